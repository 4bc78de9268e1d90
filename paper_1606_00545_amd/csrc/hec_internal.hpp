// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hec.h"
#include "plan.hpp"

namespace hec {

// ------------------------------------------------------------------ errors

struct Error : std::runtime_error {
    hec_status code;
    Error(hec_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &msg);

[[noreturn]] inline void fail(hec_status c, const std::string &m) { throw Error(c, m); }

#define HEC_HIP(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            ::hec::fail(e_ == hipErrorOutOfMemory ? HEC_ERR_NOMEM : HEC_ERR_HIP,               \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                    \
    } while (0)

#define HEC_CHECK_LAUNCH() HEC_HIP(hipGetLastError())

// Run `body` and translate exceptions into a status + thread-local message.
template <class F>
hec_status guarded(F &&body) {
    try {
        body();
        set_last_error("");
        return HEC_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return HEC_ERR_NOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return HEC_ERR_HIP;
    }
}

// ------------------------------------------------------------------ device memory

// The stream on which the calling thread's current entry point allocates
// (set by StreamScope). Allocation is stream-ordered (hipMallocAsync /
// hipFreeAsync by default, or the hooks of hec_set_allocator, which get the
// stream), so setting up or releasing one system never synchronises the whole
// device while other systems run on other streams.
hipStream_t &alloc_stream();
void ensure_pool();

struct StreamScope {
    hipStream_t prev;
    explicit StreamScope(hipStream_t s) : prev(alloc_stream()) {
        ensure_pool();
        alloc_stream() = s;
    }
    ~StreamScope() { alloc_stream() = prev; }
};

// The allocator in force when a buffer was allocated (alloc == NULL: the default
// hipMallocAsync / hipFreeAsync); a buffer is always freed by the allocator that
// made it, whatever hec_set_allocator says by then.
struct Allocator {
    hec_alloc_fn alloc = nullptr;
    hec_free_fn free = nullptr;
    void *ctx = nullptr;
};
Allocator current_allocator();
void *dev_alloc(size_t bytes, hipStream_t s, const Allocator &a);  // throws NOMEM on failure
void dev_free(void *p, size_t bytes, hipStream_t s, const Allocator &a);

// The byte counter of the handle that owns the buffers the calling thread
// allocates (set by OwnerScope; NULL: nobody counts them). hec_footprint reports
// these counters.
int64_t *&alloc_owner();

struct OwnerScope {
    int64_t *prev;
    explicit OwnerScope(int64_t *owner) : prev(alloc_owner()) { alloc_owner() = owner; }
    ~OwnerScope() { alloc_owner() = prev; }
};

// Owning device buffer, allocated and freed in order on the stream that was
// current when it was allocated, by the allocator current then; its bytes count
// towards the owner that was current then.
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    hipStream_t st = nullptr;
    Allocator al;
    int64_t *owner = nullptr;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    bool borrowed = false;  // a view of memory owned elsewhere: never freed or counted here
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n), st(o.st), al(o.al), owner(o.owner), borrowed(o.borrowed) {
        o.p = nullptr;
        o.n = 0;
        o.owner = nullptr;
        o.borrowed = false;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p; n = o.n; st = o.st; al = o.al; owner = o.owner; borrowed = o.borrowed;
            o.p = nullptr; o.n = 0; o.owner = nullptr; o.borrowed = false;
        }
        return *this;
    }
    // Points the buffer at `count` elements of memory owned elsewhere (no allocation).
    void borrow(T *ptr, size_t count) {
        release();
        p = ptr;
        n = count;
        borrowed = true;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        st = alloc_stream();
        al = current_allocator();
        if (count) {
            p = (T *)dev_alloc(count * sizeof(T), st, al);
            n = count;
            owner = alloc_owner();
            if (owner) *owner += (int64_t)(count * sizeof(T));
        }
    }
    void release() {
        if (p && !borrowed) {
            dev_free(p, n * sizeof(T), st, al);
            if (owner) *owner -= (int64_t)(n * sizeof(T));
        }
        p = nullptr;
        n = 0;
        owner = nullptr;
        borrowed = false;
    }
    void upload(const T *h, size_t count, hipStream_t s) {
        if (count) HEC_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
    }
    void download(T *h, size_t count, hipStream_t s) const {
        if (count) HEC_HIP(hipMemcpyAsync(h, p, count * sizeof(T), hipMemcpyDeviceToHost, s));
    }
    T *get() const { return p; }
};

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline unsigned ceil_div(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

// ------------------------------------------------------------------ host CSR checks

// Validates a host CSR (Ap monotone from 0, columns strictly ascending and in range).
// ncols < 0: a square matrix (columns < n)
void validate_csr(int32_t n, const int32_t *Ap, const int32_t *Aj, const double *Ax, int32_t ncols = -1);

}  // namespace hec

// ------------------------------------------------------------------ handles

namespace hec {
struct KrylovWS;  // solver workspace, cached on the matrix handle (defined in krylov.hip)
struct KrylovWSDeleter {
    void operator()(KrylovWS *) const;
};
}  // namespace hec

struct hec_matrix_s {
    int64_t dev_bytes = 0;    // device bytes held by the matrix (its solver workspace included)
    int32_t n = 0, K = 0, ld = 0;
    int64_t nnz = 0, nnz_rem = 0;
    int32_t n_rem_rows = 0;   // rows with a nonempty remainder of fewer than 1024 entries
    int32_t n_rem_long = 0;   // rows with a remainder of 1024 entries or more
    int32_t rem_lanes = 64;   // lanes per remainder row in the CSR kernel
    bool has_f32 = false;
    hec::DevBuf<int32_t> ell_col;
    hec::DevBuf<double> ell_val;
    hec::DevBuf<float> ell_val32;
    hec::DevBuf<int32_t> rem_ptr;   // n+1
    hec::DevBuf<int32_t> rem_col;
    hec::DevBuf<double> rem_val;
    hec::DevBuf<float> rem_val32;
    hec::DevBuf<int32_t> rem_rows;  // ascending short-remainder rows (all short rows when K == 0)
    hec::DevBuf<int32_t> rem_long;  // ascending long-remainder rows, one workgroup each
    // COO remainder (HEC_COO_REMAINDER: the HYB layout): the row of every remainder
    // entry, multiplied entry-parallel in tiles; partial sums of the rows cut by tile
    // boundaries (2 per tile: row, then value) are finished by a second launch
    bool coo = false;
    int64_t coo_tiles = 0;
    hec::DevBuf<int32_t> rem_row;
    hec::DevBuf<int32_t> carry_row;  // 2 * coo_tiles
    hec::DevBuf<double> carry_val;   // 2 * coo_tiles slots of 8 bytes (holds FP32 sums for FP32 values)
    std::unique_ptr<hec::KrylovWS, hec::KrylovWSDeleter> ws;
};

namespace hec {
// HEC (HYB, ELL, CSR) form of an n x ncols CSR matrix already validated; hec_from_csr's
// ell_width and flags.
std::unique_ptr<hec_matrix_s> make_hec(int32_t n, int32_t ncols, const int32_t *Ap, const int32_t *Aj,
                                       const double *Ax, int32_t ell_width, uint32_t flags, hipStream_t s);
}  // namespace hec

struct hec_ilu_s {
    int64_t dev_bytes = 0;  // device bytes held by the factor
    int32_t n = 0, k = 0;   // n: size of the factor (the stacked extended blocks for RAS)
    // restricted additive Schwarz (Sec. 2.5): system size, blocks of the stacked factor
    // (rows hblocks[b] .. hblocks[b+1]-1), the system row of each stacked row, and the
    // stacked row that owns each system row. Without RAS: n_sys == n, hblocks empty.
    int32_t n_sys = 0, nblocks = 1, overlap = 0;
    std::vector<int32_t> hblocks, hext_row, hown;
    int32_t gnx = 0, gny = 0, gnz = 0;  // natural-order grid of A's stencil, if recognised (0: none)
    int64_t nnz = 0;
    bool has_f32 = false;
    std::vector<int32_t> hLUp, hLUj;  // host copy of the pattern S_k (used by level_schedule)
    std::vector<int32_t> hdiag;       // position of the diagonal in each row
    hec::DevBuf<int32_t> LUp, LUj, diag;
    hec::DevBuf<double> LUx;
    hec::DevBuf<float> LUx32;
};

// Level-ordered copy of one triangle for the batched small-system solver:
// positions in Alg. 3 order cut into chunks of at most 64 rows of one level;
// entry s of position q at s*ldq + q holds the dependency's row (INT_MIN pad)
// and its value; piv: u_ii per position (upper only).
struct hec_flat {
    int32_t K = 0, ldq = 0, nchunks = 0;
    hec::DevBuf<int32_t> chunk_ptr, row, col;
    hec::DevBuf<double> val, piv;
    hec::DevBuf<float> val32, piv32;
};

// One triangle of the factor with its level schedule (Eq. (11), Alg. 3) and
// the blocked execution plan of the triangular solve: rows are cut into parts
// (contiguous row ranges in the order the triangle is solved), each part's rows
// are laid out at consecutive positions sorted by (level, row), and each part is
// cut into sub-segments of at most 64 rows of one level. Entry s of position q
// is stored at s*ldq + q.
// Wavefront plan of a grid triangle (plan.hpp's GridPlan) on the device.
struct hec_grid {
    bool on = false;
    int32_t TA = 8;  // tile side along a: 8 (8 x 8 tiles, 3D grid) or 64 (64 x 1, 2D grid)
    int32_t NA = 0, NB = 0, NC = 0, PA = 0, PB = 0, S = 0;
    int64_t sa = 0, sb = 0, sc = 0;
    hec::DevBuf<double> coef;  // [claim][step][k][lane]; k = 3 (upper): the reciprocal pivot
    hec::DevBuf<float> coef32;
    int64_t face_elems() const { return (int64_t)PA * PB * 2 * S * 8; }
    int64_t pad_elems() const { return (int64_t)PA * PB * S * 64; }  // positions (claim, step, lane)
};

struct hec_tri {
    int32_t nlev = 0;
    std::vector<int32_t> hlevel_ptr, hperm;  // Alg. 3: level start pointers, rows by (level, row)
    hec_flat flat;                           // small systems only: level-ordered copy for the batched solver
    int32_t K = 0, KC = 4, ldq = 0, nparts = 0, nss = 0, W = 0, S = 0;  // KC: K padded to 4/8/16/32
    int32_t NS = 1;                          // solver wavefronts per workgroup
    int32_t D64 = 0, D32 = 0;                // ring depths for the FP64 / FP32 solve
    bool blocked = true;                     // false: rows too long for LDS slots, per-row polling kernel
    int32_t nchunks = 0;                     // fallback plan: 64-row chunks of one level
    hec::DevBuf<int32_t> chunk_ptr;
    size_t lds64 = 0, lds32 = 0;             // dynamic LDS bytes of the solve kernels
    hec::DevBuf<int32_t> part_ss;   // nparts+1: sub-segment range of each part
    hec::DevBuf<int32_t> part_pos;  // nparts+1: first position of each part
    hec::DevBuf<int32_t> ss_pos;    // nss+1: first position of each sub-segment
    hec::DevBuf<int32_t> ss_need;   // nss (NS > 1): dependency bound of each sub-segment in its part
    hec::DevBuf<int32_t> grow;      // position -> row
    std::vector<int32_t> hgrow;     // host copy of grow
    hec::DevBuf<int32_t> other;     // lower: the row's position in the upper plan; upper with RAS: the
                                    // system row an owned stacked row is written to (-1: overlap row)
    hec::DevBuf<int32_t> bmap;      // lower with RAS: the system row whose right-hand side a position reads
    hec::DevBuf<int32_t> enc;       // K*ldq: -(local position+1) inside the part, position outside, INT_MIN pad
    hec::DevBuf<double> val;
    hec::DevBuf<float> val32;
    hec::DevBuf<double> piv;        // upper only: u_ii per position
    hec::DevBuf<float> piv32;
    hec_grid grid;                  // wavefront plan (7-point ILU(0) grids); when on, the blocked
                                    // plan above is not built (levels only)
};

namespace hec {
// Words of hec_levels_s::sync: part tickets and finished-workgroup counters of the
// lower (0, 1) and upper (2, 3) solves, then the error word a triangular-solve wait
// sets when it gives up (read and cleared by the host).
constexpr int kLevelsErrWord = 4;
constexpr int kLevelsSyncWords = 8;

// Polls a device-side wait of the triangular solves makes before it gives up
// (hec_set_spin_limit).
uint32_t spin_limit();

// Whether level_schedule gives wavefront plans where they apply (hec_set_trsv_grid;
// default on).
bool trsv_grid_enabled();

// Reads and clears the error word of lv after synchronising s; HEC_ERR_TIMEOUT if a
// triangular-solve wait gave up since the last check.
void check_levels(const hec_levels_s &lv, hipStream_t s);
}  // namespace hec

struct hec_levels_s {
    int64_t dev_bytes = 0;  // device bytes held by the schedules, plans and solve scratch
    int32_t n = 0;    // system size (vectors the caller passes)
    int32_t nf = 0;   // factor size (the stacked extended blocks for RAS)
    bool ras = false;
    hec_tri lower, upper;
    hec::DevBuf<uint32_t> sync;  // part tickets + finished-workgroup counters
    // Internal vectors over the factor's rows. qL/qU: each triangle's results in its own
    // plan's position order, the copy dependent rows poll (qL is sentinel-filled between
    // solves; qU is filled by every lower launch, or before a lone upper solve). yp:
    // L^{-1} b in the upper plan's order, the upper solve's right-hand side (with the
    // wavefront plans: by claim, step and lane of the lower plan, padded).
    hec::DevBuf<double> qL64, qU64, yp64;
    hec::DevBuf<float> qL32, qU32, yp32;
    // Face buffers of the wavefront solves (when both triangles have a grid plan): the
    // values tiles hand to the next tiles, sentinel-filled before a launch. fL serves
    // the lower solve of an L-then-U chain (filled by every upper launch), fU the upper
    // one (filled by every lower launch) and lone solves (filled right before).
    hec::DevBuf<double> fL64, fU64;
    hec::DevBuf<float> fL32, fU32;
};

namespace hec {

// SpMV launcher used by the API and the solvers: y = alpha*A*x + beta*z (z may be y).
// VT: value type, XT: x type, YT: y/z type.
// `skip` (device flag, may be NULL): when nonzero at launch time the kernels return at once.
template <class VT, class XT, class YT>
void spmv_launch(const hec_matrix_s &A, double alpha, const XT *x, double beta, const YT *z, YT *y,
                 hipStream_t s, const int32_t *skip = nullptr);

// Preconditioner solve pieces (launchers). T = double (FP64 factor) or float (FP32 copy).
template <class T>
void trsv_launch(const hec_levels_s &lv, uint32_t which, const T *b, T *x, hipStream_t s,
                 const int32_t *skip = nullptr);

// Sets the internal lower-solve outputs of lv to the sentinel (once, after allocation).
void trsv_init_levels(hec_levels_s &lv, hipStream_t s);

// Builds tri.grid (the wavefront plan) when the factor's triangle admits one.
void build_grid(const hec_ilu_s &M, bool upper, hec_grid &g, hipStream_t s);

// Only the level schedule of a triangle (Eq. (11), Alg. 3): nlev, hlevel_ptr, hperm.
void level_only(const hec_ilu_s &M, bool upper, hec_tri &tri);

// Builds the level schedule and blocked solve plan of one triangle of M (the
// upper plan must be built first: the lower plan records positions in it).
void build_tri(const hec_ilu_s &M, bool upper, hec_tri &tri, const hec_tri *upper_plan, hipStream_t s);

// Builds tri.flat (level-ordered copy for the batched solver) for one triangle of M.
void build_flat(const hec_ilu_s &M, bool upper, hec_tri &tri, hipStream_t s);

}  // namespace hec
