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

// Owning device buffer (hipMalloc/hipFree).
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        n = count;
        if (count) HEC_HIP(hipMalloc(&p, count * sizeof(T)));
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
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
void validate_csr(int32_t n, const int32_t *Ap, const int32_t *Aj, const double *Ax);

}  // namespace hec

// ------------------------------------------------------------------ handles

namespace hec {
struct KrylovWS;  // solver workspace, cached on the matrix handle (defined in krylov.hip)
struct KrylovWSDeleter {
    void operator()(KrylovWS *) const;
};
}  // namespace hec

struct hec_matrix_s {
    int32_t n = 0, K = 0, ld = 0;
    int64_t nnz = 0, nnz_rem = 0;
    int32_t n_rem_rows = 0;   // rows with a nonempty remainder
    int32_t rem_lanes = 64;   // lanes per remainder row in the CSR kernel
    bool has_f32 = false;
    hec::DevBuf<int32_t> ell_col;
    hec::DevBuf<double> ell_val;
    hec::DevBuf<float> ell_val32;
    hec::DevBuf<int32_t> rem_ptr;   // n+1
    hec::DevBuf<int32_t> rem_col;
    hec::DevBuf<double> rem_val;
    hec::DevBuf<float> rem_val32;
    hec::DevBuf<int32_t> rem_rows;  // ascending rows with remainder entries (all rows when K == 0)
    std::unique_ptr<hec::KrylovWS, hec::KrylovWSDeleter> ws;
};

struct hec_ilu_s {
    int32_t n = 0, k = 0;
    int64_t nnz = 0;
    bool has_f32 = false;
    std::vector<int32_t> hLUp, hLUj;  // host copy of the pattern S_k (used by level_schedule)
    std::vector<int32_t> hdiag;       // position of the diagonal in each row
    hec::DevBuf<int32_t> LUp, LUj, diag;
    hec::DevBuf<double> LUx;
    hec::DevBuf<float> LUx32;
};

// One triangle in level order, stored as a column-major ELL slab over the
// level-ordered positions q = 0..n-1 (entry s of position q at s*ldq + q).
struct hec_tri {
    int32_t nlev = 0, K = 0, ldq = 0, nchunks = 0;
    std::vector<int32_t> hlevel_ptr, hperm;
    hec::DevBuf<int32_t> perm;         // position -> row
    hec::DevBuf<int32_t> chunk_ptr;    // nchunks+1 positions; chunks never straddle a level
    hec::DevBuf<int32_t> col;          // dependency row, -1 for padding
    hec::DevBuf<double> val;
    hec::DevBuf<float> val32;
    hec::DevBuf<double> dinv_src;      // U only: the pivot u_ii per position
    hec::DevBuf<float> d32;
};

struct hec_levels_s {
    int32_t n = 0;
    hec_tri lower, upper;
    hec::DevBuf<uint32_t> sync;       // ticket + done counters for the solve kernels
    hec::DevBuf<double> tmp64;        // intermediate y of an LU solve
    hec::DevBuf<float> tmp32;
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

}  // namespace hec
