// Batched restarted GMRES for many small systems (the serving path): one
// persistent launch solves every system of a batch, one workgroup per system,
// and the launch (descriptor upload, kernel, result download) is recorded once
// into a hipGraph per batch context and replayed for each batch.
//
// Per system the method is that of gmres_solve (Sec. 2.7; right preconditioning
// with M = LU of Eq. (7)-(8); Alg. 3 level order for the triangular solves),
// carried out by the workgroup alone:
//  * SpMV over the HEC arrays (Alg. 1: the ELL slab, then the CSR remainder),
//    one row per thread, FP64 accumulation;
//  * the preconditioner solve in level order (Eq. (11), Alg. 3) over a
//    level-ordered copy of each triangle: 64-row chunks of one level are taken
//    by the 16 wavefronts in turn, and a row reads each dependency from LDS as
//    soon as it is final (the LDS vectors start filled with a signalling-NaN
//    pattern that arithmetic never produces), so no barrier separates levels;
//  * classical Gram-Schmidt applied twice, deterministic block reductions,
//    Givens rotations and the small least-squares solve in FP64 in LDS;
//  * cycles restart from the FP64 true residual. precision 1: each cycle uses the
//    FP32 copies of the matrix and factor values (FP64 vectors and arithmetic),
//    asked for a reduction of inner_rtol, and the FP64 true residual refines.
// Nothing a workgroup computes depends on the other systems of the batch, so a
// system's result is bit-identical alone and in any batch.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <mutex>

#include "hec_internal.hpp"

namespace hec {
namespace {

constexpr int kBT = 1024;         // threads per system
constexpr int kBW = kBT / 64;     // wavefronts per system
constexpr int kBMaxM = 32;        // largest restart length
constexpr int kBRedStride = 33;   // per-wavefront partial sums in LDS
constexpr int kRows = (HEC_BATCH_MAX_N + kBT - 1) / kBT;  // rows per thread at most

struct BatchSys {
    int32_t n, K, ld, has_rem;
    const int32_t *ell_col;
    const double *ell_val;
    const float *ell_val32;
    const int32_t *rem_ptr, *rem_col;
    const double *rem_val;
    const float *rem_val32;
    // level-ordered triangles (lower, upper): chunk starts, position -> row,
    // dependency rows and values at s*ldq + q, pivots (upper)
    int32_t KL, KU, ldq, nchL, nchU;
    const int32_t *chL, *rowL, *colL, *chU, *rowU, *colU;
    const double *valL, *valU, *pivU;
    const float *valL32, *valU32, *pivU32;
    const double *b;
    double *x;
    double *ws;  // (2m + 3) * n doubles: V (m+1), Z (m), r, w
};

struct BatchHead {
    int32_t count, restart, maxit, precision, x0_zero;
    uint32_t spin;  // polls a wait for a dependency makes before it gives up
    double rtol, target, inner_rtol;
};

struct BatchOut {
    int32_t status, iterations, restarts, ir_steps;
    double rel_res_true, rel_res_est;
};

// LDS layout of one system (dynamic): ly[max_n] | lz[max_n] | red[kBW][33] |
// H[(m+1)][m] | cs[m] | sn[m] | g[m+1] | y[m] | sc[8] (sc[7]: the give-up flag, an int)
struct Lds {
    double *ly, *lz, *red, *H, *cs, *sn, *g, *y, *sc;
};

__host__ __device__ inline size_t batch_lds_bytes(int max_n, int m) {
    return sizeof(double) * (2 * (size_t)max_n + kBW * kBRedStride + (size_t)(m + 1) * m + 4 * (size_t)m + 1 + 8);
}

constexpr unsigned long long kSent = 0x7FF4DEADBEEF1234ull;  // signalling NaN: never produced by arithmetic
constexpr unsigned long long kQNaN = 0x7FF8000000000000ull;

template <class VT> __device__ __forceinline__ const VT *ellv(const BatchSys &S);
template <> __device__ __forceinline__ const double *ellv<double>(const BatchSys &S) { return S.ell_val; }
template <> __device__ __forceinline__ const float *ellv<float>(const BatchSys &S) { return S.ell_val32; }
template <class VT> __device__ __forceinline__ const VT *remv(const BatchSys &S);
template <> __device__ __forceinline__ const double *remv<double>(const BatchSys &S) { return S.rem_val; }
template <> __device__ __forceinline__ const float *remv<float>(const BatchSys &S) { return S.rem_val32; }
template <class VT> __device__ __forceinline__ const VT *fval(const BatchSys &S, bool up);
template <> __device__ __forceinline__ const double *fval<double>(const BatchSys &S, bool up) {
    return up ? S.valU : S.valL;
}
template <> __device__ __forceinline__ const float *fval<float>(const BatchSys &S, bool up) {
    return up ? S.valU32 : S.valL32;
}
template <class VT> __device__ __forceinline__ const VT *fpiv(const BatchSys &S);
template <> __device__ __forceinline__ const double *fpiv<double>(const BatchSys &S) { return S.pivU; }
template <> __device__ __forceinline__ const float *fpiv<float>(const BatchSys &S) { return S.pivU32; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sums of the per-thread partials p[0..nv) over the workgroup, in a fixed order;
// out[k] (LDS) receives sum k. Ends with a barrier.
template <int NV>
__device__ void block_sums(const double (&p)[NV], int nv, const Lds &L, double *out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        if (k < nv) {
            const double s = wave_sum(p[k]);
            if (lane == 0) L.red[wave * kBRedStride + k] = s;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nv) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kBW; ++w) t += L.red[w * kBRedStride + threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

__device__ double block_norm(const double *v, int n, const Lds &L) {
    double p[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += kBT) p[0] += v[i] * v[i];
    block_sums<1>(p, 1, L, L.sc);
    return sqrt(L.sc[0]);
}

// y = A x (z == nullptr) or y = z - A x; Alg. 1 order: ELL entries, then remainder.
template <class VT>
__device__ void b_spmv(const BatchSys &S, const double *x, double *y, const double *z) {
    const VT *ev = ellv<VT>(S);
    const VT *rv = remv<VT>(S);
    for (int i = threadIdx.x; i < S.n; i += kBT) {
        double s = 0.0;
        for (int k = 0; k < S.K; ++k) {
            const size_t e = (size_t)k * S.ld + i;
            s += (double)ev[e] * x[S.ell_col[e]];
        }
        if (S.has_rem)
            for (int e = S.rem_ptr[i]; e < S.rem_ptr[i + 1]; ++e) s += (double)rv[e] * x[S.rem_col[e]];
        y[i] = z ? z[i] - s : s;
    }
    __syncthreads();
}

__device__ __forceinline__ unsigned long long lds_load_bits(const double *p) {
    return __hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One triangle in level order: wavefront w takes chunks w, w + 16, ... (each at
// most 64 rows of one level); a row waits in LDS for each dependency to leave the
// sentinel. Every dependency lies in an earlier chunk, so the lowest unfinished
// chunk can always proceed. Lower: dst = L^{-1} src (src in global memory, unit
// diagonal). Upper: dst = U^{-1} src (src in LDS), also stored to out.
template <class VT, bool UPPER>
__device__ void b_tri(const BatchSys &S, const double *src, double *dst, double *out, uint32_t spin,
                      int *timed_out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nch = UPPER ? S.nchU : S.nchL, K = UPPER ? S.KU : S.KL, ldq = S.ldq;
    const int32_t *ch = UPPER ? S.chU : S.chL, *rowp = UPPER ? S.rowU : S.rowL, *colp = UPPER ? S.colU : S.colL;
    const VT *valp = fval<VT>(S, UPPER);
    for (int c = wave; c < nch; c += kBW) {
        const int q = ch[c] + lane;
        if (q >= ch[c + 1]) continue;
        const int row = rowp[q];
        double acc = src[row];
        for (int s0 = 0; s0 < K; s0 += 8) {
            int j[8];
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int s = s0 + u;
                j[u] = s < K ? colp[(size_t)s * ldq + q] : INT_MIN;
                a[u] = j[u] >= 0 ? (double)valp[(size_t)s * ldq + q] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (j[u] < 0) continue;
                unsigned long long bits = lds_load_bits(dst + j[u]);
                uint32_t it = 0;
                while (bits == kSent) {
                    if (++it > spin) {  // give up: the row goes on with a NaN, the system reports it
                        *timed_out = 1;
                        bits = kQNaN;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    bits = lds_load_bits(dst + j[u]);
                }
                acc -= a[u] * __longlong_as_double((long long)bits);
            }
        }
        if constexpr (UPPER) acc = acc / (double)fpiv<VT>(S)[q];
        unsigned long long r = (unsigned long long)__double_as_longlong(acc);
        if (r == kSent) r = kQNaN;  // keep a final value distinguishable from "not ready"
        if (out) out[row] = __longlong_as_double((long long)r);
        __hip_atomic_store((unsigned long long *)(dst + row), r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// out = U^{-1} L^{-1} v (Eq. (7)-(8)). Ends with a barrier.
template <class VT>
__device__ void b_prec(const BatchSys &S, const double *v, double *out, const Lds &L, uint32_t spin,
                       int *timed_out) {
    const double sent = __longlong_as_double((long long)kSent);
    for (int i = threadIdx.x; i < S.n; i += kBT) {
        L.ly[i] = sent;
        L.lz[i] = sent;
    }
    __syncthreads();
    b_tri<VT, false>(S, v, L.ly, nullptr, spin, timed_out);
    __syncthreads();
    b_tri<VT, true>(S, L.ly, L.lz, out, spin, timed_out);
    __syncthreads();
}

// One GMRES cycle from the residual r (norm beta > 0): at most mcyc Arnoldi
// steps, stopping once the rotated residual estimate is <= tol; x += Z y.
// Returns the steps taken; *est receives the last estimate.
template <class VT>
__device__ int b_cycle(const BatchSys &S, int m, int mcyc, double tol, const double *r, double beta, const Lds &L,
                       double *est, uint32_t spin, int *timed_out) {
    const int n = S.n;
    double *V = S.ws, *Z = V + (size_t)(m + 1) * n, *w = Z + (size_t)m * n + n;
    for (int i = threadIdx.x; i < n; i += kBT) V[i] = r[i] / beta;
    if (threadIdx.x == 0) L.g[0] = beta;
    __syncthreads();
    int j = 0;
    double res = beta;
    while (j < mcyc) {
        double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
        b_prec<VT>(S, vj, zj, L, spin, timed_out);
        b_spmv<VT>(S, zj, w, nullptr);
        // classical Gram-Schmidt, twice: h = V^T w, w -= V h
        for (int pass = 0; pass < 2; ++pass) {
            // the thread's rows of w in registers; one wavefront sum per basis vector
            double wr[kRows];
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const int i = threadIdx.x + r * kBT;
                wr[r] = i < n ? w[i] : 0.0;
            }
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
            for (int k = 0; k <= j; ++k) {
                const double *vk = V + (size_t)k * n;
                double p = 0.0;
#pragma unroll
                for (int r = 0; r < kRows; ++r) {
                    const int i = threadIdx.x + r * kBT;
                    if (i < n) p += vk[i] * wr[r];
                }
                p = wave_sum(p);
                if (lane == 0) L.red[wave * kBRedStride + k] = p;
            }
            __syncthreads();
            if ((int)threadIdx.x <= j) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < kBW; ++q) t += L.red[q * kBRedStride + threadIdx.x];
                L.y[threadIdx.x] = t;
            }
            __syncthreads();
            for (int i = threadIdx.x; i < n; i += kBT) {
                double wi = w[i];
                for (int k = 0; k <= j; ++k) wi -= V[(size_t)k * n + i] * L.y[k];
                w[i] = wi;
            }
            if ((int)threadIdx.x <= j) L.H[threadIdx.x * m + j] = (pass ? L.H[threadIdx.x * m + j] : 0.0) + L.y[threadIdx.x];
            __syncthreads();
        }
        const double hn = block_norm(w, n, L);
        if (threadIdx.x == 0) {
            // previous rotations, then the one that zeroes H[j+1][j]
            for (int k = 0; k < j; ++k) {
                const double a = L.H[k * m + j], b = L.H[(k + 1) * m + j];
                L.H[k * m + j] = L.cs[k] * a + L.sn[k] * b;
                L.H[(k + 1) * m + j] = -L.sn[k] * a + L.cs[k] * b;
            }
            const double a = L.H[j * m + j];
            const double d = hypot(a, hn);
            const double c = d > 0.0 ? a / d : 1.0, s = d > 0.0 ? hn / d : 0.0;
            L.cs[j] = c;
            L.sn[j] = s;
            L.H[j * m + j] = d;
            L.g[j + 1] = -s * L.g[j];
            L.g[j] = c * L.g[j];
            L.sc[1] = fabs(L.g[j + 1]);
        }
        __syncthreads();
        res = L.sc[1];
        ++j;
        if (res <= tol || hn == 0.0 || j == mcyc) break;
        double *vn = V + (size_t)j * n;
        for (int i = threadIdx.x; i < n; i += kBT) vn[i] = w[i] / hn;
        __syncthreads();
    }
    // y = H(0:j, 0:j)^{-1} g(0:j), then x += Z y
    if (threadIdx.x == 0) {
        for (int k = j - 1; k >= 0; --k) {
            double t = L.g[k];
            for (int c = k + 1; c < j; ++c) t -= L.H[k * m + c] * L.y[c];
            L.y[k] = L.H[k * m + k] != 0.0 ? t / L.H[k * m + k] : 0.0;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kBT) {
        double xi = S.x[i];
        for (int k = 0; k < j; ++k) xi += Z[(size_t)k * n + i] * L.y[k];
        S.x[i] = xi;
    }
    __syncthreads();
    *est = res;
    return j;
}

__global__ __launch_bounds__(kBT) void k_gmres_batch(const BatchHead *__restrict__ head,
                                                     const BatchSys *__restrict__ sys, BatchOut *__restrict__ out,
                                                     int max_n) {
    const BatchHead H = *head;
    if ((int)blockIdx.x >= H.count) return;
    const BatchSys S = sys[blockIdx.x];
    extern __shared__ __align__(16) char bsmem[];
    const int m = H.restart;
    Lds L;
    L.ly = (double *)bsmem;
    L.lz = L.ly + max_n;
    L.red = L.lz + max_n;
    L.H = L.red + kBW * kBRedStride;
    L.cs = L.H + (size_t)(m + 1) * m;
    L.sn = L.cs + m;
    L.g = L.sn + m;
    L.y = L.g + m + 1;
    L.sc = L.y + m;
    const int n = S.n;
    double *r = S.ws + (size_t)(2 * m + 1) * n;
    BatchOut o{HEC_OK, 0, 0, 0, 0.0, 0.0};
    // a wait for a dependency gave up in this system's solves (a word of the scalar area;
    // no static LDS: the kernel's dynamic LDS may take the whole workgroup limit)
    int *const timed_out = (int *)(L.sc + 7);
    if (threadIdx.x == 0) *timed_out = 0;
    const double bnorm = block_norm(S.b, n, L);  // (its barriers publish the flag's reset)
    if (bnorm == 0.0 || n == 0) {
        for (int i = threadIdx.x; i < n; i += kBT) S.x[i] = 0.0;
    } else {
        if (H.x0_zero)
            for (int i = threadIdx.x; i < n; i += kBT) S.x[i] = 0.0;
        __syncthreads();
        b_spmv<double>(S, S.x, r, S.b);
        double res = block_norm(r, n, L);
        int cycles = 0;
        while (res / bnorm > H.target && o.iterations < H.maxit) {
            const int mcyc = min(m, H.maxit - o.iterations);
            double est = 0.0;
            int jd;
            if (H.precision == 0) {
                jd = b_cycle<double>(S, m, mcyc, H.target * bnorm, r, res, L, &est, H.spin, timed_out);
            } else {
                const double tol = fmax(H.inner_rtol * res, 0.5 * H.target * bnorm);
                jd = b_cycle<float>(S, m, mcyc, tol, r, res, L, &est, H.spin, timed_out);
                o.ir_steps++;
            }
            o.rel_res_est = est / bnorm;
            o.iterations += jd;
            cycles++;
            b_spmv<double>(S, S.x, r, S.b);
            res = block_norm(r, n, L);
            if (jd == 0) break;
        }
        o.restarts = max(0, cycles - 1);
        o.rel_res_true = res / bnorm;
        if (!(res / bnorm <= H.target)) o.status = HEC_ERR_NOT_CONVERGED;
    }
    __syncthreads();
    if (*timed_out) o.status = HEC_ERR_TIMEOUT;
    if (threadIdx.x == 0) out[blockIdx.x] = o;
}

}  // namespace
}  // namespace hec

// Batch context: pinned descriptor staging, device descriptors and results,
// per-system workspaces, and the recorded graph.
struct hec_batch_s {
    int32_t capacity = 0, restart = 0, max_n = 0;
    bool use_graph = true;
    size_t lds = 0;
    hipStream_t bs = nullptr;   // the context's own stream (graphs are recorded and replayed on it)
    hipEvent_t ev = nullptr;
    hec::BatchHead *h_head = nullptr;
    hec::BatchSys *h_sys = nullptr;
    hec::BatchOut *h_out = nullptr;
    int64_t dev_bytes = 0;      // device bytes of the buffers below
    hec::DevBuf<hec::BatchHead> d_head;
    hec::DevBuf<hec::BatchSys> d_sys;
    hec::DevBuf<hec::BatchOut> d_out;
    hec::DevBuf<double> d_ws;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~hec_batch_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (bs) (void)hipStreamSynchronize(bs);
        d_ws.release();  // in order on bs, before it is destroyed
        d_out.release();
        d_sys.release();
        d_head.release();
        if (h_out) (void)hipHostFree(h_out);
        if (h_sys) (void)hipHostFree(h_sys);
        if (h_head) (void)hipHostFree(h_head);
        if (ev) (void)hipEventDestroy(ev);
        if (bs) (void)hipStreamDestroy(bs);
    }
};

namespace hec {
namespace {

// Kernel launch plus the copies around it, on the context's stream.
void enqueue_batch(hec_batch_s &B) {
    HEC_HIP(hipMemcpyAsync(B.d_head.get(), B.h_head, sizeof(BatchHead), hipMemcpyHostToDevice, B.bs));
    HEC_HIP(hipMemcpyAsync(B.d_sys.get(), B.h_sys, sizeof(BatchSys) * B.capacity, hipMemcpyHostToDevice, B.bs));
    k_gmres_batch<<<B.capacity, kBT, B.lds, B.bs>>>(B.d_head.get(), B.d_sys.get(), B.d_out.get(), B.max_n);
    HEC_CHECK_LAUNCH();
    HEC_HIP(hipMemcpyAsync(B.h_out, B.d_out.get(), sizeof(BatchOut) * B.capacity, hipMemcpyDeviceToHost, B.bs));
}

int max_dyn_lds() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        return 64 * 1024;
    return std::min(v, 160 * 1024);
}

}  // namespace
}  // namespace hec

using namespace hec;

extern "C" {

hec_status batch_create(int32_t capacity, int32_t restart, int32_t max_n, int32_t use_graph, hec_batch *out) {
    return guarded([&] {
        if (!out) fail(HEC_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (capacity < 1 || capacity > 65535) fail(HEC_ERR_INVALID_ARG, "capacity must be in [1, 65535]");
        if (restart < 1 || restart > kBMaxM) fail(HEC_ERR_INVALID_ARG, "restart must be in [1, 32]");
        if (max_n < 1 || max_n > HEC_BATCH_MAX_N) fail(HEC_ERR_INVALID_ARG, "max_n must be in [1, HEC_BATCH_MAX_N]");
        std::unique_ptr<hec_batch_s> B(new hec_batch_s());
        B->capacity = capacity;
        B->restart = restart;
        B->max_n = max_n;
        B->use_graph = use_graph != 0;
        B->lds = batch_lds_bytes(max_n, restart);
        if ((int64_t)B->lds > max_dyn_lds()) fail(HEC_ERR_INVALID_ARG, "max_n too large for the workgroup's LDS");
        // once per process; a failure is reported (and taken off the runtime's last-error
        // slot, where it would otherwise surface in the caller's next HIP call)
        static const hipError_t attr = hipFuncSetAttribute((const void *)k_gmres_batch,
                                                           hipFuncAttributeMaxDynamicSharedMemorySize, max_dyn_lds());
        if (attr != hipSuccess) {
            (void)hipGetLastError();
            fail(HEC_ERR_HIP, std::string("hipFuncSetAttribute(k_gmres_batch): ") + hipGetErrorString(attr));
        }
        HEC_HIP(hipStreamCreateWithFlags(&B->bs, hipStreamNonBlocking));
        HEC_HIP(hipEventCreateWithFlags(&B->ev, hipEventDisableTiming));
        HEC_HIP(hipHostMalloc((void **)&B->h_head, sizeof(BatchHead), hipHostMallocDefault));
        HEC_HIP(hipHostMalloc((void **)&B->h_sys, sizeof(BatchSys) * capacity, hipHostMallocDefault));
        HEC_HIP(hipHostMalloc((void **)&B->h_out, sizeof(BatchOut) * capacity, hipHostMallocDefault));
        std::memset(B->h_sys, 0, sizeof(BatchSys) * capacity);
        {
            StreamScope scope(B->bs);
            OwnerScope own(&B->dev_bytes);
            B->d_head.alloc(1);
            B->d_sys.alloc(capacity);
            B->d_out.alloc(capacity);
            B->d_ws.alloc((size_t)(2 * restart + 3) * max_n * capacity);
            HEC_HIP(hipStreamSynchronize(B->bs));
        }
        *out = B.release();
    });
}

hec_status batch_destroy(hec_batch B) {
    return guarded([&] { delete B; });
}

hec_status gmres_solve_batched(hec_batch B, int32_t count, const hec_matrix *A, const hec_ilu *M,
                               const hec_levels *lv, const double *const *b, double *const *x,
                               const hec_solve_opts *o, hec_solve_info *info, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    hec_status st = guarded([&] {
        if (!B || !o) fail(HEC_ERR_INVALID_ARG, "null batch context or options");
        if (count < 0 || count > B->capacity) fail(HEC_ERR_INVALID_ARG, "count must be in [0, capacity]");
        if (count > 0 && (!A || !M || !lv || !b || !x)) fail(HEC_ERR_INVALID_ARG, "null array argument");
        if (o->restart != B->restart) fail(HEC_ERR_INVALID_ARG, "restart differs from the batch context's");
        if (o->maxit < 0) fail(HEC_ERR_INVALID_ARG, "maxit < 0");
        if (!(o->rtol > 0.0)) fail(HEC_ERR_INVALID_ARG, "rtol must be > 0");
        if (o->precision != 0 && o->precision != 1) fail(HEC_ERR_INVALID_ARG, "precision must be 0 or 1");
        const bool mixed = o->precision == 1;
        const size_t per = (size_t)(2 * B->restart + 3) * B->max_n;
        // the previous batch (if any) has completed: every call synchronises before it returns
        for (int32_t i = 0; i < count; ++i) {
            hec_matrix a = A[i];
            hec_ilu f = M[i];
            hec_levels l = lv[i];
            if (!a || !f || !l) fail(HEC_ERR_INVALID_ARG, "null handle in the batch");
            if (a->n != f->n || a->n != l->n || f->n != f->n_sys)
                fail(HEC_ERR_INVALID_ARG, "matrix, factor and levels differ in size (or a RAS factor)");
            if (a->n > B->max_n) fail(HEC_ERR_INVALID_ARG, "system larger than the batch context's max_n");
            if (a->n > 0 && (!b[i] || !x[i])) fail(HEC_ERR_INVALID_ARG, "b or x is NULL");
            if (mixed && (!a->has_f32 || !f->has_f32))
                fail(HEC_ERR_INVALID_ARG, "mixed precision needs HEC_KEEP_F32 on the matrix and the factor");
            if (a->n > 0 && (l->lower.flat.nchunks == 0 || l->upper.flat.nchunks == 0))
                fail(HEC_ERR_INVALID_ARG, "levels handle has no level-ordered copy (n above HEC_BATCH_MAX_N)");
            BatchSys &S = B->h_sys[i];
            S.n = a->n;
            S.K = a->K;
            S.ld = a->ld;
            S.has_rem = a->nnz_rem > 0;
            S.ell_col = a->ell_col.get();
            S.ell_val = a->ell_val.get();
            S.ell_val32 = a->ell_val32.get();
            S.rem_ptr = a->rem_ptr.get();
            S.rem_col = a->rem_col.get();
            S.rem_val = a->rem_val.get();
            S.rem_val32 = a->rem_val32.get();
            const hec_flat &fl = l->lower.flat, &fu = l->upper.flat;
            S.KL = fl.K;
            S.KU = fu.K;
            S.ldq = fl.ldq;
            S.nchL = fl.nchunks;
            S.nchU = fu.nchunks;
            S.chL = fl.chunk_ptr.get();
            S.rowL = fl.row.get();
            S.colL = fl.col.get();
            S.valL = fl.val.get();
            S.valL32 = fl.val32.get();
            S.chU = fu.chunk_ptr.get();
            S.rowU = fu.row.get();
            S.colU = fu.col.get();
            S.valU = fu.val.get();
            S.valU32 = fu.val32.get();
            S.pivU = fu.piv.get();
            S.pivU32 = fu.piv32.get();
            S.b = b[i];
            S.x = x[i];
            S.ws = B->d_ws.get() + per * i;
        }
        BatchHead &Hh = *B->h_head;
        Hh.count = count;
        Hh.restart = B->restart;
        Hh.maxit = o->maxit;
        Hh.precision = o->precision;
        Hh.x0_zero = o->x0_zero;
        Hh.spin = spin_limit();
        Hh.rtol = o->rtol;
        Hh.target = mixed && o->ir_rtol > 0.0 ? std::min(o->ir_rtol, o->rtol) : o->rtol;
        Hh.inner_rtol = o->inner_rtol > 0.0 ? o->inner_rtol : 1e-4;
        if (count == 0) return;
        // order after the caller's stream (b, x and the handles' setup), run, wait
        hipStream_t us = as_stream(stream);
        HEC_HIP(hipEventRecord(B->ev, us));
        HEC_HIP(hipStreamWaitEvent(B->bs, B->ev, 0));
        if (B->use_graph) {
            if (!B->exec) {
                HEC_HIP(hipStreamBeginCapture(B->bs, hipStreamCaptureModeThreadLocal));
                try {
                    enqueue_batch(*B);
                } catch (...) {
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(B->bs, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                HEC_HIP(hipStreamEndCapture(B->bs, &B->graph));
                HEC_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
            }
            HEC_HIP(hipGraphLaunch(B->exec, B->bs));
        } else {
            enqueue_batch(*B);
        }
        HEC_HIP(hipStreamSynchronize(B->bs));
    });
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info && B && o) {
        for (int32_t i = 0; i < count && i <= B->capacity - 1; ++i) {
            hec_solve_info &f = info[i];
            f = hec_solve_info{};
            if (st == HEC_OK) {
                const BatchOut &r = B->h_out[i];
                f.status = r.status;
                f.iterations = r.iterations;
                f.restarts = r.restarts;
                f.ir_steps = r.ir_steps;
                f.rel_res_true = r.rel_res_true;
                f.rel_res_est = r.rel_res_est;
            } else {
                f.status = st;
            }
            f.seconds = secs;
        }
    }
    if (st == HEC_OK && B) {
        for (int32_t i = 0; i < count; ++i)
            if (B->h_out[i].status == HEC_ERR_TIMEOUT) {
                set_last_error("a wait of a system's triangular solve gave up (hec_set_spin_limit)");
                return HEC_ERR_TIMEOUT;
            }
        for (int32_t i = 0; i < count; ++i)
            if (B->h_out[i].status != HEC_OK) {
                set_last_error("a system of the batch did not converge");
                return HEC_ERR_NOT_CONVERGED;
            }
    }
    return st;
}

}  // extern "C"
