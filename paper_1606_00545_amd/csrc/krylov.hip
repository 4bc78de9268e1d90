// Krylov solvers (Sec. 2.7): restarted right-preconditioned GMRES(m),
// BiCGSTAB (Alg. 4) and preconditioned CG, built from the vector operations of
// Sec. 2.3 (Eq. (2)-(6)), the HEC SpMV and the level-scheduled preconditioner solve.
//
// Every scalar of the methods (rho, alpha, omega, the Hessenberg matrix, the
// Givens rotations, the residual estimate, the convergence flags) lives in
// device memory and is produced by the one-workgroup finishing launch of the
// reduction that needs it, so an iteration is a fixed sequence of stream-ordered
// launches with no host round trip. Once the device sets the "done" flag, the remaining
// launches of the sequence return at entry. The host looks at the flag through
// mapped pinned memory one iteration behind the device.
//
// Reductions are deterministic: the grid size depends only on n, each
// workgroup sums a fixed set of rows in a fixed order, and the finishing launch
// combines the per-workgroup partial sums in a fixed order.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "hec_internal.hpp"

namespace hec {

namespace {

constexpr int RB = 256;          // threads per reduction workgroup
constexpr int kMaxRedBlocks = 1024;
// Basis vectors are 64-element aligned plus this offset (8.5 KiB in FP64), so that
// the vectors a Gram-Schmidt pass reads together do not start at addresses that
// are equal modulo a large power of two (n = 2^21 rows otherwise puts every vector
// 16 MiB apart); measured 2-4% faster passes at 128^3.
#ifndef HEC_BASIS_PAD
#define HEC_BASIS_PAD 1088
#endif
constexpr int kMaxRestart = 32;  // the orthogonalisation keeps up to 32 basis coefficients in registers
constexpr int kDSums = 2 * kMaxRestart + 4;  // sums of one Gram-Schmidt dot pass: 2 per final vector + 3

inline int red_blocks(int64_t n) {
    int64_t b = (n + RB * 2 - 1) / (RB * 2);
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, kMaxRedBlocks));
}

// ------------------------------------------------------------------ device state layout

// Integer flags (device + mapped host mirror).
enum : int { SI_DONE = 0, SI_JDONE = 1, SI_BREAK = 2, SI_STOP_S = 3, SI_ITERS = 4, SI_COUNT = 8 };
// Double scalars.
enum : int {
    SD_BNORM = 0, SD_TOL = 1, SD_BETA = 2, SD_HNEXT = 3, SD_RES = 4,  // GMRES
    SD_RHO = 5, SD_RHO_PREV = 6, SD_ALPHA = 7, SD_OMEGA = 8,       // BiCGSTAB
    SD_SNORM2 = 9, SD_RNORM2 = 10, SD_CGBETA = 11,                 // CG: beta
    SD_TRUE = 12,                                                  // GMRES: true residual norm after a cycle
    SD_PROV = 13,  // GMRES: norm of the last once-orthogonalised vector (its column's provisional subdiagonal)
    SD_SCALARS = 16
};

struct GLayout {
    int m;
    int H, cs, sn, g, y, h1, h2, ds, total;  // ds: the sums of a Gram-Schmidt dot pass
    explicit GLayout(int m_ = 0) : m(m_) {
        H = SD_SCALARS;
        cs = H + (m + 1) * m;
        sn = cs + m;
        g = sn + m;
        y = g + m + 1;
        h1 = y + m;
        h2 = h1 + kMaxRestart;
        ds = h2 + kMaxRestart;
        total = ds + kDSums;
    }
    __host__ __device__ int Hij(int i, int j) const { return H + j * (m + 1) + i; }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sum acc[0..nv) over the workgroup; the totals land in tot[0..nv) (shared).
template <int NV>
__device__ __forceinline__ void block_sum(const double (&acc)[NV], int nv, double *red, double *tot) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        if (k < nv) {
            double v = wave_sum(acc[k]);
            if (lane == 0) red[wid * NV + k] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        int k = threadIdx.x;
        tot[k] = ((red[k] + red[NV + k]) + red[2 * NV + k]) + red[3 * NV + k];
    }
    __syncthreads();
}

// Generic fused pass: every row i runs op.row(i, acc) (which may also update
// vectors) and each workgroup writes its NV partial sums; k_pass_finish (one
// workgroup, launched right after) adds them in a fixed order and calls
// op.finish(totals) on one thread. Two launches instead of a last-workgroup
// handshake: a device-scope fence and counter per workgroup costs about 20 ns
// each, serialised over the grid.
template <int NV, class Op>
__global__ __launch_bounds__(RB) void k_pass(int64_t n, Op op, int nv, double *part, const int32_t *skip) {
    if (skip && *skip) return;
    __shared__ double red[4 * NV];
    __shared__ double tot[NV];
    __shared__ double sh[kMaxRestart + 1];
    op.init(sh);
    __syncthreads();
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * RB;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += stride) op.row(i, acc, sh);
    block_sum<NV>(acc, nv, red, tot);
    if (threadIdx.x < nv) part[(size_t)blockIdx.x * NV + threadIdx.x] = tot[threadIdx.x];
}

template <int NV, class Op>
__global__ __launch_bounds__(RB) void k_pass_finish(Op op, int nv, const double *part, int nblocks,
                                                    const int32_t *skip) {
    if (skip && *skip) return;
    __shared__ double red[4 * NV];
    __shared__ double tot[NV];
    // all partials of this thread loaded at once from in-bounds addresses, then added in order
    constexpr int NR = kMaxRedBlocks / RB;
    double v[NR][NV];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int b = threadIdx.x + r * RB;
#pragma unroll
        for (int k = 0; k < NV; ++k) v[r][k] = part[(size_t)(b < nblocks ? b : 0) * NV + k];
    }
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        acc[k] = 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (threadIdx.x + r * RB < nblocks && k < nv) acc[k] += v[r][k];
    }
    block_sum<NV>(acc, nv, red, tot);
    if (threadIdx.x == 0) op.finish(tot);
}

__device__ __forceinline__ void mirror(int32_t *hostflags, int idx, int32_t v) {
    if (hostflags) __hip_atomic_store(hostflags + idx, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

struct NoInit {
    __device__ void init(double *) const {}
};

// ---------------------------------------------------------------- ops

// *out = ||a||_2 (Eq. (6))
template <class T>
struct OpNorm : NoInit {
    const T *a;
    double *out;
    __device__ void row(int64_t i, double (&acc)[1], double *) const {
        double v = a[i];
        acc[0] += v * v;
    }
    __device__ void finish(const double *t) const { *out = sqrt(t[0]); }
};

// GMRES cycle start: beta = ||r||, g = beta e1, flags cleared; done if beta <= tol.
struct OpCycleStart : NoInit {
    const double *r;
    double *sd;
    int32_t *si, *hf;
    GLayout L;
    __device__ void row(int64_t i, double (&acc)[1], double *) const { acc[0] += r[i] * r[i]; }
    __device__ void finish(const double *t) const {
        double beta = sqrt(t[0]);
        sd[SD_BETA] = beta;
        sd[SD_RES] = beta;
        sd[L.g] = beta;
        for (int k = 1; k <= L.m; ++k) sd[L.g + k] = 0.0;
        int done = !(beta > sd[SD_TOL]);
        si[SI_DONE] = done;
        si[SI_JDONE] = 0;
        mirror(hf, SI_DONE, done);
        mirror(hf, SI_JDONE, 0);
    }
};

// Givens step of column j by a workgroup: H(:, j) = h1 + h2, h_{j+1,j} = hn, the
// earlier rotations applied to the column, a new rotation zeroing h_{j+1,j}, g
// updated, and the convergence test |g_{j+1}| <= tol (or hn == 0). The column and
// the rotations are read in parallel into LDS; one thread applies the rotations.
__device__ void givens_col(int j, double hn, const double *src, double *sd, int32_t *si, int32_t *hf,
                           const GLayout &L) {
    __shared__ double col[kMaxRestart + 1];
    __shared__ double rcs[kMaxRestart], rsn[kMaxRestart];
    const int t = threadIdx.x;
    if (t <= j) col[t] = src[t];
    if (t < j) {
        rcs[t] = sd[L.cs + t];
        rsn[t] = sd[L.sn + t];
    }
    __syncthreads();
    if (t == 0) {
        sd[SD_HNEXT] = hn;
        double a = col[0];  // entry k of the column, rotated by rotations 0..k-1
        for (int k = 0; k < j; ++k) {
            const double c = col[k + 1], cs = rcs[k], sn = rsn[k];
            col[k] = cs * a + sn * c;
            a = -sn * a + cs * c;
        }
        const double c = hn;
        const double rr = hypot(a, c);
        double cs = 1.0, sn = 0.0;
        if (c != 0.0) {
            cs = a / rr;
            sn = c / rr;
        }
        sd[L.cs + j] = cs;
        sd[L.sn + j] = sn;
        col[j] = cs * a + sn * c;
        const double gj = sd[L.g + j];
        sd[L.g + j + 1] = -sn * gj;
        sd[L.g + j] = cs * gj;
        const double res = fabs(sd[L.g + j + 1]);
        sd[SD_RES] = res;
        si[SI_JDONE] = j + 1;
        mirror(hf, SI_JDONE, j + 1);
        if (!(res > sd[SD_TOL]) || hn == 0.0 || !isfinite(res)) {
            si[SI_DONE] = 1;
            mirror(hf, SI_DONE, 1);
        }
    }
    __syncthreads();
    if (t <= j) sd[L.Hij(t, j)] = col[t];
}

// The same with the column h1 + h2 (the two Gram-Schmidt passes' coefficients).
__device__ void givens_block(int j, double hn, double *sd, int32_t *si, int32_t *hf, const GLayout &L) {
    __shared__ double sum[kMaxRestart + 1];
    if ((int)threadIdx.x <= j) sum[threadIdx.x] = sd[L.h1 + threadIdx.x] + sd[L.h2 + threadIdx.x];
    __syncthreads();
    givens_col(j, hn, sum, sd, si, hf, L);
}

// Element i of a vector; NT: a non-temporal (streaming) load.
template <class VT, bool NT>
__device__ __forceinline__ VT load_elem(const VT *p, int64_t i) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p + i);
    else
        return p[i];
}

// Sums of NS values over the 64 lanes of a wavefront at once: each butterfly
// step halves the number of values a lane holds (the lanes with the step's bit
// set keep the upper half, added to their partner's), then the lanes that share
// an index finish with a plain butterfly. Returns the sum with index cgs_sum_index(lane); every sum is
// added in a fixed order.
template <int NS>
constexpr int log2_of() {
    return NS <= 1 ? 0 : 1 + log2_of<NS / 2>();
}

template <int NS>
__device__ __forceinline__ double multi_wave_sum(double (&v)[NS], int lane) {
    constexpr int LG = log2_of<NS>();
#pragma unroll
    for (int st = 0; st < LG; ++st) {
        const int h = NS >> (st + 1), o = 32 >> st;
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < NS / 2; ++i) {
            if (i < h) {
                // both halves cross, then each lane keeps the sum of its half (a
                // select between two values, not between two array elements, so
                // that the array stays in registers)
                const double lo = v[i], hi = v[i + h];
                const double rlo = __shfl_xor(lo, o), rhi = __shfl_xor(hi, o);
                v[i] = up ? hi + rhi : lo + rlo;
            }
        }
    }
    double x = v[0];
#pragma unroll
    for (int st = LG; st < 6; ++st) x += __shfl_xor(x, 32 >> st);
    return x;
}

template <int NS>
__device__ __forceinline__ int cgs_sum_index(int lane) {
    int idx = 0;
#pragma unroll
    for (int st = 0; st < log2_of<NS>(); ++st)
        if (lane & (32 >> st)) idx += NS >> (st + 1);
    return idx;
}

// Classical Gram-Schmidt passes over the basis V (vectors of type VT, FP64 sums):
//   MODE 1: hout[k] = <V_k, w>                                  k < nv
//   MODE 2: w -= V hin;  hout[k] = <V_k, w>
//   MODE 3: w -= V hin;  ||w||^2
// for nv <= NB basis vectors. Every wavefront works alone (no barrier in its
// loop) on steps of U = 32 / NB chunks of 64 rows (one element per vector, chunk
// and lane), so that a pass over few vectors keeps as many loads in flight per
// wavefront as one over many. Steps are dealt to the grid's wavefronts
// round-robin; each keeps its sums in registers, and the workgroup adds its 4
// wavefronts' sums in a fixed order (deterministic). The grid's per-workgroup sums
// go to part[k * gridDim.x + block].
template <class VT, int MODE, int NB>
__global__ __launch_bounds__(RB) void k_cgs(int64_t n, const VT *__restrict__ V, int64_t ldv, VT *w, int nv,
                                            const double *__restrict__ hin, double *part, const int32_t *skip) {
    constexpr int U = kMaxRestart / NB;
    constexpr int64_t TR = 64 * U;          // rows per wavefront step
    constexpr int NS = MODE == 3 ? 1 : NB;  // sums per wavefront
    if (skip && *skip) return;
    __shared__ double red[4][NS];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    double acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0.0;
    // Streaming (non-temporal) loads when the basis may hold more than 16 vectors
    // (more than the memory-side cache holds at 128^3), and always for an FP32 basis;
    // FP64 passes over a smaller basis read part of it from that cache in passes 2
    // and 3 instead (measured).
    constexpr bool NT = NB == kMaxRestart || sizeof(VT) == 4;
    const int64_t nsteps = (n + TR - 1) / TR;
    for (int64_t t = (int64_t)blockIdx.x * 4 + q; t < nsteps; t += (int64_t)gridDim.x * 4) {
        VT vk[U][NB];
        VT wv[U];
        double wi[U];
        // A step inside the vectors (uniform over the wavefront) loads without per-lane
        // bounds checks: one straight run of loads, all in flight before the first is
        // used (per-lane checks become branches, and the compiler then waits for each
        // load inside its branch). Rows past n read zero.
        const bool inside = (t + 1) * TR <= n;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = t * TR + 64 * u + lane;
            if (inside) {
                wv[u] = load_elem<VT, NT>(w, i);
#pragma unroll
                for (int k = 0; k < NB; ++k) vk[u][k] = k < nv ? load_elem<VT, NT>(V + k * ldv, i) : (VT)0;
            } else {
                wv[u] = i < n ? load_elem<VT, NT>(w, i) : (VT)0;
#pragma unroll
                for (int k = 0; k < NB; ++k) vk[u][k] = k < nv && i < n ? load_elem<VT, NT>(V + k * ldv, i) : (VT)0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) wi[u] = (double)wv[u];
        if constexpr (MODE != 1) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                double ps = 0.0;
#pragma unroll
                for (int k = 0; k < NB; ++k)
                    if (k < nv) ps += hin[k] * (double)vk[u][k];  // uniform: scalar loads
                wv[u] = (VT)(wi[u] - ps);  // w is stored (and used) in its own precision
                wi[u] = (double)wv[u];
                const int64_t i = t * TR + 64 * u + lane;
                if (i < n) w[i] = wv[u];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (MODE == 3) {
                acc[0] += wi[u] * wi[u];
            } else {
#pragma unroll
                for (int k = 0; k < NB; ++k) acc[k] += (double)vk[u][k] * wi[u];
            }
        }
    }
    const double v = multi_wave_sum<NS>(acc, lane);
    if ((lane & (64 / NS - 1)) == 0) red[q][cgs_sum_index<NS>(lane)] = v;
    __syncthreads();
    const int cnt = MODE == 3 ? 1 : nv;
    if ((int)threadIdx.x < cnt) {
        const int k = threadIdx.x;
        part[(size_t)k * gridDim.x + blockIdx.x] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

// The nblocks partial sums p[0..nblocks), added in a fixed order by one workgroup;
// every thread gets the total.
__device__ __forceinline__ double block_sum_fixed(const double *p, int nblocks) {
    constexpr int NR = kMaxRedBlocks / RB;  // partials per thread
    __shared__ double tot[RB / 64];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    double v[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int b = (int)threadIdx.x + RB * r;
        v[r] = b < nblocks ? p[b] : 0.0;
    }
    double a = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) a += v[r];
    a = wave_sum(a);
    if (lane == 0) tot[q] = a;
    __syncthreads();
    return ((tot[0] + tot[1]) + tot[2]) + tot[3];
}

// The grid's sums of a k_cgs pass 1 or 2: workgroup k of the finishing launch adds
// the nblocks partial sums of dot product k (contiguous) in a fixed order.
__global__ __launch_bounds__(RB) void k_cgs_finish(const double *part, int nblocks, double *hout,
                                                   const int32_t *skip) {
    if (skip && *skip) return;
    const double sum = block_sum_fixed(part + (size_t)blockIdx.x * nblocks, nblocks);
    if (threadIdx.x == 0) hout[blockIdx.x] = sum;
}

// After pass 3: every workgroup adds the norm's partial sums in the same fixed order
// (so all hold the same h_{j+1,j}); workgroup 0 takes the Givens step of column nv-1;
// then, when vnext is given, v_{j+1} = w / h_{j+1,j} (a grid-stride loop). One launch
// instead of a one-workgroup finish followed by the scaling launch.
template <class VT>
__global__ __launch_bounds__(RB) void k_finish_scale(int64_t n, const VT *__restrict__ w, VT *__restrict__ vnext,
                                                     const double *part, int nblocks, int nv, const int32_t *skip,
                                                     double *sd, int32_t *si, int32_t *hf, GLayout L) {
    if (skip && *skip) return;
    const double hn = sqrt(block_sum_fixed(part, nblocks));
    if (blockIdx.x == 0) givens_block(nv - 1, hn, sd, si, hf, L);
    if (!vnext) return;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB)
        vnext[i] = (VT)((double)w[i] / hn);
}

// ------------------------------------------------ Gram-Schmidt with delayed reorthogonalisation
// Classical Gram-Schmidt applied twice, with the second application to each vector
// lagged into the next Arnoldi step (delayed CGS2, Hernandez, Roman and Tomas 2007), so
// that a step reads the basis twice instead of three times. At step s the basis holds
// the final vectors V_0 .. V_{s-1} (nf = s of them) and u = V_s, orthogonalised once and
// scaled to unit norm. One dot pass gives a = V_f^T u, t = V_f^T w, c = u.u, d = u.w and
// e = w.w for w = A z_s, z_s = M^{-1} u. Then u' = (u - V_f a) / alpha, alpha^2 = c - a.a,
// is the final v_s; the previous column is completed for it (A z_{s-1} was expressed with
// u: its entries gain its subdiagonal times a, its subdiagonal is multiplied by alpha);
// w is orthogonalised once against [V_f, u'] with the coefficients t and
// h_ss = (d - a.t) / alpha, and its norm follows from Pythagoras, beta^2 = e - t.t - h_ss^2
// (w is orthogonalised a second time, against the final basis, in the next step). One
// update pass writes v_s = u' and v_{s+1} = (w - V_f (t - a h_ss / alpha) - u h_ss / alpha)
// / beta. The stored z_s = M^{-1} u keeps A Z = V H exact (as flexible GMRES does), so
// x = x0 + Z y is unchanged in kind. A cycle ends with a dot pass over u alone that
// completes the last column.

// Dot pass: per workgroup the 2 nf + 3 partial sums [a_0..a_{nf-1}, t_0.., c, d, e] at
// part[k * gridDim.x + block]; w == NULL (a cycle's tail): t, d, e are 0.
template <class VT, int NB>
__global__ __launch_bounds__(RB) void k_dgs_dots(int64_t n, const VT *__restrict__ V, int64_t ldv, int nf,
                                                 const VT *__restrict__ w, double *part, const int32_t *skip) {
    constexpr int U = kMaxRestart / NB;
    constexpr int64_t TR = 64 * U;
    if (skip && *skip) return;
    __shared__ double red[4][2 * NB + 4];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    double aa[NB], at[NB], sc[4];
#pragma unroll
    for (int k = 0; k < NB; ++k) aa[k] = at[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) sc[k] = 0.0;
    constexpr bool NT = NB == kMaxRestart || sizeof(VT) == 4;
    const VT *u = V + (int64_t)nf * ldv;
    const int64_t nsteps = (n + TR - 1) / TR;
    for (int64_t t = (int64_t)blockIdx.x * 4 + q; t < nsteps; t += (int64_t)gridDim.x * 4) {
        VT vk[U][NB];
        VT uv[U], wv[U];
        const bool inside = (t + 1) * TR <= n;
#pragma unroll
        for (int c = 0; c < U; ++c) {
            const int64_t i = t * TR + 64 * c + lane;
            const bool live = inside || i < n;
            uv[c] = live ? load_elem<VT, NT>(u, i) : (VT)0;
            wv[c] = live && w ? load_elem<VT, NT>(w, i) : (VT)0;
#pragma unroll
            for (int k = 0; k < NB; ++k) vk[c][k] = live && k < nf ? load_elem<VT, NT>(V + k * ldv, i) : (VT)0;
        }
#pragma unroll
        for (int c = 0; c < U; ++c) {
            const double ud = (double)uv[c], wd = (double)wv[c];
            sc[0] += ud * ud;
            sc[1] += ud * wd;
            sc[2] += wd * wd;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                aa[k] += (double)vk[c][k] * ud;
                at[k] += (double)vk[c][k] * wd;
            }
        }
    }
    const double va = multi_wave_sum<NB>(aa, lane);
    const double vt = multi_wave_sum<NB>(at, lane);
    const double vs = multi_wave_sum<4>(sc, lane);
    if ((lane & (64 / NB - 1)) == 0) {
        red[q][cgs_sum_index<NB>(lane)] = va;
        red[q][NB + cgs_sum_index<NB>(lane)] = vt;
    }
    if ((lane & 15) == 0) red[q][2 * NB + cgs_sum_index<4>(lane)] = vs;
    __syncthreads();
    const int cnt = 2 * nf + 3;
    if ((int)threadIdx.x < cnt) {
        const int k = threadIdx.x;
        const int src = k < nf ? k : k < 2 * nf ? NB + (k - nf) : 2 * NB + (k - 2 * nf);
        part[(size_t)k * gridDim.x + blockIdx.x] = ((red[0][src] + red[1][src]) + red[2][src]) + red[3][src];
    }
}

// Update pass of step s (nf = s), after the dot pass's sums were finished into sd[L.ds].
// Every workgroup first forms the step's scalars from those sums in the same order (so all
// agree); workgroup 0 also completes column s-1 (its Givens step and convergence test) and
// stores column s, provisional until the next step (a happy breakdown, beta = 0, completes
// it at once). Then v_s = u' and v_{s+1} are written in one pass over the rows.
// w == NULL: the cycle's tail (column s-1 only; no vector work).
template <class VT, int NB>
__global__ __launch_bounds__(RB) void k_dgs_update(int64_t n, VT *V, int64_t ldv, int nf, const VT *__restrict__ w,
                                                   const int32_t *skip, double *sd, int32_t *si, int32_t *hf,
                                                   GLayout L) {
    constexpr int U = kMaxRestart / NB;
    constexpr int64_t TR = 64 * U;
    if (skip && *skip) return;
    __shared__ double ca[NB], ct[NB], sv[4], col[kMaxRestart + 1];
    const double *ds = sd + L.ds;
    if (threadIdx.x == 0) {
        double alpha = 1.0;  // v_0 = r / ||r|| is final as it stands
        if (nf > 0) {
            double aa = 0.0;
            for (int k = 0; k < nf; ++k) aa += ds[k] * ds[k];
            alpha = sqrt(fmax(ds[2 * nf] - aa, 0.0));
            if (!(alpha > 0.0)) alpha = 1.0;  // u in the span of V_f: only after a breakdown the flags already stop
        }
        double h = 0.0, beta = 0.0;
        if (w) {
            double at = 0.0, tt = 0.0;
            for (int k = 0; k < nf; ++k) {
                at += ds[k] * ds[nf + k];
                tt += ds[nf + k] * ds[nf + k];
            }
            h = (ds[2 * nf + 1] - at) / alpha;
            beta = sqrt(fmax(ds[2 * nf + 2] - tt - h * h, 0.0));
        }
        sv[0] = alpha;
        sv[1] = h;
        sv[2] = beta;
    }
    __syncthreads();
    const double alpha = sv[0], h = sv[1], beta = sv[2];
    const double cu = h / alpha;
    if ((int)threadIdx.x < nf) {
        const int k = threadIdx.x;
        ca[k] = ds[k];
        ct[k] = ds[nf + k] - ds[k] * cu;
    }
    if (blockIdx.x == 0) {
        // column s - 1, complete now: entries += its provisional subdiagonal times a
        if (nf > 0) {
            const double hp = sd[SD_PROV];
            if ((int)threadIdx.x < nf) col[threadIdx.x] = sd[L.h2 + threadIdx.x] + hp * ds[threadIdx.x];
            __syncthreads();
            givens_col(nf - 1, hp * alpha, col, sd, si, hf, L);
        }
        __syncthreads();
        if (w && !si[SI_DONE]) {
            // column s, provisional: [t, h]; the subdiagonal beta is completed next step
            if ((int)threadIdx.x < nf) sd[L.h2 + threadIdx.x] = ds[nf + threadIdx.x];
            if (threadIdx.x == 0) {
                sd[L.h2 + nf] = h;
                sd[SD_PROV] = beta;
            }
            __syncthreads();
            if (beta == 0.0) {  // happy breakdown: nothing left to orthogonalise, the column is final
                if ((int)threadIdx.x <= nf) col[threadIdx.x] = sd[L.h2 + threadIdx.x];
                __syncthreads();
                givens_col(nf, 0.0, col, sd, si, hf, L);
            }
        }
    }
    __syncthreads();
    if (!w) return;
    const double bdiv = beta > 0.0 ? beta : 1.0;
    VT *const u = V + (int64_t)nf * ldv;
    VT *const vn = u + ldv;
    constexpr bool NT = NB == kMaxRestart || sizeof(VT) == 4;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t nsteps = (n + TR - 1) / TR;
    for (int64_t t = (int64_t)blockIdx.x * 4 + q; t < nsteps; t += (int64_t)gridDim.x * 4) {
        VT vk[U][NB];
        VT uv[U], wv[U];
        const bool inside = (t + 1) * TR <= n;
#pragma unroll
        for (int c = 0; c < U; ++c) {
            const int64_t i = t * TR + 64 * c + lane;
            const bool live = inside || i < n;
            uv[c] = live ? load_elem<VT, NT>(u, i) : (VT)0;
            wv[c] = live ? load_elem<VT, NT>(w, i) : (VT)0;
#pragma unroll
            for (int k = 0; k < NB; ++k) vk[c][k] = live && k < nf ? load_elem<VT, NT>(V + k * ldv, i) : (VT)0;
        }
#pragma unroll
        for (int c = 0; c < U; ++c) {
            double sa = 0.0, st = 0.0;
#pragma unroll
            for (int k = 0; k < NB; ++k)
                if (k < nf) {
                    sa += (double)vk[c][k] * ca[k];
                    st += (double)vk[c][k] * ct[k];
                }
            const int64_t i = t * TR + 64 * c + lane;
            if (i < n) {
                const double ud = (double)uv[c];
                if (nf > 0) u[i] = (VT)((ud - sa) / alpha);
                vn[i] = (VT)(((double)wv[c] - st - ud * cu) / bdiv);
            }
        }
    }
}

template <class VT>
void launch_dgs(unsigned gd, unsigned gu, int64_t n, VT *V, int64_t ldv, int nf, const VT *w, double *part,
                const int32_t *skip, double *sd, int32_t *si, int32_t *hf, const GLayout &L, hipStream_t s) {
    auto go = [&](auto nb) {
        constexpr int NB = decltype(nb)::value;
        k_dgs_dots<VT, NB><<<gd, RB, 0, s>>>(n, V, ldv, nf, w, part, skip);
        HEC_CHECK_LAUNCH();
        k_cgs_finish<<<2 * nf + 3, RB, 0, s>>>(part, gd, sd + L.ds, skip);
        HEC_CHECK_LAUNCH();
        k_dgs_update<VT, NB><<<w ? gu : 1u, RB, 0, s>>>(n, V, ldv, nf, w, skip, sd, si, hf, L);
        HEC_CHECK_LAUNCH();
    };
    if (nf <= 4)
        go(std::integral_constant<int, 4>());
    else if (nf <= 8)
        go(std::integral_constant<int, 8>());
    else if (nf <= 16)
        go(std::integral_constant<int, 16>());
    else
        go(std::integral_constant<int, 32>());
}

// A Gram-Schmidt pass with the smallest vector bound NB >= nv.
template <class VT, int MODE>
void launch_cgs(unsigned g, int64_t n, const VT *V, int64_t ldv, VT *w, int nv, const double *hin, double *part,
                const int32_t *skip, hipStream_t s) {
    if (nv <= 4)
        k_cgs<VT, MODE, 4><<<g, RB, 0, s>>>(n, V, ldv, w, nv, hin, part, skip);
    else if (nv <= 8)
        k_cgs<VT, MODE, 8><<<g, RB, 0, s>>>(n, V, ldv, w, nv, hin, part, skip);
    else if (nv <= 16)
        k_cgs<VT, MODE, 16><<<g, RB, 0, s>>>(n, V, ldv, w, nv, hin, part, skip);
    else
        k_cgs<VT, MODE, 32><<<g, RB, 0, s>>>(n, V, ldv, w, nv, hin, part, skip);
    HEC_CHECK_LAUNCH();
}

// v = r / beta (start of a cycle)
template <class VT, class RT>
__global__ __launch_bounds__(256) void k_scale_start(int64_t n, const RT *r, VT *v, const double *sd) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    v[i] = (VT)((double)r[i] / sd[SD_BETA]);
}


// H y = g back substitution on the jdone x jdone upper triangle.
// One wavefront, column by column: lane t holds row t of the triangle (loaded
// once, in parallel) and g_t; y_i = g_i / H_ii is broadcast and every lane t < i
// subtracts H_ti y_i (g_i ends as g_i - sum over q > i of H_iq y_q, q descending).
__global__ __launch_bounds__(64) void k_backsolve(double *sd, const int32_t *si, GLayout L) {
    const int t = threadIdx.x;
    const int jd = si[SI_JDONE];
    double h[kMaxRestart];
#pragma unroll
    for (int q = 0; q < kMaxRestart; ++q) h[q] = (t < jd && q < jd && q >= t) ? sd[L.Hij(t, q)] : 0.0;
    double g = t < jd ? sd[L.g + t] : 0.0;
#pragma unroll
    for (int i = kMaxRestart - 1; i >= 0; --i) {
        if (i < jd) {
            const double yi = __shfl(g, i) / __shfl(h[i], i);
            if (t == i) sd[L.y + i] = yi;
            g -= h[i] * yi;  // rows t < i; h[i] is zero below the diagonal
        }
    }
}

// x += Z y (first jdone columns)
template <class VT>
__global__ __launch_bounds__(256) void k_update_x(int64_t n, const VT *Z, int64_t ldz, double *x,
                                                  const double *sd, const int32_t *si, GLayout L) {
    __shared__ double y[kMaxRestart];
    int jd = si[SI_JDONE];
    if ((int)threadIdx.x < jd) y[threadIdx.x] = sd[L.y + threadIdx.x];
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = x[i];
    for (int k = 0; k < jd; ++k) acc += y[k] * (double)Z[k * ldz + i];
    x[i] = acc;
}

template <class T>
__global__ __launch_bounds__(256) void k_fill(int64_t n, T *a, T v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

template <class S, class D>
__global__ __launch_bounds__(256) void k_copy(int64_t n, const S *a, D *b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (D)a[i];
}

// ---------------------------------------------------------------- BiCGSTAB ops (Alg. 4)

// r0 = r (shadow), rho = (r0, r) = ||r||^2, flags reset: start / restart.
struct OpBiStart : NoInit {
    const double *r;
    double *r0;
    double *sd;
    int32_t *si, *hf;
    __device__ void row(int64_t i, double (&acc)[1], double *) const {
        double v = r[i];
        r0[i] = v;
        acc[0] += v * v;
    }
    __device__ void finish(const double *t) const {
        sd[SD_RHO] = t[0];
        sd[SD_RNORM2] = t[0];
        int done = !(sqrt(t[0]) > sd[SD_TOL]);
        si[SI_DONE] = done;
        si[SI_STOP_S] = 0;
        si[SI_BREAK] = 0;
        si[SI_JDONE] = 0;  // loop passes in this run
        mirror(hf, SI_DONE, done);
        mirror(hf, SI_BREAK, 0);
        mirror(hf, SI_JDONE, 0);
        if (!done && (t[0] == 0.0 || !isfinite(t[0]))) {
            si[SI_DONE] = 1;
            si[SI_BREAK] = 1;
            mirror(hf, SI_DONE, 1);
            mirror(hf, SI_BREAK, 1);
        }
    }
};

// k == 1: p = r; else p = r + beta (p - omega v), beta = (rho/rho_prev)(alpha/omega)
__global__ __launch_bounds__(256) void k_bi_p(int64_t n, const double *r, double *p, const double *v,
                                              const double *sd, const int32_t *si, int first) {
    if (si[SI_DONE]) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (first) {
        p[i] = r[i];
    } else {
        double beta = (sd[SD_RHO] / sd[SD_RHO_PREV]) * (sd[SD_ALPHA] / sd[SD_OMEGA]);
        p[i] = r[i] + beta * (p[i] - sd[SD_OMEGA] * v[i]);
    }
}

// alpha = rho / (r0, v); breakdown if (r0, v) == 0
struct OpBiAlpha : NoInit {
    const double *r0, *v;
    double *sd;
    int32_t *si, *hf;
    __device__ void row(int64_t i, double (&acc)[1], double *) const { acc[0] += r0[i] * v[i]; }
    __device__ void finish(const double *t) const {
        if (t[0] == 0.0 || !isfinite(t[0])) {
            si[SI_DONE] = 1;
            si[SI_BREAK] = 1;
            mirror(hf, SI_DONE, 1);
            mirror(hf, SI_BREAK, 1);
            return;
        }
        sd[SD_ALPHA] = sd[SD_RHO] / t[0];
    }
};

// s = r - alpha v, ||s||; if ||s|| is small: x += alpha p* (k_bi_xs of the same pass) and stop.
struct OpBiS : NoInit {
    const double *r, *v, *ps;
    double *s, *x;
    double *sd;
    int32_t *si, *hf;
    __device__ void row(int64_t i, double (&acc)[1], double *) const {
        double si_ = r[i] - sd[SD_ALPHA] * v[i];
        s[i] = si_;
        acc[0] += si_ * si_;
    }
    __device__ void finish(const double *t) const {
        sd[SD_SNORM2] = t[0];
        const int32_t pass = si[SI_JDONE] + 1;
        si[SI_JDONE] = pass;
        mirror(hf, SI_JDONE, pass);
        if (!(sqrt(t[0]) > sd[SD_TOL])) {  // the pass that stops is recorded for k_bi_xs
            si[SI_STOP_S] = pass;
            si[SI_DONE] = 1;
            mirror(hf, SI_DONE, 1);
        }
    }
};

// early exit of Alg. 4: x += alpha p* when ||s|| was small enough in this pass (the
// pass number, counted from the run's start, is what OpBiS recorded; the rest of the
// pass is skipped by the done flag OpBiS set)
__global__ __launch_bounds__(256) void k_bi_xs(int64_t n, double *x, const double *ps, const double *sd,
                                               const int32_t *si, int32_t pass) {
    if (si[SI_STOP_S] != pass) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += sd[SD_ALPHA] * ps[i];
}

// (t, s) and (t, t) -> omega
struct OpBiOmega : NoInit {
    const double *t_, *s;
    double *sd;
    __device__ void row(int64_t i, double (&acc)[2], double *) const {
        double tv = t_[i];
        acc[0] += tv * s[i];
        acc[1] += tv * tv;
    }
    __device__ void finish(const double *t) const { sd[SD_OMEGA] = t[1] == 0.0 ? 0.0 : t[0] / t[1]; }
};

// x += alpha p* + omega s*; r = s - omega t; ||r||^2 and (r0, r) -> next rho
struct OpBiXR : NoInit {
    double *x, *r;
    const double *ps, *ss, *s, *t_, *r0;
    double *sd;
    int32_t *si, *hf;
    __device__ void row(int64_t i, double (&acc)[2], double *) const {
        double al = sd[SD_ALPHA], om = sd[SD_OMEGA];
        x[i] = x[i] + al * ps[i] + om * ss[i];
        double ri = s[i] - om * t_[i];
        r[i] = ri;
        acc[0] += ri * ri;
        acc[1] += r0[i] * ri;
    }
    __device__ void finish(const double *t) const {
        sd[SD_RNORM2] = t[0];
        sd[SD_RHO_PREV] = sd[SD_RHO];
        sd[SD_RHO] = t[1];
        if (!(sqrt(t[0]) > sd[SD_TOL]) || sd[SD_OMEGA] == 0.0) {
            si[SI_DONE] = 1;
            mirror(hf, SI_DONE, 1);
        } else if (t[1] == 0.0 || !isfinite(t[1])) {
            // Alg. 4 tests rho at the start of the next pass: a breakdown only if that pass runs
            si[SI_DONE] = 1;
            si[SI_BREAK] = 2;
            mirror(hf, SI_DONE, 1);
            mirror(hf, SI_BREAK, 2);
        }
    }
};

}  // namespace

// ---------------------------------------------------------------- workspace

// Mapped pinned flag blocks are recycled: freeing pinned host memory can
// synchronise the whole device, which would stall other streams' solves.
// ---------------------------------------------------------------- CG ops (Sec. 2.7, preconditioned CG)

// p = z, rho = (r, z), ||r||^2; start / restart. A non-positive rho (M not SPD) is a breakdown.
struct OpCgStart : NoInit {
    const double *r, *z;
    double *p;
    double *sd;
    int32_t *si, *hf;
    __device__ void row(int64_t i, double (&acc)[2], double *) const {
        const double zi = z[i], ri = r[i];
        p[i] = zi;
        acc[0] += ri * zi;
        acc[1] += ri * ri;
    }
    __device__ void finish(const double *t) const {
        sd[SD_RHO] = t[0];
        sd[SD_RNORM2] = t[1];
        int done = !(sqrt(t[1]) > sd[SD_TOL]);
        si[SI_DONE] = done;
        si[SI_BREAK] = 0;
        si[SI_JDONE] = 0;  // iterations in this run
        mirror(hf, SI_DONE, done);
        mirror(hf, SI_BREAK, 0);
        mirror(hf, SI_JDONE, 0);
        if (!done && !(t[0] > 0.0 && isfinite(t[0]))) {
            si[SI_DONE] = 1;
            si[SI_BREAK] = 1;
            mirror(hf, SI_DONE, 1);
            mirror(hf, SI_BREAK, 1);
        }
    }
};

// alpha = rho / (p, q); (p, q) <= 0 is a breakdown (A not SPD)
struct OpCgAlpha : NoInit {
    const double *p, *q;
    double *sd;
    int32_t *si, *hf;
    __device__ void row(int64_t i, double (&acc)[1], double *) const { acc[0] += p[i] * q[i]; }
    __device__ void finish(const double *t) const {
        if (!(t[0] > 0.0 && isfinite(t[0]))) {
            si[SI_DONE] = 1;
            si[SI_BREAK] = 1;
            mirror(hf, SI_DONE, 1);
            mirror(hf, SI_BREAK, 1);
            return;
        }
        sd[SD_ALPHA] = sd[SD_RHO] / t[0];
    }
};

// x += alpha p, r -= alpha q, ||r||^2: stop when ||r|| <= tol
struct OpCgUpdate : NoInit {
    const double *p, *q;
    double *x, *r;
    double *sd;
    int32_t *si, *hf;
    __device__ void row(int64_t i, double (&acc)[1], double *) const {
        const double a = sd[SD_ALPHA];
        x[i] = x[i] + a * p[i];
        const double ri = r[i] - a * q[i];
        r[i] = ri;
        acc[0] += ri * ri;
    }
    __device__ void finish(const double *t) const {
        sd[SD_RNORM2] = t[0];
        si[SI_JDONE] += 1;
        mirror(hf, SI_JDONE, si[SI_JDONE]);
        if (!(sqrt(t[0]) > sd[SD_TOL]) || !isfinite(t[0])) {
            si[SI_DONE] = 1;
            mirror(hf, SI_DONE, 1);
        }
    }
};

// rho' = (r, z), beta = rho' / rho, rho = rho'
struct OpCgRho : NoInit {
    const double *r, *z;
    double *sd;
    int32_t *si, *hf;
    __device__ void row(int64_t i, double (&acc)[1], double *) const { acc[0] += r[i] * z[i]; }
    __device__ void finish(const double *t) const {
        if (!(t[0] > 0.0 && isfinite(t[0]))) {
            si[SI_DONE] = 1;
            si[SI_BREAK] = 1;
            mirror(hf, SI_DONE, 1);
            mirror(hf, SI_BREAK, 1);
            return;
        }
        sd[SD_CGBETA] = t[0] / sd[SD_RHO];
        sd[SD_RHO] = t[0];
    }
};

// p = z + beta p
__global__ __launch_bounds__(256) void k_cg_p(int64_t n, const double *z, double *p, const double *sd,
                                              const int32_t *si) {
    if (si[SI_DONE]) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = z[i] + sd[SD_CGBETA] * p[i];
}

static std::mutex g_flag_mu;
static std::vector<int32_t *> g_flag_pool;

// A pooled block of mapped pinned memory: the SI_COUNT flags at offset 0, then at
// kScalarsOffset bytes the host copy of the SD_SCALARS scalars (one read per GMRES
// cycle). Blocks are never freed, only recycled (freeing pinned host memory can
// synchronise the whole device).
constexpr size_t kScalarsOffset = 64;
constexpr size_t kFlagBlockBytes = kScalarsOffset + SD_SCALARS * sizeof(double);
static_assert(SI_COUNT * sizeof(int32_t) <= kScalarsOffset, "flags overlap the scalars");

static int32_t *take_flags() {
    {
        std::lock_guard<std::mutex> lk(g_flag_mu);
        if (!g_flag_pool.empty()) {
            int32_t *p = g_flag_pool.back();
            g_flag_pool.pop_back();
            return p;
        }
    }
    int32_t *p = nullptr;
    HEC_HIP(hipHostMalloc((void **)&p, kFlagBlockBytes, hipHostMallocMapped));
    return p;
}

static void give_flags(int32_t *p) {
    std::lock_guard<std::mutex> lk(g_flag_mu);
    g_flag_pool.push_back(p);
}

struct KrylovWS {
    int64_t n = 0, ldv = 0;
    int m = 0;
    int nred = 1;
    bool mixed = false, bicg = false;
    DevBuf<double> V, Z;         // FP64 basis (m+1) x ldv, preconditioned basis m x ldv
    DevBuf<float> V32, Z32;      // mixed inner basis
    DevBuf<double> w, r, v6;     // w, r, and 6 more vectors for BiCGSTAB
    DevBuf<float> w32;
    DevBuf<double> sd;           // scalars + Hessenberg
    DevBuf<int32_t> si;
    DevBuf<double> part;         // partial sums, nred x kMaxRestart
    int32_t *hflags = nullptr;   // mapped pinned mirror of si (NULL: none; flags are copied to hsi)
    int32_t *dflags = nullptr;   // its device address
    double *hsd = nullptr;       // host copy of the scalars: in the pooled pinned block, or hsd_plain
    int32_t hsi[SI_COUNT] = {};  // host copy of si when there are no mapped flags
    double hsd_plain[SD_SCALARS] = {};
    std::vector<hipEvent_t> ev;
    ~KrylovWS() {
        for (auto e : ev) (void)hipEventDestroy(e);
        if (hflags) give_flags(hflags);
    }
};

void KrylovWSDeleter::operator()(KrylovWS *w) const { delete w; }

static KrylovWS &get_ws(hec_matrix_s &A, int m, bool mixed, bool bicg, hipStream_t s) {
    auto *w = A.ws.get();
    bool ok = w && w->m >= m && (!mixed || w->mixed) && (!bicg || w->bicg);
    if (ok) return *w;
    int mm = std::max(m, w ? w->m : 0);
    bool mx = mixed || (w && w->mixed);
    bool bc = bicg || (w && w->bicg);
    A.ws.reset();
    OwnerScope own(&A.dev_bytes);  // the workspace counts towards the matrix's footprint
    auto nw = std::unique_ptr<KrylovWS, KrylovWSDeleter>(new KrylovWS());
    nw->n = A.n;
    nw->ldv = ((int64_t)A.n + 63) / 64 * 64 + HEC_BASIS_PAD;
    nw->m = mm;
    nw->mixed = mx;
    nw->bicg = bc;
    nw->nred = red_blocks(A.n);
    size_t ldv = nw->ldv;
    if (mm > 0) {
        nw->V.alloc((mm + 1) * ldv);
        nw->Z.alloc(mm * ldv);
        if (mx) {
            nw->V32.alloc((mm + 1) * ldv);
            nw->Z32.alloc(mm * ldv);
        }
    }
    nw->w.alloc(ldv);
    nw->r.alloc(ldv);
    if (mx) nw->w32.alloc(ldv);
    if (bc) nw->v6.alloc(6 * ldv);
    GLayout L(std::max(mm, 1));
    nw->sd.alloc(std::max(L.total, SD_SCALARS + 8));
    nw->si.alloc(SI_COUNT);
    nw->part.alloc((size_t)nw->nred * kDSums);
    HEC_HIP(hipMemsetAsync(nw->si.get(), 0, SI_COUNT * sizeof(int32_t), s));
    nw->hflags = take_flags();
    nw->hsd = (double *)((char *)nw->hflags + kScalarsOffset);
    std::memset(nw->hflags, 0, kFlagBlockBytes);
    HEC_HIP(hipHostGetDevicePointer((void **)&nw->dflags, nw->hflags, 0));
    nw->ev.resize(kMaxRestart + 2);
    for (auto &e : nw->ev) HEC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HEC_HIP(hipStreamSynchronize(s));
    A.ws = std::move(nw);
    return *A.ws;
}

template <int NV, class Op>
static void launch_pass(KrylovWS &ws, int64_t n, const Op &op, int nv, hipStream_t s, const int32_t *skip) {
    k_pass<NV, Op><<<ws.nred, RB, 0, s>>>(n, op, nv, ws.part.get(), skip);
    HEC_CHECK_LAUNCH();
    k_pass_finish<NV, Op><<<1, RB, 0, s>>>(op, nv, ws.part.get(), ws.nred, skip);
    HEC_CHECK_LAUNCH();
}

static inline volatile int32_t *hf(KrylovWS &ws) { return (volatile int32_t *)ws.hflags; }

// One GMRES cycle on the basis of type VT (double, or float for the mixed
// inner solve), with r (FP64) holding the cycle's starting residual and
// sd[SD_TOL] the absolute target. Returns the Arnoldi steps taken; x += Z y.
template <class VT>
static int gmres_cycle(hec_matrix_s &A, hec_levels_s &lv, KrylovWS &ws, int mcyc, int m, double *x,
                       hipStream_t s, bool sync_end = true) {
    const int64_t n = A.n, ldv = ws.ldv;
    VT *V, *Z, *w;
    if constexpr (sizeof(VT) == 8) {
        V = (VT *)ws.V.get();
        Z = (VT *)ws.Z.get();
        w = (VT *)ws.w.get();
    } else {
        V = (VT *)ws.V32.get();
        Z = (VT *)ws.Z32.get();
        w = (VT *)ws.w32.get();
    }
    GLayout L(m);
    double *sd = ws.sd.get();
    int32_t *si = ws.si.get();
    const int32_t *done = si + SI_DONE;
    // beta = ||r||, g = beta e1
    OpCycleStart st{{}, ws.r.get(), sd, si, ws.dflags, L};
    launch_pass<1>(ws, n, st, 1, s, nullptr);
    k_scale_start<VT, double><<<ceil_div(n, 256), 256, 0, s>>>(n, ws.r.get(), V, sd);
    HEC_CHECK_LAUNCH();
    // no wait here: if the start is already converged, the queued steps return at entry
    // (the device's done flag) and the cycle adds no columns to x
    if constexpr (sizeof(VT) == 8) {
        // FP64 basis: delayed reorthogonalisation, two passes over the basis per step
        const unsigned gd = ws.nred;
        const unsigned gu = (unsigned)std::min<int64_t>(ceil_div(n, (int64_t)RB * 8), kMaxRedBlocks);
        for (int j = 0; j <= mcyc; ++j) {
            // look two iterations behind, every other iteration: stop issuing work once the
            // device is done. An event record costs the stream about 6 us (it waits for the
            // previous kernel and flushes to system scope), so only odd steps record one.
            if (j >= 3 && (j & 1) && ws.hflags) {  // (without mapped flags every step is queued)
                HEC_HIP(hipEventSynchronize(ws.ev[j - 1]));
                if (hf(ws)[SI_DONE]) break;
            }
            // step j: z_j = M^{-1} v_j, w = A z_j, then the two Gram-Schmidt passes (delayed
            // reorthogonalisation); j == mcyc: only the pass that completes the last column
            const bool tail = j == mcyc;
            if (!tail) {
                VT *vj = V + j * ldv, *zj = Z + j * ldv;
                trsv_launch<VT>(lv, HEC_LU, vj, zj, s, done);
                spmv_launch<VT, VT, VT>(A, 1.0, zj, 0.0, w, w, s, done);
            }
            launch_dgs<VT>(gd, gu, n, V, ldv, j, tail ? nullptr : w, ws.part.get(), done, sd, si, ws.dflags, L, s);
            if ((j & 1) && ws.hflags) HEC_HIP(hipEventRecord(ws.ev[j + 1], s));
        }
    } else {
        // FP32 basis: classical Gram-Schmidt twice in each step (three passes: the
        // delayed form's fused dot pass keeps twice the FP64 accumulators of a pass
        // here, and on FP32 data it ran 5x slower than these: 189 against 38 us)
        for (int j = 0; j < mcyc; ++j) {
            if (j >= 3 && (j & 1) && ws.hflags) {
                HEC_HIP(hipEventSynchronize(ws.ev[j - 1]));
                if (hf(ws)[SI_DONE]) break;
            }
            VT *vj = V + j * ldv, *zj = Z + j * ldv;
            trsv_launch<VT>(lv, HEC_LU, vj, zj, s, done);
            spmv_launch<VT, VT, VT>(A, 1.0, zj, 0.0, w, w, s, done);
            const int nv = j + 1;
            const unsigned g = ws.nred;
            double *part = ws.part.get();
            launch_cgs<VT, 1>(g, n, V, ldv, w, nv, nullptr, part, done, s);
            k_cgs_finish<<<nv, RB, 0, s>>>(part, g, sd + L.h1, done);
            HEC_CHECK_LAUNCH();
            launch_cgs<VT, 2>(g, n, V, ldv, w, nv, sd + L.h1, part, done, s);
            k_cgs_finish<<<nv, RB, 0, s>>>(part, g, sd + L.h2, done);
            HEC_CHECK_LAUNCH();
            launch_cgs<VT, 3>(g, n, V, ldv, w, nv, sd + L.h2, part, done, s);
            {
                VT *vnext = j + 1 < mcyc ? V + (j + 1) * ldv : nullptr;  // the cycle's last step scales nothing
                const unsigned gs =
                    vnext ? (unsigned)std::min<int64_t>(ceil_div(n, (int64_t)RB * 8), kMaxRedBlocks) : 1u;
                k_finish_scale<VT><<<gs, RB, 0, s>>>(n, w, vnext, part, g, nv, done, sd, si, ws.dflags, L);
                HEC_CHECK_LAUNCH();
            }
            if ((j & 1) && ws.hflags) HEC_HIP(hipEventRecord(ws.ev[j + 1], s));
        }
    }
    k_backsolve<<<1, 64, 0, s>>>(sd, si, L);
    HEC_CHECK_LAUNCH();
    k_update_x<VT><<<ceil_div(n, 256), 256, 0, s>>>(n, Z, ldv, x, sd, si, L);
    HEC_CHECK_LAUNCH();
    if (!sync_end) return -1;  // the caller reads the step count after its own synchronisation
    HEC_HIP(hipStreamSynchronize(s));
    return hf(ws)[SI_JDONE];
}

static double read_scalar(KrylovWS &ws, int idx, hipStream_t s) {
    double v = 0.0;
    HEC_HIP(hipMemcpyAsync(&v, ws.sd.get() + idx, sizeof(double), hipMemcpyDeviceToHost, s));
    HEC_HIP(hipStreamSynchronize(s));
    return v;
}

static void set_scalar(KrylovWS &ws, int idx, double v, hipStream_t s) {
    HEC_HIP(hipMemcpyAsync(ws.sd.get() + idx, &v, sizeof(double), hipMemcpyHostToDevice, s));
    HEC_HIP(hipStreamSynchronize(s));
}

__global__ void k_set_scalar(double *p, double v) {
    if (threadIdx.x == 0) *p = v;
}

// The same without a host round trip: the value travels as a kernel argument.
static void set_scalar_async(KrylovWS &ws, int idx, double v, hipStream_t s) {
    k_set_scalar<<<1, 64, 0, s>>>(ws.sd.get() + idx, v);
    HEC_CHECK_LAUNCH();
}

// ||b - A x|| for the FP64 matrix into ws.r; returns the norm
static double true_residual(hec_matrix_s &A, KrylovWS &ws, const double *b, const double *x, hipStream_t s) {
    spmv_launch<double, double, double>(A, -1.0, x, 1.0, b, ws.r.get(), s);
    OpNorm<double> op{{}, ws.r.get(), ws.sd.get() + SD_RES};
    launch_pass<1>(ws, A.n, op, 1, s, nullptr);
    return read_scalar(ws, SD_RES, s);
}

static double vec_norm(KrylovWS &ws, int64_t n, const double *v, hipStream_t s) {
    OpNorm<double> op{{}, v, ws.sd.get() + SD_BNORM};
    launch_pass<1>(ws, n, op, 1, s, nullptr);
    return read_scalar(ws, SD_BNORM, s);
}

static void check_solve_args(hec_matrix A, hec_ilu M, hec_levels lv, const double *b, double *x,
                             const hec_solve_opts *o) {
    if (!A || !M || !lv || !o) fail(HEC_ERR_INVALID_ARG, "null handle or options");
    if (A->n != M->n_sys || A->n != lv->n || M->n != lv->nf)
        fail(HEC_ERR_INVALID_ARG, "matrix, factor and levels differ in size");
    if (A->n > 0 && (!b || !x)) fail(HEC_ERR_INVALID_ARG, "b or x is NULL");
    if (o->maxit < 0) fail(HEC_ERR_INVALID_ARG, "maxit < 0");
    if (!(o->rtol > 0.0)) fail(HEC_ERR_INVALID_ARG, "rtol must be > 0");
    if (o->precision != 0 && o->precision != 1) fail(HEC_ERR_INVALID_ARG, "precision must be 0 or 1");
}

// The restarted GMRES driver on a prepared workspace: x0, the FP64 true residual, then
// cycles (FP64, or FP32 inner solves inside FP64 refinement) until the target or maxit.
static void gmres_run(hec_matrix_s &A, hec_levels_s &lv, KrylovWS &ws, const double *b, double *x,
                      const hec_solve_opts *o, hec_solve_info &inf, hipStream_t s) {
    const int64_t n = A.n;
    const bool mixed = o->precision == 1;
    const double bnorm = vec_norm(ws, n, b, s);
    if (bnorm == 0.0) {
        k_fill<double><<<ceil_div(n, 256), 256, 0, s>>>(n, x, 0.0);
        HEC_CHECK_LAUNCH();
        HEC_HIP(hipStreamSynchronize(s));
        return;
    }
    if (o->x0_zero) {
        k_fill<double><<<ceil_div(n, 256), 256, 0, s>>>(n, x, 0.0);
        HEC_CHECK_LAUNCH();
    }
    const double target = mixed && o->ir_rtol > 0.0 ? std::min(o->ir_rtol, o->rtol) : o->rtol;
    double res = true_residual(A, ws, b, x, s);
    int it = 0, cycles = 0;
    // mixed precision: a refinement that stalls (eight steps in a row without halving the
    // smallest true residual so far: the FP32 inner solves no longer resolve the
    // correction) gives up, and the solve starts again in FP64 from x = 0 (restarted FP64
    // cycles from the stalled iterate were measured far slower: its residual is left in
    // the components GMRES(m) converges worst, 3700 further steps against 627 from zero)
    bool fp64_tail = false;
    int stalls = 0;
    double res_mark = res;
    while (res / bnorm > target && it < o->maxit) {
        int mcyc = std::min(o->restart, o->maxit - it);
        if (!mixed || fp64_tail) {
            set_scalar_async(ws, SD_TOL, target * bnorm, s);
            gmres_cycle<double>(A, lv, ws, mcyc, o->restart, x, s, false);
        } else {
            // inner solve of A d = r in FP32 storage, one cycle, to inner_rtol
            double inner = o->inner_rtol > 0.0 ? o->inner_rtol : 1e-4;
            set_scalar_async(ws, SD_TOL, std::max(inner * res, 0.5 * target * bnorm), s);
            gmres_cycle<float>(A, lv, ws, mcyc, o->restart, x, s, false);
            inf.ir_steps++;
        }
        // the true residual after the cycle, then one copy of the scalars and one
        // synchronisation for the cycle's estimate, the true residual and the step count
        spmv_launch<double, double, double>(A, -1.0, x, 1.0, b, ws.r.get(), s);
        launch_pass<1>(ws, n, OpNorm<double>{{}, ws.r.get(), ws.sd.get() + SD_TRUE}, 1, s, nullptr);
        int jd;
        if (ws.hflags) {  // the step count is mirrored in the mapped flags
            HEC_HIP(hipMemcpyAsync(ws.hsd, ws.sd.get(), SD_SCALARS * sizeof(double), hipMemcpyDeviceToHost, s));
            HEC_HIP(hipStreamSynchronize(s));
            jd = hf(ws)[SI_JDONE];
        } else {  // plain copies into the workspace's host arrays
            HEC_HIP(hipMemcpyAsync(ws.hsd, ws.sd.get(), SD_SCALARS * sizeof(double), hipMemcpyDeviceToHost, s));
            HEC_HIP(hipMemcpyAsync(ws.hsi, ws.si.get(), SI_COUNT * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HEC_HIP(hipStreamSynchronize(s));
            jd = ws.hsi[SI_JDONE];
        }
        inf.rel_res_est = ws.hsd[SD_RES] / bnorm;
        res = ws.hsd[SD_TRUE];
        it += jd;
        cycles++;
        if (mixed && !fp64_tail) {
            if (res <= 0.5 * res_mark) {
                res_mark = res;
                stalls = 0;
            } else if (++stalls >= 8) {
                fp64_tail = true;
                k_fill<double><<<ceil_div(n, 256), 256, 0, s>>>(n, x, 0.0);
                HEC_CHECK_LAUNCH();
                res = true_residual(A, ws, b, x, s);  // r = b for the FP64 cycles that follow
                continue;
            }
        }
        if (jd == 0) break;  // no progress possible (breakdown at the start of a cycle)
    }
    inf.iterations = it;
    inf.restarts = std::max(0, cycles - 1);
    inf.rel_res_true = res / bnorm;
    check_levels(lv, s);  // a triangular-solve wait that gave up invalidates the iterate
    if (!(res / bnorm <= target)) fail(HEC_ERR_NOT_CONVERGED, "GMRES did not reach the tolerance");
}

// ---------------------------------------------------------------- workspace without allocation
// gmres_solve_noalloc keeps its workspace (basis, preconditioned basis, w, r,
// scalars, partial sums, flags) in this file-scope array instead of allocating it.
// In host code `scratch` only names the symbol: its device address, one per GPU,
// comes from hipGetSymbolAddress on the first call made with that device current.
constexpr int64_t kNoAllocLdv = HEC_NOALLOC_MAX_N + HEC_BASIS_PAD;  // widest basis vector (n rounded to 64)
constexpr int64_t kNoAllocSd = 2048;                                // scalars + Hessenberg (GLayout(32) needs 1265)
constexpr int64_t kNoAllocPart = 4096;                              // partial sums: nred * 68 (32 * 68 at most)
constexpr int64_t kNoAllocSi = 64;                                  // SI_COUNT int32 flags, in doubles
constexpr int64_t kNoAllocDoubles = (2 * kMaxRestart + 3) * kNoAllocLdv + kNoAllocSd + kNoAllocPart + kNoAllocSi;
static_assert(HEC_NOALLOC_MAX_N % 64 == 0, "the no-allocation bound keeps basis vectors 64-aligned");
static_assert(SI_COUNT * sizeof(int32_t) <= kNoAllocSi * sizeof(double), "flags fit");

static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up once per device).
static double *scratch_address() {
    int dev = 0;
    HEC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(HEC_ERR_INVALID_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HEC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(HEC_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = (double *)p;
    }
    return g_scratch_ptr[dev];
}

// A workspace of views into the scratch array (n <= HEC_NOALLOC_MAX_N, FP64 basis of
// m + 1 vectors): no mapped flags and no events, so the driver queues whole cycles and
// reads the flags and scalars by plain copies. The flags are cleared (with a fill
// kernel); everything else is written before it is read.
static void noalloc_workspace(KrylovWS &ws, int64_t n, int m, hipStream_t s) {
    double *base = scratch_address();
    ws.n = n;
    ws.ldv = (n + 63) / 64 * 64 + HEC_BASIS_PAD;
    ws.m = m;
    ws.nred = red_blocks(n);
    const int64_t ldv = ws.ldv;
    if (GLayout(m).total > kNoAllocSd || (int64_t)ws.nred * kDSums > kNoAllocPart || ldv > kNoAllocLdv)
        fail(HEC_ERR_INVALID_ARG, "system too large for the no-allocation scratch");
    double *q = base;
    ws.V.borrow(q, (size_t)(m + 1) * ldv);
    q += (m + 1) * ldv;
    ws.Z.borrow(q, (size_t)m * ldv);
    q += m * ldv;
    ws.w.borrow(q, ldv);
    q += ldv;
    ws.r.borrow(q, ldv);
    q = base + (2 * kMaxRestart + 3) * kNoAllocLdv;
    ws.sd.borrow(q, kNoAllocSd);
    q += kNoAllocSd;
    ws.part.borrow(q, kNoAllocPart);
    q += kNoAllocPart;
    ws.si.borrow((int32_t *)q, SI_COUNT);
    ws.hsd = ws.hsd_plain;
    k_fill<int32_t><<<1, 256, 0, s>>>(SI_COUNT, ws.si.get(), 0);
    HEC_CHECK_LAUNCH();
}

}  // namespace hec

using namespace hec;

extern "C" {

hec_status gmres_solve(hec_matrix A, hec_ilu M, hec_levels lv, const double *b, double *x,
                       const hec_solve_opts *o, hec_solve_info *info, void *stream) {
    hec_solve_info inf{};
    auto t0 = std::chrono::steady_clock::now();
    hec_status st = guarded([&] {
        check_solve_args(A, M, lv, b, x, o);
        if (o->restart < 1 || o->restart > kMaxRestart)
            fail(HEC_ERR_INVALID_ARG, "restart must be in [1, 32]");
        const bool mixed = o->precision == 1;
        if (mixed && (!A->has_f32 || !M->has_f32))
            fail(HEC_ERR_INVALID_ARG, "mixed precision needs HEC_KEEP_F32 on the matrix and the factor");
        hipStream_t s = as_stream(stream);
        StreamScope scope(s);
        const int64_t n = A->n;
        inf.status = HEC_OK;
        if (n == 0) return;
        KrylovWS &ws = get_ws(*A, o->restart, mixed, false, s);
        gmres_run(*A, *lv, ws, b, x, o, inf, s);
    });
    inf.status = st;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return st;
}

hec_status gmres_solve_noalloc(hec_matrix A, hec_ilu M, hec_levels lv, const double *b, double *x,
                               const hec_solve_opts *o, hec_solve_info *info, void *stream) {
    hec_solve_info inf{};
    auto t0 = std::chrono::steady_clock::now();
    hec_status st = guarded([&] {
        check_solve_args(A, M, lv, b, x, o);
        if (o->restart < 1 || o->restart > kMaxRestart)
            fail(HEC_ERR_INVALID_ARG, "restart must be in [1, 32]");
        if (o->precision != 0) fail(HEC_ERR_INVALID_ARG, "gmres_solve_noalloc runs in FP64 only (precision 0)");
        if (A->n > HEC_NOALLOC_MAX_N)
            fail(HEC_ERR_INVALID_ARG, "gmres_solve_noalloc: n = " + std::to_string(A->n) +
                                          " exceeds its static scratch (at most " +
                                          std::to_string(HEC_NOALLOC_MAX_N) + " rows)");
        hipStream_t s = as_stream(stream);
        const int64_t n = A->n;
        inf.status = HEC_OK;
        if (n == 0) return;
        KrylovWS ws;
        noalloc_workspace(ws, n, o->restart, s);
        gmres_run(*A, *lv, ws, b, x, o, inf, s);
    });
    inf.status = st;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return st;
}

hec_status bicgstab_solve(hec_matrix A, hec_ilu M, hec_levels lv, const double *b, double *x,
                          const hec_solve_opts *o, hec_solve_info *info, void *stream) {
    hec_solve_info inf{};
    auto t0 = std::chrono::steady_clock::now();
    hec_status st = guarded([&] {
        check_solve_args(A, M, lv, b, x, o);
        if (o->precision != 0) fail(HEC_ERR_INVALID_ARG, "BiCGSTAB runs in FP64 only");
        hipStream_t s = as_stream(stream);
        StreamScope scope(s);
        const int64_t n = A->n;
        if (n == 0) return;
        KrylovWS &ws = get_ws(*A, 0, false, true, s);
        const int64_t ldv = ws.ldv;
        double *r = ws.r.get(), *r0 = ws.v6.get(), *p = r0 + ldv, *ps = p + ldv, *v = ps + ldv, *sv = v + ldv,
               *ss = sv + ldv, *t = ws.w.get();
        double *sd = ws.sd.get();
        int32_t *si = ws.si.get();
        const double bnorm = vec_norm(ws, n, b, s);
        if (bnorm == 0.0) {
            k_fill<double><<<ceil_div(n, 256), 256, 0, s>>>(n, x, 0.0);
            HEC_CHECK_LAUNCH();
            HEC_HIP(hipStreamSynchronize(s));
            return;
        }
        if (o->x0_zero) {
            k_fill<double><<<ceil_div(n, 256), 256, 0, s>>>(n, x, 0.0);
            HEC_CHECK_LAUNCH();
        }
        set_scalar(ws, SD_TOL, o->rtol * bnorm, s);
        double res = true_residual(*A, ws, b, x, s);
        int it = 0, cycles = 0;  // a cycle starts from the current x with a new shadow residual
        bool broke = false;
        const unsigned g = ceil_div(n, 256);
        while (res / bnorm > o->rtol && it < o->maxit && cycles < 4) {
            ++cycles;
            OpBiStart bs{{}, r, r0, sd, si, ws.dflags};
            launch_pass<1>(ws, n, bs, 1, s, nullptr);
            HEC_HIP(hipStreamSynchronize(s));
            broke = false;
            if (!hf(ws)[SI_DONE]) {
                int k = 0;
                for (; it + k < o->maxit; ++k) {
                    if (k >= 3 && (k & 1)) {  // every other pass: wait for pass k-2, keep k-1 queued
                        HEC_HIP(hipEventSynchronize(ws.ev[1]));
                        if (hf(ws)[SI_DONE]) break;
                    }
                    const int32_t *done = si + SI_DONE;
                    k_bi_p<<<g, 256, 0, s>>>(n, r, p, v, sd, si, k == 0);
                    HEC_CHECK_LAUNCH();
                    trsv_launch<double>(*lv, HEC_LU, p, ps, s, done);
                    spmv_launch<double, double, double>(*A, 1.0, ps, 0.0, v, v, s, done);
                    launch_pass<1>(ws, n, OpBiAlpha{{}, r0, v, sd, si, ws.dflags}, 1, s, done);
                    launch_pass<1>(ws, n, OpBiS{{}, r, v, ps, sv, x, sd, si, ws.dflags}, 1, s, done);
                    k_bi_xs<<<g, 256, 0, s>>>(n, x, ps, sd, si, k + 1);
                    HEC_CHECK_LAUNCH();
                    trsv_launch<double>(*lv, HEC_LU, sv, ss, s, done);
                    spmv_launch<double, double, double>(*A, 1.0, ss, 0.0, t, t, s, done);
                    launch_pass<2>(ws, n, OpBiOmega{{}, t, sv, sd}, 2, s, done);
                    launch_pass<2>(ws, n, OpBiXR{{}, x, r, ps, ss, sv, t, r0, sd, si, ws.dflags}, 2, s, done);
                    if (k & 1) HEC_HIP(hipEventRecord(ws.ev[1], s));  // an event record costs ~6 us of stream time
                }
                HEC_HIP(hipStreamSynchronize(s));
                it += hf(ws)[SI_JDONE];
                // 1: (r0, v) or the cycle's first rho was zero; 2: the rho of the pass after the
                // last one was, which breaks down only if the iteration limit lets that pass run
                const int32_t bk = hf(ws)[SI_BREAK];
                broke = bk == 1 || (bk == 2 && it < o->maxit);
            }
            inf.rel_res_est = std::sqrt(std::min(read_scalar(ws, SD_RNORM2, s), read_scalar(ws, SD_SNORM2, s))) / bnorm;
            res = true_residual(*A, ws, b, x, s);
        }
        inf.iterations = it;
        inf.restarts = std::max(0, cycles - 1);
        inf.rel_res_true = res / bnorm;
        check_levels(*lv, s);
        if (!(res / bnorm <= o->rtol)) {
            if (broke) fail(HEC_ERR_BREAKDOWN, "BiCGSTAB breakdown (rho or (r0,v) == 0)");
            fail(HEC_ERR_NOT_CONVERGED, "BiCGSTAB did not reach the tolerance");
        }
    });
    inf.status = st;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return st;
}

hec_status cg_solve(hec_matrix A, hec_ilu M, hec_levels lv, const double *b, double *x, const hec_solve_opts *o,
                    hec_solve_info *info, void *stream) {
    hec_solve_info inf{};
    auto t0 = std::chrono::steady_clock::now();
    hec_status st = guarded([&] {
        check_solve_args(A, M, lv, b, x, o);
        if (o->precision != 0) fail(HEC_ERR_INVALID_ARG, "CG runs in FP64 only");
        hipStream_t s = as_stream(stream);
        StreamScope scope(s);
        const int64_t n = A->n;
        if (n == 0) return;
        KrylovWS &ws = get_ws(*A, 0, false, true, s);
        const int64_t ldv = ws.ldv;
        double *r = ws.r.get(), *z = ws.v6.get(), *p = z + ldv, *q = p + ldv;
        double *sd = ws.sd.get();
        int32_t *si = ws.si.get();
        const double bnorm = vec_norm(ws, n, b, s);
        if (bnorm == 0.0) {
            k_fill<double><<<ceil_div(n, 256), 256, 0, s>>>(n, x, 0.0);
            HEC_CHECK_LAUNCH();
            HEC_HIP(hipStreamSynchronize(s));
            return;
        }
        if (o->x0_zero) {
            k_fill<double><<<ceil_div(n, 256), 256, 0, s>>>(n, x, 0.0);
            HEC_CHECK_LAUNCH();
        }
        set_scalar(ws, SD_TOL, o->rtol * bnorm, s);
        double res = true_residual(*A, ws, b, x, s);  // r = b - A x
        int it = 0, restarts = 0;
        bool broke = false;
        const unsigned g = ceil_div(n, 256);
        while (res / bnorm > o->rtol && it < o->maxit && restarts <= 3) {
            trsv_launch<double>(*lv, HEC_LU, r, z, s, nullptr);
            launch_pass<2>(ws, n, OpCgStart{{}, r, z, p, sd, si, ws.dflags}, 2, s, nullptr);
            HEC_HIP(hipStreamSynchronize(s));
            broke = hf(ws)[SI_BREAK] != 0;
            if (!hf(ws)[SI_DONE]) {
                const int32_t *done = si + SI_DONE;
                for (int k = 0; it + k < o->maxit; ++k) {
                    if (k >= 3 && (k & 1)) {  // every other iteration: wait for k-2, keep k-1 queued
                        HEC_HIP(hipEventSynchronize(ws.ev[1]));
                        if (hf(ws)[SI_DONE]) break;
                    }
                    spmv_launch<double, double, double>(*A, 1.0, p, 0.0, q, q, s, done);
                    launch_pass<1>(ws, n, OpCgAlpha{{}, p, q, sd, si, ws.dflags}, 1, s, done);
                    launch_pass<1>(ws, n, OpCgUpdate{{}, p, q, x, r, sd, si, ws.dflags}, 1, s, done);
                    trsv_launch<double>(*lv, HEC_LU, r, z, s, done);
                    launch_pass<1>(ws, n, OpCgRho{{}, r, z, sd, si, ws.dflags}, 1, s, done);
                    k_cg_p<<<g, 256, 0, s>>>(n, z, p, sd, si);
                    HEC_CHECK_LAUNCH();
                    if (k & 1) HEC_HIP(hipEventRecord(ws.ev[1], s));  // an event record costs ~6 us of stream time
                }
                HEC_HIP(hipStreamSynchronize(s));
                it += hf(ws)[SI_JDONE];
                broke = hf(ws)[SI_BREAK] != 0;
            }
            inf.rel_res_est = std::sqrt(read_scalar(ws, SD_RNORM2, s)) / bnorm;
            res = true_residual(*A, ws, b, x, s);
            if (res / bnorm > o->rtol) {
                if (broke) break;
                ++restarts;
            }
        }
        inf.iterations = it;
        inf.restarts = restarts;
        inf.rel_res_true = res / bnorm;
        check_levels(*lv, s);
        if (!(res / bnorm <= o->rtol)) {
            if (broke) fail(HEC_ERR_BREAKDOWN, "CG breakdown ((r, z) or (p, A p) not positive)");
            fail(HEC_ERR_NOT_CONVERGED, "CG did not reach the tolerance");
        }
    });
    inf.status = st;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return st;
}

}  // extern "C"
