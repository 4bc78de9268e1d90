// HEC matrix: conversion from CSR (Sec. 2.1) and SpMV (Sec. 2.2, Alg. 1, Eq. (2)).
//
// Layout in HBM: the ELL slab is column-major (entry s of row i at s*ld + i,
// ld = n rounded up to 256), so a wavefront's load of slot s touches 64
// consecutive values: one 512-byte (FP64) or 256-byte (FP32/int32) segment.
// The remainder is plain CSR plus a list of the rows that have one; in the HYB
// layout (HEC_COO_REMAINDER) it is also kept as COO, the row of every entry.
#include <algorithm>
#include <cmath>
#include <memory>
#include <atomic>
#include <mutex>

#include "hec_internal.hpp"

namespace hec {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string &msg) { g_last_error = msg; }

hipStream_t &alloc_stream() {
    thread_local hipStream_t s = nullptr;
    return s;
}

int64_t *&alloc_owner() {
    thread_local int64_t *o = nullptr;
    return o;
}

namespace {
std::mutex g_alloc_mu;
Allocator g_alloc;  // alloc == NULL: hipMallocAsync / hipFreeAsync
// 2^26 polls: about 2 s for a wait on LDS, far longer for one on global memory; a
// legitimate wait lasts at most one solve (milliseconds)
constexpr uint32_t kDefaultSpin = 1u << 26;
std::atomic<uint32_t> g_spin{kDefaultSpin};
}  // namespace

uint32_t spin_limit() { return g_spin.load(std::memory_order_relaxed); }
std::atomic<bool> g_trsv_grid{true};
bool trsv_grid_enabled() { return g_trsv_grid.load(std::memory_order_relaxed); }

Allocator current_allocator() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

void *dev_alloc(size_t bytes, hipStream_t s, const Allocator &a) {
    void *p = nullptr;
    if (a.alloc) {
        p = a.alloc(a.ctx, bytes, (void *)s);
        if (!p) fail(HEC_ERR_NOMEM, "the allocator set by hec_set_allocator returned NULL for " +
                                        std::to_string(bytes) + " bytes");
        return p;
    }
    HEC_HIP(hipMallocAsync(&p, bytes, s));
    return p;
}

void dev_free(void *p, size_t bytes, hipStream_t s, const Allocator &a) {
    if (!p) return;
    if (a.alloc)
        a.free(a.ctx, p, bytes, (void *)s);
    else
        (void)hipFreeAsync(p, s);
}

// Keep freed stream-ordered memory in the device pool for reuse instead of
// returning it to the driver at every synchronisation.
void ensure_pool() {
    thread_local int done_dev = -1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev == done_dev) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    done_dev = dev;
}

void validate_csr(int32_t n, const int32_t *Ap, const int32_t *Aj, const double *Ax, int32_t ncols) {
    if (ncols < 0) ncols = n;
    if (n < 0) fail(HEC_ERR_INVALID_ARG, "n < 0");
    if (!Ap) fail(HEC_ERR_INVALID_ARG, "Ap is NULL");
    if (Ap[0] != 0) fail(HEC_ERR_INVALID_ARG, "Ap[0] != 0");
    for (int32_t i = 0; i < n; ++i)
        if (Ap[i + 1] < Ap[i]) fail(HEC_ERR_INVALID_ARG, "Ap is not non-decreasing at row " + std::to_string(i));
    if (Ap[n] > 0 && (!Aj || !Ax)) fail(HEC_ERR_INVALID_ARG, "Aj or Ax is NULL");
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t e = Ap[i]; e < Ap[i + 1]; ++e) {
            int32_t j = Aj[e];
            if (j < 0 || j >= ncols)
                fail(HEC_ERR_INVALID_ARG, "column index out of range in row " + std::to_string(i));
            if (e > Ap[i] && j <= Aj[e - 1])
                fail(HEC_ERR_INVALID_ARG, "columns not strictly ascending in row " + std::to_string(i));
        }
    }
}

// ------------------------------------------------------------------ conversion kernels

// One thread per slab row i < ld: writes the K slots of row i (coalesced across i).
__global__ __launch_bounds__(256) void k_hec_fill_ell(int32_t n, int32_t ncols, int32_t K, int32_t ld,
                                                      const int32_t *__restrict__ Ap,
                                                      const int32_t *__restrict__ Aj,
                                                      const double *__restrict__ Ax,
                                                      int32_t *__restrict__ ell_col,
                                                      double *__restrict__ ell_val,
                                                      float *__restrict__ ell_val32) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ld) return;
    int32_t a = 0, len = 0;
    if (i < n) {
        a = Ap[i];
        len = Ap[i + 1] - a;
    }
    for (int32_t s = 0; s < K; ++s) {
        size_t slot = (size_t)s * ld + i;
        int32_t c;
        double v;
        if (s < len) {
            c = Aj[a + s];
            v = Ax[a + s];
        } else {
            c = i < n && i < ncols ? i : 0;  // padding: any valid column, value 0
            v = 0.0;
        }
        ell_col[slot] = c;
        ell_val[slot] = v;
        if (ell_val32) ell_val32[slot] = (float)v;  // round to nearest even
    }
}

// One thread per row: copies entries K.. of row i to the remainder CSR.
__global__ __launch_bounds__(256) void k_hec_fill_rem(int32_t n, int32_t K,
                                                      const int32_t *__restrict__ Ap,
                                                      const int32_t *__restrict__ Aj,
                                                      const double *__restrict__ Ax,
                                                      const int32_t *__restrict__ rem_ptr,
                                                      int32_t *__restrict__ rem_col,
                                                      double *__restrict__ rem_val,
                                                      float *__restrict__ rem_val32) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t src = Ap[i] + K, end = Ap[i + 1], dst = rem_ptr[i];
    for (; src < end; ++src, ++dst) {
        rem_col[dst] = Aj[src];
        double v = Ax[src];
        rem_val[dst] = v;
        if (rem_val32) rem_val32[dst] = (float)v;
    }
}

// ------------------------------------------------------------------ SpMV kernels

// ELL part (Alg. 1, first loop): one thread per row, slab loads are
// non-temporal (streamed once), x is gathered through the caches.
// y[i] = alpha * sum_s val[s*ld+i] * x[col[s*ld+i]] + beta * z[i].
// KT > 0: the width is KT, known at compile time, so that all 2 KT slab loads and
// then all KT gathers of a row are issued before the first is used (a run-time
// width leaves the entries past the last group of four to load one after another).
template <class VT, class XT, class YT, class AT, int KT = 0>
__global__ __launch_bounds__(256) void k_spmv_ell(int32_t n, int32_t Kd, int32_t ld,
                                                  const int32_t *__restrict__ col,
                                                  const VT *__restrict__ val, AT alpha,
                                                  const XT *__restrict__ x, AT beta,
                                                  const YT *z, YT *y, const int32_t *skip) {
    if (skip && *skip) return;
    // Workgroups are dispatched round-robin over the 8 XCDs (each with its own
    // L2): give XCD k the k-th contiguous eighth of the rows, so that the x
    // entries a row gathers from its neighbours (also those nx*ny rows away)
    // are mostly cached in the same L2. The grid is a multiple of 8.
    const uint32_t per = gridDim.x >> 3;
    const uint32_t blk = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
    int32_t i = blk * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t *c = col + i;
    const VT *v = val + i;
    AT acc = 0;
    if constexpr (KT > 0) {
        int32_t j[KT];
        VT a[KT];
#pragma unroll
        for (int s = 0; s < KT; ++s) j[s] = __builtin_nontemporal_load(c + (size_t)s * ld);
#pragma unroll
        for (int s = 0; s < KT; ++s) a[s] = __builtin_nontemporal_load(v + (size_t)s * ld);
        XT xs[KT];
#pragma unroll
        for (int s = 0; s < KT; ++s) xs[s] = x[j[s]];
#pragma unroll
        for (int s = 0; s < KT; ++s) acc += (AT)a[s] * (AT)xs[s];
        AT r = alpha * acc;
        if (beta != (AT)0) r += beta * (AT)z[i];
        y[i] = (YT)r;
        return;
    }
    const int32_t K = Kd;
    int32_t s = 0;
    for (; s + 4 <= K; s += 4) {
        int32_t j0 = __builtin_nontemporal_load(c + (size_t)(s + 0) * ld);
        int32_t j1 = __builtin_nontemporal_load(c + (size_t)(s + 1) * ld);
        int32_t j2 = __builtin_nontemporal_load(c + (size_t)(s + 2) * ld);
        int32_t j3 = __builtin_nontemporal_load(c + (size_t)(s + 3) * ld);
        VT a0 = __builtin_nontemporal_load(v + (size_t)(s + 0) * ld);
        VT a1 = __builtin_nontemporal_load(v + (size_t)(s + 1) * ld);
        VT a2 = __builtin_nontemporal_load(v + (size_t)(s + 2) * ld);
        VT a3 = __builtin_nontemporal_load(v + (size_t)(s + 3) * ld);
        XT x0 = x[j0], x1 = x[j1], x2 = x[j2], x3 = x[j3];
        acc += (AT)a0 * (AT)x0;
        acc += (AT)a1 * (AT)x1;
        acc += (AT)a2 * (AT)x2;
        acc += (AT)a3 * (AT)x3;
    }
    for (; s < K; ++s) {
        int32_t j = __builtin_nontemporal_load(c + (size_t)s * ld);
        VT a = __builtin_nontemporal_load(v + (size_t)s * ld);
        acc += (AT)a * (AT)x[j];
    }
    AT r = alpha * acc;
    if (beta != (AT)0) r += beta * (AT)z[i];
    y[i] = (YT)r;
}

// Sum of rval[e] * x[rcol[e]] over e = e0 + t, e0 + t + step, ... < e1, in that
// order. The loads of four consecutive terms are issued before their products
// are added, so that a lane keeps four gathers in flight instead of one.
template <class VT, class XT, class AT>
__device__ __forceinline__ AT rem_strided_sum(int32_t e0, int32_t e1, int32_t t, int32_t step,
                                              const int32_t *__restrict__ rcol,
                                              const VT *__restrict__ rval, const XT *__restrict__ x) {
    AT acc = 0;
    int32_t e = e0 + t;
    for (; e + 3 * step < e1; e += 4 * step) {
        int32_t j0 = __builtin_nontemporal_load(rcol + e);
        int32_t j1 = __builtin_nontemporal_load(rcol + e + step);
        int32_t j2 = __builtin_nontemporal_load(rcol + e + 2 * step);
        int32_t j3 = __builtin_nontemporal_load(rcol + e + 3 * step);
        VT a0 = __builtin_nontemporal_load(rval + e);
        VT a1 = __builtin_nontemporal_load(rval + e + step);
        VT a2 = __builtin_nontemporal_load(rval + e + 2 * step);
        VT a3 = __builtin_nontemporal_load(rval + e + 3 * step);
        XT x0 = x[j0], x1 = x[j1], x2 = x[j2], x3 = x[j3];
        acc += (AT)a0 * (AT)x0;
        acc += (AT)a1 * (AT)x1;
        acc += (AT)a2 * (AT)x2;
        acc += (AT)a3 * (AT)x3;
    }
    for (; e < e1; e += step) acc += (AT)__builtin_nontemporal_load(rval + e) * (AT)x[__builtin_nontemporal_load(rcol + e)];
    return acc;
}

// Finish remainder row r with its sum t. first == true (no ELL part):
// y = alpha*t + beta*z; otherwise y += alpha*t.
template <class YT, class AT>
__device__ __forceinline__ void rem_finish(int32_t r, AT t, AT alpha, AT beta, const YT *z, YT *y, bool first) {
    if (first) {
        AT v = alpha * t;
        if (beta != (AT)0) v += beta * (AT)z[r];
        y[r] = (YT)v;
    } else {
        y[r] = (YT)((AT)y[r] + alpha * t);
    }
}

// CSR remainder (Alg. 1, second loop), rows shorter than kLongRem: LANES lanes
// per row (a sub-wavefront), lanes stride the row, then a butterfly reduction
// inside the group.
template <class VT, class XT, class YT, class AT, int LANES>
__global__ __launch_bounds__(256) void k_spmv_rem(int32_t nrows, const int32_t *__restrict__ rows,
                                                  const int32_t *__restrict__ rptr,
                                                  const int32_t *__restrict__ rcol,
                                                  const VT *__restrict__ rval, AT alpha,
                                                  const XT *__restrict__ x, AT beta, const YT *z,
                                                  YT *y, bool first, const int32_t *skip) {
    if (skip && *skip) return;
    int32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    int32_t grp = gid / LANES;  // uniform over the LANES lanes of the group
    int32_t lane = threadIdx.x % LANES;
    if (grp >= nrows) return;
    int32_t r = rows[grp];
    AT acc = rem_strided_sum<VT, XT, AT>(rptr[r], rptr[r + 1], lane, LANES, rcol, rval, x);
#pragma unroll
    for (int off = LANES / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LANES);
    if (lane == 0) rem_finish<YT, AT>(r, acc, alpha, beta, z, y, first);
}

// CSR remainder rows of kLongRem entries or more (a few very long rows, as in
// circuit matrices): one workgroup of kLongThreads per row, so that such a row
// does not leave a single wavefront working through it while the rest of the
// chip idles. Threads stride the row; each wavefront reduces by butterfly, and
// thread 0 adds the wavefronts' sums in wavefront order (deterministic).
constexpr int32_t kLongRem = 1024;
constexpr int kLongThreads = 1024;

template <class VT, class XT, class YT, class AT>
__global__ __launch_bounds__(kLongThreads) void k_spmv_rem_long(const int32_t *__restrict__ rows,
                                                                const int32_t *__restrict__ rptr,
                                                                const int32_t *__restrict__ rcol,
                                                                const VT *__restrict__ rval, AT alpha,
                                                                const XT *__restrict__ x, AT beta,
                                                                const YT *z, YT *y, bool first,
                                                                const int32_t *skip) {
    if (skip && *skip) return;
    __shared__ AT part[kLongThreads / 64];
    const int32_t r = rows[blockIdx.x];
    AT acc = rem_strided_sum<VT, XT, AT>(rptr[r], rptr[r + 1], (int32_t)threadIdx.x, kLongThreads, rcol, rval, x);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        AT t = part[0];
        for (int w = 1; w < kLongThreads / 64; ++w) t += part[w];
        rem_finish<YT, AT>(r, t, alpha, beta, z, y, first);
    }
}

// COO remainder (HYB): entry-parallel, deterministic. A wavefront takes a tile of
// kCooTile consecutive entries (row order), kCooE per lane. A lane sums its own
// entries row by row and adds every row that begins and ends inside its entries
// to y. The rows at the lanes' edges are summed by the lane where the row begins
// in the tile, over the following lanes in order (through LDS). A row that
// continues from the previous tile or into the next one is not added here: its
// partial sum goes to the tile's carry slots (first / last row), and k_coo_carry
// adds them in tile order.
constexpr int kCooE = 8;
constexpr int kCooTile = 64 * kCooE;

template <class VT, class XT, class YT, class AT>
__global__ __launch_bounds__(256) void k_spmv_coo(int64_t nnz, const int32_t *__restrict__ row,
                                                  const int32_t *__restrict__ col, const VT *__restrict__ val,
                                                  AT alpha, const XT *__restrict__ x, YT *y, int32_t *crow,
                                                  AT *cval, const int32_t *skip) {
    if (skip && *skip) return;
    __shared__ int32_t s_hr[4][64], s_tr[4][64];  // first and last row of each lane's entries (-1: none)
    __shared__ AT s_hs[4][64], s_ts[4][64];       // sums of its first and last row
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t base = tile * kCooTile;
    const bool live = base < nnz;  // uniform over the wavefront
    int32_t hr = -1, tr = -1;
    AT hs = 0, ts = 0;
    if (live) {
        const int64_t e0 = base + (int64_t)lane * kCooE;
        int32_t cur = -1;
        AT run = 0;
        bool head_done = false;
#pragma unroll
        for (int j = 0; j < kCooE; ++j) {
            const int64_t e = e0 + j;
            if (e < nnz) {
                const int32_t r = __builtin_nontemporal_load(row + e);
                const AT p = (AT)__builtin_nontemporal_load(val + e) * (AT)x[__builtin_nontemporal_load(col + e)];
                if (cur < 0) {
                    cur = hr = r;
                    run = p;
                } else if (r == cur) {
                    run += p;
                } else {
                    if (!head_done) {
                        hs = run;
                        head_done = true;
                    } else {
                        y[cur] = (YT)((AT)y[cur] + alpha * run);  // begins and ends in this lane
                    }
                    cur = r;
                    run = p;
                }
            }
        }
        tr = cur;
        ts = run;
        if (!head_done) hs = run;
    }
    s_hr[wv][lane] = hr;
    s_tr[wv][lane] = tr;
    s_hs[wv][lane] = hs;
    s_ts[wv][lane] = ts;
    __syncthreads();
    if (!live || hr < 0) return;
    const int32_t prev_row = base > 0 ? row[base - 1] : -1;
    const int64_t nb = base + kCooTile;
    const int32_t next_row = nb < nnz ? row[nb] : -1;
    if (lane == 0) {  // which of the tile's edge rows continue across it
        const int32_t first_r = s_hr[wv][0];
        const int32_t last_r = row[(nb < nnz ? nb : nnz) - 1];
        const bool cf = first_r == prev_row, ct = last_r == next_row;
        crow[2 * tile] = cf ? first_r : -1;
        crow[2 * tile + 1] = ct ? (cf && first_r == last_r ? -2 : last_r) : -1;
    }
    auto finish = [&](int32_t r, AT total) {
        const bool cf = r == prev_row, ct = r == next_row;
        if (!cf && !ct) y[r] = (YT)((AT)y[r] + alpha * total);
        else if (cf) cval[2 * tile] = total;  // also a tile that is one row throughout
        else cval[2 * tile + 1] = total;
    };
    if (hr != tr && (lane == 0 || s_tr[wv][lane - 1] != hr)) finish(hr, hs);  // first row, ends in this lane
    if (hr == tr && lane > 0 && s_tr[wv][lane - 1] == tr) return;  // one row, begun in an earlier lane
    AT total = ts;
    for (int m = lane + 1; m < 64; ++m) {  // the last row, on through the following lanes
        if (s_hr[wv][m] != tr) break;
        total += s_hs[wv][m];
        if (s_tr[wv][m] != tr) break;
    }
    finish(tr, total);
}

// Rows cut by COO tile boundaries: the tile where such a row begins adds the
// partial sums of the following tiles in order.
template <class YT, class AT>
__global__ __launch_bounds__(256) void k_coo_carry(int64_t ntiles, const int32_t *__restrict__ crow,
                                                   const AT *__restrict__ cval, AT alpha, YT *y,
                                                   const int32_t *skip) {
    if (skip && *skip) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const int32_t r = crow[2 * t + 1];
    if (r < 0) return;
    AT total = cval[2 * t + 1];
    for (int64_t u = t + 1; u < ntiles; ++u) {
        total += cval[2 * u];
        if (crow[2 * u + 1] != -2) break;  // the row ends in tile u
    }
    y[r] = (YT)((AT)y[r] + alpha * total);
}

// y = beta * z (0 when beta == 0): the start of a product without an ELL part.
template <class YT, class AT>
__global__ __launch_bounds__(256) void k_spmv_beta(int32_t n, AT beta, const YT *z, YT *y, const int32_t *skip) {
    if (skip && *skip) return;
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = beta != (AT)0 ? (YT)(beta * (AT)z[i]) : (YT)0;
}

// The ELL kernel with the width fixed at compile time for widths 1..8 (stencil
// and most HEC slabs), else the run-time width.
template <class VT, class XT, class YT, class AT>
static void launch_ell(const hec_matrix_s &A, const VT *ev, AT alpha, const XT *x, AT beta, const YT *z, YT *y,
                       hipStream_t s, const int32_t *skip) {
    const unsigned grid = (ceil_div(A.n, 256) + 7u) / 8u * 8u;  // a multiple of 8 (XCD mapping)
#define HEC_ELL_K(KK)                                                                                  \
    case KK:                                                                                           \
        k_spmv_ell<VT, XT, YT, AT, KK><<<grid, 256, 0, s>>>(A.n, A.K, A.ld, A.ell_col.get(), ev, alpha, x, \
                                                            beta, z, y, skip);                         \
        break;
    switch (A.K) {
        HEC_ELL_K(1)
        HEC_ELL_K(2)
        HEC_ELL_K(3)
        HEC_ELL_K(4)
        HEC_ELL_K(5)
        HEC_ELL_K(6)
        HEC_ELL_K(7)
        HEC_ELL_K(8)
        default:
            k_spmv_ell<VT, XT, YT, AT><<<grid, 256, 0, s>>>(A.n, A.K, A.ld, A.ell_col.get(), ev, alpha, x, beta, z,
                                                            y, skip);
    }
#undef HEC_ELL_K
    HEC_CHECK_LAUNCH();
}

template <class VT, class XT, class YT, class AT, int LANES>
static void launch_rem(const hec_matrix_s &A, const VT *rval, AT alpha, const XT *x, AT beta,
                       const YT *z, YT *y, bool first, hipStream_t s, const int32_t *skip) {
    size_t threads = (size_t)A.n_rem_rows * LANES;
    k_spmv_rem<VT, XT, YT, AT, LANES><<<ceil_div(threads, 256), 256, 0, s>>>(
        A.n_rem_rows, A.rem_rows.get(), A.rem_ptr.get(), A.rem_col.get(), rval, alpha, x, beta, z, y,
        first, skip);
}

template <class VT, class XT, class YT>
void spmv_launch(const hec_matrix_s &A, double alpha_d, const XT *x, double beta_d, const YT *z, YT *y,
                 hipStream_t s, const int32_t *skip) {
    using AT = VT;  // accumulate in the value precision
    AT alpha = (AT)alpha_d, beta = (AT)beta_d;
    if (A.n == 0) return;
    const VT *ev, *rv;
    if constexpr (sizeof(VT) == 8) {
        ev = (const VT *)A.ell_val.get();
        rv = (const VT *)A.rem_val.get();
    } else {
        ev = (const VT *)A.ell_val32.get();
        rv = (const VT *)A.rem_val32.get();
    }
    bool first = A.K == 0;
    if (A.coo) {
        // HYB: ELL part (or y = beta z without one), then the COO remainder and its carries
        if (first) {
            k_spmv_beta<YT, AT><<<ceil_div(A.n, 256), 256, 0, s>>>(A.n, beta, z, y, skip);
            HEC_CHECK_LAUNCH();
        } else {
            launch_ell<VT, XT, YT, AT>(A, ev, alpha, x, beta, z, y, s, skip);
        }
        if (A.nnz_rem > 0) {
            AT *cval = (AT *)A.carry_val.get();
            k_spmv_coo<VT, XT, YT, AT><<<ceil_div((size_t)A.coo_tiles * 64, 256), 256, 0, s>>>(
                A.nnz_rem, A.rem_row.get(), A.rem_col.get(), rv, alpha, x, y, A.carry_row.get(), cval, skip);
            HEC_CHECK_LAUNCH();
            k_coo_carry<YT, AT><<<ceil_div((size_t)A.coo_tiles, 256), 256, 0, s>>>(A.coo_tiles, A.carry_row.get(),
                                                                                 cval, alpha, y, skip);
            HEC_CHECK_LAUNCH();
        }
        return;
    }
    if (!first) launch_ell<VT, XT, YT, AT>(A, ev, alpha, x, beta, z, y, s, skip);
    if (A.n_rem_rows > 0) {
        switch (A.rem_lanes) {
            case 2: launch_rem<VT, XT, YT, AT, 2>(A, rv, alpha, x, beta, z, y, first, s, skip); break;
            case 4: launch_rem<VT, XT, YT, AT, 4>(A, rv, alpha, x, beta, z, y, first, s, skip); break;
            case 8: launch_rem<VT, XT, YT, AT, 8>(A, rv, alpha, x, beta, z, y, first, s, skip); break;
            case 16: launch_rem<VT, XT, YT, AT, 16>(A, rv, alpha, x, beta, z, y, first, s, skip); break;
            case 32: launch_rem<VT, XT, YT, AT, 32>(A, rv, alpha, x, beta, z, y, first, s, skip); break;
            default: launch_rem<VT, XT, YT, AT, 64>(A, rv, alpha, x, beta, z, y, first, s, skip); break;
        }
        HEC_CHECK_LAUNCH();
    }
    if (A.n_rem_long > 0) {
        k_spmv_rem_long<VT, XT, YT, AT><<<A.n_rem_long, kLongThreads, 0, s>>>(
            A.rem_long.get(), A.rem_ptr.get(), A.rem_col.get(), rv, alpha, x, beta, z, y, first, skip);
        HEC_CHECK_LAUNCH();
    }
}

template void spmv_launch<double, double, double>(const hec_matrix_s &, double, const double *, double,
                                                  const double *, double *, hipStream_t,
                                                  const int32_t *);
template void spmv_launch<double, float, double>(const hec_matrix_s &, double, const float *, double,
                                                  const double *, double *, hipStream_t,
                                                  const int32_t *);
template void spmv_launch<double, double, float>(const hec_matrix_s &, double, const double *, double,
                                                  const float *, float *, hipStream_t,
                                                  const int32_t *);
template void spmv_launch<double, float, float>(const hec_matrix_s &, double, const float *, double,
                                                  const float *, float *, hipStream_t,
                                                  const int32_t *);
template void spmv_launch<float, float, float>(const hec_matrix_s &, double, const float *, double,
                                                  const float *, float *, hipStream_t,
                                                  const int32_t *);
template void spmv_launch<float, double, double>(const hec_matrix_s &, double, const double *, double,
                                                  const double *, double *, hipStream_t,
                                                  const int32_t *);
template void spmv_launch<float, float, double>(const hec_matrix_s &, double, const float *, double,
                                                  const double *, double *, hipStream_t,
                                                  const int32_t *);
template void spmv_launch<float, double, float>(const hec_matrix_s &, double, const double *, double,
                                                  const float *, float *, hipStream_t,
                                                  const int32_t *);

// The HEC (or HYB, ELL, CSR) form of an n x ncols CSR matrix (validated by the
// caller); also used for the rectangular transfer operators of AMG.
std::unique_ptr<hec_matrix_s> make_hec(int32_t n, int32_t ncols, const int32_t *Ap, const int32_t *Aj,
                                       const double *Ax, int32_t ell_width, uint32_t flags, hipStream_t s) {
    auto A = std::make_unique<hec_matrix_s>();
    OwnerScope own(&A->dev_bytes);
    A->n = n;
    A->nnz = Ap[n];
    int32_t maxrow = 0;
    for (int32_t i = 0; i < n; ++i) maxrow = std::max(maxrow, Ap[i + 1] - Ap[i]);
    int32_t K = ell_width >= 0 ? ell_width : 20;
    if (ell_width == HEC_WIDTH_HYB) {
        // HYB rule: the largest K such that at least max(4096, n/3) rows hold K or more entries
        std::vector<int64_t> atleast((size_t)maxrow + 2, 0);
        for (int32_t i = 0; i < n; ++i) atleast[Ap[i + 1] - Ap[i]]++;
        for (int32_t k = maxrow - 1; k >= 0; --k) atleast[k] += atleast[k + 1];
        const int64_t need = std::max<int64_t>(4096, n / 3);
        K = 0;
        for (int32_t k = 1; k <= maxrow; ++k)
            if (atleast[k] >= need) K = k;
    }
    A->K = std::min(K, maxrow);
    A->ld = (int32_t)(((int64_t)n + 255) / 256 * 256);
    A->has_f32 = (flags & HEC_KEEP_F32) != 0;
    // remainder row pointer and row list (host prefix sum)
    std::vector<int32_t> rptr(n + 1);
    std::vector<int32_t> rrows, rlong;
    int64_t r = 0, rshort = 0;
    rptr[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t len = Ap[i + 1] - Ap[i];
        int32_t extra = len > A->K ? len - A->K : 0;
        if (extra >= kLongRem) {
            rlong.push_back(i);
        } else if (A->K == 0 || extra > 0) {
            rrows.push_back(i);
            rshort += extra;
        }
        r += extra;
        rptr[i + 1] = (int32_t)r;
    }
    A->nnz_rem = r;
    A->n_rem_rows = (int32_t)rrows.size();
    A->n_rem_long = (int32_t)rlong.size();
    {
        // lanes per short remainder row: the power of two nearest their mean length
        double mean = rrows.empty() ? 0.0 : (double)rshort / rrows.size();
        int lanes = 2;
        while (lanes < 64 && lanes * 1.5 < mean) lanes *= 2;
        A->rem_lanes = lanes;
    }
    size_t slab = (size_t)A->K * A->ld;
    A->ell_col.alloc(slab);
    A->ell_val.alloc(slab);
    if (A->has_f32) A->ell_val32.alloc(slab);
    A->rem_ptr.alloc(n + 1);
    A->rem_col.alloc(r);
    A->rem_val.alloc(r);
    if (A->has_f32) A->rem_val32.alloc(r);
    A->rem_rows.alloc(rrows.size());
    A->rem_ptr.upload(rptr.data(), n + 1, s);
    A->rem_rows.upload(rrows.data(), rrows.size(), s);
    A->rem_long.alloc(rlong.size());
    A->rem_long.upload(rlong.data(), rlong.size(), s);
    std::vector<int32_t> rrow;
    if (flags & HEC_COO_REMAINDER) {
        A->coo = true;
        rrow.resize(r);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t e = rptr[i]; e < rptr[i + 1]; ++e) rrow[e] = i;
        A->coo_tiles = (r + kCooTile - 1) / kCooTile;
        A->rem_row.alloc(r);
        A->rem_row.upload(rrow.data(), r, s);
        A->carry_row.alloc(2 * A->coo_tiles);
        A->carry_val.alloc(2 * A->coo_tiles);
    }
    // stage the CSR on the device and scatter it into the two parts
    DevBuf<int32_t> dAp(n + 1), dAj(A->nnz);
    DevBuf<double> dAx(A->nnz);
    dAp.upload(Ap, n + 1, s);
    dAj.upload(Aj, A->nnz, s);
    dAx.upload(Ax, A->nnz, s);
    if (slab) {
        k_hec_fill_ell<<<ceil_div(A->ld, 256), 256, 0, s>>>(n, ncols, A->K, A->ld, dAp.get(), dAj.get(),
                                                            dAx.get(), A->ell_col.get(), A->ell_val.get(),
                                                            A->ell_val32.get());
        HEC_CHECK_LAUNCH();
    }
    if (r && n) {
        k_hec_fill_rem<<<ceil_div(n, 256), 256, 0, s>>>(n, A->K, dAp.get(), dAj.get(), dAx.get(),
                                                        A->rem_ptr.get(), A->rem_col.get(),
                                                        A->rem_val.get(), A->rem_val32.get());
        HEC_CHECK_LAUNCH();
    }
    HEC_HIP(hipStreamSynchronize(s));
    return A;
}

}  // namespace hec

using namespace hec;

extern "C" {

const char *hec_last_error(void) { return g_last_error.c_str(); }

hec_status hec_from_csr(int32_t n, const int32_t *Ap, const int32_t *Aj, const double *Ax,
                        int32_t ell_width, uint32_t flags, void *stream, hec_matrix *out) {
    return guarded([&] {
        if (!out) fail(HEC_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        validate_csr(n, Ap, Aj, Ax);
        if (flags & ~(HEC_KEEP_F32 | HEC_COO_REMAINDER)) fail(HEC_ERR_INVALID_ARG, "unknown flags");
        hipStream_t s = as_stream(stream);
        StreamScope scope(s);
        *out = make_hec(n, n, Ap, Aj, Ax, ell_width, flags, s).release();
    });
}

hec_status hec_info(hec_matrix A, int32_t *n, int32_t *K, int32_t *ld, int64_t *nnz, int64_t *nnz_rem) {
    return guarded([&] {
        if (!A) fail(HEC_ERR_INVALID_ARG, "null matrix");
        if (n) *n = A->n;
        if (K) *K = A->K;
        if (ld) *ld = A->ld;
        if (nnz) *nnz = A->nnz;
        if (nnz_rem) *nnz_rem = A->nnz_rem;
    });
}

hec_status hec_export(hec_matrix A, int32_t *ell_col, double *ell_val, int32_t *rem_ptr, int32_t *rem_col,
                      double *rem_val, float *ell_val32, float *rem_val32) {
    return guarded([&] {
        if (!A) fail(HEC_ERR_INVALID_ARG, "null matrix");
        if ((ell_val32 || rem_val32) && !A->has_f32) fail(HEC_ERR_INVALID_ARG, "matrix has no FP32 copy");
        size_t slab = (size_t)A->K * A->ld;
        hipStream_t s = A->ell_col.st;
        if (ell_col) A->ell_col.download(ell_col, slab, s);
        if (ell_val) A->ell_val.download(ell_val, slab, s);
        if (ell_val32) A->ell_val32.download(ell_val32, slab, s);
        if (rem_ptr) A->rem_ptr.download(rem_ptr, A->n + 1, s);
        if (rem_col) A->rem_col.download(rem_col, A->nnz_rem, s);
        if (rem_val) A->rem_val.download(rem_val, A->nnz_rem, s);
        if (rem_val32) A->rem_val32.download(rem_val32, A->nnz_rem, s);
        HEC_HIP(hipStreamSynchronize(s));
    });
}

hec_status hec_spmv(hec_matrix A, hec_dtype vals, double alpha, const void *x, hec_dtype xt, double beta,
                    void *y, hec_dtype yt, void *stream) {
    return guarded([&] {
        if (!A) fail(HEC_ERR_INVALID_ARG, "null matrix");
        if (A->n > 0 && (!x || !y)) fail(HEC_ERR_INVALID_ARG, "x or y is NULL");
        if (vals == HEC_F32 && !A->has_f32) fail(HEC_ERR_INVALID_ARG, "matrix has no FP32 copy (HEC_KEEP_F32)");
        if ((vals != HEC_F64 && vals != HEC_F32) || (xt != HEC_F64 && xt != HEC_F32) ||
            (yt != HEC_F64 && yt != HEC_F32))
            fail(HEC_ERR_INVALID_ARG, "bad dtype");
        if (!std::isfinite(alpha) || !std::isfinite(beta)) fail(HEC_ERR_INVALID_ARG, "alpha/beta not finite");
        hipStream_t s = as_stream(stream);
        StreamScope scope(s);
        int key = (vals << 2) | (xt << 1) | yt;
        switch (key) {
#define CASE(V, X, Y, TV, TX, TY)                                                                       \
    case ((V << 2) | (X << 1) | Y):                                                                     \
        spmv_launch<TV, TX, TY>(*A, alpha, (const TX *)x, beta, (const TY *)y, (TY *)y, s);             \
        break;
            CASE(0, 0, 0, double, double, double)
            CASE(0, 1, 0, double, float, double)
            CASE(0, 0, 1, double, double, float)
            CASE(0, 1, 1, double, float, float)
            CASE(1, 1, 1, float, float, float)
            CASE(1, 0, 0, float, double, double)
            CASE(1, 1, 0, float, float, double)
            CASE(1, 0, 1, float, double, float)
#undef CASE
        }
    });
}

hec_status hec_set_spin_limit(int64_t polls) {
    return guarded([&] {
        if (polls > (int64_t)UINT32_MAX) fail(HEC_ERR_INVALID_ARG, "spin limit above 2^32 - 1 polls");
        g_spin.store(polls < 0 ? kDefaultSpin : (uint32_t)polls);
    });
}

hec_status hec_set_trsv_grid(int32_t enable) {
    return guarded([&] {
        if (enable != 0 && enable != 1) fail(HEC_ERR_INVALID_ARG, "enable must be 0 or 1");
        g_trsv_grid.store(enable != 0);
    });
}

hec_status hec_set_allocator(hec_alloc_fn alloc, hec_free_fn free_fn, void *ctx) {
    return guarded([&] {
        if ((alloc == nullptr) != (free_fn == nullptr))
            fail(HEC_ERR_INVALID_ARG, "alloc and free must both be set or both be NULL");
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        g_alloc.alloc = alloc;
        g_alloc.free = free_fn;
        g_alloc.ctx = alloc ? ctx : nullptr;
    });
}

hec_status hec_footprint(hec_matrix A, hec_ilu M, hec_levels lv, int64_t *bytes) {
    return guarded([&] {
        if (!bytes) fail(HEC_ERR_INVALID_ARG, "bytes is NULL");
        *bytes = (A ? A->dev_bytes : 0) + (M ? M->dev_bytes : 0) + (lv ? lv->dev_bytes : 0);
    });
}

hec_status hec_destroy(hec_matrix A) {
    delete A;
    return HEC_OK;
}

}  // extern "C"
