// ILU(k) (Sec. 2.4, Eq. (7)-(10), Alg. 2), level schedules (Sec. 2.6, Eq. (11),
// Alg. 3) and the level-scheduled triangular solves.
//
// Symbolic work (the fill pattern S_k, the levels) is integer work done once
// per matrix on the host. The numeric factorisation runs on the device, one
// launch per level of L. The triangular solves run as one persistent launch
// per triangle in which a row starts as soon as its dependencies are final:
//
//  * rows are laid out in level order (position q = 0..n-1) and cut into
//    64-row chunks that never straddle a level, so the 64 lanes of a
//    wavefront solve 64 independent rows;
//  * wavefronts take chunks in increasing order from a ticket counter, so a
//    chunk only ever waits for chunks already taken by running wavefronts
//    (no deadlock, whatever the grid size or occupancy);
//  * the solution vector itself is the readiness flag: it is pre-filled with
//    a signalling-NaN bit pattern that arithmetic never produces, results are
//    written with device-coherent stores and dependencies are polled with
//    device-coherent loads. Only single-location coherence is needed, so no
//    cache-wide fence is issued anywhere in the solve.
#include <algorithm>
#include <cmath>
#include <memory>

#include "hec_internal.hpp"

namespace hec {

// ------------------------------------------------------------------ host symbolic work

// Symbolic ILU(k): S_k = {(i,j) : level(i,j) <= k} with the level rule of
// Eq. (9)-(10). Row i starts from A's pattern at level 0; pivots p < i are
// taken in increasing order and each merges the kept upper part of row p with
// level lev(i,p) + lev(p,j) + 1. Candidates above k are never inserted: they
// can neither be kept nor act as pivots.
static void symbolic_iluk(int32_t n, const int32_t *Ap, const int32_t *Aj, int32_t k,
                          std::vector<int32_t> &LUp, std::vector<int32_t> &LUj, std::vector<int32_t> &diag) {
    LUp.assign(n + 1, 0);
    diag.assign(n, -1);
    LUj.clear();
    if (k == 0) {
        LUj.assign(Aj, Aj + Ap[n]);
        for (int32_t i = 0; i <= n; ++i) LUp[i] = Ap[i];
        for (int32_t i = 0; i < n; ++i)
            for (int32_t e = Ap[i]; e < Ap[i + 1]; ++e)
                if (Aj[e] == i) diag[i] = e;
        return;
    }
    LUj.reserve((size_t)Ap[n] * 2);
    std::vector<int32_t> LUlev;
    LUlev.reserve((size_t)Ap[n] * 2);
    std::vector<std::pair<int32_t, int32_t>> row;  // (column, level), ascending column
    for (int32_t i = 0; i < n; ++i) {
        row.clear();
        for (int32_t e = Ap[i]; e < Ap[i + 1]; ++e) row.emplace_back(Aj[e], 0);
        for (size_t t = 0; t < row.size() && row[t].first < i; ++t) {
            int32_t p = row[t].first, lp = row[t].second;
            // merge the upper part of row p (final, kept entries only)
            size_t pos = t + 1;
            for (int32_t u = diag[p] + 1; u < LUp[p + 1]; ++u) {
                int32_t j = LUj[u];
                int32_t lv = lp + LUlev[u] + 1;
                if (lv > k) continue;
                while (pos < row.size() && row[pos].first < j) ++pos;
                if (pos < row.size() && row[pos].first == j) {
                    if (lv < row[pos].second) row[pos].second = lv;
                } else {
                    row.insert(row.begin() + pos, std::make_pair(j, lv));
                }
            }
        }
        for (auto &cl : row) {
            if (cl.first == i) diag[i] = (int32_t)LUj.size();
            LUj.push_back(cl.first);
            LUlev.push_back(cl.second);
        }
        LUp[i + 1] = (int32_t)LUj.size();
    }
}

// Eq. (11): level of each row, 0-based, for the strict lower (upper == false)
// or strict upper triangle, then Alg. 3's grouping: level_ptr and perm with
// rows ascending inside each level (stable counting sort).
static int32_t compute_levels(int32_t n, const std::vector<int32_t> &LUp, const std::vector<int32_t> &LUj,
                              const std::vector<int32_t> &diag, bool upper, std::vector<int32_t> &level_ptr,
                              std::vector<int32_t> &perm) {
    std::vector<int32_t> lev(n);
    int32_t nlev = 0;
    if (!upper) {
        for (int32_t i = 0; i < n; ++i) {
            int32_t l = 0;
            for (int32_t e = LUp[i]; e < diag[i]; ++e) l = std::max(l, lev[LUj[e]] + 1);
            lev[i] = l;
            nlev = std::max(nlev, l + 1);
        }
    } else {
        for (int32_t i = n - 1; i >= 0; --i) {
            int32_t l = 0;
            for (int32_t e = diag[i] + 1; e < LUp[i + 1]; ++e) l = std::max(l, lev[LUj[e]] + 1);
            lev[i] = l;
            nlev = std::max(nlev, l + 1);
        }
    }
    level_ptr.assign(nlev + 1, 0);
    for (int32_t i = 0; i < n; ++i) level_ptr[lev[i] + 1]++;
    for (int32_t l = 0; l < nlev; ++l) level_ptr[l + 1] += level_ptr[l];
    std::vector<int32_t> next(level_ptr.begin(), level_ptr.end() - 1);
    perm.resize(n);
    for (int32_t i = 0; i < n; ++i) perm[next[lev[i]]++] = i;
    return nlev;
}

// ------------------------------------------------------------------ numeric ILU kernel

// Rows of one level of L, one thread per row (Alg. 2 restricted to S_k):
// for each stored p < i in ascending order, l_ip = a_ip / u_pp, then
// a_ij -= l_ip * u_pj for every stored (p, j), j > p, that is also in row i.
// All rows p were finished by earlier launches.
__global__ __launch_bounds__(256) void k_ilu_level(int32_t cnt, const int32_t *__restrict__ rows,
                                                   const int32_t *__restrict__ LUp,
                                                   const int32_t *__restrict__ LUj,
                                                   const int32_t *__restrict__ diag, double *LUx,
                                                   int32_t *zero_pivot) {
    int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    int32_t i = rows[t];
    int32_t b = LUp[i + 1], di = diag[i];
    for (int32_t e = LUp[i]; e < di; ++e) {
        int32_t p = LUj[e];
        int32_t dp = diag[p];
        double upp = LUx[dp];
        if (upp == 0.0) {
            atomicMax(zero_pivot, p + 1);
            return;
        }
        double lip = LUx[e] / upp;
        LUx[e] = lip;
        int32_t f = e + 1;
        int32_t pe = LUp[p + 1];
        for (int32_t u = dp + 1; u < pe && f < b; ++u) {
            int32_t j = LUj[u];
            while (f < b && LUj[f] < j) ++f;
            if (f < b && LUj[f] == j) LUx[f] -= lip * LUx[u];
        }
    }
}

__global__ __launch_bounds__(256) void k_check_diag(int32_t n, const int32_t *__restrict__ diag,
                                                    const double *__restrict__ LUx, int32_t *zero_pivot) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && LUx[diag[i]] == 0.0) atomicMax(zero_pivot, i + 1);
}

template <class S, class D>
__global__ __launch_bounds__(256) void k_convert(size_t n, const S *__restrict__ src, D *__restrict__ dst) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (D)src[i];
}

// dst[q] = src[map[q]] (0 where map[q] < 0), optional FP32 copy.
__global__ __launch_bounds__(256) void k_gather(size_t n, const int32_t *__restrict__ map,
                                                const double *__restrict__ src, double *__restrict__ dst,
                                                float *__restrict__ dst32) {
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int32_t m = map[q];
    double v = m >= 0 ? src[m] : 0.0;
    dst[q] = v;
    if (dst32) dst32[q] = (float)v;
}

// ------------------------------------------------------------------ triangular solve kernels

template <class T> struct Sentinel;
template <> struct Sentinel<double> {
    using U = unsigned long long;
    static constexpr U bits = 0x7FF4DEADBEEF1234ull;  // signalling NaN: never produced by arithmetic
    static constexpr U qnan = 0x7FF8000000000000ull;
};
template <> struct Sentinel<float> {
    using U = unsigned int;
    static constexpr U bits = 0x7FA0BEEFu;
    static constexpr U qnan = 0x7FC00000u;
};

template <class T>
__device__ __forceinline__ typename Sentinel<T>::U load_coherent(const T *p) {
    using U = typename Sentinel<T>::U;
    return __hip_atomic_load((U *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publishes a solved value. A right-hand side that carries the sentinel's own
// bit pattern (and reaches the output untouched by arithmetic) is replaced by
// a quiet NaN, so no waiting row can mistake a final value for "not ready".
template <class T>
__device__ __forceinline__ void store_coherent(T *p, T v) {
    using U = typename Sentinel<T>::U;
    U u;
    __builtin_memcpy(&u, &v, sizeof(T));
    if (u == Sentinel<T>::bits) u = Sentinel<T>::qnan;
    __hip_atomic_store((U *)p, u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ T from_bits(typename Sentinel<T>::U u) {
    T v;
    __builtin_memcpy(&v, &u, sizeof(T));
    return v;
}

template <class T>
__global__ __launch_bounds__(256) void k_fill_sentinel(size_t n, T *a, T *b, const int32_t *skip) {
    if (skip && *skip) return;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T s = from_bits<T>(Sentinel<T>::bits);
    a[i] = s;
    if (b) b[i] = s;
}

// Sync-free level-scheduled substitution for one triangle (Alg. 3 with the
// level barrier replaced by per-row readiness). Lower: x_i = b_i - sum L_ij x_j.
// Upper: x_i = (b_i - sum U_ij x_j) / U_ii. Terms are taken in ascending column
// order. x must be pre-filled with the sentinel. sync[0] is the chunk ticket,
// sync[1] counts finished wavefronts; the last one resets both for the next launch.
template <class T, bool UPPER>
__global__ __launch_bounds__(256) void k_trsv(int32_t nchunks, const int32_t *__restrict__ chunk_ptr,
                                              const int32_t *__restrict__ perm, int32_t K, int32_t ldq,
                                              const int32_t *__restrict__ col, const T *__restrict__ val,
                                              const T *__restrict__ dpiv, const T *__restrict__ b, T *x,
                                              uint32_t *sync, const int32_t *skip) {
    if (skip && *skip) return;  // uniform: no wavefront touches the counters
    using U = typename Sentinel<T>::U;
    constexpr U SENT = Sentinel<T>::bits;
    constexpr int B = 8;  // dependencies loaded per batch
    const int lane = threadIdx.x & 63;
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(&sync[0], 1u);
        t = __shfl(t, 0);
        if (t >= (uint32_t)nchunks) break;
        const int32_t q = chunk_ptr[t] + lane;
        if (q < chunk_ptr[t + 1]) {
            const int32_t i = perm[q];
            T acc = b[i];
            for (int32_t s0 = 0; s0 < K; s0 += B) {
                int32_t js[B];
                T vs[B];
                U xs[B];
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    int32_t s = s0 + u;
                    js[u] = s < K ? col[(size_t)s * ldq + q] : -1;
                    vs[u] = s < K ? val[(size_t)s * ldq + q] : (T)0;
                }
                bool pend = false;
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    xs[u] = 0;
                    if (js[u] >= 0) {
                        xs[u] = load_coherent(x + js[u]);
                        pend |= xs[u] == SENT;
                    }
                }
                while (pend) {
                    __builtin_amdgcn_s_sleep(1);
                    pend = false;
#pragma unroll
                    for (int u = 0; u < B; ++u) {
                        if (xs[u] == SENT) {
                            xs[u] = load_coherent(x + js[u]);
                            pend |= xs[u] == SENT;
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < B; ++u)
                    if (js[u] >= 0) acc -= vs[u] * from_bits<T>(xs[u]);
            }
            if constexpr (UPPER) acc = acc / dpiv[q];
            store_coherent(x + i, acc);
        }
    }
    if (lane == 0) {
        const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
        uint32_t d = atomicAdd(&sync[1], 1u);
        if (d == nwaves - 1) {
            __hip_atomic_store(&sync[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&sync[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

static constexpr int kChunk = 64;
static constexpr int kMaxTrsvWaves = 1024;

template <class T, bool UPPER>
static void launch_tri(const hec_tri &tri, const uint32_t *sync_const, const T *b, T *x, hipStream_t s,
                       const int32_t *skip) {
    if (tri.nchunks == 0) return;
    uint32_t *sync = const_cast<uint32_t *>(sync_const);
    int waves = std::min(tri.nchunks, kMaxTrsvWaves);
    int blocks = (waves + 3) / 4;
    const T *val, *dp = nullptr;
    if constexpr (sizeof(T) == 8) {
        val = (const T *)tri.val.get();
        if (UPPER) dp = (const T *)tri.dinv_src.get();
    } else {
        val = (const T *)tri.val32.get();
        if (UPPER) dp = (const T *)tri.d32.get();
    }
    k_trsv<T, UPPER><<<blocks, 256, 0, s>>>(tri.nchunks, tri.chunk_ptr.get(), tri.perm.get(), tri.K, tri.ldq,
                                            tri.col.get(), val, dp, b, x, sync, skip);
    HEC_CHECK_LAUNCH();
}

template <class T>
void trsv_launch(const hec_levels_s &lv, uint32_t which, const T *b, T *x, hipStream_t s, const int32_t *skip) {
    size_t n = lv.n;
    if (n == 0) return;
    T *tmp;
    if constexpr (sizeof(T) == 8) tmp = (T *)lv.tmp64.get();
    else tmp = (T *)lv.tmp32.get();
    if (which == HEC_LU) {
        k_fill_sentinel<T><<<ceil_div(n, 256), 256, 0, s>>>(n, tmp, x, skip);
        HEC_CHECK_LAUNCH();
        launch_tri<T, false>(lv.lower, lv.sync.get(), b, tmp, s, skip);
        launch_tri<T, true>(lv.upper, lv.sync.get() + 2, tmp, x, s, skip);
    } else {
        k_fill_sentinel<T><<<ceil_div(n, 256), 256, 0, s>>>(n, x, (T *)nullptr, skip);
        HEC_CHECK_LAUNCH();
        if (which == HEC_LOWER) launch_tri<T, false>(lv.lower, lv.sync.get(), b, x, s, skip);
        else launch_tri<T, true>(lv.upper, lv.sync.get() + 2, b, x, s, skip);
    }
}

template void trsv_launch<double>(const hec_levels_s &, uint32_t, const double *, double *, hipStream_t,
                                  const int32_t *);
template void trsv_launch<float>(const hec_levels_s &, uint32_t, const float *, float *, hipStream_t,
                                 const int32_t *);

// Builds one level-ordered triangle from the factor pattern (host) and gathers
// its values from the device factor.
static void build_tri(const hec_ilu_s &M, bool upper, hec_tri &tri, hipStream_t s) {
    const int32_t n = M.n;
    tri.nlev = compute_levels(n, M.hLUp, M.hLUj, M.hdiag, upper, tri.hlevel_ptr, tri.hperm);
    // chunks of up to 64 positions inside each level
    std::vector<int32_t> chunks;
    chunks.push_back(0);
    for (int32_t l = 0; l < tri.nlev; ++l) {
        for (int32_t q = tri.hlevel_ptr[l]; q < tri.hlevel_ptr[l + 1]; q += kChunk)
            chunks.push_back(std::min(q + kChunk, tri.hlevel_ptr[l + 1]));
    }
    tri.nchunks = (int32_t)chunks.size() - 1;
    int32_t K = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t c = upper ? M.hLUp[i + 1] - M.hdiag[i] - 1 : M.hdiag[i] - M.hLUp[i];
        K = std::max(K, c);
    }
    tri.K = K;
    tri.ldq = (int32_t)(((int64_t)n + 63) / 64 * 64);
    size_t slab = (size_t)K * tri.ldq;
    std::vector<int32_t> col(slab, -1), src(slab, -1), dsrc;
    if (upper) dsrc.assign(tri.ldq, -1);
    for (int32_t q = 0; q < n; ++q) {
        int32_t i = tri.hperm[q];
        int32_t a = upper ? M.hdiag[i] + 1 : M.hLUp[i];
        int32_t e1 = upper ? M.hLUp[i + 1] : M.hdiag[i];
        for (int32_t e = a, s2 = 0; e < e1; ++e, ++s2) {
            col[(size_t)s2 * tri.ldq + q] = M.hLUj[e];
            src[(size_t)s2 * tri.ldq + q] = e;
        }
        if (upper) dsrc[q] = M.hdiag[i];
    }
    tri.perm.alloc(n);
    tri.perm.upload(tri.hperm.data(), n, s);
    tri.chunk_ptr.alloc(chunks.size());
    tri.chunk_ptr.upload(chunks.data(), chunks.size(), s);
    tri.col.alloc(slab);
    tri.col.upload(col.data(), slab, s);
    tri.val.alloc(slab);
    if (M.has_f32) tri.val32.alloc(slab);
    DevBuf<int32_t> dsrc_map(slab);
    if (slab) {
        dsrc_map.upload(src.data(), slab, s);
        k_gather<<<ceil_div(slab, 256), 256, 0, s>>>(slab, dsrc_map.get(), M.LUx.get(), tri.val.get(),
                                                     tri.val32.get());
        HEC_CHECK_LAUNCH();
    }
    if (upper) {
        tri.dinv_src.alloc(tri.ldq);
        if (M.has_f32) tri.d32.alloc(tri.ldq);
        DevBuf<int32_t> dmap(tri.ldq);
        dmap.upload(dsrc.data(), tri.ldq, s);
        k_gather<<<ceil_div(tri.ldq, 256), 256, 0, s>>>(tri.ldq, dmap.get(), M.LUx.get(), tri.dinv_src.get(),
                                                         tri.d32.get());
        HEC_CHECK_LAUNCH();
        HEC_HIP(hipStreamSynchronize(s));
    }
    HEC_HIP(hipStreamSynchronize(s));
}

}  // namespace hec

using namespace hec;

extern "C" {

hec_status ilu_factor(int32_t n, const int32_t *Ap, const int32_t *Aj, const double *Ax, int32_t k, uint32_t flags,
                      void *stream, hec_ilu *out) {
    return guarded([&] {
        if (!out) fail(HEC_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        validate_csr(n, Ap, Aj, Ax);
        if (k < 0) fail(HEC_ERR_INVALID_ARG, "k < 0");
        if (flags & ~HEC_KEEP_F32) fail(HEC_ERR_INVALID_ARG, "unknown flags");
        for (int32_t i = 0; i < n; ++i) {
            bool d = false;
            for (int32_t e = Ap[i]; e < Ap[i + 1] && !d; ++e) d = Aj[e] == i;
            if (!d) fail(HEC_ERR_INVALID_ARG, "row " + std::to_string(i) + " has no stored diagonal");
        }
        hipStream_t s = as_stream(stream);
        auto M = std::make_unique<hec_ilu_s>();
        M->n = n;
        M->k = k;
        M->has_f32 = (flags & HEC_KEEP_F32) != 0;
        symbolic_iluk(n, Ap, Aj, k, M->hLUp, M->hLUj, M->hdiag);
        M->nnz = M->hLUp[n];
        // A's values scattered into S_k, fill entries start at 0
        std::vector<double> x0(M->nnz, 0.0);
        for (int32_t i = 0; i < n; ++i) {
            int32_t f = M->hLUp[i];
            for (int32_t e = Ap[i]; e < Ap[i + 1]; ++e) {
                while (M->hLUj[f] < Aj[e]) ++f;
                x0[f] = Ax[e];
            }
        }
        M->LUp.alloc(n + 1);
        M->LUj.alloc(M->nnz);
        M->diag.alloc(n);
        M->LUx.alloc(M->nnz);
        M->LUp.upload(M->hLUp.data(), n + 1, s);
        M->LUj.upload(M->hLUj.data(), M->nnz, s);
        M->diag.upload(M->hdiag.data(), n, s);
        M->LUx.upload(x0.data(), M->nnz, s);
        // numeric elimination, one launch per level of L
        std::vector<int32_t> lptr, perm;
        int32_t nlev = compute_levels(n, M->hLUp, M->hLUj, M->hdiag, false, lptr, perm);
        DevBuf<int32_t> dperm(n), dflag(1);
        dperm.upload(perm.data(), n, s);
        HEC_HIP(hipMemsetAsync(dflag.get(), 0, sizeof(int32_t), s));
        for (int32_t l = 1; l < nlev; ++l) {  // level 0 rows have no L entries: nothing to do
            int32_t a = lptr[l], cnt = lptr[l + 1] - lptr[l];
            k_ilu_level<<<ceil_div(cnt, 256), 256, 0, s>>>(cnt, dperm.get() + a, M->LUp.get(), M->LUj.get(),
                                                           M->diag.get(), M->LUx.get(), dflag.get());
            HEC_CHECK_LAUNCH();
        }
        int32_t zp = 0;
        dflag.download(&zp, 1, s);
        HEC_HIP(hipStreamSynchronize(s));
        if (zp) fail(HEC_ERR_ZERO_PIVOT, "zero pivot in row " + std::to_string(zp - 1));
        // every pivot u_ii must be nonzero for the backward substitution, also
        // those of rows that no later row uses
        if (n) {
            k_check_diag<<<ceil_div(n, 256), 256, 0, s>>>(n, M->diag.get(), M->LUx.get(), dflag.get());
            HEC_CHECK_LAUNCH();
            dflag.download(&zp, 1, s);
            HEC_HIP(hipStreamSynchronize(s));
            if (zp) fail(HEC_ERR_ZERO_PIVOT, "zero pivot in row " + std::to_string(zp - 1));
        }
        if (M->has_f32) {
            M->LUx32.alloc(M->nnz);
            if (M->nnz)
                k_convert<double, float><<<ceil_div(M->nnz, 256), 256, 0, s>>>(M->nnz, M->LUx.get(),
                                                                               M->LUx32.get());
            HEC_CHECK_LAUNCH();
            HEC_HIP(hipStreamSynchronize(s));
        }
        *out = M.release();
    });
}

hec_status ilu_info(hec_ilu M, int32_t *n, int64_t *nnz) {
    return guarded([&] {
        if (!M) fail(HEC_ERR_INVALID_ARG, "null factor");
        if (n) *n = M->n;
        if (nnz) *nnz = M->nnz;
    });
}

hec_status ilu_export(hec_ilu M, int32_t *LUp, int32_t *LUj, double *LUx) {
    return guarded([&] {
        if (!M) fail(HEC_ERR_INVALID_ARG, "null factor");
        if (LUp) std::copy(M->hLUp.begin(), M->hLUp.end(), LUp);
        if (LUj) std::copy(M->hLUj.begin(), M->hLUj.end(), LUj);
        if (LUx) {
            M->LUx.download(LUx, M->nnz, nullptr);
            HEC_HIP(hipStreamSynchronize(nullptr));
        }
    });
}

hec_status ilu_destroy(hec_ilu M) {
    delete M;
    return HEC_OK;
}

hec_status level_schedule(hec_ilu M, hec_levels *out) {
    return guarded([&] {
        if (!out) fail(HEC_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (!M) fail(HEC_ERR_INVALID_ARG, "null factor");
        hipStream_t s = nullptr;
        auto lv = std::make_unique<hec_levels_s>();
        lv->n = M->n;
        build_tri(*M, false, lv->lower, s);
        build_tri(*M, true, lv->upper, s);
        lv->sync.alloc(4);
        HEC_HIP(hipMemsetAsync(lv->sync.get(), 0, 4 * sizeof(uint32_t), s));
        lv->tmp64.alloc(M->n);
        if (M->has_f32) lv->tmp32.alloc(M->n);
        HEC_HIP(hipStreamSynchronize(s));
        *out = lv.release();
    });
}

hec_status levels_info(hec_levels lv, int32_t *n, int32_t *nlev_lower, int32_t *nlev_upper) {
    return guarded([&] {
        if (!lv) fail(HEC_ERR_INVALID_ARG, "null levels");
        if (n) *n = lv->n;
        if (nlev_lower) *nlev_lower = lv->lower.nlev;
        if (nlev_upper) *nlev_upper = lv->upper.nlev;
    });
}

hec_status levels_export(hec_levels lv, int32_t *lower_ptr, int32_t *lower_perm, int32_t *upper_ptr,
                         int32_t *upper_perm) {
    return guarded([&] {
        if (!lv) fail(HEC_ERR_INVALID_ARG, "null levels");
        if (lower_ptr) std::copy(lv->lower.hlevel_ptr.begin(), lv->lower.hlevel_ptr.end(), lower_ptr);
        if (lower_perm) std::copy(lv->lower.hperm.begin(), lv->lower.hperm.end(), lower_perm);
        if (upper_ptr) std::copy(lv->upper.hlevel_ptr.begin(), lv->upper.hlevel_ptr.end(), upper_ptr);
        if (upper_perm) std::copy(lv->upper.hperm.begin(), lv->upper.hperm.end(), upper_perm);
    });
}

hec_status levels_destroy(hec_levels lv) {
    delete lv;
    return HEC_OK;
}

hec_status trsv_levels(hec_ilu M, hec_levels lv, uint32_t which, hec_dtype prec, const void *b, void *x,
                       void *stream) {
    return guarded([&] {
        if (!M || !lv) fail(HEC_ERR_INVALID_ARG, "null factor or levels");
        if (M->n != lv->n) fail(HEC_ERR_INVALID_ARG, "factor and levels differ in size");
        if (which != HEC_LOWER && which != HEC_UPPER && which != HEC_LU) fail(HEC_ERR_INVALID_ARG, "bad `which`");
        if (lv->n > 0 && (!b || !x)) fail(HEC_ERR_INVALID_ARG, "b or x is NULL");
        if (b == x && lv->n > 0) fail(HEC_ERR_INVALID_ARG, "b and x must not overlap");
        hipStream_t s = as_stream(stream);
        if (prec == HEC_F64) {
            trsv_launch<double>(*lv, which, (const double *)b, (double *)x, s);
        } else if (prec == HEC_F32) {
            if (!M->has_f32 || (!lv->tmp32.get() && lv->n > 0))
                fail(HEC_ERR_INVALID_ARG, "factor has no FP32 copy (HEC_KEEP_F32)");
            trsv_launch<float>(*lv, which, (const float *)b, (float *)x, s);
        } else {
            fail(HEC_ERR_INVALID_ARG, "bad dtype");
        }
    });
}

}  // extern "C"
