// ILU(k) (Sec. 2.4, Eq. (7)-(10), Alg. 2) and level schedules (Sec. 2.6,
// Eq. (11), Alg. 3), plus their C entry points and trsv_levels'.
//
// Symbolic work (the fill pattern S_k, the levels) is integer work done once
// per matrix on the host. The numeric factorisation runs on the device, one
// launch per level of L.
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

}  // namespace hec

using namespace hec;

// ILU(k) of a CSR matrix (validated, every diagonal stored): host symbolic phase
// (Eq. (9)-(10)), device numeric phase level by level (Alg. 2 restricted to S_k).
static std::unique_ptr<hec_ilu_s> factor_csr(int32_t n, const int32_t *Ap, const int32_t *Aj, const double *Ax,
                                            int32_t k, uint32_t flags, hipStream_t s) {
    auto M = std::make_unique<hec_ilu_s>();
    OwnerScope own(&M->dev_bytes);
    M->n = n;
    M->k = k;
    M->has_f32 = (flags & HEC_KEEP_F32) != 0;
    symbolic_iluk(n, Ap, Aj, k, M->hLUp, M->hLUj, M->hdiag);
    plan::detect_grid(n, Ap, Aj, M->gnx, M->gny, M->gnz);
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
    int32_t nlev = plan::compute_levels(n, M->hLUp.data(), M->hLUj.data(), M->hdiag.data(), false, lptr, perm);
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
    M->n_sys = n;
    return M;
}

// Sec. 2.5, restricted additive Schwarz on one device: the rows are cut into
// nblocks contiguous blocks (the sequence partition), each block is extended by
// `overlap` layers of graph neighbours (rows reached through A's stored
// entries), and the extended blocks are stacked into one block-diagonal matrix
// that keeps only the entries of A inside each extended block. ext_row: system
// row of each stacked row; bstart: first stacked row of each block; own: the
// stacked row (inside its own block) of each system row.
static void ras_stack(int32_t n, const int32_t *Ap, const int32_t *Aj, const double *Ax, int32_t nblocks,
                      int32_t overlap, std::vector<int32_t> &Sp, std::vector<int32_t> &Sj, std::vector<double> &Sx,
                      std::vector<int32_t> &ext_row, std::vector<int32_t> &bstart, std::vector<int32_t> &own) {
    const int32_t R = (int32_t)(((int64_t)n + nblocks - 1) / nblocks);
    const int32_t nb = n ? (n + R - 1) / R : 0;
    std::vector<int32_t> stamp(n, -1), loc(n, 0);
    own.assign(n, -1);
    ext_row.clear();
    bstart.assign(1, 0);
    Sp.assign(1, 0);
    Sj.clear();
    Sx.clear();
    std::vector<int32_t> cur, layer, next;
    for (int32_t b = 0; b < nb; ++b) {
        const int32_t s0 = b * R, e0 = std::min(n, s0 + R);
        cur.clear();
        for (int32_t i = s0; i < e0; ++i) {
            stamp[i] = b;
            cur.push_back(i);
        }
        layer = cur;
        for (int32_t l = 0; l < overlap; ++l) {
            next.clear();
            for (int32_t i : layer)
                for (int32_t e = Ap[i]; e < Ap[i + 1]; ++e)
                    if (stamp[Aj[e]] != b) {
                        stamp[Aj[e]] = b;
                        next.push_back(Aj[e]);
                    }
            cur.insert(cur.end(), next.begin(), next.end());
            layer.swap(next);
        }
        std::sort(cur.begin(), cur.end());
        const int32_t base = (int32_t)ext_row.size();
        for (size_t t = 0; t < cur.size(); ++t) loc[cur[t]] = (int32_t)t;
        for (size_t t = 0; t < cur.size(); ++t) {
            const int32_t i = cur[t];
            ext_row.push_back(i);
            if (i >= s0 && i < e0) own[i] = base + (int32_t)t;
            for (int32_t e = Ap[i]; e < Ap[i + 1]; ++e)
                if (stamp[Aj[e]] == b) {
                    Sj.push_back(base + loc[Aj[e]]);
                    Sx.push_back(Ax[e]);
                }
            Sp.push_back((int32_t)Sj.size());
        }
        bstart.push_back((int32_t)ext_row.size());
    }
}

namespace hec {

void check_levels(const hec_levels_s &lv, hipStream_t s) {
    if (!lv.sync.get()) return;
    uint32_t *errw = const_cast<uint32_t *>(lv.sync.get()) + kLevelsErrWord;
    uint32_t e = 0;
    HEC_HIP(hipMemcpyAsync(&e, errw, sizeof(e), hipMemcpyDeviceToHost, s));
    HEC_HIP(hipStreamSynchronize(s));
    if (e) {
        const uint32_t zero = 0;
        HEC_HIP(hipMemcpyAsync(errw, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
        HEC_HIP(hipStreamSynchronize(s));
        fail(HEC_ERR_TIMEOUT, "a wait of the triangular solve gave up (its dependency never became ready); "
                              "the results of the solves since the last check are not valid");
    }
}

}  // namespace hec

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
        StreamScope scope(s);
        auto M = factor_csr(n, Ap, Aj, Ax, k, flags, s);
        *out = M.release();
    });
}

hec_status ilu_factor_ras(int32_t n, const int32_t *Ap, const int32_t *Aj, const double *Ax, int32_t k,
                          int32_t nblocks, int32_t overlap, uint32_t flags, void *stream, hec_ilu *out) {
    return guarded([&] {
        if (!out) fail(HEC_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        validate_csr(n, Ap, Aj, Ax);
        if (k < 0) fail(HEC_ERR_INVALID_ARG, "k < 0");
        if (nblocks < 1) fail(HEC_ERR_INVALID_ARG, "nblocks < 1");
        if (overlap < 0) fail(HEC_ERR_INVALID_ARG, "overlap < 0");
        if (flags & ~HEC_KEEP_F32) fail(HEC_ERR_INVALID_ARG, "unknown flags");
        for (int32_t i = 0; i < n; ++i) {
            bool d = false;
            for (int32_t e = Ap[i]; e < Ap[i + 1] && !d; ++e) d = Aj[e] == i;
            if (!d) fail(HEC_ERR_INVALID_ARG, "row " + std::to_string(i) + " has no stored diagonal");
        }
        std::vector<int32_t> Sp, Sj, ext_row, bstart, own;
        std::vector<double> Sx;
        ras_stack(n, Ap, Aj, Ax, nblocks, overlap, Sp, Sj, Sx, ext_row, bstart, own);
        const int64_t nf = (int64_t)ext_row.size();
        if (nf > INT32_MAX / 2 || (int64_t)Sj.size() > INT32_MAX)
            fail(HEC_ERR_INVALID_ARG, "extended blocks too large for 32-bit indices");
        hipStream_t s = as_stream(stream);
        StreamScope scope(s);
        auto M = factor_csr((int32_t)nf, Sp.data(), Sj.data(), Sx.data(), k, flags, s);
        M->n_sys = n;
        M->nblocks = (int32_t)bstart.size() - 1;
        M->overlap = overlap;
        M->gnx = M->gny = M->gnz = 0;
        M->hblocks.swap(bstart);
        M->hext_row.swap(ext_row);
        M->hown.swap(own);
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
            M->LUx.download(LUx, M->nnz, M->LUx.st);
            HEC_HIP(hipStreamSynchronize(M->LUx.st));
        }
    });
}

hec_status ilu_ras_export(hec_ilu M, int32_t *n_sys, int32_t *nblocks, int32_t *block_start, int32_t *ext_row,
                          int32_t *own) {
    return guarded([&] {
        if (!M) fail(HEC_ERR_INVALID_ARG, "null factor");
        const bool ras = !M->hext_row.empty();
        if (n_sys) *n_sys = M->n_sys;
        if (nblocks) *nblocks = ras ? M->nblocks : 1;
        if (block_start) {
            if (ras) {
                std::copy(M->hblocks.begin(), M->hblocks.end(), block_start);
            } else {
                block_start[0] = 0;
                block_start[1] = M->n;
            }
        }
        if (ext_row) {
            if (ras) std::copy(M->hext_row.begin(), M->hext_row.end(), ext_row);
            else for (int32_t i = 0; i < M->n; ++i) ext_row[i] = i;
        }
        if (own) {
            if (ras) std::copy(M->hown.begin(), M->hown.end(), own);
            else for (int32_t i = 0; i < M->n; ++i) own[i] = i;
        }
    });
}

hec_status ilu_destroy(hec_ilu M) {
    delete M;
    return HEC_OK;
}

hec_status level_schedule(hec_ilu M, void *stream, hec_levels *out) {
    return guarded([&] {
        if (!out) fail(HEC_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (!M) fail(HEC_ERR_INVALID_ARG, "null factor");
        hipStream_t s = as_stream(stream);
        StreamScope scope(s);
        auto lv = std::make_unique<hec_levels_s>();
        OwnerScope own(&lv->dev_bytes);
        lv->n = M->n_sys;
        lv->nf = M->n;
        lv->ras = !M->hext_row.empty();
        if (!lv->ras && trsv_grid_enabled()) {  // the wavefront plans: both triangles or neither
            build_grid(*M, true, lv->upper.grid, s);
            if (lv->upper.grid.on) build_grid(*M, false, lv->lower.grid, s);
            const hec_grid &gl = lv->lower.grid, &gu = lv->upper.grid;
            if (gl.on && (gl.PA != gu.PA || gl.PB != gu.PB || gl.S != gu.S))  // (one padded order serves both)
                lv->lower.grid = hec_grid();
            if (!lv->lower.grid.on) lv->upper.grid = hec_grid();
        }
        if (lv->lower.grid.on) {  // the level schedules only (levels_export, the batched copies)
            level_only(*M, true, lv->upper);
            level_only(*M, false, lv->lower);
        } else {
            build_tri(*M, true, lv->upper, nullptr, s);
            build_tri(*M, false, lv->lower, &lv->upper, s);
        }
        if (!lv->ras && M->n <= HEC_BATCH_MAX_N) {  // small enough for the batched solver
            build_flat(*M, false, lv->lower, s);
            build_flat(*M, true, lv->upper, s);
        }
        lv->sync.alloc(kLevelsSyncWords);
        HEC_HIP(hipMemsetAsync(lv->sync.get(), 0, kLevelsSyncWords * sizeof(uint32_t), s));
        lv->qL64.alloc(M->n);
        lv->qU64.alloc(M->n);
        const int64_t ny = lv->lower.grid.on ? std::max<int64_t>(M->n, lv->lower.grid.pad_elems()) : M->n;
        lv->yp64.alloc(ny);
        if (M->has_f32) {
            lv->qL32.alloc(M->n);
            lv->qU32.alloc(M->n);
            lv->yp32.alloc(ny);
        }
        if (lv->lower.grid.on) {
            const int64_t nface = lv->lower.grid.face_elems();
            lv->fL64.alloc(nface);
            lv->fU64.alloc(nface);
            if (M->has_f32) {
                lv->fL32.alloc(nface);
                lv->fU32.alloc(nface);
            }
        }
        trsv_init_levels(*lv, s);
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

hec_status levels_grid(hec_levels lv, int32_t *grid) {
    return guarded([&] {
        if (!lv || !grid) fail(HEC_ERR_INVALID_ARG, "null levels or output");
        *grid = lv->lower.grid.on && lv->upper.grid.on ? 1 : 0;
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

hec_status levels_check(hec_levels lv, void *stream) {
    return guarded([&] {
        if (!lv) fail(HEC_ERR_INVALID_ARG, "null levels");
        check_levels(*lv, as_stream(stream));
    });
}

hec_status trsv_levels(hec_ilu M, hec_levels lv, uint32_t which, hec_dtype prec, const void *b, void *x,
                       void *stream) {
    return guarded([&] {
        if (!M || !lv) fail(HEC_ERR_INVALID_ARG, "null factor or levels");
        if (M->n_sys != lv->n || M->n != lv->nf) fail(HEC_ERR_INVALID_ARG, "factor and levels differ in size");
        if (which != HEC_LOWER && which != HEC_UPPER && which != HEC_LU) fail(HEC_ERR_INVALID_ARG, "bad `which`");
        if (lv->ras && which != HEC_LU)
            fail(HEC_ERR_INVALID_ARG, "a RAS factor is applied as a whole (HEC_LU): its triangles are over the stacked blocks");
        if (lv->n > 0 && (!b || !x)) fail(HEC_ERR_INVALID_ARG, "b or x is NULL");
        if (b == x && lv->n > 0) fail(HEC_ERR_INVALID_ARG, "b and x must not overlap");
        hipStream_t s = as_stream(stream);
        StreamScope scope(s);
        if (prec == HEC_F64) {
            trsv_launch<double>(*lv, which, (const double *)b, (double *)x, s);
        } else if (prec == HEC_F32) {
            if (!M->has_f32 || (!lv->qL32.get() && lv->n > 0))
                fail(HEC_ERR_INVALID_ARG, "factor has no FP32 copy (HEC_KEEP_F32)");
            trsv_launch<float>(*lv, which, (const float *)b, (float *)x, s);
        } else {
            fail(HEC_ERR_INVALID_ARG, "bad dtype");
        }
    });
}

}  // extern "C"
