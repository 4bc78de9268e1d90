// Algebraic multigrid (Sec. 2.8, Alg. 5): host setup (Ruge-Stueben coarsening,
// direct interpolation, Galerkin coarse operators) and a device V-cycle with
// damped Jacobi smoothing built on the HEC SpMV.
//
// Setup, per level (plain C++ on the host; the same steps, in the same order of
// operations, as a reference implementation can follow by hand):
//  * strength: j strongly influences i when -a_ij >= theta * max_{k!=i}(-a_ik) > 0;
//  * Ruge-Stueben first pass: points with no strong connection either way are F;
//    the undecided point that strongly influences the most undecided points
//    (smallest index on ties) becomes C, the undecided points it strongly
//    influences become F, the undecided points that strongly influence a new F
//    point gain 1, those that strongly influence the new C point lose 1;
//  * direct interpolation ("RSD"): a C point injects its coarse value; an F point
//    i takes w_ij = -alpha_i a_ij / a_ii from its strong negative C neighbours j
//    and w_ij = -beta_i a_ij / a_ii from its strong positive C neighbours (a_ij > 0
//    and a_ij >= theta * the row's largest positive off-diagonal entry; positive
//    couplings play no part in the coarsening), alpha_i, beta_i the ratios of the
//    row's negative (positive) off-diagonal sum to that over those neighbours; with
//    no strong positive C neighbour the positive entries are lumped onto the diagonal;
//  * Galerkin: A_c = P^T A P with R = P^T, (AP)_iJ summed over row i of A in
//    column order, (A_c)_IJ over the fine rows i in ascending order;
// until a level has at most coarse_size rows, max_levels levels exist, or no
// coarsening happens. The coarsest level is solved exactly with its inverse
// (Gauss-Jordan with partial pivoting on the host), applied as a dense SpMV.
//
// Solve: x = 0, then V-cycles (Alg. 5) until ||b - A x|| <= rtol ||b||: nu1
// damped Jacobi sweeps x += omega D^{-1} (b - A x), the residual restricted with
// R, the coarse correction (from zero) prolongated with P and added, nu2 sweeps.
// The other smoother is the Chebyshev polynomial one of Sec. 2.8 ("Chev"), read
// as the Chebyshev semi-iteration on D^{-1} A over [cheb_lower * lmax, lmax] with
// lmax the Gershgorin bound max_i sum_j |a_ij| / |a_ii| (computed on the host per
// level): z = D^{-1} (b - A x), d = z / theta, then per sweep x += d and, before
// the next, z -= D^{-1} A d and d = c1 d + c2 z with the recurrence's coefficients
// (host scalars, the same for every cycle); one product with A per sweep.
// A level whose rows are of about the same length (plain ELL wastes at most 30%
// of its slab) is stored as plain ELL, so that one launch does a whole sweep
// (the residual and the update, into a second vector); other levels keep the
// HEC layout and sweep with an SpMV for the residual and an update. One cycle
// with its residual norm is captured once into a HIP graph on the handle's own
// stream and replayed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <set>
#include <vector>

#include "hec_internal.hpp"

namespace hec {
namespace amgs {

struct Csr {
    int32_t n = 0, m = 0;  // rows, columns
    std::vector<int32_t> p, j;
    std::vector<double> x;
};

#pragma clang fp contract(off)

void strength(const Csr &A, double theta, std::vector<int32_t> &Sp, std::vector<int32_t> &Sj) {
    Sp.assign(1, 0);
    Sj.clear();
    for (int32_t i = 0; i < A.n; ++i) {
        double m = 0.0;
        for (int32_t e = A.p[i]; e < A.p[i + 1]; ++e)
            if (A.j[e] != i) m = std::max(m, -A.x[e]);
        if (m > 0.0)
            for (int32_t e = A.p[i]; e < A.p[i + 1]; ++e)
                if (A.j[e] != i && -A.x[e] >= theta * m) Sj.push_back(A.j[e]);
        Sp.push_back((int32_t)Sj.size());
    }
}

void rs_split(int32_t n, const std::vector<int32_t> &Sp, const std::vector<int32_t> &Sj, std::vector<int8_t> &cf) {
    std::vector<int32_t> Tp(n + 1, 0), Tj(Sj.size());
    for (int32_t j : Sj) Tp[j + 1]++;
    for (int32_t i = 0; i < n; ++i) Tp[i + 1] += Tp[i];
    {
        std::vector<int32_t> fill(Tp.begin(), Tp.end() - 1);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t e = Sp[i]; e < Sp[i + 1]; ++e) Tj[fill[Sj[e]]++] = i;
    }
    enum : int8_t { U = 0, C = 1, F = 2 };
    std::vector<int8_t> state(n, U);
    std::vector<int64_t> lam(n);
    std::set<std::pair<int64_t, int32_t>> q;  // (-lambda, i): the first element is the next C point
    for (int32_t i = 0; i < n; ++i) {
        lam[i] = Tp[i + 1] - Tp[i];
        if (Sp[i + 1] == Sp[i] && Tp[i + 1] == Tp[i])
            state[i] = F;
        else
            q.insert({-lam[i], i});
    }
    auto bump = [&](int32_t k, int64_t d) {
        q.erase({-lam[k], k});
        lam[k] += d;
        q.insert({-lam[k], k});
    };
    while (!q.empty()) {
        const int32_t i = q.begin()->second;
        q.erase(q.begin());
        state[i] = C;
        for (int32_t e = Tp[i]; e < Tp[i + 1]; ++e) {
            const int32_t j = Tj[e];
            if (state[j] != U) continue;
            state[j] = F;
            q.erase({-lam[j], j});
            for (int32_t f = Sp[j]; f < Sp[j + 1]; ++f)
                if (state[Sj[f]] == U) bump(Sj[f], 1);
        }
        for (int32_t e = Sp[i]; e < Sp[i + 1]; ++e)
            if (state[Sj[e]] == U) bump(Sj[e], -1);
    }
    cf.resize(n);
    for (int32_t i = 0; i < n; ++i) cf[i] = state[i] == C ? 1 : 0;
}

Csr direct_interpolation(const Csr &A, const std::vector<int32_t> &Sp, const std::vector<int32_t> &Sj,
                         const std::vector<int8_t> &cf, double theta) {
    const int32_t n = A.n;
    std::vector<int32_t> cidx(n);
    int32_t nc = 0;
    for (int32_t i = 0; i < n; ++i) cidx[i] = cf[i] ? nc++ : -1;
    Csr P;
    P.n = n;
    P.m = nc;
    P.p.assign(1, 0);
    std::vector<int8_t> strong(n, 0);
    for (int32_t i = 0; i < n; ++i) {
        if (cf[i]) {
            P.j.push_back(cidx[i]);
            P.x.push_back(1.0);
            P.p.push_back((int32_t)P.j.size());
            continue;
        }
        for (int32_t e = Sp[i]; e < Sp[i + 1]; ++e) strong[Sj[e]] = 1;  // strong negative couplings
        double mpos = 0.0;                                                 // and strong positive ones
        for (int32_t e = A.p[i]; e < A.p[i + 1]; ++e)
            if (A.j[e] != i && A.x[e] > 0.0) mpos = std::max(mpos, A.x[e]);
        for (int32_t e = A.p[i]; e < A.p[i + 1]; ++e)
            if (A.j[e] != i && A.x[e] > 0.0 && A.x[e] >= theta * mpos) strong[A.j[e]] = 1;
        double aii = 0.0, sneg = 0.0, spos = 0.0, cneg = 0.0, cpos = 0.0;
        for (int32_t e = A.p[i]; e < A.p[i + 1]; ++e) {
            const int32_t j = A.j[e];
            const double v = A.x[e];
            if (j == i) aii = v;
            else if (v < 0) sneg += v;
            else spos += v;
        }
        for (int32_t e = A.p[i]; e < A.p[i + 1]; ++e) {
            const int32_t j = A.j[e];
            if (j == i || !strong[j] || !cf[j]) continue;
            if (A.x[e] < 0) cneg += A.x[e];
            else cpos += A.x[e];
        }
        if (cpos == 0.0) aii += spos;
        const double alpha = cneg != 0.0 ? sneg / cneg : 0.0;
        const double beta = cpos != 0.0 ? spos / cpos : 0.0;
        for (int32_t e = A.p[i]; e < A.p[i + 1]; ++e) {
            const int32_t j = A.j[e];
            if (j == i || !strong[j] || !cf[j]) continue;
            const double v = A.x[e];
            P.j.push_back(cidx[j]);
            P.x.push_back((-(v < 0 ? alpha : beta) * v) / aii);
        }
        P.p.push_back((int32_t)P.j.size());
        for (int32_t e = A.p[i]; e < A.p[i + 1]; ++e) strong[A.j[e]] = 0;
    }
    return P;
}

// Rows of a sparse accumulator: values in touch order, then sorted by column.
struct RowAcc {
    std::vector<double> val;
    std::vector<int32_t> pos;  // column -> slot + 1 (0: untouched)
    std::vector<int32_t> cols;
    explicit RowAcc(int32_t m) : val(m, 0.0), pos(m, 0) {}
    void add(int32_t c, double v) {
        if (!pos[c]) {
            pos[c] = 1;
            cols.push_back(c);
            val[c] = v;
        } else {
            val[c] = val[c] + v;
        }
    }
    void flush(Csr &out) {
        std::sort(cols.begin(), cols.end());
        for (int32_t c : cols) {
            out.j.push_back(c);
            out.x.push_back(val[c]);
            pos[c] = 0;
        }
        cols.clear();
        out.p.push_back((int32_t)out.j.size());
    }
};

Csr transpose(const Csr &P) {
    Csr R;
    R.n = P.m;
    R.m = P.n;
    R.p.assign(P.m + 1, 0);
    for (int32_t c : P.j) R.p[c + 1]++;
    for (int32_t i = 0; i < P.m; ++i) R.p[i + 1] += R.p[i];
    R.j.resize(P.j.size());
    R.x.resize(P.x.size());
    std::vector<int32_t> fill(R.p.begin(), R.p.end() - 1);
    for (int32_t i = 0; i < P.n; ++i)  // fine rows ascending inside every row of R
        for (int32_t e = P.p[i]; e < P.p[i + 1]; ++e) {
            const int32_t d = fill[P.j[e]]++;
            R.j[d] = i;
            R.x[d] = P.x[e];
        }
    return R;
}

Csr galerkin(const Csr &A, const Csr &P, const Csr &R) {
    Csr AP;
    AP.n = A.n;
    AP.m = P.m;
    AP.p.assign(1, 0);
    {
        RowAcc acc(P.m);
        for (int32_t i = 0; i < A.n; ++i) {
            for (int32_t e = A.p[i]; e < A.p[i + 1]; ++e) {
                const int32_t k = A.j[e];
                const double a = A.x[e];
                for (int32_t f = P.p[k]; f < P.p[k + 1]; ++f) acc.add(P.j[f], a * P.x[f]);
            }
            acc.flush(AP);
        }
    }
    Csr Ac;
    Ac.n = Ac.m = P.m;
    Ac.p.assign(1, 0);
    RowAcc acc(P.m);
    for (int32_t I = 0; I < P.m; ++I) {
        for (int32_t e = R.p[I]; e < R.p[I + 1]; ++e) {  // fine rows i ascending
            const int32_t i = R.j[e];
            const double r = R.x[e];
            for (int32_t f = AP.p[i]; f < AP.p[i + 1]; ++f) acc.add(AP.j[f], r * AP.x[f]);
        }
        acc.flush(Ac);
    }
    return Ac;
}

#pragma clang fp contract(on)

// Inverse of a small dense matrix (row-major), Gauss-Jordan with partial pivoting.
// max_i sum_j |a_ij| / |a_ii|, the row sums in column order: Gershgorin's bound on
// the spectral radius of D^{-1} A (every eigenvalue lies within sum_{j != i}
// |a_ij| / |a_ii| of 1 for some row i).
double gershgorin_dinv_a(const Csr &A) {
    double lmax = 0.0;
    for (int32_t i = 0; i < A.n; ++i) {
        double s = 0.0, d = 0.0;
        for (int32_t e = A.p[i]; e < A.p[i + 1]; ++e) {
            s += std::fabs(A.x[e]);
            if (A.j[e] == i) d = A.x[e];
        }
        lmax = std::max(lmax, s / std::fabs(d));
    }
    return lmax;
}

// Coefficients of the Chebyshev smoother on [lo_frac * lmax, lmax] for `degree`
// sweeps: theta, then (c1, c2) of sweeps 2..degree (d = c1 d + c2 z).
void chebyshev_coefficients(double lmax, double lo_frac, int degree, double &theta, std::vector<double> &c1,
                            std::vector<double> &c2) {
    const double hi = lmax, lo = lo_frac * lmax;
    theta = (hi + lo) / 2.0;
    const double delta = (hi - lo) / 2.0;
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    c1.clear();
    c2.clear();
    for (int k = 1; k < degree; ++k) {
        const double rho_new = 1.0 / (2.0 * sigma - rho);
        c1.push_back(rho_new * rho);
        c2.push_back(2.0 * rho_new / delta);
        rho = rho_new;
    }
}

std::vector<double> dense_inverse(const Csr &A) {
    const int32_t n = A.n;
    std::vector<double> a((size_t)n * n, 0.0), inv((size_t)n * n, 0.0);
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t e = A.p[i]; e < A.p[i + 1]; ++e) a[(size_t)i * n + A.j[e]] = A.x[e];
        inv[(size_t)i * n + i] = 1.0;
    }
    for (int32_t c = 0; c < n; ++c) {
        int32_t piv = c;
        for (int32_t r = c + 1; r < n; ++r)
            if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)piv * n + c])) piv = r;
        if (a[(size_t)piv * n + c] == 0.0) fail(HEC_ERR_ZERO_PIVOT, "singular coarsest AMG level");
        if (piv != c)
            for (int32_t k = 0; k < n; ++k) {
                std::swap(a[(size_t)piv * n + k], a[(size_t)c * n + k]);
                std::swap(inv[(size_t)piv * n + k], inv[(size_t)c * n + k]);
            }
        const double d = a[(size_t)c * n + c];
        for (int32_t k = 0; k < n; ++k) {
            a[(size_t)c * n + k] /= d;
            inv[(size_t)c * n + k] /= d;
        }
        for (int32_t r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = a[(size_t)r * n + c];
            if (f == 0.0) continue;
            for (int32_t k = 0; k < n; ++k) {
                a[(size_t)r * n + k] -= f * a[(size_t)c * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
            }
        }
    }
    return inv;
}

}  // namespace amgs

namespace {

// x += omega * dinv * r
__global__ __launch_bounds__(256) void k_jacobi_update(int32_t n, double omega, const double *__restrict__ dinv,
                                                       const double *__restrict__ r, double *__restrict__ x) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += omega * dinv[i] * r[i];
}

// One damped Jacobi sweep on an ELL matrix (slab entry s of row i at s*ld + i):
// xo = xi + omega * dinv * (b - A xi).
__global__ __launch_bounds__(256) void k_jacobi_ell(int32_t n, int32_t K, int32_t ld, const int32_t *__restrict__ col,
                                                    const double *__restrict__ val, const double *__restrict__ dinv,
                                                    double omega, const double *__restrict__ xi,
                                                    const double *__restrict__ b, double *__restrict__ xo) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int32_t s = 0; s < K; ++s) acc += val[(size_t)s * ld + i] * xi[col[(size_t)s * ld + i]];
    xo[i] = xi[i] + omega * dinv[i] * (b[i] - acc);
}

// The first damped Jacobi sweep from x = 0: x = omega * dinv * b (the residual is b).
__global__ __launch_bounds__(256) void k_jacobi_first(int32_t n, double omega, const double *__restrict__ dinv,
                                                      const double *__restrict__ b, double *__restrict__ x) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = omega * dinv[i] * b[i];
}

// First Chebyshev sweep: z = D^{-1} r (r = b - A x, or b from a zero iterate),
// d = z / theta, x += d (x = d from a zero iterate). r may be z.
__global__ __launch_bounds__(256) void k_cheb_first(int32_t n, double theta, const double *__restrict__ dinv,
                                                    const double *r, double *z, double *__restrict__ d,
                                                    double *__restrict__ x, int32_t zero_start) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double zi = dinv[i] * r[i];
    z[i] = zi;
    const double di = zi / theta;
    d[i] = di;
    x[i] = zero_start ? di : x[i] + di;
}

// Later Chebyshev sweeps, with w = A d: z -= D^{-1} w, d = c1 d + c2 z, x += d.
__global__ __launch_bounds__(256) void k_cheb_step(int32_t n, double c1, double c2, const double *__restrict__ dinv,
                                                   const double *__restrict__ w, double *__restrict__ z,
                                                   double *__restrict__ d, double *__restrict__ x) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double zi = z[i] - dinv[i] * w[i];
    z[i] = zi;
    const double di = c1 * d[i] + c2 * zi;
    d[i] = di;
    x[i] += di;
}

__global__ __launch_bounds__(256) void k_copy(int32_t n, const double *__restrict__ a, double *__restrict__ b) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ __launch_bounds__(256) void k_zero(int32_t n, double *__restrict__ x) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

constexpr int kNormBlocks = 256;

// Sum of squares in a fixed order: block b sums rows b, b + 256, ... per thread, a
// fixed tree in the block; the finishing launch adds the 256 block sums in order.
__global__ __launch_bounds__(256) void k_sumsq(int32_t n, const double *__restrict__ v, double *part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s += v[i] * v[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(64) void k_sumsq_finish(const double *part, double *out) {
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < kNormBlocks; ++b) s += part[b];
        *out = s;
    }
}

}  // namespace

}  // namespace hec

using namespace hec;

struct hec_amg_level {
    amgs::Csr A, P;                      // host copies (A_l, and P_l for l < L)
    std::vector<int8_t> cf;              // C/F splitting of this level (l < L)
    std::unique_ptr<hec_matrix_s> dA;    // plain ELL when `fused`, else HEC
    bool fused = false;
    std::unique_ptr<hec_matrix_s> dP, dR;
    DevBuf<double> dinv, x, y, b, r;     // x, y: the iterate and the other buffer of a sweep
    // Chebyshev smoothing: the Gershgorin bound of D^{-1} A, the sweep coefficients for
    // nu1 and nu2 sweeps, and the product A d (the direction d lives in y, z in r)
    double lmax = 0.0, theta = 0.0;
    std::vector<double> c1_pre, c2_pre, c1_post, c2_post;
    DevBuf<double> t;
};

struct hec_amg_s {
    hec_amg_opts opts{};
    std::vector<std::unique_ptr<hec_amg_level>> lev;
    std::unique_ptr<hec_matrix_s> coarse_inv;  // dense inverse of the coarsest level
    DevBuf<double> part, nrm;
    hipStream_t hs = nullptr;                  // the handle's stream (the cycle graph replays on it)
    hipEvent_t ev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~hec_amg_s() {
        if (hs) (void)hipStreamSynchronize(hs);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        lev.clear();
        coarse_inv.reset();
        part.release();
        nrm.release();
        if (ev) (void)hipEventDestroy(ev);
        if (hs) (void)hipStreamDestroy(hs);
    }
};

namespace {

std::unique_ptr<hec_matrix_s> upload(const amgs::Csr &M, int32_t width, hipStream_t s) {
    return make_hec(M.n, M.m, M.p.data(), M.j.data(), M.x.data(), width, 0, s);
}

// y = alpha * M x + beta * z
void spmv(const hec_matrix_s &M, double alpha, const double *x, double beta, const double *z, double *y,
          hipStream_t s) {
    spmv_launch<double, double, double>(M, alpha, x, beta, z, y, s);
}

void sumsq(hec_amg_s &H, int32_t n, const double *v, hipStream_t s) {
    k_sumsq<<<kNormBlocks, 256, 0, s>>>(n, v, H.part.get());
    HEC_CHECK_LAUNCH();
    k_sumsq_finish<<<1, 64, 0, s>>>(H.part.get(), H.nrm.get());
    HEC_CHECK_LAUNCH();
}

double read_norm(hec_amg_s &H, hipStream_t s) {
    double h = 0.0;
    H.nrm.download(&h, 1, s);
    HEC_HIP(hipStreamSynchronize(s));
    return std::sqrt(h);
}

// `sweeps` damped Jacobi sweeps from *cur, alternating between the level's x and y;
// *cur ends on the buffer that holds the result. zero_start: the iterate is zero,
// so the first sweep is x = omega D^{-1} b (one elementwise launch, nothing to zero).
void smooth(hec_amg_level &L, double omega, int sweeps, double *&cur, const double *b, hipStream_t s,
            bool zero_start = false) {
    const hec_matrix_s &M = *L.dA;
    int k = 0;
    if (zero_start && sweeps > 0) {
        k_jacobi_first<<<ceil_div(M.n, 256), 256, 0, s>>>(M.n, omega, L.dinv.get(), b, cur);
        HEC_CHECK_LAUNCH();
        k = 1;
    }
    for (; k < sweeps; ++k) {
        if (!L.fused) {  // r = b - A x, then x += omega D^{-1} r in place
            spmv(M, -1.0, cur, 1.0, b, L.r.get(), s);
            k_jacobi_update<<<ceil_div(M.n, 256), 256, 0, s>>>(M.n, omega, L.dinv.get(), L.r.get(), cur);
            HEC_CHECK_LAUNCH();
            continue;
        }
        double *nxt = cur == L.x.get() ? L.y.get() : L.x.get();
        k_jacobi_ell<<<ceil_div(M.n, 256), 256, 0, s>>>(M.n, M.K, M.ld, M.ell_col.get(), M.ell_val.get(),
                                                       L.dinv.get(), omega, cur, b, nxt);
        HEC_CHECK_LAUNCH();
        cur = nxt;
    }
}

// `sweeps` Chebyshev sweeps on the iterate *cur (which stays where it is; the
// direction goes to the level's other vector, z to r, A d to t). zero_start: the
// iterate is zero, so the first residual is b (no product).
void smooth_cheb(hec_amg_level &L, int sweeps, const std::vector<double> &c1, const std::vector<double> &c2,
                 double *cur, const double *b, hipStream_t s, bool zero_start = false) {
    if (sweeps == 0) return;
    const hec_matrix_s &M = *L.dA;
    const unsigned g = ceil_div(M.n, 256);
    double *d = cur == L.x.get() ? L.y.get() : L.x.get();
    if (!zero_start) spmv(M, -1.0, cur, 1.0, b, L.r.get(), s);  // r = b - A x
    k_cheb_first<<<g, 256, 0, s>>>(M.n, L.theta, L.dinv.get(), zero_start ? b : L.r.get(), L.r.get(), d, cur,
                                   zero_start ? 1 : 0);
    HEC_CHECK_LAUNCH();
    for (int k = 1; k < sweeps; ++k) {
        spmv(M, 1.0, d, 0.0, L.t.get(), L.t.get(), s);  // t = A d
        k_cheb_step<<<g, 256, 0, s>>>(M.n, c1[k - 1], c2[k - 1], L.dinv.get(), L.t.get(), L.r.get(), d, cur);
        HEC_CHECK_LAUNCH();
    }
}

// Alg. 5 from level l (iterate in L.x, right-hand side in L.b); returns the buffer
// holding the result.
double *vcycle(hec_amg_s &H, size_t l, hipStream_t s) {
    hec_amg_level &L = *H.lev[l];
    if (l + 1 == H.lev.size()) {
        spmv(*H.coarse_inv, 1.0, L.b.get(), 0.0, L.b.get(), L.x.get(), s);  // x_L = A_L^{-1} b_L
        return L.x.get();
    }
    const hec_amg_opts &o = H.opts;
    const bool cheb = o.smoother == 1;
    double *cur = L.x.get();
    if (cheb)
        smooth_cheb(L, o.nu1, L.c1_pre, L.c2_pre, cur, L.b.get(), s, l > 0);
    else
        smooth(L, o.omega, o.nu1, cur, L.b.get(), s, l > 0);  // below level 0 the iterate starts at zero
    spmv(*L.dA, -1.0, cur, 1.0, L.b.get(), L.r.get(), s);  // r = b - A x
    hec_amg_level &C = *H.lev[l + 1];
    spmv(*L.dR, 1.0, L.r.get(), 0.0, L.r.get(), C.b.get(), s);  // b_{l+1} = R r
    if (l + 2 < H.lev.size() && o.nu1 == 0) {  // no pre-smoothing to start from zero with
        k_zero<<<ceil_div(C.A.n, 256), 256, 0, s>>>(C.A.n, C.x.get());
        HEC_CHECK_LAUNCH();
    }
    const double *xc = vcycle(H, l + 1, s);
    spmv(*L.dP, 1.0, xc, 1.0, cur, cur, s);  // x += P x_{l+1}
    if (cheb)
        smooth_cheb(L, o.nu2, L.c1_post, L.c2_post, cur, L.b.get(), s);
    else
        smooth(L, o.omega, o.nu2, cur, L.b.get(), s);
    return cur;
}

// One cycle on level 0 ending with the iterate back in x, then ||b - A x||^2 into nrm.
void enqueue_cycle(hec_amg_s &H, hipStream_t s) {
    hec_amg_level &L0 = *H.lev[0];
    const int32_t n = L0.A.n;
    double *res = vcycle(H, 0, s);
    if (res != L0.x.get()) {
        k_copy<<<ceil_div(n, 256), 256, 0, s>>>(n, res, L0.x.get());
        HEC_CHECK_LAUNCH();
    }
    spmv(*L0.dA, -1.0, L0.x.get(), 1.0, L0.b.get(), L0.r.get(), s);
    sumsq(H, n, L0.r.get(), s);
}

}  // namespace

extern "C" {

hec_status amg_setup(int32_t n, const int32_t *Ap, const int32_t *Aj, const double *Ax, const hec_amg_opts *opts,
                     void *stream, hec_amg *out) {
    return guarded([&] {
        if (!out) fail(HEC_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        validate_csr(n, Ap, Aj, Ax);
        if (n == 0) fail(HEC_ERR_INVALID_ARG, "empty matrix");
        hec_amg_opts o{0.25, 8, 64, 2.0 / 3.0, 3, 3, 1, 0, 0.3};
        if (opts) o = *opts;
        if (!(o.theta > 0.0 && o.theta <= 1.0) || o.max_levels < 1 || o.max_levels > 32 || o.coarse_size < 1 ||
            o.coarse_size > 4096 || !(o.omega > 0.0 && o.omega < 2.0) || o.nu1 < 0 || o.nu2 < 0 || o.nu1 > 64 ||
            o.nu2 > 64 || (o.use_graph != 0 && o.use_graph != 1) || (o.smoother != 0 && o.smoother != 1) ||
            !(o.cheb_lower > 0.0 && o.cheb_lower < 1.0))
            fail(HEC_ERR_INVALID_ARG, "bad AMG options");
        hipStream_t s = as_stream(stream);
        StreamScope scope(s);
        auto H = std::make_unique<hec_amg_s>();
        H->opts = o;
        amgs::Csr A;
        A.n = A.m = n;
        A.p.assign(Ap, Ap + n + 1);
        A.j.assign(Aj, Aj + Ap[n]);
        A.x.assign(Ax, Ax + Ap[n]);
        for (;;) {
            auto L = std::make_unique<hec_amg_level>();
            L->A = std::move(A);
            const int32_t nl = L->A.n;
            std::vector<double> dinv(nl, 0.0);
            for (int32_t i = 0; i < nl; ++i) {
                for (int32_t e = L->A.p[i]; e < L->A.p[i + 1]; ++e)
                    if (L->A.j[e] == i) dinv[i] = 1.0 / L->A.x[e];
                if (dinv[i] == 0.0 || !std::isfinite(dinv[i]))
                    fail(HEC_ERR_ZERO_PIVOT, "AMG level " + std::to_string(H->lev.size()) + ": zero or missing diagonal in row " + std::to_string(i));
            }
            int32_t width = 0;
            for (int32_t i = 0; i < nl; ++i) width = std::max(width, L->A.p[i + 1] - L->A.p[i]);
            L->fused = (double)width * nl <= 1.3 * (double)L->A.p[nl];
            L->dA = upload(L->A, L->fused ? width : -1, s);
            L->dinv.alloc(nl);
            L->dinv.upload(dinv.data(), nl, s);
            L->x.alloc(nl);
            L->y.alloc(nl);
            L->b.alloc(nl);
            L->r.alloc(nl);
            if (o.smoother == 1) {
                L->lmax = amgs::gershgorin_dinv_a(L->A);
                amgs::chebyshev_coefficients(L->lmax, o.cheb_lower, o.nu1, L->theta, L->c1_pre, L->c2_pre);
                amgs::chebyshev_coefficients(L->lmax, o.cheb_lower, o.nu2, L->theta, L->c1_post, L->c2_post);
                L->t.alloc(nl);
            }
            const bool last = nl <= o.coarse_size || (int32_t)H->lev.size() + 1 == o.max_levels;
            amgs::Csr Ac;
            if (!last) {
                std::vector<int32_t> Sp, Sj;
                amgs::strength(L->A, o.theta, Sp, Sj);
                amgs::rs_split(nl, Sp, Sj, L->cf);
                int32_t nc = 0;
                for (int8_t c : L->cf) nc += c;
                if (nc > 0 && nc < nl) {
                    L->P = amgs::direct_interpolation(L->A, Sp, Sj, L->cf, o.theta);
                    amgs::Csr R = amgs::transpose(L->P);
                    Ac = amgs::galerkin(L->A, L->P, R);
                    L->dP = upload(L->P, -1, s);
                    L->dR = upload(R, -1, s);
                } else {
                    L->cf.clear();
                }
            }
            const bool more = !L->P.p.empty();
            H->lev.push_back(std::move(L));
            if (!more) break;
            A = std::move(Ac);
            HEC_HIP(hipStreamSynchronize(s));  // host arrays of the uploads end with this iteration
        }
        // the coarsest level: its dense inverse as a matrix
        const amgs::Csr &Lc = H->lev.back()->A;
        std::vector<double> inv = amgs::dense_inverse(Lc);
        const int32_t nc = Lc.n;
        std::vector<int32_t> ip(nc + 1), ij((size_t)nc * nc);
        for (int32_t i = 0; i <= nc; ++i) ip[i] = i * nc;
        for (size_t e = 0; e < ij.size(); ++e) ij[e] = (int32_t)(e % nc);
        H->coarse_inv = make_hec(nc, nc, ip.data(), ij.data(), inv.data(), -1, 0, s);
        H->part.alloc(kNormBlocks);
        H->nrm.alloc(1);
        HEC_HIP(hipStreamSynchronize(s));
        HEC_HIP(hipStreamCreateWithFlags(&H->hs, hipStreamNonBlocking));
        HEC_HIP(hipEventCreateWithFlags(&H->ev, hipEventDisableTiming));
        *out = H.release();
    });
}

hec_status amg_info(hec_amg H, int32_t *nlevels, int32_t *n, int64_t *nnz, int64_t *nnz_p) {
    return guarded([&] {
        if (!H) fail(HEC_ERR_INVALID_ARG, "null AMG handle");
        if (nlevels) *nlevels = (int32_t)H->lev.size();
        for (size_t l = 0; l < H->lev.size(); ++l) {
            const hec_amg_level &L = *H->lev[l];
            if (n) n[l] = L.A.n;
            if (nnz) nnz[l] = L.A.p.back();
            if (nnz_p) nnz_p[l] = L.P.p.empty() ? 0 : L.P.p.back();
        }
    });
}

hec_status amg_export_level(hec_amg H, int32_t level, int8_t *cf, int32_t *Ap, int32_t *Aj, double *Ax,
                            int32_t *Pp, int32_t *Pj, double *Px) {
    return guarded([&] {
        if (!H) fail(HEC_ERR_INVALID_ARG, "null AMG handle");
        if (level < 0 || level >= (int32_t)H->lev.size()) fail(HEC_ERR_INVALID_ARG, "level out of range");
        const hec_amg_level &L = *H->lev[level];
        if (Ap) std::copy(L.A.p.begin(), L.A.p.end(), Ap);
        if (Aj) std::copy(L.A.j.begin(), L.A.j.end(), Aj);
        if (Ax) std::copy(L.A.x.begin(), L.A.x.end(), Ax);
        if (cf) std::copy(L.cf.begin(), L.cf.end(), cf);
        if (Pp) std::copy(L.P.p.begin(), L.P.p.end(), Pp);
        if (Pj) std::copy(L.P.j.begin(), L.P.j.end(), Pj);
        if (Px) std::copy(L.P.x.begin(), L.P.x.end(), Px);
    });
}

hec_status amg_solve(hec_amg H, const double *b, double *x, int32_t maxit, double rtol, void *stream,
                     hec_solve_info *info) {
    return guarded([&] {
        if (!H) fail(HEC_ERR_INVALID_ARG, "null AMG handle");
        if (!b || !x) fail(HEC_ERR_INVALID_ARG, "b or x is NULL");
        if (b == x) fail(HEC_ERR_INVALID_ARG, "b and x must not overlap");
        if (maxit < 0 || !(rtol >= 0.0)) fail(HEC_ERR_INVALID_ARG, "bad maxit or rtol");
        const auto t0 = std::chrono::steady_clock::now();
        hipStream_t us = as_stream(stream), s = H->hs;
        StreamScope scope(s);
        HEC_HIP(hipEventRecord(H->ev, us));  // after the caller's work on b and x
        HEC_HIP(hipStreamWaitEvent(s, H->ev, 0));
        hec_amg_level &L0 = *H->lev[0];
        const int32_t n = L0.A.n;
        HEC_HIP(hipMemcpyAsync(L0.b.get(), b, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
        k_zero<<<ceil_div(n, 256), 256, 0, s>>>(n, L0.x.get());
        HEC_CHECK_LAUNCH();
        sumsq(*H, n, L0.b.get(), s);
        const double nb = read_norm(*H, s);
        int32_t it = 0;
        double res = nb > 0.0 ? 1.0 : 0.0;
        hec_status st = HEC_OK;
        if (nb > 0.0) {
            st = HEC_ERR_NOT_CONVERGED;
            if (H->opts.use_graph && !H->exec && maxit > 0) {
                HEC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                try {
                    enqueue_cycle(*H, s);
                } catch (...) {
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(s, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                HEC_HIP(hipStreamEndCapture(s, &H->graph));
                HEC_HIP(hipGraphInstantiate(&H->exec, H->graph, nullptr, nullptr, 0));
            }
            while (it < maxit) {
                if (H->opts.use_graph)
                    HEC_HIP(hipGraphLaunch(H->exec, s));
                else
                    enqueue_cycle(*H, s);
                ++it;
                res = read_norm(*H, s) / nb;
                if (!std::isfinite(res)) {
                    st = HEC_ERR_BREAKDOWN;
                    break;
                }
                if (res <= rtol) {
                    st = HEC_OK;
                    break;
                }
            }
        }
        HEC_HIP(hipMemcpyAsync(x, L0.x.get(), (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
        HEC_HIP(hipEventRecord(H->ev, s));
        HEC_HIP(hipStreamWaitEvent(us, H->ev, 0));  // the caller's later work sees x
        HEC_HIP(hipStreamSynchronize(s));
        if (info) {
            *info = hec_solve_info{};
            info->status = st;
            info->iterations = it;
            info->rel_res_true = res;
            info->rel_res_est = res;
            info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        if (st == HEC_ERR_BREAKDOWN) fail(st, "AMG iteration produced a non-finite residual");
        if (st == HEC_ERR_NOT_CONVERGED) fail(st, "AMG did not reach the tolerance");
    });
}

hec_status amg_destroy(hec_amg H) {
    delete H;
    return HEC_OK;
}

}  // extern "C"
