/*
 * FP64 CPU oracle for the HEC / ILU(k) / level-schedule / Krylov path.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
 * GPU library is checked against. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never calls it.
 * It shares no code with the GPU library.
 *
 * Everything is sequential double precision, built with -O3 -ffp-contract=off
 * so that every product and sum is rounded exactly as written. Each function
 * names the passage of the paper (Yang, Liu, Chen, "Development of Krylov and
 * AMG linear solvers for large-scale sparse matrices on GPUs") that it follows.
 *
 * Conventions: CSR arrays Ap (row starts, n+1), Aj (column indices, strictly
 * ascending within a row), Ax (values), as named in Sec. 2.1. 0-based indices.
 * Return codes: 0 ok, 1 invalid argument, 2 out of memory, 3 zero pivot,
 * 4 breakdown, 5 not converged.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OK = 0, ORC_INVALID = 1, ORC_NOMEM = 2, ORC_ZERO_PIVOT = 3,
       ORC_BREAKDOWN = 4, ORC_NOT_CONVERGED = 5 };

void orc_free(void *p) { free(p); }

/* ------------------------------------------------------------------------ */
/* Sec. 2.2 Alg. 1 / Eq. (2): y = alpha*A*x + beta*y, one row at a time,
 * the row's terms summed in stored (ascending column) order. When beta == 0,
 * y is not read (so an uninitialised y is allowed). */
static inline void csr_row(int i, const int *Ap, const int *Aj, const double *Ax,
                           double alpha, const double *x, double beta, double *y)
{
    double t = 0.0;
    for (int e = Ap[i]; e < Ap[i + 1]; ++e)
        t += Ax[e] * x[Aj[e]];
    if (beta == 0.0)
        y[i] = alpha * t;
    else
        y[i] = alpha * t + beta * y[i];
}

void orc_csr_spmv(int n, const int *Ap, const int *Aj, const double *Ax,
                  double alpha, const double *x, double beta, double *y)
{
    for (int i = 0; i < n; ++i)
        csr_row(i, Ap, Aj, Ax, alpha, x, beta, y);
}

/* The same product with the rows shared among `nthreads` OpenMP threads (static
 * schedule). Every row is summed exactly as above, so the result is identical
 * bit for bit; this is the all-cores CPU figure that the benchmark reports beside
 * the single-threaded one, and nothing else in the oracle runs threaded. */
void orc_csr_spmv_omp(int n, const int *Ap, const int *Aj, const double *Ax,
                      double alpha, const double *x, double beta, double *y, int nthreads)
{
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int i = 0; i < n; ++i)
        csr_row(i, Ap, Aj, Ax, alpha, x, beta, y);
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.1: HEC = a regular ELL part stored column by column (Eq. (1): the
 * product is a sum of scaled columns), with a leading dimension that is a
 * multiple of the warp width (the paper uses 256), plus the irregular rest of
 * each row in CSR. The boundary between the two parts is the ELL width; the
 * paper's recommended value is 20.
 *
 * Readings: K = ell_width if ell_width >= 0, else min(20, longest row), and
 * never more than the longest row; ld = n rounded up to a multiple of 256;
 * the first K entries of a row (ascending column) go to ELL slot s = 0..K-1 at
 * position s*ld + i, the rest to the CSR remainder in order. Empty ELL slots of
 * a real row hold value 0 and column i; rows n..ld-1 hold value 0, column 0. */
void orc_hec_sizes(int n, const int *Ap, int ell_width, int *K, int *ld, long *nnz_rem)
{
    int maxrow = 0;
    for (int i = 0; i < n; ++i) {
        int len = Ap[i + 1] - Ap[i];
        if (len > maxrow) maxrow = len;
    }
    int k = ell_width >= 0 ? ell_width : 20;
    if (k > maxrow) k = maxrow;
    long rem = 0;
    for (int i = 0; i < n; ++i) {
        int len = Ap[i + 1] - Ap[i];
        if (len > k) rem += len - k;
    }
    *K = k;
    *ld = ((n + 255) / 256) * 256;
    *nnz_rem = rem;
}

void orc_hec_fill(int n, const int *Ap, const int *Aj, const double *Ax, int K, int ld,
                  int *ell_col, double *ell_val, int *rem_ptr, int *rem_col, double *rem_val)
{
    for (int s = 0; s < K; ++s) {
        for (int i = 0; i < ld; ++i) {
            long slot = (long)s * ld + i;
            if (i < n && Ap[i] + s < Ap[i + 1]) {
                ell_col[slot] = Aj[Ap[i] + s];
                ell_val[slot] = Ax[Ap[i] + s];
            } else if (i < n) {
                ell_col[slot] = i;
                ell_val[slot] = 0.0;
            } else {
                ell_col[slot] = 0;
                ell_val[slot] = 0.0;
            }
        }
    }
    int r = 0;
    rem_ptr[0] = 0;
    for (int i = 0; i < n; ++i) {
        for (int e = Ap[i] + K; e < Ap[i + 1]; ++e) {
            rem_col[r] = Aj[e];
            rem_val[r] = Ax[e];
            ++r;
        }
        rem_ptr[i + 1] = r;
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.4, Eq. (7)-(10), Alg. 2: ILU(k) with L and U stored in place of A.
 *
 * Each row i is copied into a working row; the entries of A get level 0
 * (Eq. (9)). Pivots p < i are visited in increasing column order, and only
 * those whose level is <= k are used (Alg. 2's condition on L_ip): the
 * multiplier a_ip = a_ip / a_pp is formed, then for every stored entry (p, j),
 * j > p, of the already factored row p, a_ij -= a_ip * a_pj and the level is
 * updated as L_ij = min(L_ij, L_ip + L_pj + 1) (Eq. (10)); a column that was
 * not yet present enters with value 0 and level infinity. Finally every entry of
 * row i with level > k is dropped. This is the paper's algorithm with the drop
 * step applied per row (reading of the garbled Alg. 2; levels of the entries
 * left of the diagonal are final before they are used as pivots because a
 * pivot p only updates columns j > p).
 *
 * Output: the factored rows in CSR (LUp, LUj, LUx, and each kept entry's level
 * in LUlev), allocated here and released with orc_free. L is the strict lower
 * part (unit diagonal implied), U the upper part with the diagonal.
 * A zero pivot (u_ii == 0 exactly, whether or not a later row uses it)
 * returns ORC_ZERO_PIVOT; a missing diagonal returns ORC_INVALID. */
int orc_iluk(int n, const int *Ap, const int *Aj, const double *Ax, int k,
             int **LUp_out, int **LUj_out, double **LUx_out, int **LUlev_out)
{
    const int INF = 0x3fffffff;
    int *LUp = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int *lev = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *next = (int *)malloc(sizeof(int) * (size_t)(n + 1)); /* sorted linked list of the working row */
    int *diag = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    size_t cap = (size_t)(Ap[n] > 16 ? Ap[n] : 16);
    int *LUj = (int *)malloc(sizeof(int) * cap);
    double *LUx = (double *)malloc(sizeof(double) * cap);
    int *LUlev = (int *)malloc(sizeof(int) * cap);
    if (!LUp || !w || !lev || !next || !diag || !LUj || !LUx || !LUlev) {
        free(LUp); free(w); free(lev); free(next); free(diag); free(LUj); free(LUx); free(LUlev);
        return ORC_NOMEM;
    }
    const int HEAD = n; /* list head sentinel index; list ends with -1 */
    size_t nz = 0;
    LUp[0] = 0;
    int status = ORC_OK;
    for (int i = 0; i < n && status == ORC_OK; ++i) {
        /* load row i of A: values and level 0 */
        next[HEAD] = -1;
        int tail = HEAD;
        int has_diag = 0;
        for (int e = Ap[i]; e < Ap[i + 1]; ++e) {
            int j = Aj[e];
            w[j] = Ax[e];
            lev[j] = 0;
            next[tail] = j;
            next[j] = -1;
            tail = j;
            if (j == i) has_diag = 1;
        }
        if (!has_diag) { status = ORC_INVALID; break; }
        /* eliminate with pivots p < i in increasing order */
        for (int p = next[HEAD]; p != -1 && p < i; p = next[p]) {
            if (lev[p] > k) continue;
            double upp = LUx[diag[p]];
            if (upp == 0.0) { status = ORC_ZERO_PIVOT; break; }
            w[p] = w[p] / upp;
            int ins = p; /* the list position after which column j may be inserted */
            for (int e = diag[p] + 1; e < LUp[p + 1]; ++e) {
                int j = LUj[e];
                /* find j in the sorted list starting from ins */
                while (next[ins] != -1 && next[ins] < j) ins = next[ins];
                if (next[ins] != j) {
                    int nx = next[ins];
                    next[ins] = j;
                    next[j] = nx;
                    w[j] = 0.0;
                    lev[j] = INF;
                }
                ins = j;
                w[j] = w[j] - w[p] * LUx[e];
                int cand = lev[p] + LUlev[e] + 1;
                if (cand < lev[j]) lev[j] = cand;
            }
        }
        if (status != ORC_OK) break;
        /* drop entries whose level exceeds k, store the row */
        for (int j = next[HEAD]; j != -1; j = next[j]) {
            if (lev[j] > k) continue;
            if (nz == cap) {
                cap *= 2;
                int *a = (int *)realloc(LUj, sizeof(int) * cap);
                if (a) LUj = a;
                double *b = (double *)realloc(LUx, sizeof(double) * cap);
                if (b) LUx = b;
                int *c = (int *)realloc(LUlev, sizeof(int) * cap);
                if (c) LUlev = c;
                if (!a || !b || !c) { status = ORC_NOMEM; break; }
            }
            if (j == i) diag[i] = (int)nz;
            LUj[nz] = j;
            LUx[nz] = w[j];
            LUlev[nz] = lev[j];
            ++nz;
        }
        LUp[i + 1] = (int)nz;
        /* U_ii is the divisor of the backward substitution: a zero pivot is an
         * error even in a row that no later row eliminates with */
        if (status == ORC_OK && LUx[diag[i]] == 0.0) status = ORC_ZERO_PIVOT;
    }
    free(w); free(lev); free(next); free(diag);
    if (status != ORC_OK) {
        free(LUp); free(LUj); free(LUx); free(LUlev);
        return status;
    }
    *LUp_out = LUp; *LUj_out = LUj; *LUx_out = LUx; *LUlev_out = LUlev;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.6, Eq. (11), Alg. 3: level schedule of a triangular factor.
 *
 * Lower (which == 0): l(i) = 1 + max l(j) over the stored entries j < i of row
 * i, with l initialised to 0 (a row with no such entry gets level 1).
 * Upper (which == 1): the mirrored definition, rows visited from n-1 down to 0
 * and j > i. Levels are returned 0-based in lev[]. The rows are then grouped
 * level by level (Alg. 3's level(k) start pointers): level_ptr[nlev+1] and
 * perm[n] = rows ordered by (level, row index), by a stable counting sort.
 * level_ptr must hold n+1 entries. Returns nlev. */
int orc_level_schedule(int n, const int *Lp, const int *Lj, int which,
                       int *lev, int *level_ptr, int *perm)
{
    int nlev = 0;
    for (int t = 0; t < n; ++t) {
        int i = which == 0 ? t : n - 1 - t;
        int l = 0;
        for (int e = Lp[i]; e < Lp[i + 1]; ++e) {
            int j = Lj[e];
            if ((which == 0 && j < i) || (which == 1 && j > i)) {
                if (lev[j] + 1 > l) l = lev[j] + 1;
            }
        }
        /* 1 + max over dependencies, stored 0-based: a free row is level 0 */
        lev[i] = l;
        if (l + 1 > nlev) nlev = l + 1;
    }
    for (int q = 0; q <= nlev; ++q) level_ptr[q] = 0;
    for (int i = 0; i < n; ++i) level_ptr[lev[i] + 1]++;
    for (int q = 0; q < nlev; ++q) level_ptr[q + 1] += level_ptr[q];
    int *fill = (int *)malloc(sizeof(int) * (size_t)(nlev > 0 ? nlev : 1));
    for (int q = 0; q < nlev; ++q) fill[q] = level_ptr[q];
    for (int i = 0; i < n; ++i) perm[fill[lev[i]]++] = i;
    free(fill);
    return nlev;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.6: triangular solves with the in-place factor of Sec. 2.4.
 * Forward: y_i = b_i - sum_{j<i} L_ij y_j (unit diagonal), i = 0..n-1.
 * Backward: x_i = (y_i - sum_{j>i} U_ij x_j) / U_ii, i = n-1..0.
 * Terms in ascending column order; division by the pivot. x may alias b. */
void orc_trsv_lower(int n, const int *LUp, const int *LUj, const double *LUx,
                    const double *b, double *y)
{
    for (int i = 0; i < n; ++i) {
        double t = b[i];
        for (int e = LUp[i]; e < LUp[i + 1]; ++e) {
            int j = LUj[e];
            if (j < i) t = t - LUx[e] * y[j];
        }
        y[i] = t;
    }
}

void orc_trsv_upper(int n, const int *LUp, const int *LUj, const double *LUx,
                    const double *y, double *x)
{
    for (int i = n - 1; i >= 0; --i) {
        double t = y[i];
        double d = 0.0;
        for (int e = LUp[i]; e < LUp[i + 1]; ++e) {
            int j = LUj[e];
            if (j > i) t = t - LUx[e] * x[j];
            else if (j == i) d = LUx[e];
        }
        x[i] = t / d;
    }
}

/* M^{-1} r = U^{-1} L^{-1} r (Eq. (7)-(8)) */
static void apply_prec(int n, const int *LUp, const int *LUj, const double *LUx,
                       const double *r, double *z, double *tmp)
{
    orc_trsv_lower(n, LUp, LUj, LUx, r, tmp);
    orc_trsv_upper(n, LUp, LUj, LUx, tmp, z);
}

/* Sec. 2.3 Eq. (5)-(6) */
static double dot(int n, const double *x, const double *y)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

static double nrm2(int n, const double *x) { return sqrt(dot(n, x, x)); }

/* true residual r = b - A x (Alg. 4 first line), returns ||r|| */
static double residual(int n, const int *Ap, const int *Aj, const double *Ax,
                       const double *b, const double *x, double *r)
{
    for (int i = 0; i < n; ++i) r[i] = b[i];
    orc_csr_spmv(n, Ap, Aj, Ax, -1.0, x, 1.0, r);
    return nrm2(n, r);
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.7: restarted GMRES(m), right-preconditioned with M = LU.
 *
 * The paper names GMRES and refers to Saad's textbook for the algorithm. One
 * cycle: r = b - A x, beta = ||r||, v_1 = r / beta, g = beta e_1. For j = 1..m:
 * z_j = M^{-1} v_j, w = A z_j; modified Gram-Schmidt h_ij = <w, v_i>,
 * w -= h_ij v_i (i = 1..j); h_{j+1,j} = ||w||; the earlier Givens rotations are
 * applied to column j, a new rotation (c, s) = (h_jj, h_{j+1,j}) / hypot(...)
 * zeroes h_{j+1,j} and is applied to g. The cycle stops when
 * |g_{j+1}| / ||b|| <= rtol or h_{j+1,j} == 0; then H y = g is back-solved and
 * x += M^{-1} (V y). The true residual decides convergence, otherwise the
 * method restarts from x. iters counts Arnoldi steps; maxit bounds them.
 * LU is the in-place factor (L strict lower, U upper with diagonal).
 *
 * Optional outputs of the last cycle (NULL to skip), for checking the Arnoldi
 * relation A M^{-1} V_j = V_{j+1} Hbar_j: V_out gets the basis vectors computed
 * in it, (m+1) x n, vector i at V_out + i*n; Hbar_out the (m+1) x m Hessenberg
 * matrix as Gram-Schmidt produced it, before the rotations (row i, column j at
 * Hbar_out[i*m + j]); steps_out the number of its Arnoldi steps. */
int orc_gmres(int n, const int *Ap, const int *Aj, const double *Ax,
              const int *LUp, const int *LUj, const double *LUx,
              const double *b, double *x, int m, int maxit, double rtol,
              int *iters_out, double *relres_out,
              double *V_out, double *Hbar_out, int *steps_out)
{
    *iters_out = 0;
    double bnorm = nrm2(n, b);
    if (bnorm == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        *relres_out = 0.0;
        return ORC_OK;
    }
    if (m < 1) return ORC_INVALID;
    size_t N = (size_t)(n > 0 ? n : 1);
    double *V = (double *)malloc(sizeof(double) * N * (size_t)(m + 1));
    double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double)); /* H[i*m + j] */
    double *cs = (double *)malloc(sizeof(double) * (size_t)m);
    double *sn = (double *)malloc(sizeof(double) * (size_t)m);
    double *g = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *yv = (double *)malloc(sizeof(double) * (size_t)m);
    double *r = (double *)malloc(sizeof(double) * N);
    double *z = (double *)malloc(sizeof(double) * N);
    double *w = (double *)malloc(sizeof(double) * N);
    double *tmp = (double *)malloc(sizeof(double) * N);
    if (!V || !H || !cs || !sn || !g || !yv || !r || !z || !w || !tmp) {
        free(V); free(H); free(cs); free(sn); free(g); free(yv); free(r); free(z); free(w); free(tmp);
        return ORC_NOMEM;
    }
    int status = ORC_NOT_CONVERGED;
    int it = 0;
    double relres = residual(n, Ap, Aj, Ax, b, x, r) / bnorm;
    while (relres > rtol && it < maxit) {
        double beta = nrm2(n, r);
        for (int i = 0; i < n; ++i) V[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        if (Hbar_out)
            for (int i = 0; i < (m + 1) * m; ++i) Hbar_out[i] = 0.0;
        int jdone = 0, vdone = 1;
        for (int j = 0; j < m && it < maxit; ++j) {
            double *vj = V + (size_t)j * N;
            apply_prec(n, LUp, LUj, LUx, vj, z, tmp);
            orc_csr_spmv(n, Ap, Aj, Ax, 1.0, z, 0.0, w);
            for (int i = 0; i <= j; ++i) {
                double *vi = V + (size_t)i * N;
                double h = dot(n, w, vi);
                H[i * m + j] = h;
                for (int q = 0; q < n; ++q) w[q] = w[q] - h * vi[q];
            }
            double hn = nrm2(n, w);
            H[(j + 1) * m + j] = hn;
            if (Hbar_out)
                for (int i = 0; i <= j + 1; ++i) Hbar_out[i * m + j] = H[i * m + j];
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], c = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[j * m + j], c = H[(j + 1) * m + j];
            double rr = hypot(a, c);
            if (c == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
            else { cs[j] = a / rr; sn[j] = c / rr; }
            H[j * m + j] = cs[j] * a + sn[j] * c;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            jdone = j + 1;
            if (fabs(g[j + 1]) / bnorm <= rtol || hn == 0.0) break;
            double *vn = V + (size_t)(j + 1) * N;
            for (int q = 0; q < n; ++q) vn[q] = w[q] / hn;
            vdone = j + 2;
        }
        if (V_out) memcpy(V_out, V, sizeof(double) * (size_t)n * (size_t)vdone);
        if (steps_out) *steps_out = jdone;
        /* back-solve the triangular H y = g */
        for (int i = jdone - 1; i >= 0; --i) {
            double t = g[i];
            for (int q = i + 1; q < jdone; ++q) t = t - H[i * m + q] * yv[q];
            yv[i] = t / H[i * m + i];
        }
        for (int q = 0; q < n; ++q) w[q] = 0.0;
        for (int i = 0; i < jdone; ++i) {
            double *vi = V + (size_t)i * N;
            for (int q = 0; q < n; ++q) w[q] = w[q] + yv[i] * vi[q];
        }
        apply_prec(n, LUp, LUj, LUx, w, z, tmp);
        for (int q = 0; q < n; ++q) x[q] = x[q] + z[q];
        relres = residual(n, Ap, Aj, Ax, b, x, r) / bnorm;
    }
    if (relres <= rtol) status = ORC_OK;
    *iters_out = it;
    *relres_out = relres;
    free(V); free(H); free(cs); free(sn); free(g); free(yv); free(r); free(z); free(w); free(tmp);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.7, Alg. 4: preconditioned BiCGSTAB, step by step in the paper's
 * notation (r0 = shadow residual = the initial residual, p*, s* = M^{-1} p,
 * M^{-1} s). "||s|| is satisfied" is read as ||s|| / ||b|| <= rtol, likewise for
 * ||r||. rho == 0 or (r0, v) == 0 is a breakdown; omega == 0 stops. After the
 * recurrence stops, the true residual b - A x decides; if it is not below rtol
 * the method restarts from x (new r0), at most 3 times, within maxit passes of
 * the loop. iters counts loop passes (2 products each); restarts_out (may be
 * NULL) the cycles started after the first. */
int orc_bicgstab(int n, const int *Ap, const int *Aj, const double *Ax,
                 const int *LUp, const int *LUj, const double *LUx,
                 const double *b, double *x, int maxit, double rtol,
                 int *iters_out, double *relres_out, int *restarts_out)
{
    *iters_out = 0;
    if (restarts_out) *restarts_out = 0;
    double bnorm = nrm2(n, b);
    if (bnorm == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        *relres_out = 0.0;
        return ORC_OK;
    }
    size_t N = (size_t)(n > 0 ? n : 1);
    double *r0 = (double *)malloc(sizeof(double) * N);
    double *r = (double *)malloc(sizeof(double) * N);
    double *p = (double *)malloc(sizeof(double) * N);
    double *ps = (double *)malloc(sizeof(double) * N);
    double *v = (double *)malloc(sizeof(double) * N);
    double *s = (double *)malloc(sizeof(double) * N);
    double *ss = (double *)malloc(sizeof(double) * N);
    double *t = (double *)malloc(sizeof(double) * N);
    double *tmp = (double *)malloc(sizeof(double) * N);
    if (!r0 || !r || !p || !ps || !v || !s || !ss || !t || !tmp) {
        free(r0); free(r); free(p); free(ps); free(v); free(s); free(ss); free(t); free(tmp);
        return ORC_NOMEM;
    }
    int it = 0, status = ORC_NOT_CONVERGED;
    double relres = residual(n, Ap, Aj, Ax, b, x, r) / bnorm;
    int cycles = 0;
    int broke = 0;
    while (relres > rtol && it < maxit && cycles < 4) {
        ++cycles;
        /* r0 = b - A x0 */
        for (int i = 0; i < n; ++i) r0[i] = r[i];
        double rho_prev = 0.0, alpha = 0.0, omega = 0.0;
        broke = 0;
        for (int k = 1; it < maxit; ++k) {
            double rho = dot(n, r0, r);
            if (rho == 0.0 || !isfinite(rho)) { broke = 1; break; }
            if (k == 1) {
                for (int i = 0; i < n; ++i) p[i] = r[i];
            } else {
                double beta = (rho / rho_prev) * (alpha / omega);
                for (int i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            }
            apply_prec(n, LUp, LUj, LUx, p, ps, tmp);
            orc_csr_spmv(n, Ap, Aj, Ax, 1.0, ps, 0.0, v);
            double r0v = dot(n, r0, v);
            if (r0v == 0.0 || !isfinite(r0v)) { broke = 1; break; }
            alpha = rho / r0v;
            for (int i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
            ++it;
            if (nrm2(n, s) / bnorm <= rtol) {
                for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * ps[i];
                break;
            }
            apply_prec(n, LUp, LUj, LUx, s, ss, tmp);
            orc_csr_spmv(n, Ap, Aj, Ax, 1.0, ss, 0.0, t);
            double tt = dot(n, t, t);
            omega = tt == 0.0 ? 0.0 : dot(n, t, s) / tt;
            for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * ps[i] + omega * ss[i];
            for (int i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
            if (nrm2(n, r) / bnorm <= rtol || omega == 0.0) break;
            rho_prev = rho;
        }
        relres = residual(n, Ap, Aj, Ax, b, x, r) / bnorm;
    }
    if (relres <= rtol) status = ORC_OK;
    else if (broke) status = ORC_BREAKDOWN;
    *iters_out = it;
    *relres_out = relres;
    if (restarts_out) *restarts_out = cycles > 0 ? cycles - 1 : 0;
    free(r0); free(r); free(p); free(ps); free(v); free(s); free(ss); free(t); free(tmp);
    return status;
}

/* Sec. 2.7 names CG among the implemented Krylov solvers (its steps are the
 * textbook preconditioned conjugate gradient the paper defers to): with
 * r = b - A x, z = M^{-1} r, p = z, rho = (r, z), repeat: q = A p,
 * alpha = rho / (p, q), x += alpha p, r -= alpha q, stop when ||r|| / ||b|| <=
 * rtol, z = M^{-1} r, rho' = (r, z), p = z + (rho'/rho) p. M = LU must be
 * symmetric positive definite (an ILU(k) of an SPD M-matrix with a symmetric
 * pattern is). rho <= 0 or (p, q) <= 0 (or non-finite) is a breakdown. After the
 * recurrence stops the true residual decides; if it is above rtol the method
 * restarts from x, at most 3 times, within maxit iterations. */
int orc_cg(int n, const int *Ap, const int *Aj, const double *Ax,
           const int *LUp, const int *LUj, const double *LUx,
           const double *b, double *x, int maxit, double rtol,
           int *iters_out, double *relres_out)
{
    *iters_out = 0;
    double bnorm = nrm2(n, b);
    if (bnorm == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        *relres_out = 0.0;
        return ORC_OK;
    }
    size_t N = (size_t)(n > 0 ? n : 1);
    double *r = (double *)malloc(sizeof(double) * N);
    double *z = (double *)malloc(sizeof(double) * N);
    double *p = (double *)malloc(sizeof(double) * N);
    double *q = (double *)malloc(sizeof(double) * N);
    double *tmp = (double *)malloc(sizeof(double) * N);
    if (!r || !z || !p || !q || !tmp) {
        free(r); free(z); free(p); free(q); free(tmp);
        return ORC_NOMEM;
    }
    int it = 0, restarts = 0, broke = 0;
    double relres = residual(n, Ap, Aj, Ax, b, x, r) / bnorm;
    while (relres > rtol && it < maxit && restarts <= 3) {
        broke = 0;
        apply_prec(n, LUp, LUj, LUx, r, z, tmp);
        for (int i = 0; i < n; ++i) p[i] = z[i];
        double rho = dot(n, r, z);
        if (!(rho > 0.0) || !isfinite(rho)) { broke = 1; break; }
        while (it < maxit) {
            orc_csr_spmv(n, Ap, Aj, Ax, 1.0, p, 0.0, q);
            double pq = dot(n, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) { broke = 1; break; }
            double alpha = rho / pq;
            for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
            for (int i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
            ++it;
            if (nrm2(n, r) / bnorm <= rtol) break;
            apply_prec(n, LUp, LUj, LUx, r, z, tmp);
            double rho_new = dot(n, r, z);
            if (!(rho_new > 0.0) || !isfinite(rho_new)) { broke = 1; break; }
            double beta = rho_new / rho;
            for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
            rho = rho_new;
        }
        relres = residual(n, Ap, Aj, Ax, b, x, r) / bnorm;
        if (relres > rtol) {
            if (broke) break;
            ++restarts;
        }
    }
    int status = relres <= rtol ? ORC_OK : broke ? ORC_BREAKDOWN : ORC_NOT_CONVERGED;
    *iters_out = it;
    *relres_out = relres;
    free(r); free(z); free(p); free(q); free(tmp);
    return status;
}
