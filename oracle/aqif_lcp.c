/*
 * Oracle (test infrastructure only) -- plain FP64 CPU reference for the
 * banded AQIF / PAQIF solve and the banded linear complementarity problem.
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may call this code.  It shares nothing with the HIP library.
 *
 * Paper: Singh & Dutt, "Total Variation Diminishing (TVD) method for
 * Elastohydrodynamic Lubrication (EHL) problem on Parallel Computers".
 *
 *  - LCP statement: Sec. 2.1, eq. (14): find U >= 0 with LU >= F and
 *    U^T (LU - F) = 0.
 *  - W0 / Z0 factor shapes: Sec. 2.2 (definitions of w_ij, z_ij; the
 *    "hourglass" W0 and "butterfly" Z0 matrices), banded forms in
 *    Sec. 2.2.2.
 *  - Factorisation, centre-out: Sec. 2.2 "Evaluation of W0 and Z0":
 *    at level k the rows s-k+1 and s+k of the reduced matrix L^(k) become
 *    rows of Z0, columns s-k+1 and s+k of W0 come from a 2x2 system per
 *    remaining row, and L^(k+1) = L^(k) - w z^T for the two pivots.
 *  - Solves: Sec. 2.2.2 "Solution of the complementarity problem":
 *    W0 Y = F from the centre outwards, Z0 U = Y from both ends inwards,
 *    one 2x2 system per level, then projection onto U >= 0.
 *  - Projected splitting iteration (Cryer): Sec. 3.2, theorem on the
 *    projected splitting; used here as an independent LCP solver.
 *
 * Readings (where the text is silent or garbled):
 *  - n odd: the paper assumes n = 2s.  For odd n = 2m+1 the centre row m
 *    is a 1x1 pivot (level 0), then levels k = 1..m pivot (m-k, m+k).
 *  - The Z-solve equation prints z_{k,k} x_{n-k+1}; it is read as
 *    z_{k,n-k+1} x_{n-k+1}.  The level ranges "2 <= k <= s-1" are read as
 *    2 <= k <= s.
 *  - The convex set K of the projection is ill-posed as printed; the
 *    projection is read as componentwise max(0, .).  An exact LCP mode
 *    (primal-dual active set on top of the AQIF solve) is provided too.
 *
 * Storage.  A band system of order n and half-bandwidth q is stored row
 * major, band[i*(2q+1) + d] = a(i, i+d-q); entries whose column falls
 * outside [0, n) are ignored.  During the centre-out elimination the only
 * fill appears next to the anti-diagonal j = n-1-i (the two frontier
 * blocks are coupled through the eliminated centre), so the working
 * matrix is kept as a main band of half-width q plus an anti band of
 * half-width q-1 around j = n-1-i.  Any write outside that pattern is a
 * bug and aborts.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ZERO_PIVOT 1
#define OR_NONFINITE 2
#define OR_LCP_NOT_CONVERGED 3

#define OR_LINEAR 0
#define OR_CLIP 1
#define OR_EXACT 2

/* ----------------------------------------------------------------------- */
/* working matrix: main band + anti band                                    */
/* ----------------------------------------------------------------------- */
typedef struct {
    int64_t n;
    int q;
    double *mb; /* n x (2q+1) */
    double *ab; /* n x (2q-1) */
} xmat;

static double *xref(xmat *S, int64_t i, int64_t j)
{
    int64_t n = S->n;
    int q = S->q;
    if (i < 0 || j < 0 || i >= n || j >= n) return NULL;
    int64_t d = j - i;
    if (d >= -q && d <= q) return &S->mb[i * (2 * q + 1) + (d + q)];
    int64_t e = j - (n - 1 - i);
    if (q >= 1 && e >= -(q - 1) && e <= q - 1) return &S->ab[i * (2 * q - 1) + (e + q - 1)];
    return NULL;
}

static double xget(xmat *S, int64_t i, int64_t j)
{
    double *p = xref(S, i, j);
    return p ? *p : 0.0;
}

static void xsub(xmat *S, int64_t i, int64_t j, double v)
{
    if (v == 0.0) return;
    double *p = xref(S, i, j);
    if (!p) {
        fprintf(stderr, "oracle: fill outside the X pattern at (%lld,%lld)\n", (long long)i,
                (long long)j);
        abort();
    }
    *p -= v;
}

static void xset(xmat *S, int64_t i, int64_t j, double v)
{
    double *p = xref(S, i, j);
    if (p) {
        *p = v;
    } else if (v != 0.0) {
        fprintf(stderr, "oracle: write outside the X pattern at (%lld,%lld)\n", (long long)i,
                (long long)j);
        abort();
    }
}

/* Effective matrix entry: rows/columns listed in `pinned` are replaced by
 * the identity (they carry u_i = 0 in the active-set solve). */
static double a_eff(int64_t n, int q, const double *band, const uint8_t *pinned, int64_t i,
                    int64_t j)
{
    if (i < 0 || j < 0 || i >= n || j >= n) return 0.0;
    int64_t d = j - i;
    if (d < -q || d > q) return 0.0;
    if (pinned && (pinned[i] || pinned[j])) return i == j ? 1.0 : 0.0;
    return band[i * (2 * q + 1) + (d + q)];
}

static int xinit(xmat *S, int64_t n, int q, const double *band, const uint8_t *pinned)
{
    S->n = n;
    S->q = q;
    S->mb = (double *)calloc((size_t)(n * (2 * q + 1)), sizeof(double));
    S->ab = (double *)calloc((size_t)(n * (2 * q - 1) + 1), sizeof(double));
    if (!S->mb || !S->ab) return -1;
    for (int64_t i = 0; i < n; i++)
        for (int d = -q; d <= q; d++) xset(S, i, i + d, a_eff(n, q, band, pinned, i, i + d));
    return 0;
}

static void xfree(xmat *S)
{
    free(S->mb);
    free(S->ab);
}

/* W0 columns: for pivot column p the 2q multipliers of the rows
 * [p1-q, p1-1] and [p2+1, p2+q] of its level (q values each side).  For
 * the odd-n centre the 2q rows are [m-q, m-1] and [m+1, m+q]. */
typedef struct {
    double *w; /* n x 2q */
} wcols;

static int level_count(int64_t n) { return (int)((n + 1) / 2); }

/* Pivot pair of level k (k = 1..): p1 = c1 - (k-1), p2 = c2 + (k-1). */
static void level_pivots(int64_t n, int k, int64_t *p1, int64_t *p2)
{
    if (n % 2 == 0) {
        int64_t s = n / 2;
        *p1 = s - k;
        *p2 = s + k - 1;
    } else {
        int64_t m = (n - 1) / 2;
        *p1 = m - k;
        *p2 = m + k;
    }
}

/* Centre-out factorisation of S in place (S becomes Z0), with the forward
 * solve W0 y = f fused (y overwritten in place).  Returns a status. */
static int aqif_factor(xmat *S, double *y, wcols *W)
{
    int64_t n = S->n;
    int q = S->q;
    int status = OR_OK;
    if (n <= 0) return OR_OK;
    int npair;
    if (n % 2 == 1) {
        /* level 0: 1x1 centre pivot */
        int64_t m = (n - 1) / 2;
        double piv = xget(S, m, m);
        if (piv == 0.0 || !isfinite(piv)) return OR_ZERO_PIVOT;
        for (int side = 0; side < 2; side++)
            for (int t = 1; t <= q; t++) {
                int64_t r = side == 0 ? m - t : m + t;
                if (r < 0 || r >= n) continue;
                double w = xget(S, r, m) / piv;
                if (W) W->w[m * 2 * q + (side == 0 ? (q - t) : (q + t - 1))] = w;
                for (int side2 = 0; side2 < 2; side2++)
                    for (int t2 = 1; t2 <= q; t2++) {
                        int64_t c = side2 == 0 ? m - t2 : m + t2;
                        if (c < 0 || c >= n) continue;
                        xsub(S, r, c, w * xget(S, m, c));
                    }
                if (y) y[r] -= w * y[m];
                xset(S, r, m, 0.0);
            }
        npair = (int)((n - 1) / 2);
    } else {
        npair = (int)(n / 2);
    }
    for (int k = 1; k <= npair; k++) {
        int64_t p1, p2;
        level_pivots(n, k, &p1, &p2);
        double a = xget(S, p1, p1), b = xget(S, p1, p2);
        double c = xget(S, p2, p1), d = xget(S, p2, p2);
        double det = a * d - b * c;
        if (det == 0.0 || !isfinite(det)) return OR_ZERO_PIVOT;
        /* remaining rows touched by this level: [p1-q, p1-1] u [p2+1, p2+q] */
        for (int side = 0; side < 2; side++)
            for (int t = 1; t <= q; t++) {
                int64_t r = side == 0 ? p1 - t : p2 + t;
                if (r < 0 || r >= n) continue;
                double l1 = xget(S, r, p1), l2 = xget(S, r, p2);
                /* [w1 w2] [[a b][c d]] = [l1 l2] */
                double w1 = (l1 * d - l2 * c) / det;
                double w2 = (l2 * a - l1 * b) / det;
                if (W) {
                    int slot = side == 0 ? (q - t) : (q + t - 1);
                    W->w[p1 * 2 * q + slot] = w1;
                    W->w[p2 * 2 * q + slot] = w2;
                }
                for (int side2 = 0; side2 < 2; side2++)
                    for (int t2 = 1; t2 <= q; t2++) {
                        int64_t cc = side2 == 0 ? p1 - t2 : p2 + t2;
                        if (cc < 0 || cc >= n) continue;
                        xsub(S, r, cc, w1 * xget(S, p1, cc) + w2 * xget(S, p2, cc));
                    }
                if (y) y[r] -= w1 * y[p1] + w2 * y[p2];
                xset(S, r, p1, 0.0);
                xset(S, r, p2, 0.0);
            }
    }
    return status;
}

/* Z0 x = y, from both ends inwards. */
static int aqif_back(xmat *S, const double *y, double *x)
{
    int64_t n = S->n;
    int q = S->q;
    if (n <= 0) return OR_OK;
    for (int64_t i = 0; i < n; i++) x[i] = 0.0;
    int npair = (int)(n % 2 ? (n - 1) / 2 : n / 2);
    for (int k = npair; k >= 1; k--) {
        int64_t p1, p2;
        level_pivots(n, k, &p1, &p2);
        double r1 = y[p1], r2 = y[p2];
        /* Z row p1 spans [p1-q, p1] u [p2, p2+q-1]; Z row p2 spans
         * [p1-q+1, p1] u [p2, p2+q].  Columns other than the pivots are
         * the already-solved outer unknowns. */
        for (int side = 0; side < 2; side++) {
            const int64_t c0 = side == 0 ? p1 - q : p2 + 1;
            for (int64_t cc = c0; cc < c0 + q; cc++) {
                if (cc < 0 || cc >= n) continue;
                r1 -= xget(S, p1, cc) * x[cc];
                r2 -= xget(S, p2, cc) * x[cc];
            }
        }
        double a = xget(S, p1, p1), b = xget(S, p1, p2);
        double c = xget(S, p2, p1), d = xget(S, p2, p2);
        double det = a * d - b * c;
        if (det == 0.0 || !isfinite(det)) return OR_ZERO_PIVOT;
        x[p1] = (d * r1 - b * r2) / det;
        x[p2] = (a * r2 - c * r1) / det;
    }
    if (n % 2 == 1) {
        int64_t m = (n - 1) / 2;
        double r = y[m];
        for (int64_t cc = m - q; cc <= m + q; cc++) {
            if (cc < 0 || cc >= n || cc == m) continue;
            r -= xget(S, m, cc) * x[cc];
        }
        x[m] = r / xget(S, m, m);
    }
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(x[i])) return OR_NONFINITE;
    return OR_OK;
}

/* Solve A_eff x = f_eff with AQIF (pinned rows: identity, f = 0). */
int or_aqif_solve(int64_t n, int q, const double *band, const uint8_t *pinned, const double *f,
                  double *x)
{
    if (n <= 0) return OR_OK;
    if (q < 1) return -1;
    xmat S;
    if (xinit(&S, n, q, band, pinned)) return -1;
    double *y = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; i++) y[i] = (pinned && pinned[i]) ? 0.0 : f[i];
    int st = aqif_factor(&S, y, NULL);
    if (st == OR_OK) st = aqif_back(&S, y, x);
    free(y);
    xfree(&S);
    return st;
}

/* Dense W0 and Z0 (row major, n x n each) for small n, for the WZ = A
 * reconstruction and zero-pattern checks. */
int or_aqif_factor_dense(int64_t n, int q, const double *band, const uint8_t *pinned, double *Wd,
                         double *Zd)
{
    if (n <= 0) return OR_OK;
    if (q < 1) return -1;
    xmat S;
    if (xinit(&S, n, q, band, pinned)) return -1;
    wcols W;
    W.w = (double *)calloc((size_t)(n * 2 * q), sizeof(double));
    int st = aqif_factor(&S, NULL, &W);
    memset(Wd, 0, (size_t)(n * n) * sizeof(double));
    memset(Zd, 0, (size_t)(n * n) * sizeof(double));
    for (int64_t i = 0; i < n; i++) {
        Wd[i * n + i] = 1.0;
        for (int64_t j = 0; j < n; j++) Zd[i * n + j] = xget(&S, i, j);
    }
    /* scatter the W columns */
    if (n % 2 == 1) {
        int64_t m = (n - 1) / 2;
        for (int t = 1; t <= q; t++) {
            if (m - t >= 0) Wd[(m - t) * n + m] = W.w[m * 2 * q + (q - t)];
            if (m + t < n) Wd[(m + t) * n + m] = W.w[m * 2 * q + (q + t - 1)];
        }
    }
    int npair = (int)(n % 2 ? (n - 1) / 2 : n / 2);
    for (int k = 1; k <= npair; k++) {
        int64_t p1, p2;
        level_pivots(n, k, &p1, &p2);
        for (int t = 1; t <= q; t++) {
            if (p1 - t >= 0) {
                Wd[(p1 - t) * n + p1] = W.w[p1 * 2 * q + (q - t)];
                Wd[(p1 - t) * n + p2] = W.w[p2 * 2 * q + (q - t)];
            }
            if (p2 + t < n) {
                Wd[(p2 + t) * n + p1] = W.w[p1 * 2 * q + (q + t - 1)];
                Wd[(p2 + t) * n + p2] = W.w[p2 * 2 * q + (q + t - 1)];
            }
        }
    }
    free(W.w);
    xfree(&S);
    return st;
}

/* w = A u - f with the original (unpinned) band. */
static void band_residual(int64_t n, int q, const double *band, const double *u, const double *f,
                          double *w)
{
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int d = -q; d <= q; d++) {
            int64_t j = i + d;
            if (j < 0 || j >= n) continue;
            s += band[i * (2 * q + 1) + (d + q)] * u[j];
        }
        w[i] = s - f[i];
    }
}

/*
 * Banded LCP:  u >= 0, w = A u - f >= 0, u_i w_i = 0 on the rows marked in
 * `bounded` (NULL: every row); unmarked rows are free (w_i = 0).
 *
 * mode OR_LINEAR: u = A^{-1} f (no projection).
 * mode OR_CLIP:   u = max(0, A^{-1} f) on bounded rows (projection of the
 *                 linear solve, the literal PAQIF step).
 * mode OR_EXACT:  primal-dual active set from a start set A_0: solve with
 *                 the rows and columns of A_k replaced by the identity and
 *                 f = 0 there; w = A u - f;
 *                 A_{k+1} = {i in A_k : w_i > 0} u {i not in A_k : u_i < 0}
 *                 (bounded rows only); stop when A_{k+1} = A_k.
 *                 or_lcp_solve_start takes A_0 from the caller (NULL: the
 *                 empty set); or_lcp_solve starts from {bounded i : f_i <= 0},
 *                 which predicts the binding constraints of a diagonally
 *                 dominant system.  Where the LCP has one solution (a
 *                 P-matrix) the start changes only the number of solves.
 * `iters` returns the number of AQIF solves.
 */
static int lcp_solve_impl(int64_t n, int q, const double *band, const double *f,
                          const uint8_t *bounded, int mode, int max_iter, int sign_start,
                          const uint8_t *start, double *u, double *w, uint8_t *active, int *iters)
{
    if (iters) *iters = 0;
    if (n <= 0) return OR_OK;
    uint8_t *act = (uint8_t *)calloc((size_t)n, 1);
    uint8_t *nxt = (uint8_t *)calloc((size_t)n, 1);
    double *wt = (double *)malloc((size_t)n * sizeof(double));
    int st = OR_OK;
    int it = 0;
    if (mode == OR_EXACT) {
        st = OR_LCP_NOT_CONVERGED;
        for (int64_t i = 0; i < n; i++) {
            int in0 = sign_start ? f[i] <= 0.0 : (start ? start[i] != 0 : 0);
            act[i] = (uint8_t)((bounded ? bounded[i] != 0 : 1) && in0);
        }
        while (it < max_iter) {
            int s2 = or_aqif_solve(n, q, band, act, f, u);
            it++;
            if (s2 != OR_OK) {
                st = s2;
                break;
            }
            band_residual(n, q, band, u, f, wt);
            int64_t changes = 0;
            for (int64_t i = 0; i < n; i++) {
                int b = bounded ? bounded[i] != 0 : 1;
                int a = 0;
                if (b) a = act[i] ? (wt[i] > 0.0) : (u[i] < 0.0);
                nxt[i] = (uint8_t)a;
                changes += a != act[i];
            }
            memcpy(act, nxt, (size_t)n);
            if (changes == 0) {
                st = OR_OK;
                break;
            }
        }
    } else {
        st = or_aqif_solve(n, q, band, NULL, f, u);
        it = 1;
        if (mode == OR_CLIP && st == OR_OK)
            for (int64_t i = 0; i < n; i++) {
                int b = bounded ? bounded[i] != 0 : 1;
                if (b && u[i] < 0.0) {
                    u[i] = 0.0;
                    act[i] = 1;
                }
            }
        band_residual(n, q, band, u, f, wt);
    }
    if (w) memcpy(w, wt, (size_t)n * sizeof(double));
    if (active) memcpy(active, act, (size_t)n);
    if (iters) *iters = it;
    free(act);
    free(nxt);
    free(wt);
    return st;
}

int or_lcp_solve(int64_t n, int q, const double *band, const double *f, const uint8_t *bounded,
                 int mode, int max_iter, double *u, double *w, uint8_t *active, int *iters)
{
    return lcp_solve_impl(n, q, band, f, bounded, mode, max_iter, 1, NULL, u, w, active, iters);
}

int or_lcp_solve_start(int64_t n, int q, const double *band, const double *f,
                       const uint8_t *bounded, const uint8_t *start, int max_iter, double *u,
                       double *w, uint8_t *active, int *iters)
{
    return lcp_solve_impl(n, q, band, f, bounded, OR_EXACT, max_iter, 0, start, u, w, active,
                          iters);
}

/*
 * Start sweeps of the exact LCP (a starting active set, not part of the
 * paper's method): k projected Jacobi sweeps from u = 0,
 *   u_i <- (f_i - sum_{j != i} a_ij u_j) / a_ii, clipped at 0 on bounded rows,
 * every sweep reading only the previous iterate.  The sum runs over the
 * row's band columns in increasing order, each term one fused
 * multiply-add.  The active-set iteration may start from
 * A_0 = {bounded i : u_i <= 0}.
 */
int or_start_sweeps(int64_t n, int q, const double *band, const double *f,
                    const uint8_t *bounded, int k, double *u)
{
    const int bw = 2 * q + 1;
    double *prev = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int64_t i = 0; i < n; i++) u[i] = 0.0;
    for (int s = 0; s < k; s++) {
        memcpy(prev, u, (size_t)n * sizeof(double));
        for (int64_t i = 0; i < n; i++) {
            double sum = f[i];
            for (int d = 0; d < bw; d++) {
                const int64_t j = i + d - q;
                if (d == q || j < 0 || j >= n) continue;
                sum = fma(-band[i * bw + d], prev[j], sum);
            }
            const double x = sum / band[i * bw + q];
            const int b = bounded ? bounded[i] != 0 : 1;
            u[i] = b ? fmax(x, 0.0) : x;
        }
    }
    free(prev);
    return OR_OK;
}

/*
 * Projected SOR for the banded LCP (Cryer's projected splitting
 * iteration): sweep i = 0..n-1,
 *   u_i <- max(0, u_i + omega * (f_i - (A u)_i) / a_ii)   (bounded rows)
 * until max_i |change| <= tol * max(1, |u|_inf).  Independent of AQIF; used
 * to pin the active-set solver.  Requires a_ii > 0.
 */
int or_lcp_pgs(int64_t n, int q, const double *band, const double *f, const uint8_t *bounded,
               double omega, int max_sweeps, double tol, double *u, int *sweeps)
{
    for (int64_t i = 0; i < n; i++) u[i] = 0.0;
    int sw = 0;
    int st = OR_LCP_NOT_CONVERGED;
    while (sw < max_sweeps) {
        double dmax = 0.0, umax = 0.0;
        for (int64_t i = 0; i < n; i++) {
            double s = 0.0;
            for (int d = -q; d <= q; d++) {
                int64_t j = i + d;
                if (j < 0 || j >= n) continue;
                s += band[i * (2 * q + 1) + (d + q)] * u[j];
            }
            double aii = band[i * (2 * q + 1) + q];
            double v = u[i] + omega * (f[i] - s) / aii;
            int b = bounded ? bounded[i] != 0 : 1;
            if (b && v < 0.0) v = 0.0;
            double ch = fabs(v - u[i]);
            if (ch > dmax) dmax = ch;
            u[i] = v;
            if (fabs(v) > umax) umax = fabs(v);
        }
        sw++;
        if (dmax <= tol * (umax > 1.0 ? umax : 1.0)) {
            st = OR_OK;
            break;
        }
    }
    if (sweeps) *sweeps = sw;
    return st;
}

/* Batch of band LCPs of one half-bandwidth; systems concatenated by row
 * offsets.  OpenMP over systems, largest first. */
int or_lcp_batch(int count, int q, const int64_t *offsets, const double *band, const double *f,
                 const uint8_t *bounded, int mode, int max_iter, double *u, double *w,
                 uint8_t *active, int32_t *status, int32_t *iters, int nthreads)
{
    int *order = (int *)malloc((size_t)(count > 0 ? count : 1) * sizeof(int));
    for (int s = 0; s < count; s++) order[s] = s;
    /* insertion sort by descending size (count is small enough) */
    for (int a = 1; a < count; a++) {
        int v = order[a];
        int64_t nv = offsets[v + 1] - offsets[v];
        int b = a - 1;
        while (b >= 0 && offsets[order[b] + 1] - offsets[order[b]] < nv) {
            order[b + 1] = order[b];
            b--;
        }
        order[b + 1] = v;
    }
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int t = 0; t < count; t++) {
        int s = order[t];
        int64_t o = offsets[s];
        int64_t n = offsets[s + 1] - o;
        int it = 0;
        int st = or_lcp_solve(n, q, band + o * (2 * q + 1), f + o, bounded ? bounded + o : NULL,
                              mode, max_iter, u + o, w ? w + o : NULL, active ? active + o : NULL,
                              &it);
        if (status) status[s] = st;
        if (iters) iters[s] = it;
    }
    free(order);
    return 0;
}
