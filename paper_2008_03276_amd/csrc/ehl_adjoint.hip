// Adjoint of the converged line contact on gfx950.
//
// At the converged state of the hybrid Newton line method (Sec. 3.3) the
// pressurised interior nodes I satisfy R_i(P, H0; theta) = 0 and the load
// balance G = h sum P - pi/2 = 0 (eq. 75 at its fixed point); cavitated nodes
// hold P = 0.  For an output J with cotangents gP (pressures), gH0 (offset)
// and gH (film H = H0 + X^2/2 + K P + roughness), with the active set held
// fixed,
//     dJ/dtheta = explicit - lambda^T dF/dtheta,
//     [J_I^T  h 1] [lambda_P]   [gP_I + (K gH)_I ]
//     [c^T    0  ] [lambda_H] = [gH0 + sum gH    ],
// where J_I = (dR/dP + dR/dH K) restricted to I x I (dense through the log
// kernel K) and c = dR/dH0.  The bordered system is split by its Schur
// complement into two transposed solves per instance,
//     z1 = J_I^-T (gP_I + (K gH)_I),  z2 = J_I^-T 1,
//     lambda_H = (c^T z1 - gH0 - sum gH) / (h c^T z2),
//     lambda_P = z1 - h lambda_H z2,
// so one batched solve covers 2B right-hand sides.  Each is GMRES(40),
// right-preconditioned by the Newton step's own band matrix: J_I D ~ -A
// (A = -dR/dsigma of half-bandwidth 4, D the weighted-change matrix of
// eqs. 69-74), hence J_I^-T ~ -A^-T D^T, applied as a PAQIF solve
// (Sec. 2.2) of the transposed band with the cavitated rows pinned.  The
// operator J_I^T v = (dR/dP)^T v + K ((dR/dH)^T v) is a banded gather plus
// the FP64 MFMA deformation product (K is symmetric).
//
// Gradients: M enters through lambda-bar and p_h, L through p_h, the
// roughness value at node m through the film at m.
//
// The paper has no adjoint; these are the exact derivatives of its discrete
// equations (the limiter derivatives are taken on the branch of the
// converged state).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "ehl_internal.h"
#include "ehl_model.h"
#include "paqif_args.h"

namespace pq {

namespace {
constexpr int PT = 256;  // rows per partial-derivative tile
constexpr int PH = 3;    // halo (the band spans nodes i-2 .. i+2)
constexpr int PW = PT + 2 * PH;
constexpr int GM = 40;   // GMRES restart length
constexpr int CHK = 4;   // Arnoldi steps between host checks of the states
constexpr int BT = 256;  // threads of the per-system kernels

enum : int { RUN = 0, HOLD = 1, DONE = 2 };

PQ_DEV double block_sum(double v, double* sh)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}
}  // namespace

// ---------------------------------------------------------------------------
// Partial derivatives of the interior residual rows: band of dR/dP (fixed
// film) and dR/dH over nodes i-2 .. i+1, and the parameter derivatives
// FM = dR/dM, FL = dR/dL at fixed (P, H).
// ---------------------------------------------------------------------------
struct AdjPartialArgs {
    int N, B;
    double h, x0;
    const ehl_params* params;
    const double *P, *Hel, *H0, *rough;
    double *RPb, *RHb, *FM, *FL;
    int conv = 0;  // 0 van Leer slope, 1 kappa-scheme slope (Sec. 3.3, eqs. 56-59)
    double kappa = 0.0;
};

__global__ void __launch_bounds__(PT) line_adjoint_partials_kernel(AdjPartialArgs a)
{
    const int b = blockIdx.y;
    const int N = a.N, n = N - 2;
    const int r0 = blockIdx.x * PT;
    const int t = threadIdx.x;
    const double h = a.h;
    const double M = a.params[b].M, L = a.params[b].L;
    const LineConst lc = line_const(M, L);
    const double H0 = a.H0[b];
    const double* P = a.P + (int64_t)b * N;
    const double* Hel = a.Hel + (int64_t)b * N;
    const double* rough = a.rough ? a.rough + (int64_t)b * N : nullptr;
    __shared__ double sP[PW], sEps[PW], sRH[PW], sEP[PW], sEH[PW], sRho[PW], sDrhoH[PW];
    const int mbase = r0 + 1 - PH;
    for (int w = t; w < PW; w += PT) {
        const int m = mbase + w;
        NodeState q{0, 0, 0, 0, 0, 0, 0};
        double Pm = 0.0;
        if (m >= 0 && m < N) {
            const double x = a.x0 + h * m;
            Pm = P[m];
            q = node_state(Pm, H0 + 0.5 * x * x + Hel[m] + (rough ? rough[m] : 0.0), lc);
        }
        sP[w] = Pm;
        sEps[w] = q.eps;
        sRH[w] = q.rH;
        sEP[w] = q.eP;
        sEH[w] = q.eH;
        sRho[w] = q.rho;
        sDrhoH[w] = q.drhoH;
    }
    __syncthreads();
    const int r = r0 + t;
    if (r >= n) return;
    const int i = r + 1;
    auto at = [&](const double* s, int m) { return s[m - mbase]; };
    const double h2 = h * h;
    const double dPp = at(sP, i + 1) - at(sP, i), dPm = at(sP, i) - at(sP, i - 1);
    const double eph = 0.5 * (at(sEps, i) + at(sEps, i + 1));
    const double epm = 0.5 * (at(sEps, i - 1) + at(sEps, i));
    // coefficients on nodes i-2+d, d = 0..3:
    //   cE: d R / d eps_m,  cF: d R / d (rho H)_m,  cP: d R / d P_m (fixed eps)
    double cE[4] = {0.0, -0.5 * dPm / h2, 0.5 * (dPp - dPm) / h2, 0.5 * dPp / h2};
    double cP[4] = {0.0, epm / h2, -(eph + epm) / h2, eph / h2};
    double cF[4] = {0.0, 0.0, 0.0, 0.0};
    {
        // -(f_i - f_{i-1}) / h with f_t = (rho H)_t + psi_t / 2 (t >= 1), f_0 = (rho H)_0
        double psi, pa, pb;
        // exact slope derivatives (limiter_jacobian mode 0)
        convective_slope(a.conv, a.kappa, 0, at(sRH, i) - at(sRH, i - 1),
                         at(sRH, i + 1) - at(sRH, i), psi, pa, pb);
        const double sg = -1.0 / h;
        cF[1] += sg * 0.5 * (-pb);
        cF[2] += sg * (1.0 + 0.5 * (pb - pa));
        cF[3] += sg * 0.5 * pa;
        const double sm = 1.0 / h;
        if (i - 1 == 0) {
            cF[1] += sm;
        } else {
            convective_slope(a.conv, a.kappa, 0, at(sRH, i - 1) - at(sRH, i - 2),
                             at(sRH, i) - at(sRH, i - 1), psi, pa, pb);
            cF[0] += sm * 0.5 * (-pb);
            cF[1] += sm * (1.0 + 0.5 * (pb - pa));
            cF[2] += sm * 0.5 * pa;
        }
    }
    double Rlam = 0.0, Rph = 0.0;
    double* rp = a.RPb + ((int64_t)b * n + r) * 4;
    double* rh = a.RHb + ((int64_t)b * n + r) * 4;
#pragma unroll
    for (int d = 0; d < 4; d++) {
        const int m = i - 2 + d;
        double vp = 0.0, vh = 0.0;
        if (m >= 0) {
            vp = cE[d] * at(sEP, m) + cF[d] * at(sDrhoH, m) + cP[d];
            vh = cE[d] * at(sEH, m) + cF[d] * at(sRho, m);
            Rlam += cE[d] * (-at(sEps, m) / lc.lam);
            Rph += (at(sP, m) / lc.ph) * (cE[d] * at(sEP, m) + cF[d] * at(sDrhoH, m));
        }
        rp[d] = vp;
        rh[d] = vh;
    }
    // lambda-bar = 3 pi^2 / (8 M^2), p_h proportional to L sqrt(M)
    a.FM[(int64_t)b * n + r] = Rlam * (-2.0 * lc.lam / M) + Rph * (lc.ph / (2.0 * M));
    a.FL[(int64_t)b * n + r] = Rph * (lc.ph / L);
}

// ---------------------------------------------------------------------------
// Transposed Newton band (both right-hand-side kinds) and the pinned mask.
// ---------------------------------------------------------------------------
__global__ void adj_transpose_kernel(int N, int B, int S, const double* band, const double* P,
                                     double* bandT, uint8_t* pin)
{
    const int n = N - 2;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)S * n) return;
    const int s = (int)(idx / n), r = (int)(idx % n), b = s % B;
    const double* A = band + (int64_t)b * n * 9;
    double* o = bandT + idx * 9;
#pragma unroll
    for (int e = -4; e <= 4; e++) {
        const int c = r + e;  // A^T[r][r+e] = A[r+e][r]
        o[4 + e] = (c >= 0 && c < n) ? A[(int64_t)c * 9 + 4 - e] : 0.0;
    }
    pin[idx] = P[(int64_t)b * N + r + 1] > 0.0 ? 0 : 1;
}

__global__ void adj_offsets_kernel(int S, int n, int64_t* offs)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= S) offs[i] = (int64_t)i * n;
}

__global__ void adj_fill_kernel(int64_t count, double* p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

// right-hand sides: kind 0 (s < B) gP_I + (K gH)_I, kind 1 the ones vector on I
__global__ void adj_rhs_kernel(int N, int B, const double* gP, const double* KgH,
                               const uint8_t* pin, double* g)
{
    const int n = N - 2, S = 2 * B;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)S * n) return;
    const int s = (int)(idx / n), j = (int)(idx % n);
    double v = 0.0;
    if (!pin[idx]) {
        if (s >= B) {
            v = 1.0;
        } else {
            if (gP) v += gP[(int64_t)s * N + j + 1];
            if (KgH) v += KgH[(int64_t)s * N + j + 1];
        }
    }
    g[idx] = v;
}

// ---------------------------------------------------------------------------
// Batched GMRES state.
// ---------------------------------------------------------------------------
struct GmArgs {
    int N, n, B, S, max_iter;
    double rtol, loose;
    const uint8_t* pin;     // n x S
    const uint8_t* direct;  // N x B (forward hybrid classification)
    const double *RPb, *RHb;
    const double* g;        // n x S
    double *x, *zt, *zz, *wpre, *tN, *uN;
    double* V;              // (GM+1) x S x n
    double *Rm, *cs, *sn, *gv, *bnorm, *prevb;
    int32_t *state, *sstat, *kcount, *siters;
};

PQ_DEV bool skipped(const GmArgs& g, int s, bool run_only)
{
    const int st = g.state[s];
    return run_only ? st != RUN : st == DONE;
}

// zt = -D^T v on I (0 on pinned rows): the first half of the preconditioner
__global__ void adj_prec_in_kernel(GmArgs g, const double* src, int run_only)
{
    const int n = g.n;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)g.S * n) return;
    const int s = (int)(idx / n), j = (int)(idx % n);
    if (skipped(g, s, run_only)) return;
    const int b = s % g.B;
    const uint8_t* pin = g.pin + (int64_t)s * n;
    const double* v = src + (int64_t)s * n;
    double y = 0.0;
    if (!pin[j]) {
        y = v[j];
        if (!g.direct[(int64_t)b * g.N + j + 1]) {  // distributive column j
            const double vm = (j > 0 && !pin[j - 1]) ? v[j - 1] : 0.0;
            const double vp = (j + 1 < n && !pin[j + 1]) ? v[j + 1] : 0.0;
            y -= 0.5 * (vm + vp);
        }
    }
    g.zt[idx] = -y;
}

// tN = (dR/dH)^T z (all N nodes), wpre = (dR/dP)^T z (interior nodes), rows in I
__global__ void adj_apply_pre_kernel(GmArgs g, const double* src, int run_only)
{
    const int N = g.N, n = g.n;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)g.S * N) return;
    const int s = (int)(idx / N), m = (int)(idx % N);
    if (skipped(g, s, run_only)) return;
    const int b = s % g.B;
    const uint8_t* pin = g.pin + (int64_t)s * n;
    const double* z = src + (int64_t)s * n;
    const double* RP = g.RPb + (int64_t)b * n * 4;
    const double* RH = g.RHb + (int64_t)b * n * 4;
    double th = 0.0, tp = 0.0;
#pragma unroll
    for (int r = m - 2; r <= m + 1; r++) {
        if (r < 0 || r >= n || pin[r]) continue;
        const int d = m - r + 1;
        th += RH[(int64_t)r * 4 + d] * z[r];
        tp += RP[(int64_t)r * 4 + d] * z[r];
    }
    g.tN[idx] = th;
    if (m >= 1 && m <= N - 2) g.wpre[(int64_t)s * n + m - 1] = tp;
}

// One Arnoldi step (classical Gram-Schmidt, twice) and the Givens update of
// the least-squares problem; one workgroup per system.
__global__ void __launch_bounds__(BT) adj_arnoldi_kernel(GmArgs g, int k)
{
    const int s = blockIdx.x;
    if (g.state[s] != RUN) return;
    const int n = g.n, S = g.S, t = threadIdx.x;
    __shared__ double sh[4];
    __shared__ double hd[GM + 1], hc[GM + 2];
    const uint8_t* pin = g.pin + (int64_t)s * n;
    const double* zz = g.zz + (int64_t)s * n;
    const double* wp = g.wpre + (int64_t)s * n;
    const double* u = g.uN + (int64_t)s * g.N;
    auto Vp = [&](int i) { return g.V + ((int64_t)i * S + s) * n; };
    double* w = Vp(k + 1);
    for (int j = t; j < n; j += BT) w[j] = pin[j] ? zz[j] : wp[j] + u[j + 1];
    if (t <= k + 1) hc[t] = 0.0;
    for (int pass = 0; pass < 2; pass++) {
        for (int i = 0; i <= k; i++) {
            const double* vi = Vp(i);
            double d = 0.0;
            for (int j = t; j < n; j += BT) d += w[j] * vi[j];
            d = block_sum(d, sh);
            if (t == 0) hd[i] = d;
        }
        __syncthreads();
        for (int j = t; j < n; j += BT) {
            double v = w[j];
            for (int i = 0; i <= k; i++) v -= hd[i] * Vp(i)[j];
            w[j] = v;
        }
        if (t <= k) hc[t] += hd[t];
        __syncthreads();
    }
    double nn = 0.0;
    for (int j = t; j < n; j += BT) nn += w[j] * w[j];
    const double nrm = sqrt(block_sum(nn, sh));
    if (nrm > 0.0) {
        const double inv = 1.0 / nrm;
        for (int j = t; j < n; j += BT) w[j] *= inv;
    }
    if (t == 0) {
        hc[k + 1] = nrm;
        double* cs = g.cs + (int64_t)s * GM;
        double* sn = g.sn + (int64_t)s * GM;
        double* gv = g.gv + (int64_t)s * (GM + 1);
        for (int i = 0; i < k; i++) {
            const double a0 = hc[i], a1 = hc[i + 1];
            hc[i] = cs[i] * a0 + sn[i] * a1;
            hc[i + 1] = -sn[i] * a0 + cs[i] * a1;
        }
        const double den = hypot(hc[k], hc[k + 1]);
        const double c = den > 0.0 ? hc[k] / den : 1.0;
        const double sv = den > 0.0 ? hc[k + 1] / den : 0.0;
        cs[k] = c;
        sn[k] = sv;
        hc[k] = den;
        const double gk = gv[k];
        gv[k] = c * gk;
        gv[k + 1] = -sv * gk;
        double* R = g.Rm + (int64_t)s * GM * GM + (int64_t)k * GM;
        for (int i = 0; i <= k; i++) R[i] = hc[i];
        g.kcount[s] = k + 1;
        g.siters[s] += 1;
        const double est = fabs(gv[k + 1]);
        if (!(est > g.rtol * g.bnorm[s]) || k + 1 == GM || nrm == 0.0 || den == 0.0 ||
            g.siters[s] >= g.max_iter)
            g.state[s] = HOLD;
    }
}

// u = V y with R y = gv (the cycle's least-squares solution), into wpre
__global__ void __launch_bounds__(BT) adj_combine_kernel(GmArgs g)
{
    const int s = blockIdx.x;
    if (g.state[s] == DONE) return;
    const int n = g.n, S = g.S, t = threadIdx.x;
    __shared__ double y[GM];
    const int k = g.kcount[s];
    if (t == 0) {
        const double* R = g.Rm + (int64_t)s * GM * GM;
        const double* gv = g.gv + (int64_t)s * (GM + 1);
        for (int i = k - 1; i >= 0; i--) {
            double v = gv[i];
            for (int l = i + 1; l < k; l++) v -= R[(int64_t)l * GM + i] * y[l];
            const double d = R[(int64_t)i * GM + i];
            y[i] = d != 0.0 ? v / d : 0.0;
        }
    }
    __syncthreads();
    double* out = g.wpre + (int64_t)s * n;
    for (int j = t; j < n; j += BT) {
        double v = 0.0;
        for (int i = 0; i < k; i++) v += y[i] * g.V[((int64_t)i * S + s) * n + j];
        out[j] = v;
    }
}

__global__ void adj_axpy_kernel(GmArgs g)
{
    const int n = g.n;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)g.S * n) return;
    const int s = (int)(idx / n);
    if (g.state[s] == DONE) return;
    g.x[idx] += g.zz[idx];
}

// r = g - A x (first: x = 0); convergence and restart decisions
__global__ void __launch_bounds__(BT) adj_restart_kernel(GmArgs g, int first)
{
    const int s = blockIdx.x;
    // the first call initialises every system (the state array starts undefined)
    if (!first && g.state[s] == DONE) return;
    const int n = g.n, t = threadIdx.x;
    __shared__ double sh[4];
    const uint8_t* pin = g.pin + (int64_t)s * n;
    const double* gg = g.g + (int64_t)s * n;
    double* x = g.x + (int64_t)s * n;
    const double* wp = g.wpre + (int64_t)s * n;
    const double* u = g.uN + (int64_t)s * g.N;
    double* v0 = g.V + (int64_t)s * n;
    double nn = 0.0;
    for (int j = t; j < n; j += BT) {
        double r = gg[j];
        if (first)
            x[j] = 0.0;
        else
            r -= pin[j] ? x[j] : wp[j] + u[j + 1];
        v0[j] = r;
        nn += r * r;
    }
    const double beta = sqrt(block_sum(nn, sh));
    if (first && t == 0) g.bnorm[s] = beta;
    const double bn = first ? beta : g.bnorm[s];
    int next = RUN, st = SYS_OK;
    if (!isfinite(beta)) {
        next = DONE;
        st = SYS_NONFINITE;
    } else if (beta <= g.rtol * bn) {
        next = DONE;
    } else if (!first && (beta > 0.5 * g.prevb[s] || g.siters[s] >= g.max_iter)) {
        // no further progress from a restart: the residual has reached the
        // rounding floor of J^T x (or the iteration cap)
        next = DONE;
        st = beta <= g.loose * bn ? SYS_OK : SYS_ADJOINT_NOT_CONVERGED;
    }
    if (next == RUN) {
        const double inv = 1.0 / beta;
        for (int j = t; j < n; j += BT) v0[j] *= inv;
    }
    if (t == 0) {
        g.state[s] = next;
        g.sstat[s] = st;
        g.prevb[s] = beta;
        g.kcount[s] = 0;
        double* gv = g.gv + (int64_t)s * (GM + 1);
        gv[0] = beta;
        if (first) g.siters[s] = 0;
    }
}

// Schur combination and gradients, one workgroup per instance
struct AdjFinalArgs {
    int N, B;
    double h;
    const uint8_t* pin;
    const double *x, *RHb, *FM, *FL, *gH0, *gH;
    const int32_t *sstat, *siters, *fstat;
    double *lam, *dM, *dL, *drough;
    int32_t *status, *iters;
};

__global__ void __launch_bounds__(BT) adj_final_kernel(AdjFinalArgs a)
{
    const int b = blockIdx.x, t = threadIdx.x;
    const int N = a.N, n = N - 2, B = a.B;
    __shared__ double sh[4];
    const uint8_t* pin = a.pin + (int64_t)b * n;
    const double* z1 = a.x + (int64_t)b * n;
    const double* z2 = a.x + (int64_t)(B + b) * n;
    const double* RH = a.RHb + (int64_t)b * n * 4;
    const double* gH = a.gH ? a.gH + (int64_t)b * N : nullptr;
    double s1 = 0.0, s2 = 0.0, sg = 0.0;
    for (int r = t; r < n; r += BT) {
        if (pin[r]) continue;
        const double c = (RH[r * 4] + RH[r * 4 + 1]) + (RH[r * 4 + 2] + RH[r * 4 + 3]);
        s1 += c * z1[r];
        s2 += c * z2[r];
    }
    if (gH)
        for (int m = t; m < N; m += BT) sg += gH[m];
    s1 = block_sum(s1, sh);
    s2 = block_sum(s2, sh);
    sg = block_sum(sg, sh);
    const double gHtot = (a.gH0 ? a.gH0[b] : 0.0) + sg;
    const double lamH = (s1 - gHtot) / (a.h * s2);
    double* lam = a.lam + (int64_t)b * n;
    double fm = 0.0, fl = 0.0;
    for (int r = t; r < n; r += BT) {
        const double l = pin[r] ? 0.0 : z1[r] - a.h * lamH * z2[r];
        lam[r] = l;
        fm += l * a.FM[(int64_t)b * n + r];
        fl += l * a.FL[(int64_t)b * n + r];
    }
    fm = block_sum(fm, sh);  // also orders the lam stores before the gather
    fl = block_sum(fl, sh);
    for (int m = t; m < N; m += BT) {
        double v = gH ? gH[m] : 0.0;
        for (int r = m - 2; r <= m + 1; r++)
            if (r >= 0 && r < n) v -= RH[(int64_t)r * 4 + (m - r + 1)] * lam[r];
        a.drough[(int64_t)b * N + m] = v;
    }
    if (t == 0) {
        a.dM[b] = -fm;
        a.dL[b] = -fl;
        const int s0 = a.sstat[b], s1s = a.sstat[B + b];
        int st = SYS_OK;
        if (a.fstat[b] != SYS_OK || a.fstat[B + b] != SYS_OK)
            st = SYS_ZERO_PIVOT;
        else if (s0 == SYS_NONFINITE || s1s == SYS_NONFINITE || !isfinite(lamH) || !isfinite(fm) ||
            !isfinite(fl))
            st = SYS_NONFINITE;
        else if (s0 != SYS_OK)
            st = s0;
        else if (s1s != SYS_OK)
            st = s1s;
        a.status[b] = st;
        a.iters[b] = a.siters[b] + a.siters[B + b];
    }
}

}  // namespace pq

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct AdjLayout {
    size_t kvec, hel, RPb, RHb, FM, FL, band, rhs, bounded, direct, bandT, pin, offs, fstat,
        factors, g, x, zt, zz, wpre, tN, uN, V, Rm, cs, sn, gv, bnorm, prevb, state, sstat,
        kcount, siters, lam, total;
};

AdjLayout adj_layout(int N, int B)
{
    const size_t n = N - 2, b = B, S = 2 * b;
    AdjLayout L;
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p += a256(bytes);
        return at;
    };
    const size_t d = sizeof(double);
    L.kvec = take(N * d);
    L.hel = take(N * b * d);
    L.RPb = take(n * 4 * b * d);
    L.RHb = take(n * 4 * b * d);
    L.FM = take(n * b * d);
    L.FL = take(n * b * d);
    L.band = take(n * 9 * b * d);
    L.rhs = take(n * b * d);
    L.bounded = take(n * b);
    L.direct = take(N * b);
    L.bandT = take(n * 9 * S * d);
    L.pin = take(n * S);
    L.offs = take((S + 1) * sizeof(int64_t));
    L.fstat = take(S * sizeof(int32_t));
    const size_t recs = (S * n + S) / 2 + 1;
    L.factors = take(recs * (size_t)pq::record_stride(4, true) * d);
    L.g = take(n * S * d);
    L.x = take(n * S * d);
    L.zt = take(n * S * d);
    L.zz = take(n * S * d);
    L.wpre = take(n * S * d);
    L.tN = take(N * S * d);
    L.uN = take(N * S * d);
    L.V = take((pq::GM + 1) * n * S * d);
    L.Rm = take((size_t)pq::GM * pq::GM * S * d);
    L.cs = take(pq::GM * S * d);
    L.sn = take(pq::GM * S * d);
    L.gv = take((pq::GM + 1) * S * d);
    L.bnorm = take(S * d);
    L.prevb = take(S * d);
    L.state = take(S * sizeof(int32_t));
    L.sstat = take(S * sizeof(int32_t));
    L.kcount = take(S * sizeof(int32_t));
    L.siters = take(S * sizeof(int32_t));
    L.lam = take(n * b * d);
    L.total = p;
    return L;
}

bool adj_valid_grid(const ehl_grid* g)
{
    return g && g->ny == 1 && g->nx >= 5 && g->nx <= 8192 && g->x1 > g->x0;
}

unsigned blocks_for(int64_t count) { return (unsigned)((count + 255) / 256); }

}  // namespace

extern "C" {

size_t ehl_adjoint_workspace_bytes(paqif_handle handle, const ehl_grid* grid, int B)
{
    (void)handle;
    if (!adj_valid_grid(grid) || B <= 0) return 0;
    return adj_layout(grid->nx, B).total;
}

int ehl_adjoint_solve(paqif_handle handle, const ehl_grid* grid, const ehl_params* params, int B,
                      const ehl_opts* opts, const double* rough, const double* P,
                      const double* H0, const double* gP, const double* gH0, const double* gH,
                      double rtol, int max_iter, double* dM, double* dL, double* drough,
                      int32_t* status, int32_t* iters, void* workspace, void* stream)
{
    using namespace pq;
    if (!handle || !adj_valid_grid(grid) || B < 0 || !opts) return PAQIF_EINVAL;
    if (!(opts->kernel_terms == 1 || opts->kernel_terms == 2)) return PAQIF_EINVAL;
    if (opts->limiter_jacobian < 0 || opts->limiter_jacobian > 2) return PAQIF_EINVAL;
    if (!(opts->convection == 0 ||
          (opts->convection == 1 && opts->kappa >= -1.0 && opts->kappa <= 1.0)))
        return PAQIF_EINVAL;
    if (!(rtol > 0.0 && rtol < 1.0) || max_iter < 1) return PAQIF_EINVAL;
    if (B == 0) return PAQIF_OK;
    if (!params || !P || !H0 || !dM || !dL || !drough || !status || !iters || !workspace)
        return PAQIF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int N = grid->nx, n = N - 2, S = 2 * B;
    const double h = (grid->x1 - grid->x0) / (N - 1);
    const AdjLayout L = adj_layout(N, B);
    char* ws = static_cast<char*>(workspace);
    auto D = [&](size_t off) { return reinterpret_cast<double*>(ws + off); };
    auto U8 = [&](size_t off) { return reinterpret_cast<uint8_t*>(ws + off); };
    auto I32 = [&](size_t off) { return reinterpret_cast<int32_t*>(ws + off); };
    double* kvec = D(L.kvec);
    double* hel = D(L.hel);
    int st;
    if ((st = launch_line_kernel_vec(N, h, kvec, s))) return st;
    if ((st = launch_line_deform(N, B, PREC_FP64, kvec, P, hel, s))) return st;

    AdjPartialArgs pa{N, B, h, grid->x0, params, P, hel, H0, rough,
                      D(L.RPb), D(L.RHb), D(L.FM), D(L.FL)};
    pa.conv = opts->convection;
    pa.kappa = opts->kappa;
    hipLaunchKernelGGL(line_adjoint_partials_kernel, dim3((n + PT - 1) / PT, B), dim3(PT), 0, s,
                       pa);

    // the Newton band at the converged state: the preconditioner
    LineAssembleArgs aa;
    aa.N = N;
    aa.B = B;
    aa.kterms = opts->kernel_terms;
    aa.limjac = opts->limiter_jacobian;
    aa.conv = opts->convection;  // the preconditioner uses the same slope
    aa.kappa = opts->kappa;
    aa.h = h;
    aa.x0 = grid->x0;
    aa.switch_ratio = opts->switch_ratio;
    aa.params = params;
    aa.kvec = kvec;
    aa.P = P;
    aa.Hel = hel;
    aa.H0 = H0;
    aa.rough = rough;
    aa.skip = nullptr;
    aa.R = nullptr;
    aa.band = D(L.band);
    aa.rhs = D(L.rhs);
    aa.bounded = U8(L.bounded);
    aa.direct = U8(L.direct);
    if ((st = launch_line_assemble(aa, s))) return st;

    int64_t* offs = reinterpret_cast<int64_t*>(ws + L.offs);
    uint8_t* pin = U8(L.pin);
    hipLaunchKernelGGL(adj_offsets_kernel, dim3((S + 256) / 256), dim3(256), 0, s, S, n, offs);
    hipLaunchKernelGGL(adj_transpose_kernel, dim3(blocks_for((int64_t)S * n)), dim3(256), 0, s, N,
                       B, S, D(L.band), P, D(L.bandT), pin);
    FactorArgs fa;
    fa.count = S;
    fa.offsets = offs;
    fa.order = nullptr;
    fa.band = D(L.bandT);
    fa.pinned = pin;
    fa.rec = ws + L.factors;
    fa.status = I32(L.fstat);
    if ((st = dispatch_factor(4, fa, s))) return st;
    SolveArgs sa;
    sa.count = S;
    sa.offsets = offs;
    sa.order = nullptr;
    sa.pinned = pin;
    sa.rec = ws + L.factors;
    sa.rhs = D(L.zt);
    sa.x = D(L.zz);

    GmArgs g;
    g.N = N;
    g.n = n;
    g.B = B;
    g.S = S;
    g.max_iter = max_iter;
    g.rtol = rtol;
    g.loose = std::max(1e-8, rtol);
    g.pin = pin;
    g.direct = U8(L.direct);
    g.RPb = D(L.RPb);
    g.RHb = D(L.RHb);
    g.g = D(L.g);
    g.x = D(L.x);
    g.zt = D(L.zt);
    g.zz = D(L.zz);
    g.wpre = D(L.wpre);
    g.tN = D(L.tN);
    g.uN = D(L.uN);
    g.V = D(L.V);
    g.Rm = D(L.Rm);
    g.cs = D(L.cs);
    g.sn = D(L.sn);
    g.gv = D(L.gv);
    g.bnorm = D(L.bnorm);
    g.prevb = D(L.prevb);
    g.state = I32(L.state);
    g.sstat = I32(L.sstat);
    g.kcount = I32(L.kcount);
    g.siters = I32(L.siters);

    // defined contents for every system's work vectors (skipped systems
    // still pass through the factored solve and the deformation product)
    for (size_t off : {L.zt, L.zz, L.wpre})
        hipLaunchKernelGGL(adj_fill_kernel, dim3(blocks_for((int64_t)S * n)), dim3(256), 0, s,
                           (int64_t)S * n, D(off));
    for (size_t off : {L.tN, L.uN})
        hipLaunchKernelGGL(adj_fill_kernel, dim3(blocks_for((int64_t)S * N)), dim3(256), 0, s,
                           (int64_t)S * N, D(off));
    const double* KgH = nullptr;
    if (gH) {
        if ((st = launch_line_deform(N, B, PREC_FP64, kvec, gH, D(L.uN), s))) return st;
        KgH = D(L.uN);
    }
    hipLaunchKernelGGL(adj_rhs_kernel, dim3(blocks_for((int64_t)S * n)), dim3(256), 0, s, N, B,
                       gP, KgH, pin, D(L.g));
    hipLaunchKernelGGL(adj_restart_kernel, dim3(S), dim3(BT), 0, s, g, 1);

    const dim3 gn(blocks_for((int64_t)S * n)), gN(blocks_for((int64_t)S * N));
    auto apply = [&](const double* src, int run_only) -> int {
        hipLaunchKernelGGL(adj_apply_pre_kernel, gN, dim3(256), 0, s, g, src, run_only);
        return launch_line_deform(N, S, PREC_FP64, kvec, D(L.tN), D(L.uN), s);
    };
    auto precond = [&](const double* src, int run_only) -> int {
        hipLaunchKernelGGL(adj_prec_in_kernel, gn, dim3(256), 0, s, g, src, run_only);
        return dispatch_solve(4, sa, s);
    };
    std::vector<int32_t> hstate(S);
    auto fetch = [&]() -> bool {
        return hipMemcpyAsync(hstate.data(), g.state, S * sizeof(int32_t), hipMemcpyDeviceToHost,
                              s) == hipSuccess &&
               hipStreamSynchronize(s) == hipSuccess;
    };
    const int max_cycles = max_iter + 2;
    for (int cyc = 0; cyc < max_cycles; cyc++) {
        if (!fetch()) return PAQIF_EHIP;
        if (std::all_of(hstate.begin(), hstate.end(), [](int32_t v) { return v == DONE; })) break;
        for (int k = 0; k < GM; k++) {
            if ((st = precond(g.V + (int64_t)k * S * n, 1))) return st;
            if ((st = apply(g.zz, 1))) return st;
            hipLaunchKernelGGL(adj_arnoldi_kernel, dim3(S), dim3(BT), 0, s, g, k);
            if ((k + 1) % CHK == 0 && k + 1 < GM) {
                if (!fetch()) return PAQIF_EHIP;
                if (std::none_of(hstate.begin(), hstate.end(), [](int32_t v) { return v == RUN; }))
                    break;
            }
        }
        hipLaunchKernelGGL(adj_combine_kernel, dim3(S), dim3(BT), 0, s, g);
        if ((st = precond(g.wpre, 0))) return st;
        hipLaunchKernelGGL(adj_axpy_kernel, gn, dim3(256), 0, s, g);
        if ((st = apply(g.x, 0))) return st;
        hipLaunchKernelGGL(adj_restart_kernel, dim3(S), dim3(BT), 0, s, g, 0);
    }
    AdjFinalArgs fa2{N,      B,        h,          pin,      g.x,      g.RHb,
                     D(L.FM), D(L.FL), gH0,        gH,       g.sstat,  g.siters,
                     I32(L.fstat), D(L.lam), dM,   dL,       drough,   status,
                     iters};
    hipLaunchKernelGGL(adj_final_kernel, dim3(B), dim3(BT), 0, s, fa2);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

}  // extern "C"
