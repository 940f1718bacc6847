// EHL point contact on gfx950: alternating x/y line sweeps, each colour of
// lines one batched PAQIF complementarity solve.
//
// Paper Sec. 3.3 (point contact, Example 5): Reynolds operator on the 2D
// grid with the TVD flux in the rolling direction x (eqs. 62-65), hybrid
// switch min(eps/hx, eps/hy) > 0.6 (eq. 60), weighted change with quarter
// weights to the four neighbours (eq. 69), the film's response through the
// distributed kernel (eqs. 66-67, 74), load balance 2 pi / 3 with the H0
// relaxation (eq. 75).
//
// One Newton step = x-sweep then y-sweep; a sweep solves its lines in two
// colours (odd line index, then even), the film being re-evaluated (2D MFMA
// deformation) before each colour.  With all lines at once, weighted changes
// of neighbouring lines can cancel (nonzero sigma, zero net change), and for
// y-lines the x-flux ties each column to its upstream neighbours.  y-lines
// act on the direct nodes only (a weighted-change node keeps its pressure):
// in the Hertzian zone a y-line couples to the flux only through the
// x-difference of the film response, which does not give a usable line
// matrix; the x-lines carry those nodes.
//
// Layout: node (b, i, j) at (b*Nx + i)*Ny + j (i along x).  A line of the
// x-sweep is one j (positions i), of the y-sweep one i (positions j).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "ehl_internal.h"
#include "ehl_model.h"
#include "paqif_args.h"

namespace pq {

// Moes point-contact map: alpha-bar = (L/pi)(3M/2)^(1/3),
// lambda-bar = (128 pi^3 / (3 M^4))^(1/3), p_h = alpha-bar / alpha.
PQ_DEV LineConst point_const(double M, double L)
{
    LineConst c;
    const double abar = (L / M_PI) * cbrt(1.5 * M);
    c.lam = cbrt(128.0 * M_PI * M_PI * M_PI / (3.0 * M * M * M * M));
    c.ph = abar / lub::ALPHA;
    return c;
}

// node quantities of every node and the hybrid classification
__global__ void point_node_kernel(PointNodeArgs a)
{
    const int64_t per = (int64_t)a.Nx * a.Ny;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per * a.B) return;
    const int b = (int)(idx / per);
    if (a.skip && a.skip[b]) return;
    const int rem = (int)(idx % per), i = rem / a.Ny, j = rem % a.Ny;
    const LineConst lc = point_const(a.params[b].M, a.params[b].L);
    const double x = a.x0 + a.hx * i, y = a.y0 + a.hy * j;
    const double Pm = a.P[idx];
    const double H = a.H0[b] + 0.5 * x * x + 0.5 * y * y + a.Hel[idx];
    const NodeState q = node_state(Pm, H, lc);
    a.eps[idx] = q.eps;
    a.rH[idx] = q.rH;
    a.rho[idx] = q.rho;
    a.drhoH[idx] = q.drhoH;
    a.eP[idx] = q.eP;
    a.eH[idx] = q.eH;
    uint8_t dir = 1;
    if (i > 0 && i < a.Nx - 1 && j > 0 && j < a.Ny - 1) {
        const double* P = a.P + (int64_t)b * per;
        const bool cav = Pm <= 0.0 || P[(i - 1) * a.Ny + j] <= 0.0 ||
                         P[(i + 1) * a.Ny + j] <= 0.0 || P[i * a.Ny + j - 1] <= 0.0 ||
                         P[i * a.Ny + j + 1] <= 0.0;
        dir = (fmin(q.eps / a.hx, q.eps / a.hy) > a.switch_ratio) || cav;
    }
    a.direct[idx] = dir;
}

int launch_point_nodes(const PointNodeArgs& a, hipStream_t s)
{
    const int64_t cnt = (int64_t)a.Nx * a.Ny * a.B;
    if (cnt <= 0) return PAQIF_OK;
    hipLaunchKernelGGL(point_node_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                       a);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

// Line geometry of one (axis, colour)
struct LineGeo {
    int axis, nl, nn, first, nlc;
    PQ_DEV int64_t node(int b, int Nx, int Ny, int l, int m) const
    {
        return axis == 0 ? ((int64_t)b * Nx + m) * Ny + l : ((int64_t)b * Nx + l) * Ny + m;
    }
};

PQ_DEV LineGeo line_geo(int Nx, int Ny, int axis, int color)
{
    LineGeo g;
    g.axis = axis;
    g.nl = axis == 0 ? Ny : Nx;
    g.nn = axis == 0 ? Nx : Ny;
    g.first = color == 1 ? 1 : 2;
    g.nlc = g.first <= g.nl - 2 ? (g.nl - 2 - g.first) / 2 + 1 : 0;
    return g;
}

int point_color_lines(int Nx, int Ny, int axis, int color)
{
    const int nl = axis == 0 ? Ny : Nx, first = color == 1 ? 1 : 2;
    return first <= nl - 2 ? (nl - 2 - first) / 2 + 1 : 0;
}

// Sixteen lanes per row of a line of the colour: lane 4 + s (s = -4..4)
// computes band entry s of -dR/dsigma, the row's rhs R + sum_s A_s P_(p+s)
// is a 16-lane shuffle sum, lane 4 writes it and the bounded mask (layout of
// paqif_solve_lcp, system = b * nlc + slot).  One thread per row had left a
// few hundred dependent loads per thread on a few waves per CU.
__global__ void __launch_bounds__(256) point_assemble_kernel(PointAssembleArgs a)
{
    const LineGeo g = line_geo(a.Nx, a.Ny, a.axis, a.color);
    const int n = g.nn - 2;
    const int64_t tid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;  // row
    const int lane_s = (int)(threadIdx.x & 15) - 4;  // band offset of this lane (-4..11)
    if (tid >= (int64_t)a.B * g.nlc * n) return;     // whole 16-lane groups
    const int r = (int)(tid % n);
    const int64_t sys = tid / n;
    const int b = (int)(sys / g.nlc), slot = (int)(sys % g.nlc);
    if (a.skip && a.skip[b]) return;
    const int l = g.first + 2 * slot, p = r + 1;
    const int Nx = a.Nx, Ny = a.Ny, nn = g.nn, nl = g.nl, kt = a.kterms;
    const double h_a = a.axis == 0 ? a.hx : a.hy, h_p = a.axis == 0 ? a.hy : a.hx;
    auto id = [&](int ll, int m) { return g.node(b, Nx, Ny, ll, m); };
    auto Pn = [&](int ll, int m) { return a.P[id(ll, m)]; };
    auto dist = [&](int ll, int m) { return a.direct[id(ll, m)] == 0; };
    auto ipos = [&](int m) { return m >= 1 && m <= nn - 2; };
    auto iline = [&](int ll) { return ll >= 1 && ll <= nl - 2; };
    const bool up_in = iline(l + 1), dn_in = iline(l - 1);
    // kernel at across-offset aa and along-offset d
    auto G = [&](int aa, int d) -> double {
        aa = abs(aa);
        d = abs(d);
        if (d >= nn || aa >= nl) return 0.0;
        return a.axis == 0 ? a.k2[(int64_t)d * Ny + aa] : a.k2[(int64_t)aa * Ny + d];
    };
    auto dPd = [&](int aa, int m, int k) -> double {
        if (aa == 0) {
            if (m == k) return 1.0;
            return (abs(m - k) == 1 && dist(l, k) && ipos(m)) ? -0.25 : 0.0;
        }
        if (abs(aa) == 1)
            return (m == k && dist(l, k) && ipos(m) && iline(l + aa)) ? -0.25 : 0.0;
        return 0.0;
    };
    auto dHd = [&](int aa, int m, int k) -> double {
        if (abs(m - k) > kt) return 0.0;
        double v = G(aa, m - k);
        if (dist(l, k)) {
            double c = 0.0;
            if (ipos(k - 1)) c += G(aa, m - k + 1);
            if (ipos(k + 1)) c += G(aa, m - k - 1);
            if (up_in) c += G(aa - 1, m - k);
            if (dn_in) c += G(aa + 1, m - k);
            v -= 0.25 * c;
        }
        return v;
    };
    // (splitting matrices: eps and rho held at the current iterate)
    const bool frozen = a.split != 0;
    auto dEps = [&](int m, int k) -> double {
        if (frozen || m < 0 || m >= nn) return 0.0;
        const int64_t q = id(l, m);
        return a.eP[q] * dPd(0, m, k) + a.eH[q] * dHd(0, m, k);
    };
    auto dRH = [&](int aa, int m, int k) -> double {
        if (m < 0 || m >= nn || l + aa < 0 || l + aa >= nl) return 0.0;
        const int64_t q = id(l + aa, m);
        return (frozen ? 0.0 : a.drhoH[q] * dPd(aa, m, k)) + a.rho[q] * dHd(aa, m, k);
    };
    auto eps = [&](int ll, int m) { return a.eps[id(ll, m)]; };
    auto rH = [&](int ll, int m) { return a.rH[id(ll, m)]; };

    // residual of the node (i, j) in grid terms
    double R;
    {
        const int i = a.axis == 0 ? p : l, j = a.axis == 0 ? l : p;
        const int64_t base = (int64_t)b * Nx * Ny;
        auto at = [&](const double* arr, int ii, int jj) { return arr[base + (int64_t)ii * Ny + jj]; };
        const double* P = a.P;
        const double exp_ = 0.5 * (at(a.eps, i, j) + at(a.eps, i + 1, j));
        const double exm = 0.5 * (at(a.eps, i, j) + at(a.eps, i - 1, j));
        const double eyp = 0.5 * (at(a.eps, i, j) + at(a.eps, i, j + 1));
        const double eym = 0.5 * (at(a.eps, i, j) + at(a.eps, i, j - 1));
        const double Pc = at(P, i, j);
        double psi, pa, pb;
        convective_slope(a.conv, a.kappa, a.limjac, at(a.rH, i, j) - at(a.rH, i - 1, j),
                         at(a.rH, i + 1, j) - at(a.rH, i, j), psi, pa, pb);
        const double fi = at(a.rH, i, j) + 0.5 * psi;
        double fm;
        if (i - 1 >= 1) {
            convective_slope(a.conv, a.kappa, a.limjac, at(a.rH, i - 1, j) - at(a.rH, i - 2, j),
                             at(a.rH, i, j) - at(a.rH, i - 1, j), psi, pa, pb);
            fm = at(a.rH, i - 1, j) + 0.5 * psi;
        } else {
            fm = at(a.rH, 0, j);
        }
        R = (exp_ * (at(P, i + 1, j) - Pc) - exm * (Pc - at(P, i - 1, j))) / (a.hx * a.hx) +
            (eyp * (at(P, i, j + 1) - Pc) - eym * (Pc - at(P, i, j - 1))) / (a.hy * a.hy) -
            (fi - fm) / a.hx;
    }

    double* brow = a.band + (sys * n + r) * 9;
    const int64_t ro = sys * n + r;
    const bool active = lane_s <= 4;
    if (a.axis == 1 && dist(l, p)) {  // y-lines leave weighted-change nodes alone
        if (active) brow[lane_s + 4] = lane_s == 0 ? 1.0 : 0.0;
        if (lane_s == 0) {
            a.rhs[ro] = Pn(l, p);
            a.bounded[ro] = 0;
        }
        return;
    }
    const double eph = 0.5 * (eps(l, p) + eps(l, p + 1));
    const double epm = 0.5 * (eps(l, p - 1) + eps(l, p));
    const double e_up = 0.5 * (eps(l, p) + eps(l + 1, p));
    const double e_dn = 0.5 * (eps(l, p) + eps(l - 1, p));
    double pa0 = 0, pb0 = 0, pa1 = 0, pb1 = 0;
    const int lj = a.limjac;
    if (a.axis == 0) {
        slope_partials(a.conv, a.kappa, lj, rH(l, p) - rH(l, p - 1), rH(l, p + 1) - rH(l, p), pa0,
                       pb0);
        if (p - 1 >= 1)
            slope_partials(a.conv, a.kappa, lj, rH(l, p - 1) - rH(l, p - 2),
                           rH(l, p) - rH(l, p - 1), pa1, pb1);
    } else {
        slope_partials(a.conv, a.kappa, lj, rH(l, p) - rH(l - 1, p), rH(l + 1, p) - rH(l, p), pa0,
                       pb0);
        if (l - 1 >= 1)
            slope_partials(a.conv, a.kappa, lj, rH(l - 1, p) - rH(l - 2, p),
                           rH(l, p) - rH(l - 1, p), pa1, pb1);
    }
    double contrib = 0.0;
    {
        const int s = lane_s;
        const int k = p + s;
        double Av = 0.0;
        if (active && k >= 1 && k <= nn - 2) {
            const double de_p = 0.5 * (dEps(p, k) + dEps(p + 1, k));
            const double de_m = 0.5 * (dEps(p - 1, k) + dEps(p, k));
            const double dPi = dPd(0, p, k);
            const double dA = de_p * (Pn(l, p + 1) - Pn(l, p)) + eph * (dPd(0, p + 1, k) - dPi);
            const double dB = de_m * (Pn(l, p) - Pn(l, p - 1)) + epm * (dPi - dPd(0, p - 1, k));
            const double along = (dA - dB) / (h_a * h_a);
            const double dEi = dEps(p, k);
            const double moved = (s == 0 && dist(l, p)) ? -0.25 : 0.0;
            const double d_up = up_in ? moved : 0.0, d_dn = dn_in ? moved : 0.0;
            const double across = (0.5 * dEi * (Pn(l + 1, p) - Pn(l, p)) + e_up * (d_up - dPi) -
                                   0.5 * dEi * (Pn(l, p) - Pn(l - 1, p)) - e_dn * (dPi - d_dn)) /
                                  (h_p * h_p);
            double conv;
            if (a.axis == 0) {
                const double fi = dRH(0, p, k) + 0.5 * (pa0 * (dRH(0, p + 1, k) - dRH(0, p, k)) +
                                                        pb0 * (dRH(0, p, k) - dRH(0, p - 1, k)));
                double fm;
                if (p - 1 >= 1)
                    fm = dRH(0, p - 1, k) + 0.5 * (pa1 * (dRH(0, p, k) - dRH(0, p - 1, k)) +
                                                   pb1 * (dRH(0, p - 1, k) - dRH(0, p - 2, k)));
                else
                    fm = dRH(0, 0, k);
                conv = (fi - fm) / h_a;
            } else {
                const double dm1 = dRH(-1, p, k), d0 = dRH(0, p, k), dp1 = dRH(1, p, k);
                const double fi = -0.5 * pb0 * dm1 + (1.0 + 0.5 * (pb0 - pa0)) * d0 + 0.5 * pa0 * dp1;
                double fm;
                if (l - 1 >= 1)
                    fm = -0.5 * pb1 * dRH(-2, p, k) + (1.0 + 0.5 * (pb1 - pa1)) * dm1 +
                         0.5 * pa1 * d0;
                else
                    fm = dm1;
                conv = (fi - fm) / h_p;
            }
            Av = -(along + across - a.csplit * conv);
            contrib = Av * Pn(l, k);
        }
        if (active) brow[s + 4] = Av;
    }
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1) contrib += __shfl_xor(contrib, m, 16);
    if (lane_s == 0) {
        a.rhs[ro] = R + contrib;
        a.bounded[ro] = (!dist(l, p) && !dist(l, p - 1) && !dist(l, p + 1)) ? 1 : 0;
    }
}

int launch_point_assemble(const PointAssembleArgs& a, hipStream_t s)
{
    const int nlc = point_color_lines(a.Nx, a.Ny, a.axis, a.color);
    const int n = (a.axis == 0 ? a.Nx : a.Ny) - 2;
    const int64_t cnt = (int64_t)a.B * nlc * n;  // rows, 16 lanes each
    if (cnt <= 0) return PAQIF_OK;
    hipLaunchKernelGGL(point_assemble_kernel, dim3((unsigned)((cnt * 16 + 255) / 256)), dim3(256),
                       0, s, a);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

// Weighted-change update after one colour: delta = sigma - (sigma / 4 of
// the distributive interior neighbours); P_out = max(0, P + omega delta).
__global__ void point_update_kernel(PointUpdateArgs a)
{
    const int64_t per = (int64_t)a.Nx * a.Ny;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per * a.B) return;
    const int b = (int)(idx / per);
    if (a.skip && a.skip[b]) return;
    const int rem = (int)(idx % per), i = rem / a.Ny, j = rem % a.Ny;
    const int Nx = a.Nx, Ny = a.Ny;
    const LineGeo g = line_geo(Nx, Ny, a.axis, a.color);
    const int n = g.nn - 2;
    const double* P = a.P + (int64_t)b * per;
    const uint8_t* dir = a.direct + (int64_t)b * per;
    auto interior = [&](int ii, int jj) { return ii >= 1 && ii <= Nx - 2 && jj >= 1 && jj <= Ny - 2; };
    auto sigma = [&](int ii, int jj) -> double {
        if (!interior(ii, jj)) return 0.0;
        const int ll = a.axis == 0 ? jj : ii, m = a.axis == 0 ? ii : jj;
        if ((ll & 1) != a.color) return 0.0;
        if (a.axis == 1 && !dir[ii * Ny + jj]) return 0.0;
        const int slot = (ll - g.first) / 2;
        return a.v[((int64_t)b * g.nlc + slot) * n + m - 1] - P[ii * Ny + jj];
    };
    double out = P[i * Ny + j];
    if (interior(i, j)) {
        double d = sigma(i, j);
        auto nb = [&](int ii, int jj) {
            return (interior(ii, jj) && !dir[ii * Ny + jj]) ? sigma(ii, jj) : 0.0;
        };
        d -= 0.25 * (nb(i - 1, j) + nb(i + 1, j) + nb(i, j - 1) + nb(i, j + 1));
        out = fmax(0.0, out + a.omega * d);
    }
    a.Pout[idx] = out;
}

int launch_point_update(const PointUpdateArgs& a, hipStream_t s)
{
    const int64_t cnt = (int64_t)a.Nx * a.Ny * a.B;
    if (cnt <= 0) return PAQIF_OK;
    hipLaunchKernelGGL(point_update_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                       a);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

// H0 relaxation (eq. 75, load 2 pi / 3) after a sweep direction; with
// check, the end-of-step convergence test against the step's start.
__global__ void __launch_bounds__(1024) point_h0_kernel(PointH0Args a, int check)
{
    const int b = blockIdx.x;
    if (a.done[b]) return;
    const int64_t per = (int64_t)a.Nx * a.Ny;
    const double* P = a.P + (int64_t)b * per;
    double* Ps = a.Pstart + (int64_t)b * per;
    __shared__ double sh[3][32];
    double sum = 0.0, dmax = 0.0, pmax = 0.0;
    bool fin = true;
    for (int64_t q = threadIdx.x; q < per; q += blockDim.x) {
        const double v = P[q];
        sum += v;
        if (!isfinite(v)) fin = false;
        if (check) {
            dmax = fmax(dmax, fabs(v - Ps[q]));
            pmax = fmax(pmax, v);
            Ps[q] = v;
        }
    }
    if (!fin) dmax = INFINITY;
    // wave reductions, then across the 16 waves in a fixed order
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        sum += __shfl_xor(sum, m, 64);
        dmax = fmax(dmax, __shfl_xor(dmax, m, 64));
        pmax = fmax(pmax, __shfl_xor(pmax, m, 64));
    }
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = sum;
        sh[1][w] = dmax;
        sh[2][w] = pmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double S = 0.0, D = 0.0, Pm = 0.0;
        for (int k = 0; k < nw; k++) {
            S += sh[0][k];
            D = fmax(D, sh[1][k]);
            Pm = fmax(Pm, sh[2][k]);
        }
        const double err = a.load_target - a.hx * a.hy * S;
        a.H0[b] -= a.c_h0 * err;
        if (check) {
            // end of an x+y step: the worst LCP status of its four colour passes
            const int lst = a.step_lcp[b];
            a.step_lcp[b] = SYS_OK;
            const int fails = lcp_failed(lst) ? a.lcp_fails[b] + 1 : 0;
            a.lcp_fails[b] = fails;
            a.iters[b] += 1;
            if (!isfinite(D) || !isfinite(S)) {
                a.status[b] = SYS_NONFINITE;
                a.done[b] = 1;
            } else if (lcp_fatal(lst)) {
                a.status[b] = lst;
                a.done[b] = 1;
            } else if (D <= a.tol * fmax(1.0, Pm) && fabs(err) <= a.tol) {
                a.status[b] = SYS_OK;
                a.done[b] = 1;
            } else if (fails >= a.fail_steps) {
                a.status[b] = lst;
                a.done[b] = 1;
            }
        }
    }
}

// One wavefront per instance: the worst (by lcp_severity) status over the
// instance's lines of one colour pass, folded into its step status.
__global__ void __launch_bounds__(64) point_lcp_status_kernel(int nlc, const int32_t* lst,
                                                             const uint8_t* done, int32_t* step)
{
    const int b = blockIdx.x;
    if (done[b]) return;
    int worst = SYS_OK, sev = 0;
    for (int l = threadIdx.x; l < nlc; l += 64) {
        const int st = lst[(int64_t)b * nlc + l];
        const int sv = lcp_severity(st);
        if (sv > sev) {
            sev = sv;
            worst = st;
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const int os = __shfl_xor(sev, m, 64), ow = __shfl_xor(worst, m, 64);
        if (os > sev) {
            sev = os;
            worst = ow;
        }
    }
    if (threadIdx.x == 0 && sev > lcp_severity(step[b])) step[b] = worst;
}

int launch_point_lcp_status(int B, int nlc, const int32_t* lst, const uint8_t* done,
                            int32_t* step_lcp, hipStream_t s)
{
    if (B <= 0 || nlc <= 0) return PAQIF_OK;
    hipLaunchKernelGGL(point_lcp_status_kernel, dim3(B), dim3(64), 0, s, nlc, lst, done, step_lcp);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

int launch_point_h0(const PointH0Args& a, int check, hipStream_t s)
{
    if (a.B <= 0) return PAQIF_OK;
    hipLaunchKernelGGL(point_h0_kernel, dim3(a.B), dim3(1024), 0, s, a, check);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

// Hertzian start on the 2D grid and the start rule for H0:
// H0 = 0.4 / sqrt(M) - min over the unit circle of (X^2 + Y^2)/2 + H_el.
__global__ void point_hertz_kernel(int Nx, int Ny, int B, double x0, double y0, double hx,
                                   double hy, double* P)
{
    const int64_t per = (int64_t)Nx * Ny;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per * B) return;
    const int rem = (int)(idx % per), i = rem / Ny, j = rem % Ny;
    const double x = x0 + hx * i, y = y0 + hy * j;
    const bool edge = i == 0 || j == 0 || i == Nx - 1 || j == Ny - 1;
    P[idx] = edge ? 0.0 : sqrt(fmax(0.0, 1.0 - x * x - y * y));
}

__global__ void __launch_bounds__(256) point_h0_rule_kernel(int Nx, int Ny, double x0, double y0,
                                                            double hx, double hy,
                                                            const ehl_params* params,
                                                            const double* Hel, double* H0)
{
    const int b = blockIdx.x;
    const int64_t per = (int64_t)Nx * Ny;
    __shared__ double sh[4];
    double mn = INFINITY;
    for (int64_t q = threadIdx.x; q < per; q += blockDim.x) {
        const int i = (int)(q / Ny), j = (int)(q % Ny);
        const double x = x0 + hx * i, y = y0 + hy * j;
        if (x * x + y * y <= 1.0) mn = fmin(mn, 0.5 * (x * x + y * y) + Hel[(int64_t)b * per + q]);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) mn = fmin(mn, __shfl_xor(mn, m, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mn;
    __syncthreads();
    if (threadIdx.x == 0)
        H0[b] = 0.4 / sqrt(params[b].M) - fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
}

int launch_point_start(int Nx, int Ny, int B, double x0, double y0, double hx, double hy,
                       double* P, hipStream_t s)
{
    const int64_t cnt = (int64_t)Nx * Ny * B;
    if (cnt <= 0) return PAQIF_OK;
    hipLaunchKernelGGL(point_hertz_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                       Nx, Ny, B, x0, y0, hx, hy, P);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

int launch_point_h0_rule(int Nx, int Ny, int B, double x0, double y0, double hx, double hy,
                         const ehl_params* params, const double* Hel, double* H0, hipStream_t s)
{
    if (B <= 0) return PAQIF_OK;
    hipLaunchKernelGGL(point_h0_rule_kernel, dim3(B), dim3(256), 0, s, Nx, Ny, x0, y0, hx, hy,
                       params, Hel, H0);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

// film H = H0 + (X^2 + Y^2)/2 + H_el and its minimum per instance
__global__ void __launch_bounds__(256) point_film_kernel(int Nx, int Ny, double x0, double y0,
                                                         double hx, double hy, const double* Hel,
                                                         const double* H0, double* H,
                                                         double* Hmin)
{
    const int b = blockIdx.x;
    const int64_t per = (int64_t)Nx * Ny;
    __shared__ double sh[4];
    double mn = INFINITY;
    for (int64_t q = threadIdx.x; q < per; q += blockDim.x) {
        const int i = (int)(q / Ny), j = (int)(q % Ny);
        const double x = x0 + hx * i, y = y0 + hy * j;
        const double v = H0[b] + 0.5 * (x * x + y * y) + Hel[(int64_t)b * per + q];
        if (H) H[(int64_t)b * per + q] = v;
        mn = fmin(mn, v);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) mn = fmin(mn, __shfl_xor(mn, m, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mn;
    __syncthreads();
    if (threadIdx.x == 0 && Hmin) Hmin[b] = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
}

int launch_point_film(int Nx, int Ny, int B, double x0, double y0, double hx, double hy,
                      const double* Hel, const double* H0, double* H, double* Hmin, hipStream_t s)
{
    if (B <= 0) return PAQIF_OK;
    hipLaunchKernelGGL(point_film_kernel, dim3(B), dim3(256), 0, s, Nx, Ny, x0, y0, hx, hy, Hel,
                       H0, H, Hmin);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

}  // namespace pq
