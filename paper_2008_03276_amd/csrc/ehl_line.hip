// EHL line contact on gfx950: assembly of the linearised complementarity
// problem of the hybrid Newton line method, pressure update with the
// load-balance relaxation, Hertzian start and film evaluation.
//
// Paper Sec. 3.3 (line contact): Reynolds operator with the TVD
// finite-volume flux (eqs. 62-65), hybrid switch (eq. 60), weighted change
// (eqs. 69-74, one-dimensional form), H0 relaxation (eq. 75); lubricant
// models (Roelands viscosity, Dowson-Higginson density) and Moes parameters
// of the appendix.
//
// Assembly: one workgroup per tile of 256 interior rows of one instance.
// The node quantities (film, density, viscosity, eps, rho*H and their
// pressure/film derivatives) of the tile plus a halo of 5 nodes are computed
// once into LDS; every thread then forms its residual and the 9 band
// entries of dR/dsigma through the chain rule on that window.
#include "common.h"
#include "ehl_internal.h"
#include "ehl_model.h"

namespace pq {

namespace {
constexpr int TILE = 256;
constexpr int HALO = 5;
constexpr int WIN = TILE + 2 * HALO;
}  // namespace

__global__ void __launch_bounds__(TILE) line_assemble_kernel(LineAssembleArgs a)
{
    const int b = blockIdx.y;
    if (a.skip && a.skip[b]) return;
    const int N = a.N, n = N - 2;
    const int r0 = blockIdx.x * TILE;  // first interior row (node r0+1)
    const int t = threadIdx.x;
    const double h = a.h;
    const LineConst lc = line_const(a.params[b].M, a.params[b].L);
    const double H0 = a.H0[b];
    const double* P = a.P + (int64_t)b * N;
    const double* Hel = a.Hel + (int64_t)b * N;
    const double* rough = a.rough ? a.rough + (int64_t)b * N : nullptr;

    __shared__ double sP[WIN], sH[WIN], sEps[WIN], sRH[WIN], sEP[WIN], sEH[WIN], sRho[WIN],
        sDrhoH[WIN];
    __shared__ unsigned char sDist[WIN], sDirect[WIN];
    const int mbase = r0 + 1 - HALO;  // node of window slot 0

    for (int w = t; w < WIN; w += TILE) {
        const int m = mbase + w;
        double Pm = 0, Hm = 0, eps = 0, rH = 0, eP = 0, eH = 0, rho = 0, drhoH = 0;
        if (m >= 0 && m < N) {
            const double x = a.x0 + h * m;
            Pm = P[m];
            Hm = H0 + 0.5 * x * x + Hel[m] + (rough ? rough[m] : 0.0);
            const NodeState q = node_state(Pm, Hm, lc);
            eps = q.eps;
            rH = q.rH;
            eP = q.eP;
            eH = q.eH;
            rho = q.rho;
            drhoH = q.drhoH;
        }
        sP[w] = Pm;
        sH[w] = Hm;
        sEps[w] = eps;
        sRH[w] = rH;
        sEP[w] = eP;
        sEH[w] = eH;
        sRho[w] = rho;
        sDrhoH[w] = drhoH;
    }
    __syncthreads();
    // hybrid switch: direct where eps/h > switch or next to cavitation
    for (int w = t; w < WIN; w += TILE) {
        const int m = mbase + w;
        unsigned char dir = 1, dist = 0;
        if (m >= 0 && m < N && w > 0 && w < WIN - 1) {
            const bool cav = sP[w - 1] <= 0.0 || sP[w] <= 0.0 || sP[w + 1] <= 0.0;
            dir = (sEps[w] / h > a.switch_ratio) || cav;
            dist = (!dir) && m >= 1 && m <= N - 2;
        }
        sDirect[w] = dir;
        sDist[w] = dist;
    }
    __syncthreads();
    if (a.direct) {
        for (int w = HALO + t; w < HALO + TILE; w += TILE) {
            const int m = mbase + w;
            if (m >= 1 && m <= N - 2) a.direct[(int64_t)b * N + m] = sDirect[w];
        }
        if (r0 == 0 && t == 0) {
            a.direct[(int64_t)b * N] = 1;
            a.direct[(int64_t)b * N + N - 1] = 1;
        }
    }

    const int r = r0 + t;
    if (r >= n) return;
    const int i = r + 1;
    const int wi = i - mbase;  // window slot of node i
    const int kt = a.kterms;
    double kap[4];
#pragma unroll
    for (int e = 0; e < 4; e++) kap[e] = e < N ? (a.kvec ? a.kvec[e] : a.kap[e]) : 0.0;
    auto K = [&](int d) { d = abs(d); return d < 4 ? kap[d] : 0.0; };
    auto interior = [&](int m) { return m >= 1 && m <= N - 2; };
    auto distk = [&](int k) { return sDist[k - mbase] != 0; };
    // D[m][k] and (K D)[m][k] (cut to |m-k| <= kt) for interior column k
    auto Dc = [&](int k, int m) -> double {
        if (m == k) return 1.0;
        if (abs(m - k) == 1 && distk(k) && interior(m)) return -0.5;
        return 0.0;
    };
    auto KDc = [&](int k, int m) -> double {
        const int d = m - k;
        if (abs(d) > kt) return 0.0;
        double v = K(d);
        if (distk(k)) {
            if (interior(k - 1)) v -= 0.5 * K(d + 1);
            if (interior(k + 1)) v -= 0.5 * K(d - 1);
        }
        return v;
    };
    // node quantities
    auto Pn = [&](int m) { return sP[m - mbase]; };
    auto epsn = [&](int m) { return sEps[m - mbase]; };
    auto rHn = [&](int m) { return sRH[m - mbase]; };
    // derivatives of node quantities wrt sigma_k
    auto dP = [&](int m, int k) { return (m < 0 || m >= N) ? 0.0 : Dc(k, m); };
    // (splitting matrices: eps and rho held at the current iterate, so only
    // the pressure and the film move)
    const bool frozen = a.split != 0;
    auto dEps = [&](int m, int k) {
        if (frozen || m < 0 || m >= N) return 0.0;
        const int w = m - mbase;
        return sEP[w] * Dc(k, m) + sEH[w] * KDc(k, m);
    };
    auto dRH = [&](int m, int k) {
        if (m < 0 || m >= N) return 0.0;
        const int w = m - mbase;
        return (frozen ? 0.0 : sDrhoH[w] * Dc(k, m)) + sRho[w] * KDc(k, m);
    };
    // limiter at node tt (1 <= tt <= N-2)
    auto limiter = [&](int tt, double& psi, double& pa, double& pb) {
        const double dm = rHn(tt) - rHn(tt - 1), dp = rHn(tt + 1) - rHn(tt);
        convective_slope(a.conv, a.kappa, a.limjac, dm, dp, psi, pa, pb);
    };
    // residual
    const double eph = 0.5 * (epsn(i) + epsn(i + 1));
    const double epm = 0.5 * (epsn(i - 1) + epsn(i));
    double psi_i, pa_i, pb_i, psi_m, pa_m, pb_m;
    limiter(i, psi_i, pa_i, pb_i);
    const double f_i = rHn(i) + 0.5 * psi_i;
    double f_m;
    if (i - 1 >= 1) {
        limiter(i - 1, psi_m, pa_m, pb_m);
        f_m = rHn(i - 1) + 0.5 * psi_m;
    } else {
        psi_m = pa_m = pb_m = 0.0;
        f_m = rHn(0);
    }
    const double Rres =
        (eph * (Pn(i + 1) - Pn(i)) - epm * (Pn(i) - Pn(i - 1))) / (h * h) - (f_i - f_m) / h;

    double* brow = a.band + ((int64_t)b * n + r) * 9;
    double rhs = Rres;
#pragma unroll
    for (int s = -4; s <= 4; s++) {
        const int k = i + s;
        double Aval = 0.0;
        if (k >= 1 && k <= N - 2) {
            const double de_p = 0.5 * (dEps(i, k) + dEps(i + 1, k));
            const double de_m = 0.5 * (dEps(i - 1, k) + dEps(i, k));
            const double dA = de_p * (Pn(i + 1) - Pn(i)) + eph * (dP(i + 1, k) - dP(i, k));
            const double dB = de_m * (Pn(i) - Pn(i - 1)) + epm * (dP(i, k) - dP(i - 1, k));
            const double df_i =
                dRH(i, k) +
                0.5 * (pa_i * (dRH(i + 1, k) - dRH(i, k)) + pb_i * (dRH(i, k) - dRH(i - 1, k)));
            double df_m;
            if (i - 1 >= 1)
                df_m = dRH(i - 1, k) + 0.5 * (pa_m * (dRH(i, k) - dRH(i - 1, k)) +
                                              pb_m * (dRH(i - 1, k) - dRH(i - 2, k)));
            else
                df_m = dRH(0, k);
            const double J = (dA - dB) / (h * h) - a.csplit * (df_i - df_m) / h;
            Aval = -J;
            rhs += Aval * Pn(k);
        }
        brow[s + 4] = Aval;
    }
    if (a.R) a.R[(int64_t)b * n + r] = Rres;
    a.rhs[(int64_t)b * n + r] = rhs;
    a.bounded[(int64_t)b * n + r] =
        (sDirect[wi] && sDirect[wi - 1] && sDirect[wi + 1]) ? 1 : 0;
}

int launch_line_assemble(const LineAssembleArgs& a, hipStream_t s)
{
    const int n = a.N - 2;
    if (n <= 0 || a.B <= 0) return PAQIF_OK;
    dim3 grid((n + TILE - 1) / TILE, a.B);
    hipLaunchKernelGGL(line_assemble_kernel, grid, dim3(TILE), 0, s, a);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

// --------------------------------------------------------------------------
// Pressure update and load balance, one workgroup per instance.
// --------------------------------------------------------------------------
template <typename T, typename Op>
PQ_DEV T block_reduce(T v, T* sh, Op op)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] = op(sh[t], sh[t + w]);
        __syncthreads();
    }
    const T r = sh[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(256) line_update_kernel(LineUpdateArgs a, double* Pnew)
{
    const int b = blockIdx.x;
    if (a.done[b]) return;
    const int N = a.N, n = N - 2;
    double* P = a.P + (int64_t)b * N;
    double* Pn = Pnew + (int64_t)b * N;
    const double* v = a.v + (int64_t)b * n;
    const uint8_t* dir = a.direct + (int64_t)b * N;
    __shared__ double sh[256];
    double dmax = 0.0, pmax = 0.0, sum = 0.0;
    bool finite = true;
    auto sigma = [&](int k) { return (k >= 1 && k <= N - 2) ? v[k - 1] - P[k] : 0.0; };
    auto dist = [&](int k) { return k >= 1 && k <= N - 2 && !dir[k]; };
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double pn = 0.0;
        if (i >= 1 && i <= N - 2) {
            double d = sigma(i);
            if (dist(i - 1)) d -= 0.5 * sigma(i - 1);
            if (dist(i + 1)) d -= 0.5 * sigma(i + 1);
            pn = fmax(0.0, P[i] + a.omega * d);
            if (!isfinite(P[i] + a.omega * d)) finite = false;
        }
        Pn[i] = pn;
        dmax = fmax(dmax, fabs(pn - P[i]));
        pmax = fmax(pmax, pn);
        sum += pn;
    }
    dmax = block_reduce(dmax, sh, [](double x, double y) { return fmax(x, y); });
    pmax = block_reduce(pmax, sh, [](double x, double y) { return fmax(x, y); });
    sum = block_reduce(sum, sh, [](double x, double y) { return x + y; });
    const double fin = block_reduce(finite ? 0.0 : 1.0, sh,
                                    [](double x, double y) { return fmax(x, y); });
    for (int i = threadIdx.x; i < N; i += blockDim.x) P[i] = Pn[i];
    if (threadIdx.x == 0) {
        const double load = a.h * sum;
        const double err = a.load_target - load;
        a.H0[b] = a.H0[b] - a.c_h0 * err;
        a.iters[b] += 1;
        a.dP[b] = dmax;
        a.load_err[b] = err;
        const int lst = a.lcp_status[b];
        const int fails = lcp_failed(lst) ? a.lcp_fails[b] + 1 : 0;
        a.lcp_fails[b] = fails;
        if (fin != 0.0 || !isfinite(dmax) || !isfinite(sum)) {
            a.status[b] = SYS_NONFINITE;
            a.done[b] = 1;
        } else if (lcp_fatal(lst)) {
            a.status[b] = lst;
            a.done[b] = 1;
        } else if (dmax <= a.tol * fmax(1.0, pmax) && fabs(err) <= a.tol) {
            a.status[b] = SYS_OK;
            a.done[b] = 1;
        } else if (fails >= a.fail_steps) {
            a.status[b] = lst;
            a.done[b] = 1;
        } else if (dmax < a.best_dP[b]) {
            a.best_dP[b] = dmax;
            a.best_step[b] = a.iters[b];
        } else if (a.stall_steps > 0 && a.iters[b] - a.best_step[b] >= a.stall_steps) {
            // stalled: a limit cycle or a drift above the rounding floor
            a.status[b] = SYS_NEWTON_NOT_CONVERGED;
            a.done[b] = 1;
        }
    }
}

int launch_line_update_ws(const LineUpdateArgs& a, double* Pnew, hipStream_t s)
{
    if (a.B <= 0) return PAQIF_OK;
    hipLaunchKernelGGL(line_update_kernel, dim3(a.B), dim3(256), 0, s, a, Pnew);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

// --------------------------------------------------------------------------
// Hertzian start, H0 start rule, film and its minimum.
// --------------------------------------------------------------------------
__global__ void line_hertz_kernel(int N, int B, double h, double x0, double* P)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * B) return;
    const int i = (int)(idx % N);
    const double x = x0 + h * i;
    P[idx] = (i == 0 || i == N - 1) ? 0.0 : sqrt(fmax(0.0, 1.0 - x * x));
}

int launch_line_hertz(const LineInitArgs& a, hipStream_t s)
{
    const int64_t cnt = (int64_t)a.N * a.B;
    if (cnt <= 0) return PAQIF_OK;
    hipLaunchKernelGGL(line_hertz_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                       a.N, a.B, a.h, a.x0, a.P);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

__global__ void __launch_bounds__(256) line_h0_kernel(int N, double h, double x0,
                                                      const ehl_params* params,
                                                      const double* Hel, double* H0)
{
    const int b = blockIdx.x;
    __shared__ double sh[256];
    double mn = INFINITY;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double x = x0 + h * i;
        if (fabs(x) <= 1.0) mn = fmin(mn, 0.5 * x * x + Hel[(int64_t)b * N + i]);
    }
    mn = block_reduce(mn, sh, [](double x, double y) { return fmin(x, y); });
    if (threadIdx.x == 0) H0[b] = 0.4 / sqrt(params[b].M) - mn;
}

int launch_line_h0_rule(int N, int B, double h, double x0, const ehl_params* params,
                        const double* Hel, double* H0, hipStream_t s)
{
    if (B <= 0) return PAQIF_OK;
    hipLaunchKernelGGL(line_h0_kernel, dim3(B), dim3(256), 0, s, N, h, x0, params, Hel, H0);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

__global__ void __launch_bounds__(256) line_film_kernel(int N, double h, double x0,
                                                        const double* Hel, const double* H0,
                                                        const double* rough, double* H,
                                                        double* Hmin, int32_t* argmin)
{
    const int b = blockIdx.x;
    __shared__ double sv[256];
    __shared__ int si[256];
    double mn = INFINITY;
    int mi = N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double x = x0 + h * i;
        const int64_t g = (int64_t)b * N + i;
        const double v = H0[b] + 0.5 * x * x + Hel[g] + (rough ? rough[g] : 0.0);
        if (H) H[g] = v;
        if (v < mn) {
            mn = v;
            mi = i;
        }
    }
    const int t = threadIdx.x;
    sv[t] = mn;
    si[t] = mi;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w) {
            const double a2 = sv[t + w];
            const int i2 = si[t + w];
            if (a2 < sv[t] || (a2 == sv[t] && i2 < si[t])) {
                sv[t] = a2;
                si[t] = i2;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        if (Hmin) Hmin[b] = sv[0];
        if (argmin) argmin[b] = si[0];
    }
}

int launch_line_film(int N, int B, double h, double x0, const double* Hel, const double* H0,
                     const double* rough, double* H, double* Hmin, int32_t* argmin,
                     hipStream_t s)
{
    if (B <= 0) return PAQIF_OK;
    hipLaunchKernelGGL(line_film_kernel, dim3(B), dim3(256), 0, s, N, h, x0, Hel, H0, rough, H,
                       Hmin, argmin);
    return hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

}  // namespace pq
