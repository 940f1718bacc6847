// C ABI of the EHL part: deformation, assembly and the Newton line driver.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "ehl_internal.h"
#include "paqif_args.h"

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

bool valid_line(const ehl_grid* g) { return g && g->ny == 1 && g->nx >= 5 && g->nx <= 8192 && g->x1 > g->x0; }

bool valid_point(const ehl_grid* g)
{
    return g && g->ny > 1 && g->nx >= 2 && g->nx <= 2048 && g->ny <= 2048 && g->x1 > g->x0 &&
           g->y1 > g->y0;
}

double hx_of(const ehl_grid* g) { return (g->x1 - g->x0) / (g->nx - 1); }
double hy_of(const ehl_grid* g) { return (g->y1 - g->y0) / (g->ny - 1); }

// deformation workspace: kernel vector / table, then point partial sums
size_t deform_ws_bytes(const ehl_grid* g, int B)
{
    if (valid_line(g)) return a256((size_t)g->nx * sizeof(double));
    if (valid_point(g))
        return a256((size_t)pq::point_workspace_doubles(g->nx, g->ny, B) * sizeof(double));
    return 0;
}

int run_deformation(const ehl_grid* g, const double* P, int B, int prec, double* out, char* ws,
                    bool kernel_ready, hipStream_t s)
{
    double* k = reinterpret_cast<double*>(ws);
    if (valid_line(g)) {
        if (!kernel_ready) {
            const int st = pq::launch_line_kernel_vec(g->nx, hx_of(g), k, s);
            if (st) return st;
        }
        return pq::launch_line_deform(g->nx, B, prec, k, P, out, s);
    }
    if (!kernel_ready) {
        const int st = pq::launch_point_kernel_tab(g->nx, g->ny, hx_of(g), hy_of(g), k, s);
        if (st) return st;
    }
    double* part = k + (size_t)g->nx * g->ny;
    return pq::launch_point_deform(g->nx, g->ny, B, prec, k, P, out, part, s);
}

// k[0..3] of the line kernel on the host (same closed form as the device
// kernel vector): k[m] = -(1/pi) (F((m+1/2)h) - F((m-1/2)h)), F(t) = t ln|t| - t.
void host_kernel_head(double h, double kap[4])
{
    auto F = [](double t) { return t == 0.0 ? 0.0 : t * std::log(std::fabs(t)) - t; };
    for (int m = 0; m < 4; m++) kap[m] = -(F((m + 0.5) * h) - F((m - 0.5) * h)) / M_PI;
}

// Consecutive failed linearised LCPs after which an instance stops.
int fail_steps(const ehl_opts* o) { return o->lcp_fail_steps > 0 ? o->lcp_fail_steps : 16; }

// Rounding floor of the Newton change in FP64 on a line of n nodes: the
// stopping test uses max(tol, 4 n eps), eps = 2^-52 (measured floors: about
// 1.5e-13 at n = 1025 and 6e-13 at n = 2049, which a fixed 1e-13 never meets).
double fp64_floor(int n) { return 4.0 * n * 2.220446049250313e-16; }

bool valid_convection(const ehl_opts* o)
{
    return o->convection == 0 || (o->convection == 1 && o->kappa >= -1.0 && o->kappa <= 1.0);
}

// Weight of the upwind convective derivative in the splitting matrices
// (Sec. 3.3.2): Lhs1 (2-k)/2, Lhs2 (2-k)/2 + (1-k)/4, k = kappa for the
// kappa-scheme, 0 for the limited slope.
double splitting_weight(const ehl_opts* o)
{
    const double k = o->convection == 1 ? o->kappa : 0.0;
    if (o->splitting == 1) return 0.5 * (2.0 - k);
    if (o->splitting == 2) return 0.5 * (2.0 - k) + 0.25 * (1.0 - k);
    return 1.0;
}

// Assembly arguments shared by the line and point kernels: slope, limiter
// matrix and splitting.
template <typename Args>
void set_scheme(Args& a, const ehl_opts* o)
{
    a.conv = o->convection;
    a.kappa = o->kappa;
    a.split = o->splitting;
    a.csplit = splitting_weight(o);
    a.limjac = o->splitting != 0 ? 2 : o->limiter_jacobian;
}

bool valid_opts(const ehl_opts* o)
{
    return o && o->omega > 0 && o->omega <= 1.0 && o->c_h0 > 0 && o->tol > 0 &&
           o->max_newton >= 1 && (o->kernel_terms == 1 || o->kernel_terms == 2) &&
           o->lcp_max_iter >= 1 &&
           (o->deform_prec == PREC_FP64 || o->deform_prec == PREC_FP32 ||
            o->deform_prec == PREC_SPLIT_BF16) &&
           (o->lcp_prec == PREC_FP64 || o->lcp_prec == PREC_FP32_IR) &&
           o->steps_per_graph >= 1 && o->steps_per_graph <= 64 && o->limiter_jacobian >= 0 &&
           o->limiter_jacobian <= 2 && o->stall_steps >= 0 && o->lcp_fail_steps >= 0 &&
           o->splitting >= 0 && o->splitting <= 2 && valid_convection(o);
}

// Newton workspace layout (line contact)
struct NewtonLayout {
    size_t kvec, hel, band, rhs, v, pn, bounded, direct, done, dP, lerr, offs, lst, lit, lfail,
        best, bstep, lcp, total;
};

size_t lcp_ws_bytes(int B, int n, int prec)
{
    // same as paqif_workspace_bytes for a batch of B systems of order n, q = 4
    const size_t recs = (size_t)(((int64_t)B * n + B) / 2 + 1);
    const size_t elt = prec == PREC_FP32_IR ? sizeof(float) : sizeof(double);
    size_t t = a256(recs * (size_t)pq::record_stride(4, true) * elt);
    t += a256((size_t)B * n);
    if (prec == PREC_FP32_IR) t += a256((size_t)B * n * sizeof(double));
    return t;
}

NewtonLayout newton_layout(const ehl_grid* g, int B, const ehl_opts* o)
{
    const size_t N = g->nx, n = N - 2, b = B;
    NewtonLayout L;
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p += a256(bytes);
        return at;
    };
    L.kvec = take(N * sizeof(double));
    L.hel = take(N * b * sizeof(double));
    L.band = take(n * b * 9 * sizeof(double));
    L.rhs = take(n * b * sizeof(double));
    L.v = take(n * b * sizeof(double));
    L.pn = take(N * b * sizeof(double));
    L.bounded = take(n * b);
    L.direct = take(N * b);
    L.done = take(b);
    L.dP = take(b * sizeof(double));
    L.lerr = take(b * sizeof(double));
    L.offs = take((b + 1) * sizeof(int64_t));
    L.lst = take(b * sizeof(int32_t));
    L.lit = take(b * sizeof(int32_t));
    L.lfail = take(b * sizeof(int32_t));
    L.best = take(b * sizeof(double));
    L.bstep = take(b * sizeof(int32_t));
    L.lcp = take(lcp_ws_bytes(B, (int)n, o ? o->lcp_prec : PREC_FP64));
    L.total = p;
    return L;
}

__global__ void init_newton_kernel(int B, int n, int64_t* offs, uint8_t* done, int32_t* status,
                                   int32_t* iters)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= B) offs[i] = (int64_t)i * n;
    if (i < B) {
        done[i] = 0;
        status[i] = SYS_NEWTON_NOT_CONVERGED;
        iters[i] = 0;
    }
}

// Before an FP64 refresh phase: instances that converged under the
// low-precision deformation go on; non-finite ones and those whose band
// matrix had a singular pivot stay stopped.
__global__ void reopen_kernel(int B, uint8_t* done, int32_t* status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B && status[i] != SYS_NONFINITE && status[i] != SYS_ZERO_PIVOT) {
        done[i] = 0;
        status[i] = SYS_NEWTON_NOT_CONVERGED;
    }
}

__global__ void stall_init_kernel(int B, double* best, int32_t* step, const int32_t* iters)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B) {
        best[i] = INFINITY;
        step[i] = iters[i];
    }
}

__global__ void final_status_kernel(int B, const uint8_t* done, const double* Hmin,
                                    int32_t* status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B) {
        if (!done[i])
            status[i] = SYS_NEWTON_NOT_CONVERGED;
        else if (status[i] == SYS_OK && !(Hmin[i] > 0.0))
            status[i] = SYS_NEGATIVE_FILM;
    }
}


// ---------------------------------------------------------------------------
// Point contact (2D grid): workspace and driver.
// ---------------------------------------------------------------------------
struct PointLayout {
    size_t dws, hel, nodes, direct, q, pstart, band, rhs, v, bounded, done, offs[4], act[4], lst,
        lit, pst, pfail, lcp, total;
    int nlc[4], nrow[4];  // (axis, colour) -> lines per instance, rows per line
};

PointLayout point_layout(const ehl_grid* g, int B, const ehl_opts* o)
{
    PointLayout L;
    const size_t cells = (size_t)g->nx * g->ny * B;
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p += a256(bytes);
        return at;
    };
    L.dws = take(deform_ws_bytes(g, B));
    L.hel = take(cells * sizeof(double));
    L.nodes = take(6 * cells * sizeof(double));
    L.direct = take(cells);
    L.q = take(cells * sizeof(double));
    L.pstart = take(cells * sizeof(double));
    size_t rows_max = 0;
    int cnt_max = 0, n_max = 0;
    for (int ax = 0; ax < 2; ax++)
        for (int c = 0; c < 2; c++) {
            const int k = 2 * ax + c;
            L.nlc[k] = pq::point_color_lines(g->nx, g->ny, ax, c);
            L.nrow[k] = (ax == 0 ? g->nx : g->ny) - 2;
            rows_max = std::max(rows_max, (size_t)L.nlc[k] * L.nrow[k] * B);
            cnt_max = std::max(cnt_max, L.nlc[k] * B);
            n_max = std::max(n_max, L.nrow[k]);
        }
    L.band = take(rows_max * 9 * sizeof(double));
    L.rhs = take(rows_max * sizeof(double));
    L.v = take(rows_max * sizeof(double));
    L.bounded = take(rows_max);
    L.done = take(B);
    for (int k = 0; k < 4; k++) L.offs[k] = take((size_t)(L.nlc[k] * B + 1) * sizeof(int64_t));
    // active flags of each colour pass, kept from one step to the next
    for (int k = 0; k < 4; k++) L.act[k] = take((size_t)L.nlc[k] * L.nrow[k] * B);
    L.lst = take((size_t)cnt_max * sizeof(int32_t));
    L.lit = take((size_t)cnt_max * sizeof(int32_t));
    L.pst = take((size_t)B * sizeof(int32_t));
    L.pfail = take((size_t)B * sizeof(int32_t));
    L.lcp = take(lcp_ws_bytes(cnt_max, n_max, o ? o->lcp_prec : PREC_FP64));
    L.total = p;
    return L;
}

__global__ void point_init_kernel(int B, uint8_t* done, int32_t* status, int32_t* iters,
                                  int32_t* pst, int32_t* pfail)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B) {
        done[i] = 0;
        status[i] = SYS_NEWTON_NOT_CONVERGED;
        iters[i] = 0;
        pst[i] = SYS_OK;
        pfail[i] = 0;
    }
}

__global__ void point_offsets_kernel(int count, int n, int64_t* offs)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= count) offs[i] = (int64_t)i * n;
}

int point_newton(paqif_handle handle, const ehl_grid* grid, const ehl_params* params, int B,
                 const ehl_opts* opts, double* P, double* H0, double* H, double* Hmin,
                 int32_t* status, int32_t* iters, char* ws, hipStream_t s, bool capture)
{
    const PointLayout L = point_layout(grid, B, opts);
    const int Nx = grid->nx, Ny = grid->ny;
    const double hx = hx_of(grid), hy = hy_of(grid);
    const size_t cells = (size_t)Nx * Ny * B;
    double* dws = reinterpret_cast<double*>(ws + L.dws);  // k2 table first
    double* hel = reinterpret_cast<double*>(ws + L.hel);
    double* nodes = reinterpret_cast<double*>(ws + L.nodes);
    uint8_t* direct = reinterpret_cast<uint8_t*>(ws + L.direct);
    double* Q = reinterpret_cast<double*>(ws + L.q);
    double* Pst = reinterpret_cast<double*>(ws + L.pstart);
    double* band = reinterpret_cast<double*>(ws + L.band);
    double* rhs = reinterpret_cast<double*>(ws + L.rhs);
    double* v = reinterpret_cast<double*>(ws + L.v);
    uint8_t* bounded = reinterpret_cast<uint8_t*>(ws + L.bounded);
    uint8_t* done = reinterpret_cast<uint8_t*>(ws + L.done);
    int32_t* lst = reinterpret_cast<int32_t*>(ws + L.lst);
    int32_t* lit = reinterpret_cast<int32_t*>(ws + L.lit);
    int32_t* pst = reinterpret_cast<int32_t*>(ws + L.pst);
    int32_t* pfail = reinterpret_cast<int32_t*>(ws + L.pfail);
    char* lcpws = ws + L.lcp;
    int st;
    // kernel table, offsets, flags, start
    if ((st = run_deformation(grid, P, B, PREC_FP64, hel, ws + L.dws, false, s))) return st;
    for (int k = 0; k < 4; k++) {
        const int cnt = L.nlc[k] * B;
        hipLaunchKernelGGL(point_offsets_kernel, dim3((cnt + 256) / 256), dim3(256), 0, s, cnt,
                           L.nrow[k], reinterpret_cast<int64_t*>(ws + L.offs[k]));
    }
    hipLaunchKernelGGL(point_init_kernel, dim3((B + 255) / 256), dim3(256), 0, s, B, done, status,
                       iters, pst, pfail);
    if (opts->start_rule) {
        if ((st = pq::launch_point_start(Nx, Ny, B, grid->x0, grid->y0, hx, hy, P, s))) return st;
        if ((st = run_deformation(grid, P, B, PREC_FP64, hel, ws + L.dws, true, s))) return st;
        if ((st = pq::launch_point_h0_rule(Nx, Ny, B, grid->x0, grid->y0, hx, hy, params, hel, H0,
                                           s)))
            return st;
    }
    if (hipMemcpyAsync(Pst, P, cells * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return PAQIF_EHIP;

    pq::PointNodeArgs na;
    na.Nx = Nx;
    na.Ny = Ny;
    na.B = B;
    na.x0 = grid->x0;
    na.y0 = grid->y0;
    na.hx = hx;
    na.hy = hy;
    na.switch_ratio = opts->switch_ratio;
    na.params = params;
    na.Hel = hel;
    na.H0 = H0;
    na.skip = done;
    na.eps = nodes;
    na.rH = nodes + cells;
    na.rho = nodes + 2 * cells;
    na.drhoH = nodes + 3 * cells;
    na.eP = nodes + 4 * cells;
    na.eH = nodes + 5 * cells;
    na.direct = direct;

    pq::PointAssembleArgs pa;
    pa.Nx = Nx;
    pa.Ny = Ny;
    pa.B = B;
    pa.kterms = opts->kernel_terms;
    set_scheme(pa, opts);
    pa.hx = hx;
    pa.hy = hy;
    pa.k2 = dws;
    pa.eps = na.eps;
    pa.rH = na.rH;
    pa.rho = na.rho;
    pa.drhoH = na.drhoH;
    pa.eP = na.eP;
    pa.eH = na.eH;
    pa.direct = direct;
    pa.skip = done;
    pa.band = band;
    pa.rhs = rhs;
    pa.bounded = bounded;

    pq::LcpArgs la;
    la.order = nullptr;
    la.band = band;
    la.b = rhs;
    la.bounded = bounded;
    la.mode = LCP_EXACT;
    la.max_iter = opts->lcp_max_iter;
    la.refine_tol = 1e-12;
    la.u = v;
    la.w = nullptr;
    la.active_out = nullptr;
    la.status = lst;
    la.iters = lit;
    la.rec = lcpws;
    {
        int cnt_max = 0, n_max = 0;
        for (int k = 0; k < 4; k++) {
            cnt_max = std::max(cnt_max, L.nlc[k] * B);
            n_max = std::max(n_max, L.nrow[k]);
        }
        const size_t recs = (size_t)(((int64_t)cnt_max * n_max + cnt_max) / 2 + 1);
        const size_t elt = opts->lcp_prec == PREC_FP32_IR ? sizeof(float) : sizeof(double);
        const size_t rb = a256(recs * (size_t)pq::record_stride(4, true) * elt);
        la.act = reinterpret_cast<uint8_t*>(lcpws + rb);
        la.r = opts->lcp_prec == PREC_FP32_IR
                   ? reinterpret_cast<double*>(lcpws + rb + a256((size_t)cnt_max * n_max))
                   : nullptr;
    }
    la.skip = nullptr;
    // each colour pass keeps its own active flags: a pass's LCP starts from
    // the set its lines ended with one step earlier (first step: empty set)
    la.warm = 1;
    for (int k = 0; k < 4; k++)
        if (hipMemsetAsync(ws + L.act[k], 0, (size_t)L.nlc[k] * L.nrow[k] * B, s) != hipSuccess)
            return PAQIF_EHIP;

    pq::PointUpdateArgs ua;
    ua.Nx = Nx;
    ua.Ny = Ny;
    ua.B = B;
    ua.omega = opts->omega;
    ua.v = v;
    ua.direct = direct;
    ua.skip = done;

    pq::PointH0Args ha;
    ha.Nx = Nx;
    ha.Ny = Ny;
    ha.B = B;
    ha.hx = hx;
    ha.hy = hy;
    ha.c_h0 = opts->c_h0;
    ha.load_target = 2.0 * M_PI / 3.0;
    ha.Pstart = Pst;
    ha.H0 = H0;
    ha.done = done;
    ha.status = status;
    ha.iters = iters;
    ha.step_lcp = pst;
    ha.lcp_fails = pfail;
    ha.fail_steps = fail_steps(opts);

    const int layout = handle->layout[1][opts->lcp_prec == PREC_FP32_IR];
    auto one_step = [&](int dprec) -> int {
        int e;
        double* cur = P;
        double* nxt = Q;
        for (int ax = 0; ax < 2; ax++) {
            for (int c = 1; c >= 0; c--) {
                const int k = 2 * ax + c;
                if ((e = run_deformation(grid, cur, B, dprec, hel, ws + L.dws, true, s))) return e;
                na.P = cur;
                if ((e = pq::launch_point_nodes(na, s))) return e;
                pa.axis = ax;
                pa.color = c;
                pa.P = cur;
                if ((e = pq::launch_point_assemble(pa, s))) return e;
                la.count = L.nlc[k] * B;
                la.offsets = reinterpret_cast<const int64_t*>(ws + L.offs[k]);
                la.act = reinterpret_cast<uint8_t*>(ws + L.act[k]);
                if (la.count > 0 && (e = pq::dispatch_lcp(4, la, opts->lcp_prec, layout, s)))
                    return e;
                // worst LCP status of each instance's lines, folded into its step status
                if ((e = pq::launch_point_lcp_status(B, L.nlc[k], lst, done, pst, s))) return e;
                ua.axis = ax;
                ua.color = c;
                ua.P = cur;
                ua.Pout = nxt;
                if ((e = pq::launch_point_update(ua, s))) return e;
                std::swap(cur, nxt);
            }
            ha.P = cur;
            ha.tol = std::max(opts->tol, fp64_floor(std::max(Nx, Ny)));
            if ((e = pq::launch_point_h0(ha, ax == 1 ? 1 : 0, s))) return e;
        }
        return PAQIF_OK;  // four colour updates: the state is back in P
    };

    std::vector<uint8_t> hdone(B);
    const int K = opts->steps_per_graph;
    const int dprec = opts->deform_prec;
    hipGraphExec_t exec = nullptr;
    bool use_graph = capture;
    if (use_graph) {
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
            use_graph = false;
        else {
            int e = 0;
            for (int k = 0; k < K && !e; k++) e = one_step(dprec);
            const hipError_t ce = hipStreamEndCapture(s, &graph);
            if (e || ce != hipSuccess || !graph) {
                if (graph) (void)hipGraphDestroy(graph);
                (void)hipGetLastError();
                use_graph = false;
            } else {
                if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                    exec = nullptr;
                    use_graph = false;
                }
                (void)hipGraphDestroy(graph);
            }
        }
    }
    int steps = 0;
    while (steps < opts->max_newton) {
        if (use_graph) {
            if (hipGraphLaunch(exec, s) != hipSuccess) {
                (void)hipGraphExecDestroy(exec);
                return PAQIF_EHIP;
            }
        } else {
            for (int k = 0; k < K; k++)
                if ((st = one_step(dprec))) return st;
        }
        steps += K;
        if (hipMemcpyAsync(hdone.data(), done, B, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            if (exec) (void)hipGraphExecDestroy(exec);
            return PAQIF_EHIP;
        }
        if (std::all_of(hdone.begin(), hdone.end(), [](uint8_t d) { return d != 0; })) break;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if ((st = run_deformation(grid, P, B, PREC_FP64, hel, ws + L.dws, true, s))) return st;
    if ((st = pq::launch_point_film(Nx, Ny, B, grid->x0, grid->y0, hx, hy, hel, H0, H, Hmin, s)))
        return st;
    hipLaunchKernelGGL(final_status_kernel, dim3((B + 255) / 256), dim3(256), 0, s, B, done, Hmin,
                       status);
    return pq::hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

// node arrays + kernel table for the standalone point assembly
size_t point_assemble_ws(const ehl_grid* g, int B)
{
    return a256(deform_ws_bytes(g, B)) + a256(6 * (size_t)g->nx * g->ny * B * sizeof(double)) +
           a256((size_t)g->nx * g->ny * B);
}

}  // namespace

extern "C" {

size_t ehl_deformation_workspace_bytes(const ehl_grid* grid, int B)
{
    if (B <= 0) return 0;
    return deform_ws_bytes(grid, B);
}

int ehl_deformation(paqif_handle handle, const ehl_grid* grid, const double* P, int B, int prec,
                    double* H_el, void* workspace, void* stream)
{
    if (!handle || !grid || B < 0) return PAQIF_EINVAL;
    if (!(valid_line(grid) || valid_point(grid))) return PAQIF_EINVAL;
    if (prec != PREC_FP64 && prec != PREC_FP32 && prec != PREC_SPLIT_BF16) return PAQIF_EINVAL;
    if (B == 0) return PAQIF_OK;
    if (!P || !H_el || !workspace || P == H_el) return PAQIF_EINVAL;
    return run_deformation(grid, P, B, prec, H_el, static_cast<char*>(workspace), false,
                           (hipStream_t)stream);
}

int ehl_jacobian_assemble(paqif_handle handle, const ehl_grid* grid, const ehl_params* params,
                          int B, const ehl_opts* opts, const double* P, const double* H_el,
                          const double* H0, const double* rough, double* R, double* band,
                          double* rhs, uint8_t* bounded, uint8_t* direct, void* stream)
{
    if (!handle || !valid_line(grid) || B < 0 || !opts) return PAQIF_EINVAL;
    if (!(opts->kernel_terms == 1 || opts->kernel_terms == 2)) return PAQIF_EINVAL;
    if (opts->limiter_jacobian < 0 || opts->limiter_jacobian > 2) return PAQIF_EINVAL;
    if (!valid_convection(opts)) return PAQIF_EINVAL;
    if (B == 0) return PAQIF_OK;
    if (!params || !P || !H_el || !H0 || !band || !rhs || !bounded) return PAQIF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int N = grid->nx;
    pq::LineAssembleArgs a;
    a.N = N;
    a.B = B;
    a.kterms = opts->kernel_terms;
    set_scheme(a, opts);
    a.h = hx_of(grid);
    a.x0 = grid->x0;
    a.switch_ratio = opts->switch_ratio;
    a.params = params;
    a.kvec = nullptr;
    host_kernel_head(hx_of(grid), a.kap);
    a.P = P;
    a.Hel = H_el;
    a.H0 = H0;
    a.rough = rough;
    a.skip = nullptr;
    a.R = R;
    a.band = band;
    a.rhs = rhs;
    a.bounded = bounded;
    a.direct = direct;
    return pq::launch_line_assemble(a, s);
}

size_t ehl_newton_workspace_bytes(paqif_handle handle, const ehl_grid* grid, int B,
                                  const ehl_opts* opts)
{
    (void)handle;
    if (B <= 0 || !valid_opts(opts)) return 0;
    if (valid_point(grid)) return point_layout(grid, B, opts).total;
    if (!valid_line(grid)) return 0;
    return newton_layout(grid, B, opts).total;
}

int ehl_newton_tvd(paqif_handle handle, const ehl_grid* grid, const ehl_params* params, int B,
                   const ehl_opts* opts, const double* rough, double* P, double* H0, double* H,
                   double* Hmin, int32_t* status, int32_t* iters, void* workspace, void* stream)
{
    if (!handle || B < 0 || !valid_opts(opts)) return PAQIF_EINVAL;
    if (!valid_line(grid) && !(valid_point(grid) && grid->nx >= 5 && grid->ny >= 5))
        return PAQIF_EINVAL;
    if (B == 0) return PAQIF_OK;
    if (!params || !P || !H0 || !Hmin || !status || !iters || !workspace) return PAQIF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (valid_point(grid)) {
        if (rough) return PAQIF_EINVAL;  // roughness is a line-contact input
        return point_newton(handle, grid, params, B, opts, P, H0, H, Hmin, status, iters,
                            static_cast<char*>(workspace), s, stream != nullptr);
    }
    const NewtonLayout L = newton_layout(grid, B, opts);
    char* ws = static_cast<char*>(workspace);
    const int N = grid->nx, n = N - 2;
    const double h = hx_of(grid);
    double* kvec = reinterpret_cast<double*>(ws + L.kvec);
    double* hel = reinterpret_cast<double*>(ws + L.hel);
    double* band = reinterpret_cast<double*>(ws + L.band);
    double* rhs = reinterpret_cast<double*>(ws + L.rhs);
    double* v = reinterpret_cast<double*>(ws + L.v);
    double* pn = reinterpret_cast<double*>(ws + L.pn);
    uint8_t* bounded = reinterpret_cast<uint8_t*>(ws + L.bounded);
    uint8_t* direct = reinterpret_cast<uint8_t*>(ws + L.direct);
    uint8_t* done = reinterpret_cast<uint8_t*>(ws + L.done);
    double* dP = reinterpret_cast<double*>(ws + L.dP);
    double* lerr = reinterpret_cast<double*>(ws + L.lerr);
    int64_t* offs = reinterpret_cast<int64_t*>(ws + L.offs);
    int32_t* lst = reinterpret_cast<int32_t*>(ws + L.lst);
    int32_t* lit = reinterpret_cast<int32_t*>(ws + L.lit);
    char* lcpws = ws + L.lcp;

    int st = pq::launch_line_kernel_vec(N, h, kvec, s);
    if (st) return st;
    hipLaunchKernelGGL(init_newton_kernel, dim3((B + 256) / 256), dim3(256), 0, s, B, n, offs,
                       done, status, iters);
    if (opts->start_rule) {
        pq::LineInitArgs ia{N, B, h, grid->x0, P};
        if ((st = pq::launch_line_hertz(ia, s))) return st;
        if ((st = pq::launch_line_deform(N, B, PREC_FP64, kvec, P, hel, s))) return st;
        if ((st = pq::launch_line_h0_rule(N, B, h, grid->x0, params, hel, H0, s))) return st;
    }

    pq::LineAssembleArgs aa;
    aa.N = N;
    aa.B = B;
    aa.kterms = opts->kernel_terms;
    set_scheme(aa, opts);
    aa.h = h;
    aa.x0 = grid->x0;
    aa.switch_ratio = opts->switch_ratio;
    aa.params = params;
    aa.kvec = kvec;
    aa.P = P;
    aa.Hel = hel;
    aa.H0 = H0;
    aa.rough = rough;
    aa.skip = done;
    aa.R = nullptr;
    aa.band = band;
    aa.rhs = rhs;
    aa.bounded = bounded;
    aa.direct = direct;

    pq::LcpArgs la;
    la.count = B;
    la.offsets = offs;
    la.order = nullptr;
    la.band = band;
    la.b = rhs;
    la.bounded = bounded;
    la.mode = LCP_EXACT;
    la.max_iter = opts->lcp_max_iter;
    la.refine_tol = 1e-12;
    la.u = v;
    la.w = nullptr;
    la.active_out = nullptr;
    la.status = lst;
    la.iters = lit;
    la.rec = lcpws;
    {
        const size_t recs = (size_t)(((int64_t)B * n + B) / 2 + 1);
        const size_t elt = opts->lcp_prec == PREC_FP32_IR ? sizeof(float) : sizeof(double);
        const size_t rb = a256(recs * (size_t)pq::record_stride(4, true) * elt);
        la.act = reinterpret_cast<uint8_t*>(lcpws + rb);
        la.r = opts->lcp_prec == PREC_FP32_IR
                   ? reinterpret_cast<double*>(lcpws + rb + a256((size_t)B * n))
                   : nullptr;
    }
    la.skip = done;
    // each Newton step's LCP starts from the previous step's final active
    // set (the same rows every step); the first starts from the empty set
    la.warm = 1;
    if (hipMemsetAsync(la.act, 0, (size_t)B * n, s) != hipSuccess) return PAQIF_EHIP;

    pq::LineUpdateArgs ua;
    ua.N = N;
    ua.B = B;
    ua.h = h;
    ua.omega = opts->omega;
    ua.c_h0 = opts->c_h0;
    ua.load_target = M_PI / 2.0;
    ua.v = v;
    ua.direct = direct;
    ua.P = P;
    ua.H0 = H0;
    ua.done = done;
    ua.status = status;
    ua.iters = iters;
    ua.dP = dP;
    ua.load_err = lerr;
    ua.lcp_status = lst;
    ua.lcp_fails = reinterpret_cast<int32_t*>(ws + L.lfail);
    ua.best_dP = reinterpret_cast<double*>(ws + L.best);
    ua.best_step = reinterpret_cast<int32_t*>(ws + L.bstep);
    ua.stall_steps = opts->stall_steps;
    ua.fail_steps = fail_steps(opts);

    auto one_step = [&](int dprec) -> int {
        int e;
        if ((e = pq::launch_line_deform(N, B, dprec, kvec, P, hel, s))) return e;
        if ((e = pq::launch_line_assemble(aa, s))) return e;
        if ((e = pq::dispatch_lcp(4, la, opts->lcp_prec,
                                  handle->layout[1][opts->lcp_prec == PREC_FP32_IR], s)))
            return e;
        return pq::launch_line_update_ws(ua, pn, s);
    };

    std::vector<uint8_t> hdone(B);
    const int K = opts->steps_per_graph;
    std::vector<int> phases;
    if (opts->deform_prec != PREC_FP64) phases.push_back(opts->deform_prec);
    phases.push_back(PREC_FP64);
    int steps = 0;
    for (size_t ph = 0; ph < phases.size(); ph++) {
        const int dprec = phases[ph];
        // a low-precision deformation only gets the iterate close (its noise
        // floor is far above tol); the FP64 phase finishes the convergence
        const bool low = dprec != PREC_FP64;
        ua.tol = low ? std::max(opts->tol, 1e-5) : std::max(opts->tol, fp64_floor(N));
        const int phase_cap = low ? opts->max_newton / 2 : opts->max_newton;
        if (ph > 0)
            hipLaunchKernelGGL(reopen_kernel, dim3((B + 255) / 256), dim3(256), 0, s, B, done,
                               status);
        if (hipMemsetAsync(ua.lcp_fails, 0, (size_t)B * sizeof(int32_t), s) != hipSuccess)
            return PAQIF_EHIP;
        // stall tracking restarts with every phase
        hipLaunchKernelGGL(stall_init_kernel, dim3((B + 255) / 256), dim3(256), 0, s, B,
                           ua.best_dP, ua.best_step, iters);
        hipGraphExec_t exec = nullptr;
        bool use_graph = stream != nullptr;
        if (use_graph) {
            hipGraph_t graph = nullptr;
            if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
                use_graph = false;
            else {
                int e = 0;
                for (int k = 0; k < K && !e; k++) e = one_step(dprec);
                const hipError_t ce = hipStreamEndCapture(s, &graph);
                if (e || ce != hipSuccess || !graph) {
                    if (graph) (void)hipGraphDestroy(graph);
                    (void)hipGetLastError();
                    use_graph = false;
                } else {
                    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                        exec = nullptr;
                        use_graph = false;
                    }
                    (void)hipGraphDestroy(graph);
                }
            }
        }
        while (steps < phase_cap) {
            if (use_graph) {
                if (hipGraphLaunch(exec, s) != hipSuccess) {
                    (void)hipGraphExecDestroy(exec);
                    return PAQIF_EHIP;
                }
            } else {
                for (int k = 0; k < K; k++)
                    if ((st = one_step(dprec))) return st;
            }
            steps += K;
            if (hipMemcpyAsync(hdone.data(), done, B, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                if (exec) (void)hipGraphExecDestroy(exec);
                return PAQIF_EHIP;
            }
            if (std::all_of(hdone.begin(), hdone.end(), [](uint8_t d) { return d != 0; })) break;
        }
        if (exec) (void)hipGraphExecDestroy(exec);
    }
    // film with the final pressure (FP64 deformation)
    if ((st = pq::launch_line_deform(N, B, PREC_FP64, kvec, P, hel, s))) return st;
    if ((st = pq::launch_line_film(N, B, h, grid->x0, hel, H0, rough, H, Hmin, nullptr, s)))
        return st;
    hipLaunchKernelGGL(final_status_kernel, dim3((B + 255) / 256), dim3(256), 0, s, B, done, Hmin,
                       status);
    return pq::hip_ok(hipGetLastError()) ? PAQIF_OK : PAQIF_EHIP;
}

size_t ehl_point_assemble_workspace_bytes(const ehl_grid* grid, int B)
{
    if (!valid_point(grid) || B <= 0) return 0;
    return point_assemble_ws(grid, B);
}

int ehl_point_sweep_assemble(paqif_handle handle, const ehl_grid* grid, const ehl_params* params,
                             int B, const ehl_opts* opts, int axis, int color, const double* P,
                             const double* H_el, const double* H0, double* band, double* rhs,
                             uint8_t* bounded, uint8_t* direct, void* workspace, void* stream)
{
    if (!handle || !valid_point(grid) || grid->nx < 5 || grid->ny < 5 || B < 0 || !opts)
        return PAQIF_EINVAL;
    if ((axis != 0 && axis != 1) || (color != 0 && color != 1)) return PAQIF_EINVAL;
    if (!(opts->kernel_terms == 1 || opts->kernel_terms == 2)) return PAQIF_EINVAL;
    if (!valid_convection(opts)) return PAQIF_EINVAL;
    if (opts->limiter_jacobian < 0 || opts->limiter_jacobian > 2) return PAQIF_EINVAL;
    if (B == 0) return PAQIF_OK;
    if (!params || !P || !H_el || !H0 || !band || !rhs || !bounded || !workspace)
        return PAQIF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int Nx = grid->nx, Ny = grid->ny;
    const size_t cells = (size_t)Nx * Ny * B;
    char* ws = static_cast<char*>(workspace);
    double* k2 = reinterpret_cast<double*>(ws);
    double* nodes = reinterpret_cast<double*>(ws + a256(deform_ws_bytes(grid, B)));
    uint8_t* dir = direct ? direct
                          : reinterpret_cast<uint8_t*>(ws + a256(deform_ws_bytes(grid, B)) +
                                                       a256(6 * cells * sizeof(double)));
    int st;
    if ((st = pq::launch_point_kernel_tab(Nx, Ny, hx_of(grid), hy_of(grid), k2, s))) return st;
    pq::PointNodeArgs na;
    na.Nx = Nx;
    na.Ny = Ny;
    na.B = B;
    na.x0 = grid->x0;
    na.y0 = grid->y0;
    na.hx = hx_of(grid);
    na.hy = hy_of(grid);
    na.switch_ratio = opts->switch_ratio;
    na.params = params;
    na.P = P;
    na.Hel = H_el;
    na.H0 = H0;
    na.skip = nullptr;
    na.eps = nodes;
    na.rH = nodes + cells;
    na.rho = nodes + 2 * cells;
    na.drhoH = nodes + 3 * cells;
    na.eP = nodes + 4 * cells;
    na.eH = nodes + 5 * cells;
    na.direct = dir;
    if ((st = pq::launch_point_nodes(na, s))) return st;
    pq::PointAssembleArgs pa;
    pa.Nx = Nx;
    pa.Ny = Ny;
    pa.B = B;
    pa.axis = axis;
    pa.color = color;
    pa.kterms = opts->kernel_terms;
    set_scheme(pa, opts);
    pa.hx = na.hx;
    pa.hy = na.hy;
    pa.k2 = k2;
    pa.P = P;
    pa.eps = na.eps;
    pa.rH = na.rH;
    pa.rho = na.rho;
    pa.drhoH = na.drhoH;
    pa.eP = na.eP;
    pa.eH = na.eH;
    pa.direct = dir;
    pa.skip = nullptr;
    pa.band = band;
    pa.rhs = rhs;
    pa.bounded = bounded;
    return pq::launch_point_assemble(pa, s);
}

}  // extern "C"
