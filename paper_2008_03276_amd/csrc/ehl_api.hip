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

bool valid_opts(const ehl_opts* o)
{
    return o && o->omega > 0 && o->omega <= 1.0 && o->c_h0 > 0 && o->tol > 0 &&
           o->max_newton >= 1 && (o->kernel_terms == 1 || o->kernel_terms == 2) &&
           o->lcp_max_iter >= 1 &&
           (o->deform_prec == PREC_FP64 || o->deform_prec == PREC_FP32 ||
            o->deform_prec == PREC_SPLIT_BF16) &&
           (o->lcp_prec == PREC_FP64 || o->lcp_prec == PREC_FP32_IR) &&
           o->steps_per_graph >= 1 && o->steps_per_graph <= 64;
}

// Newton workspace layout (line contact)
struct NewtonLayout {
    size_t kvec, hel, band, rhs, v, pn, bounded, direct, done, dP, lerr, offs, lst, lit, lcp,
        total;
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
// low-precision deformation go on; non-finite ones stay stopped.
__global__ void reopen_kernel(int B, uint8_t* done, int32_t* status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B && status[i] != SYS_NONFINITE) {
        done[i] = 0;
        status[i] = SYS_NEWTON_NOT_CONVERGED;
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
    if (B == 0) return PAQIF_OK;
    if (!params || !P || !H_el || !H0 || !band || !rhs || !bounded) return PAQIF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int N = grid->nx;
    pq::LineAssembleArgs a;
    a.N = N;
    a.B = B;
    a.kterms = opts->kernel_terms;
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
    if (!valid_line(grid) || B <= 0 || !valid_opts(opts)) return 0;
    return newton_layout(grid, B, opts).total;
}

int ehl_newton_tvd(paqif_handle handle, const ehl_grid* grid, const ehl_params* params, int B,
                   const ehl_opts* opts, const double* rough, double* P, double* H0, double* H,
                   double* Hmin, int32_t* status, int32_t* iters, void* workspace, void* stream)
{
    if (!handle || !valid_line(grid) || B < 0 || !valid_opts(opts)) return PAQIF_EINVAL;
    if (B == 0) return PAQIF_OK;
    if (!params || !P || !H0 || !Hmin || !status || !iters || !workspace) return PAQIF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
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
        ua.tol = low ? std::max(opts->tol, 1e-5) : opts->tol;
        const int phase_cap = low ? opts->max_newton / 2 : opts->max_newton;
        if (ph > 0)
            hipLaunchKernelGGL(reopen_kernel, dim3((B + 255) / 256), dim3(256), 0, s, B, done,
                               status);
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

}  // extern "C"
