// C ABI of the library: argument validation, workspace layout, launches.
#include <mutex>
#include <new>

#include "common.h"

#include "paqif_args.h"

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static bool valid_batch(const paqif_batch* b)
{
    if (!b) return false;
    if (b->count < 0) return false;
    if (!(b->q == 2 || b->q == 4 || b->q == 8)) return false;
    if (b->count > 0 && !b->offsets) return false;
    if (b->total_rows < 0 || b->max_n < 0) return false;
    if (b->max_n > (int64_t)1 << 30) return false;
    return true;
}

static size_t n_records(const paqif_batch* b) { return (size_t)((b->total_rows + b->count) / 2 + 1); }

// workspace: [records][active flags][refinement residual]
struct LcpLayout {
    size_t rec_bytes, act_off, r_off, total;
};

static LcpLayout lcp_layout(const paqif_batch* b, int prec)
{
    LcpLayout L;
    const bool mixed = prec == PREC_FP32_IR;
    const size_t elt = mixed ? sizeof(float) : sizeof(double);
    // records are sized with room for the W0 part (paqif_factor and the
    // mixed-precision path store it; the FP64 LCP path uses a shorter stride)
    L.rec_bytes = align256(n_records(b) * (size_t)pq::record_stride(b->q, true) * elt);
    L.act_off = L.rec_bytes;
    L.r_off = L.act_off + align256((size_t)b->total_rows);
    L.total = L.r_off + (mixed ? align256((size_t)b->total_rows * sizeof(double)) : 0);
    return L;
}

// Scratch of paqif_solve_lcp_noalloc: one array per GPU, held until the
// process ends.  Host code never uses the array's name as a device address:
// its address on each device comes from hipGetSymbolAddress (taken once per
// device, with that device current, when a handle is created there).
static __device__ __align__(256) unsigned char scratch[PAQIF_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Address of `scratch` on the current device `dev` (nullptr on failure).
void* scratch_address(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

// Tight workspace of one LCP solve: level records at the stride the LCP
// kernel uses (FP64: Z0 part only; FP32 + refinement: with W0), active
// flags, refinement residual.
LcpLayout lcp_layout_tight(const paqif_batch* b, int prec)
{
    LcpLayout L;
    const bool mixed = prec == PREC_FP32_IR;
    const size_t elt = mixed ? sizeof(float) : sizeof(double);
    L.rec_bytes = align256(n_records(b) * (size_t)pq::record_stride(b->q, mixed) * elt);
    L.act_off = L.rec_bytes;
    L.r_off = L.act_off + align256((size_t)b->total_rows);
    L.total = L.r_off + (mixed ? align256((size_t)b->total_rows * sizeof(double)) : 0);
    return L;
}
}  // namespace

// Kernel arguments of one LCP solve (a.sweeps: the start sweeps to run
// first, 0 for none, 1 with LCP_EXACT_FROM_U whose start is u as passed in).
static pq::LcpArgs lcp_args(paqif_handle handle, const paqif_batch* batch, const double* band,
                            const double* b, const uint8_t* bounded, int mode, int prec,
                            double refine_tol, int max_iter, double* u, double* w,
                            uint8_t* active_out, int32_t* sys_status, int32_t* sys_iters,
                            char* ws, const LcpLayout& L)
{
    pq::LcpArgs a;
    a.count = batch->count;
    a.offsets = batch->offsets;
    a.order = batch->order;
    a.band = band;
    a.b = b;
    a.bounded = bounded;
    // LCP_EXACT_FROM_U: the exact kernels, reading their start from u
    const bool from_u = mode == LCP_EXACT_FROM_U;
    a.mode = from_u ? LCP_EXACT : mode;
    a.max_iter = max_iter;
    a.refine_tol = refine_tol;
    a.u = u;
    a.w = w;
    a.active_out = active_out;
    a.status = sys_status;
    a.iters = sys_iters;
    a.rec = ws;
    a.act = reinterpret_cast<uint8_t*>(ws + L.act_off);
    a.r = prec == PREC_FP32_IR ? reinterpret_cast<double*>(ws + L.r_off) : nullptr;
    a.skip = nullptr;
    a.warm = 0;
    a.sweeps = mode == LCP_EXACT ? handle->sweeps[pq::q_index(batch->q)][prec != 0] : 0;
    // every system starts from the sweeps: as a kernel of their own they
    // cost a band read per launch, and they bring the active-set solves per
    // LCP to about one (from about three from the sign of b)
    a.sweep_min = 0;
    if (from_u) a.sweeps = 1;  // the kernels' start is then the sign of u as passed in
    return a;
}

// The start sweeps of a (none for LCP_EXACT_FROM_U, whose u is the start);
// second sweep buffer: the record area, free until the solve.
static int run_sweeps(const paqif_batch* batch, const pq::LcpArgs& a, int mode, char* ws,
                      hipStream_t s)
{
    if (mode == LCP_EXACT_FROM_U || a.sweeps <= 0) return PAQIF_OK;
    return pq::dispatch_sweeps(batch->q, a, (int)batch->max_n, reinterpret_cast<double*>(ws), s);
}

static int launch_lcp(paqif_handle handle, const paqif_batch* batch, const double* band,
                      const double* b, const uint8_t* bounded, int mode, int prec,
                      double refine_tol, int max_iter, double* u, double* w,
                      uint8_t* active_out, int32_t* sys_status, int32_t* sys_iters, char* ws,
                      const LcpLayout& L, void* stream)
{
    const pq::LcpArgs a = lcp_args(handle, batch, band, b, bounded, mode, prec, refine_tol,
                                   max_iter, u, w, active_out, sys_status, sys_iters, ws, L);
    const int e = run_sweeps(batch, a, mode, ws, (hipStream_t)stream);
    if (e) return e;
    return pq::dispatch_lcp(batch->q, a, prec, handle->layout[pq::q_index(batch->q)][prec != 0],
                            (hipStream_t)stream);
}

extern "C" {

int paqif_create(paqif_handle* handle)
{
    if (!handle) return PAQIF_EINVAL;
    paqif_handle_s* h = new (std::nothrow) paqif_handle_s;
    if (!h) return PAQIF_EINVAL;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return PAQIF_EHIP;
    }
    h->cu_count = 0;
    if (hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, h->device) !=
        hipSuccess)
        h->cu_count = 0;
    // FP64 solves default to the row layout (one system per lane group of
    // 16 rows), FP32 solves with refinement to the lane-per-system layout.
    // Start sweeps of exact solves: measured on 4096 systems of 513-4097
    // rows, the sweep count that gave the fastest solve (q = 2, 4, 8).
    static const int default_sweeps[3] = {16, 16, 12};
    for (int qi = 0; qi < 3; qi++) {
        h->layout[qi][PREC_FP64] = 3;
        h->layout[qi][PREC_FP32_IR] = 0;
        h->sweeps[qi][PREC_FP64] = h->sweeps[qi][PREC_FP32_IR] = default_sweeps[qi];
    }
    h->scratch = scratch_address(h->device);
    if (!h->scratch) {
        delete h;
        return PAQIF_EHIP;
    }
    *handle = h;
    return PAQIF_OK;
}

int paqif_destroy(paqif_handle handle)
{
    delete handle;
    return PAQIF_OK;
}

const char* paqif_status_str(int code)
{
    switch (code) {
    case PAQIF_OK: return "ok";
    case PAQIF_EINVAL: return "invalid argument";
    case PAQIF_EWORKSPACE: return "workspace too small";
    case PAQIF_EHIP: return "HIP launch error";
    case SYS_ZERO_PIVOT: return "zero or non-finite pivot";
    case SYS_NONFINITE: return "non-finite solution";
    case SYS_LCP_NOT_CONVERGED: return "active-set iteration not converged";
    case SYS_REFINE_STALLED: return "iterative refinement stalled";
    case SYS_NEGATIVE_FILM: return "negative film thickness";
    case SYS_NEWTON_NOT_CONVERGED: return "Newton iteration not converged";
    default: return "unknown status";
    }
}

size_t paqif_workspace_bytes(paqif_handle handle, const paqif_batch* batch, int prec, int mode)
{
    (void)handle;
    (void)mode;
    if (!valid_batch(batch)) return 0;
    if (prec != PREC_FP64 && prec != PREC_FP32_IR) return 0;
    return lcp_layout(batch, prec).total;
}

int paqif_factor(paqif_handle handle, const paqif_batch* batch, const double* band,
                 const uint8_t* pinned, int prec, void* factors, int32_t* sys_status,
                 void* stream)
{
    if (!handle || !valid_batch(batch)) return PAQIF_EINVAL;
    if (prec != PREC_FP64 && prec != PREC_FP32_IR) return PAQIF_EINVAL;
    if (batch->count == 0) return PAQIF_OK;
    if (!band || !factors || !sys_status) return PAQIF_EINVAL;
    pq::FactorArgs a;
    a.count = batch->count;
    a.offsets = batch->offsets;
    a.order = batch->order;
    a.band = band;
    a.pinned = pinned;
    a.rec = factors;
    a.status = sys_status;
    a.prec = prec;
    return pq::dispatch_factor(batch->q, a, (hipStream_t)stream);
}

int paqif_solve_factored(paqif_handle handle, const paqif_batch* batch, const void* factors,
                         int prec, const uint8_t* pinned, const double* rhs, double* x,
                         void* stream)
{
    if (!handle || !valid_batch(batch)) return PAQIF_EINVAL;
    if (prec != PREC_FP64 && prec != PREC_FP32_IR) return PAQIF_EINVAL;
    if (batch->count == 0) return PAQIF_OK;
    if (!factors || !rhs || !x || (const void*)rhs == (const void*)x) return PAQIF_EINVAL;
    pq::SolveArgs a;
    a.count = batch->count;
    a.offsets = batch->offsets;
    a.order = batch->order;
    a.pinned = pinned;
    a.rec = const_cast<void*>(factors);
    a.rhs = rhs;
    a.x = x;
    a.prec = prec;
    return pq::dispatch_solve(batch->q, a, (hipStream_t)stream);
}

int paqif_solve_lcp(paqif_handle handle, const paqif_batch* batch, const double* band,
                    const double* b, const uint8_t* bounded, int mode, int prec,
                    double refine_tol, int max_iter, double* u, double* w, uint8_t* active_out,
                    int32_t* sys_status, int32_t* sys_iters, void* workspace, void* stream)
{
    if (!handle || !valid_batch(batch)) return PAQIF_EINVAL;
    if (mode != LCP_LINEAR && mode != LCP_CLIP && mode != LCP_EXACT && mode != LCP_EXACT_FROM_U)
        return PAQIF_EINVAL;
    if (prec != PREC_FP64 && prec != PREC_FP32_IR) return PAQIF_EINVAL;
    if (batch->count == 0) return PAQIF_OK;
    if (!band || !b || !u || !sys_status || !workspace) return PAQIF_EINVAL;
    if ((mode == LCP_EXACT || mode == LCP_EXACT_FROM_U) && max_iter < 1) return PAQIF_EINVAL;
    if (prec == PREC_FP32_IR && !(refine_tol > 0.0)) return PAQIF_EINVAL;
    const LcpLayout L = lcp_layout(batch, prec);
    return launch_lcp(handle, batch, band, b, bounded, mode, prec, refine_tol, max_iter, u, w,
                      active_out, sys_status, sys_iters, static_cast<char*>(workspace), L,
                      stream);
}

int paqif_solve_lcp_noalloc(paqif_handle handle, const paqif_batch* batch, const double* band,
                            const double* b, const uint8_t* bounded, int mode, int prec,
                            double refine_tol, int max_iter, double* u, double* w,
                            uint8_t* active_out, int32_t* sys_status, int32_t* sys_iters,
                            void* stream)
{
    if (!handle || !valid_batch(batch)) return PAQIF_EINVAL;
    if (mode != LCP_LINEAR && mode != LCP_CLIP && mode != LCP_EXACT && mode != LCP_EXACT_FROM_U)
        return PAQIF_EINVAL;
    if (prec != PREC_FP64 && prec != PREC_FP32_IR) return PAQIF_EINVAL;
    if (batch->count == 0) return PAQIF_OK;
    if (!band || !b || !u || !sys_status) return PAQIF_EINVAL;
    if ((mode == LCP_EXACT || mode == LCP_EXACT_FROM_U) && max_iter < 1) return PAQIF_EINVAL;
    if (prec == PREC_FP32_IR && !(refine_tol > 0.0)) return PAQIF_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return PAQIF_EHIP;
    if (dev != handle->device || !handle->scratch) return PAQIF_EINVAL;
    const LcpLayout L = lcp_layout_tight(batch, prec);
    if (L.total > (size_t)PAQIF_NOALLOC_SCRATCH_BYTES) return PAQIF_EWORKSPACE;
    // every byte of the scratch that the kernel reads it wrote first in the
    // same launch (records, flags, residual): nothing needs clearing
    return launch_lcp(handle, batch, band, b, bounded, mode, prec, refine_tol, max_iter, u, w,
                      active_out, sys_status, sys_iters, static_cast<char*>(handle->scratch), L,
                      stream);
}

int paqif_solve_lcp_many(paqif_handle handle, int ncalls, const paqif_lcp_call* calls, int mode,
                         int prec, double refine_tol, int max_iter, void* stream)
{
    if (!handle || ncalls < 0 || ncalls > PAQIF_MAX_LCP_CALLS || (ncalls > 0 && !calls))
        return PAQIF_EINVAL;
    if (mode != LCP_LINEAR && mode != LCP_CLIP && mode != LCP_EXACT && mode != LCP_EXACT_FROM_U)
        return PAQIF_EINVAL;
    if (prec != PREC_FP64 && prec != PREC_FP32_IR) return PAQIF_EINVAL;
    if ((mode == LCP_EXACT || mode == LCP_EXACT_FROM_U) && max_iter < 1) return PAQIF_EINVAL;
    if (prec == PREC_FP32_IR && !(refine_tol > 0.0)) return PAQIF_EINVAL;
    for (int c = 0; c < ncalls; c++) {
        const paqif_lcp_call& k = calls[c];
        if (!valid_batch(k.batch)) return PAQIF_EINVAL;
        if (k.batch->count > 0 && (!k.band || !k.b || !k.u || !k.sys_status || !k.workspace))
            return PAQIF_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    // every call's start sweeps first (bandwidth-bound, the whole chip), then
    // the solves: the FP64 row-layout ones in one launch, the others each in
    // its own kernel
    pq::RowsManyArgs m;
    m.n = 0;
    static_assert(PAQIF_MAX_LCP_CALLS <= pq::kMaxManyCalls, "many-call launch size");
    pq::LcpArgs args[PAQIF_MAX_LCP_CALLS];
    for (int c = 0; c < ncalls; c++) {
        const paqif_lcp_call& k = calls[c];
        if (k.batch->count == 0) continue;
        const LcpLayout L = lcp_layout(k.batch, prec);
        char* ws = static_cast<char*>(k.workspace);
        args[c] = lcp_args(handle, k.batch, k.band, k.b, k.bounded, mode, prec, refine_tol,
                           max_iter, k.u, k.w, k.active_out, k.sys_status, k.sys_iters, ws, L);
        const int e = run_sweeps(k.batch, args[c], mode, ws, s);
        if (e) return e;
    }
    for (int c = 0; c < ncalls; c++) {
        const paqif_lcp_call& k = calls[c];
        if (k.batch->count == 0) continue;
        const int layout = handle->layout[pq::q_index(k.batch->q)][prec != 0];
        if (prec == PREC_FP64 && layout == 3) {
            m.a[m.n] = args[c];
            m.q[m.n] = k.batch->q;
            m.waves[m.n] = pq::rows_waves(k.batch->count);
            m.n++;
        } else {
            const int e = pq::dispatch_lcp(k.batch->q, args[c], prec, layout, s);
            if (e) return e;
        }
    }
    return m.n > 0 ? pq::dispatch_lcp_rows_many(m, s) : PAQIF_OK;
}

int paqif_start_sweeps(paqif_handle handle, const paqif_batch* batch, const double* band,
                       const double* b, const uint8_t* bounded, int prec, double* u,
                       void* workspace, void* stream)
{
    if (!handle || !valid_batch(batch)) return PAQIF_EINVAL;
    if (prec != PREC_FP64 && prec != PREC_FP32_IR) return PAQIF_EINVAL;
    if (batch->count == 0) return PAQIF_OK;
    if (!band || !b || !u || !workspace) return PAQIF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int k = handle->sweeps[pq::q_index(batch->q)][prec != 0];
    if (k == 0)  // the sign start: u = b
        return pq::hip_ok(hipMemcpyAsync(u, b, (size_t)batch->total_rows * sizeof(double),
                                     hipMemcpyDeviceToDevice, s))
                   ? PAQIF_OK
                   : PAQIF_EHIP;
    pq::LcpArgs a;
    a.count = batch->count;
    a.offsets = batch->offsets;
    a.band = band;
    a.b = b;
    a.bounded = bounded;
    a.u = u;
    a.sweeps = k;
    a.sweep_min = 0;
    return pq::dispatch_sweeps(batch->q, a, (int)batch->max_n, static_cast<double*>(workspace), s);
}

int paqif_layout_count(int q) { return pq::layouts_for(q); }

int paqif_set_layout(paqif_handle handle, int q, int prec, int layout)
{
    if (!handle || pq::layouts_for(q) == 0) return PAQIF_EINVAL;
    if (prec != PREC_FP64 && prec != PREC_FP32_IR) return PAQIF_EINVAL;
    if (layout < 0 || layout >= pq::layouts_for(q)) return PAQIF_EINVAL;
    handle->layout[pq::q_index(q)][prec != 0] = layout;
    return PAQIF_OK;
}

int paqif_get_layout(paqif_handle handle, int q, int prec)
{
    if (!handle || pq::layouts_for(q) == 0) return PAQIF_EINVAL;
    if (prec != PREC_FP64 && prec != PREC_FP32_IR) return PAQIF_EINVAL;
    return handle->layout[pq::q_index(q)][prec != 0];
}

int paqif_set_start_sweeps(paqif_handle handle, int q, int prec, int sweeps)
{
    if (!handle || pq::layouts_for(q) == 0) return PAQIF_EINVAL;
    if (prec != PREC_FP64 && prec != PREC_FP32_IR) return PAQIF_EINVAL;
    if (sweeps < 0 || sweeps > PAQIF_MAX_START_SWEEPS) return PAQIF_EINVAL;
    handle->sweeps[pq::q_index(q)][prec != 0] = sweeps;
    return PAQIF_OK;
}

int paqif_get_start_sweeps(paqif_handle handle, int q, int prec)
{
    if (!handle || pq::layouts_for(q) == 0) return PAQIF_EINVAL;
    if (prec != PREC_FP64 && prec != PREC_FP32_IR) return PAQIF_EINVAL;
    return handle->sweeps[pq::q_index(q)][prec != 0];
}

int paqif_autotune(paqif_handle handle, const paqif_batch* batch, const double* band,
                   const double* b, const uint8_t* bounded, int mode, int prec, int max_iter,
                   double* u, int32_t* sys_status, void* workspace, void* stream,
                   float* times_ms)
{
    if (!handle || !valid_batch(batch)) return PAQIF_EINVAL;
    // u is scratch here: a start from u is timed as the sweeps' start
    if (mode == LCP_EXACT_FROM_U) mode = LCP_EXACT;
    const int nl = pq::layouts_for(batch->q);
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return PAQIF_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return PAQIF_EHIP;
    }
    int best = 0;
    float best_ms = 0.0f;
    int st = PAQIF_OK;
    for (int l = 0; l < nl && st == PAQIF_OK; l++) {
        handle->layout[pq::q_index(batch->q)][prec != 0] = l;
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && st == PAQIF_OK; rep++) {  // warm-up, then timed
            if (hipEventRecord(e0, s) != hipSuccess) st = PAQIF_EHIP;
            if (st == PAQIF_OK)
                st = paqif_solve_lcp(handle, batch, band, b, bounded, mode, prec, 1e-10, max_iter,
                                     u, nullptr, nullptr, sys_status, nullptr, workspace, stream);
            if (st == PAQIF_OK && (hipEventRecord(e1, s) != hipSuccess ||
                                   hipEventSynchronize(e1) != hipSuccess ||
                                   hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = PAQIF_EHIP;
        }
        if (times_ms) times_ms[l] = ms;
        if (st == PAQIF_OK && (l == 0 || ms < best_ms)) {
            best = l;
            best_ms = ms;
        }
    }
    handle->layout[pq::q_index(batch->q)][prec != 0] = best;
    // exact mode: then the start sweeps with that layout
    if (st == PAQIF_OK && mode == LCP_EXACT) {
        static const int cand[] = {0, 2, 4, 6, 8, 12, 16, 20, 24, 32};
        int& sw = handle->sweeps[pq::q_index(batch->q)][prec != 0];
        int best_sw = sw;
        float best_sw_ms = -1.0f;
        for (int c : cand) {
            if (st != PAQIF_OK) break;
            sw = c;
            float ms = 0.0f;
            for (int rep = 0; rep < 2 && st == PAQIF_OK; rep++) {
                if (hipEventRecord(e0, s) != hipSuccess) st = PAQIF_EHIP;
                if (st == PAQIF_OK)
                    st = paqif_solve_lcp(handle, batch, band, b, bounded, mode, prec, 1e-10,
                                         max_iter, u, nullptr, nullptr, sys_status, nullptr,
                                         workspace, stream);
                if (st == PAQIF_OK && (hipEventRecord(e1, s) != hipSuccess ||
                                       hipEventSynchronize(e1) != hipSuccess ||
                                       hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    st = PAQIF_EHIP;
            }
            if (st == PAQIF_OK && (best_sw_ms < 0.0f || ms < best_sw_ms)) {
                best_sw = c;
                best_sw_ms = ms;
            }
        }
        sw = best_sw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // extern "C"
