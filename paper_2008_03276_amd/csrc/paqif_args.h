// Launch arguments of the PAQIF kernels (internal; shared by paqif.hip and
// api.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Library handle: device properties and the tuned lane layout of the
// PAQIF kernel per half-bandwidth (q = 2, 4, 8) and precision (FP64, FP32+IR).
struct paqif_handle_s {
    int device;
    int cu_count;
    int layout[3][2];
    int sweeps[3][2];  // start sweeps of the exact LCP per (q, precision)
    // device address of the library-owned scratch array on `device` (the
    // allocation-free LCP entry point), from hipGetSymbolAddress
    void* scratch;
};



namespace pq {

inline int q_index(int q) { return q == 2 ? 0 : (q == 4 ? 1 : 2); }

struct LcpArgs {
    int32_t count;
    const int64_t* offsets;
    const int32_t* order;
    const double* band;
    const double* b;
    const uint8_t* bounded;
    int mode;
    int max_iter;
    double refine_tol;
    double* u;
    double* w;
    uint8_t* active_out;
    int32_t* status;
    int32_t* iters;
    void* rec;     // level records
    uint8_t* act;  // working active flags (total_rows)
    double* r;     // refinement residual (total_rows), FP32_IR only
    const uint8_t* skip;  // per system: nonzero = leave untouched (may be null)
    int warm;  // exact mode: start from the flags already in act (bounded rows only)
    // per system: first row of its band rows in `band` (null = offsets[sys]);
    // lets several systems (e.g. one matrix with several right-hand sides) share rows
    const int64_t* band_off = nullptr;
    // exact mode without a warm start: the systems with at least sweep_min
    // elimination levels (paqif_solve_lcp: 0, every system) start from the
    // iterate that `sweeps` projected Jacobi sweeps (dispatch_sweeps, run
    // before the solve) left in u, the others (and all when sweeps == 0)
    // from the sign of b
    int sweeps = 0;
    int sweep_min = 0;
};

// Start sweeps (paqif_sweep_kernel): rows of a system as in b and u.
constexpr int SWC = 256;  // rows of one system per workgroup
struct SweepArgs {
    int32_t count;
    const int64_t* offsets;
    const int64_t* band_off;  // null: offsets
    const double* band;
    const double* b;
    const uint8_t* bounded;  // null: all bounded
    const double* src;       // iterate the sweeps start from (null: zero)
    double* dst;
    int kp;                  // sweeps of this launch
    int sweep_min;           // systems with fewer elimination levels: untouched
};

struct FactorArgs {
    int32_t count;
    const int64_t* offsets;
    const int32_t* order;
    const double* band;
    const uint8_t* pinned;
    void* rec;
    int32_t* status;
    int prec = PREC_FP64;  // records in FP64, or FP32 (PREC_FP32_IR)
};

struct SolveArgs {
    int32_t count;
    const int64_t* offsets;
    const int32_t* order;
    const uint8_t* pinned;
    void* rec;
    const double* rhs;
    double* x;
    int prec = PREC_FP64;  // precision of the records in rec
};

int dispatch_lcp(int q, const LcpArgs& a, int prec, int layout, hipStream_t s);

// Several FP64 row-layout solves in one launch (paqif_lcp_rows_many_kernel):
// call c has half-bandwidth q[c] and waves[c] = rows_waves(count) waves.
constexpr int kMaxManyCalls = 8;
struct RowsManyArgs {
    LcpArgs a[kMaxManyCalls];
    int q[kMaxManyCalls];
    int waves[kMaxManyCalls];
    int n;
};
int dispatch_lcp_rows_many(const RowsManyArgs& m, hipStream_t s);
int rows_waves(int count);
// The start sweeps of an exact solve (a.sweeps of them, into a.u; tmp: a
// second buffer of total-rows doubles when they take several launches).
int dispatch_sweeps(int q, const LcpArgs& a, int max_n, double* tmp, hipStream_t s);
int layouts_for(int q);
int dispatch_factor(int q, const FactorArgs& a, hipStream_t s);
int dispatch_solve(int q, const SolveArgs& a, hipStream_t s);
int record_stride(int q, bool with_w);

}  // namespace pq
