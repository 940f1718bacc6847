// Internal declarations of the EHL kernels (deformation, assembly, update).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "paqif_ehl.h"

namespace pq {

// deform.hip
int launch_line_kernel_vec(int N, double h, double* k, hipStream_t s);
int launch_point_kernel_tab(int Nx, int Ny, double hx, double hy, double* k2, hipStream_t s);
int launch_line_deform(int N, int B, int prec, const double* k, const double* P, double* out,
                       hipStream_t s);
size_t point_workspace_doubles(int Nx, int Ny, int B);
int launch_point_deform(int Nx, int Ny, int B, int prec, const double* k2, const double* P,
                        double* out, double* part, hipStream_t s);

// ehl_line.hip
struct LineAssembleArgs {
    int N, B, kterms, limjac;
    int conv;       // 0 van Leer slope, 1 kappa-scheme
    double kappa;
    // splitting matrix (Lhs1 / Lhs2): eps and rho frozen, upwind convective
    // derivative weighted by csplit (limjac must be 2); 0: Newton band
    int split = 0;
    double csplit = 1.0;
    double h, x0, switch_ratio;
    const ehl_params* params;  // device, B
    const double* kvec;        // N (device) or null: use kap
    double kap[4];             // k[0..3] when kvec is null
    const double* P;           // N x B
    const double* Hel;         // N x B
    const double* H0;          // B
    const double* rough;       // N x B or null
    const uint8_t* skip;       // B or null
    double* R;                 // (N-2) x B or null
    double* band;              // (N-2) x 9 per instance
    double* rhs;               // (N-2) x B
    uint8_t* bounded;          // (N-2) x B
    uint8_t* direct;           // N x B or null
};
int launch_line_assemble(const LineAssembleArgs& a, hipStream_t s);

struct LineUpdateArgs {
    int N, B;
    double h, omega, c_h0, tol, load_target;
    const double* v;     // (N-2) x B, LCP solution (new pressure before weighting)
    const uint8_t* direct;  // N x B
    double* P;           // N x B
    double* H0;          // B
    uint8_t* done;       // B
    int32_t* status;     // B
    int32_t* iters;      // B
    double* dP;          // B (last max change)
    double* load_err;    // B
    const int32_t* lcp_status;  // B, status of this step's LCP solve
    int32_t* lcp_fails;  // B, consecutive steps whose LCP hit its active-set cap
    double* best_dP;     // B, smallest max |P change| of the phase so far
    int32_t* best_step;  // B, step (iters count) at which it was reached
    int stall_steps;     // stop after this many steps without a new minimum (0: never)
    int fail_steps;      // stop after this many consecutive failed step LCPs
};
// Severity of a band LCP's status for an EHL instance: a singular or
// non-finite pivot stops the instance at once; a capped active-set
// iteration or a stalled refinement counts as a failed step, and an
// instance whose step LCP failed in fail_steps consecutive Newton steps
// stops with the last failure's status (the active-set iteration cycles,
// or the FP32 factors cannot be refined: the step's linearisation has no
// solution the iteration reaches).
PQ_DEV int lcp_severity(int st)
{
    switch (st) {
    case SYS_LCP_NOT_CONVERGED: return 1;
    case SYS_REFINE_STALLED: return 2;
    case SYS_NONFINITE: return 3;
    case SYS_ZERO_PIVOT: return 4;
    default: return 0;
    }
}
PQ_DEV int lcp_fatal(int st) { return st == SYS_ZERO_PIVOT || st == SYS_NONFINITE; }
PQ_DEV int lcp_failed(int st) { return st == SYS_LCP_NOT_CONVERGED || st == SYS_REFINE_STALLED; }
int launch_line_update_ws(const LineUpdateArgs& a, double* Pnew, hipStream_t s);

struct LineInitArgs {
    int N, B;
    double h, x0;
    double* P;  // N x B (Hertzian start written)
};
int launch_line_hertz(const LineInitArgs& a, hipStream_t s);
int launch_line_h0_rule(int N, int B, double h, double x0, const ehl_params* params,
                        const double* Hel, double* H0, hipStream_t s);
int launch_line_film(int N, int B, double h, double x0, const double* Hel, const double* H0,
                     const double* rough, double* H, double* Hmin, int32_t* argmin,
                     hipStream_t s);


// ehl_point.hip (point contact, alternating line sweeps in two colours)
struct PointNodeArgs {
    int Nx, Ny, B;
    double x0, y0, hx, hy, switch_ratio;
    const ehl_params* params;
    const double *P, *Hel, *H0;
    const uint8_t* skip;  // B or null
    double *eps, *rH, *rho, *drhoH, *eP, *eH;
    uint8_t* direct;
};
int launch_point_nodes(const PointNodeArgs& a, hipStream_t s);

struct PointAssembleArgs {
    int Nx, Ny, B, axis, color, kterms, limjac;
    int conv;      // 0 van Leer slope, 1 kappa-scheme slope (Sec. 3.3, eqs. 56-59)
    double kappa;
    int split = 0;  // as LineAssembleArgs
    double csplit = 1.0;
    double hx, hy;
    const double* k2;  // Nx x Ny kernel table
    const double *P, *eps, *rH, *rho, *drhoH, *eP, *eH;
    const uint8_t* direct;
    const uint8_t* skip;
    double *band, *rhs;
    uint8_t* bounded;
};
int point_color_lines(int Nx, int Ny, int axis, int color);
int launch_point_assemble(const PointAssembleArgs& a, hipStream_t s);

struct PointUpdateArgs {
    int Nx, Ny, B, axis, color;
    double omega;
    const double *P, *v;
    const uint8_t* direct;
    const uint8_t* skip;
    double* Pout;
};
int launch_point_update(const PointUpdateArgs& a, hipStream_t s);

struct PointH0Args {
    int Nx, Ny, B;
    double hx, hy, c_h0, tol, load_target;
    const double* P;
    double *Pstart, *H0;
    uint8_t* done;
    int32_t *status, *iters;
    int32_t* step_lcp;   // B: worst LCP status of the step's colour passes (reset per step)
    int32_t* lcp_fails;  // B: consecutive steps with a failed LCP
    int fail_steps;
};
int launch_point_h0(const PointH0Args& a, int check, hipStream_t s);
// fold the worst LCP status of each instance's nlc lines into step_lcp
int launch_point_lcp_status(int B, int nlc, const int32_t* lst, const uint8_t* done,
                            int32_t* step_lcp, hipStream_t s);
int launch_point_start(int Nx, int Ny, int B, double x0, double y0, double hx, double hy,
                       double* P, hipStream_t s);
int launch_point_h0_rule(int Nx, int Ny, int B, double x0, double y0, double hx, double hy,
                         const ehl_params* params, const double* Hel, double* H0, hipStream_t s);
int launch_point_film(int Nx, int Ny, int B, double x0, double y0, double hx, double hy,
                      const double* Hel, const double* H0, double* H, double* Hmin, hipStream_t s);

}  // namespace pq
