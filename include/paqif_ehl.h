/*
 * paqif_ehl.h -- C ABI of the MI355X (gfx950) PAQIF / EHL library.
 *
 * Paper: P. Singh, P. Dutt, "Total Variation Diminishing (TVD) method for
 * Elastohydrodynamic Lubrication (EHL) problem on Parallel Computers".
 *
 * Conventions for every entry point
 *  - All functions are extern "C", never throw, and return an int call
 *    status (PAQIF_OK or a negative PAQIF_E* code).
 *  - Array arguments are DEVICE pointers owned by the caller, unless the
 *    comment says "host".  The library never frees caller memory.
 *  - Work is enqueued on the caller's stream (hipStream_t passed as void*;
 *    NULL = default stream) and is asynchronous: the call returns once the
 *    kernels are queued.  Numerical outcomes are written per system into
 *    int32 status arrays on the device; read them after synchronising.
 *  - Argument errors (NULL where a pointer is required, sizes out of range,
 *    unsupported half-bandwidth, workspace too small) are detected on the
 *    host before anything is launched and return PAQIF_EINVAL /
 *    PAQIF_EWORKSPACE.  A failing HIP launch returns PAQIF_EHIP.
 *  - Entry points do not allocate device memory; scratch space is passed
 *    in as `workspace`, sized by the matching *_workspace_bytes query.
 *
 * Band layout (all band arguments): a system of order n with half-bandwidth
 * q is stored row major with 2q+1 doubles per row,
 *     band[i*(2q+1) + d] = a(i, i+d-q),   d = 0..2q,
 * entries whose column falls outside [0, n) are ignored.  A batch
 * concatenates its systems; system s owns rows offsets[s] .. offsets[s+1]-1
 * of band, right-hand sides and solutions.
 */
#ifndef PAQIF_EHL_H
#define PAQIF_EHL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* call-level status */
enum {
    PAQIF_OK = 0,
    PAQIF_EINVAL = -1,
    PAQIF_EWORKSPACE = -2,
    PAQIF_EHIP = -3
};

/* per-system numerical status (device int32 arrays) */
enum {
    SYS_OK = 0,
    SYS_ZERO_PIVOT = 1,          /* a 2x2 (or centre 1x1) pivot block was singular or not finite */
    SYS_NONFINITE = 2,           /* a non-finite value appeared in the solution */
    SYS_LCP_NOT_CONVERGED = 3,   /* active-set iteration hit max_iter */
    SYS_REFINE_STALLED = 4,      /* iterative refinement did not reach the tolerance */
    SYS_NEGATIVE_FILM = 5,       /* EHL: film thickness H <= 0 somewhere */
    SYS_NEWTON_NOT_CONVERGED = 6, /* EHL: Newton iteration hit max_newton */
    SYS_ADJOINT_NOT_CONVERGED = 7 /* EHL adjoint: the transposed solve missed its tolerance */
};

/* arithmetic of the band factorisation */
enum {
    PREC_FP64 = 0,    /* factor, solve and decisions in FP64 */
    PREC_FP32_IR = 1, /* FP32 factors, FP64 residuals, iterative refinement */
    PREC_SPLIT_BF16 = 2,
    PREC_FP32 = 3
};

/* complementarity handling of paqif_solve_lcp */
enum {
    LCP_LINEAR = 0, /* u = A^{-1} b, no projection                         */
    LCP_CLIP = 1,   /* u = max(0, A^{-1} b) on bounded rows (projection)    */
    LCP_EXACT = 2,  /* exact LCP by a primal-dual active-set iteration      */
    LCP_EXACT_FROM_U = 3 /* LCP_EXACT started from the u passed in          */
};

/* Library handle: device properties.  Create once per process/device. */
typedef struct paqif_handle_s *paqif_handle;
int paqif_create(paqif_handle *handle);
int paqif_destroy(paqif_handle handle);
const char *paqif_status_str(int code);

/* A batch of band systems sharing one half-bandwidth q (q in {2, 4, 8}).
 * offsets: DEVICE int64[count+1], offsets[0] = 0, non-decreasing.
 * max_n: largest system order; total_rows = offsets[count] (host copies).
 * order: optional DEVICE int32[count] permutation giving the processing
 *        order (largest systems first is best); NULL = natural order. */
typedef struct {
    int32_t count;
    int32_t q;
    const int64_t *offsets;
    int64_t max_n;
    int64_t total_rows;
    const int32_t *order;
} paqif_batch;

/*
 * Workspace for paqif_solve_lcp / paqif_factor, in bytes (host query).
 * Holds, per system, one record per elimination level (the two Z0 rows on
 * the frontier, the inverse 2x2 pivot, the forward-solve values and, for
 * paqif_factor and PREC_FP32_IR, the W0 multipliers) plus the active-set
 * flags.  Returns 0 for an invalid batch.
 */
size_t paqif_workspace_bytes(paqif_handle handle, const paqif_batch *batch, int prec, int mode);

/*
 * paqif_factor -- alternate quadrant interlocking factorisation A = W0 Z0
 * of every system, centre-out (Sec. 2.2, "The Factorization" and
 * "Evaluation of W0 and Z0": at level k the two central rows of the reduced
 * matrix become rows of Z0, the two columns of W0 come from one 2x2 solve
 * per remaining row, then the rank-2 update).  n odd: the centre row is a
 * 1x1 pivot first.
 *  band     : DEVICE, total_rows x (2q+1) doubles (layout above).
 *  pinned   : DEVICE uint8[total_rows] or NULL; rows/columns with a nonzero
 *             flag are replaced by the identity before factorising.
 *  prec     : PREC_FP64, or PREC_FP32_IR: the factorisation computed and
 *             stored in FP32 (half the record bytes; the layout of the
 *             FP32 + refinement LCP path).  PAQIF_EINVAL otherwise.
 *  factors  : DEVICE, paqif_workspace_bytes(handle, batch, prec, LCP_LINEAR)
 *             bytes; receives the level records (layout in the library
 *             source; consumed by paqif_solve_factored with the same prec).
 *  sys_status: DEVICE int32[count]: SYS_OK or SYS_ZERO_PIVOT.
 */
int paqif_factor(paqif_handle handle, const paqif_batch *batch, const double *band,
                 const uint8_t *pinned, int prec, void *factors, int32_t *sys_status,
                 void *stream);

/*
 * paqif_solve_factored -- x = (W0 Z0)^{-1} rhs with factors from
 * paqif_factor: W0 y = rhs from the centre outwards, Z0 x = y from both ends
 * inwards (Sec. 2.2.2).  rhs entries of pinned rows are treated as 0.
 *  prec   : the prec the factors were made with (PAQIF_EINVAL otherwise).
 *           With PREC_FP32_IR the solve runs on the FP32 records (FP64 rhs
 *           and x): an FP32-accurate solution, which serves as the
 *           correction step of an iterative refinement whose residual the
 *           caller forms in FP64 with its band.
 *  rhs, x : DEVICE, total_rows doubles each (may not alias).
 *  pinned : the same mask given to paqif_factor (or NULL).
 */
int paqif_solve_factored(paqif_handle handle, const paqif_batch *batch, const void *factors,
                         int prec, const uint8_t *pinned, const double *rhs, double *x,
                         void *stream);

/*
 * paqif_solve_lcp -- PAQIF solve of the banded linear complementarity
 * problem of Sec. 2.1 eq. (14):  u >= 0, w = A u - b >= 0, u_i w_i = 0,
 * on the rows flagged in `bounded` (NULL = all rows); other rows are free.
 *  mode LCP_LINEAR: u = A^{-1} b.
 *  mode LCP_CLIP  : u = max(0, A^{-1} b) on bounded rows (the paper's
 *                   projection of the AQIF solution onto u >= 0).
 *  mode LCP_EXACT : active sets A_0 (the handle's start rule, see
 *                   paqif_set_start_sweeps), solve with the rows of A_k
 *                   replaced by identity rows and b = 0 there (so u = 0 on
 *                   A_k), w = A u - b,
 *                   A_{k+1} = {i in A_k : w_i > 0} u {i not in A_k : u_i < 0}
 *                   (bounded rows), until A_{k+1} = A_k or max_iter solves.
 *  mode LCP_EXACT_FROM_U: LCP_EXACT with A_0 = {bounded i : u_i <= 0} for
 *                   the u passed in (DEVICE in and out; typically the
 *                   iterate of paqif_start_sweeps, which makes the result
 *                   that of LCP_EXACT bit for bit); no start sweeps run.
 *  prec       : PREC_FP64, or PREC_FP32_IR (FP32 factors; every solve is
 *               refined with FP64 residuals until |r|_inf <= refine_tol *
 *               max(|b|_inf, 1) or 8 refinement steps, else
 *               SYS_REFINE_STALLED).
 *  u          : DEVICE out, total_rows doubles (in and out with
 *               LCP_EXACT_FROM_U).
 *  w          : DEVICE out or NULL, total_rows doubles, w = A u - b.
 *  active_out : DEVICE out or NULL, uint8 per row (1 = u_i pinned at 0).
 *  sys_status : DEVICE out, int32[count].
 *  sys_iters  : DEVICE out or NULL, int32[count], number of AQIF solves.
 *  workspace  : DEVICE, paqif_workspace_bytes(handle, batch, prec, mode).
 */
int paqif_solve_lcp(paqif_handle handle, const paqif_batch *batch, const double *band,
                    const double *b, const uint8_t *bounded, int mode, int prec,
                    double refine_tol, int max_iter, double *u, double *w, uint8_t *active_out,
                    int32_t *sys_status, int32_t *sys_iters, void *workspace, void *stream);


/*
 * paqif_solve_lcp_noalloc -- paqif_solve_lcp for callers that cannot
 * allocate device memory or pass a workspace (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * kernels and results as paqif_solve_lcp, without `workspace`: the level
 * records, active flags and refinement residual live in a library-owned
 * device array of PAQIF_NOALLOC_SCRATCH_BYTES per GPU, reserved when the
 * library is loaded on that GPU and held until the process ends.  The call
 * allocates nothing.  Its address on the device is taken (hipGetSymbolAddress)
 * when paqif_create runs there; the handle's device must be the current one
 * (else PAQIF_EINVAL).
 * Size limit: with R = total_rows, C = count, K = (R + C)/2 + 1 records and
 * a(x) = x rounded up to a multiple of 256,
 *   FP64:     a(K * (4q+6) * 8) + a(R)                    bytes
 *   FP32_IR:  a(K * (8q+6) * 4) + a(R) + a(8 R)           bytes
 * must not exceed PAQIF_NOALLOC_SCRATCH_BYTES, else PAQIF_EWORKSPACE (host
 * check, nothing launched).  Every call on one GPU shares that GPU's array
 * (its contents are those of the last call; nothing in it needs clearing),
 * so calls that overlap on one GPU -- on different streams or from
 * different threads -- race: serialise them.
 */
#define PAQIF_NOALLOC_SCRATCH_BYTES (64u << 20)
int paqif_solve_lcp_noalloc(paqif_handle handle, const paqif_batch *batch, const double *band,
                            const double *b, const uint8_t *bounded, int mode, int prec,
                            double refine_tol, int max_iter, double *u, double *w,
                            uint8_t *active_out, int32_t *sys_status, int32_t *sys_iters,
                            void *stream);

/*
 * Lane layouts of the PAQIF LCP kernel (how many frontier elements a lane
 * owns and how many systems share a wavefront; see the library source).
 * paqif_layout_count(q): number of layouts for half-bandwidth q (0 if q is
 * unsupported).  Layouts 0-2 spread each system's frontier over the lanes of
 * a wavefront (q = 2 layout 2: one system per lane); layout 3 gives each
 * system a group of 16 lanes, one frontier row per lane, with pivot rows
 * broadcast by DPP (FP64 only; with PREC_FP32_IR it runs layout 0).  A new
 * handle uses layout 3 for PREC_FP64 and layout 0 for PREC_FP32_IR.
 * paqif_set_layout / paqif_get_layout: the layout used by paqif_solve_lcp
 * (and the EHL Newton drivers) for (q, prec) on this handle; PAQIF_EINVAL for
 * an unknown q, prec or layout.
 * paqif_set_start_sweeps / paqif_get_start_sweeps: the starting active set
 * of mode LCP_EXACT for (q, prec) on this handle: A_0 = {bounded i : u_i <=
 * 0} for u after `sweeps` projected Jacobi sweeps from u = 0,
 * u_i <- (b_i - sum_{j != i} a_ij u_j) / a_ii, clipped at 0 on bounded rows
 * (0 or 1 sweep: A_0 = {bounded i : b_i <= 0}).  The solution does not
 * depend on the start (the active-set iteration ends at the LCP's solution);
 * the number of active-set solves does (about one per LCP from the sweeps
 * on the synthetic batches, about three from the sign of b).  The sweeps
 * run for every system, as a kernel of their own before the solve: each
 * workgroup holds 512 rows of a system, two per thread with their band
 * rows in registers, and runs up to 1 + 128 / q sweeps on them (one band
 * read per launch).  0 <= sweeps <= PAQIF_MAX_START_SWEEPS; a new handle
 * uses 16 for q = 2 and 4 and 12 for q = 8.  The sweeps write u (and,
 * above 1 + 128 / q sweeps, the workspace's record area).
 * paqif_autotune: times every layout on the caller's batch (one warm-up and
 * one timed solve each, HIP events on `stream`, which it synchronises),
 * stores the fastest in the handle and, if times_ms (host, float[count]) is
 * not NULL, the measured times; in mode LCP_EXACT it then times the start
 * sweeps 0, 2, 4, 6, 8, 12, 16, 20, 24, 32 with that layout and keeps the
 * fastest.  Arguments as for paqif_solve_lcp; u, sys_status and workspace
 * are used as scratch.
 */
#define PAQIF_MAX_START_SWEEPS 32
int paqif_layout_count(int q);
int paqif_set_layout(paqif_handle handle, int q, int prec, int layout);
int paqif_get_layout(paqif_handle handle, int q, int prec);
int paqif_set_start_sweeps(paqif_handle handle, int q, int prec, int sweeps);
int paqif_get_start_sweeps(paqif_handle handle, int q, int prec);

/*
 * paqif_solve_lcp_many -- several paqif_solve_lcp calls on one stream (each
 * its own batch, e.g. one per half-bandwidth q), with the results of calling
 * paqif_solve_lcp for each in turn with the same mode, prec, refine_tol and
 * max_iter, bit for bit.  Their order on the chip differs: every call's start
 * sweeps run first (bandwidth-bound kernels that fill the chip), then the
 * FP64 solves of the calls whose (q, prec) uses the row layout run in ONE
 * launch, workgroup g taking wave g / ncalls' of call g mod ncalls' (ncalls'
 * of them), so that the first waves of every call, which hold its largest
 * systems in LPT order, start together and the batches share the chip from
 * the start; the other calls' solves follow, one kernel each.  (Sec. 2
 * algorithm, batched; the scheduling is this library's.)
 *  ncalls : 0 <= ncalls <= PAQIF_MAX_LCP_CALLS.
 *  calls  : HOST, ncalls entries; each entry's pointers as for
 *           paqif_solve_lcp.  Calls may not share an output array or a
 *           workspace (they run concurrently).
 * Returns PAQIF_EINVAL for a bad count, batch, mode or prec, or a null
 * pointer a non-empty call needs.
 */
#define PAQIF_MAX_LCP_CALLS 8
typedef struct paqif_lcp_call {
    const paqif_batch *batch;
    const double *band;
    const double *b;
    const uint8_t *bounded;
    double *u;
    double *w;
    uint8_t *active_out;
    int32_t *sys_status;
    int32_t *sys_iters;
    void *workspace;
} paqif_lcp_call;
int paqif_solve_lcp_many(paqif_handle handle, int ncalls, const paqif_lcp_call *calls, int mode,
                         int prec, double refine_tol, int max_iter, void *stream);

/*
 * paqif_start_sweeps -- the starting iterate of LCP_EXACT on its own: the
 * handle's start sweeps for (batch->q, prec) from u = 0 into u (with 0
 * sweeps, u = b, whose signs give the same A_0).  A following
 * paqif_solve_lcp in mode LCP_EXACT_FROM_U with this u solves exactly as one
 * LCP_EXACT call; split in two, the sweeps of several batches can run
 * before their solves (a bandwidth-bound kernel that fills the chip ahead of
 * latency-bound ones).
 *  band, b, bounded : as for paqif_solve_lcp.
 *  u         : DEVICE out, total_rows doubles.
 *  workspace : DEVICE, paqif_workspace_bytes(handle, batch, prec,
 *              LCP_EXACT); its record area holds the iterate between
 *              launches when the sweeps take several (above 1 + 128 / q).
 * Returns PAQIF_EINVAL for a bad batch, prec or null pointer.
 */
int paqif_start_sweeps(paqif_handle handle, const paqif_batch *batch, const double *band,
                       const double *b, const uint8_t *bounded, int prec, double *u,
                       void *workspace, void *stream);
int paqif_autotune(paqif_handle handle, const paqif_batch *batch, const double *band,
                   const double *b, const uint8_t *bounded, int mode, int prec, int max_iter,
                   double *u, int32_t *sys_status, void *workspace, void *stream,
                   float *times_ms);

/*
 * Partitioned PAQIF solve of ONE long band system (Sec. 2.1 eqs. 15-18 and
 * Sec. 2.2 "PAQIF method", Steps 1-7), spread over many wavefronts.
 * The order-n system (half-bandwidth q, band layout above, one system) is
 * cut into r blocks, block m owning rows floor(m n / r) .. floor((m+1) n / r)
 * - 1; its first q and last q unknowns are coupled to the neighbouring
 * blocks.  Every block's inner unknowns are eliminated in parallel (one
 * batched PAQIF launch over the r blocks and their 2q+1 right-hand sides),
 * the reduced system on the 2 q r outer unknowns (a band of half-bandwidth
 * 2q - 1, solved directly in place of the paper's normal equations; for
 * q = 2 and at least 512 reduced rows by the same scheme once more) is
 * solved and, in LCP_CLIP mode, projected (Step 5), then the inner unknowns
 * follow from their blocks and are projected (Steps 6-7).
 *  n, q, r  : q in {2, 4}; every block needs at least 2q+1 rows
 *             (n / r >= 2q + 1); n <= 2^31.
 *  band     : DEVICE, n x (2q+1) doubles; b: DEVICE, n doubles.
 *  bounded  : DEVICE uint8[n] or NULL (all rows bounded); clip and exact.
 *  mode     : LCP_LINEAR (u = A^{-1} b); LCP_CLIP (the paper's projected
 *             partitioned solve; not the same as clipping A^{-1} b, since the
 *             inner unknowns use the projected outer ones); LCP_EXACT (the
 *             LCP of eq. 14 by the active-set iteration of paqif_solve_lcp,
 *             A_0 = {bounded i : b_i <= 0}, each iteration one partitioned
 *             solve with the rows and columns of A_k replaced by the identity
 *             and b = 0 there; the host reads the number of changes after
 *             every solve, so this mode synchronises `stream`).
 *  max_iter : exact mode: at most this many solves (>= 1); else ignored.
 *  u        : DEVICE out, n doubles.
 *  active_out: DEVICE out or NULL, uint8[n]: exact mode the final active
 *             set, clip mode the projected rows, linear mode zeros.
 *  status   : DEVICE out, int32[1]: the largest SYS_* code of the block and
 *             reduced solves of the last solve (SYS_OK, SYS_ZERO_PIVOT,
 *             SYS_NONFINITE), or SYS_LCP_NOT_CONVERGED after max_iter solves.
 *  iters    : DEVICE out or NULL, int32[1]: number of partitioned solves.
 *  workspace: DEVICE, paqif_partitioned_workspace_bytes(n, q, r) bytes
 *             (about (2q+1)(4q+5) n doubles; 0 = invalid arguments).
 * Returns PAQIF_EINVAL for invalid arguments before any launch.
 * The block solves use the handle's lane layout for q; the reduced system
 * (one system) runs with layout 0.
 */
size_t paqif_partitioned_workspace_bytes(int64_t n, int q, int32_t r);
int paqif_solve_partitioned(paqif_handle handle, int64_t n, int q, int32_t r, const double *band,
                            const double *b, const uint8_t *bounded, int mode, int max_iter,
                            double *u, uint8_t *active_out, int32_t *status, int32_t *iters,
                            void *workspace, void *stream);

/* ------------------------------------------------------------------------
 * Elastohydrodynamic lubrication (Sec. 3.3 of the paper)
 * ------------------------------------------------------------------------ */

/* Uniform grid: nx x ny nodes on [x0, x1] x [y0, y1]; ny == 1 is a line
 * contact (y0, y1 ignored).  Line contact requires 5 <= nx <= 8192. */
typedef struct {
    int32_t nx, ny;
    double x0, x1, y0, y1;
} ehl_grid;

/* Moes dimensionless load M and material parameter L of one instance.
 * Line contact: alpha_bar = L sqrt(M / 2 pi), lam = 3 pi^2 / (8 M^2),
 * p_h = alpha_bar / alpha with alpha = 1.7e-8 1/Pa, p0 = 1.98e8 Pa,
 * z = 0.68 (appendix of the paper; line-contact forms derived from the
 * Hertzian half width). */
typedef struct {
    double M, L;
} ehl_params;

/* Options of the hybrid line iteration (eqs. 60-75). */
typedef struct {
    double omega;        /* relaxation of the pressure change, (0, 1]          */
    double c_h0;         /* load-balance relaxation c of eq. 75                */
    double switch_ratio; /* hybrid switch threshold on eps/h (paper: 0.6)      */
    double tol;          /* convergence: max|dP| <= tol max(1,|P|), |load err| <= tol */
    int32_t max_newton;  /* iteration cap (then SYS_NEWTON_NOT_CONVERGED)       */
    int32_t kernel_terms;/* elastic coupling kept in the band: |k - j| <= 1 or 2 */
    int32_t lcp_max_iter;/* active-set cap of the linearised LCP per step       */
    int32_t deform_prec; /* PREC_FP64, PREC_FP32 or PREC_SPLIT_BF16 for K P;
                            a low-precision run is finished by FP64 steps       */
    int32_t lcp_prec;    /* PREC_FP64 or PREC_FP32_IR for the band LCP          */
    int32_t steps_per_graph; /* Newton steps per captured HIP graph replay    */
    int32_t start_rule;  /* 1: Hertzian P and H0 = 0.4/sqrt(M) - min_{|X|<=1}
                            (X^2/2 + H_el); 0: use P and H0 as given           */
    int32_t limiter_jacobian; /* limiter terms of the Newton matrix (the
                            residual always has the full limiter): 0 exact
                            derivatives, 1 ratio phi(r) frozen at the current
                            iterate (eqs. 64-65), 2 first-order flux           */
    int32_t stall_steps; /* line contact: stop an instance (status
                            SYS_NEWTON_NOT_CONVERGED) once max|dP| has set no
                            new minimum for this many steps; 0 = never       */
    int32_t convection;  /* convective face value (rho H)_{i+1/2} = (rho H)_i
                            + psi/2: 0 van Leer limited slope (TVD, default);
                            1 kappa-scheme psi = (1+kappa)/2 D+ + (1-kappa)/2
                            D- (Sec. 3.3, eqs. 56-59; line and point contact
                            and the line-contact adjoint)                    */
    double kappa;        /* -1 <= kappa <= 1 for convection 1                */
    int32_t lcp_fail_steps; /* stop an instance whose linearised LCP failed in this
                             many consecutive Newton steps (active-set cap hit:
                             SYS_LCP_NOT_CONVERGED; FP32 + refinement stalled:
                             SYS_REFINE_STALLED, the status of the last failure);
                             0 = 16.  A zero or non-finite pivot stops the
                             instance at once (SYS_ZERO_PIVOT / SYS_NONFINITE).
                             Point contact: a step fails if any line of any of
                             its four colour passes failed.                    */
    int32_t splitting;   /* matrix of each step's linearised problem (the
                            residual and the fixed point do not change):
                            0 the Newton band (limiter_jacobian applies);
                            1 / 2 the implicit operator of the hybrid
                            splitting Lhs1 / Lhs2 (Sec. 3.3.2, eqs. 60 / 61:
                            Ls1 or Ls0 for a direct change, eqs. 48-49; Ls4
                            or Ls5 for a weighted change, eqs. 56-59) --
                            eps and rho held at the current iterate, the
                            convective flux first-order upwind with weight
                            (2-k)/2 (Lhs1) or (2-k)/2 + (1-k)/4 (Lhs2), k =
                            kappa with convection 1, 0 with the limited
                            slope.  Line and point contact.                   */
} ehl_opts;

/*
 * ehl_deformation -- elastic film contribution H_el of B pressure fields on
 * one grid (Sec. 3.3.1).  Line (ny == 1): H_el = K P with
 * K[i][j] = -(1/pi) * integral of ln|x_i - x'| over the cell of node j;
 * P, H_el: DEVICE, nx x B column major (P[i + nx*b]).  Point (ny > 1):
 * H_el[i][j] = (2/pi^2) sum k2[|i-i'|][|j-j'|] P[i'][j'] with the closed-form
 * 1/r cell integrals; P, H_el: DEVICE, B blocks of nx*ny, row major in x
 * (P[b*nx*ny + i*ny + j]).
 * prec: PREC_FP64 (MFMA f64), PREC_FP32 (MFMA f32) or PREC_SPLIT_BF16.
 * workspace: DEVICE, ehl_deformation_workspace_bytes(grid, B) bytes.
 */
size_t ehl_deformation_workspace_bytes(const ehl_grid *grid, int B);
int ehl_deformation(paqif_handle handle, const ehl_grid *grid, const double *P, int B, int prec,
                    double *H_el, void *workspace, void *stream);

/*
 * ehl_jacobian_assemble -- line contact: residual R of the TVD
 * finite-volume Reynolds operator (eqs. 62-65; van Leer limited flux) and
 * the band Jacobian of the hybrid change (eq. 60: direct change where
 * eps/h > switch_ratio and next to cavitation, weighted change e_i -
 * (e_{i-1}+e_{i+1})/2 elsewhere; the distributed elastic kernel kept for
 * |k - j| <= kernel_terms, eqs. 66-67, 74), returned as the linearised
 * complementarity problem of each instance:  band = -dR/dsigma (rows of the
 * nx-2 interior nodes, half-bandwidth 4, layout of paqif_solve_lcp), rhs =
 * band * P + R, bounded = 1 where the node and both neighbours are direct.
 *  params: DEVICE ehl_params[B];  P, H_el: DEVICE nx x B;  H0: DEVICE [B];
 *  rough: DEVICE nx x B or NULL (added to the film);  R, rhs: DEVICE
 *  (nx-2) x B (R may be NULL);  band: DEVICE (nx-2)*B*9;  bounded: DEVICE
 *  uint8 (nx-2) x B;  direct: DEVICE uint8 nx x B or NULL.
 */
int ehl_jacobian_assemble(paqif_handle handle, const ehl_grid *grid, const ehl_params *params,
                          int B, const ehl_opts *opts, const double *P, const double *H_el,
                          const double *H0, const double *rough, double *R, double *band,
                          double *rhs, uint8_t *bounded, uint8_t *direct, void *stream);

/*
 * ehl_point_sweep_assemble -- point contact: the band systems of one colour
 * of one sweep direction of the alternating line method (Sec. 3.3, eqs. 60,
 * 62-65, 66-67, 69-70, 74): for every line of the colour (axis 0: x-lines,
 * one per interior y index j with j % 2 == color; axis 1: y-lines, one per
 * interior x index i), rows = interior positions along the line, band =
 * -dR/dsigma (half-bandwidth 4, layout of paqif_solve_lcp, system = b *
 * lines + line slot, slots in increasing line index), rhs = band * P + R,
 * bounded = 1 where the node and both along-line neighbours are direct.  The
 * film responds through the distributed kernel cut to |k - i| <=
 * kernel_terms; on y-lines the rows of weighted-change nodes are v = P.
 *  grid: 2D (ny > 1), nx, ny >= 5;  P, H_el: DEVICE B x nx x ny (node (i, j)
 *  at (b*nx + i)*ny + j);  H0: DEVICE [B];  band: DEVICE rows*9, rhs: DEVICE
 *  rows, bounded: DEVICE uint8 rows (rows = B * lines * (line length - 2));
 *  direct: DEVICE uint8 B x nx x ny out or NULL;  workspace: DEVICE,
 *  ehl_point_assemble_workspace_bytes(grid, B).
 */
size_t ehl_point_assemble_workspace_bytes(const ehl_grid *grid, int B);
int ehl_point_sweep_assemble(paqif_handle handle, const ehl_grid *grid, const ehl_params *params,
                             int B, const ehl_opts *opts, int axis, int color, const double *P,
                             const double *H_el, const double *H0, double *band, double *rhs,
                             uint8_t *bounded, uint8_t *direct, void *workspace, void *stream);

/*
 * ehl_newton_tvd -- line contact: the hybrid Newton line iteration (Lhs1)
 * for B instances on one grid until each converges or hits max_newton:
 * deformation (MFMA), assembly, PAQIF solve of the linearised LCP (exact
 * active set; each step's active-set iteration starts from the previous
 * step's final set, the first from the empty set: the LCP solution does not
 * depend on the start), P <- max(0, P + omega D (v - P)), H0 <- H0 - c (pi/2 -
 * h sum P) (eq. 75).  Steps are captured in HIP graphs of steps_per_graph
 * steps; the host reads the per-instance done flags after every replay
 * (this call synchronises the stream).
 *  P: DEVICE nx x B, in: start (ignored with start_rule 1), out: solution.
 *  H0: DEVICE [B], in/out.  H: DEVICE nx x B out (film).  Hmin: DEVICE [B].
 *  status: DEVICE int32[B] (SYS_OK, SYS_NEWTON_NOT_CONVERGED,
 *  SYS_NEGATIVE_FILM, SYS_NONFINITE; line contact also
 *  SYS_LCP_NOT_CONVERGED when the step's LCP hit lcp_max_iter in 16
 *  consecutive steps: the active-set iteration cycles and the instance is
 *  stopped).  iters: DEVICE int32[B].
 *  workspace: DEVICE, ehl_newton_workspace_bytes(handle, grid, B, opts).
 * Point contact (grid with ny > 1; nx, ny >= 5): alternating x/y line sweeps,
 * each sweep direction in two colours of lines (odd line index, then even,
 * the film re-evaluated in between), every colour one batched PAQIF solve of
 * its lines (its active-set iteration starts from the set the same lines
 * ended with one step earlier); weighted change with quarter weights to the four neighbours
 * (eq. 69); y-lines change the direct nodes only; H0 <- H0 - c (2 pi/3 -
 * hx hy sum P) after each direction (eq. 75); convergence tested after each
 * x+y step.  P, H: DEVICE B x nx x ny; rough must be NULL.
 */
size_t ehl_newton_workspace_bytes(paqif_handle handle, const ehl_grid *grid, int B,
                                  const ehl_opts *opts);
int ehl_newton_tvd(paqif_handle handle, const ehl_grid *grid, const ehl_params *params, int B,
                   const ehl_opts *opts, const double *rough, double *P, double *H0, double *H,
                   double *Hmin, int32_t *status, int32_t *iters, void *workspace, void *stream);


/*
 * ehl_adjoint_solve -- line contact: gradients of a scalar output of the
 * converged solution (P, H0) with respect to M, L and the roughness profile.
 * The paper has no adjoint; this is the exact derivative of its discrete
 * equations at the fixed point of Sec. 3.3 (Reynolds residual with the TVD
 * flux of eqs. 62-65 on the pressurised nodes, load balance of eq. 75), with
 * the cavitated set, the limiter branches and the film's arg-min held fixed.
 * The caller supplies the cotangents of the output,
 *    gP (d out / d P), gH0 (d out / d H0), gH (d out / d H, H the film),
 * e.g. gH0 = 1 for out = H0, or gH = e_m at the arg-min m for out = Hmin.
 * The transposed bordered Jacobian is solved for both right-hand sides of its
 * Schur split by GMRES(40), right-preconditioned with a PAQIF solve of the
 * transposed Newton band (cavitated rows pinned); the dense part K (dR/dH)^T
 * v is the FP64 MFMA deformation product.
 *  params: DEVICE ehl_params[B];  rough: DEVICE nx x B or NULL (as in the
 *  forward solve);  P: DEVICE nx x B, H0: DEVICE [B] -- the converged state
 *  (P > 0 marks the pressurised nodes).
 *  gP, gH: DEVICE nx x B or NULL (zero);  gH0: DEVICE [B] or NULL.
 *  rtol: relative residual target of the transposed solves (0 < rtol < 1);
 *  max_iter: cap on Arnoldi steps per solve.
 *  dM, dL: DEVICE [B];  drough: DEVICE nx x B (d out / d roughness_m).
 *  status: DEVICE int32[B] (SYS_OK, SYS_ADJOINT_NOT_CONVERGED: the residual
 *  stalled above max(1e-8, rtol), SYS_NONFINITE);  iters: DEVICE int32[B],
 *  Arnoldi steps of the two solves together.
 *  opts: switch_ratio and kernel_terms select the preconditioning band (use
 *  the forward solve's options).
 *  workspace: DEVICE, ehl_adjoint_workspace_bytes(handle, grid, B).  The
 *  call synchronises the stream (convergence checks on the host).
 */
size_t ehl_adjoint_workspace_bytes(paqif_handle handle, const ehl_grid *grid, int B);
int ehl_adjoint_solve(paqif_handle handle, const ehl_grid *grid, const ehl_params *params, int B,
                      const ehl_opts *opts, const double *rough, const double *P,
                      const double *H0, const double *gP, const double *gH0, const double *gH,
                      double rtol, int max_iter, double *dM, double *dL, double *drough,
                      int32_t *status, int32_t *iters, void *workspace, void *stream);

/* ------------------------------------------------------------------------
 * Linear convection-diffusion workload (Sec. 4, linear case study of
 * Example 1, kappa-schemes of Sec. 3.1): the banded solver on non-symmetric,
 * non-complementarity line systems.
 * ------------------------------------------------------------------------ */

/*
 * (a u)_x + (b u)_y - eps (u_xx + u_yy) = f on [-1, 1]^2, Dirichlet data, a,
 * b > 0 constant (the paper does not give a(x, y), b(x, y)).  Grid n x n
 * nodes, h = 2/(n-1), arrays row major: u[i*n + j] = u(x_i, y_j).
 * Convection: kappa-scheme flux difference c (u_{i+1/2} - u_{i-1/2}) / h,
 * u_{i+1/2} = u_i + (1+kappa)/4 (u_{i+1} - u_i) + (1-kappa)/4 (u_i - u_{i-1}),
 * ghost u_{-1} = 2 u_0 - u_1 next to the inflow boundary; diffusion 5-point.
 *
 * cd_example: f for the exact solution u = x^4 + y^4 and the start iterate
 * (exact boundary values, zero inside).  f, u: DEVICE n x n, out.
 *
 * cd_line_relax: line relaxation as a defect correction (the paper's line
 * splittings): a half-step solves, on all n-2 lines of one direction in one
 * batched PAQIF launch (plain linear mode, half-bandwidth 2), M sigma =
 * f - L_h u with M the line's whole operator along the line plus the
 * diagonal of the across-line part, then u += omega sigma; x- and y-lines
 * alternate.  Stops after the first full iteration with
 * max|f - L_h u| <= tol max|f| (interior nodes), or after max_iter.
 *  n >= 5; -1 <= kappa < 1; eps >= 0; a, b > 0; 0 < omega < 2.
 *  f: DEVICE n x n in;  u: DEVICE n x n in/out (boundary values are kept).
 *  iters, defect: HOST out (iterations done, final max |f - L_h u|; a
 *  non-finite defect stops the iteration and is returned as infinity).
 *  workspace: DEVICE, cd_workspace_bytes(n) bytes.  Synchronises the stream
 *  once per iteration (the stopping test is read on the host).
 */
size_t cd_workspace_bytes(int n);
int cd_example(int n, double eps, double a, double b, double *f, double *u, void *stream);
int cd_line_relax(paqif_handle handle, int n, double kappa, double eps, double a, double b,
                  double omega, double tol, int max_iter, const double *f, double *u,
                  int32_t *iters, double *defect, void *workspace, void *stream);

/*
 * cd_split_relax -- the paper's x-line splittings Ls0 (which = 0, Sec. 3.1
 * eq. 48) and Ls1 (which = 1, eq. 49) of the same problem, as a defect
 * correction: x-line j solves L0 sigma = f - L_h u with the tridiagonal
 * implicit operator u_{i-1}: -eps/h^2 - w a/h, u_i: w a/h + 4 eps/h^2 +
 * b/h (3 - 3 kappa)/4 (the line's own y-convection coefficient; (1 -
 * kappa)/2 on the first line), u_{i+1}: -eps/h^2, w = (2 - kappa)/2 (Ls1)
 * or (2 - kappa)/2 + (1 - kappa)/4 (Ls0), then u += omega sigma on the line
 * (omega < 1: the paper's under-relaxation).  The paper sweeps the x-lines
 * in lexicographic order; here one iteration solves the odd lines, then the
 * even ones, each colour in one batched PAQIF launch (linear mode,
 * half-bandwidth 2), each on the defect after the other colour's update.
 * Arguments as for cd_line_relax (workspace: cd_workspace_bytes(n) bytes);
 * PAQIF_EINVAL for which not 0 or 1.
 */
int cd_split_relax(paqif_handle handle, int n, int which, double kappa, double eps, double a,
                   double b, double omega, double tol, int max_iter, const double *f, double *u,
                   int32_t *iters, double *defect, void *workspace, void *stream);

/*
 * cd_distributive_relax -- the distributive line relaxation (Ls3 of Sec. 3.1,
 * eqs. 51-54) of the same problem: a node's change is distributed,
 * u_ij += s_ij - (s_{i+-1,j} + s_{i,j+-1}) / 4, and every line solves for
 * ghost changes s whose distributed pattern cancels its defect (row (i, l),
 * column k: L_h of the pattern of a unit ghost change at the line's node k,
 * read at (i, l); half-bandwidth 3, one batched PAQIF launch in plain linear
 * mode per colour).  One iteration: x-lines odd then even, y-lines odd then
 * even (line index parity; neighbouring lines' patterns overlap), then the
 * defect test.  The paper notes this splitting is not robust: it converges
 * far more slowly than cd_line_relax.  Arguments as for cd_line_relax;
 * workspace: cd_ls3_workspace_bytes(n) bytes (0 = invalid n).
 */
size_t cd_ls3_workspace_bytes(int n);
int cd_distributive_relax(paqif_handle handle, int n, double kappa, double eps, double a,
                          double b, double omega, double tol, int max_iter, const double *f,
                          double *u, int32_t *iters, double *defect, void *workspace,
                          void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PAQIF_EHL_H */
