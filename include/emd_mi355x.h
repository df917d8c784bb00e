/*
 * emd_mi355x.h -- C ABI of the MI355X (gfx950) library for the Earth Mover's
 * Distance misfit between predicted and observed seismic shot gathers, in the
 * dynamic (Beckmann) form solved by primal-dual hybrid gradient with linesearch.
 *
 * Method: Yong, Liao, Huang, Li, Lin, "Misfit function for full waveform
 * inversion based on Earth Mover's Distance with dynamic formulation"
 * (arXiv 1808.07284).  Section 2.1 gives the signed-data recombination, Section
 * 2.2 the grid, the difference operators, the objective
 * Phi = ||u||_{1,1} + eps/2 ||u||_2^2 with EMD = Phi dx dt, the closed-form
 * primal/dual updates and Algorithm 1 (PDHG with linesearch); Section 2.3 makes
 * the dual potential phi the adjoint source of full waveform inversion.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout.  A batch holds `ngather` gathers.  Gather g is a dense row-major array
 *   [nr][nt] (receiver index i, time index j contiguous: the paper's (i, j)),
 *   starting `offset` elements into each batch buffer.  Element type is float in
 *   EMD_F32 precision and double in EMD_F64 precision, for every field buffer.
 *   The flux u is two such batches back to back: u^x at [0, N) and u^t at
 *   [N, 2N), N = the batch length given to emd_plan_create.
 * Operators.  grad is the backward difference with a zero first row/column
 *   (Section 2.2); div is minus its transpose, the forward difference of Section
 *   2.2 in the interior, -u/dx (-u/dt) on the last row (column), so that the
 *   adjoint identity <u, grad phi> = -<div u, phi> of Section 2.2 holds exactly.
 *   The constraint is div u + s = 0, s = Pcal - Pobs after normalisation (the
 *   paper's div u + Pcal - Pobs = 0), and the adjoint source is +phi.
 * Memory.  Every data pointer is a device pointer owned by the caller; the library
 *   never frees or retains it past the call.  The plan owns its workspace
 *   (padded solver state, per-gather scalars, reduction partials).
 * Streams.  Work is enqueued on `stream` (0 = the null stream).  emd_decompose
 *   and emd_adjoint_source never synchronise.  emd_pdhg_solve (and its resume and
 *   replay forms) synchronises the stream before its first chunk of sweeps, after
 *   every chunk of `sweeps_per_sync` sweeps (to read the number of finished
 *   gathers, and whenever some have finished their states, to narrow the sweeps
 *   to the running ones) and at the end (to read the per-gather states); with
 *   sweeps_per_sync = 0 it enqueues a fixed budget of sweeps and never
 *   synchronises (see emd_params).
 * Errors.  A call returns EMD_SUCCESS or an error code; emd_last_error() gives a
 *   message (per thread).  Bad arguments are reported before anything is
 *   enqueued.  Numerical outcomes are per-gather statuses (EMD_GATHER_*) in the
 *   emd_solve_info array, never call failures.
 * Device.  Calls run on the current HIP device, which must be the gfx950 device
 *   the plan was created on.
 * Threads.  A plan serves one call at a time: calls on one plan from several
 *   threads, or on streams whose work overlaps, race on its workspace.  Distinct
 *   plans are independent.
 */
#ifndef EMD_MI355X_H
#define EMD_MI355X_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t emd_status;

/* call status */
#define EMD_SUCCESS 0
#define EMD_ERR_INVALID_ARGUMENT 1 /* a size, spacing, mode or parameter is out of range */
#define EMD_ERR_NULL_POINTER 2     /* a required pointer is NULL                        */
#define EMD_ERR_DEVICE 3           /* the current device is not gfx950 / not the plan's */
#define EMD_ERR_HIP 4              /* a HIP runtime call failed                         */
#define EMD_ERR_OUT_OF_MEMORY 5    /* workspace allocation failed                       */
#define EMD_ERR_UNSUPPORTED 6      /* valid request that the library does not implement */

/* per-gather solve status, written into emd_solve_info.status */
#define EMD_GATHER_RUNNING 0
#define EMD_GATHER_CONVERGED 1      /* ||div u + s||_2 / ||s||_2 <= tol_res at a check   */
#define EMD_GATHER_MAX_ITER 2       /* max_iter iterations done without converging      */
#define EMD_GATHER_ZERO_SOURCE 3    /* s == 0: EMD = 0, u = phi = 0, no iteration        */
#define EMD_GATHER_NONFINITE 4      /* NaN/Inf in the source or during the iteration    */
#define EMD_GATHER_LS_FAIL 5        /* more than max_ls_trials backtracking steps       */
#define EMD_GATHER_MASS_IMBALANCE 6 /* mass mode none and |M_f - M_g| > mass_tol max M  */

typedef enum { EMD_MASS_BALANCE = 0, EMD_MASS_UNIT = 1, EMD_MASS_NONE = 2 } emd_mass_mode;
typedef enum { EMD_LS_L2 = 0, EMD_LS_L1 = 1, EMD_LS_FIXED = 2 } emd_ls_mode;
typedef enum { EMD_F32 = 0, EMD_F64 = 1 } emd_precision;

/* One gather of the batch (host array passed to emd_plan_create).
 * nr, nt >= 1; dx, dt > 0 are the spacings of the EMD grid (Section 2.2:
 * dx = X/(nr - 1), dt = T/(nt - 1)); an axis of length one drops its difference
 * terms and contributes 1 to the cell measure dx dt.  offset >= 0 is the element
 * offset of the gather in every batch buffer; gathers must not overlap. */
typedef struct {
    int32_t nr, nt;
    double dx, dt;
    int64_t offset;
} emd_gather_desc;

/* Solver parameters.  emd_params_default() fills the paper's constants:
 * eps = 1e-4 (Section 2.2), xi = 0.5, zeta = 0.99, delta = 1e5 (parameters of
 * Algorithm 1), theta_1 = 1.
 *   alpha1 <= 0 selects alpha_1 = (delta lambda)^(-1/2), lambda = 4/dx^2 + 4/dt^2
 *     the Gershgorin bound of Section 2.2, so that alpha_1 beta_1 = 1/lambda.
 *   alpha_max_factor > 0 caps every step at alpha_max_factor * alpha_1.
 *   tol_res: stop when ||div u + s||_2 / ||s||_2 <= tol_res, checked every
 *     check_every iterations (this certifies feasibility, not optimality).
 *   ls_mode: EMD_LS_L2 uses Euclidean norms in the linesearch test (the
 *     Malitsky-Pock setting); EMD_LS_L1 the l1 norms printed in Algorithm 1 (each
 *     sweep sums the test for the first 6 backtracking candidates of the next
 *     iteration; should all 6 fail, one extra sweep without an iteration sums the
 *     next 6); EMD_LS_FIXED is plain PDHG with theta = 1 and the fixed steps
 *     alpha_1, beta_1 = delta alpha_1.
 *   mass_mode: how emd_decompose builds s (see there) and emd_adjoint_source chains.
 *   precision: element type of all field buffers (EMD_F32: float fields, FP64
 *     reductions and scalars; EMD_F64: double throughout).
 *   sweeps_per_sync: iterations enqueued between reads of the finished count
 *     (even, 2..4096), or 0: the fixed-budget solve, which enqueues every sweep
 *     the budget allows (max_iter + 2, times up to max_ls_trials / 6 + 2 with the
 *     l1 test) and reads nothing back.  The stop rule still ends each gather's
 *     iterations on the device (its later sweeps only carry its state), and the
 *     results are bitwise those of the chunked solve.  Such a call neither
 *     synchronises nor allocates, so it can be captured into a HIP graph; the
 *     graph then uses the plan's workspace, tile table and parameters as they were
 *     at capture (keep the plan, and its tiling, while the graph may run).
 *     emd_plan_query and emd_solver_state synchronise the device before reading
 *     the state such a solve left.
 *   iters_per_sweep: 1 (or 0): one PDHG iteration per sweep of the fields; K = 2 or
 *     3: with EMD_LS_FIXED only, K iterations per sweep (one HBM pass reads u, phi, s
 *     and writes u, phi for K iterations; the fields are bitwise those of one
 *     iteration per sweep), with check_every a multiple of K: the stop rule is
 *     checked on multiples of K.  K = 3 needs EMD_F32. */
typedef struct {
    double eps, xi, zeta, delta, alpha1, alpha_max_factor, tol_res, mass_tol;
    int32_t max_iter, check_every, max_ls_trials, ls_mode;
    int32_t mass_mode, precision, sweeps_per_sync, iters_per_sweep;
} emd_params;

/* Per-gather result (device array written by emd_pdhg_solve).
 * The EMD estimate is the Lagrangian of Section 2.2 at the returned pair,
 *   emd = dx dt (Phi(u) + <phi, div u + s>),  Phi(u) = ||u||_{1,1} + eps/2 ||u||_2^2,
 * which equals the objective dx dt Phi(u) (`primal`) wherever the flux meets the
 * constraint and, at a stop-rule iterate that misses it by the residual, prices
 * that miss with the potential (the derivative of the optimal value with respect
 * to s).  On the seismic batches it is 5-6 times closer to the converged EMD than
 * `primal` at the same iteration. */
typedef struct {
    int32_t status;    /* EMD_GATHER_*                                    */
    int32_t iters;     /* accepted PDHG iterations                        */
    int32_t ls_trials; /* backtracking steps over the whole solve         */
    int32_t pad;
    double rel_res;    /* ||div u + s||_2 / ||s||_2 of the returned u      */
    double emd;        /* dx dt L(u, phi), as above (also in d_emd)       */
    double transport;  /* dx dt ||u||_{1,1}                                */
    double alpha;      /* last accepted primal step                        */
    double primal;     /* dx dt (||u||_{1,1} + eps/2 ||u||_2^2)            */
} emd_solve_info;

/* Solver state of one gather at the end of a solve (host struct): the step alpha_k
 * and theta_k of its last accepted iteration k, the counts, and its outcome (status,
 * and for a finished gather the residual, EMD and transport it reported).  With the
 * flux u_k and potential phi_k the solve returned, it is all a resumed solve needs
 * (see emd_pdhg_solve_resume); the EMD estimate of a finished gather is recomputed
 * from those fields. */
typedef struct {
    double alpha, theta;
    int32_t iters, ls_trials, status, pad;
    double rel_res, primal, transport;  /* primal: dx dt Phi(u) */
} emd_gather_state;

/* Plan statistics (host struct filled by emd_plan_query). */
typedef struct {
    int32_t ngather, tiles, rows_per_tile, samples_per_tile;
    int64_t batch_len;        /* N                                             */
    int64_t cells;            /* sum of nr * nt                                */
    int64_t workspace_bytes;  /* device memory owned by the plan               */
    int64_t last_sweeps;      /* sweep launches of the last emd_pdhg_solve     */
    int64_t last_cell_updates;/* sum over gathers of nr * nt * iterations      */
    double last_sweep_ms;     /* GPU time from the first to the last sweep     */
    int64_t last_table_rebuilds; /* times the last solve narrowed the sweep's tile
                                  * table to its running gathers                  */
} emd_plan_stats;

typedef struct emd_plan emd_plan;

/* Fill *p with the defaults above (max_iter 100000, check_every 10,
 * max_ls_trials 40, tol_res 1e-5, alpha_max_factor 1e6, mass_tol 1e-6,
 * sweeps_per_sync 64, EMD_LS_L2, EMD_MASS_BALANCE, EMD_F32). */
emd_status emd_params_default(emd_params* p);

/* Create a plan for `ngather` gathers described by the host array h_desc, in a
 * batch of `batch_len` elements, on the current device.  Validates every
 * descriptor and parameter, copies them, and allocates the workspace (9 field
 * copies of the padded batch plus per-tile scalars).  *out receives the
 * plan; it is NULL on failure. */
emd_status emd_plan_create(const emd_gather_desc* h_desc, int32_t ngather, int64_t batch_len,
                           const emd_params* p, emd_plan** out);

/* Release the plan and its workspace (synchronises the device first). NULL is a no-op. */
emd_status emd_plan_destroy(emd_plan* plan);

/* Replace the solver parameters of an existing plan (precision must not change).
 * Synchronises the device. */
emd_status emd_plan_set_params(emd_plan* plan, const emd_params* p);

/* Choose the tile height (receiver rows per wavefront tile, 1..1024) of every
 * gather's solver sweeps; 0 restores the default (16).  The fields a solve returns
 * do not depend on the tiling for a fixed step schedule; the linesearch inner
 * products are summed per tile, so free-running results may differ in the last
 * bits between tilings (each tiling is bitwise reproducible).  Synchronises the
 * device. */
emd_status emd_plan_set_tiling(emd_plan* plan, int32_t rows_per_tile);

/* Per-gather tile heights: h_rows is a host array of ngather values in [1, 1024]
 * (set) or receives them (get).  set synchronises the device. */
emd_status emd_plan_set_gather_tiling(emd_plan* plan, const int32_t* h_rows);
emd_status emd_plan_get_gather_tiling(const emd_plan* plan, int32_t* h_rows);

/* Tile-height autotuner.  Puts the gathers in 3 x 3 size buckets (tertiles of nt
 * and of nr over the batch) and, bucket by bucket (largest first), tries heights
 * 8, 12 and 16 for that bucket, timing a fixed-step solve of `sweeps` sweeps (even,
 * 4..4096; 0 = 48) of the whole batch from the source s (as given to
 * emd_pdhg_solve) in the production launch configuration (the fastest of three
 * runs after a warm-up), and keeps a height when it is faster by more than 0.3 %.
 * (Taller tiles are not tried: they lengthen each launch of the last few running
 * gathers, which a whole-batch timing does not see.)  The chosen heights stay in
 * the plan (read them with emd_plan_get_gather_tiling to reuse them).  The plan's
 * parameters are left unchanged; its workspace is overwritten; synchronises the
 * device.  Timing-based, so the choice can differ from run to run. */
emd_status emd_plan_autotune(emd_plan* plan, const void* s, int32_t sweeps, hipStream_t stream);

/* Residual history: in every later solve on the plan (emd_pdhg_solve and its
 * resume and replay forms), each gather's relative residual ||div u + s|| / ||s||
 * at every stop-rule check (iterations c * check_every, c = 1, 2, ...; the test of
 * Algorithm 1's stopping rule, Section 2.2) is written as a double to
 * d_hist[g * capacity + (c - 1) % capacity]: a ring holding each gather's last
 * `capacity` checks.  A resumed solve continues the count of its checkpoint.
 * Entries of checks a solve does not reach are not written, and the autotuner's
 * timing solves write none.  d_hist: caller-owned device memory of
 * ngather * capacity doubles that must stay valid while solves on the plan may
 * run; (NULL, 0) turns the history off (the default).  Never synchronises. */
emd_status emd_plan_set_history(emd_plan* plan, double* d_hist, int32_t capacity);

/* Fill *out with the plan's sizes and the counters of its last solve. */
emd_status emd_plan_query(const emd_plan* plan, emd_plan_stats* out);

/* Signed-data recombination and mass normalisation (Section 2.1).
 *   f = Pcal^+ + Pobs^-, g = Pobs^+ + Pcal^- (so f - g = Pcal - Pobs),
 *   d_mass[3 g + 0] = M_f = dx dt sum f,  d_mass[3 g + 1] = M_g = dx dt sum g,
 *   d_mass[3 g + 2] = mean(Pcal - Pobs)   (FP64 sums in a fixed order),
 *   s_out = (Pcal - Pobs) - mean(Pcal - Pobs)  (EMD_MASS_BALANCE),
 *         = f / M_f - g / M_g                  (EMD_MASS_UNIT),
 *         = Pcal - Pobs                        (EMD_MASS_NONE).
 * pcal, pobs, s_out: batch buffers of the plan's precision; f_out, g_out: optional
 * batch buffers (NULL to skip); d_mass: device double[3 ngather].  s_out must not
 * alias pcal or pobs. */
emd_status emd_decompose(emd_plan* plan, const void* pcal, const void* pobs, void* s_out,
                         void* f_out, void* g_out, double* d_mass, hipStream_t stream);

/* emd_decompose without a plan, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It computes what emd_decompose computes, with the same conventions
 * and outputs, for the gathers described by the host array h_desc (validated as by
 * emd_plan_create; the batch buffers must cover every gather's [offset, offset +
 * nr nt)), in `precision` and `mass_mode` (the emd_params values).  It calls no
 * allocating routine: the per-gather partial sums live in a file-scope device array
 * of the library, EMD_NOALLOC_MAX_GATHERS x 256 x 3 doubles (384 KiB) per device,
 * which each device holds until the process ends; more gathers than that are
 * rejected (EMD_ERR_INVALID_ARGUMENT).  The sums are taken in another fixed order
 * than emd_decompose's, so the two agree to the rounding of FP64 sums.  Every call
 * rewrites all of the partial sums it reads, but all calls on one device share the
 * array: calls that overlap on a device (other streams, other threads) race on it
 * and must be ordered by the caller.  Never synchronises. */
#define EMD_NOALLOC_MAX_GATHERS 64
emd_status emd_decompose_noalloc(const emd_gather_desc* h_desc, int32_t ngather, int32_t precision,
                                 int32_t mass_mode, const void* pcal, const void* pobs, void* s_out,
                                 void* f_out, void* g_out, double* d_mass, hipStream_t stream);

/* Solve min Phi(u) s.t. div u + s = 0 for every gather by PDHG with linesearch
 * (Algorithm 1, Section 2.2), all gathers in one batch of fused sweeps.
 *   s: source batch (from emd_decompose).
 *   u: optional flux, 2 batches [u^x | u^t]; read as the start point when
 *      warm_start != 0, and receives the final flux (NULL: cold start, not returned).
 *   phi: dual potential batch; read as the start point when warm_start != 0, and
 *      receives the final potential (required: it is the adjoint source).
 *   d_mass: optional device double[3 ngather] from emd_decompose; with
 *      EMD_MASS_NONE it flags gathers whose masses differ (MASS_IMBALANCE).
 *   d_emd: optional device double[ngather] receiving the EMD values.
 *   d_info: optional device emd_solve_info[ngather].
 * s must not alias u or phi (the same holds for the resume and replay forms). */
emd_status emd_pdhg_solve(emd_plan* plan, const void* s, void* u, void* phi, int32_t warm_start,
                          const double* d_mass, double* d_emd, emd_solve_info* d_info,
                          hipStream_t stream);

/* Checkpoint: the per-gather solver state at the end of the plan's last solve
 * (h_state: host emd_gather_state[ngather]).  Together with that solve's u and phi
 * it is a checkpoint of the iteration. */
emd_status emd_solver_state(const emd_plan* plan, emd_gather_state* h_state);

/* Resume: emd_pdhg_solve continued from a checkpoint instead of a cold start.
 * u and phi (required) hold the checkpoint's flux and potential on entry and the
 * final ones on return; h_state is the checkpoint's host emd_gather_state[ngather].
 * Each gather continues from iteration iters with steps alpha, theta: the first
 * sweep redoes the checkpointed iteration's primal update (the dual step was
 * applied), which rebuilds the previous residual and the linesearch inner
 * products, so a solve of K iterations resumed to 2K (max_iter counts from 0)
 * reproduces a single solve of 2K iterations bitwise.  A gather whose checkpointed
 * status is RUNNING or MAX_ITER continues; any other status (it met the stop rule,
 * or failed) is final: the gather is not iterated, keeps its status, residual, EMD
 * and transport, and its u and phi pass through unchanged, as in the uninterrupted
 * solve.  (A gather whose source is zero reports ZERO_SOURCE either way.)  alpha
 * must be finite and > 0 for the gathers that continue. */
emd_status emd_pdhg_solve_resume(emd_plan* plan, const void* s, void* u, void* phi,
                                 const emd_gather_state* h_state, const double* d_mass,
                                 double* d_emd, emd_solve_info* d_info, hipStream_t stream);

/* The same solve with the step sizes taken from a schedule instead of the
 * linesearch: iteration k of gather g uses alpha_{k+1} = d_alpha[g * ld_alpha + k]
 * (theta_{k+1} = alpha_{k+1} / alpha_k, beta_{k+1} = delta alpha_{k+1}) and
 * counts no backtracking.  Replaying the accepted steps of another solve of the
 * same problem reproduces its iterates up to rounding; the stop rule and
 * max_iter (<= ld_alpha) apply as usual. */
emd_status emd_pdhg_solve_replay(emd_plan* plan, const void* s, void* u, void* phi,
                                 int32_t warm_start, const double* d_alpha, int32_t ld_alpha,
                                 double* d_emd, emd_solve_info* d_info, hipStream_t stream);

/* Adjoint source psi = d EMD / d Pcal (Section 2.3: the dual potential phi is the
 * derivative of the misfit with respect to the data), chained through the mass
 * normalisation and scaled by the upstream gradient gbar_g:
 *   EMD_MASS_BALANCE: psi = dx dt gbar (phi - mean phi),
 *   EMD_MASS_UNIT:    psi = dx dt gbar [H (phi - pf)/M_f + (1 - H)(phi - pg)/M_g],
 *                     pf = <phi, f>/sum f, pg = <phi, g>/sum g, H = [Pcal > 0],
 *   EMD_MASS_NONE:    psi = dx dt gbar phi.
 * phi, psi_out: batch buffers; pcal, pobs: needed for EMD_MASS_UNIT only (else may
 * be NULL); d_mass: from emd_decompose (needed for EMD_MASS_UNIT); d_gbar: optional
 * device double[ngather] (NULL means 1).  psi_out must not alias any input. */
emd_status emd_adjoint_source(emd_plan* plan, const void* phi, const void* pcal,
                              const void* pobs, const double* d_mass, const double* d_gbar,
                              void* psi_out, hipStream_t stream);

/* The conventional least-squares misfit the paper compares the EMD with (Section
 * 2.1) and its adjoint source (Section 2.3), per gather:
 *   d_value[g] = 1/2 dx dt sum (Pcal - Pobs)^2      (FP64 sums in a fixed order),
 *   psi_out    = gbar dx dt (Pcal - Pobs)           (the exact gradient; optional).
 * pcal, pobs, psi_out: batch buffers of the plan's precision (psi_out NULL: value
 * only; it must not alias pcal or pobs); d_gbar: device double[ngather] upstream
 * gradients or NULL (= 1); d_value: device double[ngather].  Never synchronises. */
emd_status emd_lsd_misfit(emd_plan* plan, const void* pcal, const void* pobs, const double* d_gbar,
                          double* d_value, void* psi_out, hipStream_t stream);

/* Grid transfer for the multi-grid strategy (Section 2.2 closes on it: compute the
 * EMD on a coarse grid first, then run the primal-dual method on the fine grid;
 * Section 3.3 resamples each shot and interpolates the coarse solution back).
 * `fine` and `coarse` are plans of the same gathers in the same order, same
 * precision and device; the coarse gather g groups fr receivers by ft samples:
 * its size must be ceil(nr/fr) x ceil(nt/ft), and its spacings should be fr dx
 * and ft dt (then the flux, an integral of the source, and the potential, a
 * distance, keep their scale, so no values are rescaled).  Buffers are batch
 * buffers of each plan's layout; neither call synchronises.
 *
 * emd_restrict: coarse_out[I][J] = mean of fine_in over the block i in
 *   [fr I, min(fr I + fr, nr)), j in [ft J, min(ft J + ft, nt)) (FP64 sum), for
 *   each gather (use it on Pcal and on Pobs before emd_decompose on the coarse
 *   plan).  coarse_out must not alias fine_in. */
emd_status emd_restrict(const emd_plan* fine, const emd_plan* coarse, int32_t fr, int32_t ft,
                        const void* fine_in, void* coarse_out, hipStream_t stream);

/* emd_prolong: bilinear interpolation of a coarse solution onto the fine grid, for
 * a warm start (emd_pdhg_solve with warm_start = 1).  Each field keeps its
 * staggering: phi at cell centres (fine cell i at coarse coordinate
 * (i - (fr - 1)/2)/fr, clamped to the coarse cells); u^x on the receiver edges
 * (fine edge i, between cells i - 1 and i, at coarse coordinate i/fr on the coarse
 * edges 0..ceil(nr/fr), of which the first and last are boundary edges with no
 * flux) and at time cell centres; u^t likewise with the axes swapped.  u_c / u_f:
 * [u^x | u^t] batches of the coarse / fine plan; phi_c / phi_f: batches.  Either
 * output may be NULL (then its input is not read); outputs must not alias inputs. */
emd_status emd_prolong(const emd_plan* coarse, const emd_plan* fine, int32_t fr, int32_t ft,
                       const void* u_c, const void* phi_c, void* u_f, void* phi_f,
                       hipStream_t stream);

/* Human-readable name of a call status. */
const char* emd_status_string(emd_status status);

/* Message of the last failed call on this thread ("" if none). */
const char* emd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EMD_MI355X_H */
