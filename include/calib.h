/* calib.h - C ABI of the MI355X consensus-ADMM calibration library.
 *
 * The library solves the distributed calibration problem of Yatawatta (2015), "Distributed
 * radio interferometric calibration": for every subband f (one compute agent of the paper) and
 * direction k it estimates 2x2 complex Jones matrices J_fkp of N stations such that the model
 * visibilities sum_k J_fkp C_fkpq J_fkq^H (Section 2, visibility model) fit the observed
 * V_fpq in least squares (Section 2, cost), while the Jones matrices of all subbands are tied
 * to a polynomial in frequency J_fk = B_f Z_k (Section 3, smoothness constraint) by consensus
 * ADMM (Section 3, minimisations M1-M3 and steps D1-D3).  All subbands live on one GPU; the
 * paper's network exchange becomes a device-wide reduction over subbands.
 *
 * Local step (M1): per direction a SAGE expectation (Section 3) and a Levenberg-Marquardt
 * minimisation of the augmented Lagrangian
 *     L_fk(J) = sum ||V_fk - c J_p J_q^H||^2 + Re tr(Y_fk^H (J - B_f Z_k)) + rho_k/2 ||J - B_f Z_k||^2
 * (the linear term in the trace form of Appendix A).  The paper minimises M1 with a Riemannian
 * trust region; this library uses Levenberg-Marquardt with Nielsen's damping rule on the
 * Gauss-Newton normal equations, solved by a batched FP64 Cholesky factorisation.
 *
 * Data conventions
 *   - Baselines b enumerate station pairs p<q row-major (no autocorrelations); 2x2 matrices are
 *     row-major complex, interleaved (re, im).
 *   - Visibilities: per subband, sample s = (b*T + t)*n_chan[f] + ch; vis holds
 *     sum_f B*T*n_chan[f] samples of 2x2 complex (8 reals).
 *   - Coherencies: the paper's C = c * I2 for an unpolarised point source (Section 2), so one
 *     complex scalar per sample and direction; per subband laid out [k][b][t][ch] for
 *     k < n_dirs[f]; coh holds sum_f n_dirs[f]*B*T*n_chan[f] complex scalars.
 *   - Element type of vis/coh: double for CALIB_FP64, float for CALIB_FP32_MIXED.  J, Z, Y and
 *     B_f Z are always double complex: J/Y/BZ [P][K][N][2][2], Z [K][Q][N][2][2] (monomial basis
 *     b_l(f) = ((f - f0)/f0)^(l-1), Section 3).
 *   - Flags: one byte per (subband, baseline), 1 = baseline flagged in that subband; flagged
 *     baselines are excluded from every sum and never read after calib_init.
 *
 * Ownership and execution
 *   - Pointers marked "device" are GPU memory owned by the caller; calib_init and calib_set_data
 *     read them into the context (a packed copy and the statistics, or the statistics alone with
 *     CALIB_OPT_STATS_ONLY), so the caller may release them once the stream has synchronised.
 *     Pointers marked "host" are read during the call only.
 *   - All work is enqueued on the stream given to calib_init (a hipStream_t, NULL = default
 *     stream).  Entry points return once the work is enqueued, except where stated.
 *   - A context is not thread-safe; distinct contexts are independent.
 *
 * Errors: every entry point returns a calib_status; nothing aborts or throws across the ABI.
 * calib_last_error gives a message for the last failure of a context (or of calib_init, with a
 * NULL context).
 */
#ifndef CALIB_MI355X_H
#define CALIB_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct calib_ctx calib_ctx;

typedef enum {
  CALIB_OK = 0,
  CALIB_E_INVAL = 1,    /* bad argument or configuration                                      */
  CALIB_E_NOMEM = 2,    /* device allocation failed                                           */
  CALIB_E_DEVICE = 3,   /* a HIP call failed                                                  */
  CALIB_E_RANK = 4,     /* fewer than Q distinct subband frequencies carry a direction (the
                           rank condition P >= F of the Z update, Section 3)                  */
  CALIB_E_NUMERIC = 5,  /* non-finite values in the inputs (calib_init); or, from admm_solve, a
                           subband whose LM objective is not finite at the start of a run or
                           whose damped normal equations cannot be solved even at a damping
                           1e16 times the run's initial one (that subband's runs then stop;
                           CALIB_FIELD_STATUS names it)                                       */
  CALIB_E_STATE = 6     /* entry point called out of order, or the device's local-step
                           schedule did not finish within its LM iterations                   */
} calib_status;

typedef enum { CALIB_FP64 = 0, CALIB_FP32_MIXED = 1 } calib_precision;

/* options */
#define CALIB_OPT_GPA_FIRST_ITER 1u  /* align the unitary ambiguity across subbands after the first
                                        local step (Section 3, initialisation)                  */
#define CALIB_OPT_UNREG_FIRST 2u     /* first local step without the consensus terms            */
#define CALIB_OPT_STATS_ONLY 4u      /* keep only the per-baseline coherency statistics, no packed
                                        copy of the samples (the matrix-free solver works from the
                                        statistics alone; a new interval is then one read of the
                                        inputs): needs solver 3 (else CALIB_E_INVAL);
                                        CALIB_FIELD_MODEL_VIS returns CALIB_E_STATE and
                                        CALIB_FIELD_COST comes from the statistics              */

typedef struct {
  int32_t n_stations;      /* N >= 2                                                           */
  int32_t n_subbands;      /* P >= 1 (the paper's compute agents)                              */
  int32_t n_basis;         /* Q >= 1 polynomial terms (the paper's F)                          */
  int32_t n_dirs_max;      /* K >= 1                                                           */
  int32_t n_times;         /* T >= 1 time slots of the solution interval                       */
  const int32_t *n_chan;   /* host [P], channels per subband, >= 1                             */
  const int32_t *n_dirs;   /* host [P], directions per subband 1..K (nested 0..K_f-1); NULL = K */
  const double *freq_hz;   /* host [P], subband frequency at which b_f is evaluated             */
  double f0_hz;            /* basis reference frequency (> 0)                                  */
  const double *rho;       /* host [K], per-direction rho >= 0 (0 = normal calibration)        */
  calib_precision precision;
  int32_t lm_iters;        /* LM iterations per direction per local step, >= 1                  */
  int32_t sage_sweeps;     /* SAGE sweeps over the directions per local step, >= 1              */
  uint32_t options;        /* CALIB_OPT_* bits                                                  */
  int32_t tile_group;      /* lanes per baseline in the streaming passes: 4, 8, 16, 32 or 64
                              (a tile holds 256 / tile_group baselines); 0 = chosen from the
                              samples per baseline among 8..64 (tile-shape tuner output), or 4
                              with solver 3 (its per-baseline kernels take one lane per
                              baseline of a tile)                                              */
  int32_t stream_grid;     /* workgroups of the streaming passes: 0 = one per tile, > 0 = a
                              persistent grid striding over the tiles                          */
  double lm_tol;           /* LM stopping rule: a direction's LM run ends after an iteration whose
                              step predicts a decrease ell <= lm_tol * F (F the objective before
                              the step); 0 = always lm_iters iterations.  Skipped iterations
                              launch nothing for that subband; their CALIB_FIELD_LM_TRACE rows
                              repeat (F, lambda) with accepted = 0                             */
  int32_t solver;          /* solver of the damped normal equations of each LM step: 1 = Cholesky,
                              one workgroup per subband matrix; 2 = Cholesky in 64-column panels
                              spread over many workgroups per matrix (for batches that leave
                              compute units idle); 3 = matrix-free preconditioned conjugate
                              gradients on the Gauss-Newton operator (no dense matrix is formed:
                              the operator is applied from S_b and J, Section 3 and Appendix A
                              operator form), stopped at cg_tol; 0 = Cholesky, chosen from the
                              number of subbands                                               */
  double cg_tol;           /* solver 3: stop once ||G + (H + (rho + lambda) I) delta|| <= cg_tol ||G||
                              (or after 8N iterations); 0 = 1e-10                              */
} calib_config;

/* Field selectors for calib_get. */
#define CALIB_FIELD_J 0          /* double complex [P][K][N][2][2]                              */
#define CALIB_FIELD_Z 1          /* double complex [K][Q][N][2][2]                              */
#define CALIB_FIELD_BZ 2         /* double complex [P][K][N][2][2], B_f Z_k                     */
#define CALIB_FIELD_Y 3          /* double complex [P][K][N][2][2], Lagrange multipliers        */
#define CALIB_FIELD_MODEL_VIS 4  /* vis layout and element type: sum_k c J_p J_q^H, zero on
                                    flagged baselines (Section 2, visibility model)           */
#define CALIB_FIELD_COST 5       /* double [P]: data cost g_f at the current J (Section 2): a
                                    pass over the samples, or with CALIB_OPT_STATS_ONLY the
                                    expansion over the coherency statistics                    */
#define CALIB_FIELD_TRACE 6      /* double [admm iterations run][4]: data cost after the local
                                    step, augmented Lagrangian, primal, dual residual         */
#define CALIB_FIELD_LM_TRACE 7   /* double [P][K][lm_iters][3] of the last SAGE sweep of the last
                                    local step: objective after each LM iteration, damping
                                    lambda, 1 if the step was accepted                        */
#define CALIB_FIELD_LM_STEP 8    /* double [P][2][8N]: gradient G and solution delta of
                                    (H_GN + (rho + lambda) I) delta = -G of the last LM
                                    iteration (real parameters p*8 + (i*2+j)*2 + re/im)       */
#define CALIB_FIELD_WORK 11      /* double [P][2]: conjugate-gradient iterations and LM solves
                                    of solver 3 per subband since calib_set_kernel_timing last
                                    enabled timing (measurement aid: the algorithmic work of the
                                    local step's launches)                                     */
#define CALIB_FIELD_STATUS 10    /* int32 [P]: CALIB_OK, or CALIB_E_NUMERIC for a subband whose
                                    objective became non-finite or whose normal equations could
                                    not be solved (reset by calib_set_jones / calib_set_state)  */

/* Validate the configuration, pack the inputs into the library's baseline-major layout (dropping
 * flagged baselines, converting nothing: the element type must match cfg->precision; no packed
 * copy with CALIB_OPT_STATS_ONLY), compute the per-baseline coherency statistics
 * S_b = sum |c|^2, U_l = sum conj(c_l) V, X_lm = sum conj(c_l) c_m and sum ||V||^2 (everything
 * the matrix-free local steps need from the samples), set J to jones0 (or identity blocks, Section 3 initialisation) and
 * Z = Y = 0.
 *   vis    device, see layout above;       coh    device, see layout above
 *   flags  device [P*B] or NULL;           jones0 device double complex [P][K][N][2][2] or NULL
 *   hip_stream  hipStream_t or NULL;       out    receives the new context
 * Returns CALIB_E_RANK when some direction has fewer than Q subbands or the basis matrix of its
 * subband frequencies is rank deficient. */
calib_status calib_init(const calib_config *cfg, const void *vis, const void *coh,
                        const uint8_t *flags, const void *jones0, void *hip_stream,
                        calib_ctx **out);

/* Step D1/S1 for all subbands at ADMM iteration admm_iter (minimisation M1): the residual's
 * energy (one pass over the samples) and every direction's per-baseline statistics of the
 * residual, then for each SAGE sweep and direction lm_iters Levenberg-Marquardt iterations on
 * L_fk with Y and B_f Z from the previous consensus update (fewer under the stopping rule).  At admm_iter 0 with
 * CALIB_OPT_UNREG_FIRST the consensus terms are left out. */
calib_status admm_local_step(calib_ctx *ctx, int32_t admm_iter);

/* Steps D2 and D3 (minimisations M2 and M3): at admm_iter 0 with CALIB_OPT_GPA_FIRST_ITER first
 * align the unitary ambiguity of each direction across subbands; then per direction
 * Z_k = argmin sum_f ||J_fk + Y_fk/rho_k - B_f Z_k||^2 (the closed-form Z of Section 3, solved by
 * QR of the basis matrix), B_f Z_k, Y_fk += rho_k (J_fk - B_f Z_k), and the primal and dual
 * residuals of Section 4.1 into the trace row of admm_iter. */
calib_status admm_consensus_update(calib_ctx *ctx, int32_t admm_iter);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the fusion-centre part of admm_consensus_update at an
 * iteration after the first, on caller-owned arrays and without a context - Z_k, B_f Z_k, the
 * dual update of Y and the primal and dual residuals - computed by the same kernels.  Their
 * working memory (basis values, the per-direction least-squares operator, residual partials,
 * direction counts, a rank flag) is a fixed 4 MiB device array inside the library, one per GPU,
 * held until the process ends; nothing is allocated or freed.
 *   n_stations N in [2, 128], n_subbands P >= 1, n_basis Q in [1, 8], n_dirs_max K in [1, 16], with
 *   P*(Q + K*Q + K) + 16K + 4 + (P + 3)/2 <= 524288 (else CALIB_E_INVAL, nothing enqueued)
 *   n_dirs   device int32 [P] directions per subband (nested 0..K_f-1), or NULL = K for all
 *   freq_hz  device double [P];  f0_hz > 0;  rho  device double [K], >= 0
 *   jones    device double complex [P][K][N][2][2] (read only)
 *   y        device, same layout: Y in, Y + rho (J - B_f Z) out
 *   z        device double complex [K][Q][N][2][2]: the previous Z in (for the dual residual), the
 *            new Z out
 *   bz       device, J's layout: B_f Z out (slots of directions a subband does not carry are
 *            left as they are, as are those of y)
 *   residuals device double [2] (primal, dual of Section 4.1) or NULL
 *   status   device int32 [1] or NULL: CALIB_OK, or CALIB_E_RANK when the basis matrix of the
 *            subbands carrying some direction is rank deficient (then y, z, bz and residuals are
 *            left unchanged)
 * Enqueued on hip_stream (of the current device), returns without synchronising.  Calls that
 * overlap on one GPU share the working memory and race; each call rewrites all of it.  Errors are
 * reported by calib_last_error(NULL). */
calib_status calib_consensus_noalloc(int32_t n_stations, int32_t n_subbands, int32_t n_basis,
                                     int32_t n_dirs_max, const int32_t *n_dirs,
                                     const double *freq_hz, double f0_hz, const double *rho,
                                     const double *jones, double *y, double *z, double *bz,
                                     double *residuals, int32_t *status, void *hip_stream);

/* The whole C-ADMM loop: iterations 0..max_iters-1 of local step + consensus update.  Iteration
 * 0 is enqueued kernel by kernel; the launch sequence of the later iterations is identical, so it
 * is captured once into a HIP graph and replayed (not while kernel timing is enabled).  With
 * solver 3 the whole local step is one launch whose workgroups apply the LM stopping rule
 * themselves, so the graph is replayed whatever lm_tol is.  With a Cholesky solver and
 * lm_tol > 0 the local step is launched directly instead, one LM iteration of every unfinished
 * subband per step, each subband moving through its own directions and SAGE sweeps; after each
 * step's solve the host reads a word of pinned memory that the device writes (whether every
 * subband has finished its local step) and launches the next step only if not; results per
 * subband are those of the iteration-by-iteration schedule of admm_local_step.  When
 * rel_cost_tol > 0 it stops after an iteration whose data cost changed by less than
 * rel_cost_tol relative to the previous one (this check synchronises the stream each
 * iteration).  trace_out (host, may be NULL) receives [iters][4] as CALIB_FIELD_TRACE;
 * iters_done (host, may be NULL) the number of iterations run.  Synchronises the stream.
 * Returns CALIB_E_NUMERIC (after the iterations) when some subband's state became non-finite or
 * its normal equations could not be solved; CALIB_FIELD_STATUS names the subbands. */
calib_status admm_solve(calib_ctx *ctx, int32_t max_iters, double rel_cost_tol, double *trace_out,
                        int32_t *iters_done);

/* Copy a field into caller memory.  dst is device memory for every field except
 * CALIB_FIELD_TRACE (host).  Enqueued on the context's stream. */
calib_status calib_get(calib_ctx *ctx, int32_t field, void *dst);

/* Overwrite J (device double complex [P][K][N][2][2]) - a warm start for a new solve on the
 * same data, e.g. the previous solution interval's J (Section 3) or a learned prediction -
 * and reset Y, Z and B_f Z to zero. */
calib_status calib_set_jones(calib_ctx *ctx, const void *jones);

/* Overwrite the whole C-ADMM state for a warm start that carries the dual variables as well:
 * J (required), Y, Z and B_f Z (each may be NULL = zero), device double complex in the layouts
 * above (Z [K][Q][N][2][2]).  bz must equal B_f Z for this context's frequencies, e.g. the previous
 * solution interval's.  The next admm_solve or admm_local_step(0) continues the iteration from
 * this state; a context initialised without CALIB_OPT_GPA_FIRST_ITER keeps its gauge. */
calib_status calib_set_state(calib_ctx *ctx, const void *jones, const void *y, const void *z,
                             const void *bz);

/* A new solution interval of the same observation (Section 3 calibrates interval after interval):
 * visibilities and coherencies of the same array, subband frequencies, channel and direction
 * counts and flags as at calib_init (device, same layouts and element type).  Repacks them into
 * the context's buffers (unless CALIB_OPT_STATS_ONLY) and recomputes the per-baseline coherency
 * statistics (S_b, U_l, X_lm, sum ||V||^2) in one pass over the inputs; J, Y, Z and B_f Z are kept - the previous interval's solution, the
 * paper's warm start (Section 3, initialisation) - until calib_set_state or calib_set_jones
 * replaces them.  Allocates nothing and does not synchronise.  Non-finite inputs mark their
 * subbands CALIB_E_NUMERIC in CALIB_FIELD_STATUS, and the next admm_solve returns it. */
calib_status calib_set_data(calib_ctx *ctx, const void *vis, const void *coh);

/* Kernel classes reported by CALIB_FIELD_KERNEL_TIMES. */
#define CALIB_KERNEL_REFRESH 0      /* every direction's per-baseline residual statistics and
                                       the residual's energy (from the coherency statistics
                                       with solver 3, over the samples otherwise)              */
#define CALIB_KERNEL_LM_BEGIN 1     /* initial objective and damping of a direction            */
#define CALIB_KERNEL_ASSEMBLE 2     /* gradient and dense Gauss-Newton normal equations (the
                                       Cholesky solvers only)                                   */
#define CALIB_KERNEL_CHOL_SOLVE 3   /* batched FP64 solve of the damped normal equations
                                       (Cholesky factorisation, or the gradient and conjugate
                                       gradients of solver 3)                                   */
#define CALIB_KERNEL_TRIAL 4        /* cost and per-baseline statistics at the LM trial point    */
#define CALIB_KERNEL_LM_UPDATE 5    /* gain ratio, accept/reject, damping update                */
#define CALIB_KERNEL_COMMIT 6       /* SAGE commit: every later direction's statistics and the
                                       residual energy updated for the direction just solved    */
#define CALIB_KERNEL_CONSENSUS 7    /* Lagrangian trace, alignment, Z, B_f Z, Y, residuals      */
#define CALIB_KERNEL_LOCAL_STEP 8   /* solver 3: every subband's whole local step (LM runs with
                                       the matrix-free solve, stopping rule, SAGE commits) in one
                                       launch after the refresh                               */
#define CALIB_KERNEL_PACK 9         /* calib_set_data: the interval's coherency statistics (and,
                                       unless statistics-only, the packed samples), and the
                                       dense S table rebuilt                                    */
#define CALIB_NUM_KERNELS 10
#define CALIB_FIELD_KERNEL_TIMES 9  /* host double [CALIB_NUM_KERNELS][2]: launches and total
                                       milliseconds since timing was enabled (synchronises)     */

/* Measurement aid: when enable != 0, every kernel launch of the context is bracketed by a pair
 * of HIP events recorded on the context's stream, and CALIB_FIELD_KERNEL_TIMES accumulates the
 * launch count and elapsed time per kernel class.  Enabling resets the counters. */
calib_status calib_set_kernel_timing(calib_ctx *ctx, int32_t enable);

/* ---- Warm start of a new solution interval ----------------------------------------------------
 * Section 3 initialises a new interval's C-ADMM iteration from the previous interval's solution.
 * The learned warm start refines that: a small network maps per-station features of the new
 * data at the previous solution to a correction of each station's Jones matrix, and a per-subband
 * cost comparison keeps the correction only where it does not raise the data cost.  The features
 * and the fallback run here; the network is the calib_mlp API below.
 *
 * Rows r = (f*K + k)*N + p; a row of a direction the subband does not carry is zero. */
#define CALIB_WS_FEATURES 32   /* features per row                                             */
#define CALIB_WS_OUTPUTS 8     /* network outputs per row                                      */
#define CALIB_WS_SCALE 10.0    /* scale s of the difference features and of the outputs        */

/* Features at the context's current J (the previous interval's solution, set by calib_set_jones
 * with the new interval's data loaded by calib_init), device float [P*K*N][32]:
 *   [0,8)   J_p
 *   [8,16)  s (J_p - J2_p)            J2 = jones_prev2 (the interval before; device double
 *                                     [P][K][N][2][2]) or zero when jones_prev2 is NULL
 *   [16,24) s (-1/2) G_p Q_p^-1       per-station Gauss-Newton step of the new data with the other
 *                                     stations held (G_p: gradient of the data cost of direction k
 *                                     after the SAGE expectation of Section 3; Q_p = sum_q S_pq
 *                                     J_q^H J_q); zero if Q_p is singular
 *   [24,32) s (BZ_p - J_p)            BZ = bz_prev (previous interval's B_f Z_k, device double
 *                                     [P][K][N][2][2]) or zero when bz_prev is NULL
 * J is unchanged on return. */
calib_status calib_warmstart_features(calib_ctx *ctx, const void *jones_prev2, const void *bz_prev,
                                      float *features);

/* Training target of the network for the interval whose converged J the context holds:
 * device float [P*K*N][8], row (f, k, p) = s (J_p U - Jprev_p) with U the unitary polar factor of
 * sum_p J_p^H Jprev_p, so that the target is free of the unitary ambiguity of the solution
 * (Section 3).  jones_prev: device double [P][K][N][2][2], the previous interval's solution. */
calib_status calib_warmstart_target(calib_ctx *ctx, const void *jones_prev, float *target);

/* J_learned = J + delta / s (delta: device float [P*K*N][8], the network output), then per
 * subband keep J_learned if its data cost is finite and not above that of the current J, else
 * restore the current J.  kept (device int32 [P], may be NULL) receives 1 where the learned value
 * was kept.  Y, Z and B_f Z are left as they are (set them first with calib_set_state to carry
 * the previous interval's dual variables, or calib_set_jones to start them at zero); the next
 * admm_solve starts at iteration 0 from this state. */
calib_status calib_warmstart_apply(calib_ctx *ctx, const float *delta, int32_t *kept);

/* ---- Warm-start network ------------------------------------------------------------------------
 * A fully connected network y = W_L^T(... GELU(W_1^T x + b_1) ...) + b_L with GELU(x) =
 * x Phi(x) between layers.  GEMM operands (inputs, activations, weights, output gradients) are
 * rounded to BF16 (round to nearest even) and multiplied on the matrix cores with FP32
 * accumulation; master weights, biases, pre-activations, gradients and the Adam moments are FP32.
 * Parameters are packed per layer l as W_l [dims[l]][dims[l+1]] row-major followed by
 * b_l [dims[l+1]]. */
typedef struct calib_mlp calib_mlp;

/* n_layers >= 1 layers of widths dims[0..n_layers] (host); params host FP32 (copied); max_rows
 * bounds the rows of every later call; work is enqueued on hip_stream.  Adam state starts at 0. */
calib_status calib_mlp_create(int32_t n_layers, const int32_t *dims, const float *params,
                              int64_t max_rows, void *hip_stream, calib_mlp **out);

/* y (device float [rows][dims[L]]) = network(x) (device float [rows][dims[0]]), 1 <= rows <=
 * max_rows. */
calib_status calib_mlp_forward(calib_mlp *m, const float *x, int64_t rows, float *y);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with the 1-based step) on the
 * mean square error mean((y - target)^2) over rows x dims[L] values; loss (device float [1], may
 * be NULL) receives the loss before the step.  lr = 0 computes the gradients only. */
calib_status calib_mlp_train_step(calib_mlp *m, const float *x, const float *target, int64_t rows,
                                  float lr, int32_t step, float *loss);

/* Copy the FP32 parameters (what = 0) or the last gradients (what = 1) into host memory in the
 * packed layout.  Synchronises the stream. */
calib_status calib_mlp_get(calib_mlp *m, int32_t what, float *dst);

/* Free the network's device memory (synchronises its stream). NULL is accepted. */
void calib_mlp_destroy(calib_mlp *m);

/* Message of the last failure on m, or of the last calib_mlp_create failure when m is NULL. */
const char *calib_mlp_last_error(const calib_mlp *m);

/* Free every device buffer of the context (synchronises its stream). NULL is accepted. */
void calib_destroy(calib_ctx *ctx);

/* Message of the last failure on ctx, or of the last calib_init failure when ctx is NULL. */
const char *calib_last_error(const calib_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* CALIB_MI355X_H */
