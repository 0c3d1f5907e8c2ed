/*
 * chebgame.h -- C ABI of libchebgame.so, a gfx950 (MI355X) implementation of
 * the tensorial Chebyshev value iteration for the J-player transboundary
 * pollution game of de Castro, Gaton & Gomez (arXiv 2307.04688).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an int status: CG_OK (0) on success, a negative
 *    CG_E* code on error, or the positive warning CG_ENOTCONVERGED.  On error
 *    nothing observable has been written unless stated, and cg_last_error()
 *    returns a message for the calling thread.  No C++ exception crosses the
 *    ABI.
 *  - Device pointers ("_dev") are addresses in the memory of the current HIP
 *    device; they are owned by the caller and must stay valid until the work
 *    queued on 'stream' has finished.  Host pointers are read during the
 *    call only.  'stream' is a hipStream_t passed as void* (NULL = the null
 *    stream).  Work is queued asynchronously on it unless a function says it
 *    synchronises.
 *  - Tensors are FP64, C order (last mode fastest).  A value tensor of shape
 *    N x ... x N holds the values at the Chebyshev-Lobatto nodes
 *    x_k = cos(pi k / (N-1)), k = 0..N-1, so index 0 is x = +1 (Section 3.1);
 *    a coefficient tensor holds c_k of sum_k c_k T_{k_1}(x_1)...T_{k_d}(x_d).
 *  - State arrays of a game are [d][N^d]: player-major, then node index in
 *    C order.  State coordinates are physical, p in [0, p_max]^d, mapped to
 *    [-1,1]^d by x = 2 p / p_max - 1 (Section 3.4).
 */
#ifndef CHEBGAME_H
#define CHEBGAME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define CG_OK 0
#define CG_ENOTCONVERGED 1   /* warning: max_steps reached before the tolerance */
#define CG_EINVAL (-1)       /* invalid argument (message says which) */
#define CG_EUNSUPPORTED (-2) /* size or precision outside the compiled set */
#define CG_EDEVICE (-3)      /* HIP runtime error or no gfx950 device */
#define CG_ENOMEM (-4)       /* workspace too small */
#define CG_ENONFINITE (-5)   /* a non-finite value appeared in the iterate */

/* Arithmetic of the contractions.  CG_FP64: everything in binary64 (MFMA
 * f64).  CG_FP32 / CG_BF16 (cg_chebyshev_eval only): basis and coefficients
 * rounded to binary32 / bfloat16, products accumulated in binary32 on MFMA.
 * CG_FP32_CORR (games only): the contraction is split into an FP64 part
 * (value and first-order Taylor term at the node, computed by small mode
 * products) and a second-order remainder contracted at binary32 accuracy on
 * MFMA: for d = 3 with N rounded up to a multiple of 4 at least 20, both
 * operands are rounded to binary32 and split exactly into three bfloat16
 * pieces, and the six leading piece products run on bf16 MFMA with binary32
 * sums; otherwise on binary32 MFMA.  The transform, line fit, argmax, step
 * accumulation and residual stay FP64. */
#define CG_FP64 0
#define CG_FP32 1
#define CG_BF16 2
#define CG_FP32_CORR 3
/* cg_chebyshev_eval only: binary32 accuracy on the bf16 MFMA.  Basis
 * products and coefficients rounded to binary32 and split exactly into three
 * bfloat16 pieces; the six piece products of leading order (hi hi, hi mid,
 * mid hi, hi lo, mid mid, lo hi; the three dropped ones are below 2^-24 of
 * the product) accumulated in binary32.  Output float, like CG_FP32. */
#define CG_FP32_SPLIT 4

/* Sizes compiled into the library. */
#define CG_MAX_D 4   /* players (state dimension) */
#define CG_MAX_N 32  /* nodes per dimension */

/* Game description: the discrete-space LQ game of Section 2 with the time
 * discretisation of Section 2.1 and the grids of Section 3.4.
 *   drift      g_i(p,u) = (K p)_i / m_i - c_i p_i + beta_i u_i
 *              (K in the graph-Laplacian convention of the paper's examples:
 *              off-diagonal k_ij >= 0, diagonal = -(exchange + leakage))
 *   payoff     G_i(p,u) = u_i (A_i - u_i / 2) - phi_i p_i^2 / 2
 *   Bellman    V_i(p) = max_{0 <= u <= u_max} { h G_i(p_i,u)
 *                       + (1 - rho h) V_i(p + h g(p, [u, u_{-i}])) }
 * All host arrays are copied by cg_init_game. */
typedef struct cg_game_desc {
    int32_t d;          /* players = state dimension, 2..CG_MAX_D */
    int32_t n_nodes;    /* N: Lobatto nodes per state dimension, 3..CG_MAX_N */
    int32_t n_unodes;   /* control nodes per player on [0,u_max], 3..N rounded up to a
                           multiple of 4; 0 = N */
    int32_t reserved;   /* must be 0 */
    double h;           /* time step, > 0 */
    double rho;         /* discount rate; requires 0 < rho h < 1 */
    double p_max;       /* state box [0, p_max]^d, > 0 */
    double u_max;       /* control interval [0, u_max], > 0 */
    const double *K;    /* d*d row-major exchange matrix */
    const double *m;    /* d region measures (NULL = all 1), > 0 */
    const double *c;    /* d decay rates */
    const double *beta; /* d emission-to-stock factors */
    const double *A;    /* d benefit coefficients */
    const double *phi;  /* d damage coefficients */
} cg_game_desc;

typedef struct cg_game cg_game;

/* Message for the last failing call on this thread ("" if none). */
const char *cg_last_error(void);
/* Static description of a status code. */
const char *cg_strerror(int status);

/* Bytes of device workspace cg_init_game needs for this game and precision
 * (0 if the description is invalid; cg_last_error says why). */
size_t cg_workspace_bytes(const cg_game_desc *desc, int precision);

/* Step 0 of Section 2.1 (offline set-up).  Validates the description, builds
 * the node and control grids (Section 3.4) and the constants, carves the
 * caller-owned workspace ws_dev (>= cg_workspace_bytes, 256-byte aligned)
 * and queues on 'stream' the start V^{[0]} = 0 (zero terminal value),
 * u^{[0]} = A.  *out receives a handle that owns no device memory; the
 * workspace must outlive it.  precision: CG_FP64 or CG_FP32_CORR.
 * Errors: CG_EINVAL (bad description), CG_EUNSUPPORTED (d or N outside the
 * compiled set), CG_ENOMEM (workspace too small), CG_EDEVICE. */
int cg_init_game(const cg_game_desc *desc, int precision, void *ws_dev, size_t ws_bytes,
                 void *stream, cg_game **out);

/* Releases the handle (not the workspace).  NULL is accepted. */
int cg_destroy(cg_game *game);

/* Re-initialises an existing game in place with another description of the
 * same d, n_nodes and number of control nodes (its precision is kept): the
 * constants of Step 0 are rebuilt and V^{[0]} = 0, u^{[0]} = A, the iteration
 * count and the convergence test are reset.  The workspace layout does not
 * change, so a batch that holds the game stays valid: a finished game's slot
 * can take the next game of a stream.  Synchronises the game's stream.
 * Errors: CG_EINVAL (invalid or differently sized description), CG_EDEVICE. */
int cg_reset_game(cg_game *game, const cg_game_desc *desc);

/* Algorithm Cnv (Section 3.1, eq. (forcoef) along every mode): coefficient
 * tensors of 'batch' value tensors of shape n[0] x ... x n[d-1], stored one
 * after the other in vals_dev; coef_dev receives them in the same layout and
 * must not overlap vals_dev.  1 <= d <= CG_MAX_D, 2 <= n[l] <= CG_MAX_N.
 * Queued on 'stream'.  Errors: CG_EINVAL, CG_EUNSUPPORTED, CG_EDEVICE. */
int cg_chebyshev_transform(int d, const int32_t *n, const double *vals_dev, double *coef_dev,
                           int64_t batch, void *stream);

/* Value of the series sum_k c_k T_{k_1}(x_1)...T_{k_d}(x_d) (Definition of
 * the n-dimensional interpolant, Section 3.1; evaluation by mode products as
 * in Section 3.2) at npts points.  coef_dev: shape n[0] x ... x n[d-1] FP64;
 * x_dev: npts x d FP64 row-major, normalised coordinates (points outside
 * [-1,1]^d are evaluated by polynomial continuation); out_dev: npts values,
 * double for CG_FP64, float for CG_FP32, CG_BF16 and CG_FP32_SPLIT.  1 <= d <= CG_MAX_D,
 * 2 <= n[l] <= CG_MAX_N.  Needs cg_eval_workspace_bytes() bytes of device
 * workspace in ws_dev.  Queued on 'stream'. */
size_t cg_eval_workspace_bytes(int d, const int32_t *n, int precision);
int cg_chebyshev_eval(int d, const int32_t *n, const double *coef_dev, const double *x_dev,
                      int64_t npts, void *out_dev, int precision, void *ws_dev, size_t ws_bytes,
                      void *stream);

/* cg_chebyshev_eval without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * cg_chebyshev_eval (bitwise equal output); the packed coefficient operand
 * goes to a static device array of the library, 8 MiB + 256 bytes per GPU
 * (enough for every size in the compiled set; CG_EUNSUPPORTED beyond it),
 * held until the process ends.  The call allocates nothing.  Every call on a
 * GPU shares that GPU's array: calls that may overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller; calls
 * queued on one stream are ordered and safe. */
int cg_chebyshev_eval_noalloc(int d, const int32_t *n, const double *coef_dev, const double *x_dev,
                              int64_t npts, void *out_dev, int precision, void *stream);

/* nsteps iterations r -> r+1 of Steps 1-4 (Section 2.1, implemented as in
 * Section 3.4): coefficient transform of every V_i^{[r]}, evaluation of V_i at
 * every node's update points p + h g(p, [u_m, u^{[r]}_{-i}(p)]) for the control
 * nodes u_m, fit in u, argmax over [0, u_max], new value and control.  All
 * players use the same u^{[r]} (simultaneous update).  If residual_out is not
 * NULL the call synchronises 'stream' and stores max_{i,j} |V^{[r+1]} - V^{[r]}|
 * of the last iteration there; otherwise it only queues the work.  Errors:
 * CG_EINVAL, CG_EDEVICE, CG_ENONFINITE (only when synchronising). */
int cg_step(cg_game *game, int32_t nsteps, double *residual_out);

/* Iterates until the residual of an iteration is < tol (strict, the TOL test
 * of Step 4, taken on the nodes) or max_steps iterations are done.  tol <= 0
 * runs exactly max_steps iterations.  The test runs on the device: once an
 * iteration meets it, later queued iterations leave the state unchanged, so
 * the state is that of the first iteration below tol.  Synchronises 'stream'.
 * *steps_done and *residual (either may be NULL) receive the iterations done
 * by this call and the last residual.  Returns CG_ENOTCONVERGED if tol > 0 and
 * it was not met. */
int cg_solve(cg_game *game, int32_t max_steps, double tol, int32_t *steps_done, double *residual);

/* Checkpoint / warm start.  cg_get_state copies the current V and U
 * ([d][N^d] FP64 each, device) and stores the iteration count in *r (host,
 * nullable); it queues the copies on the game's stream.  cg_set_state
 * replaces them (U_dev NULL = u_i = A_i everywhere) and resets the
 * convergence test; the iteration count is kept. */
int cg_get_state(cg_game *game, double *V_dev, double *U_dev, int32_t *r);
int cg_set_state(cg_game *game, const double *V_dev, const double *U_dev);

/* Batched value iteration: many games, of uneven d, N and parameters,
 * advanced together.  Games with the same d, N, precision and control-fit
 * path form a group; one iteration of every group is a fixed sequence of
 * kernel launches, each covering all games of its group (blocks are mapped
 * to (game, player, node tile) through a device table).  One iteration of
 * all groups is captured once in a hipGraph, the groups spread over up to
 * four parallel branches (balanced by their contraction work) so that small
 * groups run beside large ones, and replayed per iteration.  Each game keeps
 * its own state, status and convergence test (Step 4): a converged game's
 * blocks return at once.
 *
 * cg_batch_create: 'games' (count >= 1 distinct, initialised handles; host
 * array, copied) must stay valid and must not be used on other streams while
 * the batch works; ws_dev (>= cg_batch_workspace_bytes(count), 256-byte
 * aligned, device) holds the device tables; work is queued on 'stream'.
 * cg_batch_autotune: for every group, times the contraction's tile shapes
 * (16, 32 or 64 nodes per wave; one or two values of the outer modes per
 * coefficient slab) over 'trial_steps' iterations and keeps the fastest;
 * then times 'trial_steps' replays of the captured iteration with 1 to 4
 * parallel branches and keeps the fastest (more branches only when 2 %
 * faster); it resets every game of the batch to V = 0, u = A.
 * Synchronises.
 * cg_batch_solve: like cg_solve for every game at once; steps_done and
 * residuals (host arrays of count entries, nullable) receive each game's
 * iteration count and last residual.  Synchronises.  Returns
 * CG_ENOTCONVERGED if tol > 0 and some game did not reach it, CG_ENONFINITE
 * if some game produced a non-finite value: that game stopped at that
 * iteration, its residuals entry is non-finite, and every other game ran on
 * unaffected (its entries are valid).
 * cg_batch_groups: number of groups and, for arrays that are not NULL (host,
 * CG_MAX_GROUPS entries each), the row blocks of 16 per wave (rb) and the
 * outer values per coefficient slab (ocb) chosen per group.
 * cg_batch_branches: number of parallel branches of the captured iteration
 * (1 to 4; builds the graph if there is none yet), or a negative error. */
#define CG_MAX_GROUPS 64
typedef struct cg_batch cg_batch;
size_t cg_batch_workspace_bytes(int32_t count);
int cg_batch_create(cg_game *const *games, int32_t count, void *ws_dev, size_t ws_bytes, void *stream,
                    cg_batch **out);
int cg_batch_autotune(cg_batch *batch, int32_t trial_steps);
int cg_batch_solve(cg_batch *batch, int32_t max_steps, double tol, int32_t *steps_done, double *residuals);
int cg_batch_groups(cg_batch *batch, int32_t *rb, int32_t *ocb);
int cg_batch_branches(cg_batch *batch);
int cg_batch_destroy(cg_batch *batch);

/* Learned warm start (an addition to the method: Section 2.2 leaves the
 * starting iterate V^[0] free; the network only chooses it, and the iteration
 * that follows is the plain method, which also decides the result).
 *
 * Network: 9 inputs (the six game parameters (A, beta, phi, c, kappa, rho) as
 * theta/nominal - 1, then the three normalised state coordinates x in
 * [-1,1]^3 of a node) -> 256 -> 256 -> 256 GELU units (gelu(z) = z Phi(z)) ->
 * 3 outputs (the players' values at the node, scaled).  binary32 throughout.
 * Parameters: one device array of cg_mlp_param_count() floats, per layer W
 * ([fan_in][fan_out], row-major) then b, layers in order.  Loss: mean over
 * samples and outputs of (y - t)^2.  Samples X are [n][9], outputs and
 * targets [n][3], device, binary32.
 *
 * Workspaces (device, 256-byte aligned, >= cg_mlp_workspace_bytes(batch)):
 * scratch of the calls below for minibatches of up to 'batch' rows (1 ..
 * 65536); 0 = batch out of range.  All calls queue work on 'stream' (the
 * game's stream for the game-level calls) and return at once unless stated.
 *
 * cg_mlp_forward: Y = net(X) for n rows, 'batch' rows at a time.
 * cg_mlp_grad: loss (device float, nullable) and gradient (device, same
 *   layout as the parameters) of one minibatch of n <= 65536 rows; ws must
 *   fit n rows.  Sums are taken in a fixed order: reruns are bitwise equal.
 * cg_mlp_adam: one Adam step t >= 1 (Kingma and Ba, bias-corrected) of the
 *   parameters with moment arrays m, v (device, parameter layout).
 * cg_mlp_train: 'steps' Adam steps t0+1 .. t0+steps at learning rate lr
 *   (beta1 0.9, beta2 0.999, eps 1e-8), each on 'batch' rows drawn with
 *   replacement from the n_samples rows of (X, T) by SplitMix64 of (seed,
 *   step, row); losses (device, 'steps' floats, nullable) gets each step's
 *   minibatch loss.
 * theta (game-level calls): host array of the six normalised parameters.
 * cg_mlp_features: writes the N^3 feature rows of a d = 3 game's nodes into X
 *   (node order of V) and, if T is not NULL, t_scale * V_i of the game's
 *   current state into T: training pairs from a solved game.
 * cg_warm_start: V^[0] = out_scale * net(features) at every node and u^[0]_i
 *   = clip(A_i + delta_h beta_i dV^[0]_i/dp_i, 0, U_M), the maximiser of
 *   Step 3's objective with V^[0] expanded to first order at the node.  If
 *   any value of V^[0] is non-finite the game is set to the zero start
 *   (V = 0, u = A) instead and *nonfinite (host, nullable) is 1.
 *   Synchronises.
 * cg_solve_warm: cg_solve to tol from the warm start, with the plain method as
 *   fallback: one iteration from the zero start gives the bar r0; after the
 *   warm start, probe_steps iterations must leave a finite residual <= r0, or
 *   the game restarts from zero and is solved plainly (*fell_back = 1).
 *   *steps_done counts every iteration spent (the bar, the probe, the rest).
 *   Synchronises; returns as cg_solve.
 * Calls other than cg_mlp_param_count and cg_mlp_workspace_bytes return
 * CG_EUNSUPPORTED for games with d != 3. */
#define CG_MLP_IN 9
#define CG_MLP_HIDDEN 256
#define CG_MLP_OUT 3
int64_t cg_mlp_param_count(void);
size_t cg_mlp_workspace_bytes(int32_t batch);
int cg_mlp_forward(const float *params, const float *X, int64_t n, float *Y, int32_t batch, void *ws,
                   size_t ws_bytes, void *stream);
int cg_mlp_grad(const float *params, const float *X, const float *T, int32_t n, float *grad, float *loss, void *ws,
                size_t ws_bytes, void *stream);
int cg_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t t, float lr, float beta1, float beta2,
                float eps, void *stream);
int cg_mlp_train(float *params, float *m, float *v, const float *X, const float *T, int64_t n_samples, int32_t batch,
                 int32_t steps, int32_t t0, float lr, uint64_t seed, float *losses, void *ws, size_t ws_bytes,
                 void *stream);
int cg_mlp_features(cg_game *game, const float *theta, double t_scale, float *X, float *T);
int cg_warm_start(cg_game *game, const float *params, const float *theta, double out_scale, void *ws,
                  size_t ws_bytes, int32_t batch, int32_t *nonfinite);
int cg_solve_warm(cg_game *game, const float *params, const float *theta, double out_scale, int32_t max_steps,
                  double tol, int32_t probe_steps, void *ws, size_t ws_bytes, int32_t batch, int32_t *steps_done,
                  double *residual, int32_t *fell_back);

/* Equilibrium time paths (the emission and pollution paths of Section 4):
 * for each of n_paths initial states (p0, device, [n_paths][d], physical
 * units) the state recursion p_{n+1} = p_n + h g(p_n, u*(p_n)) over n_steps,
 * with u*_i the Chebyshev interpolant (Section 3.1) of the game's current
 * nodal controls U_i at p, kept in [0, U_M]; points outside [0, P_M]^d use the
 * polynomial continuation.  paths (device, [n_paths][n_steps+1][d], row 0 =
 * p0) and controls (device, nullable, [n_paths][n_steps][d]).  Queued on the
 * game's stream; uses the game's transform buffer, so it must not overlap the
 * game's iterations (same stream: it does not). */
int cg_simulate(cg_game *game, const double *p0_dev, int32_t n_paths, int32_t n_steps, double *paths_dev,
                double *controls_dev);

/* Timing of the contraction kernel (the kernel that carries the mode-n
 * contractions).  With enable = k >= 1, every k-th later step (the first,
 * then every k-th) records a pair of HIP events on the game's stream around
 * that kernel's launch; enable = 0 stops timing.  If kernel_ms or launches
 * is not NULL the call first synchronises the stream and returns the summed
 * elapsed time and the number of timed launches since the previous
 * cg_profile call; the record is then cleared.  Costs one event pair per
 * timed step.  CG_EINVAL for enable < 0. */
int cg_profile(cg_game *game, int enable, double *kernel_ms, int64_t *launches);

/* Tile shapes of the game's contraction kernel: rb row blocks of 16 nodes per
 * wave (1, 2 or 4) and ocb values of the outer modes per coefficient slab
 * (1 or 2; 1 when d = 2).  Defaults: rb = 2 when the game has rows for
 * three waves per SIMD at that shape (d * N^d >= 98304), else 1 (always 1
 * for d = 4 and for CG_FP32_CORR outside the split bfloat16 form), ocb = 2
 * (d = 2: 1).  Results do not depend on rb;
 * ocb changes where the binary32 partial sums of CG_FP32_CORR enter FP64
 * (not in the split bfloat16 form, whose remainder enters FP64 once).
 * CG_EINVAL for other values. */
int cg_set_tiles(cg_game *game, int32_t rb, int32_t ocb);

/* ------------------------------------------------------------------------
 * General form (Section 2.1's algorithm for dynamics that are not separable
 * in the controls, with the node-wise control polynomials of Section 3.3 and
 * the offline Step 0 of Section 3.4).
 *
 * The game is given by samples instead of a formula:
 *   drift   g_k(p, u), k = 0..d-1   (dp/dt = g(p, u))
 *   payoff  G_i(p, u), i = 0..d-1
 * at every state node p_j of an anisotropic Lobatto grid (n_nodes[l] nodes
 * along state dimension l) and every control node u of the tensor grid of
 * control nodes (n_unodes[i] nodes for player i).  Step 0 interpolates them
 * in u (one control polynomial per node, component and payoff; Algorithm
 * Cnv).  Each iteration, for every player i and node p_j:
 *   Step 1  the control polynomials are evaluated along the line
 *           u -> [u, u^{[r]}_{-i}(p_j)] at player i's control nodes u_m;
 *   Step 2  V_i^{[r]} is evaluated at the update points p_j + h g(p_j, .)
 *           (a full d-dimensional evaluation per control node) and the
 *           samples h G_i + (1 - rho h) V_i^{[r]} are formed;
 *   Step 3  the samples are fitted in u (eq. (forcoef)) and the fit's
 *           maximiser over [0, u_max] is the new control;
 *   Step 4  the fit there is the new value; residual max |V^{[r+1]} - V^{[r]}|.
 * All players use u^{[r]} (simultaneous update).
 *
 * Grids: state node k of dimension l is p = p_max (x_k + 1) / 2 with
 * x_k = cos(pi k / (n_nodes[l] - 1)); control node m of player i is
 * u = u_max (cos(pi m / (n_unodes[i] - 1)) + 1) / 2 (index 0 = u_max).
 * N_P = prod n_nodes, U_P = prod n_unodes; node and control indices run in C
 * order over their grids (last dimension fastest).  State arrays are
 * [d][N_P].
 * ---------------------------------------------------------------------- */
#define CG_MAX_NU 16 /* control nodes per player in the general form */

typedef struct cg_general_desc {
    int32_t d;                      /* players = state dimension, 2..CG_MAX_D */
    int32_t n_nodes[CG_MAX_D];      /* state nodes per dimension, 3..CG_MAX_N */
    int32_t n_unodes[CG_MAX_D];     /* control nodes per player, 3..CG_MAX_NU */
    double h;                       /* time step, > 0 */
    double rho;                     /* discount rate; requires 0 < rho h < 1 */
    double p_max;                   /* state box [0, p_max]^d, > 0 */
    double u_max;                   /* control interval [0, u_max], > 0 */
    double u_init[CG_MAX_D];        /* u^{[0]} of each player, in [0, u_max] (V^{[0]} = 0) */
    const double *drift_dev;        /* device [d][N_P][U_P]: g_k(p_j, u_t) */
    const double *payoff_dev;       /* device [d][N_P][U_P]: G_i(p_j, u_t) */
} cg_general_desc;

typedef struct cg_general cg_general;

/* Grid coordinates of the description (host arrays): pnodes receives the
 * physical state nodes of dimension 0, then 1, ... (sum n_nodes doubles);
 * unodes the control nodes of player 0, 1, ... (sum n_unodes doubles).
 * Either may be NULL.  The drift and payoff samples are taken there.
 * Errors: CG_EINVAL, CG_EUNSUPPORTED (sizes outside the compiled set). */
int cg_general_nodes(const cg_general_desc *desc, double *pnodes, double *unodes);

/* Bytes of device workspace cg_general_init needs (0 if the description is
 * invalid; cg_last_error says why).  It holds the control-polynomial
 * coefficients (2 d N_P U_P doubles), the update points (d N_P sum n_unodes
 * x (d + 2) doubles) and the state. */
size_t cg_general_workspace_bytes(const cg_general_desc *desc);

/* Step 0: validates the description, interpolates the drift and payoff
 * samples into control polynomials (in the workspace), sets V^{[0]} = 0 and
 * u^{[0]} = u_init.  The work runs on 'stream' and the call synchronises it,
 * so drift_dev and payoff_dev may be released on return.  The workspace
 * (>= cg_general_workspace_bytes, 256-byte aligned) must outlive the handle;
 * later calls queue their work on the same stream.
 * Errors: CG_EINVAL, CG_EUNSUPPORTED, CG_ENOMEM, CG_EDEVICE. */
int cg_general_init(const cg_general_desc *desc, void *ws_dev, size_t ws_bytes, void *stream,
                    cg_general **out);

/* nsteps iterations (Steps 1-4 above).  If residual_out is not NULL the call
 * synchronises the stream and stores the last residual; CG_ENONFINITE if a
 * non-finite value appeared. */
int cg_general_step(cg_general *game, int32_t nsteps, double *residual_out);

/* Iterate until the residual is < tol (strict; tol <= 0: exactly max_steps
 * iterations) or max_steps; synchronises.  Returns CG_OK, CG_ENOTCONVERGED
 * or CG_ENONFINITE; *steps_done and *residual (nullable) as for cg_solve.
 * The host checks the device-side test every 8 iterations; the iterations
 * queued after convergence leave the state unchanged. */
int cg_general_solve(cg_general *game, int32_t max_steps, double tol, int32_t *steps_done, double *residual);

/* Copies of the current V and u ([d][N_P] each, device, nullable) and the
 * iterations done since init (host, nullable; synchronises).  set_state
 * replaces them (U_dev NULL keeps u).  Queued on the game's stream. */
int cg_general_get_state(cg_general *game, double *V_dev, double *U_dev, int32_t *r);
int cg_general_set_state(cg_general *game, const double *V_dev, const double *U_dev);

/* Per-phase timing with HIP events on the game's stream.  With enable != 0
 * every later iteration records events between its phases.  If phase_ms is
 * not NULL the call synchronises and stores the summed milliseconds since the
 * previous call of [0] the coefficient transform (and the packing of the
 * coefficients for the evaluation), [1] Step 1 (control polynomials and
 * update points), [2] Step 2 (the evaluation kernel of V, all players in one
 * launch) and [3] Steps 3-4 (fit, argmax, residual); *steps the iterations
 * timed. */
int cg_general_profile(cg_general *game, int enable, double *phase_ms, int64_t *steps);

/* Releases the handle (not the workspace).  NULL is accepted. */
int cg_general_destroy(cg_general *game);

#ifdef __cplusplus
}
#endif

#endif /* CHEBGAME_H */
