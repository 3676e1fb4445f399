/*
 * af.h -- C ABI of the MI355X (gfx950) implementation of the compact
 * fourth-order positivity-preserving Active Flux (AF) method for the 1D/2D
 * compressible Navier-Stokes equations on Cartesian meshes (Duan, Barsukow,
 * Klingenberg).
 *
 * Problem statement (Sec. 1 of the paper): conservative variables
 * U = (rho, rho u, E) (1D) or (rho, rho u, rho v, E) (2D), ideal gas
 * p = (gamma-1)(E - |rho u|^2/(2 rho)), Newtonian stress with constant
 * viscosity mu >= 0, Fourier heat flux with kappa = gamma mu/((gamma-1) Pr),
 * temperature T = p/rho.  mu = 0 gives the Euler equations.
 *
 * Degrees of freedom (Sec. 2.1, Sec. 2.2): cell averages and point values
 * shared by neighbouring cells.  A state is ONE contiguous FP64 device buffer:
 *   1D: [avg: 3 x n1][pts: 3 x n1x]
 *   2D: [avg: 4 x n2 x n1][xe: 4 x n2 x n1x][ye: 4 x n2y x n1][co: 4 x n2y x n1x]
 * component-major, x fastest; n1x = n1 if the x axis is periodic else n1+1
 * (n2y likewise).  Cell (i,j) spans [x0+i dx, x0+(i+1)dx] x [y0+j dy, ...];
 * xe(i,j) is the point (x0+i dx, y0+(j+1/2)dy), ye(i,j) is
 * (x0+(i+1/2)dx, y0+j dy), co(i,j) is (x0+i dx, y0+j dy); 1D point k is x0+k dx.
 *
 * Memory and streams: the library never allocates device memory.  The caller
 * allocates state and workspace buffers (sizes below) and passes a HIP
 * stream (hipStream_t as void*; NULL = the default stream).  All entry points
 * that take a stream enqueue work on it; only the ones documented as
 * synchronous wait for it.  All pointers to state/workspace are device
 * pointers (8-byte aligned at least, 256-byte recommended).
 *
 * Errors: every call returns af_status; AF_OK = 0.  Nothing aborts; a
 * human-readable message for the last error of the calling thread is
 * available from af_last_error().
 */
#ifndef AF_H
#define AF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AF_OK = 0,
  AF_E_ARG = 1,       /* invalid argument (message says which)              */
  AF_E_HIP = 2,       /* a HIP runtime call failed                           */
  AF_E_PP = 3,        /* step halving exhausted: low-order states inadmissible */
  AF_E_NONFINITE = 4  /* a non-finite value appeared in the solution          */
} af_status;

/* boundary kinds (Sec. 4 names periodic, outflow, no-slip adiabatic wall and
 * symmetry boundaries; ghost values are images of interior lattice sites:
 * wrap, zero-order copy, or a mirror about the wall line with the normal
 * momentum (symmetry) or both momenta (no-slip) negated; point values on a
 * wall are projected after every stage onto zero normal (symmetry) or zero
 * (no-slip) momentum at unchanged density and internal energy).
 * AF_DIRICHLET (1D only; the paper prescribes boundary values in its 1D
 * viscous-shock test, Sec. 4): the ghost cells and lattice sites hold the
 * side's state (af_set_bc_state) and the boundary point value is set to it
 * after every stage. */
typedef enum {
  AF_PERIODIC = 0, AF_OUTFLOW = 1, AF_NOSLIP = 2, AF_SYMMETRY = 3, AF_DIRICHLET = 4
} af_bc;
typedef enum { AF_XLO = 0, AF_XHI = 1, AF_YLO = 2, AF_YHI = 3 } af_side;

/* limiter switches (Sec. 3.2-3.4) */
enum {
  AF_LIM_SMOOTH = 1, /* smoothness-indicator blend theta^s of the cell fluxes    */
  AF_LIM_PP = 2,     /* density/pressure blend theta^rho theta^p of cell fluxes  */
  AF_LIM_POINT = 4,  /* scaling limiter of point values toward the point LLF     */
  AF_LIM_CENTRE = 8, /* scaling of Simpson centre values toward the cell average */
  AF_LIM_ALL = 15,
  /* diagnostic: the low-order schemes alone (blend parameters 0): LLF cell
     fluxes (Sec. 3.1) and, together with AF_LIM_POINT, the low-order point
     values (Sec. 3.4) */
  AF_LIM_LOWONLY = 16,
  /* 2D: the learned blend.  The smoothness blend theta^s of the cell fluxes
     (Sec. 3.2) is replaced by a small network's proposal theta_nn per face,
     computed from the stage input's cell averages (af_blend_infer, with the
     network set by af_set_blend_net).  The density/pressure blend then acts
     on the candidate F^L + theta_nn (F^H - F^L) exactly as it acts on the
     smoothness-blended one: F = F^L + theta_nn theta^rho theta^p (F^H - F^L)
     with AF_LIM_PP, so the coefficient never exceeds theta_nn nor the
     admissible bound (Sec. 3.3), and positivity and conservation are as in
     the plain method; theta_nn = theta^s gives the plain stage.
     AF_LIM_SMOOTH is ignored. */
  AF_LIM_LEARNED = 32,
  /* the pressure factor theta^p of every density-then-pressure blend (cell
     fluxes, point values, centres; Sec. 3.3) solved exactly: the largest
     blend keeping p >= eps along the whole segment, the root of the
     quadratic that p(blend) = eps becomes once multiplied by the blended
     density, in place of the linear bound that the concavity of p gives;
     0 where the low-order state's pressure is at the 1e-13 floor, as with
     the linear rule.  Never below the linear one.  1D and 2D, both
     precisions (computed in FP64).  Blends then sit at p = eps, and on
     strong shock tubes steps are rejected far more often than with the
     linear rule. */
  AF_LIM_PEXACT = 64
};

/* sticky status flags accumulated in the workspace by af_rk_stage */
enum {
  AF_FLAG_CELL_LOW = 1,  /* a low-order intermediate cell state left the admissible set */
  AF_FLAG_POINT_LOW = 2, /* a low-order point state left the admissible set           */
  AF_FLAG_NONFINITE = 4  /* a non-finite value was written                             */
};

typedef struct af_params {
  int dim;              /* 1 or 2                                                 */
  int n1, n2;           /* cells along x (>= 4) and y (>= 4; ignored in 1D)       */
  double x0, x1, y0, y1;/* box; x1 > x0, y1 > y0                                  */
  double gamma;         /* ratio of specific heats, > 1                           */
  double mu;            /* dynamic viscosity, >= 0                                */
  double Pr;            /* Prandtl number, > 0                                    */
  double cfl_c, cfl_v;  /* C^c and C^v of the CFL condition (eq. cfl), > 0.  Under
                           SSP-RK3 the scheme's linearisation about a uniform
                           state is stable for viscous numbers (dt max(4mu/3rho,
                           gamma mu/(Pr rho))/dx^2) up to about 0.157 in 1D and
                           0.061 in 2D, so cfl_v <= 0.15 (1D) and <= 0.06 (2D)  */
  double Cs;            /* smoothness-limiter strength (paper: 1), >= 0           */
  int limiter;          /* AF_LIM_* bits                                          */
  int max_halvings;     /* retries of a step with halved dt (>= 0)               */
  int precision;        /* AF_PREC_FP64, or AF_PREC_MIXED (2D only)               */
  int rk;               /* time integrator of af_step / af_run: 3 (SSP-RK3) or 54
                           (SSP-RK54, the five-stage fourth-order SSP method of
                           Sec. 2.3; the paper pairs it with cfl_c = 1.04/d and
                           cfl_v = 0.33/d, which the 2D scheme's linearisation
                           exceeds when viscosity dominates: its viscous limit
                           under SSP-RK54 is about 0.13 in 2D)                   */
} af_params;

/* arithmetic of the 2D stage.  AF_PREC_MIXED: the stencils, fluxes and
 * residuals run in FP32; the density/pressure blends (Theta rule, Sec. 3.3
 * and 3.4), the cell-average update and the point-value update run in FP64
 * on FP64 data.  The state stays FP64 in both; results differ from the FP64
 * stage by the FP32 rounding of the fluxes and residuals. */
enum { AF_PREC_FP64 = 0, AF_PREC_MIXED = 1 };

typedef struct af_ctx af_ctx;

/* Fill p with defaults: 2D 64x64 on [0,1]^2, gamma 1.4, mu 1e-3, Pr 0.72,
 * cfl_c 0.2, cfl_v 0.05, Cs 1, all limiters, max_halvings 40, FP64,
 * SSP-RK3. */
af_status af_default_params(af_params* p);

/* Validate p and create a context (host memory only; no device work).
 * All boundaries default to AF_OUTFLOW.  Free with af_destroy. */
af_status af_init_grid(const af_params* p, af_ctx** out);
void af_destroy(af_ctx* ctx);

/* Set the boundary kind of one side.  A periodic axis must be periodic on
 * both sides before any compute call (checked there: AF_E_ARG). */
af_status af_set_bc(af_ctx* ctx, int side, int kind);
/* The state of a Dirichlet side (1D, side AF_XLO or AF_XHI): state[3] =
 * (rho, rho u, E) on the host, copied.  Defaults to (1, 0, 1). */
af_status af_set_bc_state(af_ctx* ctx, int side, const double* state);

/* Number of doubles in one state buffer, its size in bytes, and the bytes of
 * the workspace (0 for a NULL or inconsistent context). */
size_t af_state_len(const af_ctx* ctx);
size_t af_state_bytes(const af_ctx* ctx);
size_t af_workspace_bytes(const af_ctx* ctx);

/* Copy a whole state between a host buffer (af_state_len doubles, in the
 * layout above) and a device state buffer, on `stream`; synchronous (the
 * call returns when the copy is done).  AF_E_ARG for NULL pointers. */
af_status af_set_state(af_ctx* ctx, double* U_dev, const double* U_host, void* stream);
af_status af_get_state(af_ctx* ctx, const double* U_dev, double* U_host, void* stream);

/* Number of DOF sites (cell averages and point values) of the device state
 * U whose density or pressure p = (gamma-1)(E - |rho u|^2/(2 rho)) is not
 * positive, NaN included: the admissible set of Sec. 3 (synchronous; uses
 * the workspace).  *count receives the number. */
af_status af_check_admissible(af_ctx* ctx, const double* U, void* ws, void* stream,
                              long* count);

/* One SSP-RK3 stage (Shu-Osher form), asynchronous on `stream`:
 *   Uout = a_k Un + b_k FE(Uk, dt),  (a,b) = (0,1), (3/4,1/4), (1/3,2/3)
 * for k = 0, 1, 2, where FE is the limited forward-Euler update of cell
 * averages (eq. of the limited cell update, Sec. 3.3) and point values
 * (Sec. 2 point update with the Sec. 3.4 scaling limiter).  dt is read from
 * the device scalar dt_dev if it is not NULL, else dt_host is used.  Un may
 * be NULL for k = 0.  Uout must not alias Un or Uk.  Flags (AF_FLAG_*) are
 * OR-ed into the workspace; see af_read_flags / af_reset_flags. */
af_status af_rk_stage(af_ctx* ctx, int k, const double* dt_dev, double dt_host,
                      const double* Un, const double* Uk, double* Uout, void* ws,
                      void* stream);

/* CFL time step (eq. cfl) from the cell averages of U, clipped to
 * t_final - t and written to the device scalar *dt_dev; asynchronous. */
af_status af_cfl_dt(af_ctx* ctx, const double* U, double t, double t_final, double* dt_dev,
                    void* ws, void* stream);

/* One full step of U in place (SSP-RK3, or SSP-RK54 when params.rk is 54:
 * five forward-Euler stages with their own fractions of dt and two state
 * combinations), synchronous.  dt <= 0 selects the CFL
 * step.  dt is clipped to t_final - t.  If any flag is raised the state is
 * restored and the step recomputed with dt/2, up to max_halvings times
 * (Remark on the time step, Sec. 3.4): then AF_E_PP (or AF_E_NONFINITE) is
 * returned and U holds the state before the step.  *dt_used and *halvings
 * (either may be NULL) receive the step actually taken. */
af_status af_step(af_ctx* ctx, double* U, void* ws, void* stream, double dt, double t,
                  double t_final, double* dt_used, int* halvings);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): af_step with its
 * workspace taken from a fixed array inside the library instead of a caller
 * buffer.  The array holds AF_NOALLOC_SCRATCH_BYTES bytes on every GPU the
 * library runs on, for the life of the process.  A grid whose
 * af_workspace_bytes exceeds it is rejected with AF_E_ARG before any device
 * work (the FP64 2D workspace is about 512 bytes per cell: up to about
 * 32,000 cells, e.g. 256 x 128).  All calls on one GPU share its array, and
 * each call leaves its contents behind: calls that overlap on one GPU
 * (from several host threads or on several streams) race, so the caller
 * serialises them.  Arguments, synchronisation, halving and results are as
 * in af_step; the call allocates nothing. */
#define AF_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
af_status af_step_noalloc(af_ctx* ctx, double* U, void* stream, double dt, double t,
                          double t_final, double* dt_used, int* halvings);

/* Steps with a source term (manufactured solutions: the paper's Taylor-Green
 * test, Sec. 4, adds an energy source).  af_stage_times writes the times of
 * the stage inputs of integrator rk (3 or 54) as fractions of dt into c
 * (3 or 5 values) and returns their number (-1 for another rk).
 * af_step_source takes one step of dU/dt = L(U) + S(t) with the given dt
 * (no CFL, no halving): every forward-Euler step of the integrator is the
 * limited update of L followed by + tau S_k, where src[k] is a device state
 * (same layout as U) holding S at the k-th stage input's time.  nsrc must
 * be 3 (SSP-RK3) or 5 (SSP-RK54).  Synchronous.  If a flag is raised the
 * state is restored and AF_E_PP (or AF_E_NONFINITE) returned. */
int af_stage_times(int rk, double* c);
af_status af_step_source(af_ctx* ctx, double* U, void* ws, void* stream, double dt,
                         const double* const* src, int nsrc);

/* Advance U from t0 until t_final or max_steps steps.  Steps run with the
 * time step kept on the device; every check_every steps (>= 1) the stream is
 * synchronised and the flags read; a block whose flags are raised is redone
 * from its saved start with af_step semantics (halving).  *nsteps_out and
 * *t_out (may be NULL) receive the steps taken and the final time. */
af_status af_run(af_ctx* ctx, double* U, void* ws, void* stream, double t0, double t_final,
                 long max_steps, int check_every, long* nsteps_out, double* t_out);

/* af_run with every step decision on the device (2D, SSP-RK3, without the
 * learned blend): a round opens a step with the CFL dt of eq. (cfl) when the
 * previous one was accepted (clipped to t_final - t), runs one RK3 attempt,
 * and accepts it or redoes it with dt/2 in the next round (the remark on the
 * time step at the end of Sec. 3.4), up to max_halvings times.  Rounds are
 * enqueued in slots of attempts_per_slot (>= 1), captured once in a HIP graph
 * and replayed on `stream`; the host synchronises only once per four slots,
 * to stop (rounds after the last step do nothing).  The state rotates through U and the workspace's two stage buffers
 * and ends in U.  Results equal af_run's bit for bit.  Synchronous.
 * *nsteps_out, *t_out and *attempts_out (RK3 attempts, accepted and rejected;
 * any may be NULL) receive the counts and the final time; AF_E_PP or
 * AF_E_NONFINITE as in af_run, U then holding the state before the failed
 * step. */
af_status af_run_graph(af_ctx* ctx, double* U, void* ws, void* stream, double t0,
                       double t_final, long max_steps, int attempts_per_slot, long* nsteps_out,
                       double* t_out, long* attempts_out);

/* Flags accumulated in the workspace (synchronous read), and their reset
 * (asynchronous). */
af_status af_read_flags(af_ctx* ctx, const void* ws, int* flags, void* stream);
af_status af_reset_flags(af_ctx* ctx, void* ws, void* stream);

/* Kernel timing (diagnostics for the benchmark).  While enabled, every kernel
 * the library launches for this context is bracketed by HIP events on its
 * stream.  af_timing_read waits for the recorded events and returns, for
 * each kernel kind below, the number of launches and their summed duration
 * in milliseconds since the previous read (arrays of AF_K_COUNT entries). */
enum {
  AF_K_LATTICE = 0,  /* 1D: half-lattice values, centres, auxiliaries */
  AF_K_GRAD = 1,     /* 1D: lattice gradients                          */
  AF_K_CELLPRE = 2,  /* 1D: per-cell low-order data                    */
  AF_K_FACE = 3,     /* 1D: limited face fluxes                         */
  AF_K_CELLS = 4,    /* 1D: cell-average update                         */
  AF_K_POINTS = 5,   /* 1D: point-value update                          */
  AF_K_CFL = 6,      /* time-step reduction                             */
  AF_K_STAGE2D = 7,  /* 2D: the fused stage kernel                      */
  AF_K_BLEND = 8,    /* 2D: the learned blend's features and network   */
  AF_K_COUNT = 9
};
af_status af_timing(af_ctx* ctx, int enable);
af_status af_timing_read(af_ctx* ctx, long* launches, double* ms);

/* ---- batches: many independent 2D instances advanced together ----
 *
 * A batch groups n contexts (2D, one precision; each with its own grid, gas,
 * boundaries and switches).  Every stage of every instance of a step attempt
 * is ONE persistent kernel launch over the tiles of all instances.  Each
 * instance keeps its own CFL time step (eq. cfl) and its own halving (the
 * remark on the time step at the end of Sec. 3.4), decided on the device
 * after each attempt, so no host round trip separates the attempts.  The
 * contexts must outlive the batch; 1 <= n <= 512. */
typedef struct af_batch af_batch;
af_status af_batch_create(af_ctx* const* ctxs, int n, af_batch** out);
void af_batch_destroy(af_batch* b);
/* Workspace of a batch run (descriptors and two stage buffers per instance). */
size_t af_batch_workspace_bytes(const af_batch* b);
/* Advance the device states U[i] (af_state_len doubles of ctxs[i] each) from
 * t0 until t_final or max_steps accepted steps per instance; synchronous.
 * Work is enqueued in slots of attempts_per_slot (>= 1) rounds: a round
 * opens a step (fresh CFL dt) for every instance that is between steps and
 * runs one RK3 attempt of every instance inside a step; the attempt is then
 * accepted or redone with dt/2 in the next round (af_run's halving rule).
 * use_graph != 0 captures one slot in a HIP graph and replays it.  steps[i], t[i], status[i] (AF_OK, AF_E_PP, AF_E_NONFINITE: the state
 * is then the one before the failed step) and attempts[i] (RK3 attempts,
 * accepted and rejected) receive per-instance results; any may be NULL. */
af_status af_batch_run(af_batch* b, double* const* U, void* ws, void* stream, double t0,
                       double t_final, long max_steps, int attempts_per_slot, int use_graph,
                       long* steps, double* t, int* status, long* attempts);

/* Compiled variants of the 2D stage kernel.  Each is the same arithmetic
 * (results are identical to the last bit) over a different tile shape:
 * tiles are 16 cells wide and tile_height cells high, and the taller the
 * tile the fewer halo sites are recomputed but the more LDS a workgroup
 * takes, so fewer workgroups are resident per CU.  The first variant of
 * each precision is the one af_rk_stage, af_step, af_run and new batches
 * use. */
int af_stage_variant_count(void);
/* name (static storage), precision (AF_PREC_*) and tile height of variant
 * i in [0, af_stage_variant_count()); any output may be NULL. */
af_status af_stage_variant_info(int i, const char** name, int* precision, int* tile_height);
/* Index of the variant the batch's stage launches use. */
int af_batch_variant(const af_batch* b);
/* Use variant i for the batch; it must have the batch's precision. */
af_status af_batch_set_variant(af_batch* b, int i);
/* Autotuner: for every variant of the batch's precision, time one step slot
 * (CFL step opening, one RK3 attempt of every instance from the states U at
 * time t0, and the accept/halve decision) reps times after one untimed slot,
 * and keep the fastest variant for the batch's later runs.  Synchronous; U
 * is read, never written (ws must be the batch's workspace).  us_per_slot,
 * if not NULL, receives af_stage_variant_count() entries: the fastest time
 * of each variant in microseconds, -1 for variants of the other precision. */
af_status af_batch_tune(af_batch* b, double* const* U, void* ws, void* stream, double t0,
                        double t_final, int reps, double* us_per_slot);

/* ---- the learned blend coefficient (2D; AF_LIM_LEARNED) ----
 *
 * Faces are numbered x-faces first, [n2][n1+1] (face (i, j) at x = x0 +
 * i dx between cells i-1 and i of row j), then y-faces, [n2+1][n1].  On a
 * periodic axis the last face of a line is the first one again: stages read
 * the first one's entry.
 *
 * The network is 40 -> 64 -> 64 -> 1 with tanh hidden units:
 * h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), z = w3.h2 + b3,
 * theta_nn = min(max(z, 0), 1).  Its parameters are one device array of
 * af_mlp_param_count() floats: [W1 (64 x 40, row-major W1[o][i]), b1 (64),
 * W2 (64 x 64), b2 (64), w3 (64), b3].  Inference stores W1, W2, w3 and the
 * layer inputs in bfloat16 and accumulates in FP32 on the matrix cores.
 *
 * Features of a face (40 floats), in the face's frame (normal n along its
 * axis, tangent t along the other): the 4 x 3 block of cell averages at
 * normal offsets -2, -1, +1, +2 (cells -1 and +1 adjoin the face) and
 * tangential offsets -1, 0, +1, ghost cells being the stage's boundary
 * images.  With rho_f, p_f, u_nf, u_tf the means over the two adjoining
 * cells and c_f = sqrt(gamma p_f / rho_f): for s = -1, 0, +1 and
 * m = -2, -1, +1, +2 the triple ln(p/p_f), (u_n - u_nf)/c_f,
 * (u_t - u_tf)/c_f; then ln(rho/rho_f) for m = -2, -1, +1, +2 at s = 0. */
long af_face_count(const af_ctx* ctx);
size_t af_mlp_param_count(void);

/* Features of every face of the device state U into feat (af_face_count x
 * 40 floats, device), asynchronous. */
af_status af_blend_features(af_ctx* ctx, const double* U, float* feat, void* stream);

/* The network of the learned blend: a device array of af_mlp_param_count()
 * floats owned by the caller, read at every later inference (it must stay
 * valid while the context uses AF_LIM_LEARNED); NULL clears it. */
af_status af_set_blend_net(af_ctx* ctx, const float* params);

/* theta_nn of every face of U into theta (af_face_count floats, device),
 * asynchronous; uses the workspace for the packed weights. */
af_status af_blend_infer(af_ctx* ctx, const double* U, float* theta, void* ws, void* stream);

/* af_rk_stage (2D) with explicit blend arrays: theta (af_face_count floats,
 * values in [0, 1]) takes the place of theta^s as under AF_LIM_LEARNED, or
 * NULL for the context's own rule; theta_s_out, if not NULL, receives the
 * coefficient that took theta^s's place at every face: theta^s itself for
 * a plain stage (the training targets of the learned blend), theta where it
 * is given, 1 with the smoothness blend off, 0 under AF_LIM_LOWONLY. */
af_status af_rk_stage_blend(af_ctx* ctx, int k, const double* dt_dev, double dt_host,
                            const double* Un, const double* Uk, double* Uout,
                            const float* theta, float* theta_s_out, void* ws, void* stream);

/* Training.  af_mlp_grad: mean of (z - y)^2 over the n rows of X (n x 40
 * floats) and targets y, its gradient (af_mlp_param_count floats) and the
 * loss (one float; may be NULL), all device arrays, asynchronous, FP32 and
 * deterministic; gws is a device scratch array of
 * af_mlp_grad_workspace_bytes(n) bytes.  af_mlp_adam: one Adam update
 * (beta1 0.9, beta2 0.999, eps 1e-8, step counted from 1) of params with
 * moment arrays m and v.  af_mlp_train: `steps` minibatches of `batch` rows
 * taken in order (wrapping around the n rows), gradient and Adam each,
 * steps counted from step0 + 1; *loss_out (device, may be NULL) receives the
 * last minibatch's loss. */
size_t af_mlp_grad_workspace_bytes(long n);
af_status af_mlp_grad(const float* X, const float* y, long n, const float* params, float* grad,
                      float* loss, void* gws, void* stream);
af_status af_mlp_adam(float* params, const float* grad, float* m, float* v, long step, float lr,
                      void* stream);
af_status af_mlp_train(const float* X, const float* y, long n, float* params, float* grad,
                       float* m, float* v, long step0, int steps, int batch, float lr,
                       float* loss_out, void* gws, void* stream);

/* Message of the last error raised on the calling thread ("" if none). */
const char* af_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
