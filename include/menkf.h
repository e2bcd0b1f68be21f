/*
 * menkf.h - C ABI of the MI355X (gfx950) multigrid ensemble Kalman filter
 * (MEnKF) hot path.
 *
 * The calls follow the paper's statement of the problem and its MEnKF
 * algorithm (Moldovan, Lehnasch, Cordier & Meldi, "A multigrid/ensemble
 * Kalman filter strategy for assimilation of unsteady flows", J. Comput.
 * Phys., arXiv 2012.10091):
 *   model        x_k = M(x_{k-1}) (+ eta)                   Sec. 2.1.1, state-evolution equation
 *   observation  y^o = H(x_k) + eps,  eps ~ N(0, R)        Sec. 2.1.1, observation equation
 *   one cycle    Algo. 4 steps 2-6 with the state part of Algo. 3
 *       menkf_forecast(FINE)      Algo. 4 step 2   fine forecast x^F_f
 *       menkf_forecast(COARSE)    Algo. 3 step 2   ensemble forecast on the coarse grid
 *       menkf_restrict            Algo. 4 step 4   x* = Pi_C(x^F_f)
 *       menkf_gain                Algo. 3 steps 3,4,7,8 (gain) and Algo. 4 step 5 (gain of x*)
 *       menkf_update              Algo. 3 step 8 (member update) and Algo. 4 step 5 (delta^C)
 *       menkf_prolong_smooth      Algo. 4 steps 5-6: x' = x^F_f + Pi_F(delta^C), relaxed iteration
 *   dual estimation of inlet parameters (Sec. 2.1.3, Algo. 2), inlet-forced models only
 *       menkf_forecast_inlet, menkf_param_perturb, menkf_param_update, menkf_dual_cycle
 *
 * Conventions shared by every call
 *   - Every pointer argument named *_dev is DEVICE memory on the context's
 *     device, owned by the caller; the library never frees or retains it
 *     beyond the call, except the probe tables (menkf_set_probes) and the
 *     workspace (menkf_set_workspace), which must stay valid while the
 *     context uses them.
 *   - State arrays hold float (MENKF_F32 contexts) or double (MENKF_F64
 *     contexts), passed as void*.  Layout: [nb][F][ny][nx], x fastest,
 *     members outermost; F = 1 (Burgers, ny = 1), 3 (1D Euler: rho, rho u,
 *     rho E; ny = 1) or 4 (rho, rho u, rho v, E).
 *   - Calls are asynchronous on the given stream (NULL = default stream),
 *     allocate nothing, never synchronise and never read device results
 *     on the host, so a sequence of them can be captured in a HIP graph.
 *     The only exceptions are menkf_get_status (synchronises the stream)
 *     and the menkf_graph_* helpers.
 *   - Argument and shape errors are detected on the host before any launch
 *     and returned as negative codes; menkf_last_error gives the text.
 *     Failures found on the device (a non-positive Cholesky pivot) are
 *     written to a device status word read by menkf_get_status; the calls
 *     that follow (menkf_update, menkf_prolong_smooth) test it on the
 *     device and leave their outputs untouched when it is set.
 */
#ifndef MENKF_H
#define MENKF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct menkf_ctx menkf_ctx;
typedef struct menkf_graph menkf_graph;
typedef void *menkf_stream; /* a hipStream_t */

typedef enum {
    MENKF_OK = 0,
    MENKF_E_ARG = -1,         /* bad argument (null pointer, bad enum, bad count) */
    MENKF_E_SHAPE = -2,       /* sizes inconsistent with the configuration */
    MENKF_E_NOT_SPD = -3,     /* innovation covariance not positive definite (device) */
    MENKF_E_NONFINITE = -4,   /* NaN/Inf found by a diagnostic */
    MENKF_E_HIP = -5,         /* a HIP runtime call failed */
    MENKF_E_UNSUPPORTED = -6, /* valid request outside what this build implements */
    MENKF_E_WORKSPACE = -7    /* workspace missing or too small */
} menkf_status;

enum { MENKF_BURGERS1D = 1, MENKF_NS2D = 2, MENKF_BURGERS1D_INLET = 3, MENKF_EULER1D_INLET = 4 };   /* model */
enum { MENKF_F32 = 0, MENKF_F64 = 1 };                 /* precision */
enum { MENKF_GAIN_EXACT_R = 0, MENKF_GAIN_SAMPLE_EE = 1, MENKF_GAIN_ENSEMBLE_SPACE = 2 };
enum { MENKF_FINE = 0, MENKF_COARSE = 1 };             /* grid level */
enum { MENKF_PROLONG_PLAIN = 0, MENKF_PROLONG_LEARNED = 1, MENKF_PROLONG_LEARNED_FALLBACK = 2 };
enum { MENKF_TIME_SSPRK3 = 0, MENKF_TIME_FIRST_ORDER = 1 };   /* time scheme (inlet-forced Burgers) */

/*
 * Configuration of one assimilation instance.
 *   model      MENKF_BURGERS1D: u_t + u u_x = nu u_xx (Sec. 4, Burgers equation),
 *              second-order centred differences, three-stage SSP Runge-Kutta.
 *              MENKF_NS2D: compressible Navier-Stokes in conservative form
 *              (Sec. 6, mass/momentum/energy equations), fourth-order centred
 *              differences, classical four-stage Runge-Kutta.
 *              Both periodic on [0, length)^dim.
 *              MENKF_BURGERS1D_INLET: the Burgers equation on the open
 *              interval of the inlet case of Sec. 4: nodes x_i = i length/nx,
 *              Dirichlet inlet u(0, t) = u0 (1 + theta_1 sin(omega t + theta_2))
 *              with per-state parameters theta (menkf_forecast_inlet),
 *              imposed at every Runge-Kutta stage time, outlet node the
 *              linear extrapolation 2 u_{n-2} - u_{n-3}.  Pi_F uses one-sided
 *              cubic stencils at both ends (coarse nodes b..b+3,
 *              b = clamp(j - 1, 0, n_c - 4) for the fine nodes of coarse
 *              cell j); Pi_C is injection; the fine correction and the
 *              relaxed sweeps leave the inlet node to the boundary
 *              condition.  A state row lives in LDS during a forecast, so
 *              nx <= 5290 (F64) or 8192 (F32).
 *              MENKF_EULER1D_INLET: the inviscid 1D Euler equations of the
 *              acoustic case of Sec. 5 in conservative variables (rho,
 *              rho u, rho E; F = 3) on the same open grid, in
 *              characteristic units (u0 + a = 1, rho0 = 1, so a = 1/(1+mach),
 *              u0 = mach a, p0 = a^2/gamma; the u0 field is not used):
 *              centred second-order flux differences, forward Euler in time
 *              (a single matrix-splitting iteration from x_{k-1} is that
 *              step, the centred inviscid operator having no diagonal),
 *              then the centred explicit filter x + (-1)^(p+1) filter_sigma
 *              delta^(2p) x / 4^p of order 2p = 6 on nodes 3..n-4, 4 on
 *              nodes 2 and n-3, 2 on nodes 1 and n-2.  Inlet node (rho0,
 *              rho0 u0 (1 + theta_1 sin(omega t + theta_2)), rho0 E0) at the
 *              end of every step, outlet node extrapolated linearly after
 *              the filter.  Observations read rho u (component 0 = rho u);
 *              the relaxed sweeps use the diagonal 1.  nx <= 1792 (F64) or
 *              3612 (F32), coarse grid >= 8 nodes.
 *   precision  MENKF_F32: float states and stencils, BF16 member-update
 *              products with FP32 accumulation, FP64 innovation covariance
 *              (S = Y Y^T + R), Cholesky and gain of x*.
 *              MENKF_F64: everything in double.
 *   gain_mode  MENKF_GAIN_EXACT_R: S = Y Y^T + obs_sigma^2 I.
 *              MENKF_GAIN_SAMPLE_EE: S = Y Y^T + E E^T (Algo. 1 step 6 as
 *              printed; singular when n_probes > 2 n_members - 2).
 *              MENKF_GAIN_ENSEMBLE_SPACE: the same gain as EXACT_R through
 *              the identity Y^T (Y Y^T + s^2 I)^-1 = (s^2 I + Y^T Y)^-1 Y^T
 *              (s = obs_sigma): Z = (s^2 I + Y^T Y)^-1 Y^T [D | d*], an
 *              N_e x N_e FP64 Cholesky instead of the N_y x N_y one.
 *   nx, ny     fine grid points (ny = 1 for the 1D model); ratio = coarsening
 *              ratio r_C per direction, must divide nx (and ny in 2D).
 *   n_members  ensemble size 2 <= N_e <= 256 (anomalies scaled by 1/sqrt(N_e - 1)).
 *   n_probes   number of scalar observations N_y >= 1.
 *   dt         time step of both levels; nu Burgers viscosity; gamma, mach,
 *              reynolds, prandtl the non-dimensional gas constants
 *              (rho0 = U0 = T0 = 1, mu = 1/Re, p = (gamma-1)(E - rho|u|^2/2)).
 *   obs_sigma  observation noise standard deviation (R = obs_sigma^2 I).
 *   anomaly_terms  MENKF_F32 member update X Z on BF16 MFMA: 1 = plain BF16
 *              operands; 3 (or 0 = default) = each operand split into a BF16
 *              pair hi + lo, product hi*hi + hi*lo + lo*hi (FP32-level accuracy).
 */
typedef struct {
    int32_t model, precision, gain_mode;
    int32_t nx, ny, ratio;
    int32_t n_members, n_probes;
    double length, dt, nu;
    double gamma, mach, reynolds, prandtl;
    double obs_sigma;
    int32_t anomaly_terms;
    /* MENKF_BURGERS1D_INLET only: inlet mean velocity and angular
     * frequency, and the standard deviations of the random walk
     * theta^f = theta + tau, tau ~ N(0, diag(theta_sigma^2)), of the dual
     * filter's parameter forecast (Algo. 2 step 1). */
    double u0, omega;
    double theta_sigma[2];
    /* MENKF_EULER1D_INLET only: strength of the explicit filter, in [0, 1]. */
    double filter_sigma;
    /* MENKF_BURGERS1D_INLET: MENKF_TIME_SSPRK3 (0, the default: three-stage
     * SSP Runge-Kutta) or MENKF_TIME_FIRST_ORDER, the paper's first-order
     * scheme (Sec. 4; implementation notes after Algo. 4): forward-Euler
     * steps, and the last step of every forecast call (the analysis step)
     * as a single Jacobi iteration of the implicit-Euler system
     * x_k - dt L(x_k) = x_{k-1} started from x_{k-1}, the convective
     * coefficient frozen there: x_k = x_{k-1} + dt / D L(x_{k-1}),
     * D = 1 + 2 nu dt / h^2 (centred convection has a zero diagonal).  The
     * inlet value is imposed at t_k and the outlet extrapolated after
     * every step.  Other models take 0 only. */
    int32_t time_scheme;
} menkf_config;

/* Create / destroy a context for the current HIP device.  The context owns
 * only host-side metadata; on failure *out is NULL and the status says why
 * (menkf_last_error(NULL) gives the text). */
menkf_status menkf_create(const menkf_config *cfg, menkf_ctx **out);
void menkf_destroy(menkf_ctx *ctx);
const char *menkf_last_error(const menkf_ctx *ctx);

/* Bytes of device workspace the context needs (no GPU call made). */
menkf_status menkf_workspace_size(const menkf_ctx *ctx, size_t *bytes);
/* Attach caller-owned device workspace of at least menkf_workspace_size
 * bytes, 256-byte aligned.  Its contents are the library's between calls. */
menkf_status menkf_set_workspace(menkf_ctx *ctx, void *ws_dev, size_t bytes);

/* Observation probes (observation equation of Sec. 2.1.1): probe p
 * observes the fine node idx_dev[p] (linear index y*nx + x) and component
 * comp_dev[p] (0: u = (rho u)/rho in 2D or u in 1D; 1: v = (rho v)/rho).
 * On the coarse level the operator is H^C = H^F o Pi_F at the probe node.
 * Device arrays of n_probes int32, kept by reference.  A set-up call: it
 * copies the tables to the host once (synchronously) and rejects nodes
 * outside the fine grid or components other than 0 (1D) / 0, 1 (2D). */
menkf_status menkf_set_probes(menkf_ctx *ctx, const int32_t *idx_dev, const int32_t *comp_dev);
/* The same call under the name of the observation-setting step: identical
 * arguments, contract and errors. */
menkf_status menkf_set_observations(menkf_ctx *ctx, const int32_t *idx_dev, const int32_t *comp_dev);

/* Explicit forecast (state-evolution equation; Algo. 4 step 2 for
 * level = MENKF_FINE with nb = 1, Algo. 3 step 2 for level = MENKF_COARSE
 * with nb <= n_members states).  Advances state_dev in place by nsteps
 * time steps.  If prev_dev is not NULL it receives the state one step
 * before the end (the right-hand side x_{k-1} of the fine-grid implicit
 * system used by the relaxed iteration).  nsteps >= 1. */
menkf_status menkf_forecast(menkf_ctx *ctx, int32_t level, void *state_dev, int32_t nb,
                            int32_t nsteps, void *prev_dev, menkf_stream stream);

/* Forecast schedule of one grid level: how the explicit stencil of the
 * state-evolution equation is tiled and ordered on the GPU.  It changes
 * speed only, never results: every tile shape and chunking evaluates the
 * same arithmetic per grid point, so forecasts are bitwise identical.
 *   tile_x, tile_y  grid points per 256-thread workgroup of the 2D stencil,
 *                   one of 32x16, 64x8, 32x8, 16x16, 64x4 (FP32) or
 *                   32x8, 16x8, 16x16, 64x4 (FP64); 0, 0 = the first of
 *                   the list (32x16 / 32x8).  FP32 also takes 0x16, the
 *                   row march: a workgroup of nx threads advances 16 whole
 *                   periodic rows of one state (nx = 64, 128, 192 or 256,
 *                   ny a multiple of 16; other grids run the 32x16 tile
 *                   instead); it is the coarse level's initial schedule
 *                   when it applies.  Ignored by the 1D model.
 *   member_chunk    states advanced together through a whole forecast
 *                   window, chunk after chunk, so that a chunk's state and
 *                   Runge-Kutta temporaries stay in the last-level cache;
 *                   0 = all nb states at once.  Ignored by the 1D model. */
typedef struct {
    int32_t tile_x, tile_y;
    int32_t member_chunk;
    int32_t reserved;
} menkf_schedule;

/* Set / read the schedule of level MENKF_FINE or MENKF_COARSE (host only;
 * applies to forecasts issued afterwards, also the relaxed sweeps and the
 * residual for MENKF_FINE).  Unknown tile shapes or a negative chunk give
 * MENKF_E_ARG and leave the schedule unchanged. */
menkf_status menkf_set_schedule(menkf_ctx *ctx, int32_t level, const menkf_schedule *sched);
menkf_status menkf_get_schedule(const menkf_ctx *ctx, int32_t level, menkf_schedule *sched);

/* Autotuner of the forecast schedule: times every tile shape of the
 * context's precision against member chunks nb, nb/2, nb/4, ... (coarse
 * level), each as one warm-up and reps individually timed forecasts of
 * nsteps steps of nb states held in scratch_dev (overwritten: pass a copy
 * of real states, the timing depends only on the shape), with HIP events on
 * stream; a schedule scores its fastest repetition.  The level's current
 * schedule is timed first and is replaced only by a candidate at least 3 %
 * faster (so timing noise does not flip it); the winner becomes the
 * level's schedule and is returned in *best with its time per forecast in
 * *best_ms (either may be NULL).  A set-up
 * call: it synchronises the stream and must not be captured into a graph. */
menkf_status menkf_autotune(menkf_ctx *ctx, int32_t level, void *scratch_dev, int32_t nb, int32_t nsteps,
                            int32_t reps, menkf_schedule *best, float *best_ms, menkf_stream stream);

/* x* = Pi_C(x^F_f) (Algo. 4 step 4): the fourth-order Lagrange restriction
 * of Sec. 2.2 on nested vertex-centred grids, i.e. injection of every
 * ratio-th node.  xf_dev: one fine state; xc_dev: one coarse state. */
menkf_status menkf_restrict(menkf_ctx *ctx, const void *xf_dev, void *xc_dev, menkf_stream stream);

/* Ensemble gain (Algo. 3 steps 3, 4, 7, 8; Algo. 1 steps 2-6).
 *   members_dev  the N_e forecast members (coarse states), unchanged
 *   xstar_dev    x* (coarse state)
 *   yobs_dev     N_y double observations y^o
 *   eps_dev      NULL: draw eps^(i) ~ N(0, obs_sigma^2) with Philox4x32-10
 *                keyed by seed and counter (probe/2, member, cycle, 0x5045),
 *                Box-Muller in FP64; else N_e x N_y doubles used as given.
 * Computes H^C of every member and of x*, secant anomalies Y, the
 * perturbed-observation innovations D = y^o + eps^(i) - y^(i) and
 * d* = y^o - H^C(x*), S = Y Y^T + R (or + E E^T), its FP64 Cholesky
 * factor, and the gain factors Z = Y^T S^-1 [D | d*] kept in the
 * workspace for menkf_update.  A non-positive pivot sets the device status
 * to column+1 (MENKF_E_NOT_SPD via menkf_get_status). */
menkf_status menkf_gain(menkf_ctx *ctx, const void *members_dev, const void *xstar_dev,
                        const double *yobs_dev, uint64_t seed, uint64_t cycle,
                        const double *eps_dev, menkf_stream stream);

/* cycle = MENKF_CYCLE_DEVICE makes menkf_gain take the cycle number from a
 * counter kept in the workspace and advance it by one on the device, so a
 * captured cycle replayed many times draws new perturbations each time.
 * menkf_set_cycle sets that counter (stream-ordered, no allocation). */
#define MENKF_CYCLE_DEVICE (~(uint64_t)0)
menkf_status menkf_set_cycle(menkf_ctx *ctx, uint64_t cycle, menkf_stream stream);

/* Copy the gain factors Z of the last menkf_gain into z_dev, laid out as
 * (N_e + 1) x N_e doubles, row j = column j of Z (j < N_e: member j's
 * innovation; j = N_e: the x* innovation). */
menkf_status menkf_get_gain(menkf_ctx *ctx, double *z_dev, menkf_stream stream);

/* Member update and coarse correction (Algo. 3 step 8; Algo. 4 step 5):
 *   members_dev  in/out: x^a(i) = x^(i) + X Z[:, i], X the normalised anomalies
 *   deltac_dev   out: delta^C = X Z[:, N_e] (= x^C' - x*), computed in FP64
 * Uses the factors of the preceding menkf_gain on the same members.  A no-op
 * on the device if the status word is set. */
menkf_status menkf_update(menkf_ctx *ctx, void *members_dev, void *deltac_dev, menkf_stream stream);

/* Fine-grid correction and regularisation (Algo. 4 steps 5-6):
 *   xf_dev       in: x^F_f, out: x^F_a
 *   deltac_dev   delta^C (coarse state)
 *   xprev_dev    x^F_{k-1}, the fine state one step before x^F_f
 *   MENKF_PROLONG_PLAIN: x' = x^F_f + Pi_F(delta^C) (cubic Lagrange,
 *   Sec. 2.2), then n_sweeps damped Jacobi sweeps of the implicit-Euler
 *   system x - dt F(x) = x^F_{k-1}:  x <- x + alpha/D (x_{k-1} + dt F(x) - x),
 *   D the viscous diagonal (one sweep with alpha = 0.5 in the paper's
 *   implementation notes).
 *   MENKF_PROLONG_LEARNED: x' = x^F_f + Pi_F(delta^C) + NN(Pi_F(delta^C), x^F_f)
 *   with the network net (2D, MENKF_F32 contexts), no sweeps.
 *   MENKF_PROLONG_LEARNED_FALLBACK: the network's correction, with the plain
 *   correction (Pi_F(delta^C) and n_sweeps sweeps, as MENKF_PROLONG_PLAIN)
 *   as its judge and its fallback; the network's output is not swept.
 *   Every net->judge_every-th call of the context (the first included;
 *   0 = never) also forms the plain correction x_plain and the distance
 *   |x_net - x_plain| / |x_plain - x^F_f| (whole fine state, FP64 sums):
 *   above net->judge_tol the plain correction is used, in this call and in
 *   every call up to the next judged one (which may return to the
 *   network).  Independently, a 16x16 pixel tile whose network output is
 *   non-finite or whose norm exceeds guard * |Pi_F(delta^C)| on that tile
 *   (counted in net->fallback_count_dev if given) makes that call use the
 *   plain correction for the whole state.  The decisions are taken on the
 *   device (graph-capturable); their state lives in the workspace and is
 *   reset by menkf_set_workspace.
 * A no-op on the device if the status word is set.
 *
 * The network (not part of the paper; its closing section names better
 * coarse-to-fine projectors as future work): conv3x3(8->32), ReLU,
 * conv3x3(32->32), ReLU, conv3x3(32->4), circular padding, cross-
 * correlation.  Input channels: Pi_F(delta^C) and x^F_f, each field mapped
 * to (v - in_offset) * in_scale; the fine correction is
 * Pi_F(delta^C) + out / out_scale.  BF16 weights and activations, FP32
 * accumulation on MFMA. */
#define MENKF_NET_NPARAM 12740   /* FP32 parameter vector, see menkf_net_pack */
#define MENKF_NET_NPACKED 20736  /* BF16 elements of the packed kernel weights */
typedef struct {
    const void *wpacked;   /* BF16 kernel-layout weights written by menkf_net_pack */
    const float *params;   /* FP32 parameter vector (the biases are read from it) */
    float in_scale[8], in_offset[8], out_scale[4];
    float guard;           /* fallback amplitude guard (LEARNED_FALLBACK) */
    int32_t *fallback_count_dev; /* optional: incremented per guarded tile */
    int32_t judge_every;   /* LEARNED_FALLBACK: judge every judge_every-th call; 0 = never */
    float judge_tol;       /* LEARNED_FALLBACK: largest accepted relative distance to the plain correction */
    double *judge_dev;     /* optional, 4 doubles accumulated by LEARNED_FALLBACK calls: [0] distance of
                            * the last judged call, [1] judged calls, [2] calls corrected by the plain
                            * path, [3] calls with a guarded tile */
} menkf_net;

menkf_status menkf_prolong_smooth(menkf_ctx *ctx, const void *deltac_dev, void *xf_dev,
                                  const void *xprev_dev, int32_t n_sweeps, double alpha,
                                  int32_t mode, const menkf_net *net, menkf_stream stream);

/* Pack the FP32 parameter vector (params_dev, MENKF_NET_NPARAM floats laid
 * out as w1[32][8][3][3], b1[32], w2[32][32][3][3], b2[32], w3[4][32][3][3],
 * b3[4], the PyTorch convolution order) into the BF16 kernel layout
 * (MENKF_NET_NPACKED elements: w1 as [32][3][3][8], w2 as [32][3][3][32],
 * w3 as [32][3][3][32] with output rows 4..31 zero). */
menkf_status menkf_net_pack(const float *params_dev, void *wpacked_dev, menkf_stream stream);

/* One training step of the network on a batch of periodic crops (Adam,
 * Kingma & Ba 2015; mean-squared error of the scaled residual
 * (correction - Pi_F(delta^C)) * out_scale).  Inputs are npairs full
 * periodic fine fields [npairs][4][H][W] (FP32): dproj = Pi_F(delta^C),
 * xf = x^F_f, target = the fine correction to learn.  crops_dev holds
 * batch (pair, y0, x0) triples; each crop is crop x crop output pixels,
 * evaluated with the periodic halo of the full field.  BF16 activations and
 * weights, FP32 arithmetic and master weights.  apply_adam = 0 computes the
 * loss and the gradient (grad, same layout as params) only.  step is the
 * 1-based Adam step.  loss_dev receives the batch loss (double). */
typedef struct {
    float *params, *grad, *adam_m, *adam_v;  /* MENKF_NET_NPARAM each, device */
    void *wpacked;                           /* refreshed after the update */
    const float *dproj, *xf, *target;        /* [npairs][4][H][W], device */
    int32_t npairs, H, W;
    const int32_t *crops_dev;                /* [batch][3] */
    int32_t batch, crop;
    float in_scale[8], in_offset[8], out_scale[4];
    float lr, beta1, beta2, eps;
    int32_t step, apply_adam;
    double *loss_dev;
    void *workspace_dev;                     /* menkf_net_train_workspace_size bytes */
    size_t workspace_bytes;
} menkf_net_train;

menkf_status menkf_net_train_workspace_size(int32_t batch, int32_t crop, size_t *bytes);
menkf_status menkf_net_train_step(const menkf_net_train *t, menkf_stream stream);

/* The training step in its three phases, on the same descriptor and
 * workspace (menkf_net_train_step = forward, backward, and Adam when
 * apply_adam is set; the three calls in that order give bitwise its
 * results):
 *   menkf_net_forward:  layer activations of the crops into the workspace,
 *                       the batch loss into loss_dev and its gradient with
 *                       respect to the network output (workspace);
 *   menkf_net_backward: the parameter gradient into grad, from what the
 *                       last menkf_net_forward on this workspace left
 *                       (calling it without one reads stale activations);
 *   menkf_net_adam:     the Adam update of params (moments adam_m, adam_v,
 *                       1-based step; apply_adam is not read) from grad,
 *                       then the BF16 repack into wpacked if it is set.
 * Argument checks as for menkf_net_train_step (Adam needs its moment
 * buffers and step >= 1). */
menkf_status menkf_net_forward(const menkf_net_train *t, menkf_stream stream);
menkf_status menkf_net_backward(const menkf_net_train *t, menkf_stream stream);
menkf_status menkf_net_adam(const menkf_net_train *t, menkf_stream stream);

/* Synchronise the stream and read the device status word into *info
 * (0 = fine, j+1 = first non-positive pivot at column j).  Returns
 * MENKF_E_NOT_SPD if it is set.  Clears the word when clear != 0. */
menkf_status menkf_get_status(menkf_ctx *ctx, int32_t *info, int32_t clear, menkf_stream stream);

/* Fine-to-coarse feedback (driving the coarse ensemble by the fine-grid
 * analysis, which the paper's closing section names as future work):
 * x^(i) <- x^(i) - mean_i x^(i) + Pi_C(xf) for every member, so the
 * ensemble mean becomes the injected fine state while every anomaly is
 * kept; mean and shift in FP64.  members_dev: n_members coarse states
 * (in/out); xf_dev: one fine state (the analysis x^F_a).  A no-op on the
 * device if the status word is set. */
menkf_status menkf_recentre(menkf_ctx *ctx, void *members_dev, const void *xf_dev, menkf_stream stream);

/* Observation operator on nb states: level MENKF_FINE applies H^F (state =
 * fine), MENKF_COARSE applies H^C = H^F o Pi_F; y_dev gets nb x N_y doubles. */
menkf_status menkf_observe(menkf_ctx *ctx, int32_t level, const void *state_dev, int32_t nb,
                           double *y_dev, menkf_stream stream);

/* Diagnostics of a fine state against a reference (Sec. 4 relative RMSE):
 * out_dev[0] = sum (xa - xt)^2, out_dev[1] = sum xt^2 over the observed
 * quantity (u in 1D; (u, v) in 2D), out_dev[2] = number of non-finite
 * entries of xa, accumulated in FP64. */
menkf_status menkf_diagnostics(menkf_ctx *ctx, const void *xa_dev, const void *xt_dev,
                               double *out_dev, menkf_stream stream);

/* menkf_diagnostics for callers that cannot allocate device memory or
 * attach a workspace (code under HIP graph capture, serving loops, hosts
 * that forbid hipMalloc): the same outputs from the same kernels, with the
 * reduction partials (at most 3 x 512 doubles) in a static device array of
 * 2048 doubles (16 KiB) that the library holds on every GPU it runs on until
 * the process ends, instead of the context workspace.  The context needs no
 * workspace.  Allocates nothing: no hipMalloc, hipFree or allocating library
 * call.  The first call on a device looks the array's address up once
 * (hipGetSymbolAddress) and keeps it; make that first call outside a graph
 * capture.  A request needing more partials than the array holds returns
 * MENKF_E_WORKSPACE (none does with the present block cap).  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (on two
 * streams, or from two threads) race and must be serialised by the caller. */
menkf_status menkf_diagnostics_noalloc(menkf_ctx *ctx, const void *xa_dev, const void *xt_dev, double *out_dev,
                                       menkf_stream stream);

/* Ensemble spread of the coarse members (the ensemble estimate of the error
 * covariance, P^e = X X^T with X = (x^(i) - mean) / sqrt(N_e - 1), Sec. 2.1.2),
 * over the observed quantity (u in 1D Burgers, rho u in 1D Euler, the
 * velocity pair (u, v) = (rho u, rho v) / rho in 2D), accumulated in FP64:
 *   out_dev[0] = trace of P^e = sum_points sum_i (q^(i) - mean q)^2 / (nb - 1)
 *   out_dev[1] = sum_points (mean q)^2   (sqrt(out[0] / out[1]) is the
 *                relative spread, comparable with the relative RMSE)
 *   out_dev[2] = number of non-finite values of q.
 * members_dev: nb coarse states [nb][F][ny_c][nx_c], 2 <= nb <= n_members.
 * Needs the workspace (reduction partials); asynchronous on stream. */
menkf_status menkf_spread(menkf_ctx *ctx, const void *members_dev, int32_t nb, double *out_dev, menkf_stream stream);

/* Residual of the fine-grid implicit-Euler system of the last step,
 * r = x_{k-1} + dt F(x) - x (fine states, r must not alias the inputs).
 * The conservativity indicator of Sec. 6 for a conserved field is
 * Gamma = -r / dt on that field (e.g. field 2, rho v, in 2D). */
menkf_status menkf_residual(menkf_ctx *ctx, const void *x_dev, const void *xprev_dev, void *r_dev,
                            menkf_stream stream);

/* ----------------------------------------------------------------------
 * Dual estimation of the inlet parameters (Sec. 2.1.3, Algo. 2, applied to
 * the coarse ensemble as in Algo. 3, the fine run of Algo. 4 driven by the
 * mean analysed parameters), MENKF_BURGERS1D_INLET contexts only.
 * Parameters are FP64 pairs theta = (amplitude theta_1, phase theta_2),
 * one row of 2 doubles per state.
 * ---------------------------------------------------------------------- */

/* Forecast of the inlet-forced model (state-evolution equation with the
 * inlet value of each state's own parameters): as menkf_forecast, plus
 *   theta_dev  nb x 2 doubles, row i = parameters of state i
 *   t0_dev     one double: the time at the start of the window (read when
 *              the forecast runs, so a captured call sees updates)
 * menkf_forecast on such a context returns MENKF_E_ARG. */
menkf_status menkf_forecast_inlet(menkf_ctx *ctx, int32_t level, void *state_dev, int32_t nb, int32_t nsteps,
                                  void *prev_dev, const double *theta_dev, const double *t0_dev,
                                  menkf_stream stream);

/* Parameter forecast (Algo. 2 step 1): theta_f = theta + tau for the
 * n_members rows, tau_k ~ N(0, theta_sigma[k]^2) drawn with Philox4x32-10
 * keyed by seed at counter (k/2, member, cycle, 0x5041), Box-Muller in FP64
 * (cos for k = 0, sin for k = 1).  cycle = MENKF_CYCLE_DEVICE reads the
 * context's device counter without advancing it.  theta_f may alias theta. */
menkf_status menkf_param_perturb(menkf_ctx *ctx, const double *theta_dev, double *theta_f_dev, uint64_t seed,
                                 uint64_t cycle, menkf_stream stream);

/* Parameter analysis (Algo. 2 step 5): theta_a(j) = theta_f(j) +
 * sum_i Theta_i Z[i, j], Theta_i = (theta_f(i) - mean) / sqrt(N_e - 1), with
 * the gain factors Z of the preceding menkf_gain, which must have been
 * computed on the members forecast with theta_f.  theta_mean_dev (2
 * doubles) receives the mean of theta_a.  theta_a may alias theta_f.  A
 * no-op on the device if the status word is set. */
menkf_status menkf_param_update(menkf_ctx *ctx, const double *theta_f_dev, double *theta_a_dev,
                                double *theta_mean_dev, menkf_stream stream);

/* One dual cycle, issued on stream as
 *   theta_f = theta + tau (as menkf_param_perturb), trial = members      (workspace)
 *   menkf_forecast_inlet(COARSE, trial, theta_f, clock)
 *   menkf_gain(trial, members[0], yobs, seed, cycle)  any x* (only Z[:, :N] is used
 *                                                    next); the cycle counter is not
 *                                                    advanced here
 *   menkf_param_update(theta_f -> theta, theta_mean)
 *   menkf_forecast_inlet(FINE, fine, theta_mean, clock), x_{k-1} into fine_prev
 *   menkf_forecast_inlet(COARSE, members, theta, clock)
 *   menkf_restrict(fine, xstar)
 *   menkf_gain(members, xstar, yobs, seed, cycle)    the same perturbed observations
 *   menkf_update(members, deltac)
 *   menkf_prolong_smooth(deltac, fine, fine_prev, n_sweeps, alpha, PLAIN)
 *   clock += nsteps dt
 * theta (n_members x 2 doubles) is in/out, theta_mean (2 doubles) out,
 * clock (one double) in/out; the other buffers as for menkf_cycle.
 * aux_stream (optional, NULL = none, not stream itself): the fine forecast
 * is issued there, forked from and joined back into stream with the
 * context's two events, so it runs beside the member forecast; results are
 * the same.  A non-positive pivot of the parameter gain leaves theta as it
 * was; the status word then reports the state gain's outcome only. */
typedef struct {
    menkf_ctx *ctx;
    void *fine, *fine_prev, *members, *xstar, *deltac;
    const double *yobs;
    double *theta, *theta_mean, *clock;
    uint64_t seed, cycle;
    int32_t nsteps, n_sweeps;
    double alpha;
    menkf_stream aux_stream;
} menkf_dual_args;

menkf_status menkf_dual_cycle(const menkf_dual_args *args, menkf_stream stream);

/* Normalised RAM requirement R_RAM = 1 + N_e / r_C^dim of one fine
 * simulation plus N_e coarse members (Sec. 3).  Host only. */
double menkf_ram_ratio(int32_t dim, int32_t ratio, int32_t n_members);

/* One assimilation cycle of one instance (Algo. 4 steps 2-6 with the
 * member forecast and analysis of Algo. 3), issued on stream as
 *   menkf_forecast(FINE, fine, 1, nsteps, fine_prev)
 *   menkf_forecast(COARSE, members, n_members, nsteps, NULL)
 *   menkf_restrict(fine, xstar)
 *   menkf_gain(members, xstar, yobs, seed, cycle, NULL)
 *   menkf_update(members, deltac)
 *   menkf_prolong_smooth(deltac, fine, fine_prev, n_sweeps, alpha, prolong_mode, net)
 *   [menkf_recentre(members, fine) if feedback]
 * with the contracts of those calls.  All pointers are device buffers owned
 * by the caller: fine and fine_prev one fine state each, members n_members
 * coarse states, xstar and deltac one coarse state each, yobs n_probes
 * doubles (read when the cycle runs, so a captured cycle can be fed new
 * observations in place).  cycle = MENKF_CYCLE_DEVICE uses the context's
 * device counter.  aux_stream (optional, NULL = none, not stream itself):
 * the fine forecast is issued there, forked from and joined back into
 * stream with two events the context owns.  With MENKF_GAIN_EXACT_R it
 * runs beside the N_y x N_y factorisation: the member forecast comes
 * first, the factorisation runs with d* = 0 (the fine forecast is forked
 * from it once each remaining trailing update has at most four tiles per
 * compute unit, so that it fills the GPU beside the latency-bound late
 * block steps rather than the throughput-bound early ones), and the x*
 * column of the gain
 * follows once x* is known through the identity
 *   z* = Y^T (Y Y^T + s^2 I)^-1 d* = (s^2 I + Y^T Y)^-1 Y^T d*
 * (the N_e x N_e system, which needs only the anomalies, is factored on
 * aux_stream too, forked right after the gain's front end).  The member columns
 * of Z are bitwise those of menkf_gain; z*, delta^C and the fine state
 * agree with it to FP64 roundoff.  In the other gain modes the fine
 * forecast runs beside the member forecast and results are bitwise the
 * same as without aux_stream.
 *
 * pipelined = 1 defers the fine-grid correction (Algo. 4 steps 5-6) by one
 * call, software pipelining of consecutive cycles: the call begins with the
 * correction left pending by the previous pipelined call,
 *   menkf_prolong_smooth(deltac, fine, fine_prev, n_sweeps, alpha, prolong_mode, net),
 * and ends with menkf_update, leaving its own delta^C pending in deltac
 * (a device word of the context records whether a correction is pending:
 * none after menkf_set_workspace or menkf_cycle_flush, so the first
 * pipelined call corrects nothing; whether one is pending is read when the
 * call starts).  With aux_stream the pending correction runs there ahead of
 * the fine forecast (with MENKF_GAIN_EXACT_R beside the early block steps of
 * the factorisation, after the x* system), off the member chain that bounds
 * the cycle.  After the call fine holds the uncorrected forecast x^F_f;
 * menkf_cycle_flush applies the pending correction, after which K
 * pipelined calls have given bitwise the results of K calls with
 * pipelined = 0.  Flush before reading fine as an analysis, before a call
 * with pipelined = 0 and before changing n_sweeps, alpha, prolong_mode or
 * net.  feedback must be 0 (it needs the corrected state). */
typedef struct {
    menkf_ctx *ctx;
    void *fine, *fine_prev, *members, *xstar, *deltac;
    const double *yobs;
    uint64_t seed, cycle;
    int32_t nsteps, n_sweeps;
    double alpha;
    int32_t prolong_mode;
    const menkf_net *net;
    menkf_stream aux_stream;
    int32_t feedback;    /* 1: end the cycle with menkf_recentre(members, fine) */
    int32_t pipelined;   /* 1: correction deferred to the next call (above) */
} menkf_cycle_args;

menkf_status menkf_cycle(const menkf_cycle_args *args, menkf_stream stream);

/* The correction left pending by the last pipelined menkf_cycle of
 * args->ctx (fine, fine_prev, deltac, n_sweeps, alpha, prolong_mode and net
 * of args, as that call had them; nothing when none is pending), issued on
 * stream; clears the pending word.  Capturable. */
menkf_status menkf_cycle_flush(const menkf_cycle_args *args, menkf_stream stream);

/* Batch of independent instances of uneven sizes advanced together: a
 * batch owns n_lanes HIP streams (default priority) and their events.
 * menkf_batch_cycle forks the lanes from stream, assigns the n instances to
 * lanes longest-first by an estimated cost (autotuned forecast times when
 * menkf_autotune has run on the instance, otherwise a model of stencil
 * points and Cholesky block steps), issues one menkf_cycle per instance on
 * its lane and joins every lane back into stream.  Capturable: inside a
 * graph capture of stream the whole batch becomes one graph.  Instances
 * must not share contexts or buffers.  menkf_batch_lane gives the lane
 * each instance went to in the last call (lane_of has n entries). */
typedef struct menkf_batch menkf_batch;
menkf_status menkf_batch_create(int32_t n_lanes, menkf_batch **out);
void menkf_batch_destroy(menkf_batch *b);
menkf_status menkf_batch_cycle(menkf_batch *b, const menkf_cycle_args *inst, int32_t n, menkf_stream stream);
menkf_status menkf_batch_lanes(const menkf_batch *b, int32_t *lane_of, int32_t n);

/* HIP graph helpers: capture the menkf_* calls issued on stream between
 * begin and end into a graph, then replay it.  The stream must not be the
 * legacy default stream. */
menkf_status menkf_graph_begin(menkf_stream stream);
menkf_status menkf_graph_end(menkf_stream stream, menkf_graph **out);
menkf_status menkf_graph_launch(menkf_graph *g, menkf_stream stream);
void menkf_graph_destroy(menkf_graph *g);

#ifdef __cplusplus
}
#endif
#endif /* MENKF_H */
