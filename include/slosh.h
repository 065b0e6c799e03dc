/*
 * slosh.h -- C ABI of the MI355X (gfx950) sloshing simulator.
 *
 * The library steps a 2D weakly compressible SPH fluid in a partially filled
 * tank, in the tank's body frame, coupled to the planar rigid-body dynamics of
 * the spacecraft that carries it, and evaluates a small MLP surrogate of the
 * slosh wrench.  The operations follow the paper's problem statement
 * (Section 2: input u = [u_x, u_y, tau] at the centre of mass, output
 * y = [r_x, r_y, theta, rdot_x, rdot_y, thetadot]) and its simulator
 * (Section 3: eqs. density_update, EOS, momentum, viscous, pressure_b2f,
 * viscous_b2f, tankdynamics, cubicspline, spiky3; Algorithm "state transition
 * function"; first-order symplectic Euler).
 *
 * Conventions for every call:
 *   - "dev" pointers are device (HBM) pointers on the current HIP device;
 *     "host" pointers are ordinary host memory.  All float arrays are
 *     little-endian IEEE binary32, row-major, with no padding.
 *   - The caller owns all device memory: particle arrays, logs and a
 *     workspace sized by sph_workspace_bytes / mlp_workspace_bytes.  The
 *     library never allocates device memory; it allocates only its opaque
 *     host handle (freed by *_destroy) and, for rollouts, HIP graphs.
 *   - Work is enqueued on the stream given at init (a hipStream_t passed as
 *     void*; NULL = the legacy default stream) and is asynchronous unless a
 *     call says it synchronises.  One handle per stream; no internal locking.
 *   - Every call returns 0 on success or a negative SPH_E_* code; no C++
 *     exception crosses the ABI.  sph_strerror gives a message.
 *   - Particle outputs are in the caller's particle order (the order of the
 *     arrays given to sph_init); the library reorders particles internally.
 */
#ifndef SLOSH_H
#define SLOSH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define SPH_OK 0
#define SPH_E_INVAL (-1)      /* bad argument, size or parameter */
#define SPH_E_HIP (-2)        /* a HIP runtime call failed; see sph_strerror */
#define SPH_E_CAPACITY (-3)   /* workspace too small / grid too large */
#define SPH_E_STATE (-4)      /* device status word non-zero (see sph_status) */

/* ---- device status bits (latched on device, read by sph_status) -------- */
#define SPH_ST_ESCAPED 1u     /* a fluid particle left the domain box */
#define SPH_ST_NONFINITE 2u   /* a NaN or Inf position or velocity appeared */
#define SPH_ST_SORT 4u        /* a particle moved farther than the cell list's
                               * skin allows since the last rebuild */
#define SPH_ST_CFL 8u         /* a fluid particle's speed put the step's Courant
                               * number dt (c + |w|) / h above 0.4 (c: sound
                               * speed at rest, c0 or sqrt(k_lin)) */

/* ---- method options ----------------------------------------------------- */
#define SPH_EOS_TAIT 0        /* P = B((rho/rho0)^gamma - 1), B = rho0 c0^2/gamma */
#define SPH_EOS_LINEAR 1      /* P = k (rho - rho0)  (eq. EOS) */
#define SPH_EOS_LINEAR_CLAMPED 2  /* P = max(k (rho - rho0), 0): eq. EOS without tension */
#define SPH_EOS_TAIT_CLAMPED 3    /* P = max(B((rho/rho0)^gamma - 1), 0): Tait without tension */
#define SPH_MOTION_FREE 0     /* Newton-Euler rigid body (eq. tankdynamics) */
#define SPH_MOTION_SINE 1     /* prescribed theta = A sin(2 pi f t), r = 0 */
#define SPH_CTRL_NONE 0
#define SPH_CTRL_PD_ZOH 1     /* tau = kp (ref_k - theta) - kd thetadot, held (Section 5.1) */
#define SPH_KNORM_UNIT 0      /* cubic spline constant 5/(14 pi h^2): unit integral */
#define SPH_KNORM_PRINTED 1   /* constant 15/(14 pi h^2) as printed in eq. cubicspline */
#define SPH_FRAME_BODY 0
#define SPH_FRAME_WORLD 1

/* Scenario constants.  SI units; masses per unit depth (2D). */
typedef struct sph_params {
  int32_t eos, motion, ctrl, kernel_norm;
  double h;            /* smoothing length; cubic-spline support is 2h */
  double h_spiky;      /* support of the spiky kernel used for wall forces */
  double rho0;         /* rest density */
  double mass;         /* particle mass (fluid and ghost) */
  double c0;           /* Tait sound speed */
  double tait_gamma;   /* Tait exponent */
  double k_lin;        /* linear EOS stiffness */
  double visc_alpha;   /* fluid artificial-viscosity coefficient (eq. viscous) */
  double visc_beta;    /* fluid-wall viscosity coefficient (eq. viscous_b2f) */
  double eps;          /* singularity guard, eps h^2 */
  double gamma1;       /* ghost density correction (eq. density_update) */
  double dt;           /* fixed time step */
  double body_mass, body_inertia;
  double kp, kd;       /* PD gains */
  int32_t ctrl_period; /* zero-order-hold period in steps */
  int32_t reserved;
  double sine_amp, sine_freq;
  double domain_min[2], domain_max[2];  /* body-frame box holding every particle */
} sph_params;

typedef struct sph_handle sph_handle;

/* Device bytes of the workspace for N fluid and G ghost particles, or
 * SPH_E_INVAL for bad parameters (non-positive h, dt, mass; empty domain;
 * a cell grid above 2^26 cells). */
int sph_workspace_bytes(const sph_params* p, int32_t n_fluid, int32_t n_ghost, size_t* bytes);

/* Creates a simulator of the system of the problem statement (Section 2:
 * the spacecraft's planar rigid body carrying a partially filled tank, state
 * x = [r, theta, r_if, rdot, thetadot, rdot_if] of Section 3.4) at its
 * initial state: the fluid's particles (Section 3.1) and the tank wall's
 * fixed ghost particles (Section 3.2, which the paper moves with the tank by
 * eq. kinematicghost and this library keeps static in the tank's body
 * frame).  s0_dev, w0_dev: [n_fluid][2] body-frame positions and
 * velocities; g_dev: [n_ghost][2] static body-frame ghost positions; rigid0:
 * host [6] = r_x, r_y, theta, rdot_x, rdot_y, thetadot (world frame, double).
 * ws_dev: workspace of at least sph_workspace_bytes, 256-byte aligned, which
 * the caller keeps alive until sph_destroy.  Input arrays are copied and may
 * be freed after the call returns (the call synchronises the stream).
 * Builds the static ghost cell list and sorts the fluid into cells.
 * Returns SPH_E_INVAL on bad sizes/pointers, a particle outside the domain
 * box, or a time step above the Courant limit at rest (dt c > 0.4 h, c the
 * sound speed of the equation of state, for a tank that holds fluid);
 * SPH_E_CAPACITY if ws_bytes is too small. */
int sph_init(const sph_params* p, int32_t n_fluid, const float* s0_dev, const float* w0_dev,
             int32_t n_ghost, const float* g_dev, const double* rigid0, void* ws_dev,
             size_t ws_bytes, void* stream, sph_handle** out);

/* ---- many tanks in one handle ------------------------------------------- */
/*
 * A batch handle advances n_tanks independent tanks (each its own sph_params,
 * particle counts, cell grid, time step, rigid body and inputs) in the same
 * kernel launches.  Tank t's fluid particles are rows [P_t, P_t + n_fluid[t])
 * of the concatenated arrays, P_t = sum of the earlier n_fluid; ghosts
 * likewise.  For a batch, every per-tank argument of the calls below is
 * tank-major: rigid0 / rigid [T][6], u_dev [T][3], u_seq_dev [T][n_steps][3],
 * theta_ref_dev [T][n_ref], logs [T][n_log][...], wrench / acc [T][3],
 * tau_ctrl and step [T] in sph_get_state; particle arrays are concatenated.
 * A tank gives bitwise the same results alone or in a batch.
 */
int sph_batch_workspace_bytes(int32_t n_tanks, const sph_params* params, const int32_t* n_fluid,
                              const int32_t* n_ghost, size_t* bytes);

/* Like sph_init for n_tanks tanks: params [T] (host), n_fluid [T], n_ghost
 * [T] (host), s0_dev / w0_dev [sum n_fluid][2], g_dev [sum n_ghost][2],
 * rigid0 host [T][6]. */
int sph_batch_init(int32_t n_tanks, const sph_params* params, const int32_t* n_fluid, const float* s0_dev,
                   const float* w0_dev, const int32_t* n_ghost, const float* g_dev, const double* rigid0,
                   void* ws_dev, size_t ws_bytes, void* stream, sph_handle** out);

/* Number of tanks of a handle (1 for sph_init). */
int sph_num_tanks(sph_handle* h, int32_t* n_tanks);

/* Autotuner of the neighbour kernels: times, at the current state and
 * without advancing it, `reps` evaluations of one rebuild interval of the
 * step kernels (density, forces, wrench) for each supported number of lanes
 * per particle (4, 8, 16, 32; the tile is 256 / lanes particles), with and
 * without near lists, and keeps the fastest; *lanes receives the lanes (may
 * be NULL; sph_get_tuning reports both choices).  Rebuilds the cell list.
 * The choice changes the summation order, so results are reproducible for a
 * fixed choice (sph_set_lanes, sph_set_near_lists). */
int sph_autotune(sph_handle* h, int32_t reps, int32_t* lanes);

/* Selects the lanes per particle (4, 8, 16 or 32; default 8). */
int sph_set_lanes(sph_handle* h, int32_t lanes);

/* Near lists on (1) or off (0, default).  On: at the first step after each
 * cell-list rebuild every particle lists the candidates of its 3x3 cell
 * block that lie within 2h + skin of it (fluid) or S + skin/2 (boundary)
 * at the rebuild positions, and the other kernels of the interval walk only
 * those; off: every kernel walks the whole block.  Both give the same
 * neighbour sets (the sums differ in order only). */
int sph_set_near_lists(sph_handle* h, int32_t on);

/* Steps between cell-list rebuilds of the multi-kernel path: 1, 2, 4, 8,
 * 16, 32 or 64 (default 4); anything else is SPH_E_INVAL.  The neighbour sets
 * are those of an exact search at every step for any interval as long as
 * every fluid particle stays within skin/2 = h/2 of its position at the last
 * rebuild; the density kernel checks that bound at every step and latches
 * SPH_ST_SORT in the status word when it fails, so a run whose status stays
 * clean computed the same pairs as a rebuild at every step.  A rebuild
 * reorders the particles, so intervals differ in summation order (rounding)
 * only.  A change drops the handle's captured graphs; a rebuild that a
 * shorter interval makes overdue runs at the start of the next rollout. */
int sph_set_rebuild_interval(sph_handle* h, int32_t steps);

/* The current rebuild interval in steps. */
int sph_get_rebuild_interval(sph_handle* h, int32_t* steps);

/* The current tuning choices: lanes per particle and near lists (0/1);
 * either pointer may be NULL. */
int sph_get_tuning(sph_handle* h, int32_t* lanes, int32_t* near_lists);

/* Frees the host handle and its graphs (the workspace stays the caller's). */
int sph_destroy(sph_handle* h);

/* One symplectic-Euler step of the coupled system (Algorithm "state
 * transition function" + Section 3.4 integrator): cell-list build, density and
 * EOS, fluid and wall forces, slosh wrench, controller, rigid body, fictitious
 * accelerations and fluid update.  u_dev: device [3] = F_x, F_y (world frame)
 * and torque, or NULL for zero.  Asynchronous. */
int sph_step(sph_handle* h, const float* u_dev);

/* n_steps steps of the closed-loop simulation of Section 3.5 (each step is
 * sph_step: Algorithm "state transition function" followed by first-order
 * symplectic Euler, Section 3.4) under its multi-rate scheme: the SPH state
 * advances every step, the attitude law of Section 5.1 is sampled and held
 * every ctrl_period steps (zero-order hold), and the outputs are logged every
 * log_stride steps.  The steps are replayed from captured HIP graphs.
 * u_seq_dev: [n_steps][3]
 * inputs or NULL (zero); theta_ref_dev: [n_ref] double angle references at the
 * control instants (global step / ctrl_period) or NULL (zero), used by
 * SPH_CTRL_PD_ZOH.  Every log_stride steps (log_stride > 0) entry k receives
 * the state at local step k*log_stride and the wrench evaluated there:
 * y_log_dev [n_log][6] = r, theta, rdot, thetadot; wrench_log_dev [n_log][3]
 * = body-frame slosh force and torque; u_log_dev [n_log][3] = applied F_x,
 * F_y and total torque (input + controller); wmean_log_dev [n_log][3] = mean
 * body-frame wrench over the steps of the log interval.  n_log =
 * ceil(n_steps / log_stride); any log pointer may be NULL.  Asynchronous;
 * inputs and logs must stay valid until the stream reaches the end. */
int sph_rollout(sph_handle* h, int32_t n_steps, const float* u_seq_dev,
                const double* theta_ref_dev, int32_t n_ref, int32_t log_stride,
                float* y_log_dev, float* wrench_log_dev, float* u_log_dev,
                float* wmean_log_dev);

/* sph_rollout for small tanks, with the same arguments and results: one
 * workgroup per tank keeps the fluid, the ghosts, a cell list (cells of
 * side 2h) and the rigid state in LDS and runs up to 4,096 steps per launch,
 * each step being the same terms as the multi-kernel path (Algorithm "state
 * transition function": density, EOS, pair and wall forces, wrench, attitude
 * law, rigid body, symplectic Euler) separated by workgroup barriers.  Needs
 * every tank to hold at most 2,048 fluid particles, 1,024 ghosts and 2,048
 * cells of side 2h over its domain box (sph_resident_fits), else returns
 * SPH_E_CAPACITY without doing anything.  The summation order differs from
 * sph_rollout's, so the two agree to rounding, not bitwise.  Asynchronous;
 * ends with a rebuild of the multi-kernel path's cell list. */
int sph_rollout_resident(sph_handle* h, int32_t n_steps, const float* u_seq_dev, const double* theta_ref_dev,
                         int32_t n_ref, int32_t log_stride, float* y_log_dev, float* wrench_log_dev,
                         float* u_log_dev, float* wmean_log_dev);

/* *fits (host) = 1 if every tank of the handle fits sph_rollout_resident. */
int sph_resident_fits(sph_handle* h, int32_t* fits);

/* The slosh wrench (F_x, F_y, torque) of the fluid on the tank (the reaction
 * sums of eq. tankdynamics, torque about the centre of mass) at the last
 * evaluated state, in SPH_FRAME_BODY or SPH_FRAME_WORLD.  out_dev: device [3]. */
int sph_slosh_wrench(sph_handle* h, int32_t frame, float* out_dev);

/* Evaluates x_dot = f(x, u) at the current state without advancing it, with
 * the controller torque held as it is.  u_dev: device [3] or NULL.  Outputs
 * (device, caller order, any may be NULL): rho_dev [N], p_dev [N] pressure,
 * a_sph_dev [N][2] SPH acceleration, wdot_dev [N][2] body-frame fluid
 * acceleration including fictitious terms, wrench_dev [3] body frame,
 * acc_dev [3] = r''_x, r''_y, theta''.  Uses the neighbour lists of the last
 * rebuild (rebuilds first if one is due). */
int sph_rhs(sph_handle* h, const float* u_dev, float* rho_dev, float* p_dev, float* a_sph_dev,
            float* wdot_dev, float* wrench_dev, float* acc_dev);

/* Copies the state out: s_dev, w_dev [N][2] (caller order, may be NULL);
 * rigid: host [6] (may be NULL); tau_ctrl, step: host (may be NULL).
 * Synchronises the stream. */
int sph_get_state(sph_handle* h, float* s_dev, float* w_dev, double* rigid, double* tau_ctrl,
                  int64_t* step);

/* Replaces the state (checkpoint restore): s_dev, w_dev [N][2] in caller
 * order; rigid host [6]; held controller torque; global step counter.
 * Clears the status word.  Synchronises the stream. */
int sph_set_state(sph_handle* h, const float* s_dev, const float* w_dev, const double* rigid,
                  double tau_ctrl, int64_t step);

/* Synchronises the stream and returns the latched SPH_ST_* bits in *flags;
 * returns SPH_E_STATE if any bit is set, else SPH_OK. */
int sph_status(sph_handle* h, uint32_t* flags);

/* Test hook of the cell-list traversal that every particle sum uses: for each
 * fluid particle (caller order) the caller-order indices of the fluid
 * particles j != i with fmaf(dy, dy, dx*dx) < (2h)^2 in binary32, ascending,
 * in nbr_dev [N][max_nbr], and their number in count_dev [N] (counts above
 * max_nbr are reported but only max_nbr indices stored).  Reorders particles
 * internally like a step does. */
int sph_neighbours(sph_handle* h, int32_t max_nbr, int32_t* nbr_dev, int32_t* count_dev);

/* Measurement hook: advances the state by n_steps steps like sph_rollout (no
 * logs), launching each step's kernels directly with HIP events between them,
 * and writes the mean event-to-event time in microseconds of the six step
 * kernels to avg_us [6]: cell binning, count scan, stable placement (these
 * three per rebuild), density/EOS (with the deferred fluid update),
 * forces with the per-workgroup wrench partials, and the per-tank wrench sum
 * with the rigid-body update (these three per step).  Synchronises the stream. */
int sph_time_kernels(sph_handle* h, int32_t n_steps, const float* u_seq_dev,
                     const double* theta_ref_dev, int32_t n_ref, float* avg_us);

/* Terms of the analytic wall correction (eq. gamma1): for every fluid
 * particle i of fluid_dev [n_fluid][2] (FP32 positions, body frame) against
 * ghost_dev [n_ghost][2], num_dev[i] = rho0/m - sum_f W(r_if) (the fluid sum of
 * the density, self term included) and den_dev[i] = sum_g W(r_ig), FP64,
 * with the cubic spline and kernel normalisation of p (the printed
 * denominator index is read as a sum over the ghosts).  gamma1 = num/den is
 * the value that puts particle i at rest density; the paper evaluates it for
 * a representative particle next to the wall (Section 3.5).  O(n (n + ng))
 * set-up work; enqueued on `stream`. */
int sph_gamma1_terms(const sph_params* p, const float* fluid_dev, int32_t n_fluid, const float* ghost_dev,
                     int32_t n_ghost, double* num_dev, double* den_dev, void* stream);

/* A representative value of eq. gamma1 for a fluid state: the terms of
 * sph_gamma1_terms (written to the caller's num_dev / den_dev [n_fluid]),
 * then, on the host, the median of num/den over the fraction `top` (0, 1]
 * of the particles with a non-zero ghost sum that have the largest ghost
 * sums (ties by index; of an even count the lower middle value).  Those are
 * the particles against the wall with a full fluid neighbourhood on the
 * other side, the configuration the paper evaluates eq. gamma1 for (a
 * particle next to the wall, Section 3.2).  Synchronises the default stream
 * (the terms are computed on it); *gamma1 is host memory.  SPH_E_INVAL if no
 * particle sees a ghost. */
int sph_gamma1_estimate(const sph_params* p, const float* fluid_dev, int32_t n_fluid, const float* ghost_dev,
                        int32_t n_ghost, double top, double* num_dev, double* den_dev, double* gamma1);

/* ---- linearization: tangent-linear rollout ---------------------------- */
/*
 * Forward-mode derivative of the coupled step (the linearization of
 * x_{k+1} = f(x_k, u_k) that the paper obtains by automatic differentiation,
 * Section 3.5; each step follows Algorithm 1 and the symplectic Euler
 * update), propagated over n_steps steps along n_dir directions (1..64).
 * A direction perturbs the initial fluid state (ds0_dev, dw0_dev: device
 * [n_dir][N][2] caller order, or both NULL = zero), the initial rigid state
 * (drigid0: host [n_dir][6] r_x, r_y, theta, r'_x, r'_y, theta', or NULL =
 * zero) and the applied force/torque sequence (du_seq_dev: device
 * [n_dir][n_steps][3], or NULL = zero).  The primal starts from the handle's
 * state with u_seq_dev [n_steps][3] (or NULL) and theta_ref_dev [n_ref] as
 * in sph_rollout; the handle's state is not changed.  Neighbour sets are
 * those of the primal (rebuilt every step).  Single-tank handles only.
 * Outputs (any may be NULL): wrench host [3] = the slosh wrench of the last
 * step (body frame), dwrench host [n_dir][3] its derivative along each
 * direction; rigid host [6] the final rigid state, drigid host [n_dir][6]
 * its derivatives; ds_dev, dw_dev device [n_dir][N][2] the final fluid
 * tangents.  ws_dev: caller-owned, 256-byte aligned, of at least
 * sph_jvp_workspace_bytes.  Synchronises the stream.
 */
int sph_jvp_workspace_bytes(sph_handle* h, int32_t n_dir, size_t* bytes);
int sph_jvp_rollout(sph_handle* h, int32_t n_dir, int32_t n_steps, const float* u_seq_dev,
                    const float* du_seq_dev, const double* theta_ref_dev, int32_t n_ref,
                    const double* drigid0, const float* ds0_dev, const float* dw0_dev, void* ws_dev,
                    size_t ws_bytes, double* wrench, double* dwrench, double* rigid, double* drigid,
                    float* ds_dev, float* dw_dev);

/* ---- linearization: adjoint rollout ------------------------------------ */
/*
 * Reverse-mode derivative (the transpose of sph_jvp_rollout) of n_steps
 * steps from the handle's state: given the adjoint wbar (host [3]) of the
 * slosh wrench of the last step, optionally rbar (host [6]) of the final
 * rigid state and sbar_dev / wbar_dev (device [N][2], both or neither) of
 * the final fluid state, returns the adjoints of the inputs: grad_rigid0
 * (host [6]) of the initial rigid state, grad_u_dev (device [n_steps][3]) of
 * the applied force/torque sequence, grad_s0_dev / grad_w0_dev (device
 * [N][2], caller order) of the initial fluid state; any output may be NULL.
 * wrench (host [3]) receives the primal wrench of the last step.  The
 * state is stored every `every` steps on a forward sweep; the reverse sweep
 * recomputes one segment at a time and reverses its steps.  Inputs as in
 * sph_jvp_rollout; the handle's state is not changed; single-tank handles
 * only.  ws_dev: caller-owned, 256-byte aligned, of at least
 * sph_vjp_workspace_bytes(h, n_steps, every).  Synchronises the stream.
 */
int sph_vjp_workspace_bytes(sph_handle* h, int32_t n_steps, int32_t every, size_t* bytes);
int sph_vjp_rollout(sph_handle* h, int32_t n_steps, int32_t every, const float* u_seq_dev,
                    const double* theta_ref_dev, int32_t n_ref, const double* wbar, const double* rbar,
                    const float* sbar_dev, const float* wbar_dev, void* ws_dev, size_t ws_bytes,
                    double* wrench, double* grad_rigid0, float* grad_u_dev, float* grad_s0_dev,
                    float* grad_w0_dev);

/* Message for an error code (static storage). */
const char* sph_strerror(int code);

/* ---- slosh-wrench surrogate (an MLP, trained on rollouts) -------------- */
/*
 * Network: x [B][128] (32 samples x 4 channels) -> 4 x (Linear 256 + GELU,
 * tanh form) -> Linear 3.  Weights are BF16 on the MFMA path with FP32
 * accumulation, FP32 master weights for Adam.  Parameter packing, used by
 * every weights argument: for l = 0..4, W_l [out_l][in_l] then b_l [out_l],
 * concatenated, FP32; dims 128, 256, 256, 256, 256, 3 (231,171 values).
 */
typedef struct mlp_handle mlp_handle;

#define MLP_N_PARAMS 231171

/* Workspace bytes for batches of up to max_batch rows. */
int mlp_workspace_bytes(int32_t max_batch, size_t* bytes);

/* Creates a network with FP32 master weights copied from params_dev [231171]. */
int mlp_init(const float* params_dev, int32_t max_batch, void* ws_dev, size_t ws_bytes,
             void* stream, mlp_handle** out);

int mlp_destroy(mlp_handle* h);

/* y_dev [B][3] FP32 = net(x_dev [B][128] FP32), inputs rounded to BF16; one
 * fused kernel (activations stay on chip).  Asynchronous.  x_dev must be
 * 16-byte aligned (here and in mlp_train_step and mlp_backward), else
 * SPH_E_INVAL. */
int mlp_forward(mlp_handle* h, const float* x_dev, int32_t batch, float* y_dev);

/* One training step on the mean squared error: forward, backward (gradients
 * in FP32, written to grad_dev [231171] if non-NULL), then Adam with bias
 * correction (step counter kept in the handle).  target_dev [B][3].  The
 * batch loss is written to loss_dev [1] if non-NULL. */
int mlp_train_step(mlp_handle* h, const float* x_dev, const float* target_dev, int32_t batch,
                   float lr, float beta1, float beta2, float eps, float* grad_dev,
                   float* loss_dev);

/* Back-propagation of a given output gradient (Section 4 trains its
 * surrogate by gradient descent on a simulation-error loss; this is the
 * gradient half of such a step for the network above): the forward pass of
 * x_dev [B][128] is recomputed with its activations kept, then dy_dev
 * [B][3] = dL/dy is propagated back through the head and the four GELU
 * layers.  grads_dev [231171] receives dL/dparams in the packing above
 * (FP32; BF16 activations and weights, FP32 accumulation).  B is a multiple
 * of 32 in [32, max_batch]; SPH_E_INVAL otherwise.  The weights do not
 * change.  Asynchronous. */
int mlp_backward(mlp_handle* h, const float* x_dev, const float* dy_dev, int32_t batch, float* grads_dev);

/* One Adam step (Kingma and Ba; the optimizer Section 4 starts its fits
 * with) on the FP32 master weights from grads_dev [231171], bias-corrected
 * for step t >= 1 (1 - beta^t); moments are kept in the handle and start at
 * zero; the BF16 copies used by the kernels are refreshed.  The handle's
 * step counter (used by mlp_train_step) becomes t.  SPH_E_INVAL for t < 1,
 * lr < 0, betas outside [0, 1) or eps <= 0.  Asynchronous. */
int mlp_adam_step(mlp_handle* h, const float* grads_dev, float lr, float beta1, float beta2, float eps,
                  int32_t t);

/* Builds standardised surrogate inputs and targets from rollout logs.
 * feat_dev [n_roll][n_t][3] = theta, thetadot, input torque per log sample;
 * static_dev [n_roll][n_static] per-rollout constants (the fill ratio, and
 * optionally tank descriptors such as shape and particle spacing), 1 <=
 * n_static <= min(8, window); wrench_dev [n_roll][n_t][3] body-frame slosh
 * force and torque (may be NULL when y_dev is NULL); norm: host
 * [2 (3 + n_static) + 6] = input means [3 + n_static] (theta, thetadot,
 * torque, then each constant), input stds [3 + n_static], output means [3],
 * output stds [3] (stds > 0; with n_static = 1 the 14 numbers of the four
 * channels theta, thetadot, torque, fill).  With n_win = n_t - window + 1
 * windows per rollout, x_dev [n_roll * n_win][window * 4] receives window w
 * of rollout r as samples t = w .. w + window - 1, 4 channels per sample:
 * theta, thetadot, torque and, in the fourth, constant (t - w) % n_static of
 * the rollout (n_static = 1: the fill ratio in every sample); y_dev
 * [n_roll * n_win][3] the wrench at sample w + window - 1 (the surrogate's
 * target, Section 2 eq. surrogate as a one-step map).  Enqueued on
 * `stream`; asynchronous. */
int mlp_make_windows(const float* feat_dev, const float* static_dev, int32_t n_static, const float* wrench_dev,
                     int32_t n_roll, int32_t n_t, int32_t window, const float* norm, float* x_dev, float* y_dev,
                     void* stream);

/* Bit of mlp_coupled_rollout's per-rollout flags: a window input lay further
 * than z_max standard deviations from the training mean (or was not a
 * number). */
#define MLP_FLAG_OUT_OF_RANGE 1u

/* Rigid body driven by the surrogate instead of SPH: the use the paper makes
 * of its surrogate, standing in for the fluid in the spacecraft's simulation
 * (Section 4; the closed-loop validation of Section 5.3, Table 3).  For n_roll
 * rollouts (at most the handle's max_batch) of n_steps steps logged every
 * log_stride steps (T = ceil(n_steps / log_stride) >= window samples;
 * window = 32, the network's 128 inputs), for k = window - 1 .. T - 1: the
 * standardised window of samples k - window + 1 .. k (the layout and norm of
 * mlp_make_windows, constants from static_dev) goes through the network; its
 * output, de-standardised, is the mean body-frame slosh wrench over log
 * interval k (the target sph_rollout logs in wmean_log_dev); the rigid body
 * integrates the interval's steps with that wrench held and the applied
 * inputs, by eq. tankdynamics for a free body and the first-order symplectic
 * Euler of Section 3.4 (sph_rollout's rigid-body update without an attitude
 * law); then sample k + 1 is logged.
 * body_dev [n_roll][3] = body mass, inertia, dt; u_seq_dev
 * [n_roll][n_steps][3] = applied F_x, F_y, torque per step; rigid_dev
 * [n_roll][6] = r_x, r_y, theta, rdot_x, rdot_y, thetadot, in: the state at
 * sample window - 1, out: the state after the last step; feat_dev
 * [n_roll][T][3] = theta, thetadot, input torque per sample, in: samples
 * 0 .. window - 1 (for instance sph_rollout's logs of the same inputs), out:
 * samples window .. T - 1; y_log_dev [n_roll][T][6] (sph_rollout's y_log
 * layout) receives samples window .. T - 1 and wrench_log_dev [n_roll][T][3]
 * intervals window - 1 .. T - 1 (other rows are left as they are);
 * flags_dev [n_roll] is cleared, then receives MLP_FLAG_OUT_OF_RANGE for a
 * rollout any of whose window inputs lay further than z_max standard
 * deviations from the training mean: it left the data the network was fitted
 * on, and the caller runs it on SPH instead.  One workgroup advances 16
 * rollouts through every interval in one launch (the last 32 samples in
 * LDS).  SPH_E_INVAL for window != 32, n_roll outside
 * [1, max_batch], T < window, n_static outside mlp_make_windows' range,
 * z_max <= 0, a std that is not positive or a NULL pointer.  Enqueued on the
 * handle's stream; asynchronous. */
int mlp_coupled_rollout(mlp_handle* h, int32_t n_roll, int32_t n_steps, int32_t log_stride, int32_t window,
                        const double* body_dev, const float* u_seq_dev, const float* static_dev, int32_t n_static,
                        const float* norm, float z_max, double* rigid_dev, float* feat_dev, float* y_log_dev,
                        float* wrench_log_dev, uint32_t* flags_dev);

/* Copies the FP32 master weights to params_dev [231171]. */
int mlp_get_params(mlp_handle* h, float* params_dev);

/* ---- LPV state-space surrogate (Section 4, Section 5.3) ------------------ */
/*
 * The paper's surrogate of the velocity-level dynamics u = [u_x, u_y, tau] ->
 * y = [rdot_x, rdot_y, thetadot] (Section 5.3): eq. surrogate_form with
 * n_x = 4, n_u = 3, n_y = 3, one scheduling variable and D = 0,
 *     p_k     = W3 tanh(W2 tanh(W1 [x_k; u_k] + b1) + b2) + b3   (2 x 4 tanh)
 *     y_k     = (C0 + p_k C1) x_k
 *     x_{k+1} = (A0 + p_k A1) x_k + (B0 + p_k B1) u_k            (eq. LPVparametrization)
 * fitted by minimising eq. pem plus eq. regularization,
 *     L = (1/n) sum_k |y_k - yhat_k|^2 + sigma2/2 |theta|^2 + sigmax/2 |x0|^2,
 * with Adam followed by L-BFGS (Section 4).  A model is LPV_N_PARAM FP64
 * numbers: theta = A0 (4x4), B0 (4x3), C0 (3x4), A1, B1, C1, W1 (4x7: four
 * state then three input columns), b1 (4), W2 (4x4), b2 (4), W3 (1x4), b3,
 * each row-major, then the initial state x0 (4).  Data are the caller's
 * scaled samples: u_dev, y_dev device [n_samples][3] FP64, shared by all
 * n_models models (independent restarts).  Every entry point enqueues work on
 * `stream` (a hipStream_t as void*); lpv_lbfgs alone synchronises it (it
 * polls the per-model status between launches).  Models run one per quad of
 * lanes, 16 per wave: any n_models >= 1 is accepted and 16 cost the same as 1.
 */
#define LPV_N_THETA 137
#define LPV_N_PARAM 141

typedef struct lpv_opts {
  double sigma2;         /* weight of |theta|^2 in eq. regularization */
  double sigmax;         /* weight of |x0|^2 */
  double lr, beta1, beta2, eps;    /* Adam (Kingma and Ba) */
  double c1;             /* Armijo constant of the L-BFGS line search */
  double gtol;           /* L-BFGS stops when max |grad| <= gtol ... */
  double ftol;           /* ... or when f_old - f <= ftol max(|f_old|, |f|) */
  int32_t max_backtracks;  /* rejected steps before the line search fails */
  int32_t lti_only;      /* 1: only A0, B0, C0 and x0 move (their LTI fit); others keep their values */
} lpv_opts;

/* Workspace (device, caller-owned, any content) for n_models models over
 * n_samples samples: the reverse sweep's per-step record and the optimizer
 * state.  About 8 (4 n_samples + 900) bytes per 4 lanes of a padded model. */
int lpv_workspace_bytes(int32_t n_models, int32_t n_samples, size_t* bytes);

/* Open-loop simulation: params_dev [n_models][141]; u_dev [n_samples][3]
 * (u_per_model = 0) or [n_models][n_samples][3] (1); writes yhat to y_dev
 * [n_models][n_samples][3] and, if p_dev is non-NULL, the scheduling variable
 * to p_dev [n_models][n_samples].  Starts from each model's x0. */
int lpv_simulate(const double* params_dev, int32_t n_models, const double* u_dev, int32_t u_per_model,
                 int32_t n_samples, double* y_dev, double* p_dev, void* stream);

/* Loss L of each model at params_dev to loss_dev [n_models] and, if grad_dev
 * is non-NULL, its gradient to grad_dev [n_models][141] (reverse sweep;
 * entries that opts->lti_only freezes get 0; needs the workspace). */
int lpv_loss_grad(const double* params_dev, int32_t n_models, const double* u_dev, const double* y_dev,
                  int32_t n_samples, const lpv_opts* opts, double* loss_dev, double* grad_dev, void* ws_dev,
                  size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory or hand over a workspace
 * (code under HIP graph capture, tight serving or fitting loops, harnesses
 * that forbid allocation): lpv_loss_grad without the workspace arguments.
 * The reverse sweep's record lives in a fixed array of
 * LPV_NOALLOC_SCRATCH_BYTES in device memory, one per GPU, reserved when the
 * library's code is loaded on that GPU and held until the process ends; the
 * call itself allocates nothing.  It needs n_samples * 4 * 64 *
 * ceil(n_models / 16) * 8 bytes (16 models share one wave), so 2,200 samples
 * fit up to 112 models and one wave of 16 models fits 16,384 samples; larger
 * requests return SPH_E_CAPACITY without launching anything.  The record is
 * written before it is read, so nothing needs clearing between calls.  Every
 * call on one GPU shares that GPU's array: calls that overlap in time on one
 * GPU (two streams, or two host threads) race and give undefined results;
 * calls on one stream are ordered and safe.  Results equal lpv_loss_grad's
 * bit for bit.  Arguments, outputs and errors are those of lpv_loss_grad;
 * SPH_E_HIP if the array's device address cannot be obtained. */
#define LPV_NOALLOC_SCRATCH_BYTES (32u << 20)
int lpv_loss_grad_noalloc(const double* params_dev, int32_t n_models, const double* u_dev, const double* y_dev,
                          int32_t n_samples, const lpv_opts* opts, double* loss_dev, double* grad_dev,
                          void* stream);

/* `iters` Adam steps from zero moments on every model; params_dev is updated
 * in place; loss_dev [n_models] (may be NULL) gets the loss at the last
 * evaluated point (before the last update). */
int lpv_adam(double* params_dev, int32_t n_models, const double* u_dev, const double* y_dev, int32_t n_samples,
             const lpv_opts* opts, int32_t iters, double* loss_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* L-BFGS (memory 10, two-loop recursion, initial matrix gamma I from the
 * newest pair; steepest descent and a cleared memory when the direction is
 * not one of descent; trial steps 1, or 1/max(1, |g|_2) on the first
 * iteration, until the Armijo condition holds, each rejected step replaced by
 * the minimiser of the interpolating quadratic clamped to [0.1, 0.5] of it
 * (0.1 after a non-finite loss); a pair is kept only if
 * s'y > 1e-10 |s| |y|) on every model, from params_dev, updated in place.
 * Per model (device, each may be NULL): loss_dev the final loss, status_dev
 * 1 gradient tolerance, 2 no further decrease, 3 line search failed,
 * 4 max_iter accepted steps; iters_dev the accepted steps.  Synchronises. */
int lpv_lbfgs(double* params_dev, int32_t n_models, const double* u_dev, const double* y_dev, int32_t n_samples,
              const lpv_opts* opts, int32_t max_iter, double* loss_dev, int32_t* status_dev, int32_t* iters_dev,
              void* ws_dev, size_t ws_bytes, void* stream);

/* Closed-loop simulation of the model augmented with position integrators
 * (Section 5.3) under the sampled attitude law of Section 5.1,
 * tau_k = kp (ref_k - theta_k) - kd thetadot_k, held for one sample of
 * length ts.  The law reads the velocity the model predicts while the
 * previous input is still held, C(eta(x_k, u_{k-1})) x_k (the model's output
 * map depends on u_k through the scheduling map, so reading the output of
 * the new input would be an algebraic loop); the integrators advance by ts
 * C(p_k) x_k with the input applied.  Physical units: force_dev
 * [n_samples][2] (force_per_model = 0) or [n_models][n_samples][2] world
 * forces; ref_dev [n_samples] or [n_models][n_samples] angle reference;
 * scales host [6] = u scales (3) then y scales (3): the model sees u / u_scale
 * and predicts y / y_scale.  x0_dev [n_models][4] initial model state, or NULL
 * for zero.  Writes y_dev [n_models][n_samples][6] = r_x, r_y, theta, rdot_x,
 * rdot_y, thetadot at the start of each sample, and tau_dev
 * [n_models][n_samples] (may be NULL) the torque applied. */
int lpv_closed_loop(const double* params_dev, int32_t n_models, const double* x0_dev, const double* force_dev,
                    int32_t force_per_model, const double* ref_dev, int32_t ref_per_model, int32_t n_samples,
                    double ts, double kp, double kd, const double* scales, double* y_dev, double* tau_dev,
                    void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SLOSH_H */
