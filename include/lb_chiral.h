/*
 * lb_chiral.h -- C ABI of the coupled hybrid lattice-Boltzmann step for
 * chiral active droplets (Carenza, Gonnella, Negro, "Lattice Boltzmann
 * simulations of self-propelling chiral active droplets").
 *
 * One time step (Sec. 2 Eqs. (1)-(5), Sec. 3 Eqs. (6)-(11)):
 *   - chemical potential mu = dF/dphi and molecular field H = -dF/dQ of the
 *     free energy of Eq. (5) (second-order central stencils);
 *   - stress sigma = passive (interfacial + Ericksen + Beris-Edwards reactive
 *     + antisymmetric) + active -zeta*phi*Q (Eqs. (3)-(4));
 *   - D3Q19 BGK collide + pull-stream of the populations (Eqs. (6)-(8), (11)),
 *     forced by F = div(sigma) in the Guo form (force moments of Eq. (10));
 *   - explicit Euler finite-difference Beris-Edwards update of Q (Eq. (2)) and
 *     Cahn-Hilliard update of phi in conservative flux form (Eq. (1)).
 *
 * Conventions
 *   - Periodic box nx x ny x nz, each >= 3, at most 2^29 sites.  Lattice
 *     spacing = time step = 1.
 *   - Every host field array is float64, component-major [c][z][y][x] with x
 *     fastest; N = nx*ny*nz sites.  Q is passed as its 5 independent
 *     components (xx, xy, xz, yy, yz); Q_zz = -Q_xx - Q_yy.
 *   - Populations are deviations g_i = f_i - w_i*rho0, D3Q19 order:
 *     0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = the 12 edge vectors in
 *     opposite pairs (7,8) = (+x+y, -x-y), (9,10) = (+x-y, -x+y),
 *     (11,12) = (+x+z, -x-z), (13,14) = (+x-z, -x+z), (15,16) = (+y+z, -y-z),
 *     (17,18) = (+y-z, -y+z).
 *   - The state at time t is (post-stream g, Q, phi).  u reported at t is
 *     (sum_i c_i g_i + F/2)/rho.
 *
 * Ownership and streams
 *   - The caller owns every host array: lb_init / lb_set_* copy in, lb_moments /
 *     lb_populations copy out.  The library owns all device memory of a context.
 *   - hip_stream is borrowed (NULL = the default stream) and must outlive the
 *     context; every kernel of the context runs on it.  Device pointers passed
 *     to lb_get_state / lb_set_state / lb_adjoint_* must be valid on the
 *     context's device and ordered with respect to that stream by the caller.
 *
 * Errors
 *   - Every call returns lb_status (0 = LB_OK); no exception crosses the ABI.
 *     lb_last_error() gives a thread-local message for the last failure.
 *   - lb_step only enqueues work; a launch failure returns LB_EDEVICE.
 *     Non-finite values are reported by the next lb_free_energy
 *     (LB_ENONFINITE).  After any error the context is still valid for
 *     lb_destroy and for lb_set_state (recovery from a checkpoint).
 */
#ifndef LB_CHIRAL_H
#define LB_CHIRAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LB_OK = 0,
  LB_EINVAL = -1,     /* invalid argument or parameter                     */
  LB_ENOMEM = -2,     /* device allocation failed or box too large          */
  LB_EDEVICE = -3,    /* HIP runtime or kernel launch error                 */
  LB_ENONFINITE = -4, /* NaN/Inf found in the state by a reduction          */
  LB_ESTATE = -5      /* state buffer of the wrong size / context mismatch  */
} lb_status;

typedef enum {
  LB_FP64 = 0,  /* populations, Q, phi stored and computed in float64        */
  LB_FP32 = 1,  /* stored and computed in float32                            */
  LB_FP16S = 2  /* populations stored as float16 (scaled by 64/w_i), Q and phi
                   float32, all arithmetic float32                            */
} lb_precision;

typedef enum {
  LB_D3Q19 = 0, /* D3Q19; the whole stress acts as a Guo body force F = div(sigma) */
  LB_D3Q15 = 1  /* the paper's scheme (Sec. 3): D3Q15 (Fig. 1), the symmetric
                   stress in the second moment of the equilibrium (Eqs. (9),
                   (11)), the antisymmetric stress as a Guo forcing term
                   (Eq. (10)); all three precisions, with its adjoint       */
} lb_lattice;

typedef enum {
  LB_FD_EULER2 = 0, /* explicit Euler, second-order central differences (D0, the
                       7-point Laplacian), central advection                   */
  LB_FD_PC4 = 1     /* the paper's integrator of Eqs. (1)-(2) (Sec. 3): Heun
                       predictor-corrector at the time-t velocity, first-order
                       upwind advection (donor-cell flux for phi), fourth-order
                       stencils in mu, H, grad u and the Laplacian of mu; the
                       LB stress and force keep the second-order stencils.
                       Stable where M*16*(f'' + 16 k_phi) < 2 (e.g. M = 0.05 with
                       the droplet parameters); with its adjoint               */
} lb_fd_scheme;

/* Model parameters (Eqs. (1)-(5), (7)).  K is the single elastic constant
 * K_Q of Eq. (5); Gamma is the rotational mobility multiplying H in the
 * Beris-Edwards update; xi the flow-alignment parameter; zeta the activity
 * (> 0 extensile).  chi(phi) = chi0 + chi_s*phi. */
typedef struct {
  int32_t nx, ny, nz;
  int32_t prec; /* lb_precision */
  double tau, rho0;
  double a, phi0, phi_cr, k_phi, M;
  double A0, chi0, chi_s, K, q0, W;
  double Gamma, xi, zeta;
  double body_force[3]; /* uniform external force density, added to F */
  int32_t lattice;      /* lb_lattice; 0 (a zero-initialised struct) = LB_D3Q19 */
  int32_t fd_scheme;    /* lb_fd_scheme; 0 = LB_FD_EULER2 */
} lb_params;

/* Global sums, accumulated in float64 on the device.  mass = N*rho0 + sum g;
 * momentum = sum rho*u (u with F/2); free_energy = F_h (Eq. (5) on the
 * lattice, forward differences in the squared-gradient terms); kinetic
 * energy = sum rho |u|^2 / 2. */
typedef struct {
  double mass;
  double momentum[3];
  double phi_total;
  double free_energy;
  double kinetic_energy;
  int64_t step;
} lb_totals;

typedef struct lb_ctx lb_ctx;

/* Create a context: validates p (tau > 0.5, n >= 3, finite values), allocates
 * the device state and uploads phi [N], q5 [5][N] and u0 [3][N] (NULL = 0).
 * The populations start at the second-order equilibrium of (rho0, u0).
 * Device memory: two buffers of populations, Q and phi, plus u and mu, i.e.
 * 2 (19 s_g + 6 s_f) + 4 s bytes per site (s_g, s_f, s: population, field and
 * arithmetic sizes; 232 B in LB_FP32).  lb_moments (rho, u), lb_free_energy
 * and the adjoint's recomputation allocate 14 s more per site on first use.
 * Errors: LB_EINVAL, LB_ENOMEM, LB_EDEVICE; *out is NULL on error. */
lb_status lb_init(const lb_params* p, const double* phi, const double* q5, const double* u0,
                  void* hip_stream, lb_ctx** out);

/* Launch configuration of a context, for tests and tuning.  lb_init uses the
 * defaults; lb_init_tuned with t = NULL, or with a zero-initialised struct,
 * reproduces them.  The configuration changes the launch shapes and, through
 * them, the floating-point rounding order, never the method.  The library
 * reads no environment variables. */
typedef enum {
  LB_PATH_DEFAULT = 0,      /* LB_PATH_TWO_LAUNCHES */
  LB_PATH_ONE_LAUNCH = 1,   /* the whole step in one z-marching kernel: Q, phi read once, u and
                               mu kept on chip, at the price of recomputing the stress on a
                               frame two sites wide and the moments of the tile's edge sites
                               (LB_FD_EULER2 only; slower than two launches on MI355X) */
  LB_PATH_TWO_LAUNCHES = 2, /* stress + collision kernel (writes u, mu), then the
                               order-parameter kernel (LB_FD_PC4: its four launches) */
  LB_PATH_SITE = 3          /* site-parallel kernels, the reference the tiled kernels are
                               tested against (adjoint only with LB_D3Q19 + LB_FD_EULER2) */
} lb_path;

typedef struct {
  int32_t path;          /* lb_path */
  int32_t lb_tile;       /* stress + collision kernel tile; 0 = default,
                            1..5 = 32x8, 32x16, 64x4, 16x16, 16x8 (float64: 32x16 -> 16x16) */
  int32_t order_tile;    /* order-parameter kernel tile; 0 = default,
                            1..5 = 32x8, 64x4, 32x16, 64x8, 64x16 (float64: 64x16 -> 64x8) */
  int32_t pc_tile;       /* LB_FD_PC4 stage kernel tile; 0 = default, 1..4 = 32x8, 32x16, 16x16, 64x8 */
  int32_t pcmu_tile;     /* LB_FD_PC4 mu kernel tile; same table as pc_tile */
  int32_t adj_tile;      /* stress + gather adjoint tile; 0 = default (32x16; float64 16x8),
                            1 = 32x8, 2 = 32x16 (float64: 16x8, 16x16) */
  int32_t adj_order_tile; /* order-parameter adjoint tile; 0 = default (float 32x16, float64 32x8),
                             1 = 32x8, 2 = 32x16 */
  int32_t step_tile;     /* one-launch kernel tile; 0 = default, 1..3 = 32x8, 32x16, 64x8
                            (float64: 32x8 only) */
  int32_t tz_step;       /* z-slab depths in planes, 0 = automatic: one-launch kernel, */
  int32_t tz_lb;         /* stress + collision kernel, */
  int32_t tz_order;      /* order-parameter kernel, */
  int32_t tz_pc;         /* LB_FD_PC4 stage kernel, */
  int32_t tz_pcmu;       /* LB_FD_PC4 mu kernel, */
  int32_t tz_adj;        /* fused stress + gather adjoint, */
  int32_t tz_adj_order;  /* order-parameter adjoint, */
  int32_t tz_pc_adj;     /* LB_FD_PC4 reverse product kernel */
  int32_t pc_adj;        /* LB_FD_PC4 reverse: 0 = default (one z-marching kernel per Heun
                            product where every tile along a split axis is at least two sites
                            wide, else the site-parallel kernels), 1 = site-parallel kernels */
} lb_tuning;

/* lb_init with an explicit launch configuration (t may be NULL).  Errors as
 * lb_init, plus LB_EINVAL for an unknown path or tile index, a negative slab
 * depth, pc_adj other than 0 or 1, or LB_PATH_ONE_LAUNCH with LB_FD_PC4. */
lb_status lb_init_tuned(const lb_params* p, const lb_tuning* t, const double* phi, const double* q5,
                        const double* u0, void* hip_stream, lb_ctx** out);

/* Enqueue nsteps coupled steps on the context's stream (nsteps >= 0).  One
 * step: mu and H of the Eq. (5) free energy, the stress of Eqs. (3)-(4), the
 * BGK collision with its forcing and the pull stream (Eqs. (6)-(8), (10)-(11)),
 * the Q update of Eq. (2) and the phi update of Eq. (1). */
lb_status lb_step(lb_ctx* c, int32_t nsteps);

/* Replace the model parameters that do not change the allocation (every
 * field except nx, ny, nz, prec, which must match).  Errors: LB_EINVAL. */
lb_status lb_set_params(lb_ctx* c, const lb_params* p);

/* Copy rho [N], u [3][N] (with F/2), phi [N] and q5 [5][N] at the current
 * time to host float64 arrays; any pointer may be NULL.  rho and u are the
 * moments of Eq. (8), u with half the force of the stress of Eqs. (3)-(4) in
 * the forcing form of Eq. (10).  Synchronises.
 * Errors: LB_ENOMEM when device scratch for rho, u cannot be allocated. */
lb_status lb_moments(lb_ctx* c, double* rho, double* u3, double* phi, double* q5);

/* Post-stream population deviations g [Q][N] at the current time (float64
 * host array; Q = 19 for LB_D3Q19, 15 for LB_D3Q15, in the velocity order of
 * the lattice).  Synchronises. */
lb_status lb_populations(lb_ctx* c, double* g19);

/* Overwrite the state at the current time from host float64 arrays:
 * g19 [Q][N] post-stream deviations (Q as in lb_populations), phi [N],
 * q5 [5][N] (NULL = keep). */
lb_status lb_set_fields(lb_ctx* c, const double* g19, const double* phi, const double* q5);

/* Global float64 sums of the current state (see lb_totals).  Returns
 * LB_ENONFINITE if any of them is not finite, LB_ENOMEM if device scratch
 * cannot be allocated.  Synchronises. */
lb_status lb_free_energy(lb_ctx* c, lb_totals* out);

/* phi-weighted droplet centre.  out[0..2] = linear centre (x, y, z) with
 * coordinates in [0, n); out[3..5] = circular-mean centre per axis,
 * n/(2 pi) atan2(sum phi sin(2 pi x/n), sum phi cos(2 pi x/n)) in [0, n);
 * *phi_total = sum phi.  float64 device sums.  Synchronises. */
lb_status lb_centre(lb_ctx* c, double out[6], double* phi_total);

/* Allocation-free variant of lb_centre, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Computes the centre of lb_centre (same kernels, same
 * fixed-order float64 sums) from a caller-owned device array without a
 * context, and allocates nothing.
 *   nx, ny, nz  periodic box, each >= 1, N = nx*ny*nz <= LB_NOALLOC_MAX_SITES
 *               (2^25; larger boxes return LB_EINVAL before any work)
 *   prec        LB_FP64: dev_phi is float64; LB_FP32 or LB_FP16S: float32
 *   dev_phi     [N] concentration, [z][y][x] with x fastest (caller-owned)
 *   dev_out     7 float64 on the device (caller-owned): linear centre (x, y, z),
 *               circular-mean centre (x, y, z) in [0, n), sum phi
 *   hip_stream  stream the work is enqueued on (NULL = default stream)
 * The call only enqueues work and does not synchronise.  Its block partials
 * live in one static device array of LB_NOALLOC_SCRATCH_BYTES per GPU, held
 * until the process ends; every call on a GPU shares it and nothing in it
 * needs clearing between calls.  Calls that overlap on one GPU (several
 * streams or host threads) race on that array: order them.  dev_phi, dev_out
 * and the stream must belong to the current device.
 * Errors: LB_EINVAL (box, precision, null pointer), LB_EDEVICE. */
#define LB_NOALLOC_MAX_SITES (1 << 25)
#define LB_NOALLOC_SCRATCH_BYTES (11u << 20)
lb_status lb_centre_noalloc(int32_t nx, int32_t ny, int32_t nz, int32_t prec, const void* dev_phi,
                            double* dev_out, void* hip_stream);

/* Size in bytes of the opaque state buffer (populations, Q, phi in storage
 * precision, plus the step counter). */
size_t lb_state_bytes(const lb_ctx* c);

/* Copy the state to / from a caller-owned device buffer of lb_state_bytes()
 * bytes (checkpoint / resume; resuming is bitwise identical).  Ordered on the
 * context's stream.  Errors: LB_ESTATE on a size mismatch. */
lb_status lb_get_state(lb_ctx* c, void* dev_dst, size_t bytes);
lb_status lb_set_state(lb_ctx* c, const void* dev_src, size_t bytes);

/* ---------------------------------------------------------------------------
 * Adjoint (reverse mode) of the coupled step.
 *
 * The adjoint of a state is a device buffer of lb_adjoint_bytes() bytes in the
 * context's arithmetic type (double for LB_FP64, float otherwise), laid out
 * as g_bar [Q][N] (adjoint of the post-stream population deviations; Q = 19
 * for LB_D3Q19, 15 for LB_D3Q15), q_bar [5][N] (adjoint of the 5 stored Q
 * components) and phi_bar [N].  The caller owns it (e.g. a torch tensor on
 * the context's device).  On LB_D3Q15 the reverse of the collision also
 * carries the adjoint of the symmetric stress in the equilibrium (Eq. (9))
 * into the stress; the force is the divergence of the antisymmetric part only
 * (Eq. (10)).
 * The adjoint covers both lattices and both integrators (on LB_FD_PC4 it is
 * the reverse of Heun's two stages, Sec. 3).  Only when the library runs its
 * site-parallel test kernels (LB_PATH_SITE) is it limited to LB_D3Q19
 * with LB_FD_EULER2: there, for the other schemes, lb_adjoint_bytes,
 * lb_record_bytes and lb_lean_record_bytes return 0 and the calls below
 * return LB_EINVAL.
 * ------------------------------------------------------------------------- */
size_t lb_adjoint_bytes(const lb_ctx* c);

/* Size of a step record: u [3][N], F [3][N] and drho [N] (the velocity with
 * F/2, the force of Eq. (3) and rho - rho0 = sum g) of one time t, in the
 * context's arithmetic type; with LB_FD_PC4 followed by the predictor stage
 * X* = (Q* [5][N], phi* [N]) of that step in the storage type, which the
 * reverse of the step then reads instead of recomputing it. */
size_t lb_record_bytes(const lb_ctx* c);

/* One forward step from the state buffer dev_state_in (time t, lb_get_state
 * format) into dev_state_out (time t+1, a different buffer), writing u, F and
 * drho of time t into dev_rec_out.  The context's own state is not touched.  This is
 * the replay of a checkpoint segment before its reverse steps.  dev_state_out
 * may be NULL: then only the record is written (the last step of a replayed
 * segment, whose output state the reverse never reads), and the populations
 * and order parameters of t+1 are not formed. */
lb_status lb_step_record(lb_ctx* c, const void* dev_state_in, void* dev_state_out, void* dev_rec_out,
                         size_t state_bytes, size_t rec_bytes);

/* One reverse step: dev_adj_out <- (d step / d state_t)^T dev_adj_in, the
 * vector-Jacobian product of one coupled step at the forward state dev_state_t
 * with the context's current parameters.  dev_rec_t is that step's record
 * from lb_step_record (NULL: u and F are recomputed and the collision's
 * reverse reads the populations of dev_state_t; with a record it reads drho
 * and u from it).  adj_in and adj_out must differ.
 * The step's contributions to dL/dzeta and dL/dq0 are summed in float64 on
 * the device and kept there across calls.  When zeta_bar or q0_bar is
 * non-NULL, every contribution kept since the last such call (this one's
 * included) is added to *zeta_bar and *q0_bar (a NULL one is dropped), the
 * device sums are cleared, and the call synchronises the stream.  With both
 * NULL the call only enqueues work, so a reverse sweep passes pointers on its
 * last step only.
 * Errors: LB_ESTATE on a buffer size mismatch, LB_EINVAL, LB_EDEVICE. */
lb_status lb_adjoint_step(lb_ctx* c, const void* dev_state_t, size_t state_bytes, const void* dev_rec_t,
                          size_t rec_bytes, const void* dev_adj_in, void* dev_adj_out, size_t adj_bytes,
                          double* zeta_bar, double* q0_bar);

/* Size of a lean step record: Q [5][N] and phi [N] of time t in the storage
 * type, then drho [N] (the sum of the population deviations), u [3][N] and
 * F [3][N] of the step from t, in the arithmetic type, and with LB_FD_PC4 the
 * predictor stage Q* [5][N], phi* [N] (storage type); each part starts on a
 * 256-byte boundary (about 52 B per site in float32, 76 B with LB_FD_PC4).  The populations enter
 * the collision only through drho and u, so a lean record holds everything
 * the reverse of its step reads: a reverse sweep over lean records needs no
 * state buffers and no replay. */
size_t lb_lean_record_bytes(const lb_ctx* c);

/* Record the context's current time t into dev_rec_out (lean format) and
 * advance the context's own state by one step, as lb_step(c, 1) does.
 * Errors: LB_ESTATE on a size mismatch, LB_EINVAL (incl. a scheme without
 * adjoint), LB_EDEVICE. */
lb_status lb_step_record_lean(lb_ctx* c, void* dev_rec_out, size_t rec_bytes);

/* One reverse step of the step recorded in dev_rec_t (lean format); the
 * adjoint buffers and the parameter sums behave as in lb_adjoint_step. */
lb_status lb_adjoint_step_lean(lb_ctx* c, const void* dev_rec_t, size_t rec_bytes, const void* dev_adj_in,
                               void* dev_adj_out, size_t adj_bytes, double* zeta_bar, double* q0_bar);

/* Seed of the droplet-displacement loss L = (z_c - z_ref)^2 with z_c the
 * phi-weighted linear centre along z of the current state (the loss of a
 * differentiable rollout).  Writes dL/d(state) into dev_adj and L into *loss. */
lb_status lb_adjoint_seed_centre(lb_ctx* c, double z_ref, void* dev_adj, size_t adj_bytes, double* loss);

/* Average device time per launch of each kernel of the step, measured with
 * HIP events recorded on the context's stream around every launch of
 * nsteps steps (the state advances by nsteps).  kernel_ms must hold
 * LB_MAX_KERNELS entries; *count receives the number of kernels per step. */
#define LB_MAX_KERNELS 8
lb_status lb_profile_step(lb_ctx* c, int32_t nsteps, double* kernel_ms, int32_t* count);

/* Name of kernel i of the step (as it appears in a kernel trace), or NULL. */
const char* lb_kernel_name(const lb_ctx* c, int32_t i);

/* Block until the context's stream is idle. */
lb_status lb_sync(lb_ctx* c);

/* Free the context (NULL-safe). */
void lb_destroy(lb_ctx* c);

/* Thread-local message of the last failing call ("" if none). */
const char* lb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LB_CHIRAL_H */
