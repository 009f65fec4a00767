/* C ABI of the two-dimensional bulk active nematic (D2Q9 lattice Boltzmann
 * coupled to a 2x2 Q tensor): the 2D counterpart of the coupled step, for the
 * activity regimes of the paper's Fig. 4 (quiescent, spontaneous flow,
 * chaotic) and its 2D workload of Fig. 3.
 *
 * Model (per step, units dx = dt = 1, periodic nx x ny box, arrays [c][y][x]
 * with x fastest):
 *   Q = [[Q_xx, Q_xy], [Q_xy, -Q_xx]], stored as q2[2][ny][nx];
 *   H = -A0 (1 - chi/3) Q - A0 chi tr(Q^2) Q + K lap Q   (Eq. (5) in 2D, no phi);
 *   sigma = f I - 2K (grad Q_xx grad Q_xx + grad Q_xy grad Q_xy) - xi H
 *           + 2 xi (Q:H) Q + (Q H - H Q) - zeta Q          (Eqs. (3)-(4) in 2D);
 *   F = D0 . sigma + body force; D2Q9 BGK with Guo forcing (Eqs. (6)-(8), (10)-(11));
 *   Q(t+1) = Q + [-u.D0 Q + S + Gamma H]                  (Eq. (2), explicit Euler),
 * with second-order central differences and the 5-point Laplacian.  Status
 * codes and precisions are those of lb_chiral.h (LB_FP64 or LB_FP32 only).
 * All host arrays are float64 and owned by the caller; a context is used from
 * one thread at a time.  Errors leave the context unchanged; the message of
 * the last error of the calling thread is lb2d_last_error(). */
#ifndef LB_NEMATIC2D_H
#define LB_NEMATIC2D_H

#include <stdint.h>

#include "lb_chiral.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t nx, ny;   /* box, each >= 3, nx * ny <= 2^28 */
  int32_t prec;     /* LB_FP64 or LB_FP32 (storage and arithmetic) */
  double tau, rho0; /* BGK relaxation time (> 1/2) and rest density */
  double A0, chi;   /* bulk: nematic for chi > 3, S_eq = sqrt(2 (chi/3 - 1)/chi) */
  double K;         /* elastic constant */
  double Gamma, xi; /* rotational mobility, flow-alignment parameter */
  double zeta;      /* activity (> 0 extensile) */
  double body_force[2];
} lb2d_params;

typedef struct {
  double mass;           /* N rho0 + sum g */
  double momentum[2];    /* sum rho u (u with F/2) */
  double free_energy;    /* F_h, forward differences in the gradient term */
  double kinetic_energy; /* sum rho |u|^2 / 2 */
  int64_t step;
} lb2d_totals;

typedef struct lb2d_ctx lb2d_ctx;

/* New context: Q from q2 [2][ny][nx], populations at the second-order
 * equilibrium of (rho0, u0) (u0 [2][ny][nx], NULL = at rest).  stream: a
 * hipStream_t (NULL = default stream).  LB_EINVAL for invalid parameters,
 * LB_ENOMEM when the device cannot hold the state (2 x 9 + 2 x 2 + 2 values
 * per site). */
lb_status lb2d_init(const lb2d_params* p, const double* q2, const double* u0, void* stream, lb2d_ctx** out);

/* Enqueue nsteps (>= 0) coupled steps on the context's stream. */
lb_status lb2d_step(lb2d_ctx* c, int32_t nsteps);

/* Synchronise the context's stream. */
lb_status lb2d_sync(lb2d_ctx* c);

/* rho [ny][nx], u [2][ny][nx] (with F/2) and q2 [2][ny][nx] at the current
 * time; any pointer may be NULL.  Synchronises. */
lb_status lb2d_moments(lb2d_ctx* c, double* rho, double* u, double* q2);

/* Post-stream population deviations g_i = f_i - w_i rho0 at the current time,
 * g9 [9][ny][nx] in the order rest, +x, -x, +y, -y, (+,+), (-,-), (+,-), (-,+). */
lb_status lb2d_populations(lb2d_ctx* c, double* g9);

/* Replace the populations (g9 [9][ny][nx] post-stream deviations) and / or Q
 * (q2 [2][ny][nx]); NULL leaves that field. */
lb_status lb2d_set_fields(lb2d_ctx* c, const double* g9, const double* q2);

/* Global sums in float64 (summed in a fixed order on the host). */
lb_status lb2d_free_energy(lb2d_ctx* c, lb2d_totals* t);

/* Average ms per launch of each kernel of the step over nsteps steps (the
 * state advances); kernel_ms has room for 4 entries. */
lb_status lb2d_profile_step(lb2d_ctx* c, int32_t nsteps, double* kernel_ms, int32_t* count);
const char* lb2d_kernel_name(const lb2d_ctx* c, int32_t i);

void lb2d_destroy(lb2d_ctx* c);
const char* lb2d_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
