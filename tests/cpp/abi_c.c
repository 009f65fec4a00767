/* A plain C consumer of the library: only include/lb_chiral.h and the shared
 * library, no Python and no HIP headers.  Runs on the GPU:
 *   1. a uniform body force f on a fluid without order parameters (Q = 0,
 *      phi = 0) in float64, on both lattices: the total momentum (u with F/2)
 *      is N f (t + 1/2) exactly after t steps;
 *   2. a small chiral droplet in float64 and float32: mass and sum(phi) are
 *      conserved over 50 steps, the step counter advances;
 *   3. error paths: invalid parameters, unknown or unsupported lattices and
 *      integrators, negative step counts, NULL contexts, shape, lattice or
 *      integrator changes.
 * Prints "C ABI OK" and exits 0 when every check holds. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lb_chiral.h"

static const double kPi = 3.14159265358979323846;
static int failures = 0;

#define CHECK(cond, ...)                    \
  do {                                      \
    if (!(cond)) {                          \
      printf("FAIL %s:%d: ", __FILE__, __LINE__); \
      printf(__VA_ARGS__);                  \
      printf("\n");                         \
      ++failures;                           \
    }                                       \
  } while (0)

static lb_params base_params(int nx, int ny, int nz, int prec) {
  lb_params p;
  memset(&p, 0, sizeof p);
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.prec = prec;
  p.tau = 2.5;
  p.rho0 = 1.0;
  p.a = 0.07;
  p.phi0 = 2.0;
  p.phi_cr = 1.0;
  p.k_phi = 0.1;
  p.M = 0.1;
  p.A0 = 1.0;
  p.chi0 = 2.4;
  p.chi_s = 0.3;
  p.K = 0.02;
  p.q0 = 2.0 * kPi / 8.0;
  p.W = 0.02;
  p.Gamma = 0.3;
  p.xi = 0.7;
  p.zeta = 0.01;
  return p;
}

static void body_force_case(int lattice) {
  const int nx = 9, ny = 7, nz = 6, N = nx * ny * nz;
  lb_params p = base_params(nx, ny, nz, LB_FP64);
  p.lattice = lattice;
  p.zeta = 0.0;
  p.body_force[0] = 1e-6;
  p.body_force[2] = -3e-7;
  double* phi = calloc(N, sizeof(double));
  double* q5 = calloc(5 * (size_t)N, sizeof(double));
  lb_ctx* c = NULL;
  lb_status st = lb_init(&p, phi, q5, NULL, NULL, &c);
  CHECK(st == LB_OK && c, "lb_init: %d %s", st, lb_last_error());
  if (c) {
    const int t = 25;
    CHECK(lb_step(c, t) == LB_OK, "lb_step");
    lb_totals tot;
    CHECK(lb_free_energy(c, &tot) == LB_OK, "lb_free_energy: %s", lb_last_error());
    for (int a = 0; a < 3; ++a) {
      const double want = N * p.body_force[a] * (t + 0.5);
      const double got = tot.momentum[a];
      CHECK(fabs(got - want) <= 1e-12 * fabs(N * 1e-6 * t), "momentum[%d] %.17g vs %.17g", a, got, want);
    }
    CHECK(fabs(tot.mass - N * p.rho0) <= 1e-12 * N, "mass %.17g", tot.mass);
    CHECK(tot.step == t, "step %lld", (long long)tot.step);
    lb_destroy(c);
  }
  free(phi);
  free(q5);
}

static void droplet_case(int prec, double tol) {
  const int nx = 16, ny = 14, nz = 12, N = nx * ny * nz;
  lb_params p = base_params(nx, ny, nz, prec);
  double* phi = malloc(sizeof(double) * N);
  double* q5 = calloc(5 * (size_t)N, sizeof(double));
  const double R = 4.5;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int s = (z * ny + y) * nx + x;
        const double dx = x - nx / 2.0, dy = y - ny / 2.0, dz = z - nz / 2.0;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        phi[s] = 0.5 * p.phi0 * (1.0 + tanh(R - r));
        if (phi[s] > p.phi_cr) { /* helix n = (cos q0 z, sin q0 z, 0), S = 0.5 */
          const double cz = cos(p.q0 * z), sz = sin(p.q0 * z), S = 0.5;
          q5[0 * (size_t)N + s] = S * (cz * cz - 1.0 / 3.0);
          q5[1 * (size_t)N + s] = S * cz * sz;
          q5[3 * (size_t)N + s] = S * (sz * sz - 1.0 / 3.0);
        }
      }
  lb_ctx* c = NULL;
  CHECK(lb_init(&p, phi, q5, NULL, NULL, &c) == LB_OK && c, "lb_init: %s", lb_last_error());
  if (c) {
    lb_totals t0, t1;
    CHECK(lb_free_energy(c, &t0) == LB_OK, "totals 0: %s", lb_last_error());
    CHECK(lb_step(c, 50) == LB_OK, "lb_step");
    CHECK(lb_sync(c) == LB_OK, "lb_sync");
    CHECK(lb_free_energy(c, &t1) == LB_OK, "totals 1: %s", lb_last_error());
    CHECK(fabs(t1.mass - t0.mass) <= tol * t0.mass, "mass %.17g -> %.17g", t0.mass, t1.mass);
    CHECK(fabs(t1.phi_total - t0.phi_total) <= tol * t0.phi_total, "sum phi %.17g -> %.17g", t0.phi_total,
          t1.phi_total);
    CHECK(t1.step == 50, "step %lld", (long long)t1.step);
    double centre[6], ptot = 0.0;
    CHECK(lb_centre(c, centre, &ptot) == LB_OK, "lb_centre");
    CHECK(fabs(centre[2] - nz / 2.0) < 0.5, "centre z %.6f", centre[2]);
    double* rho = malloc(sizeof(double) * N);
    CHECK(lb_moments(c, rho, NULL, NULL, NULL) == LB_OK, "lb_moments");
    double sum = 0.0;
    for (int s = 0; s < N; ++s) sum += rho[s];
    CHECK(fabs(sum - t1.mass) <= 1e-6 * t1.mass, "sum rho %.17g vs mass %.17g", sum, t1.mass);
    free(rho);
    lb_destroy(c);
  }
  free(phi);
  free(q5);
}

static void error_paths(void) {
  double phi[4 * 4 * 4] = {0}, q5[5 * 4 * 4 * 4] = {0};
  lb_params p = base_params(4, 4, 4, LB_FP32);
  p.tau = 0.4;
  lb_ctx* c = (lb_ctx*)1;
  CHECK(lb_init(&p, phi, q5, NULL, NULL, &c) == LB_EINVAL && c == NULL, "tau <= 1/2 accepted");
  CHECK(strlen(lb_last_error()) > 0, "empty error message");
  p = base_params(2, 4, 4, LB_FP32);
  CHECK(lb_init(&p, phi, q5, NULL, NULL, &c) == LB_EINVAL, "n < 3 accepted");
  p = base_params(4, 4, 4, 7);
  CHECK(lb_init(&p, phi, q5, NULL, NULL, &c) == LB_EINVAL, "unknown precision accepted");
  p = base_params(4, 4, 4, LB_FP32);
  p.lattice = 3;
  CHECK(lb_init(&p, phi, q5, NULL, NULL, &c) == LB_EINVAL, "unknown lattice accepted");
  p = base_params(4, 4, 4, LB_FP16S);
  p.lattice = LB_D3Q15;
  CHECK(lb_init(&p, phi, q5, NULL, NULL, &c) == LB_OK && c, "float16 storage on D3Q15: %s", lb_last_error());
  lb_destroy(c);
  c = NULL;
  p = base_params(4, 4, 4, LB_FP32);
  p.fd_scheme = 2;
  CHECK(lb_init(&p, phi, q5, NULL, NULL, &c) == LB_EINVAL, "unknown integrator accepted");
  p = base_params(4, 4, 4, LB_FP32);
  CHECK(lb_init(&p, phi, q5, NULL, NULL, &c) == LB_OK && c, "lb_init: %s", lb_last_error());
  CHECK(lb_step(c, -1) == LB_EINVAL, "negative step count accepted");
  CHECK(lb_step(NULL, 1) == LB_EINVAL, "NULL context accepted");
  lb_params q = p;
  q.nx = 5;
  CHECK(lb_set_params(c, &q) == LB_EINVAL, "shape change accepted");
  q = p;
  q.lattice = LB_D3Q15;
  CHECK(lb_set_params(c, &q) == LB_EINVAL, "lattice change accepted");
  q = p;
  q.fd_scheme = LB_FD_PC4;
  CHECK(lb_set_params(c, &q) == LB_EINVAL, "integrator change accepted");
  lb_destroy(c);
  lb_destroy(NULL);
}

int main(void) {
  body_force_case(LB_D3Q19);
  body_force_case(LB_D3Q15);
  droplet_case(LB_FP64, 1e-12);
  droplet_case(LB_FP32, 1e-6);
  error_paths();
  if (failures) {
    printf("%d check(s) failed\n", failures);
    return 1;
  }
  printf("C ABI OK\n");
  return 0;
}
