// Host-side check of the per-site reverse derivatives in adjoint.hpp against
// central differences of the forward functions in physics.hpp (float64).
// For random inputs x, output weights v and input direction d it compares
// <v, (f(x + h d) - f(x - h d)) / 2h> with <J^T v, d> from the *_bwd code.
// Prints one line per check and exits nonzero on failure.
#include <cmath>
#include <cstdio>
#include <random>

#include "adjoint.hpp"

using namespace lbc;
using R = double;

static std::mt19937_64 rng(1234);
static double U(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

static Params<R> params() {
  Params<R> P;
  P.omega = 1.0 / 2.5;
  P.guo = 1.0 - 0.5 / 2.5;
  P.rho0 = 1.0;
  P.a = 0.07; P.phi0 = 2.0; P.inv_phicr2 = 1.0; P.k_phi = 0.1; P.M = 0.1;
  P.A0 = 1.0; P.chi0 = 2.4; P.chi_s = 0.3; P.K = 0.02; P.q0 = 0.7; P.W = 0.02;
  P.Gamma = 0.3; P.xi = 0.7; P.zeta = 0.01;
  P.bf[0] = P.bf[1] = P.bf[2] = 0.0;
  return P;
}

static void rand_grad(Grad<R>& G) {
  G.phi = U(0.2, 1.9);
  for (int g = 0; g < 3; ++g) G.dphi[g] = U(-0.5, 0.5);
  G.lapphi = U(-0.5, 0.5);
  G.divv = U(-0.5, 0.5);
  for (int k = 0; k < 5; ++k) {
    G.q[k] = U(-0.3, 0.3);
    G.lapq[k] = U(-0.2, 0.2);
    for (int g = 0; g < 3; ++g) G.dq[g][k] = U(-0.2, 0.2);
  }
}

// flatten Grad into 31 values (phi, dphi, lapphi, divv, q, dq, lapq)
static void flat(const Grad<R>& G, double* v) {
  int n = 0;
  v[n++] = G.phi;
  for (int g = 0; g < 3; ++g) v[n++] = G.dphi[g];
  v[n++] = G.lapphi;
  v[n++] = G.divv;
  for (int k = 0; k < 5; ++k) v[n++] = G.q[k];
  for (int g = 0; g < 3; ++g)
    for (int k = 0; k < 5; ++k) v[n++] = G.dq[g][k];
  for (int k = 0; k < 5; ++k) v[n++] = G.lapq[k];
}
static void unflat(const double* v, Grad<R>& G) {
  int n = 0;
  G.phi = v[n++];
  for (int g = 0; g < 3; ++g) G.dphi[g] = v[n++];
  G.lapphi = v[n++];
  G.divv = v[n++];
  for (int k = 0; k < 5; ++k) G.q[k] = v[n++];
  for (int g = 0; g < 3; ++g)
    for (int k = 0; k < 5; ++k) G.dq[g][k] = v[n++];
  for (int k = 0; k < 5; ++k) G.lapq[k] = v[n++];
}
static void flatb(const GradBar<R>& G, double* v) {
  int n = 0;
  v[n++] = G.phi;
  for (int g = 0; g < 3; ++g) v[n++] = G.dphi[g];
  v[n++] = G.lapphi;
  v[n++] = G.divv;
  for (int k = 0; k < 5; ++k) v[n++] = G.q[k];
  for (int g = 0; g < 3; ++g)
    for (int k = 0; k < 5; ++k) v[n++] = G.dq[g][k];
  for (int k = 0; k < 5; ++k) v[n++] = G.lapq[k];
}

static int failures = 0;
static void report(const char* name, double fd, double ad) {
  const double err = std::fabs(fd - ad) / std::fmax(1e-12, std::fabs(fd) + std::fabs(ad));
  const bool ok = err < 1e-7;
  std::printf("%-28s fd % .12e  adj % .12e  rel %.2e %s\n", name, fd, ad, err, ok ? "ok" : "FAIL");
  if (!ok) ++failures;
}

static void check_sigma(int trial) {
  Params<R> P = params();
  Grad<R> G;
  rand_grad(G);
  double v[15], d[31], x[31];
  for (double& t : v) t = U(-1, 1);
  for (double& t : d) t = U(-1, 1);
  flat(G, x);
  // v: cotangents of sigma (9), H (5) and mu at the site (1)
  auto f = [&](const Grad<R>& g, const Params<R>& p) {
    R sig[9], h[5];
    sigma_site(p, g, sig, h);
    double s = 0;
    for (int k = 0; k < 9; ++k) s += v[k] * sig[k];
    for (int k = 0; k < 5; ++k) s += v[9 + k] * h[k];
    return s + v[14] * mu_site(p, g.phi, g.lapphi, g.divv, g.q);
  };
  const double hstep = 1e-6;
  double xp[31], xm[31];
  for (int i = 0; i < 31; ++i) { xp[i] = x[i] + hstep * d[i]; xm[i] = x[i] - hstep * d[i]; }
  Grad<R> Gp, Gm;
  unflat(xp, Gp);
  unflat(xm, Gm);
  const double fd = (f(Gp, P) - f(Gm, P)) / (2 * hstep);
  GradBar<R> Gb;
  Gb.zero();
  ParBar<R> Pb{0, 0, 0};
  sigma_site_bwd(P, G, v, v + 9, Gb, Pb, v[14]);
  double gb[31];
  flatb(Gb, gb);
  double ad = 0;
  for (int i = 0; i < 31; ++i) ad += gb[i] * d[i];
  char name[64];
  std::snprintf(name, sizeof name, "sigma+h+mu wrt G #%d", trial);
  report(name, fd, ad);
  // parameters: zeta and q0
  Params<R> pp = P, pm = P;
  pp.zeta += hstep; pm.zeta -= hstep;
  report("sigma+h wrt zeta", (f(G, pp) - f(G, pm)) / (2 * hstep), Pb.zeta);
  pp = P; pm = P;
  pp.q0 += hstep; pm.q0 -= hstep;
  report("sigma+h wrt q0", (f(G, pp) - f(G, pm)) / (2 * hstep), 2 * P.K * Pb.kq + 8 * P.K * P.q0 * Pb.kq2);
}

static void check_mu() {
  Params<R> P = params();
  Grad<R> G;
  rand_grad(G);
  const double v = U(-1, 1);
  double d[8];
  for (double& t : d) t = U(-1, 1);
  auto f = [&](double phi, double lp, double dv, const R* q) { return v * mu_site(P, phi, lp, dv, q); };
  const double h = 1e-6;
  R qp[5], qm[5];
  for (int k = 0; k < 5; ++k) { qp[k] = G.q[k] + h * d[3 + k]; qm[k] = G.q[k] - h * d[3 + k]; }
  const double fd = (f(G.phi + h * d[0], G.lapphi + h * d[1], G.divv + h * d[2], qp) -
                     f(G.phi - h * d[0], G.lapphi - h * d[1], G.divv - h * d[2], qm)) / (2 * h);
  R phib = 0, lpb = 0, dvb = 0, qb[5] = {0, 0, 0, 0, 0};
  mu_site_bwd(P, G.phi, G.q, v, phib, lpb, dvb, qb);
  double ad = phib * d[0] + lpb * d[1] + dvb * d[2];
  for (int k = 0; k < 5; ++k) ad += qb[k] * d[3 + k];
  report("mu wrt phi, lap, divv, q", fd, ad);
}

static void check_corotation() {
  R q[5], W[3][3], v[5], dq[5], dW[3][3];
  for (int k = 0; k < 5; ++k) { q[k] = U(-0.3, 0.3); v[k] = U(-1, 1); dq[k] = U(-1, 1); }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) { W[a][b] = U(-0.05, 0.05); dW[a][b] = U(-1, 1); }
  const double xi = 0.7, h = 1e-6;
  auto f = [&](double s) {
    R qq[5], WW[3][3], out[5];
    for (int k = 0; k < 5; ++k) qq[k] = q[k] + s * dq[k];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) WW[a][b] = W[a][b] + s * dW[a][b];
    corotation_site(xi, qq, WW, out);
    double r = 0;
    for (int k = 0; k < 5; ++k) r += v[k] * out[k];
    return r;
  };
  const double fd = (f(h) - f(-h)) / (2 * h);
  R qb[5] = {0, 0, 0, 0, 0}, Wb[3][3] = {};
  corotation_site_bwd(xi, q, W, v, qb, Wb);
  double ad = 0;
  for (int k = 0; k < 5; ++k) ad += qb[k] * dq[k];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) ad += Wb[a][b] * dW[a][b];
  report("corotation wrt q, W", fd, ad);
}

static void check_collide() {
  Params<R> P = params();
  R g[19], F[3], vg[19], vu[3], dg[19], dF[3];
  for (int i = 0; i < 19; ++i) { g[i] = U(-2e-2, 2e-2); vg[i] = U(-1, 1); dg[i] = U(-1, 1); }
  for (int a = 0; a < 3; ++a) { F[a] = U(-1e-2, 1e-2); vu[a] = U(-1, 1); dF[a] = U(-1, 1); }
  const double h = 1e-6;
  auto f = [&](double s) {
    R gg[19], FF[3], u[3];
    for (int i = 0; i < 19; ++i) gg[i] = g[i] + s * dg[i];
    for (int a = 0; a < 3; ++a) FF[a] = F[a] + s * dF[a];
    collide_site(P, gg, FF, u);
    double r = 0;
    for (int i = 0; i < 19; ++i) r += vg[i] * gg[i];
    for (int a = 0; a < 3; ++a) r += vu[a] * u[a];
    return r;
  };
  const double fd = (f(h) - f(-h)) / (2 * h);
  R gb[19], Fb[3] = {0, 0, 0};
  collide_site_bwd(P, g, F, vg, vu, gb, Fb);
  double ad = 0;
  for (int i = 0; i < 19; ++i) ad += gb[i] * dg[i];
  for (int a = 0; a < 3; ++a) ad += Fb[a] * dF[a];
  report("collide wrt g, F", fd, ad);
}

// the paper's D3Q15 collision with the symmetric stress in the equilibrium
static void check_collide_eq() {
  Params<R> P = params();
  R g[15], F[3], S[6], vg[15], vu[3], dg[15], dF[3], dS[6];
  for (int i = 0; i < 15; ++i) { g[i] = U(-2e-2, 2e-2); vg[i] = U(-1, 1); dg[i] = U(-1, 1); }
  for (int a = 0; a < 3; ++a) { F[a] = U(-1e-2, 1e-2); vu[a] = U(-1, 1); dF[a] = U(-1, 1); }
  for (int k = 0; k < 6; ++k) { S[k] = U(-1e-2, 1e-2); dS[k] = U(-1, 1); }
  const double h = 1e-6;
  auto f = [&](double s) {
    R gg[15], FF[3], SS[6], u[3];
    for (int i = 0; i < 15; ++i) gg[i] = g[i] + s * dg[i];
    for (int a = 0; a < 3; ++a) FF[a] = F[a] + s * dF[a];
    for (int k = 0; k < 6; ++k) SS[k] = S[k] + s * dS[k];
    collide_site_eq(P, gg, FF, SS, u);
    double r = 0;
    for (int i = 0; i < 15; ++i) r += vg[i] * gg[i];
    for (int a = 0; a < 3; ++a) r += vu[a] * u[a];
    return r;
  };
  const double fd = (f(h) - f(-h)) / (2 * h);
  R gb[15], Fb[3] = {0, 0, 0}, Sb[6] = {0, 0, 0, 0, 0, 0};
  collide_eq_site_bwd(P, g, F, vg, vu, gb, Fb, Sb);
  double ad = 0;
  for (int i = 0; i < 15; ++i) ad += gb[i] * dg[i];
  for (int a = 0; a < 3; ++a) ad += Fb[a] * dF[a];
  for (int k = 0; k < 6; ++k) ad += Sb[k] * dS[k];
  report("D3Q15 collide wrt g, F, S", fd, ad);
}

int main() {
  for (int t = 0; t < 4; ++t) check_sigma(t);
  for (int t = 0; t < 3; ++t) check_mu();
  for (int t = 0; t < 3; ++t) check_corotation();
  for (int t = 0; t < 3; ++t) check_collide();
  for (int t = 0; t < 3; ++t) check_collide_eq();
  std::printf("%s\n", failures ? "FAILED" : "ALL OK");
  return failures ? 1 : 0;
}
