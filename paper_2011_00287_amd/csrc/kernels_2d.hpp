// Two-dimensional bulk active nematic on D2Q9: the 2D coupled step of the
// activity regimes of Fig. 4 (quiescent, spontaneous flow, chaotic).
//
// Q is the 2x2 traceless symmetric tensor [[a, b], [b, -a]], stored as
// (Q_xx, Q_xy) = (a, b).  Free energy: bulk A0/2 (1 - chi/3) tr Q^2 +
// A0 chi/4 (tr Q^2)^2 (no cubic invariant in 2D) and K/2 |grad Q|^2, so
//   H = -A0 (1 - chi/3) Q - A0 chi tr(Q^2) Q + K lap Q.
// Stress (index a = force component, b = derivative index):
//   f delta - 2K (D0_a a D0_b a + D0_a b D0_b b) - xi H + 2 xi (Q:H) Q
//   + (Q H - H Q) - zeta Q,
// the 2D form of the Beris-Edwards reactive stress with P = Q + I/2 (in 2D
// Q H + H Q = (Q:H) I, so -xi (H P + P H) + 2 xi P (Q:H) = -xi H + 2 xi (Q:H) Q).
// LB: D2Q9 (rest, +-x, +-y, (+,+)/(-,-), (+,-)/(-,+)), BGK with Guo forcing of
// F = D0 . sigma (+ body force), pull streaming of post-collision deviations.
// Q: explicit Euler of -u.D0 Q + S + Gamma H with the 2D co-rotation term
//   S = (xi D + Om) P + P (xi D - Om) - 2 xi P tr(Q W), made traceless.
// A step is two launches: k2_lb (stress on the tile and its ring in LDS, force,
// pull, collision; writes g*, u) and k2_order (the Q update).
#pragma once
#include <hip/hip_runtime.h>

namespace lbc2 {

template <class R>
struct Params2 {
  R omega, guo, rho0;
  R A0, chi, K, Gamma, xi, zeta;
  R bf[2];
};

struct Box2 {
  int nx, ny, N;
};

__host__ __device__ constexpr int CX9(int i) {
  return (i == 1 || i == 5 || i == 7) ? 1 : ((i == 2 || i == 6 || i == 8) ? -1 : 0);
}
__host__ __device__ constexpr int CY9(int i) {
  return (i == 3 || i == 5 || i == 8) ? 1 : ((i == 4 || i == 6 || i == 7) ? -1 : 0);
}
template <class R>
__host__ __device__ constexpr R W9(int i) {
  return i == 0 ? R(4) / R(9) : (i <= 4 ? R(1) / R(9) : R(1) / R(36));
}

__device__ __forceinline__ int wrap2(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }
__device__ __forceinline__ int pmod2(int a, int n) {
  const int r = a % n;
  return r < 0 ? r + n : r;
}

// H (2 stored components) from Q and its 5-point Laplacian.
template <class R>
__device__ __forceinline__ void h2_site(const Params2<R>& P, R a, R b, R lapa, R lapb, R h[2]) {
  const R t2 = R(2) * (a * a + b * b);
  const R c = -P.A0 * (R(1) - P.chi * R(1.0 / 3.0)) - P.A0 * P.chi * t2;
  h[0] = c * a + P.K * lapa;
  h[1] = c * b + P.K * lapb;
}

// stress sig[2*a + b] of one site from Q = (a, b), its central differences
// da[g] = D0_g a, db[g] = D0_g b and the molecular field h.
template <class R>
__device__ __forceinline__ void sigma2_site(const Params2<R>& P, R a, R b, const R da[2], const R db[2],
                                            const R h[2], R sig[4]) {
  const R t2 = R(2) * (a * a + b * b);
  const R f = P.A0 * (R(0.5) * (R(1) - P.chi * R(1.0 / 3.0)) * t2 + R(0.25) * P.chi * t2 * t2) +
              P.K * ((da[0] * da[0] + da[1] * da[1]) + (db[0] * db[0] + db[1] * db[1]));
  const R qh = R(2) * (a * h[0] + b * h[1]);
  const R anti = R(2) * (a * h[1] - b * h[0]);  // (Q H - H Q)_xy
  const R k2 = R(2) * P.K;
  const R exx = -k2 * (da[0] * da[0] + db[0] * db[0]);
  const R eyy = -k2 * (da[1] * da[1] + db[1] * db[1]);
  const R exy = -k2 * (da[0] * da[1] + db[0] * db[1]);
  const R rxx = -P.xi * h[0] + R(2) * P.xi * qh * a - P.zeta * a;  // traceless symmetric part (xx)
  const R rxy = -P.xi * h[1] + R(2) * P.xi * qh * b - P.zeta * b;
  sig[0] = (f + exx) + rxx;
  sig[1] = (exy + rxy) + anti;
  sig[2] = (exy + rxy) - anti;
  sig[3] = (f + eyy) - rxx;
}

// traceless co-rotation term s[2] from Q = (a, b) and W[a][b] = D0_b u_a
template <class R>
__device__ __forceinline__ void corot2_site(R xi, R a, R b, const R W[2][2], R s[2]) {
  const R Pm[2][2] = {{a + R(0.5), b}, {b, -a + R(0.5)}};
  R A[2][2], B[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const R D = R(0.5) * (W[i][j] + W[j][i]), Om = R(0.5) * (W[i][j] - W[j][i]);
      A[i][j] = xi * D + Om;
      B[i][j] = xi * D - Om;
    }
  const R trQW = a * W[0][0] + b * W[1][0] + b * W[0][1] - a * W[1][1];
  R S[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      S[i][j] = (A[i][0] * Pm[0][j] + A[i][1] * Pm[1][j]) + (Pm[i][0] * B[0][j] + Pm[i][1] * B[1][j]) -
                R(2) * xi * Pm[i][j] * trQW;
  s[0] = R(0.5) * (S[0][0] - S[1][1]);
  s[1] = S[0][1];
}

// ---------------------------------------------------------------------------
// k2_lb: one TX x TY tile per workgroup.  Q on the tile with a ring of 2 in LDS;
// the stress on the tile with a ring of 1 (whose divergence is the force) in
// LDS; then each thread pulls its 9 populations, collides and writes g*, u.
// ---------------------------------------------------------------------------
template <class R, int TX, int TY>
__global__ void __launch_bounds__(TX* TY) k2_lb(Box2 b, Params2<R> P, int ntx, const R* __restrict__ Bin,
                                                 R* __restrict__ Bout, const R* __restrict__ q,
                                                 R* __restrict__ u_out) {
  constexpr int NT = TX * TY;
  constexpr int QX = TX + 4, QY = TY + 4, NQF = QX * QY;  // Q frame (ring 2)
  constexpr int SX = TX + 2, SY = TY + 2, NSF = SX * SY;  // stress frame (ring 1)
  __shared__ R sQ[2][NQF];
  __shared__ R sS[4][NSF];
  const int bid = blockIdx.x;
  const int x0 = (bid % ntx) * TX, y0 = (bid / ntx) * TY;
  const int tid = threadIdx.x;
  const size_t N = b.N;
  for (int k = tid; k < NQF; k += NT) {
    const int gx = pmod2(x0 - 2 + k % QX, b.nx), gy = pmod2(y0 - 2 + k / QX, b.ny);
    const int s = gy * b.nx + gx;
    sQ[0][k] = q[s];
    sQ[1][k] = q[N + s];
  }
  __syncthreads();
  for (int k = tid; k < NSF; k += NT) {
    const int f = (k / SX + 1) * QX + (k % SX + 1);  // Q-frame slot of stress slot k
    const R a = sQ[0][f], bb = sQ[1][f];
    const R da[2] = {R(0.5) * (sQ[0][f + 1] - sQ[0][f - 1]), R(0.5) * (sQ[0][f + QX] - sQ[0][f - QX])};
    const R db[2] = {R(0.5) * (sQ[1][f + 1] - sQ[1][f - 1]), R(0.5) * (sQ[1][f + QX] - sQ[1][f - QX])};
    const R la = ((sQ[0][f + 1] + sQ[0][f - 1]) + (sQ[0][f + QX] + sQ[0][f - QX])) - R(4) * a;
    const R lb = ((sQ[1][f + 1] + sQ[1][f - 1]) + (sQ[1][f + QX] + sQ[1][f - QX])) - R(4) * bb;
    R h[2], sig[4];
    h2_site(P, a, bb, la, lb, h);
    sigma2_site(P, a, bb, da, db, h, sig);
#pragma unroll
    for (int c = 0; c < 4; ++c) sS[c][k] = sig[c];
  }
  __syncthreads();
  const int lx = tid % TX, ly = tid / TX;
  const int x = x0 + lx, y = y0 + ly;
  if (x >= b.nx || y >= b.ny) return;
  const int k = (ly + 1) * SX + (lx + 1);
  R F[2];
  F[0] = (R(0.5) * (sS[0][k + 1] - sS[0][k - 1]) + R(0.5) * (sS[1][k + SX] - sS[1][k - SX])) + P.bf[0];
  F[1] = (R(0.5) * (sS[2][k + 1] - sS[2][k - 1]) + R(0.5) * (sS[3][k + SX] - sS[3][k - SX])) + P.bf[1];
  R g[9];
#pragma unroll
  for (int i = 0; i < 9; ++i)
    g[i] = Bin[i * N + wrap2(y - CY9(i), b.ny) * b.nx + wrap2(x - CX9(i), b.nx)];
  R drho = g[0], j[2] = {R(0), R(0)};
  // lattice-velocity products from the nonzero components only (a product
  // with 0 is not dropped by the compiler under IEEE rules; same results)
  auto cadd9 = [](int c, R v, R& acc) {
    if (c != 0) acc += c > 0 ? v : -v;
  };
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    drho += g[i];
    cadd9(CX9(i), g[i], j[0]);
    cadd9(CY9(i), g[i], j[1]);
  }
  const R rho = P.rho0 + drho;
  const R u[2] = {(j[0] + R(0.5) * F[0]) / rho, (j[1] + R(0.5) * F[1]) / rho};
  const R uu = u[0] * u[0] + u[1] * u[1], uF = u[0] * F[0] + u[1] * F[1];
  const int s = y * b.nx + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    R cu = R(-0.0), cF = R(-0.0);  // -0 + x == x: the first add folds
    cadd9(CX9(i), u[0], cu);
    cadd9(CY9(i), u[1], cu);
    cadd9(CX9(i), F[0], cF);
    cadd9(CY9(i), F[1], cF);
    const R w = W9<R>(i);
    const R geq = w * (drho + rho * ((R(3) * cu + R(4.5) * cu * cu) - R(1.5) * uu));
    const R src = P.guo * w * (R(3) * (cF - uF) + R(9) * cu * cF);
    Bout[i * N + s] = (g[i] - P.omega * (g[i] - geq)) + src;
  }
  u_out[s] = u[0];
  u_out[N + s] = u[1];
}

// ---------------------------------------------------------------------------
// k2_order: Q(t+1) = Q + [-u.D0 Q + S + Gamma H], one thread per site.
// ---------------------------------------------------------------------------
template <class R>
__global__ void __launch_bounds__(256) k2_order(Box2 b, Params2<R> P, const R* __restrict__ q,
                                                const R* __restrict__ u, R* __restrict__ q_out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  const int x = s % b.nx, y = s / b.nx;
  const size_t N = b.N;
  const int xp = y * b.nx + wrap2(x + 1, b.nx), xm = y * b.nx + wrap2(x - 1, b.nx);
  const int yp = wrap2(y + 1, b.ny) * b.nx + x, ym = wrap2(y - 1, b.ny) * b.nx + x;
  const R a = q[s], bb = q[N + s];
  const R da[2] = {R(0.5) * (q[xp] - q[xm]), R(0.5) * (q[yp] - q[ym])};
  const R db[2] = {R(0.5) * (q[N + xp] - q[N + xm]), R(0.5) * (q[N + yp] - q[N + ym])};
  const R la = ((q[xp] + q[xm]) + (q[yp] + q[ym])) - R(4) * a;
  const R lb = ((q[N + xp] + q[N + xm]) + (q[N + yp] + q[N + ym])) - R(4) * bb;
  R h[2];
  h2_site(P, a, bb, la, lb, h);
  const R ux = u[s], uy = u[N + s];
  R W[2][2];
  W[0][0] = R(0.5) * (u[xp] - u[xm]);
  W[0][1] = R(0.5) * (u[yp] - u[ym]);
  W[1][0] = R(0.5) * (u[N + xp] - u[N + xm]);
  W[1][1] = R(0.5) * (u[N + yp] - u[N + ym]);
  R S[2];
  corot2_site(P.xi, a, bb, W, S);
  q_out[s] = a + ((-(ux * da[0] + uy * da[1]) + S[0]) + P.Gamma * h[0]);
  q_out[N + s] = bb + ((-(ux * db[0] + uy * db[1]) + S[1]) + P.Gamma * h[1]);
}

// ------------------------------------------------------------ auxiliaries
// post-stream populations at time t (pull of B)
template <class R>
__global__ void k2_pull(Box2 b, const R* __restrict__ B, double* __restrict__ g) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  const int x = s % b.nx, y = s / b.nx;
  const size_t N = b.N;
#pragma unroll
  for (int i = 0; i < 9; ++i) g[i * N + s] = double(B[i * N + wrap2(y - CY9(i), b.ny) * b.nx + wrap2(x - CX9(i), b.nx)]);
}

// B_i(x) = g_i(x + c_i), the inverse of the pull
template <class R>
__global__ void k2_push(Box2 b, const double* __restrict__ g, R* __restrict__ B) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  const int x = s % b.nx, y = s / b.nx;
  const size_t N = b.N;
#pragma unroll
  for (int i = 0; i < 9; ++i) B[i * N + s] = R(g[i * N + wrap2(y + CY9(i), b.ny) * b.nx + wrap2(x + CX9(i), b.nx)]);
}

// second-order equilibrium deviations of (rho0, u0), in float64
__global__ void k2_equilibrium(Box2 b, double rho0, const double* __restrict__ u0, double* __restrict__ g) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  const size_t N = b.N;
  const double ux = u0 ? u0[s] : 0.0, uy = u0 ? u0[N + s] : 0.0;
  const double uu = ux * ux + uy * uy;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double cu = CX9(i) * ux + CY9(i) * uy;
    g[i * N + s] = W9<double>(i) * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

// float64 per-site observables at time t: rho, u (with F/2), F_h density terms;
// written to out[0..5][N] = rho, u_x, u_y, free-energy density (forward
// differences), kinetic energy density, momentum helpers are rho u.
template <class R>
__global__ void __launch_bounds__(256) k2_observe(Box2 b, Params2<double> P, const R* __restrict__ B,
                                                  const R* __restrict__ q, double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  const int x = s % b.nx, y = s / b.nx;
  const size_t N = b.N;
  // stress at the four neighbours (in float64 from the stored Q)
  auto qa = [&](int xx, int yy, int c) { return double(q[c * N + wrap2(yy, b.ny) * b.nx + wrap2(xx, b.nx)]); };
  auto sig_at = [&](int xx, int yy, double sg[4]) {
    const double a = qa(xx, yy, 0), bb = qa(xx, yy, 1);
    const double da[2] = {0.5 * (qa(xx + 1, yy, 0) - qa(xx - 1, yy, 0)), 0.5 * (qa(xx, yy + 1, 0) - qa(xx, yy - 1, 0))};
    const double db[2] = {0.5 * (qa(xx + 1, yy, 1) - qa(xx - 1, yy, 1)), 0.5 * (qa(xx, yy + 1, 1) - qa(xx, yy - 1, 1))};
    const double la = qa(xx + 1, yy, 0) + qa(xx - 1, yy, 0) + qa(xx, yy + 1, 0) + qa(xx, yy - 1, 0) - 4.0 * a;
    const double lb = qa(xx + 1, yy, 1) + qa(xx - 1, yy, 1) + qa(xx, yy + 1, 1) + qa(xx, yy - 1, 1) - 4.0 * bb;
    double h[2];
    h2_site(P, a, bb, la, lb, h);
    sigma2_site(P, a, bb, da, db, h, sg);
  };
  double sxp[4], sxm[4], syp[4], sym[4];
  sig_at(x + 1, y, sxp);
  sig_at(x - 1, y, sxm);
  sig_at(x, y + 1, syp);
  sig_at(x, y - 1, sym);
  const double F[2] = {0.5 * (sxp[0] - sxm[0]) + 0.5 * (syp[1] - sym[1]) + P.bf[0],
                       0.5 * (sxp[2] - sxm[2]) + 0.5 * (syp[3] - sym[3]) + P.bf[1]};
  double drho = 0.0, j[2] = {0.0, 0.0};
  for (int i = 0; i < 9; ++i) {
    const double gi = double(B[i * N + wrap2(y - CY9(i), b.ny) * b.nx + wrap2(x - CX9(i), b.nx)]);
    drho += gi;
    j[0] += CX9(i) * gi;
    j[1] += CY9(i) * gi;
  }
  const double rho = P.rho0 + drho;
  const double ux = (j[0] + 0.5 * F[0]) / rho, uy = (j[1] + 0.5 * F[1]) / rho;
  const double a = qa(x, y, 0), bb = qa(x, y, 1);
  const double t2 = 2.0 * (a * a + bb * bb);
  const double dxa = qa(x + 1, y, 0) - a, dya = qa(x, y + 1, 0) - a;
  const double dxb = qa(x + 1, y, 1) - bb, dyb = qa(x, y + 1, 1) - bb;
  const double fh = P.A0 * (0.5 * (1.0 - P.chi / 3.0) * t2 + 0.25 * P.chi * t2 * t2) +
                    P.K * (dxa * dxa + dya * dya + dxb * dxb + dyb * dyb);
  out[s] = rho;
  out[N + s] = ux;
  out[2 * N + s] = uy;
  out[3 * N + s] = drho;
  out[4 * N + s] = fh;
  out[5 * N + s] = 0.5 * rho * (ux * ux + uy * uy);
}

}  // namespace lbc2
