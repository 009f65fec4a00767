// Site-parallel kernels of the coupled step: one thread per lattice site,
// stencil neighbours read through the cache hierarchy.
//
// The population buffer holds post-collision values of the previous step,
// B_i(x) = g*_i(x, t-1), so that the post-stream deviation at time t is the
// pull g_i(x, t) = B_i(x - c_i).  A step is three launches:
//   thermo  : Q, phi -> mu, H, sigma            (Eq. (5); Eqs. (3)-(4))
//   collide : B, sigma -> B', u                 (Eqs. (6)-(8), (10)-(11))
//   order   : Q, phi, u, H, mu -> Q', phi'      (Eqs. (1)-(2))
#pragma once
#include "physics.hpp"
#include "storage.hpp"

namespace lbc {

// Row a of Q at site k from the 5 stored components (stride N).
template <class R, class FS>
__device__ __forceinline__ void qrow(const FS* __restrict__ q, size_t N, int k, int a, R r[3]) {
  const R xx = R(q[k]), xy = R(q[N + k]), xz = R(q[2 * N + k]), yy = R(q[3 * N + k]), yz = R(q[4 * N + k]);
  if (a == 0) { r[0] = xx; r[1] = xy; r[2] = xz; }
  else if (a == 1) { r[0] = xy; r[1] = yy; r[2] = yz; }
  else { r[0] = xz; r[1] = yz; r[2] = -xx - yy; }
}

// Gather the local gradient data of site (x, y, z) from Q and phi.
template <class R, class FS>
__device__ __forceinline__ void gather_grad(const Box& b, const FS* __restrict__ phi, const FS* __restrict__ q,
                                            int x, int y, int z, Grad<R>& G) {
  const size_t N = b.N;
  const int s0 = (z * b.ny + y) * b.nx + x;
  const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  G.phi = R(phi[s0]);
  R lap = R(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) { G.q[k] = R(q[k * N + s0]); G.lapq[k] = R(0); }
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const int sp = sidx(b, x + off[g][0], y + off[g][1], z + off[g][2]);
    const int sm = sidx(b, x - off[g][0], y - off[g][1], z - off[g][2]);
    const R pp = R(phi[sp]), pm = R(phi[sm]);
    G.dphi[g] = R(0.5) * (pp - pm);
    lap += pp + pm;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const R a = R(q[k * N + sp]), c = R(q[k * N + sm]);
      G.dq[g][k] = R(0.5) * (a - c);
      G.lapq[k] += a + c;
    }
  }
  G.lapphi = lap - R(6) * G.phi;
#pragma unroll
  for (int k = 0; k < 5; ++k) G.lapq[k] -= R(6) * G.q[k];
  // divv = sum_a D0_a v_a,  v_a(y) = Q_ab(y) D0_b phi(y)
  R divv = R(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R va[2];
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
      const int dd = sg == 0 ? 1 : -1;
      const int X = x + dd * off[a][0], Y = y + dd * off[a][1], Z = z + dd * off[a][2];
      const int sy = sidx(b, X, Y, Z);
      R row[3];
      qrow<R>(q, N, sy, a, row);
      R v = R(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const R pp = R(phi[sidx(b, X + off[c][0], Y + off[c][1], Z + off[c][2])]);
        const R pm = R(phi[sidx(b, X - off[c][0], Y - off[c][1], Z - off[c][2])]);
        v += row[c] * (R(0.5) * (pp - pm));
      }
      va[sg] = v;
    }
    divv += R(0.5) * (va[0] - va[1]);
  }
  G.divv = divv;
}

template <class R, class FS>
__global__ void __launch_bounds__(256) k_thermo(Box b, Params<R> P, const FS* __restrict__ phi,
                                                const FS* __restrict__ q, R* __restrict__ mu_out,
                                                R* __restrict__ h_out, R* __restrict__ sig_out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  Grad<R> G;
  gather_grad<R>(b, phi, q, x, y, z, G);
  R h[5], sig[9];
  sigma_site(P, G, sig, h);
  const size_t N = b.N;
  mu_out[s] = mu_site(P, G.phi, G.lapphi, G.divv, G.q);
#pragma unroll
  for (int k = 0; k < 5; ++k) h_out[k * N + s] = h[k];
#pragma unroll
  for (int k = 0; k < 9; ++k) sig_out[k * N + s] = sig[k];
}

// sum_b D0_b of the stress components the lattice's forcing carries: the
// whole stress (D3Q19), or its antisymmetric part (sigma_ab - sigma_ba)/2
// (D3Q15, whose equilibrium carries the symmetric part).  No body force.
template <class L, class R>
__device__ __forceinline__ void force_sig(const Box& b, const R* __restrict__ sig, int x, int y, int z, R F[3]) {
  const size_t N = b.N;
  const int sp[3] = {sidx(b, x + 1, y, z), sidx(b, x, y + 1, z), sidx(b, x, y, z + 1)};
  const int sm[3] = {sidx(b, x - 1, y, z), sidx(b, x, y - 1, z), sidx(b, x, y, z - 1)};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R d = R(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const R* sac = sig + size_t(3 * a + c) * N;
      if constexpr (L::kStressInEq) {
        const R* sca = sig + size_t(3 * c + a) * N;
        d += R(0.5) * (R(0.5) * (sac[sp[c]] - sca[sp[c]]) - R(0.5) * (sac[sm[c]] - sca[sm[c]]));
      } else {
        d += R(0.5) * (sac[sp[c]] - sac[sm[c]]);
      }
    }
    F[a] = d;
  }
}

template <class L, class R>
__device__ __forceinline__ void force_at(const Box& b, const Params<R>& P, const R* __restrict__ sig, int x, int y,
                                         int z, R F[3]) {
  force_sig<L>(b, sig, x, y, z, F);
#pragma unroll
  for (int a = 0; a < 3; ++a) F[a] += P.bf[a];
}

template <class R, class GS, class L>
__global__ void __launch_bounds__(256) k_collide(Box b, Params<R> P, const GS* __restrict__ Bin,
                                                 GS* __restrict__ Bout, const R* __restrict__ sig,
                                                 R* __restrict__ u_out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  R F[3];
  force_at<L>(b, P, sig, x, y, z, F);
  R g[L::Q];
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    g[i] = GPol<GS, L>::template ld<R>(Bin, i * N + sidx(b, x - L::cx(i), y - L::cy(i), z - L::cz(i)), i);
  R u[3];
  if constexpr (L::kStressInEq) {
    const R S[6] = {sig[s], R(0.5) * (sig[N + s] + sig[3 * N + s]), R(0.5) * (sig[2 * N + s] + sig[6 * N + s]),
                    sig[4 * N + s], R(0.5) * (sig[5 * N + s] + sig[7 * N + s]), sig[8 * N + s]};
    collide_site_eq(P, g, F, S, u);
  } else {
    collide_site(P, g, F, u);
  }
#pragma unroll
  for (int i = 0; i < L::Q; ++i) GPol<GS, L>::template st<R>(Bout, i * N + s, i, g[i]);
#pragma unroll
  for (int a = 0; a < 3; ++a) u_out[a * N + s] = u[a];
}

template <class R, class FS>
__global__ void __launch_bounds__(256) k_order(Box b, Params<R> P, const FS* __restrict__ phi,
                                               const FS* __restrict__ q, const R* __restrict__ u,
                                               const R* __restrict__ h, const R* __restrict__ mu,
                                               FS* __restrict__ phi_out, FS* __restrict__ q_out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  R qc[5], dq[3][5], W[3][3], uc[3];
#pragma unroll
  for (int k = 0; k < 5; ++k) qc[k] = R(q[k * N + s]);
#pragma unroll
  for (int a = 0; a < 3; ++a) uc[a] = u[a * N + s];
  R flux = R(0), lapmu = R(0);
  const R muc = mu[s];
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const int sp = sidx(b, x + off[g][0], y + off[g][1], z + off[g][2]);
    const int sm = sidx(b, x - off[g][0], y - off[g][1], z - off[g][2]);
#pragma unroll
    for (int k = 0; k < 5; ++k) dq[g][k] = R(0.5) * (R(q[k * N + sp]) - R(q[k * N + sm]));
#pragma unroll
    for (int a = 0; a < 3; ++a) W[a][g] = R(0.5) * (u[a * N + sp] - u[a * N + sm]);
    flux += R(0.5) * (u[g * N + sp] * R(phi[sp]) - u[g * N + sm] * R(phi[sm]));
    lapmu += mu[sp] + mu[sm];
  }
  lapmu -= R(6) * muc;
  R S[5];
  corotation_site(P.xi, qc, W, S);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const R adv = uc[0] * dq[0][k] + uc[1] * dq[1][k] + uc[2] * dq[2][k];
    q_out[k * N + s] = FS(qc[k] + (-adv + S[k] + P.Gamma * h[k * N + s]));
  }
  phi_out[s] = FS(R(phi[s]) - flux + P.M * lapmu);
}

// ------------------------------------------------------------ auxiliary kernels
// Post-stream populations at time t (pull of B) converted to R.
template <class R, class GS, class L>
__global__ void k_pull(Box b, const GS* __restrict__ B, R* __restrict__ g) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    g[i * N + s] = GPol<GS, L>::template ld<R>(B, i * N + sidx(b, x - L::cx(i), y - L::cy(i), z - L::cz(i)), i);
}

// B_i(x) = g_i(x + c_i): the inverse of the pull, from float64 deviations.
template <class GS, class L>
__global__ void k_push(Box b, const double* __restrict__ g, GS* __restrict__ B) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    GPol<GS, L>::template st<double>(B, i * N + s, i, g[i * N + sidx(b, x + L::cx(i), y + L::cy(i), z + L::cz(i))]);
}

// Second-order equilibrium deviations of (rho0, u0) in float64 (Eq. (11) with
// no stress term).
template <class L>
__global__ void k_equilibrium(Box b, double rho0, const double* __restrict__ u0, double* __restrict__ g) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  const size_t N = b.N;
  double u[3] = {0.0, 0.0, 0.0};
  if (u0)
    for (int a = 0; a < 3; ++a) u[a] = u0[a * N + s];
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const double cu = L::cx(i) * u[0] + L::cy(i) * u[1] + L::cz(i) * u[2];
    g[i * N + s] = L::template w<double>(i) * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

// rho and u (with F/2) at time t.
template <class R, class GS, class L>
__global__ void k_moments(Box b, Params<R> P, const GS* __restrict__ B, const R* __restrict__ sig,
                          R* __restrict__ rho_out, R* __restrict__ u_out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  R F[3];
  force_at<L>(b, P, sig, x, y, z, F);
  R sum = R(0), j[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    const R gi = GPol<GS, L>::template ld<R>(B, i * N + sidx(b, x - L::cx(i), y - L::cy(i), z - L::cz(i)), i);
    sum += gi;
    cadd(L::cx(i), gi, j[0]);
    cadd(L::cy(i), gi, j[1]);
    cadd(L::cz(i), gi, j[2]);
  }
  const R rho = P.rho0 + sum;
  rho_out[s] = rho;
#pragma unroll
  for (int a = 0; a < 3; ++a) u_out[a * N + s] = (j[a] + R(0.5) * F[a]) / rho;
}

template <class T, class S>
__global__ void k_convert(size_t n, const S* __restrict__ src, T* __restrict__ dst) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = T(src[k]);
}

}  // namespace lbc
