// Per-site physics of the coupled step, templated on the arithmetic type R.
//
// Every function here is pure register math on values a kernel has already
// gathered; the kernels decide where the values come from (HBM, L2, LDS).
//
// Free energy (Eq. (5)), with chi(phi) = chi0 + chi_s*phi and the one-constant
// elastic term written on a periodic box as
//   (K/2)|grad Q|^2 + 2 K q0 Q:curl(Q) + 2 K q0^2 Q:Q,   curl(Q)_ab = eps_agd d_g Q_db.
// mu = dF/dphi, H = -(dF/dQ) projected traceless symmetric (Eqs. (1), (2)).
// Stress (Eqs. (3), (4)): interfacial + Ericksen + Beris-Edwards reactive +
// antisymmetric + active (-zeta phi Q); a is the force component and b the
// derivative index, F_a = sum_b D0_b sigma_ab.
#pragma once
#include <hip/hip_runtime.h>

namespace lbc {

template <class R>
struct Params {
  R omega;      // 1/tau
  R guo;        // 1 - 1/(2 tau)
  R rho0;
  R a, phi0, inv_phicr2, k_phi, M;
  R A0, chi0, chi_s, K, q0, W;
  R Gamma, xi, zeta;
  R bf[3];
};

// D3Q19 velocity set, same order as the public header.
__host__ __device__ constexpr int CX(int i) {
  return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
       : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int CY(int i) {
  return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
       : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr int CZ(int i) {
  return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
       : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
template <class R>
__host__ __device__ constexpr R WQ(int i) {
  return i == 0 ? R(1) / R(3) : (i <= 6 ? R(1) / R(18) : R(1) / R(36));
}

// ------------------------------------------------------------- tensor helpers
template <class R>
__device__ __forceinline__ void full3(const R q[5], R Q[3][3]) {
  Q[0][0] = q[0]; Q[0][1] = q[1]; Q[0][2] = q[2];
  Q[1][0] = q[1]; Q[1][1] = q[3]; Q[1][2] = q[4];
  Q[2][0] = q[2]; Q[2][1] = q[4]; Q[2][2] = -q[0] - q[3];
}

template <class R>
__device__ __forceinline__ void matmul3(const R A[3][3], const R B[3][3], R C[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) C[a][b] = A[a][0] * B[0][b] + A[a][1] * B[1][b] + A[a][2] * B[2][b];
}

// A:B = sum_ab A_ab B_ab
template <class R>
__device__ __forceinline__ R ddot3(const R A[3][3], const R B[3][3]) {
  R s = R(0);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) s += A[a][b] * B[a][b];
  return s;
}

// curl(Q)_ab = eps_agd dQ[g][d][b]; dQ[g] = D0_g Q.
template <class R>
__device__ __forceinline__ void curl3(const R dQ[3][3][3], R C[3][3]) {
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    C[0][b] = dQ[1][2][b] - dQ[2][1][b];
    C[1][b] = dQ[2][0][b] - dQ[0][2][b];
    C[2][b] = dQ[0][1][b] - dQ[1][0][b];
  }
}

// Local gradient data of one site, gathered by a kernel.
template <class R>
struct Grad {
  R phi;          // phi(x)
  R dphi[3];      // D0 phi
  R lapphi;       // 7-point laplacian of phi
  R divv;         // sum_a D0_a (Q_ab D0_b phi)
  R q[5];         // stored Q components at x
  R dq[3][5];     // D0_g of the stored components
  R lapq[5];      // laplacian of the stored components
};

// mu, H (stored 5 components) and the central-difference free-energy density.
template <class R>
__device__ __forceinline__ void thermo_site(const Params<R>& P, const Grad<R>& G, R& mu, R h[5], R& fc) {
  R Q[3][3], dQ[3][3][3], Q2[3][3], C[3][3];
  full3(G.q, Q);
#pragma unroll
  for (int g = 0; g < 3; ++g) full3(G.dq[g], dQ[g]);
  matmul3(Q, Q, Q2);
  R tr2 = ddot3(Q, Q);
  R tr3 = ddot3(Q2, Q);
  const R phi = G.phi;
  const R chi = P.chi0 + P.chi_s * phi;
  const R dp2 = G.dphi[0] * G.dphi[0] + G.dphi[1] * G.dphi[1] + G.dphi[2] * G.dphi[2];

  mu = P.a * phi * (phi - P.phi0) * (R(2) * phi - P.phi0) * P.inv_phicr2
     + P.A0 * P.chi_s * (-tr2 / R(6) - tr3 / R(3) + tr2 * tr2 / R(4))
     - P.k_phi * G.lapphi - R(2) * P.W * G.divv;

  curl3(dQ, C);
  const R c1 = R(1) - chi / R(3);
  const R kq = R(2) * P.K * P.q0;
  const R kq2 = R(4) * P.K * P.q0 * P.q0;
  // stored components: (0,0) (0,1) (0,2) (1,1) (1,2)
  const int ia[5] = {0, 0, 0, 1, 1};
  const int ib[5] = {0, 1, 2, 1, 2};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int a = ia[k], b = ib[k];
    const R de = (a == b) ? R(1) : R(0);
    h[k] = -P.A0 * (c1 * Q[a][b] - chi * (Q2[a][b] - de * tr2 / R(3)) + chi * Q[a][b] * tr2)
         + P.K * G.lapq[k] - kq * (C[a][b] + C[b][a]) - kq2 * Q[a][b]
         - P.W * (G.dphi[a] * G.dphi[b] - de * dp2 / R(3));
  }

  R gq2 = R(0);
#pragma unroll
  for (int g = 0; g < 3; ++g) gq2 += ddot3(dQ[g], dQ[g]);
  R qc = ddot3(Q, C);
  R anch = R(0);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) anch += G.dphi[a] * Q[a][b] * G.dphi[b];
  const R dw = phi * (phi - P.phi0);
  fc = R(0.5) * P.a * dw * dw * P.inv_phicr2
     + P.A0 * (R(0.5) * c1 * tr2 - chi / R(3) * tr3 + chi / R(4) * tr2 * tr2)
     + R(0.5) * kq2 * tr2 + R(0.5) * P.k_phi * dp2 + R(0.5) * P.K * gq2 + kq * qc + P.W * anch;
}

// Full 3x3 stress (row a = force component, column b = derivative index).
template <class R>
__device__ __forceinline__ void stress_site(const Params<R>& P, const Grad<R>& G, const R h[5], R fc,
                                            R sig[3][3]) {
  R Q[3][3], H[3][3], dQ[3][3][3];
  full3(G.q, Q);
  full3(h, H);
#pragma unroll
  for (int g = 0; g < 3; ++g) full3(G.dq[g], dQ[g]);
  R Qd[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) Qd[b] = Q[b][0] * G.dphi[0] + Q[b][1] * G.dphi[1] + Q[b][2] * G.dphi[2];
  R QH[3][3], HQ[3][3];
  matmul3(Q, H, QH);
  matmul3(H, Q, HQ);
  const R qh = ddot3(Q, H);
  const R xi = P.xi;
  const R kq = R(2) * P.K * P.q0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // Ericksen (Q): -K dQ[a]:dQ[b] - 2 K q0 axial_b(dQ[a] Q), axial_b(M) = eps_bgl M_gl
    R M[3][3];
    matmul3(dQ[a], Q, M);
    const R ax[3] = {M[1][2] - M[2][1], M[2][0] - M[0][2], M[0][1] - M[1][0]};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const R de = (a == b) ? R(1) : R(0);
      const R P_ab = Q[a][b] + de / R(3);
      R s = fc * de - G.dphi[a] * (P.k_phi * G.dphi[b] + R(2) * P.W * Qd[b]);
      s -= P.K * ddot3(dQ[a], dQ[b]) + kq * ax[b];
      s += -xi * (HQ[a][b] + QH[a][b] + R(2) * H[a][b] / R(3)) + R(2) * xi * P_ab * qh + (QH[a][b] - HQ[a][b]);
      s -= P.zeta * G.phi * Q[a][b];
      sig[a][b] = s;
    }
  }
}

// Traceless co-rotational term S of the Beris-Edwards material derivative
// (Eq. (2)), from the velocity gradient W_ab = D0_b u_a.
template <class R>
__device__ __forceinline__ void corotation_site(R xi, const R Q[3][3], const R W[3][3], R S[3][3]) {
  R A[3][3], B[3][3], Pm[3][3];
  R trQW = R(0);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const R D = R(0.5) * (W[a][b] + W[b][a]);
      const R O = R(0.5) * (W[a][b] - W[b][a]);
      A[a][b] = xi * D + O;
      B[a][b] = xi * D - O;
      Pm[a][b] = Q[a][b] + ((a == b) ? R(1) / R(3) : R(0));
      trQW += Q[a][b] * W[b][a];
    }
  R AP[3][3], PB[3][3];
  matmul3(A, Pm, AP);
  matmul3(Pm, B, PB);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) S[a][b] = AP[a][b] + PB[a][b] - R(2) * xi * Pm[a][b] * trQW;
  const R tr = (S[0][0] + S[1][1] + S[2][2]) / R(3);
  S[0][0] -= tr; S[1][1] -= tr; S[2][2] -= tr;
}

// BGK collision with Guo forcing on the 19 deviations g (in place).
// rho = rho0 + sum g, u = (sum c g + F/2)/rho; returns u.
template <class R>
__device__ __forceinline__ void collide_site(const Params<R>& P, R g[19], const R F[3], R u[3]) {
  R s = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    s += g[i];
    if (CX(i)) jx += CX(i) > 0 ? g[i] : -g[i];
    if (CY(i)) jy += CY(i) > 0 ? g[i] : -g[i];
    if (CZ(i)) jz += CZ(i) > 0 ? g[i] : -g[i];
  }
  const R drho = s;
  const R rho = P.rho0 + drho;
  const R inv = R(1) / rho;
  u[0] = (jx + R(0.5) * F[0]) * inv;
  u[1] = (jy + R(0.5) * F[1]) * inv;
  u[2] = (jz + R(0.5) * F[2]) * inv;
  const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const R uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const R cu = R(CX(i)) * u[0] + R(CY(i)) * u[1] + R(CZ(i)) * u[2];
    const R cF = R(CX(i)) * F[0] + R(CY(i)) * F[1] + R(CZ(i)) * F[2];
    const R w = WQ<R>(i);
    const R geq = w * (drho + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu));
    const R src = P.guo * w * (R(3) * (cF - uF) + R(9) * cu * cF);
    g[i] = g[i] - (g[i] - geq) * P.omega + src;
  }
}

}  // namespace lbc
