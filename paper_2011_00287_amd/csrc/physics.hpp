// Per-site physics of the coupled step, templated on the arithmetic type R.
//
// Every function here is pure register math on values a kernel has already
// gathered; the kernels decide where the values come from (HBM, L2, LDS).
// Symmetric traceless tensors are handled through their 5 stored components
// (xx, xy, xz, yy, yz; zz = -xx - yy) with explicit scalar formulas, so no
// work is spent on entries that symmetry already fixes.
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

// c . v and acc += c v for lattice-velocity components c in {-1, 0, 1} known
// at compile time, from the nonzero components only.  Under IEEE rules the
// compiler may not drop a product with 0 (0 * inf is NaN), so R(c) * v would
// cost an instruction for every zero component.  For finite v the results
// equal those of the full sums exactly.
template <class R>
__host__ __device__ __forceinline__ R cdot(int cx, int cy, int cz, const R v[3]) {
  R s = R(-0.0);  // -0 + x == x for every x: the first term is exact and the add folds
  if (cx != 0) s += cx > 0 ? v[0] : -v[0];
  if (cy != 0) s += cy > 0 ? v[1] : -v[1];
  if (cz != 0) s += cz > 0 ? v[2] : -v[2];
  return s;
}
template <class R>
__host__ __device__ __forceinline__ void cadd(int c, R v, R& acc) {
  if (c != 0) acc += c > 0 ? v : -v;
}

// Velocity sets as traits.  D3Q19 (the order above) carries the whole stress as
// a Guo body force.  D3Q15, the paper's lattice (Fig. 1), carries the symmetric
// stress in the second moment of the equilibrium (Eqs. (9), (11)) and only the
// antisymmetric stress as forcing (Eq. (10)).  D3Q15 order: 0 rest; 1-6 = +x,
// -x, +y, -y, +z, -z; 7-14 = body diagonals in opposite pairs (+,+,+)/(-,-,-),
// (+,+,-)/(-,-,+), (+,-,+)/(-,+,-), (-,+,+)/(+,-,-); weights 2/9, 1/9, 1/72.
struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr bool kStressInEq = false;
  __host__ __device__ static constexpr int cx(int i) { return CX(i); }
  __host__ __device__ static constexpr int cy(int i) { return CY(i); }
  __host__ __device__ static constexpr int cz(int i) { return CZ(i); }
  template <class R>
  __host__ __device__ static constexpr R w(int i) { return WQ<R>(i); }
};
struct D3Q15 {
  static constexpr int Q = 15;
  static constexpr bool kStressInEq = true;
  __host__ __device__ static constexpr int cx(int i) {
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 14) ? 1
         : (i == 2 || i == 8 || i == 10 || i == 12 || i == 13) ? -1 : 0;
  }
  __host__ __device__ static constexpr int cy(int i) {
    return (i == 3 || i == 7 || i == 9 || i == 12 || i == 13) ? 1
         : (i == 4 || i == 8 || i == 10 || i == 11 || i == 14) ? -1 : 0;
  }
  __host__ __device__ static constexpr int cz(int i) {
    return (i == 5 || i == 7 || i == 10 || i == 11 || i == 13) ? 1
         : (i == 6 || i == 8 || i == 9 || i == 12 || i == 14) ? -1 : 0;
  }
  template <class R>
  __host__ __device__ static constexpr R w(int i) {
    return i == 0 ? R(2) / R(9) : (i <= 6 ? R(1) / R(9) : R(1) / R(72));
  }
};

template <class R>
struct C3 {
  static constexpr R third = R(1) / R(3);
  static constexpr R sixth = R(1) / R(6);
};

// Local gradient data of one site, gathered by a kernel.
template <class R>
struct Grad {
  R phi;          // phi(x)
  R dphi[3];      // D0 phi
  R lapphi;       // 7-point laplacian of phi (mu only)
  R divv;         // sum_a D0_a (Q_ab D0_b phi) (mu only)
  R q[5];         // stored Q components at x
  R dq[3][5];     // D0_g of the stored components
  R lapq[5];      // laplacian of the stored components
};

// Quantities shared by H, the free-energy density and the stress.
template <class R>
struct Local {
  R xx, xy, xz, yy, yz, zz;                        // Q
  R q2xx, q2xy, q2xz, q2yy, q2yz, q2zz, tr2, tr3;  // Q.Q and invariants
  R cxx, cyy, sxy, sxz, syz;                       // C_xx, C_yy, (C + C^T) off-diagonals
  R qc;                                            // Q : curl(Q)
  R dp2, chi;
  R h[5];                                          // molecular field
};

template <class R>
__host__ __device__ __forceinline__ void local_thermo(const Params<R>& P, const Grad<R>& G, Local<R>& L) {
  const R xx = G.q[0], xy = G.q[1], xz = G.q[2], yy = G.q[3], yz = G.q[4], zz = -xx - yy;
  L.xx = xx; L.xy = xy; L.xz = xz; L.yy = yy; L.yz = yz; L.zz = zz;
  L.q2xx = xx * xx + xy * xy + xz * xz;
  L.q2xy = xx * xy + xy * yy + xz * yz;
  L.q2xz = xx * xz + xy * yz + xz * zz;
  L.q2yy = xy * xy + yy * yy + yz * yz;
  L.q2yz = xy * xz + yy * yz + yz * zz;
  L.q2zz = xz * xz + yz * yz + zz * zz;
  L.tr2 = L.q2xx + L.q2yy + L.q2zz;
  L.tr3 = xx * L.q2xx + yy * L.q2yy + zz * L.q2zz + R(2) * (xy * L.q2xy + xz * L.q2xz + yz * L.q2yz);
  // d[g] = D0_g Q;  C_ab = eps_agd d[g]_db
  const R* d0 = G.dq[0];
  const R* d1 = G.dq[1];
  const R* d2 = G.dq[2];
  const R d0zz = -d0[0] - d0[3], d1zz = -d1[0] - d1[3];
  L.cxx = d1[2] - d2[1];
  L.cyy = d2[1] - d0[4];
  const R czz = -L.cxx - L.cyy;
  L.sxy = (d1[4] - d2[3]) + (d2[0] - d0[2]);
  L.sxz = (d1zz - d2[4]) + (d0[1] - d1[0]);
  L.syz = (d2[2] - d0zz) + (d0[3] - d1[1]);
  L.qc = xx * L.cxx + yy * L.cyy + zz * czz + xy * L.sxy + xz * L.sxz + yz * L.syz;

  const R dx = G.dphi[0], dy = G.dphi[1], dz = G.dphi[2];
  L.dp2 = dx * dx + dy * dy + dz * dz;
  L.chi = P.chi0 + P.chi_s * G.phi;
  const R kq = R(2) * P.K * P.q0;
  const R kq2 = R(4) * P.K * P.q0 * P.q0;
  const R c1 = R(1) - L.chi * C3<R>::third;
  const R alpha = -P.A0 * (c1 + L.chi * L.tr2) - kq2;
  const R beta = P.A0 * L.chi;
  const R t3 = L.tr2 * C3<R>::third;
  const R dd3 = L.dp2 * C3<R>::third;
  L.h[0] = alpha * xx + beta * (L.q2xx - t3) + P.K * G.lapq[0] - kq * (R(2) * L.cxx) - P.W * (dx * dx - dd3);
  L.h[1] = alpha * xy + beta * L.q2xy + P.K * G.lapq[1] - kq * L.sxy - P.W * (dx * dy);
  L.h[2] = alpha * xz + beta * L.q2xz + P.K * G.lapq[2] - kq * L.sxz - P.W * (dx * dz);
  L.h[3] = alpha * yy + beta * (L.q2yy - t3) + P.K * G.lapq[3] - kq * (R(2) * L.cyy) - P.W * (dy * dy - dd3);
  L.h[4] = alpha * yz + beta * L.q2yz + P.K * G.lapq[4] - kq * L.syz - P.W * (dy * dz);
}

// Molecular field only (5 stored components).
template <class R>
__host__ __device__ __forceinline__ void h_site(const Params<R>& P, const Grad<R>& G, R h[5]) {
  Local<R> L;
  local_thermo(P, G, L);
#pragma unroll
  for (int k = 0; k < 5; ++k) h[k] = L.h[k];
}

// A:B for symmetric traceless tensors given by 5 components.
template <class R>
__host__ __device__ __forceinline__ R sdot(const R* A, const R* B) {
  const R azz = -A[0] - A[3], bzz = -B[0] - B[3];
  return A[0] * B[0] + A[3] * B[3] + azz * bzz + R(2) * (A[1] * B[1] + A[2] * B[2] + A[4] * B[4]);
}

// Full stress sig[3*a + b] (a = force component, b = derivative index), the
// molecular field h (5 components) and the anchoring vector vq_a = Q_ab D0_b phi
// (whose divergence enters mu) of one site.
template <class R>
__host__ __device__ __forceinline__ void sigma_site(const Params<R>& P, const Grad<R>& G, R sig[9], R h[5],
                                                   R vq[3]) {
  Local<R> L;
  local_thermo(P, G, L);
  const R xx = L.xx, xy = L.xy, xz = L.xz, yy = L.yy, yz = L.yz, zz = L.zz;
  const R dp[3] = {G.dphi[0], G.dphi[1], G.dphi[2]};
  const R kq = R(2) * P.K * P.q0;
  const R kq2 = R(4) * P.K * P.q0 * P.q0;

  // Ericksen (Q) part: D_ab = dQ[a]:dQ[b]; ax[a]_b = eps_bgl (dQ[a] Q)_gl
  R D[3][3], ax[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      D[a][b] = sdot(G.dq[a], G.dq[b]);
      D[b][a] = D[a][b];
    }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const R dxx = G.dq[a][0], dxy = G.dq[a][1], dxz = G.dq[a][2], dyy = G.dq[a][3], dyz = G.dq[a][4];
    const R dzz = -dxx - dyy;
    ax[a][0] = (dxy * xz + dyy * yz + dyz * zz) - (dxz * xy + dyz * yy + dzz * yz);
    ax[a][1] = (dxz * xx + dyz * xy + dzz * xz) - (dxx * xz + dxy * yz + dxz * zz);
    ax[a][2] = (dxx * xy + dxy * yy + dxz * yz) - (dxy * xx + dyy * xy + dyz * xz);
  }
  // free-energy density (central differences)
  const R Qd[3] = {xx * dp[0] + xy * dp[1] + xz * dp[2], xy * dp[0] + yy * dp[1] + yz * dp[2],
                   xz * dp[0] + yz * dp[1] + zz * dp[2]};
  const R anch = dp[0] * Qd[0] + dp[1] * Qd[1] + dp[2] * Qd[2];
  const R dw = G.phi * (G.phi - P.phi0);
  const R c1 = R(1) - L.chi * C3<R>::third;
  const R fc = R(0.5) * P.a * dw * dw * P.inv_phicr2 +
               P.A0 * (R(0.5) * c1 * L.tr2 - L.chi * C3<R>::third * L.tr3 + R(0.25) * L.chi * L.tr2 * L.tr2) +
               R(0.5) * kq2 * L.tr2 + R(0.5) * P.k_phi * L.dp2 + R(0.5) * P.K * (D[0][0] + D[1][1] + D[2][2]) +
               kq * L.qc + P.W * anch;
  // reactive + antisymmetric:
  //   -(xi+1) (QH)^T + (1-xi) QH - (2xi/3) H + (2xi/3)(Q:H) I + 2 xi (Q:H) Q
  const R hxx = L.h[0], hxy = L.h[1], hxz = L.h[2], hyy = L.h[3], hyz = L.h[4], hzz = -hxx - hyy;
  const R Qm[3][3] = {{xx, xy, xz}, {xy, yy, yz}, {xz, yz, zz}};
  const R Hm[3][3] = {{hxx, hxy, hxz}, {hxy, hyy, hyz}, {hxz, hyz, hzz}};
  R QH[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) QH[a][b] = Qm[a][0] * Hm[0][b] + Qm[a][1] * Hm[1][b] + Qm[a][2] * Hm[2][b];
  const R qh = QH[0][0] + QH[1][1] + QH[2][2];
  const R xi = P.xi;
  const R cA = -(xi + R(1)), cB = R(1) - xi, cH = -R(2) * xi * C3<R>::third;
  const R cQ = R(2) * xi * qh - P.zeta * G.phi;
  const R iso = fc - cH * qh;  // fc + (2 xi/3) qh
  const R t[3] = {P.k_phi * dp[0] + R(2) * P.W * Qd[0], P.k_phi * dp[1] + R(2) * P.W * Qd[1],
                  P.k_phi * dp[2] + R(2) * P.W * Qd[2]};
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      R s = -dp[a] * t[b] - P.K * D[a][b] - kq * ax[a][b] + cA * QH[b][a] + cB * QH[a][b] + cH * Hm[a][b] +
            cQ * Qm[a][b];
      if (a == b) s += iso;
      sig[3 * a + b] = s;
    }
#pragma unroll
  for (int k = 0; k < 5; ++k) h[k] = L.h[k];
#pragma unroll
  for (int a = 0; a < 3; ++a) vq[a] = Qd[a];
}

template <class R>
__host__ __device__ __forceinline__ void sigma_site(const Params<R>& P, const Grad<R>& G, R sig[9], R h[5]) {
  R vq[3];
  sigma_site(P, G, sig, h, vq);
}

// Chemical potential mu = dF/dphi from phi, its laplacian, the anchoring
// divergence divv = D0_a(Q_ab D0_b phi) and the stored Q components.
template <class R>
__host__ __device__ __forceinline__ R mu_site(const Params<R>& P, R phi, R lapphi, R divv, const R q[5]) {
  const R xx = q[0], xy = q[1], xz = q[2], yy = q[3], yz = q[4], zz = -xx - yy;
  const R q2xx = xx * xx + xy * xy + xz * xz;
  const R q2xy = xx * xy + xy * yy + xz * yz;
  const R q2xz = xx * xz + xy * yz + xz * zz;
  const R q2yy = xy * xy + yy * yy + yz * yz;
  const R q2yz = xy * xz + yy * yz + yz * zz;
  const R q2zz = xz * xz + yz * yz + zz * zz;
  const R tr2 = q2xx + q2yy + q2zz;
  const R tr3 = xx * q2xx + yy * q2yy + zz * q2zz + R(2) * (xy * q2xy + xz * q2xz + yz * q2yz);
  return P.a * phi * (phi - P.phi0) * (R(2) * phi - P.phi0) * P.inv_phicr2 +
         P.A0 * P.chi_s * (-tr2 * C3<R>::sixth - tr3 * C3<R>::third + R(0.25) * tr2 * tr2) - P.k_phi * lapphi -
         R(2) * P.W * divv;
}

// Traceless co-rotational term of the Beris-Edwards material derivative
// (Eq. (2)) as 5 stored components, from the velocity gradient W_ab = D0_b u_a:
// S = A P + P A^T - 2 xi P tr(Q W), A = xi D + Om, P = Q + I/3, minus its trace/3.
template <class R>
__host__ __device__ __forceinline__ void corotation_site(R xi, const R q[5], const R W[3][3], R s5[5]) {
  const R xx = q[0], xy = q[1], xz = q[2], yy = q[3], yz = q[4], zz = -xx - yy;
  const R Pm[3][3] = {{xx + C3<R>::third, xy, xz}, {xy, yy + C3<R>::third, yz}, {xz, yz, zz + C3<R>::third}};
  const R Qm[3][3] = {{xx, xy, xz}, {xy, yy, yz}, {xz, yz, zz}};
  R A[3][3];
  R trQW = R(0);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      A[a][b] = R(0.5) * ((xi + R(1)) * W[a][b] + (xi - R(1)) * W[b][a]);
      trQW += Qm[a][b] * W[b][a];
    }
  R M[3][3];  // A P
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) M[a][b] = A[a][0] * Pm[0][b] + A[a][1] * Pm[1][b] + A[a][2] * Pm[2][b];
  const R c = R(2) * xi * trQW;
  const R sxx = R(2) * M[0][0] - c * Pm[0][0];
  const R syy = R(2) * M[1][1] - c * Pm[1][1];
  const R szz = R(2) * M[2][2] - c * Pm[2][2];
  const R tr = (sxx + syy + szz) * C3<R>::third;
  s5[0] = sxx - tr;
  s5[1] = (M[0][1] + M[1][0]) - c * Pm[0][1];
  s5[2] = (M[0][2] + M[2][0]) - c * Pm[0][2];
  s5[3] = syy - tr;
  s5[4] = (M[1][2] + M[2][1]) - c * Pm[1][2];
}

// BGK collision with Guo forcing on the 19 deviations g (in place).
// rho = rho0 + sum g, u = (sum c g + F/2)/rho; writes u and returns
// drho = sum g of the pre-collision populations.  With cu = c_i.u,
// cF = c_i.F, the equilibrium and source of population i are
//   g_eq_i = w (A + 3 rho cu + 4.5 rho cu^2),  A = (rho - rho0) - 1.5 rho u.u
//   src_i  = guo w (-3 u.F + 3 cF + 9 cu cF)
// and opposite pairs (i, i+1) share the even part in cu and differ in the
// sign of the odd part.  The weight w and the relaxation factors are folded
// into per-class constants, so a pair costs a few fused multiply-adds.
template <class R>
__host__ __device__ __forceinline__ R collide_site(const Params<R>& P, R g[19], const R F[3], R u[3]) {
  R drho = g[0];
#pragma unroll
  for (int i = 1; i < 19; ++i) drho += g[i];
  const R e1 = g[1] - g[2], e3 = g[3] - g[4], e5 = g[5] - g[6], e7 = g[7] - g[8], e9 = g[9] - g[10];
  const R e11 = g[11] - g[12], e13 = g[13] - g[14], e15 = g[15] - g[16], e17 = g[17] - g[18];
  const R jx = e1 + e7 + e9 + e11 + e13;
  const R jy = e3 + e7 - e9 + e15 + e17;
  const R jz = e5 + e11 - e13 + e15 - e17;
  const R rho = P.rho0 + drho;
  const R inv = R(1) / rho;
  u[0] = (jx + R(0.5) * F[0]) * inv;
  u[1] = (jy + R(0.5) * F[1]) * inv;
  u[2] = (jz + R(0.5) * F[2]) * inv;
  const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const R uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
  const R om = P.omega, om1 = R(1) - P.omega;
  // w-free coefficients: even = w (base + cu (a45 cu + g9 cF)), odd = w (r3 cu + g3 cF)
  const R base = om * (drho - R(1.5) * rho * uu) - R(3) * P.guo * uF;
  const R a45 = R(4.5) * om * rho, g9 = R(9) * P.guo;
  const R r3 = R(3) * om * rho, g3 = R(3) * P.guo;
  R cb[2], ca[2], cg9[2], cr[2], cg3[2];  // class 0: axis (w = 1/18), class 1: edge (w = 1/36)
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const R w = WQ<R>(k == 0 ? 1 : 7);
    cb[k] = w * base;
    ca[k] = w * a45;
    cg9[k] = w * g9;
    cr[k] = w * r3;
    cg3[k] = w * g3;
  }
  g[0] = om1 * g[0] + WQ<R>(0) * base;
#pragma unroll
  for (int i = 1; i < 19; i += 2) {
    const int k = i < 7 ? 0 : 1;
    const R cu = cdot(CX(i), CY(i), CZ(i), u);
    const R cF = cdot(CX(i), CY(i), CZ(i), F);
    const R even = cb[k] + cu * (ca[k] * cu + cg9[k] * cF);
    const R odd = cr[k] * cu + cg3[k] * cF;
    const R gi = g[i], gj = g[i + 1];
    g[i] = (om1 * gi + even) + odd;
    g[i + 1] = (om1 * gj + even) - odd;
  }
  return drho;
}

// BGK collision of the paper's scheme on the 15 D3Q15 deviations g (in place).
// The symmetric stress S (xx, xy, xz, yy, yz, zz) sits in the equilibrium,
//   g_eq_i = w (drho + 3 rho cu + 9/2 c.T.c - 3/2 tr T),  T = rho u u - S,
// and F (the force of the antisymmetric stress plus the body force) enters as
// the Guo source guo w (-3 u.F + 3 cF + 9 cu cF) with u = (sum c g + F/2)/rho.
// Opposite pairs (i, i+1) share the even part, as in collide_site.
template <class R>
__host__ __device__ __forceinline__ R collide_site_eq(const Params<R>& P, R g[15], const R F[3], const R S[6],
                                                      R u[3]) {
  using L = D3Q15;
  R drho = g[0];
#pragma unroll
  for (int i = 1; i < 15; ++i) drho += g[i];
  R j[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 1; i < 15; i += 2) {
    const R e = g[i] - g[i + 1];
    cadd(L::cx(i), e, j[0]);
    cadd(L::cy(i), e, j[1]);
    cadd(L::cz(i), e, j[2]);
  }
  const R rho = P.rho0 + drho;
  const R inv = R(1) / rho;
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = (j[a] + R(0.5) * F[a]) * inv;
  const R Txx = rho * u[0] * u[0] - S[0], Txy = rho * u[0] * u[1] - S[1], Txz = rho * u[0] * u[2] - S[2];
  const R Tyy = rho * u[1] * u[1] - S[3], Tyz = rho * u[1] * u[2] - S[4], Tzz = rho * u[2] * u[2] - S[5];
  const R trT = Txx + Tyy + Tzz;
  const R uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
  const R om = P.omega, om1 = R(1) - P.omega;
  const R base = om * (drho - R(1.5) * trT) - R(3) * P.guo * uF;
  const R a45 = R(4.5) * om, g9 = R(9) * P.guo, r3 = R(3) * om * rho, g3 = R(3) * P.guo;
  g[0] = om1 * g[0] + L::w<R>(0) * base;
#pragma unroll
  for (int i = 1; i < 15; i += 2) {
    const int ex = L::cx(i), ey = L::cy(i), ez = L::cz(i);
    const R cu = cdot(ex, ey, ez, u);
    const R cF = cdot(ex, ey, ez, F);
    R cd = R(-0.0), co = R(-0.0);  // c.T.c = sum c_a^2 T_aa + 2 sum_{a<b} c_a c_b T_ab
    cadd(ex * ex, Txx, cd);
    cadd(ey * ey, Tyy, cd);
    cadd(ez * ez, Tzz, cd);
    cadd(ex * ey, Txy, co);
    cadd(ex * ez, Txz, co);
    cadd(ey * ez, Tyz, co);
    const R cTc = cd + R(2) * co;
    const R w = L::w<R>(i);
    const R even = w * (base + a45 * cTc + g9 * cu * cF);
    const R odd = w * (r3 * cu + g3 * cF);
    const R gi = g[i], gj = g[i + 1];
    g[i] = (om1 * gi + even) + odd;
    g[i + 1] = (om1 * gj + even) - odd;
  }
  return drho;
}

}  // namespace lbc
