// Reverse-mode derivatives (vector-Jacobian products) of the per-site physics.
//
// Each *_bwd function recomputes the forward intermediates it needs from the
// same inputs as its forward counterpart in physics.hpp and accumulates (+=)
// the adjoints of those inputs, given the adjoints of the outputs.  The
// derivatives are written out by hand, statement by statement in reverse
// order of the forward code; the host build of this header is checked against
// central differences of the forward functions.
#pragma once
#include "physics.hpp"

namespace lbc {

// Adjoint of the gradient data of one site.
template <class R>
struct GradBar {
  R phi, dphi[3], lapphi, divv, q[5], dq[3][5], lapq[5];
  __host__ __device__ void zero() {
    phi = lapphi = divv = R(0);
    for (int g = 0; g < 3; ++g) {
      dphi[g] = R(0);
      for (int k = 0; k < 5; ++k) dq[g][k] = R(0);
    }
    for (int k = 0; k < 5; ++k) q[k] = lapq[k] = R(0);
  }
};

// Parameter adjoints accumulated per site.
template <class R>
struct ParBar {
  R zeta, kq, kq2;  // kq = 2 K q0, kq2 = 4 K q0^2
};

// Adjoint of the 9 entries of a symmetric traceless tensor (treated as
// independent) pulled back to its 5 stored components (zz = -xx - yy).
template <class R>
__host__ __device__ __forceinline__ void full_to_stored(const R T[3][3], R out[5]) {
  out[0] += T[0][0] - T[2][2];
  out[1] += T[0][1] + T[1][0];
  out[2] += T[0][2] + T[2][0];
  out[3] += T[1][1] - T[2][2];
  out[4] += T[1][2] + T[2][1];
}

// Reverse of Q.Q (6 entries), tr2 = tr(Q^2), tr3 = tr(Q^3) as computed in
// local_thermo / mu_site; accumulates into the stored-component adjoint qb.
template <class R>
__host__ __device__ __forceinline__ void invariants_bwd(const R q[5], R q2b[6], R tr2b, R tr3b, R qb[5]) {
  const R xx = q[0], xy = q[1], xz = q[2], yy = q[3], yz = q[4], zz = -xx - yy;
  const R q2xx = xx * xx + xy * xy + xz * xz;
  const R q2xy = xx * xy + xy * yy + xz * yz;
  const R q2xz = xx * xz + xy * yz + xz * zz;
  const R q2yy = xy * xy + yy * yy + yz * yz;
  const R q2yz = xy * xz + yy * yz + yz * zz;
  const R q2zz = xz * xz + yz * yz + zz * zz;
  // q2b order: xx, xy, xz, yy, yz, zz
  R xxb = R(0), xyb = R(0), xzb = R(0), yyb = R(0), yzb = R(0), zzb = R(0);
  // tr3 = xx q2xx + yy q2yy + zz q2zz + 2 (xy q2xy + xz q2xz + yz q2yz)
  xxb += q2xx * tr3b;
  yyb += q2yy * tr3b;
  zzb += q2zz * tr3b;
  xyb += R(2) * q2xy * tr3b;
  xzb += R(2) * q2xz * tr3b;
  yzb += R(2) * q2yz * tr3b;
  q2b[0] += xx * tr3b;
  q2b[3] += yy * tr3b;
  q2b[5] += zz * tr3b;
  q2b[1] += R(2) * xy * tr3b;
  q2b[2] += R(2) * xz * tr3b;
  q2b[4] += R(2) * yz * tr3b;
  // tr2 = q2xx + q2yy + q2zz
  q2b[0] += tr2b;
  q2b[3] += tr2b;
  q2b[5] += tr2b;
  // q2xx = xx^2 + xy^2 + xz^2
  xxb += R(2) * xx * q2b[0];
  xyb += R(2) * xy * q2b[0];
  xzb += R(2) * xz * q2b[0];
  // q2xy = xx xy + xy yy + xz yz
  xxb += xy * q2b[1];
  xyb += (xx + yy) * q2b[1];
  yyb += xy * q2b[1];
  xzb += yz * q2b[1];
  yzb += xz * q2b[1];
  // q2xz = xx xz + xy yz + xz zz
  xxb += xz * q2b[2];
  xzb += (xx + zz) * q2b[2];
  xyb += yz * q2b[2];
  yzb += xy * q2b[2];
  zzb += xz * q2b[2];
  // q2yy = xy^2 + yy^2 + yz^2
  xyb += R(2) * xy * q2b[3];
  yyb += R(2) * yy * q2b[3];
  yzb += R(2) * yz * q2b[3];
  // q2yz = xy xz + yy yz + yz zz
  xyb += xz * q2b[4];
  xzb += xy * q2b[4];
  yyb += yz * q2b[4];
  yzb += (yy + zz) * q2b[4];
  zzb += yz * q2b[4];
  // q2zz = xz^2 + yz^2 + zz^2
  xzb += R(2) * xz * q2b[5];
  yzb += R(2) * yz * q2b[5];
  zzb += R(2) * zz * q2b[5];
  // zz = -xx - yy
  xxb -= zzb;
  yyb -= zzb;
  qb[0] += xxb;
  qb[1] += xyb;
  qb[2] += xzb;
  qb[3] += yyb;
  qb[4] += yzb;
}

// Reverse of local_thermo: adjoints of h[5], tr2, tr3, qc, dp2, chi -> G.
template <class R>
__host__ __device__ __forceinline__ void local_thermo_bwd(const Params<R>& P, const Grad<R>& G, const Local<R>& L,
                                                          const R hb[5], R tr2b, R tr3b, R qcb, R dp2b, R chib,
                                                          GradBar<R>& Gb, ParBar<R>& Pb) {
  const R xx = L.xx, xy = L.xy, xz = L.xz, yy = L.yy, yz = L.yz, zz = L.zz;
  const R dx = G.dphi[0], dy = G.dphi[1], dz = G.dphi[2];
  const R kq = R(2) * P.K * P.q0;
  const R c1 = R(1) - L.chi * C3<R>::third;
  const R alpha = -P.A0 * (c1 + L.chi * L.tr2) - R(4) * P.K * P.q0 * P.q0;
  const R beta = P.A0 * L.chi;
  const R t3 = L.tr2 * C3<R>::third;
  R xxb = R(0), xyb = R(0), xzb = R(0), yyb = R(0), yzb = R(0), zzb = R(0);
  R q2b[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
  // h_k = alpha Q_k + beta (Q2_k - delta t3) + K lapq_k - kq S_k - W (dd_k - delta dp2/3)
  const R alphab = hb[0] * xx + hb[1] * xy + hb[2] * xz + hb[3] * yy + hb[4] * yz;
  const R betab = hb[0] * (L.q2xx - t3) + hb[1] * L.q2xy + hb[2] * L.q2xz + hb[3] * (L.q2yy - t3) + hb[4] * L.q2yz;
  xxb += alpha * hb[0];
  xyb += alpha * hb[1];
  xzb += alpha * hb[2];
  yyb += alpha * hb[3];
  yzb += alpha * hb[4];
  q2b[0] += beta * hb[0];
  q2b[1] += beta * hb[1];
  q2b[2] += beta * hb[2];
  q2b[3] += beta * hb[3];
  q2b[4] += beta * hb[4];
  const R t3b = -beta * (hb[0] + hb[3]);
#pragma unroll
  for (int k = 0; k < 5; ++k) Gb.lapq[k] += P.K * hb[k];
  R cxxb = -R(2) * kq * hb[0], cyyb = -R(2) * kq * hb[3];
  R sxyb = -kq * hb[1], sxzb = -kq * hb[2], syzb = -kq * hb[4];
  Pb.kq -= R(2) * L.cxx * hb[0] + L.sxy * hb[1] + L.sxz * hb[2] + R(2) * L.cyy * hb[3] + L.syz * hb[4];
  R dxb = -P.W * (R(2) * dx * hb[0] + dy * hb[1] + dz * hb[2]);
  R dyb = -P.W * (dx * hb[1] + R(2) * dy * hb[3] + dz * hb[4]);
  R dzb = -P.W * (dx * hb[2] + dy * hb[4]);
  const R dd3b = P.W * (hb[0] + hb[3]);
  // t3 = tr2/3, dd3 = dp2/3
  tr2b += t3b * C3<R>::third;
  dp2b += dd3b * C3<R>::third;
  // beta = A0 chi; alpha = -A0 (c1 + chi tr2) - kq2
  chib += P.A0 * betab;
  const R c1b = -P.A0 * alphab;
  chib += -P.A0 * L.tr2 * alphab;
  tr2b += -P.A0 * L.chi * alphab;
  Pb.kq2 -= alphab;
  (void)c1;
  // c1 = 1 - chi/3
  chib -= c1b * C3<R>::third;
  // chi = chi0 + chi_s phi
  Gb.phi += P.chi_s * chib;
  // dp2 = dx^2 + dy^2 + dz^2
  dxb += R(2) * dx * dp2b;
  dyb += R(2) * dy * dp2b;
  dzb += R(2) * dz * dp2b;
  Gb.dphi[0] += dxb;
  Gb.dphi[1] += dyb;
  Gb.dphi[2] += dzb;
  // qc = xx cxx + yy cyy + zz czz + xy sxy + xz sxz + yz syz
  const R czz = -L.cxx - L.cyy;
  xxb += L.cxx * qcb;
  yyb += L.cyy * qcb;
  zzb += czz * qcb;
  xyb += L.sxy * qcb;
  xzb += L.sxz * qcb;
  yzb += L.syz * qcb;
  cxxb += xx * qcb;
  cyyb += yy * qcb;
  const R czzb = zz * qcb;
  sxyb += xy * qcb;
  sxzb += xz * qcb;
  syzb += yz * qcb;
  // czz = -cxx - cyy
  cxxb -= czzb;
  cyyb -= czzb;
  // cxx = d1[2] - d2[1]; cyy = d2[1] - d0[4]
  R* d0b = Gb.dq[0];
  R* d1b = Gb.dq[1];
  R* d2b = Gb.dq[2];
  d1b[2] += cxxb;
  d2b[1] -= cxxb;
  d2b[1] += cyyb;
  d0b[4] -= cyyb;
  // sxy = (d1[4] - d2[3]) + (d2[0] - d0[2])
  d1b[4] += sxyb;
  d2b[3] -= sxyb;
  d2b[0] += sxyb;
  d0b[2] -= sxyb;
  // sxz = (d1zz - d2[4]) + (d0[1] - d1[0]), d1zz = -d1[0] - d1[3]
  d1b[0] -= sxzb;
  d1b[3] -= sxzb;
  d2b[4] -= sxzb;
  d0b[1] += sxzb;
  d1b[0] -= sxzb;
  // syz = (d2[2] - d0zz) + (d0[3] - d1[1]), d0zz = -d0[0] - d0[3]
  d2b[2] += syzb;
  d0b[0] += syzb;
  d0b[3] += syzb;
  d0b[3] += syzb;
  d1b[1] -= syzb;
  // zz = -xx - yy (then the invariants)
  xxb -= zzb;
  yyb -= zzb;
  Gb.q[0] += xxb;
  Gb.q[1] += xyb;
  Gb.q[2] += xzb;
  Gb.q[3] += yyb;
  Gb.q[4] += yzb;
  invariants_bwd(G.q, q2b, tr2b, tr3b, Gb.q);
}

// The reverse of mu_site except its path through Q: accumulates the phi,
// lapphi and divv adjoints and the adjoints of tr(Q^2) (tr2b) and tr(Q^3)
// (tr3b), so that a caller which also reverses H reverses the invariants once.
//   mu = a phi (phi - phi0)(2 phi - phi0) ipc2 + A0 chi_s (-tr2/6 - tr3/3 + tr2^2/4)
//        - k_phi lapphi - 2 W divv
template <class R>
__host__ __device__ __forceinline__ void mu_site_bwd_local(const Params<R>& P, R phi, R tr2, R mub, R& phib,
                                                           R& lapphib, R& divvb, R& tr2b, R& tr3b) {
  phib += P.a * P.inv_phicr2 * (R(6) * phi * phi - R(6) * phi * P.phi0 + P.phi0 * P.phi0) * mub;
  tr2b += P.A0 * P.chi_s * (-C3<R>::sixth + R(0.5) * tr2) * mub;
  tr3b -= P.A0 * P.chi_s * C3<R>::third * mub;
  lapphib -= P.k_phi * mub;
  divvb -= R(2) * P.W * mub;
}

// Reverse of sigma_site: adjoint of the stress (sb[3*a+b]), of the
// molecular field output (hb_out[5], e.g. from the Beris-Edwards update) and
// of the chemical potential mu_site at the same site (mub; its divv adjoint
// goes to Gb.divv) -> gradient-data adjoint and parameter adjoints.  mu shares
// tr(Q^2) and tr(Q^3) with H, so their reverse through Q runs once.  MU =
// false: no mu adjoint (mub is ignored and its terms are not formed).
template <class R, bool MU = true>
__host__ __device__ __forceinline__ void sigma_site_bwd(const Params<R>& P, const Grad<R>& G, const R sb[9],
                                                        const R hb_out[5], GradBar<R>& Gb, ParBar<R>& Pb,
                                                        R mub = R(0)) {
  Local<R> L;
  local_thermo(P, G, L);
  const R xx = L.xx, xy = L.xy, xz = L.xz, yy = L.yy, yz = L.yz, zz = L.zz;
  const R dp[3] = {G.dphi[0], G.dphi[1], G.dphi[2]};
  const R kq = R(2) * P.K * P.q0;
  const R kq2 = R(4) * P.K * P.q0 * P.q0;
  // forward intermediates
  const R Qm[3][3] = {{xx, xy, xz}, {xy, yy, yz}, {xz, yz, zz}};
  const R Qd[3] = {xx * dp[0] + xy * dp[1] + xz * dp[2], xy * dp[0] + yy * dp[1] + yz * dp[2],
                   xz * dp[0] + yz * dp[1] + zz * dp[2]};
  const R dw = G.phi * (G.phi - P.phi0);
  const R c1 = R(1) - L.chi * C3<R>::third;
  const R hxx = L.h[0], hxy = L.h[1], hxz = L.h[2], hyy = L.h[3], hyz = L.h[4], hzz = -hxx - hyy;
  const R Hm[3][3] = {{hxx, hxy, hxz}, {hxy, hyy, hyz}, {hxz, hyz, hzz}};
  R QH[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) QH[a][b] = Qm[a][0] * Hm[0][b] + Qm[a][1] * Hm[1][b] + Qm[a][2] * Hm[2][b];
  const R qh = QH[0][0] + QH[1][1] + QH[2][2];
  const R xi = P.xi;
  const R cA = -(xi + R(1)), cB = R(1) - xi, cH = -R(2) * xi * C3<R>::third;
  const R cQ = R(2) * xi * qh - P.zeta * G.phi;
  const R t[3] = {P.k_phi * dp[0] + R(2) * P.W * Qd[0], P.k_phi * dp[1] + R(2) * P.W * Qd[1],
                  P.k_phi * dp[2] + R(2) * P.W * Qd[2]};

  // ---- reverse of sig_ab = -dp_a t_b - K D_ab - kq ax_ab + cA QH_ba + cB QH_ab + cH H_ab + cQ Q_ab + d_ab iso
  // (the ax term is reversed below with sb itself as the cotangent, then scaled by -kq)
  R Qmb[3][3] = {}, Hmb[3][3] = {}, QHb[3][3] = {}, Db[3][3] = {};
  R dpb[3] = {R(0), R(0), R(0)}, tb[3] = {R(0), R(0), R(0)};
  R cQb = R(0);
  const R isob = sb[0] + sb[4] + sb[8];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const R s = sb[3 * a + b];
      dpb[a] -= s * t[b];
      tb[b] -= s * dp[a];
      Db[a][b] -= P.K * s;
      QHb[b][a] += cA * s;
      QHb[a][b] += cB * s;
      Hmb[a][b] += cH * s;
      Qmb[a][b] += cQ * s;
      cQb += s * Qm[a][b];
    }
  // iso = fc - cH qh
  R fcb = isob;
  R qhb = -cH * isob;
  // cQ = 2 xi qh - zeta phi
  qhb += R(2) * xi * cQb;
  Gb.phi -= P.zeta * cQb;
  Pb.zeta -= G.phi * cQb;
  // t_b = k_phi dp_b + 2 W Qd_b
  R Qdb[3];
  for (int b = 0; b < 3; ++b) {
    dpb[b] += P.k_phi * tb[b];
    Qdb[b] = R(2) * P.W * tb[b];
  }
  // qh = tr(QH); QH = Q H
  for (int a = 0; a < 3; ++a) QHb[a][a] += qhb;
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      R sq = R(0), sh = R(0);
      for (int b = 0; b < 3; ++b) {
        sq += QHb[a][b] * Hm[c][b];  // dQ_ac
        sh += Qm[b][a] * QHb[b][c];  // dH_ac
      }
      Qmb[a][c] += sq;
      Hmb[a][c] += sh;
    }
  // fc = (a/2) dw^2 ipc2 + A0 ((1/2) c1 tr2 - chi/3 tr3 + chi/4 tr2^2) + (1/2) kq2 tr2
  //      + (1/2) k_phi dp2 + (1/2) K (D00 + D11 + D22) + kq qc + W anch
  const R dwb = P.a * dw * P.inv_phicr2 * fcb;
  const R c1b = P.A0 * R(0.5) * L.tr2 * fcb;
  R tr2b = (P.A0 * (R(0.5) * c1 + R(0.5) * L.chi * L.tr2) + R(0.5) * kq2) * fcb;
  R tr3b = -P.A0 * L.chi * C3<R>::third * fcb;
  R chib = P.A0 * (-L.tr3 * C3<R>::third + R(0.25) * L.tr2 * L.tr2) * fcb;
  chib -= c1b * C3<R>::third;
  Pb.kq2 += R(0.5) * L.tr2 * fcb;
  R dp2b = R(0.5) * P.k_phi * fcb;
  for (int a = 0; a < 3; ++a) Db[a][a] += R(0.5) * P.K * fcb;
  Pb.kq += L.qc * fcb;
  const R qcb = kq * fcb;
  const R anchb = P.W * fcb;
  // dw = phi (phi - phi0)
  Gb.phi += (R(2) * G.phi - P.phi0) * dwb;
  // anch = dp . Qd
  for (int b = 0; b < 3; ++b) {
    dpb[b] += Qd[b] * anchb;
    Qdb[b] += dp[b] * anchb;
  }
  // Qd_b = Q_bc dp_c
  for (int b = 0; b < 3; ++b)
    for (int c = 0; c < 3; ++c) {
      Qmb[b][c] += Qdb[b] * dp[c];
      dpb[c] += Qm[b][c] * Qdb[b];
    }
  // ax (per a), from dq[a] and Q, bilinear: with sb as its cotangent the reverse
  // gives r = d(sb:ax)/d(dq, Q); the stress takes -kq ax, so G.dq and Q get
  // -kq r, and since ax is linear in dq, sb:ax = sum r_dq . dq (kq's adjoint)
  R qb5[5] = {R(0), R(0), R(0), R(0), R(0)};
  R xxb = R(0), xyb = R(0), xzb = R(0), yyb = R(0), yzb = R(0), zzb = R(0);
  R sax = R(0);
  for (int a = 0; a < 3; ++a) {
    const R dxx = G.dq[a][0], dxy = G.dq[a][1], dxz = G.dq[a][2], dyy = G.dq[a][3], dyz = G.dq[a][4];
    const R dzz = -dxx - dyy;
    const R a0b = sb[3 * a], a1b = sb[3 * a + 1], a2b = sb[3 * a + 2];
    R dxxb = R(0), dxyb = R(0), dxzb = R(0), dyyb = R(0), dyzb = R(0), dzzb = R(0);
    // ax0 = (dxy xz + dyy yz + dyz zz) - (dxz xy + dyz yy + dzz yz)
    dxyb += a0b * xz; xzb += a0b * dxy;
    dyyb += a0b * yz; yzb += a0b * dyy;
    dyzb += a0b * zz; zzb += a0b * dyz;
    dxzb -= a0b * xy; xyb -= a0b * dxz;
    dyzb -= a0b * yy; yyb -= a0b * dyz;
    dzzb -= a0b * yz; yzb -= a0b * dzz;
    // ax1 = (dxz xx + dyz xy + dzz xz) - (dxx xz + dxy yz + dxz zz)
    dxzb += a1b * xx; xxb += a1b * dxz;
    dyzb += a1b * xy; xyb += a1b * dyz;
    dzzb += a1b * xz; xzb += a1b * dzz;
    dxxb -= a1b * xz; xzb -= a1b * dxx;
    dxyb -= a1b * yz; yzb -= a1b * dxy;
    dxzb -= a1b * zz; zzb -= a1b * dxz;
    // ax2 = (dxx xy + dxy yy + dxz yz) - (dxy xx + dyy xy + dyz xz)
    dxxb += a2b * xy; xyb += a2b * dxx;
    dxyb += a2b * yy; yyb += a2b * dxy;
    dxzb += a2b * yz; yzb += a2b * dxz;
    dxyb -= a2b * xx; xxb -= a2b * dxy;
    dyyb -= a2b * xy; xyb -= a2b * dyy;
    dyzb -= a2b * xz; xzb -= a2b * dyz;
    // dzz = -dxx - dyy
    dxxb -= dzzb;
    dyyb -= dzzb;
    sax += dxxb * dxx + dxyb * dxy + dxzb * dxz + dyyb * dyy + dyzb * dyz;
    Gb.dq[a][0] -= kq * dxxb;
    Gb.dq[a][1] -= kq * dxyb;
    Gb.dq[a][2] -= kq * dxzb;
    Gb.dq[a][3] -= kq * dyyb;
    Gb.dq[a][4] -= kq * dyzb;
  }
  Pb.kq -= sax;
  // D_ab = dq[a] : dq[b] = dq[a]^T J dq[b] with J the metric of sdot, so
  // dq_bar[a] += J sum_b (Db_ab + Db_ba) dq[b]
  for (int a = 0; a < 3; ++a) {
    R T[5];
    for (int k = 0; k < 5; ++k) T[k] = R(0);
    for (int b = 0; b < 3; ++b) {
      const R m = Db[a][b] + Db[b][a];
      for (int k = 0; k < 5; ++k) T[k] += m * G.dq[b][k];
    }
    Gb.dq[a][0] += R(2) * T[0] + T[3];
    Gb.dq[a][1] += R(2) * T[1];
    Gb.dq[a][2] += R(2) * T[2];
    Gb.dq[a][3] += T[0] + R(2) * T[3];
    Gb.dq[a][4] += R(2) * T[4];
  }
  // Q from its explicit uses (Qm and the ax/xx.. scalars) -> stored components
  xxb -= zzb;
  yyb -= zzb;
  qb5[0] -= kq * xxb;
  qb5[1] -= kq * xyb;
  qb5[2] -= kq * xzb;
  qb5[3] -= kq * yyb;
  qb5[4] -= kq * yzb;
  full_to_stored(Qmb, qb5);
  for (int k = 0; k < 5; ++k) Gb.q[k] += qb5[k];
  for (int g = 0; g < 3; ++g) Gb.dphi[g] += dpb[g];
  // H -> stored components, plus the adjoint of the molecular-field output
  R hb[5] = {hb_out[0], hb_out[1], hb_out[2], hb_out[3], hb_out[4]};
  full_to_stored(Hmb, hb);
  if constexpr (MU) mu_site_bwd_local(P, G.phi, L.tr2, mub, Gb.phi, Gb.lapphi, Gb.divv, tr2b, tr3b);
  // back through local_thermo
  local_thermo_bwd(P, G, L, hb, tr2b, tr3b, qcb, dp2b, chib, Gb, Pb);
}

// Reverse of mu_site(phi, lapphi, divv, q).
template <class R>
__host__ __device__ __forceinline__ void mu_site_bwd(const Params<R>& P, R phi, const R q[5], R mub, R& phib,
                                                     R& lapphib, R& divvb, R qb[5]) {
  const R xx = q[0], xy = q[1], xz = q[2], yy = q[3], yz = q[4], zz = -xx - yy;
  const R tr2 = (xx * xx + xy * xy + xz * xz) + (xy * xy + yy * yy + yz * yz) + (xz * xz + yz * yz + zz * zz);
  R tr2b = R(0), tr3b = R(0);
  mu_site_bwd_local(P, phi, tr2, mub, phib, lapphib, divvb, tr2b, tr3b);
  R q2b[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
  invariants_bwd(q, q2b, tr2b, tr3b, qb);
}

// Reverse of corotation_site: s5b -> qb (stored components) and Wb (3x3).
template <class R>
__host__ __device__ __forceinline__ void corotation_site_bwd(R xi, const R q[5], const R W[3][3], const R s5b[5],
                                                             R qb[5], R Wb[3][3]) {
  const R xx = q[0], xy = q[1], xz = q[2], yy = q[3], yz = q[4], zz = -xx - yy;
  const R Pm[3][3] = {{xx + C3<R>::third, xy, xz}, {xy, yy + C3<R>::third, yz}, {xz, yz, zz + C3<R>::third}};
  const R Qm[3][3] = {{xx, xy, xz}, {xy, yy, yz}, {xz, yz, zz}};
  R A[3][3];
  R trQW = R(0);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      A[a][b] = R(0.5) * ((xi + R(1)) * W[a][b] + (xi - R(1)) * W[b][a]);
      trQW += Qm[a][b] * W[b][a];
    }
  const R c = R(2) * xi * trQW;
  // s5: xx = S_xx - tr/3, xy = S_xy, xz = S_xz, yy = S_yy - tr/3, yz = S_yz
  const R tb = -(s5b[0] + s5b[3]) * C3<R>::third;
  const R Sb_diag[3] = {s5b[0] + tb, s5b[3] + tb, tb};
  R Mb[3][3] = {}, Pmb[3][3] = {};
  R cb = R(0);
  // S_aa = 2 M_aa - c Pm_aa
  for (int a = 0; a < 3; ++a) {
    Mb[a][a] += R(2) * Sb_diag[a];
    cb -= Sb_diag[a] * Pm[a][a];
    Pmb[a][a] -= c * Sb_diag[a];
  }
  // S_ab = M_ab + M_ba - c Pm_ab for (0,1), (0,2), (1,2)
  const int oa[3] = {0, 0, 1}, ob[3] = {1, 2, 2};
  const R ofs[3] = {s5b[1], s5b[2], s5b[4]};
  for (int k = 0; k < 3; ++k) {
    const int a = oa[k], b = ob[k];
    Mb[a][b] += ofs[k];
    Mb[b][a] += ofs[k];
    cb -= ofs[k] * Pm[a][b];
    Pmb[a][b] -= c * ofs[k];
  }
  // M = A Pm
  R Ab[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      R sa = R(0), sp = R(0);
      for (int k = 0; k < 3; ++k) {
        sa += Mb[a][k] * Pm[b][k];  // dA_ab = sum_k Mb_ak Pm_bk
        sp += A[k][a] * Mb[k][b];   // dPm_ab = sum_k A_ka Mb_kb
      }
      Ab[a][b] = sa;
      Pmb[a][b] += sp;
    }
  // c = 2 xi trQW; trQW = sum Q_ab W_ba
  const R trb = R(2) * xi * cb;
  R Qb[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      Qb[a][b] = Pmb[a][b] + trb * W[b][a];
      Wb[b][a] += trb * Qm[a][b];
    }
  // A_ab = (1/2)((xi+1) W_ab + (xi-1) W_ba)
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      Wb[a][b] += R(0.5) * (xi + R(1)) * Ab[a][b];
      Wb[b][a] += R(0.5) * (xi - R(1)) * Ab[a][b];
    }
  full_to_stored(Qb, qb);
}

// The W part of corotation_site_bwd alone.  S is linear in W, so its W
// adjoint depends on Q and on the adjoint s5b of S only:
//   Wb = (xi+1)/2 Ab + (xi-1)/2 Ab^T + 2 xi cb Q,   Ab = Mb P,
// with Mb the symmetric tensor whose diagonal is twice the trace-projected
// diagonal of s5b and whose off-diagonals are those of s5b, and
// cb = -(the diagonal and each off-diagonal of the projected s5b, once) : P.
template <class R>
__host__ __device__ __forceinline__ void corotation_wbar(R xi, const R q[5], const R s5b[5], R Wb[3][3]) {
  const R xx = q[0], xy = q[1], xz = q[2], yy = q[3], yz = q[4], zz = -xx - yy;
  const R Pm[3][3] = {{xx + C3<R>::third, xy, xz}, {xy, yy + C3<R>::third, yz}, {xz, yz, zz + C3<R>::third}};
  const R Qm[3][3] = {{xx, xy, xz}, {xy, yy, yz}, {xz, yz, zz}};
  const R tb = -(s5b[0] + s5b[3]) * C3<R>::third;
  const R d[3] = {s5b[0] + tb, s5b[3] + tb, tb};
  const R Mb[3][3] = {{R(2) * d[0], s5b[1], s5b[2]}, {s5b[1], R(2) * d[1], s5b[4]}, {s5b[2], s5b[4], R(2) * d[2]}};
  const R cb = -((d[0] * Pm[0][0] + d[1] * Pm[1][1] + d[2] * Pm[2][2]) +
                 (s5b[1] * Pm[0][1] + s5b[2] * Pm[0][2] + s5b[4] * Pm[1][2]));
  R Ab[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) Ab[a][b] = Mb[a][0] * Pm[b][0] + Mb[a][1] * Pm[b][1] + Mb[a][2] * Pm[b][2];
  const R trb = R(2) * xi * cb;
  const R cp = R(0.5) * (xi + R(1)), cm = R(0.5) * (xi - R(1));
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) Wb[a][b] = (cp * Ab[a][b] + cm * Ab[b][a]) + trb * Qm[a][b];
}

// Reverse of collide_site from the moments of the pre-collision populations:
// drho = sum g, u = (j + F/2)/rho (rho = rho0 + drho), the force F, the
// adjoint of the post-collision populations gsb[19] and of the velocity
// output ub_in[3]; writes the adjoint of the pre-collision populations gb[19]
// and accumulates Fb[3].  The populations enter the collision only through
// drho and j, so their moments are all the reverse needs.
template <class R>
__host__ __device__ __forceinline__ void collide_site_bwd_m(const Params<R>& P, R drho, const R u[3], const R F[3],
                                                            const R gsb[19], const R ub_in[3], R gb[19], R Fb[3]) {
  const R rho = P.rho0 + drho;
  const R inv = R(1) / rho;
  const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const R om = P.omega, om1 = R(1) - P.omega;
  // g*_i = om1 g_i + w_i [om (A + 3 rho cu_i + 4.5 rho cu_i^2) + guo (Bs + 3 cF_i + 9 cu_i cF_i)]
  // A = drho - 1.5 rho uu, Bs = -3 uF
  R Ab = R(0), Bsb = R(0), rhob = R(0);
  R ub[3] = {ub_in[0], ub_in[1], ub_in[2]};
  for (int i = 0; i < 19; ++i) {
    const R cu = cdot(CX(i), CY(i), CZ(i), u);
    const R cF = cdot(CX(i), CY(i), CZ(i), F);
    const R e = WQ<R>(i) * gsb[i];
    gb[i] = om1 * gsb[i];
    Ab += om * e;
    Bsb += P.guo * e;
    rhob += om * e * (R(3) * cu + R(4.5) * cu * cu);
    const R cub = e * (om * (R(3) * rho + R(9) * rho * cu) + P.guo * R(9) * cF);
    const R cFb = e * P.guo * (R(3) + R(9) * cu);
    cadd(CX(i), cub, ub[0]);
    cadd(CY(i), cub, ub[1]);
    cadd(CZ(i), cub, ub[2]);
    cadd(CX(i), cFb, Fb[0]);
    cadd(CY(i), cFb, Fb[1]);
    cadd(CZ(i), cFb, Fb[2]);
  }
  R drhob = Ab;
  rhob += R(-1.5) * uu * Ab;
  const R uub = R(-1.5) * rho * Ab;
  const R uFb = R(-3) * Bsb;
  for (int a = 0; a < 3; ++a) {
    ub[a] += R(2) * u[a] * uub + F[a] * uFb;
    Fb[a] += u[a] * uFb;
  }
  // u = (j + F/2) / rho
  R jb[3];
  for (int a = 0; a < 3; ++a) {
    jb[a] = ub[a] * inv;
    Fb[a] += R(0.5) * ub[a] * inv;
    rhob -= ub[a] * u[a] * inv;
  }
  drhob += rhob;
  for (int i = 0; i < 19; ++i) {
    R t = drhob;
    cadd(CX(i), jb[0], t);
    cadd(CY(i), jb[1], t);
    cadd(CZ(i), jb[2], t);
    gb[i] += t;
  }
}

// Reverse of collide_site from the pre-collision populations g[19].
template <class R>
__host__ __device__ __forceinline__ void collide_site_bwd(const Params<R>& P, const R g[19], const R F[3],
                                                          const R gsb[19], const R ub_in[3], R gb[19], R Fb[3]) {
  R drho = R(0);
  for (int i = 0; i < 19; ++i) drho += g[i];
  R j[3] = {R(0), R(0), R(0)};
  for (int i = 0; i < 19; ++i) {
    cadd(CX(i), g[i], j[0]);
    cadd(CY(i), g[i], j[1]);
    cadd(CZ(i), g[i], j[2]);
  }
  const R inv = R(1) / (P.rho0 + drho);
  R u[3];
  for (int a = 0; a < 3; ++a) u[a] = (j[a] + R(0.5) * F[a]) * inv;
  collide_site_bwd_m(P, drho, u, F, gsb, ub_in, gb, Fb);
}

// Reverse of collide_site_eq (the paper's D3Q15 scheme with the symmetric
// stress S in the equilibrium) from the moments drho and u:
//   g*_i = om1 g_i + w_i [om (drho - 1.5 trT + 3 rho cu_i + 4.5 c.T.c) + guo (-3 uF + 3 cF_i + 9 cu_i cF_i)],
//   T = rho u u - S.
// The collision is linear in S with constant coefficients, so its adjoint
// Sb[6] (xx, xy, xz, yy, yz, zz, stored components) needs no forward value of
// S.  gsb, ub_in: adjoints of the post-collision populations and of the
// velocity output; gb gets the pre-collision adjoints, Fb and Sb accumulate.
template <class R>
__host__ __device__ __forceinline__ void collide_eq_site_bwd_m(const Params<R>& P, R drho, const R u[3],
                                                               const R F[3], const R gsb[15], const R ub_in[3],
                                                               R gb[15], R Fb[3], R Sb[6]) {
  using L = D3Q15;
  const R rho = P.rho0 + drho;
  const R inv = R(1) / rho;
  const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const R om = P.omega, om1 = R(1) - P.omega;
  // with c.T.c = rho cu^2 - c.S.c and trT = rho uu - trS:
  // g*_i = om1 g_i + w_i [om (drho - 1.5 rho uu + 1.5 trS + 3 rho cu + 4.5 rho cu^2 - 4.5 c.S.c) + guo (...)]
  R Ab = R(0), Bsb = R(0), rhob = R(0);
  R ub[3] = {ub_in[0], ub_in[1], ub_in[2]};
  for (int i = 0; i < 15; ++i) {
    const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
    const R cu = cdot(cx, cy, cz, u);
    const R cF = cdot(cx, cy, cz, F);
    const R e = L::w<R>(i) * gsb[i];
    gb[i] = om1 * gsb[i];
    Ab += om * e;
    Bsb += P.guo * e;
    rhob += om * e * (R(3) * cu + R(4.5) * cu * cu);
    const R cub = e * (om * (R(3) * rho + R(9) * rho * cu) + P.guo * R(9) * cF);
    const R cFb = e * P.guo * (R(3) + R(9) * cu);
    cadd(cx, cub, ub[0]);
    cadd(cy, cub, ub[1]);
    cadd(cz, cub, ub[2]);
    cadd(cx, cFb, Fb[0]);
    cadd(cy, cFb, Fb[1]);
    cadd(cz, cFb, Fb[2]);
    // -4.5 om c.S.c, with c.S.c = cx^2 Sxx + cy^2 Syy + cz^2 Szz + 2 (cx cy Sxy + cx cz Sxz + cy cz Syz)
    const R es = R(-4.5) * om * e, es2 = R(2) * es;
    cadd(cx * cx, es, Sb[0]);
    cadd(cx * cy, es2, Sb[1]);
    cadd(cx * cz, es2, Sb[2]);
    cadd(cy * cy, es, Sb[3]);
    cadd(cy * cz, es2, Sb[4]);
    cadd(cz * cz, es, Sb[5]);
  }
  // +1.5 om trS, summed over i through Ab = om sum w_i gsb_i
  Sb[0] += R(1.5) * Ab;
  Sb[3] += R(1.5) * Ab;
  Sb[5] += R(1.5) * Ab;
  R drhob = Ab;
  rhob += R(-1.5) * uu * Ab;
  const R uub = R(-1.5) * rho * Ab;
  const R uFb = R(-3) * Bsb;
  for (int a = 0; a < 3; ++a) {
    ub[a] += R(2) * u[a] * uub + F[a] * uFb;
    Fb[a] += u[a] * uFb;
  }
  // u = (j + F/2) / rho
  R jb[3];
  for (int a = 0; a < 3; ++a) {
    jb[a] = ub[a] * inv;
    Fb[a] += R(0.5) * ub[a] * inv;
    rhob -= ub[a] * u[a] * inv;
  }
  drhob += rhob;
  for (int i = 0; i < 15; ++i) {
    R t = drhob;
    cadd(L::cx(i), jb[0], t);
    cadd(L::cy(i), jb[1], t);
    cadd(L::cz(i), jb[2], t);
    gb[i] += t;
  }
}

// Reverse of collide_site_eq from the pre-collision populations g[15].
template <class R>
__host__ __device__ __forceinline__ void collide_eq_site_bwd(const Params<R>& P, const R g[15], const R F[3],
                                                             const R gsb[15], const R ub_in[3], R gb[15], R Fb[3],
                                                             R Sb[6]) {
  using L = D3Q15;
  R drho = R(0), j[3] = {R(0), R(0), R(0)};
  for (int i = 0; i < 15; ++i) {
    drho += g[i];
    cadd(L::cx(i), g[i], j[0]);
    cadd(L::cy(i), g[i], j[1]);
    cadd(L::cz(i), g[i], j[2]);
  }
  const R inv = R(1) / (P.rho0 + drho);
  R u[3];
  for (int a = 0; a < 3; ++a) u[a] = (j[a] + R(0.5) * F[a]) * inv;
  collide_eq_site_bwd_m(P, drho, u, F, gsb, ub_in, gb, Fb, Sb);
}

}  // namespace lbc
