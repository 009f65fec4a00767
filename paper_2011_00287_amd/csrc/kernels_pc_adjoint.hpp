// Reverse of the paper's finite-difference integrator of the order parameters
// (Sec. 3: Heun predictor-corrector, first-order upwind advection, fourth-order
// stencils; the forward is kernels_pc.hpp).
//
// Forward, with u the LB velocity of time t in both stages:
//   X* = X + R(X),   X(t+1) = ((X + X*) + R(X*))/2,
//   R_Q   = -upwind(u, Q) + S(D4 u, Q) + Gamma H4(Q, phi),
//   R_phi = -div_donor(u, phi) + M L4 mu4(phi, Q),
//   mu4   = mu_site(phi, L4 phi, D4 . v, Q),  v = Q D4 phi.
// Reverse, given X_bar(t+1):
//   X*_bar = X_bar(t+1)/2 + R'(X*)^T V2,          V2 = X_bar(t+1)/2,
//   X_bar  = X_bar(t+1)/2 + X*_bar + R'(X)^T X*_bar,
//   u_bar  = the u parts of both products.
// One product R'(X)^T V takes three site-parallel passes:
//   k_pcb_local: the local reverses at each site (H4 through local_thermo_bwd
//     with H_bar = Gamma V_Q, the co-rotation, mu4 with mu_bar = M L4 V_phi, the
//     site's own upwind terms) -> the adjoints of the site's stencil data
//     (D4 phi, D4 Q, L4 Q, L4 phi, D4 . v, W = D4 u) and its local adjoints;
//   k_pcb_v: v_bar = -D4 (D4.v)_bar (D4^T = -D4), then the adjoints of Q and D4 phi
//     through v = Q D4 phi;
//   k_pcb_gather: the transposed stencils (D4^T = -D4, L4^T = L4) of those
//     adjoints, and the neighbour terms of the upwind and donor-cell operators,
//     along x and y (NAX = 2; their neighbours share the plane, so they come
//     from L2), then k_pcb_gather_z adds the z terms marching each column
//     through a slab with the z neighbours in register rings (reading the 23
//     fields of the z stencils once instead of from five planes at a time).
// The upwind and donor-cell terms are max(w, 0) a + min(w, 0) b of a velocity
// w; at w = 0 their w-derivative is taken as a + b (both one-sided parts), the
// convention of the clamp form the oracle writes them in.
#pragma once
#include "adjoint.hpp"
#include "kernels_pc.hpp"
#include "kernels_reduce.hpp"

namespace lbc {

// fields of the per-site scratch of one product (arithmetic type, [NPB][N])
constexpr int PB_DPHI = 0;     // adjoint of D4 phi (3)
constexpr int PB_DQ = 3;       // adjoint of D4_g Q_k at 3 + 5 g + k (15)
constexpr int PB_LAPQ = 18;    // adjoint of L4 Q (5)
constexpr int PB_LAPPHI = 23;  // adjoint of L4 phi in mu4
constexpr int PB_DIVV = 24;    // adjoint of D4 . v in mu4
constexpr int PB_W = 25;       // adjoint of W_ag = D4_g u_a at 25 + 3 a + g (9)
constexpr int PB_Q = 34;       // local adjoint of Q (5)
constexpr int PB_PHI = 39;     // local adjoint of phi
constexpr int PB_U = 40;       // local adjoint of u (upwind) (3)
constexpr int NPB = 43;

// The local reverses of R at each site for the adjoint V = vs (vq, vphi) of R.
// partial: one float64 (zeta, q0) pair per block, overwritten (accumulate = 0)
// or added to (accumulate = 1); R depends on q0 through H4 and not on zeta.
template <class R, class FS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1)))
k_pcb_local(Box b, Params<R> P, const FS* __restrict__ phi, const FS* __restrict__ q, const R* __restrict__ u,
            const R* __restrict__ vq, const R* __restrict__ vphi, R vs, R* __restrict__ pb,
            double* __restrict__ partial, int accumulate) {
  const int s = site_xcd();
  double v2[2] = {0.0, 0.0};
  if (s < b.N) {
    int x, y, z;
    coords(b, s, x, y, z);
    const size_t N = b.N;
    int n[3][4];
    star2(b, x, y, z, n);
    Grad<R> G;
    G.phi = R(phi[s]);
    G.lapphi = R(0);
    G.divv = R(0);
    R qm1[3][5], qp1[3][5], W[3][3], uc[3];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      G.q[k] = R(q[k * N + s]);
      G.lapq[k] = R(-7.5) * G.q[k];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) uc[a] = u[a * N + s];
    R lapv = R(-7.5) * vphi[s];
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      G.dphi[g] = d4c(R(phi[n[g][0]]), R(phi[n[g][1]]), R(phi[n[g][2]]), R(phi[n[g][3]]));
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const FS* qk = q + size_t(k) * N;
        const R m2 = R(qk[n[g][0]]), m1 = R(qk[n[g][1]]), p1 = R(qk[n[g][2]]), p2 = R(qk[n[g][3]]);
        G.dq[g][k] = d4c(m2, m1, p1, p2);
        G.lapq[k] += l4c(m2, m1, p1, p2);
        qm1[g][k] = m1;
        qp1[g][k] = p1;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const R* ua = u + size_t(a) * N;
        W[a][g] = d4c(ua[n[g][0]], ua[n[g][1]], ua[n[g][2]], ua[n[g][3]]);
      }
      lapv += l4c(vphi[n[g][0]], vphi[n[g][1]], vphi[n[g][2]], vphi[n[g][3]]);
    }
    R VQ[5], hb[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      VQ[k] = vs * vq[k * N + s];
      hb[k] = P.Gamma * VQ[k];
    }
    const R mub = P.M * vs * lapv;  // (M L4)^T V_phi = M L4 V_phi
    // H4 through local_thermo
    Local<R> Lc;
    local_thermo(P, G, Lc);
    GradBar<R> Gb;
    Gb.zero();
    ParBar<R> Pb{R(0), R(0), R(0)};
    // mu4 (its own adjoints of L4 phi and D4 . v go to the next passes) shares
    // the invariants of Q with H4, whose reverse takes both
    R lapphib = R(0), divvb = R(0), tr2b = R(0), tr3b = R(0);
    mu_site_bwd_local(P, G.phi, Lc.tr2, mub, Gb.phi, lapphib, divvb, tr2b, tr3b);
    local_thermo_bwd(P, G, Lc, hb, tr2b, tr3b, R(0), R(0), R(0), Gb, Pb);
    // co-rotation S(W, Q)
    R qb[5], Wb[3][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
#pragma unroll
    for (int k = 0; k < 5; ++k) qb[k] = Gb.q[k];
    corotation_site_bwd(P.xi, G.q, W, VQ, qb, Wb);
    const R phb = Gb.phi;
    // the site's own upwind terms: R_Q gets -sum_g max(u_g,0)(Q - Q(x-e_g)) + min(u_g,0)(Q(x+e_g) - Q)
    R ub[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const R ug = uc[g], up = ug > R(0) ? ug : R(0), um = ug < R(0) ? ug : R(0);
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const R a = -VQ[k];
        const R back = G.q[k] - qm1[g][k], fwd = qp1[g][k] - G.q[k];
        qb[k] += a * (up - um);
        ub[g] += a * ((ug >= R(0) ? back : R(0)) + (ug <= R(0) ? fwd : R(0)));
      }
    }
#pragma unroll
    for (int g = 0; g < 3; ++g) pb[(PB_DPHI + g) * N + s] = Gb.dphi[g];
#pragma unroll
    for (int g = 0; g < 3; ++g)
#pragma unroll
      for (int k = 0; k < 5; ++k) pb[(PB_DQ + 5 * g + k) * N + s] = Gb.dq[g][k];
#pragma unroll
    for (int k = 0; k < 5; ++k) pb[(PB_LAPQ + k) * N + s] = Gb.lapq[k];
    pb[PB_LAPPHI * N + s] = lapphib;
    pb[PB_DIVV * N + s] = divvb;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int g = 0; g < 3; ++g) pb[(PB_W + 3 * a + g) * N + s] = Wb[a][g];
#pragma unroll
    for (int k = 0; k < 5; ++k) pb[(PB_Q + k) * N + s] = qb[k];
    pb[PB_PHI * N + s] = phb;
#pragma unroll
    for (int a = 0; a < 3; ++a) pb[(PB_U + a) * N + s] = ub[a];
    par_adjoints(P, Pb, v2);
  }
  block_reduce_store<2>(v2, partial + size_t(blockIdx.x) * 2, accumulate != 0);
}

// v = Q D4 phi: v_bar = D4^T (D4 . v)_bar = -D4 (D4 . v)_bar, then
// Q_bar_ab += v_bar_a D4_b phi and (D4 phi)_bar_b += Q_ab v_bar_a at the site.
template <class R, class FS>
__global__ void __launch_bounds__(256) k_pcb_v(Box b, const FS* __restrict__ phi, const FS* __restrict__ q,
                                               R* __restrict__ pb) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  int n[3][4];
  star2(b, x, y, z, n);
  const R* dv = pb + size_t(PB_DIVV) * N;
  R vb[3], dp[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    vb[a] = -d4c(dv[n[a][0]], dv[n[a][1]], dv[n[a][2]], dv[n[a][3]]);
    dp[a] = d4c(R(phi[n[a][0]]), R(phi[n[a][1]]), R(phi[n[a][2]]), R(phi[n[a][3]]));
  }
  const R xx = R(q[s]), xy = R(q[N + s]), xz = R(q[2 * N + s]), yy = R(q[3 * N + s]), yz = R(q[4 * N + s]);
  const R zz = -xx - yy;
  const R Qm[3][3] = {{xx, xy, xz}, {xy, yy, yz}, {xz, yz, zz}};
  R Qb[3][3], qb[5] = {R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int c = 0; c < 3; ++c) Qb[a][c] = vb[a] * dp[c];
    pb[(PB_DPHI + a) * N + s] += Qm[a][0] * vb[0] + Qm[a][1] * vb[1] + Qm[a][2] * vb[2];
  }
  full_to_stored(Qb, qb);
#pragma unroll
  for (int k = 0; k < 5; ++k) pb[(PB_Q + k) * N + s] += qb[k];
}

// The transposed stencils and neighbour terms of one product along the first
// NAX axes, combined with the Heun weights: out = c1 X_bar(t+1) + c2 Xs +
// R'^T V at each site (the z terms follow in k_pcb_gather_z when NAX = 2),
// and u_bar (ub_out) written (accumulate = 0) or added to (accumulate = 1).
// phi, u: the stage's phi and the velocity; V = vs (vq, vphi).
template <class R, class FS, int NAX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2)))
k_pcb_gather(Box b, const FS* __restrict__ phi, const R* __restrict__ u, const R* __restrict__ vq,
             const R* __restrict__ vphi, R vs, const R* __restrict__ pb, const R* __restrict__ xq1,
             const R* __restrict__ xp1, R c1, const R* __restrict__ xsq, const R* __restrict__ xsp, R c2,
             R* __restrict__ q_out, R* __restrict__ phi_out, R* __restrict__ ub_out, int accumulate) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  int n[3][4];
  star2(b, x, y, z, n);
  auto l4t = [&](const R* f) {  // L4^T = L4
    R r = R(-7.5) * f[s];
#pragma unroll
    for (int g = 0; g < NAX; ++g) r += l4c(f[n[g][0]], f[n[g][1]], f[n[g][2]], f[n[g][3]]);
    return r;
  };
  auto d4t = [&](const R* f, int g) { return -d4c(f[n[g][0]], f[n[g][1]], f[n[g][2]], f[n[g][3]]); };
  // one output field's gathers at a time (not unrolled): the loads of all
  // fields at once would need more registers than four waves per SIMD allow
  R qo[5], po, ub[3];
#pragma unroll 1
  for (int k = 0; k < 5; ++k) {
    R r = pb[(PB_Q + k) * N + s] + l4t(pb + size_t(PB_LAPQ + k) * N);
#pragma unroll
    for (int g = 0; g < NAX; ++g) r += d4t(pb + size_t(PB_DQ + 5 * g + k) * N, g);
    qo[k] = r;
  }
  {
    R r = pb[PB_PHI * N + s] + l4t(pb + size_t(PB_LAPPHI) * N);
#pragma unroll
    for (int g = 0; g < NAX; ++g) r += d4t(pb + size_t(PB_DPHI + g) * N, g);
    po = r;
  }
#pragma unroll 1
  for (int a = 0; a < 3; ++a) {
    R r = pb[(PB_U + a) * N + s];
#pragma unroll
    for (int g = 0; g < NAX; ++g) r += d4t(pb + size_t(PB_W + 3 * a + g) * N, g);
    ub[a] = r;
  }
  const R ph = R(phi[s]), vp0 = vs * vphi[s];
#pragma unroll
  for (int g = 0; g < NAX; ++g) {
    const int m1 = n[g][1], p1 = n[g][2];
    const R* ug = u + size_t(g) * N;
    // upwind terms of the neighbours: x = y + e_g reads Q(y) backward, x = y - e_g forward
    const R upx = ug[p1] > R(0) ? ug[p1] : R(0), umx = ug[m1] < R(0) ? ug[m1] : R(0);
#pragma unroll
    for (int k = 0; k < 5; ++k) qo[k] += (vs * vq[k * N + p1]) * upx - (vs * vq[k * N + m1]) * umx;
    // donor-cell faces y + e_g/2 and y - e_g/2; the flux's adjoint is V_phi(right) - V_phi(left)
    const R fp = R(0.5) * (ug[s] + ug[p1]), fm = R(0.5) * (ug[m1] + ug[s]);
    const R cp = vs * vphi[p1] - vp0, cm = vp0 - vs * vphi[m1];
    const R php = R(phi[p1]), phm = R(phi[m1]);
    po += cp * (fp > R(0) ? fp : R(0)) + cm * (fm < R(0) ? fm : R(0));
    const R dfp = (fp >= R(0) ? ph : R(0)) + (fp <= R(0) ? php : R(0));
    const R dfm = (fm >= R(0) ? phm : R(0)) + (fm <= R(0) ? ph : R(0));
    ub[g] += R(0.5) * (cp * dfp + cm * dfm);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    R r = c1 * xq1[k * N + s] + qo[k];
    if (xsq) r += c2 * xsq[k * N + s];
    q_out[k * N + s] = r;
  }
  {
    R r = c1 * xp1[s] + po;
    if (xsp) r += c2 * xsp[s];
    phi_out[s] = r;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) ub_out[a * N + s] = accumulate ? ub_out[a * N + s] + ub[a] : ub[a];
}

// The z terms of one product (after k_pcb_gather<R, FS, 2>), added to q_out,
// phi_out and ub_out.  One thread per (x, y) column marches the planes of a
// slab of TZ; the 15 fields with a radius-2 z stencil (the adjoints of
// D4_z Q, L4 Q, D4_z phi, L4 phi, W_az) sit in five-plane register rings, the
// 8 with a radius-1 one (V, u_z, phi) in three-plane rings.
template <class R, class FS>
__global__ void __launch_bounds__(256) k_pcb_gather_z(Box b, int TZ, const FS* __restrict__ phi,
                                                      const R* __restrict__ u, const R* __restrict__ vq,
                                                      const R* __restrict__ vphi, R vs, const R* __restrict__ pb,
                                                      R* __restrict__ q_out, R* __restrict__ phi_out,
                                                      R* __restrict__ ub_out) {
  const int plane = b.nx * b.ny;
  const int ncb = (plane + 255) / 256;
  const int col = (blockIdx.x % ncb) * 256 + threadIdx.x;
  if (col >= plane) return;
  const int z0 = (blockIdx.x / ncb) * TZ, z1 = min(z0 + TZ, b.nz);
  const size_t N = b.N;
  constexpr int N2 = 15, N1 = 8;
  // radius-2 fields: D4_z Q adjoint (5), L4 Q adjoint (5), D4_z phi, L4 phi adjoints, W_az adjoint (3)
  const R* f2[N2];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    f2[k] = pb + size_t(PB_DQ + 10 + k) * N;
    f2[5 + k] = pb + size_t(PB_LAPQ + k) * N;
  }
  f2[10] = pb + size_t(PB_DPHI + 2) * N;
  f2[11] = pb + size_t(PB_LAPPHI) * N;
#pragma unroll
  for (int a = 0; a < 3; ++a) f2[12 + a] = pb + size_t(PB_W + 3 * a + 2) * N;
  auto at = [&](int zz) { return size_t(pmod(zz, b.nz)) * plane + col; };
  auto ld1 = [&](int zz, R v[N1]) {
    const size_t k = at(zz);
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = vs * vq[c * N + k];
    v[5] = vs * vphi[k];
    v[6] = u[2 * N + k];
    v[7] = R(phi[k]);
  };
  R r2[5][N2], r1[3][N1];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const size_t k = at(z0 - 2 + j);
#pragma unroll
    for (int f = 0; f < N2; ++f) r2[j][f] = f2[f][k];
  }
  ld1(z0 - 1, r1[0]);
  ld1(z0, r1[1]);
  for (int zc = z0; zc < z1; ++zc) {
    {
      const size_t k = at(zc + 2);
#pragma unroll
      for (int f = 0; f < N2; ++f) r2[4][f] = f2[f][k];
    }
    ld1(zc + 1, r1[2]);
    auto d4z = [&](int f) { return -d4c(r2[0][f], r2[1][f], r2[3][f], r2[4][f]); };
    auto l4z = [&](int f) { return l4c(r2[0][f], r2[1][f], r2[3][f], r2[4][f]); };
    const size_t s = size_t(zc) * plane + col;
    // upwind terms of the z neighbours; donor-cell faces z + 1/2 and z - 1/2
    const R uzp = r1[2][6], uzm = r1[0][6], uz = r1[1][6];
    const R upx = uzp > R(0) ? uzp : R(0), umx = uzm < R(0) ? uzm : R(0);
#pragma unroll
    for (int k = 0; k < 5; ++k)
      q_out[k * N + s] += (d4z(k) + l4z(5 + k)) + (r1[2][k] * upx - r1[0][k] * umx);
    const R fp = R(0.5) * (uz + uzp), fm = R(0.5) * (uzm + uz);
    const R cp = r1[2][5] - r1[1][5], cm = r1[1][5] - r1[0][5];
    const R ph = r1[1][7], php = r1[2][7], phm = r1[0][7];
    phi_out[s] += (d4z(10) + l4z(11)) + (cp * (fp > R(0) ? fp : R(0)) + cm * (fm < R(0) ? fm : R(0)));
    const R dfp = (fp >= R(0) ? ph : R(0)) + (fp <= R(0) ? php : R(0));
    const R dfm = (fm >= R(0) ? phm : R(0)) + (fm <= R(0) ? ph : R(0));
    ub_out[s] += d4z(12);
    ub_out[N + s] += d4z(13);
    ub_out[2 * N + s] += d4z(14) + R(0.5) * (cp * dfp + cm * dfm);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int f = 0; f < N2; ++f) r2[j][f] = r2[j + 1][f];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int f = 0; f < N1; ++f) r1[j][f] = r1[j + 1][f];
  }
}

}  // namespace lbc
