// Site-parallel kernels of the adjoint (reverse) of one coupled step.
//
// Given the state at time t and the adjoint of the state at t+1 (adjoints of
// the post-stream populations g, the 5 stored Q components and phi), the
// kernels produce the adjoint at time t and the per-block float64 partial
// sums of the activity and chirality derivatives.  Transposes of the
// stencils used: (D0)^T = -D0, (lap)^T = lap, and the transpose of the pull
// stream g'_i(x) = g*_i(x - c_i) is the push gs_bar_i(x) = g'_bar_i(x + c_i).
//
// Order (each a launch; the forward u and F of time t come from a recording
// step, or are recomputed by k_thermo and k_fwd_force):
//   k_adj_order   : phi, Q updates (Eqs. (1), (2))  -> mu_bar, W_bar, partial u_bar, Q_bar, phi_bar
//   k_adj_collide : collision + stream (Eqs. (6)-(8), (10)-(11)) -> g_bar(t), F_bar
//   k_adj_stress  : stress, H, mu (Eqs. (3)-(5)), including the anchoring
//                   divergence D0_a(Q_ab D0_b phi) of mu, whose adjoint
//                   v_bar_a = W (mu_bar(x + e_a) - mu_bar(x - e_a)) is formed
//                   from mu_bar at the neighbours -> gradient-data adjoints
//                   (the site-local ones already summed with the Q, phi
//                   adjoints of k_adj_order), zeta / q0 block partials
//   k_adj_gather  : stencil transposes of the gradient data -> Q_bar(t), phi_bar(t)
// H_bar = Gamma Q_bar(t+1) is formed where it is used.
#pragma once
#include "adjoint.hpp"
#include "kernels_reduce.hpp"

namespace lbc {

// Forward force F = div(sigma) + body force and u = (j + F/2)/rho at time t.
template <class R, class GS>
__global__ void __launch_bounds__(256) k_fwd_force(Box b, Params<R> P, const GS* __restrict__ B,
                                                   const R* __restrict__ sig, R* __restrict__ F_out,
                                                   R* __restrict__ u_out) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  R F[3];
  force_at(b, P, sig, x, y, z, F);
  R sum = R(0), j[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const R gi = GPol<GS>::template ld<R>(B, i * N + sidx(b, x - CX(i), y - CY(i), z - CZ(i)), i);
    sum += gi;
    j[0] += R(CX(i)) * gi;
    j[1] += R(CY(i)) * gi;
    j[2] += R(CZ(i)) * gi;
  }
  const R rho = P.rho0 + sum;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    F_out[a * N + s] = F[a];
    u_out[a * N + s] = (j[a] + R(0.5) * F[a]) / rho;
  }
}

// Reverse of the Q and phi updates at one site.
//   phi' = phi - sum_g D0_g(u_g phi) + M lap(mu)
//   q'   = q - u.D0 q + S(q, W(u)) + Gamma h
template <class R, class FS>
__global__ void __launch_bounds__(256) k_adj_order(Box b, Params<R> P, const FS* __restrict__ phi,
                                                   const FS* __restrict__ q, const R* __restrict__ u,
                                                   const R* __restrict__ adj_phi, const R* __restrict__ adj_q,
                                                   R* __restrict__ mub, R* __restrict__ Wb_out,
                                                   R* __restrict__ ubp, R* __restrict__ qbp,
                                                   R* __restrict__ phibp) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  R qc[5], qbar[5], W[3][3], uc[3], dq[3][5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    qc[k] = R(q[k * N + s]);
    qbar[k] = adj_q[k * N + s];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) uc[a] = u[a * N + s];
  const R ph = R(phi[s]);
  const R pb0 = adj_phi[s];
  R lap_pb = R(0), vb[3];
  R qb_out[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) qb_out[k] = qbar[k];
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const int sp = sidx(b, x + off[g][0], y + off[g][1], z + off[g][2]);
    const int sm = sidx(b, x - off[g][0], y - off[g][1], z - off[g][2]);
    const R pbp = adj_phi[sp], pbm = adj_phi[sm];
    lap_pb += pbp + pbm;
    vb[g] = R(0.5) * (pbp - pbm);  // adjoint of u_g phi at this site
#pragma unroll
    for (int a = 0; a < 3; ++a) W[a][g] = R(0.5) * (u[a * N + sp] - u[a * N + sm]);
    const R ugp = u[g * N + sp], ugm = u[g * N + sm];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      dq[g][k] = R(0.5) * (R(q[k * N + sp]) - R(q[k * N + sm]));
      // transpose of the advection: D0_g (u_g q_bar_k)
      qb_out[k] += R(0.5) * (ugp * adj_q[k * N + sp] - ugm * adj_q[k * N + sm]);
    }
  }
  lap_pb -= R(6) * pb0;
  mub[s] = P.M * lap_pb;
  R ub[3], phib = pb0;
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    ub[g] = vb[g] * ph;
    phib += vb[g] * uc[g];
#pragma unroll
    for (int k = 0; k < 5; ++k) ub[g] -= qbar[k] * dq[g][k];
  }
  R Wb[3][3] = {};
  corotation_site_bwd(P.xi, qc, W, qbar, qb_out, Wb);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) Wb_out[(a * 3 + c) * N + s] = Wb[a][c];
#pragma unroll
  for (int a = 0; a < 3; ++a) ubp[a * N + s] = ub[a];
#pragma unroll
  for (int k = 0; k < 5; ++k) qbp[k * N + s] = qb_out[k];
  phibp[s] = phib;
}

// Reverse of the collision and the pull stream at one site.
template <class R, class GS>
__global__ void __launch_bounds__(256) k_adj_collide(Box b, Params<R> P, const GS* __restrict__ B,
                                                     const R* __restrict__ F, const R* __restrict__ Wb,
                                                     const R* __restrict__ ubp, const R* __restrict__ adj_g,
                                                     R* __restrict__ g_out, R* __restrict__ Fb_out) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  // u_bar = partial - sum_b D0_b W_bar_ab   (W_ab = D0_b u_a)
  R ub[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) ub[a] = ubp[a * N + s];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int sp = sidx(b, x + off[c][0], y + off[c][1], z + off[c][2]);
    const int sm = sidx(b, x - off[c][0], y - off[c][1], z - off[c][2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) ub[a] -= R(0.5) * (Wb[(a * 3 + c) * N + sp] - Wb[(a * 3 + c) * N + sm]);
  }
  R g[19], gsb[19], Fs[3];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    g[i] = GPol<GS>::template ld<R>(B, i * N + sidx(b, x - CX(i), y - CY(i), z - CZ(i)), i);
    gsb[i] = adj_g[i * N + sidx(b, x + CX(i), y + CY(i), z + CZ(i))];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) Fs[a] = F[a * N + s];
  R gb[19], Fb[3] = {R(0), R(0), R(0)};
  collide_site_bwd(P, g, Fs, gsb, ub, gb, Fb);
#pragma unroll
  for (int i = 0; i < 19; ++i) g_out[i * N + s] = gb[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) Fb_out[a * N + s] = Fb[a];
}

// Number of per-site gradient-data adjoint values stored between kernels.
constexpr int NGB = 30;  // phi, dphi[3], lapphi, q[5], dq[3][5], lapq[5]
// offsets of the fields in the gradient-data adjoint buffer
constexpr int GB_PHI = 0, GB_DPHI = 1, GB_LAPPHI = 4, GB_Q = 5, GB_DQ = 10, GB_LAPQ = 25;

template <class R>
__device__ __forceinline__ void store_gb(const GradBar<R>& Gb, R* __restrict__ out, size_t N, int s) {
  out[GB_PHI * N + s] = Gb.phi;
#pragma unroll
  for (int g = 0; g < 3; ++g) out[(GB_DPHI + g) * N + s] = Gb.dphi[g];
  out[GB_LAPPHI * N + s] = Gb.lapphi;
#pragma unroll
  for (int k = 0; k < 5; ++k) out[(GB_Q + k) * N + s] = Gb.q[k];
#pragma unroll
  for (int g = 0; g < 3; ++g)
#pragma unroll
    for (int k = 0; k < 5; ++k) out[(GB_DQ + 5 * g + k) * N + s] = Gb.dq[g][k];
#pragma unroll
  for (int k = 0; k < 5; ++k) out[(GB_LAPQ + k) * N + s] = Gb.lapq[k];
}

// Reverse of the stress (through H), of H as used by the Q update and of mu.
// qbp, phibp: the site-local Q and phi adjoints from k_adj_order, added to
// the gradient data's own.  partial: one float64 pair (zeta, q0) per block,
// overwritten (accumulate = 0) or added to (accumulate = 1).
template <class R, class FS>
__global__ void __launch_bounds__(256) k_adj_stress(Box b, Params<R> P, const FS* __restrict__ phi,
                                                    const FS* __restrict__ q, const R* __restrict__ Fb,
                                                    const R* __restrict__ adj_q, const R* __restrict__ mub,
                                                    const R* __restrict__ qbp, const R* __restrict__ phibp,
                                                    R* __restrict__ gbar, double* __restrict__ partial,
                                                    int accumulate) {
  const int s = site_xcd();
  double v[2] = {0.0, 0.0};
  if (s < b.N) {
    int x, y, z;
    coords(b, s, x, y, z);
    const size_t N = b.N;
    const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    // sigma_bar_ab = -D0_b F_bar_a;  v_bar_a = -D0_a divv_bar with divv_bar = -2 W mu_bar
    R sb[9], vb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int sp = sidx(b, x + off[c][0], y + off[c][1], z + off[c][2]);
      const int sm = sidx(b, x - off[c][0], y - off[c][1], z - off[c][2]);
#pragma unroll
      for (int a = 0; a < 3; ++a) sb[3 * a + c] = -R(0.5) * (Fb[a * N + sp] - Fb[a * N + sm]);
      vb[c] = P.W * (mub[sp] - mub[sm]);
    }
    Grad<R> G;
    gather_grad<R>(b, phi, q, x, y, z, G);
    R hbs[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) hbs[k] = P.Gamma * adj_q[k * N + s];
    GradBar<R> Gb;
    Gb.zero();
    ParBar<R> Pb{R(0), R(0), R(0)};
    sigma_site_bwd(P, G, sb, hbs, Gb, Pb);
    mu_site_bwd(P, G.phi, G.q, mub[s], Gb.phi, Gb.lapphi, Gb.divv, Gb.q);
    // anchoring divergence: v_a = Q_ab D0_b phi  ->  Q_bar_ab += v_bar_a D0_b phi,
    // (D0_b phi)_bar += Q_ab v_bar_a
    {
      R Qb[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) Qb[a][c] = vb[a] * G.dphi[c];
      full_to_stored(Qb, Gb.q);
      const R xx = G.q[0], xy = G.q[1], xz = G.q[2], yy = G.q[3], yz = G.q[4], zz = -xx - yy;
      Gb.dphi[0] += xx * vb[0] + xy * vb[1] + xz * vb[2];
      Gb.dphi[1] += xy * vb[0] + yy * vb[1] + yz * vb[2];
      Gb.dphi[2] += xz * vb[0] + yz * vb[1] + zz * vb[2];
    }
    Gb.phi += phibp[s];
#pragma unroll
    for (int k = 0; k < 5; ++k) Gb.q[k] += qbp[k * N + s];
    store_gb(Gb, gbar, N, s);
    v[0] = double(Pb.zeta);
    v[1] = 2.0 * double(P.K) * double(Pb.kq) + 8.0 * double(P.K) * double(P.q0) * double(Pb.kq2);
  }
  block_reduce_store<2>(v, partial + size_t(blockIdx.x) * 2, accumulate != 0);
}

// Stencil transposes of the gradient data; writes Q_bar(t), phi_bar(t).
template <class R>
__global__ void __launch_bounds__(256) k_adj_gather(Box b, const R* __restrict__ gbar, R* __restrict__ adj_phi,
                                                    R* __restrict__ adj_q) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  R pb = gbar[size_t(GB_PHI) * N + s];
  R qb[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) qb[k] = gbar[size_t(GB_Q + k) * N + s];
  R lp = R(0), lq[5] = {R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const int sp = sidx(b, x + off[g][0], y + off[g][1], z + off[g][2]);
    const int sm = sidx(b, x - off[g][0], y - off[g][1], z - off[g][2]);
    pb -= R(0.5) * (gbar[size_t(GB_DPHI + g) * N + sp] - gbar[size_t(GB_DPHI + g) * N + sm]);
    lp += gbar[size_t(GB_LAPPHI) * N + sp] + gbar[size_t(GB_LAPPHI) * N + sm];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      qb[k] -= R(0.5) * (gbar[size_t(GB_DQ + 5 * g + k) * N + sp] - gbar[size_t(GB_DQ + 5 * g + k) * N + sm]);
      lq[k] += gbar[size_t(GB_LAPQ + k) * N + sp] + gbar[size_t(GB_LAPQ + k) * N + sm];
    }
  }
  pb += lp - R(6) * gbar[size_t(GB_LAPPHI) * N + s];
  adj_phi[s] = pb;
#pragma unroll
  for (int k = 0; k < 5; ++k) adj_q[k * N + s] = qb[k] + lq[k] - R(6) * gbar[size_t(GB_LAPQ + k) * N + s];
}

// out = in + 1 for the step counter of a recorded state (one thread, vector memory).
__global__ void k_step_count(const int64_t* __restrict__ in, int64_t* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = in[0] + 1;
}

// Seed of the displacement loss L = (z_c - z_ref)^2, z_c = sum phi z / sum phi:
// dL/dphi(x) = 2 (z_c - z_ref)(z - z_c) / sum phi; zero for g and Q.
template <class R>
__global__ void __launch_bounds__(256) k_seed_centre(Box b, double zc, double zref, double phitot,
                                                     R* __restrict__ adj) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  const size_t N = b.N;
  const int z = s / (b.nx * b.ny);
#pragma unroll
  for (int i = 0; i < 24; ++i) adj[i * N + s] = R(0);
  adj[24 * N + s] = R(2.0 * (zc - zref) * (double(z) - zc) / phitot);
}

}  // namespace lbc
