// Kernels of the adjoint (reverse) of one coupled step.
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
//                   (site-parallel, or z-marching over LDS tiles: k_adj_order_fused,
//                   which also applies the transpose of the velocity gradient
//                   and writes the whole u_bar)
//   k_adj_collide : collision + stream (Eqs. (6)-(8), (10)-(11)) -> g_bar(t), F_bar
//   k_adj_stress  : stress, H, mu (Eqs. (3)-(5)), including the anchoring
//                   divergence D0_a(Q_ab D0_b phi) of mu, whose adjoint
//                   v_bar_a = W (mu_bar(x + e_a) - mu_bar(x - e_a)) is formed
//                   from mu_bar at the neighbours -> gradient-data adjoints
//                   (the site-local ones already summed with the Q, phi
//                   adjoints of k_adj_order), zeta / q0 block partials
//   k_adj_gather  : stencil transposes of the gradient data -> Q_bar(t), phi_bar(t)
//   (k_adj_sg_fused does k_adj_stress and k_adj_gather in one z-marching pass)
// H_bar = Gamma Q_bar(t+1) is formed where it is used.
#pragma once
#include "adjoint.hpp"
#include "kernels_reduce.hpp"

namespace lbc {

// Forward force F = div(sigma) + body force (div of the antisymmetric part
// on the D3Q15 scheme), u = (j + F/2)/rho and (when drho_out is not null)
// drho = sum g at time t.
template <class R, class GS, class L>
__global__ void __launch_bounds__(256) k_fwd_force(Box b, Params<R> P, const GS* __restrict__ B,
                                                   const R* __restrict__ sig, R* __restrict__ F_out,
                                                   R* __restrict__ u_out, R* __restrict__ drho_out) {
  const int s = site_xcd();
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
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    F_out[a * N + s] = F[a];
    u_out[a * N + s] = (j[a] + R(0.5) * F[a]) / rho;
  }
  if (drho_out) drho_out[s] = sum;
}

// Reverse of the Q and phi updates at one site.
//   phi' = phi - sum_g D0_g(u_g phi) + M lap(mu)
//   q'   = q - u.D0 q + S(q, W(u)) + Gamma h
// Own values: qc, u, phi at x; qbar, pb0 the adjoints of q', phi' at x.
// Neighbour values at x + e_g (index [g][0]) and x - e_g ([g][1]): phi
// adjoint pbn, u, q and q adjoint aqn.  Outputs: mu_bar, W_bar (3x3),
// the local parts of u_bar, Q_bar, phi_bar.
template <class R>
__device__ __forceinline__ void adj_order_site(const Params<R>& P, const R qc[5], const R qbar[5], const R uc[3], R ph,
                                               R pb0, const R pbn[3][2], const R un[3][2][3], const R qn[3][2][5],
                                               const R aqn[3][2][5], R& mub, R Wb[3][3], R ub[3], R qb_out[5],
                                               R& phib) {
  R lap_pb = -R(6) * pb0, vb[3], W[3][3], dq[3][5];
#pragma unroll
  for (int k = 0; k < 5; ++k) qb_out[k] = qbar[k];
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    lap_pb += pbn[g][0] + pbn[g][1];
    vb[g] = R(0.5) * (pbn[g][0] - pbn[g][1]);  // adjoint of u_g phi at this site
#pragma unroll
    for (int a = 0; a < 3; ++a) W[a][g] = R(0.5) * (un[g][0][a] - un[g][1][a]);
    const R ugp = un[g][0][g], ugm = un[g][1][g];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      dq[g][k] = R(0.5) * (qn[g][0][k] - qn[g][1][k]);
      // transpose of the advection: D0_g (u_g q_bar_k)
      qb_out[k] += R(0.5) * (ugp * aqn[g][0][k] - ugm * aqn[g][1][k]);
    }
  }
  mub = P.M * lap_pb;
  phib = pb0;
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    ub[g] = vb[g] * ph;
    phib += vb[g] * uc[g];
#pragma unroll
    for (int k = 0; k < 5; ++k) ub[g] -= qbar[k] * dq[g][k];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) Wb[a][c] = R(0);
  corotation_site_bwd(P.xi, qc, W, qbar, qb_out, Wb);
}

template <class R>
__device__ __forceinline__ void store_adj_order(size_t N, size_t s, R mub, const R Wb[3][3], const R ub[3],
                                                const R qb[5], R phib, R* __restrict__ mub_out,
                                                R* __restrict__ Wb_out, R* __restrict__ ubp, R* __restrict__ qbp,
                                                R* __restrict__ phibp) {
  mub_out[s] = mub;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) Wb_out[(a * 3 + c) * N + s] = Wb[a][c];
#pragma unroll
  for (int a = 0; a < 3; ++a) ubp[a * N + s] = ub[a];
#pragma unroll
  for (int k = 0; k < 5; ++k) qbp[k * N + s] = qb[k];
  phibp[s] = phib;
}

// Site-parallel form: all loads of a site (own values and the 6 neighbours)
// are issued before the arithmetic.
template <class R, class FS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4)))
k_adj_order(Box b, Params<R> P, const FS* __restrict__ phi, const FS* __restrict__ q, const R* __restrict__ u,
            const R* __restrict__ adj_phi, const R* __restrict__ adj_q, R* __restrict__ mub, R* __restrict__ Wb_out,
            R* __restrict__ ubp, R* __restrict__ qbp, R* __restrict__ phibp) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  R qc[5], qbar[5], uc[3];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    qc[k] = R(q[k * N + s]);
    qbar[k] = adj_q[k * N + s];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) uc[a] = u[a * N + s];
  const R ph = R(phi[s]);
  const R pb0 = adj_phi[s];
  R pbn[3][2], un[3][2][3], qn[3][2][5], aqn[3][2][5];
#pragma unroll
  for (int g = 0; g < 3; ++g)
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int sg = d == 0 ? 1 : -1;
      const int sn = sidx(b, x + sg * off[g][0], y + sg * off[g][1], z + sg * off[g][2]);
      pbn[g][d] = adj_phi[sn];
#pragma unroll
      for (int a = 0; a < 3; ++a) un[g][d][a] = u[a * N + sn];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        qn[g][d][k] = R(q[k * N + sn]);
        aqn[g][d][k] = adj_q[k * N + sn];
      }
    }
  R m, Wb[3][3], ub[3], qb[5], pb;
  adj_order_site(P, qc, qbar, uc, ph, pb0, pbn, un, qn, aqn, m, Wb, ub, qb, pb);
  store_adj_order(N, size_t(s), m, Wb, ub, qb, pb, mub, Wb_out, ubp, qbp, phibp);
}

// z-marching form of k_adj_order: LDS holds plane z of the 14 stencil fields
// (q[5], u[3], phi adjoint, q adjoint[5]) on a TX x TY tile plus the halo the
// stencils read (no corners), the owned column keeps planes z-1, z, z+1 in
// registers, and the halo of plane z+1 is loaded while plane z is computed.
// It also applies the transpose of the velocity gradient,
// u_bar_a -= sum_c D0_c W_bar_ac, and writes the whole u_bar (ub_out [3][N]).
// W_bar at a site depends only on Q and Q_bar(t+1) there (the co-rotation is
// linear in W), so the W_bar the transposes read beyond the owned sites (the
// halo columns and rows of the plane, and the own column at z +- 1) is formed
// from the staged fields (corotation_wbar) instead of being exchanged
// between tiles or launches.  In float it fits 128 registers without spills,
// so four waves per SIMD hide the latency of the plane loads.
template <class R, class FS, int TX, int TY>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1)))
k_adj_order_fused(Box b, Params<R> P, int TZ, int ntx, int nty, const FS* __restrict__ phi,
                  const FS* __restrict__ q, const R* __restrict__ u, const R* __restrict__ adj_phi,
                  const R* __restrict__ adj_q, R* __restrict__ mub, R* __restrict__ ub_out,
                  R* __restrict__ qbp, R* __restrict__ phibp) {
  constexpr int NT = TX * TY;
  constexpr int SX = TX + 2, SY = TY + 2, NS = SX * SY;
  constexpr int NH = 2 * (TX + TY);
  static_assert(NH <= NT, "one halo slot per thread");
  constexpr int NV = 14;  // q[5], u[3], phi adjoint, q adjoint[5]
  __shared__ R sV[NV][NS];
  __shared__ R sW[6][NS];  // W_bar_ax, then W_bar_ay (a = 0..2) on the tile and its halo
  __shared__ int sGX[SX], sGY[SY];

  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = l % ntx, ty = (l / ntx) % nty, sl = l / (ntx * nty);
  const int x0 = tx * TX, y0 = ty * TY, z0 = sl * TZ;
  const int z1 = min(z0 + TZ, b.nz);
  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = tid / TX;
  const bool active = (x0 + lx < b.nx) && (y0 + ly < b.ny);
  const size_t N = b.N;
  const int plane = b.nx * b.ny;

  for (int k = tid; k < SX; k += NT) sGX[k] = pmod(x0 - 1 + k, b.nx);
  for (int k = tid; k < SY; k += NT) sGY[k] = pmod(y0 - 1 + k, b.ny);
  __syncthreads();
  // every thread, active or not, stages the (wrapped) site of its slot: on a
  // ragged tile the slot right of the last active column holds that
  // column's neighbour
  const int col = sGY[ly + 1] * b.nx + sGX[lx + 1];

  // global accesses: uniform field base plus a 32-bit byte offset per lane
  // (component arrays are below 4 GiB)
  auto load_at = [&](uint32_t k, R v[NV]) {
    const uint32_t kf = k * uint32_t(sizeof(FS)), kr = k * uint32_t(sizeof(R));
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = R(ldo(q + c * N, kf));
#pragma unroll
    for (int a = 0; a < 3; ++a) v[5 + a] = ldo(u + a * N, kr);
    v[8] = ldo(adj_phi, kr);
#pragma unroll
    for (int c = 0; c < 5; ++c) v[9 + c] = ldo(adj_q + c * N, kr);
  };
  auto load_col = [&](int zz, R v[NV]) { load_at(uint32_t(pmod(zz, b.nz)) * uint32_t(plane) + uint32_t(col), v); };
  R vm[NV], v0[NV], vp[NV];
  load_col(z0 - 1, vm);
  load_col(z0, v0);
  load_col(z0 + 1, vp);

  // halo slot of this thread: rows y0-1, y0+TY for tid < 2 TX (they need
  // W_bar_ay), then columns x0-1, x0+TX (W_bar_ax)
  const bool has_halo = tid < NH;
  const bool halo_row = tid < 2 * TX;
  int hs = 0, hcol = 0;
  if (has_halo) {
    int hx, hy;
    if (halo_row) {
      hx = 1 + (tid % TX);
      hy = tid < TX ? 0 : SY - 1;
    } else {
      const int r = tid - 2 * TX;
      hx = r < TY ? 0 : SX - 1;
      hy = 1 + (r % TY);
    }
    hs = hy * SX + hx;
    hcol = sGY[hy] * b.nx + sGX[hx];
  }
  R hv[NV];
  if (has_halo) load_at(uint32_t(z0) * uint32_t(plane) + uint32_t(hcol), hv);

  // W_bar_az of the owned column at plane z - 1 (carried from the previous plane)
  R wz_m[3];
  {
    R Wt[3][3];
    corotation_wbar(P.xi, vm, vm + 9, Wt);
#pragma unroll
    for (int a = 0; a < 3; ++a) wz_m[a] = Wt[a][2];
  }

  const int sc = (ly + 1) * SX + (lx + 1);
  for (int zc = z0; zc < z1; ++zc) {
    __syncthreads();  // previous plane's reads are done
#pragma unroll
    for (int c = 0; c < NV; ++c) sV[c][sc] = v0[c];
    if (has_halo) {
#pragma unroll
      for (int c = 0; c < NV; ++c) sV[c][hs] = hv[c];
      if (zc + 1 < z1) load_at(uint32_t(zc + 1) * uint32_t(plane) + uint32_t(hcol), hv);  // next plane's halo
    }
    __syncthreads();
    R Wb[3][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}, {R(0), R(0), R(0)}}, ub[3] = {R(0), R(0), R(0)};
    const uint32_t site = uint32_t(zc) * uint32_t(plane) + uint32_t(col);
    const uint32_t sr = site * uint32_t(sizeof(R));
    if (active) {
      const R ph = R(ldo(phi, site * uint32_t(sizeof(FS))));
      R qc[5], qbar[5], uc[3];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        qc[k] = v0[k];
        qbar[k] = v0[9 + k];
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) uc[a] = v0[5 + a];
      R pbn[3][2], un[3][2][3], qn[3][2][5], aqn[3][2][5];
      const int nb[2][2] = {{sc + 1, sc - 1}, {sc + SX, sc - SX}};
#pragma unroll
      for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          const int t = nb[g][d];
          pbn[g][d] = sV[8][t];
#pragma unroll
          for (int a = 0; a < 3; ++a) un[g][d][a] = sV[5 + a][t];
#pragma unroll
          for (int k = 0; k < 5; ++k) {
            qn[g][d][k] = sV[k][t];
            aqn[g][d][k] = sV[9 + k][t];
          }
        }
      pbn[2][0] = vp[8];
      pbn[2][1] = vm[8];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        un[2][0][a] = vp[5 + a];
        un[2][1][a] = vm[5 + a];
      }
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        qn[2][0][k] = vp[k];
        qn[2][1][k] = vm[k];
        aqn[2][0][k] = vp[9 + k];
        aqn[2][1][k] = vm[9 + k];
      }
      R m, qb[5], pb;
      adj_order_site(P, qc, qbar, uc, ph, v0[8], pbn, un, qn, aqn, m, Wb, ub, qb, pb);
      sto(mub, sr, m);
#pragma unroll
      for (int k = 0; k < 5; ++k) sto(qbp + k * N, sr, qb[k]);
      sto(phibp, sr, pb);
    } else {
      corotation_wbar(P.xi, v0, v0 + 9, Wb);  // a neighbour of the tile's last column or row
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      sW[a][sc] = Wb[a][0];
      sW[3 + a][sc] = Wb[a][1];
    }
    if (has_halo) {  // the halo slot's W_bar_ay (rows) or W_bar_ax (columns), from its staged Q and Q_bar
      R qh[5], sh[5], Wh[3][3];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        qh[k] = sV[k][hs];
        sh[k] = sV[9 + k][hs];
      }
      corotation_wbar(P.xi, qh, sh, Wh);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (halo_row)
          sW[3 + a][hs] = Wh[a][1];
        else
          sW[a][hs] = Wh[a][0];
      }
    }
    // W_bar_az of the owned column at plane z + 1
    R wz_p[3];
    {
      R Wt[3][3];
      corotation_wbar(P.xi, vp, vp + 9, Wt);
#pragma unroll
      for (int a = 0; a < 3; ++a) wz_p[a] = Wt[a][2];
    }
    __syncthreads();  // W_bar of the tile and its halo are in place
    if (active) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
        sto(ub_out + a * N, sr, ub[a] - ((R(0.5) * (sW[a][sc + 1] - sW[a][sc - 1]) +
                                          R(0.5) * (sW[3 + a][sc + SX] - sW[3 + a][sc - SX])) +
                                         R(0.5) * (wz_p[a] - wz_m[a])));
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) wz_m[a] = Wb[a][2];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      vm[c] = v0[c];
      v0[c] = vp[c];
    }
    if (zc + 1 < z1) load_col(zc + 2, vp);
  }
}

// Where the velocity adjoint u_bar comes from.  Site path (whole == 0): the
// order kernel's local part u (ubp [3][N]) and W_bar (W [9][N]), and
//   u_bar_a = ubp_a - sum_c D0_c W_bar_ac.
// whole == 1: u is the whole u_bar (k_adj_order_fused, the pc4 reverse).
template <class R>
struct UbarIn {
  const R* W;
  const R* u;
  int whole;
};

template <class R>
__device__ __forceinline__ void ubar_at(const Box& b, const UbarIn<R>& in, int s, int x, int y, int z, R ub[3]) {
  const size_t N = b.N;
  const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
#pragma unroll
  for (int a = 0; a < 3; ++a) ub[a] = ldo(in.u + a * N, uint32_t(s) * uint32_t(sizeof(R)));
  if (in.whole) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int sp = sidx(b, x + off[c][0], y + off[c][1], z + off[c][2]);
    const int sm = sidx(b, x - off[c][0], y - off[c][1], z - off[c][2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) ub[a] -= R(0.5) * (in.W[(a * 3 + c) * N + sp] - in.W[(a * 3 + c) * N + sm]);
  }
}

// The collision reverse of one site on lattice L from its moments; on the
// D3Q15 scheme it also writes the adjoint of the symmetric stress (Sb_out,
// 6 stored components), which enters that collision.
template <class R, class L>
__device__ __forceinline__ void collide_bwd_site_l(const Params<R>& P, R drho, const R u[3], const R F[3],
                                                   const R gsb[L::Q], const R ub[3], R gb[L::Q], R Fb[3],
                                                   R* __restrict__ Sb_out, size_t N, int s) {
  if constexpr (L::kStressInEq) {
    R Sb[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    collide_eq_site_bwd_m(P, drho, u, F, gsb, ub, gb, Fb, Sb);
#pragma unroll
    for (int k = 0; k < 6; ++k) Sb_out[k * N + s] = Sb[k];
  } else {
    collide_site_bwd_m(P, drho, u, F, gsb, ub, gb, Fb);
  }
}

// Reverse of the collision and the pull stream at one site (the moments are
// formed from the pulled populations B).
template <class R, class GS, class L>
__global__ void __launch_bounds__(256) k_adj_collide(Box b, Params<R> P, const GS* __restrict__ B,
                                                     const R* __restrict__ F, UbarIn<R> ubin,
                                                     const R* __restrict__ adj_g, R* __restrict__ g_out,
                                                     R* __restrict__ Fb_out, R* __restrict__ Sb_out) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  R ub[3];
  ubar_at(b, ubin, s, x, y, z, ub);
  R g[L::Q], gsb[L::Q], Fs[3];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    // pulled populations and pushed adjoints are read once: streaming loads
    // (32/64-bit storage; half storage keeps ordinary loads)
    const int sp = sidx(b, x - L::cx(i), y - L::cy(i), z - L::cz(i));
    if constexpr (sizeof(GS) >= 4)
      g[i] = R(__builtin_nontemporal_load(B + i * N + sp));
    else
      g[i] = GPol<GS, L>::template ld<R>(B, i * N + sp, i);
    gsb[i] = __builtin_nontemporal_load(adj_g + i * N + sidx(b, x + L::cx(i), y + L::cy(i), z + L::cz(i)));
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) Fs[a] = F[a * N + s];
  R drho = R(0), j[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    drho += g[i];
    cadd(L::cx(i), g[i], j[0]);
    cadd(L::cy(i), g[i], j[1]);
    cadd(L::cz(i), g[i], j[2]);
  }
  const R inv = R(1) / (P.rho0 + drho);
  R us[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) us[a] = (j[a] + R(0.5) * Fs[a]) * inv;
  R gb[L::Q], Fb[3] = {R(0), R(0), R(0)};
  collide_bwd_site_l<R, L>(P, drho, us, Fs, gsb, ub, gb, Fb, Sb_out, N, s);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) __builtin_nontemporal_store(gb[i], g_out + i * N + s);
#pragma unroll
  for (int a = 0; a < 3; ++a) Fb_out[a * N + s] = Fb[a];
}

// Reverse of the collision and the pull stream from a record: the
// pre-collision populations enter only through drho = sum g and u, which the
// record holds, so they are not read.
template <class R, class L>
__global__ void __launch_bounds__(256) k_adj_collide_lean(Box b, Params<R> P, const R* __restrict__ drho,
                                                          const R* __restrict__ u, const R* __restrict__ F,
                                                          UbarIn<R> ubin, const R* __restrict__ adj_g,
                                                          R* __restrict__ g_out, R* __restrict__ Fb_out,
                                                          R* __restrict__ Sb_out) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  R ub[3];
  ubar_at(b, ubin, s, x, y, z, ub);
  // global accesses: uniform field base plus a 32-bit byte offset per lane
  const uint32_t so = uint32_t(s) * uint32_t(sizeof(R));
  R gsb[L::Q], Fs[3], us[3];
#pragma unroll
  for (int i = 0; i < L::Q; ++i)
    gsb[i] = ldo_nt(adj_g + i * N,
                    uint32_t(sidx(b, x + L::cx(i), y + L::cy(i), z + L::cz(i))) * uint32_t(sizeof(R)));
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Fs[a] = ldo(F + a * N, so);
    us[a] = ldo(u + a * N, so);
  }
  R gb[L::Q], Fb[3] = {R(0), R(0), R(0)};
  collide_bwd_site_l<R, L>(P, ldo(drho, so), us, Fs, gsb, ub, gb, Fb, Sb_out, N, s);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) sto_nt(g_out + i * N, so, gb[i]);
#pragma unroll
  for (int a = 0; a < 3; ++a) sto(Fb_out + a * N, so, Fb[a]);
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

// Gradient-data adjoint of one site: the reverse of its stress (through H), of
// H as used by the Q update (H_bar = Gamma Q_bar(t+1)) and of mu, including
// the anchoring vector v = Q D0 phi whose divergence enters mu.  G: the
// site's forward gradient data (G.divv unused); Fn[g][d][a], mbn[g][d]: F_bar
// and mu_bar at x + e_g (d = 0) and x - e_g (d = 1); mb0, aq: mu_bar and
// Q_bar(t+1) at the site.  On the D3Q15 scheme (SYM) the force is the
// divergence of the antisymmetric part A = (sigma - sigma^T)/2 only, and the
// symmetric part S enters the site's own collision, whose adjoint Ssb (6
// stored components) is added here.  Gb gets the gradient-data adjoints
// (without the order kernel's site-local Q and phi adjoints), Pb the
// parameter adjoints.  HM = false (the pc4 reverse, whose order-parameter
// update takes neither this H nor this mu): mu_bar and Q_bar(t+1) are zero,
// mbn, mb0 and aq are not read, and their terms are not formed.
template <class R, bool SYM = false, bool HM = true>
__device__ __forceinline__ void adj_stress_site(const Params<R>& P, const Grad<R>& G, const R Fn[3][2][3],
                                                const R mbn[3][2], R mb0, const R aq[5], GradBar<R>& Gb,
                                                ParBar<R>& Pb, const R* Ssb = nullptr) {
  // sigma_bar_ab = -D0_b F_bar_a;  v_bar_a = -D0_a divv_bar with divv_bar = -2 W mu_bar
  R sb[9], vb[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int a = 0; a < 3; ++a) sb[3 * a + c] = -R(0.5) * (Fn[c][0][a] - Fn[c][1][a]);
    if constexpr (HM) vb[c] = P.W * (mbn[c][0] - mbn[c][1]);
  }
  if constexpr (SYM) {
    // A_ac = (sigma_ac - sigma_ca)/2, S_ac = (sigma_ac + sigma_ca)/2 (S stored xx, xy, xz, yy, yz, zz)
    R t[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) t[3 * a + c] = R(0.5) * (sb[3 * a + c] - sb[3 * c + a]);
    t[0] += Ssb[0];
    t[4] += Ssb[3];
    t[8] += Ssb[5];
    t[1] += R(0.5) * Ssb[1];
    t[3] += R(0.5) * Ssb[1];
    t[2] += R(0.5) * Ssb[2];
    t[6] += R(0.5) * Ssb[2];
    t[5] += R(0.5) * Ssb[4];
    t[7] += R(0.5) * Ssb[4];
#pragma unroll
    for (int k = 0; k < 9; ++k) sb[k] = t[k];
  }
  R hbs[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) hbs[k] = HM ? P.Gamma * aq[k] : R(0);
  Gb.zero();
  Pb = ParBar<R>{R(0), R(0), R(0)};
  sigma_site_bwd<R, HM>(P, G, sb, hbs, Gb, Pb, HM ? mb0 : R(0));
  if constexpr (!HM) return;
  // anchoring divergence: v_a = Q_ab D0_b phi  ->  Q_bar_ab += v_bar_a D0_b phi,
  // (D0_b phi)_bar += Q_ab v_bar_a
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

// the (zeta, q0) adjoint contributions of one site
template <class R>
__device__ __forceinline__ void par_adjoints(const Params<R>& P, const ParBar<R>& Pb, double v[2]) {
  v[0] += double(Pb.zeta);
  v[1] += 2.0 * double(P.K) * double(Pb.kq) + 8.0 * double(P.K) * double(P.q0) * double(Pb.kq2);
}

// Reverse of the stress (through H), of H as used by the Q update and of mu.
// qbp, phibp: the site-local Q and phi adjoints from k_adj_order, added to
// the gradient data's own.  partial: one float64 pair (zeta, q0) per block,
// overwritten (accumulate = 0) or added to (accumulate = 1).
template <class R, class FS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 3)))
k_adj_stress(Box b, Params<R> P, const FS* __restrict__ phi, const FS* __restrict__ q, const R* __restrict__ Fb,
             const R* __restrict__ adj_q, const R* __restrict__ mub, const R* __restrict__ qbp,
             const R* __restrict__ phibp, R* __restrict__ gbar, double* __restrict__ partial, int accumulate) {
  const int s = site_xcd();
  double v[2] = {0.0, 0.0};
  if (s < b.N) {
    int x, y, z;
    coords(b, s, x, y, z);
    const size_t N = b.N;
    const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    int sn[3][2];
#pragma unroll
    for (int g = 0; g < 3; ++g)
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const int sg = d == 0 ? 1 : -1;
        sn[g][d] = sidx(b, x + sg * off[g][0], y + sg * off[g][1], z + sg * off[g][2]);
      }
    // ---- every load of the site first
    R ph0 = R(phi[s]), q0[5], aq[5], qp[5];
    const R mb0 = mub[s], pbp = phibp[s];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      q0[k] = R(q[k * N + s]);
      aq[k] = adj_q[k * N + s];
      qp[k] = qbp[k * N + s];
    }
    R phn[3][2], mbn[3][2], qn[3][2][5], Fn[3][2][3];
#pragma unroll
    for (int g = 0; g < 3; ++g)
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const int t = sn[g][d];
        phn[g][d] = R(phi[t]);
        mbn[g][d] = mub[t];
#pragma unroll
        for (int k = 0; k < 5; ++k) qn[g][d][k] = R(q[k * N + t]);
#pragma unroll
        for (int a = 0; a < 3; ++a) Fn[g][d][a] = Fb[a * N + t];
      }
    // ---- gradient data of the site (as the forward gathers it)
    Grad<R> G;
    G.phi = ph0;
    R lap = R(0);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      G.q[k] = q0[k];
      G.lapq[k] = R(0);
    }
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      G.dphi[g] = R(0.5) * (phn[g][0] - phn[g][1]);
      lap += phn[g][0] + phn[g][1];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        G.dq[g][k] = R(0.5) * (qn[g][0][k] - qn[g][1][k]);
        G.lapq[k] += qn[g][0][k] + qn[g][1][k];
      }
    }
    G.lapphi = lap - R(6) * G.phi;
#pragma unroll
    for (int k = 0; k < 5; ++k) G.lapq[k] -= R(6) * G.q[k];
    G.divv = R(0);  // mu's anchoring divergence is reversed through v_bar
    GradBar<R> Gb;
    ParBar<R> Pb;
    adj_stress_site(P, G, Fn, mbn, mb0, aq, Gb, Pb);
    Gb.phi += pbp;
#pragma unroll
    for (int k = 0; k < 5; ++k) Gb.q[k] += qp[k];
    store_gb(Gb, gbar, N, s);
    par_adjoints(P, Pb, v);
  }
  block_reduce_store<2>(v, partial + size_t(blockIdx.x) * 2, accumulate != 0);
}

// Stencil transposes of the gradient data at one site.
// own: phi, q[5], lapphi, lapq[5] of the site; nb[g][d] at x + e_g (d = 0) and
// x - e_g (d = 1): dphi_g, lapphi, dq_g[5], lapq[5].
template <class R>
__device__ __forceinline__ void gather_site(const R own[12], const R nb[3][2][12], R& pb, R qb[5]) {
  pb = own[0] - R(6) * own[6];
#pragma unroll
  for (int g = 0; g < 3; ++g) pb += (nb[g][0][1] + nb[g][1][1]) - R(0.5) * (nb[g][0][0] - nb[g][1][0]);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    qb[k] = own[1 + k] - R(6) * own[7 + k];
#pragma unroll
    for (int g = 0; g < 3; ++g)
      qb[k] += (nb[g][0][7 + k] + nb[g][1][7 + k]) - R(0.5) * (nb[g][0][2 + k] - nb[g][1][2 + k]);
  }
}

// Site-parallel form: all 84 loads of a site are issued before any
// arithmetic (a wave keeps them in flight together; the register budget
// allows 4 waves per SIMD).
template <class R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4)))
k_adj_gather(Box b, const R* __restrict__ gbar, R* __restrict__ adj_phi, R* __restrict__ adj_q) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  R own[12], nb[3][2][12];
  own[0] = gbar[size_t(GB_PHI) * N + s];
  own[6] = gbar[size_t(GB_LAPPHI) * N + s];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    own[1 + k] = gbar[size_t(GB_Q + k) * N + s];
    own[7 + k] = gbar[size_t(GB_LAPQ + k) * N + s];
  }
#pragma unroll
  for (int g = 0; g < 3; ++g)
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int sg = d == 0 ? 1 : -1;
      const int sn = sidx(b, x + sg * off[g][0], y + sg * off[g][1], z + sg * off[g][2]);
      R* v = nb[g][d];
      v[0] = gbar[size_t(GB_DPHI + g) * N + sn];
      v[1] = gbar[size_t(GB_LAPPHI) * N + sn];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        v[2 + k] = gbar[size_t(GB_DQ + 5 * g + k) * N + sn];
        v[7 + k] = gbar[size_t(GB_LAPQ + k) * N + sn];
      }
    }
  R pb, qb[5];
  gather_site(own, nb, pb, qb);
  adj_phi[s] = pb;
#pragma unroll
  for (int k = 0; k < 5; ++k) adj_q[k * N + s] = qb[k];
}

// ---------------------------------------------------------------------------
// k_adj_sg_fused: k_adj_stress and k_adj_gather in one z-marching pass, so the
// 30 gradient-data adjoints never leave the chip.  One workgroup marches a
// TX x TY tile through a slab of planes, one site per thread; at plane p it
//   * takes phi, Q, mu_bar, F_bar of planes p-1, p, p+1 from an LDS ring of
//     three planes on the tile with a halo of 1;
//   * forms the gradient-data adjoint (adj_stress_site) at its own site and
//     puts the 18 values the in-plane transposes read in LDS;
//   * applies the in-plane transposes from the neighbours inside the tile,
//     and the z transposes from the own column's values at p-1 and p+1 held
//     in registers, so the adjoint of plane p-1 is complete one step later
//     except for the terms of neighbours in other tiles;
//   * an edge site of an owned plane writes the term it owes the neighbour
//     across the tile face to the face buffers (hx, hy), which k_adj_faces
//     then adds.  Every wave does one stress adjoint per
//     plane: no site's adjoint is recomputed by a second tile.
// Face buffers: hx[f][side][k][z][y] for the face between x tiles k and k+1
// (mod ntx), hy[f][side][k][z][x] for y tiles; side 0 is the term sent in the
// + direction, side 1 the term sent in the - direction; f = phi, q[5].  They
// are written only when the box has more than one tile along that axis.  hx
// has two more sides: the adjoint of the first (2) and last (3) column of
// tile k without its face terms.  Those columns are left out of adj_phi and
// adj_qo here, and k_adj_faces writes them whole (a plain store instead of
// a read-modify-write of every cache line that holds a tile edge).
// The (zeta, q0) partials count owned sites only.  HM = false (the pc4
// reverse): no mu_bar or Q_bar(t+1) seeds; mub and adj_q are not read.
// ---------------------------------------------------------------------------
template <class R, class FS, int TX, int TY, bool SYM = false, bool HM = true>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(1, 2)))
k_adj_sg_fused(Box b, Params<R> P, int TZ, int ntx, int nty, const FS* __restrict__ phi,
               const FS* __restrict__ q, const R* __restrict__ Fb, const R* __restrict__ adj_q,
               const R* __restrict__ mub, const R* __restrict__ qbp, const R* __restrict__ phibp,
               const R* __restrict__ Sbar, R* __restrict__ adj_phi, R* __restrict__ adj_qo, R* __restrict__ hx,
               R* __restrict__ hy, double* __restrict__ partial, int accumulate) {
  constexpr int NT = TX * TY;
  constexpr int IX = TX + 2, IY = TY + 2, NI = IX * IY;  // input frame (halo 1)
  constexpr int NF = 10;                                 // phi, q[5], mu_bar, F_bar[3]
  constexpr int KI = (NI + NT - 1) / NT;
  constexpr int NGB = 18;  // lapphi, lapq[5], dphi_x, dphi_y, dq_x[5], dq_y[5]
  __shared__ R sIn[3][NF][NI];
  __shared__ R sGB[NGB][NT];
  __shared__ int sGX[IX], sGY[IY];

  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = l % ntx, ty = (l / ntx) % nty, sl = l / (ntx * nty);
  // with several x tiles, tile tx starts one column early (x0 = tx TX - 1,
  // mod nx): the edge columns of neighbouring tiles are then adjacent in
  // memory, and so are the two columns k_adj_faces writes per face
  const int x0 = tx * TX - (ntx > 1 ? 1 : 0), y0 = ty * TY, z0 = sl * TZ;
  const int z1 = min(z0 + TZ, b.nz);
  const int w = min(TX, b.nx - tx * TX), h = min(TY, b.ny - y0);  // the tile's extent in the box
  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = tid / TX;
  const bool active = lx < w && ly < h;
  const size_t N = b.N;
  const int plane = b.nx * b.ny;

  for (int k = tid; k < IX; k += NT) sGX[k] = pmod(x0 - 1 + k, b.nx);
  for (int k = tid; k < IY; k += NT) sGY[k] = pmod(y0 - 1 + k, b.ny);
  __syncthreads();

  // input-frame slots this thread loads (padding repeats the frame origin)
  int icol[KI];
#pragma unroll
  for (int j = 0; j < KI; ++j) {
    const int k = tid + j * NT;
    icol[j] = k < NI ? sGY[k / IX] * b.nx + sGX[k % IX] : sGY[0] * b.nx + sGX[0];
  }
  // plane w of the inputs into ring slot `slot` (the loads of one frame slot are
  // stored before the next slot's are issued, which keeps few registers live)
  auto fill_plane = [&](int wp, int slot) {
    const size_t base = size_t(pmod(wp, b.nz)) * plane;
#pragma unroll
    for (int j = 0; j < KI; ++j) {
      const int k = tid + j * NT;
      const size_t g = base + icol[j];
      R v[NF];
      v[0] = R(phi[g]);
#pragma unroll
      for (int c = 0; c < 5; ++c) v[1 + c] = R(q[c * N + g]);
      v[6] = HM ? mub[g] : R(0);
#pragma unroll
      for (int a = 0; a < 3; ++a) v[7 + a] = Fb[a * N + g];
      if (k < NI) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
          if (HM || f != 6) sIn[slot][f][k] = v[f];
      }
    }
  };
  // float, D3Q19: the next plane is loaded into registers before the stress
  // adjoint of this plane (which hides the loads) and stored after it
  constexpr bool kEarly = sizeof(R) == 4 && !SYM;
  auto fill_load = [&](int wp, R v[KI][NF]) {
    const size_t base = size_t(pmod(wp, b.nz)) * plane;
#pragma unroll
    for (int j = 0; j < KI; ++j) {
      const size_t g = base + icol[j];
      v[j][0] = R(phi[g]);
#pragma unroll
      for (int c = 0; c < 5; ++c) v[j][1 + c] = R(q[c * N + g]);
      v[j][6] = HM ? mub[g] : R(0);
#pragma unroll
      for (int a = 0; a < 3; ++a) v[j][7 + a] = Fb[a * N + g];
    }
  };

  // in-plane neighbours inside the tile (a lone tile along an axis wraps
  // periodically inside itself); -1 where the neighbour is in another tile
  const int nxp = ntx == 1 ? (lx + 1) % w : (lx + 1 < w ? lx + 1 : -1);
  const int nxm = ntx == 1 ? (lx + w - 1) % w : (lx > 0 ? lx - 1 : -1);
  const int nyp = nty == 1 ? (ly + 1) % h : (ly + 1 < h ? ly + 1 : -1);
  const int nym = nty == 1 ? (ly + h - 1) % h : (ly > 0 ? ly - 1 : -1);
  const int sxp = nxp < 0 ? tid : ly * TX + nxp, sxm = nxm < 0 ? tid : ly * TX + nxm;
  const int syp = nyp < 0 ? tid : nyp * TX + lx, sym = nym < 0 ? tid : nym * TX + lx;
  // the tile faces this site sends across (owned planes only)
  const bool send_xp = active && ntx > 1 && lx == w - 1, send_xm = active && ntx > 1 && lx == 0;
  const bool send_yp = active && nty > 1 && ly == h - 1, send_ym = active && nty > 1 && ly == 0;
  const size_t fxs = size_t(ntx) * b.nz * b.ny, fys = size_t(nty) * b.nz * b.nx;  // one field-side block
  const bool xedge = active && ntx > 1 && (lx == 0 || lx == w - 1);  // adjoint goes to hx side 2 / 3
  const int kxm = (tx + ntx - 1) % ntx, kym = (ty + nty - 1) % nty;

  const int f0 = (ly + 1) * IX + (lx + 1);
  const int col = sGY[ly + 1] * b.nx + sGX[lx + 1];
  // the gradient-data adjoint of the own site at plane p (input slots rm, r0, rp = planes p-1, p, p+1)
  auto site_adjoint = [&](int rm, int r0, int rp, const R aq[5], const R ssb[6], GradBar<R>& Gb, ParBar<R>& Pb) {
    const int f = f0;
    const int nb[3][2] = {{f + 1, f - 1}, {f + IX, f - IX}, {f, f}};
    auto at = [&](int fld, int g, int d) {
      return g < 2 ? sIn[r0][fld][nb[g][d]] : sIn[d == 0 ? rp : rm][fld][f];
    };
    Grad<R> G;
    G.phi = sIn[r0][0][f];
    R lap = R(0);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      G.q[k] = sIn[r0][1 + k][f];
      G.lapq[k] = R(0);
    }
    R Fn[3][2][3], mbn[3][2];
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const R pp = at(0, g, 0), pm = at(0, g, 1);
      G.dphi[g] = R(0.5) * (pp - pm);
      lap += pp + pm;
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const R a = at(1 + k, g, 0), c = at(1 + k, g, 1);
        G.dq[g][k] = R(0.5) * (a - c);
        G.lapq[k] += a + c;
      }
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        mbn[g][d] = HM ? at(6, g, d) : R(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) Fn[g][d][a] = at(7 + a, g, d);
      }
    }
    G.lapphi = lap - R(6) * G.phi;
#pragma unroll
    for (int k = 0; k < 5; ++k) G.lapq[k] -= R(6) * G.q[k];
    G.divv = R(0);
    adj_stress_site<R, SYM, HM>(P, G, Fn, mbn, HM ? sIn[r0][6][f] : R(0), aq, Gb, Pb, ssb);
  };
  auto load_site = [&](int wp, R aq[5], R qp[5], R& pp, R ssb[6], bool with_s = true) {
    const size_t k = size_t(pmod(wp, b.nz)) * plane + col;
#pragma unroll
    for (int c = 0; c < 5; ++c) aq[c] = HM ? adj_q[c * N + k] : R(0);
#pragma unroll
    for (int c = 0; c < 5; ++c) qp[c] = qbp[c * N + k];
    pp = phibp[k];
    if (SYM && with_s) {
#pragma unroll
      for (int c = 0; c < 6; ++c) ssb[c] = Sbar[c * N + k];
    }
  };
  // the term a site sends across a face: lap + (sgn/2) d, for phi and q[5]
  // (fields fstride apart)
  auto send = [&](R* __restrict__ buf, size_t fstride, size_t off, R sgn, const GradBar<R>& Gb, int g) {
    buf[off] = Gb.lapphi + sgn * R(0.5) * Gb.dphi[g];
#pragma unroll
    for (int k = 0; k < 5; ++k) buf[size_t(1 + k) * fstride + off] = Gb.lapq[k] + sgn * R(0.5) * Gb.dq[g][k];
  };

  // planes z0-2 .. z0 into the ring, the site inputs of plane z0-1 into registers
  int rm = 0, r0 = 1, rp = 2;  // ring slots of planes p-1, p, p+1
  fill_plane(z0 - 2, rm);
  fill_plane(z0 - 1, r0);
  fill_plane(z0, rp);
  R aq_o[5], qp_o[5], pp_o = R(0), ss_o[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
  load_site(z0 - 1, aq_o, qp_o, pp_o, ss_o);

  // own column: z-transpose values of the previous plane and the running adjoint
  R zp_lapphi = R(0), zp_dphi = R(0), zp_lapq[5], zp_dq[5];
  R acc_p = R(0), acc_q[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) zp_lapq[k] = zp_dq[k] = acc_q[k] = R(0);
  double v[2] = {0.0, 0.0};

  for (int p = z0 - 1; p <= z1; ++p) {
    const bool more = p < z1;
    __syncthreads();  // plane p+1 in place; the previous plane's reads of sGB are done
    R fv[kEarly ? KI : 1][kEarly ? NF : 1];
    if constexpr (kEarly) {
      if (more) fill_load(p + 2, fv);
    }
    // D3Q15: the next plane's collision S adjoint, loaded before this plane's stress adjoint
    R ss_n[SYM ? 6 : 1];
    if constexpr (SYM) {
      if (more) {
        const size_t k = size_t(pmod(p + 1, b.nz)) * plane + col;
#pragma unroll
        for (int c = 0; c < 6; ++c) ss_n[c] = Sbar[c * N + k];
      }
    }
    GradBar<R> Gb;
    ParBar<R> Pb;
    site_adjoint(rm, r0, rp, aq_o, ss_o, Gb, Pb);
    const bool own_plane = p >= z0 && p < z1;
    if (own_plane && active) par_adjoints(P, Pb, v);
    Gb.phi += pp_o;
#pragma unroll
    for (int k = 0; k < 5; ++k) Gb.q[k] += qp_o[k];
    sGB[0][tid] = Gb.lapphi;
#pragma unroll
    for (int k = 0; k < 5; ++k) sGB[1 + k][tid] = Gb.lapq[k];
    sGB[6][tid] = Gb.dphi[0];
    sGB[7][tid] = Gb.dphi[1];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      sGB[8 + k][tid] = Gb.dq[0][k];
      sGB[13 + k][tid] = Gb.dq[1][k];
    }
    if (own_plane) {
      const int pz = pmod(p, b.nz);
      const int gy = sGY[ly + 1], gx = sGX[lx + 1];
      if (send_xp) send(hx, 4 * fxs, (size_t(tx) * b.nz + pz) * b.ny + gy, R(1), Gb, 0);
      if (send_xm) send(hx + fxs, 4 * fxs, (size_t(kxm) * b.nz + pz) * b.ny + gy, R(-1), Gb, 0);
      if (send_yp) send(hy, 2 * fys, (size_t(ty) * b.nz + pz) * b.nx + gx, R(1), Gb, 1);
      if (send_ym) send(hy + fys, 2 * fys, (size_t(kym) * b.nz + pz) * b.nx + gx, R(-1), Gb, 1);
    }
    __syncthreads();  // the gradient adjoints of plane p are in place
    const size_t site = size_t(pmod(p - 1, b.nz)) * plane + col;
    // plane p-1 is complete with the z+ neighbour's terms (this plane)
    if (p - 1 >= z0 && active) {
      R* op = adj_phi;
      R* oq = adj_qo;
      size_t off = site, qs = N;
      if (xedge) {  // a tile-edge column: its adjoint without the face terms goes to hx
        op = hx + (lx == 0 ? 2 : 3) * fxs;
        oq = op + 4 * fxs;
        qs = 4 * fxs;
        off = (size_t(tx) * b.nz + pmod(p - 1, b.nz)) * b.ny + sGY[ly + 1];
      }
      op[off] = acc_p + (Gb.lapphi - R(0.5) * Gb.dphi[2]);
#pragma unroll
      for (int k = 0; k < 5; ++k) oq[k * qs + off] = acc_q[k] + (Gb.lapq[k] - R(0.5) * Gb.dq[2][k]);
    }
    if (own_plane) {
      // own terms, the z- neighbour's terms (previous plane), and the in-plane
      // transposes of the neighbours in this tile: lap - d/2 from the + side,
      // lap + d/2 from the - side
      auto nbr = [&](int fl, int fd, int s, bool in, R sgn) {
        return in ? sGB[fl][s] + sgn * R(0.5) * sGB[fd][s] : R(0);
      };
      acc_p = (Gb.phi - R(6) * Gb.lapphi) + (zp_lapphi + R(0.5) * zp_dphi);
      acc_p += nbr(0, 6, sxp, nxp >= 0, R(-1)) + nbr(0, 6, sxm, nxm >= 0, R(1));
      acc_p += nbr(0, 7, syp, nyp >= 0, R(-1)) + nbr(0, 7, sym, nym >= 0, R(1));
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        R a = (Gb.q[k] - R(6) * Gb.lapq[k]) + (zp_lapq[k] + R(0.5) * zp_dq[k]);
        a += nbr(1 + k, 8 + k, sxp, nxp >= 0, R(-1)) + nbr(1 + k, 8 + k, sxm, nxm >= 0, R(1));
        a += nbr(1 + k, 13 + k, syp, nyp >= 0, R(-1)) + nbr(1 + k, 13 + k, sym, nym >= 0, R(1));
        acc_q[k] = a;
      }
    }
    zp_lapphi = Gb.lapphi;
    zp_dphi = Gb.dphi[2];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      zp_lapq[k] = Gb.lapq[k];
      zp_dq[k] = Gb.dq[2][k];
    }
    if (more) {
      // plane p-1 is read by no one any more (all passed the barrier above):
      // plane p+2 takes its slot; the site inputs of plane p+1
      if constexpr (kEarly) {
#pragma unroll
        for (int j = 0; j < KI; ++j) {
          const int k = tid + j * NT;
          if (k < NI) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
              if (HM || f != 6) sIn[rm][f][k] = fv[j][f];
          }
        }
      } else {
        fill_plane(p + 2, rm);
      }
      load_site(p + 1, aq_o, qp_o, pp_o, ss_o, false);
      if constexpr (SYM) {
#pragma unroll
        for (int c = 0; c < 6; ++c) ss_o[c] = ss_n[c];
      }
    }
    const int t = rm;
    rm = r0;
    r0 = rp;
    rp = t;
  }
  block_reduce_store<2>(v, partial + size_t(blockIdx.x) * 2, accumulate != 0);
}

// The face terms of k_adj_sg_fused, in one launch of two block ranges (grid
// x: the rows or columns of a plane, y: the (field, face) pairs, z: the plane).
// Fields f = 0..5: phi, q[5].
// * x faces, one thread per (field, face j, z, y) when there are several x
//   tiles.  Tile j covers the columns j TX - 1 .. j TX + w_j - 2 (mod nx), so
//   the last column of tile j and the first of tile j+1 are neighbours in
//   memory; the thread writes both whole: the last column of tile j (its
//   adjoint without face terms plus the term sent in the - direction across
//   face j) and the first column of tile j+1 (the same, with the term sent in
//   the + direction).  A tile one column wide (only the last tile can be) gets
//   both of its terms from the thread of the face before it.  On a row that is
//   the first or last of its y tile, the thread adds that row's y-face terms
//   as well, so the corner sites are complete.
// * y faces, one thread per (field, y tile i, z, x) when there are several y
//   tiles: the first row of tile i takes the term sent in the + direction
//   across face i-1, its last row the term sent in the - direction across
//   face i (read-modify-write of what k_adj_sg_fused stored), at every column
//   except the x-edge columns, which the first range writes.
template <class R>
__global__ void __launch_bounds__(256) k_adj_faces(Box b, int TX, int ntx, int TY, int nty,
                                                   const R* __restrict__ hx, const R* __restrict__ hy,
                                                   R* __restrict__ adj_phi, R* __restrict__ adj_q) {
  // grid: x = the rows (columns) of a plane in blocks (of up to 256), y = (field,
  // face) of the x faces then of the y faces, z = the plane: the indices
  // come from the block, no division per thread.  32-bit index arithmetic:
  // every index below is under 6 N < 2^32.
  const uint32_t nx = b.nx, ny = b.ny, nz = b.nz;
  const uint32_t z = blockIdx.z;
  const uint32_t nxb = ntx > 1 ? 6u * uint32_t(ntx) : 0u;
  const uint32_t fxs = uint32_t(ntx) * nz * ny, fys = uint32_t(nty) * nz * nx;  // one field-side block of hx, hy
  if (blockIdx.y < nxb) {
    const uint32_t y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= ny) return;
    const uint32_t f = blockIdx.y / uint32_t(ntx), j = blockIdx.y - f * uint32_t(ntx);
    const uint32_t zy = z * ny + y;
    const uint32_t jn = j + 1 < uint32_t(ntx) ? j + 1 : 0;
    const int wj = min(TX, b.nx - int(j) * TX), wn = min(TX, b.nx - int(jn) * TX);
    const uint32_t xf = jn > 0 ? jn * TX - 1 : nx - 1;  // first column of tile jn; tile j's last is xf - 1
    R* out = (f == 0 ? adj_phi : adj_q + size_t(f - 1) * b.N) + size_t(zy) * nx;  // row (z, y)
    const R* hs = hx + size_t(4 * f) * fxs;
    const uint32_t fj = j * nz * ny + zy, fn = jn * nz * ny + zy;
    R vl = hs[3 * fxs + fj] + hs[fxs + fj];
    R vf = hs[2 * fxs + fn] + hs[fj];
    if (wn == 1) vf += hs[fxs + fn];
    if (nty > 1) {  // the y-face terms of a first or last row of a y tile
      const uint32_t i = y / uint32_t(TY), ly = y - i * uint32_t(TY);
      const uint32_t h = min(uint32_t(TY), ny - i * uint32_t(TY));
      const R* ys = hy + size_t(2 * f) * fys + z * nx;
      if (ly == 0) {
        const R* s0 = ys + ((i + nty - 1) % nty) * nz * nx;
        vl += s0[xf - 1];
        vf += s0[xf];
      }
      if (ly == h - 1) {
        const R* s1 = ys + fys + i * nz * nx;
        vl += s1[xf - 1];
        vf += s1[xf];
      }
    }
    if (wj > 1) out[xf - 1] = vl;
    out[xf] = vf;
    return;
  }
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nx) return;
  const uint32_t fi = blockIdx.y - nxb;
  const uint32_t f = fi / uint32_t(nty), i = fi - f * uint32_t(nty);
  // the x-edge columns (first and last of every x tile) belong to the first range
  if (ntx > 1 && ((x + 1) % TX == 0 || (x + 2) % TX == 0 || x + 2 >= nx)) return;
  const uint32_t zx = z * nx + x;
  const uint32_t ya = i * TY, yb = min(ya + TY, ny) - 1;
  R* out = (f == 0 ? adj_phi : adj_q + size_t(f - 1) * b.N) + size_t(z) * ny * nx + x;
  const R* hs = hy + size_t(2 * f) * fys;
  out[ya * nx] += hs[((i + nty - 1) % nty) * nz * nx + zx];
  out[yb * nx] += hs[fys + i * nz * nx + zx];
}

// out = in + 1 for the step counter of a recorded state (one thread, vector memory).
__global__ void k_step_count(const int64_t* __restrict__ in, int64_t* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = in[0] + 1;
}

// Seed of the displacement loss L = (z_c - z_ref)^2, z_c = sum phi z / sum phi:
// dL/dphi(x) = 2 (z_c - z_ref)(z - z_c) / sum phi; zero for g and Q.
template <class R>
__global__ void __launch_bounds__(256) k_seed_centre(Box b, int nq, double zc, double zref, double phitot,
                                                     R* __restrict__ adj) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.N) return;
  const size_t N = b.N;
  const int z = s / (b.nx * b.ny);
  for (int i = 0; i < nq + 5; ++i) adj[i * N + s] = R(0);
  adj[(nq + 5) * N + s] = R(2.0 * (zc - zref) * (double(z) - zc) / phitot);
}

}  // namespace lbc
