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
//                   (site-parallel, or z-marching over LDS tiles: k_adj_order_fused)
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
  force_at<D3Q19>(b, P, sig, x, y, z, F);
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
template <class R, class FS, int TX, int TY>
__global__ void __launch_bounds__(TX* TY)
k_adj_order_fused(Box b, Params<R> P, int TZ, int ntx, int nty, const FS* __restrict__ phi,
                  const FS* __restrict__ q, const R* __restrict__ u, const R* __restrict__ adj_phi,
                  const R* __restrict__ adj_q, R* __restrict__ mub, R* __restrict__ Wb_out, R* __restrict__ ubp,
                  R* __restrict__ qbp, R* __restrict__ phibp) {
  constexpr int NT = TX * TY;
  constexpr int SX = TX + 2, SY = TY + 2, NS = SX * SY;
  constexpr int NH = 2 * (TX + TY);
  static_assert(NH <= NT, "one halo slot per thread");
  constexpr int NV = 14;  // q[5], u[3], phi adjoint, q adjoint[5]
  __shared__ R sV[NV][NS];
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
  const int col = sGY[ly + 1] * b.nx + sGX[lx + 1];

  auto load_at = [&](size_t k, R v[NV]) {
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = R(q[c * N + k]);
#pragma unroll
    for (int a = 0; a < 3; ++a) v[5 + a] = u[a * N + k];
    v[8] = adj_phi[k];
#pragma unroll
    for (int c = 0; c < 5; ++c) v[9 + c] = adj_q[c * N + k];
  };
  auto load_col = [&](int zz, R v[NV]) { load_at(size_t(pmod(zz, b.nz)) * plane + col, v); };
  R vm[NV], v0[NV], vp[NV];
  load_col(z0 - 1, vm);
  load_col(z0, v0);
  load_col(z0 + 1, vp);

  const bool has_halo = tid < NH;
  int hs = 0, hcol = 0;
  if (has_halo) {
    int hx, hy;
    if (tid < 2 * TX) {
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
  if (has_halo) load_at(size_t(z0) * plane + hcol, hv);

  const int sc = (ly + 1) * SX + (lx + 1);
  for (int zc = z0; zc < z1; ++zc) {
    __syncthreads();  // previous plane's reads are done
#pragma unroll
    for (int c = 0; c < NV; ++c) sV[c][sc] = v0[c];
    if (has_halo) {
#pragma unroll
      for (int c = 0; c < NV; ++c) sV[c][hs] = hv[c];
      if (zc + 1 < z1) load_at(size_t(zc + 1) * plane + hcol, hv);  // next plane's halo
    }
    __syncthreads();
    if (active) {
      const size_t site = size_t(zc) * plane + col;
      const R ph = R(phi[site]);
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
      R m, Wb[3][3], ub[3], qb[5], pb;
      adj_order_site(P, qc, qbar, uc, ph, v0[8], pbn, un, qn, aqn, m, Wb, ub, qb, pb);
      store_adj_order(N, site, m, Wb, ub, qb, pb, mub, Wb_out, ubp, qbp, phibp);
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      vm[c] = v0[c];
      v0[c] = vp[c];
    }
    if (zc + 1 < z1) load_col(zc + 2, vp);
  }
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
    // pulled populations and pushed adjoints are read once: streaming loads
    // (32/64-bit storage; half storage keeps ordinary loads)
    const int sp = sidx(b, x - CX(i), y - CY(i), z - CZ(i));
    if constexpr (sizeof(GS) >= 4)
      g[i] = R(__builtin_nontemporal_load(B + i * N + sp));
    else
      g[i] = GPol<GS>::template ld<R>(B, i * N + sp, i);
    gsb[i] = __builtin_nontemporal_load(adj_g + i * N + sidx(b, x + CX(i), y + CY(i), z + CZ(i)));
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) Fs[a] = F[a * N + s];
  R gb[19], Fb[3] = {R(0), R(0), R(0)};
  collide_site_bwd(P, g, Fs, gsb, ub, gb, Fb);
#pragma unroll
  for (int i = 0; i < 19; ++i) __builtin_nontemporal_store(gb[i], g_out + i * N + s);
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
    G.divv = R(0);  // mu's anchoring divergence is reversed below through v_bar
    // sigma_bar_ab = -D0_b F_bar_a;  v_bar_a = -D0_a divv_bar with divv_bar = -2 W mu_bar
    R sb[9], vb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int a = 0; a < 3; ++a) sb[3 * a + c] = -R(0.5) * (Fn[c][0][a] - Fn[c][1][a]);
      vb[c] = P.W * (mbn[c][0] - mbn[c][1]);
    }
    R hbs[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) hbs[k] = P.Gamma * aq[k];
    GradBar<R> Gb;
    Gb.zero();
    ParBar<R> Pb{R(0), R(0), R(0)};
    sigma_site_bwd(P, G, sb, hbs, Gb, Pb);
    mu_site_bwd(P, G.phi, G.q, mb0, Gb.phi, Gb.lapphi, Gb.divv, Gb.q);
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
    Gb.phi += pbp;
#pragma unroll
    for (int k = 0; k < 5; ++k) Gb.q[k] += qp[k];
    store_gb(Gb, gbar, N, s);
    v[0] = double(Pb.zeta);
    v[1] = 2.0 * double(P.K) * double(Pb.kq) + 8.0 * double(P.K) * double(P.q0) * double(Pb.kq2);
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
