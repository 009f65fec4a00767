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
// One product R'(X)^T V is, by default, k_pcb_mub (mu_bar = M L4 V_phi),
// k_pcb_fused (the local reverses and the x, y transposes in one z-march, with
// the terms owed across tile faces handed to the next pass) and
// k_pcb_gather_z (the z transposes and those face terms).  Where the tiling
// leaves a tile one site wide, and on request (lb_tuning.pc_adj = 1), it takes
// three site-parallel passes and the z pass instead:
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
#include <type_traits>
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

// mu_bar = M vs L4 vphi of one product at every site: the adjoint of mu4,
// which the fused product reads with a D4 stencil (v_bar = 2 W D4 mu_bar).
// A workgroup covers a TX x TY tile of NP planes: it loads the NP + 4 planes
// of vphi the stencils read (the tile with an in-plane halo of 2) at once,
// puts them in LDS and forms the laplacian of its NP planes, summing the x,
// y, z stencils in that order.
template <class R, int TX, int TY, int NP>
__global__ void __launch_bounds__(TX* TY) k_pcb_mub(Box b, Params<R> P, int ntx, int nty,
                                                   const R* __restrict__ vphi, R vs, R* __restrict__ mub) {
  constexpr int NT = TX * TY, SX = TX + 4, SY = TY + 4, NF = SX * SY, KR = (NF + NT - 1) / NT;
  constexpr int NL = NP + 4;  // planes z0 - 2 .. z0 + NP + 1
  __shared__ R sF[NL][NF];
  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = l % ntx, ty = (l / ntx) % nty, sl = l / (ntx * nty);
  const int x0 = tx * TX, y0 = ty * TY, z0 = sl * NP;
  const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
  const uint32_t plane = uint32_t(b.nx) * uint32_t(b.ny);
  R v[NL][KR];
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    const int k = tid + j * NT;
    if (k < NF) {
      const uint32_t col = uint32_t(pmod(y0 - 2 + k / SX, b.ny) * b.nx + pmod(x0 - 2 + k % SX, b.nx));
#pragma unroll
      for (int i = 0; i < NL; ++i)
        v[i][j] = ldo(vphi, (uint32_t(pmod(z0 - 2 + i, b.nz)) * plane + col) * uint32_t(sizeof(R)));
    }
  }
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    const int k = tid + j * NT;
    if (k < NF) {
#pragma unroll
      for (int i = 0; i < NL; ++i) sF[i][k] = v[i][j];
    }
  }
  __syncthreads();
  if (x0 + lx >= b.nx || y0 + ly >= b.ny) return;
  const int c = (ly + 2) * SX + (lx + 2);
  const uint32_t own = (uint32_t(y0 + ly) * uint32_t(b.nx) + uint32_t(x0 + lx)) * uint32_t(sizeof(R));
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int p = z0 + i;
    if (p >= b.nz) break;
    const R* f = sF[i + 2];
    R lapv = R(-7.5) * f[c];
    lapv += l4c(f[c - 2], f[c - 1], f[c + 1], f[c + 2]);
    lapv += l4c(f[c - 2 * SX], f[c - SX], f[c + SX], f[c + 2 * SX]);
    lapv += l4c(sF[i][c], sF[i + 1][c], sF[i + 3][c], sF[i + 4][c]);
    sto(mub, uint32_t(p) * plane * uint32_t(sizeof(R)) + own, P.M * vs * lapv);
  }
}

// Coefficients of the transposed axis stencils: a site x gathers
// L4^T f = sum_d l4w(d) f(x + d) (plus -7.5 f(x), once over the axes) and
// D4^T f = -D4 f = sum_d d4w(d) f(x + d), d = -2, -1, 1, 2.
template <class R>
__device__ __forceinline__ R l4w(int d) {
  return (d == 1 || d == -1) ? R(16.0 / 12.0) : R(-1.0 / 12.0);
}
template <class R>
__device__ __forceinline__ R d4w(int d) {
  return d == 1 ? R(-8.0 / 12.0) : d == -1 ? R(8.0 / 12.0) : d == 2 ? R(1.0 / 12.0) : R(-1.0 / 12.0);
}

// One 32-bit value per lane from global memory straight into LDS
// (global_load_lds_dword): lane i of the wave writes lds_wave[i].  The data
// is visible to the workgroup after s_waitcnt and a barrier.
__device__ __forceinline__ void g2lds(const float* src, float* lds_wave) {
  __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)(src),
                                   (__attribute__((address_space(3))) void*)(lds_wave), 4, 0, 0);
}

// A face record along x: the 9 output fields of one owed term, padded to 12
// values so that it moves as three 16-byte (float) or six 16-byte (double)
// accesses (a receiving site of an x face reads its record alone; y faces are
// whole rows and keep one array per field).
constexpr int kRec = 12;
template <class R>
__device__ __forceinline__ void st_rec(R* __restrict__ p, const R v[9]) {
  if constexpr (sizeof(R) == 4) {
    float4* q = reinterpret_cast<float4*>(p);
    q[0] = make_float4(v[0], v[1], v[2], v[3]);
    q[1] = make_float4(v[4], v[5], v[6], v[7]);
    q[2] = make_float4(v[8], 0.0f, 0.0f, 0.0f);
  } else {
    double2* q = reinterpret_cast<double2*>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = make_double2(v[2 * i], v[2 * i + 1]);
    q[4] = make_double2(v[8], 0.0);
  }
}
template <class R>
__device__ __forceinline__ void ld_rec(const R* __restrict__ p, R t[9]) {
  if constexpr (sizeof(R) == 4) {
    const float4* q = reinterpret_cast<const float4*>(p);
    const float4 a = q[0], c = q[1], d = q[2];
    t[0] = a.x; t[1] = a.y; t[2] = a.z; t[3] = a.w;
    t[4] = c.x; t[5] = c.y; t[6] = c.z; t[7] = c.w;
    t[8] = d.x;
  } else {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double2 a = q[i];
      t[2 * i] = a.x;
      t[2 * i + 1] = a.y;
    }
    t[8] = q[4].x;
  }
}
template <class R>
__device__ __forceinline__ void add_rec(const R* __restrict__ p, R t[9]) {
  if constexpr (sizeof(R) == 4) {
    const float4* q = reinterpret_cast<const float4*>(p);
    const float4 a = q[0], c = q[1], d = q[2];
    t[0] += a.x; t[1] += a.y; t[2] += a.z; t[3] += a.w;
    t[4] += c.x; t[5] += c.y; t[6] += c.z; t[7] += c.w;
    t[8] += d.x;
  } else {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double2 a = q[i];
      t[2 * i] += a.x;
      t[2 * i + 1] += a.y;
    }
    t[8] += q[4].x;
  }
}

// ---------------------------------------------------------------------------
// k_pcb_fused: one product R'(X)^T V of the pc4 reverse (k_pcb_local, k_pcb_v
// and k_pcb_gather together) in one z-march over a TX x TY tile and a slab of
// TZ planes, with the Heun combination out = c1 X_bar(t+1) + c2 Xs + R'^T V
// and u_bar written (accumulate = 0) or added to (accumulate = 1).
//   Per plane, LDS holds the 16 input fields (Q, phi, u, mu_bar for the
//   stencils of the local reverse; V for the neighbour terms of the upwind
//   and donor-cell operators) on the tile with an in-plane cross-shaped halo
//   of 2; the owned column keeps Q, phi, u, mu_bar of planes z-2 .. z+2 in
//   registers.  Each thread forms the local reverse of its own site (the
//   stencil-data adjoints of H4, mu4, the co-rotation and the site's own
//   upwind terms, with v_bar = -D4 (-2 W mu_bar) folded in) and puts the 24
//   stencil-data adjoints the x and y transposes read in LDS.  A site then
//   gathers the x and y transposes from the neighbours in its tile (a lone
//   tile along an axis wraps inside itself).  Two kinds of terms are left to
//   k_pcb_gather_z:
//   * the z transposes: of the 15 stencil-data adjoints with z stencils, the
//     9 that depend on the site's reverse go to zf[9][N] (D4_z Q adjoints,
//     the D4_z phi adjoint, W_az adjoints); the L4 Q and L4 phi adjoints are
//     K Gamma V_Q and -k_phi mu_bar, which k_pcb_gather_z forms from V and
//     mu_bar itself;
//   * the terms a site owes the two columns (rows) across a tile face: the
//     last two columns of tile j send to the first two of tile j+1 and back.
//     Per output field (q[5], phi, u[3]) the edge column owes the whole
//     term of the first site across (its own part and its inner neighbour's,
//     read from LDS; pos 0) and of the second (pos 1); side 0 holds what
//     tile j sends in the + direction across face j, side 1 what tile j+1
//     sends in the - direction.  These terms are formed as work items spread
//     over the waves after the transposes.  x faces as records of the 9 fields,
//     fx[(((((side 2 + pos) ntx + j) nz + z) ny + y) kRec + f], y faces one
//     array per field, fy[((((f 2 + side) 2 + pos) nty + i) nz + z) nx + x].
//     Every tile along a split axis is at least two sites wide (checked by
//     the caller).
// partial: one float64 (zeta, q0) pair per block, overwritten (pacc = 0) or
// added to (pacc = 1).
// ---------------------------------------------------------------------------
template <class R, class FS, int TX, int TY>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 2 : 1)))
k_pcb_fused(Box b, Params<R> P, int TZ, int ntx, int nty, const FS* __restrict__ phi, const FS* __restrict__ q,
            const R* __restrict__ u, const R* __restrict__ vq, const R* __restrict__ vphi, R vs,
            const R* __restrict__ mub, const R* __restrict__ xq1, const R* __restrict__ xp1, R c1,
            const R* __restrict__ xsq, const R* __restrict__ xsp, R c2, R* __restrict__ q_out,
            R* __restrict__ phi_out, R* __restrict__ ub_out, int accumulate, R* __restrict__ zf,
            R* __restrict__ fx, R* __restrict__ fy, double* __restrict__ partial, int pacc) {
  constexpr int NT = TX * TY;
  constexpr int HR = 2;
  constexpr int SX = TX + 2 * HR, SY = TY + 2 * HR, NS = SX * SY;
  constexpr int NH = 2 * HR * (TX + TY);  // halo slots of the axis stencils (no corners)
  static_assert(NH <= NT, "one halo slot per thread");
  constexpr int NZ = 10;  // fields with z stencils: q[5], phi, u[3], mu_bar
  constexpr int NV = 16;  // and V: vq[5], vphi
  // x, y stencil-data adjoints: lapq[5], lapphi, dq_x[5], dq_y[5], dphi_x, dphi_y, W_ax[3], W_ay[3]
  constexpr int XL = 0, XLP = 5, XDQ = 6, XDP = 16, XW = 18, NXF = 24;
  __shared__ R sV[NV][NS];
  // the tile's x, y stencil-data adjoints, each row padded with two zero
  // columns on both sides: the x transposes read fixed offsets, and a site
  // beyond the tile's last column (or a ragged tile's width) reads zeros (a
  // lone x tile wraps inside itself instead)
  constexpr int PX = TX + 4, NTP = TY * PX;
  __shared__ R sX[NXF][NTP];
  __shared__ int sGX[SX], sGY[SY];
  // float: the next plane's V and halo, and this plane's inputs of the Heun
  // combination, go from global memory to LDS staging buffers while the local
  // reverse runs (global_load_lds, no registers); double loads them where used
  constexpr bool kStage = sizeof(R) == 4;
  constexpr int NHP = (NH + 63) / 64 * 64;  // whole waves of halo slots
  constexpr int NO = 15;                    // xq1[5], xp1, xsq[5], xsp, ub_out[3]
  __shared__ R sStV[kStage ? 6 : 1][kStage ? NT : 1];
  __shared__ R sStH[kStage ? NV : 1][kStage ? NHP : 1];
  __shared__ R sStO[kStage ? NO : 1][kStage ? NT : 1];

  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = l % ntx, ty = (l / ntx) % nty, sl = l / (ntx * nty);
  const int x0 = tx * TX, y0 = ty * TY, z0 = sl * TZ;
  const int z1 = min(z0 + TZ, b.nz);
  const int w = min(TX, b.nx - x0), h = min(TY, b.ny - y0);
  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = tid / TX;
  const bool active = lx < w && ly < h;
  const size_t N = b.N;
  const int plane = b.nx * b.ny;

  for (int k = tid; k < SX; k += NT) sGX[k] = pmod(x0 - HR + k, b.nx);
  for (int k = tid; k < SY; k += NT) sGY[k] = pmod(y0 - HR + k, b.ny);
  for (int k = tid; k < NXF * NTP; k += NT) (&sX[0][0])[k] = R(0);  // pads and inactive sites stay zero
  __syncthreads();
  const int col = sGY[ly + HR] * b.nx + sGX[lx + HR];

  // global accesses: uniform field base plus a 32-bit byte offset per lane
  // (component arrays are below 4 GiB)
  constexpr uint32_t SR = sizeof(R), SF = sizeof(FS);
  auto load_z = [&](int zz, R v[NZ]) {
    const uint32_t k = uint32_t(pmod(zz, b.nz)) * uint32_t(plane) + uint32_t(col);
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = R(ldo(q + c * N, k * SF));
    v[5] = R(ldo(phi, k * SF));
#pragma unroll
    for (int a = 0; a < 3; ++a) v[6 + a] = ldo(u + a * N, k * SR);
    v[9] = ldo(mub, k * SR);
  };
  auto load_v = [&](uint32_t k, R v[6]) {
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = ldo(vq + c * N, k * SR);
    v[5] = ldo(vphi, k * SR);
  };
  // owned column: planes z-2 .. z+2 of the z-stencil fields
  R zr[5][NZ];
#pragma unroll
  for (int j = 0; j < 5; ++j) load_z(z0 - 2 + j, zr[j]);

  // this thread's halo slot: 2 HR rows of TX, then 2 HR columns of TY
  const bool has_halo = tid < NH;
  int hs = 0, hcol = 0;
  if (has_halo) {
    int hx, hy;
    if (tid < 2 * HR * TX) {
      const int r = tid / TX;
      hx = HR + tid % TX;
      hy = r < HR ? r : TY + r;
    } else {
      const int t = tid - 2 * HR * TX;
      const int c = t / TY;
      hy = HR + t % TY;
      hx = c < HR ? c : TX + c;
    }
    hs = hy * SX + hx;
    hcol = sGY[hy] * b.nx + sGX[hx];
  }
  auto load_all = [&](int zz, R v[NV]) {
    const uint32_t k = uint32_t(zz) * uint32_t(plane) + uint32_t(hcol);
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = R(ldo(q + c * N, k * SF));
    v[5] = R(ldo(phi, k * SF));
#pragma unroll
    for (int a = 0; a < 3; ++a) v[6 + a] = ldo(u + a * N, k * SR);
    v[9] = ldo(mub, k * SR);
#pragma unroll
    for (int c = 0; c < 5; ++c) v[10 + c] = ldo(vq + c * N, k * SR);
    v[15] = ldo(vphi, k * SR);
  };

  // in-tile neighbour at offset d (|d| <= 2) along x (y); -1 where it is in
  // another tile (a lone tile wraps: t in [-2, n + 1] folds into [0, n))
  auto wrap2 = [](int t, int n) {
    t += t < 0 ? n : 0;
    t += t < 0 ? n : 0;
    t -= t >= n ? n : 0;
    t -= t >= n ? n : 0;
    return t;
  };
  // (indices into the padded rows of sX)
  auto nbx = [&](int d) {
    const int t = lx + d;
    if (ntx == 1) return ly * PX + wrap2(t, w) + 2;
    return (t >= 0 && t < w) ? ly * PX + t + 2 : -1;
  };
  auto nby = [&](int d) {
    const int t = ly + d;
    if (nty == 1) return wrap2(t, h) * PX + lx + 2;
    return (t >= 0 && t < h) ? t * PX + lx + 2 : -1;
  };
  const int xs = ly * PX + lx + 2;  // this site's slot in sX
  const size_t fxs = size_t(ntx) * b.nz * b.ny, fys = size_t(nty) * b.nz * b.nx;  // one (side, pos) block of records / of a field
  const int kxm = (tx + ntx - 1) % ntx, kym = (ty + nty - 1) % nty;

  const int sc = (ly + HR) * SX + (lx + HR);
  const int wb = (tid >> 6) << 6;  // first thread of this wave
  // staging (float): V and the halo of plane zz; the combination inputs of plane zz
  auto stage_vh = [&](int zz) {
    if constexpr (kStage) {
      const uint32_t k = uint32_t(zz) * uint32_t(plane) + uint32_t(col);
#pragma unroll
      for (int c = 0; c < 5; ++c) g2lds(reinterpret_cast<const float*>(vq + c * N) + k, reinterpret_cast<float*>(&sStV[c][wb]));
      g2lds(reinterpret_cast<const float*>(vphi) + k, reinterpret_cast<float*>(&sStV[5][wb]));
      if (has_halo) {
        const uint32_t kh = uint32_t(zz) * uint32_t(plane) + uint32_t(hcol);
        const float* src[NV] = {};
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          src[c] = reinterpret_cast<const float*>(q + c * N);
          src[10 + c] = reinterpret_cast<const float*>(vq + c * N);
        }
        src[5] = reinterpret_cast<const float*>(phi);
#pragma unroll
        for (int a = 0; a < 3; ++a) src[6 + a] = reinterpret_cast<const float*>(u + a * N);
        src[9] = reinterpret_cast<const float*>(mub);
        src[15] = reinterpret_cast<const float*>(vphi);
#pragma unroll
        for (int c = 0; c < NV; ++c) g2lds(src[c] + kh, reinterpret_cast<float*>(&sStH[c][wb]));
      }
    }
  };
  auto stage_o = [&](int zz) {
    if constexpr (kStage) {
      const uint32_t k = uint32_t(zz) * uint32_t(plane) + uint32_t(col);
#pragma unroll
      for (int c = 0; c < 5; ++c) g2lds(reinterpret_cast<const float*>(xq1 + c * N) + k, reinterpret_cast<float*>(&sStO[c][wb]));
      g2lds(reinterpret_cast<const float*>(xp1) + k, reinterpret_cast<float*>(&sStO[5][wb]));
      if (xsq) {
#pragma unroll
        for (int c = 0; c < 5; ++c) g2lds(reinterpret_cast<const float*>(xsq + c * N) + k, reinterpret_cast<float*>(&sStO[6 + c][wb]));
        g2lds(reinterpret_cast<const float*>(xsp) + k, reinterpret_cast<float*>(&sStO[11][wb]));
      }
      if (accumulate) {
#pragma unroll
        for (int a = 0; a < 3; ++a) g2lds(reinterpret_cast<const float*>(ub_out + a * N) + k, reinterpret_cast<float*>(&sStO[12 + a][wb]));
      }
    }
  };
  stage_vh(z0);
  double v2[2] = {0.0, 0.0};
  for (int zc = z0; zc < z1; ++zc) {
    if constexpr (kStage) __builtin_amdgcn_s_waitcnt(0);  // this thread's staging loads have landed
    __syncthreads();  // the previous plane's reads are done; the staged V and halo are in place
#pragma unroll
    for (int c = 0; c < NZ; ++c) sV[c][sc] = zr[2][c];
    if constexpr (kStage) {
#pragma unroll
      for (int c = 0; c < 6; ++c) sV[NZ + c][sc] = sStV[c][tid];
      if (has_halo) {
#pragma unroll
        for (int c = 0; c < NV; ++c) sV[c][hs] = sStH[c][tid];
      }
    } else {
      R vv[6];  // V of the owned site
      load_v(uint32_t(zc) * uint32_t(plane) + uint32_t(col), vv);
#pragma unroll
      for (int c = 0; c < 6; ++c) sV[NZ + c][sc] = vv[c];
      if (has_halo) {  // the halo of this plane
        R hv[NV];
        load_all(zc, hv);
#pragma unroll
        for (int c = 0; c < NV; ++c) sV[c][hs] = hv[c];
      }
    }
    __syncthreads();
    // in flight during the local reverse: the combination inputs of this plane, V and halo of the next
    stage_o(zc);
    if (zc + 1 < z1) stage_vh(zc + 1);
    // ---- local reverse at the own site
    R qbl[5], pbl = R(0), ubl[3] = {R(0), R(0), R(0)};
    if (active) {
      auto nb = [&](int f, int g, R& m2, R& m1, R& p1, R& p2) {
        if (g == 0) {
          m2 = sV[f][sc - 2]; m1 = sV[f][sc - 1]; p1 = sV[f][sc + 1]; p2 = sV[f][sc + 2];
        } else if (g == 1) {
          m2 = sV[f][sc - 2 * SX]; m1 = sV[f][sc - SX]; p1 = sV[f][sc + SX]; p2 = sV[f][sc + 2 * SX];
        } else {
          m2 = zr[0][f]; m1 = zr[1][f]; p1 = zr[3][f]; p2 = zr[4][f];
        }
      };
      Grad<R> G;
      G.phi = zr[2][5];
      G.lapphi = R(0);
      G.divv = R(0);
      R W[3][3], vb[3], VQ[5], uq[5] = {R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        G.q[k] = zr[2][k];
        G.lapq[k] = R(-7.5) * G.q[k];
        VQ[k] = vs * sV[NZ + k][sc];
      }
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        R m2, m1, p1, p2;
        nb(5, g, m2, m1, p1, p2);
        G.dphi[g] = d4c(m2, m1, p1, p2);
        // the site's own upwind terms along g: R_Q gets
        // -max(u_g,0)(Q - Q(x-e_g)) - min(u_g,0)(Q(x+e_g) - Q)
        const R ug = zr[2][6 + g], up = ug > R(0) ? ug : R(0), um = ug < R(0) ? ug : R(0);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          nb(k, g, m2, m1, p1, p2);
          G.dq[g][k] = d4c(m2, m1, p1, p2);
          G.lapq[k] += l4c(m2, m1, p1, p2);
          const R a = -VQ[k];
          const R back = G.q[k] - m1, fwd = p1 - G.q[k];
          uq[k] += a * (up - um);
          ubl[g] += a * ((ug >= R(0) ? back : R(0)) + (ug <= R(0) ? fwd : R(0)));
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          nb(6 + a, g, m2, m1, p1, p2);
          W[a][g] = d4c(m2, m1, p1, p2);
        }
        // v = Q D4 phi: v_bar_g = -D4_g divv_bar with divv_bar = -2 W mu_bar
        nb(9, g, m2, m1, p1, p2);
        const R w2 = R(2) * P.W;
        vb[g] = -d4c(-(w2 * m2), -(w2 * m1), -(w2 * p1), -(w2 * p2));
      }
      R hb[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) hb[k] = P.Gamma * VQ[k];
      Local<R> Lc;
      local_thermo(P, G, Lc);
      GradBar<R> Gb;
      Gb.zero();
      ParBar<R> Pb{R(0), R(0), R(0)};
      R lapphib = R(0), divvb = R(0), tr2b = R(0), tr3b = R(0);
      mu_site_bwd_local(P, G.phi, Lc.tr2, zr[2][9], Gb.phi, lapphib, divvb, tr2b, tr3b);
      local_thermo_bwd(P, G, Lc, hb, tr2b, tr3b, R(0), R(0), R(0), Gb, Pb);
      R Wb[3][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
#pragma unroll
      for (int k = 0; k < 5; ++k) qbl[k] = Gb.q[k];
      corotation_site_bwd(P.xi, G.q, W, VQ, qbl, Wb);
      pbl = Gb.phi;
#pragma unroll
      for (int k = 0; k < 5; ++k) qbl[k] += uq[k];
      // v = Q D4 phi at the site: Q_bar_ab += v_bar_a D4_b phi, (D4 phi)_bar_b += Q_ab v_bar_a
      {
        const R xx = G.q[0], xy = G.q[1], xz = G.q[2], yy = G.q[3], yz = G.q[4], zz = -xx - yy;
        const R Qm[3][3] = {{xx, xy, xz}, {xy, yy, yz}, {xz, yz, zz}};
        R Qb[3][3], qv[5] = {R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
          for (int c = 0; c < 3; ++c) Qb[a][c] = vb[a] * G.dphi[c];
          Gb.dphi[a] += Qm[a][0] * vb[0] + Qm[a][1] * vb[1] + Qm[a][2] * vb[2];
        }
        full_to_stored(Qb, qv);
#pragma unroll
        for (int k = 0; k < 5; ++k) qbl[k] += qv[k];
      }
      par_adjoints(P, Pb, v2);
      // x, y stencil-data adjoints to LDS; z ones to zf
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        sX[XL + k][xs] = Gb.lapq[k];
        sX[XDQ + k][xs] = Gb.dq[0][k];
        sX[XDQ + 5 + k][xs] = Gb.dq[1][k];
      }
      sX[XLP][xs] = lapphib;
      sX[XDP][xs] = Gb.dphi[0];
      sX[XDP + 1][xs] = Gb.dphi[1];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sX[XW + a][xs] = Wb[a][0];
        sX[XW + 3 + a][xs] = Wb[a][1];
      }
      const uint32_t so = (uint32_t(zc) * uint32_t(plane) + uint32_t(col)) * SR;
#pragma unroll
      for (int k = 0; k < 5; ++k) sto(zf + k * N, so, Gb.dq[2][k]);
      sto(zf + 5 * N, so, Gb.dphi[2]);
#pragma unroll
      for (int a = 0; a < 3; ++a) sto(zf + (6 + a) * N, so, Wb[a][2]);
    }
    if constexpr (kStage) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();  // the stencil-data adjoints of the tile (and the staged inputs) are in place
    // the own column's plane zc + 3, loaded while the transposes are gathered
    // (planes zc - 2 and zc +- 1, +2 of the ring are not read after the local reverse)
    R zn[NZ];
    if (zc + 1 < z1) load_z(zc + 3, zn);
    if (active) {
      const uint32_t so = (uint32_t(zc) * uint32_t(plane) + uint32_t(col)) * SR;
      constexpr int dd[4] = {-2, -1, 1, 2};
      int iy[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) iy[k] = nby(dd[k]);
      auto vy = [&](int f, int k) { return iy[k] >= 0 ? sX[f][iy[k]] : R(0); };
      auto l4y = [&](int f) { return l4c(vy(f, 0), vy(f, 1), vy(f, 2), vy(f, 3)); };
      auto d4y = [&](int f) { return -d4c(vy(f, 0), vy(f, 1), vy(f, 2), vy(f, 3)); };
      R qo[5], po, ub[3];
      // the transposes; x neighbours at fixed offsets in the padded rows, or
      // wrapped inside a lone x tile (two copies of the code, one branch)
      auto transposes = [&](auto lone) {
        constexpr bool LONE = decltype(lone)::value;
        int ix[4];
        if constexpr (LONE) {
#pragma unroll
          for (int k = 0; k < 4; ++k) ix[k] = nbx(dd[k]);
        }
        auto vx = [&](int f, int k) {
          if constexpr (LONE)
            return sX[f][ix[k]];
          else
            return sX[f][xs + dd[k]];
        };
        auto l4x = [&](int f) { return l4c(vx(f, 0), vx(f, 1), vx(f, 2), vx(f, 3)); };
        auto d4x = [&](int f) { return -d4c(vx(f, 0), vx(f, 1), vx(f, 2), vx(f, 3)); };
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          R r = qbl[k] + ((R(-7.5) * sX[XL + k][xs] + l4x(XL + k)) + l4y(XL + k));
          r += d4x(XDQ + k);
          r += d4y(XDQ + 5 + k);
          qo[k] = r;
        }
        {
          R r = pbl + ((R(-7.5) * sX[XLP][xs] + l4x(XLP)) + l4y(XLP));
          r += d4x(XDP);
          r += d4y(XDP + 1);
          po = r;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          R r = ubl[a];
          r += d4x(XW + a);
          r += d4y(XW + 3 + a);
          ub[a] = r;
        }
      };
      if (ntx == 1)
        transposes(std::true_type{});
      else
        transposes(std::false_type{});
      // the x and y neighbour terms of the upwind and donor-cell operators
      const R ph = zr[2][5], vp0 = vs * sV[NZ + 5][sc];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const int m1 = g == 0 ? sc - 1 : sc - SX, p1 = g == 0 ? sc + 1 : sc + SX;
        const R ugp = sV[6 + g][p1], ugm = sV[6 + g][m1], ugs = zr[2][6 + g];
        const R upx = ugp > R(0) ? ugp : R(0), umx = ugm < R(0) ? ugm : R(0);
#pragma unroll
        for (int k = 0; k < 5; ++k) qo[k] += (vs * sV[NZ + k][p1]) * upx - (vs * sV[NZ + k][m1]) * umx;
        const R fp = R(0.5) * (ugs + ugp), fm = R(0.5) * (ugm + ugs);
        const R cp = vs * sV[NZ + 5][p1] - vp0, cm = vp0 - vs * sV[NZ + 5][m1];
        const R php = sV[5][p1], phm = sV[5][m1];
        po += cp * (fp > R(0) ? fp : R(0)) + cm * (fm < R(0) ? fm : R(0));
        const R dfp = (fp >= R(0) ? ph : R(0)) + (fp <= R(0) ? php : R(0));
        const R dfm = (fm >= R(0) ? phm : R(0)) + (fm <= R(0) ? ph : R(0));
        ub[g] += R(0.5) * (cp * dfp + cm * dfm);
      }
      // the combination inputs of this site: staged (float) or loaded
      auto in_o = [&](int c, const R* base) { return kStage ? sStO[c][tid] : ldo(base, so); };
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        R r = c1 * in_o(k, xq1 + k * N) + qo[k];
        if (xsq) r += c2 * in_o(6 + k, xsq + k * N);
        sto(q_out + k * N, so, r);
      }
      {
        R r = c1 * in_o(5, xp1) + po;
        if (xsp) r += c2 * in_o(11, xsp);
        sto(phi_out, so, r);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) sto(ub_out + a * N, so, accumulate ? in_o(12 + a, ub_out + a * N) + ub[a] : ub[a]);
    }
    // the terms owed across the tile faces, per output field q[5], phi, u[3]:
    // an edge site sends, for the first site across, its own term and that of
    // its inner neighbour, and its own for the second.  They are formed from
    // the stencil-data adjoints in LDS as one work item per (row, side, pos)
    // of the x faces and (column, side, pos) of the y faces, spread evenly
    // over the waves (an edge lane of every row would leave the other lanes
    // of its wave idle through the whole branch).
    {
      auto owed = [&](int t, int g, int d, R o[9], bool add) {
        const R lw = l4w<R>(-d), dw = d4w<R>(-d);  // the sender is at offset -d from the receiver
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const R v = sX[XL + k][t] * lw + sX[XDQ + 5 * g + k][t] * dw;
          o[k] = add ? o[k] + v : v;
        }
        const R v5 = sX[XLP][t] * lw + sX[XDP + g][t] * dw;
        o[5] = add ? o[5] + v5 : v5;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const R v = sX[XW + 3 * g + a][t] * dw;
          o[6 + a] = add ? o[6 + a] + v : v;
        }
      };
      // side 0: sent in the + direction by the last column (row) of the tile,
      // side 1: in the - direction by the first; pos 0 / 1: the first / second
      // site across
      auto owed_item = [&](int t, int g, int side, int pos, int step, R o[9]) {
        const int dir = side == 0 ? 1 : -1;
        if (pos == 0) {
          owed(t, g, dir, o, false);
          owed(t - dir * step, g, 2 * dir, o, true);
        } else {
          owed(t, g, 2 * dir, o, false);
        }
      };
      constexpr int NXI = 4 * TY, NYI = 4 * TX, NW = NT / 64;
      constexpr int NWI = (NXI + NYI + NW - 1) / NW;  // items per wave
      static_assert(NWI <= 64, "face items fit the lanes");
      // the item of this lane, formed from the thread id in each plane (an
      // empty asm keeps it from being hoisted and held across the march)
      int tf = tid;
      asm volatile("" : "+v"(tf));
      const int lane = tf & 63, it = (tf >> 6) * NWI + lane;
      if (lane < NWI) {
        if (it < NXI) {
          // consecutive lanes take consecutive rows of one (side, pos): whole runs of records
          const int r = it % TY, side = it / (2 * TY), pos = (it / TY) & 1;
          if (ntx > 1 && r < h) {
            R o[9];
            owed_item(r * PX + (side == 0 ? w - 1 : 0) + 2, 0, side, pos, 1, o);
            const size_t off = (size_t(side == 0 ? tx : kxm) * b.nz + zc) * b.ny + sGY[r + HR];
            st_rec(fx + (size_t(side * 2 + pos) * fxs + off) * kRec, o);
          }
        } else if (it < NXI + NYI) {
          const int i2 = it - NXI;
          const int cc = i2 % TX, side = i2 / (2 * TX), pos = (i2 / TX) & 1;
          if (nty > 1 && cc < w) {
            R o[9];
            owed_item((side == 0 ? h - 1 : 0) * PX + cc + 2, 1, side, pos, PX, o);
            // uniform field base plus a 32-bit byte offset (one field block of fy is below 4 GiB)
            const uint32_t off = (uint32_t(side * 2 + pos) * uint32_t(fys) +
                                  (uint32_t(side == 0 ? ty : kym) * uint32_t(b.nz) + uint32_t(zc)) * uint32_t(b.nx) +
                                  uint32_t(sGX[cc + HR])) * SR;
#pragma unroll
            for (int f = 0; f < 9; ++f) sto(fy + size_t(4 * f) * fys, off, o[f]);
          }
        }
      }
    }
    if (zc + 1 < z1) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int c = 0; c < NZ; ++c) zr[j][c] = zr[j + 1][c];
#pragma unroll
      for (int c = 0; c < NZ; ++c) zr[4][c] = zn[c];
    }
  }
  block_reduce_store<2>(v2, partial + size_t(blockIdx.x) * 2, pacc != 0);
}

// The z terms of one product (after k_pcb_gather<R, FS, 2> or k_pcb_fused),
// added to q_out, phi_out and ub_out.  One thread per (x, y) column marches
// the planes of a slab of TZ; the 15 fields with a radius-2 z stencil (the
// adjoints of D4_z Q, L4 Q, D4_z phi, L4 phi, W_az: pb's fields, or zf of
// k_pcb_fused, zstride apart) sit in five-plane register rings, the 8 with a
// radius-1 one (V, u_z, phi) in three-plane rings.  After k_pcb_fused (fx or
// fy not null) a column among the first or last two of its TX x TY tile also
// takes the terms the neighbouring tile owes it across the face.
template <class R, class FS, bool FACES>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 2 : 1)))
k_pcb_gather_z(Box b, Params<R> P, int TZ, const FS* __restrict__ phi,
                                                      const R* __restrict__ u, const R* __restrict__ vq,
                                                      const R* __restrict__ vphi, R vs, const R* __restrict__ pb,
                                                      R* __restrict__ q_out, R* __restrict__ phi_out,
                                                      R* __restrict__ ub_out, const R* __restrict__ zf,
                                                      const R* __restrict__ mub, int TX, int TY, int ntx, int nty,
                                                      const R* __restrict__ fx, const R* __restrict__ fy) {
  const int plane = b.nx * b.ny;
  const int ncb = (plane + 255) / 256;
  const int col = (blockIdx.x % ncb) * 256 + threadIdx.x;
  if (col >= plane) return;
  const int z0 = (blockIdx.x / ncb) * TZ, z1 = min(z0 + TZ, b.nz);
  const size_t N = b.N;
  constexpr int N2 = 15, N1 = 8;
  // radius-2 fields: D4_z Q adjoint (5), L4 Q adjoint (5), D4_z phi, L4 phi adjoints, W_az adjoint (3)
  const R* f2[N2];
  if constexpr (FACES) {  // zf: D4_z Q (5), D4_z phi, W_az (3); L4 Q, L4 phi formed from V, mu_bar below
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      f2[k] = zf + size_t(k) * N;
      f2[5 + k] = vq + size_t(k) * N;
    }
    f2[10] = zf + size_t(5) * N;
    f2[11] = mub;
#pragma unroll
    for (int a = 0; a < 3; ++a) f2[12 + a] = zf + size_t(6 + a) * N;
  } else {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      f2[k] = pb + size_t(PB_DQ + 10 + k) * N;
      f2[5 + k] = pb + size_t(PB_LAPQ + k) * N;
    }
    f2[10] = pb + size_t(PB_DPHI + 2) * N;
    f2[11] = pb + size_t(PB_LAPPHI) * N;
#pragma unroll
    for (int a = 0; a < 3; ++a) f2[12 + a] = pb + size_t(PB_W + 3 * a + 2) * N;
  }
  // face terms of this column (k_pcb_fused): up to one source per side and
  // axis, each a (face, side, pos) block of fx or fy
  const int cx = col % b.nx, cy = col / b.nx;
  int xsrc[2] = {-1, -1}, ysrc[2] = {-1, -1};  // ((face 2 + side) 2 + pos)
  if (FACES && ntx > 1) {
    const int j = cx / TX, lx = cx - j * TX, wj = min(TX, b.nx - j * TX);
    if (lx < 2) xsrc[0] = ((((j + ntx - 1) % ntx) * 2 + 0) * 2) + lx;  // sent by tile j - 1 across face j - 1
    if (lx >= wj - 2) xsrc[1] = ((j * 2 + 1) * 2) + (wj - 1 - lx);     // sent by tile j + 1 across face j
  }
  if (FACES && nty > 1) {
    const int i = cy / TY, ly = cy - i * TY, hi = min(TY, b.ny - i * TY);
    if (ly < 2) ysrc[0] = ((((i + nty - 1) % nty) * 2 + 0) * 2) + ly;
    if (ly >= hi - 2) ysrc[1] = ((i * 2 + 1) * 2) + (hi - 1 - ly);
  }
  const size_t fxs = size_t(ntx) * b.nz * b.ny, fys = size_t(nty) * b.nz * b.nx;
  // the owed terms at plane zz: a record of fx, or 9 values of one fy row
  // (sp = side 2 + pos)
  auto xrec = [&](int src, int zz) {
    return fx + (size_t(src & 3) * fxs + (size_t(src >> 2) * b.nz + zz) * b.ny + cy) * kRec;
  };
  auto yrow = [&](int src, int zz) { return fy + size_t(src & 3) * fys + (size_t(src >> 2) * b.nz + zz) * b.nx + cx; };
  // the first x and the first y source of the column are loaded one plane
  // ahead; a second one along an axis (tiles under four sites wide) is
  // loaded where it is added
  const int xa = xsrc[0] >= 0 ? xsrc[0] : xsrc[1], xb = xsrc[0] >= 0 ? xsrc[1] : -1;
  const int ya = ysrc[0] >= 0 ? ysrc[0] : ysrc[1], yb = ysrc[0] >= 0 ? ysrc[1] : -1;
  auto ld_faces = [&](int zz, R px[9], R py[9]) {
    if (xa >= 0) ld_rec(xrec(xa, zz), px);
    if (ya >= 0) {
      const R* r = yrow(ya, zz);
#pragma unroll
      for (int f = 0; f < 9; ++f) py[f] = r[size_t(4 * f) * fys];
    }
  };
  const bool faces = xsrc[0] >= 0 || xsrc[1] >= 0 || ysrc[0] >= 0 || ysrc[1] >= 0;
  auto at = [&](int zz) { return size_t(pmod(zz, b.nz)) * plane + col; };
  // the radius-1 fields (vs V_Q, vs V_phi, u_z, phi); with FACES vs V_Q is
  // formed from the radius-2 ring, which holds V_Q itself
  auto ld1 = [&](int zz, R v[N1]) {
    const size_t k = at(zz);
    if constexpr (!FACES) {
#pragma unroll
      for (int c = 0; c < 5; ++c) v[c] = vs * vq[c * N + k];
    }
    v[5] = vs * vphi[k];
    v[6] = u[2 * N + k];
    v[7] = R(phi[k]);
  };
  R r2[5][N2], r1[3][N1];
  // a plane of the radius-2 ring; with FACES its L4 Q and L4 phi slots hold
  // V_Q and mu_bar, whose adjoints K (Gamma (vs V_Q)) and -(k_phi mu_bar) (as
  // the local reverse forms them) are taken where the stencil reads them
  auto ld2 = [&](size_t k, R v[N2]) {
#pragma unroll
    for (int f = 0; f < N2; ++f) v[f] = f2[f][k];
  };
  auto r2v = [&](int j, int f) {
    if constexpr (FACES) {
      if (f >= 5 && f < 10) return P.K * (P.Gamma * (vs * r2[j][f]));
      if (f == 11) return -(P.k_phi * r2[j][f]);
    }
    return r2[j][f];
  };
  // vs V_Q at planes zc - 1, zc, zc + 1 (j = 0, 1, 2)
  auto vq1 = [&](int j, int c) {
    if constexpr (FACES) return vs * r2[1 + j][5 + c];
    return r1[j][c];
  };
#pragma unroll
  for (int j = 0; j < 4; ++j) ld2(at(z0 - 2 + j), r2[j]);
  ld1(z0 - 1, r1[0]);
  ld1(z0, r1[1]);
  // the loads of a plane are issued one iteration ahead: the ring planes
  // zc + 2 (radius 2) and zc + 1 (radius 1), and the 9 outputs at zc it adds to
  R n2[N2], n1[N1], no[9];
  R nfx[9], nfy[9];  // the face sources of the next plane
  auto ld_out = [&](int zz, R o[9]) {
    const size_t k = size_t(zz) * plane + col;
#pragma unroll
    for (int c = 0; c < 5; ++c) o[c] = q_out[c * N + k];
    o[5] = phi_out[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) o[6 + a] = ub_out[a * N + k];
  };
  if (z0 < z1) {
    ld_out(z0, no);
    ld2(at(z0 + 2), n2);
    ld1(z0 + 1, n1);
    if constexpr (FACES) ld_faces(z0, nfx, nfy);
  }
  for (int zc = z0; zc < z1; ++zc) {
    R o[9];
#pragma unroll
    for (int f = 0; f < N2; ++f) r2[4][f] = n2[f];
#pragma unroll
    for (int f = 0; f < N1; ++f) r1[2][f] = n1[f];
#pragma unroll
    for (int f = 0; f < 9; ++f) o[f] = no[f];
    // the face terms of this plane: the prefetched sources, then any second one
    R ft[9] = {R(0), R(0), R(0), R(0), R(0), R(0), R(0), R(0), R(0)};
    if (FACES && faces) {
      if (xa >= 0) {
#pragma unroll
        for (int f = 0; f < 9; ++f) ft[f] += nfx[f];
      }
      if (ya >= 0) {
#pragma unroll
        for (int f = 0; f < 9; ++f) ft[f] += nfy[f];
      }
      if (xb >= 0) add_rec(xrec(xb, zc), ft);
      if (yb >= 0) {
        const R* r = yrow(yb, zc);
#pragma unroll
        for (int f = 0; f < 9; ++f) ft[f] += r[size_t(4 * f) * fys];
      }
    }
    if (zc + 1 < z1) {
      ld_out(zc + 1, no);
      ld2(at(zc + 3), n2);
      ld1(zc + 2, n1);
      if constexpr (FACES) ld_faces(zc + 1, nfx, nfy);
    }
    auto d4z = [&](int f) { return -d4c(r2[0][f], r2[1][f], r2[3][f], r2[4][f]); };
    auto l4z = [&](int f) { return l4c(r2v(0, f), r2v(1, f), r2v(3, f), r2v(4, f)); };
    const size_t s = size_t(zc) * plane + col;
    // upwind terms of the z neighbours; donor-cell faces z + 1/2 and z - 1/2
    const R uzp = r1[2][6], uzm = r1[0][6], uz = r1[1][6];
    const R upx = uzp > R(0) ? uzp : R(0), umx = uzm < R(0) ? uzm : R(0);
#pragma unroll
    for (int k = 0; k < 5; ++k)
      q_out[k * N + s] = o[k] + (((d4z(k) + l4z(5 + k)) + (vq1(2, k) * upx - vq1(0, k) * umx)) + ft[k]);
    const R fp = R(0.5) * (uz + uzp), fm = R(0.5) * (uzm + uz);
    const R cp = r1[2][5] - r1[1][5], cm = r1[1][5] - r1[0][5];
    const R ph = r1[1][7], php = r1[2][7], phm = r1[0][7];
    phi_out[s] = o[5] + (((d4z(10) + l4z(11)) + (cp * (fp > R(0) ? fp : R(0)) + cm * (fm < R(0) ? fm : R(0)))) + ft[5]);
    const R dfp = (fp >= R(0) ? ph : R(0)) + (fp <= R(0) ? php : R(0));
    const R dfm = (fm >= R(0) ? phm : R(0)) + (fm <= R(0) ? ph : R(0));
    ub_out[s] = o[6] + (d4z(12) + ft[6]);
    ub_out[N + s] = o[7] + (d4z(13) + ft[7]);
    ub_out[2 * N + s] = o[8] + ((d4z(14) + R(0.5) * (cp * dfp + cm * dfm)) + ft[8]);
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
