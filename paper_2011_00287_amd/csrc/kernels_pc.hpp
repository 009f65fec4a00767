// The paper's integrator of the order parameters (Sec. 3): predictor-corrector
// time stepping (Heun), first-order upwind advection and fourth-order
// accurate stencils for the space derivatives of Eqs. (1)-(2).
//
// With R the right-hand side of Eqs. (1)-(2) at the fixed LB velocity u of
// time t (with F/2), one update is
//   X* = X + R(X),   X(t+1) = X + R(X)/2 + R(X*)/2,      X = (Q, phi).
// R uses
//   D4 f  = [8 (f(x+1) - f(x-1)) - (f(x+2) - f(x-2))] / 12          (radius 2)
//   L4 f  = sum_g [16 (f(x+e) + f(x-e)) - (f(x+2e) + f(x-2e))] / 12 - 7.5 f
// in mu (L4 phi, D4 of v = Q D4 phi), in H (L4 Q, the curl and D4 phi), in
// W_ab = D4_b u_a and in L4 mu; the advection of Q is upwind, u_g times the
// one-sided difference on the side the flow comes from; that of phi is the
// donor-cell flux form with face velocity (u(x) + u(x+e))/2, so sum phi is
// conserved exactly.
//
// Each stage is mu, then the stage update: two z-marching launches
// (k_pc_mu_z, k_pc_stage_z), or three site-parallel ones (k_pc_v, k_pc_mu,
// k_pc_predict / k_pc_correct).  The predictor writes X*; the corrector reads
// X* (stencils) and X (own site) and writes X(t+1) = ((X + X*) + R(X*))/2.
#pragma once
#include "physics.hpp"
#include "storage.hpp"

namespace lbc {

template <class R>
__device__ __forceinline__ R d4c(R m2, R m1, R p1, R p2) {
  return (R(8) * (p1 - m1) - (p2 - m2)) * R(1.0 / 12.0);
}
// one axis of L4 without the centre term; the 3-axis sum takes -7.5 f
template <class R>
__device__ __forceinline__ R l4c(R m2, R m1, R p1, R p2) {
  return (R(16) * (p1 + m1) - (p2 + m2)) * R(1.0 / 12.0);
}

// site indices of x +- e_g, x +- 2 e_g: n[g][0..3] = (-2, -1, +1, +2)
__device__ __forceinline__ void star2(const Box& b, int x, int y, int z, int n[3][4]) {
  const int d[4] = {-2, -1, 1, 2};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    n[0][k] = sidx(b, x + d[k], y, z);
    n[1][k] = sidx(b, x, y + d[k], z);
    n[2][k] = sidx(b, x, y, z + d[k]);
  }
}

// v_a = Q_ab D4_b phi
template <class R, class FS>
__global__ void __launch_bounds__(256) k_pc_v(Box b, const FS* __restrict__ phi, const FS* __restrict__ q,
                                              R* __restrict__ v) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  int n[3][4];
  star2(b, x, y, z, n);
  R dp[3];
#pragma unroll
  for (int g = 0; g < 3; ++g)
    dp[g] = d4c(R(phi[n[g][0]]), R(phi[n[g][1]]), R(phi[n[g][2]]), R(phi[n[g][3]]));
  const R xx = R(q[s]), xy = R(q[N + s]), xz = R(q[2 * N + s]), yy = R(q[3 * N + s]), yz = R(q[4 * N + s]);
  const R zz = -xx - yy;
  v[s] = xx * dp[0] + xy * dp[1] + xz * dp[2];
  v[N + s] = xy * dp[0] + yy * dp[1] + yz * dp[2];
  v[2 * N + s] = xz * dp[0] + yz * dp[1] + zz * dp[2];
}

// mu = local part - k_phi L4 phi - 2 W sum_a D4_a v_a
template <class R, class FS>
__global__ void __launch_bounds__(256) k_pc_mu(Box b, Params<R> P, const FS* __restrict__ phi,
                                               const FS* __restrict__ q, const R* __restrict__ v,
                                               R* __restrict__ mu) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  int n[3][4];
  star2(b, x, y, z, n);
  const R ph = R(phi[s]);
  R lap = R(-7.5) * ph, divv = R(0);
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    lap += l4c(R(phi[n[g][0]]), R(phi[n[g][1]]), R(phi[n[g][2]]), R(phi[n[g][3]]));
    const R* va = v + size_t(g) * N;
    divv += d4c(va[n[g][0]], va[n[g][1]], va[n[g][2]], va[n[g][3]]);
  }
  R qs[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) qs[k] = R(q[k * N + s]);
  mu[s] = mu_site(P, ph, lap, divv, qs);
}

// R(X) at site s: rq[5] = -upwind(u, Q) + S(D4 u, Q) + Gamma H4, rphi = -div_donor(u phi) + M L4 mu
template <class R, class FS>
__device__ __forceinline__ void pc_rhs(const Box& b, const Params<R>& P, const FS* __restrict__ phi,
                                       const FS* __restrict__ q, const R* __restrict__ u,
                                       const R* __restrict__ mu, int s, int x, int y, int z, R rq[5], R& rphi) {
  const size_t N = b.N;
  int n[3][4];
  star2(b, x, y, z, n);
  Grad<R> G;
  G.phi = R(phi[s]);
  G.lapphi = R(0);
  G.divv = R(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    G.q[k] = R(q[k * N + s]);
    G.lapq[k] = R(-7.5) * G.q[k];
  }
  R uc[3], W[3][3], adv[5] = {R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
  for (int a = 0; a < 3; ++a) uc[a] = u[a * N + s];
  R lapmu = R(-7.5) * mu[s], div = R(0);
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const int m2 = n[g][0], m1 = n[g][1], p1 = n[g][2], p2 = n[g][3];
    const R fm1 = R(phi[m1]), fp1 = R(phi[p1]);
    G.dphi[g] = d4c(R(phi[m2]), fm1, fp1, R(phi[p2]));
    const R ug = uc[g];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const FS* qk = q + size_t(k) * N;
      const R qm1 = R(qk[m1]), qp1 = R(qk[p1]), qm2 = R(qk[m2]), qp2 = R(qk[p2]);
      G.dq[g][k] = d4c(qm2, qm1, qp1, qp2);
      G.lapq[k] += l4c(qm2, qm1, qp1, qp2);
      adv[k] += ug > R(0) ? ug * (G.q[k] - qm1) : ug * (qp1 - G.q[k]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const R* ua = u + size_t(a) * N;
      W[a][g] = d4c(ua[m2], ua[m1], ua[p1], ua[p2]);
    }
    // donor-cell fluxes through the faces x + e_g/2 and x - e_g/2
    const R* ugp = u + size_t(g) * N;
    const R fp = R(0.5) * (ug + ugp[p1]);
    const R fm = R(0.5) * (ugp[m1] + ug);
    const R flux_p = fp > R(0) ? fp * G.phi : fp * fp1;
    const R flux_m = fm > R(0) ? fm * fm1 : fm * G.phi;
    div += flux_p - flux_m;
    lapmu += l4c(mu[m2], mu[m1], mu[p1], mu[p2]);
  }
  R h[5], S[5];
  h_site(P, G, h);
  corotation_site(P.xi, G.q, W, S);
#pragma unroll
  for (int k = 0; k < 5; ++k) rq[k] = (-adv[k] + S[k]) + P.Gamma * h[k];
  rphi = -div + P.M * lapmu;
}

// Predictor: X* = X + R(X).
template <class R, class FS>
__global__ void __launch_bounds__(256) k_pc_predict(Box b, Params<R> P, const FS* __restrict__ phi,
                                                    const FS* __restrict__ q, const R* __restrict__ u,
                                                    const R* __restrict__ mu, FS* __restrict__ phi_s,
                                                    FS* __restrict__ q_s) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  R rq[5], rphi;
  pc_rhs(b, P, phi, q, u, mu, s, x, y, z, rq, rphi);
#pragma unroll
  for (int k = 0; k < 5; ++k) q_s[k * N + s] = FS(R(q[k * N + s]) + rq[k]);
  phi_s[s] = FS(R(phi[s]) + rphi);
}

// Corrector: X(t+1) = X + R(X)/2 + R(X*)/2 = ((X + X*) + R(X*))/2.
template <class R, class FS>
__global__ void __launch_bounds__(256) k_pc_correct(Box b, Params<R> P, const FS* __restrict__ phi_s,
                                                    const FS* __restrict__ q_s, const R* __restrict__ u,
                                                    const R* __restrict__ mu, const FS* __restrict__ phi_x,
                                                    const FS* __restrict__ q_x, FS* __restrict__ phi_o,
                                                    FS* __restrict__ q_o) {
  const int s = site_xcd();
  if (s >= b.N) return;
  int x, y, z;
  coords(b, s, x, y, z);
  const size_t N = b.N;
  R rq[5], rphi;
  pc_rhs(b, P, phi_s, q_s, u, mu, s, x, y, z, rq, rphi);
#pragma unroll
  for (int k = 0; k < 5; ++k)
    q_o[k * N + s] = FS(R(0.5) * ((R(q_x[k * N + s]) + R(q_s[k * N + s])) + rq[k]));
  phi_o[s] = FS(R(0.5) * ((R(phi_x[s]) + R(phi_s[s])) + rphi));
}

// ---------------------------------------------------------------------------
// z-marching stage kernel: the predictor (PRED) or the corrector on a TX x TY
// tile and a slab of TZ planes.  Per plane, the 10 fields the right-hand side
// reads (Q, phi, u, mu) sit in LDS with an in-plane cross-shaped halo of 2
// (one halo slot per thread, loaded one plane ahead); the z neighbours at
// +-1, +-2 of the owned column stay in registers, and (float) the column at
// +3 is loaded at the start of the plane so that its latency hides behind it.
// ---------------------------------------------------------------------------
template <class R, class FS, int TX, int TY, int MINW, bool PRED>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(MINW)))
k_pc_stage_z(Box b, Params<R> P, int TZ, int ntx, int nty, const FS* __restrict__ phi, const FS* __restrict__ q,
             const R* __restrict__ u, const R* __restrict__ mu, const FS* __restrict__ phi_x,
             const FS* __restrict__ q_x, FS* __restrict__ phi_out, FS* __restrict__ q_out) {
  constexpr int NT = TX * TY;
  constexpr int HR = 2;
  constexpr int SX = TX + 2 * HR, SY = TY + 2 * HR, NS = SX * SY;
  constexpr int NH = 2 * HR * (TX + TY);  // halo slots the axis stencils read (no corners)
  static_assert(NH <= NT, "one halo slot per thread");
  constexpr int NV = 10;  // q[5], phi, u[3], mu
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

  for (int k = tid; k < SX; k += NT) sGX[k] = pmod(x0 - HR + k, b.nx);
  for (int k = tid; k < SY; k += NT) sGY[k] = pmod(y0 - HR + k, b.ny);
  __syncthreads();
  const int col = sGY[ly + HR] * b.nx + sGX[lx + HR];

  auto load_at = [&](size_t k, R v[NV]) {
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = R(q[c * N + k]);
    v[5] = R(phi[k]);
#pragma unroll
    for (int a = 0; a < 3; ++a) v[6 + a] = u[a * N + k];
    v[9] = mu[k];
  };
  auto load_col = [&](int zz, R v[NV]) { load_at(size_t(pmod(zz, b.nz)) * plane + col, v); };
  // column registers: planes zc-2 .. zc+2
  R cm2[NV], cm1[NV], c0[NV], cp1[NV], cp2[NV];
  load_col(z0 - 2, cm2);
  load_col(z0 - 1, cm1);
  load_col(z0, c0);
  load_col(z0 + 1, cp1);
  load_col(z0 + 2, cp2);

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
  R hv[NV];
  if (has_halo) load_at(size_t(z0) * plane + hcol, hv);

  const int sc = (ly + HR) * SX + (lx + HR);
  // float: the column at zc+3 is in flight during the plane; double has no
  // registers to spare and loads it after the plane
  constexpr bool kStaged = sizeof(R) == 4;
  R cn[kStaged ? NV : 1];
  for (int zc = z0; zc < z1; ++zc) {
    __syncthreads();  // previous plane's reads are done
    if constexpr (kStaged) {
      if (zc + 1 < z1) load_col(zc + 3, cn);
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) sV[c][sc] = c0[c];
    if (has_halo) {
#pragma unroll
      for (int c = 0; c < NV; ++c) sV[c][hs] = hv[c];
      if (zc + 1 < z1) load_at(size_t(zc + 1) * plane + hcol, hv);  // next plane's halo
    }
    __syncthreads();
    if (active) {
      // neighbours of field f: x and y from LDS, z from the column registers
      auto nb = [&](int f, int g, R& m2, R& m1, R& p1, R& p2) {
        if (g == 0) {
          m2 = sV[f][sc - 2]; m1 = sV[f][sc - 1]; p1 = sV[f][sc + 1]; p2 = sV[f][sc + 2];
        } else if (g == 1) {
          m2 = sV[f][sc - 2 * SX]; m1 = sV[f][sc - SX]; p1 = sV[f][sc + SX]; p2 = sV[f][sc + 2 * SX];
        } else {
          m2 = cm2[f]; m1 = cm1[f]; p1 = cp1[f]; p2 = cp2[f];
        }
      };
      Grad<R> G;
      G.phi = c0[5];
      G.lapphi = R(0);
      G.divv = R(0);
      R adv[5] = {R(0), R(0), R(0), R(0), R(0)}, W[3][3];
      R lapmu = R(-7.5) * c0[9], div = R(0);
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        G.q[k] = c0[k];
        G.lapq[k] = R(-7.5) * c0[k];
      }
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        R m2, m1, p1, p2;
        nb(5, g, m2, m1, p1, p2);
        G.dphi[g] = d4c(m2, m1, p1, p2);
        const R fm1 = m1, fp1 = p1;
        const R ug = c0[6 + g];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          nb(k, g, m2, m1, p1, p2);
          G.dq[g][k] = d4c(m2, m1, p1, p2);
          G.lapq[k] += l4c(m2, m1, p1, p2);
          adv[k] += ug > R(0) ? ug * (c0[k] - m1) : ug * (p1 - c0[k]);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          nb(6 + a, g, m2, m1, p1, p2);
          W[a][g] = d4c(m2, m1, p1, p2);
          if (a == g) {  // donor-cell fluxes through the faces x +- e_g/2
            const R fp = R(0.5) * (ug + p1);
            const R fm = R(0.5) * (m1 + ug);
            const R flux_p = fp > R(0) ? fp * G.phi : fp * fp1;
            const R flux_m = fm > R(0) ? fm * fm1 : fm * G.phi;
            div += flux_p - flux_m;
          }
        }
        nb(9, g, m2, m1, p1, p2);
        lapmu += l4c(m2, m1, p1, p2);
      }
      R h[5], S[5];
      h_site(P, G, h);
      corotation_site(P.xi, G.q, W, S);
      const R rphi = -div + P.M * lapmu;
      const size_t site = size_t(zc) * plane + col;
      if constexpr (PRED) {
#pragma unroll
        for (int k = 0; k < 5; ++k) q_out[k * N + site] = FS(c0[k] + ((-adv[k] + S[k]) + P.Gamma * h[k]));
        phi_out[site] = FS(c0[5] + rphi);
      } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const R rk = (-adv[k] + S[k]) + P.Gamma * h[k];
          q_out[k * N + site] = FS(R(0.5) * ((R(q_x[k * N + site]) + c0[k]) + rk));
        }
        phi_out[site] = FS(R(0.5) * ((R(phi_x[site]) + c0[5]) + rphi));
      }
    }
    if (zc + 1 < z1) {
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        cm2[c] = cm1[c];
        cm1[c] = c0[c];
        c0[c] = cp1[c];
        cp1[c] = cp2[c];
        if constexpr (kStaged) cp2[c] = cn[c];
      }
      if constexpr (!kStaged) load_col(zc + 3, cp2);
    }
  }
}

// ---------------------------------------------------------------------------
// z-marching mu: the anchoring vector v = Q D4 phi and mu of one stage in one
// pass (the site-parallel pair k_pc_v + k_pc_mu writes and re-reads v).
// March step p computes v at plane p on the tile and its cross-shaped halo of
// 2, then mu at plane p-2, whose z stencils reach v_z and phi at p-4 .. p.
//   LDS: phi planes on the tile with halo 4 (v at a halo slot takes D4 phi
//        around it), a ring of 8 plane slots of which p-2 .. p+2 are live;
//        v_x, v_y on the cross, a ring of 4 of which p-2 .. p are live.  The
//        slot a step writes was last read two steps earlier, so one barrier
//        per half-step suffices;
//   registers: the owned column's phi and v_z at p-4 .. p, Q at p-2 .. p.
// ---------------------------------------------------------------------------
template <class R, class FS, int TX, int TY, int MINW>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(MINW)))
k_pc_mu_z(Box b, Params<R> P, int TZ, int ntx, int nty, const FS* __restrict__ phi, const FS* __restrict__ q,
          R* __restrict__ mu) {
  constexpr int NT = TX * TY;
  constexpr int HP = 4, HV = 2, OFF = HP - HV;
  constexpr int PX = TX + 2 * HP, PY = TY + 2 * HP, NP = PX * PY;  // phi frame
  constexpr int KP = (NP + NT - 1) / NT;                           // phi plane loads per thread
  constexpr int NPP = KP * NT;                                     // padded frame (no load guards)
  constexpr int VX = TX + 2 * HV, VY = TY + 2 * HV, NV = VX * VY;  // v frame
  constexpr int NH = 2 * HV * (TX + TY);                           // v halo slots (no corners)
  static_assert(NH <= NT, "one v halo slot per thread");
  __shared__ R sPhi[8][NPP];
  __shared__ R sVx[4][NV], sVy[4][NV];
  __shared__ int sGX[PX], sGY[PY];

  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = l % ntx, ty = (l / ntx) % nty, sl = l / (ntx * nty);
  const int x0 = tx * TX, y0 = ty * TY, z0 = sl * TZ;
  const int z1 = min(z0 + TZ, b.nz);
  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = tid / TX;
  const bool active = (x0 + lx < b.nx) && (y0 + ly < b.ny);
  const size_t N = b.N;
  const int plane = b.nx * b.ny;

  for (int k = tid; k < PX; k += NT) sGX[k] = pmod(x0 - HP + k, b.nx);
  for (int k = tid; k < PY; k += NT) sGY[k] = pmod(y0 - HP + k, b.ny);
  __syncthreads();

  // phi-plane slots this thread loads (padding slots load the frame origin)
  int pcol[KP];
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const int k = tid + j * NT;
    pcol[j] = k < NP ? sGY[k / PX] * b.nx + sGX[k % PX] : sGY[0] * b.nx + sGX[0];
  }
  // plane offsets advance by one plane per step, wrapping at the box
  auto next_plane = [&](int off) { return off + plane == int(N) ? 0 : off + plane; };
  auto load_phi_plane = [&](int off, R v[KP]) {
#pragma unroll
    for (int j = 0; j < KP; ++j) v[j] = R(phi[size_t(off) + pcol[j]]);
  };
  auto store_phi_plane = [&](int w, const R v[KP]) {
#pragma unroll
    for (int j = 0; j < KP; ++j) sPhi[w & 7][tid + j * NT] = v[j];
  };

  // v slots: the owned site, and (tid < NH) one halo slot of the cross
  const int ovx = lx + HV, ovy = ly + HV;
  int hvx = 0, hvy = 0;
  const bool has_halo = tid < NH;
  if (has_halo) {
    if (tid < 2 * HV * TX) {
      const int r = tid / TX;
      hvx = HV + tid % TX;
      hvy = r < HV ? r : TY + r;
    } else {
      const int t = tid - 2 * HV * TX;
      const int c = t / TY;
      hvy = HV + t % TY;
      hvx = c < HV ? c : TX + c;
    }
  }
  const int ocol = sGY[ovy + OFF] * b.nx + sGX[ovx + OFF];
  const int hcol = sGY[hvy + OFF] * b.nx + sGX[hvx + OFF];
  auto load_q = [&](int off, int colx, R v[5]) {
    const size_t k = size_t(off) + colx;
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = R(q[c * N + k]);
  };
  // v at v-frame slot (vx, vy) of plane w, from the phi ring and Q there
  auto v_at = [&](int w, int vx, int vy, const R qv[5], R v[3]) {
    const int f = (vy + OFF) * PX + (vx + OFF);
    const R* p0 = sPhi[w & 7];
    R d[3];
    d[0] = d4c(p0[f - 2], p0[f - 1], p0[f + 1], p0[f + 2]);
    d[1] = d4c(p0[f - 2 * PX], p0[f - PX], p0[f + PX], p0[f + 2 * PX]);
    d[2] = d4c(sPhi[(w - 2) & 7][f], sPhi[(w - 1) & 7][f], sPhi[(w + 1) & 7][f], sPhi[(w + 2) & 7][f]);
    const R xx = qv[0], xy = qv[1], xz = qv[2], yy = qv[3], yz = qv[4], zz = -xx - yy;
    v[0] = xx * d[0] + xy * d[1] + xz * d[2];
    v[1] = xy * d[0] + yy * d[1] + yz * d[2];
    v[2] = xz * d[0] + yz * d[1] + zz * d[2];
  };

  // ring slots are indexed by (plane - z0 + 8) & 7 through w = p - z0 + 8 >= 4
  const int wb = 8 - z0;
  // planes z0-4 .. z0-1 into the ring; plane z0 and Q of plane z0-2 prefetched
  int off_phi = pmod(z0 - 4, b.nz) * plane;  // offset of the next phi plane to load
  {
    R t[KP];
    for (int w = z0 - 4; w < z0; ++w) {
      load_phi_plane(off_phi, t);
      store_phi_plane(w + wb, t);
      off_phi = next_plane(off_phi);
    }
  }
  R pf[KP], qo_n[5], qh_n[5] = {R(0), R(0), R(0), R(0), R(0)};
  load_phi_plane(off_phi, pf);
  off_phi = next_plane(off_phi);
  int off_q = pmod(z0 - 2, b.nz) * plane;  // offset of the Q plane of the next v step
  load_q(off_q, ocol, qo_n);
  if (has_halo) load_q(off_q, hcol, qh_n);
  off_q = next_plane(off_q);
  R phc[5] = {R(0), R(0), R(0), R(0), R(0)};  // owned phi at p-4 .. p
  R vzc[5] = {R(0), R(0), R(0), R(0), R(0)};  // owned v_z at p-4 .. p
  R qc[3][5];                                  // owned Q at p-2 .. p
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int c = 0; c < 5; ++c) qc[j][c] = R(0);

  const int ov = ovy * VX + ovx, hv = hvy * VX + hvx;
  const int op = (ovy + OFF) * PX + (ovx + OFF);
  int off_mu = z0 * plane + ocol;  // output site of plane p-2 once p-2 >= z0
  R qo_f[5], qh_f[5];              // Q of plane p+1, in flight during the step
  for (int p = z0 - 2; p < z1 + 2; ++p) {
    const int w = p + wb;
    store_phi_plane(w + 2, pf);
    const bool more = p + 1 < z1 + 2;
    if (more) {  // prefetch: phi plane p+3, Q of plane p+1
      load_phi_plane(off_phi, pf);
      off_phi = next_plane(off_phi);
      load_q(off_q, ocol, qo_f);
      if (has_halo) load_q(off_q, hcol, qh_f);
      off_q = next_plane(off_q);
    }
    __syncthreads();  // phi plane p+2 is in place
    // v at plane p: owned slot and halo slot
    R v[3];
    v_at(w, ovx, ovy, qo_n, v);
    sVx[w & 3][ov] = v[0];
    sVy[w & 3][ov] = v[1];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      vzc[j] = vzc[j + 1];
      phc[j] = phc[j + 1];
    }
    vzc[4] = v[2];
    phc[4] = sPhi[w & 7][op];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      qc[0][c] = qc[1][c];
      qc[1][c] = qc[2][c];
      qc[2][c] = qo_n[c];
    }
    if (has_halo) {
      R vh[3];
      v_at(w, hvx, hvy, qh_n, vh);
      sVx[w & 3][hv] = vh[0];
      sVy[w & 3][hv] = vh[1];
    }
    __syncthreads();  // v of plane p is in place
    if (p - 2 >= z0) {
      if (active) {
        const R* pl = sPhi[(w - 2) & 7];
        const R* vx = sVx[(w - 2) & 3];
        const R* vy = sVy[(w - 2) & 3];
        const R ph = phc[2];
        const R lap = (R(-7.5) * ph + l4c(pl[op - 2], pl[op - 1], pl[op + 1], pl[op + 2])) +
                      l4c(pl[op - 2 * PX], pl[op - PX], pl[op + PX], pl[op + 2 * PX]) +
                      l4c(phc[0], phc[1], phc[3], phc[4]);
        const R divv = d4c(vx[ov - 2], vx[ov - 1], vx[ov + 1], vx[ov + 2]) +
                       d4c(vy[ov - 2 * VX], vy[ov - VX], vy[ov + VX], vy[ov + 2 * VX]) +
                       d4c(vzc[0], vzc[1], vzc[3], vzc[4]);
        mu[off_mu] = mu_site(P, ph, lap, divv, qc[0]);
      }
      off_mu += plane;
    }
    if (more) {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        qo_n[c] = qo_f[c];
        qh_n[c] = has_halo ? qh_f[c] : R(0);
      }
    }
  }
}

}  // namespace lbc
