// Fused kernels of the coupled step: two launches per step.
//
// k_lb_fused  : stress, force, pull-stream and Guo-forced BGK collision
//               (Eqs. (3)-(4), (6)-(8), (10)-(11)) plus mu (Eq. (1), with the
//               anchoring vector v = Q D0 phi taken from the stress pass); on
//               D3Q15 the symmetric stress enters the equilibrium (Eq. (9))
//               and the force is that of the antisymmetric stress;
//               writes the post-collision populations (unless Bout is null),
//               u and mu (and the force F and the density deviation when a
//               recording step asks for them).
// k_order_fused: molecular field H (Eq. (5)), Beris-Edwards update of Q
//               (Eq. (2)) and Cahn-Hilliard update of phi (Eq. (1)).
//
// Both march along z over a slab of planes.  A workgroup owns a TX x TY tile
// of the x-y plane; thread (lx, ly) owns one column of it.  Stencil inputs
// are staged in LDS plane rings with a halo, so every neighbour read is an
// LDS access at a compile-time offset.  Values a thread needs only along its
// own column (the z-components of the stress, the in-plane force part, the
// z-neighbours of u, mu, Q, phi) stay in registers.
//
// Workgroup ids are remapped so that each XCD (8 on MI355X, ids dealt
// round-robin) receives a contiguous range of tiles, keeping the halos a
// tile shares with its neighbours in the same L2.
#pragma once
#include "physics.hpp"
#include "storage.hpp"

namespace lbc {

// ---------------------------------------------------------------------------
// k_lb_fused
//   Iteration p of the march: phi and Q rings hold planes p-2..p+2 (phi) and
//   p-1..p+1 (Q) on the tile plus a halo of 2.  The stress is computed at
//   plane p on the tile plus the halo of 1 the force reads (each thread its
//   own site, then the halo slots on rotating waves).  Thread t owns column t
//   of the tile for mu and for the collision of plane p-1, whose force needs
//   the stress of planes p-2..p.  The global loads needed after the stress
//   pass (the pull of plane p-1, the ring planes for p+1) are issued before
//   it so that their latency overlaps the stress arithmetic.
//   A recording step also passes the step counters of its input and output
//   states (step_in, step_out; null otherwise): one thread writes
//   *step_out = *step_in + 1, which spares a launch per recorded step.
// ---------------------------------------------------------------------------
template <class R, class GS, class FS, class L, int TX, int TY, int MINW>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(MINW)))
k_lb_fused(Box b, Params<R> P, int TZ, int ntx, int nty, const GS* __restrict__ Bin, GS* __restrict__ Bout,
           const FS* __restrict__ phi, const FS* __restrict__ q, R* __restrict__ u_out, R* __restrict__ mu_out,
           R* __restrict__ F_out, R* __restrict__ drho_out, const int64_t* __restrict__ step_in,
           int64_t* __restrict__ step_out) {
  constexpr int NT = TX * TY;
  if (step_out != nullptr && blockIdx.x == 0 && threadIdx.x == 0) step_out[0] = step_in[0] + 1;
  constexpr int AX = TX + 4, AY = TY + 4, NA = AX * AY;  // phi / Q slots (halo 2)
  constexpr int SX = TX + 2, SY = TY + 2, NS = SX * SY;  // stress slots (halo 1)
  __shared__ R sPhi[5][NA];
  __shared__ R sQ[3][5][NA];
  constexpr int NHALO = 2 * (TX + TY);                  // halo stress slots the force reads
  static_assert(NHALO <= NT && NT % 64 == 0, "one halo slot per thread, whole waves");
  __shared__ R sSig[6][NS];  // sigma_ax (a = 0..2), then sigma_ay
  __shared__ R sV[2][2][NS];  // anchoring vector v_x, v_y of the stress slots, planes by parity
  __shared__ int sGX[AX], sGY[AY];

  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = l % ntx, ty = (l / ntx) % nty, sl = l / (ntx * nty);
  const int x0 = tx * TX, y0 = ty * TY, z0 = sl * TZ;
  const int z1 = min(z0 + TZ, b.nz);
  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = tid / TX;
  const int x = x0 + lx, y = y0 + ly;
  const bool active = (x < b.nx) && (y < b.ny);
  const size_t N = b.N;
  const int plane = b.nx * b.ny;

  for (int k = tid; k < AX; k += NT) sGX[k] = pmod(x0 - 2 + k, b.nx);
  for (int k = tid; k < AY; k += NT) sGY[k] = pmod(y0 - 2 + k, b.ny);
  __syncthreads();

  // ring slots this thread refills each plane (fixed over the march)
  constexpr int KR = (NA + NT - 1) / NT;
  int rslot[KR];
  uint32_t rcol[KR];  // byte offset of the slot's column within a plane (FS)
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    const int k = tid + j * NT;
    rslot[j] = k < NA ? k : -1;
    rcol[j] = k < NA ? uint32_t(sGY[k / AX] * b.nx + sGX[k % AX]) * uint32_t(sizeof(FS)) : 0u;
  }
  const uint32_t plane_fs = uint32_t(plane) * uint32_t(sizeof(FS));
  auto fill = [&](int p, bool do_phi, bool do_q) {
    const uint32_t bz = uint32_t(pmod(p, b.nz)) * plane_fs;
    const int sph = pmod(p, 5), sq = pmod(p, 3);
#pragma unroll
    for (int j = 0; j < KR; ++j) {
      if (rslot[j] >= 0) {
        if (do_phi) sPhi[sph][rslot[j]] = R(ldo(phi, bz + rcol[j]));
        if (do_q) {
#pragma unroll
          for (int c = 0; c < 5; ++c) sQ[sq][c][rslot[j]] = R(ldo(q + size_t(c) * N, bz + rcol[j]));
        }
      }
    }
  };
  // prefill for the first stress plane p = z0 - 1: phi z0-3..z0+1, Q z0-2..z0
  fill(z0 - 3, true, false);
  for (int p = z0 - 2; p <= z0; ++p) fill(p, true, true);
  fill(z0 + 1, true, false);

  // column registers: sigma_az at planes p-2, p-1 and the in-plane force part at p-1
  R saz_m2[3] = {R(0), R(0), R(0)}, saz_m1[3] = {R(0), R(0), R(0)}, fin_m1[3] = {R(0), R(0), R(0)};
  R vz_m2 = R(0), vz_m1 = R(0);  // v_z of the owned column at planes p-2, p-1
  // stress in the equilibrium (D3Q15): symmetric stress of the owned site at plane p-1
  R ssym_m1[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};

  // pull offsets of the owned column: in-plane byte offsets of the 9 (x, y) neighbours
  const int xw = active ? x : 0, yw = active ? y : 0;
  const int xs[3] = {wrapi(xw - 1, b.nx), xw, wrapi(xw + 1, b.nx)};
  const int ys[3] = {wrapi(yw - 1, b.ny), yw, wrapi(yw + 1, b.ny)};
  uint32_t colb[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int i = 0; i < 3; ++i) colb[j][i] = uint32_t(ys[j] * b.nx + xs[i]) * uint32_t(sizeof(GS));
  const uint32_t plane_gs = uint32_t(plane) * uint32_t(sizeof(GS));
  const uint32_t own_r = uint32_t(yw * b.nx + xw) * uint32_t(sizeof(R));
  const uint32_t own_g = uint32_t(yw * b.nx + xw) * uint32_t(sizeof(GS));
  const uint32_t plane_r = uint32_t(plane) * uint32_t(sizeof(R));

  // loop-carried ring slots and wrapped plane indices (uniform)
  int r0 = pmod(z0 - 1, 5), c0 = pmod(z0 - 1, 3);
  int zph = pmod(z0 + 2, b.nz), zq = pmod(z0 + 1, b.nz);
  int zc_m = pmod(z0 - 3, b.nz), zc_0 = pmod(z0 - 2, b.nz), zc_p = pmod(z0 - 1, b.nz);
  for (int p = z0 - 1; p <= z1; ++p) {
    __syncthreads();  // rings for plane p are complete; last plane's stress reads are done
    const int rm = r0 == 0 ? 4 : r0 - 1, rp = r0 == 4 ? 0 : r0 + 1;
    const int rm2 = rm == 0 ? 4 : rm - 1;
    const int cm = c0 == 0 ? 2 : c0 - 1, cp = c0 == 2 ? 0 : c0 + 1;
    const int zc = p - 1;
    const bool collide = active && zc >= z0 && zc < z1;

    // ---- issue the global loads needed after the stress pass
    R g[L::Q];
    if (collide) {
      const uint32_t zb[3] = {uint32_t(zc_m) * plane_gs, uint32_t(zc_0) * plane_gs, uint32_t(zc_p) * plane_gs};
#pragma unroll
      for (int i = 0; i < L::Q; ++i)
        g[i] = GPolO<GS, L>::template ld<R>(Bin + size_t(i) * N, zb[1 - L::cz(i)] + colb[1 - L::cy(i)][1 - L::cx(i)], i);
    }
    const bool refill = p < z1;
    R nphi[KR], nq[KR][5];
    if (refill) {
      const uint32_t bph = uint32_t(zph) * plane_fs, bq = uint32_t(zq) * plane_fs;
#pragma unroll
      for (int j = 0; j < KR; ++j) {
        if (rslot[j] >= 0) {
          nphi[j] = R(ldo(phi, bph + rcol[j]));
#pragma unroll
          for (int c = 0; c < 5; ++c) nq[j][c] = R(ldo(q + size_t(c) * N, bq + rcol[j]));
        }
      }
    }

    // ---- stress at plane p: round 0 is the owned site (its sigma_az stays in
    // registers), round 1 the halo slots the in-plane force reads (rows
    // y0-1, y0+TY and columns x0-1, x0+TX; corners are not needed).  The halo
    // slots go to whole waves, starting at a wave that rotates with the plane
    // and the workgroup, so the extra round is spread over the SIMDs.
    R saz[3], vz = R(0);
    R ss[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};  // symmetric stress of the owned site (D3Q15)
    const int vbuf = p & 1;
    {
      constexpr int NW = NT / 64 > 0 ? NT / 64 : 1;
      const int shift = ((p + 1 + l) % NW) * 64;
      const int hslot = tid >= shift ? tid - shift : tid - shift + NT;
#pragma unroll 1
      for (int r = 0; r < 2; ++r) {
        int sx, sy;
        if (r == 0) {
          sx = lx + 1;
          sy = ly + 1;
        } else {
          if (hslot >= NHALO) break;
          if (hslot < 2 * TX) {
            sx = 1 + (hslot % TX);
            sy = hslot < TX ? 0 : SY - 1;
          } else {
            const int h2 = hslot - 2 * TX;
            sx = h2 < TY ? 0 : SX - 1;
            sy = 1 + (h2 % TY);
          }
        }
        const int s = sy * SX + sx;
        const int a0 = (sy + 1) * AX + (sx + 1);  // phi / Q slot of this stress slot
        Grad<R> G;
        G.phi = sPhi[r0][a0];
        G.dphi[0] = R(0.5) * (sPhi[r0][a0 + 1] - sPhi[r0][a0 - 1]);
        G.dphi[1] = R(0.5) * (sPhi[r0][a0 + AX] - sPhi[r0][a0 - AX]);
        G.dphi[2] = R(0.5) * (sPhi[rp][a0] - sPhi[rm][a0]);
        G.lapphi = R(0);
        G.divv = R(0);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          const R qc = sQ[c0][c][a0];
          const R qxp = sQ[c0][c][a0 + 1], qxm = sQ[c0][c][a0 - 1];
          const R qyp = sQ[c0][c][a0 + AX], qym = sQ[c0][c][a0 - AX];
          const R qzp = sQ[cp][c][a0], qzm = sQ[cm][c][a0];
          G.q[c] = qc;
          G.dq[0][c] = R(0.5) * (qxp - qxm);
          G.dq[1][c] = R(0.5) * (qyp - qym);
          G.dq[2][c] = R(0.5) * (qzp - qzm);
          G.lapq[c] = ((qxp + qxm) + (qyp + qym) + (qzp + qzm)) - R(6) * qc;
        }
        R h[5], sig[9], vq[3];
        sigma_site(P, G, sig, h, vq);
        if constexpr (L::kStressInEq) {
          // the symmetric part goes to the equilibrium, the force stencil sees
          // only the antisymmetric part A_ab = (sigma_ab - sigma_ba)/2
          if (r == 0) {
            ss[0] = sig[0];
            ss[1] = R(0.5) * (sig[1] + sig[3]);
            ss[2] = R(0.5) * (sig[2] + sig[6]);
            ss[3] = sig[4];
            ss[4] = R(0.5) * (sig[5] + sig[7]);
            ss[5] = sig[8];
          }
          R A[9];
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) A[3 * a + c] = R(0.5) * (sig[3 * a + c] - sig[3 * c + a]);
#pragma unroll
          for (int k = 0; k < 9; ++k) sig[k] = A[k];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          sSig[a][s] = sig[3 * a + 0];
          sSig[3 + a][s] = sig[3 * a + 1];
        }
        sV[vbuf][0][s] = vq[0];
        sV[vbuf][1][s] = vq[1];
        if (r == 0) {
#pragma unroll
          for (int a = 0; a < 3; ++a) saz[a] = sig[3 * a + 2];
          vz = vq[2];
        }
      }
    }

    // ---- mu at the owned site of plane p-1 (the collision plane): its
    // anchoring divergence D0_a v_a takes v_x, v_y of plane p-1 from the
    // stress slots and v_z of planes p-2, p from the column registers.  It
    // reads phi p-2 and Q p-1, so it runs before the rings are refilled.
    if (collide) {
      const int a0 = (ly + 2) * AX + (lx + 2);
      const int s0 = (ly + 1) * SX + (lx + 1);
      const int vb = vbuf ^ 1;
      const R ph = sPhi[rm][a0];
      const R lapphi = ((sPhi[rm][a0 + 1] + sPhi[rm][a0 - 1]) + (sPhi[rm][a0 + AX] + sPhi[rm][a0 - AX]) +
                        (sPhi[r0][a0] + sPhi[rm2][a0])) - R(6) * ph;
      const R divv = R(0.5) * (sV[vb][0][s0 + 1] - sV[vb][0][s0 - 1]) +
                     R(0.5) * (sV[vb][1][s0 + SX] - sV[vb][1][s0 - SX]) + R(0.5) * (vz - vz_m2);
      R qs[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) qs[c] = sQ[cm][c][a0];
      sto(mu_out, uint32_t(zc) * plane_r + own_r, mu_site(P, ph, lapphi, divv, qs));
    }
    __syncthreads();  // stress of plane p is complete; ring slots of phi p-2 and Q p-1 are free

    // ---- refill the rings for plane p+1 from the registers loaded above
    if (refill) {
#pragma unroll
      for (int j = 0; j < KR; ++j) {
        if (rslot[j] >= 0) {
          sPhi[rm2][rslot[j]] = nphi[j];
#pragma unroll
          for (int c = 0; c < 5; ++c) sQ[cm][c][rslot[j]] = nq[j][c];
        }
      }
    }

    // ---- in-plane force part at plane p; collision of plane p-1
    const int s0 = (ly + 1) * SX + (lx + 1);
    R fin[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      fin[a] = R(0.5) * (sSig[a][s0 + 1] - sSig[a][s0 - 1]) + R(0.5) * (sSig[3 + a][s0 + SX] - sSig[3 + a][s0 - SX]);
    if (collide) {
      R F[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) F[a] = (fin_m1[a] + R(0.5) * (saz[a] - saz_m2[a])) + P.bf[a];
      R u[3], drho = R(0);
      if constexpr (L::kStressInEq)
        drho = collide_site_eq(P, g, F, ssym_m1, u);
      else
        drho = collide_site(P, g, F, u);
      const uint32_t sg = uint32_t(zc) * plane_gs + own_g, sr = uint32_t(zc) * plane_r + own_r;
      if (Bout) {  // null on a step that only records u, F and drho
#pragma unroll
        for (int i = 0; i < L::Q; ++i) GPolO<GS, L>::template st<R>(Bout + size_t(i) * N, sg, i, g[i]);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) sto(u_out + size_t(a) * N, sr, u[a]);
      if (F_out) {  // recording step (adjoint replay): keep the force of this plane
#pragma unroll
        for (int a = 0; a < 3; ++a) sto(F_out + size_t(a) * N, sr, F[a]);
      }
      if (drho_out) sto(drho_out, sr, drho);  // lean recording step: the density deviation
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      saz_m2[a] = saz_m1[a];
      saz_m1[a] = saz[a];
      fin_m1[a] = fin[a];
    }
    vz_m2 = vz_m1;
    vz_m1 = vz;
    if constexpr (L::kStressInEq) {
#pragma unroll
      for (int k = 0; k < 6; ++k) ssym_m1[k] = ss[k];
    }
    // advance the uniform indices to plane p+1
    r0 = rp;
    c0 = cp;
    zph = zph + 1 == b.nz ? 0 : zph + 1;
    zq = zq + 1 == b.nz ? 0 : zq + 1;
    zc_m = zc_0;
    zc_0 = zc_p;
    zc_p = zc_p + 1 == b.nz ? 0 : zc_p + 1;
  }
}

// ---------------------------------------------------------------------------
// k_order_fused
//   LDS holds plane z of (Q, phi, u, mu) on the tile plus the halo the
//   stencils read (rows y0-1, y0+TY and columns x0-1, x0+TX; no corners); the
//   owned column keeps planes z-1, z, z+1 of the same fields in registers.
//   The halo of plane z+1 is loaded into registers while plane z is computed.
// ---------------------------------------------------------------------------
template <class R, class FS, int TX, int TY, int MINW>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(MINW))) k_order_fused(Box b, Params<R> P, int TZ, int ntx, int nty,
                                                        const FS* __restrict__ phi, const FS* __restrict__ q,
                                                        const R* __restrict__ u, const R* __restrict__ mu,
                                                        FS* __restrict__ phi_out, FS* __restrict__ q_out) {
  constexpr int NT = TX * TY;
  constexpr int SX = TX + 2, SY = TY + 2, NS = SX * SY;
  constexpr int NH = 2 * (TX + TY);  // halo slots read by the stencils
  static_assert(NH <= NT, "one halo slot per thread");
  constexpr int NV = 10;             // q[5], phi, u[3], mu
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
  const int x = sGX[lx + 1], y = sGY[ly + 1];  // wrapped coordinates of the column
  const int col = y * b.nx + x;

  auto load_at = [&](size_t k, R v[NV]) {
#pragma unroll
    for (int c = 0; c < 5; ++c) v[c] = R(q[c * N + k]);
    v[5] = R(phi[k]);
#pragma unroll
    for (int a = 0; a < 3; ++a) v[6 + a] = u[a * N + k];
    v[9] = mu[k];
  };
  auto load_col = [&](int zz, R v[NV]) { load_at(size_t(pmod(zz, b.nz)) * plane + col, v); };
  R vm[NV], v0[NV], vp[NV];
  load_col(z0 - 1, vm);
  load_col(z0, v0);
  load_col(z0 + 1, vp);

  // this thread's halo slot (rows first, then columns), fixed over the march
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
      // gradients: x, y from LDS, z from the column registers
      Grad<R> G;
      G.phi = v0[5];
      G.dphi[0] = R(0.5) * (sV[5][sc + 1] - sV[5][sc - 1]);
      G.dphi[1] = R(0.5) * (sV[5][sc + SX] - sV[5][sc - SX]);
      G.dphi[2] = R(0.5) * (vp[5] - vm[5]);
      G.lapphi = R(0);
      G.divv = R(0);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const R qxp = sV[c][sc + 1], qxm = sV[c][sc - 1];
        const R qyp = sV[c][sc + SX], qym = sV[c][sc - SX];
        G.q[c] = v0[c];
        G.dq[0][c] = R(0.5) * (qxp - qxm);
        G.dq[1][c] = R(0.5) * (qyp - qym);
        G.dq[2][c] = R(0.5) * (vp[c] - vm[c]);
        G.lapq[c] = ((qxp + qxm) + (qyp + qym) + (vp[c] + vm[c])) - R(6) * v0[c];
      }
      R h[5];
      h_site(P, G, h);
      // velocity gradient W_ab = D0_b u_a, conservative phi flux, laplacian of mu
      R W[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        W[a][0] = R(0.5) * (sV[6 + a][sc + 1] - sV[6 + a][sc - 1]);
        W[a][1] = R(0.5) * (sV[6 + a][sc + SX] - sV[6 + a][sc - SX]);
        W[a][2] = R(0.5) * (vp[6 + a] - vm[6 + a]);
      }
      const R flux = R(0.5) * (sV[6][sc + 1] * sV[5][sc + 1] - sV[6][sc - 1] * sV[5][sc - 1]) +
                     R(0.5) * (sV[7][sc + SX] * sV[5][sc + SX] - sV[7][sc - SX] * sV[5][sc - SX]) +
                     R(0.5) * (vp[8] * vp[5] - vm[8] * vm[5]);
      const R lapmu = ((sV[9][sc + 1] + sV[9][sc - 1]) + (sV[9][sc + SX] + sV[9][sc - SX]) + (vp[9] + vm[9])) -
                      R(6) * v0[9];
      R S[5];
      corotation_site(P.xi, G.q, W, S);
      const size_t site = size_t(zc) * plane + col;
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const R adv = v0[6] * G.dq[0][k] + v0[7] * G.dq[1][k] + v0[8] * G.dq[2][k];
        q_out[k * N + site] = FS(v0[k] + (-adv + S[k] + P.Gamma * h[k]));
      }
      phi_out[site] = FS(v0[5] - flux + P.M * lapmu);
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      vm[c] = v0[c];
      v0[c] = vp[c];
    }
    if (zc + 1 < z1) load_col(zc + 2, vp);
  }
}

}  // namespace lbc
