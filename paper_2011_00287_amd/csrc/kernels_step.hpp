// The whole coupled step in one launch (explicit Euler, second-order stencils).
//
// k_step_fused marches along z over a slab of planes, like k_lb_fused, and
// in the same pass updates the order parameters (Eqs. (1)-(2)), so that Q
// and phi are read once per step and u, mu never leave the chip.  The price
// is a wider halo: the Q and phi updates of the TX x TY tile need u and mu on
// the tile's edges (the sites one step outside it, corners excluded), so the
// workgroup also pulls the populations of those edge sites (moments only),
// computes their force and mu, and for that the stress on a frame two sites
// wide (Q and phi staged with a halo of three).
//
// Iteration p of the march (p = z0-2 .. z1+1, planes taken periodically):
//   loads     pulls of plane p-1 (own site; one edge site on some threads)
//             and the ring planes p+2 of Q and phi, issued first
//   stress    plane p at the own site and at the halo slots (edge sites and
//             the outer frame), on rotating waves
//   --- barrier ---
//   refill    rings of Q (3 planes) and phi (5 planes) with plane p+2
//   A(p)      mu(p) without the term of v_z(p+1) (anchoring divergence)
//   fin(p)    in-plane part of the force at plane p
//   collide   plane p-1: force, u, mu; full BGK + stream at the own site,
//             moments only at edge sites; u, mu of the plane go to LDS
//   order     Q and phi of plane p-2 at the own site (u, mu of planes p-3,
//             p-2, p-1 from LDS; H, D0 Q, Q of plane p-2 carried in
//             registers from the stress pass)
//   --- barrier (top of the next iteration) ---
// Every right-hand side uses time-t fields, as in the two-launch path; the
// only difference in arithmetic is that mu is summed in two parts.
//
// Frame coordinates (fx, fy) are relative to the tile origin.  Every frame
// position maps to the wrapped global site, so stencils near the periodic
// faces and on ragged tiles are those of the global box; only threads whose
// own site lies inside the box write.
#pragma once
#include "physics.hpp"
#include "storage.hpp"

namespace lbc {

template <int TX, int TY>
struct StepFrame {
  static constexpr int NT = TX * TY;
  static constexpr int AX = TX + 6, AY = TY + 6, NA = AX * AY;  // Q, phi rings (halo 3)
  static constexpr int SX = TX + 4, SY = TY + 4, NSF = SX * SY;  // stress slots (halo 2)
  static constexpr int UX = TX + 2, UY = TY + 2, NU = UX * UY;   // u, mu (halo 1)
  static constexpr int NE = 2 * (TX + TY);                        // edge sites (halo 1, no corners)
  static constexpr int NO = NE + 4;                               // outer stress slots
  static constexpr int NH = NE + NO;                              // halo stress slots
  static constexpr int NR = SX * SY + NE;                         // ring slots loaded per plane
  static constexpr int KR = (NR + NT - 1) / NT;
  __device__ static int ra(int fx, int fy) { return (fy + 3) * AX + (fx + 3); }
  __device__ static int rs(int fx, int fy) { return (fy + 2) * SX + (fx + 2); }
  __device__ static int ru(int fx, int fy) { return (fy + 1) * UX + (fx + 1); }
  // edge site e: rows y = -1, y = TY (x in [0, TX)), then columns x = -1, x = TX
  __device__ static void edge_pos(int e, int& fx, int& fy) {
    if (e < 2 * TX) {
      fx = e < TX ? e : e - TX;
      fy = e < TX ? -1 : TY;
    } else {
      const int k = e - 2 * TX;
      fx = k < TY ? -1 : TX;
      fy = k < TY ? k : k - TY;
    }
  }
  // outer slot o: rows y = -2, y = TY + 1, columns x = -2, x = TX + 1, then
  // the four corners of the edge ring
  __device__ static void outer_pos(int o, int& fx, int& fy) {
    if (o < NE) {
      if (o < 2 * TX) {
        fx = o < TX ? o : o - TX;
        fy = o < TX ? -2 : TY + 1;
      } else {
        const int k = o - 2 * TX;
        fx = k < TY ? -2 : TX + 1;
        fy = k < TY ? k : k - TY;
      }
    } else {
      const int c = o - NE;
      fx = (c & 1) ? TX : -1;
      fy = (c & 2) ? TY : -1;
    }
  }
  // ring slot j of the per-plane load list: the (TX+4) x (TY+4) rectangle,
  // then the four rows / columns three sites out
  __device__ static void ring_pos(int j, int& fx, int& fy) {
    if (j < SX * SY) {
      fx = j % SX - 2;
      fy = j / SX - 2;
    } else {
      const int k = j - SX * SY;
      if (k < 2 * TX) {
        fx = k < TX ? k : k - TX;
        fy = k < TX ? -3 : TY + 2;
      } else {
        const int m = k - 2 * TX;
        fx = m < TY ? -3 : TX + 2;
        fy = m < TY ? m : m - TY;
      }
    }
  }
};

template <class R, class GS, class FS, class L, int TX, int TY, int MINW>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(MINW)))
k_step_fused(Box b, Params<R> P, int TZ, int ntx, int nty, const GS* __restrict__ Bin, GS* __restrict__ Bout,
             const FS* __restrict__ phi, const FS* __restrict__ q, FS* __restrict__ phi_out,
             FS* __restrict__ q_out, R* __restrict__ u_rec, R* __restrict__ F_rec, R* __restrict__ drho_rec,
             const int64_t* __restrict__ step_in, int64_t* __restrict__ step_out) {
  using Fr = StepFrame<TX, TY>;
  constexpr int NT = Fr::NT, AX = Fr::AX, AY = Fr::AY, NA = Fr::NA, SX = Fr::SX, NSF = Fr::NSF;
  constexpr int UX = Fr::UX, NU = Fr::NU, NE = Fr::NE, NH = Fr::NH, KR = Fr::KR;
  static_assert(NT % 64 == 0, "whole waves");
  static_assert(NH + NE <= NT, "one halo stress slot or one edge job per thread and plane");
  if (step_out != nullptr && blockIdx.x == 0 && threadIdx.x == 0) step_out[0] = step_in[0] + 1;

  __shared__ R sPhi[5][NA];     // phi planes by p mod 5
  __shared__ R sQ[3][5][NA];    // Q planes by p mod 3
  __shared__ R sSig[6][NSF];    // sigma_ax, sigma_ay of the stress slots (plane p)
  __shared__ R sV[2][NSF];      // v_x, v_y of the stress slots (plane p)
  __shared__ R sUM[3][4][NU];   // u, mu of the tile and its edges, planes by p mod 3
  __shared__ R eSaz[3][3][NE];  // sigma_az of the edge sites, planes by p mod 3
  __shared__ R eVz[3][NE];      // v_z of the edge sites, planes by p mod 3
  __shared__ R eFin[2][3][NE];  // in-plane force of the edge sites, planes by parity
  __shared__ R eA[2][NE];       // mu(p) less its v_z(p+1) term at the edge sites, by parity
  __shared__ int sGX[AX], sGY[AY];

  const int l = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = l % ntx, ty = (l / ntx) % nty, sl = l / (ntx * nty);
  const int x0 = tx * TX, y0 = ty * TY, z0 = sl * TZ;
  const int z1 = min(z0 + TZ, b.nz);
  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = tid / TX;
  const bool active = (x0 + lx < b.nx) && (y0 + ly < b.ny);
  const size_t N = b.N;
  const int plane = b.nx * b.ny;

  for (int k = tid; k < AX; k += NT) sGX[k] = pmod(x0 - 3 + k, b.nx);
  for (int k = tid; k < AY; k += NT) sGY[k] = pmod(y0 - 3 + k, b.ny);
  __syncthreads();

  // ring slots this thread loads each plane
  int rslot[KR];
  uint32_t rcol[KR];
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    const int k = tid + j * NT;
    rslot[j] = -1;
    rcol[j] = 0u;
    if (k < Fr::NR) {
      int fx, fy;
      Fr::ring_pos(k, fx, fy);
      rslot[j] = Fr::ra(fx, fy);
      rcol[j] = uint32_t(sGY[fy + 3] * b.nx + sGX[fx + 3]) * uint32_t(sizeof(FS));
    }
  }
  const uint32_t plane_fs = uint32_t(plane) * uint32_t(sizeof(FS));
  auto fill = [&](int p, bool do_q) {
    const uint32_t bz = uint32_t(pmod(p, b.nz)) * plane_fs;
    const int sph = pmod(p, 5), sq = pmod(p, 3);
#pragma unroll
    for (int j = 0; j < KR; ++j) {
      if (rslot[j] >= 0) {
        sPhi[sph][rslot[j]] = R(ldo(phi, bz + rcol[j]));
        if (do_q) {
#pragma unroll
          for (int c = 0; c < 5; ++c) sQ[sq][c][rslot[j]] = R(ldo(q + size_t(c) * N, bz + rcol[j]));
        }
      }
    }
  };
  for (int p = z0 - 3; p <= z0 - 1; ++p) fill(p, true);

  // own site: frame slots and global byte offsets
  const int a_own = Fr::ra(lx, ly), s_own = Fr::rs(lx, ly), m_own = Fr::ru(lx, ly);
  const uint32_t plane_gs = uint32_t(plane) * uint32_t(sizeof(GS));
  const uint32_t plane_r = uint32_t(plane) * uint32_t(sizeof(R));
  const int col_own = sGY[ly + 3] * b.nx + sGX[lx + 3];
  const uint32_t own_g = uint32_t(col_own) * uint32_t(sizeof(GS));
  const uint32_t own_f = uint32_t(col_own) * uint32_t(sizeof(FS));
  const uint32_t own_r = uint32_t(col_own) * uint32_t(sizeof(R));
  uint32_t colb[3][3];  // in-plane byte offsets of the own site's 9 pull columns
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int i = 0; i < 3; ++i) colb[j][i] = uint32_t(sGY[ly + 2 + j] * b.nx + sGX[lx + 2 + i]) * uint32_t(sizeof(GS));

  // carried registers of the own column
  R saz_m1[3] = {R(0), R(0), R(0)}, saz_m2[3] = {R(0), R(0), R(0)};  // sigma_az at p-1, p-2
  R fin_m1[3] = {R(0), R(0), R(0)};  // in-plane force at p-1
  R A_m1 = R(0), vz_m1 = R(0);       // A(p-1), v_z(p-1)
  R ssym_m1[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};  // symmetric stress at p-1 (D3Q15)
  R q_m1[5], q_m2[5], p1_m1[5], p12_m2[5], dq_m1[3][5];  // Q update pieces (see the order step)
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    q_m1[c] = q_m2[c] = p1_m1[c] = p12_m2[c] = R(0);
    dq_m1[0][c] = dq_m1[1][c] = dq_m1[2][c] = R(0);
  }
  constexpr int NW = NT / 64;

  for (int p = z0 - 2; p <= z1 + 1; ++p) {
    __syncthreads();  // ring planes p-1..p+1 complete; the previous plane's LDS reads are done
    const int pc = p - 1, po = p - 2;
    const int r3p = pmod(p, 3), r3m = pmod(p - 1, 3), r3mm = pmod(p - 2, 3), r3pp = pmod(p + 1, 3);
    const int f5p = pmod(p, 5), f5m = pmod(p - 1, 5), f5mm = pmod(p - 2, 5), f5mmm = pmod(p - 3, 5),
              f5pp = pmod(p + 1, 5);
    const int par = p & 1, parc = pc & 1;
    // halo work of this plane on rotated thread indices: stress slots first, then edge jobs
    const int shift = ((p + 2 + l) % NW) * 64;
    const int rt = tid >= shift ? tid - shift : tid - shift + NT;
    const bool own_band = p >= z0 - 1 && p <= z1;          // planes whose u, mu the own column needs
    const bool edge_band = p >= z0 && p <= z1 - 1;         // planes whose u, mu the edge sites need
    const bool own_coll = pc >= z0 - 1 && pc <= z1;
    const bool own_write = pc >= z0 && pc <= z1 - 1;
    const bool edge_coll = pc >= z0 && pc <= z1 - 1;
    const int ej = rt - NH;  // edge job (A of plane p, collision of plane p-1)
    const bool has_ej = ej >= 0 && ej < NE;
    int efx = 0, efy = 0;
    if (has_ej) Fr::edge_pos(ej, efx, efy);

    // ---- loads issued before the stress pass
    R g[L::Q], ge[L::Q];
    const uint32_t zc_m = uint32_t(pmod(pc - 1, b.nz)) * plane_gs, zc_0 = uint32_t(pmod(pc, b.nz)) * plane_gs,
                   zc_p = uint32_t(pmod(pc + 1, b.nz)) * plane_gs;
    const uint32_t zb[3] = {zc_m, zc_0, zc_p};
    if (own_coll) {
#pragma unroll
      for (int i = 0; i < L::Q; ++i)
        g[i] = GPolO<GS, L>::template ld<R>(Bin + size_t(i) * N, zb[1 - L::cz(i)] + colb[1 - L::cy(i)][1 - L::cx(i)],
                                            i);
    }
    if (has_ej && edge_coll) {
      const int gx[3] = {sGX[efx + 2], sGX[efx + 3], sGX[efx + 4]};
      const int gy[3] = {sGY[efy + 2], sGY[efy + 3], sGY[efy + 4]};
#pragma unroll
      for (int i = 0; i < L::Q; ++i) {
        const uint32_t off =
            zb[1 - L::cz(i)] + uint32_t(gy[1 - L::cy(i)] * b.nx + gx[1 - L::cx(i)]) * uint32_t(sizeof(GS));
        ge[i] = GPol<GS, L>::template ld<R>(Bin + size_t(i) * N, off / sizeof(GS), i);
      }
    }
    const bool refill = p <= z1;
    R nphi[KR], nq[KR][5];
    if (refill) {
      const uint32_t bz = uint32_t(pmod(p + 2, b.nz)) * plane_fs;
#pragma unroll
      for (int j = 0; j < KR; ++j) {
        if (rslot[j] >= 0) {
          nphi[j] = R(ldo(phi, bz + rcol[j]));
#pragma unroll
          for (int c = 0; c < 5; ++c) nq[j][c] = R(ldo(q + size_t(c) * N, bz + rcol[j]));
        }
      }
    }
    const R phi_m3 = sPhi[f5mmm][a_own];  // own phi(p-3), before its ring slot is refilled

    // ---- stress at plane p: round 0 the own site, round 1 a halo slot
    R saz[3], vz = R(0), h[5], qown[5], dq[3][5];
    R ss[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll 1
    for (int r = 0; r < 2; ++r) {
      int fx, fy, e = -1;
      if (r == 0) {
        fx = lx;
        fy = ly;
      } else {
        if (rt >= NH) break;
        if (rt < NE) {
          if (!own_band) break;
          e = rt;
          Fr::edge_pos(e, fx, fy);
        } else {
          if (!edge_band) break;
          Fr::outer_pos(rt - NE, fx, fy);
        }
      }
      const int a0 = Fr::ra(fx, fy), s = Fr::rs(fx, fy);
      Grad<R> G;
      G.phi = sPhi[f5p][a0];
      G.dphi[0] = R(0.5) * (sPhi[f5p][a0 + 1] - sPhi[f5p][a0 - 1]);
      G.dphi[1] = R(0.5) * (sPhi[f5p][a0 + AX] - sPhi[f5p][a0 - AX]);
      G.dphi[2] = R(0.5) * (sPhi[f5pp][a0] - sPhi[f5m][a0]);
      G.lapphi = R(0);
      G.divv = R(0);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const R qc = sQ[r3p][c][a0];
        const R qxp = sQ[r3p][c][a0 + 1], qxm = sQ[r3p][c][a0 - 1];
        const R qyp = sQ[r3p][c][a0 + AX], qym = sQ[r3p][c][a0 - AX];
        const R qzp = sQ[r3pp][c][a0], qzm = sQ[r3m][c][a0];
        G.q[c] = qc;
        G.dq[0][c] = R(0.5) * (qxp - qxm);
        G.dq[1][c] = R(0.5) * (qyp - qym);
        G.dq[2][c] = R(0.5) * (qzp - qzm);
        G.lapq[c] = ((qxp + qxm) + (qyp + qym) + (qzp + qzm)) - R(6) * qc;
      }
      R sig[9], hh[5], vq[3];
      sigma_site(P, G, sig, hh, vq);
      if constexpr (L::kStressInEq) {
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
      sV[0][s] = vq[0];
      sV[1][s] = vq[1];
      if (r == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) saz[a] = sig[3 * a + 2];
        vz = vq[2];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          h[c] = hh[c];
          qown[c] = G.q[c];
          dq[0][c] = G.dq[0][c];
          dq[1][c] = G.dq[1][c];
          dq[2][c] = G.dq[2][c];
        }
      } else if (e >= 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) eSaz[r3p][a][e] = sig[3 * a + 2];
        eVz[r3p][e] = vq[2];
      }
    }
    __syncthreads();  // stress of plane p complete; ring slots of phi p-3 and Q p-1 are free

    // ---- refill the rings with plane p+2
    if (refill) {
      const int sph = pmod(p + 2, 5), sq = pmod(p + 2, 3);
#pragma unroll
      for (int j = 0; j < KR; ++j) {
        if (rslot[j] >= 0) {
          sPhi[sph][rslot[j]] = nphi[j];
#pragma unroll
          for (int c = 0; c < 5; ++c) sQ[sq][c][rslot[j]] = nq[j][c];
        }
      }
    }

    // ---- A(p): mu of plane p without the v_z(p+1) half of the anchoring divergence
    auto a_at = [&](int a0, int s, R vz_below) -> R {
      const R ph = sPhi[f5p][a0];
      const R lapphi = ((sPhi[f5p][a0 + 1] + sPhi[f5p][a0 - 1]) + (sPhi[f5p][a0 + AX] + sPhi[f5p][a0 - AX]) +
                        (sPhi[f5pp][a0] + sPhi[f5m][a0])) - R(6) * ph;
      const R divv = R(0.5) * (sV[0][s + 1] - sV[0][s - 1]) + R(0.5) * (sV[1][s + SX] - sV[1][s - SX]) -
                     R(0.5) * vz_below;
      R qs[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) qs[c] = sQ[r3p][c][a0];
      return mu_site(P, ph, lapphi, divv, qs);
    };
    auto fin_at = [&](int s, R f[3]) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
        f[a] = R(0.5) * (sSig[a][s + 1] - sSig[a][s - 1]) + R(0.5) * (sSig[3 + a][s + SX] - sSig[3 + a][s - SX]);
    };
    R A0 = R(0), fin[3] = {R(0), R(0), R(0)};
    if (own_band) {
      A0 = a_at(a_own, s_own, vz_m1);
      fin_at(s_own, fin);
    }
    if (has_ej && edge_band) {
      const int a0 = Fr::ra(efx, efy), s = Fr::rs(efx, efy);
      eA[par][ej] = a_at(a0, s, eVz[r3m][ej]);
      R f[3];
      fin_at(s, f);
#pragma unroll
      for (int a = 0; a < 3; ++a) eFin[par][a][ej] = f[a];
    }

    // ---- plane p-1: force, u and mu; collision at the own site, moments at an edge site
    R ucol[3] = {R(0), R(0), R(0)};
    R p12_c[5] = {R(0), R(0), R(0), R(0), R(0)};
    const int m3c = pmod(pc, 3);
    if (own_coll) {
      R F[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) F[a] = (fin_m1[a] + R(0.5) * (saz[a] - saz_m2[a])) + P.bf[a];
      R drho;
      if (own_write) {
        if constexpr (L::kStressInEq)
          drho = collide_site_eq(P, g, F, ssym_m1, ucol);
        else
          drho = collide_site(P, g, F, ucol);
        if (active) {
          const uint32_t sg = uint32_t(pmod(pc, b.nz)) * plane_gs + own_g;
          if (Bout) {  // null on a step that only records u, F and drho
#pragma unroll
            for (int i = 0; i < L::Q; ++i) GPolO<GS, L>::template st<R>(Bout + size_t(i) * N, sg, i, g[i]);
          }
          const uint32_t sr = uint32_t(pmod(pc, b.nz)) * plane_r + own_r;
          if (u_rec) {
#pragma unroll
            for (int a = 0; a < 3; ++a) sto(u_rec + size_t(a) * N, sr, ucol[a]);
          }
          if (F_rec) {
#pragma unroll
            for (int a = 0; a < 3; ++a) sto(F_rec + size_t(a) * N, sr, F[a]);
          }
          if (drho_rec) sto(drho_rec, sr, drho);
        }
      } else {
        drho = g[0];
        R j[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
          drho += g[i];
          cadd(L::cx(i), g[i], j[0]);
          cadd(L::cy(i), g[i], j[1]);
          cadd(L::cz(i), g[i], j[2]);
        }
        const R inv = R(1) / (P.rho0 + drho);
#pragma unroll
        for (int a = 0; a < 3; ++a) ucol[a] = (j[a] + R(0.5) * F[a]) * inv;
      }
      const R mu_c = A_m1 - P.W * vz;
#pragma unroll
      for (int a = 0; a < 3; ++a) sUM[m3c][a][m_own] = ucol[a];
      sUM[m3c][3][m_own] = mu_c;
      // Q(pc) + Gamma H(pc) - u(pc) . D0 Q(pc)
#pragma unroll
      for (int c = 0; c < 5; ++c)
        p12_c[c] = p1_m1[c] - (ucol[0] * dq_m1[0][c] + ucol[1] * dq_m1[1][c] + ucol[2] * dq_m1[2][c]);
    }
    if (has_ej && edge_coll) {
      R F[3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
        F[a] = (eFin[parc][a][ej] + R(0.5) * (eSaz[r3p][a][ej] - eSaz[r3mm][a][ej])) + P.bf[a];
      R drho = ge[0];
      R j[3] = {R(0), R(0), R(0)};
#pragma unroll
      for (int i = 1; i < L::Q; ++i) {
        drho += ge[i];
        cadd(L::cx(i), ge[i], j[0]);
        cadd(L::cy(i), ge[i], j[1]);
        cadd(L::cz(i), ge[i], j[2]);
      }
      const R inv = R(1) / (P.rho0 + drho);
      const int m = Fr::ru(efx, efy);
#pragma unroll
      for (int a = 0; a < 3; ++a) sUM[m3c][a][m] = (j[a] + R(0.5) * F[a]) * inv;
      sUM[m3c][3][m] = eA[parc][ej] - P.W * eVz[r3p][ej];
    }

    // ---- order parameters of plane p-2 at the own site (skipped on a record-only step)
    if (q_out != nullptr && po >= z0 && po <= z1 - 1) {
      const int m3o = pmod(po, 3), m3b = pmod(po - 1, 3);
      const R(*U0)[NU] = sUM[m3o];
      R W[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        W[a][0] = R(0.5) * (U0[a][m_own + 1] - U0[a][m_own - 1]);
        W[a][1] = R(0.5) * (U0[a][m_own + UX] - U0[a][m_own - UX]);
        W[a][2] = R(0.5) * (sUM[m3c][a][m_own] - sUM[m3b][a][m_own]);
      }
      R S[5];
      corotation_site(P.xi, q_m2, W, S);
      // conservative phi flux and laplacian of mu
      const R* Ph0 = sPhi[f5mm];
      const R flux = R(0.5) * (U0[0][m_own + 1] * Ph0[a_own + 1] - U0[0][m_own - 1] * Ph0[a_own - 1]) +
                     R(0.5) * (U0[1][m_own + UX] * Ph0[a_own + AX] - U0[1][m_own - UX] * Ph0[a_own - AX]) +
                     R(0.5) * (sUM[m3c][2][m_own] * sPhi[f5m][a_own] - sUM[m3b][2][m_own] * phi_m3);
      const R lapmu = ((U0[3][m_own + 1] + U0[3][m_own - 1]) + (U0[3][m_own + UX] + U0[3][m_own - UX]) +
                       (sUM[m3c][3][m_own] + sUM[m3b][3][m_own])) - R(6) * U0[3][m_own];
      if (active) {
        const uint32_t so = uint32_t(pmod(po, b.nz)) * plane_fs + own_f;
#pragma unroll
        for (int k = 0; k < 5; ++k) sto(q_out + size_t(k) * N, so, FS(p12_m2[k] + S[k]));
        sto(phi_out, so, FS(Ph0[a_own] - flux + P.M * lapmu));
      }
    }

    // ---- carry the own column to plane p+1
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      saz_m2[a] = saz_m1[a];
      saz_m1[a] = saz[a];
      fin_m1[a] = fin[a];
    }
    A_m1 = A0;
    vz_m1 = vz;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      q_m2[c] = q_m1[c];
      q_m1[c] = qown[c];
      p12_m2[c] = p12_c[c];
      p1_m1[c] = qown[c] + P.Gamma * h[c];
      dq_m1[0][c] = dq[0][c];
      dq_m1[1][c] = dq[1][c];
      dq_m1[2][c] = dq[2][c];
    }
    if constexpr (L::kStressInEq) {
#pragma unroll
      for (int k = 0; k < 6; ++k) ssym_m1[k] = ss[k];
    }
  }
}

}  // namespace lbc
