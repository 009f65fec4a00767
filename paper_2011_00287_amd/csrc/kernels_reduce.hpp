// Global float64 reductions: conservation totals, the discrete free energy
// F_h of Eq. (5), and the phi-weighted droplet centre.
//
// Each launch writes one partial vector per block (wave64 shuffles, then a
// fixed-order pass over the block's waves); k_final_sum adds the block
// partials in a fixed order, so results are bitwise reproducible.
#pragma once
#include "kernels_site.hpp"

namespace lbc {

// Block sum of NV doubles into out[0..NV) (added to out when accumulate).
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], double* __restrict__ out,
                                                   bool accumulate = false) {
  __shared__ double red[NV][16];  // one slot per wave, blocks of up to 1024 threads
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (int(blockDim.x) + 63) >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_down(v[k], o, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int k = threadIdx.x;
    double bs = red[k][0];
    for (int w = 1; w < nw; ++w) bs += red[k][w];  // fixed order: bitwise reproducible
    out[k] = accumulate ? out[k] + bs : bs;
  }
}

// out[g*nv + k] = sum over the blocks b of chunk g (b in [g*chunk, (g+1)*chunk)
// and below nblocks) of partial[b*nv + k]; one workgroup of 256 threads per
// chunk g (one chunk covering every block gives the plain total).
__global__ void __launch_bounds__(256) k_final_sum(const double* __restrict__ partial, int nblocks, int nv,
                                                   double* __restrict__ out, int chunk = 1 << 30) {
  __shared__ double buf[256];
  const int b0 = blockIdx.x * chunk, b1 = min(nblocks, b0 + chunk);
  for (int k = 0; k < nv; ++k) {
    double s = 0.0;
    for (int bI = b0 + threadIdx.x; bI < b1; bI += 256) s += partial[(size_t)bI * nv + k];
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (int(threadIdx.x) < w) buf[threadIdx.x] += buf[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[size_t(blockIdx.x) * nv + k] = buf[0];
    __syncthreads();
  }
}

// Plain 3x3 helpers for the float64 free-energy density (off the step path).
__device__ __forceinline__ void full3d(const double q[5], double Q[3][3]) {
  Q[0][0] = q[0]; Q[0][1] = q[1]; Q[0][2] = q[2];
  Q[1][0] = q[1]; Q[1][1] = q[3]; Q[1][2] = q[4];
  Q[2][0] = q[2]; Q[2][1] = q[4]; Q[2][2] = -q[0] - q[3];
}
__device__ __forceinline__ double ddot3d(const double A[3][3], const double B[3][3]) {
  double s = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) s += A[a][b] * B[a][b];
  return s;
}

constexpr int NTOT = 8;  // mass, jx, jy, jz, phi, F_h, E_kin, non-finite count

// Free-energy density of F_h at one site in float64: forward differences in
// the squared-gradient terms, central differences in the chiral and
// anchoring terms (the discretisation whose exact gradients are mu and -H).
template <class FS>
__device__ __forceinline__ double fh_density(const Box& b, const Params<double>& P, const FS* __restrict__ phi,
                                             const FS* __restrict__ q, int x, int y, int z) {
  const size_t N = b.N;
  const int s0 = (z * b.ny + y) * b.nx + x;
  const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double qc[5], Q[3][3], dQ[3][3][3], dphi[3];
  const double ph = double(phi[s0]);
  for (int k = 0; k < 5; ++k) qc[k] = double(q[k * N + s0]);
  full3d(qc, Q);
  double gp2 = 0.0, gq2 = 0.0;
  for (int g = 0; g < 3; ++g) {
    const int sp = sidx(b, x + off[g][0], y + off[g][1], z + off[g][2]);
    const int sm = sidx(b, x - off[g][0], y - off[g][1], z - off[g][2]);
    const double pp = double(phi[sp]), pm = double(phi[sm]);
    dphi[g] = 0.5 * (pp - pm);
    gp2 += (pp - ph) * (pp - ph);
    double qp[5], qm[5], dqk[5];
    for (int k = 0; k < 5; ++k) {
      qp[k] = double(q[k * N + sp]);
      qm[k] = double(q[k * N + sm]);
      dqk[k] = 0.5 * (qp[k] - qm[k]);
    }
    full3d(dqk, dQ[g]);
    const double f[5] = {qp[0] - qc[0], qp[1] - qc[1], qp[2] - qc[2], qp[3] - qc[3], qp[4] - qc[4]};
    const double fzz = -f[0] - f[3];
    gq2 += f[0] * f[0] + f[3] * f[3] + fzz * fzz + 2.0 * (f[1] * f[1] + f[2] * f[2] + f[4] * f[4]);
  }
  double Q2[3][3], C[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) Q2[a][c] = Q[a][0] * Q[0][c] + Q[a][1] * Q[1][c] + Q[a][2] * Q[2][c];
  const double tr2 = ddot3d(Q, Q), tr3 = ddot3d(Q2, Q);
  for (int c = 0; c < 3; ++c) {  // C_ab = eps_agd D0_g Q_db
    C[0][c] = dQ[1][2][c] - dQ[2][1][c];
    C[1][c] = dQ[2][0][c] - dQ[0][2][c];
    C[2][c] = dQ[0][1][c] - dQ[1][0][c];
  }
  const double qcurl = ddot3d(Q, C);
  double anch = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) anch += dphi[a] * Q[a][c] * dphi[c];
  const double chi = P.chi0 + P.chi_s * ph;
  const double dw = ph * (ph - P.phi0);
  return 0.5 * P.a * dw * dw * P.inv_phicr2 +
         P.A0 * (0.5 * (1.0 - chi / 3.0) * tr2 - chi / 3.0 * tr3 + chi / 4.0 * tr2 * tr2) +
         2.0 * P.K * P.q0 * P.q0 * tr2 + 0.5 * P.k_phi * gp2 + 0.5 * P.K * gq2 + 2.0 * P.K * P.q0 * qcurl +
         P.W * anch;
}

template <class R, class GS, class FS, class L>
__global__ void __launch_bounds__(256) k_totals(Box b, Params<double> P, const GS* __restrict__ B,
                                                const FS* __restrict__ phi, const FS* __restrict__ q,
                                                const R* __restrict__ sig, double* __restrict__ partial) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double v[NTOT];
#pragma unroll
  for (int k = 0; k < NTOT; ++k) v[k] = 0.0;
  if (s < b.N) {
    int x, y, z;
    coords(b, s, x, y, z);
    const size_t N = b.N;
    double sum = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < L::Q; ++i) {
      const double gi =
          double(GPol<GS, L>::template ld<R>(B, i * N + sidx(b, x - L::cx(i), y - L::cy(i), z - L::cz(i)), i));
      sum += gi;
      j[0] += L::cx(i) * gi;
      j[1] += L::cy(i) * gi;
      j[2] += L::cz(i) * gi;
    }
    R Fs[3];
    force_sig<L>(b, sig, x, y, z, Fs);
    double mom[3];
    for (int a = 0; a < 3; ++a) mom[a] = j[a] + 0.5 * double(Fs[a] + R(P.bf[a]));
    const double rho = P.rho0 + sum;
    const double fh = fh_density(b, P, phi, q, x, y, z);
    const double ph = double(phi[s]);
    v[0] = sum;
    v[1] = mom[0];
    v[2] = mom[1];
    v[3] = mom[2];
    v[4] = ph;
    v[5] = fh;
    v[6] = 0.5 * (mom[0] * mom[0] + mom[1] * mom[1] + mom[2] * mom[2]) / rho;
    double chk = sum + mom[0] + mom[1] + mom[2] + ph + fh;
    for (int k = 0; k < 5; ++k) chk += double(q[k * N + s]);
    v[7] = isfinite(chk) ? 0.0 : 1.0;
  }
  block_reduce_store<NTOT>(v, partial + (size_t)blockIdx.x * NTOT);
}

constexpr int NCEN = 10;  // phi x, phi y, phi z, phi, (phi sin, phi cos) per axis

template <class FS>
__global__ void __launch_bounds__(256) k_centre(Box b, const FS* __restrict__ phi, double* __restrict__ partial) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double v[NCEN];
#pragma unroll
  for (int k = 0; k < NCEN; ++k) v[k] = 0.0;
  if (s < b.N) {
    int x, y, z;
    coords(b, s, x, y, z);
    const double ph = double(phi[s]);
    v[0] = ph * x;
    v[1] = ph * y;
    v[2] = ph * z;
    v[3] = ph;
    double sn, cs;
    sincospi(2.0 * x / b.nx, &sn, &cs);
    v[4] = ph * sn;
    v[5] = ph * cs;
    sincospi(2.0 * y / b.ny, &sn, &cs);
    v[6] = ph * sn;
    v[7] = ph * cs;
    sincospi(2.0 * z / b.nz, &sn, &cs);
    v[8] = ph * sn;
    v[9] = ph * cs;
  }
  block_reduce_store<NCEN>(v, partial + (size_t)blockIdx.x * NCEN);
}

// Centre from the summed k_centre partials (sums[0..NCEN)) on the device:
// out[0..2] linear centre, out[3..5] circular mean per axis in [0, n),
// out[6] sum of phi.  One thread.
__global__ void k_centre_finish(Box b, const double* __restrict__ sums, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int n[3] = {b.nx, b.ny, b.nz};
  for (int a = 0; a < 3; ++a) {
    out[a] = sums[a] / sums[3];
    const double ang = atan2(sums[4 + 2 * a], sums[5 + 2 * a]);
    double c = ang * n[a] / (2.0 * M_PI);
    if (c < 0) c += n[a];
    out[3 + a] = c;
  }
  out[6] = sums[3];
}

}  // namespace lbc
