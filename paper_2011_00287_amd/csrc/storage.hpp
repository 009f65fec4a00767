// Storage policies and lattice indexing shared by all kernels.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "physics.hpp"

namespace lbc {

// Global access as a uniform base pointer plus a 32-bit per-lane byte offset
// (the SGPR-base + VGPR-offset addressing form); every component array of
// a context is below 4 GiB (sites <= 2^29).
template <class T>
__device__ __forceinline__ T ldo(const T* __restrict__ base, uint32_t byteoff) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byteoff);
}
template <class T>
__device__ __forceinline__ void sto(T* __restrict__ base, uint32_t byteoff, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byteoff) = v;
}

// Population storage.  float64 / float32 store the deviation g_i itself;
// float16 stores g_i * 64 / w_i (w_i the weights of lattice L), which keeps
// the typical O(1e-4 .. 1e-1) values of g_i / w_i inside the normal range of
// the format.
template <class GS, class L = D3Q19>
struct GPol {
  template <class R>
  __device__ __forceinline__ static R ld(const GS* p, size_t k, int) { return R(p[k]); }
  template <class R>
  __device__ __forceinline__ static void st(GS* p, size_t k, int, R v) { p[k] = GS(v); }
};

// Non-temporal (streaming) access for 32- and 64-bit populations: each value
// is pulled once and the post-collision values are not read again within the
// step, so their traffic is marked to leave the caches to the fields the
// kernels re-read (u, mu, Q, phi and their halos).
template <class T>
__device__ __forceinline__ T ldo_nt(const T* __restrict__ base, uint32_t byteoff) {
  return __builtin_nontemporal_load(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byteoff));
}
template <class T>
__device__ __forceinline__ void sto_nt(T* __restrict__ base, uint32_t byteoff, T v) {
  __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byteoff));
}

template <class GS, class L = D3Q19>
struct GPolO {
  // element of the population array starting at base, by byte offset (streaming)
  template <class R>
  __device__ __forceinline__ static R ld(const GS* base, uint32_t off, int) { return R(ldo_nt(base, off)); }
  template <class R>
  __device__ __forceinline__ static void st(GS* base, uint32_t off, int, R v) { sto_nt(base, off, GS(v)); }
};
template <class L>
struct GPolO<__half, L> {
  // ordinary (cached) access: 16-bit streaming accesses measured much slower
  template <class R>
  __device__ __forceinline__ static R ld(const __half* base, uint32_t off, int i) {
    return R(__half2float(ldo(base, off))) * (L::template w<R>(i) * R(1.0 / 64.0));
  }
  template <class R>
  __device__ __forceinline__ static void st(__half* base, uint32_t off, int i, R v) {
    sto(base, off, __float2half(float(v * (R(64) / L::template w<R>(i)))));
  }
};

template <class L>
struct GPol<__half, L> {
  template <class R>
  __device__ __forceinline__ static R ld(const __half* p, size_t k, int i) {
    return R(__half2float(p[k])) * (L::template w<R>(i) * R(1.0 / 64.0));
  }
  template <class R>
  __device__ __forceinline__ static void st(__half* p, size_t k, int i, R v) {
    p[k] = __float2half(float(v * (R(64) / L::template w<R>(i))));
  }
};

struct Box {
  int nx, ny, nz;
  int N;  // nx*ny*nz
};

__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ __forceinline__ int sidx(const Box& b, int x, int y, int z) {
  return (wrapi(z, b.nz) * b.ny + wrapi(y, b.ny)) * b.nx + wrapi(x, b.nx);
}

__device__ __forceinline__ int pmod(int a, int n) {
  const int r = a % n;
  return r < 0 ? r + n : r;
}

// Bijection of [0, nblk): XCD x (ids congruent to x mod 8 are dealt to it)
// gets a contiguous range of logical block ids, so blocks that share stencil
// neighbours share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * q + (x < r ? x : r) + k;
}

// Site of this thread in a site-parallel launch, blocks remapped by XCD.
__device__ __forceinline__ int site_xcd() {
  return xcd_remap(int(blockIdx.x), int(gridDim.x)) * int(blockDim.x) + int(threadIdx.x);
}

__device__ __forceinline__ void coords(const Box& b, int s, int& x, int& y, int& z) {
  x = s % b.nx;
  const int t = s / b.nx;
  y = t % b.ny;
  z = t / b.ny;
}

}  // namespace lbc
