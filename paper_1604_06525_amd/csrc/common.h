// Device-side building blocks shared by all energies: launch geometry,
// deterministic FP64 block reductions, the device-resident solver scalars and
// the Jacobi preconditioner.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "opt_limits.h"

namespace optmi {

// Chunk-local neighbour slots and halo lists of a graph problem: nbl[k] names the
// neighbour of incidence-list entry k by its LDS slot (u - chunk start inside the
// chunk, kBlock + halo index for a staged outside vertex, -(u + 1) for one past
// the cap); chunk c stages the hcnt[c] vertices hid[c * cap ...] (rows of a fixed
// stride, so that a count and the ids can be read at once).
struct Halo {
  const int* __restrict__ nbl;
  const int* __restrict__ hcnt;
  const int* __restrict__ hid;
};

// The per-vertex values a staged graph energy reads for a neighbour.
template <typename T, int N>
struct Vals {
  T v[N];
};

// Solver scalars that live on the device for the whole solve, so that the host
// never waits inside the loop.  Written by block 0 of one kernel and read by the
// kernels that follow it in stream order.
struct DevScalars {
  double rz[2];      // split form: r.z of PCG iteration k, stored at slot k & 1
  double gam[2];     // fused form: gamma_i and alpha_i at slot i & 1
  double alpha[2];
  double E0;         // cost at the current linearisation point
  double E1;         // LM: cost at the trial point x + d
  double m;          // LM: model decrease
  double radius, nu, lambda;  // LM trust region; lambda = 1/radius (GN: 0)
  double E_final;
  int32_t stopped;   // PCG breakdown: p.q was not positive
  int32_t accepted;  // LM: last step taken
  int32_t need_lin;  // LM: x changed since the last linearisation
  int32_t done;      // LM: radius fell below its minimum
  int32_t n_accepted;
  int32_t outer_done;
  int32_t nonfinite; // a cost was NaN or infinite
  int32_t trace_k;   // next cost-trace entry (one per outer iteration that linearises)
};

// Sum of v over the block in a fixed order: a shuffle tree inside each wave,
// then the wave totals in wave order.  The result is valid in thread 0 only.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double wsum[kWaves];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wsum[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kWaves; ++k) t += wsum[k];
  }
  __syncthreads();
  return t;
}

// The grid a kernel body sees: its block id and block count.  A plain launch
// passes the hardware grid; a batched launch passes the block's position inside
// its problem's range of blocks, so each problem is processed exactly as if it
// had been launched alone.
struct VG {
  int bid, nb;
};

// Store the block's sum of v at out[g.bid].
__device__ __forceinline__ void block_store(double v, double* out, VG g) {
  const double t = block_sum(v);
  if (threadIdx.x == 0) out[g.bid] = t;
}

// Sum of the n partials written by the previous kernel, in a fixed order that
// does not depend on the reading block, so every block obtains the same bits.
// Returned to every thread of the block.
__device__ __forceinline__ double reduce_partials(const double* __restrict__ part, int n) {
  __shared__ double total;
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += kBlock) acc += part[k];
  const double t = block_sum(acc);
  if (threadIdx.x == 0) total = t;
  __syncthreads();
  return total;
}

// block_sum of two values at once (one pair of barriers); each result has the
// bits block_sum gives it alone.  Valid in thread 0 only.
__device__ __forceinline__ void block_sum2(double a, double b, double* ta, double* tb) {
  __shared__ double wsum[2][kWaves];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    wsum[0][w] = a;
    wsum[1][w] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      sa += wsum[0][k];
      sb += wsum[1][k];
    }
  }
  __syncthreads();
  *ta = sa;
  *tb = sb;
}

// reduce_partials of two arrays in one pass (their loads are issued together);
// each result has the bits reduce_partials gives it alone.  Returned to every
// thread of the block.
__device__ __forceinline__ void reduce_partials2(const double* __restrict__ pa, const double* __restrict__ pb,
                                                 int n, double* ta, double* tb) {
  __shared__ double total[2];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < n; k += kBlock) {
    a += pa[k];
    b += pb[k];
  }
  double sa, sb;
  block_sum2(a, b, &sa, &sb);
  if (threadIdx.x == 0) {
    total[0] = sa;
    total[1] = sb;
  }
  __syncthreads();
  *ta = total[0];
  *tb = total[1];
}

// p as a pointer to global memory.  Pointers read from an argument row in
// device memory are generic; accesses through them compile to flat
// instructions, which also count against the LDS/scalar counter, so every wait
// for an LDS read would wait for outstanding HBM loads and stores as well.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ bool is_block_leader(VG g) { return g.bid == 0 && threadIdx.x == 0; }

// 1/x: the hardware reciprocal in FP32 (within 1 ulp; every kernel forms M^-1
// with it, so the preconditioner is the same everywhere), correctly rounded in
// FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Jacobi preconditioner entry for an unknown with diagonal d (Sec. 4.1): the
// inverse of the damped diagonal d + lambda*clamp(d), or 0 when that is not
// positive (an unknown no residual touches stays where it is).  Without the
// preconditioner every unknown gets 1; excluded unknowns have r = 0, so their
// z = M^-1 r is 0 either way.
template <typename T>
struct Precond {
  T lam, dmin, dmax;
  int use;
  __device__ __forceinline__ T damp(T d) const { return lam * (d < dmin ? dmin : (d > dmax ? dmax : d)); }
  // the preconditioner's entry M (the damped diagonal, or 1 without it)
  __device__ __forceinline__ T den(T d) const {
    if (!use) return T(1);
    return lam != T(0) ? d + damp(d) : d;
  }
  __device__ __forceinline__ T minv(T d) const {
    if (!use) return T(1);
    const T m = den(d);
    return m > T(0) ? recip(m) : T(0);
  }
};

__device__ __forceinline__ bool finite_d(double v) { return v - v == 0.0; }

// A raw buffer view of a device array: a scalar descriptor plus a 32-bit byte
// offset per lane.  Reads at or past `bytes` return 0 and writes there are dropped
// (hardware range check), which lets masked lanes use an out-of-range offset
// instead of a branch.  The third descriptor word is the gfx9-family raw-buffer
// format word.
constexpr unsigned kBufOutOfRange = 0xF0000000u;  // buffers must stay below 256 MB

template <typename T>
struct Buf {
  __amdgpu_buffer_rsrc_t rs;
  __device__ __forceinline__ static Buf make(const void* p, size_t bytes) {
    Buf b;
    b.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
    return b;
  }
  // voff: per-lane byte offset (range-checked); soff: wave-uniform byte offset
  // added to it (a channel plane); voff + soff must stay inside the buffer for
  // an in-range voff.
  __device__ __forceinline__ T load(unsigned voff, unsigned soff) const;
  __device__ __forceinline__ void store(unsigned voff, unsigned soff, T v) const;
};
template <>
__device__ __forceinline__ float Buf<float>::load(unsigned off, unsigned soff) const {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off, soff, 0));
}
template <>
__device__ __forceinline__ double Buf<double>::load(unsigned off, unsigned soff) const {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, soff, 0));
}
template <>
__device__ __forceinline__ uint8_t Buf<uint8_t>::load(unsigned off, unsigned soff) const {
  return __builtin_amdgcn_raw_buffer_load_b8(rs, off, soff, 0);
}
template <>
__device__ __forceinline__ void Buf<float>::store(unsigned off, unsigned soff, float v) const {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, off, soff, 0);
}
template <>
__device__ __forceinline__ void Buf<double>::store(unsigned off, unsigned soff, double v) const {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rs, off, soff, 0);
}

// K consecutive values at byte offset voff (+ soff) in one or two wide loads
// (each lane reads 4*K or 8*K contiguous bytes), and the matching store.
template <int K, typename T>
__device__ __forceinline__ void buf_loadv(const Buf<T>& b, unsigned voff, unsigned soff, T* out) {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  typedef unsigned u3 __attribute__((ext_vector_type(3)));
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  constexpr int W = (int)(K * sizeof(T) / 4);  // dwords
  static_assert(K * sizeof(T) % 4 == 0, "whole dwords");
  unsigned d[W];
  int i = 0;
#pragma unroll
  for (; i + 4 <= W; i += 4) {
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(b.rs, voff + 4 * i, soff, 0);
    d[i] = v.x; d[i + 1] = v.y; d[i + 2] = v.z; d[i + 3] = v.w;
  }
  if constexpr (W % 4 == 3) {
    const u3 v = __builtin_amdgcn_raw_buffer_load_b96(b.rs, voff + 4 * (W - 3), soff, 0);
    d[W - 3] = v.x; d[W - 2] = v.y; d[W - 1] = v.z;
  } else if constexpr (W % 4 == 2) {
    const u2 v = __builtin_amdgcn_raw_buffer_load_b64(b.rs, voff + 4 * (W - 2), soff, 0);
    d[W - 2] = v.x; d[W - 1] = v.y;
  } else if constexpr (W % 4 == 1) {
    d[W - 1] = __builtin_amdgcn_raw_buffer_load_b32(b.rs, voff + 4 * (W - 1), soff, 0);
  }
  (void)i;
  __builtin_memcpy(out, d, sizeof(d));
}

// AUX: the cache-policy bits of the store instruction (0: default).
template <int K, int AUX = 0, typename T>
__device__ __forceinline__ void buf_storev(const Buf<T>& b, unsigned voff, unsigned soff, const T* in) {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  typedef unsigned u3 __attribute__((ext_vector_type(3)));
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  constexpr int W = (int)(K * sizeof(T) / 4);
  unsigned d[W];
  __builtin_memcpy(d, in, sizeof(d));
  int i = 0;
#pragma unroll
  for (; i + 4 <= W; i += 4) {
    u4 v;
    v.x = d[i]; v.y = d[i + 1]; v.z = d[i + 2]; v.w = d[i + 3];
    __builtin_amdgcn_raw_buffer_store_b128(v, b.rs, voff + 4 * i, soff, AUX);
  }
  if constexpr (W % 4 == 3) {
    u3 v;
    v.x = d[W - 3]; v.y = d[W - 2]; v.z = d[W - 1];
    __builtin_amdgcn_raw_buffer_store_b96(v, b.rs, voff + 4 * (W - 3), soff, AUX);
  } else if constexpr (W % 4 == 2) {
    u2 v;
    v.x = d[W - 2]; v.y = d[W - 1];
    __builtin_amdgcn_raw_buffer_store_b64(v, b.rs, voff + 4 * (W - 2), soff, AUX);
  } else if constexpr (W % 4 == 1) {
    __builtin_amdgcn_raw_buffer_store_b32(d[W - 1], b.rs, voff + 4 * (W - 1), soff, AUX);
  }
  (void)i;
}

// Index of element (channel c, site s) of an internal vector of C channels:
// the channels of a site are adjacent, so one wide access reads a site.
template <int C>
__device__ __forceinline__ size_t vix(int c, int s) {
  return (size_t)s * C + c;
}

__device__ __forceinline__ void sincos_t(float v, float* s, float* c) { sincosf(v, s, c); }
__device__ __forceinline__ void sincos_t(double v, double* s, double* c) { sincos(v, s, c); }

}  // namespace optmi
