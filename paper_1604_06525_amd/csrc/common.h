// Device-side building blocks shared by all energies: launch geometry,
// deterministic FP64 block reductions, the device-resident solver scalars and
// the Jacobi preconditioner.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace optmi {

constexpr int kBlock = 256;      // threads per block (4 waves of 64)
constexpr int kWaves = kBlock / 64;
constexpr int kMaxBlocks = 1024; // cap on the grid of every site kernel; also the
                                 // length of each partial-sum buffer

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
  int32_t pad;
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

// Store the block's sum of v at out[blockIdx.x].
__device__ __forceinline__ void block_store(double v, double* out) {
  const double t = block_sum(v);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
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

__device__ __forceinline__ bool is_block_leader() { return blockIdx.x == 0 && threadIdx.x == 0; }

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
  __device__ __forceinline__ T minv(T d) const {
    if (!use) return T(1);
    const T den = lam != T(0) ? d + damp(d) : d;
    return den > T(0) ? T(1) / den : T(0);
  }
};

__device__ __forceinline__ bool finite_d(double v) { return v - v == 0.0; }

__device__ __forceinline__ void sincos_t(float v, float* s, float* c) { sincosf(v, s, c); }
__device__ __forceinline__ void sincos_t(double v, double* s, double* c) { sincos(v, s, c); }

}  // namespace optmi
