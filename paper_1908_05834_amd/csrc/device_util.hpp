// Device-side helpers: compensated sums and wave/block reductions (wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bchar {

constexpr int kWave = 64;

// Error-free transformation of a + b (Knuth's TwoSum): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Compensated accumulator: value = hi + lo, updated with TwoSum.
struct CSum {
  double hi = 0.0, lo = 0.0;
  __device__ __forceinline__ void add(double v) {
    double s, e;
    two_sum(hi, v, s, e);
    hi = s;
    lo += e;
  }
  __device__ __forceinline__ void add(const CSum& o) {
    add(o.hi);
    lo += o.lo;
  }
  __device__ __forceinline__ double value() const { return hi + lo; }
};

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ void wave_csum(CSum& c) {
  for (int o = kWave / 2; o > 0; o >>= 1) {
    CSum other;
    other.hi = __shfl_xor(c.hi, o, kWave);
    other.lo = __shfl_xor(c.lo, o, kWave);
    c.add(other);
  }
}

// Inclusive scan of an int across the wave (lane order).
__device__ __forceinline__ int wave_incl_scan_i(int v) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int o = 1; o < kWave; o <<= 1) {
    int t = __shfl_up(v, o, kWave);
    if (lane >= o) v += t;
  }
  return v;
}

// Block-wide sum (blockDim.x multiple of 64, <= 1024); result valid in all threads.
template <class T>
__device__ __forceinline__ T block_sum(T v, T* sh /* >= 16 entries */) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T r = 0;
  const int nw = blockDim.x / kWave;
  for (int i = 0; i < nw; ++i) r += sh[i];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  const int nw = blockDim.x / kWave;
  for (int i = 0; i < nw; ++i) r = fmax(r, sh[i]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ CSum block_csum(CSum c, double* sh /* >= 32 */) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  wave_csum(c);
  __syncthreads();
  if (lane == 0) {
    sh[2 * w] = c.hi;
    sh[2 * w + 1] = c.lo;
  }
  __syncthreads();
  CSum r;
  const int nw = blockDim.x / kWave;
  for (int i = 0; i < nw; ++i) {
    CSum o;
    o.hi = sh[2 * i];
    o.lo = sh[2 * i + 1];
    r.add(o);
  }
  __syncthreads();
  return r;
}

}  // namespace bchar
