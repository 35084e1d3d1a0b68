// Exclusive scans of the library (hand-written, three passes), shared by the
// kernels and the packed-layout builder.
#pragma once
#include "gtp_device.h"

namespace gtp {

// Exclusive scan, three passes: per tile (kScanTile items) local scan and
// total; scan of tile totals by one workgroup; add the tile prefix.
struct OpAdd {
  template <class T>
  __device__ __forceinline__ T operator()(T a, T b) const { return a + b; }
};
struct OpXor {
  template <class T>
  __device__ __forceinline__ T operator()(T a, T b) const { return a ^ b; }
};

template <class T, class Op>
__device__ __forceinline__ T block_exclusive(T v, T ident, Op op, T* sh, T& total) {
  // Hillis-Steele over kScanThreads values in LDS
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    T x = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : ident;
    __syncthreads();
    if (threadIdx.x >= (unsigned)off) sh[threadIdx.x] = op(x, sh[threadIdx.x]);
    __syncthreads();
  }
  const T excl = threadIdx.x == 0 ? ident : sh[threadIdx.x - 1];
  total = sh[kScanThreads - 1];
  __syncthreads();
  return excl;
}

template <class T, class Op>
__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const T* in, T* out, T* sums, int64_t n, T ident, Op op) {
  __shared__ T sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T loc[kScanItems];
  T acc = ident;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const T x = (base + k < n) ? in[base + k] : ident;
    loc[k] = acc;
    acc = op(acc, x);
  }
  T total;
  const T pre = block_exclusive(acc, ident, op, sh, total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) out[base + k] = op(pre, loc[k]);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <class T, class Op>
__global__ void __launch_bounds__(kScanThreads) k_scan_sums(T* sums, int64_t n, T ident, Op op) {
  __shared__ T sh[kScanThreads];
  T carry = ident;
  for (int64_t base0 = 0; base0 < n; base0 += kScanTile) {
    const int64_t base = base0 + (int64_t)threadIdx.x * kScanItems;
    T loc[kScanItems];
    T acc = ident;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const T x = (base + k < n) ? sums[base + k] : ident;
      loc[k] = acc;
      acc = op(acc, x);
    }
    T total;
    const T pre = block_exclusive(acc, ident, op, sh, total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
      if (base + k < n) sums[base + k] = op(carry, op(pre, loc[k]));
    carry = op(carry, total);
    __syncthreads();
  }
}

template <class T, class Op>
__global__ void __launch_bounds__(256) k_scan_add(T* out, const T* sums, int64_t n, Op op) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = op(sums[i / kScanTile], out[i]);
}

}  // namespace gtp
