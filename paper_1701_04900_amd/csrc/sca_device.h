// Device helpers for the gfx950 kernels of libsca: 16-byte vector types, Philox4x32-10,
// wave64 reductions and a 1024-thread block scan.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sca {

// ------------------------------------------------------------------ vector types
template <typename T> struct V16;
template <> struct V16<float> {
  typedef float v __attribute__((ext_vector_type(4)));
  static constexpr int N = 4;
};
template <> struct V16<double> {
  typedef double v __attribute__((ext_vector_type(2)));
  static constexpr int N = 2;
};

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw (SC'11): ten rounds; each multiplies counter words 0 and 2
// by fixed odd constants, xors the high halves with words 1/3 and the key, and bumps
// the key by the Weyl constants.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c[0];
    const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Block i is drawn in round k when Philox word 0 < T (T >= 2^32: always).
__device__ __forceinline__ bool block_drawn(uint32_t i, uint64_t k, uint32_t inst, uint64_t seed,
                                            uint64_t T) {
  if (T >= (1ull << 32)) return true;
  uint32_t c[4] = {i, (uint32_t)(k & 0xffffffffu), (uint32_t)(k >> 32), inst};
  philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  return (uint64_t)c[0] < T;
}

// ------------------------------------------------------------------ reductions
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
template <typename T> __device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Number of set bits of 'mask' strictly below this lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Workgroups are dispatched to the chip's 8 XCDs round robin (workgroup w to XCD w % 8), and
// each XCD has an L2 of its own.  xcd_order(w, W) is a position in [0, W) such that the
// workgroups of one XCD take one contiguous range of positions: workgroups whose positions
// are neighbours (and that read neighbouring data) then share an L2.  A bijection of [0, W).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_order(int w, int W) {
  const int x = w % kXcds, q = w / kXcds;
  return x * (W / kXcds) + min(x, W % kXcds) + q;
}

// Exclusive scan over a 1024-thread block (16 waves); returns the prefix, *total = sum.
// 'sh' needs 17 ints of shared memory.  Contains __syncthreads.
__device__ __forceinline__ int block_exclusive_scan_1024(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < 16; ++w) {
      const int t = sh[w];
      sh[w] = run;
      run += t;
    }
    sh[16] = run;
  }
  __syncthreads();
  const int res = sh[wave] + inc - v;
  *total = sh[16];
  __syncthreads();
  return res;
}

}  // namespace sca
