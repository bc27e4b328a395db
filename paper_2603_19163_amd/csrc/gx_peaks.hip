// gx_peaks.hip -- device ceilings the evolve kernels are measured against:
// a random-address LDS gather, the Philox4x32-10 block rate of the per-lane
// form the candidate draws use, the full-rate 32-bit VALU issue rate, a
// random-address gather from a buffer that fits the L2, and an HBM read
// stream.  Each kernel is timed with HIP events on the context's stream; the
// work per launch is fixed, so every access stays inside its buffer and
// every loop has a constant trip count.
#include "../../include/gx.h"
#include "gx_internal.hpp"

#include <vector>

namespace {

constexpr int kPeakThreads = 256;
constexpr int kLdsWords = 16384;   // 64 KiB of LDS per workgroup

__device__ __forceinline__ uint32_t lcg(uint32_t x) { return x * 1664525u + 1013904223u; }

// every lane: 8 independent streams of random 4-byte LDS reads
__global__ __launch_bounds__(kPeakThreads) void k_peak_lds(uint32_t iters, uint32_t *sink) {
  __shared__ uint32_t t[kLdsWords];
  for (int i = threadIdx.x; i < kLdsWords; i += kPeakThreads) t[i] = i * 2654435761u;
  __syncthreads();
  uint32_t x[8], acc = 0;
#pragma unroll
  for (int s = 0; s < 8; ++s) x[s] = (blockIdx.x * kPeakThreads + threadIdx.x) * 8u + s;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      x[s] = lcg(x[s]);
      acc += t[x[s] >> 18];   // 14-bit index
    }
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;   // keeps the reads
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

// Philox4x32-10 blocks with per-lane counters and a uniform key, 4 streams per lane
__global__ __launch_bounds__(kPeakThreads) void k_peak_philox(uint32_t iters, uint32_t k0i, uint32_t k1i, uint32_t *sink) {
  const uint32_t lane = blockIdx.x * kPeakThreads + threadIdx.x;
  uint32_t acc = 0;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      uint32_t c0 = it, c1 = lane, c2 = (uint32_t)s, c3 = lane ^ it, k0 = k0i, k1 = k1i;
#pragma unroll
      for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        c0 = xor3(hi1, c1, k0);
        c1 = lo1;
        c2 = xor3(hi0, c3, k1);
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
      }
      acc ^= c0 ^ c1 ^ c2 ^ c3;
    }
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

// full-rate 32-bit integer multiply-adds (24-bit operands), 16 independent chains
__global__ __launch_bounds__(kPeakThreads) void k_peak_valu(uint32_t iters, uint32_t *sink) {
  uint32_t a[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) a[s] = threadIdx.x + s;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int s = 0; s < 16; ++s) a[s] = __umul24(a[s], 3u) + (uint32_t)s;
  }
  uint32_t acc = 0;
#pragma unroll
  for (int s = 0; s < 16; ++s) acc ^= a[s];
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

// random 4-byte loads from a buffer of `mask + 1` words (a power of two that fits the L2)
__global__ __launch_bounds__(kPeakThreads) void k_peak_l2(const uint32_t *__restrict__ buf, uint32_t mask, uint32_t iters,
                                                          uint32_t *sink) {
  uint32_t x[8], acc = 0;
#pragma unroll
  for (int s = 0; s < 8; ++s) x[s] = (blockIdx.x * kPeakThreads + threadIdx.x) * 8u + s;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      x[s] = lcg(x[s]);
      acc += buf[(x[s] >> 8) & mask];
    }
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

// 16-byte loads over the whole buffer (grid-stride), summed
__global__ __launch_bounds__(kPeakThreads) void k_peak_hbm(const uint4 *__restrict__ buf, size_t n16, uint32_t *sink) {
  uint32_t acc = 0;
  const size_t stride = (size_t)gridDim.x * kPeakThreads;
  for (size_t i = (size_t)blockIdx.x * kPeakThreads + threadIdx.x; i < n16; i += stride) {
    const uint4 v = buf[i];
    acc += v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

__global__ void k_fill(uint32_t *buf, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) buf[i] = (uint32_t)(i * 2654435761u);
}

}  // namespace

namespace gxk {

hipError_t measure_peaks(int cus, hipStream_t s, gx_peaks *out) {
  uint32_t *sink = nullptr, *l2buf = nullptr;
  uint4 *hbm = nullptr;
  const size_t l2_words = size_t(1) << 20;            // 4 MiB
  const size_t hbm_bytes = size_t(2) << 30;           // 2 GiB
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipSuccess;
  auto timed = [&](auto launch, int reps) -> double {   // seconds per launch, best of reps after a warm-up
    double best = 1e30;
    for (int r = 0; r < reps + 1; ++r) {
      (void)hipEventRecord(e0, s);
      launch();
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (r > 0 && ms * 1e-3 < best) best = ms * 1e-3;
    }
    return best;
  };
  if ((err = hipMalloc(&sink, 64)) == hipSuccess && (err = hipMalloc(&l2buf, l2_words * 4)) == hipSuccess &&
      (err = hipMalloc(&hbm, hbm_bytes)) == hipSuccess && (err = hipEventCreate(&e0)) == hipSuccess &&
      (err = hipEventCreate(&e1)) == hipSuccess) {
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((l2_words + 255) / 256)), dim3(256), 0, s, l2buf, l2_words);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((hbm_bytes / 4 + 255) / 256)), dim3(256), 0, s, (uint32_t *)hbm,
                       hbm_bytes / 4);
    const unsigned grid = (unsigned)cus * 8;          // 8 workgroups of 256 threads per CU
    const double lanes = (double)grid * kPeakThreads;
    const uint32_t it_lds = 4096, it_ph = 256, it_valu = 65536, it_l2 = 1024;
    double t = timed([&] { hipLaunchKernelGGL(k_peak_lds, dim3(grid), dim3(kPeakThreads), 0, s, it_lds, sink); }, 3);
    out->lds_gather_bytes_per_s = lanes * it_lds * 8 * 4 / t;
    t = timed([&] { hipLaunchKernelGGL(k_peak_philox, dim3(grid), dim3(kPeakThreads), 0, s, it_ph, 42u, 7u, sink); }, 3);
    out->philox_blocks_per_s = lanes * it_ph * 4 / t;
    t = timed([&] { hipLaunchKernelGGL(k_peak_valu, dim3(grid), dim3(kPeakThreads), 0, s, it_valu, sink); }, 3);
    out->valu_lane_ops_per_s = lanes * it_valu * 16 * 2 / t;   // a multiply and an add per step
    out->valu_instr_per_s = lanes * it_valu * 16 / t;          // one v_mad_u32_u24 per step and lane
    t = timed([&] {
      hipLaunchKernelGGL(k_peak_l2, dim3(grid), dim3(kPeakThreads), 0, s, l2buf, (uint32_t)(l2_words - 1), it_l2, sink);
    }, 3);
    out->l2_gather_bytes_per_s = lanes * it_l2 * 8 * 4 / t;
    t = timed([&] {
      hipLaunchKernelGGL(k_peak_hbm, dim3((unsigned)cus * 32), dim3(kPeakThreads), 0, s, hbm, hbm_bytes / 16, sink);
    }, 3);
    out->hbm_read_bytes_per_s = hbm_bytes / t;
    out->cus = cus;
    err = hipStreamSynchronize(s);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  (void)hipFree(l2buf);
  (void)hipFree(hbm);
  return err;
}

}  // namespace gxk
