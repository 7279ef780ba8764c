// Device-wide exclusive scan of u32 (reduce-then-scan over a fixed grid, so
// the element count may live in device memory and the launch shape never
// depends on it), and fill kernels used instead of memset so that every
// sequence of calls can be captured into a HIP graph.
#include "tg_internal.h"

namespace tg {

__device__ __forceinline__ void chunk_of(uint32_t n, uint32_t &a, uint32_t &b) {
  uint32_t chunk = ((n + gridDim.x - 1) / gridDim.x + 255u) & ~255u;
  a = min(n, blockIdx.x * chunk);
  b = min(n, a + chunk);
}

// A block's chunk is taken kScanSub elements at a time, kScanItems per
// thread, all loads of a sub-chunk in flight at once.
constexpr uint32_t kScanItems = 16;
constexpr uint32_t kScanSub = 256 * kScanItems;

__global__ __launch_bounds__(256) void k_scan_part(const int32_t *__restrict__ gate, const uint32_t *in,
                                                   uint32_t n_host,
                                                   const uint32_t *n_dev,
                                                   uint32_t *part) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  __shared__ uint32_t sh[4];
  uint32_t n = n_dev ? *n_dev : n_host;
  uint32_t a, b;
  chunk_of(n, a, b);
  uint32_t s = 0;
  for (uint32_t t0 = a; t0 < b; t0 += kScanSub) {
#pragma unroll
    for (uint32_t j = 0; j < kScanItems; ++j) {
      const uint32_t i = t0 + 256u * j + threadIdx.x;
      s += i < b ? in[i] : 0u;
    }
  }
  uint32_t tot;
  block_exclusive_scan(s, sh, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Each block first scans the blocks' partial sums itself (there are as many
// as a block has threads) for its own offset; block 0 also stores the total.
// A sub-chunk is read into LDS with coalesced loads, each thread scans a
// contiguous run of kScanItems there, one block scan of the run totals
// places the runs, and the results leave through LDS with coalesced
// stores.  in and out may be the same array: a sub-chunk is read whole
// before any of it is written, and blocks own disjoint chunks.
static_assert(kScanBlocks <= 256, "one partial sum per thread");

__device__ __forceinline__ uint32_t scan_pad(uint32_t p) { return p + (p >> 5); }

__global__ __launch_bounds__(256) void k_scan_final(const int32_t *__restrict__ gate, const uint32_t *in,
                                                    uint32_t *out,
                                                    uint32_t n_host,
                                                    const uint32_t *n_dev,
                                                    const uint32_t *part, uint32_t *total) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  __shared__ uint32_t sh[4];
  __shared__ uint32_t s_base;
  __shared__ uint32_t buf[kScanSub + kScanSub / 32];
  const uint32_t tid = threadIdx.x;
  uint32_t n = n_dev ? *n_dev : n_host;
  uint32_t a, b;
  chunk_of(n, a, b);
  {
    const uint32_t v = tid < gridDim.x ? part[tid] : 0u;
    uint32_t tot;
    const uint32_t e = block_exclusive_scan(v, sh, tot);
    if (tid == blockIdx.x) s_base = e;
    if (blockIdx.x == 0 && tid == 0 && total) *total = tot;
    __syncthreads();
  }
  uint32_t base = s_base;
  for (uint32_t t0 = a; t0 < b; t0 += kScanSub) {
    const uint32_t m = min(kScanSub, b - t0);
#pragma unroll
    for (uint32_t j = 0; j < kScanItems; ++j) {
      const uint32_t p = 256u * j + tid;
      buf[scan_pad(p)] = p < m ? in[t0 + p] : 0u;
    }
    __syncthreads();
    uint32_t run[kScanItems], sum = 0;
#pragma unroll
    for (uint32_t j = 0; j < kScanItems; ++j) {
      run[j] = buf[scan_pad(kScanItems * tid + j)];
      sum += run[j];
    }
    uint32_t tot;
    uint32_t e = base + block_exclusive_scan(sum, sh, tot);
#pragma unroll
    for (uint32_t j = 0; j < kScanItems; ++j) {
      buf[scan_pad(kScanItems * tid + j)] = e;
      e += run[j];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kScanItems; ++j) {
      const uint32_t p = 256u * j + tid;
      if (p < m) out[t0 + p] = buf[scan_pad(p)];
    }
    base += tot;
    __syncthreads();                // the sub-chunk is written out before the next is read in
  }
}

hipError_t scan_u32(const uint32_t *in, uint32_t *out, uint32_t n_host,
                    const uint32_t *n_dev, uint32_t *total_dev, uint32_t *part,
                    hipStream_t s, const int32_t *gate) {
  hipLaunchKernelGGL(k_scan_part, dim3(kScanBlocks), dim3(256), 0, s, gate, in,
                     n_host, n_dev, part);
  hipLaunchKernelGGL(k_scan_final, dim3(kScanBlocks), dim3(256), 0, s, gate, in,
                     out, n_host, n_dev, part, total_dev);
  return hipGetLastError();
}

__global__ void k_fill_u32(const int32_t *__restrict__ gate, uint32_t *p, uint32_t v, int64_t n) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u8(const int32_t *__restrict__ gate, uint8_t *p, uint8_t v, int64_t n) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static inline int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (int)g;
}

hipError_t fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s, const int32_t *gate) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, gate, p, v,
                     n);
  return hipGetLastError();
}

hipError_t fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s, const int32_t *gate) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n, 256)), dim3(256), 0, s, gate, p, v,
                     n);
  return hipGetLastError();
}

}  // namespace tg
