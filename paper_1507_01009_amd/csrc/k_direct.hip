// Double-precision direct forces between a source set and a target set
// (SMBH <-> stars; perturber <-> chain-member corrections), softening
// max(eps_i, eps_j) per pair: Plummer, or the cubic spline with that h.
//
// Many targets (stars feeling the SMBHs): one thread per target takes every
// source of its segment (or of a source chunk, combined in a second ordered
// pass when targets are too few to fill the chip).  Few targets (SMBHs
// feeling a million stars): one 256-thread block per (target, range of
// kFewPerBlock sources), threads striding through the range with coalesced
// loads, the block's sums combined in a fixed tree order and the per-block
// partials summed in a second ordered pass.  Every sum is compensated
// (error-free TwoSum with a running correction), so the result does not
// depend on the split beyond the last bit and is deterministic.
#include "tg_internal.h"

namespace tg {

__device__ __forceinline__ int seg_of(const int64_t *off, int nseg, int64_t i) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// m/r and m/r^3 with the pair's softening ep (soft: cubic spline, h = ep).
__device__ __forceinline__ void pair_terms(double dx, double dy, double dz, double ep, double m,
                                           int soft, double &mD1, double &mD3) {
  if (soft) {
    double p0, p1;
    spline_pair_dp(sqrt(dx * dx + dy * dy + dz * dz), ep, p0, p1);
    mD1 = m * p0;
    mD3 = m * p1;
  } else {
    const double r2 = dx * dx + dy * dy + dz * dz + ep * ep;
    const double D1 = 1.0 / sqrt(r2);
    mD1 = m * D1;
    mD3 = mD1 * D1 * D1;
  }
}

__global__ void k_direct(const double *__restrict__ spos, const double *__restrict__ sm,
                         const double *__restrict__ seps, double seps_all,
                         const double *__restrict__ tpos,
                         const double *__restrict__ teps, int64_t nt,
                         const int64_t *__restrict__ sseg, const int64_t *__restrict__ tseg,
                         int nseg, int64_t chunk, int nchunks, int self_pairs,
                         int accumulate, int soft, double *__restrict__ acc,
                         double *__restrict__ pot, double *__restrict__ part) {
  const int64_t total = nt * (int64_t)nchunks;
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < total;
       w += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = w % nt;
    const int c = (int)(w / nt);
    const int s = seg_of(tseg, nseg, i);
    const int64_t j0 = sseg[s] + (int64_t)c * chunk;
    const int64_t j1 = min(sseg[s + 1], j0 + chunk);
    const double xi = tpos[3 * i], yi = tpos[3 * i + 1], zi = tpos[3 * i + 2];
    const double ei = teps[i];
    CSum ax, ay, az, ph;
    for (int64_t j = j0; j < j1; ++j) {
      if (self_pairs && j == i) continue;
      const double ep = fmax(seps ? seps[j] : seps_all, ei);
      const double dx = xi - spos[3 * j], dy = yi - spos[3 * j + 1], dz = zi - spos[3 * j + 2];
      double mD1, mD3;
      pair_terms(dx, dy, dz, ep, sm[j], soft, mD1, mD3);
      ax.add(-mD3 * dx);
      ay.add(-mD3 * dy);
      az.add(-mD3 * dz);
      ph.add(-mD1);
    }
    if (nchunks == 1) {
      double a0 = ax.get(), a1 = ay.get(), a2 = az.get(), p = ph.get();
      if (accumulate) {
        acc[3 * i] += a0; acc[3 * i + 1] += a1; acc[3 * i + 2] += a2;
        if (pot) pot[i] += p;
      } else {
        acc[3 * i] = a0; acc[3 * i + 1] = a1; acc[3 * i + 2] = a2;
        if (pot) pot[i] = p;
      }
    } else {
      double *o = part + 8 * (size_t)w;
      o[0] = ax.s; o[1] = ax.c; o[2] = ay.s; o[3] = ay.c;
      o[4] = az.s; o[5] = az.c; o[6] = ph.s; o[7] = ph.c;
    }
  }
}

// Compensated sums of a 256-thread block combined in a fixed tree order;
// thread 0 returns with the totals in ss[k][0] + sc[k][0].
__device__ void block_csum4(CSum r[4], double (*ss)[256], double (*sc)[256]) {
  for (int k = 0; k < 4; ++k) { ss[k][threadIdx.x] = r[k].s; sc[k][threadIdx.x] = r[k].c; }
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      for (int k = 0; k < 4; ++k) {
        CSum x;
        x.s = ss[k][threadIdx.x];
        x.c = sc[k][threadIdx.x] + sc[k][threadIdx.x + h];
        x.add(ss[k][threadIdx.x + h]);
        ss[k][threadIdx.x] = x.s;
        sc[k][threadIdx.x] = x.c;
      }
    }
    __syncthreads();
  }
}

constexpr int kFewPerBlock = 4096;   // sources per block in the few-target path

// grid (blocks per target, targets): block b of target i sums sources
// [b kFewPerBlock, (b + 1) kFewPerBlock) of i's segment into part[b nt + i].
__global__ __launch_bounds__(256) void k_direct_few(
    const double *__restrict__ spos, const double *__restrict__ sm,
    const double *__restrict__ seps, double seps_all, const double *__restrict__ tpos,
    const double *__restrict__ teps, int64_t nt, const int64_t *__restrict__ sseg,
    const int64_t *__restrict__ tseg, int nseg, int self_pairs, int soft,
    double *__restrict__ part) {
  __shared__ double ss[4][256], sc[4][256];
  const int64_t i = blockIdx.y;
  const int s = seg_of(tseg, nseg, i);
  const int64_t j0 = sseg[s] + (int64_t)blockIdx.x * kFewPerBlock;
  const int64_t j1 = min(sseg[s + 1], j0 + kFewPerBlock);
  const double xi = tpos[3 * i], yi = tpos[3 * i + 1], zi = tpos[3 * i + 2];
  const double ei = teps[i];
  CSum r[4];
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) {
    if (self_pairs && j == i) continue;
    const double ep = fmax(seps ? seps[j] : seps_all, ei);
    const double dx = xi - spos[3 * j], dy = yi - spos[3 * j + 1], dz = zi - spos[3 * j + 2];
    double mD1, mD3;
    pair_terms(dx, dy, dz, ep, sm[j], soft, mD1, mD3);
    r[0].add(-mD3 * dx);
    r[1].add(-mD3 * dy);
    r[2].add(-mD3 * dz);
    r[3].add(-mD1);
  }
  block_csum4(r, ss, sc);
  if (threadIdx.x == 0) {
    double *o = part + 8 * (size_t)(blockIdx.x * nt + i);
    for (int k = 0; k < 4; ++k) { o[2 * k] = ss[k][0]; o[2 * k + 1] = sc[k][0]; }
  }
}

// One block per target: each thread sums a strided subset of the chunks,
// then the block combines the compensated pairs in a fixed tree order.
__global__ __launch_bounds__(256) void k_direct_reduce(int64_t nt, int nchunks,
                                                       int accumulate,
                                                       const double *__restrict__ part,
                                                       double *__restrict__ acc,
                                                       double *__restrict__ pot) {
  __shared__ double ss[4][256], sc[4][256];
  for (int64_t i = blockIdx.x; i < nt; i += gridDim.x) {
    CSum r[4];
    for (int c = threadIdx.x; c < nchunks; c += 256) {
      const double *o = part + 8 * (size_t)(c * nt + i);
      for (int k = 0; k < 4; ++k) {
        r[k].add(o[2 * k]);
        r[k].add(o[2 * k + 1]);
      }
    }
    block_csum4(r, ss, sc);
    if (threadIdx.x == 0) {
      const double v0 = ss[0][0] + sc[0][0], v1 = ss[1][0] + sc[1][0];
      const double v2 = ss[2][0] + sc[2][0], v3 = ss[3][0] + sc[3][0];
      if (accumulate) {
        acc[3 * i] += v0; acc[3 * i + 1] += v1; acc[3 * i + 2] += v2;
        if (pot) pot[i] += v3;
      } else {
        acc[3 * i] = v0; acc[3 * i + 1] = v1; acc[3 * i + 2] = v2;
        if (pot) pot[i] = v3;
      }
    }
    __syncthreads();
  }
}

hipError_t launch_direct(tg_ctx *c, const int64_t *dseg, const double *spos,
                         const double *sm, const double *seps, double seps_all,
                         int64_t ns, const double *tpos,
                         const double *teps, int64_t nt, int nseg,
                         int64_t max_seg_src, int self_pairs, int accumulate,
                         double *acc, double *pot) {
  (void)ns;
  if (nt == 0) return hipSuccess;
  if (nt <= 4096 && max_seg_src >= 2 * kFewPerBlock) {
    const int64_t bpt = (max_seg_src + kFewPerBlock - 1) / kFewPerBlock;
    if (bpt * nt * 8 <= c->b.dpart_cap && bpt <= 65535) {
      hipLaunchKernelGGL(k_direct_few, dim3((unsigned)bpt, (unsigned)nt), dim3(256), 0,
                         c->stream, spos, sm, seps, seps_all, tpos, teps, nt, dseg,
                         dseg + (nseg + 1), nseg, self_pairs, c->soft, c->b.dpart);
      hipLaunchKernelGGL(k_direct_reduce, dim3((unsigned)std::min<int64_t>(nt, 4096)),
                         dim3(256), 0, c->stream, nt, (int)bpt, accumulate, c->b.dpart,
                         acc, pot);
      return hipGetLastError();
    }
  }
  // aim for >= 2^16 independent (target, chunk) sums
  int64_t nchunks = 1, chunk = std::max<int64_t>(max_seg_src, 1);
  if (nt < 65536 && max_seg_src > 256) {
    int64_t want = (65536 + nt - 1) / nt;
    chunk = std::max<int64_t>(256, (max_seg_src + want - 1) / want);
    nchunks = (max_seg_src + chunk - 1) / chunk;
    while (nchunks * nt * 8 > c->b.dpart_cap) {
      chunk *= 2;
      nchunks = (max_seg_src + chunk - 1) / chunk;
    }
  }
  const int64_t total = nt * nchunks;
  const int g = (int)std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_direct, dim3(g), dim3(256), 0, c->stream, spos, sm, seps,
                     seps_all, tpos, teps, nt, dseg, dseg + (nseg + 1), nseg,
                     chunk, (int)nchunks, self_pairs, accumulate, c->soft, acc, pot,
                     c->b.dpart);
  if (nchunks > 1) {
    const int g2 = (int)std::min<int64_t>(nt, 4096);
    hipLaunchKernelGGL(k_direct_reduce, dim3(g2), dim3(256), 0, c->stream, nt,
                       (int)nchunks, accumulate, c->b.dpart, acc, pot);
  }
  return hipGetLastError();
}

}  // namespace tg
