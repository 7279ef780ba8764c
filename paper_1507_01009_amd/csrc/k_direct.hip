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
// depend on the split beyond the last bit and is deterministic.  Every
// operation is rounded on its own (no FMA contraction): the TwoSum steps
// need it, and so does the fused drift-and-sum kernel, whose sums must equal
// the unfused ones bit for bit.
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
#pragma clang fp contract(off)
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
#pragma clang fp contract(off)
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
__device__ __forceinline__ void block_csum4(CSum r[4], double (*ss)[256], double (*sc)[256]) {
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
#pragma clang fp contract(off)
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

// The stars' drift fused with the SMBH <- star sums of a block substep
// (one system, at most kDriftSmbhMax SMBHs): block b drifts the stars
// [b kFewPerBlock, (b + 1) kFewPerBlock) (x <- x + v dt with the operations
// of k_drift; frozen stars stay) and sums their pull on every SMBH at the
// drifted positions with the ranges, thread order and block reduction of
// k_direct_few, so k_direct_reduce turns the partials into the same totals.
// The stars' positions are read once instead of twice.
constexpr int kDriftSmbhMax = 4;

template <int kNB>
__global__ __launch_bounds__(256) void k_drift_smbh(
    double *__restrict__ pos, const double *__restrict__ vel, const uint8_t *__restrict__ frozen,
    int64_t n, double dt, const double *__restrict__ sm, double seps,
    const double *__restrict__ bpos, const double *__restrict__ beps, int soft,
    double *__restrict__ part) {
#pragma clang fp contract(off)
  constexpr int nb = kNB;
  __shared__ double ss[4][256], sc[4][256];
  const int64_t j0 = (int64_t)blockIdx.x * kFewPerBlock;
  const int64_t j1 = min(n, j0 + kFewPerBlock);
  double bx[nb], by[nb], bz[nb], be[nb];
#pragma unroll
  for (int i = 0; i < nb; ++i) {
    bx[i] = bpos[3 * i]; by[i] = bpos[3 * i + 1]; bz[i] = bpos[3 * i + 2]; be[i] = beps[i];
  }
  CSum r[nb][4];
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) {
    double x = pos[3 * j], y = pos[3 * j + 1], z = pos[3 * j + 2];
    if (!(frozen && frozen[j])) {
      x = x + vel[3 * j] * dt;
      y = y + vel[3 * j + 1] * dt;
      z = z + vel[3 * j + 2] * dt;
      pos[3 * j] = x; pos[3 * j + 1] = y; pos[3 * j + 2] = z;
    }
    const double m = sm[j];
#pragma unroll
    for (int i = 0; i < nb; ++i) {
      const double ep = fmax(seps, be[i]);
      const double dx = bx[i] - x, dy = by[i] - y, dz = bz[i] - z;
      double mD1, mD3;
      pair_terms(dx, dy, dz, ep, m, soft, mD1, mD3);
      r[i][0].add(-mD3 * dx);
      r[i][1].add(-mD3 * dy);
      r[i][2].add(-mD3 * dz);
      r[i][3].add(-mD1);
    }
  }
  // static indices keep the sums in registers
#pragma unroll
  for (int i = 0; i < nb; ++i) {
    block_csum4(r[i], ss, sc);
    if (threadIdx.x == 0) {
      double *o = part + 8 * (size_t)(blockIdx.x * nb + i);
      for (int k = 0; k < 4; ++k) { o[2 * k] = ss[k][0]; o[2 * k + 1] = sc[k][0]; }
    }
    __syncthreads();
  }
}

// Whether sums of n sources on nt targets take the few-target path of
// launch_direct (part_cap doubles of partials; the star sums on the SMBHs
// that take it may be fused with the drift).
static bool few_path(int64_t part_cap, int64_t n, int64_t nt) {
  if (!(nt <= 4096 && n >= 2 * kFewPerBlock)) return false;
  const int64_t bpt = (n + kFewPerBlock - 1) / kFewPerBlock;
  return bpt * nt * 8 <= part_cap && bpt <= 65535;
}

bool drift_smbh_fits(const tg_ctx *c, int64_t n, int32_t nb) {
  return nb >= 1 && nb <= kDriftSmbhMax && few_path(c->b.dpart_cap, n, nb);
}

hipError_t launch_drift_smbh(tg_ctx *c, double *pos, const double *vel, const uint8_t *frozen,
                             int64_t n, double dt, const double *mass, double eps,
                             const double *bpos, const double *beps, int32_t nb,
                             double *bacc, double *bpot) {
  const int64_t bpt = (n + kFewPerBlock - 1) / kFewPerBlock;
  const dim3 g((unsigned)bpt), b(256);
  switch (nb) {
    case 1: hipLaunchKernelGGL(k_drift_smbh<1>, g, b, 0, c->stream, pos, vel, frozen, n, dt, mass,
                               eps, bpos, beps, c->soft, c->b.dpart); break;
    case 2: hipLaunchKernelGGL(k_drift_smbh<2>, g, b, 0, c->stream, pos, vel, frozen, n, dt, mass,
                               eps, bpos, beps, c->soft, c->b.dpart); break;
    case 3: hipLaunchKernelGGL(k_drift_smbh<3>, g, b, 0, c->stream, pos, vel, frozen, n, dt, mass,
                               eps, bpos, beps, c->soft, c->b.dpart); break;
    default: hipLaunchKernelGGL(k_drift_smbh<4>, g, b, 0, c->stream, pos, vel, frozen, n, dt, mass,
                                eps, bpos, beps, c->soft, c->b.dpart); break;
  }
  hipLaunchKernelGGL(k_direct_reduce, dim3((unsigned)std::min<int64_t>(nb, 4096)), dim3(256), 0,
                     c->stream, (int64_t)nb, (int)bpt, 0, c->b.dpart, bacc, bpot);
  return hipGetLastError();
}

hipError_t launch_direct_env(const DirectEnv &e, const int64_t *dseg, const double *spos,
                             const double *sm, const double *seps, double seps_all,
                             const double *tpos, const double *teps, int64_t nt, int nseg,
                             int64_t max_seg_src, int self_pairs, int accumulate,
                             double *acc, double *pot) {
  if (nt == 0) return hipSuccess;
  if (few_path(e.part_cap, max_seg_src, nt)) {
    const int64_t bpt = (max_seg_src + kFewPerBlock - 1) / kFewPerBlock;
    hipLaunchKernelGGL(k_direct_few, dim3((unsigned)bpt, (unsigned)nt), dim3(256), 0,
                       e.stream, spos, sm, seps, seps_all, tpos, teps, nt, dseg,
                       dseg + (nseg + 1), nseg, self_pairs, e.soft, e.part);
    hipLaunchKernelGGL(k_direct_reduce, dim3((unsigned)std::min<int64_t>(nt, 4096)),
                       dim3(256), 0, e.stream, nt, (int)bpt, accumulate, e.part, acc, pot);
    return hipGetLastError();
  }
  // aim for >= 2^16 independent (target, chunk) sums; with part_cap >= 2^19
  // doubles the partials of nt < 2^16 targets always fit at some chunk
  int64_t nchunks = 1, chunk = std::max<int64_t>(max_seg_src, 1);
  if (nt < 65536 && max_seg_src > 256) {
    int64_t want = (65536 + nt - 1) / nt;
    chunk = std::max<int64_t>(256, (max_seg_src + want - 1) / want);
    nchunks = (max_seg_src + chunk - 1) / chunk;
    while (nchunks > 1 && nchunks * nt * 8 > e.part_cap) {
      chunk *= 2;
      nchunks = (max_seg_src + chunk - 1) / chunk;
    }
  }
  const int64_t total = nt * nchunks;
  const int g = (int)std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_direct, dim3(g), dim3(256), 0, e.stream, spos, sm, seps,
                     seps_all, tpos, teps, nt, dseg, dseg + (nseg + 1), nseg,
                     chunk, (int)nchunks, self_pairs, accumulate, e.soft, acc, pot,
                     e.part);
  if (nchunks > 1) {
    const int g2 = (int)std::min<int64_t>(nt, 4096);
    hipLaunchKernelGGL(k_direct_reduce, dim3(g2), dim3(256), 0, e.stream, nt,
                       (int)nchunks, accumulate, e.part, acc, pot);
  }
  return hipGetLastError();
}

hipError_t launch_direct(tg_ctx *c, const int64_t *dseg, const double *spos,
                         const double *sm, const double *seps, double seps_all,
                         int64_t ns, const double *tpos,
                         const double *teps, int64_t nt, int nseg,
                         int64_t max_seg_src, int self_pairs, int accumulate,
                         double *acc, double *pot) {
  (void)ns;
  const DirectEnv e{c->stream, c->soft, c->b.dpart, c->b.dpart_cap};
  return launch_direct_env(e, dseg, spos, sm, seps, seps_all, tpos, teps, nt, nseg,
                           max_seg_src, self_pairs, accumulate, acc, pot);
}

}  // namespace tg
