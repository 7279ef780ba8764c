// Kick-drift-kick leapfrog and power-of-two block time-steps.
//
// Element-wise double arithmetic with no contraction, in the order of the
// plain definition, so kick, drift and level decisions are bit-identical to
// any correct implementation fed the same inputs:
//   kick   v <- v + a h,  h = dt/2, or h = (dt_max 2^-level)/2 per particle
//   drift  x <- x + v dt
//   level  smallest l with (dt_l^2)^2 |a|^2 <= (tau^2)^2 eps^2, |a|^2 summed
//          x, y, z in order; then raised so that the step divides k
//   active (k mod 2^(nlev-1-level)) == 0
// Counts and the substep k are read from device memory, so a whole step can
// be captured once and replayed.
#include "tg_internal.h"

namespace tg {

__global__ void k_kick(double *__restrict__ vel, const double *__restrict__ acc,
                       int64_t n, const int32_t *__restrict__ idx,
                       const int32_t *__restrict__ n_act,
                       const uint8_t *__restrict__ level, double dt,
                       const int64_t *__restrict__ kctr, int skip_k0,
                       const uint8_t *__restrict__ frozen) {
#pragma clang fp contract(off)
  if (skip_k0 && kctr && kctr[0] == 0) return;
  const int64_t m = idx ? min((int64_t)n_act[0], n) : n;
  const double h0 = dt * 0.5;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx ? (int64_t)idx[t] : t;
    if (i < 0 || i >= n || (frozen && frozen[i])) continue;
    const double h = level ? ldexp(dt, -(int)level[i]) * 0.5 : h0;
    vel[3 * i + 0] = vel[3 * i + 0] + acc[3 * i + 0] * h;
    vel[3 * i + 1] = vel[3 * i + 1] + acc[3 * i + 1] * h;
    vel[3 * i + 2] = vel[3 * i + 2] + acc[3 * i + 2] * h;
  }
}

__global__ void k_drift(double *__restrict__ pos, const double *__restrict__ vel,
                        int64_t n3, double dt, const uint8_t *__restrict__ frozen) {
#pragma clang fp contract(off)
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!frozen || !frozen[i / 3]) pos[i] = pos[i] + vel[i] * dt;
}

// The half kicks of a whole KDK step in one pass over the stars and then
// the SMBHs, the opening one followed by the drift (the operations of
// k_kick and k_drift, in that order, per particle): v <- v + a dt/2, and
// with drift set x <- x + v dt.
__device__ __forceinline__ void kick_drift_one(double *__restrict__ x, double *__restrict__ v,
                                               const double *__restrict__ a, double h, double dt,
                                               int drift) {
#pragma clang fp contract(off)
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double vk = v[k] + a[k] * h;
    v[k] = vk;
    if (drift) x[k] = x[k] + vk * dt;
  }
}

__global__ void k_kick_drift(double *__restrict__ pos, double *__restrict__ vel,
                             const double *__restrict__ acc, const uint8_t *__restrict__ frozen,
                             int64_t n, double *__restrict__ bpos, double *__restrict__ bvel,
                             const double *__restrict__ bacc, int64_t nb, double dt, int drift) {
#pragma clang fp contract(off)
  const double h = dt * 0.5;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n + nb;
       t += (int64_t)gridDim.x * blockDim.x) {
    if (t < n) {
      if (!(frozen && frozen[t])) kick_drift_one(pos + 3 * t, vel + 3 * t, acc + 3 * t, h, dt, drift);
    } else {
      const int64_t i = t - n;
      kick_drift_one(bpos + 3 * i, bvel + 3 * i, bacc + 3 * i, h, dt, drift);
    }
  }
}

__device__ __forceinline__ int lmin_at(int64_t k, int nlev) {
  int l = 0;
  while (l < nlev - 1 && (k % ((int64_t)1 << (nlev - 1 - l))) != 0) ++l;
  return l;
}

__global__ void k_levels(const double *__restrict__ acc,
                         const double *__restrict__ vel,
                         const double *__restrict__ t4e2,
                         const double *__restrict__ t2e2v, int64_t n,
                         const int32_t *__restrict__ idx,
                         const int32_t *__restrict__ n_act, double dt_max,
                         int nlev, const int64_t *__restrict__ kctr,
                         uint8_t *__restrict__ level) {
#pragma clang fp contract(off)
  const int64_t m = idx ? min((int64_t)n_act[0], n) : n;
  const int lmin = lmin_at(kctr ? kctr[0] : 0, nlev);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx ? (int64_t)idx[t] : t;
    if (i < 0 || i >= n) continue;
    const double ax = acc[3 * i], ay = acc[3 * i + 1], az = acc[3 * i + 2];
    const double a2 = ax * ax + ay * ay + az * az;
    double v2 = 0.0;
    if (vel) {
      const double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
      v2 = vx * vx + vy * vy + vz * vz;
    }
    int l = nlev - 1;
    for (int c = 0; c < nlev; ++c) {
      const double dl = ldexp(dt_max, -c);
      const double d2 = dl * dl;
      if (d2 * d2 * a2 <= t4e2[i] && (!vel || d2 * v2 <= t2e2v[i])) { l = c; break; }
    }
    level[i] = (uint8_t)(l < lmin ? lmin : l);
  }
}

constexpr int kActItems = 4;                      // stars per thread and tile
constexpr int kActTile = 256 * kActItems;          // stars per active-set tile

__device__ __forceinline__ bool on_at(int l, int64_t k, int nlev) {
  return (k & (((int64_t)1 << (nlev - 1 - l)) - 1)) == 0;
}

// One 1024-star tile per block: the number of active stars at substep
// k + k_add, and the finest level held by a star that is not frozen (+1, 0
// for none), packed as count | (level + 1) << 16.
__global__ __launch_bounds__(256) void k_active_count(const uint8_t *__restrict__ level,
                                                      int64_t n, int nlev,
                                                      const int64_t *__restrict__ kctr,
                                                      int k_add,
                                                      const uint8_t *__restrict__ frozen,
                                                      uint32_t *__restrict__ tcount) {
  __shared__ uint32_t lds[8];
  const int64_t k = (kctr ? kctr[0] : 0) + k_add;
  const int64_t base = (int64_t)blockIdx.x * kActTile;
  uint32_t cnt = 0, top = 0;
#pragma unroll
  for (int r = 0; r < kActItems; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    if (i < n && !(frozen && frozen[i])) {
      const int l = min((int)level[i], nlev - 1);
      cnt += on_at(l, k, nlev) ? 1u : 0u;
      top = max(top, (uint32_t)l + 1u);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    cnt += (uint32_t)__shfl_xor((int)cnt, o, 64);
    top = max(top, (uint32_t)__shfl_xor((int)top, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    lds[threadIdx.x >> 6] = cnt;
    lds[4 + (threadIdx.x >> 6)] = top;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    tcount[blockIdx.x] = (lds[0] + lds[1] + lds[2] + lds[3]) |
                         (max(max(lds[4], lds[5]), max(lds[6], lds[7])) << 16);
}

// One block: exclusive offsets of the tiles' counts (toff[0..tiles]), the
// total into n_out and info[0], the finest occupied level into info[1]
// (-1 when no star is free to move).
__global__ __launch_bounds__(1024) void k_active_offsets(const uint32_t *__restrict__ tcount,
                                                         int64_t tiles,
                                                         uint32_t *__restrict__ toff,
                                                         int32_t *__restrict__ n_out,
                                                         int32_t *__restrict__ info) {
  __shared__ uint32_t sh[16];
  __shared__ uint32_t top_sh[16];
  uint32_t base = 0, top = 0;
  for (int64_t t0 = 0; t0 < tiles; t0 += 1024) {
    const int64_t t = t0 + threadIdx.x;
    const uint32_t w = t < tiles ? tcount[t] : 0u;
    top = max(top, w >> 16);
    uint32_t tot;
    const uint32_t e = block_exclusive_scan(w & 0xFFFFu, sh, tot);
    if (t < tiles) toff[t] = base + e;
    base += tot;
  }
  for (int o = 32; o > 0; o >>= 1) top = max(top, (uint32_t)__shfl_xor((int)top, o, 64));
  if ((threadIdx.x & 63) == 0) top_sh[threadIdx.x >> 6] = top;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = 0;
    for (int w = 0; w < 16; ++w) m = max(m, top_sh[w]);
    toff[tiles] = base;
    n_out[0] = (int32_t)base;
    info[0] = (int32_t)base;
    info[1] = (int32_t)m - 1;
  }
}

// One tile per block: the tile's active stars in ascending order at its
// offset (wave ballots, then the four waves in order).  Empty tiles return.
__global__ __launch_bounds__(256) void k_active_emit(const uint8_t *__restrict__ level,
                                                     int64_t n, int nlev,
                                                     const int64_t *__restrict__ kctr,
                                                     int k_add,
                                                     const uint8_t *__restrict__ frozen,
                                                     const uint32_t *__restrict__ toff,
                                                     int32_t *__restrict__ idx) {
  __shared__ uint32_t wtot[4];
  uint32_t off = toff[blockIdx.x];
  if (toff[blockIdx.x + 1] == off) return;
  const int64_t k = (kctr ? kctr[0] : 0) + k_add;
  const int64_t base = (int64_t)blockIdx.x * kActTile;
  const unsigned w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int r = 0; r < kActItems; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    const bool s = i < n && !(frozen && frozen[i]) && on_at(min((int)level[i], nlev - 1), k, nlev);
    const unsigned long long m = __ballot(s);
    __syncthreads();
    if (lane == 0) wtot[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t pre = 0;
    for (unsigned v = 0; v < w; ++v) pre += wtot[v];
    if (s) idx[off + pre + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = (int32_t)i;
    off += wtot[0] + wtot[1] + wtot[2] + wtot[3];
  }
}

// The SMBHs' part of one block substep (they sit on the finest level):
// closing half kick (not at k = 0), opening half kick, drift, all with the
// finest step and the same separately rounded operations as k_kick and
// k_drift; then the substep counter advances.  A non-null n_act is set to 0
// (a substep known to have no active star).
__global__ __launch_bounds__(64) void k_bh_substep(double *__restrict__ pos,
                                                   double *__restrict__ vel,
                                                   const double *__restrict__ acc, int n,
                                                   double dt, int64_t *__restrict__ kctr,
                                                   int32_t *__restrict__ n_act) {
#pragma clang fp contract(off)
  const int64_t k = kctr[0];
  const double h = dt * 0.5;
  for (int b = threadIdx.x; b < n; b += blockDim.x) {
    for (int d = 0; d < 3; ++d) {
      double v = vel[3 * b + d];
      const double a = acc[3 * b + d];
      if (k != 0) v = v + a * h;
      v = v + a * h;
      vel[3 * b + d] = v;
      pos[3 * b + d] = pos[3 * b + d] + v * dt;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    kctr[0] = k + 1;
    if (n_act) n_act[0] = 0;
  }
}

__global__ void k_counter_add(int64_t *k, int64_t inc) {
  if (threadIdx.x == 0) k[0] += inc;
}

static inline int grid_n(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}

hipError_t launch_kick(tg_ctx *c, double *vel, const double *acc, int64_t n,
                       const int32_t *idx, const int32_t *n_act,
                       const uint8_t *level, double dt, const int64_t *k,
                       int skip_k0, const uint8_t *frozen) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_kick, dim3(grid_n(n)), dim3(256), 0, c->stream, vel, acc,
                     n, idx, n_act, level, dt, k, skip_k0, frozen);
  return hipGetLastError();
}

hipError_t launch_drift(tg_ctx *c, double *pos, const double *vel, int64_t n,
                        double dt, const uint8_t *frozen) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_drift, dim3(grid_n(3 * n)), dim3(256), 0, c->stream, pos,
                     vel, 3 * n, dt, frozen);
  return hipGetLastError();
}

hipError_t launch_kick_drift(tg_ctx *c, double *pos, double *vel, const double *acc,
                             const uint8_t *frozen, int64_t n, double *bpos, double *bvel,
                             const double *bacc, int64_t nb, double dt, bool drift) {
  if (n + nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_kick_drift, dim3(grid_n(n + nb)), dim3(256), 0, c->stream, pos, vel,
                     acc, frozen, n, bpos, bvel, bacc, nb, dt, drift ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_levels(tg_ctx *c, const double *acc, const double *vel,
                         const double *t4e2, const double *t2e2v, int64_t n,
                         const int32_t *idx, const int32_t *n_act, double dt_max, int nlev,
                         const int64_t *k, uint8_t *level) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_levels, dim3(grid_n(n)), dim3(256), 0, c->stream, acc, vel,
                     t4e2, t2e2v, n, idx, n_act, dt_max, nlev, k, level);
  return hipGetLastError();
}

// Count, offsets, emit: three launches whose shape depends only on n.
hipError_t launch_active_set(tg_ctx *c, const uint8_t *level, int64_t n,
                             int nlev, const int64_t *k, int k_add,
                             int32_t *idx, int32_t *n_out, const uint8_t *frozen) {
  Buffers &b = c->b;
  const int64_t tiles = (n + kActTile - 1) / kActTile;
  if (n > 0) {
    hipLaunchKernelGGL(k_active_count, dim3((unsigned)tiles), dim3(256), 0, c->stream, level, n,
                       nlev, k, k_add, frozen, b.atile);
  }
  hipLaunchKernelGGL(k_active_offsets, dim3(1), dim3(1024), 0, c->stream, b.atile, tiles,
                     b.aoff, n_out, b.ainfo);
  if (n > 0) {
    hipLaunchKernelGGL(k_active_emit, dim3((unsigned)tiles), dim3(256), 0, c->stream, level, n,
                       nlev, k, k_add, frozen, b.aoff, idx);
  }
  return hipGetLastError();
}

hipError_t launch_bh_substep(tg_ctx *c, double *pos, double *vel, const double *acc, int32_t n,
                             double dt, int64_t *k, int32_t *n_act) {
  hipLaunchKernelGGL(k_bh_substep, dim3(1), dim3(64), 0, c->stream, pos, vel, acc, n, dt, k,
                     n_act);
  return hipGetLastError();
}

hipError_t launch_counter_add(tg_ctx *c, int64_t *k, int64_t inc) {
  hipLaunchKernelGGL(k_counter_add, dim3(1), dim3(64), 0, c->stream, k, inc);
  return hipGetLastError();
}

}  // namespace tg
