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

__global__ void k_active_flags(const uint8_t *__restrict__ level, int64_t n,
                               int nlev, const int64_t *__restrict__ kctr,
                               int k_add, const uint8_t *__restrict__ frozen,
                               uint32_t *__restrict__ flag) {
  const int64_t k = (kctr ? kctr[0] : 0) + k_add;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int l = min((int)level[i], nlev - 1);
    const bool on = (k % ((int64_t)1 << (nlev - 1 - l))) == 0 && !(frozen && frozen[i]);
    flag[i] = on ? 1u : 0u;
  }
}

__global__ void k_active_write(const uint32_t *__restrict__ flag,
                               const uint32_t *__restrict__ pos, int64_t n,
                               const uint32_t *__restrict__ total,
                               int32_t *__restrict__ idx,
                               int32_t *__restrict__ n_out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (flag[i]) idx[pos[i]] = (int32_t)i;
  if (blockIdx.x == 0 && threadIdx.x == 0) n_out[0] = (int32_t)total[0];
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

hipError_t launch_levels(tg_ctx *c, const double *acc, const double *vel,
                         const double *t4e2, const double *t2e2v, int64_t n,
                         const int32_t *idx, const int32_t *n_act, double dt_max, int nlev,
                         const int64_t *k, uint8_t *level) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_levels, dim3(grid_n(n)), dim3(256), 0, c->stream, acc, vel,
                     t4e2, t2e2v, n, idx, n_act, dt_max, nlev, k, level);
  return hipGetLastError();
}

// Flags and the scan share the context's active-group scratch, which is
// sized for max_particles entries.
hipError_t launch_active_set(tg_ctx *c, const uint8_t *level, int64_t n,
                             int nlev, const int64_t *k, int k_add,
                             int32_t *idx, int32_t *n_out, const uint8_t *frozen) {
  Buffers &b = c->b;
  if (n == 0) return fill_u32((uint32_t *)n_out, 0u, 1, c->stream);
  hipLaunchKernelGGL(k_active_flags, dim3(grid_n(n)), dim3(256), 0, c->stream,
                     level, n, nlev, k, k_add, frozen, b.wl_count);
  hipError_t e = scan_u32(b.wl_count, b.wl_off, (uint32_t)n, nullptr,
                          b.scan_total, b.scan_part, c->stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_active_write, dim3(grid_n(n)), dim3(256), 0, c->stream,
                     b.wl_count, b.wl_off, n, b.scan_total, idx, n_out);
  return hipGetLastError();
}

hipError_t launch_counter_add(tg_ctx *c, int64_t *k, int64_t inc) {
  hipLaunchKernelGGL(k_counter_add, dim3(1), dim3(64), 0, c->stream, k, inc);
  return hipGetLastError();
}

}  // namespace tg
