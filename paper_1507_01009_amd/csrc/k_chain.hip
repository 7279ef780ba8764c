// Coupling between the tree particles and the regularised chain (Sec. 2, the
// hybrid method): selection of the perturbers by the tidal criterion (Eq. 2),
// selection by radius (the chain start around an SMBH, absorption Eq. 4), and
// the forces the two parts exert on each other.
//
// Selection.  One pass flags every particle (FP64, each operation rounded on
// its own, so the decision equals the plain definition bit for bit):
//   tidal:  (r2 r2) r2 < (k k) rc6,  k = c m_j,  c = 2 / (gamma_crit M_chain),
//           rc6 = r_crit^6 (Eq. 2 cubed and squared: no roots),
//   radius: r2 < r r,
// with r2 = (dx dx + dy dy) + dz dz about the centre; an exclusion mask
// (ghost members) clears flags.  The flags are scanned and the indices of
// the flagged particles scattered in ascending order (stable, so the list
// is unique); a list beyond its capacity sets TG_ERR_CHAIN.  The pass is
// bound by HBM: 32 B read per particle (position, mass) and 4 B of flags.
//
// Forces (pairs with the chain are Newtonian; perturber-member pairs may be
// Plummer-softened with eps_pm):
//   stars:  each listed, non-excluded star adds the point force of the chain
//           particle (mass M at the centre of mass R), or, if it is a
//           perturber, the forces of the resolved members (members in LDS,
//           summed in member order);
//   chain particle: the point force at R of every non-perturber,
//           non-excluded star (compensated sums over a fixed grid, then an
//           ordered pass) plus the Eq. 3 correction (1 / M) sum_i m_i a_i;
//   members: a_i = force of the perturbers on member i (one block each,
//           compensated), returned for the chain integration.
#include "tg_internal.h"

namespace tg {

constexpr int kChainBlocks = 256;   // partial sums of the chain particle's force

template <bool kTidal>
__global__ __launch_bounds__(256) void k_chain_flags(const double *__restrict__ pos,
                                                     const double *__restrict__ mass, int64_t n,
                                                     const uint8_t *__restrict__ excl, double cx,
                                                     double cy, double cz, double c, double lim,
                                                     uint32_t *__restrict__ flag) {
#pragma clang fp contract(off)
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double dx = __dsub_rn(pos[3 * i], cx);
    const double dy = __dsub_rn(pos[3 * i + 1], cy);
    const double dz = __dsub_rn(pos[3 * i + 2], cz);
    const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    bool s;
    if constexpr (kTidal) {
      const double k = __dmul_rn(c, mass[i]);
      s = __dmul_rn(__dmul_rn(r2, r2), r2) < __dmul_rn(__dmul_rn(k, k), lim);
    } else {
      s = r2 < lim;
    }
    if (excl && excl[i]) s = false;
    flag[i] = s ? 1u : 0u;
  }
}

__global__ __launch_bounds__(256) void k_chain_compact(const uint32_t *__restrict__ flag,
                                                       const uint32_t *__restrict__ off, int64_t n,
                                                       const uint32_t *__restrict__ total,
                                                       int32_t *__restrict__ idx, int32_t cap,
                                                       int32_t *__restrict__ n_out,
                                                       uint32_t *__restrict__ err) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (flag[i] && off[i] < (uint32_t)cap) idx[off[i]] = (int32_t)i;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint32_t t = *total;
    *n_out = (int32_t)t;
    if (t > (uint32_t)cap) atomicOr(err, TG_ERR_CHAIN);
  }
}

// Force and potential of one source (xs, m) at target (xt): accumulate
// m (xs - xt) / (r^2 + e2)^(3/2) and -m / (r^2 + e2)^(1/2).
__device__ __forceinline__ void chain_pair(double sx, double sy, double sz, double m, double tx,
                                           double ty, double tz, double e2, double &ax,
                                           double &ay, double &az, double &ph) {
  const double dx = sx - tx, dy = sy - ty, dz = sz - tz;
  const double r2 = dx * dx + dy * dy + dz * dz + e2;
  const double D1 = 1.0 / sqrt(r2);
  const double mD1 = m * D1, mD3 = mD1 * D1 * D1;
  ax += mD3 * dx; ay += mD3 * dy; az += mD3 * dz; ph -= mD1;
}

__global__ __launch_bounds__(256) void k_chain_stars(
    const int32_t *__restrict__ idx, const int32_t *__restrict__ n_act, int64_t n,
    const double *__restrict__ pos, const uint8_t *__restrict__ excl,
    const uint32_t *__restrict__ pflag, const double *__restrict__ mpos,
    const double *__restrict__ mmass, int nc, double Rx, double Ry, double Rz, double M,
    double e2pm, double G, double *__restrict__ acc, double *__restrict__ pot) {
  __shared__ double s_m[4 * kMaxChain];
  for (int i = threadIdx.x; i < nc; i += blockDim.x) {
    s_m[4 * i] = mpos[3 * i]; s_m[4 * i + 1] = mpos[3 * i + 1];
    s_m[4 * i + 2] = mpos[3 * i + 2]; s_m[4 * i + 3] = mmass[i];
  }
  __syncthreads();
  const int64_t m = idx ? min((int64_t)max(n_act[0], 0), n) : n;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = idx ? (int64_t)idx[k] : k;
    if (j < 0 || j >= n || (excl && excl[j])) continue;
    const double x = pos[3 * j], y = pos[3 * j + 1], z = pos[3 * j + 2];
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    if (pflag[j]) {
      for (int i = 0; i < nc; ++i)
        chain_pair(s_m[4 * i], s_m[4 * i + 1], s_m[4 * i + 2], s_m[4 * i + 3], x, y, z, e2pm,
                   ax, ay, az, ph);
    } else {
      chain_pair(Rx, Ry, Rz, M, x, y, z, 0.0, ax, ay, az, ph);
    }
    acc[3 * j] += G * ax; acc[3 * j + 1] += G * ay; acc[3 * j + 2] += G * az;
    if (pot) pot[j] += G * ph;
  }
}

// Fixed-order tree reduction of three compensated sums over the block.
__device__ void block_csum3(CSum &a, CSum &b, CSum &c, double *lds) {
  const int t = threadIdx.x;
  lds[6 * t] = a.s; lds[6 * t + 1] = a.c; lds[6 * t + 2] = b.s;
  lds[6 * t + 3] = b.c; lds[6 * t + 4] = c.s; lds[6 * t + 5] = c.c;
  __syncthreads();
  for (int h = blockDim.x >> 1; h > 0; h >>= 1) {
    if (t < h) {
      CSum x, y, z, o;
      x.s = lds[6 * t]; x.c = lds[6 * t + 1];
      y.s = lds[6 * t + 2]; y.c = lds[6 * t + 3];
      z.s = lds[6 * t + 4]; z.c = lds[6 * t + 5];
      o.s = lds[6 * (t + h)]; o.c = lds[6 * (t + h) + 1]; x.merge(o);
      o.s = lds[6 * (t + h) + 2]; o.c = lds[6 * (t + h) + 3]; y.merge(o);
      o.s = lds[6 * (t + h) + 4]; o.c = lds[6 * (t + h) + 5]; z.merge(o);
      lds[6 * t] = x.s; lds[6 * t + 1] = x.c; lds[6 * t + 2] = y.s;
      lds[6 * t + 3] = y.c; lds[6 * t + 4] = z.s; lds[6 * t + 5] = z.c;
    }
    __syncthreads();
  }
  a.s = lds[0]; a.c = lds[1]; b.s = lds[2]; b.c = lds[3]; c.s = lds[4]; c.c = lds[5];
}

__global__ __launch_bounds__(256) void k_chain_com_part(
    const double *__restrict__ pos, const double *__restrict__ mass, int64_t n,
    const uint8_t *__restrict__ excl, const uint32_t *__restrict__ pflag, double Rx, double Ry,
    double Rz, double *__restrict__ part) {
  __shared__ double lds[6 * 256];
  CSum sx, sy, sz;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    if (pflag[j] || (excl && excl[j])) continue;
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    chain_pair(pos[3 * j], pos[3 * j + 1], pos[3 * j + 2], mass[j], Rx, Ry, Rz, 0.0, ax, ay,
               az, ph);
    sx.add(ax); sy.add(ay); sz.add(az);
  }
  block_csum3(sx, sy, sz, lds);
  if (threadIdx.x == 0) {
    double *o = part + 6 * (size_t)blockIdx.x;
    o[0] = sx.s; o[1] = sx.c; o[2] = sy.s; o[3] = sy.c; o[4] = sz.s; o[5] = sz.c;
  }
}

__global__ __launch_bounds__(256) void k_chain_members(
    const double *__restrict__ mpos, const int32_t *__restrict__ pidx,
    const int32_t *__restrict__ n_pert, int32_t cap, const double *__restrict__ pos,
    const double *__restrict__ mass, double e2pm, double G, double *__restrict__ macc) {
  __shared__ double lds[6 * 256];
  const int i = blockIdx.x;
  const double x = mpos[3 * i], y = mpos[3 * i + 1], z = mpos[3 * i + 2];
  const int np = min(max(n_pert[0], 0), cap);
  CSum sx, sy, sz;
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    const int64_t j = pidx[p];
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    chain_pair(pos[3 * j], pos[3 * j + 1], pos[3 * j + 2], mass[j], x, y, z, e2pm, ax, ay, az,
               ph);
    sx.add(ax); sy.add(ay); sz.add(az);
  }
  block_csum3(sx, sy, sz, lds);
  if (threadIdx.x == 0) {
    macc[3 * i] = G * sx.get(); macc[3 * i + 1] = G * sy.get(); macc[3 * i + 2] = G * sz.get();
  }
}

// The chain particle: ordered sum of the block partials, then Eq. 3.
__global__ void k_chain_com_final(const double *__restrict__ part, int nb,
                                  const double *__restrict__ macc,
                                  const double *__restrict__ mmass, int nc, double M, double G,
                                  double *__restrict__ com_acc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  CSum s[3], q[3];
  for (int b = 0; b < nb; ++b)
    for (int k = 0; k < 3; ++k) {
      CSum o;
      o.s = part[6 * b + 2 * k]; o.c = part[6 * b + 2 * k + 1];
      s[k].merge(o);
    }
  for (int i = 0; i < nc; ++i)
    for (int k = 0; k < 3; ++k) q[k].add(mmass[i] * macc[3 * i + k]);
  for (int k = 0; k < 3; ++k) com_acc[k] = G * s[k].get() + q[k].get() / M;
}

static int grid_for(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}

hipError_t launch_chain_select(tg_ctx *c, const double *pos, const double *mass, int64_t n,
                               const uint8_t *excl, const double center[3], bool tidal,
                               double cst, double lim, int32_t *idx, int32_t cap,
                               int32_t *n_out) {
  Buffers &b = c->b;
  if (tidal)
    hipLaunchKernelGGL(k_chain_flags<true>, dim3(grid_for(n)), dim3(256), 0, c->stream, pos,
                       mass, n, excl, center[0], center[1], center[2], cst, lim, b.cflag);
  else
    hipLaunchKernelGGL(k_chain_flags<false>, dim3(grid_for(n)), dim3(256), 0, c->stream, pos,
                       mass, n, excl, center[0], center[1], center[2], cst, lim, b.cflag);
  hipError_t e = scan_u32(b.cflag, b.coff, (uint32_t)n, nullptr, b.scan_total, b.scan_part,
                          c->stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chain_compact, dim3(grid_for(n)), dim3(256), 0, c->stream, b.cflag,
                     b.coff, n, b.scan_total, idx, cap, n_out, b.err);
  return hipGetLastError();
}

hipError_t launch_chain_forces(tg_ctx *c, const tg_chain *ch, const int32_t *idx,
                               const int32_t *n_act, double *acc, double *pot,
                               double *com_acc, double *member_acc) {
  Buffers &b = c->b;
  const double G = c->cfg.G;
  const double e2pm = ch->eps_pm * ch->eps_pm;
  const int64_t n = ch->n;
  if (n > 0 && acc) {
    // the grid covers all n; with a list the kernel reads its device count
    hipLaunchKernelGGL(k_chain_stars, dim3(grid_for(n)), dim3(256), 0, c->stream, idx, n_act,
                       n, ch->pos, ch->exclude, b.cflag, ch->member_pos, ch->member_mass,
                       ch->nc, ch->com[0], ch->com[1], ch->com[2], ch->m_chain, e2pm, G, acc,
                       pot);
  }
  hipLaunchKernelGGL(k_chain_com_part, dim3(kChainBlocks), dim3(256), 0, c->stream, ch->pos,
                     ch->mass, n, ch->exclude, b.cflag, ch->com[0], ch->com[1], ch->com[2],
                     b.cpart);
  hipLaunchKernelGGL(k_chain_members, dim3(ch->nc), dim3(256), 0, c->stream, ch->member_pos,
                     ch->pert_idx, ch->n_pert, ch->pert_cap, ch->pos, ch->mass, e2pm, G,
                     member_acc);
  hipLaunchKernelGGL(k_chain_com_final, dim3(1), dim3(64), 0, c->stream, b.cpart,
                     kChainBlocks, member_acc, ch->member_mass, ch->nc, ch->m_chain, G,
                     com_acc);
  return hipGetLastError();
}

}  // namespace tg
