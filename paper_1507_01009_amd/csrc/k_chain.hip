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
// (ghost members) clears flags.  Tiles of 1024 particles count their flags;
// a second pass gives each tile the sum of the earlier counts and scatters
// the flagged indices in ascending order (stable, so the list is unique); a
// list beyond its capacity sets TG_ERR_CHAIN.  Both passes are bound by HBM:
// 33 B read per particle (position, mass, exclusion) and 1 B of flags
// written, then the flags read once more.
//
// Forces (pairs with the chain are Newtonian; perturber-member pairs may be
// Plummer-softened with eps_pm):
//   stars:  each listed, non-excluded star adds the point force of the chain
//           particle (mass M at the centre of mass R), or, if it is a
//           perturber, the forces of the resolved members (members in LDS,
//           summed in member order);
//   chain particle: the point force at R of every non-perturber,
//           non-excluded star (compensated sums over a fixed grid, combined
//           in a fixed tree order) plus the Eq. 3 correction
//           (1 / M) sum_i m_i a_i;
//   members: a_i = force of the perturbers on member i (one block each,
//           compensated), returned for the chain integration.
// Prediction: the listed perturbers relative to the chain particle, moved
// to first order in time (the chain integration evaluates them at many
// sub-step times), gathered into compact arrays.
#include "tg_internal.h"

namespace tg {

constexpr int kSelItems = 4;                        // elements per thread and tile
constexpr int kSelTile = 256 * kSelItems;            // elements per selection tile

// Block sum of one value per thread (256 threads); every thread gets it.
__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t *lds) {
  for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  return lds[0] + lds[1] + lds[2] + lds[3];
}

// One tile per block: flag each element (1 byte) and count the tile.
template <bool kTidal>
__global__ __launch_bounds__(256) void k_chain_flags(const double *__restrict__ pos,
                                                     const double *__restrict__ mass, int64_t n,
                                                     const uint8_t *__restrict__ excl, double cx,
                                                     double cy, double cz, double c, double lim,
                                                     uint8_t *__restrict__ flag,
                                                     uint32_t *__restrict__ tcount) {
#pragma clang fp contract(off)
  __shared__ uint32_t lds[4];
  const int64_t base = (int64_t)blockIdx.x * kSelTile;
  uint32_t cnt = 0;
#pragma unroll 4
  for (int r = 0; r < kSelItems; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    if (i >= n) break;
    const double dx = dsub(pos[3 * i], cx);
    const double dy = dsub(pos[3 * i + 1], cy);
    const double dz = dsub(pos[3 * i + 2], cz);
    const double r2 = dadd(dadd(dmul(dx, dx), dmul(dy, dy)), dmul(dz, dz));
    bool s;
    if constexpr (kTidal) {
      const double k = dmul(c, mass[i]);
      s = dmul(dmul(r2, r2), r2) < dmul(dmul(k, k), lim);
    } else {
      s = r2 < lim;
    }
    if (excl && excl[i]) s = false;
    flag[i] = s ? 1 : 0;
    cnt += s ? 1u : 0u;
  }
  cnt = block_sum_u32(cnt, lds);
  if (threadIdx.x == 0) tcount[blockIdx.x] = cnt;
}

// One tile per block: its offset is the sum of the earlier tiles' counts;
// ranks inside the tile follow element order (wave ballots, then the four
// waves in order), so the list is ascending.  The last tile writes the total.
__global__ __launch_bounds__(256) void k_chain_compact(const uint8_t *__restrict__ flag,
                                                       const uint32_t *__restrict__ tcount,
                                                       int64_t n, int32_t *__restrict__ idx,
                                                       int32_t cap, int32_t *__restrict__ n_out,
                                                       uint32_t *__restrict__ err) {
  __shared__ uint32_t lds[4];
  __shared__ uint32_t wtot[4];
  uint32_t before = 0;
  for (uint32_t u = threadIdx.x; u < blockIdx.x; u += 256) before += tcount[u];
  uint32_t off = block_sum_u32(before, lds);
  const int64_t base = (int64_t)blockIdx.x * kSelTile;
  const unsigned w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int r = 0; r < kSelItems; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    const bool s = i < n && flag[i];
    const unsigned long long m = __ballot(s);
    __syncthreads();
    if (lane == 0) wtot[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t pre = 0;
    for (unsigned v = 0; v < w; ++v) pre += wtot[v];
    const uint32_t rank = off + pre + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    if (s && rank < (uint32_t)cap) idx[rank] = (int32_t)i;
    off += wtot[0] + wtot[1] + wtot[2] + wtot[3];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    *n_out = (int32_t)off;
    if (off > (uint32_t)cap) atomicOr(err, TG_ERR_CHAIN);
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
    const uint8_t *__restrict__ pflag, const double *__restrict__ mpos,
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
    const uint8_t *__restrict__ excl, const uint8_t *__restrict__ pflag, double Rx, double Ry,
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
    const int32_t *__restrict__ n_pert, int32_t cap, int64_t n, const double *__restrict__ pos,
    const double *__restrict__ mass, double e2pm, double G, double *__restrict__ macc) {
  __shared__ double lds[6 * 256];
  const int i = blockIdx.x;
  const double x = mpos[3 * i], y = mpos[3 * i + 1], z = mpos[3 * i + 2];
  const int np = min(max(n_pert[0], 0), cap);
  CSum sx, sy, sz;
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    const int64_t j = pidx[p];
    if (j < 0 || j >= n) continue;   // the list is this call's, so always in range
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

// The chain particle: the block partials in a fixed tree order (each thread
// first merges kChainBlocks / 256 of them in block order), then Eq. 3.
__global__ __launch_bounds__(256) void k_chain_com_final(const double *__restrict__ part,
                                                         const double *__restrict__ macc,
                                                         const double *__restrict__ mmass,
                                                         int nc, double M, double G,
                                                         double *__restrict__ com_acc) {
  __shared__ double lds[6 * 256];
  CSum sx, sy, sz;
  for (int b = threadIdx.x * (kChainBlocks / 256); b < (threadIdx.x + 1) * (kChainBlocks / 256);
       ++b) {
    CSum o;
    o.s = part[6 * b]; o.c = part[6 * b + 1]; sx.merge(o);
    o.s = part[6 * b + 2]; o.c = part[6 * b + 3]; sy.merge(o);
    o.s = part[6 * b + 4]; o.c = part[6 * b + 5]; sz.merge(o);
  }
  block_csum3(sx, sy, sz, lds);
  if (threadIdx.x == 0) {
    CSum q[3];
    for (int i = 0; i < nc; ++i)
      for (int k = 0; k < 3; ++k) q[k].add(mmass[i] * macc[3 * i + k]);
    com_acc[0] = G * sx.get() + q[0].get() / M;
    com_acc[1] = G * sy.get() + q[1].get() / M;
    com_acc[2] = G * sz.get() + q[2].get() / M;
  }
}

// Perturbers relative to the chain particle, predicted to first order:
// x_rel = (x + v dt) - Rp, v_rel = v - V (Rp = R + V dt formed on the host).
__global__ __launch_bounds__(256) void k_chain_predict(
    const int32_t *__restrict__ pidx, const int32_t *__restrict__ n_pert, int32_t cap,
    int64_t n, const double *__restrict__ pos, const double *__restrict__ vel,
    const double *__restrict__ mass, double dt, double Rx, double Ry, double Rz, double Vx,
    double Vy, double Vz, double *__restrict__ out_pos, double *__restrict__ out_vel,
    double *__restrict__ out_mass) {
#pragma clang fp contract(off)
  const int np = min(max(n_pert[0], 0), cap);
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < np; k += gridDim.x * blockDim.x) {
    const int64_t j = pidx[k];
    if (j < 0 || j >= n) {   // a list not made for these stars: NaN rows
      const double nanv = __longlong_as_double(0x7ff8000000000000ll);
      for (int a = 0; a < 3; ++a) out_pos[3 * k + a] = out_vel[3 * k + a] = nanv;
      if (out_mass) out_mass[k] = nanv;
      continue;
    }
    const double R[3] = {Rx, Ry, Rz}, V[3] = {Vx, Vy, Vz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double x = pos[3 * j + a], v = vel[3 * j + a];
      out_pos[3 * k + a] = dsub(dadd(x, dmul(v, dt)), R[a]);
      out_vel[3 * k + a] = dsub(v, V[a]);
    }
    if (out_mass) out_mass[k] = mass[j];
  }
}

static int grid_for(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}

hipError_t launch_chain_select(tg_ctx *c, const double *pos, const double *mass, int64_t n,
                               const uint8_t *excl, const double center[3], bool tidal,
                               double cst, double lim, int32_t *idx, int32_t cap,
                               int32_t *n_out) {
  Buffers &b = c->b;
  const int tiles = (int)((n + kSelTile - 1) / kSelTile);
  if (tidal)
    hipLaunchKernelGGL(k_chain_flags<true>, dim3(tiles), dim3(256), 0, c->stream, pos, mass, n,
                       excl, center[0], center[1], center[2], cst, lim, b.cflag, b.ctile);
  else
    hipLaunchKernelGGL(k_chain_flags<false>, dim3(tiles), dim3(256), 0, c->stream, pos, mass, n,
                       excl, center[0], center[1], center[2], cst, lim, b.cflag, b.ctile);
  hipLaunchKernelGGL(k_chain_compact, dim3(tiles), dim3(256), 0, c->stream, b.cflag, b.ctile, n,
                     idx, cap, n_out, b.err);
  return hipGetLastError();
}

hipError_t launch_chain_predict(tg_ctx *c, const tg_chain *ch, const double *vel, double dt,
                                const double rp[3], const double v[3], double *out_pos,
                                double *out_vel, double *out_mass) {
  hipLaunchKernelGGL(k_chain_predict, dim3(grid_for(ch->pert_cap)), dim3(256), 0, c->stream,
                     ch->pert_idx, ch->n_pert, ch->pert_cap, ch->n, ch->pos, vel, ch->mass, dt, rp[0],
                     rp[1], rp[2], v[0], v[1], v[2], out_pos, out_vel, out_mass);
  return hipGetLastError();
}

// Several chains: out[k] += add.v[k] for k < n3 (the chain particles' mutual
// point-mass forces, formed on the host from the host centres of mass).
__global__ void k_add_host_vector(double *__restrict__ out, ChainVec add, int n3) {
  const int k = (int)threadIdx.x;
  if (k < n3) out[k] += add.v[k];
}

hipError_t launch_add_host_vector(tg_ctx *c, double *out, const ChainVec &add, int n3) {
  hipLaunchKernelGGL(k_add_host_vector, dim3(1), dim3(64), 0, c->stream, out, add, n3);
  return hipGetLastError();
}

// Rows of 3 doubles between a packed list and indexed rows of an array
// (the hybrid driver's members and ghosts): to_rows != 0: dst[idx[r]] =
// src[r], else dst[r] = src[idx[r]], for r < n.
__global__ void k_move_rows(double *__restrict__ dst, const double *__restrict__ src,
                            const int32_t *__restrict__ idx, int n, int to_rows) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const size_t a = 3 * (size_t)(to_rows ? idx[r] : r), b = 3 * (size_t)(to_rows ? r : idx[r]);
    dst[a] = src[b]; dst[a + 1] = src[b + 1]; dst[a + 2] = src[b + 2];
  }
}

// Per-row scalars and flags: mass[idx[r]] = val[r] and flag[idx[r]] = f[r].
__global__ void k_set_rows(double *__restrict__ mass, uint8_t *__restrict__ flag,
                           const int32_t *__restrict__ idx, const double *__restrict__ val,
                           const uint8_t *__restrict__ f, int n) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    mass[idx[r]] = val[r];
    flag[idx[r]] = f[r];
  }
}

// Bytes of listed rows: dst[r] = src[idx[r]] (levels of a few stars).
__global__ void k_gather_bytes(uint8_t *__restrict__ dst, const uint8_t *__restrict__ src,
                               const int32_t *__restrict__ idx, int n) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    dst[r] = src[idx[r]];
}

hipError_t launch_gather_bytes(tg_ctx *c, uint8_t *dst, const uint8_t *src, const int32_t *idx,
                               int n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_bytes, dim3((n + 255) / 256), dim3(256), 0, c->stream, dst, src,
                     idx, n);
  return hipGetLastError();
}

hipError_t launch_move_rows(tg_ctx *c, double *dst, const double *src, const int32_t *idx, int n,
                            bool to_rows) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_move_rows, dim3((n + 255) / 256), dim3(256), 0, c->stream, dst, src, idx, n,
                     to_rows ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_set_rows(tg_ctx *c, double *mass, uint8_t *flag, const int32_t *idx,
                           const double *val, const uint8_t *f, int n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_rows, dim3((n + 255) / 256), dim3(256), 0, c->stream, mass, flag, idx,
                     val, f, n);
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
                     ch->pert_idx, ch->n_pert, ch->pert_cap, ch->n, ch->pos, ch->mass, e2pm, G,
                     member_acc);
  hipLaunchKernelGGL(k_chain_com_final, dim3(1), dim3(256), 0, c->stream, b.cpart, member_acc,
                     ch->member_mass, ch->nc, ch->m_chain, G, com_acc);
  return hipGetLastError();
}

}  // namespace tg
