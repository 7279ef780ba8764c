// Monopole and quadrupole moments about each node's centre of mass (the
// multipole expansion of a distant group about its centre of mass).
//
// Leaves first, all in one launch: a leaf sums its particles in sorted
// order, two passes (mass and first moment, then the second moment about
// the centre of mass) with no contraction, so leaf moments equal the plain
// definition bit for bit.  Then internal nodes, one launch per level from
// 20 to 0, each combining its children with the parallel-axis theorem:
//   M = sum M_c,  com = (sum M_c com_c) / M,
//   S = sum (S_c + M_c d d^T),  d = com_c - com.
// The cell side s = L 2^-level (exact) is stored squared beside the centre
// of mass for the opening-angle test, and as the node's opening size.
//
// Refit (the tree is an earlier build, the particles have moved): the same
// passes also take each node's particle bounding box (exact min / max,
// leaves from their particles, internal nodes from their children) and the
// opening size becomes s' = max(s, 2 e), e the largest distance from the
// cell's geometric centre to the box: the smallest cube about the centre
// that holds the cell and all its particles.
#include "tg_internal.h"

namespace tg {

__global__ void k_mass_gather(const int32_t *__restrict__ gate, const double *__restrict__ mass,
                              const uint32_t *__restrict__ perm, int64_t n,
                              double4 *__restrict__ spart, uint32_t *err) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  bool bad = false;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    double m = mass[perm[r]];
    bad |= !(m > 0.0) || !isfinite(m);
    spart[r].w = m;
  }
  if (bad) set_err(err, TG_ERR_MASS);
}

// Opening size of node v: the cell side s, or with a refit its refitted
// size from the bounding box [lo, hi] (every operation rounded separately).
__device__ __forceinline__ double open_size(uint32_t v, int l, const uint32_t *first,
                                           const uint32_t *nsys, const uint64_t *skey,
                                           const double *cube, const double lo[3],
                                           const double hi[3], bool refit) {
  double g[3];
  const double s = cell_centre(v, l, first, nsys, skey, cube, g);
  if (!refit) return s;
  double e = 0.0;
  for (int k = 0; k < 3; ++k) e = fmax(fmax(e, dsub(hi[k], g[k])), dsub(g[k], lo[k]));
  return 2.0 * e > s ? 2.0 * e : s;
}

__device__ __forceinline__ void store_moments(uint32_t v, double s, double M, double cx,
                                              double cy, double cz, const double S[6],
                                              double4 *com, double *mom, double *side) {
  com[v] = make_double4(cx, cy, cz, dmul(s, s));
  side[v] = s;
  double *o = mom + 8 * (size_t)v;
  o[0] = M;
  for (int k = 0; k < 6; ++k) o[1 + k] = S[k];
  o[7] = 0.0;
}

// Every leaf of the tree (nodes without children), any level.  The first
// kLeafRegs particles of a leaf are loaded into registers at once, so both
// passes over them wait for memory once; particles beyond (over-full leaves
// of the deepest level, or leaves of a larger leaf size) are read in the
// passes.  The sums take the particles in the same order either way.
constexpr uint32_t kLeafRegs = 8;

template <bool kBox>
__global__ __launch_bounds__(256) void k_moments_leaves(const int32_t *__restrict__ gate,
    const TreeCounters *ctr, const double *__restrict__ cube,
    const uint8_t *__restrict__ level, const uint8_t *__restrict__ nchild,
    const uint32_t *__restrict__ first, const uint32_t *__restrict__ count,
    const uint32_t *__restrict__ nsys, const double4 *__restrict__ spart,
    const uint64_t *__restrict__ skey, const int32_t *__restrict__ refit,
    double4 *__restrict__ com, double *__restrict__ mom, double *__restrict__ side,
    double4 *__restrict__ bbox, uint32_t *err) {
#pragma clang fp contract(off)
  if (gate && *gate <= 0) return;   // nothing active: skipped
  const uint32_t nn = ctr->n_nodes;
  bool bad = false;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nn;
       v += gridDim.x * blockDim.x) {
    // every per-node read at once, before the leaf test
    const uint32_t nc = nchild[v], f = first[v], n = count[v];
    const int lv = level[v];
    const double cside = kBox ? 0.0 : cube[4 * nsys[v] + 3];
    if (nc != 0) continue;
    double4 pr[kLeafRegs];
#pragma unroll
    for (uint32_t q = 0; q < kLeafRegs; ++q)
      if (q < n) pr[q] = spart[f + q];
    // compensated sums: a leaf may hold any number of coincident particles
    CSum Mc, sxc, syc, szc;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    auto first_moments = [&](const double4 &p) {
      Mc.add(p.w);
      sxc.add(p.w * p.x);
      syc.add(p.w * p.y);
      szc.add(p.w * p.z);
      if constexpr (kBox) {
        lo[0] = fmin(lo[0], p.x); lo[1] = fmin(lo[1], p.y); lo[2] = fmin(lo[2], p.z);
        hi[0] = fmax(hi[0], p.x); hi[1] = fmax(hi[1], p.y); hi[2] = fmax(hi[2], p.z);
        bad |= !isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z);
      }
    };
#pragma unroll
    for (uint32_t q = 0; q < kLeafRegs; ++q)
      if (q < n) first_moments(pr[q]);
    for (uint32_t j = f + kLeafRegs; j < f + n; ++j) first_moments(spart[j]);
    const double M = Mc.get();
    const double cx = sxc.get() / M, cy = syc.get() / M, cz = szc.get() / M;
    CSum Sc[6];
    auto second_moments = [&](const double4 &p) {
      const double dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
      Sc[0].add(p.w * dx * dx); Sc[1].add(p.w * dy * dy); Sc[2].add(p.w * dz * dz);
      Sc[3].add(p.w * dx * dy); Sc[4].add(p.w * dx * dz); Sc[5].add(p.w * dy * dz);
    };
#pragma unroll
    for (uint32_t q = 0; q < kLeafRegs; ++q)
      if (q < n) second_moments(pr[q]);
    for (uint32_t j = f + kLeafRegs; j < f + n; ++j) second_moments(spart[j]);
    double S[6];
    for (int k = 0; k < 6; ++k) S[k] = Sc[k].get();
    double so;
    if constexpr (kBox) {
      bbox[2 * (size_t)v] = make_double4(lo[0], lo[1], lo[2], 0.0);
      bbox[2 * (size_t)v + 1] = make_double4(hi[0], hi[1], hi[2], 0.0);
      so = open_size(v, lv, first, nsys, skey, cube, lo, hi, *refit > 0);
    } else {
      so = ldexp(cside, -lv);
    }
    store_moments(v, so, M, cx, cy, cz, S, com, mom, side);
  }
  if (kBox && bad) set_err(err, TG_ERR_NONFINITE);
}

// Sum over the 8 lanes of an aligned lane octet (xor tree: deterministic).
__device__ __forceinline__ double oct_sum(double v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  return v;
}
__device__ __forceinline__ double oct_min(double v) {
  v = fmin(v, __shfl_xor(v, 1, 64));
  v = fmin(v, __shfl_xor(v, 2, 64));
  return fmin(v, __shfl_xor(v, 4, 64));
}
__device__ __forceinline__ double oct_max(double v) {
  v = fmax(v, __shfl_xor(v, 1, 64));
  v = fmax(v, __shfl_xor(v, 2, 64));
  return fmax(v, __shfl_xor(v, 4, 64));
}

// Internal nodes of level l from their children (level l + 1, done): eight
// lanes per node, lane k holding child k.
template <bool kBox>
__global__ __launch_bounds__(256) void k_moments_level(const int32_t *__restrict__ gate,
    int l, const TreeCounters *ctr, const double *__restrict__ cube,
    const uint8_t *__restrict__ nchild, const uint32_t *__restrict__ child,
    const uint32_t *__restrict__ nsys, const uint32_t *__restrict__ first,
    const uint64_t *__restrict__ skey, const int32_t *__restrict__ refit,
    double4 *__restrict__ com, double *__restrict__ mom, double *__restrict__ side,
    double4 *__restrict__ bbox) {
#pragma clang fp contract(off)
  if (gate && *gate <= 0) return;   // nothing active: skipped
  const uint32_t a = ctr->lvl[l], e = ctr->lvl[l + 1];
  const uint32_t k = threadIdx.x & 7u;
  const uint32_t oct = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const uint32_t n_oct = (gridDim.x * blockDim.x) >> 3;
  for (uint32_t v0 = a; v0 < e; v0 += n_oct) {      // uniform over the wave
    const uint32_t v = v0 + oct;
    const bool live = v < e;
    // the node's reads at once: child count, first child, cell side
    const uint32_t nch = live ? nchild[v] : 0u;
    const uint32_t c0 = live ? child[v] : 0u;
    const double cside = (!kBox && live) ? cube[4 * nsys[v] + 3] : 0.0;
    const bool mine = k < nch;
    const uint32_t c = mine ? c0 + k : 0u;
    double mc = 0.0, cx_ = 0.0, cy_ = 0.0, cz_ = 0.0;
    double4 cc = make_double4(0.0, 0.0, 0.0, 0.0);
    double o1 = 0.0, o2 = 0.0, o3 = 0.0, o4 = 0.0, o5 = 0.0, o6 = 0.0;
    if (mine) {
      const double *o = mom + 8 * (size_t)c;
      cc = com[c];
      mc = o[0];
      o1 = o[1]; o2 = o[2]; o3 = o[3]; o4 = o[4]; o5 = o[5]; o6 = o[6];
      cx_ = mc * cc.x; cy_ = mc * cc.y; cz_ = mc * cc.z;
    }
    const double M = oct_sum(mc);
    const double cx = oct_sum(cx_) / M, cy = oct_sum(cy_) / M, cz = oct_sum(cz_) / M;
    const double dx = cc.x - cx, dy = cc.y - cy, dz = cc.z - cz;
    double S[6];
    S[0] = oct_sum(mine ? o1 + mc * dx * dx : 0.0);
    S[1] = oct_sum(mine ? o2 + mc * dy * dy : 0.0);
    S[2] = oct_sum(mine ? o3 + mc * dz * dz : 0.0);
    S[3] = oct_sum(mine ? o4 + mc * dx * dy : 0.0);
    S[4] = oct_sum(mine ? o5 + mc * dx * dz : 0.0);
    S[5] = oct_sum(mine ? o6 + mc * dy * dz : 0.0);
    double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
    if constexpr (kBox) {
      double4 b0 = make_double4(INFINITY, INFINITY, INFINITY, 0.0);
      double4 b1 = make_double4(-INFINITY, -INFINITY, -INFINITY, 0.0);
      if (mine) { b0 = bbox[2 * (size_t)c]; b1 = bbox[2 * (size_t)c + 1]; }
      lo[0] = oct_min(b0.x); lo[1] = oct_min(b0.y); lo[2] = oct_min(b0.z);
      hi[0] = oct_max(b1.x); hi[1] = oct_max(b1.y); hi[2] = oct_max(b1.z);
    }
    if (live && nch > 0 && k == 0) {
      double so;
      if constexpr (kBox) {
        bbox[2 * (size_t)v] = make_double4(lo[0], lo[1], lo[2], 0.0);
        bbox[2 * (size_t)v + 1] = make_double4(hi[0], hi[1], hi[2], 0.0);
        so = open_size(v, l, first, nsys, skey, cube, lo, hi, *refit > 0);
      } else {
        so = ldexp(cside, -l);
      }
      store_moments(v, so, M, cx, cy, cz, S, com, mom, side);
    }
  }
}

template <bool kBox>
static void launch_moment_passes(tg_ctx *c) {
  Buffers &b = c->b;
  hipLaunchKernelGGL((k_moments_leaves<kBox>), dim3(1024), dim3(256), 0, c->stream, c->gate,
                     b.ctr, b.cube, b.level, b.nchild, b.first, b.count, b.nsys, b.spart,
                     b.key[0], b.refit_flag, b.com, b.mom, b.side, b.bbox, b.err);
  for (int l = c->max_level - 1; l >= 0; --l)    // the deepest level holds only leaves
    hipLaunchKernelGGL((k_moments_level<kBox>), dim3(512), dim3(256), 0, c->stream, c->gate, l,
                       b.ctr, b.cube, b.nchild, b.child, b.nsys, b.first, b.key[0],
                       b.refit_flag, b.com, b.mom, b.side, b.bbox);
}

hipError_t launch_moments(tg_ctx *c, const double *mass, bool gathered, bool refit) {
  Buffers &b = c->b;
  if (c->n == 0) return hipSuccess;
  int g = (int)std::min<int64_t>((c->n + 255) / 256, 4096);
  if (!gathered)        // else the build's gather brought the masses already
    hipLaunchKernelGGL(k_mass_gather, dim3(g), dim3(256), 0, c->stream, c->gate, mass,
                       b.val[0], c->n, b.spart, b.err);
  if (refit)
    launch_moment_passes<true>(c);
  else
    launch_moment_passes<false>(c);
  return hipGetLastError();
}

}  // namespace tg
