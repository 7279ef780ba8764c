// a5-a6: octree over the sorted keys, level by level, and the walk groups.
//
// Level l is the node-id range [lvl[l], lvl[l+1]).  For every node of the
// level that holds more than n_L particles (and l < 21) the starts of its
// non-empty octants inside its sorted particle range are found (from the
// common-prefix lengths of neighbouring keys, or for the largest nodes by a
// wave-wide search on the next key digit); they become its children.
// Children ids come from an exclusive scan of the child counts over the
// level, so the numbering is breadth first with children in octant order,
// exactly the canonical order, without atomics.  Three launches per level,
// each of fixed shape, reading its range from device memory (graph-
// capturable): find the children, scan their counts, write them.
#include "tg_internal.h"

namespace tg {

// Contiguous share of [0, n) for this block (no rounding, so that a small
// level still spreads over every block).
__device__ __forceinline__ void chunk_range(uint32_t n, uint32_t &a, uint32_t &b) {
  const uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  a = min(n, blockIdx.x * chunk);
  b = min(n, a + chunk);
}

// Exclusive prefix of v over the wave; tot = wave sum.
__device__ __forceinline__ uint32_t wave_prefix(uint32_t v, uint32_t &tot) {
  const unsigned lane = lane_id();
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= (unsigned)o) x += y;
  }
  tot = (uint32_t)__shfl((int)x, 63, 64);
  return x - v;
}

__device__ __forceinline__ uint32_t digit_at(const uint64_t *__restrict__ skey,
                                             uint32_t i, int shift) {
  return (uint32_t)(skey[i] >> shift) & 7u;
}

// Octant starts of one node's sorted range [first, first + count), found by
// the whole wave: b[o] = first index whose digit (at bit `shift`) is >= o,
// for o = 1..7 (digits are sorted inside a node).  Up to 64 particles: one
// load per lane and one ballot per octant.  Larger nodes: lane group o
// (8 lanes) narrows the interval holding b[o] nine-fold per round with 8
// probes, so a million-particle node needs 7 rounds of parallel loads
// instead of 7 x 20 dependent ones.  The result is the same in every lane.
__device__ void wave_octants(const uint64_t *__restrict__ skey, uint32_t first,
                             uint32_t count, int shift, uint32_t b[9]) {
  const unsigned lane = lane_id();
  if (count <= 64) {
    const bool valid = lane < count;
    const uint32_t d = valid ? digit_at(skey, first + lane, shift) : 8u;
#pragma unroll
    for (uint32_t o = 1; o < 8; ++o)
      b[o] = first + (uint32_t)__popcll(__ballot(valid && d < o));
    return;
  }
  const uint32_t o = lane >> 3, k = lane & 7u;
  uint32_t lo = first, hi = first + count;   // b[o] lies in [lo, hi]
  while (__ballot(hi - lo > 8u)) {
    const bool act = hi - lo > 8u;
    const uint32_t step = act ? (hi - lo + 8u) / 9u : 0u;
    const uint32_t p = lo + (k + 1u) * step;
    const bool valid = act && p < hi;
    const bool pred = valid && digit_at(skey, p, shift) < o;
    const uint32_t c = (uint32_t)__popcll((__ballot(pred) >> (8 * o)) & 0xffull);
    const uint32_t nv = (uint32_t)__popcll((__ballot(valid) >> (8 * o)) & 0xffull);
    if (act) {
      const uint32_t lo0 = lo;
      if (c > 0) lo = lo0 + c * step + 1u;       // probe c-1 is below o
      if (c < nv) hi = lo0 + (c + 1u) * step;     // probe c is not
    }
  }
  const uint32_t p = lo + k;
  const bool pred = p < hi && digit_at(skey, p, shift) < o;
  const uint32_t mine = lo + (uint32_t)__popcll((__ballot(pred) >> (8 * o)) & 0xffull);
#pragma unroll
  for (int q = 1; q < 8; ++q) b[q] = (uint32_t)__shfl((int)mine, 8 * q, 64);
}

// Roots: one per non-empty system, in system order.
__global__ __launch_bounds__(256) void k_roots(const int64_t *__restrict__ sysoff,
                                               int S, TreeCounters *ctr,
                                               uint32_t *root_of, uint8_t *level,
                                               uint8_t *nchild, uint32_t *first,
                                               uint32_t *count, uint32_t *child,
                                               uint32_t *parent, uint32_t *nsys) {
  __shared__ uint32_t sh[4];
  const int s = threadIdx.x;
  int64_t ns = s < S ? sysoff[s + 1] - sysoff[s] : 0;
  uint32_t ne = ns > 0 ? 1u : 0u;
  uint32_t tot;
  uint32_t id = block_exclusive_scan(ne, sh, tot);
  if (s < S) root_of[s] = ne ? id : kNone;
  if (ne) {
    level[id] = 0; nchild[id] = 0; child[id] = 0; parent[id] = kNone;
    first[id] = (uint32_t)sysoff[s]; count[id] = (uint32_t)ns; nsys[id] = (uint32_t)s;
  }
  if (s == 0) {
    ctr->lvl[0] = 0;
    for (int l = 1; l < kLevels + 2; ++l) ctr->lvl[l] = tot;
    ctr->overflow = 0;
    ctr->big_n = 0;
    ctr->n_nodes = tot;
  }
}

// Common leading key digits of each sorted particle with its predecessor:
// d[i] = number of equal top digits of key[i-1] and key[i] (21 if equal).
// Inside a node of level l every d >= l, and its children start at the
// node's first particle and wherever d == l (the digit of level l+1 changes).
__global__ void k_lcp(const uint64_t *__restrict__ skey, int64_t n,
                      uint8_t *__restrict__ d) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t v = 0;
    if (i > 0) {
      const uint64_t x = skey[i - 1] ^ skey[i];
      v = x == 0 ? 21u : (uint32_t)(__clzll((long long)x) - 1) / 3u;   // bit 63 is 0
    }
    d[i] = (uint8_t)v;
  }
}

// 0x80 in every byte of w equal to l, 0 elsewhere (no false positives).
__device__ __forceinline__ uint64_t bytes_equal(uint64_t w, uint32_t l) {
  const uint64_t x = w ^ (0x0101010101010101ull * l);
  const uint64_t t = (x & 0x7f7f7f7f7f7f7f7full) + 0x7f7f7f7f7f7f7f7full;
  return ~(t | x | 0x7f7f7f7f7f7f7f7full);
}

// Bytes of the aligned word at p (p multiple of 8) that lie in [lo, hi).
__device__ __forceinline__ uint64_t byte_window(uint32_t p, uint32_t lo, uint32_t hi) {
  const int a = (int)lo - (int)p, b = (int)hi - (int)p;   // keep bytes j in [a, b)
  const uint64_t upto_b = b >= 8 ? ~0ull : (b <= 0 ? 0ull : (1ull << (8 * b)) - 1ull);
  const uint64_t from_a = a <= 0 ? ~0ull : (a >= 8 ? 0ull : ~((1ull << (8 * a)) - 1ull));
  return upto_b & from_a;
}

// Children of the nodes of level l that split, and per-block sums of their
// counts.  The children of a node [f, e) start at f and at every i in
// (f, e) with d[i] == l, stored in order: bnd[8 k + j] = start of child j
// (j >= 1).  Nodes of at most 512 particles: one lane scans their d bytes
// eight words (64 bytes) per batch with the loads of a batch independent;
// bigger ones are listed for k_level_big.
__global__ __launch_bounds__(256) void k_level_count(int l, int nleaf,
                                                     TreeCounters *ctr,
                                                     const uint64_t *__restrict__ skey,
                                                     const uint8_t *__restrict__ dl,
                                                     const uint32_t *__restrict__ first,
                                                     const uint32_t *__restrict__ count,
                                                     uint32_t *__restrict__ tmp,
                                                     uint32_t *__restrict__ bnd,
                                                     uint32_t *__restrict__ part,
                                                     uint32_t *__restrict__ biglist) {
  __shared__ uint32_t sh[4];
  const uint32_t a0 = ctr->lvl[l], n = ctr->lvl[l + 1] - a0;
  uint32_t ca, cb;
  chunk_range(n, ca, cb);
  const unsigned lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint64_t *dw = reinterpret_cast<const uint64_t *>(dl);
  uint32_t sum = 0;
  for (uint32_t base = ca + 64u * w; base < cb; base += 256u) {
    const uint32_t i = base + lane;
    const bool in = i < cb;
    const uint32_t cnt = in ? count[a0 + i] : 0u;
    const uint32_t fst = in ? first[a0 + i] : 0u;
    const bool split = in && cnt > (uint32_t)nleaf;
    const bool small = split && cnt <= 512u;
    if (in && !split) tmp[i] = 0u;
    if (small) {
      // d bytes of (fst, fst + cnt), eight aligned words per batch, every
      // load of a batch independent of the others
      const uint32_t lo = fst + 1u, hi = fst + cnt;
      const uint32_t p0 = lo & ~7u;
      uint32_t nch = 1;
      for (uint32_t pb = p0; pb < hi; pb += 64u) {
        uint64_t wd[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const uint32_t p = pb + 8u * q;
          wd[q] = p < hi ? dw[p >> 3] : 0ull;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const uint32_t p = pb + 8u * q;
          uint64_t m = p < hi ? bytes_equal(wd[q], (uint32_t)l) & byte_window(p, lo, hi) : 0ull;
          while (m) {
            const uint32_t j = (uint32_t)(__ffsll((long long)m) - 1) / 8u;   // byte of the 0x80 bit
            m &= m - 1ull;
            if (nch < 8u) bnd[8 * (size_t)i + nch] = p + j;
            ++nch;
          }
        }
      }
      nch = min(nch, 8u);
      tmp[i] = nch;
      sum += nch;
    }
    // nodes above 512 particles go to a work list for k_level_big, which
    // spreads them over the whole grid (they cluster in the dense centre)
    const unsigned long long bigm = __ballot(split && !small);
    if (bigm) {
      uint32_t b0 = 0;
      if (lane == 0) b0 = atomicAdd(&ctr->big_n, (uint32_t)__popcll(bigm));
      b0 = (uint32_t)__shfl((int)b0, 0, 64);
      if (split && !small) biglist[b0 + lanes_below(bigm)] = i;
    }
  }
  uint32_t tot;
  block_exclusive_scan(sum, sh, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Splitting nodes of more than 512 particles listed by k_level_count: one
// wave per node over the whole grid.  Up to 4096 particles the wave scans
// the d bytes coalesced (512 per round); bigger nodes are narrowed on the
// keys (wave_octants).  The child count is added to the sum of the block
// chunk that owns the node.
__global__ __launch_bounds__(256) void k_level_big(int l, const TreeCounters *ctr,
                                                   const uint64_t *__restrict__ skey,
                                                   const uint8_t *__restrict__ dl,
                                                   const uint32_t *__restrict__ first,
                                                   const uint32_t *__restrict__ count,
                                                   const uint32_t *__restrict__ biglist,
                                                   uint32_t *__restrict__ tmp,
                                                   uint32_t *__restrict__ bnd,
                                                   uint32_t *__restrict__ part) {
  const uint32_t nbig = ctr->big_n;
  if (nbig == 0) return;
  const uint32_t a0 = ctr->lvl[l], n = ctr->lvl[l + 1] - a0;
  const uint32_t chunk = (n + kLevelBlocks - 1) / kLevelBlocks;   // as k_level_count
  const int shift = 3 * (kMaxLevel - 1 - l);
  const unsigned lane = threadIdx.x & 63u;
  const uint32_t wid = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint32_t nw = gridDim.x * (blockDim.x >> 6);
  const uint64_t *dw = reinterpret_cast<const uint64_t *>(dl);
  for (uint32_t e = wid; e < nbig; e += nw) {
    const uint32_t vi = biglist[e];
    const uint32_t f = first[a0 + vi], c = count[a0 + vi];
    uint32_t nch;
    if (c <= 4096u) {
      const uint32_t lo = f + 1u, hi = f + c, p0 = lo & ~7u;
      uint32_t found = 0;
      for (uint32_t r = p0; r < hi; r += 512u) {
        const uint32_t p = r + 8u * lane;
        uint64_t m = p < hi ? bytes_equal(dw[p >> 3], (uint32_t)l) & byte_window(p, lo, hi) : 0ull;
        uint32_t tot;
        const uint32_t pre = wave_prefix(__popcll(m), tot);
        uint32_t k = 1u + found + pre;
        while (m) {
          const uint32_t j = (uint32_t)(__ffsll((long long)m) - 1) / 8u;
          m &= m - 1ull;
          if (k < 8u) bnd[8 * (size_t)vi + k] = p + j;
          ++k;
        }
        found += tot;
      }
      nch = min(1u + found, 8u);
    } else {
      uint32_t b[9];
      wave_octants(skey, f, c, shift, b);
      b[0] = f;
      b[8] = f + c;
      nch = 0;
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        if (b[o + 1] > b[o]) {
          if (nch > 0 && lane == 0) bnd[8 * (size_t)vi + nch] = b[o];
          ++nch;
        }
      }
    }
    if (lane == 0) {
      tmp[vi] = nch;
      atomicAdd(&part[vi / chunk], nch);
    }
  }
}

// Exclusive scan of the per-block child counts (one block, 4 per thread);
// sets the end of level l+1, guarding the node capacity.  A separate launch:
// a "last block" hand-off inside k_level_count would need an agent-scope
// fence in every block, which writes back the per-XCD L2 caches.
__global__ __launch_bounds__(256) void k_level_top(int l, int64_t max_nodes,
                                                   TreeCounters *ctr,
                                                   uint32_t *__restrict__ part,
                                                   uint32_t *err) {
  __shared__ uint32_t sh[4];
  constexpr int per = kLevelBlocks / 256;
  uint32_t loc[per];
  uint32_t my = 0;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    loc[q] = part[threadIdx.x * per + q];
    my += loc[q];
  }
  uint32_t all;
  uint32_t e = block_exclusive_scan(my, sh, all);
#pragma unroll
  for (int q = 0; q < per; ++q) {
    part[threadIdx.x * per + q] = e;
    e += loc[q];
  }
  if (threadIdx.x == 0) {
    ctr->big_n = 0;
    const uint32_t start = ctr->lvl[l + 1];
    if (ctr->overflow || (int64_t)start + all > max_nodes) {
      if (!ctr->overflow) set_err(err, TG_ERR_NODES);
      ctr->overflow = 1;
      all = 0;
    }
    ctr->lvl[l + 2] = start + all;
    ctr->n_nodes = start + all;
  }
}

// Emit the children of level l's nodes from the stored octant starts.
__global__ __launch_bounds__(256) void k_level_emit(int l, const TreeCounters *ctr,
                                                    const uint32_t *__restrict__ bnd,
                                                    const uint32_t *__restrict__ tmp,
                                                    const uint32_t *__restrict__ part,
                                                    uint8_t *level, uint8_t *nchild,
                                                    uint32_t *first, uint32_t *count,
                                                    uint32_t *child, uint32_t *parent,
                                                    uint32_t *nsys) {
  __shared__ uint32_t sh[4];
  const uint32_t a0 = ctr->lvl[l], n = ctr->lvl[l + 1] - a0;
  const uint32_t c_start = ctr->lvl[l + 1];
  const bool ovf = ctr->overflow != 0;
  uint32_t ca, cb;
  chunk_range(n, ca, cb);
  uint32_t base = part[blockIdx.x];
  for (uint32_t t0 = ca; t0 < cb; t0 += 256u) {
    const uint32_t i = t0 + threadIdx.x;
    const bool in = i < cb;
    uint32_t nch = (in && !ovf) ? tmp[i] : 0u;
    uint32_t tot;
    uint32_t off = block_exclusive_scan(nch, sh, tot);
    if (in) {
      const uint32_t v = a0 + i;
      if (nch > 0) {
        const uint32_t f = first[v], e = f + count[v];
        uint32_t c = c_start + base + off;
        child[v] = c;
        nchild[v] = (uint8_t)nch;
        const uint32_t sy = nsys[v];
        uint32_t st = f;
        for (uint32_t k = 0; k < nch; ++k, ++c) {
          const uint32_t nx = k + 1 < nch ? bnd[8 * (size_t)i + k + 1] : e;
          level[c] = (uint8_t)(l + 1);
          nchild[c] = 0;
          child[c] = 0;
          first[c] = st;
          count[c] = nx - st;
          parent[c] = v;
          nsys[c] = sy;
          st = nx;
        }
      } else {
        child[v] = 0;
        nchild[v] = 0;
      }
    }
    base += tot;
  }
}

hipError_t launch_tree_build(tg_ctx *c) {
  Buffers &b = c->b;
  if (c->n > 0)
    hipLaunchKernelGGL(k_lcp, dim3((int)std::min<int64_t>((c->n + 255) / 256, 4096)),
                       dim3(256), 0, c->stream, b.key[0], c->n, b.lcp);
  hipLaunchKernelGGL(k_roots, dim3(1), dim3(256), 0, c->stream, b.sysoff, c->S,
                     b.ctr, b.root_of, b.level, b.nchild, b.first, b.count,
                     b.child, b.parent, b.nsys);
  for (int l = 0; l < kMaxLevel; ++l) {
    hipLaunchKernelGGL(k_level_count, dim3(kLevelBlocks), dim3(256), 0,
                       c->stream, l, c->leaf_size, b.ctr, b.key[0], b.lcp,
                       b.first, b.count, b.lvl_tmp, b.lvl_bnd, b.lvl_part,
                       b.lvl_big);
    hipLaunchKernelGGL(k_level_big, dim3(kLevelBlocks), dim3(256), 0, c->stream,
                       l, b.ctr, b.key[0], b.lcp, b.first, b.count, b.lvl_big,
                       b.lvl_tmp, b.lvl_bnd, b.lvl_part);
    hipLaunchKernelGGL(k_level_top, dim3(1), dim3(256), 0, c->stream, l,
                       c->max_nodes, b.ctr, b.lvl_part, b.err);
    hipLaunchKernelGGL(k_level_emit, dim3(kLevelBlocks), dim3(256), 0,
                       c->stream, l, b.ctr, b.lvl_bnd, b.lvl_tmp, b.lvl_part,
                       b.level, b.nchild, b.first, b.count, b.child, b.parent,
                       b.nsys);
  }
  return hipGetLastError();
}

// ---- groups --------------------------------------------------------------
// A group is a node holding at most n_G particles whose parent holds more
// (or a root holding at most n_G); a leaf holding more than n_G is cut into
// runs of n_G.  Group starts are flagged per particle and numbered by a scan,
// so groups come out ordered by first particle.
__device__ __forceinline__ bool is_group(uint32_t v, uint32_t ng,
                                         const uint32_t *count,
                                         const uint32_t *parent) {
  const uint32_t p = parent[v];
  return count[v] <= ng && (p == kNone || count[p] > ng);
}

__global__ void k_group_flags(const TreeCounters *ctr, uint32_t ng,
                              const uint8_t *__restrict__ nchild,
                              const uint32_t *__restrict__ first,
                              const uint32_t *__restrict__ count,
                              const uint32_t *__restrict__ parent,
                              uint32_t *__restrict__ gflag) {
  const uint32_t nn = ctr->n_nodes;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nn;
       v += gridDim.x * blockDim.x) {
    if (is_group(v, ng, count, parent)) {
      gflag[first[v]] = 1;
    } else if (count[v] > ng && nchild[v] == 0) {
      for (uint32_t k = 0; k < count[v]; k += ng) gflag[first[v] + k] = 1;
    }
  }
}

__global__ void k_group_write(const TreeCounters *ctr, uint32_t ng,
                              const uint8_t *__restrict__ nchild,
                              const uint32_t *__restrict__ first,
                              const uint32_t *__restrict__ count,
                              const uint32_t *__restrict__ parent,
                              const uint32_t *__restrict__ nsys,
                              const uint32_t *__restrict__ gidx,
                              uint4 *__restrict__ groups) {
  const uint32_t nn = ctr->n_nodes;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nn;
       v += gridDim.x * blockDim.x) {
    if (is_group(v, ng, count, parent)) {
      groups[gidx[first[v]]] = make_uint4(first[v], count[v], v, nsys[v]);
    } else if (count[v] > ng && nchild[v] == 0) {
      for (uint32_t k = 0; k < count[v]; k += ng)
        groups[gidx[first[v] + k]] =
            make_uint4(first[v] + k, min(ng, count[v] - k), v, nsys[v]);
    }
  }
}

hipError_t launch_groups(tg_ctx *c) {
  Buffers &b = c->b;
  if (c->n == 0) {
    return fill_u32(&b.ctr->n_groups, 0u, 1, c->stream);
  }
  hipError_t e = fill_u32(b.gflag, 0u, c->n + 1, c->stream);
  if (e != hipSuccess) return e;
  const int g = 1024;
  hipLaunchKernelGGL(k_group_flags, dim3(g), dim3(256), 0, c->stream, b.ctr,
                     (uint32_t)c->group_size, b.nchild, b.first, b.count,
                     b.parent, b.gflag);
  e = scan_u32(b.gflag, b.gflag, (uint32_t)c->n, nullptr, &b.ctr->n_groups,
               b.scan_part, c->stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_group_write, dim3(g), dim3(256), 0, c->stream, b.ctr,
                     (uint32_t)c->group_size, b.nchild, b.first, b.count,
                     b.parent, b.nsys, b.gflag, b.groups);
  return hipGetLastError();
}

}  // namespace tg
