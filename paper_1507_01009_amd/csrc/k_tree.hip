// a5-a6: octree over the sorted keys, level by level, and the walk groups.
//
// Level l is the node-id range [lvl[l], lvl[l+1]).  For every node of the
// level that holds more than n_L particles (and l < 21) the boundaries of its
// eight octants inside its sorted particle range are found by binary search
// on the next key digit; the non-empty ones become its children.  Children
// ids come from an exclusive scan of the child counts over the level, so the
// numbering is breadth first with children in octant order, exactly the
// canonical order, without atomics.  Every launch has a fixed shape and
// reads its range from device memory (graph-capturable).
#include "tg_internal.h"

namespace tg {

__device__ __forceinline__ void chunk_range(uint32_t n, uint32_t &a, uint32_t &b) {
  uint32_t chunk = ((n + gridDim.x - 1) / gridDim.x + 255u) & ~255u;
  a = min(n, blockIdx.x * chunk);
  b = min(n, a + chunk);
}

// Octant boundaries of the sorted range [first, first + count) on the digit
// at bit `shift`: bnd[o] = first index whose digit >= o.
__device__ __forceinline__ void octant_bounds(const uint64_t *__restrict__ skey,
                                              uint32_t first, uint32_t count,
                                              int shift, uint32_t bnd[9]) {
  const uint32_t end = first + count;
  bnd[0] = first;
  bnd[8] = end;
  uint32_t lo = first;
  for (uint32_t o = 1; o < 8; ++o) {
    uint32_t a = lo, b = end;
    while (a < b) {
      uint32_t m = (a + b) >> 1;
      if (((uint32_t)(skey[m] >> shift) & 7u) < o) a = m + 1; else b = m;
    }
    bnd[o] = a;
    lo = a;
  }
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
    ctr->n_nodes = tot;
  }
}

// Child counts of the nodes of level l (and per-block sums for the scan).
__global__ __launch_bounds__(256) void k_level_count(int l, int nleaf,
                                                     const TreeCounters *ctr,
                                                     const uint64_t *__restrict__ skey,
                                                     const uint32_t *__restrict__ first,
                                                     const uint32_t *__restrict__ count,
                                                     uint32_t *__restrict__ tmp,
                                                     uint32_t *__restrict__ part) {
  __shared__ uint32_t sh[4];
  const uint32_t a0 = ctr->lvl[l], n = ctr->lvl[l + 1] - a0;
  uint32_t ca, cb;
  chunk_range(n, ca, cb);
  const int shift = 3 * (kMaxLevel - 1 - l);
  uint32_t sum = 0;
  for (uint32_t i = ca + threadIdx.x; i < cb; i += 256u) {
    const uint32_t v = a0 + i;
    uint32_t nch = 0;
    if (count[v] > (uint32_t)nleaf) {
      uint32_t bnd[9];
      octant_bounds(skey, first[v], count[v], shift, bnd);
#pragma unroll
      for (int o = 0; o < 8; ++o) nch += bnd[o + 1] > bnd[o] ? 1u : 0u;
    }
    tmp[i] = nch;
    sum += nch;
  }
  uint32_t tot;
  block_exclusive_scan(sum, sh, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Scan of the block sums; sets the end of level l+1, guarding capacity.
__global__ __launch_bounds__(256) void k_level_top(int l, int64_t max_nodes,
                                                   TreeCounters *ctr,
                                                   uint32_t *part, uint32_t *err) {
  __shared__ uint32_t sh[4];
  uint32_t v = part[threadIdx.x];
  uint32_t tot;
  uint32_t e = block_exclusive_scan(v, sh, tot);
  part[threadIdx.x] = e;
  if (threadIdx.x == 0) {
    const uint32_t start = ctr->lvl[l + 1];
    if (ctr->overflow || (int64_t)start + tot > max_nodes) {
      if (!ctr->overflow) set_err(err, TG_ERR_NODES);
      ctr->overflow = 1;
      tot = 0;
    }
    ctr->lvl[l + 2] = start + tot;
    ctr->n_nodes = start + tot;
  }
}

// Emit the children of level l's nodes.
__global__ __launch_bounds__(256) void k_level_emit(int l, const TreeCounters *ctr,
                                                    const uint64_t *__restrict__ skey,
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
  const int shift = 3 * (kMaxLevel - 1 - l);
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
        uint32_t bnd[9];
        octant_bounds(skey, first[v], count[v], shift, bnd);
        uint32_t c = c_start + base + off;
        child[v] = c;
        nchild[v] = (uint8_t)nch;
        const uint32_t sy = nsys[v];
        for (int o = 0; o < 8; ++o) {
          if (bnd[o + 1] > bnd[o]) {
            level[c] = (uint8_t)(l + 1);
            nchild[c] = 0;
            child[c] = 0;
            first[c] = bnd[o];
            count[c] = bnd[o + 1] - bnd[o];
            parent[c] = v;
            nsys[c] = sy;
            ++c;
          }
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
  hipLaunchKernelGGL(k_roots, dim3(1), dim3(256), 0, c->stream, b.sysoff, c->S,
                     b.ctr, b.root_of, b.level, b.nchild, b.first, b.count,
                     b.child, b.parent, b.nsys);
  for (int l = 0; l < kMaxLevel; ++l) {
    hipLaunchKernelGGL(k_level_count, dim3(kScanBlocks), dim3(256), 0,
                       c->stream, l, c->leaf_size, b.ctr, b.key[0], b.first,
                       b.count, b.lvl_tmp, b.scan_part);
    hipLaunchKernelGGL(k_level_top, dim3(1), dim3(kScanBlocks), 0, c->stream,
                       l, c->max_nodes, b.ctr, b.scan_part, b.err);
    hipLaunchKernelGGL(k_level_emit, dim3(kScanBlocks), dim3(256), 0,
                       c->stream, l, b.ctr, b.key[0], b.lvl_tmp, b.scan_part,
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
