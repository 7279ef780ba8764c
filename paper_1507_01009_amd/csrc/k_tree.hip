// Octree over the sorted keys, all levels at once, and the walk groups.
//
// d[i] = number of equal leading key digits of sorted particles i-1 and i
// (0 at the first particle of every system and at the end, D for equal
// keys, D = 21 with one key word and 42 with two).  A level-l run is a
// maximal range of equal first l digits; one starts at i exactly when
// d[i] < l (l >= 1; level 0 is the whole system).  A node is a run whose
// parent run holds more than n_L particles (and splits only if l < D), so
// with lo = d[i] + 1 the nodes starting at i are the levels [lo, top] with
//   top = min(D, max(lo, m + 1)),  m = min(d[i+1 .. i+n_L]),
// provided the parent run of the first of them is longer than n_L, which
// is decided inside a window of n_L bytes on either side of i.  A system's
// root always exists and splits if the system holds more than n_L.
//
// Canonical ids order the nodes by level, then by first particle, which is
// the breadth-first order with children in octant order.  So a node's id is
// the start of its level plus its rank among the level's node starts,
// counted with per-level bitmaps and per-tile prefix sums; its parent is
// the last node of the level above starting at or before it, its children
// the nodes of the level below starting inside it, and its end the first
// position after it with d < l (searched inside the tile, else taken from
// a per-tile suffix minimum of the run starts of later tiles).
//
// Four launches, each of fixed shape for a given N (graph-capturable):
// k_lcp, k_flat_flags (per 256-particle tile: node levels per particle,
// bitmaps, counts, first run starts), k_flat_scan (one block per level:
// prefix of the counts, suffix minimum of the run starts), k_flat_emit.
#include "tg_internal.h"

namespace tg {

constexpr int kFT = 256;                 // particles per tile of the flat build
constexpr int kHalo = 16;                // >= max leaf size

__device__ __forceinline__ int sys_of(const int64_t *so, int S, int64_t i) {
  int lo = 0, hi = S - 1;                // last s with so[s] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (so[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ void load_sysoff(int64_t *so, const int64_t *sysoff, int S) {
  for (int k = threadIdx.x; k <= S; k += blockDim.x) so[k] = sysoff[k];
  __syncthreads();
}

__device__ __forceinline__ uint32_t common_digits(uint64_t a, uint64_t b) {
  const uint64_t x = a ^ b;
  return x == 0 ? 21u : (uint32_t)(__clzll((long long)x) - 1) / 3u;   // bit 63 is 0
}

// d for [0, n + 64): the common leading digits with the predecessor, 0 at
// every system start and from n on.  With second key words (skey_lo not
// null) the digits continue into them when the first words are equal.
__global__ __launch_bounds__(256) void k_lcp(const int32_t *__restrict__ gate, const uint64_t *__restrict__ skey,
                                             const uint64_t *__restrict__ skey_lo, int64_t n,
                                             const int64_t *__restrict__ sysoff, int S,
                                             uint8_t *__restrict__ d, uint32_t *__restrict__ gflag) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  __shared__ int64_t so[kMaxSys + 1];
  load_sysoff(so, sysoff, S);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n + 64;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i <= n) gflag[i] = 0u;   // the group-start flags [0, n], cleared for k_group_flags
    uint32_t v = 0;
    if (i > 0 && i < n && so[sys_of(so, S, i)] != i) {
      v = common_digits(skey[i - 1], skey[i]);
      if (skey_lo && v == 21u) v += common_digits(skey_lo[i - 1], skey_lo[i]);
    }
    d[i] = (uint8_t)v;
  }
}

// Per tile b of kFT particles: lt[i] = lo | top << 8 of the nodes starting
// at i (0xffff: none); bits[l][4 b + w] = ballot of "a level-l node starts
// here" of wave w; cnt[l][b] = nodes of level l in the tile; fst[l][b] =
// first run start of level l in the tile (first i with d[i] < l).  ML is
// the deepest level.
template <int ML>
__global__ __launch_bounds__(kFT) void k_flat_flags(const int32_t *__restrict__ gate, int64_t n, int nleaf, int S,
                                                    const int64_t *__restrict__ sysoff,
                                                    const uint8_t *__restrict__ d,
                                                    uint16_t *__restrict__ lt,
                                                    uint64_t *__restrict__ bits, int64_t wl,
                                                    uint32_t *__restrict__ cnt,
                                                    uint32_t *__restrict__ fst, int64_t tl) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  __shared__ uint8_t sd[kHalo + kFT + 2 * kHalo];
  __shared__ int64_t so[kMaxSys + 1];
  constexpr int kL = ML + 1;
  __shared__ uint32_t wc[kFT / 64][kL];
  __shared__ unsigned long long wm[kFT / 64][kL];
  __shared__ uint32_t mj[kL];
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.x, t0 = b * kFT, i = t0 + tid;
  for (int k = tid; k < kHalo + kFT + 2 * kHalo; k += kFT) {
    const int64_t p = t0 - kHalo + k;
    sd[k] = (p >= 0 && p < n + 64) ? d[p] : (uint8_t)0;
  }
  if (tid < kL) mj[tid] = 0xffffffffu;
  load_sysoff(so, sysoff, S);
  const bool valid = i < n;
  bool ex = false;
  uint32_t lo = 0, top = 0;
  const uint8_t *di = sd + kHalo + tid;       // di[k] = d[i + k]
  if (valid) {
    const int s = sys_of(so, S, i);
    const int64_t size = so[s + 1] - so[s];
    const bool seg = so[s] == i;
    uint32_t m = 255;
    for (int k = 1; k <= nleaf; ++k) m = min(m, (uint32_t)di[k]);
    if (seg) {
      ex = true;
      lo = 0;
      top = size > nleaf ? min((uint32_t)ML, max(1u, m + 1)) : 0u;
    } else {
      const uint32_t p = di[0];
      lo = p + 1;
      if (lo <= (uint32_t)ML) {
        if (p == 0) {
          ex = size > nleaf;                  // the parent is the root
        } else {
          // parent run [s0, e0) at level p: short iff e0 - s0 <= n_L
          int back = 0;
          for (int k = 1; k < nleaf; ++k)
            if (di[-k] < p) { back = k; break; }
          ex = true;
          if (back > 0) {
            for (int k = 1; k <= nleaf - back; ++k)
              if (di[k] < p) { ex = false; break; }
          }
        }
        top = min((uint32_t)ML, max(lo, m + 1));
      }
    }
    atomicMin(&mj[di[0]], (uint32_t)i);
  }
  if (valid) lt[i] = ex ? (uint16_t)(lo | (top << 8)) : (uint16_t)0xffff;
  const int w = tid >> 6, lane = tid & 63;
  // the wave's mask of every level first, then lane l stores level l's
  unsigned long long msk[kL];
#pragma unroll
  for (int l = 0; l < kL; ++l)
    msk[l] = __ballot(ex && lo <= (uint32_t)l && (uint32_t)l <= top);
  if (lane == 0) {
#pragma unroll
    for (int l = 0; l < kL; ++l) wm[w][l] = msk[l];
  }
  // one wave's LDS accesses execute in order
  if (lane < kL) {
    const unsigned long long m = wm[w][lane];
    bits[lane * wl + 4 * b + w] = m;
    wc[w][lane] = (uint32_t)__popcll(m);
  }
  __syncthreads();
  if (tid < kL) {
    const int l = tid;
    uint32_t c = 0;
    for (int q = 0; q < kFT / 64; ++q) c += wc[q][l];
    cnt[l * tl + b] = c;
    uint32_t f = 0xffffffffu;
    for (int v = 0; v < l; ++v) f = min(f, mj[v]);
    fst[l * tl + b] = f;
  }
}

// One block per level: exclusive prefix of cnt[l][0..T) in place with
// cnt[l][T] = total (also tot[l]); fst[l][b] <- first run start of level l
// after tile b (suffix minimum over later tiles; n past the last).  The
// tiles are taken kFSSub at a time: read into LDS with all loads in flight,
// each thread combining a contiguous run of kFSItems, one block-wide pass
// over the run totals, and written back from LDS.
constexpr int kFSItems = 4;
constexpr int kFSSub = 1024 * kFSItems;
__device__ __forceinline__ int fs_pad(int p) { return p + (p >> 5); }

__global__ __launch_bounds__(1024) void k_flat_scan(const int32_t *__restrict__ gate, int64_t T, int64_t n,
                                                    uint32_t *__restrict__ cnt,
                                                    uint32_t *__restrict__ fst, int64_t tl,
                                                    uint32_t *__restrict__ tot) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  __shared__ uint32_t sh[16];
  __shared__ uint32_t buf[kFSSub + kFSSub / 32];
  const int l = blockIdx.x;
  uint32_t *c = cnt + l * tl, *f = fst + l * tl;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint32_t run = 0;
  for (int64_t base = 0; base < T; base += kFSSub) {
    const int m = (int)min<int64_t>(kFSSub, T - base);
#pragma unroll
    for (int j = 0; j < kFSItems; ++j) {
      const int q = 1024 * j + tid;
      buf[fs_pad(q)] = q < m ? c[base + q] : 0u;
    }
    __syncthreads();
    uint32_t r[kFSItems], sum = 0;
#pragma unroll
    for (int j = 0; j < kFSItems; ++j) {
      r[j] = buf[fs_pad(kFSItems * tid + j)];
      sum += r[j];
    }
    uint32_t t;
    uint32_t e = run + block_exclusive_scan(sum, sh, t);
#pragma unroll
    for (int j = 0; j < kFSItems; ++j) {
      buf[fs_pad(kFSItems * tid + j)] = e;
      e += r[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kFSItems; ++j) {
      const int q = 1024 * j + tid;
      if (q < m) c[base + q] = buf[fs_pad(q)];
    }
    run += t;
    __syncthreads();
  }
  if (tid == 0) { c[T] = run; tot[l] = run; }
  // suffix minimum, chunks from the end; positions past the chunk's m hold
  // the identity
  uint32_t carry = (uint32_t)n;
  for (int64_t hi = T; hi > 0; hi -= kFSSub) {
    const int m = (int)min<int64_t>(kFSSub, hi);
    const int64_t lo = hi - m;
#pragma unroll
    for (int j = 0; j < kFSItems; ++j) {
      const int q = 1024 * j + tid;
      buf[fs_pad(q)] = q < m ? f[lo + q] : 0xffffffffu;
    }
    __syncthreads();
    uint32_t r[kFSItems], rm = 0xffffffffu;
#pragma unroll
    for (int j = 0; j < kFSItems; ++j) {
      r[j] = buf[fs_pad(kFSItems * tid + j)];
      rm = min(rm, r[j]);
    }
    // minimum over the later runs: inclusive suffix over the wave's lanes,
    // then over the later waves
    uint32_t x = rm;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_down(x, o, 64);
      if (lane + o < 64) x = min(x, y);
    }
    if (lane == 0) sh[wv] = x;
    __syncthreads();
    uint32_t later = carry, all = carry;
    for (int q = 0; q < 16; ++q) {
      const uint32_t v = sh[q];
      if (q > wv) later = min(later, v);
      all = min(all, v);
    }
    const uint32_t xl = __shfl_down(x, 1, 64);   // later lanes of the wave
    if (lane < 63) later = min(later, xl);
    uint32_t cur = later;
#pragma unroll
    for (int j = kFSItems - 1; j >= 0; --j) {
      buf[fs_pad(kFSItems * tid + j)] = cur;
      cur = min(cur, r[j]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kFSItems; ++j) {
      const int q = 1024 * j + tid;
      if (q < m) f[lo + q] = buf[fs_pad(q)];
    }
    carry = all;
    __syncthreads();
  }
}

// rank of x among the level-l node starts: base of x's tile + bits before x
// (All four bitmap words of x's tile are read at once and masked; a tile's
// words are allocated up to and including the tile past the last.)
__device__ __forceinline__ uint32_t rank_of(const uint64_t *__restrict__ bl,
                                            const uint32_t *__restrict__ cl, int64_t x) {
  const int64_t q = x >> 8;
  const uint32_t wq = (uint32_t)((x & 255) >> 6), bq = (uint32_t)(x & 63);
  const uint64_t *wv = bl + 4 * q;
  const uint64_t part = bq ? (1ull << bq) - 1ull : 0ull;
  uint32_t r = cl[q];
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k)
    r += (uint32_t)__popcll(wv[k] & (k < wq ? ~0ull : k == wq ? part : 0ull));
  return r;
}

// Nodes of tile b written at their canonical ids (ML: the deepest level).
template <int ML>
__global__ __launch_bounds__(kFT) void k_flat_emit(const int32_t *__restrict__ gate, 
    int64_t n, int S, const int64_t *__restrict__ sysoff, const uint8_t *__restrict__ d,
    const uint16_t *__restrict__ lt, const uint64_t *__restrict__ bits, int64_t wl,
    const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ fst, int64_t tl,
    const uint32_t *__restrict__ tot, int64_t max_nodes, TreeCounters *ctr, uint32_t *err,
    uint32_t *__restrict__ root_of, uint8_t *__restrict__ level,
    uint8_t *__restrict__ nchild, uint32_t *__restrict__ first,
    uint32_t *__restrict__ count, uint32_t *__restrict__ child,
    uint32_t *__restrict__ parent, uint32_t *__restrict__ nsys, uint4 *__restrict__ ninfo) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  __shared__ uint8_t sd[kFT];
  __shared__ uint8_t mn8[kFT / 8], mn64[kFT / 64];
  __shared__ int64_t so[kMaxSys + 1];
  constexpr int kL = ML + 1;
  __shared__ uint32_t lv[kL + 1];
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.x, t0 = b * kFT, i = t0 + tid;
  if (tid == 0) {
    uint32_t a = 0;
    for (int l = 0; l < kL; ++l) { lv[l] = a; a += tot[l]; }
    lv[kL] = a;
  }
  sd[tid] = i < n + 64 ? d[i] : (uint8_t)0;
  load_sysoff(so, sysoff, S);               // (includes a barrier)
  const uint32_t nn = lv[kL];
  const bool ovf = (int64_t)nn > max_nodes;
  if (b == 0 && tid == 0) {
    for (int l = 0; l <= kL; ++l) ctr->lvl[l] = ovf ? 0u : lv[l];
    ctr->lvl[kL + 1] = ovf ? 0u : nn;
    ctr->n_nodes = ovf ? 0u : nn;
    ctr->overflow = ovf ? 1u : 0u;
    if (ovf) set_err(err, TG_ERR_NODES);
  }
  if (ovf) return;
  if (b == 0) {
    for (int s = tid; s < S; s += kFT)
      root_of[s] = so[s + 1] > so[s] ? rank_of(bits, cnt, so[s]) : kNone;
  }
  if (tid < kFT / 8) {
    uint8_t v = 255;
    for (int k = 0; k < 8; ++k) v = min(v, sd[8 * tid + k]);
    mn8[tid] = v;
  }
  __syncthreads();
  if (tid < kFT / 64) {
    uint8_t v = 255;
    for (int k = 0; k < 8; ++k) v = min(v, mn8[8 * tid + k]);
    mn64[tid] = v;
  }
  __syncthreads();
  // one slot per (particle, level) node starting in this tile, spread over
  // the block so that a particle starting many nodes is not one long thread
  __shared__ uint32_t pre[kFT + 1];
  __shared__ uint16_t codes[kFT];
  __shared__ uint32_t scan_sh[kFT / 64];
  const uint16_t code_i = i < n ? lt[i] : (uint16_t)0xffff;
  const uint32_t nl_i = code_i == 0xffff ? 0u : (uint32_t)(code_i >> 8) - (code_i & 0xffu) + 1u;
  uint32_t n_slots;
  pre[tid] = block_exclusive_scan(nl_i, scan_sh, n_slots);
  codes[tid] = code_i;
  if (tid == 0) pre[kFT] = n_slots;
  __syncthreads();
  for (uint32_t slot = tid; slot < n_slots; slot += kFT) {
    int jl = 0, jh = kFT - 1;             // last j with pre[j] <= slot
    while (jl < jh) {
      const int mid = (jl + jh + 1) >> 1;
      if (pre[mid] <= slot) jl = mid; else jh = mid - 1;
    }
    const int j = jl;
    const uint32_t lo = codes[j] & 0xffu, top = codes[j] >> 8;
    const uint32_t l = lo + (slot - pre[j]);
    const int64_t i = t0 + j;
    const int sk = j;                     // position of i inside the tile
    const int s = sys_of(so, S, i);
    {
    const uint64_t *bl = bits + l * wl;
    const uint32_t *cl = cnt + l * tl;
    // the ranks that do not depend on the node's end, read together: the
    // node's own, its parent's (last level-(l - 1) start at or before i) and
    // its first child's
    const bool inner = l < top;
    const uint64_t *bc = bits + (inner ? l + 1 : l) * wl;
    const uint32_t *cc = cnt + (inner ? l + 1 : l) * tl;
    const uint32_t rid = rank_of(bl, cl, i);
    const uint32_t rpar = l == 0 ? 0u : rank_of(bits + (l - 1) * wl, cnt + (l - 1) * tl, i + 1);
    const uint32_t r0 = inner ? rank_of(bc, cc, i) : 0u;
    const uint32_t id = lv[l] + rid;
    // end: first j > i with d[j] < l (root: the system end)
    int64_t e;
    if (l == 0) {
      e = so[s + 1];
    } else {
      int k = sk + 1;
      int found = -1;
      for (; k < kFT && (k & 7); ++k)
        if (sd[k] < l) { found = k; break; }
      if (found < 0) {
        for (; k < kFT && (k & 63); k += 8)
          if (mn8[k >> 3] < l) break;
        if (k < kFT && (k & 63) == 0)
          for (; k < kFT; k += 64)
            if (mn64[k >> 6] < l) {
              while (mn8[k >> 3] >= l) k += 8;
              break;
            }
        if (k < kFT)
          for (int q = 0; q < 8; ++q)
            if (sd[k + q] < l) { found = k + q; break; }
      }
      e = found >= 0 ? t0 + found : (int64_t)fst[l * tl + b];
    }
    level[id] = (uint8_t)l;
    first[id] = (uint32_t)i;
    count[id] = (uint32_t)(e - i);
    nsys[id] = (uint32_t)s;
    parent[id] = l == 0 ? kNone : lv[l - 1] + rpar - 1u;
    uint32_t ch = 0, nch = 0;
    if (inner) {
      ch = lv[l + 1] + r0;
      nch = rank_of(bc, cc, e) - r0;
    }
    child[id] = ch;
    nchild[id] = (uint8_t)nch;
    ninfo[id] = make_uint4((uint32_t)i, (uint32_t)(e - i), ch, nch);
    }
  }
}

template <int ML>
static void launch_flat(tg_ctx *c, int64_t T) {
  Buffers &b = c->b;
  const int64_t n = c->n;
  const int64_t wl = 4 * (c->flat_tiles + 1), tl = c->flat_tiles + 1;
  if (T > 0)
    hipLaunchKernelGGL(k_flat_flags<ML>, dim3((unsigned)T), dim3(kFT), 0, c->stream, c->gate, n,
                       c->leaf_size, c->S, b.sysoff, b.lcp, b.fl_lt, b.fl_bits, wl,
                       b.fl_cnt, b.fl_fst, tl);
  hipLaunchKernelGGL(k_flat_scan, dim3(ML + 1), dim3(1024), 0, c->stream, c->gate, T, n,
                     b.fl_cnt, b.fl_fst, tl, b.fl_tot);
  hipLaunchKernelGGL(k_flat_emit<ML>, dim3((unsigned)std::max<int64_t>(T, 1)), dim3(kFT), 0,
                     c->stream, c->gate, n, c->S, b.sysoff, b.lcp, b.fl_lt, b.fl_bits, wl,
                     b.fl_cnt, b.fl_fst, tl, b.fl_tot, c->max_nodes, b.ctr, b.err,
                     b.root_of, b.level, b.nchild, b.first, b.count, b.child, b.parent,
                     b.nsys, b.ninfo);
}

hipError_t launch_tree_build(tg_ctx *c) {
  Buffers &b = c->b;
  const int64_t n = c->n, T = (n + kFT - 1) / kFT;
  const bool deep = c->max_level > kMaxLevel;
  hipLaunchKernelGGL(k_lcp, dim3((int)std::min<int64_t>((n + 64 + 255) / 256, 4096)),
                     dim3(256), 0, c->stream, c->gate, b.key[0], deep ? b.klo[0] : nullptr, n,
                     b.sysoff, c->S, b.lcp, b.gflag);
  if (deep)
    launch_flat<kMaxLevelDeep>(c, T);
  else
    launch_flat<kMaxLevel>(c, T);
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

__global__ void k_group_flags(const int32_t *__restrict__ gate, const TreeCounters *ctr, uint32_t ng,
                              const uint8_t *__restrict__ nchild,
                              const uint32_t *__restrict__ first,
                              const uint32_t *__restrict__ count,
                              const uint32_t *__restrict__ parent,
                              uint32_t *__restrict__ gflag) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
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

__global__ void k_group_write(const int32_t *__restrict__ gate, const TreeCounters *ctr, uint32_t ng,
                              const uint8_t *__restrict__ nchild,
                              const uint32_t *__restrict__ first,
                              const uint32_t *__restrict__ count,
                              const uint32_t *__restrict__ parent,
                              const uint32_t *__restrict__ nsys,
                              const uint32_t *__restrict__ gidx,
                              uint4 *__restrict__ groups) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
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
  // the flags were cleared by k_lcp in the build
  const int g = 1024;
  hipLaunchKernelGGL(k_group_flags, dim3(g), dim3(256), 0, c->stream, c->gate, b.ctr,
                     (uint32_t)c->group_size, b.nchild, b.first, b.count,
                     b.parent, b.gflag);
  hipError_t e = scan_u32(b.gflag, b.gflag, (uint32_t)c->n, nullptr, &b.ctr->n_groups,
               b.scan_part, c->stream, c->gate);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_group_write, dim3(g), dim3(256), 0, c->stream, c->gate, b.ctr,
                     (uint32_t)c->group_size, b.nchild, b.first, b.count,
                     b.parent, b.nsys, b.gflag, b.groups);
  return hipGetLastError();
}

// Block steps with a rebuild period: rebuild at substeps k that are
// multiples of it (or when no build exists yet), refit otherwise; neither
// when no star is active.
__global__ void k_refit_gates(const int32_t *__restrict__ n_act, const int64_t *__restrict__ k,
                              int32_t every, int32_t *__restrict__ gates,
                              int32_t *__restrict__ refit_flag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const bool any = !n_act || n_act[0] > 0;
  const bool build = any && (k[0] % every == 0 || gates[2] == 0);
  const bool refit = any && !build;
  gates[0] = build ? 1 : 0;
  gates[1] = refit ? 1 : 0;
  refit_flag[0] = refit ? 1 : 0;
}

hipError_t launch_refit_gates(tg_ctx *c, const int32_t *n_act, const int64_t *k, int32_t every) {
  hipLaunchKernelGGL(k_refit_gates, dim3(1), dim3(64), 0, c->stream, n_act, k, every,
                     c->b.refit_gates, c->b.refit_flag);
  return hipGetLastError();
}

}  // namespace tg
