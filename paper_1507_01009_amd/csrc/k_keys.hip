// Bounding cube per system, 21-bit Morton keys (or 42-bit, as two words),
// stable LSD radix sort of (key, index), and the gather of positions into
// sorted order.
//
// Work is cut into tiles of kSortTile consecutive particles that never cross
// a system boundary, so one launch handles every system of a batch.  One
// kernel counts each system's digits for all passes; in each pass a tile
// ranks its keys, publishes its per-digit counts and adds those of the
// earlier tiles of its own system (a look-back that ends at the system's
// first tile).  A key's place is the system's first index + the system's
// keys of smaller digits + the earlier tiles' keys of its digit + its rank
// in the tile, so the sort is segmented by system.
//
// Bit-exactness: the quantisation is t = x - lo, u = t * (2^21 / L), floor,
// clamp, with no contraction possible (one subtract, one multiply), and the
// division 2^21 / L is IEEE-rounded; keys and the stable permutation are
// therefore identical to any correct implementation of the same definition.
#include "tg_internal.h"

namespace tg {

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Per-tile min/max of each coordinate; flags non-finite positions.
__global__ __launch_bounds__(256) void k_cube_part(const int32_t *__restrict__ gate, const double *__restrict__ pos,
                                                   const Tile *__restrict__ tiles,
                                                   double *__restrict__ part,
                                                   uint32_t *err) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  __shared__ double sh[4][6];
  const Tile t = tiles[blockIdx.x];
  double lo[3] = {INFINITY, INFINITY, INFINITY};
  double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
#pragma unroll 4
  for (uint32_t i = t.start + threadIdx.x; i < t.end; i += 256u) {   // unrolled: loads in flight together
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double x = pos[3 * (size_t)i + k];
      bad |= !isfinite(x);
      lo[k] = fmin(lo[k], x);
      hi[k] = fmax(hi[k], x);
    }
  }
  if (bad) set_err(err, TG_ERR_NONFINITE);
  const unsigned lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = wave_min(lo[k]);
    hi[k] = wave_max(hi[k]);
  }
  if (lane == 0)
    for (int k = 0; k < 3; ++k) { sh[w][k] = lo[k]; sh[w][3 + k] = hi[k]; }
  __syncthreads();
  if (threadIdx.x < 6) {
    double v = sh[0][threadIdx.x];
    for (int i = 1; i < 4; ++i)
      v = threadIdx.x < 3 ? fmin(v, sh[i][threadIdx.x]) : fmax(v, sh[i][threadIdx.x]);
    part[6 * (size_t)blockIdx.x + threadIdx.x] = v;
  }
}

// One block per system: lo = coordinate minimum, L = largest extent (1 if
// every particle coincides or the system is empty).
__global__ __launch_bounds__(256) void k_cube_final(const int32_t *__restrict__ gate, const double *__restrict__ part,
                                                    const uint32_t *__restrict__ sys_tile0,
                                                    double *__restrict__ cube) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  __shared__ double sh[4][6];
  const int s = blockIdx.x;
  const uint32_t a = sys_tile0[s], b = sys_tile0[s + 1];
  double lo[3] = {INFINITY, INFINITY, INFINITY};
  double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (uint32_t t = a + threadIdx.x; t < b; t += 256u)
    for (int k = 0; k < 3; ++k) {
      lo[k] = fmin(lo[k], part[6 * (size_t)t + k]);
      hi[k] = fmax(hi[k], part[6 * (size_t)t + 3 + k]);
    }
  const unsigned lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  for (int k = 0; k < 3; ++k) { lo[k] = wave_min(lo[k]); hi[k] = wave_max(hi[k]); }
  if (lane == 0)
    for (int k = 0; k < 3; ++k) { sh[w][k] = lo[k]; sh[w][3 + k] = hi[k]; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double L = 1.0, l3[3] = {0.0, 0.0, 0.0};
    if (b > a) {
      double h3[3];
      for (int k = 0; k < 3; ++k) {
        l3[k] = fmin(fmin(sh[0][k], sh[1][k]), fmin(sh[2][k], sh[3][k]));
        h3[k] = fmax(fmax(sh[0][3 + k], sh[1][3 + k]), fmax(sh[2][3 + k], sh[3][3 + k]));
      }
      L = 0.0;
      for (int k = 0; k < 3; ++k) L = fmax(L, h3[k] - l3[k]);
      if (L == 0.0) L = 1.0;
    }
    cube[4 * s + 0] = l3[0]; cube[4 * s + 1] = l3[1]; cube[4 * s + 2] = l3[2];
    cube[4 * s + 3] = L;
  }
}

// Spread the low 21 bits of v so that bit j lands on bit 3j.
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  v &= 0x1FFFFFull;
  v = (v | (v << 32)) & 0x1F00000000FFFFull;
  v = (v | (v << 16)) & 0x1F0000FF0000FFull;
  v = (v | (v << 8)) & 0x100F00F00F00F00Full;
  v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

// q = min(floor((x - lo) sigma), qmax), sigma = 2^bits / L.
__device__ __forceinline__ uint64_t quantise(double x, double lo, double sigma, uint64_t qmax) {
  double t = dsub(x, lo);
  double u = dmul(t, sigma);
  double f = floor(u);
  uint64_t q = f <= 0.0 ? 0ull : (uint64_t)f;
  return q > qmax ? qmax : q;
}

// Interleave the low 21 bits of three coordinates (x above y above z).
__device__ __forceinline__ uint64_t morton21(uint64_t qx, uint64_t qy, uint64_t qz) {
  return (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
}

// 42 levels: 2^42 / L is 2^21 / L scaled by a power of two, so the top 21
// bits of each 42-bit coordinate are the 21-bit coordinate and the first
// key word is the 21-level key; the second word holds the last 21 digits.
__device__ __forceinline__ void keys42(const double *p, const double *c, double sigma,
                                       uint64_t &hi, uint64_t &lo) {
  const uint64_t m = (1ull << 42) - 1ull;
  const uint64_t qx = quantise(p[0], c[0], sigma, m), qy = quantise(p[1], c[1], sigma, m),
                 qz = quantise(p[2], c[2], sigma, m);
  hi = morton21(qx >> 21, qy >> 21, qz >> 21);
  lo = morton21(qx, qy, qz);
}

__device__ __forceinline__ int system_of_tile(const uint32_t *sys_tile0, int S, uint32_t t) {
  int lo_s = 0, hi_s = S - 1;     // last s with sys_tile0[s] <= t
  while (lo_s < hi_s) {
    int mid = (lo_s + hi_s + 1) >> 1;
    if (sys_tile0[mid] <= t) lo_s = mid; else hi_s = mid - 1;
  }
  return lo_s;
}

// Keys (x bit above y above z at every level) and the identity values;
// with kDeep the 42-level key's first word goes to key and its second to
// klo.
template <bool kDeep>
__global__ __launch_bounds__(256) void k_keys(const int32_t *__restrict__ gate, const double *__restrict__ pos,
                                              const Tile *__restrict__ tiles,
                                              const uint32_t *__restrict__ sys_tile0,
                                              int S, const double *__restrict__ cube,
                                              uint64_t *__restrict__ key,
                                              uint64_t *__restrict__ klo,
                                              uint32_t *__restrict__ val,
                                              uint32_t *__restrict__ zero, int64_t nzero) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  // the sort's counters and tile status, cleared for the sort that follows
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nzero;
       w += (int64_t)gridDim.x * blockDim.x)
    zero[w] = 0u;
  const Tile t = tiles[blockIdx.x];
  const double *c = cube + 4 * system_of_tile(sys_tile0, S, blockIdx.x);
  const double sigma = (kDeep ? 4398046511104.0 : 2097152.0) / c[3];
#pragma unroll 4
  for (uint32_t i = t.start + threadIdx.x; i < t.end; i += 256u) {   // unrolled: loads in flight together
    if constexpr (kDeep) {
      uint64_t hi, lo;
      keys42(pos + 3 * (size_t)i, c, sigma, hi, lo);
      key[i] = hi;
      klo[i] = lo;
    } else {
      const uint64_t m = 0x1FFFFFull;
      key[i] = morton21(quantise(pos[3 * (size_t)i + 0], c[0], sigma, m),
                        quantise(pos[3 * (size_t)i + 1], c[1], sigma, m),
                        quantise(pos[3 * (size_t)i + 2], c[2], sigma, m));
    }
    val[i] = i;
  }
}

// 42 levels, after the sort: the second key words in sorted order, from
// the positions of the sorted particles (slo[r] for perm[r]).
__global__ void k_keys_lo_sorted(const int32_t *__restrict__ gate, const double *__restrict__ pos,
                                 const uint32_t *__restrict__ perm, int64_t n,
                                 const int64_t *__restrict__ sysoff, int S,
                                 const double *__restrict__ cube, uint64_t *__restrict__ slo) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    int a = 0, b = S - 1;          // last s with sysoff[s] <= r
    while (a < b) {
      const int mid = (a + b + 1) >> 1;
      if (sysoff[mid] <= r) a = mid; else b = mid - 1;
    }
    const double *c = cube + 4 * a;
    uint64_t hi, lo;
    keys42(pos + 3 * (size_t)perm[r], c, 4398046511104.0 / c[3], hi, lo);
    slo[r] = lo;
  }
}

// ---- radix sort, 9-bit digits ----------------------------------------
// Stable LSD sort of (key, index), 7 passes of 9 bits (the 63 bits of a key
// word), each system sorted on its own (tiles never straddle systems).  One
// counting kernel gives the digit totals of all passes per system; then one
// kernel per pass: a tile (taken in dispatch order from a ticket) ranks its
// keys in LDS, publishes its per-digit counts, adds up the counts of the
// earlier tiles of its system by looking back through their published words
// (each a flag and a count in one 32-bit word, written and read with
// agent-scope atomics), and scatters.  The lowest waiting tile never waits
// on a later one, so every wait ends; a wait is still bounded and reports
// TG_ERR_SORT if exceeded.
constexpr uint32_t kSortMask = kSortDigits - 1;
static_assert(kSortBits * kSortPasses == 63, "a key word holds 63 bits");
static_assert(kSortDigits == kSortThreads, "each thread owns one digit");
constexpr uint32_t kStAgg = 1u << 30, kStIncl = 2u << 30, kStVal = (1u << 30) - 1u;

__device__ __forceinline__ int tile_system(const uint32_t *sys_tile0, int S, uint32_t t) {
  int lo = 0, hi = S - 1;      // last s with sys_tile0[s] <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sys_tile0[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// cnt[s][p][d]: keys of system s with digit d in pass p (cleared beforehand)
__global__ __launch_bounds__(256) void k_sort_count(const int32_t *__restrict__ gate, const uint64_t *__restrict__ key,
                                                    const Tile *__restrict__ tiles,
                                                    const uint32_t *__restrict__ sys_tile0,
                                                    int S, uint32_t *__restrict__ cnt) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  __shared__ uint32_t c[kSortPasses][kSortDigits];
  const Tile t = tiles[blockIdx.x];
  const int s = tile_system(sys_tile0, S, blockIdx.x);
#pragma unroll
  for (int p = 0; p < kSortPasses; ++p) {
    c[p][threadIdx.x] = 0;
    c[p][threadIdx.x + 256] = 0;
  }
  __syncthreads();
  for (uint32_t i = t.start + threadIdx.x; i < t.end; i += 256u) {
    const uint64_t k = key[i];
#pragma unroll
    for (int p = 0; p < kSortPasses; ++p)
      atomicAdd(&c[p][(uint32_t)(k >> (kSortBits * p)) & kSortMask], 1u);
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < kSortPasses; ++p) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t d = threadIdx.x + 256u * h;
      const uint32_t v = c[p][d];
      if (v) atomicAdd(&cnt[(size_t)(s * kSortPasses + p) * kSortDigits + d], v);
    }
  }
}

// Exclusive prefix sums over the block of two values per thread at once
// (one barrier).  The wave totals stay in sh; the caller's next barrier
// comes before sh is written again.
__device__ __forceinline__ void block_exclusive_scan2(uint32_t a, uint32_t b, uint2 *sh,
                                                      uint32_t &ea, uint32_t &eb) {
  const unsigned lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  uint32_t x = a, y = b;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t xo = __shfl_up(x, o, 64), yo = __shfl_up(y, o, 64);
    if (lane >= (unsigned)o) { x += xo; y += yo; }
  }
  if (lane == 63u) sh[w] = make_uint2(x, y);
  __syncthreads();
  uint32_t ba = 0, bb = 0;
  for (unsigned q = 0; q < w; ++q) { ba += sh[q].x; bb += sh[q].y; }
  ea = ba + x - a;
  eb = bb + y - b;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_pass(const int32_t *__restrict__ gate, 
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
    const Tile *__restrict__ tiles, const uint32_t *__restrict__ sys_tile0, int S,
    const int64_t *__restrict__ sysoff, int pass, const uint32_t *__restrict__ cnt,
    uint32_t *status, uint32_t *ticket, uint32_t *err, uint32_t *__restrict__ rank) {
  constexpr int kWaves = kSortThreads / 64;
  if (gate && *gate <= 0) return;   // nothing active: skipped
  __shared__ uint64_t sk[kSortTile];
  __shared__ uint32_t sv[kSortTile];
  __shared__ uint32_t wcnt[kWaves][kSortDigits];
  __shared__ uint32_t loc_off[kSortDigits];
  __shared__ uint32_t glob_off[kSortDigits];
  __shared__ uint2 scan_sh[kWaves];
  __shared__ uint32_t s_tile;
  const unsigned tid = threadIdx.x, w = tid >> 6, lane = tid & 63u;
  const int shift = kSortBits * pass;
  if (tid == 0) s_tile = atomicAdd(ticket, 1u);
#pragma unroll
  for (int q = 0; q < kWaves; ++q) wcnt[q][tid] = 0;
  __syncthreads();
  const uint32_t tb = s_tile;
  const Tile t = tiles[tb];
  const int s = tile_system(sys_tile0, S, tb);
  const uint32_t first_tile = sys_tile0[s];
  const uint32_t n_in = t.end - t.start;
  // the system's count of digit tid (all tiles) and its first index
  const uint32_t gcnt = cnt[(size_t)(s * kSortPasses + pass) * kSortDigits + tid];
  const int64_t soff = sysoff[s];

  // wave w holds the tile's keys [64 kSortItems w, 64 kSortItems (w + 1)) in index order
  uint64_t k[kSortItems];
  uint32_t v[kSortItems], rk[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t idx = 64u * kSortItems * w + 64u * r + lane;
    k[r] = idx < n_in ? kin[t.start + idx] : 0ull;
    v[r] = idx < n_in ? vin[t.start + idx] : 0u;
  }
  // stable ranks inside each wave: rounds of 64 keys in index order, peers
  // of equal digit found with ballots, counts kept in the wave's own LDS row
  // (one wave's LDS accesses execute in order: no barrier between rounds)
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t idx = 64u * kSortItems * w + 64u * r + lane;
    const bool valid = idx < n_in;
    const uint32_t d = (uint32_t)(k[r] >> shift) & kSortMask;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kSortBits; ++bit) {
      const unsigned long long bb = __ballot((d >> bit) & 1u);
      peers &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    const uint32_t lr = lanes_below(peers);
    const uint32_t base = valid ? wcnt[w][d] : 0u;
    rk[r] = base + lr;
    if (valid && lr == 0) wcnt[w][d] = base + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // digit tid: counts of the waves -> their exclusive offsets in place
  uint32_t mine = 0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) {
    const uint32_t cq = wcnt[q][tid];
    wcnt[q][tid] = mine;
    mine += cq;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t d = (uint32_t)(k[r] >> shift) & kSortMask;
    rk[r] += wcnt[w][d];
  }
  // publish this tile's count of digit tid
  uint32_t *st = status + (size_t)tb * kSortDigits + tid;
  __hip_atomic_store(st, (tb == first_tile ? kStIncl : kStAgg) | mine, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  // before waiting on the predecessors: the digit starts inside the system
  // (counts of smaller digits) and inside the tile, and the tile's keys
  // placed in LDS in digit order
  uint32_t dbase, lbase;
  block_exclusive_scan2(gcnt, mine, scan_sh, dbase, lbase);
  loc_off[tid] = lbase;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t idx = 64u * kSortItems * w + 64u * r + lane;
    if (idx < n_in) {
      const uint32_t d = (uint32_t)(k[r] >> shift) & kSortMask;
      const uint32_t p = loc_off[d] + rk[r];
      sk[p] = k[r];
      sv[p] = v[r];
    }
  }
  // look back for the prefix of digit tid over the earlier tiles
  uint32_t prefix = 0;
  if (tb != first_tile) {
    // windows of up to 16 predecessors read at once; walk down from the
    // nearest, adding counts, until a tile that holds its inclusive prefix
    uint32_t q = tb;                 // tiles [first_tile, q) remain
    uint32_t spin = 0;
    for (;;) {
      constexpr int kW = 16;
      const uint32_t avail = min(q - first_tile, (uint32_t)kW);
      uint32_t x[kW];
#pragma unroll
      for (int j = 0; j < kW; ++j)
        x[j] = (uint32_t)j < avail
                   ? __hip_atomic_load(status + (size_t)(q - 1 - j) * kSortDigits + tid,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                   : 0u;
      uint32_t used = 0;
      bool done = false;
#pragma unroll
      for (int j = 0; j < kW; ++j) {
        if (done || (uint32_t)j != used || used >= avail) continue;
        if ((x[j] >> 30) == 0u) continue;          // not published yet: poll again
        prefix += x[j] & kStVal;
        ++used;
        done = (x[j] & kStIncl) != 0u;
      }
      if (done) break;
      q -= used;                                   // q > first_tile: the first tile is inclusive
      if (used == 0) {
        if (++spin >= (1u << 18)) {
          set_err(err, TG_ERR_SORT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __hip_atomic_store(st, kStIncl | (prefix + mine), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  glob_off[tid] = (uint32_t)soff + dbase + prefix;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t idx = r * (uint32_t)kSortThreads + tid;
    if (idx < n_in) {
      const uint64_t kk = sk[idx];
      const uint32_t d = (uint32_t)(kk >> shift) & kSortMask;
      const uint32_t dst = glob_off[d] + (idx - loc_off[d]);
      kout[dst] = kk;
      vout[dst] = sv[idx];
      if (rank) rank[sv[idx]] = dst;   // last pass: caller index -> sorted position
    }
  }
}

// Sorted particles {x, y, z, m}; the masses come with them when the caller
// has them at build time (else the moments pass fills them in).
__global__ void k_gather(const int32_t *__restrict__ gate, const double *__restrict__ pos,
                         const double *__restrict__ mass, const uint32_t *__restrict__ rank,
                         int64_t n, double4 *__restrict__ spart, uint32_t *err) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  bool bad = false;
  // caller order in, sorted order out: the reads are coalesced, each
  // particle is one 32-byte write (reading the caller's arrays in sorted
  // order would fetch a cache line per 24-byte position and 8-byte mass)
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double m = 0.0;
    if (mass) {
      m = mass[i];
      bad |= !(m > 0.0) || !isfinite(m);
    }
    spart[rank[i]] = make_double4(pos[3 * (size_t)i], pos[3 * (size_t)i + 1],
                                  pos[3 * (size_t)i + 2], m);
  }
  if (bad) set_err(err, TG_ERR_MASS);
}

hipError_t launch_cube_keys(tg_ctx *c, const double *pos) {
  Buffers &b = c->b;
  const int nt = (int)c->n_tiles;
  if (nt > 0)
    hipLaunchKernelGGL(k_cube_part, dim3(nt), dim3(256), 0, c->stream, c->gate, pos,
                       b.tiles, b.cube_part, b.err);
  hipLaunchKernelGGL(k_cube_final, dim3(c->S), dim3(256), 0, c->stream, c->gate,
                     b.cube_part, b.sys_tile0, b.cube);
  // the sort takes its input from the second buffers (an odd number of
  // passes leaves the result in the first)
  if (nt > 0 && c->max_level > kMaxLevel)
    // first words in caller order to key[0], second words to klo[1] (sorted first)
    hipLaunchKernelGGL(k_keys<true>, dim3(nt), dim3(256), 0, c->stream, c->gate, pos, b.tiles,
                       b.sys_tile0, c->S, b.cube, b.key[0], b.klo[1], b.val[1], b.hist,
                       sort_hist_words(c->S, nt));
  else if (nt > 0)
    hipLaunchKernelGGL(k_keys<false>, dim3(nt), dim3(256), 0, c->stream, c->gate, pos, b.tiles,
                       b.sys_tile0, c->S, b.cube, b.key[1], nullptr, b.val[1], b.hist,
                       sort_hist_words(c->S, nt));
  return hipGetLastError();
}

// The passes of a sort whose input is in (kb, vb): passes alternate
// between the two buffer pairs and the result ends in (ka, va).
// rank (may be null): the last pass also writes each caller index's sorted
// position.
static hipError_t sort_passes(tg_ctx *c, uint64_t *ka, uint32_t *va, uint64_t *kb, uint32_t *vb,
                              uint32_t *rank) {
  static_assert(kSortPasses % 2 == 1, "the input starts in the second buffers");
  Buffers &b = c->b;
  const int nt = (int)c->n_tiles;
  // [tickets | pad | counts [S][passes][digits] | status [passes][nt][digits]],
  // all zero: cleared by the kernel before the sort (k_keys, k_gather_hi)
  uint32_t *tickets = b.hist, *cnt = b.hist + kSortStatusBase;
  uint32_t *status = cnt + (size_t)c->S * kSortPasses * kSortDigits;
  hipLaunchKernelGGL(k_sort_count, dim3(nt), dim3(256), 0, c->stream, c->gate, kb, b.tiles,
                     b.sys_tile0, c->S, cnt);
  uint64_t *k2[2] = {ka, kb};
  uint32_t *v2[2] = {va, vb};
  for (int pass = 0; pass < kSortPasses; ++pass) {
    const int dst = pass & 1, src = dst ^ 1;
    hipLaunchKernelGGL(k_sort_pass, dim3(nt), dim3(kSortThreads), 0, c->stream, c->gate, k2[src],
                       v2[src], k2[dst], v2[dst], b.tiles, b.sys_tile0, c->S, b.sysoff, pass,
                       cnt, status + (size_t)pass * kSortDigits * nt, tickets + pass,
                       b.err, pass == kSortPasses - 1 ? rank : nullptr);
  }
  return hipGetLastError();
}

// 42 levels, between the two sort phases: first words in the order of the
// first phase (sorted by the second word) and that order itself, both into
// the second buffers where the next phase starts.
__global__ void k_gather_hi(const int32_t *__restrict__ gate, const uint64_t *__restrict__ hi,
                            const uint32_t *__restrict__ perm, int64_t n,
                            uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                            uint32_t *__restrict__ zero, int64_t nzero) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  // the sort's counters and tile status, cleared for the second sort
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nzero;
       w += (int64_t)gridDim.x * blockDim.x)
    zero[w] = 0u;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = perm[r];
    kout[r] = hi[p];
    vout[r] = p;
  }
}

hipError_t launch_sort(tg_ctx *c) {
  Buffers &b = c->b;
  const int nt = (int)c->n_tiles;
  if (nt == 0) return hipSuccess;
  if (c->max_level <= kMaxLevel)      // key[1] / val[1] -> key[0] / val[0]
    return sort_passes(c, b.key[0], b.val[0], b.key[1], b.val[1], b.rank);
  // 42 levels, least significant word first: sort by the second words,
  // carry the first words into that order, sort them (stable), then the
  // second words of the final order from the positions
  hipError_t e = sort_passes(c, b.klo[0], b.val[0], b.klo[1], b.val[1], nullptr);
  if (e != hipSuccess) return e;
  const int g = (int)std::min<int64_t>((c->n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_gather_hi, dim3(g), dim3(256), 0, c->stream, c->gate, b.key[0],
                     b.val[0], c->n, b.key[1], b.val[1], b.hist, sort_hist_words(c->S, nt));
  return sort_passes(c, b.key[0], b.val[0], b.key[1], b.val[1], b.rank);
}

// 42 levels: the second key words of the sorted particles (klo[0]).
hipError_t launch_keys_lo(tg_ctx *c, const double *pos) {
  Buffers &b = c->b;
  if (c->max_level <= kMaxLevel || c->n == 0) return hipSuccess;
  const int g = (int)std::min<int64_t>((c->n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_keys_lo_sorted, dim3(g), dim3(256), 0, c->stream, c->gate, pos,
                     b.val[0], c->n, b.sysoff, c->S, b.cube, b.klo[0]);
  return hipGetLastError();
}

hipError_t launch_gather(tg_ctx *c, const double *pos, const double *mass) {
  if (c->n == 0) return hipSuccess;
  int g = (int)std::min<int64_t>((c->n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_gather, dim3(g), dim3(256), 0, c->stream, c->gate, pos, mass,
                     c->b.rank, c->n, c->b.spart, c->b.err);
  return hipGetLastError();
}

}  // namespace tg
