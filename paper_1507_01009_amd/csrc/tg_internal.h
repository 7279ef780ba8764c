// Internal declarations shared by the HIP translation units of libtg.so.
// Device data layouts (all in HBM, owned by the context):
//   sorted particles   spart[N]   double4 {x, y, z, m}      (32 B each)
//   sort keys / perm   key[N] u64, perm[N] u32 (sorted rank -> caller index),
//                      rank[N] u32 (caller index -> sorted rank, written by
//                      the last sort pass)
//   nodes (SoA)        level u8, nchild u8, first u32, count u32, child u32,
//                      parent u32, sys u32; com double4 {cx, cy, cz, side^2};
//                      mom double[8] {M, Sxx, Syy, Szz, Sxy, Sxz, Syz, 0}
//   groups             uint4 {first, count, node, system}
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "tg.h"

namespace tg {

constexpr int kBits = 21;             // key bits per axis (one key word)
constexpr int kMaxLevel = 21;         // deepest octree level of one key word
constexpr int kLevels = kMaxLevel + 1;
constexpr int kMaxLevelDeep = 42;     // two key words (tg_config.key_levels = 42)
constexpr int kLevelsMax = kMaxLevelDeep + 1;
constexpr uint32_t kNone = 0xffffffffu;
constexpr int kQueueStride = 64;      // words between the walk's queue counters (256 bytes)
constexpr int kMaxLeaf = 16;          // largest n_L (bounds the walk's LDS queue)
constexpr int kMaxGroup = 128;        // targets of one walk (one wave, up to 3 per lane)
constexpr int kMaxSys = 256;
constexpr int kSortThreads = 512;             // one digit per thread in the sort passes
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;   // 4096 keys per tile
constexpr int kSortStatusBase = 64;               // words before the digit counts (tickets + pad)
constexpr int kSortBits = 9, kSortDigits = 1 << kSortBits, kSortPasses = 7;
// sort scratch words: tickets and pad, digit counts [S][passes][digits],
// tile status [passes][tiles][digits]
constexpr int64_t sort_hist_words(int64_t S, int64_t tiles) {
  return kSortStatusBase + (int64_t)kSortPasses * kSortDigits * (S + tiles);
}
constexpr int kScanBlocks = 256;
constexpr int kMaxWavesPerCU = 16;
constexpr int kMaxExternal = 1024;               // SMBHs / external point masses
constexpr int kMaxChain = 256;                   // chain members
constexpr int kChainBlocks = 1024;               // partial sums of the chain particle's force
constexpr int kSegSlots = 8;                     // cached direct-sum segment tables
constexpr int kSegSlotLen = 2 * (kMaxSys + 1);

// A tile of consecutive particles inside one system (sort, cube, keys).
struct Tile {
  uint32_t start, end;    // particle range
};

// Per-level bookkeeping kept on the device so that graph replays need no
// host round trip.  lvl[l] = first node id of level l, lvl[l+1] = end.
struct TreeCounters {
  uint32_t lvl[kLevelsMax + 2];
  uint32_t n_nodes;
  uint32_t n_groups;
  uint32_t n_active_groups;
  uint32_t overflow;         // node capacity exceeded during this build
  uint32_t pad[11];
  unsigned long long n_p2p, n_p2m, n_targets, n_walked;      // last walk
  unsigned long long cum_p2p, cum_p2m, cum_targets, cum_walked;  // since reset
  // walk work counters, one queue per XCD, each on a line of its own
  // (kQueueStride words apart): eight counters on one line made every
  // group's fetch wait on the other XCDs' atomics (walk 2.4% slower)
  alignas(256) uint32_t xq[8 * kQueueStride];
};

struct Buffers {
  // system layout
  int64_t *sysoff = nullptr;      // [S+1]
  double *cube = nullptr;         // [S][4]
  double *cube_part = nullptr;    // [tiles][6] per-tile min / max
  Tile *tiles = nullptr;          // [tiles]
  uint32_t *sys_tile0 = nullptr;  // [S+1] first tile of each system
  uint32_t *root_of = nullptr;    // [S]
  // sort
  uint64_t *key[2] = {nullptr, nullptr};
  uint64_t *klo[2] = {nullptr, nullptr};   // 42 levels: the keys' last 21 digits
  uint32_t *val[2] = {nullptr, nullptr};
  uint32_t *hist = nullptr;       // sort: [tickets | digit counts [S][7][512] | tile status [7][tiles][512]]
  uint32_t *rank = nullptr;       // [N]
  double4 *spart = nullptr;       // [N]
  // nodes
  uint8_t *level = nullptr, *nchild = nullptr;
  uint32_t *first = nullptr, *count = nullptr, *child = nullptr,
           *parent = nullptr, *nsys = nullptr;
  double4 *com = nullptr;
  double *mom = nullptr;          // [nodes][8]
  uint4 *ninfo = nullptr;         // [nodes] {first, count, child, nchild} for the walk
  double4 *rel = nullptr;         // [nodes][2] relative test {enlarged cube lo, (G M) s^2} {hi, 0}
  double *side = nullptr;         // [nodes] opening size: the cell side, or refitted
  double4 *bbox = nullptr;        // [nodes][2] particle bounding box {lo, -} {hi, -} (refit)
  int32_t *refit_flag = nullptr;  // [1] > 0: moments with bounding boxes take refitted sizes
  int32_t *refit_gates = nullptr; // [3] block steps: rebuild now, refit now, a build exists
  double4 *cell = nullptr;        // [nodes][2] walk records {Qxx,Qyy,Qzz,-T eps^2} {Qxy,Qxz,Qyz,M}
                                  // (FP64; the mixed path uses the first half as float4[nodes][2])
  uint8_t *lcp = nullptr;         // [N + 64] common leading digits with predecessor
  // flat octree build, per 256-particle tile (FT = tiles of max_particles)
  uint16_t *fl_lt = nullptr;      // [N] first | last node level starting at a particle
  uint64_t *fl_bits = nullptr;    // [levels][4 (FT + 1)] node-start bitmaps
  uint32_t *fl_cnt = nullptr;     // [levels][FT + 1] nodes per tile -> prefix
  uint32_t *fl_fst = nullptr;     // [levels][FT + 1] first run start -> next after tile
  uint32_t *fl_tot = nullptr;     // [levels] nodes per level
  // groups
  uint32_t *gflag = nullptr;      // [N + 1] group starts / scan
  uint4 *groups = nullptr;        // [N]
  uint32_t *aflag = nullptr;      // [N + 1] active-group flags / scan
  uint32_t *alist = nullptr;      // [N] active group ids
  uint32_t *acnt = nullptr;       // [N] active targets per group
  uint32_t *gorder = nullptr;     // [N] active group ids in the force walk's order
  double *abox = nullptr;         // [N][6] box of active targets per group
  double *arel = nullptr;         // [N] relative test: (alpha alpha) min |a_old|^2 per group
  // chain coupling
  uint8_t *cflag = nullptr;       // [N + 1] selection flags (the perturber mask after Eq. 2)
  uint32_t *ctile = nullptr;      // [N / 1024 + 2] flags per 1024-particle tile
  double *cpart = nullptr;        // [kChainBlocks][6] compensated partials of the chain particle's force
  uint8_t *sact = nullptr;        // [N] active flag per sorted particle
  // active sets of block steps, per 1024-star tile
  uint32_t *atile = nullptr;      // [N / 1024 + 2] count | (finest level + 1) << 16
  uint32_t *aoff = nullptr;       // [N / 1024 + 2] exclusive offsets, then the total
  int32_t *ainfo = nullptr;       // [2] active count, finest occupied level of free stars
  // walk
  uint32_t *frontier = nullptr;   // [waves][2][frontier_cap]
  unsigned long long *wtot = nullptr;   // [waves][4] force walk totals per workgroup
  uint32_t *wl_count = nullptr;   // [N][2] list sizes (list mode)
  uint32_t *wl_off = nullptr;     // [2N + 1] list offsets (list mode)
  // scan scratch and counters
  uint32_t *scan_part = nullptr;  // [kScanBlocks + 1]
  uint32_t *scan_total = nullptr; // [4]
  TreeCounters *ctr = nullptr;
  uint32_t *err = nullptr;        // device error bits
  // direct sums
  double *dpart = nullptr;        // partial sums for few-target direct sums
  int64_t *dseg = nullptr;        // [kSegSlots][2 * (S+1)] segment offsets
  int32_t *ext_seg = nullptr;     // [S+1] external masses of each system
  int64_t dpart_cap = 0;
};

}  // namespace tg

struct tg_ctx {
  tg_config cfg;
  hipStream_t stream = nullptr;
  int device = 0;
  int n_cu = 256;
  int64_t n = 0;
  int32_t S = 0;
  int32_t leaf_size = 8, group_size = 64, waves_per_cu = 8;
  int32_t max_level = tg::kMaxLevel;   // octree depth: 21, or 42 with two key words
  int64_t max_nodes = 0;
  int64_t max_tiles = 0;
  int64_t flat_tiles = 0;          // 256-particle tiles of max_particles
  // device count that gates the build, moments and walk kernels (they
  // return at once when it is <= 0: no active particle); null = always run
  const int32_t *gate = nullptr;
  // opening test of the walk: TG_MAC_GEOMETRIC, or TG_MAC_RELATIVE with
  // alpha and the old accelerations (null: the system's acc in tg_forces)
  int32_t mac = 0;
  // pair softening of the walk, the SMBH terms and the direct sums:
  // TG_SOFT_PLUMMER or TG_SOFT_SPLINE
  int32_t soft = 0;
  double alpha = 0.0;
  const double *acc_old = nullptr;
  // masses gathered into the sorted particles by the last build (or null)
  const double *mass_gathered = nullptr;
  int64_t n_tiles = 0;
  bool have_tree = false, have_moments = false;
  bool capturing = false;
  // walk-kernel timing (tg_set_profiling): ring of event pairs
  bool profiling = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  int64_t ev_head = 0, ev_tail = 0;     // recorded / resolved pairs
  double prof_ms = 0.0;
  int64_t prof_n = 0;
  std::vector<int64_t> sysoff_host;   // layout of the last build
  // external point masses (tg_set_external)
  const double *ext_pos = nullptr, *ext_mass = nullptr, *ext_eps = nullptr;
  int32_t n_ext = 0;
  std::vector<int32_t> ext_seg_host;
  std::vector<std::vector<int64_t>> dseg_host;  // tables held in the device slots
  int dseg_next = 0;
  // bumped whenever a device table that a captured graph may point into is
  // overwritten (system layout and tiles, an evicted segment slot, the
  // external segments); a graph replays only at its capture's generation
  uint64_t layout_gen = 0;
  int64_t *host_words = nullptr;  // pinned [4]: device words read back by tg_step_blocks
  tg::Buffers b;
};

struct tg_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const tg_ctx *ctx = nullptr;   // the context it was captured on
  uint64_t gen = 0;              // ctx->layout_gen at the end of the capture
};

namespace tg {

// error reporting (tg_runtime.hip)
tg_status fail(tg_status st, const std::string &msg);
tg_status hip_fail(hipError_t e, const char *what);
// msg must outlive the thread's next error (a literal or a HIP string)
tg_status fail_literal(tg_status st, const char *msg);

// Host exceptions never cross the C ABI: the entry points (and the helpers)
// that build host containers are function-try-blocks ending in this
// handler, which turns an allocation failure into TG_ENOMEM and any other
// exception (e.g. a thread that cannot start) into TG_EINTERNAL.
#define TG_HOST_CATCH(name)                                               \
  catch (const std::bad_alloc &) {                                        \
    return tg::fail(TG_ENOMEM, name ": host allocation failed");          \
  }                                                                       \
  catch (const std::exception &e_) {                                      \
    return tg::fail(TG_EINTERNAL, std::string(name ": ") + e_.what());    \
  }

#define TG_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return tg::hip_fail(e_, #call); \
  } while (0)

// ---- launchers (each .hip file owns its kernels) ----
// k_scan.hip: exclusive scan of u32; n from n_dev (if non-null) else n_host.
// Writes the total to *total_dev (if non-null).  in may equal out.
hipError_t scan_u32(const uint32_t *in, uint32_t *out, uint32_t n_host,
                    const uint32_t *n_dev, uint32_t *total_dev,
                    uint32_t *part, hipStream_t s,
                    const int32_t *gate = nullptr);
hipError_t fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s,
                    const int32_t *gate = nullptr);
hipError_t fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s,
                   const int32_t *gate = nullptr);

// Separately rounded double operations for the decisions that must equal
// the plain definition bit for bit (keys, opening tests, selections): the
// operations are created without the contraction flag, so the backend never
// fuses them into FMAs, whatever the caller's contraction setting.
__device__ __forceinline__ double dmul(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}
__device__ __forceinline__ double dadd(double a, double b) {
#pragma clang fp contract(off)
  return a + b;
}
__device__ __forceinline__ double dsub(double a, double b) {
#pragma clang fp contract(off)
  return a - b;
}

// Geometric centre g of node v's cell, from the integer cell coordinates in
// the key prefix of its first particle: g_k = lo_k + (i_k + 0.5) s, with
// s = L 2^-level returned; every operation rounded separately.  Reads one
// key word, so l <= 21 (trees of 42 levels have neither refits nor the
// relative test, the two callers).
__device__ __forceinline__ double cell_centre(uint32_t v, int l, const uint32_t *first,
                                              const uint32_t *nsys, const uint64_t *skey,
                                              const double *cube, double g[3]) {
  const double *cb = cube + 4 * (size_t)nsys[v];
  const double s = ldexp(cb[3], -l);
  const uint64_t pre = l ? skey[first[v]] >> (3 * (kMaxLevel - l)) : 0ull;
  uint32_t ic[3] = {0u, 0u, 0u};
  for (int j = 0; j < l; ++j) {
    const uint32_t d = (uint32_t)(pre >> (3 * j)) & 7u;
    ic[0] |= ((d >> 2) & 1u) << j;
    ic[1] |= ((d >> 1) & 1u) << j;
    ic[2] |= (d & 1u) << j;
  }
  for (int k = 0; k < 3; ++k) g[k] = dadd(cb[k], dmul(dadd((double)ic[k], 0.5), s));
  return s;
}

// Cubic-spline softening (the Monaghan-Lattanzio kernel with support 2h,
// h = the pair's softening): psi and psi_1 of a pair at distance r, in
// double with correctly rounded divisions and square roots, for the SMBH
// terms and the direct sums.  A pair's acceleration is -m psi_1 x and its
// potential -m psi; beyond 2h (and for h = 0) they are 1/r and 1/r^3.
__device__ __forceinline__ void spline_pair_dp(double r, double h, double &p0, double &p1) {
#pragma clang fp contract(off)
  if (!(r < 2.0 * h)) {
    p0 = 1.0 / r;
    p1 = p0 * p0 * p0;
    return;
  }
  const double ih = 1.0 / h, u = r * ih, u2 = u * u, ih3 = ih * ih * ih;
  if (u < 1.0) {
    p0 = ih * (1.4 + u2 * (-2.0 / 3.0 + u2 * (0.3 - 0.1 * u)));
    p1 = ih3 * (4.0 / 3.0 + u2 * (-1.2 + 0.5 * u));
  } else {
    const double iu = 1.0 / u;
    p0 = ih * (1.6 + u2 * (-4.0 / 3.0 + u * (1.0 + u * (-0.3 + u / 30.0))) - iu / 15.0);
    p1 = ih3 * (8.0 / 3.0 + u * (-3.0 + u * (1.2 - u / 6.0)) - iu * iu * iu / 15.0);
  }
}

// Compensated double sum (error-free TwoSum with a running correction),
// used by the direct sums, the chain coupling and the leaf moments.
struct CSum {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double x) {
    double t = s + x;
    double bp = t - s;
    c += (s - (t - bp)) + (x - bp);
    s = t;
  }
  __device__ __forceinline__ void merge(const CSum &o) {
    add(o.s);
    c += o.c;
  }
  __device__ __forceinline__ double get() const { return s + c; }
};

// k_keys.hip
hipError_t launch_cube_keys(tg_ctx *c, const double *pos);
hipError_t launch_sort(tg_ctx *c);
// 42 levels: second key words of the sorted particles (after launch_sort)
hipError_t launch_keys_lo(tg_ctx *c, const double *pos);
hipError_t launch_gather(tg_ctx *c, const double *pos, const double *mass);

// k_tree.hip
hipError_t launch_tree_build(tg_ctx *c);
hipError_t launch_groups(tg_ctx *c);
// gates[0] = rebuild, gates[1] = refit (and the refit flag) for substep k
hipError_t launch_refit_gates(tg_ctx *c, const int32_t *n_act, const int64_t *k, int32_t every);

// k_moments.hip
// refit: bounding boxes and refitted opening sizes (the tree is an earlier
// build; the gather with its permutation was done by the caller)
hipError_t launch_moments(tg_ctx *c, const double *mass, bool gathered, bool refit = false);

// k_walk.hip
// acc_old != nullptr: also the relative test's per-group thresholds
hipError_t launch_active_groups(tg_ctx *c, const int32_t *idx,
                                const int32_t *n_act, const double *acc_old,
                                double alpha);
// rel: relative opening test (needs launch_active_groups with acc_old)
hipError_t launch_walk_forces(tg_ctx *c, double eps, double theta,
                              double *acc, double *pot, hipEvent_t before,
                              hipEvent_t after, bool rel);
hipError_t launch_counts_reset(tg_ctx *c);
hipError_t launch_walk_lists(tg_ctx *c, double theta, int pass,
                             int64_t *info, int64_t cap_groups, uint32_t *ids,
                             int64_t cap_ids, bool rel);

// k_chain.hip
hipError_t launch_chain_select(tg_ctx *c, const double *pos, const double *mass, int64_t n,
                               const uint8_t *excl, const double center[3], bool tidal,
                               double cst, double lim, int32_t *idx, int32_t cap,
                               int32_t *n_out);
hipError_t launch_chain_predict(tg_ctx *c, const tg_chain *ch, const double *vel, double dt,
                                const double rp[3], const double v[3], double *out_pos,
                                double *out_vel, double *out_mass);
// the stars' part of a block substep in two stages (tg_runtime.hip)
tg_status block_stars_kick(tg_ctx *c, const tg_system *y, const tg_blocks *b);
tg_status block_stars_drift(tg_ctx *c, const tg_system *y, const tg_blocks *b);

// several chains (tg_chains_forces): at most kMaxChains, the chain
// particles' mutual forces added from the host
constexpr int kMaxChains = 16;
struct ChainVec { double v[3 * kMaxChains]; };
hipError_t launch_add_host_vector(tg_ctx *c, double *out, const ChainVec &add, int n3);
// hybrid driver: rows of 3 doubles to (to_rows) or from indexed rows, and
// per-row masses and flags
hipError_t launch_gather_bytes(tg_ctx *c, uint8_t *dst, const uint8_t *src, const int32_t *idx,
                               int n);
hipError_t launch_move_rows(tg_ctx *c, double *dst, const double *src, const int32_t *idx, int n,
                            bool to_rows);
hipError_t launch_set_rows(tg_ctx *c, double *mass, uint8_t *flag, const int32_t *idx,
                           const double *val, const uint8_t *f, int n);
hipError_t launch_chain_forces(tg_ctx *c, const tg_chain *ch, const int32_t *idx,
                               const int32_t *n_act, double *acc, double *pot,
                               double *com_acc, double *member_acc);

// k_direct.hip
// stars' drift fused with their sums on the SMBHs (one system); fits says
// whether the few-target sum path applies (then the totals are bit-equal)
bool drift_smbh_fits(const tg_ctx *c, int64_t n, int32_t nb);
hipError_t launch_drift_smbh(tg_ctx *c, double *pos, const double *vel, const uint8_t *frozen,
                             int64_t n, double dt, const double *mass, double eps,
                             const double *bpos, const double *beps, int32_t nb,
                             double *bacc, double *bpot);
hipError_t launch_direct(tg_ctx *c, const int64_t *dseg, const double *spos,
                         const double *sm, const double *seps, double seps_all,
                         int64_t ns, const double *tpos,
                         const double *teps, int64_t nt, int nseg,
                         int64_t max_seg_src, int self_pairs, int accumulate,
                         double *acc, double *pot);
// The same sums on any stream, softening and partial-sum buffer (part_cap
// doubles, at least 2^19): the context's own, or the allocation-free one.
struct DirectEnv {
  hipStream_t stream;
  int soft;
  double *part;
  int64_t part_cap;
};
hipError_t launch_direct_env(const DirectEnv &e, const int64_t *dseg, const double *spos,
                             const double *sm, const double *seps, double seps_all,
                             const double *tpos, const double *teps, int64_t nt, int nseg,
                             int64_t max_seg_src, int self_pairs, int accumulate,
                             double *acc, double *pot);

// k_integrate.hip
// frozen: [n] nonzero = star held still (ghost chain members in whole steps)
hipError_t launch_kick(tg_ctx *c, double *vel, const double *acc, int64_t n,
                       const int32_t *idx, const int32_t *n_act,
                       const uint8_t *level, double dt, const int64_t *k,
                       int skip_k0, const uint8_t *frozen = nullptr);
hipError_t launch_kick_drift(tg_ctx *c, double *pos, double *vel, const double *acc,
                             const uint8_t *frozen, int64_t n, double *bpos, double *bvel,
                             const double *bacc, int64_t nb, double dt, bool drift);
hipError_t launch_drift(tg_ctx *c, double *pos, const double *vel, int64_t n,
                        double dt, const uint8_t *frozen = nullptr);
hipError_t launch_levels(tg_ctx *c, const double *acc, const double *vel,
                         const double *t4e2, const double *t2e2v, int64_t n,
                         const int32_t *idx, const int32_t *n_act, double dt_max, int nlev,
                         const int64_t *k, uint8_t *level);
hipError_t launch_active_set(tg_ctx *c, const uint8_t *level, int64_t n,
                             int nlev, const int64_t *k, int k_add,
                             int32_t *idx, int32_t *n_out, const uint8_t *frozen = nullptr);
hipError_t launch_counter_add(tg_ctx *c, int64_t *k, int64_t inc);
// SMBH kicks and drift of one block substep, then k += 1 (and *n_act = 0 if
// n_act is given)
hipError_t launch_bh_substep(tg_ctx *c, double *pos, double *vel, const double *acc, int32_t n,
                             double dt, int64_t *k, int32_t *n_act);

// ---- small device helpers ----
__device__ __forceinline__ unsigned lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// number of set bits of `mask` in lanes below this one
__device__ __forceinline__ unsigned lanes_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}
__device__ __forceinline__ void set_err(uint32_t *err, uint32_t bit) {
  atomicOr(err, bit);
}

// Exclusive scan of one value per thread across the block (multiple of 64
// threads); sh needs blockDim/64 entries.  Contains two barriers.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh,
                                         uint32_t &total) {
  const unsigned lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= (unsigned)o) x += y;
  }
  if (lane == 63u) sh[w] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  const unsigned nw = blockDim.x >> 6;
  for (unsigned i = 0; i < nw; ++i) {
    uint32_t t = sh[i];
    base += (i < w) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return base + x - v;
}

}  // namespace tg
