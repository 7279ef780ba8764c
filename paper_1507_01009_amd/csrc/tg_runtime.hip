// Host side of libtg.so: the C ABI declared in include/tg.h.  Validates
// arguments on the host, owns every device buffer (allocated once in
// tg_create, so any sequence of calls is graph-capturable), sequences the
// kernel launches of each step on the context's stream, and reports device
// error bits through tg_sync.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "tg_internal.h"

namespace {
thread_local std::string g_last_error;
}

namespace tg {

// A message that is a string literal (or a HIP runtime string) is kept by
// pointer, so reporting it allocates nothing.
thread_local const char *g_last_literal = nullptr;

tg_status fail(tg_status st, const std::string &msg) {
  g_last_error = msg;
  g_last_literal = nullptr;
  return st;
}

tg_status fail_literal(tg_status st, const char *msg) {
  g_last_literal = msg;
  return st;
}

tg_status hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  g_last_literal = nullptr;
  return TG_EHIP;
}

template <class T>
static hipError_t dalloc(T **p, size_t count) {
  return hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
}

}  // namespace tg

using namespace tg;

extern "C" {

const char *tg_last_error(void) { return g_last_literal ? g_last_literal : g_last_error.c_str(); }

const char *tg_version(void) {
  return "libtg gfx950 (HIP, wave64, FP64 + mixed walk)";
}

void tg_default_config(tg_config *cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->max_particles = 1;
  cfg->max_systems = 1;
  cfg->leaf_size = 8;
  cfg->group_size = 64;
  cfg->precision = TG_FP64;
  cfg->max_nodes = 0;
  cfg->frontier_cap = 0;
  cfg->waves_per_cu = 0;
  cfg->G = 1.0;
}

static void free_all(tg_ctx *c) {
  Buffers &b = c->b;
  void *ptrs[] = {b.sysoff, b.cube, b.cube_part, b.tiles, b.sys_tile0,
                  b.root_of, b.key[0], b.key[1], b.val[0], b.val[1], b.hist,
                  b.rank, b.spart, b.level, b.nchild, b.first, b.count,
                  b.child, b.parent, b.nsys, b.com, b.mom, b.ninfo, b.cell, b.lcp, b.fl_lt, b.fl_bits, b.fl_cnt, b.fl_fst, b.fl_tot, b.gflag,
                  b.groups, b.aflag, b.alist, b.acnt, b.gorder, b.abox, b.sact, b.frontier, b.wtot,
                  b.wl_count, b.wl_off, b.scan_part, b.scan_total, b.ctr,
                  b.err, b.dpart, b.dseg, b.ext_seg, b.rel, b.side, b.bbox,
                  b.refit_flag, b.refit_gates, b.arel, b.cflag, b.ctile, b.cpart,
                  b.atile, b.aoff, b.ainfo, b.klo[0], b.klo[1]};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  b = Buffers();
  if (c->host_words) (void)hipHostFree(c->host_words);
  c->host_words = nullptr;
}

tg_status tg_create(const tg_config *cfg_in, void *stream, tg_ctx **out) {
  if (!cfg_in || !out) return fail(TG_EINVAL, "tg_create: NULL argument");
  *out = nullptr;
  tg_config cfg = *cfg_in;
  if (cfg.max_particles < 1 || cfg.max_particles > (int64_t)0x7fffffff / 2)
    return fail(TG_EINVAL, "tg_create: max_particles out of range");
  if (cfg.max_systems < 1 || cfg.max_systems > kMaxSys)
    return fail(TG_EINVAL, "tg_create: max_systems must be in 1..256");
  if (cfg.leaf_size < 1 || cfg.leaf_size > kMaxLeaf)
    return fail(TG_EINVAL, "tg_create: leaf_size must be in 1..16");
  if (cfg.group_size < 1 || cfg.group_size > kMaxGroup)
    return fail(TG_EINVAL, "tg_create: group_size must be in 1..128");
  if (cfg.precision != TG_FP64 && cfg.precision != TG_MIXED)
    return fail(TG_EINVAL, "tg_create: unknown precision");
  if (!(cfg.G > 0.0) || !std::isfinite(cfg.G))
    return fail(TG_EINVAL, "tg_create: G must be positive");
  if (cfg.max_nodes == 0)
    cfg.max_nodes = 2 * cfg.max_particles + 64 * (int64_t)cfg.max_systems;
  if (cfg.max_nodes < cfg.max_systems || cfg.max_nodes > (int64_t)0xfffffff0)
    return fail(TG_EINVAL, "tg_create: max_nodes out of range");
  if (cfg.frontier_cap == 0) cfg.frontier_cap = 16384;
  if (cfg.frontier_cap < 64) return fail(TG_EINVAL, "tg_create: frontier_cap < 64");
  if (cfg.waves_per_cu == 0) cfg.waves_per_cu = 16;
  if (cfg.waves_per_cu < 1 || cfg.waves_per_cu > kMaxWavesPerCU)
    return fail(TG_EINVAL, "tg_create: waves_per_cu must be in 1..16");
  if (cfg.key_levels == 0) cfg.key_levels = kMaxLevel;
  if (cfg.key_levels != kMaxLevel && cfg.key_levels != kMaxLevelDeep)
    return fail(TG_EINVAL, "tg_create: key_levels must be 21 or 42");

  tg_ctx *c = new tg_ctx();
  c->cfg = cfg;
  c->stream = (hipStream_t)stream;
  c->leaf_size = cfg.leaf_size;
  c->group_size = cfg.group_size;
  c->waves_per_cu = cfg.waves_per_cu;
  c->max_nodes = cfg.max_nodes;
  c->max_level = cfg.key_levels;
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount,
                              c->device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "tg_create: device query");
  }
  const int64_t N = cfg.max_particles, S = cfg.max_systems, NN = cfg.max_nodes;
  c->max_tiles = (N + kSortTile - 1) / kSortTile + S;
  Buffers &b = c->b;
  b.dpart_cap = (int64_t)8 * 131072;
  const int64_t waves = (int64_t)c->n_cu * kMaxWavesPerCU;
  hipError_t a = hipSuccess;
  auto A = [&](hipError_t r) { if (a == hipSuccess) a = r; };
  A(dalloc(&b.sysoff, S + 1));
  A(dalloc(&b.cube, 4 * S));
  A(dalloc(&b.cube_part, 6 * c->max_tiles));
  A(dalloc(&b.tiles, c->max_tiles));
  A(dalloc(&b.sys_tile0, S + 1));
  A(dalloc(&b.root_of, S));
  A(dalloc(&b.key[0], N)); A(dalloc(&b.key[1], N));
  if (c->max_level > kMaxLevel) { A(dalloc(&b.klo[0], N)); A(dalloc(&b.klo[1], N)); }
  A(dalloc(&b.val[0], N)); A(dalloc(&b.val[1], N));
  A(dalloc(&b.hist, sort_hist_words(S, c->max_tiles)));
  A(dalloc(&b.rank, N));
  A(dalloc(&b.spart, N));
  A(dalloc(&b.level, NN)); A(dalloc(&b.nchild, NN));
  A(dalloc(&b.first, NN)); A(dalloc(&b.count, NN)); A(dalloc(&b.child, NN));
  A(dalloc(&b.parent, NN)); A(dalloc(&b.nsys, NN));
  A(dalloc(&b.com, NN)); A(dalloc(&b.mom, 8 * NN));
  A(dalloc(&b.ninfo, NN)); A(dalloc(&b.cell, 2 * NN)); A(dalloc(&b.rel, 2 * NN));
  A(dalloc(&b.side, NN)); A(dalloc(&b.bbox, 2 * NN)); A(dalloc(&b.refit_flag, 1));
  A(dalloc(&b.refit_gates, 3));
  c->flat_tiles = (N + 255) / 256;
  A(dalloc(&b.lcp, N + 64));
  A(dalloc(&b.fl_lt, std::max<int64_t>(N, 1)));
  const int64_t levels = c->max_level + 1;
  A(dalloc(&b.fl_bits, levels * 4 * (c->flat_tiles + 1)));
  A(dalloc(&b.fl_cnt, levels * (c->flat_tiles + 1)));
  A(dalloc(&b.fl_fst, levels * (c->flat_tiles + 1)));
  A(dalloc(&b.fl_tot, levels + 2));
  A(dalloc(&b.gflag, N + 1));
  A(dalloc(&b.groups, N));
  A(dalloc(&b.aflag, N + 1));
  A(dalloc(&b.alist, N)); A(dalloc(&b.acnt, N)); A(dalloc(&b.gorder, N));
  A(dalloc(&b.abox, 6 * N)); A(dalloc(&b.arel, N));
  A(dalloc(&b.cflag, N + 1)); A(dalloc(&b.ctile, N / 1024 + 2)); A(dalloc(&b.cpart, 6 * kChainBlocks));
  A(dalloc(&b.sact, N));
  A(dalloc(&b.atile, N / 1024 + 2)); A(dalloc(&b.aoff, N / 1024 + 2)); A(dalloc(&b.ainfo, 2));
  A(dalloc(&b.frontier, waves * 2 * (int64_t)cfg.frontier_cap));
  A(dalloc(&b.wtot, waves * 4));
  A(dalloc(&b.wl_count, 2 * N + 2));
  A(dalloc(&b.wl_off, 2 * N + 2));
  A(dalloc(&b.scan_part, kScanBlocks + 1));
  A(dalloc(&b.scan_total, 4));
  A(dalloc(&b.ctr, 1));
  A(dalloc(&b.err, 1));
  A(dalloc(&b.dpart, b.dpart_cap));
  A(dalloc(&b.dseg, kSegSlots * kSegSlotLen));
  A(dalloc(&b.ext_seg, kMaxSys + 1));
  if (a != hipSuccess) {
    free_all(c);
    delete c;
    return fail(TG_ENOMEM, std::string("tg_create: hipMalloc: ") + hipGetErrorString(a));
  }
  A(hipMemset(b.ctr, 0, sizeof(TreeCounters)));
  A(hipMemset(b.err, 0, sizeof(uint32_t)));
  A(hipMemset(b.refit_gates, 0, 3 * sizeof(int32_t)));
  A(hipHostMalloc((void **)&c->host_words, 4 * sizeof(int64_t), hipHostMallocDefault));
  A(hipDeviceSynchronize());
  if (a != hipSuccess) {
    free_all(c);
    delete c;
    return hip_fail(a, "tg_create: init");
  }
  *out = c;
  return TG_OK;
}

void tg_destroy(tg_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev_start) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev_stop) (void)hipEventDestroy(e);
  free_all(c);
  delete c;
}

tg_status tg_set_stream(tg_ctx *c, void *stream) {
  if (!c) return fail(TG_EINVAL, "tg_set_stream: NULL context");
  if (c->capturing) return fail(TG_ESTATE, "tg_set_stream: during capture");
  c->stream = (hipStream_t)stream;
  return TG_OK;
}

tg_status tg_set_sizes(tg_ctx *c, int32_t leaf_size, int32_t group_size) {
  if (!c) return fail(TG_EINVAL, "tg_set_sizes: NULL context");
  if (leaf_size < 1 || leaf_size > kMaxLeaf)
    return fail(TG_EINVAL, "tg_set_sizes: leaf_size must be in 1..16");
  if (group_size < 1 || group_size > kMaxGroup)
    return fail(TG_EINVAL, "tg_set_sizes: group_size must be in 1..128");
  c->leaf_size = leaf_size;
  c->group_size = group_size;
  c->have_tree = c->have_moments = false;
  return TG_OK;
}

// Upload the system layout and tile table if it changed since the last
// build (never during graph capture).
static tg_status set_layout(tg_ctx *c, int64_t n, const int64_t *off, int32_t S) try {
  std::vector<int64_t> so(S + 1);
  if (off) {
    for (int s = 0; s <= S; ++s) so[s] = off[s];
  } else {
    so[0] = 0;
    so[1] = n;
  }
  if (so[0] != 0 || so[S] != n)
    return fail(TG_EINVAL, "tg_build_tree: sys_off must start at 0 and end at N");
  for (int s = 0; s < S; ++s)
    if (so[s + 1] < so[s]) return fail(TG_EINVAL, "tg_build_tree: sys_off not ascending");
  if (so == c->sysoff_host && c->n == n && c->S == S) return TG_OK;
  if (c->capturing)
    return fail(TG_ESTATE, "tg_build_tree: system layout changed during graph capture");
  std::vector<Tile> tiles;
  std::vector<uint32_t> t0(S + 1);
  for (int s = 0; s < S; ++s) {
    t0[s] = (uint32_t)tiles.size();
    const int64_t ns = so[s + 1] - so[s];
    const uint32_t nts = (uint32_t)((ns + kSortTile - 1) / kSortTile);
    for (uint32_t k = 0; k < nts; ++k) {
      Tile t;
      t.start = (uint32_t)(so[s] + (int64_t)k * kSortTile);
      t.end = (uint32_t)std::min<int64_t>(so[s + 1], so[s] + (int64_t)(k + 1) * kSortTile);
      tiles.push_back(t);
    }
  }
  t0[S] = (uint32_t)tiles.size();
  if ((int64_t)tiles.size() > c->max_tiles)
    return fail(TG_ECAPACITY, "tg_build_tree: tile table too large");
  Buffers &b = c->b;
  ++c->layout_gen;
  TG_HIP(hipMemcpyAsync(b.sysoff, so.data(), sizeof(int64_t) * (S + 1),
                        hipMemcpyHostToDevice, c->stream));
  TG_HIP(hipMemcpyAsync(b.sys_tile0, t0.data(), sizeof(uint32_t) * (S + 1),
                        hipMemcpyHostToDevice, c->stream));
  if (!tiles.empty())
    TG_HIP(hipMemcpyAsync(b.tiles, tiles.data(), sizeof(Tile) * tiles.size(),
                          hipMemcpyHostToDevice, c->stream));
  TG_HIP(hipStreamSynchronize(c->stream));
  c->sysoff_host = so;
  c->n = n;
  c->S = S;
  c->n_tiles = (int64_t)tiles.size();
  return TG_OK;
} TG_HOST_CATCH("set_layout")

// mass (may be null): gathered with the positions when the caller has it
static tg_status build_tree_impl(tg_ctx *c, const double *pos, const double *mass,
                                 int64_t n, const int64_t *sys_off, int32_t S) {
  if (!c) return fail(TG_EINVAL, "tg_build_tree: NULL context");
  if (n < 0 || n > c->cfg.max_particles)
    return fail(TG_EINVAL, "tg_build_tree: N exceeds max_particles");
  if (S < 1 || S > c->cfg.max_systems)
    return fail(TG_EINVAL, "tg_build_tree: number of systems out of range");
  if (!sys_off && S != 1)
    return fail(TG_EINVAL, "tg_build_tree: sys_off required for S > 1");
  if (n > 0 && !pos) return fail(TG_EINVAL, "tg_build_tree: NULL positions");
  tg_status st = set_layout(c, n, sys_off, S);
  if (st != TG_OK) return st;
  c->have_tree = c->have_moments = false;
  TG_HIP(launch_cube_keys(c, pos));
  TG_HIP(launch_sort(c));
  TG_HIP(launch_keys_lo(c, pos));
  TG_HIP(launch_gather(c, pos, mass));
  TG_HIP(launch_tree_build(c));
  TG_HIP(launch_groups(c));
  // a build exists now (read by the device-side rebuild / refit choice)
  TG_HIP(fill_u32((uint32_t *)(c->b.refit_gates + 2), 1u, 1, c->stream, c->gate));
  c->have_tree = true;
  c->mass_gathered = mass;
  return TG_OK;
}

tg_status tg_build_tree(tg_ctx *c, const double *pos, int64_t n,
                        const int64_t *sys_off, int32_t S) {
  return build_tree_impl(c, pos, nullptr, n, sys_off, S);
}

tg_status tg_compute_moments(tg_ctx *c, const double *mass) {
  if (!c) return fail(TG_EINVAL, "tg_compute_moments: NULL context");
  if (!c->have_tree) return fail(TG_ESTATE, "tg_compute_moments: no tree");
  if (c->n > 0 && !mass) return fail(TG_EINVAL, "tg_compute_moments: NULL mass");
  // the build gathered these masses only for the moments right after it
  const bool gathered = mass == c->mass_gathered;
  c->mass_gathered = nullptr;
  TG_HIP(launch_moments(c, mass, gathered));
  c->have_moments = true;
  return TG_OK;
}

tg_status tg_refit_tree(tg_ctx *c, const double *pos, const double *mass) {
  if (!c) return fail(TG_EINVAL, "tg_refit_tree: NULL context");
  if (c->max_level > kMaxLevel) return fail(TG_EINVAL, "tg_refit_tree: takes a 21-level tree");
  if (!c->have_tree) return fail(TG_ESTATE, "tg_refit_tree: no tree to refit");
  if (c->n > 0 && (!pos || !mass)) return fail(TG_EINVAL, "tg_refit_tree: NULL positions or masses");
  if (c->n == 0) {
    c->have_moments = true;
    return TG_OK;
  }
  c->have_moments = false;
  c->mass_gathered = nullptr;
  TG_HIP(fill_u32((uint32_t *)c->b.refit_flag, 1u, 1, c->stream, c->gate));
  TG_HIP(launch_gather(c, pos, mass));
  TG_HIP(launch_moments(c, mass, true, true));
  c->have_moments = true;
  return TG_OK;
}

static tg_status check_walk_args(tg_ctx *c, double theta, const int32_t *idx,
                                 const int32_t *n_act, const char *who) {
  if (!c) return fail(TG_EINVAL, std::string(who) + ": NULL context");
  if (!c->have_moments) return fail(TG_ESTATE, std::string(who) + ": no tree/moments");
  if (c->mac == TG_MAC_GEOMETRIC && (!(theta >= 0.0) || !(theta * theta * 3.0 < 1.0)))
    return fail(TG_EINVAL, std::string(who) + ": theta must be in [0, 1/sqrt(3))");
  if (idx && !n_act) return fail(TG_EINVAL, std::string(who) + ": n_active required");
  return TG_OK;
}

// Old accelerations of the relative test for a walk (nullptr: the opening-
// angle test); sys_acc stands in when the context holds none.
static tg_status mac_acc_old(tg_ctx *c, const double *sys_acc, const char *who,
                             const double **out) {
  *out = nullptr;
  if (c->mac != TG_MAC_RELATIVE) return TG_OK;
  *out = c->acc_old ? c->acc_old : sys_acc;
  if (!*out && c->n > 0)
    return fail(TG_ESTATE, std::string(who) + ": relative test without old accelerations");
  return TG_OK;
}

static tg_status tree_forces_impl(tg_ctx *c, double eps, double theta,
                                  const int32_t *idx, const int32_t *n_act, double *acc,
                                  double *pot, const double *sys_acc) {
  tg_status st = check_walk_args(c, theta, idx, n_act, "tg_tree_forces");
  if (st != TG_OK) return st;
  const double *aold = nullptr;
  if ((st = mac_acc_old(c, sys_acc, "tg_tree_forces", &aold)) != TG_OK) return st;
  if (!(eps > 0.0) || !std::isfinite(eps))
    return fail(TG_EINVAL, "tg_tree_forces: eps must be positive");
  if (c->n > 0 && !acc) return fail(TG_EINVAL, "tg_tree_forces: NULL acc");
  if (c->n == 0) return TG_OK;
  // with an active list, every kernel of the evaluation returns at once when
  // the device-side count is 0 (graph replays of block steps)
  struct Gate {
    tg_ctx *c; const int32_t *saved;
    Gate(tg_ctx *c_, const int32_t *g) : c(c_), saved(c_->gate) { if (g) c->gate = g; }
    ~Gate() { c->gate = saved; }
  } gate(c, idx ? n_act : nullptr);
  TG_HIP(launch_active_groups(c, idx, n_act, aold, c->alpha));
  hipEvent_t before = nullptr, after = nullptr;
  if (c->profiling && !c->capturing) {
    const int64_t ring = (int64_t)c->ev_start.size();
    if (c->ev_head - c->ev_tail == ring) {      // ring full: resolve the oldest
      const int64_t k = c->ev_tail % ring;
      float ms = 0.f;
      TG_HIP(hipEventSynchronize(c->ev_stop[k]));
      TG_HIP(hipEventElapsedTime(&ms, c->ev_start[k], c->ev_stop[k]));
      c->prof_ms += ms;
      c->prof_n += 1;
      c->ev_tail += 1;
    }
    const int64_t k = c->ev_head % ring;
    before = c->ev_start[k];
    after = c->ev_stop[k];
    c->ev_head += 1;
  }
  TG_HIP(launch_walk_forces(c, eps, theta, acc, pot, before, after, aold != nullptr));
  return TG_OK;
}

tg_status tg_tree_forces(tg_ctx *c, double eps, double theta,
                         const int32_t *idx, const int32_t *n_act, double *acc,
                         double *pot) {
  return tree_forces_impl(c, eps, theta, idx, n_act, acc, pot, nullptr);
}

tg_status tg_set_mac(tg_ctx *c, int32_t kind, double alpha, const double *acc_old) {
  if (!c) return fail(TG_EINVAL, "tg_set_mac: NULL context");
  if (kind == TG_MAC_GEOMETRIC) {
    c->mac = kind; c->alpha = 0.0; c->acc_old = nullptr;
    return TG_OK;
  }
  if (kind != TG_MAC_RELATIVE) return fail(TG_EINVAL, "tg_set_mac: unknown kind");
  if (c->max_level > kMaxLevel)
    return fail(TG_EINVAL, "tg_set_mac: the relative test takes a 21-level tree");
  if (!(alpha >= 0.0) || !std::isfinite(alpha))
    return fail(TG_EINVAL, "tg_set_mac: alpha must be finite and >= 0");
  c->mac = kind; c->alpha = alpha; c->acc_old = acc_old;
  return TG_OK;
}

tg_status tg_set_softening(tg_ctx *c, int32_t kind) {
  if (!c) return fail(TG_EINVAL, "tg_set_softening: NULL context");
  if (kind != TG_SOFT_PLUMMER && kind != TG_SOFT_SPLINE)
    return fail(TG_EINVAL, "tg_set_softening: unknown kind");
  c->soft = kind;
  return TG_OK;
}

tg_status tg_set_profiling(tg_ctx *c, int32_t on) {
  if (!c) return fail(TG_EINVAL, "tg_set_profiling: NULL context");
  if (c->capturing) return fail(TG_ESTATE, "tg_set_profiling: during capture");
  if (on && c->ev_start.empty()) {
    const int ring = 256;
    c->ev_start.resize(ring);
    c->ev_stop.resize(ring);
    for (int k = 0; k < ring; ++k) {
      TG_HIP(hipEventCreate(&c->ev_start[k]));
      TG_HIP(hipEventCreate(&c->ev_stop[k]));
    }
  }
  if (c->profiling) TG_HIP(hipStreamSynchronize(c->stream));
  c->profiling = on != 0;
  c->ev_head = c->ev_tail = 0;
  c->prof_ms = 0.0;
  c->prof_n = 0;
  return TG_OK;
}

tg_status tg_get_profile(tg_ctx *c, double *walk_ms, int64_t *n_walks) {
  if (!c || !walk_ms || !n_walks) return fail(TG_EINVAL, "tg_get_profile: NULL argument");
  if (c->capturing) return fail(TG_ESTATE, "tg_get_profile: during capture");
  const int64_t ring = (int64_t)c->ev_start.size();
  while (c->ev_tail < c->ev_head) {
    const int64_t k = c->ev_tail % ring;
    float ms = 0.f;
    TG_HIP(hipEventSynchronize(c->ev_stop[k]));
    TG_HIP(hipEventElapsedTime(&ms, c->ev_start[k], c->ev_stop[k]));
    c->prof_ms += ms;
    c->prof_n += 1;
    c->ev_tail += 1;
  }
  *walk_ms = c->prof_ms;
  *n_walks = c->prof_n;
  return TG_OK;
}

tg_status tg_reset_counts(tg_ctx *c) {
  if (!c) return fail(TG_EINVAL, "tg_reset_counts: NULL context");
  TG_HIP(launch_counts_reset(c));
  return TG_OK;
}

tg_status tg_get_counts(tg_ctx *c, int64_t out[8]) {
  if (!c || !out) return fail(TG_EINVAL, "tg_get_counts: NULL argument");
  if (c->capturing) return fail(TG_ESTATE, "tg_get_counts: during capture");
  TreeCounters h;
  TG_HIP(hipMemcpyAsync(&h, c->b.ctr, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  TG_HIP(hipStreamSynchronize(c->stream));
  out[0] = (int64_t)h.n_p2p;
  out[1] = (int64_t)h.n_p2m;
  out[2] = (int64_t)h.n_targets;
  out[3] = (int64_t)h.n_walked;
  out[4] = (int64_t)h.cum_p2p;
  out[5] = (int64_t)h.cum_p2m;
  out[6] = (int64_t)h.cum_targets;
  out[7] = (int64_t)h.cum_walked;
  return TG_OK;
}

tg_status tg_walk_lists(tg_ctx *c, double theta, const int32_t *idx,
                        const int32_t *n_act, int64_t *info, int64_t cap_groups,
                        uint32_t *ids, int64_t cap_ids, int64_t *n_groups_out,
                        int64_t *n_ids_out) try {
  tg_status st = check_walk_args(c, theta, idx, n_act, "tg_walk_lists");
  if (st != TG_OK) return st;
  const double *aold = nullptr;
  if ((st = mac_acc_old(c, nullptr, "tg_walk_lists", &aold)) != TG_OK) return st;
  if (c->capturing) return fail(TG_ESTATE, "tg_walk_lists: during capture");
  if (!n_groups_out || !n_ids_out) return fail(TG_EINVAL, "tg_walk_lists: NULL outputs");
  *n_groups_out = 0;
  *n_ids_out = 0;
  if (c->n == 0) return TG_OK;
  Buffers &b = c->b;
  TG_HIP(launch_active_groups(c, idx, n_act, aold, c->alpha));
  TG_HIP(launch_walk_lists(c, theta, 0, nullptr, 0, nullptr, 0, aold != nullptr));
  TreeCounters h;
  TG_HIP(hipMemcpyAsync(&h, b.ctr, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  TG_HIP(hipStreamSynchronize(c->stream));
  const uint32_t nag = h.n_active_groups;
  TG_HIP(scan_u32(b.wl_count, b.wl_off, 2u * nag, nullptr, b.scan_total,
                  b.scan_part, c->stream));
  uint32_t total = 0;
  TG_HIP(hipMemcpyAsync(&total, b.scan_total, sizeof(uint32_t),
                        hipMemcpyDeviceToHost, c->stream));
  TG_HIP(hipStreamSynchronize(c->stream));
  *n_groups_out = nag;
  *n_ids_out = total;
  if ((int64_t)nag > cap_groups || (int64_t)total > cap_ids || !info || !ids)
    return fail(TG_ECAPACITY, "tg_walk_lists: output capacity too small");
  TG_HIP(launch_walk_lists(c, theta, 1, nullptr, 0, ids, cap_ids, aold != nullptr));
  std::vector<uint32_t> cnt(2 * (size_t)nag), off(2 * (size_t)nag), al(nag);
  if (nag) {
    TG_HIP(hipMemcpyAsync(cnt.data(), b.wl_count, sizeof(uint32_t) * 2 * nag,
                          hipMemcpyDeviceToHost, c->stream));
    TG_HIP(hipMemcpyAsync(off.data(), b.wl_off, sizeof(uint32_t) * 2 * nag,
                          hipMemcpyDeviceToHost, c->stream));
    TG_HIP(hipMemcpyAsync(al.data(), b.alist, sizeof(uint32_t) * nag,
                          hipMemcpyDeviceToHost, c->stream));
  }
  TG_HIP(hipStreamSynchronize(c->stream));
  std::vector<int64_t> inf(4 * (size_t)nag);
  for (uint32_t g = 0; g < nag; ++g) {
    inf[4 * g + 0] = al[g];
    inf[4 * g + 1] = off[2 * g];
    inf[4 * g + 2] = cnt[2 * g];
    inf[4 * g + 3] = cnt[2 * g + 1];
  }
  if (nag)
    TG_HIP(hipMemcpy(info, inf.data(), sizeof(int64_t) * inf.size(), hipMemcpyHostToDevice));
  return TG_OK;
} TG_HOST_CATCH("tg_walk_lists")

tg_status tg_direct_fp64(tg_ctx *c, const double *spos, const double *sm,
                         const double *seps, int64_t ns, const double *tpos,
                         const double *teps, int64_t nt, const int64_t *sseg,
                         const int64_t *tseg, int32_t nseg, int32_t self_pairs,
                         int32_t accumulate, double *acc, double *pot) try {
  if (!c) return fail(TG_EINVAL, "tg_direct_fp64: NULL context");
  if (ns < 0 || nt < 0) return fail(TG_EINVAL, "tg_direct_fp64: negative size");
  if (nt == 0) return TG_OK;
  if (!tpos || !teps || !acc || (ns > 0 && (!spos || !sm || !seps)))
    return fail(TG_EINVAL, "tg_direct_fp64: NULL pointer");
  if (nseg < 0 || nseg > kMaxSys)
    return fail(TG_EINVAL, "tg_direct_fp64: nseg must be in 0..256");
  if (self_pairs && ns != nt)
    return fail(TG_EINVAL, "tg_direct_fp64: self_pairs needs ns == nt");
  std::vector<int64_t> seg;
  int ns_eff = nseg;
  if (nseg == 0) {
    seg = {0, ns, 0, nt};
    ns_eff = 1;
  } else {
    if (!sseg || !tseg) return fail(TG_EINVAL, "tg_direct_fp64: NULL segments");
    seg.resize(2 * (nseg + 1));
    for (int s = 0; s <= nseg; ++s) { seg[s] = sseg[s]; seg[nseg + 1 + s] = tseg[s]; }
    if (seg[0] != 0 || seg[nseg] != ns || seg[nseg + 1] != 0 || seg[2 * nseg + 1] != nt)
      return fail(TG_EINVAL, "tg_direct_fp64: segment offsets must span 0..n");
    for (int s = 0; s < nseg; ++s)
      if (seg[s + 1] < seg[s] || seg[nseg + 2 + s] < seg[nseg + 1 + s])
        return fail(TG_EINVAL, "tg_direct_fp64: segment offsets not ascending");
  }
  int64_t max_src = 0;
  for (int s = 0; s < ns_eff; ++s) max_src = std::max(max_src, seg[s + 1] - seg[s]);
  // segment tables live in a few device slots keyed by their contents, so
  // a step that uses several tables can still be graph-captured once each
  // table has been seen eagerly
  int slot = -1;
  for (int k = 0; k < (int)c->dseg_host.size(); ++k)
    if (c->dseg_host[k] == seg) slot = k;
  if (slot < 0) {
    if (c->capturing)
      return fail(TG_ESTATE, "tg_direct_fp64: new segment layout during capture");
    if ((int)c->dseg_host.size() < kSegSlots) {
      c->dseg_host.push_back(seg);
      slot = (int)c->dseg_host.size() - 1;
    } else {
      slot = c->dseg_next;
      c->dseg_next = (c->dseg_next + 1) % kSegSlots;
      c->dseg_host[slot] = seg;
      ++c->layout_gen;          // an evicted slot is overwritten
    }
    TG_HIP(hipMemcpyAsync(c->b.dseg + slot * kSegSlotLen, seg.data(),
                          sizeof(int64_t) * seg.size(), hipMemcpyHostToDevice,
                          c->stream));
    TG_HIP(hipStreamSynchronize(c->stream));
  }
  const int64_t *dseg = c->b.dseg + slot * kSegSlotLen;
  TG_HIP(launch_direct(c, dseg, spos, sm, seps, 0.0, ns, tpos, teps, nt, ns_eff,
                       max_src, self_pairs, accumulate, acc, pot));
  return TG_OK;
} TG_HOST_CATCH("tg_direct_fp64")

// Direct sums where every source shares one softening (stars): the same
// kernels with a broadcast softening.
static tg_status tg_direct_fp64_eps(tg_ctx *c, const double *spos, const double *sm,
                             double seps, int64_t ns, const double *tpos,
                             const double *teps, int64_t nt,
                             const int64_t *sseg, const int64_t *tseg, int32_t nseg,
                             double *acc, double *pot) try {
  if (!c) return fail(TG_EINVAL, "tg_direct_fp64_eps: NULL context");
  if (nt == 0) return TG_OK;
  int slot = -1;
  std::vector<int64_t> seg(2 * (nseg + 1));
  for (int s = 0; s <= nseg; ++s) { seg[s] = sseg[s]; seg[nseg + 1 + s] = tseg[s]; }
  int64_t max_src = 0;
  for (int s = 0; s < nseg; ++s) max_src = std::max(max_src, seg[s + 1] - seg[s]);
  for (int k = 0; k < (int)c->dseg_host.size(); ++k)
    if (c->dseg_host[k] == seg) slot = k;
  if (slot < 0) {
    if (c->capturing)
      return fail(TG_ESTATE, "tg_direct_fp64_eps: new segment layout during capture");
    if ((int)c->dseg_host.size() < kSegSlots) {
      c->dseg_host.push_back(seg);
      slot = (int)c->dseg_host.size() - 1;
    } else {
      slot = c->dseg_next;
      c->dseg_next = (c->dseg_next + 1) % kSegSlots;
      c->dseg_host[slot] = seg;
      ++c->layout_gen;          // an evicted slot is overwritten
    }
    TG_HIP(hipMemcpyAsync(c->b.dseg + slot * kSegSlotLen, seg.data(),
                          sizeof(int64_t) * seg.size(), hipMemcpyHostToDevice, c->stream));
    TG_HIP(hipStreamSynchronize(c->stream));
  }
  TG_HIP(launch_direct(c, c->b.dseg + slot * kSegSlotLen, spos, sm, nullptr, seps, ns,
                       tpos, teps, nt, nseg, max_src, 0, 0, acc, pot));
  return TG_OK;
} TG_HOST_CATCH("tg_direct_fp64_eps")

// Kick, drift and active set with an optional mask of frozen stars (ghost
// chain members inside whole steps: no kick, no drift, never active).
static tg_status kick_impl(tg_ctx *c, double *vel, const double *acc, int64_t n,
                           const int32_t *idx, const int32_t *n_act, const uint8_t *level,
                           double dt, const int64_t *k, int32_t skip_k0,
                           const uint8_t *frozen) {
  if (!c) return fail(TG_EINVAL, "tg_kick: NULL context");
  if (n < 0) return fail(TG_EINVAL, "tg_kick: negative n");
  if (n > 0 && (!vel || !acc)) return fail(TG_EINVAL, "tg_kick: NULL pointer");
  if (idx && !n_act) return fail(TG_EINVAL, "tg_kick: n_active required");
  if (skip_k0 && !k) return fail(TG_EINVAL, "tg_kick: skip_at_k0 needs k");
  if (!std::isfinite(dt)) return fail(TG_EINVAL, "tg_kick: dt not finite");
  TG_HIP(launch_kick(c, vel, acc, n, idx, n_act, level, dt, k, skip_k0, frozen));
  return TG_OK;
}

tg_status tg_kick(tg_ctx *c, double *vel, const double *acc, int64_t n,
                  const int32_t *idx, const int32_t *n_act,
                  const uint8_t *level, double dt, const int64_t *k,
                  int32_t skip_k0) {
  return kick_impl(c, vel, acc, n, idx, n_act, level, dt, k, skip_k0, nullptr);
}

static tg_status drift_impl(tg_ctx *c, double *pos, const double *vel, int64_t n, double dt,
                            const uint8_t *frozen) {
  if (!c) return fail(TG_EINVAL, "tg_drift: NULL context");
  if (n < 0) return fail(TG_EINVAL, "tg_drift: negative n");
  if (n > 0 && (!pos || !vel)) return fail(TG_EINVAL, "tg_drift: NULL pointer");
  if (!std::isfinite(dt)) return fail(TG_EINVAL, "tg_drift: dt not finite");
  TG_HIP(launch_drift(c, pos, vel, n, dt, frozen));
  return TG_OK;
}

tg_status tg_drift(tg_ctx *c, double *pos, const double *vel, int64_t n, double dt) {
  return drift_impl(c, pos, vel, n, dt, nullptr);
}

tg_status tg_levels_v(tg_ctx *c, const double *acc, const double *vel,
                      const double *t4e2, const double *t2e2v, int64_t n,
                      const int32_t *idx, const int32_t *n_act, double dt_max,
                      int32_t nlev, const int64_t *k, uint8_t *level) {
  if (!c) return fail(TG_EINVAL, "tg_levels: NULL context");
  if (n < 0) return fail(TG_EINVAL, "tg_levels: negative n");
  if (nlev < 1 || nlev > 30) return fail(TG_EINVAL, "tg_levels: nlev must be in 1..30");
  if (!(dt_max > 0.0)) return fail(TG_EINVAL, "tg_levels: dt_max must be positive");
  if (n > 0 && (!acc || !t4e2 || !level)) return fail(TG_EINVAL, "tg_levels: NULL pointer");
  if (idx && !n_act) return fail(TG_EINVAL, "tg_levels: n_active required");
  if ((vel == nullptr) != (t2e2v == nullptr))
    return fail(TG_EINVAL, "tg_levels_v: vel and tau2eps2v go together");
  TG_HIP(launch_levels(c, acc, vel, t4e2, t2e2v, n, idx, n_act, dt_max, nlev, k, level));
  return TG_OK;
}

tg_status tg_levels(tg_ctx *c, const double *acc, const double *t4e2, int64_t n,
                    const int32_t *idx, const int32_t *n_act, double dt_max,
                    int32_t nlev, const int64_t *k, uint8_t *level) {
  return tg_levels_v(c, acc, nullptr, t4e2, nullptr, n, idx, n_act, dt_max, nlev, k, level);
}

static tg_status active_set_impl(tg_ctx *c, const uint8_t *level, int64_t n, int32_t nlev,
                                 const int64_t *k, int32_t k_add, int32_t *idx,
                                 int32_t *n_out, const uint8_t *frozen) {
  if (!c) return fail(TG_EINVAL, "tg_active_set: NULL context");
  if (n < 0 || n > c->cfg.max_particles)
    return fail(TG_EINVAL, "tg_active_set: n out of range");
  if (nlev < 1 || nlev > 30) return fail(TG_EINVAL, "tg_active_set: nlev must be in 1..30");
  if (!n_out || (n > 0 && (!level || !idx)))
    return fail(TG_EINVAL, "tg_active_set: NULL pointer");
  TG_HIP(launch_active_set(c, level, n, nlev, k, k_add, idx, n_out, frozen));
  return TG_OK;
}

tg_status tg_active_set(tg_ctx *c, const uint8_t *level, int64_t n, int32_t nlev,
                        const int64_t *k, int32_t k_add, int32_t *idx,
                        int32_t *n_out) {
  return active_set_impl(c, level, n, nlev, k, k_add, idx, n_out, nullptr);
}

tg_status tg_counter_add(tg_ctx *c, int64_t *k, int64_t inc) {
  if (!c || !k) return fail(TG_EINVAL, "tg_counter_add: NULL argument");
  TG_HIP(launch_counter_add(c, k, inc));
  return TG_OK;
}

tg_status tg_graph_begin(tg_ctx *c) {
  if (!c) return fail(TG_EINVAL, "tg_graph_begin: NULL context");
  if (c->capturing) return fail(TG_ESTATE, "tg_graph_begin: already capturing");
  if (!c->stream) return fail(TG_ESTATE, "tg_graph_begin: needs a non-default stream");
  TG_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  return TG_OK;
}

tg_status tg_graph_end(tg_ctx *c, tg_graph **out) {
  if (!c || !out) return fail(TG_EINVAL, "tg_graph_end: NULL argument");
  if (!c->capturing) return fail(TG_ESTATE, "tg_graph_end: not capturing");
  c->capturing = false;
  tg_graph *g = new tg_graph();
  hipError_t e = hipStreamEndCapture(c->stream, &g->graph);
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return hip_fail(e, "tg_graph_end");
  }
  g->ctx = c;
  g->gen = c->layout_gen;
  *out = g;
  return TG_OK;
}

tg_status tg_graph_launch(tg_graph *g, void *stream) {
  if (!g) return fail(TG_EINVAL, "tg_graph_launch: NULL graph");
  if (g->ctx && g->ctx->layout_gen != g->gen)
    return fail(TG_ESTATE, "tg_graph_launch: the context's system layout or segment tables "
                           "changed since the capture (capture again)");
  TG_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return TG_OK;
}

void tg_graph_destroy(tg_graph *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

tg_status tg_get_tree(tg_ctx *c, tg_tree_view *v) {
  if (!c || !v) return fail(TG_EINVAL, "tg_get_tree: NULL argument");
  if (!c->have_tree) return fail(TG_ESTATE, "tg_get_tree: no tree");
  if (c->capturing) return fail(TG_ESTATE, "tg_get_tree: during capture");
  TreeCounters h;
  TG_HIP(hipMemcpyAsync(&h, c->b.ctr, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  TG_HIP(hipStreamSynchronize(c->stream));
  Buffers &b = c->b;
  v->n = c->n;
  v->n_nodes = c->n ? h.n_nodes : 0;
  v->n_groups = c->n ? h.n_groups : 0;
  v->n_sys = c->S;
  v->skeys = b.key[0];
  v->skeys_lo = c->max_level > kMaxLevel ? b.klo[0] : nullptr;
  v->perm = b.val[0];
  v->level = b.level;
  v->nchild = b.nchild;
  v->first = b.first;
  v->count = b.count;
  v->child = b.child;
  v->parent = b.parent;
  v->cube = b.cube;
  v->com = (const double *)b.com;
  v->mom = b.mom;
  v->groups = (const uint32_t *)b.groups;
  return TG_OK;
}

tg_status tg_autotune(tg_ctx *c, const double *pos, const double *mass,
                      int64_t n, const int64_t *sys_off, int32_t S, double eps,
                      double theta, const int32_t *leaf_list,
                      const int32_t *group_list, const int32_t *waves_list,
                      int32_t repeats, int32_t best[3], double *best_ms,
                      double *times) {
  if (!c || !best || !best_ms) return fail(TG_EINVAL, "tg_autotune: NULL argument");
  if (c->capturing) return fail(TG_ESTATE, "tg_autotune: during capture");
  static const int32_t dl[] = {4, 8, 12, 16, 0};
  static const int32_t dg[] = {16, 32, 48, 64, 0};
  static const int32_t dw[] = {4, 8, 12, 0};
  if (!leaf_list) leaf_list = dl;
  if (!group_list) group_list = dg;
  if (!waves_list) waves_list = dw;
  if (repeats < 1) repeats = 3;
  double *acc = nullptr;
  TG_HIP(hipMalloc((void **)&acc, sizeof(double) * 3 * std::max<int64_t>(n, 1)));
  hipEvent_t e0, e1;
  TG_HIP(hipEventCreate(&e0));
  TG_HIP(hipEventCreate(&e1));
  double bms = 1e300;
  int32_t b3[3] = {c->leaf_size, c->group_size, c->waves_per_cu};
  tg_status st = TG_OK;
  int64_t cand = 0;
  for (const int32_t *L = leaf_list; *L && st == TG_OK; ++L)
    for (const int32_t *Gs = group_list; *Gs && st == TG_OK; ++Gs)
      for (const int32_t *W = waves_list; *W && st == TG_OK; ++W) {
        if (*W < 1 || *W > kMaxWavesPerCU) { st = fail(TG_EINVAL, "tg_autotune: bad waves"); break; }
        if ((st = tg_set_sizes(c, *L, *Gs)) != TG_OK) break;
        c->waves_per_cu = *W;
        double tmin = 1e300;
        for (int r = 0; r < repeats + 1 && st == TG_OK; ++r) {
          (void)hipEventRecord(e0, c->stream);
          st = tg_build_tree(c, pos, n, sys_off, S);
          if (st == TG_OK) st = tg_compute_moments(c, mass);
          if (st == TG_OK) st = tg_tree_forces(c, eps, theta, nullptr, nullptr, acc, nullptr);
          (void)hipEventRecord(e1, c->stream);
          (void)hipEventSynchronize(e1);
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (r > 0) tmin = std::min(tmin, (double)ms);   // first run warms up
        }
        uint32_t bits = 0;
        if (st == TG_OK) st = tg_sync(c, &bits);
        if (st == TG_OK && times) times[cand] = tmin;
        ++cand;
        if (st == TG_OK && tmin < bms) {
          bms = tmin;
          b3[0] = *L; b3[1] = *Gs; b3[2] = *W;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(acc);
  if (st != TG_OK) return st;
  tg_set_sizes(c, b3[0], b3[1]);
  c->waves_per_cu = b3[2];
  best[0] = b3[0]; best[1] = b3[1]; best[2] = b3[2];
  *best_ms = bms;
  return TG_OK;
}

tg_status tg_set_external(tg_ctx *c, const double *pos, const double *mass,
                          const double *eps, int32_t n_ext,
                          const int64_t *seg_host, int32_t n_sys) try {
  if (!c) return fail(TG_EINVAL, "tg_set_external: NULL context");
  if (n_ext < 0 || n_ext > kMaxExternal)
    return fail(TG_EINVAL, "tg_set_external: n_ext must be in 0..1024");
  if (n_ext == 0) {
    c->n_ext = 0;
    c->ext_pos = c->ext_mass = c->ext_eps = nullptr;
    return TG_OK;
  }
  if (!pos || !mass || !eps) return fail(TG_EINVAL, "tg_set_external: NULL pointer");
  if (n_sys < 1 || n_sys > c->cfg.max_systems)
    return fail(TG_EINVAL, "tg_set_external: n_sys out of range");
  std::vector<int32_t> seg(kMaxSys + 1, 0);
  if (seg_host) {
    if (seg_host[0] != 0 || seg_host[n_sys] != n_ext)
      return fail(TG_EINVAL, "tg_set_external: segments must span 0..n_ext");
    for (int s = 0; s <= n_sys; ++s) {
      if (s > 0 && seg_host[s] < seg_host[s - 1])
        return fail(TG_EINVAL, "tg_set_external: segments not ascending");
      seg[s] = (int32_t)seg_host[s];
    }
  } else {
    if (n_sys != 1) return fail(TG_EINVAL, "tg_set_external: segments needed for n_sys > 1");
    seg[0] = 0;
    seg[1] = n_ext;
  }
  seg.resize(n_sys + 1);
  if (seg != c->ext_seg_host) {
    if (c->capturing)
      return fail(TG_ESTATE, "tg_set_external: new segment layout during capture");
    ++c->layout_gen;
    TG_HIP(hipMemcpyAsync(c->b.ext_seg, seg.data(), sizeof(int32_t) * (n_sys + 1),
                          hipMemcpyHostToDevice, c->stream));
    TG_HIP(hipStreamSynchronize(c->stream));
    c->ext_seg_host = seg;
  }
  c->ext_pos = pos;
  c->ext_mass = mass;
  c->ext_eps = eps;
  c->n_ext = n_ext;
  return TG_OK;
} TG_HOST_CATCH("tg_set_external")

static tg_status check_system(const tg_system *y, const char *who) {
  if (!y) return fail(TG_EINVAL, std::string(who) + ": NULL system");
  if (y->n < 0 || (y->n > 0 && (!y->pos || !y->vel || !y->acc || !y->mass)))
    return fail(TG_EINVAL, std::string(who) + ": star arrays missing");
  if (y->n_bh < 0 || (y->n_bh > 0 && (!y->bh_pos || !y->bh_vel || !y->bh_acc ||
                                      !y->bh_mass || !y->bh_eps)))
    return fail(TG_EINVAL, std::string(who) + ": SMBH arrays missing");
  if (y->n_bh > 0 && y->n_sys > 1 && !y->bh_seg)
    return fail(TG_EINVAL, std::string(who) + ": bh_seg needed for several systems");
  return TG_OK;
}

// Forces for the listed stars.  With a rebuild period (block steps) the
// tree is rebuilt when the substep counter k is a multiple of it (or no
// build exists yet) and refitted otherwise; both choices are made on the
// device, so a captured substep replays correctly.
static tg_status smbh_sums(tg_ctx *c, const tg_system *y, bool stars_done = false);

static tg_status forces_impl(tg_ctx *c, const tg_system *y, const int32_t *idx,
                             const int32_t *n_act, const int64_t *k, int32_t rebuild_every) {
  tg_status st = check_system(y, "tg_forces");
  if (st != TG_OK) return st;
  if (rebuild_every > 1 && c->max_level > kMaxLevel)
    return fail(TG_EINVAL, "block steps: refit between rebuilds takes a 21-level tree");
  // with an active list, the build, moments and walk are skipped on the
  // device when it is empty (the SMBH sums below always run)
  const int32_t *gate = idx ? n_act : nullptr;
  if (rebuild_every > 1 && k && y->n > 0 && c->have_tree && y->n == c->n &&
      y->n_sys == c->S) {
    int32_t *gb = c->b.refit_gates, *gr = c->b.refit_gates + 1;
    TG_HIP(launch_refit_gates(c, gate, k, rebuild_every));
    c->gate = gb;
    st = build_tree_impl(c, y->pos, y->mass, y->n, y->sys_off, y->n_sys);
    if (st == TG_OK) {
      c->gate = gr;
      if (hipError_t e = launch_gather(c, y->pos, y->mass); e != hipSuccess)
        st = hip_fail(e, "launch_gather");
    }
    if (st == TG_OK) {
      c->gate = gate;
      c->mass_gathered = nullptr;
      if (hipError_t e = launch_moments(c, y->mass, true, true); e != hipSuccess)
        st = hip_fail(e, "launch_moments");
      c->have_moments = st == TG_OK;
    }
  } else {
    c->gate = gate;
    st = build_tree_impl(c, y->pos, y->mass, y->n, y->sys_off, y->n_sys);
    if (st == TG_OK) st = tg_compute_moments(c, y->mass);
  }
  c->gate = nullptr;
  if (st != TG_OK) return st;
  if ((st = tg_set_external(c, y->bh_pos, y->bh_mass, y->bh_eps, y->n_bh,
                            y->n_bh ? y->bh_seg : nullptr, y->n_sys)) != TG_OK)
    return st;
  // relative test: the system's current accelerations are the old ones
  // (each group's threshold is formed before any of them is overwritten)
  if ((st = tree_forces_impl(c, y->eps, y->theta, idx, n_act, y->acc, y->pot, y->acc)) !=
      TG_OK)
    return st;
  return smbh_sums(c, y);
}

// SMBH <- star sums over each system's stars (skipped with stars_done: a
// fused launch already formed them), then SMBH <-> SMBH.
static tg_status smbh_sums(tg_ctx *c, const tg_system *y, bool stars_done) try {
  tg_status st = TG_OK;
  if (y->n_bh > 0) {
    // SMBHs feel the stars of their own system, then each other
    std::vector<int64_t> so = c->sysoff_host;
    std::vector<int64_t> bs(y->n_sys + 1);
    for (int s = 0; s <= y->n_sys; ++s) bs[s] = y->bh_seg ? y->bh_seg[s] : (s ? y->n_bh : 0);
    const int nseg = y->n_sys;
    // star softening: the stars' eps for every star
    if (!stars_done) {
      st = tg_direct_fp64_eps(c, y->pos, y->mass, y->eps, y->n, y->bh_pos, y->bh_eps,
                              y->n_bh, so.data(), bs.data(), nseg, y->bh_acc, y->bh_pot);
      if (st != TG_OK) return st;
    }
    st = tg_direct_fp64(c, y->bh_pos, y->bh_mass, y->bh_eps, y->n_bh, y->bh_pos,
                        y->bh_eps, y->n_bh, bs.data(), bs.data(), nseg, 1, 1, y->bh_acc,
                        y->bh_pot);
    if (st != TG_OK) return st;
  }
  return TG_OK;
} TG_HOST_CATCH("smbh_sums")

tg_status tg_forces(tg_ctx *c, const tg_system *y, const int32_t *idx,
                    const int32_t *n_act) {
  return forces_impl(c, y, idx, n_act, nullptr, 0);
}

tg_status tg_step_kdk(tg_ctx *c, const tg_system *y, double dt) {
  tg_status st = check_system(y, "tg_step_kdk");
  if (st != TG_OK) return st;
  if (!c) return fail(TG_EINVAL, "tg_step_kdk: NULL context");
  if (!std::isfinite(dt)) return fail(TG_EINVAL, "tg_step_kdk: dt not finite");
  // opening half kicks and drifts of stars and SMBHs, one launch
  TG_HIP(launch_kick_drift(c, y->pos, y->vel, y->acc, y->frozen, y->n, y->bh_pos, y->bh_vel,
                           y->bh_acc, y->n_bh, dt, true));
  if ((st = tg_forces(c, y, nullptr, nullptr))) return st;
  // closing half kicks, one launch
  TG_HIP(launch_kick_drift(c, y->pos, y->vel, y->acc, y->frozen, y->n, y->bh_pos, y->bh_vel,
                           y->bh_acc, y->n_bh, dt, false));
  return TG_OK;
}

tg_status tg_step_dkd(tg_ctx *c, const tg_system *y, double dt) {
  tg_status st = check_system(y, "tg_step_dkd");
  if (st != TG_OK) return st;
  // tg_kick applies half of its dt: 2 dt gives the full kick
  if ((st = drift_impl(c, y->pos, y->vel, y->n, 0.5 * dt, y->frozen))) return st;
  if ((st = tg_drift(c, y->bh_pos, y->bh_vel, y->n_bh, 0.5 * dt))) return st;
  if ((st = tg_forces(c, y, nullptr, nullptr))) return st;
  if ((st = kick_impl(c, y->vel, y->acc, y->n, nullptr, nullptr, nullptr, 2.0 * dt, nullptr, 0,
                       y->frozen)))
    return st;
  if ((st = tg_kick(c, y->bh_vel, y->bh_acc, y->n_bh, nullptr, nullptr, nullptr, 2.0 * dt,
                    nullptr, 0)))
    return st;
  if ((st = drift_impl(c, y->pos, y->vel, y->n, 0.5 * dt, y->frozen))) return st;
  return tg_drift(c, y->bh_pos, y->bh_vel, y->n_bh, 0.5 * dt);
}

tg_status tg_step_block(tg_ctx *c, const tg_system *y, const tg_blocks *b) {
  tg_status st = check_system(y, "tg_step_block");
  if (st != TG_OK) return st;
  if (!b || !b->level || !b->tau4eps2 || !b->active_idx || !b->n_active || !b->k)
    return fail(TG_EINVAL, "tg_step_block: block arrays missing");
  if (b->nlev < 1 || b->nlev > 30 || !(b->dt_max > 0.0))
    return fail(TG_EINVAL, "tg_step_block: bad levels");
  const double dt_min = std::ldexp(b->dt_max, -(b->nlev - 1));
  // closing half kicks of the particles whose step ends now (not at k = 0)
  if ((st = active_set_impl(c, b->level, y->n, b->nlev, b->k, 0, b->active_idx, b->n_active,
                             y->frozen)))
    return st;
  if ((st = kick_impl(c, y->vel, y->acc, y->n, b->active_idx, b->n_active, b->level,
                      b->dt_max, b->k, 1, y->frozen)))
    return st;
  // new levels, then opening half kicks with the new steps
  if ((st = tg_levels_v(c, y->acc, b->tau2eps2v ? y->vel : nullptr, b->tau4eps2,
                        b->tau2eps2v, y->n, b->active_idx, b->n_active, b->dt_max, b->nlev,
                        b->k, b->level)))
    return st;
  if ((st = kick_impl(c, y->vel, y->acc, y->n, b->active_idx, b->n_active, b->level,
                      b->dt_max, nullptr, 0, y->frozen)))
    return st;
  // everyone drifts by the smallest step (the SMBHs, on the finest level,
  // are kicked and drifted in one launch that also advances k); then forces
  // for the next active set
  if ((st = drift_impl(c, y->pos, y->vel, y->n, dt_min, y->frozen))) return st;
  TG_HIP(launch_bh_substep(c, y->bh_pos, y->bh_vel, y->bh_acc, y->n_bh, dt_min, b->k, nullptr));
  if ((st = active_set_impl(c, b->level, y->n, b->nlev, b->k, 0, b->active_idx, b->n_active,
                             y->frozen)))
    return st;
  return forces_impl(c, y, b->active_idx, b->n_active, b->k, b->rebuild_every);
}

}  // extern "C"

namespace tg {

// The stars' part of a block substep, in two stages around whatever the
// caller moves with them (the hybrid driver's chain particle): first the
// active set at k, the closing half kicks (not at k = 0), new levels and
// the opening half kicks; then the drift of every star that is not frozen,
// k += 1 and the active set at the new k.  The same launches as
// tg_step_block's, without the SMBHs and the forces.
tg_status block_stars_kick(tg_ctx *c, const tg_system *y, const tg_blocks *b) {
  tg_status st = check_system(y, "block substep");
  if (st != TG_OK) return st;
  if (!b || !b->level || !b->tau4eps2 || !b->active_idx || !b->n_active || !b->k)
    return fail(TG_EINVAL, "block substep: block arrays missing");
  if (b->nlev < 1 || b->nlev > 30 || !(b->dt_max > 0.0))
    return fail(TG_EINVAL, "block substep: bad levels");
  if ((st = active_set_impl(c, b->level, y->n, b->nlev, b->k, 0, b->active_idx, b->n_active,
                             y->frozen)))
    return st;
  if ((st = kick_impl(c, y->vel, y->acc, y->n, b->active_idx, b->n_active, b->level,
                      b->dt_max, b->k, 1, y->frozen)))
    return st;
  if ((st = tg_levels_v(c, y->acc, b->tau2eps2v ? y->vel : nullptr, b->tau4eps2,
                        b->tau2eps2v, y->n, b->active_idx, b->n_active, b->dt_max, b->nlev,
                        b->k, b->level)))
    return st;
  return kick_impl(c, y->vel, y->acc, y->n, b->active_idx, b->n_active, b->level, b->dt_max,
                   nullptr, 0, y->frozen);
}

tg_status block_stars_drift(tg_ctx *c, const tg_system *y, const tg_blocks *b) {
  const double dt_min = std::ldexp(b->dt_max, -(b->nlev - 1));
  tg_status st;
  if ((st = drift_impl(c, y->pos, y->vel, y->n, dt_min, y->frozen))) return st;
  TG_HIP(launch_counter_add(c, b->k, 1));
  return active_set_impl(c, b->level, y->n, b->nlev, b->k, 0, b->active_idx, b->n_active,
                         y->frozen);
}

}  // namespace tg

extern "C" {

// A substep in which no star is active at its start or at its end: the
// SMBHs' kicks and drift (k advances, the active count becomes 0), the
// stars' drift and the SMBH sums.  These are exactly the launches of
// tg_step_block that do any work when both active sets are empty.
// With one system and a few SMBHs the stars' drift and their sums on the
// SMBHs are one launch (the SMBHs move first; the sums come out bit for
// bit as in tg_step_block).
static tg_status idle_substep(tg_ctx *c, const tg_system *y, const tg_blocks *b, double dt_min) {
  tg_status st;
  const bool fused = y->n_sys == 1 && c->sysoff_host.size() == 2 &&
                     c->sysoff_host[0] == 0 && c->sysoff_host[1] == y->n &&
                     drift_smbh_fits(c, y->n, y->n_bh);
  if (fused) {
    TG_HIP(launch_bh_substep(c, y->bh_pos, y->bh_vel, y->bh_acc, y->n_bh, dt_min, b->k,
                             b->n_active));
    TG_HIP(launch_drift_smbh(c, y->pos, y->vel, y->frozen, y->n, dt_min, y->mass, y->eps,
                             y->bh_pos, y->bh_eps, y->n_bh, y->bh_acc, y->bh_pot));
    return smbh_sums(c, y, true);
  }
  if ((st = drift_impl(c, y->pos, y->vel, y->n, dt_min, y->frozen))) return st;
  TG_HIP(launch_bh_substep(c, y->bh_pos, y->bh_vel, y->bh_acc, y->n_bh, dt_min, b->k,
                           b->n_active));
  return smbh_sums(c, y);
}

tg_status tg_step_blocks(tg_ctx *c, const tg_system *y, const tg_blocks *b, int64_t n_sub,
                         int64_t *n_idle) {
  if (!c) return fail(TG_EINVAL, "tg_step_blocks: NULL context");
  if (n_sub < 0) return fail(TG_EINVAL, "tg_step_blocks: n_sub must be >= 0");
  if (c->capturing) return fail(TG_ESTATE, "tg_step_blocks: reads the device back, not capturable");
  if (n_idle) *n_idle = 0;
  int64_t done = 0, idle_total = 0;
  while (done < n_sub) {
    tg_status st = tg_step_block(c, y, b);
    if (st != TG_OK) return st;
    ++done;
    if (done == n_sub) break;
    // the substep counter and the finest level held by a star free to move,
    // as left by the active set of the new substep
    TG_HIP(hipMemcpyAsync(c->host_words, b->k, sizeof(int64_t), hipMemcpyDeviceToHost,
                          c->stream));
    TG_HIP(hipMemcpyAsync(c->host_words + 1, c->b.ainfo, 2 * sizeof(int32_t),
                          hipMemcpyDeviceToHost, c->stream));
    TG_HIP(hipStreamSynchronize(c->stream));
    const int64_t k = c->host_words[0];
    int32_t info[2];
    std::memcpy(info, c->host_words + 1, sizeof(info));
    const int lf = info[1];
    // levels change only for active stars, so until the next multiple m of
    // the finest occupied level's step nobody is active: substeps k .. m-2
    // have empty active sets at both ends
    int64_t idle = 0;
    if (k >= 0 && info[0] == 0) {
      if (lf < 0) {
        idle = n_sub - done;
      } else {
        const int64_t p = (int64_t)1 << (b->nlev - 1 - std::min(lf, b->nlev - 1));
        const int64_t m = (k + p - 1) / p * p;
        idle = std::max<int64_t>(0, m - 1 - k);
      }
    }
    idle = std::min(idle, n_sub - done);
    const double dt_min = std::ldexp(b->dt_max, -(b->nlev - 1));
    for (int64_t i = 0; i < idle; ++i) {
      st = idle_substep(c, y, b, dt_min);
      if (st != TG_OK) return st;
    }
    done += idle;
    idle_total += idle;
  }
  if (n_idle) *n_idle = idle_total;
  return TG_OK;
}

static tg_status check_chain(tg_ctx *c, const tg_chain *ch, const char *who) {
  if (!c) return fail(TG_EINVAL, std::string(who) + ": NULL context");
  if (!ch) return fail(TG_EINVAL, std::string(who) + ": NULL chain");
  if (ch->n < 0 || ch->n > c->cfg.max_particles)
    return fail(TG_EINVAL, std::string(who) + ": n out of range");
  if (ch->n > 0 && (!ch->pos || !ch->mass))
    return fail(TG_EINVAL, std::string(who) + ": NULL star arrays");
  if (ch->nc < 1 || ch->nc > kMaxChain)
    return fail(TG_EINVAL, std::string(who) + ": nc must be in 1..256");
  if (!ch->member_pos || !ch->member_mass)
    return fail(TG_EINVAL, std::string(who) + ": NULL member arrays");
  if (!(ch->m_chain > 0.0) || !std::isfinite(ch->m_chain))
    return fail(TG_EINVAL, std::string(who) + ": m_chain must be positive");
  if (!(ch->r_crit >= 0.0) || !std::isfinite(ch->r_crit) || !(ch->gamma_crit > 0.0) ||
      !std::isfinite(ch->gamma_crit))
    return fail(TG_EINVAL, std::string(who) + ": r_crit >= 0 and gamma_crit > 0 required");
  if (!(ch->eps_pm >= 0.0) || !std::isfinite(ch->eps_pm))
    return fail(TG_EINVAL, std::string(who) + ": eps_pm must be >= 0");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(ch->com[k])) return fail(TG_EINVAL, std::string(who) + ": com not finite");
  if (!ch->pert_idx || !ch->n_pert || ch->pert_cap < 0)
    return fail(TG_EINVAL, std::string(who) + ": perturber list required");
  return TG_OK;
}

tg_status tg_perturbers(tg_ctx *c, const tg_chain *ch) {
  tg_status st = check_chain(c, ch, "tg_perturbers");
  if (st != TG_OK) return st;
  // Eq. 2 without roots: (r2 r2) r2 < (k k) rc6, k = c m_j
  const double cst = 2.0 / (ch->gamma_crit * ch->m_chain);
  const double rc2 = ch->r_crit * ch->r_crit;
  const double rc6 = (rc2 * rc2) * rc2;
  if (ch->n == 0) {
    TG_HIP(fill_u32((uint32_t *)ch->n_pert, 0u, 1, c->stream));
    return TG_OK;
  }
  TG_HIP(launch_chain_select(c, ch->pos, ch->mass, ch->n, ch->exclude, ch->com, true, cst, rc6,
                             ch->pert_idx, ch->pert_cap, ch->n_pert));
  return TG_OK;
}

tg_status tg_chain_forces(tg_ctx *c, const tg_chain *ch, const int32_t *idx,
                          const int32_t *n_act, double *acc, double *pot, double *com_acc,
                          double *member_acc) {
  tg_status st = check_chain(c, ch, "tg_chain_forces");
  if (st != TG_OK) return st;
  if (idx && !n_act) return fail(TG_EINVAL, "tg_chain_forces: n_active required");
  if (!com_acc || !member_acc) return fail(TG_EINVAL, "tg_chain_forces: NULL outputs");
  if ((st = tg_perturbers(c, ch)) != TG_OK) return st;
  TG_HIP(launch_chain_forces(c, ch, idx, n_act, acc, pot, com_acc, member_acc));
  return TG_OK;
}

tg_status tg_chains_forces(tg_ctx *c, const tg_chain *chains, int32_t n_chains,
                           const int32_t *idx, const int32_t *n_act, double *acc, double *pot,
                           double *com_acc, double *member_acc) {
  if (!c) return fail(TG_EINVAL, "tg_chains_forces: NULL context");
  if (!chains || n_chains < 1 || n_chains > kMaxChains)
    return fail(TG_EINVAL, "tg_chains_forces: n_chains must be in 1..16");
  if (!com_acc || !member_acc) return fail(TG_EINVAL, "tg_chains_forces: NULL outputs");
  const tg_chain &c0 = chains[0];
  for (int k = 0; k < n_chains; ++k) {
    tg_status st = check_chain(c, &chains[k], "tg_chains_forces");
    if (st != TG_OK) return st;
    const tg_chain &ck = chains[k];
    if (ck.pos != c0.pos || ck.mass != c0.mass || ck.n != c0.n || ck.exclude != c0.exclude)
      return fail(TG_EINVAL, "tg_chains_forces: chains must share the star arrays and mask");
    if (ck.pert_idx == c0.pert_idx && k > 0)
      return fail(TG_EINVAL, "tg_chains_forces: each chain needs its own perturber list");
  }
  // every chain couples to the stars on its own (the mask holds all ghosts)
  int64_t moff = 0;
  for (int k = 0; k < n_chains; ++k) {
    tg_status st = tg_chain_forces(c, &chains[k], idx, n_act, acc, pot, com_acc + 3 * k,
                                   member_acc + 3 * moff);
    if (st != TG_OK) return st;
    moff += chains[k].nc;
  }
  // the chain particles feel each other as point masses (Newtonian)
  if (n_chains > 1) {
    ChainVec add{};
    const double G = c->cfg.G;
    for (int a = 0; a < n_chains; ++a) {
      for (int d = 0; d < n_chains; ++d) {
        if (d == a) continue;
        const double dx = chains[d].com[0] - chains[a].com[0];
        const double dy = chains[d].com[1] - chains[a].com[1];
        const double dz = chains[d].com[2] - chains[a].com[2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 > 0.0)) return fail(TG_EINVAL, "tg_chains_forces: two chains share a centre");
        const double D1 = 1.0 / std::sqrt(r2);
        const double w = G * chains[d].m_chain * D1 * D1 * D1;
        add.v[3 * a] += w * dx;
        add.v[3 * a + 1] += w * dy;
        add.v[3 * a + 2] += w * dz;
      }
    }
    TG_HIP(launch_add_host_vector(c, com_acc, add, 3 * n_chains));
  }
  return TG_OK;
}

tg_status tg_predict_perturbers(tg_ctx *c, const tg_chain *ch, const double *vel,
                                const double com_vel[3], double dt, double *out_pos,
                                double *out_vel, double *out_mass) {
#pragma clang fp contract(off)
  tg_status st = check_chain(c, ch, "tg_predict_perturbers");
  if (st != TG_OK) return st;
  if (!com_vel || !std::isfinite(dt))
    return fail(TG_EINVAL, "tg_predict_perturbers: NULL com_vel or non-finite dt");
  if (ch->pert_cap > 0 && (!out_pos || !out_vel || (ch->n > 0 && !vel)))
    return fail(TG_EINVAL, "tg_predict_perturbers: NULL outputs");
  if (ch->pert_cap == 0 || ch->n == 0) return TG_OK;
  double rp[3], v[3];
  for (int k = 0; k < 3; ++k) {
    const double t = com_vel[k] * dt;
    rp[k] = ch->com[k] + t;
    v[k] = com_vel[k];
  }
  TG_HIP(launch_chain_predict(c, ch, vel, dt, rp, v, out_pos, out_vel, out_mass));
  return TG_OK;
}

tg_status tg_select_within(tg_ctx *c, const double *pos, int64_t n, const uint8_t *exclude,
                           const double center[3], double r, int32_t *idx, int32_t cap,
                           int32_t *n_out) {
  if (!c) return fail(TG_EINVAL, "tg_select_within: NULL context");
  if (n < 0 || n > c->cfg.max_particles) return fail(TG_EINVAL, "tg_select_within: n out of range");
  if ((n > 0 && !pos) || !center || !idx || !n_out || cap < 0)
    return fail(TG_EINVAL, "tg_select_within: NULL pointer or negative capacity");
  if (!(r >= 0.0) || !std::isfinite(r)) return fail(TG_EINVAL, "tg_select_within: r must be >= 0");
  if (n == 0) {
    TG_HIP(fill_u32((uint32_t *)n_out, 0u, 1, c->stream));
    return TG_OK;
  }
  TG_HIP(launch_chain_select(c, pos, nullptr, n, exclude, center, false, 0.0, r * r, idx, cap,
                             n_out));
  return TG_OK;
}

tg_status tg_sync(tg_ctx *c, uint32_t *bits) {
  if (!c) return fail(TG_EINVAL, "tg_sync: NULL context");
  if (c->capturing) return fail(TG_ESTATE, "tg_sync: during capture");
  uint32_t h = 0;
  TG_HIP(hipStreamSynchronize(c->stream));
  TG_HIP(hipMemcpy(&h, c->b.err, sizeof(h), hipMemcpyDeviceToHost));
  if (h) TG_HIP(hipMemset(c->b.err, 0, sizeof(uint32_t)));
  if (bits) *bits = h;
  if (h & (TG_ERR_NONFINITE | TG_ERR_MASS))
    return fail(TG_EDATA, "device: non-finite position or non-positive mass");
  if (h & (TG_ERR_NODES | TG_ERR_FRONTIER | TG_ERR_LISTS | TG_ERR_CHAIN))
    return fail(TG_ECAPACITY, "device: node, frontier, list or selection capacity exceeded");
  if (h & TG_ERR_SORT)
    return fail(TG_EINTERNAL, "device: radix-sort tile hand-off gave up waiting");
  return TG_OK;
}

}  // extern "C"
