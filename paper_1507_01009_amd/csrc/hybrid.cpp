// The hybrid step (Sec. 2) on the host: tree stars advanced by kick-drift-
// kick steps on the GPU, the stars near the SMBH regularised in one chain
// (AR-chain, host FP64), the two coupled through the perturbers (Eq. 2),
// the chain particle with the correction of Eq. 3, and the membership
// rules (Eq. 4, Eq. 5).  Every GPU stage is one of the library's calls;
// this file holds the bookkeeping: which stars are members (ghosts in the
// star arrays, never advanced: their rows keep the state they had when they
// joined), the chain's centre of mass, and the order of the stages (the
// chain step before the tree forces; membership when chain and tree share
// a time; in block substeps every velocity brought into step at a
// hand-off).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "tg_internal.h"

using namespace tg;

struct tg_hybrid {
  tg_ctx *c = nullptr;
  tg_system sys{};
  tg_hybrid_config cfg{};
  double G = 1.0;
  bool active = false;
  // members: star index (-1 for the SMBH), coordinates relative to the
  // centre of mass, masses (the stars' own, not the ghost masses)
  std::vector<int32_t> star;
  std::vector<double> x, v, m;
  // the AR-chain's chain state kept between steps (order, chain vectors);
  // rebuilt from x, v whenever the membership changes
  std::vector<int32_t> chain;
  std::vector<double> cx, cv;
  int32_t chain_valid = 0;
  double R[3] = {0, 0, 0}, V[3] = {0, 0, 0}, M = 0.0;
  double B = 0.0, ds = 0.0;
  double a_com[3] = {0, 0, 0};
  double r_chain = 0.0;
  int32_t n_pert = 0;
  double energy_error = 0.0;
  int64_t steps = 0, starts = 0, absorbed = 0, escaped = 0, ended = 0;
  double ar_s = 0.0, step_s = 0.0;   // host wall time: AR-chain, whole steps
  // device buffers
  uint8_t *d_excl = nullptr, *d_flag = nullptr;
  int32_t *d_pidx = nullptr, *d_sel = nullptr, *d_nsel = nullptr;
  double *d_macc = nullptr, *d_px = nullptr, *d_pv = nullptr, *d_pm = nullptr,
         *d_vals = nullptr;
  // what a step uploads, in one device block with a pinned host image (one
  // copy per upload): member star ids | their rows (positions, then
  // velocities) | all members' positions | masses | SMBH position, velocity
  char *d_stage = nullptr, *h_stage = nullptr;
  int32_t *d_ids = nullptr;
  double *d_rows = nullptr, *d_mpos = nullptr, *d_mmass = nullptr, *d_bh = nullptr;
  // the chain particle's force [3] and the perturber count, adjacent (one read)
  double *d_com = nullptr;
  int32_t *d_np = nullptr;
  // pinned landing area for reads: force and count [4], then the
  // perturbers' positions, velocities, masses [7 pert_cap] and ids
  double *h_read = nullptr;
};

namespace {

constexpr size_t kOffIds = 0;
constexpr size_t kOffRows = (sizeof(int32_t) * kMaxChain + 255) / 256 * 256;
constexpr size_t kOffMpos = kOffRows + sizeof(double) * 6 * kMaxChain;
constexpr size_t kOffMmass = kOffMpos + sizeof(double) * 3 * kMaxChain;
constexpr size_t kOffBh = kOffMmass + sizeof(double) * kMaxChain;
constexpr size_t kStageBytes = kOffBh + sizeof(double) * 6;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Adds the wall time of a scope to an accumulator.
struct Timer {
  double &acc;
  double t0;
  explicit Timer(double &a) : acc(a), t0(now_s()) {}
  ~Timer() { acc += now_s() - t0; }
};

template <class T>
hipError_t dalloc(T **p, int64_t n) {
  return hipMalloc((void **)p, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
}

tg_status to_dev(tg_hybrid *h, void *dst, const void *src, size_t bytes) {
  if (!bytes) return TG_OK;
  TG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->c->stream));
  return TG_OK;
}

tg_status to_host(tg_hybrid *h, void *dst, const void *src, size_t bytes) {
  if (!bytes) return TG_OK;
  TG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->c->stream));
  TG_HIP(hipStreamSynchronize(h->c->stream));
  return TG_OK;
}

int nc(const tg_hybrid *h) { return (int)h->m.size(); }

// Centre of mass from the members' global coordinates (X, W), then the
// coordinates relative to it.
void reform(tg_hybrid *h, const std::vector<double> &X, const std::vector<double> &W) {
#pragma clang fp contract(off)
  const int n = (int)h->m.size();
  double M = 0.0, R[3] = {0, 0, 0}, V[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i) {
    M += h->m[i];
    for (int k = 0; k < 3; ++k) {
      R[k] += h->m[i] * X[3 * i + k];
      V[k] += h->m[i] * W[3 * i + k];
    }
  }
  for (int k = 0; k < 3; ++k) {
    h->R[k] = R[k] / M;
    h->V[k] = V[k] / M;
  }
  h->M = M;
  h->x.assign(3 * n, 0.0);
  h->v.assign(3 * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) {
      h->x[3 * i + k] = X[3 * i + k] - h->R[k];
      h->v[3 * i + k] = W[3 * i + k] - h->V[k];
    }
}

double max_radius(const tg_hybrid *h) {
#pragma clang fp contract(off)
  double r2 = 0.0;
  for (int i = 0; i < nc(h); ++i) {
    const double *a = &h->x[3 * i];
    r2 = std::max(r2, (a[0] * a[0] + a[1] * a[1]) + a[2] * a[2]);
  }
  return std::sqrt(r2);
}

// Stage the members' global positions and masses for the coupling, and
// write the SMBH member's global coordinates (velocity relative to Vref)
// into its arrays (reference only: it is not a tree particle).  One upload
// of the staged block and, with the SMBH a member, two device copies.  The
// ghosts' rows are not touched.
tg_status stage_members(tg_hybrid *h, const double *Vref) {
#pragma clang fp contract(off)
  const int n = nc(h);
  double *mpos = reinterpret_cast<double *>(h->h_stage + kOffMpos);
  double *mmass = reinterpret_cast<double *>(h->h_stage + kOffMmass);
  double *bh = reinterpret_cast<double *>(h->h_stage + kOffBh);
  bool smbh = false;
  for (int i = 0; i < n; ++i) {
    for (int d = 0; d < 3; ++d) mpos[3 * i + d] = h->R[d] + h->x[3 * i + d];
    mmass[i] = h->m[i];
    if (h->star[i] < 0) {
      for (int d = 0; d < 3; ++d) {
        bh[d] = mpos[3 * i + d];
        bh[3 + d] = Vref[d] + h->v[3 * i + d];
      }
      smbh = true;
    }
  }
  hipStream_t sm = h->c->stream;
  TG_HIP(hipMemcpyAsync(h->d_stage, h->h_stage, kStageBytes, hipMemcpyHostToDevice, sm));
  if (smbh) {
    TG_HIP(hipMemcpyAsync(h->sys.bh_pos, h->d_bh, 3 * sizeof(double), hipMemcpyDeviceToDevice,
                          sm));
    TG_HIP(hipMemcpyAsync(h->sys.bh_vel, h->d_bh + 3, 3 * sizeof(double),
                          hipMemcpyDeviceToDevice, sm));
  }
  TG_HIP(hipStreamSynchronize(sm));
  return TG_OK;
}

// The SMBH's arrays := X, W (a freed SMBH, or the member's reference copy).
tg_status write_smbh(tg_hybrid *h, const double *X, const double *W) {
  double *bh = reinterpret_cast<double *>(h->h_stage + kOffBh);
  for (int d = 0; d < 3; ++d) {
    bh[d] = X[d];
    bh[3 + d] = W[d];
  }
  hipStream_t sm = h->c->stream;
  TG_HIP(hipMemcpyAsync(h->sys.bh_pos, bh, 3 * sizeof(double), hipMemcpyHostToDevice, sm));
  TG_HIP(hipMemcpyAsync(h->sys.bh_vel, bh + 3, 3 * sizeof(double), hipMemcpyHostToDevice, sm));
  TG_HIP(hipStreamSynchronize(sm));
  return TG_OK;
}

tg_status set_ghosts(tg_hybrid *h, const std::vector<int32_t> &ids,
                     const std::vector<double> &mass, bool ghost);

// Stars that leave the chain: rows := their global coordinates (X, W per
// star, [k][3]), mass restored, no longer excluded.
tg_status restore_rows(tg_hybrid *h, const std::vector<int32_t> &ids,
                       const std::vector<double> &X, const std::vector<double> &W,
                       const std::vector<double> &mass) {
  const int k = (int)ids.size();
  if (!k) return TG_OK;
  int32_t *sid = reinterpret_cast<int32_t *>(h->h_stage + kOffIds);
  double *rows = reinterpret_cast<double *>(h->h_stage + kOffRows);
  for (int i = 0; i < k; ++i) {
    sid[i] = ids[i];
    for (int d = 0; d < 3; ++d) {
      rows[3 * i + d] = X[3 * i + d];
      rows[3 * kMaxChain + 3 * i + d] = W[3 * i + d];
    }
  }
  hipStream_t sm = h->c->stream;
  TG_HIP(hipMemcpyAsync(h->d_stage, h->h_stage, kStageBytes, hipMemcpyHostToDevice, sm));
  TG_HIP(launch_move_rows(h->c, h->sys.pos, h->d_rows, h->d_ids, k, true));
  TG_HIP(launch_move_rows(h->c, h->sys.vel, h->d_rows + 3 * kMaxChain, h->d_ids, k, true));
  TG_HIP(hipStreamSynchronize(sm));
  return set_ghosts(h, ids, mass, false);
}

// The chain particle's force and the perturber count of the last coupling
// (the stream is synchronised by the read).
tg_status read_coupling(tg_hybrid *h) {
  TG_HIP(hipMemcpyAsync(h->h_read, h->d_com, 4 * sizeof(double), hipMemcpyDeviceToHost,
                        h->c->stream));
  TG_HIP(hipStreamSynchronize(h->c->stream));
  for (int k = 0; k < 3; ++k) h->a_com[k] = h->h_read[k];
  std::memcpy(&h->n_pert, h->h_read + 3, sizeof(int32_t));
  return TG_OK;
}

// Stars become ghosts (ghost = 1: mass times ghost_mass, excluded) or get
// their mass back (ghost = 0).
tg_status set_ghosts(tg_hybrid *h, const std::vector<int32_t> &ids,
                     const std::vector<double> &mass, bool ghost) {
  const int k = (int)ids.size();
  if (!k) return TG_OK;
  std::vector<double> val(k);
  std::vector<uint8_t> f(k, ghost ? 1 : 0);
  for (int i = 0; i < k; ++i) val[i] = ghost ? mass[i] * h->cfg.ghost_mass : mass[i];
  tg_status st;
  if ((st = to_dev(h, h->d_ids, ids.data(), sizeof(int32_t) * k))) return st;
  if ((st = to_dev(h, h->d_vals, val.data(), sizeof(double) * k))) return st;
  if ((st = to_dev(h, h->d_flag, f.data(), k))) return st;
  TG_HIP(launch_set_rows(h->c, const_cast<double *>(h->sys.mass), h->d_excl, h->d_ids, h->d_vals,
                         h->d_flag, k));
  TG_HIP(hipStreamSynchronize(h->c->stream));
  return TG_OK;
}

tg_chain chain_of(tg_hybrid *h) {
  tg_chain ch{};
  ch.pos = h->sys.pos;
  ch.mass = h->sys.mass;
  ch.n = h->sys.n;
  ch.exclude = h->d_excl;
  ch.member_pos = h->d_mpos;
  ch.member_mass = h->d_mmass;
  ch.nc = nc(h);
  for (int k = 0; k < 3; ++k) ch.com[k] = h->R[k];
  ch.m_chain = h->M;
  ch.r_crit = std::min(h->r_chain, h->cfg.r_chain0);   // Eq. 2
  ch.gamma_crit = h->cfg.gamma_crit;
  ch.eps_pm = 0.0;
  ch.pert_idx = h->d_pidx;
  ch.pert_cap = h->cfg.pert_cap;
  ch.n_pert = h->d_np;
  return ch;
}

// Forces of the current state: the tree (without the SMBH while it is in
// the chain) and the coupling with the chain.
tg_status forces(tg_hybrid *h) {
  tg_status st;
  if (!h->active) {
    if ((st = tg_forces(h->c, &h->sys, nullptr, nullptr))) return st;
    return tg_sync(h->c, nullptr);
  }
  if ((st = stage_members(h, h->V))) return st;
  tg_system y = h->sys;
  y.n_bh = 0;
  if ((st = tg_forces(h->c, &y, nullptr, nullptr))) return st;
  tg_chain ch = chain_of(h);
  if ((st = tg_chain_forces(h->c, &ch, nullptr, nullptr, h->sys.acc, h->sys.pot, h->d_com,
                            h->d_macc)))
    return st;
  if ((st = tg_sync(h->c, nullptr))) return st;
  return read_coupling(h);
}

// The coupling alone (the tree forces of the same positions are queued
// already): members written, chain forces added, the chain particle's force
// and the perturber count read back.
tg_status coupling(tg_hybrid *h) {
  tg_status st;
  if ((st = stage_members(h, h->V))) return st;
  tg_chain ch = chain_of(h);
  if ((st = tg_chain_forces(h->c, &ch, nullptr, nullptr, h->sys.acc, h->sys.pot, h->d_com,
                            h->d_macc)))
    return st;
  if ((st = tg_sync(h->c, nullptr))) return st;
  return read_coupling(h);
}

// The perturbers of the last coupling relative to the chain particle, at
// the current time (first-order prediction with dt = 0).
tg_status perturbers(tg_hybrid *h, std::vector<double> &px, std::vector<double> &pv,
                     std::vector<double> &pm, std::vector<int32_t> *ids) {
  const int np = std::min(h->n_pert, h->cfg.pert_cap);
  px.assign(3 * np, 0.0);
  pv.assign(3 * np, 0.0);
  pm.assign(np, 0.0);
  if (ids) ids->assign(np, 0);
  if (!np) return TG_OK;
  tg_chain ch = chain_of(h);
  tg_status st;
  if ((st = tg_predict_perturbers(h->c, &ch, h->sys.vel, h->V, 0.0, h->d_px, h->d_pv, h->d_pm)))
    return st;
  // four reads queued into the pinned area, one wait
  const int cap = h->cfg.pert_cap;
  double *rx = h->h_read + 4, *rv = rx + 3 * cap, *rm = rv + 3 * cap;
  int32_t *ri = reinterpret_cast<int32_t *>(rm + cap);
  hipStream_t sm = h->c->stream;
  TG_HIP(hipMemcpyAsync(rx, h->d_px, sizeof(double) * 3 * np, hipMemcpyDeviceToHost, sm));
  TG_HIP(hipMemcpyAsync(rv, h->d_pv, sizeof(double) * 3 * np, hipMemcpyDeviceToHost, sm));
  TG_HIP(hipMemcpyAsync(rm, h->d_pm, sizeof(double) * np, hipMemcpyDeviceToHost, sm));
  if (ids)
    TG_HIP(hipMemcpyAsync(ri, h->d_pidx, sizeof(int32_t) * np, hipMemcpyDeviceToHost, sm));
  TG_HIP(hipStreamSynchronize(sm));
  std::copy(rx, rx + 3 * np, px.begin());
  std::copy(rv, rv + 3 * np, pv.begin());
  std::copy(rm, rm + np, pm.begin());
  if (ids) std::copy(ri, ri + np, ids->begin());
  return TG_OK;
}

// Global coordinates and masses of the listed stars.
tg_status read_stars(tg_hybrid *h, const std::vector<int32_t> &ids, std::vector<double> &X,
                     std::vector<double> &W, std::vector<double> &mass) {
  const int k = (int)ids.size();
  X.assign(3 * k, 0.0);
  W.assign(3 * k, 0.0);
  mass.assign(k, 0.0);
  if (!k) return TG_OK;
  tg_status st;
  if ((st = to_dev(h, h->d_ids, ids.data(), sizeof(int32_t) * k))) return st;
  TG_HIP(launch_move_rows(h->c, h->d_rows, h->sys.pos, h->d_ids, k, false));
  if ((st = to_host(h, X.data(), h->d_rows, sizeof(double) * 3 * k))) return st;
  TG_HIP(launch_move_rows(h->c, h->d_rows, h->sys.vel, h->d_ids, k, false));
  if ((st = to_host(h, W.data(), h->d_rows, sizeof(double) * 3 * k))) return st;
  for (int i = 0; i < k; ++i)
    if ((st = to_host(h, &mass[i], h->sys.mass + ids[i], sizeof(double)))) return st;
  return TG_OK;
}

// The AR-chain's view of the members (with the kept chain state).
tg_archain archain_of(tg_hybrid *h) {
  tg_archain s{};
  s.n = nc(h);
  s.x = h->x.data();
  s.v = h->v.data();
  s.m = h->m.data();
  s.t = 0.0;
  s.B = h->B;
  s.ds = h->ds;
  s.chain = h->chain.data();
  s.cx = h->cx.data();
  s.cv = h->cv.data();
  s.chain_valid = h->chain_valid;
  return s;
}

tg_status ar_init(tg_hybrid *h) {
  const int n = nc(h);
  h->chain.assign(n, 0);
  h->cx.assign(3 * (n - 1), 0.0);
  h->cv.assign(3 * (n - 1), 0.0);
  h->chain_valid = 0;
  h->ds = 0.0;
  tg_archain s = archain_of(h);
  tg_status st = tg_archain_init(&s, h->G);
  if (st) return st;
  h->B = s.B;
  h->ds = s.ds;
  h->chain_valid = s.chain_valid;
  h->r_chain = max_radius(h);
  h->energy_error = 0.0;
  return TG_OK;
}

// A chain starts when stars come within r_chain0 of the SMBH.
tg_status maybe_start(tg_hybrid *h) {
  double bp[3], bv[3], bm;
  tg_status st;
  if ((st = to_host(h, bp, h->sys.bh_pos, sizeof(bp)))) return st;
  if ((st = tg_select_within(h->c, h->sys.pos, h->sys.n, nullptr, bp, h->cfg.r_chain0, h->d_sel,
                             kMaxChain - 1, h->d_nsel)))
    return st;
  if ((st = tg_sync(h->c, nullptr))) return st;
  int32_t k = 0;
  if ((st = to_host(h, &k, h->d_nsel, sizeof(int32_t)))) return st;
  if (k < 1) return TG_OK;
  std::vector<int32_t> ids(k);
  if ((st = to_host(h, ids.data(), h->d_sel, sizeof(int32_t) * k))) return st;
  std::vector<double> X, W, mass;
  if ((st = read_stars(h, ids, X, W, mass))) return st;
  if ((st = to_host(h, bv, h->sys.bh_vel, sizeof(bv)))) return st;
  if ((st = to_host(h, &bm, h->sys.bh_mass, sizeof(double)))) return st;
  // member 0 is the SMBH, then the stars in ascending order
  std::vector<double> GX(bp, bp + 3), GW(bv, bv + 3);
  GX.insert(GX.end(), X.begin(), X.end());
  GW.insert(GW.end(), W.begin(), W.end());
  h->star.assign(1, -1);
  h->star.insert(h->star.end(), ids.begin(), ids.end());
  h->m.assign(1, bm);
  h->m.insert(h->m.end(), mass.begin(), mass.end());
  reform(h, GX, GW);
  if ((st = ar_init(h))) return st;
  if ((st = set_ghosts(h, ids, mass, true))) return st;
  h->active = true;
  ++h->starts;
  return forces(h);
}

// Accelerations of the listed stars ([k][3]).
tg_status read_acc(tg_hybrid *h, const std::vector<int32_t> &ids, std::vector<double> &A) {
  const int k = (int)ids.size();
  A.assign(3 * k, 0.0);
  if (!k) return TG_OK;
  tg_status st;
  if ((st = to_dev(h, h->d_ids, ids.data(), sizeof(int32_t) * k))) return st;
  TG_HIP(launch_move_rows(h->c, h->d_rows, h->sys.acc, h->d_ids, k, false));
  return to_host(h, A.data(), h->d_rows, sizeof(double) * 3 * k);
}

// Block levels of the listed stars (in batches of kMaxChain).
tg_status read_levels(tg_hybrid *h, const tg_blocks *b, const std::vector<int32_t> &ids,
                      std::vector<uint8_t> &lv) {
  lv.assign(ids.size(), 0);
  tg_status st;
  for (size_t o = 0; o < ids.size(); o += kMaxChain) {
    const int k = (int)std::min<size_t>(kMaxChain, ids.size() - o);
    if ((st = to_dev(h, h->d_ids, ids.data() + o, sizeof(int32_t) * k))) return st;
    TG_HIP(launch_gather_bytes(h->c, h->d_flag, b->level, h->d_ids, k));
    if ((st = to_host(h, lv.data() + o, h->d_flag, (size_t)k))) return st;
  }
  return TG_OK;
}

// Whether a star on level l ends a step at substep k.
bool ends_at(uint8_t l, int64_t k, int nlev) {
  const int64_t per = (int64_t)1 << (nlev - 1 - (int)l);
  return k % per == 0;
}

// Velocities of stars at the end of their own step: W = v + a h with the
// pending closing half kick h = (dt_max 2^-level) / 2 (the kick's rounding).
void sync_vel(const std::vector<double> &v, const std::vector<double> &a,
              const std::vector<uint8_t> &lv, double dt_max, std::vector<double> &W) {
#pragma clang fp contract(off)
  W.resize(v.size());
  for (size_t i = 0; i < lv.size(); ++i) {
    const double hk = std::ldexp(dt_max, -(int)lv[i]) * 0.5;
    for (int d = 0; d < 3; ++d) W[3 * i + d] = v[3 * i + d] + a[3 * i + d] * hk;
  }
}

// The membership routine on the members and the listed perturber offsets.
tg_status decide(tg_hybrid *h, const std::vector<double> &px, int np,
                 std::vector<int32_t> &ab, std::vector<int32_t> &es, tg_membership_out &out) {
  const int n = nc(h);
  std::vector<uint8_t> massive(n, 0);
  for (int i = 0; i < n; ++i) massive[i] = h->star[i] < 0 ? 1 : 0;
  ab.assign(std::max(np, 1), 0);
  es.assign(std::max(n, 1), 0);
  tg_membership_in in{};
  in.n = n;
  in.x = h->x.data();
  in.v = h->v.data();
  in.m = h->m.data();
  in.massive = massive.data();
  in.designated = 0;
  in.r_chain = h->r_chain;
  in.r_chain0 = h->cfg.r_chain0;
  in.gamma = h->cfg.gamma_esc;
  in.np = np;
  in.px = px.data();
  out = tg_membership_out{};
  out.absorb = ab.data();
  out.escape = es.data();
  return tg_chain_membership(&in, &out);
}

// The chain after a membership decision: the leaving members go back to
// the tree with their global coordinates (velocities relative to Vref),
// the joining stars (global X, W given) are appended and become ghosts.
// Returns the rows of the stars that left in *back.
tg_status apply_membership(tg_hybrid *h, const tg_membership_out &out,
                           const std::vector<int32_t> &es, const double *Vref,
                           const std::vector<int32_t> &join, const std::vector<double> &JX,
                           const std::vector<double> &JW, const std::vector<double> &jm,
                           std::vector<int32_t> *back) {
#pragma clang fp contract(off)
  const int n = nc(h);
  std::vector<double> X(3 * n), W(3 * n);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) {
      X[3 * i + k] = h->R[k] + h->x[3 * i + k];
      W[3 * i + k] = Vref[k] + h->v[3 * i + k];
    }
  std::vector<bool> leaves(n, out.terminate != 0);
  for (int e = 0; e < out.n_escape; ++e) leaves[es[e]] = true;
  std::vector<int32_t> star;
  std::vector<double> m, GX, GW, BX, BW, bm;
  back->clear();
  tg_status st;
  for (int i = 0; i < n; ++i) {
    if (leaves[i]) {
      if (h->star[i] >= 0) {
        back->push_back(h->star[i]);
        bm.push_back(h->m[i]);
        BX.insert(BX.end(), &X[3 * i], &X[3 * i] + 3);
        BW.insert(BW.end(), &W[3 * i], &W[3 * i] + 3);
      } else if ((st = write_smbh(h, &X[3 * i], &W[3 * i]))) {
        return st;
      }
      continue;
    }
    star.push_back(h->star[i]);
    m.push_back(h->m[i]);
    GX.insert(GX.end(), &X[3 * i], &X[3 * i] + 3);
    GW.insert(GW.end(), &W[3 * i], &W[3 * i] + 3);
  }
  if ((st = restore_rows(h, *back, BX, BW, bm))) return st;
  h->escaped += (int64_t)back->size();
  if (out.terminate) {
    h->active = false;
    h->star.clear();
    h->x.clear();
    h->v.clear();
    h->m.clear();
    h->n_pert = 0;
    for (int k = 0; k < 3; ++k) h->a_com[k] = 0.0;
    ++h->ended;
    return TG_OK;
  }
  star.insert(star.end(), join.begin(), join.end());
  m.insert(m.end(), jm.begin(), jm.end());
  GX.insert(GX.end(), JX.begin(), JX.end());
  GW.insert(GW.end(), JW.begin(), JW.end());
  h->star = star;
  h->m = m;
  reform(h, GX, GW);
  if ((st = ar_init(h))) return st;
  if ((st = set_ghosts(h, join, jm, true))) return st;
  h->absorbed += (int64_t)join.size();
  return TG_OK;
}

// Membership at the end of a step (positions and velocities in step):
// absorb, escape, or end the chain; the forces again after a change.
tg_status membership(tg_hybrid *h) {
  std::vector<double> px, pv, pm;
  std::vector<int32_t> pids, ab, es;
  tg_status st;
  if ((st = perturbers(h, px, pv, pm, &pids))) return st;
  tg_membership_out out;
  if ((st = decide(h, px, (int)pids.size(), ab, es, out))) return st;
  if (!out.terminate && out.n_absorb == 0 && out.n_escape == 0) return TG_OK;
  if (nc(h) - out.n_escape + out.n_absorb > kMaxChain && !out.terminate)
    return fail(TG_ECAPACITY, "tg_hybrid_step: more than 256 chain members");
  std::vector<int32_t> join, back;
  std::vector<double> JX, JW, jm;
  if (!out.terminate) {
    for (int a = 0; a < out.n_absorb; ++a) join.push_back(pids[ab[a]]);
    if ((st = read_stars(h, join, JX, JW, jm))) return st;
  }
  const double V0[3] = {h->V[0], h->V[1], h->V[2]};
  if ((st = apply_membership(h, out, es, V0, join, JX, JW, jm, &back))) return st;
  return forces(h);
}

// Forces for a device list of stars (idx, n_act on the device; NULL: all):
// the tree without the SMBH while it is a member, then the coupling for the
// same list; the chain particle's force and the perturber list always.
tg_status forces_list(tg_hybrid *h, const int32_t *idx, const int32_t *n_act) {
  tg_status st;
  if (!h->active) {
    if ((st = tg_forces(h->c, &h->sys, idx, n_act))) return st;
    return tg_sync(h->c, nullptr);
  }
  if ((st = stage_members(h, h->V))) return st;
  tg_system y = h->sys;
  y.n_bh = 0;
  if ((st = tg_forces(h->c, &y, idx, n_act))) return st;
  tg_chain ch = chain_of(h);
  if ((st = tg_chain_forces(h->c, &ch, idx, n_act, h->sys.acc, h->sys.pot, h->d_com,
                            h->d_macc)))
    return st;
  if ((st = tg_sync(h->c, nullptr))) return st;
  return read_coupling(h);
}

// Block substeps: stars that return to the tree (escaped, or all members of
// a chain that ends) go to the finest level, which ends a step at every
// substep, and get their forces now (with a chain, the chain particle's
// force is formed again for the new membership; without, the SMBH's).
// Their velocities, in step, are then stored half a kick back, so the next
// substep's closing half kick brings them into step.
tg_status returned_stars(tg_hybrid *h, const tg_blocks *b, const std::vector<int32_t> &back) {
  const int k = (int)back.size();
  std::vector<uint8_t> lv(k, (uint8_t)(b->nlev - 1));
  tg_status st;
  for (int i = 0; i < k; ++i)
    if ((st = to_dev(h, b->level + back[i], &lv[i], 1))) return st;
  if ((st = to_dev(h, h->d_sel, back.data(), sizeof(int32_t) * k))) return st;
  if ((st = to_dev(h, h->d_nsel, &k, sizeof(int32_t)))) return st;
  if ((st = forces_list(h, h->d_sel, h->d_nsel))) return st;
  if (k)
    TG_HIP(launch_kick(h->c, h->sys.vel, h->sys.acc, h->sys.n, h->d_sel, h->d_nsel, b->level,
                       -b->dt_max, nullptr, 0, nullptr));
  return TG_OK;
}

// Membership at substep k (the new counter), every velocity in step: the
// chain particle's with its pending closing half kick; perturbers are
// absorbed only at a substep where their own step ends.
tg_status membership_block(tg_hybrid *h, const tg_blocks *b, int64_t k) {
#pragma clang fp contract(off)
  const double dt_min = std::ldexp(b->dt_max, -(b->nlev - 1));
  double Vs[3];
  for (int d = 0; d < 3; ++d) Vs[d] = h->V[d] + h->a_com[d] * (0.5 * dt_min);
  std::vector<double> px, pv, pm;
  std::vector<int32_t> pids, ab, es;
  tg_status st;
  if ((st = perturbers(h, px, pv, pm, &pids))) return st;
  const int np = (int)pids.size();
  tg_membership_out out;
  if ((st = decide(h, px, np, ab, es, out))) return st;
  if (out.n_absorb > 0) {
    // candidates whose step does not end now are out of reach this substep
    std::vector<int32_t> cand;
    for (int a = 0; a < out.n_absorb; ++a) cand.push_back(pids[ab[a]]);
    std::vector<uint8_t> lv;
    if ((st = read_levels(h, b, cand, lv))) return st;
    bool again = false;
    for (int a = 0; a < out.n_absorb; ++a)
      if (!ends_at(lv[a], k, b->nlev)) {
        for (int d = 0; d < 3; ++d) px[3 * ab[a] + d] = 1e100;
        again = true;
      }
    if (again && (st = decide(h, px, np, ab, es, out))) return st;
  }
  if (!out.terminate && out.n_absorb == 0 && out.n_escape == 0) return TG_OK;
  if (nc(h) - out.n_escape + out.n_absorb > kMaxChain && !out.terminate)
    return fail(TG_ECAPACITY, "tg_hybrid_step_block: more than 256 chain members");
  std::vector<int32_t> join, back;
  std::vector<double> JX, JV, JW, jm, JA;
  if (!out.terminate) {
    for (int a = 0; a < out.n_absorb; ++a) join.push_back(pids[ab[a]]);
    std::vector<uint8_t> jl;
    if ((st = read_stars(h, join, JX, JV, jm))) return st;
    if ((st = read_acc(h, join, JA))) return st;
    if ((st = read_levels(h, b, join, jl))) return st;
    sync_vel(JV, JA, jl, b->dt_max, JW);
  }
  const bool ends = out.terminate != 0;
  if ((st = apply_membership(h, out, es, Vs, join, JX, JW, jm, &back))) return st;
  if ((st = returned_stars(h, b, back))) return st;
  if (ends) {
    TG_HIP(launch_kick(h->c, h->sys.bh_vel, h->sys.bh_acc, 1, nullptr, nullptr, nullptr,
                       -dt_min, nullptr, 0, nullptr));
    return tg_sync(h->c, nullptr);
  }
  for (int d = 0; d < 3; ++d) h->V[d] = h->V[d] - h->a_com[d] * (0.5 * dt_min);
  return tg_sync(h->c, nullptr);
}

// A chain starting at substep k (the new counter): the stars within
// r_chain0 of the SMBH whose own step ends at k join it; every velocity is
// brought into step (the SMBH's and the stars' pending closing half
// kicks); then only the chain particle's force (no star gets new forces),
// and the chain particle is stored half a kick back.
tg_status maybe_start_block(tg_hybrid *h, const tg_blocks *b, int64_t kk) {
#pragma clang fp contract(off)
  double bp[3], bv[3], ba[3], bm;
  tg_status st;
  if ((st = to_host(h, bp, h->sys.bh_pos, sizeof(bp)))) return st;
  if ((st = tg_select_within(h->c, h->sys.pos, h->sys.n, nullptr, bp, h->cfg.r_chain0, h->d_sel,
                             kMaxChain - 1, h->d_nsel)))
    return st;
  if ((st = tg_sync(h->c, nullptr))) return st;
  int32_t k = 0;
  if ((st = to_host(h, &k, h->d_nsel, sizeof(int32_t)))) return st;
  if (k < 1) return TG_OK;
  std::vector<int32_t> all(k), ids;
  if ((st = to_host(h, all.data(), h->d_sel, sizeof(int32_t) * k))) return st;
  std::vector<uint8_t> lv;
  if ((st = read_levels(h, b, all, lv))) return st;
  for (int i = 0; i < k; ++i)
    if (ends_at(lv[i], kk, b->nlev)) ids.push_back(all[i]);
  if (ids.empty()) return TG_OK;
  std::vector<double> X, V, A, W, mass;
  std::vector<uint8_t> il;
  if ((st = read_stars(h, ids, X, V, mass))) return st;
  if ((st = read_acc(h, ids, A))) return st;
  if ((st = read_levels(h, b, ids, il))) return st;
  sync_vel(V, A, il, b->dt_max, W);
  if ((st = to_host(h, bv, h->sys.bh_vel, sizeof(bv)))) return st;
  if ((st = to_host(h, ba, h->sys.bh_acc, sizeof(ba)))) return st;
  if ((st = to_host(h, &bm, h->sys.bh_mass, sizeof(double)))) return st;
  const double dt_min = std::ldexp(b->dt_max, -(b->nlev - 1));
  for (int d = 0; d < 3; ++d) bv[d] = bv[d] + ba[d] * (dt_min * 0.5);
  std::vector<double> GX(bp, bp + 3), GW(bv, bv + 3);
  GX.insert(GX.end(), X.begin(), X.end());
  GW.insert(GW.end(), W.begin(), W.end());
  h->star.assign(1, -1);
  h->star.insert(h->star.end(), ids.begin(), ids.end());
  h->m.assign(1, bm);
  h->m.insert(h->m.end(), mass.begin(), mass.end());
  reform(h, GX, GW);
  if ((st = ar_init(h))) return st;
  if ((st = set_ghosts(h, ids, mass, true))) return st;
  h->active = true;
  ++h->starts;
  const int32_t zero = 0;
  if ((st = to_dev(h, h->d_nsel, &zero, sizeof(int32_t)))) return st;
  if ((st = forces_list(h, h->d_sel, h->d_nsel))) return st;
  for (int d = 0; d < 3; ++d) h->V[d] = h->V[d] - h->a_com[d] * (0.5 * dt_min);
  return TG_OK;
}

}  // namespace

extern "C" {

tg_status tg_hybrid_create(tg_ctx *c, const tg_system *y, const tg_hybrid_config *cfg,
                           tg_hybrid **out) try {
  if (!c || !y || !cfg || !out) return fail(TG_EINVAL, "tg_hybrid_create: NULL argument");
  *out = nullptr;
  if (y->n_bh != 1 || y->n_sys != 1 || y->n < 1 || y->frozen)
    return fail(TG_EINVAL, "tg_hybrid_create: one system, one SMBH, no frozen mask");
  if (!(cfg->r_chain0 > 0.0) || !(cfg->gamma_crit > 0.0) || !(cfg->gamma_esc > 0.0) ||
      !(cfg->tol > 0.0) || !(cfg->ghost_mass > 0.0 && cfg->ghost_mass < 1.0) ||
      cfg->pert_cap < 1)
    return fail(TG_EINVAL, "tg_hybrid_create: bad configuration");
  tg_hybrid *h = new tg_hybrid();
  h->c = c;
  h->sys = *y;
  h->cfg = *cfg;
  h->G = c->cfg.G;
  hipError_t a = hipSuccess;
  auto A = [&](hipError_t r) { if (a == hipSuccess) a = r; };
  A(dalloc(&h->d_excl, y->n));
  A(dalloc(&h->d_flag, kMaxChain));
  A(dalloc(&h->d_pidx, cfg->pert_cap));
  A(dalloc(&h->d_sel, kMaxChain));
  A(dalloc(&h->d_nsel, 1));
  A(dalloc(&h->d_com, 4));
  A(dalloc(&h->d_macc, 3 * kMaxChain));
  A(dalloc(&h->d_px, 3 * (int64_t)cfg->pert_cap));
  A(dalloc(&h->d_pv, 3 * (int64_t)cfg->pert_cap));
  A(dalloc(&h->d_pm, cfg->pert_cap));
  A(dalloc(&h->d_vals, kMaxChain));
  A(dalloc(&h->d_stage, (int64_t)kStageBytes));
  A(hipHostMalloc((void **)&h->h_stage, kStageBytes, hipHostMallocDefault));
  A(hipHostMalloc((void **)&h->h_read,
                  sizeof(double) * (4 + 7 * (size_t)cfg->pert_cap) +
                      sizeof(int32_t) * (size_t)cfg->pert_cap,
                  hipHostMallocDefault));
  if (h->d_stage) {
    h->d_ids = reinterpret_cast<int32_t *>(h->d_stage + kOffIds);
    h->d_rows = reinterpret_cast<double *>(h->d_stage + kOffRows);
    h->d_mpos = reinterpret_cast<double *>(h->d_stage + kOffMpos);
    h->d_mmass = reinterpret_cast<double *>(h->d_stage + kOffMmass);
    h->d_bh = reinterpret_cast<double *>(h->d_stage + kOffBh);
  }
  if (h->d_com) h->d_np = reinterpret_cast<int32_t *>(h->d_com + 3);
  if (h->h_stage) std::memset(h->h_stage, 0, kStageBytes);
  if (a == hipSuccess) A(hipMemset(h->d_excl, 0, (size_t)y->n));
  if (a == hipSuccess) A(hipDeviceSynchronize());
  h->sys.frozen = h->d_excl;   // ghosts are held still in block substeps
  if (a != hipSuccess) {
    tg_hybrid_destroy(h);
    return hip_fail(a, "tg_hybrid_create");
  }
  *out = h;
  return TG_OK;
} TG_HOST_CATCH("tg_hybrid_create")

tg_status tg_hybrid_begin(tg_hybrid *h) try {
  if (!h) return fail(TG_EINVAL, "tg_hybrid_begin: NULL");
  tg_status st = forces(h);
  if (st) return st;
  return h->active ? TG_OK : maybe_start(h);
} TG_HOST_CATCH("tg_hybrid_begin")

tg_status tg_hybrid_step(tg_hybrid *h, double dt) try {
#pragma clang fp contract(off)
  if (!h) return fail(TG_EINVAL, "tg_hybrid_step: NULL");
  Timer whole(h->step_s);
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(TG_EINVAL, "tg_hybrid_step: dt must be > 0");
  tg_status st;
  ++h->steps;
  if (!h->active) {
    if ((st = tg_step_kdk(h->c, &h->sys, dt))) return st;
    if ((st = tg_sync(h->c, nullptr))) return st;
    return maybe_start(h);
  }
  const int64_t n = h->sys.n;
  // (6) opening half kick of the stars (ghosts stay) and of the chain particle
  TG_HIP(launch_kick(h->c, h->sys.vel, h->sys.acc, n, nullptr, nullptr, nullptr, dt, nullptr, 0,
                     h->d_excl));
  for (int k = 0; k < 3; ++k) h->V[k] = h->V[k] + h->a_com[k] * (0.5 * dt);
  // (3) the chain step: the perturbers of the last coupling on the straight
  // lines of this step's drift, relative to the chain particle
  std::vector<double> px, pv, pm;
  if ((st = perturbers(h, px, pv, pm, nullptr))) return st;
  // (6) drift, and the tree forces at the new positions (ghosts where they
  // joined, no SMBH), queued on the GPU while the chain advances on the host
  TG_HIP(launch_drift(h->c, h->sys.pos, h->sys.vel, n, dt, h->d_excl));
  for (int k = 0; k < 3; ++k) h->R[k] = h->R[k] + h->V[k] * dt;
  {
    tg_system y = h->sys;
    y.n_bh = 0;
    if ((st = tg_forces(h->c, &y, nullptr, nullptr))) return st;
  }
  tg_archain s = archain_of(h);
  tg_archain_perturbers P{};
  P.np = (int32_t)pm.size();
  P.x = px.data();
  P.v = pv.data();
  P.m = pm.data();
  P.t0 = 0.0;
  {
    Timer tm(h->ar_s);
    st = tg_archain_advance(&s, h->G, dt, h->cfg.tol, P.np ? &P : nullptr, nullptr);
  }
  if (st) return st;
  h->B = s.B;
  h->ds = s.ds;
  h->chain_valid = s.chain_valid;
  if ((st = tg_archain_energy(&s, h->G, &h->energy_error))) return st;
  h->r_chain = max_radius(h);
  // (6b) the coupling with the members' new positions, (6c) closing half kick
  if ((st = coupling(h))) return st;
  TG_HIP(launch_kick(h->c, h->sys.vel, h->sys.acc, n, nullptr, nullptr, nullptr, dt, nullptr, 0,
                     h->d_excl));
  for (int k = 0; k < 3; ++k) h->V[k] = h->V[k] + h->a_com[k] * (0.5 * dt);
  if ((st = stage_members(h, h->V))) return st;
  // (4)-(5) with chain and tree at the same time, then (8)
  if ((st = membership(h))) return st;
  return h->active ? TG_OK : maybe_start(h);
} TG_HOST_CATCH("tg_hybrid_step")

tg_status tg_hybrid_step_block(tg_hybrid *h, const tg_blocks *b) try {
#pragma clang fp contract(off)
  if (!h || !b) return fail(TG_EINVAL, "tg_hybrid_step_block: NULL");
  Timer whole(h->step_s);
  tg_status st;
  ++h->steps;
  int64_t k0 = 0;
  if (!h->active) {
    if ((st = tg_step_block(h->c, &h->sys, b))) return st;
    if ((st = tg_sync(h->c, nullptr))) return st;
    if ((st = to_host(h, &k0, b->k, sizeof(int64_t)))) return st;
    return maybe_start_block(h, b, k0);
  }
  const double dt = std::ldexp(b->dt_max, -(b->nlev - 1));
  if ((st = to_host(h, &k0, b->k, sizeof(int64_t)))) return st;
  // the stars' closing kicks, levels and opening kicks (ghosts are frozen)
  if ((st = block_stars_kick(h->c, &h->sys, b))) return st;
  // the chain particle sits on the finest level: closing (not at k = 0)
  // and opening half kicks with the force of the last substep
  if (k0 != 0)
    for (int k = 0; k < 3; ++k) h->V[k] = h->V[k] + h->a_com[k] * (0.5 * dt);
  for (int k = 0; k < 3; ++k) h->V[k] = h->V[k] + h->a_com[k] * (0.5 * dt);
  // (3) the chain step over the substep, the perturbers on the straight
  // lines of their drift
  std::vector<double> px, pv, pm;
  if ((st = perturbers(h, px, pv, pm, nullptr))) return st;
  if ((st = block_stars_drift(h->c, &h->sys, b))) return st;
  for (int k = 0; k < 3; ++k) h->R[k] = h->R[k] + h->V[k] * dt;
  // tree forces of the stars active at the new k, queued while the chain
  // advances on the host
  {
    tg_system y = h->sys;
    y.n_bh = 0;
    if ((st = tg_forces(h->c, &y, b->active_idx, b->n_active))) return st;
  }
  tg_archain s = archain_of(h);
  tg_archain_perturbers P{};
  P.np = (int32_t)pm.size();
  P.x = px.data();
  P.v = pv.data();
  P.m = pm.data();
  P.t0 = 0.0;
  {
    Timer tm(h->ar_s);
    st = tg_archain_advance(&s, h->G, dt, h->cfg.tol, P.np ? &P : nullptr, nullptr);
  }
  if (st) return st;
  h->B = s.B;
  h->ds = s.ds;
  h->chain_valid = s.chain_valid;
  if ((st = tg_archain_energy(&s, h->G, &h->energy_error))) return st;
  h->r_chain = max_radius(h);
  // the coupling for the same stars with the members' new positions, and
  // the chain particle's force
  if ((st = stage_members(h, h->V))) return st;
  {
    tg_chain ch = chain_of(h);
    if ((st = tg_chain_forces(h->c, &ch, b->active_idx, b->n_active, h->sys.acc, h->sys.pot,
                              h->d_com, h->d_macc)))
      return st;
  }
  if ((st = tg_sync(h->c, nullptr))) return st;
  if ((st = read_coupling(h))) return st;
  // (4)-(5) with every velocity in step, then (8)
  if ((st = membership_block(h, b, k0 + 1))) return st;
  if (h->active) {
    double Vs[3];
    for (int k = 0; k < 3; ++k) Vs[k] = h->V[k] + h->a_com[k] * (0.5 * dt);
    return stage_members(h, Vs);
  }
  return maybe_start_block(h, b, k0 + 1);
} TG_HOST_CATCH("tg_hybrid_step_block")

tg_status tg_hybrid_state_get(const tg_hybrid *h, tg_hybrid_state *st, int32_t *members_out,
                              double *member_x, double *member_v) {
  if (!h || !st) return fail(TG_EINVAL, "tg_hybrid_state_get: NULL");
  st->active = h->active ? 1 : 0;
  st->n_members = h->active ? nc(h) : 0;
  st->n_perturbers = h->active ? h->n_pert : 0;
  for (int k = 0; k < 3; ++k) {
    st->com[k] = h->R[k];
    st->com_vel[k] = h->V[k];
  }
  st->m_chain = h->M;
  st->r_chain = h->r_chain;
  st->energy_error = h->energy_error;
  st->steps = h->steps;
  st->starts = h->starts;
  st->absorbed = h->absorbed;
  st->escaped = h->escaped;
  st->ended = h->ended;
  st->archain_seconds = h->ar_s;
  st->step_seconds = h->step_s;
  if (h->active) {
    if (members_out) std::copy(h->star.begin(), h->star.end(), members_out);
    if (member_x) std::copy(h->x.begin(), h->x.end(), member_x);
    if (member_v) std::copy(h->v.begin(), h->v.end(), member_v);
  }
  return TG_OK;
}

void tg_hybrid_destroy(tg_hybrid *h) {
  if (!h) return;
  void *ptrs[] = {h->d_excl, h->d_flag, h->d_pidx, h->d_sel, h->d_nsel, h->d_com,
                  h->d_macc, h->d_px, h->d_pv, h->d_pm, h->d_vals, h->d_stage};
  if (h->c) (void)hipStreamSynchronize(h->c->stream);
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (h->h_stage) (void)hipHostFree(h->h_stage);
  if (h->h_read) (void)hipHostFree(h->h_read);
  delete h;
}

}  // extern "C"
