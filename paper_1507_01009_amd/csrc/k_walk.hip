// Active groups, the group tree walk with the opening-angle
// test, and the softened P2P / quadrupole P2M force sums.
//
// One 64-lane wavefront owns one group of targets at a time (persistent
// grid, groups taken from per-XCD queues).  The walk is breadth first: the
// frontier holds the cells opened on the level above as ranges of
// consecutive children, and the wave tests the children of eight of them at
// once (eight lanes each) against the group's box,
//   accept iff side^2 < theta^2 d^2,  d = box-to-centre-of-mass distance,
// evaluated in double precision with no contraction (bit-identical decisions
// to the plain definition).  A second mode replaces it by the relative
// test (G M s^2 / d^4 <= alpha min|a_old|, group box outside the cell cube
// enlarged by 20 %; the paper's "Gadget" criterion, Sec. 3, run set-up, in
// the form of Springel 2005, Sec. 3.1).  Ballot + mbcnt compaction appends accepted
// cells to an LDS P2M list and the particles of refused leaves to an LDS
// P2P queue; a refused internal cell goes onto the next frontier as one
// {first child, child count} record.  Whenever a list holds a full tile it
// is flushed: the sources are staged in LDS once and each lane sums one
// slice of them (every slices-th entry) onto the T (1..3) targets it holds,
// on the vector ALUs.  No MFMA: a P2M pair is a chain of dependent scalar
// operations around one rsqrt, and the bilinear parts that could be cast as
// products have an N dimension of 1-9, which FP32 MFMA (twice the unpacked
// VALU rate) would mostly pad.
//
// Precision modes.  FP64: all sums in double, rsqrt from the hardware
// estimate plus one third-order correction (Householder).  MIXED: the walk
// decisions stay double; targets and sources are taken relative to the
// group's box centre c_g in double and rounded to float, the interaction
// arithmetic is float with the hardware rsqrt, and each tile's float
// partial sums (at most 128 sources per lane slice) are added into per-target
// double accumulators (one conversion and one FP64 add, both full rate).
//
// Flops per interaction as written in p2p_term / p2m_term (FMA = 2; the
// rsqrt and, in FP64, its refinement are not counted):
//   P2P 19: 3 sub, 6 for r^2 + eps^2, 3 for m D1 and m D3, 6 for the three
//          accelerations, 1 for the potential.
//   P2M 54: 3 sub, 6 for r^2 + eps^2, 3 for D2..D5, 15 for Q x, 6 for W,
//          2 for D4 W, 3 for the radial coefficient, 12 for the
//          accelerations, 4 for the potential (Q = 3S - T I, -T eps^2 and M
//          of every node are formed once per evaluation, k_cell_records).
#include <type_traits>

#include "tg_internal.h"

namespace tg {

// Most targets a lane holds (the per-group choice is 1..this), and the
// occupancy the kernel is compiled for, per precision mode.
#ifndef TG_WALK_MAXT_MIXED
#define TG_WALK_MAXT_MIXED 3
#endif
#ifndef TG_WALK_MAXT_MIXED_SPLINE
#define TG_WALK_MAXT_MIXED_SPLINE 2        // the spline terms need more registers
#endif
#ifndef TG_WALK_MAXT_FP64
#define TG_WALK_MAXT_FP64 3
#endif
#ifndef TG_WALK_WAVES_MIXED
#define TG_WALK_WAVES_MIXED 4
#endif
#ifndef TG_WALK_WAVES_FP64
#define TG_WALK_WAVES_FP64 2
#endif

constexpr int kTile = 128;                  // source tile entries (a flush uses <= 128)
constexpr int kMCap = 128 + 64;             // P2M cell list (LDS): < one flush + one append
constexpr int kQCap = 128 + 64 * 8;         // P2P particle queue (LDS); overflow goes leaf by leaf

struct WalkArgs {
  const uint4 *ninfo;       // {first, count, child, nchild} per node
  const double4 *com;
  const double4 *rel;       // relative test: per node {lo, P}, {hi, 0} (enlarged cube)
  const double *arel;       // relative test: per group (alpha alpha) min |a_old|^2
  const void *cell;         // walk records per node (float4[2] mixed, double4[2] FP64)
  const double4 *spart;
  const uint32_t *root_of;
  const uint4 *groups;
  const uint32_t *alist;
  const double *abox;
  const uint8_t *sact;
  const uint32_t *perm;
  TreeCounters *ctr;
  unsigned long long *wtot;   // force walk: per workgroup {P2P, P2M, targets, groups}
  uint32_t *err;
  uint32_t *frontier;
  int fcap;
  double th2, eps2, G;
  double *acc, *pot;
  // external point masses (SMBHs) of each system, added in FP64 per target
  const double *ext_pos, *ext_mass, *ext_eps;
  const int32_t *ext_seg;   // [S+1]: externals of system s
  double eps;
  // list mode
  uint32_t *wl_count;
  const uint32_t *wl_off;
  uint32_t *ids;
};

// ---------------------------------------------------------------- helpers
// Exclusive prefix sum over the 64 lanes and the wave total, on DPP lane
// moves: shifts by 1, 2, 4, 8 inside each row of 16, then row 0's total to
// rows 1 and 3 and the first 32 lanes' total to rows 2 and 3.
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t &tot) {
  uint32_t x = v;
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  tot = (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
  return x - v;
}

// Squared distance from the group box to the centre of mass, the same
// operations in the same order as the plain definition: d^2 = sum_k
// max(max(lo_k - c_k, c_k - hi_k), 0)^2.  fmax (one v_max_f64) equals the
// compare-and-select of the definition for the finite inputs the build
// guarantees.
__device__ __forceinline__ double box_d2(const double lo[3], const double hi[3], double4 c) {
#pragma clang fp contract(off)
  double d2 = 0.0;
  {
    double a = dsub(lo[0], c.x), b = dsub(c.x, hi[0]);
    const double m = fmax(fmax(a, b), 0.0);
    d2 = dadd(d2, dmul(m, m));
  }
  {
    double a = dsub(lo[1], c.y), b = dsub(c.y, hi[1]);
    const double m = fmax(fmax(a, b), 0.0);
    d2 = dadd(d2, dmul(m, m));
  }
  {
    double a = dsub(lo[2], c.z), b = dsub(c.z, hi[2]);
    const double m = fmax(fmax(a, b), 0.0);
    d2 = dadd(d2, dmul(m, m));
  }
  return d2;
}

// Opening-angle test: accept iff side^2 < theta^2 d^2 (c.w = side^2).
__device__ __forceinline__ bool mac_accept(const double lo[3], const double hi[3],
                                           double4 c, double th2) {
  return c.w < dmul(th2, box_d2(lo, hi, c));
}

// Relative test: accept iff P P <= A (d^2 d^2)(d^2 d^2), P = (G M) s^2,
// A = (alpha alpha) min |a_old|^2 of the group, and the box misses the
// enlarged cube [r0.xyz, r1.xyz] on some axis (touching counts as a hit).
__device__ __forceinline__ bool mac_rel(const double lo[3], const double hi[3], double4 c,
                                        double4 r0, double4 r1, double A) {
  const double d2 = box_d2(lo, hi, c);
  const double d4 = dmul(d2, d2);
  const bool near = dmul(r0.w, r0.w) <= dmul(A, dmul(d4, d4));
  const bool apart = lo[0] > r1.x || hi[0] < r0.x || lo[1] > r1.y || hi[1] < r0.y ||
                     lo[2] > r1.z || hi[2] < r0.z;
  return near && apart;
}

// 1/sqrt(x) in double: hardware estimate, then one third-order Householder
// step y <- y (1 + e/2 + 3e^2/8), e = 1 - x y^2.
__device__ __forceinline__ double rsqrt_dp(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double t = x * y;
  double e = fma(-t, y, 1.0);
  double p = fma(0.375, e, 0.5);
  return fma(y * e, p, y);
}


// ---------------------------------------------------------------- terms
template <class R> struct Vec4;
template <> struct Vec4<float> { using T = float4; };
template <> struct Vec4<double> { using T = double4; };

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return rsqrt_dp(x); }

// Softened quadrupole term of one cell on one target, x = target - com.
// Cell: a = {com, M}, b = {Qxx, Qyy, Qzz, -T eps^2}, c = {Qxy, Qxz, Qyz, -}
// with the traceless Q = 3S - T I, T = tr S.  With r^2 = |x|^2 + eps^2 and
// D_n = r^-n, the expansion of the softened potential about the centre of
// mass gives
//   W = x.Q.x - T eps^2      (= 3 x.S.x - T r^2)
//   a += -(M D3 + 2.5 D7 W) x + D5 Q x
//   phi -= M D1 + 0.5 D5 W
// (the same as -(M D3 + T D5 + 2.5 D7 W) x + 3 D5 S x, with T x folded
// into Q x).
template <class R>
__device__ __forceinline__ void p2m_term(typename Vec4<R>::T a, typename Vec4<R>::T b,
                                         typename Vec4<R>::T c, R tx, R ty, R tz, R e2,
                                         R &ax, R &ay, R &az, R &ph) {
  const R x = tx - a.x, y = ty - a.y, z = tz - a.z;
  const R r2 = fma(z, z, fma(y, y, fma(x, x, e2)));
  const R D1 = rsq(r2);
  const R u = D1 * D1, D3 = D1 * u, D5 = D3 * u;
  const R Qx = fma(c.y, z, fma(c.x, y, b.x * x));
  const R Qy = fma(c.z, z, fma(b.y, y, c.x * x));
  const R Qz = fma(b.z, z, fma(c.z, y, c.y * x));
  const R W = fma(z, Qz, fma(y, Qy, fma(x, Qx, b.w)));
  const R k = (u * W) * u;                     // D4 W
  const R C = D3 * fma(R(2.5), k, a.w);        // M D3 + 2.5 D7 W
  ax = fma(D5, Qx, fma(-C, x, ax));
  ay = fma(D5, Qy, fma(-C, y, ay));
  az = fma(D5, Qz, fma(-C, z, az));
  ph = fma(-D1, fma(R(0.5), k, a.w), ph);      // M D1 + 0.5 D5 W
}

// Softened particle term, source s = {position, m}; keep = false drops the
// pair (a target and itself).
template <class R>
__device__ __forceinline__ void p2p_term(typename Vec4<R>::T s, R tx, R ty, R tz, R e2,
                                         R &ax, R &ay, R &az, R &ph, bool keep = true) {
  const R dx = tx - s.x, dy = ty - s.y, dz = tz - s.z;
  const R r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2)));
  const R D1 = keep ? rsq(r2) : R(0);
  const R mD1 = s.w * D1;
  const R mD3 = mD1 * (D1 * D1);
  ax = fma(-mD3, dx, ax);
  ay = fma(-mD3, dy, ay);
  az = fma(-mD3, dz, az);
  ph -= mD1;
}

// Cubic-spline softening (Monaghan-Lattanzio kernel, support 2h, h = eps):
// with u = r/h, psi is the pair's softened 1/r and psi_k+1 = -(1/r) d psi_k
// / dr; beyond 2h they are 1/r, 1/r^3, 3/r^5, 15/r^7.  The Newtonian values
// come from one rsqrt; the polynomial pieces are evaluated only where some
// lane of the wave has a pair inside 2h.  At r = 0 (a particle and itself,
// coincident ones, or a zero-mass tile pad at the target) u = 0 selects the
// inner piece, which is finite; psi_3 (1/u there) is set to 0, since it
// multiplies x.S.x = 0.
template <class R>
__device__ __forceinline__ void spline_psi01(R r2, R h, R ih, R &p0, R &p1) {
  const R ir = rsq(r2);
  p0 = ir;
  p1 = ir * ir * ir;
  const R u = (r2 > R(0) ? r2 * ir : R(0)) * ih;
  if (u < R(2)) {
    const R u2 = u * u, ih3 = ih * ih * ih, iu = h * ir;
    const R a0 = ih * fma(u2, fma(u2, fma(R(-0.1), u, R(0.3)), R(-2.0 / 3.0)), R(1.4));
    const R a1 = ih3 * fma(u2, fma(R(0.5), u, R(-1.2)), R(4.0 / 3.0));
    const R b0 = ih * fma(R(-1.0 / 15.0), iu,
                          fma(u2, fma(u, fma(u, fma(u, R(1.0 / 30.0), R(-0.3)), R(1)),
                                      R(-4.0 / 3.0)), R(1.6)));
    const R b1 = ih3 * fma(R(-1.0 / 15.0), iu * iu * iu,
                           fma(u, fma(u, fma(u, R(-1.0 / 6.0), R(1.2)), R(-3)), R(8.0 / 3.0)));
    const bool in = u < R(1);
    p0 = in ? a0 : b0;
    p1 = in ? a1 : b1;
  }
}

template <class R>
__device__ __forceinline__ void spline_psi0123(R r2, R h, R ih, R &p0, R &p1, R &p2, R &p3) {
  const R ir = rsq(r2), ir2 = ir * ir;
  p0 = ir;
  p1 = ir * ir2;
  p2 = R(3) * p1 * ir2;
  p3 = R(5) * p2 * ir2;
  const R u = (r2 > R(0) ? r2 * ir : R(0)) * ih;
  if (u < R(2)) {
    const R u2 = u * u, ih2 = ih * ih, ih3 = ih2 * ih, ih5 = ih3 * ih2, ih7 = ih5 * ih2;
    const R iu = h * ir, iu2 = iu * iu, iu3 = iu2 * iu, iu5 = iu3 * iu2;
    const R a0 = ih * fma(u2, fma(u2, fma(R(-0.1), u, R(0.3)), R(-2.0 / 3.0)), R(1.4));
    const R a1 = ih3 * fma(u2, fma(R(0.5), u, R(-1.2)), R(4.0 / 3.0));
    const R a2 = ih5 * fma(R(-1.5), u, R(2.4));
    const R a3 = r2 > R(0) ? ih7 * (R(1.5) * iu) : R(0);   // multiplies V = 0 at r = 0
    const R b0 = ih * fma(R(-1.0 / 15.0), iu,
                          fma(u2, fma(u, fma(u, fma(u, R(1.0 / 30.0), R(-0.3)), R(1)),
                                      R(-4.0 / 3.0)), R(1.6)));
    const R b1 = ih3 * fma(R(-1.0 / 15.0), iu3,
                           fma(u, fma(u, fma(u, R(-1.0 / 6.0), R(1.2)), R(-3)), R(8.0 / 3.0)));
    const R b2 = ih5 * fma(R(-0.2), iu5, fma(R(3), iu, fma(R(0.5), u, R(-2.4))));
    const R b3 = ih7 * fma(R(-1), iu5 * iu2, fma(R(3), iu3, R(-0.5) * iu));
    const bool in = u < R(1);
    p0 = in ? a0 : b0;
    p1 = in ? a1 : b1;
    p2 = in ? a2 : b2;
    p3 = in ? a3 : b3;
  }
}

// Spline-softened cell term, x = target - com, cell as for p2m_term but
// b.w = T.  The second-order expansion of the kernel about the centre of
// mass, with V = x.Q.x + T |x|^2 (= 3 x.S.x):
//   a  += -(M psi_1 - 5/6 psi_2 T + psi_3 V / 6) x + (psi_2 / 3) Q x
//   phi -= M psi + psi_2 V / 6 - psi_1 T / 2
template <class R>
__device__ __forceinline__ void p2m_spline(typename Vec4<R>::T a, typename Vec4<R>::T b,
                                           typename Vec4<R>::T c, R tx, R ty, R tz, R h, R ih,
                                           R &ax, R &ay, R &az, R &ph) {
  const R x = tx - a.x, y = ty - a.y, z = tz - a.z;
  const R r2 = fma(z, z, fma(y, y, x * x));
  R p0, p1, p2, p3;
  spline_psi0123<R>(r2, h, ih, p0, p1, p2, p3);
  const R Qx = fma(c.y, z, fma(c.x, y, b.x * x));
  const R Qy = fma(c.z, z, fma(b.y, y, c.x * x));
  const R Qz = fma(b.z, z, fma(c.z, y, c.y * x));
  const R V = fma(b.w, r2, fma(z, Qz, fma(y, Qy, x * Qx)));
  const R V6 = V * R(1.0 / 6.0);
  const R C = fma(p3, V6, fma(R(-5.0 / 6.0) * p2, b.w, a.w * p1));
  const R q = p2 * R(1.0 / 3.0);
  ax = fma(q, Qx, fma(-C, x, ax));
  ay = fma(q, Qy, fma(-C, y, ay));
  az = fma(q, Qz, fma(-C, z, az));
  ph -= fma(p2, V6, fma(R(-0.5) * p1, b.w, a.w * p0));
}

// Spline-softened particle term, source s = {position, m}; keep = false
// drops the pair (a target and itself: x = 0, only the potential term).
template <class R>
__device__ __forceinline__ void p2p_spline(typename Vec4<R>::T s, R tx, R ty, R tz, R h, R ih,
                                           R &ax, R &ay, R &az, R &ph, bool keep = true) {
  const R dx = tx - s.x, dy = ty - s.y, dz = tz - s.z;
  const R r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  R p0, p1;
  spline_psi01<R>(r2, h, ih, p0, p1);
  const R mp1 = s.w * p1;
  ax = fma(-mp1, dx, ax);
  ay = fma(-mp1, dy, ay);
  az = fma(-mp1, dz, az);
  ph -= keep ? s.w * p0 : R(0);
}

// ---------------------------------------------------------------- tiles
struct P2MTileD { double4 a, b, c; };
struct P2MTileF { float4 a, b, c; };

// Targets per lane: a group of nt targets is spread over the 64 lanes as
// lt = ceil(nt / T) lane-targets (each lane holding up to T targets) times
// slices = floor(64 / lt) source slices; T is chosen per group to minimise
// the evaluations per source, T / slices.
template <bool kMixed, bool kSpline> struct Shape {
  static constexpr int kMaxT =
      kMixed ? (kSpline ? TG_WALK_MAXT_MIXED_SPLINE : TG_WALK_MAXT_MIXED) : TG_WALK_MAXT_FP64;
  static_assert(kMaxT >= 1 && kMaxT <= 3, "1..3 targets per lane");
};
template <bool kMixed>
constexpr int kRedT = Shape<kMixed, false>::kMaxT > Shape<kMixed, true>::kMaxT
                          ? Shape<kMixed, false>::kMaxT : Shape<kMixed, true>::kMaxT;

// Source tiles in LDS.  A flush of k sources fills entries [0, slices *
// trips) with trips = ceil(k / slices), the entries past k with zero mass;
// slice s evaluates the entries s, s + slices, s + 2 slices, ... (trips of
// them), so every lane runs the same trip count with no masking, and the
// slices of one trip read neighbouring entries (interleaving them measured
// 0.8% faster than contiguous runs per slice).  Full flushes take exactly
// slices * floor(128 / slices) (65..128) sources, so the fixed cost of a
// flush (two barriers, the staging set-up, the FP64 accumulation) is shared
// by as many sources as the tile holds.  `red` holds the per-lane sums of
// the final slice reduction.
template <bool kMixed> union TileMem;
template <> union __align__(16) TileMem<true> {
  P2MTileF m[kTile];
  float4 p[kTile];
  double red[kRedT<true> * 256];
};
template <> union __align__(16) TileMem<false> {
  P2MTileD m[kTile];
  double4 p[kTile];
  double red[kRedT<false> * 256];
};

// ------------------------------------------------------- force-mode sink
template <bool kMixed, bool kSpline>
struct ForceSink {
  using R = typename std::conditional<kMixed, float, double>::type;
  using R4 = typename Vec4<R>::T;
  static constexpr int kMaxT = Shape<kMixed, kSpline>::kMaxT;
  uint32_t *s_m;
  uint32_t *s_q;
  TileMem<kMixed> *tile;
  uint32_t nm, nq;
  unsigned long long cells, parts;   // wave-uniform totals
  int T, lt, slices, tfull, F, my_s;
  double cgx, cgy, cgz;              // coordinate origin of the group (0 in FP64)
  R e2;
  R h, ih;                           // spline softening length and its inverse
  R tx[kMaxT], ty[kMaxT], tz[kMaxT];
  const uint32_t *s_tgt;             // sorted indices of the nt targets (LDS)
  int nt;
  // The group's own particles [g0, g0 + gn) met in refused leaves are not
  // queued: bit b of own (own0 | own1 << 64) marks particle g0 + b, and
  // they are evaluated last, each target without its own pair.
  uint32_t g0, gn;
  unsigned long long own0, own1;     // wave-uniform
  // per-target totals in FP64 (mixed: each tile's FP32 partial sums are
  // added here, so rounding accumulates only within a tile)
  double hax[kMaxT], hay[kMaxT], haz[kMaxT], hph[kMaxT];

  __device__ void add(int k, R ax, R ay, R az, R ph) {
    hax[k] += (double)ax; hay[k] += (double)ay; haz[k] += (double)az; hph[k] += (double)ph;
  }

  template <int kT>
  __device__ void eval_m(int base, int trips_in, int st) {
    const int trips = __builtin_amdgcn_readfirstlane(trips_in);
    R ax[kT], ay[kT], az[kT], ph[kT];
#pragma unroll
    for (int k = 0; k < kT; ++k) ax[k] = ay[k] = az[k] = ph[k] = R(0);
    const auto *e = &tile->m[base];
    if constexpr (kSpline) {
      for (int it = 0; it < trips; ++it) {
        const R4 a = e[it * st].a, b = e[it * st].b, c = e[it * st].c;
#pragma unroll
        for (int k = 0; k < kT; ++k)
          p2m_spline<R>(a, b, c, tx[k], ty[k], tz[k], h, ih, ax[k], ay[k], az[k], ph[k]);
      }
    } else if constexpr (kT == 1) {
#pragma unroll 2
      for (int it = 0; it < trips; ++it)
        p2m_term<R>(e[it * st].a, e[it * st].b, e[it * st].c, tx[0], ty[0], tz[0], e2, ax[0], ay[0], az[0], ph[0]);
    } else {
      for (int it = 0; it < trips; ++it) {
        const R4 a = e[it * st].a, b = e[it * st].b, c = e[it * st].c;
#pragma unroll
        for (int k = 0; k < kT; ++k)
          p2m_term<R>(a, b, c, tx[k], ty[k], tz[k], e2, ax[k], ay[k], az[k], ph[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < kT; ++k) add(k, ax[k], ay[k], az[k], ph[k]);
  }

  // kOwn: entry et[k] of the tile is target k itself, its pair dropped
  template <int kT, bool kOwn = false>
  __device__ void eval_p(int base, int trips_in, int st, const uint32_t *et = nullptr) {
    const int trips = __builtin_amdgcn_readfirstlane(trips_in);
    R ax[kT], ay[kT], az[kT], ph[kT];
#pragma unroll
    for (int k = 0; k < kT; ++k) ax[k] = ay[k] = az[k] = ph[k] = R(0);
    const R4 *e = &tile->p[base];
    if constexpr (kOwn) {
      for (int it = 0; it < trips; ++it) {
        const R4 s = e[it * st];
        const uint32_t en = (uint32_t)(base + it * st);
#pragma unroll
        for (int k = 0; k < kT; ++k) {
          if constexpr (kSpline)
            p2p_spline<R>(s, tx[k], ty[k], tz[k], h, ih, ax[k], ay[k], az[k], ph[k], en != et[k]);
          else
            p2p_term<R>(s, tx[k], ty[k], tz[k], e2, ax[k], ay[k], az[k], ph[k], en != et[k]);
        }
      }
    } else if constexpr (kSpline) {
      for (int it = 0; it < trips; ++it) {
        const R4 s = e[it * st];
#pragma unroll
        for (int k = 0; k < kT; ++k)
          p2p_spline<R>(s, tx[k], ty[k], tz[k], h, ih, ax[k], ay[k], az[k], ph[k]);
      }
    } else if constexpr (kT == 1) {
#pragma unroll 4
      for (int it = 0; it < trips; ++it)
        p2p_term<R>(e[it * st], tx[0], ty[0], tz[0], e2, ax[0], ay[0], az[0], ph[0]);
    } else {
#pragma unroll 2
      for (int it = 0; it < trips; ++it) {
        const R4 s = e[it * st];
#pragma unroll
        for (int k = 0; k < kT; ++k)
          p2p_term<R>(s, tx[k], ty[k], tz[k], e2, ax[k], ay[k], az[k], ph[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < kT; ++k) add(k, ax[k], ay[k], az[k], ph[k]);
  }

  __device__ int trips_for(int k) const {
    return k == F ? tfull : (k + slices - 1) / slices;
  }

  // P2M tile entry of cell v, relative to the group origin
  __device__ void stage_cell(const WalkArgs &A, int e, bool live, uint32_t v) {
    if (live) {
      const double4 cm = A.com[v];
      const R4 *r = reinterpret_cast<const R4 *>(A.cell) + 2 * (size_t)v;
      const R4 q0 = r[0], q1 = r[1];
      tile->m[e].a = R4{(R)(cm.x - cgx), (R)(cm.y - cgy), (R)(cm.z - cgz), q1.w};
      tile->m[e].b = q0;
      tile->m[e].c = q1;
    } else {
      tile->m[e].a = tile->m[e].b = tile->m[e].c = R4{R(0), R(0), R(0), R(0)};
    }
  }

  __device__ void flush_p2m(const WalkArgs &A, const uint32_t *list, int k) {
    const int lane = (int)lane_id();
    const int trips = trips_for(k);
    const int ne = slices * trips;
    const int e0 = lane, e1 = lane + 64;
    const uint32_t v0 = e0 < k ? list[e0] : 0u, v1 = e1 < k ? list[e1] : 0u;
    if (e0 < ne) stage_cell(A, e0, e0 < k, v0);
    if (e1 < ne) stage_cell(A, e1, e1 < k, v1);
    __syncthreads();
    const int base = my_s;
    if (T == 1) eval_m<1>(base, trips, slices);
    else if constexpr (kMaxT >= 2) {
      if (T == 2) eval_m<2>(base, trips, slices);
      else if constexpr (kMaxT >= 3) eval_m<3>(base, trips, slices);
    }
    __syncthreads();
  }

  __device__ void stage_part(const WalkArgs &A, int e, bool live, uint32_t j) {
    R4 v = R4{R(0), R(0), R(0), R(0)};
    if (live) {
      const double4 p = A.spart[j];
      v = R4{(R)(p.x - cgx), (R)(p.y - cgy), (R)(p.z - cgz), (R)p.w};
    }
    tile->p[e] = v;
  }

  __device__ void flush_p2p(const WalkArgs &A, const uint32_t *list, int k) {
    const int lane = (int)lane_id();
    const int trips = trips_for(k);
    const int ne = slices * trips;
    const int e0 = lane, e1 = lane + 64;
    const uint32_t j0 = e0 < k ? list[e0] : 0u, j1 = e1 < k ? list[e1] : 0u;
    if (e0 < ne) stage_part(A, e0, e0 < k, j0);
    if (e1 < ne) stage_part(A, e1, e1 < k, j1);
    __syncthreads();
    const int base = my_s;
    if (T == 1) eval_p<1>(base, trips, slices);
    else if constexpr (kMaxT >= 2) {
      if (T == 2) eval_p<2>(base, trips, slices);
      else if constexpr (kMaxT >= 3) eval_p<3>(base, trips, slices);
    }
    __syncthreads();
  }

  // rank among the own particles of bit b (b < 128)
  __device__ uint32_t own_rank(uint32_t b) const {
    return b < 64u ? (uint32_t)__popcll(own0 & ((1ull << b) - 1ull))
                   : (uint32_t)__popcll(own0) +
                         (uint32_t)__popcll(own1 & ((1ull << (b - 64u)) - 1ull));
  }

  __device__ bool own_bit(uint32_t b) const {
    return b < 64u ? ((own0 >> b) & 1ull) != 0ull : ((own1 >> (b - 64u)) & 1ull) != 0ull;
  }

  // One tile of the kq queued particles s_q[0, kq) followed by the own
  // particles of ranks [o, o + k) at entries kq + rank - o, each target
  // without itself.
  __device__ void flush_own(const WalkArgs &A, int kq, uint32_t o, int k) {
    const uint32_t lane = lane_id();
    const int trips = trips_for(kq + k);
    const int ne = slices * trips;
    for (int e = (int)lane; e < kq; e += 64) stage_part(A, e, true, s_q[e]);
    for (uint32_t b = lane; b < 128u; b += 64u) {
      if (b < gn && own_bit(b)) {
        const int e = (int)(own_rank(b) - o);
        if (e >= 0 && e < k) stage_part(A, kq + e, true, g0 + b);
      }
    }
    for (int e = kq + k + (int)lane; e < ne; e += 64) stage_part(A, e, false, 0u);
    // the lane's targets as placed at the start (missing ones repeat j)
    const int j = (int)lane % lt;
    uint32_t et[kMaxT];
#pragma unroll
    for (int q = 0; q < kMaxT; ++q) {
      const int i = j + q * lt;
      const uint32_t b = s_tgt[i < nt ? i : j] - g0;   // < gn: targets lie in the group
      et[q] = own_bit(b) ? own_rank(b) - o + (uint32_t)kq : 0xffffffffu;
    }
    __syncthreads();
    const int base = my_s;
    if (T == 1) eval_p<1, true>(base, trips, slices, et);
    else if constexpr (kMaxT >= 2) {
      if (T == 2) eval_p<2, true>(base, trips, slices, et);
      else if constexpr (kMaxT >= 3) eval_p<3, true>(base, trips, slices, et);
    }
    __syncthreads();
  }

  // Queue the particles [lf, lf + lc), flushing whenever a tile is full.
  __device__ void append_run(const WalkArgs &A, uint32_t lf, uint32_t lc) {
    uint32_t o = 0;
    while (o < lc) {
      const uint32_t take = min(lc - o, (uint32_t)kQCap - nq);
      for (uint32_t j = lane_id(); j < take; j += 64u) s_q[nq + j] = lf + o + j;
      nq += take;
      o += take;
      __syncthreads();
      drain_q(A);
    }
  }

  __device__ void p2m(const WalkArgs &A, bool pred, uint32_t node) {
    const unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return;
    if (pred) s_m[nm + lanes_below(mask)] = node;
    const uint32_t c = (uint32_t)__popcll(mask);
    nm += c;
    cells += c;
    __syncthreads();
    if (nm >= (uint32_t)F) {          // nm < F + 64 <= 2 F: one flush
      flush_p2m(A, s_m + (nm - F), F);
      nm -= F;
    }
  }

  __device__ void drain_q(const WalkArgs &A) {
    while (nq >= (uint32_t)F) {
      flush_p2p(A, s_q + (nq - F), F);
      nq -= F;
    }
  }

  // pred: this lane's leaf is refused; c = its particle count (0 if not
  // pred), pre / tot = exclusive prefix and wave total of c
  __device__ void p2p(const WalkArgs &A, bool pred, uint32_t node, uint32_t f,
                      uint32_t c, uint32_t pre, uint32_t tot) {
    (void)node;
    const unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return;
    parts += tot;
    // the leaf minus the group's own particles: [f, oa) and [ob, f + c)
    uint32_t oa = f + c, ob = f + c;
    if (pred) {
      oa = min(max(f, g0), f + c);
      ob = min(max(f, g0 + gn), f + c);
    }
    const unsigned long long omask = __ballot(ob > oa);
    if (omask != 0ull) {
      // rare (the group's own leaves): mark them, queue the rest
      unsigned long long m = omask;
      while (m) {
        const int L = __ffsll((long long)m) - 1;
        m &= m - 1ull;
        const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)oa, L) - g0;
        const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)ob, L) - g0;
        for (uint32_t q = a; q < b; ++q) {     // at most gn <= 128 bits in all
          if (q < 64u) own0 |= 1ull << q; else own1 |= 1ull << (q - 64u);
        }
      }
      pre = wave_excl_scan(c - (ob - oa), tot);
    }
    const uint32_t left = oa - f, right = f + c - ob;
    if (nq + tot <= (uint32_t)kQCap) {
      for (uint32_t k = 0; k < left; ++k) s_q[nq + pre + k] = f + k;
      for (uint32_t k = 0; k < right; ++k) s_q[nq + pre + left + k] = ob + k;
      nq += tot;
      __syncthreads();
      drain_q(A);
      return;
    }
    // rare: many large leaves at once; one run at a time
    unsigned long long m = mask;
    while (m) {
      const int L = __ffsll((long long)m) - 1;
      m &= m - 1ull;
      append_run(A, (uint32_t)__shfl((int)f, L, 64), (uint32_t)__shfl((int)left, L, 64));
      append_run(A, (uint32_t)__shfl((int)ob, L, 64), (uint32_t)__shfl((int)right, L, 64));
    }
  }

  __device__ void finish(const WalkArgs &A) {
    if (nm > 0) flush_p2m(A, s_m, (int)nm);
    nm = 0;
    // the queue's rest (nq < F) and the own particles share the last tiles
    const uint32_t no = (uint32_t)(__popcll(own0) + __popcll(own1));
    uint32_t o = 0;
    while (nq + (no - o) > 0u) {
      const uint32_t k = min(no - o, (uint32_t)F - nq);
      flush_own(A, (int)nq, o, (int)k);
      nq = 0;
      o += k;
    }
    own0 = own1 = 0ull;
  }
};

// -------------------------------------------------------- list-mode sinks
struct CountSink {
  uint32_t nm = 0, np = 0;
  __device__ void p2m(const WalkArgs &, bool pred, uint32_t) {
    nm += (uint32_t)__popcll(__ballot(pred));
  }
  __device__ void p2p(const WalkArgs &, bool pred, uint32_t, uint32_t, uint32_t, uint32_t,
                      uint32_t) {
    np += (uint32_t)__popcll(__ballot(pred));
  }
  __device__ void finish(const WalkArgs &) {}
};

struct FillSink {
  uint32_t nm = 0, np = 0;
  uint32_t base_m = 0, base_p = 0;
  __device__ void p2m(const WalkArgs &A, bool pred, uint32_t node) {
    const unsigned long long mask = __ballot(pred);
    if (pred) A.ids[base_m + nm + lanes_below(mask)] = node;
    nm += (uint32_t)__popcll(mask);
  }
  __device__ void p2p(const WalkArgs &A, bool pred, uint32_t node, uint32_t, uint32_t,
                      uint32_t, uint32_t) {
    const unsigned long long mask = __ballot(pred);
    if (pred) A.ids[base_p + np + lanes_below(mask)] = node;
    np += (uint32_t)__popcll(mask);
  }
  __device__ void finish(const WalkArgs &) {}
};

// ---------------------------------------------------------- traversal
// Breadth-first walk of the group's system tree.  The frontier holds the
// cells opened on the level above as {first child, child count} (children
// have consecutive ids); a pass takes eight of them, lane 8 j + k testing
// child k of cell j, so an opened cell is pushed with one store and no
// per-child loop.  The walk starts from the range {root, 1}.  Returns false
// if the frontier overflowed (the group's results are then invalid).
template <bool kRel, class Sink>
__device__ bool traverse(const WalkArgs &A, Sink &sink, uint32_t root,
                         const double lo[3], const double hi[3], double arel) {
  const unsigned lane = lane_id();
  const uint32_t cap = (uint32_t)A.fcap >> 1;     // ranges per half (two words each)
  uint2 *cur = reinterpret_cast<uint2 *>(A.frontier + (size_t)blockIdx.x * 2 * A.fcap);
  uint2 *nxt = cur + cap;
  if (lane == 0) cur[0] = make_uint2(root, 1u);
  __threadfence_block();
  __syncthreads();
  uint32_t fsize = 1;
  const uint32_t kk = lane & 7u;
  while (fsize > 0) {
    uint32_t nf = 0;
    for (uint32_t base = 0; base < fsize; base += 8) {
      // Lanes with no child to test take the first child of their range
      // (lanes past the frontier the first range) and are masked off after
      // the test: the wave runs one path, with no branch around the loads
      // and the test.
      const uint32_t i = base + (lane >> 3);
      const uint2 r = cur[i < fsize ? i : 0u];
      const bool valid = (i < fsize) & (kk < r.y);
      const uint32_t node = r.x + (valid ? kk : 0u);
      const double4 c = A.com[node];
      const uint4 ni = A.ninfo[node];
      const uint32_t f = ni.x, cnt = ni.y, ch = ni.z, nch = ni.w;
      bool acc;
      if constexpr (kRel)
        acc = mac_rel(lo, hi, c, A.rel[2 * (size_t)node], A.rel[2 * (size_t)node + 1], arel);
      else
        acc = mac_accept(lo, hi, c, A.th2);
      acc = acc & valid;
      const bool refused = valid & !acc;
      const bool leaf = refused & (nch == 0u);
      const bool open = refused & (nch > 0u);
      // prefix sum of the particles of refused leaves (most passes have none)
      const uint32_t pc = leaf ? cnt : 0u;
      uint32_t ptot = 0, ppre = 0;
      if (__ballot(leaf) != 0ull) ppre = wave_excl_scan(pc, ptot);
      sink.p2m(A, acc, node);
      sink.p2p(A, leaf, node, f, pc, ppre, ptot);
      const unsigned long long om = __ballot(open);
      const uint32_t no = (uint32_t)__popcll(om);
      if (nf + no > cap) {
        if (lane == 0) set_err(A.err, TG_ERR_FRONTIER);
        return false;
      }
      if (open) nxt[nf + lanes_below(om)] = make_uint2(ch, nch);
      nf += no;
    }
    __threadfence_block();
    __syncthreads();
    uint2 *tmp = cur;
    cur = nxt;
    nxt = tmp;
    fsize = nf;
  }
  sink.finish(A);
  return true;
}

// Work distribution aware of the 8 XCDs (each with its own L2): queue q
// holds the contiguous, hence spatially coherent, active groups
// [q G / 8, (q + 1) G / 8); workgroups are dispatched to the XCDs round
// robin, so block b drains queue b mod 8 first and then helps the others.
struct GroupQueue {
  uint32_t q, tried;
  __device__ explicit GroupQueue(uint32_t home) : q(home & 7u), tried(0) {}
  __device__ uint32_t next(TreeCounters *ctr, uint32_t G) {
    while (tried < 8u) {
      const uint32_t lo = (uint32_t)(((uint64_t)q * G) >> 3);
      const uint32_t hi = (uint32_t)(((uint64_t)(q + 1u) * G) >> 3);
      uint32_t g = 0;
      if (lane_id() == 0) g = atomicAdd(&ctr->xq[kQueueStride * q], 1u);
      // every lane is active here: the first lane is lane 0, and the group
      // index (with all that is loaded from it) is known to be uniform
      g = (uint32_t)__builtin_amdgcn_readfirstlane((int)g);
      if (lo + g < hi) return lo + g;
      q = (q + 1u) & 7u;
      ++tried;
    }
    return G;
  }
};

// ------------------------------------------------------------ force kernel
template <bool kMixed, bool kRel, bool kSpline>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kMixed ? TG_WALK_WAVES_MIXED : TG_WALK_WAVES_FP64)))
void k_walk_forces(const int32_t *__restrict__ gate, WalkArgs A) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  __shared__ uint32_t s_tgt[kMaxGroup];
  __shared__ uint32_t s_m[kMCap];
  __shared__ uint32_t s_q[kQCap];
  __shared__ TileMem<kMixed> tile;
  using Sink = ForceSink<kMixed, kSpline>;
  using R = typename Sink::R;
  constexpr int kMaxT = Sink::kMaxT;
  const unsigned lane = lane_id();
  const uint32_t n_groups = A.ctr->n_active_groups;
  unsigned long long tot_p2p = 0, tot_p2m = 0, tot_t = 0, tot_g = 0;
  GroupQueue Q(blockIdx.x);
  for (;;) {
    const uint32_t gi = Q.next(A.ctr, n_groups);
    if (gi >= n_groups) break;
    const uint32_t g = A.alist[gi];
    const uint4 gr = A.groups[g];
    double lo[3], hi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) { lo[k] = A.abox[6 * (size_t)g + k]; hi[k] = A.abox[6 * (size_t)g + 3 + k]; }
    // compact the active targets of the group
    int nt = 0;
    for (uint32_t c0 = 0; c0 < gr.y; c0 += 64u) {
      const bool act = c0 + lane < gr.y && A.sact[gr.x + c0 + lane];
      const unsigned long long amask = __ballot(act);
      if (act) s_tgt[nt + lanes_below(amask)] = gr.x + c0 + lane;
      nt += __popcll(amask);
    }
    __syncthreads();
    if (nt == 0) continue;   // cannot happen for a listed group; keeps s_tgt reads defined
    // shape: T targets per lane (at least ceil(nt / 64)), lt lane-targets,
    // slices source slices; minimise T / slices.  Ties go to the larger T
    // (fewer tile reads per pair), except that in mixed precision three
    // targets to a lane are taken only where they evaluate strictly fewer
    // pairs: measured on the 1M cusp, ties between two and three ran slower
    // with three.
    int T = (nt + 63) / 64;
    int lt = (nt + T - 1) / T, slices = 64 / lt;
#pragma unroll
    for (int t = 2; t <= kMaxT; ++t) {
      if (t <= T) continue;
      const int l2 = (nt + t - 1) / t, s2 = 64 / l2;
      const bool better = (kMixed && t >= 3) ? t * slices < T * s2 : t * slices <= T * s2;
      if (better) { T = t; lt = l2; slices = s2; }
    }
    Sink S;
    S.s_m = s_m; S.s_q = s_q; S.tile = &tile;
    S.nm = 0; S.nq = 0; S.cells = 0; S.parts = 0;
    S.g0 = gr.x; S.gn = gr.y; S.own0 = S.own1 = 0ull;
    S.s_tgt = s_tgt; S.nt = nt;
    S.T = T; S.lt = lt; S.slices = slices;
    S.tfull = 128 / slices;
    S.F = slices * S.tfull;
    const int j = (int)lane % lt;
    const int sl = (int)lane / lt;
    S.my_s = sl < slices ? sl : 0;           // idle lanes shadow slice 0 (discarded)
    if constexpr (kMixed) {
      S.cgx = 0.5 * (lo[0] + hi[0]);
      S.cgy = 0.5 * (lo[1] + hi[1]);
      S.cgz = 0.5 * (lo[2] + hi[2]);
    } else {
      S.cgx = S.cgy = S.cgz = 0.0;
    }
    S.e2 = (R)A.eps2;
    S.h = (R)A.eps;
    S.ih = (R)(1.0 / A.eps);
#pragma unroll
    for (int k = 0; k < kMaxT; ++k) {
      // lane-target j holds targets j, j + lt, ...; missing ones repeat j
      const int i = j + k * lt;
      const double4 p = A.spart[s_tgt[i < nt ? i : j]];
      S.tx[k] = (R)(p.x - S.cgx); S.ty[k] = (R)(p.y - S.cgy); S.tz[k] = (R)(p.z - S.cgz);
      S.hax[k] = S.hay[k] = S.haz[k] = S.hph[k] = 0.0;
    }
    const bool ok = traverse<kRel>(A, S, A.root_of[gr.w], lo, hi, kRel ? A.arel[g] : 0.0);
    // per-lane totals -> LDS, [k][lane][4]
    double *red = tile.red;
#pragma unroll
    for (int k = 0; k < kMaxT; ++k) {
      double *o = red + 4 * (64 * k + (int)lane);
      o[0] = S.hax[k]; o[1] = S.hay[k]; o[2] = S.haz[k]; o[3] = S.hph[k];
    }
    __syncthreads();
    for (int i = (int)lane; i < nt; i += 64) {
      // target i sits at k = i / lt, lane-target i % lt of every slice; sum
      // the slices in slice order (deterministic)
      const int k = i / lt, jj = i % lt;
      double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
      for (int q = 0; q < slices; ++q) {
        const double *o = red + 4 * (64 * k + q * lt + jj);
        ax += o[0]; ay += o[1]; az += o[2]; ph += o[3];
      }
      const uint32_t r_t = s_tgt[i];
      const double4 p = A.spart[r_t];
      const uint32_t orig = A.perm[r_t];
      const double nanv = __longlong_as_double(0x7ff8000000000000ll);
      double ex = 0.0, ey = 0.0, ez = 0.0, ep = 0.0;
      if (A.ext_seg) {   // SMBH terms, FP64 in both precision modes
        for (int32_t e = A.ext_seg[gr.w]; e < A.ext_seg[gr.w + 1]; ++e) {
          const double es = fmax(A.eps, A.ext_eps[e]);
          const double dx = p.x - A.ext_pos[3 * e], dy = p.y - A.ext_pos[3 * e + 1],
                       dz = p.z - A.ext_pos[3 * e + 2];
          double mD1, mD3;
          if constexpr (kSpline) {
            double p0, p1;
            spline_pair_dp(sqrt(dx * dx + dy * dy + dz * dz), es, p0, p1);
            mD1 = A.ext_mass[e] * p0;
            mD3 = A.ext_mass[e] * p1;
          } else {
            const double r2 = dx * dx + dy * dy + dz * dz + es * es;
            const double D1 = 1.0 / sqrt(r2);
            mD1 = A.ext_mass[e] * D1;
            mD3 = mD1 * D1 * D1;
          }
          ex -= mD3 * dx; ey -= mD3 * dy; ez -= mD3 * dz; ep -= mD1;
        }
      }
      A.acc[3 * (size_t)orig + 0] = ok ? A.G * (ax + ex) : nanv;
      A.acc[3 * (size_t)orig + 1] = ok ? A.G * (ay + ey) : nanv;
      A.acc[3 * (size_t)orig + 2] = ok ? A.G * (az + ez) : nanv;
      if (A.pot) A.pot[orig] = ok ? A.G * (ph + ep) : nanv;
    }
    tot_p2m += S.cells * (unsigned long long)nt;
    tot_p2p += S.parts * (unsigned long long)nt - (unsigned long long)nt;
    tot_t += (unsigned long long)nt;
    tot_g += 1;
    __syncthreads();
  }
  // each workgroup stores its own totals (k_walk_sum adds them up): eight
  // atomics per wave on one line, most of them issued as the queues ran
  // dry, had kept the last waves waiting (the walk took 8% longer)
  if (lane == 0) {
    unsigned long long *w = A.wtot + 4 * (size_t)blockIdx.x;
    w[0] = tot_p2p;
    w[1] = tot_p2m;
    w[2] = tot_t;
    w[3] = tot_g;
  }
}

// The force walk's counts: the sums of the nb workgroups' totals, into the
// last walk's counts and added to the running ones.
constexpr int kSumThreads = 1024;

__global__ __launch_bounds__(kSumThreads) void k_walk_sum(const int32_t *__restrict__ gate, TreeCounters *ctr,
                                                  const unsigned long long *__restrict__ wtot,
                                                  int nb) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  __shared__ unsigned long long part[kSumThreads / 64][4];
  unsigned long long v[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += wtot[4 * (size_t)b + k];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
  const unsigned w = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) part[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x < 4) {
    const unsigned k = threadIdx.x;
    unsigned long long t = 0;
    for (int q = 0; q < kSumThreads / 64; ++q) t += part[q][k];
    (&ctr->n_p2p)[k] = t;
    (&ctr->cum_p2p)[k] += t;
  }
}

// -------------------------------------------------------- list kernels
// pass 0: sizes per active group into wl_count[2 gi + {0,1}];
// pass 1: ids at the offsets wl_off (exclusive scan of wl_count).
template <int kPass, bool kRel>
__global__ __launch_bounds__(64) void k_walk_lists(WalkArgs A) {
  const uint32_t n_groups = A.ctr->n_active_groups;
  GroupQueue Q(blockIdx.x);
  for (;;) {
    const uint32_t gi = Q.next(A.ctr, n_groups);
    if (gi >= n_groups) break;
    const uint32_t g = A.alist[gi];
    const uint4 gr = A.groups[g];
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) { lo[k] = A.abox[6 * (size_t)g + k]; hi[k] = A.abox[6 * (size_t)g + 3 + k]; }
    const double arel = kRel ? A.arel[g] : 0.0;
    if constexpr (kPass == 0) {
      // the fill pass repeats this walk exactly (also up to a frontier
      // overflow), so these counts bound what it writes
      CountSink S;
      traverse<kRel>(A, S, A.root_of[gr.w], lo, hi, arel);
      if (lane_id() == 0) {
        A.wl_count[2 * (size_t)gi] = S.nm;
        A.wl_count[2 * (size_t)gi + 1] = S.np;
      }
    } else {
      FillSink S;
      S.base_m = A.wl_off[2 * (size_t)gi];
      S.base_p = A.wl_off[2 * (size_t)gi + 1];
      traverse<kRel>(A, S, A.root_of[gr.w], lo, hi, arel);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------ active groups
__global__ void k_mark_active(const int32_t *__restrict__ gate, const int32_t *__restrict__ idx,
                              const int32_t *__restrict__ n_act, int64_t n,
                              const uint32_t *__restrict__ rank,
                              uint8_t *__restrict__ sact) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  const int64_t m = idx ? (int64_t)min((int64_t)n_act[0], n) : n;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (idx) {
      const int32_t i = idx[k];
      if (i >= 0 && i < n) sact[rank[i]] = 1;
    } else {
      sact[k] = 1;
    }
  }
}

// Min / max over the 16 lanes of a quarter wave.
__device__ __forceinline__ double qmin(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double qmax(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sixteen lanes per group (a group holds at most kMaxGroup particles):
// flag groups with an active particle and store the box of their active
// particles.  With old accelerations (caller order, reached through perm)
// also the relative test's group threshold (alpha alpha) min |a_old|^2,
// |a|^2 = (ax ax + ay ay) + az az unfused.
__global__ __launch_bounds__(256) void k_group_active(const int32_t *__restrict__ gate, const TreeCounters *ctr,
                                                      const uint4 *__restrict__ groups,
                                                      const uint8_t *__restrict__ sact,
                                                      const double4 *__restrict__ spart,
                                                      const double *__restrict__ acc_old,
                                                      const uint32_t *__restrict__ perm,
                                                      double alpha2,
                                                      uint32_t *__restrict__ aflag,
                                                      uint32_t *__restrict__ acnt,
                                                      double *__restrict__ abox,
                                                      double *__restrict__ arel) {
#pragma clang fp contract(off)
  if (gate && *gate <= 0) return;   // nothing active: skipped
  const uint32_t ng = ctr->n_groups;
  const unsigned q = threadIdx.x & 15u;
  const uint32_t qpb = blockDim.x >> 4;
  for (uint32_t g0 = blockIdx.x * qpb; g0 < ng; g0 += gridDim.x * qpb) {
    const uint32_t g = g0 + (threadIdx.x >> 4);     // quarter-waves stay in step
    const bool live = g < ng;
    const uint4 gr = live ? groups[g] : make_uint4(0, 0, 0, 0);
    double lx = INFINITY, ly = INFINITY, lz = INFINITY;
    double hx = -INFINITY, hy = -INFINITY, hz = -INFINITY;
    double a2min = INFINITY;
    bool any = false;
    uint32_t nact = 0;      // active targets of the quarter-wave's group
#pragma unroll
    for (int r = 0; r < kMaxGroup / 16; ++r) {
      const uint32_t j = q + 16u * r;
      const bool a = j < gr.y && sact[gr.x + j];
      nact += (uint32_t)__popcll((__ballot(a) >> (threadIdx.x & 48u)) & 0xffffull);
      if (a) {
        const double4 p = spart[gr.x + j];
        lx = fmin(lx, p.x); ly = fmin(ly, p.y); lz = fmin(lz, p.z);
        hx = fmax(hx, p.x); hy = fmax(hy, p.y); hz = fmax(hz, p.z);
        any = true;
        if (acc_old) {
          const double *ao = acc_old + 3 * (size_t)perm[gr.x + j];
          const double a2 = dadd(dadd(dmul(ao[0], ao[0]), dmul(ao[1], ao[1])),
                                      dmul(ao[2], ao[2]));
          a2min = fmin(a2min, a2);
        }
      }
    }
    lx = qmin(lx); ly = qmin(ly); lz = qmin(lz);
    hx = qmax(hx); hy = qmax(hy); hz = qmax(hz);
    if (acc_old) a2min = qmin(a2min);
    const unsigned long long m = __ballot(any);
    const unsigned long long mine = (m >> (threadIdx.x & 48u)) & 0xffffull;
    if (live && q == 0) {
      aflag[g] = mine ? 1u : 0u;
      acnt[g] = nact;
      double *b = abox + 6 * (size_t)g;
      b[0] = lx; b[1] = ly; b[2] = lz; b[3] = hx; b[4] = hy; b[5] = hz;
      if (acc_old) arel[g] = mine ? dmul(alpha2, a2min) : 0.0;
    }
  }
}

__global__ void k_compact_groups(const int32_t *__restrict__ gate, const TreeCounters *ctr,
                                 const uint32_t *__restrict__ aflag,
                                 const uint32_t *__restrict__ aidx,
                                 uint32_t *__restrict__ alist) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  const uint32_t ng = ctr->n_groups;
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += gridDim.x * blockDim.x)
    if (aflag[g]) alist[aidx[g]] = g;
}

// The order in which the force walk takes the active groups: each XCD's
// queue range [q G / 8, (q + 1) G / 8) of the compacted list keeps its
// groups (and so its part of the tree), taken by size class, largest class
// first (kSizeClass thresholds on the active targets), and in tree order
// within a class.  The walk's wall time ends with the last groups taken, so
// ending on the small ones shortens the tail in which few waves are left;
// keeping tree order inside a class keeps neighbouring groups, which share
// most of their cells, close in time for the XCD's L2.  One block per range:
// a first sweep counts the classes (coalesced reads), then the range is
// taken in chunks staged in LDS, each thread placing a contiguous run of
// the chunk at offsets from one block scan of its four class counts packed
// in 16-bit fields.  Stable, so deterministic.  No result depends on the
// order in which groups are walked.
constexpr int kSizeClasses = 4;
__device__ __forceinline__ uint32_t size_class(uint32_t nt) {
  return nt >= 48u ? 0u : nt >= 32u ? 1u : nt >= 16u ? 2u : 3u;
}

constexpr int kOrderThreads = 1024;
constexpr uint32_t kOrderItems = 8;                                // per thread and chunk
constexpr uint32_t kOrderChunk = kOrderThreads * kOrderItems;      // < 2^16 per class field
static_assert(kOrderChunk < 65536u, "a chunk's class counts fit 16-bit fields");

// Exclusive block prefix of a 64-bit value (four 16-bit fields; no carries
// between fields since every field's total stays below 2^16).
__device__ __forceinline__ uint64_t block_exclusive_scan64(uint64_t v, uint64_t *sh,
                                                          uint64_t &total) {
  const unsigned lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  uint64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(x, o, 64);
    if (lane >= (unsigned)o) x += y;
  }
  if (lane == 63u) sh[w] = x;
  __syncthreads();
  uint64_t base = 0, tot = 0;
  for (unsigned q = 0; q < blockDim.x / 64u; ++q) {
    const uint64_t t = sh[q];
    base += q < w ? t : 0ull;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return base + x - v;
}

__global__ __launch_bounds__(kOrderThreads) void k_order_groups(const int32_t *__restrict__ gate,
                                                      const TreeCounters *ctr,
                                                      const uint32_t *__restrict__ alist,
                                                      const uint32_t *__restrict__ acnt,
                                                      uint32_t *__restrict__ order) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  __shared__ uint64_t scan_sh[kOrderThreads / 64];
  __shared__ uint32_t s_g[kOrderChunk];
  __shared__ uint8_t s_c[kOrderChunk];
  const uint32_t tid = threadIdx.x;
  const uint32_t G = ctr->n_active_groups;
  const uint32_t lo = (uint32_t)(((uint64_t)blockIdx.x * G) >> 3);
  const uint32_t hi = (uint32_t)(((uint64_t)(blockIdx.x + 1) * G) >> 3);
  // class totals of the range
  uint32_t cnt[kSizeClasses] = {};
  for (uint32_t p0 = lo + tid; p0 < hi; p0 += kOrderThreads * kOrderItems) {
    uint32_t gg[kOrderItems];       // the loads of kOrderItems groups in flight at once
#pragma unroll
    for (uint32_t j = 0; j < kOrderItems; ++j) {
      const uint32_t p = p0 + j * kOrderThreads;
      gg[j] = p < hi ? alist[p] : 0u;
    }
#pragma unroll
    for (uint32_t j = 0; j < kOrderItems; ++j) {
      if (p0 + j * kOrderThreads >= hi) continue;
      const uint32_t k = size_class(acnt[gg[j]]);
#pragma unroll
      for (uint32_t q = 0; q < kSizeClasses; ++q) cnt[q] += k == q ? 1u : 0u;
    }
  }
  uint32_t next[kSizeClasses];      // next free slot of each class
  uint32_t base = lo;
#pragma unroll
  for (int k = 0; k < kSizeClasses; ++k) {
    uint32_t tot;
    block_exclusive_scan(cnt[k], reinterpret_cast<uint32_t *>(scan_sh), tot);
    next[k] = base;
    base += tot;
  }
  for (uint32_t c0 = lo; c0 < hi; c0 += kOrderChunk) {
    const uint32_t m = min(kOrderChunk, hi - c0);
    uint32_t gg[kOrderItems];
#pragma unroll
    for (uint32_t j = 0; j < kOrderItems; ++j) {
      const uint32_t i = tid + j * kOrderThreads;
      gg[j] = i < m ? alist[c0 + i] : 0u;
    }
#pragma unroll
    for (uint32_t j = 0; j < kOrderItems; ++j) {
      const uint32_t i = tid + j * kOrderThreads;
      if (i < m) {
        s_g[i] = gg[j];
        s_c[i] = (uint8_t)size_class(acnt[gg[j]]);
      }
    }
    __syncthreads();
    // this thread's run [kOrderItems tid, kOrderItems (tid + 1)) of the chunk
    const uint32_t r0 = kOrderItems * tid;
    uint64_t mine = 0;
#pragma unroll
    for (uint32_t j = 0; j < kOrderItems; ++j)
      if (r0 + j < m) mine += 1ull << (16u * s_c[r0 + j]);
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan64(mine, scan_sh, tot);
    uint32_t at[kSizeClasses];
#pragma unroll
    for (uint32_t q = 0; q < kSizeClasses; ++q) at[q] = next[q] + (uint32_t)((ex >> (16u * q)) & 0xffffu);
#pragma unroll
    for (uint32_t j = 0; j < kOrderItems; ++j) {
      if (r0 + j >= m) break;
      const uint32_t k = s_c[r0 + j];
      uint32_t dst = at[0];
#pragma unroll
      for (uint32_t q = 1; q < kSizeClasses; ++q) dst = k == q ? at[q] : dst;
#pragma unroll
      for (uint32_t q = 0; q < kSizeClasses; ++q) at[q] += k == q ? 1u : 0u;
      order[dst] = s_g[r0 + j];
    }
#pragma unroll
    for (uint32_t q = 0; q < kSizeClasses; ++q) next[q] += (uint32_t)((tot >> (16u * q)) & 0xffffu);
    __syncthreads();                // the chunk's LDS is read before the next is staged
  }
}

__global__ void k_counts_reset(TreeCounters *ctr) {
  if (threadIdx.x == 0) {
    ctr->cum_p2p = 0;
    ctr->cum_p2m = 0;
    ctr->cum_targets = 0;
    ctr->cum_walked = 0;
  }
}

hipError_t launch_counts_reset(tg_ctx *c) {
  hipLaunchKernelGGL(k_counts_reset, dim3(1), dim3(64), 0, c->stream, c->b.ctr);
  return hipGetLastError();
}

__global__ void k_walk_reset(TreeCounters *ctr) {
  if (threadIdx.x < 8) ctr->xq[kQueueStride * threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    ctr->n_p2p = 0;
    ctr->n_p2m = 0;
    ctr->n_targets = 0;
    ctr->n_walked = 0;
  }
}

hipError_t launch_active_groups(tg_ctx *c, const int32_t *idx,
                                const int32_t *n_act, const double *acc_old,
                                double alpha) {
  Buffers &b = c->b;
  if (c->n == 0) return fill_u32(&b.ctr->n_active_groups, 0u, 1, c->stream);
  hipError_t e = hipSuccess;
  if (idx) {   // without a list every particle is marked active below
    e = fill_u8(b.sact, 0, c->n, c->stream, c->gate);
    if (e != hipSuccess) return e;
  }
  int g = (int)std::min<int64_t>((c->n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_mark_active, dim3(g), dim3(256), 0, c->stream, c->gate, idx,
                     n_act, c->n, b.rank, b.sact);
  hipLaunchKernelGGL(k_group_active, dim3(2048), dim3(256), 0, c->stream, c->gate,
                     b.ctr, b.groups, b.sact, b.spart, acc_old, b.val[0], alpha * alpha,
                     b.aflag, b.acnt, b.abox, b.arel);
  // the group-start scan buffer is free after the build: reuse it
  e = scan_u32(b.aflag, b.gflag, 0u, &b.ctr->n_groups, &b.ctr->n_active_groups,
               b.scan_part, c->stream, c->gate);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_compact_groups, dim3(1024), dim3(256), 0, c->stream, c->gate,
                     b.ctr, b.aflag, b.gflag, b.alist);
  hipLaunchKernelGGL(k_order_groups, dim3(8), dim3(kOrderThreads), 0, c->stream, c->gate, b.ctr,
                     b.alist, b.acnt, b.gorder);
  return hipGetLastError();
}

static WalkArgs make_args(tg_ctx *c, double theta) {
  Buffers &b = c->b;
  WalkArgs A;
  A.ninfo = b.ninfo; A.com = b.com; A.cell = b.cell;
  A.rel = b.rel; A.arel = b.arel;
  A.spart = b.spart; A.root_of = b.root_of;
  A.groups = b.groups; A.alist = b.alist; A.abox = b.abox; A.sact = b.sact;
  A.perm = b.val[0]; A.ctr = b.ctr; A.wtot = b.wtot; A.err = b.err; A.frontier = b.frontier;
  A.fcap = c->cfg.frontier_cap;
  A.th2 = theta * theta;
  A.eps2 = 0.0; A.G = c->cfg.G;
  A.acc = nullptr; A.pot = nullptr;
  A.ext_pos = c->ext_pos; A.ext_mass = c->ext_mass; A.ext_eps = c->ext_eps;
  A.ext_seg = c->n_ext > 0 ? c->b.ext_seg : nullptr;
  A.eps = 0.0;
  A.wl_count = b.wl_count; A.wl_off = b.wl_off; A.ids = nullptr;
  return A;
}

// Walk records of every node: Q = 3S - T I, -T eps^2 (spline: T) and M, in
// the walk's precision, formed once per evaluation instead of once per
// staged cell.
template <class R>
__global__ __launch_bounds__(256) void k_cell_records(const int32_t *__restrict__ gate, const TreeCounters *ctr,
                                                      const double *__restrict__ mom,
                                                      double eps2, int spline, void *cell) {
  if (gate && *gate <= 0) return;   // nothing active: skipped
  using R4 = typename Vec4<R>::T;
  R4 *out = reinterpret_cast<R4 *>(cell);
  const uint32_t nn = ctr->n_nodes;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nn;
       v += gridDim.x * blockDim.x) {
    const double4 m0 = reinterpret_cast<const double4 *>(mom)[2 * (size_t)v];
    const double4 m1 = reinterpret_cast<const double4 *>(mom)[2 * (size_t)v + 1];
    // m0 = {M, Sxx, Syy, Szz}, m1 = {Sxy, Sxz, Syz, -}
    const double T = m0.y + m0.z + m0.w;
    out[2 * (size_t)v] = R4{(R)(3.0 * m0.y - T), (R)(3.0 * m0.z - T), (R)(3.0 * m0.w - T),
                            spline ? (R)T : (R)(-(T * eps2))};
    out[2 * (size_t)v + 1] = R4{(R)(3.0 * m1.x), (R)(3.0 * m1.y), (R)(3.0 * m1.z), (R)m0.x};
  }
}

// Relative-test records of every node: the cell cube enlarged by 20 %
// about its geometric centre and P = (G M) s^2, s the node's opening size
// (the cell side, or its refitted size), every operation rounded separately.
__global__ __launch_bounds__(256) void k_rel_records(const int32_t *__restrict__ gate,
                                                     const TreeCounters *ctr,
                                                     const uint8_t *__restrict__ level,
                                                     const uint32_t *__restrict__ first,
                                                     const uint32_t *__restrict__ nsys,
                                                     const uint64_t *__restrict__ skey,
                                                     const double *__restrict__ cube,
                                                     const double *__restrict__ mom,
                                                     const double *__restrict__ side, double G,
                                                     double4 *__restrict__ rel) {
#pragma clang fp contract(off)
  if (gate && *gate <= 0) return;   // nothing active: skipped
  const uint32_t nn = ctr->n_nodes;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nn;
       v += gridDim.x * blockDim.x) {
    double g[3];
    cell_centre(v, level[v], first, nsys, skey, cube, g);
    const double s = side[v];
    const double h = dmul(0.6, s);
    double lo[3], hi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lo[k] = dsub(g[k], h);
      hi[k] = dadd(g[k], h);
    }
    const double P = dmul(dmul(G, mom[8 * (size_t)v]), dmul(s, s));
    rel[2 * (size_t)v] = make_double4(lo[0], lo[1], lo[2], P);
    rel[2 * (size_t)v + 1] = make_double4(hi[0], hi[1], hi[2], 0.0);
  }
}

static hipError_t launch_rel_records(tg_ctx *c) {
  Buffers &b = c->b;
  hipLaunchKernelGGL(k_rel_records, dim3(1024), dim3(256), 0, c->stream, c->gate, b.ctr,
                     b.level, b.first, b.nsys, b.key[0], b.cube, b.mom, b.side, c->cfg.G, b.rel);
  return hipGetLastError();
}

static int walk_grid(tg_ctx *c) {
  return std::max(1, c->n_cu * c->waves_per_cu);
}

template <bool kRel, bool kSpline>
static void launch_force_kernel(tg_ctx *c, const WalkArgs &A) {
  if (c->cfg.precision == TG_MIXED)
    hipLaunchKernelGGL((k_walk_forces<true, kRel, kSpline>), dim3(walk_grid(c)), dim3(64), 0,
                       c->stream, c->gate, A);
  else
    hipLaunchKernelGGL((k_walk_forces<false, kRel, kSpline>), dim3(walk_grid(c)), dim3(64), 0,
                       c->stream, c->gate, A);
}

hipError_t launch_walk_forces(tg_ctx *c, double eps, double theta,
                              double *acc, double *pot, hipEvent_t before,
                              hipEvent_t after, bool rel) {
  WalkArgs A = make_args(c, theta);
  A.alist = c->b.gorder;      // largest groups first in each XCD's range
  A.eps2 = eps * eps;
  A.eps = eps;
  A.acc = acc;
  A.pot = pot;
  const int spline = c->soft == TG_SOFT_SPLINE ? 1 : 0;
  if (c->cfg.precision == TG_MIXED)
    hipLaunchKernelGGL(k_cell_records<float>, dim3(1024), dim3(256), 0, c->stream, c->gate, c->b.ctr,
                       c->b.mom, A.eps2, spline, (void *)c->b.cell);
  else
    hipLaunchKernelGGL(k_cell_records<double>, dim3(1024), dim3(256), 0, c->stream, c->gate, c->b.ctr,
                       c->b.mom, A.eps2, spline, (void *)c->b.cell);
  if (rel) {
    hipError_t e = launch_rel_records(c);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_walk_reset, dim3(1), dim3(64), 0, c->stream, c->b.ctr);
  if (before) {
    hipError_t e = hipEventRecord(before, c->stream);
    if (e != hipSuccess) return e;
  }
  if (spline) {
    if (rel) launch_force_kernel<true, true>(c, A);
    else launch_force_kernel<false, true>(c, A);
  } else {
    if (rel) launch_force_kernel<true, false>(c, A);
    else launch_force_kernel<false, false>(c, A);
  }
  if (after) {
    hipError_t e = hipEventRecord(after, c->stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_walk_sum, dim3(1), dim3(kSumThreads), 0, c->stream, c->gate, c->b.ctr, c->b.wtot,
                     walk_grid(c));
  return hipGetLastError();
}

hipError_t launch_walk_lists(tg_ctx *c, double theta, int pass, int64_t *info,
                             int64_t cap_groups, uint32_t *ids, int64_t cap_ids,
                             bool rel) {
  (void)info; (void)cap_groups; (void)cap_ids;
  WalkArgs A = make_args(c, theta);
  A.ids = ids;
  if (rel && pass == 0) {
    hipError_t e = launch_rel_records(c);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_walk_reset, dim3(1), dim3(64), 0, c->stream, c->b.ctr);
  const dim3 grid(walk_grid(c));
  if (pass == 0 && !rel)
    hipLaunchKernelGGL((k_walk_lists<0, false>), grid, dim3(64), 0, c->stream, A);
  else if (pass == 0)
    hipLaunchKernelGGL((k_walk_lists<0, true>), grid, dim3(64), 0, c->stream, A);
  else if (!rel)
    hipLaunchKernelGGL((k_walk_lists<1, false>), grid, dim3(64), 0, c->stream, A);
  else
    hipLaunchKernelGGL((k_walk_lists<1, true>), grid, dim3(64), 0, c->stream, A);
  return hipGetLastError();
}

}  // namespace tg
