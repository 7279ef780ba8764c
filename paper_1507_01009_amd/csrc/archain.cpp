// Algorithmic-regularization chain integrator (host, FP64): the few-body
// subsystem around the SMBH that the hybrid method integrates apart from the
// tree (Sec. 2), in the chain's centre-of-mass frame.
//
// Method (Mikkola & Tanikawa 1999, MNRAS 310, 745; Preto & Tremaine 1999,
// AJ 118, 2532; Mikkola & Aarseth 2002, CeMDA 84, 343): with the kinetic
// energy T, the (positive) potential energy U = sum_{i<j} G m_i m_j / r_ij
// and the binding energy B = U - T carried as a variable, the logarithmic
// Hamiltonian splits into two exactly solvable flows in a fictitious time s:
//   drift:  dt/ds = 1 / (T + B),  x += v dt,  t += dt       (v fixed)
//   kick:   dt/ds = 1 / U,        v += (a + f) dt,           (x, t fixed)
//           B -= dt sum_i m_i f_i . (v_old + v_new) / 2
// with a the Newtonian accelerations of the members and f an external
// perturbation.  A leapfrog D(h/2) [K(h) D(h)]^(n-1) K(h) D(h/2) follows
// two-body orbits exactly up to a time error, also through collisions, and
// its error is even in h, so a Bulirsch-Stoer extrapolation in h^2 over the
// substep counts n = 2, 4, 6, ... brings each step to the tolerance.  The
// last step before the target time is found by a secant search on its
// length, from a first trial interpolated with the time derivatives at both
// ends; a last gap much shorter than every pair's crossing time is covered
// in physical time by one drift-kick-drift.
//
// Coordinates: the chain of inter-particle vectors (Mikkola & Aarseth
// 1990, CeMDA 47, 375; 1993, CeMDA 57, 439).  The members are ordered along
// a chain c[0..n-1] and the integrated variables are X_k = x_c[k+1] -
// x_c[k], W_k = v_c[k+1] - v_c[k] (k < n - 1): a drift moves X_k by W_k dt
// and a kick moves W_k by (A_c[k+1] - A_c[k]) dt.  Pairs one or two links
// apart take their separation from X_k (or X_k + X_k+1), so a close pair
// keeps its digits however far it is from the centre of mass; the other
// pairs and the perturbers use centre-of-mass coordinates rebuilt from the
// chain.  The chain is built by force (Sec. 2: members sorted by their
// gravitational forces, not by distance): the pair with the largest
// m_i m_j / r^2 first, then at either end the member that end pulls
// hardest, until all are in.  Before every extrapolated step the chain is
// built again and, if it changed, the new vectors are sums of the old ones
// along the old chain.
//
// Perturbers: point masses moved to first order, y_p(t) = y_p + w_p (t - t0),
// relative to the chain's centre of mass; the members feel their tidal part,
// f_i - (1/M) sum_j m_j f_j, so the frame stays centred (the centre of mass
// itself is the tree's chain particle).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "tg_internal.h"

namespace {

struct Chain {
  int n = 0;
  const double *m = nullptr;
  double G = 1.0, M = 0.0;
  // perturbers
  int np = 0;
  const double *py = nullptr, *pw = nullptr, *pm = nullptr;
  double t0 = 0.0;
  // the chain: members in chain order, and each member's place in it
  std::vector<int> ord, pos;
};

// State vector: chain vectors X [3(n-1)], their velocities W [3(n-1)], t, B.
struct Y {
  std::vector<double> d;
  double *X() { return d.data(); }
  const double *X() const { return d.data(); }
  double *W(int n) { return d.data() + 3 * (n - 1); }
  const double *W(int n) const { return d.data() + 3 * (n - 1); }
  double &t(int n) { return d[6 * (n - 1)]; }
  double &B(int n) { return d[6 * (n - 1) + 1]; }
};

// Centre-of-mass coordinates [n][3] (member order) from chain vectors:
// x_c[0] = -(1/M) sum_k S_k X_k with S_k the mass after link k, then
// x_c[k+1] = x_c[k] + X_k.
void to_com(const Chain &c, const double *X, double *x) {
  double s[3] = {0.0, 0.0, 0.0}, before = 0.0;
  for (int k = 0; k < c.n - 1; ++k) {
    before += c.m[c.ord[k]];
    const double S = c.M - before;
    for (int d = 0; d < 3; ++d) s[d] += S * X[3 * k + d];
  }
  double *x0 = x + 3 * c.ord[0];
  for (int d = 0; d < 3; ++d) x0[d] = -s[d] / c.M;
  for (int k = 0; k < c.n - 1; ++k) {
    const double *a = x + 3 * c.ord[k];
    double *b = x + 3 * c.ord[k + 1];
    for (int d = 0; d < 3; ++d) b[d] = a[d] + X[3 * k + d];
  }
}

// Chain vectors of the order in c from centre-of-mass coordinates.
void from_com(const Chain &c, const double *x, double *X) {
  for (int k = 0; k < c.n - 1; ++k)
    for (int d = 0; d < 3; ++d) X[3 * k + d] = x[3 * c.ord[k + 1] + d] - x[3 * c.ord[k] + d];
}

double kinetic_com(const Chain &c, const double *v) {
  double T = 0.0;
  for (int i = 0; i < c.n; ++i)
    T += 0.5 * c.m[i] * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
  return T;
}

// The chain by force over centre-of-mass coordinates x: the strongest pair
// (largest m_i m_j / r^2; ties to the lower indices), then repeatedly the
// member outside the chain pulled hardest by either end, attached to that
// end (ties: the tail, then the lower index).
void build_order(Chain &c, const double *x) {
  const int n = c.n;
  std::vector<double> F((size_t)n * n, 0.0);
  int bi = 0, bj = 1;
  double best = -1.0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double r2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double q = x[3 * j + d] - x[3 * i + d];
        r2 += q * q;
      }
      const double f = c.m[i] * c.m[j] / r2;
      F[(size_t)i * n + j] = F[(size_t)j * n + i] = f;
      if (f > best) { best = f; bi = i; bj = j; }
    }
  std::vector<int> chain{bi, bj};
  std::vector<char> in(n, 0);
  in[bi] = in[bj] = 1;
  while ((int)chain.size() < n) {
    const int head = chain.front(), tail = chain.back();
    int k_best = -1;
    bool at_tail = true;
    double f_best = -1.0;
    for (int k = 0; k < n; ++k) {
      if (in[k]) continue;
      const double ft = F[(size_t)k * n + tail], fh = F[(size_t)k * n + head];
      if (ft > f_best) { f_best = ft; k_best = k; at_tail = true; }
      if (fh > f_best) { f_best = fh; k_best = k; at_tail = false; }
    }
    in[k_best] = 1;
    if (at_tail) chain.push_back(k_best);
    else chain.insert(chain.begin(), k_best);
  }
  c.ord = chain;
  c.pos.assign(n, 0);
  for (int k = 0; k < n; ++k) c.pos[c.ord[k]] = k;
}

// Rebuild the chain by force at the state y (chain vectors of c.ord); if
// the order changes, the new vectors are sums of the old ones along the
// old chain (no round trip through centre-of-mass coordinates).
void rechain(Chain &c, Y &y) {
  const int n = c.n;
  if (n < 3) return;
  std::vector<double> x(3 * n);
  to_com(c, y.X(), x.data());
  const std::vector<int> old_pos = c.pos;
  build_order(c, x.data());
  bool same = true;
  for (int i = 0; i < n; ++i) same = same && (c.pos[i] == old_pos[i]);
  if (same) return;
  const std::vector<double> X0(y.X(), y.X() + 3 * (n - 1)), W0(y.W(n), y.W(n) + 3 * (n - 1));
  for (int k = 0; k < n - 1; ++k) {
    const int pa = old_pos[c.ord[k]], pb = old_pos[c.ord[k + 1]];
    const int lo = std::min(pa, pb), hi = std::max(pa, pb);
    const double sg = pa < pb ? 1.0 : -1.0;
    for (int d = 0; d < 3; ++d) {
      double sx = 0.0, sw = 0.0;
      for (int l = lo; l < hi; ++l) {
        sx += X0[3 * l + d];
        sw += W0[3 * l + d];
      }
      y.X()[3 * k + d] = sg * sx;
      y.W(n)[3 * k + d] = sg * sw;
    }
  }
}

// Scratch of one thread: accelerations a (members' own) and f (perturbers'
// tidal part), [n][3]; centre-of-mass coordinates xc, vc; structure-of-
// arrays copies of the member coordinates, masses and chain places and of
// the perturbers, padded to whole vectors.
struct Work {
  std::vector<double> a, f, xc, vc;
  std::vector<double> X, Yc, Z, Mw, P;   // members
  std::vector<double> PX, PY, PZ, PM;    // perturbers at the kick's time
  explicit Work(int n = 0) : a(3 * n), f(3 * n), xc(3 * n), vc(3 * n) {}
};

// The pair sums run over 8-wide vectors (clang vector extensions); the
// same source is compiled for AVX-512, AVX2 + FMA and the baseline, and the
// widest one the CPU has is taken once per process, so every call (every
// thread) rounds the same way on a given machine.
using v8 = double __attribute__((ext_vector_type(8)));
using l8 = long long __attribute__((ext_vector_type(8)));
constexpr int kV = 8;

int padded(int n) { return (n + kV - 1) / kV * kV; }

__attribute__((always_inline)) inline v8 load8(const double *p) {
  v8 r;
  std::memcpy(&r, p, sizeof(r));
  return r;
}
// 1/sqrt(x) for positive normal x, eight lanes: the bit-level first guess
// of Lomont (2003; within 3.5%) and four Newton steps y += y (1 - x y^2) / 2,
// which end within two units in the last place.  The same arithmetic in
// every clone, and several times cheaper than a square root and a division.
__attribute__((always_inline)) inline v8 inv_sqrt(v8 x) {
  const l8 bits = (l8)x;
  v8 y = (v8)((long long)0x5FE6EB50C7B537A9ll - (bits >> 1));
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const v8 e = 1.0 - (x * y) * y;
    y = y + y * (0.5 * e);
  }
  return y;
}
// 1.0 where a comparison's lane is true (all bits set), else 0.0: the
// bits of 1.0 masked, with no integer-to-double conversion (which the
// AVX-512F clone would do lane by lane)
template <class M>
__attribute__((always_inline)) inline v8 select01(M m) {
  const v8 one = 1.0;
  return (v8)((l8)m & (l8)one);
}
__attribute__((always_inline)) inline double hsum(v8 v) {
  return ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
}

// Row i of the members' sums over the pairs more than two links apart in
// the chain: a_i = sum_j m_j (x_j - x_i) / r^3 and u_i = sum_j m_j / r.
// Other lanes (near pairs, j = i, padding) get a mass of zero and r^2 + 1,
// so no lane divides by zero.
__attribute__((always_inline)) inline void internal_row(const Work &w, int n, int i,
                                                        double *ai, double &ui) {
  const double xi = w.X[i], yi = w.Yc[i], zi = w.Z[i], pi = w.P[i];
  v8 ax = 0.0, ay = 0.0, az = 0.0, u = 0.0;
  const l8 lane = {0, 1, 2, 3, 4, 5, 6, 7};
  for (int j = 0; j < padded(n); j += kV) {
    const l8 jj = lane + (long long)j;
    const v8 dp = load8(&w.P[j]) - pi;
    const v8 live = select01(((dp > 2.5) | (dp < -2.5)) & (jj < (long long)n));
    const v8 dx = load8(&w.X[j]) - xi, dy = load8(&w.Yc[j]) - yi, dz = load8(&w.Z[j]) - zi;
    const v8 r2 = dx * dx + dy * dy + dz * dz + (1.0 - live);
    const v8 ir = inv_sqrt(r2);
    const v8 mj = load8(&w.Mw[j]) * live;
    const v8 mir = mj * ir;
    const v8 g = mir * (ir * ir);
    ax += g * dx;
    ay += g * dy;
    az += g * dz;
    u += mir;
  }
  ai[0] = hsum(ax);
  ai[1] = hsum(ay);
  ai[2] = hsum(az);
  ui = hsum(u);
}

// Member i's sum over the perturbers (positions already at the kick's time;
// padding: mass zero, r^2 + 1).
__attribute__((always_inline)) inline void external_row(const Work &w, int np, double xi,
                                                        double yi, double zi, double *fi) {
  v8 fx = 0.0, fy = 0.0, fz = 0.0;
  const l8 lane = {0, 1, 2, 3, 4, 5, 6, 7};
  for (int p = 0; p < padded(np); p += kV) {
    const v8 live = select01(lane + (long long)p < (long long)np);
    const v8 dx = load8(&w.PX[p]) - xi, dy = load8(&w.PY[p]) - yi, dz = load8(&w.PZ[p]) - zi;
    const v8 r2 = dx * dx + dy * dy + dz * dz + (1.0 - live);
    const v8 ir = inv_sqrt(r2);
    const v8 g = load8(&w.PM[p]) * (ir * (ir * ir));
    fx += g * dx;
    fy += g * dy;
    fz += g * dz;
  }
  fi[0] = hsum(fx);
  fi[1] = hsum(fy);
  fi[2] = hsum(fz);
}

#define TG_PAIR_SUMS(SUFFIX, ATTR)                                                      \
  ATTR double internal_rows##SUFFIX(const Work &w, int n, double *a) {                  \
    double U2 = 0.0;                                                                    \
    for (int i = 0; i < n; ++i) {                                                       \
      double ui;                                                                        \
      internal_row(w, n, i, &a[3 * i], ui);                                             \
      U2 += w.Mw[i] * ui;                                                               \
    }                                                                                   \
    return U2;                                                                          \
  }                                                                                     \
  ATTR void external_rows##SUFFIX(const Work &w, int n, int np, const double *x,        \
                                  double *f) {                                          \
    for (int i = 0; i < n; ++i)                                                         \
      external_row(w, np, x[3 * i], x[3 * i + 1], x[3 * i + 2], &f[3 * i]);             \
  }
// (the sources are compiled as HIP, whose device pass also parses this
// host-only file: CPU targets and CPU feature tests exist in the host pass)
#if defined(__HIP_DEVICE_COMPILE__)
#define TG_CPU_TARGET(x)
#else
#define TG_CPU_TARGET(x) __attribute__((target(x)))
#endif
TG_PAIR_SUMS(_base, )
TG_PAIR_SUMS(_avx2, TG_CPU_TARGET("avx2,fma"))
TG_PAIR_SUMS(_avx512, TG_CPU_TARGET("avx512f"))
#undef TG_PAIR_SUMS
#undef TG_CPU_TARGET

enum class Isa { base, avx2, avx512 };
Isa isa() {
#if defined(__HIP_DEVICE_COMPILE__)
  return Isa::base;
#else
  // TG_ARCHAIN_ISA = base or avx2 takes a narrower clone than the CPU
  // allows (never a wider one)
  static const Isa k = [] {
    __builtin_cpu_init();
    const char *e = std::getenv("TG_ARCHAIN_ISA");
    const std::string want = e ? e : "";
    const bool a512 = __builtin_cpu_supports("avx512f");
    const bool a2 = __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
    if (want == "base") return Isa::base;
    if (a512 && want != "avx2") return Isa::avx512;
    if (a2) return Isa::avx2;
    return Isa::base;
  }();
  return k;
#endif
}

// One pair from its separation r = x_j - x_i: a_i += m_j r / |r|^3,
// a_j -= m_i r / |r|^3; returns 2 m_i m_j / |r| (the pair counted from both
// ends, as the rows count it).
inline double near_pair(const Chain &c, int i, int j, const double r[3], double *a) {
  const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  const double ir = 1.0 / std::sqrt(r2), g = ir * ir * ir;
  for (int d = 0; d < 3; ++d) {
    a[3 * i + d] += c.m[j] * g * r[d];
    a[3 * j + d] -= c.m[i] * g * r[d];
  }
  return 2.0 * c.m[i] * c.m[j] * ir;
}

// Newtonian accelerations of the members (into w.a, member order) and the
// centre-of-mass positions (w.xc); returns U.
double internal(const Chain &c, const double *X, Work &w) {
  const int n = c.n, np8 = padded(n);
  w.xc.resize(3 * n);
  to_com(c, X, w.xc.data());
  w.X.assign(np8, 0.0);
  w.Yc.assign(np8, 0.0);
  w.Z.assign(np8, 0.0);
  w.Mw.assign(np8, 0.0);
  w.P.assign(np8, -1e9);
  for (int i = 0; i < n; ++i) {
    w.X[i] = w.xc[3 * i];
    w.Yc[i] = w.xc[3 * i + 1];
    w.Z[i] = w.xc[3 * i + 2];
    w.Mw[i] = c.m[i];
    w.P[i] = (double)c.pos[i];
  }
  w.a.resize(3 * n);
  double U2;
  switch (isa()) {
    case Isa::avx512: U2 = internal_rows_avx512(w, n, w.a.data()); break;
    case Isa::avx2: U2 = internal_rows_avx2(w, n, w.a.data()); break;
    default: U2 = internal_rows_base(w, n, w.a.data()); break;
  }
  // pairs one and two links apart, from the chain vectors
  for (int k = 0; k + 1 < n; ++k) {
    U2 += near_pair(c, c.ord[k], c.ord[k + 1], &X[3 * k], w.a.data());
    if (k + 2 < n) {
      const double r[3] = {X[3 * k] + X[3 * k + 3], X[3 * k + 1] + X[3 * k + 4],
                           X[3 * k + 2] + X[3 * k + 5]};
      U2 += near_pair(c, c.ord[k], c.ord[k + 2], r, w.a.data());
    }
  }
  for (double &q : w.a) q *= c.G;
  return 0.5 * c.G * U2;
}

// Tidal part of the perturbers' accelerations at time t on the members at
// centre-of-mass positions x (into w.f).
void external(const Chain &c, const double *x, double t, Work &w) {
  w.f.resize(3 * c.n);
  double *f = w.f.data();
  std::fill(f, f + 3 * c.n, 0.0);
  if (c.np == 0) return;
  const double dt = t - c.t0;
  const int np8 = padded(c.np);
  w.PX.assign(np8, 0.0);
  w.PY.assign(np8, 0.0);
  w.PZ.assign(np8, 0.0);
  w.PM.assign(np8, 0.0);
  for (int p = 0; p < c.np; ++p) {
    w.PX[p] = c.py[3 * p] + c.pw[3 * p] * dt;
    w.PY[p] = c.py[3 * p + 1] + c.pw[3 * p + 1] * dt;
    w.PZ[p] = c.py[3 * p + 2] + c.pw[3 * p + 2] * dt;
    w.PM[p] = c.G * c.pm[p];
  }
  switch (isa()) {
    case Isa::avx512: external_rows_avx512(w, c.n, c.np, x, f); break;
    case Isa::avx2: external_rows_avx2(w, c.n, c.np, x, f); break;
    default: external_rows_base(w, c.n, c.np, x, f); break;
  }
  double mx = 0.0, my = 0.0, mz = 0.0;
  for (int i = 0; i < c.n; ++i) {
    mx += c.m[i] * f[3 * i]; my += c.m[i] * f[3 * i + 1]; mz += c.m[i] * f[3 * i + 2];
  }
  mx /= c.M; my /= c.M; mz /= c.M;
  for (int i = 0; i < c.n; ++i) { f[3 * i] -= mx; f[3 * i + 1] -= my; f[3 * i + 2] -= mz; }
}

double kinetic(const Chain &c, const double *W, Work &w) {
  w.vc.resize(3 * c.n);
  to_com(c, W, w.vc.data());
  return kinetic_com(c, w.vc.data());
}

// x += v dt and t += dt over a physical time dt
void drift_t(const Chain &c, Y &y, double dt) {
  const int n = c.n;
  double *X = y.X();
  const double *W = y.W(n);
  for (int k = 0; k < 3 * (n - 1); ++k) X[k] += W[k] * dt;
  y.t(n) += dt;
}

void drift(const Chain &c, Y &y, double h, Work &w) {
  drift_t(c, y, h / (kinetic(c, y.W(c.n), w) + y.B(c.n)));
}

// v_i changes by (a_i + f_i) dt, so W_k by the difference along link k;
// B loses the perturbers' work at the mean velocity of the kick.
// The kick over a physical time dt; w.a and w.xc hold the members'
// accelerations and centre-of-mass positions at y (from internal).
void kick_t(const Chain &c, Y &y, double dt, Work &w) {
  const int n = c.n;
  external(c, w.xc.data(), y.t(n), w);
  w.vc.resize(3 * n);
  to_com(c, y.W(n), w.vc.data());
  const std::vector<double> &a = w.a, &f = w.f;
  double work = 0.0;
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      const double dv = (a[3 * i + d] + f[3 * i + d]) * dt;
      work += c.m[i] * f[3 * i + d] * (w.vc[3 * i + d] + 0.5 * dv);
    }
  double *W = y.W(n);
  for (int k = 0; k + 1 < n; ++k) {
    const int i = c.ord[k], j = c.ord[k + 1];
    for (int d = 0; d < 3; ++d)
      W[3 * k + d] += ((a[3 * j + d] + f[3 * j + d]) - (a[3 * i + d] + f[3 * i + d])) * dt;
  }
  y.B(n) -= work * dt;
}

void kick(const Chain &c, Y &y, double h, Work &w) {
  const double U = internal(c, y.X(), w);
  kick_t(c, y, h / U, w);
}

// Shortest |X_k| / |W_k| over the chain vectors: the time scale of the
// closest pairs.
double crossing(const Chain &c, const Y &y) {
  const int n = c.n;
  const double *X = y.X(), *W = &y.d[3 * (n - 1)];
  double best = 1e300;
  for (int k = 0; k + 1 < n; ++k) {
    const double x2 = X[3 * k] * X[3 * k] + X[3 * k + 1] * X[3 * k + 1] + X[3 * k + 2] * X[3 * k + 2];
    const double w2 = W[3 * k] * W[3 * k] + W[3 * k + 1] * W[3 * k + 1] + W[3 * k + 2] * W[3 * k + 2];
    if (w2 > 0.0) best = std::min(best, std::sqrt(x2 / w2));
  }
  return best;
}

// A remaining gap of physical time, short against every pair's crossing
// time, in one second-order drift-kick-drift.
void close_gap(const Chain &c, Y &y, double gap, Work &w) {
  drift_t(c, y, 0.5 * gap);
  internal(c, y.X(), w);
  kick_t(c, y, gap, w);
  drift_t(c, y, 0.5 * gap);
}

Y leapfrog(const Chain &c, const Y &y0, double H, int nsub, Work &w) {
  Y y = y0;
  const double h = H / nsub;
  drift(c, y, 0.5 * h, w);
  for (int k = 0; k < nsub; ++k) {
    kick(c, y, h, w);
    drift(c, y, k == nsub - 1 ? 0.5 * h : h, w);
  }
  return y;
}

constexpr int kCols = 10;
constexpr int kSeq[kCols] = {2, 4, 6, 8, 10, 12, 14, 16, 20, 24};

// Host threads for the extrapolation columns: one (no threads) for small
// chains, where starting threads costs more than a column; otherwise up to
// six, fewer with TG_ARCHAIN_THREADS.  The first batch holds the columns the
// previous step of the same call converged with (at least three, which the
// first convergence test needs), so the batch's longest column sets the time.
int column_threads(const Chain &c) {
  static const int hw = [] {
    const char *e = std::getenv("TG_ARCHAIN_THREADS");
    int t = e ? std::atoi(e) : (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(t, 6));
  }();
  const long pairs = (long)c.n * (c.n + c.np);
  return pairs < 4096 ? 1 : hw;
}

// Host threads started once (at the first threaded batch) that take the
// columns of a batch; the calling thread takes columns too.  One batch runs
// at a time in a process; the workers are never joined (they wait on a
// condition variable until the process ends).
class ColumnPool {
 public:
  static ColumnPool &get(int workers) {
    static ColumnPool *p = new ColumnPool(workers);
    return *p;
  }
  // f(q) for every q in [lo, hi); returns when all have finished.  f must
  // not throw.
  void run(int lo, int hi, const std::function<void(int)> &f) {
    std::lock_guard<std::mutex> one(batch_mu_);
    {
      std::lock_guard<std::mutex> lk(mu_);
      f_ = &f;
      next_ = lo;
      end_ = hi;
      ++gen_;
    }
    cv_.notify_all();
    work();
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return next_ >= end_ && busy_ == 0; });
    f_ = nullptr;
  }

 private:
  explicit ColumnPool(int workers) {
    for (int i = 0; i < workers; ++i) {
      try {
        std::thread(&ColumnPool::loop, this).detach();
      } catch (const std::system_error &) {
        break;   // fewer workers; the caller takes what is left
      }
    }
  }
  void work() {
    for (;;) {
      const std::function<void(int)> *f;
      int q;
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (!f_ || next_ >= end_) return;
        f = f_;
        q = next_++;
        ++busy_;
      }
      (*f)(q);
      {
        std::lock_guard<std::mutex> lk(mu_);
        --busy_;
      }
      done_cv_.notify_all();
    }
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return gen_ != seen; });
        seen = gen_;
      }
      work();
    }
  }
  std::mutex batch_mu_, mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)> *f_ = nullptr;
  int next_ = 0, end_ = 0, busy_ = 0;
  uint64_t gen_ = 0;
};

// One extrapolated step of fictitious length H.  Returns the column at which
// it converged (or -1) and the result in out.
int bs_step(const Chain &c, const Y &y0, double H, double tol, Y &out, Work &w,
            int first = 3) {
  const int n = c.n, nv = 3 * (n - 1), dim = 2 * nv + 2;
  std::vector<std::vector<double>> T(kCols, std::vector<double>(dim));
  // error scales: every chain vector and its velocity relative to their
  // own lengths (a close pair is resolved on its own scale), with floors at
  // 1e-12 of the longest vector and 1e-6 of the fastest or of the system's
  // circular speed; the step's time; |B|
  std::vector<double> sc(dim, 0.0);
  double xmax = 0.0, vmax = 0.0;
  for (int k = 0; k < n - 1; ++k) {
    const double *X = &y0.d[3 * k], *W = &y0.d[nv + 3 * k];
    const double lx = std::sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    const double lw = std::sqrt(W[0] * W[0] + W[1] * W[1] + W[2] * W[2]);
    for (int d = 0; d < 3; ++d) {
      sc[3 * k + d] = lx;
      sc[nv + 3 * k + d] = lw;
    }
    xmax = std::max(xmax, lx);
    vmax = std::max(vmax, lw);
  }
  const double vfloor = 1e-6 * std::max(vmax, std::sqrt(c.G * c.M / xmax));
  for (int q = 0; q < nv; ++q) {
    sc[q] = std::max(sc[q], 1e-12 * xmax);
    sc[nv + q] = std::max(sc[nv + q], vfloor);
  }
  // The columns' leapfrogs are independent: with a large chain they are
  // computed a batch at a time on host threads (each with its own scratch),
  // then extrapolated in order exactly as one at a time.
  const int par = column_threads(c);
  std::vector<Y> col(kCols);
  int ready = 0;
  for (int k = 0; k < kCols; ++k) {
    if (k == ready) {
      // first the columns the last step needed (at least the three of the
      // first convergence test), then pairs
      const int want = k == 0 ? std::max(3, first) : 2;
      const int hi = std::min(kCols, k + std::min(par, want));
      if (hi - k > 1) {
        // a column that fails on a pool thread is computed again on this
        // one; the result is the same on any thread
        std::vector<char> done(kCols, 0);
        const std::function<void(int)> job = [&](int q) {
          try {
            thread_local Work tw;
            col[q] = leapfrog(c, y0, H, kSeq[q], tw);
            done[q] = 1;
          } catch (...) {
          }
        };
        ColumnPool::get(par - 1).run(k, hi, job);
        for (int q = k; q < hi; ++q)
          if (!done[q]) col[q] = leapfrog(c, y0, H, kSeq[q], w);
      } else {
        col[k] = leapfrog(c, y0, H, kSeq[k], w);
      }
      ready = hi;
    }
    T[k] = col[k].d;
    for (int j = k - 1; j >= 0; --j) {
      const double r = (double)kSeq[k] / kSeq[j];
      const double den = r * r - 1.0;
      for (int q = 0; q < dim; ++q) T[j][q] = T[j + 1][q] + (T[j + 1][q] - T[j][q]) / den;
    }
    if (k >= 2) {
      // T[0] holds the newest extrapolation, T[1] the previous one
      double err = 0.0;
      const double ts = std::fabs(T[0][2 * nv] - y0.d[2 * nv]) + 1e-300;
      for (int q = 0; q < dim; ++q) {
        double s;
        if (q < 2 * nv) s = sc[q];
        else if (q == 2 * nv) s = ts;
        else s = std::fabs(y0.d[2 * nv + 1]);
        err = std::max(err, std::fabs(T[0][q] - T[1][q]) / (s + 1e-300));
      }
      if (err <= tol) {
        out.d = T[0];
        return k;
      }
    }
  }
  return -1;
}

// The chain and the chain vectors of the caller's state: the kept chain
// state when it is valid, else the chain by force over x, v.  Returns false
// if a kept chain is not a permutation of the members.
bool load_state(const tg_archain *s, Chain &c, Y &y) {
  const int n = s->n;
  y.d.assign(6 * (n - 1) + 2, 0.0);
  if (s->chain_valid && s->chain && s->cx && s->cv) {
    std::vector<char> seen(n, 0);
    for (int k = 0; k < n; ++k) {
      const int i = s->chain[k];
      if (i < 0 || i >= n || seen[i]) return false;
      seen[i] = 1;
    }
    c.ord.assign(s->chain, s->chain + n);
    c.pos.assign(n, 0);
    for (int k = 0; k < n; ++k) c.pos[c.ord[k]] = k;
    std::memcpy(y.X(), s->cx, sizeof(double) * 3 * (n - 1));
    std::memcpy(y.W(n), s->cv, sizeof(double) * 3 * (n - 1));
  } else {
    build_order(c, s->x);
    from_com(c, s->x, y.X());
    from_com(c, s->v, y.W(n));
  }
  y.t(n) = s->t;
  y.B(n) = s->B;
  return true;
}

// x, v (centre-of-mass frame) from the chain state, and the chain state
// itself where the caller keeps it.
void store_state(const Chain &c, const Y &y, tg_archain *s) {
  const int n = s->n;
  to_com(c, y.X(), s->x);
  to_com(c, y.W(n), s->v);
  if (s->chain && s->cx && s->cv) {
    std::copy(c.ord.begin(), c.ord.end(), s->chain);
    std::memcpy(s->cx, y.X(), sizeof(double) * 3 * (n - 1));
    std::memcpy(s->cv, y.W(n), sizeof(double) * 3 * (n - 1));
    s->chain_valid = 1;
  }
}

}  // namespace

using namespace tg;

extern "C" {

tg_status tg_archain_init(tg_archain *s, double G) try {
  if (!s || !s->x || !s->v || !s->m) return fail(TG_EINVAL, "tg_archain_init: NULL argument");
  if (s->n < 2 || s->n > kMaxChain) return fail(TG_EINVAL, "tg_archain_init: n must be in 2..256");
  if (!(G > 0.0)) return fail(TG_EINVAL, "tg_archain_init: G must be positive");
  Chain c;
  c.n = s->n; c.m = s->m; c.G = G;
  Work w(s->n);
  for (int i = 0; i < s->n; ++i) {
    if (!(s->m[i] > 0.0)) return fail(TG_EINVAL, "tg_archain_init: masses must be positive");
    c.M += s->m[i];
  }
  for (int i = 0; i < 3 * s->n; ++i)
    if (!std::isfinite(s->x[i]) || !std::isfinite(s->v[i]))
      return fail(TG_EINVAL, "tg_archain_init: non-finite coordinates");
  Y y;
  if (!load_state(s, c, y)) return fail(TG_EINVAL, "tg_archain_init: chain is not a permutation");
  const double U = internal(c, y.X(), w);
  if (!std::isfinite(U)) return fail(TG_EINVAL, "tg_archain_init: coincident members");
  s->B = U - kinetic(c, y.W(s->n), w);
  if (!(s->ds > 0.0)) {
    // a first step of about a hundredth of the fastest pair's dynamical time
    double tmin = INFINITY;
    for (int i = 0; i < s->n; ++i)
      for (int j = i + 1; j < s->n; ++j) {
        double r2 = 0.0;
        for (int k = 0; k < 3; ++k) {
          const double d = w.xc[3 * j + k] - w.xc[3 * i + k];
          r2 += d * d;
        }
        const double r = std::sqrt(r2);
        tmin = std::min(tmin, std::sqrt(r * r * r / (G * (s->m[i] + s->m[j]))));
      }
    s->ds = 0.01 * tmin * U;
  }
  y.B(s->n) = s->B;
  store_state(c, y, s);
  return TG_OK;
} TG_HOST_CATCH("tg_archain_init")

tg_status tg_archain_advance(tg_archain *s, double G, double dt, double tol,
                             const tg_archain_perturbers *p, int64_t *steps_out) try {
  if (!s || !s->x || !s->v || !s->m) return fail(TG_EINVAL, "tg_archain_advance: NULL argument");
  if (s->n < 2 || s->n > kMaxChain) return fail(TG_EINVAL, "tg_archain_advance: n must be in 2..256");
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(TG_EINVAL, "tg_archain_advance: dt must be >= 0");
  if (!(tol > 0.0) || !(s->ds > 0.0)) return fail(TG_EINVAL, "tg_archain_advance: tol and ds must be > 0");
  if (p && p->np > 0 && (!p->x || !p->v || !p->m))
    return fail(TG_EINVAL, "tg_archain_advance: NULL perturber arrays");
  Chain c;
  c.n = s->n; c.m = s->m; c.G = G;
  for (int i = 0; i < s->n; ++i) c.M += s->m[i];
  if (p && p->np > 0) { c.np = p->np; c.py = p->x; c.pw = p->v; c.pm = p->m; c.t0 = p->t0; }
  const int n = s->n;
  Y y;
  if (!load_state(s, c, y)) return fail(TG_EINVAL, "tg_archain_advance: chain is not a permutation");
  const double t_end = s->t + dt;
  Work w(n);
  int64_t steps = 0;
  double H = s->ds;
  Y out;
  int hint = 3;   // columns the last extrapolated step converged with
  while (y.t(n) < t_end) {
    rechain(c, y);
    int col = bs_step(c, y, H, tol, out, w, hint);
    if (col >= 0) hint = col + 1;
    if (col < 0) {
      H *= 0.5;
      if (H < 1e-300 || ++steps > 100000000) return fail(TG_EINTERNAL, "tg_archain_advance: step underflow");
      continue;
    }
    ++steps;
    if (out.t(n) > t_end) {
      // the last step: secant (regula falsi) search for the length that
      // ends at t_end; a trial that does not converge shortens the step and
      // returns to ordinary stepping.  The first trial solves the cubic in
      // the step length through t and dt/ds = 1 / (T + B) at both ends of
      // the step that overshot (Newton's method); it usually ends within
      // 1e-8 of the advance, and such a gap is closed in physical time.
      double ha = 0.0, ta = y.t(n), hb = H, tb = out.t(n);
      bool done = false, retry = false;
      double uh = (t_end - ta) / (tb - ta);
      {
        const double da = H / (kinetic(c, y.W(n), w) + y.B(n));
        const double db = H / (kinetic(c, out.W(n), w) + out.B(n));
        for (int q = 0; q < 30; ++q) {
          const double u = uh, u2 = u * u, u3 = u2 * u;
          const double f = ta * (2 * u3 - 3 * u2 + 1) + da * (u3 - 2 * u2 + u) +
                           tb * (-2 * u3 + 3 * u2) + db * (u3 - u2) - t_end;
          const double fp = ta * (6 * u2 - 6 * u) + da * (3 * u2 - 4 * u + 1) +
                            tb * (-6 * u2 + 6 * u) + db * (3 * u2 - 2 * u);
          if (!(fp > 0.0)) break;
          const double un = std::min(1.0, std::max(0.0, u - f / fp));
          if (un == uh) break;
          uh = un;
        }
      }
      for (int it = 0; it < 100 && !done; ++it) {
        const double hc = it == 0 ? uh * H : ha + (hb - ha) * (t_end - ta) / (tb - ta);
        Y yc;
        if (bs_step(c, y, hc, tol, yc, w, hint) < 0) {
          H = 0.5 * hc;
          retry = true;
          break;
        }
        const double tc = yc.t(n);
        if (std::fabs(tc - t_end) <= 1e-14 * std::max(std::fabs(t_end), std::fabs(dt))) {
          y = yc;
          done = true;
        } else if (std::fabs(t_end - tc) <= 1e-6 * std::fabs(dt) &&
                   std::fabs(t_end - tc) <= 1e-4 * crossing(c, yc)) {
          // second order: the rest's error is ~(gap / crossing time)^3
          close_gap(c, yc, t_end - tc, w);
          y = yc;
          done = true;
        } else if (tc < t_end) {
          ha = hc; ta = tc;
        } else {
          hb = hc; tb = tc;
        }
      }
      if (retry) continue;
      if (!done) return fail(TG_EINTERNAL, "tg_archain_advance: final step search did not close");
      y.t(n) = t_end;   // within the search tolerance
      break;
    }
    y = out;
    // next step: grow when the extrapolation converged early
    if (col <= 3) H *= 1.5;
    else if (col >= 6) H *= 0.7;
  }
  store_state(c, y, s);
  s->t = t_end;
  s->B = y.B(n);
  s->ds = H;
  if (steps_out) *steps_out = steps;
  return TG_OK;
} TG_HOST_CATCH("tg_archain_advance")

tg_status tg_archain_energy(const tg_archain *s, double G, double *err_out) try {
  if (!s || !s->x || !s->v || !s->m || !err_out) return fail(TG_EINVAL, "tg_archain_energy: NULL argument");
  if (s->n < 2 || s->n > kMaxChain) return fail(TG_EINVAL, "tg_archain_energy: n must be in 2..256");
  Chain c;
  c.n = s->n; c.m = s->m; c.G = G;
  for (int i = 0; i < s->n; ++i) c.M += s->m[i];
  Work w(s->n);
  Y y;
  if (!load_state(s, c, y)) return fail(TG_EINVAL, "tg_archain_energy: chain is not a permutation");
  const double U = internal(c, y.X(), w);
  const double T = kinetic(c, y.W(s->n), w);
  *err_out = (T - U + s->B) / U;
  return TG_OK;
} TG_HOST_CATCH("tg_archain_energy")

}  // extern "C"
