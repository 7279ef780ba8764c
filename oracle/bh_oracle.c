/*
 * Plain CPU oracle for the softened Barnes-Hut tree-gravity path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path.
 *
 * Every routine is the plain definition (or the algorithm's steps in order),
 * written for a reader to check by eye against the paper:
 *   - tree force = multipole expansion of a distant group about its centre of
 *     mass, near particles summed directly (Sec. 1; Sec. 2, the integration
 *     regions list),
 *   - Plummer softening of every pair (Sec. 3, the softening paragraph), or
 *     the cubic-spline softening the tree may use instead (Sec. 2, the
 *     description of the tree part; READING below, or_spline_psi),
 *   - forces only for the active particles, leapfrog driver, individual
 *     hierarchical block time-steps (Sec. 2, the hybrid time-step steps (1),
 *     (6), (7); Sec. 3 for tau_acc = 0.3 for stars and 0.003 for SMBHs).
 * Readings where the paper is silent (octree from Morton keys, geometric
 * opening angle, softened quadrupole, self term, block-step level rule) are
 * marked READING below.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no -ffast-math).
 * All floating point is IEEE double; sums run in the order stated.
 *
 * Layouts: positions are row-major [n][3] doubles.  Systems (independent
 * realisations) are contiguous index ranges off[s] .. off[s+1].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_BITS 21               /* key bits per axis */
#define OR_QMAX ((1u << OR_BITS) - 1u)
#define OR_MAXLEVEL 21           /* deepest octree level */

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---------------------------------------------------------------------- */
/* Bounding cube per system (READING: the smallest axis-aligned cube whose  */
/* low corner is the coordinate-wise minimum; side = largest extent, or 1   */
/* when every particle coincides).  cube[4s..4s+3] = lo_x, lo_y, lo_z, L.   */
/* ---------------------------------------------------------------------- */
void or_cube(const double *pos, const int64_t *off, int32_t S, double *cube) {
  for (int32_t s = 0; s < S; ++s) {
    int64_t a = off[s], b = off[s + 1];
    double *c = cube + 4 * (int64_t)s;
    if (b <= a) { c[0] = c[1] = c[2] = 0.0; c[3] = 1.0; continue; }
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) lo[k] = hi[k] = pos[3 * a + k];
    for (int64_t i = a; i < b; ++i)
      for (int k = 0; k < 3; ++k) {
        double x = pos[3 * i + k];
        if (x < lo[k]) lo[k] = x;
        if (x > hi[k]) hi[k] = x;
      }
    double L = 0.0;
    for (int k = 0; k < 3; ++k) {
      double e = hi[k] - lo[k];
      if (e > L) L = e;
    }
    if (L == 0.0) L = 1.0;
    c[0] = lo[0]; c[1] = lo[1]; c[2] = lo[2]; c[3] = L;
  }
}

/* ---------------------------------------------------------------------- */
/* Morton keys (READING: octree from 21-bit quantised coordinates).         */
/* q = min(floor((x - lo) * (2^21 / L)), 2^21 - 1); the key is the bits of */
/* (qx, qy, qz) interleaved from the top bit down, x first, so each 3-bit   */
/* digit is the octant 4*bx + 2*by + bz at one level.                       */
/* ---------------------------------------------------------------------- */
void or_keys(const double *pos, const int64_t *off, int32_t S,
             const double *cube, uint64_t *keys) {
  for (int32_t s = 0; s < S; ++s) {
    const double *c = cube + 4 * (int64_t)s;
    double sigma = 2097152.0 / c[3];
    for (int64_t i = off[s]; i < off[s + 1]; ++i) {
      uint64_t q[3];
      for (int k = 0; k < 3; ++k) {
        double t = pos[3 * i + k] - c[k];
        double u = t * sigma;
        double f = floor(u);
        uint64_t qi = (f <= 0.0) ? 0u : (uint64_t)f;
        if (qi > OR_QMAX) qi = OR_QMAX;
        q[k] = qi;
      }
      uint64_t key = 0;
      for (int j = OR_BITS - 1; j >= 0; --j)
        key = (key << 3) | (((q[0] >> j) & 1u) << 2) |
              (((q[1] >> j) & 1u) << 1) | ((q[2] >> j) & 1u);
      keys[i] = key;
    }
  }
}

/* ---------------------------------------------------------------------- */
/* Sort: within each system, order particles by key, ties by index.  This  */
/* total order makes the permutation unique.  perm[r] = original index.    */
/* ---------------------------------------------------------------------- */
typedef struct { uint64_t key; uint32_t idx; } or_kv;

static int or_kv_cmp(const void *pa, const void *pb) {
  const or_kv *a = (const or_kv *)pa, *b = (const or_kv *)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
  return 0;
}

int or_sort(const uint64_t *keys, const int64_t *off, int32_t S,
            uint32_t *perm) {
  for (int32_t s = 0; s < S; ++s) {
    int64_t a = off[s], n = off[s + 1] - off[s];
    if (n <= 0) continue;
    or_kv *kv = (or_kv *)malloc(sizeof(or_kv) * (size_t)n);
    if (!kv) return -1;
    for (int64_t i = 0; i < n; ++i) { kv[i].key = keys[a + i]; kv[i].idx = (uint32_t)(a + i); }
    qsort(kv, (size_t)n, sizeof(or_kv), or_kv_cmp);
    for (int64_t i = 0; i < n; ++i) perm[a + i] = kv[i].idx;
    free(kv);
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Octree over key prefixes (READING of the tree update, Sec. 2 step 7).   */
/* One root per non-empty system (level 0, its whole range).  A node is     */
/* refined iff it holds more than nleaf particles and its level is below   */
/* 21; its children are the non-empty octants of the next key digit, in   */
/* octant order.  Nodes are numbered breadth first: each node's children   */
/* are appended at the end, so ids run level by level and, within a level, */
/* in key order.  Leaves at level 21 may hold more than nleaf particles.    */
/* Returns the node count, or -1 when cap is too small.                     */
/* ---------------------------------------------------------------------- */
int64_t or_build(const uint64_t *skey, const int64_t *off, int32_t S,
                 int32_t nleaf, int64_t cap, uint8_t *level, uint32_t *first,
                 uint32_t *count, uint32_t *child, uint8_t *nchild,
                 int32_t *sys, uint32_t *parent) {
  int64_t nn = 0;
  for (int32_t s = 0; s < S; ++s) {
    if (off[s + 1] <= off[s]) continue;
    if (nn >= cap) return -1;
    level[nn] = 0; first[nn] = (uint32_t)off[s];
    count[nn] = (uint32_t)(off[s + 1] - off[s]);
    sys[nn] = s; parent[nn] = 0xffffffffu;
    ++nn;
  }
  for (int64_t i = 0; i < nn; ++i) {
    child[i] = 0; nchild[i] = 0;
    if (count[i] <= (uint32_t)nleaf || level[i] >= OR_MAXLEVEL) continue;
    int shift = 3 * (OR_MAXLEVEL - 1 - level[i]);
    uint32_t j = first[i], end = first[i] + count[i];
    child[i] = (uint32_t)nn;
    while (j < end) {
      uint64_t d = (skey[j] >> shift) & 7u;
      uint32_t k = j;
      while (k < end && ((skey[k] >> shift) & 7u) == d) ++k;
      if (nn >= cap) return -1;
      level[nn] = (uint8_t)(level[i] + 1); first[nn] = j; count[nn] = k - j;
      sys[nn] = sys[i]; parent[nn] = (uint32_t)i;
      ++nn; ++nchild[i];
      j = k;
    }
  }
  return nn;
}

/* ---------------------------------------------------------------------- */
/* 42 levels: the same definitions with 42-bit quantised coordinates, for   */
/* systems whose extent leaves the centre unresolved at 21 levels (escapers, */
/* untruncated initial conditions).  q = min(floor((x - lo) (2^42 / L)),    */
/* 2^42 - 1); the 126-bit key interleaves the bits from the top, x first,   */
/* and is kept as two words: khi = the first 21 digits (levels 1..21),      */
/* klo = the last 21 (levels 22..42).                                       */
/* ---------------------------------------------------------------------- */
#define OR_BITS42 42
#define OR_QMAX42 ((1ull << OR_BITS42) - 1ull)
#define OR_MAXLEVEL42 42

void or_keys42(const double *pos, const int64_t *off, int32_t S,
               const double *cube, uint64_t *khi, uint64_t *klo) {
  for (int32_t s = 0; s < S; ++s) {
    const double *c = cube + 4 * (int64_t)s;
    double sigma = 4398046511104.0 / c[3];
    for (int64_t i = off[s]; i < off[s + 1]; ++i) {
      uint64_t q[3];
      for (int k = 0; k < 3; ++k) {
        double t = pos[3 * i + k] - c[k];
        double u = t * sigma;
        double f = floor(u);
        uint64_t qi = (f <= 0.0) ? 0u : (uint64_t)f;
        if (qi > OR_QMAX42) qi = OR_QMAX42;
        q[k] = qi;
      }
      unsigned __int128 key = 0;
      for (int j = OR_BITS42 - 1; j >= 0; --j)
        key = (key << 3) | (((q[0] >> j) & 1u) << 2) |
              (((q[1] >> j) & 1u) << 1) | ((q[2] >> j) & 1u);
      khi[i] = (uint64_t)(key >> 63);
      klo[i] = (uint64_t)(key & (((unsigned __int128)1 << 63) - 1));
    }
  }
}

typedef struct { unsigned __int128 key; uint32_t idx; } or_kv42;

static int or_kv42_cmp(const void *pa, const void *pb) {
  const or_kv42 *a = (const or_kv42 *)pa, *b = (const or_kv42 *)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
  return 0;
}

/* Sort by the 126-bit key, ties by index, within each system. */
int or_sort42(const uint64_t *khi, const uint64_t *klo, const int64_t *off, int32_t S,
              uint32_t *perm) {
  for (int32_t s = 0; s < S; ++s) {
    int64_t a = off[s], n = off[s + 1] - off[s];
    if (n <= 0) continue;
    or_kv42 *kv = (or_kv42 *)malloc(sizeof(or_kv42) * (size_t)n);
    if (!kv) return -1;
    for (int64_t i = 0; i < n; ++i) {
      kv[i].key = ((unsigned __int128)khi[a + i] << 63) | klo[a + i];
      kv[i].idx = (uint32_t)(a + i);
    }
    qsort(kv, (size_t)n, sizeof(or_kv42), or_kv42_cmp);
    for (int64_t i = 0; i < n; ++i) perm[a + i] = kv[i].idx;
    free(kv);
  }
  return 0;
}

/* The octree of or_build over 126-bit sorted keys (skhi, sklo): refined    */
/* below level 42; leaves at level 42 may hold more than nleaf particles.   */
int64_t or_build42(const uint64_t *skhi, const uint64_t *sklo, const int64_t *off,
                   int32_t S, int32_t nleaf, int64_t cap, uint8_t *level,
                   uint32_t *first, uint32_t *count, uint32_t *child, uint8_t *nchild,
                   int32_t *sys, uint32_t *parent) {
  int64_t nn = 0;
  for (int32_t s = 0; s < S; ++s) {
    if (off[s + 1] <= off[s]) continue;
    if (nn >= cap) return -1;
    level[nn] = 0; first[nn] = (uint32_t)off[s];
    count[nn] = (uint32_t)(off[s + 1] - off[s]);
    sys[nn] = s; parent[nn] = 0xffffffffu;
    ++nn;
  }
  for (int64_t i = 0; i < nn; ++i) {
    child[i] = 0; nchild[i] = 0;
    if (count[i] <= (uint32_t)nleaf || level[i] >= OR_MAXLEVEL42) continue;
    int shift = 3 * (OR_MAXLEVEL42 - 1 - level[i]);
    uint32_t j = first[i], end = first[i] + count[i];
    child[i] = (uint32_t)nn;
    while (j < end) {
      unsigned __int128 kj = ((unsigned __int128)skhi[j] << 63) | sklo[j];
      uint32_t d = (uint32_t)(kj >> shift) & 7u;
      uint32_t k = j;
      while (k < end) {
        unsigned __int128 kk = ((unsigned __int128)skhi[k] << 63) | sklo[k];
        if (((uint32_t)(kk >> shift) & 7u) != d) break;
        ++k;
      }
      if (nn >= cap) return -1;
      level[nn] = (uint8_t)(level[i] + 1); first[nn] = j; count[nn] = k - j;
      sys[nn] = sys[i]; parent[nn] = (uint32_t)i;
      ++nn; ++nchild[i];
      j = k;
    }
  }
  return nn;
}

/* ---------------------------------------------------------------------- */
/* Moments about the centre of mass (Sec. 1: multipole expansion about the  */
/* group's centre of mass).  Straight from the particles of each node, in   */
/* sorted order, two passes:                                                */
/*   M = sum m,  c = (sum m x) / M,  S_ab = sum m (x_a - c_a)(x_b - c_b).   */
/* mom[10 v ..] = M, cx, cy, cz, Sxx, Syy, Szz, Sxy, Sxz, Syz.              */
/* spos/smass are the particles in sorted order.                            */
/* ---------------------------------------------------------------------- */
/* The sums are compensated (Neumaier 1974): s + x is rounded to t and its  */
/* exact error, (s - t) + x if |s| >= |x| else (x - t) + s, is added to a   */
/* running correction c; the sum is s + c.  A plain sum over the 10^5      */
/* particles of a node drifts by ~1e-12 relative, the size of the FP64     */
/* parity bar; the compensated one stays within a few ulp.                  */
typedef struct { double s, c; } or_ksum;

static void or_kadd(or_ksum *k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x))
    k->c += (k->s - t) + x;
  else
    k->c += (x - t) + k->s;
  k->s = t;
}

static double or_kget(const or_ksum *k) { return k->s + k->c; }

void or_moments(const double *spos, const double *smass, int64_t nn,
                const uint32_t *first, const uint32_t *count, double *mom) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t v = 0; v < nn; ++v) {
    uint32_t a = first[v], b = first[v] + count[v];
    or_ksum M = {0, 0}, sx = {0, 0}, sy = {0, 0}, sz = {0, 0};
    for (uint32_t j = a; j < b; ++j) {
      double m = smass[j];
      or_kadd(&M, m);
      or_kadd(&sx, m * spos[3 * (int64_t)j + 0]);
      or_kadd(&sy, m * spos[3 * (int64_t)j + 1]);
      or_kadd(&sz, m * spos[3 * (int64_t)j + 2]);
    }
    double Mt = or_kget(&M);
    double cx = or_kget(&sx) / Mt, cy = or_kget(&sy) / Mt, cz = or_kget(&sz) / Mt;
    or_ksum S[6];
    for (int k = 0; k < 6; ++k) S[k].s = S[k].c = 0.0;
    for (uint32_t j = a; j < b; ++j) {
      double m = smass[j];
      double dx = spos[3 * (int64_t)j + 0] - cx;
      double dy = spos[3 * (int64_t)j + 1] - cy;
      double dz = spos[3 * (int64_t)j + 2] - cz;
      or_kadd(&S[0], m * dx * dx); or_kadd(&S[1], m * dy * dy); or_kadd(&S[2], m * dz * dz);
      or_kadd(&S[3], m * dx * dy); or_kadd(&S[4], m * dx * dz); or_kadd(&S[5], m * dy * dz);
    }
    double *o = mom + 10 * v;
    o[0] = Mt; o[1] = cx; o[2] = cy; o[3] = cz;
    for (int k = 0; k < 6; ++k) o[4 + k] = or_kget(&S[k]);
  }
}

/* ---------------------------------------------------------------------- */
/* Groups (READING): the walk is shared by the targets of a group = a node  */
/* holding at most ngroup particles whose parent holds more (or a root that */
/* holds at most ngroup).  A leaf holding more than ngroup is cut into runs */
/* of ngroup in sorted order.  Groups come out ordered by first particle.   */
/* g[4 k ..] = first, count, node, system.  Returns count or -1 (cap).      */
/* ---------------------------------------------------------------------- */
static int64_t or_grp_rec(uint32_t v, int32_t ng, const uint32_t *first,
                          const uint32_t *count, const uint32_t *child,
                          const uint8_t *nchild, const int32_t *sys,
                          int64_t cap, int64_t n, uint32_t *g) {
  if (n < 0) return n;
  if (count[v] <= (uint32_t)ng) {
    if (n >= cap) return -1;
    g[4 * n + 0] = first[v]; g[4 * n + 1] = count[v];
    g[4 * n + 2] = v; g[4 * n + 3] = (uint32_t)sys[v];
    return n + 1;
  }
  if (nchild[v] == 0) {
    for (uint32_t c = 0; c < count[v]; c += (uint32_t)ng) {
      if (n >= cap) return -1;
      uint32_t len = count[v] - c < (uint32_t)ng ? count[v] - c : (uint32_t)ng;
      g[4 * n + 0] = first[v] + c; g[4 * n + 1] = len;
      g[4 * n + 2] = v; g[4 * n + 3] = (uint32_t)sys[v];
      ++n;
    }
    return n;
  }
  for (uint32_t c = 0; c < nchild[v]; ++c)
    n = or_grp_rec(child[v] + c, ng, first, count, child, nchild, sys, cap, n, g);
  return n;
}

int64_t or_groups(int64_t nn, const uint8_t *level, const uint32_t *first,
                  const uint32_t *count, const uint32_t *child,
                  const uint8_t *nchild, const int32_t *sys, int32_t ngroup,
                  int64_t cap, uint32_t *g) {
  int64_t n = 0;
  for (int64_t v = 0; v < nn && level[v] == 0; ++v)
    n = or_grp_rec((uint32_t)v, ngroup, first, count, child, nchild, sys, cap, n, g);
  return n;
}

/* Group box over the group's ACTIVE particles (only they are targets):     */
/* box[6 k ..] = lo x,y,z, hi x,y,z; nact[k] = number of active targets.    */
void or_group_boxes(const double *spos, const uint8_t *sactive, int64_t ng,
                    const uint32_t *g, double *box, int32_t *nact) {
  for (int64_t k = 0; k < ng; ++k) {
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    int32_t na = 0;
    for (uint32_t j = g[4 * k]; j < g[4 * k] + g[4 * k + 1]; ++j) {
      if (!sactive[j]) continue;
      for (int c = 0; c < 3; ++c) {
        double x = spos[3 * (int64_t)j + c];
        if (na == 0 || x < lo[c]) lo[c] = x;
        if (na == 0 || x > hi[c]) hi[c] = x;
      }
      ++na;
    }
    for (int c = 0; c < 3; ++c) { box[6 * k + c] = lo[c]; box[6 * k + 3 + c] = hi[c]; }
    nact[k] = na;
  }
}

/* ---------------------------------------------------------------------- */
/* Opening-angle test and walk (READING: geometric Barnes-Hut angle with    */
/* the distance d from the group box to the cell's centre of mass).         */
/*   d^2 = sum_k max(max(glo_k - c_k, c_k - ghi_k), 0)^2   (x, then y, z)   */
/*   accept (multipole) iff s*s < (theta*theta) * d^2,  s = L * 2^-level.   */
/* Accepted cells go to the P2M list; a refused leaf goes to the P2P list;  */
/* a refused internal node is replaced by its children.  With theta below   */
/* 1/sqrt(3) a cell that holds a target is never accepted.                  */
/* ---------------------------------------------------------------------- */
static int or_mac_accept(const double *glo, const double *ghi,
                         const double *com, double s2, double th2) {
  double d2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    double a = glo[k] - com[k];
    double b = com[k] - ghi[k];
    double m = a > b ? a : b;
    if (m < 0.0) m = 0.0;
    d2 = d2 + m * m;
  }
  return s2 < th2 * d2;
}

static int or_u32_cmp(const void *pa, const void *pb) {
  uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
  return a < b ? -1 : (a > b ? 1 : 0);
}

typedef struct { uint32_t *v; int64_t n, cap; } or_vec;

static int or_push(or_vec *a, uint32_t x) {
  if (a->n == a->cap) {
    int64_t nc = a->cap ? 2 * a->cap : 256;
    uint32_t *p = (uint32_t *)realloc(a->v, sizeof(uint32_t) * (size_t)nc);
    if (!p) return -1;
    a->v = p; a->cap = nc;
  }
  a->v[a->n++] = x;
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Relative opening test (READING: the paper names a "Gadget" criterion     */
/* with an error tolerance, Sec. 3, run set-up, but prints no formula; this  */
/* is the relative criterion of Springel 2005, MNRAS 364, 1105, Sec. 3.1,   */
/* taken for a group of targets).  A cell of mass M and side s is accepted  */
/* for a target with old acceleration |a| at distance r from the cell's     */
/* centre of mass iff G M s^2 / r^4 <= alpha |a|, and the target lies       */
/* outside the cell's cube enlarged by 20 % about its geometric centre.     */
/* Group form: r is the group-box distance d of the geometric test, |a| the */
/* smallest old acceleration of the group's active targets, and the whole   */
/* group box must miss the enlarged cube.  Squared to avoid roots:          */
/*   P = (G M) s^2,   accept iff  P P <= A ((d^2 d^2)(d^2 d^2))  and the     */
/*   box misses [g - h, g + h] on some axis, h = 0.6 s,                     */
/* with A = (alpha alpha) a2min per group, a2min = min (ax ax + ay ay) + az */
/* az.  Cell centre: g_k = lo_k + (i_k + 0.5) s from the integer cell       */
/* coordinates i_k in the key prefix of the cell's first particle.          */
/* rel[8 v] = {g_x - h, g_y - h, g_z - h, P, g_x + h, g_y + h, g_z + h, 0}. */
/* ---------------------------------------------------------------------- */
/* Geometric centre g of node v's cell and its side s = L 2^-level. */
static double or_cell_centre(int64_t v, const uint8_t *level, const uint32_t *first,
                             const int32_t *sys, const uint64_t *skeys,
                             const double *cube, double g[3]) {
  const double *c = cube + 4 * (int64_t)sys[v];
  int l = (int)level[v];
  double s = ldexp(c[3], -l);
  uint64_t pre = skeys[first[v]] >> (3 * (OR_MAXLEVEL - l));
  uint64_t ic[3] = {0, 0, 0};
  for (int j = 0; j < l; ++j) {            /* digit j from the bottom */
    uint64_t d = (pre >> (3 * j)) & 7u;
    ic[0] |= ((d >> 2) & 1u) << j;
    ic[1] |= ((d >> 1) & 1u) << j;
    ic[2] |= (d & 1u) << j;
  }
  for (int k = 0; k < 3; ++k) g[k] = c[k] + ((double)ic[k] + 0.5) * s;
  return s;
}

/* side == NULL: s = L 2^-level; else side[v] (a refitted tree). */
void or_rel_records(int64_t nn, const uint8_t *level, const uint32_t *first,
                    const int32_t *sys, const uint64_t *skeys,
                    const double *cube, const double *mom, double G,
                    const double *side, double *rel) {
  for (int64_t v = 0; v < nn; ++v) {
    double g[3];
    double s = or_cell_centre(v, level, first, sys, skeys, cube, g);
    if (side) s = side[v];
    double h = 0.6 * s;
    double *o = rel + 8 * v;
    for (int k = 0; k < 3; ++k) {
      o[k] = g[k] - h;
      o[4 + k] = g[k] + h;
    }
    o[3] = (G * mom[10 * v]) * (s * s);
    o[7] = 0.0;
  }
}

/* ---------------------------------------------------------------------- */
/* Refit (READING of Sec. 2 step 7, which updates the tree structure only  */
/* when needed): between full builds the sort order, nodes and groups stay; moments   */
/* come from the current positions, and each cell's opening size becomes    */
/*   s' = max(s, 2 e),  e = max_k max(hi_k - g_k, g_k - lo_k),              */
/* with [lo, hi] the bounding box of the node's particles (exact min/max)   */
/* and g the cell's geometric centre: the smallest cube about g that holds  */
/* the cell and every particle of the node.  Both opening tests take s'.    */
/* ---------------------------------------------------------------------- */
void or_refit_sides(int64_t nn, const uint8_t *level, const uint32_t *first,
                    const uint32_t *count, const int32_t *sys, const uint64_t *skeys,
                    const double *cube, const double *spos, double *side) {
  for (int64_t v = 0; v < nn; ++v) {
    double g[3];
    double s = or_cell_centre(v, level, first, sys, skeys, cube, g);
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) lo[k] = hi[k] = spos[3 * (int64_t)first[v] + k];
    for (uint32_t j = first[v]; j < first[v] + count[v]; ++j)
      for (int k = 0; k < 3; ++k) {
        double x = spos[3 * (int64_t)j + k];
        if (x < lo[k]) lo[k] = x;
        if (x > hi[k]) hi[k] = x;
      }
    double e = 0.0;
    for (int k = 0; k < 3; ++k) {
      double a = hi[k] - g[k], b = g[k] - lo[k];
      if (a > e) e = a;
      if (b > e) e = b;
    }
    side[v] = (2.0 * e > s) ? 2.0 * e : s;
  }
}

static int or_rel_accept(const double *glo, const double *ghi,
                         const double *com, const double *r, double A) {
  double d2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    double a = glo[k] - com[k];
    double b = com[k] - ghi[k];
    double m = a > b ? a : b;
    if (m < 0.0) m = 0.0;
    d2 = d2 + m * m;
  }
  double d4 = d2 * d2;
  if (!(r[3] * r[3] <= A * (d4 * d4))) return 0;
  for (int k = 0; k < 3; ++k)
    if (glo[k] > r[4 + k] || ghi[k] < r[k]) return 1;   /* box misses the cube */
  return 0;
}

/* Walk one group; lists come back sorted ascending.  rel == NULL: the      */
/* geometric test with theta; else the relative test with A = arel.  side   */
/* (refitted tree) replaces L 2^-level as the cell size.  Root of the       */
/* group's system: roots are the level-0 nodes in system order.             */
static int or_walk_one(uint32_t root, const uint8_t *level,
                       const uint32_t *child, const uint8_t *nchild,
                       const int32_t *sys, const double *mom,
                       const double *cube, const double *box, double theta,
                       const double *side, const double *rel, double arel,
                       or_vec *p2m, or_vec *p2p, or_vec *work) {
  double th2 = theta * theta;
  p2m->n = p2p->n = work->n = 0;
  if (or_push(work, root)) return -1;
  while (work->n > 0) {
    uint32_t c = work->v[--work->n];
    double s = side ? side[c] : ldexp(cube[4 * (int64_t)sys[c] + 3], -(int)level[c]);
    const double *com = mom + 10 * (int64_t)c + 1;
    int acc = rel ? or_rel_accept(box, box + 3, com, rel + 8 * (int64_t)c, arel)
                  : or_mac_accept(box, box + 3, com, s * s, th2);
    if (acc) {
      if (or_push(p2m, c)) return -1;
    } else if (nchild[c] == 0) {
      if (or_push(p2p, c)) return -1;
    } else {
      for (uint32_t k = 0; k < nchild[c]; ++k)
        if (or_push(work, child[c] + k)) return -1;
    }
  }
  /* an empty list may never have been allocated (qsort needs an array) */
  if (p2m->n > 1) qsort(p2m->v, (size_t)p2m->n, sizeof(uint32_t), or_u32_cmp);
  if (p2p->n > 1) qsort(p2p->v, (size_t)p2p->n, sizeof(uint32_t), or_u32_cmp);
  return 0;
}

static uint32_t or_root_of(int32_t s, int64_t nn, const uint8_t *level,
                           const int32_t *sys) {
  for (int64_t v = 0; v < nn && level[v] == 0; ++v)
    if (sys[v] == s) return (uint32_t)v;
  return 0xffffffffu;
}

/* Lists for selected groups.  Call with ids == NULL to get the per-group   */
/* sizes (np2m[k], np2p[k]); then with ids != NULL and lofs (exclusive      */
/* offsets, 2 per group: P2M then P2P) to fill.  Returns 0, or -1.          */
int or_walk_lists(int64_t nn, const uint8_t *level, const uint32_t *child,
                  const uint8_t *nchild, const int32_t *sys, const double *mom,
                  const double *cube, const uint32_t *g, const double *box,
                  const int32_t *sel, int64_t nsel, double theta, const double *side,
                  const double *rel, const double *arel,
                  int64_t *np2m, int64_t *np2p, const int64_t *lofs,
                  uint32_t *ids) {
  int err = 0;
#pragma omp parallel
  {
    or_vec p2m = {0, 0, 0}, p2p = {0, 0, 0}, work = {0, 0, 0};
#pragma omp for schedule(dynamic, 4)
    for (int64_t t = 0; t < nsel; ++t) {
      int64_t k = sel[t];
      uint32_t root = or_root_of((int32_t)g[4 * k + 3], nn, level, sys);
      if (or_walk_one(root, level, child, nchild, sys, mom, cube, box + 6 * k,
                      theta, side, rel, rel ? arel[k] : 0.0, &p2m, &p2p, &work)) {
        err = 1; continue;
      }
      np2m[t] = p2m.n; np2p[t] = p2p.n;
      if (ids) {
        if (p2m.n) memcpy(ids + lofs[2 * t], p2m.v, sizeof(uint32_t) * (size_t)p2m.n);
        if (p2p.n) memcpy(ids + lofs[2 * t + 1], p2p.v, sizeof(uint32_t) * (size_t)p2p.n);
      }
    }
    free(p2m.v); free(p2p.v); free(work.v);
  }
  return err ? -1 : 0;
}

/* ---------------------------------------------------------------------- */
/* Evaluation (Sec. 3: Plummer softening of every pair).                    */
/* For target i and x = x_i - c, D_n = (|x|^2 + eps^2)^(-n/2):              */
/*  P2P  (source particle j != i, mass m):                                  */
/*     a -= G m D3 x,   phi -= G m D1            (x = x_i - x_j)            */
/*  P2M  (cell: M, c, S; T = tr S, Q = 3S - T I, W = x.Q.x - T eps^2):      */
/*     a += G(-M D3 x + D5 Q x - 2.5 D7 W x),  phi += G(-M D1 - 0.5 D5 W)   */
/*  (READING: the second-order Taylor expansion of the softened kernel      */
/*   about the centre of mass; its -T eps^2 term vanishes for eps = 0.)     */
/* Order: P2M cells by ascending id, then P2P leaves by ascending id with   */
/* their particles in sorted order; plain double additions.  The self term */
/* is left out of the potential too.                                        */
/* ---------------------------------------------------------------------- */
/* ---------------------------------------------------------------------- */
/* Cubic-spline softening.  READING: the paper names spline or Plummer     */
/* softening for the tree without formulas; the spline is the kernel of    */
/* Monaghan & Lattanzio (1985) with support 2h, used for gravity as in     */
/* Hernquist & Katz (1989), with h = eps.  Its mass density is             */
/*   W(u) = (1/(pi h^3)) (1 - 3/2 u^2 + 3/4 u^3)   0 <= u < 1,             */
/*        = (1/(pi h^3)) (2 - u)^3 / 4             1 <= u < 2,  u = r/h,   */
/* and 0 beyond.  psi(r) is the potential of a unit mass so spread, with   */
/* the sign of 1/r (phi = -G m psi), and psi_{k+1} = -(1/r) d psi_k / dr:  */
/* a pair force is -G m psi_1(r) x, and beyond 2h the four are the         */
/* Newtonian 1/r, 1/r^3, 3/r^5, 15/r^7.  psi_3 grows as 1/u near 0; it is   */
/* only needed for cells, whose centre of mass never sits on the target    */
/* (it is set to 0 at u = 0, where it multiplies zero).                    */
/* ---------------------------------------------------------------------- */
static void or_spline_psi(double r, double h, double psi[4]) {
  double u = r / h;
  double ih = 1.0 / h;
  double ih2 = ih * ih;
  double ih3 = ih2 * ih, ih5 = ih3 * ih2, ih7 = ih5 * ih2;
  if (u < 1.0) {
    double u2 = u * u, u3 = u2 * u, u4 = u3 * u, u5 = u4 * u;
    psi[0] = ih * (7.0 / 5.0 - 2.0 / 3.0 * u2 + 3.0 / 10.0 * u4 - 1.0 / 10.0 * u5);
    psi[1] = ih3 * (4.0 / 3.0 - 6.0 / 5.0 * u2 + 1.0 / 2.0 * u3);
    psi[2] = ih5 * (12.0 / 5.0 - 3.0 / 2.0 * u);
    psi[3] = u > 0.0 ? ih7 * (3.0 / 2.0) / u : 0.0;
  } else if (u < 2.0) {
    double u2 = u * u, u3 = u2 * u, u4 = u3 * u, u5 = u4 * u, u7 = u5 * u2;
    psi[0] = ih * (8.0 / 5.0 - 4.0 / 3.0 * u2 + u3 - 3.0 / 10.0 * u4 + 1.0 / 30.0 * u5 -
                   1.0 / (15.0 * u));
    psi[1] = ih3 * (8.0 / 3.0 - 3.0 * u + 6.0 / 5.0 * u2 - 1.0 / 6.0 * u3 - 1.0 / (15.0 * u3));
    psi[2] = ih5 * (3.0 / u - 12.0 / 5.0 + 1.0 / 2.0 * u - 1.0 / (5.0 * u5));
    psi[3] = ih7 * (3.0 / u3 - 1.0 / (2.0 * u) - 1.0 / u7);
  } else {
    double ir = 1.0 / r;
    double ir2 = ir * ir;
    psi[0] = ir;
    psi[1] = ir * ir2;
    psi[2] = 3.0 * psi[1] * ir2;
    psi[3] = 5.0 * psi[2] * ir2;
  }
}

/* The same in long double, for the direct-sum reference.                  */
static void or_spline_psi_l(long double r, long double h, long double psi[2]) {
  long double u = r / h;
  long double ih = 1.0L / h;
  if (u < 1.0L) {
    long double u2 = u * u, u3 = u2 * u, u4 = u3 * u, u5 = u4 * u;
    psi[0] = ih * (7.0L / 5.0L - 2.0L / 3.0L * u2 + 3.0L / 10.0L * u4 - 1.0L / 10.0L * u5);
    psi[1] = ih * ih * ih * (4.0L / 3.0L - 6.0L / 5.0L * u2 + 1.0L / 2.0L * u3);
  } else if (u < 2.0L) {
    long double u2 = u * u, u3 = u2 * u, u4 = u3 * u, u5 = u4 * u;
    psi[0] = ih * (8.0L / 5.0L - 4.0L / 3.0L * u2 + u3 - 3.0L / 10.0L * u4 +
                   1.0L / 30.0L * u5 - 1.0L / (15.0L * u));
    psi[1] = ih * ih * ih *
             (8.0L / 3.0L - 3.0L * u + 6.0L / 5.0L * u2 - 1.0L / 6.0L * u3 - 1.0L / (15.0L * u3));
  } else {
    psi[0] = 1.0L / r;
    psi[1] = psi[0] * psi[0] * psi[0];
  }
}

/* Exported for the pins: psi[0..3] at r for softening length h.           */
void or_spline(double r, double h, double *psi) { or_spline_psi(r, h, psi); }

/* Spline-softened multipole term, the second-order expansion of          */
/* sum_j m_j psi(|x - y_j|) about the centre of mass for any radial psi:   */
/*   phi = -G (M psi + 1/2 psi_2 x.S.x - 1/2 psi_1 T)                      */
/*   a   =  G (-M psi_1 x + psi_2 (S x + T x / 2) - 1/2 psi_3 (x.S.x) x)   */
/* with x = target - com, S the second moments, T = tr S.  (With the       */
/* Plummer psi these reduce to or_p2m_term.)                              */
static void or_p2m_spline(const double *o, double xi, double yi, double zi,
                          double h, double G, double *out) {
  double M = o[0];
  double x = xi - o[1], y = yi - o[2], z = zi - o[3];
  double Sxx = o[4], Syy = o[5], Szz = o[6], Sxy = o[7], Sxz = o[8], Syz = o[9];
  double T = Sxx + Syy + Szz;
  double r = sqrt(x * x + y * y + z * z);
  double psi[4];
  or_spline_psi(r, h, psi);
  double Sx = Sxx * x + Sxy * y + Sxz * z;
  double Sy = Sxy * x + Syy * y + Syz * z;
  double Sz = Sxz * x + Syz * y + Szz * z;
  double xSx = x * Sx + y * Sy + z * Sz;
  out[0] += G * (-M * psi[1] * x + psi[2] * (Sx + 0.5 * T * x) - 0.5 * psi[3] * xSx * x);
  out[1] += G * (-M * psi[1] * y + psi[2] * (Sy + 0.5 * T * y) - 0.5 * psi[3] * xSx * y);
  out[2] += G * (-M * psi[1] * z + psi[2] * (Sz + 0.5 * T * z) - 0.5 * psi[3] * xSx * z);
  out[3] -= G * (M * psi[0] + 0.5 * psi[2] * xSx - 0.5 * psi[1] * T);
}

/* Spline-softened particle term (coincident particles feel no force).     */
static void or_p2p_spline(double xj, double yj, double zj, double m, double xi,
                          double yi, double zi, double h, double G, double *out) {
  double x = xi - xj, y = yi - yj, z = zi - zj;
  double r = sqrt(x * x + y * y + z * z);
  double psi[4];
  or_spline_psi(r, h, psi);
  out[0] -= G * m * psi[1] * x; out[1] -= G * m * psi[1] * y; out[2] -= G * m * psi[1] * z;
  out[3] -= G * m * psi[0];
}

/* One multipole (P2M) term: cell o = {M, cx, cy, cz, Sxx, Syy, Szz, Sxy,   */
/* Sxz, Syz}; target at (xi, yi, zi).  Adds to out[0..3] = ax, ay, az, phi. */
static void or_p2m_term(const double *o, double xi, double yi, double zi,
                        double e2, double G, double *out) {
  double M = o[0];
  double x = xi - o[1], y = yi - o[2], z = zi - o[3];
  double Sxx = o[4], Syy = o[5], Szz = o[6], Sxy = o[7], Sxz = o[8], Syz = o[9];
  double T = Sxx + Syy + Szz;
  double r2 = x * x + y * y + z * z + e2;
  double D1 = 1.0 / sqrt(r2);
  double D2 = D1 * D1;
  double D3 = D1 * D2, D5 = D3 * D2, D7 = D5 * D2;
  double Qx = 3.0 * (Sxx * x + Sxy * y + Sxz * z) - T * x;
  double Qy = 3.0 * (Sxy * x + Syy * y + Syz * z) - T * y;
  double Qz = 3.0 * (Sxz * x + Syz * y + Szz * z) - T * z;
  double W = x * Qx + y * Qy + z * Qz - T * e2;
  out[0] += G * (-M * D3 * x + D5 * Qx - 2.5 * D7 * W * x);
  out[1] += G * (-M * D3 * y + D5 * Qy - 2.5 * D7 * W * y);
  out[2] += G * (-M * D3 * z + D5 * Qz - 2.5 * D7 * W * z);
  out[3] += G * (-M * D1 - 0.5 * D5 * W);
}

/* One particle (P2P) term: source (xj, yj, zj) of mass m.                 */
static void or_p2p_term(double xj, double yj, double zj, double m, double xi,
                        double yi, double zi, double e2, double G,
                        double *out) {
  double x = xi - xj, y = yi - yj, z = zi - zj;
  double r2 = x * x + y * y + z * z + e2;
  double D1 = 1.0 / sqrt(r2);
  double D3 = D1 * D1 * D1;
  out[0] -= G * m * D3 * x; out[1] -= G * m * D3 * y; out[2] -= G * m * D3 * z;
  out[3] -= G * m * D1;
}

/* Exported single terms, so that tests can probe the expansion alone.      */
/* soft: 0 Plummer, 1 cubic spline (h = eps).                              */
void or_p2m_single(const double *cell, const double *x, double eps, double G,
                   double *out, int32_t soft) {
  out[0] = out[1] = out[2] = out[3] = 0.0;
  if (soft)
    or_p2m_spline(cell, x[0], x[1], x[2], eps, G, out);
  else
    or_p2m_term(cell, x[0], x[1], x[2], eps * eps, G, out);
}

void or_p2p_single(const double *src, double m, const double *x, double eps,
                   double G, double *out, int32_t soft) {
  out[0] = out[1] = out[2] = out[3] = 0.0;
  if (soft)
    or_p2p_spline(src[0], src[1], src[2], m, x[0], x[1], x[2], eps, G, out);
  else
    or_p2p_term(src[0], src[1], src[2], m, x[0], x[1], x[2], eps * eps, G, out);
}

static void or_eval_target(int64_t i, const double *spos, const double *smass,
                           const uint32_t *first, const uint32_t *count,
                           const double *mom, const or_vec *p2m,
                           const or_vec *p2p, double eps, double G, int32_t soft,
                           double *acc, double *pot, int64_t *n_pp) {
  double xi = spos[3 * i], yi = spos[3 * i + 1], zi = spos[3 * i + 2];
  double e2 = eps * eps;
  double out[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t t = 0; t < p2m->n; ++t) {
    const double *o = mom + 10 * (int64_t)p2m->v[t];
    if (soft)
      or_p2m_spline(o, xi, yi, zi, eps, G, out);
    else
      or_p2m_term(o, xi, yi, zi, e2, G, out);
  }
  int64_t npp = 0;
  for (int64_t t = 0; t < p2p->n; ++t) {
    uint32_t leaf = p2p->v[t];
    for (uint32_t j = first[leaf]; j < first[leaf] + count[leaf]; ++j) {
      if ((int64_t)j == i) continue;
      const double *q = spos + 3 * (int64_t)j;
      if (soft)
        or_p2p_spline(q[0], q[1], q[2], smass[j], xi, yi, zi, eps, G, out);
      else
        or_p2p_term(q[0], q[1], q[2], smass[j], xi, yi, zi, e2, G, out);
      ++npp;
    }
  }
  acc[3 * i] = out[0]; acc[3 * i + 1] = out[1]; acc[3 * i + 2] = out[2];
  pot[i] = out[3];
  *n_pp += npp;
}

/* Tree forces for the active targets of the selected groups.  Results are */
/* written in SORTED order (acc[3 r], pot[r]); counts[0] = P2P pairs,      */
/* counts[1] = particle-cell (P2M) pairs, counts[2] = targets evaluated.   */
int or_tree_forces(int64_t nn, const uint8_t *level, const uint32_t *first,
                   const uint32_t *count, const uint32_t *child,
                   const uint8_t *nchild, const int32_t *sys, const double *mom,
                   const double *cube, const uint32_t *g, const double *box,
                   const int32_t *sel, int64_t nsel, const double *spos,
                   const double *smass, const uint8_t *sactive, double eps,
                   double theta, const double *side, const double *rel,
                   const double *arel, double G, double *acc, double *pot,
                   int64_t *counts, int32_t soft) {
  int err = 0;
  int64_t npp = 0, npm = 0, ntg = 0;
#pragma omp parallel reduction(+ : npp, npm, ntg)
  {
    or_vec p2m = {0, 0, 0}, p2p = {0, 0, 0}, work = {0, 0, 0};
#pragma omp for schedule(dynamic, 4)
    for (int64_t t = 0; t < nsel; ++t) {
      int64_t k = sel[t];
      uint32_t root = or_root_of((int32_t)g[4 * k + 3], nn, level, sys);
      if (or_walk_one(root, level, child, nchild, sys, mom, cube, box + 6 * k,
                      theta, side, rel, rel ? arel[k] : 0.0, &p2m, &p2p, &work)) {
        err = 1; continue;
      }
      for (uint32_t i = g[4 * k]; i < g[4 * k] + g[4 * k + 1]; ++i) {
        if (!sactive[i]) continue;
        or_eval_target(i, spos, smass, first, count, mom, &p2m, &p2p, eps, G, soft,
                       acc, pot, &npp);
        npm += p2m.n;
        ++ntg;
      }
    }
    free(p2m.v); free(p2p.v); free(work.v);
  }
  counts[0] = npp; counts[1] = npm; counts[2] = ntg;
  return err ? -1 : 0;
}

/* ---------------------------------------------------------------------- */
/* Direct summation, the exact reference: for each listed target i, the     */
/* sum over every other particle of its own system (same softening eps),    */
/* plus nx external point masses (SMBHs) with pair softening                */
/* max(eps, xeps_k) (Sec. 2: eps = max(eps_BH, eps_star)).  Accumulated in  */
/* long double.  Outputs per listed target: acc[3 t], pot[t].  soft = 1:    */
/* every pair takes the cubic spline with that softening as h.              */
/* ---------------------------------------------------------------------- */
void or_direct(const double *pos, const double *mass, const int64_t *off,
               int32_t S, const int32_t *sysof, const int64_t *tgt, int64_t nt,
               double eps, const double *xpos, const double *xmass,
               const double *xeps, int64_t nx, double G, double *acc,
               double *pot, int32_t soft) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < nt; ++t) {
    int64_t i = tgt[t];
    int32_t s = sysof ? sysof[t] : 0;
    (void)S;
    long double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
    long double ax = 0, ay = 0, az = 0, ph = 0;
    long double e2 = (long double)eps * (long double)eps;
    for (int64_t j = off[s]; j < off[s + 1]; ++j) {
      if (j == i) continue;
      long double x = xi - pos[3 * j], y = yi - pos[3 * j + 1], z = zi - pos[3 * j + 2];
      long double D1, D3;
      if (soft) {
        long double ps[2];
        or_spline_psi_l(sqrtl(x * x + y * y + z * z), (long double)eps, ps);
        D1 = ps[0]; D3 = ps[1];
      } else {
        long double r2 = x * x + y * y + z * z + e2;
        D1 = 1.0L / sqrtl(r2);
        D3 = D1 * D1 * D1;
      }
      ax -= mass[j] * D3 * x; ay -= mass[j] * D3 * y; az -= mass[j] * D3 * z;
      ph -= mass[j] * D1;
    }
    for (int64_t j = 0; j < nx; ++j) {
      double ep = xeps[j] > eps ? xeps[j] : eps;
      long double x = xi - xpos[3 * j], y = yi - xpos[3 * j + 1], z = zi - xpos[3 * j + 2];
      long double D1, D3;
      if (soft) {
        long double ps[2];
        or_spline_psi_l(sqrtl(x * x + y * y + z * z), (long double)ep, ps);
        D1 = ps[0]; D3 = ps[1];
      } else {
        long double r2 = x * x + y * y + z * z + (long double)ep * (long double)ep;
        D1 = 1.0L / sqrtl(r2);
        D3 = D1 * D1 * D1;
      }
      ax -= xmass[j] * D3 * x; ay -= xmass[j] * D3 * y; az -= xmass[j] * D3 * z;
      ph -= xmass[j] * D1;
    }
    acc[3 * t] = (double)(G * ax); acc[3 * t + 1] = (double)(G * ay);
    acc[3 * t + 2] = (double)(G * az);
    pot[t] = (double)(G * ph);
  }
}

/* ---------------------------------------------------------------------- */
/* Direct pair forces in double between a source set and a target set       */
/* (Sec. 2: perturber <-> chain-member forces; SMBH <-> star forces), pair  */
/* softening max(eps_i, eps_j).  When the sets are the same (self != 0) the */
/* pair i == j is skipped.  Sources summed in index order.  If accumulate, */
/* the result is added to acc/pot, else it overwrites them.  soft = 1: the  */
/* cubic spline with h = max(eps_i, eps_j) (h = 0: Newtonian).              */
/* ---------------------------------------------------------------------- */
void or_direct_pairs(const double *spos, const double *sm, const double *seps,
                     int64_t ns, const double *tpos, const double *teps,
                     int64_t nt, int self, double G, int accumulate,
                     double *acc, double *pot, int32_t soft) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nt; ++i) {
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    for (int64_t j = 0; j < ns; ++j) {
      if (self && i == j) continue;
      double ep = seps[j] > teps[i] ? seps[j] : teps[i];
      double x = tpos[3 * i] - spos[3 * j], y = tpos[3 * i + 1] - spos[3 * j + 1],
             z = tpos[3 * i + 2] - spos[3 * j + 2];
      double D1, D3;
      if (soft) {
        double ps[4];
        or_spline_psi(sqrt(x * x + y * y + z * z), ep, ps);
        D1 = ps[0]; D3 = ps[1];
      } else {
        double r2 = x * x + y * y + z * z + ep * ep;
        D1 = 1.0 / sqrt(r2);
        D3 = D1 * D1 * D1;
      }
      ax -= G * sm[j] * D3 * x; ay -= G * sm[j] * D3 * y; az -= G * sm[j] * D3 * z;
      ph -= G * sm[j] * D1;
    }
    if (accumulate) {
      acc[3 * i] += ax; acc[3 * i + 1] += ay; acc[3 * i + 2] += az; pot[i] += ph;
    } else {
      acc[3 * i] = ax; acc[3 * i + 1] = ay; acc[3 * i + 2] = az; pot[i] = ph;
    }
  }
}

/* ---------------------------------------------------------------------- */
/* Leapfrog (Sec. 2, hybrid step (6); READING: kick-drift-kick).            */
/* kick: v += a * h for the listed particles (all when idx == NULL), where  */
/*   h = dt/2 for a global step, or h = (dt_max * 2^-level_i)/2 per         */
/*   particle when level != NULL.  drift: x += v * dt for every particle.   */
/* ---------------------------------------------------------------------- */
void or_kick(double *vel, const double *acc, const int32_t *idx, int64_t n,
             const uint8_t *level, double dt) {
  for (int64_t t = 0; t < n; ++t) {
    int64_t i = idx ? idx[t] : t;
    double h = level ? ldexp(dt, -(int)level[i]) * 0.5 : dt * 0.5;
    for (int k = 0; k < 3; ++k) vel[3 * i + k] = vel[3 * i + k] + acc[3 * i + k] * h;
  }
}

void or_drift(double *pos, const double *vel, int64_t n, double dt) {
  for (int64_t i = 0; i < 3 * n; ++i) pos[i] = pos[i] + vel[i] * dt;
}

/* ---------------------------------------------------------------------- */
/* Block time-step levels (Sec. 2, steps (1) and (7); Sec. 3 for tau).      */
/* READING of the acceleration criterion dt_i = tau_i sqrt(eps/|a_i|):      */
/* level l_i = the smallest l in 0..nlev-1 with dt_max 2^-l <= dt_i, else   */
/* nlev-1.  Decided without square roots on the equivalent                  */
/*   (dt_l^2)^2 * |a|^2 <= (tau^2)^2 * eps^2,  |a|^2 = ax^2 + ay^2 + az^2.  */
/* At substep k (counted in units of the smallest step) a particle may     */
/* only take a level whose step divides k: l >= lmin(k), the smallest l    */
/* with k mod 2^(nlev-1-l) == 0.  tau4eps2[i] = (tau_i^2)^2 * eps^2.  Only  */
/* the listed (active) particles are updated.                               */
/* ---------------------------------------------------------------------- */
/* Levels with an optional velocity criterion (READING: the VINE criterion  */
/* dt_vel = tau_vel eps / |v|, the paper quoting tau_vel beside tau_acc).    */
/* A level c is admissible iff (dt_c^2)^2 |a|^2 <= tau4eps2[i] and, with     */
/* vel, dt_c^2 |v|^2 <= tau2eps2v[i]; the particle takes the smallest        */
/* admissible level (else the finest), raised to the coarsest one whose step */
/* divides k.                                                                */
void or_levels_v(const double *acc, const double *vel, const double *tau4eps2,
                 const double *tau2eps2v, const int32_t *idx, int64_t n,
                 double dt_max, int32_t nlev, int64_t k, uint8_t *level) {
  int lmin = 0;
  while (lmin < nlev - 1 && (k % ((int64_t)1 << (nlev - 1 - lmin))) != 0) ++lmin;
  for (int64_t t = 0; t < n; ++t) {
    int64_t i = idx ? idx[t] : t;
    double a2 = acc[3 * i] * acc[3 * i] + acc[3 * i + 1] * acc[3 * i + 1] +
                acc[3 * i + 2] * acc[3 * i + 2];
    double v2 = 0.0;
    if (vel)
      v2 = vel[3 * i] * vel[3 * i] + vel[3 * i + 1] * vel[3 * i + 1] +
           vel[3 * i + 2] * vel[3 * i + 2];
    int l = nlev - 1;
    for (int c = 0; c < nlev; ++c) {
      double dl = ldexp(dt_max, -c);
      double d2 = dl * dl;
      if (d2 * d2 * a2 <= tau4eps2[i] && (!vel || d2 * v2 <= tau2eps2v[i])) { l = c; break; }
    }
    if (l < lmin) l = lmin;
    level[i] = (uint8_t)l;
  }
}

void or_levels(const double *acc, const double *tau4eps2, const int32_t *idx,
               int64_t n, double dt_max, int32_t nlev, int64_t k,
               uint8_t *level) {
  or_levels_v(acc, 0, tau4eps2, 0, idx, n, dt_max, nlev, k, level);
}

/* Particles active at substep k: k mod 2^(nlev-1-level) == 0, in index    */
/* order.  Returns the count.                                               */
int64_t or_active_at(const uint8_t *level, int64_t n, int32_t nlev, int64_t k,
                     int32_t *idx) {
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i)
    if ((k % ((int64_t)1 << (nlev - 1 - level[i]))) == 0) idx[m++] = (int32_t)i;
  return m;
}
