/*
 * tg.h -- C ABI of libtg.so: softened Barnes-Hut tree gravity on one MI355X
 * (gfx950), after the tree part of the hybrid tree + chain-regularisation
 * code of Karl, Aarseth, Naab, Haehnelt & Spurzem (rVINE).
 *
 * What the library computes (paper passages):
 *   - gravity of distant groups of particles from a multipole expansion about
 *     the group's centre of mass, near particles summed directly (Sec. 1 and
 *     the list of integration regions in Sec. 2);
 *   - Plummer-softened pair forces (Sec. 3, softening paragraph);
 *   - forces only for the active particles of a block-time-step scheme, a
 *     leapfrog integrator, and FP64 direct forces between the SMBHs/chain
 *     members and nearby stars (Sec. 2, the hybrid time-step steps (1), (6),
 *     (7) and the perturber force-correction paragraph).
 * Readings where the paper is silent: an octree over 21-bit Morton keys, a
 * geometric opening angle theta (cell side s, distance d from the target
 * group's box to the cell's centre of mass, accept iff s^2 < theta^2 d^2),
 * monopole + quadrupole moments with the softened expansion
 *   a += G(-M D3 x + D5 Q x - 2.5 D7 W x),  phi += G(-M D1 - 0.5 D5 W),
 *   x = x_i - com, D_n = (|x|^2 + eps^2)^(-n/2), Q = 3S - tr(S) I,
 *   W = x.Q.x - tr(S) eps^2,
 * and kick-drift-kick leapfrog with power-of-two block levels.
 *
 * Conventions for every entry point:
 *   - Pointers named *_dev are device (HBM) pointers, owned by the caller and
 *     only read or written during the call's stream work.  Pointers named
 *     *_host are host memory, read before the call returns.
 *   - Positions, velocities and accelerations are row-major [n][3] doubles in
 *     the caller's particle order; outputs come back in that order.
 *   - All work is enqueued asynchronously on the context's stream; nothing is
 *     synchronised unless stated.  tg_sync() waits and reports device-side
 *     errors.
 *   - Every function returns TG_OK or a negative tg_status; tg_last_error()
 *     gives the message of the last failure on the calling thread.  Argument
 *     errors are detected on the host before anything is enqueued.
 *   - A context allocates all of its device memory in tg_create(); no later
 *     call allocates, so any sequence of calls between tg_graph_begin() and
 *     tg_graph_end() can be captured into a HIP graph and replayed.
 *   - One context per stream and per host thread at a time.
 */
#ifndef TG_H
#define TG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TG_OK = 0,
  TG_EINVAL = -1,     /* bad argument (NULL pointer, size, range) */
  TG_ENOMEM = -2,     /* device allocation failed in tg_create, or a host allocation */
  TG_EHIP = -3,       /* a HIP runtime call failed */
  TG_ECAPACITY = -4,  /* a capacity given at tg_create was exceeded */
  TG_ESTATE = -5,     /* call out of order (e.g. forces before a tree) */
  TG_EDATA = -6,      /* device found non-finite positions or mass <= 0 */
  TG_EINTERNAL = -7   /* a bounded device-side wait gave up (TG_ERR_SORT) */
} tg_status;

typedef enum { TG_FP64 = 0, TG_MIXED = 1 } tg_precision;

/* Device error bits reported through tg_sync() / tg_error_bits(). */
#define TG_ERR_NONFINITE   0x1u  /* a position is NaN or infinite */
#define TG_ERR_MASS        0x2u  /* a mass is <= 0 or not finite */
#define TG_ERR_NODES       0x4u  /* octree needed more than max_nodes */
#define TG_ERR_FRONTIER    0x8u  /* walk frontier exceeded frontier_cap */
#define TG_ERR_LISTS       0x10u /* list dump exceeded its capacity */
#define TG_ERR_SORT        0x20u /* a radix-sort tile waited too long for its predecessor */
#define TG_ERR_CHAIN       0x40u /* a selection (perturbers, radius) exceeded its capacity */

typedef struct {
  int64_t max_particles;   /* capacity N for every call (>= 1) */
  int32_t max_systems;     /* capacity of independent systems S (1..256) */
  int32_t leaf_size;       /* n_L: a node with more particles is refined (1..16) */
  int32_t group_size;      /* n_G: particles sharing one walk (1..128) */
  int32_t precision;       /* tg_precision of the walk and P2P/P2M sums */
  int64_t max_nodes;       /* octree node capacity; 0 = 2 * max_particles + 64 * max_systems */
  int32_t frontier_cap;    /* walk frontier per wave and level, in 32-bit words
                              (an opened cell takes two); 0 = 16384 */
  int32_t waves_per_cu;    /* resident walk waves per compute unit; 0 = 16 */
  double G;                /* gravitational constant (paper units: 1) */
  int32_t key_levels;      /* octree depth: 21 (0 = 21) or 42.  42 levels quantise
                              coordinates to 42 bits and keep the 126-bit key as
                              two words (the first 21 digits are the 21-level
                              key), for escapers and untruncated initial
                              conditions that 21 levels leave in over-full
                              leaves; it costs a second 8-pass sort and 16 more
                              bytes per particle.  The relative opening test and
                              refit take 21-level trees (TG_EINVAL with 42). */
} tg_config;

typedef struct tg_ctx tg_ctx;

/* Fill *cfg with defaults: N = 1, S = 1, n_L = 8, n_G = 64, FP64, G = 1. */
void tg_default_config(tg_config *cfg);

/* Create a context on the current HIP device, working on `stream`
 * (a hipStream_t; NULL = the default stream).  Allocates every device
 * buffer for the capacities in *cfg.  Errors: TG_EINVAL, TG_ENOMEM, TG_EHIP. */
tg_status tg_create(const tg_config *cfg, void *stream, tg_ctx **out);

/* Free the context and its device memory (waits for its stream first). */
void tg_destroy(tg_ctx *ctx);

/* Use another stream for subsequent work. */
tg_status tg_set_stream(tg_ctx *ctx, void *stream);

/* Change n_L / n_G between builds (n_G also applies to tg_tree_forces);
 * bounds as in tg_config.  Takes effect at the next tg_build_tree. */
tg_status tg_set_sizes(tg_ctx *ctx, int32_t leaf_size, int32_t group_size);

/* ---- cube, Morton keys, radix sort, gather, octree, groups -----------
 * Builds the octree of N particles split into S independent systems, the
 * contiguous ranges sys_off_host[s] .. sys_off_host[s+1] (NULL with S = 1
 * means one system [0, N)).  One root per non-empty system; a node with
 * more than n_L particles below level 21 is refined into its non-empty
 * octants; node ids are breadth first with children in octant order.
 * Non-finite positions set TG_ERR_NONFINITE (reported by tg_sync).
 * N = 0 is allowed (empty tree).  Errors: TG_EINVAL (N > capacity, S out of
 * range, offsets not ascending), TG_ESTATE (system layout changed during
 * graph capture). */
tg_status tg_build_tree(tg_ctx *ctx, const double *pos_dev, int64_t n,
                        const int64_t *sys_off_host, int32_t n_sys);

/* ---- monopole + quadrupole moments about each node's centre of mass
 * (upward pass; leaves from their particles, internal nodes from children).
 * mass_dev: [N] doubles, caller order, each > 0 (else TG_ERR_MASS).
 * Requires a tree.  Errors: TG_ESTATE. */
tg_status tg_compute_moments(tg_ctx *ctx, const double *mass_dev);

/* ---- refit: update the tree without rebuilding it (Sec. 2 step 7) -----
 * For the particles of the last tg_build_tree (same n and systems), moved:
 * keeps the sort order, nodes and groups of that build, gathers the current
 * positions and masses (caller order, as for the build; masses > 0, else
 * TG_ERR_MASS; non-finite positions set TG_ERR_NONFINITE), recomputes the
 * moments, and gives each node the opening size
 *   s' = max(s, 2 e),  e = max_k max(hi_k - g_k, g_k - lo_k),
 * [lo, hi] the bounding box of the node's particles, g its cell's centre and
 * s its side: the smallest cube about the centre that holds the cell and all
 * its particles (READING of Sec. 2 step 7, which updates the tree only when
 * needed).
 * Both opening tests use s' until the next tg_build_tree; a cell holding a
 * target is still never accepted.  Replaces tg_compute_moments.
 * Errors: TG_EINVAL, TG_ESTATE (no tree). */
tg_status tg_refit_tree(tg_ctx *ctx, const double *pos_dev, const double *mass_dev);

/* ---- group walk with the opening-angle test, P2P and P2M --------------
 * Forces and potentials on the active particles from all particles of their
 * own system.  active_idx_dev: caller-order indices of the targets, int32,
 * distinct, n_active_dev[0] of them (both device; NULL active_idx_dev means
 * all particles).  Rows of acc_dev ([N][3]) and pot_dev ([N], may be NULL)
 * belonging to targets are overwritten; other rows are untouched.  The self
 * pair is excluded.  0 < eps, 0 <= theta < 1/sqrt(3).
 * Errors: TG_EINVAL, TG_ESTATE (no tree or moments). */
tg_status tg_tree_forces(tg_ctx *ctx, double eps, double theta,
                         const int32_t *active_idx_dev,
                         const int32_t *n_active_dev, double *acc_dev,
                         double *pot_dev);

/* ---- relative opening test (alternative to the opening angle) ---------
 * The paper's tree runs open cells with a relative ("Gadget") criterion and
 * an error tolerance (Sec. 3, run set-up) but print no formula; this is the
 * relative criterion of Springel 2005 (MNRAS 364, 1105, Sec. 3.1) for a
 * group of targets: a cell of mass M and side s is accepted iff
 *   (G M s^2)^2 <= alpha^2 min|a_old|^2 d^8
 * with d the distance from the group's box of active targets to the cell's
 * centre of mass and the minimum over those targets, and the box misses the
 * cell's cube enlarged by 20 % about its geometric centre (the cube with
 * corner lo + i s for integer cell coordinates i).  All in FP64 with every
 * operation rounded separately.
 * kind TG_MAC_GEOMETRIC (the default) restores the opening angle;
 * TG_MAC_RELATIVE makes every later tg_tree_forces, tg_walk_lists and
 * tg_forces (hence the steps) use it with tolerance alpha (finite, >= 0;
 * the paper's runs use 1e-3) and theta is ignored.  acc_old_dev: [N][3]
 * doubles, caller order, finite, read at walk time (before any output row
 * is written, so it may be the acc_dev of the same call); NULL makes
 * tg_forces use the system's acc and tg_tree_forces / tg_walk_lists fail
 * with TG_ESTATE.  A zero old acceleration opens every cell of its group
 * (the first evaluation of a run should use the opening angle).
 * Errors: TG_EINVAL. */
#define TG_MAC_GEOMETRIC 0
#define TG_MAC_RELATIVE 1
tg_status tg_set_mac(tg_ctx *ctx, int32_t kind, double alpha,
                     const double *acc_old_dev);

/* Pair softening for everything the context computes afterwards: the walk's
 * particle and cell terms, the SMBH terms of tg_forces and the steps, and
 * tg_direct_fp64.  The tree may use spline or Plummer softening (Sec. 2,
 * the tree part of the hybrid scheme).
 *   TG_SOFT_PLUMMER (the default): pair potential -G m / sqrt(r^2 + eps^2).
 *   TG_SOFT_SPLINE: the cubic-spline kernel of Monaghan & Lattanzio (1985)
 *     with support 2h, h = eps (pairs with an SMBH: h = max(eps_i, eps_j)),
 *     as used for gravity by Hernquist & Katz (1989): with u = r/h the pair
 *     potential is -G m psi(r), psi = (7/5 - 2/3 u^2 + 3/10 u^4 - 1/10 u^5)/h
 *     for u < 1, (8/5 - 4/3 u^2 + u^3 - 3/10 u^4 + 1/30 u^5 - 1/(15 u))/h
 *     for 1 <= u < 2, and 1/r beyond (h = 0: Newtonian).  Cells use the
 *     second-order expansion of the same kernel about their centre of mass
 *     (psi and its derivatives psi_k+1 = -(1/r) d psi_k / dr).
 * The chain-coupling kernels keep their own softening (tg_chain).  Errors:
 * TG_EINVAL for another kind. */
#define TG_SOFT_PLUMMER 0
#define TG_SOFT_SPLINE 1
tg_status tg_set_softening(tg_ctx *ctx, int32_t kind);

/* Interaction counts (synchronises the stream).  out[0..3] for the last
 * tg_tree_forces: P2P pairs (target, source particle, j != i), particle-cell
 * (P2M) pairs, targets, active groups walked; out[4..7] the same summed over
 * every tg_tree_forces since the context was created or tg_reset_counts. */
tg_status tg_get_counts(tg_ctx *ctx, int64_t out[8]);
tg_status tg_reset_counts(tg_ctx *ctx);

/* Parity/diagnostic mode of the walk: for every active group (ordered by
 * its first particle, as numbered by the groups of the current tree) write
 * its P2M cell ids and P2P leaf ids (unsorted, node ids of the current
 * tree).  group_info_dev: [cap_groups][4] int64 = group index, P2M offset,
 * P2M count, P2P count (P2P ids follow the P2M ids of the same group);
 * ids_dev: [cap_ids] uint32.  Synchronises; *n_groups_out and *n_ids_out get
 * the sizes (if larger than the caps nothing beyond the caps is written and
 * TG_ECAPACITY is returned). */
tg_status tg_walk_lists(tg_ctx *ctx, double theta,
                        const int32_t *active_idx_dev,
                        const int32_t *n_active_dev, int64_t *group_info_dev,
                        int64_t cap_groups, uint32_t *ids_dev, int64_t cap_ids,
                        int64_t *n_groups_out, int64_t *n_ids_out);

/* ---- double-precision direct forces (SMBH <-> stars, perturber <->
 * chain members; Sec. 2).  Targets [nt] at tgt_pos_dev with softening
 * tgt_eps_dev feel sources [ns] (src_pos_dev, src_mass_dev, src_eps_dev)
 * with pair softening max(eps_i, eps_j), Plummer or the cubic spline as set
 * by tg_set_softening (0: Newtonian).  With segments (nseg > 0,
 * src_seg_host/tgt_seg_host ascending offsets [nseg+1]) only pairs in the
 * same segment interact.  If self_pairs != 0 the two sets are the same
 * particles and i == j is skipped.  accumulate != 0 adds to acc/pot, else
 * overwrites.  pot_dev may be NULL.  Sums are compensated (double-double
 * style Neumaier) and deterministic. */
tg_status tg_direct_fp64(tg_ctx *ctx, const double *src_pos_dev,
                         const double *src_mass_dev, const double *src_eps_dev,
                         int64_t ns, const double *tgt_pos_dev,
                         const double *tgt_eps_dev, int64_t nt,
                         const int64_t *src_seg_host,
                         const int64_t *tgt_seg_host, int32_t nseg,
                         int32_t self_pairs, int32_t accumulate,
                         double *acc_dev, double *pot_dev);

/* ---- the same direct forces with no allocation at all ----------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sums
 * of tg_direct_fp64 with no context.  It calls no hipMalloc, hipFree or
 * other allocating routine; its scratch (the segment table and the
 * per-block compensated partial sums) is one fixed device array inside the
 * library, TG_NOALLOC_SCRATCH_BYTES long, which each GPU that calls it holds
 * until the process ends.  Arguments as for tg_direct_fp64, plus
 * softening (TG_SOFT_PLUMMER or TG_SOFT_SPLINE, pair h = max(eps_i, eps_j))
 * and stream (a hipStream_t of the current HIP device; NULL = the default
 * stream); the work is enqueued on that stream and nothing is synchronised.
 * The partial sums have the capacity of a context's, so the results equal
 * tg_direct_fp64's bit for bit.  Nothing in the scratch needs clearing:
 * every call writes what it reads.  Every call on one GPU shares that GPU's
 * array, so calls that overlap on one GPU (other streams, other host
 * threads) race: order them.  Errors (on the host, before any work):
 * TG_EINVAL as tg_direct_fp64, TG_ECAPACITY for nseg > TG_NOALLOC_MAX_SEG,
 * TG_EHIP if the scratch address or a launch fails; tg_last_error gives the
 * message without allocating. */
#define TG_NOALLOC_MAX_SEG 64
#define TG_NOALLOC_SCRATCH_BYTES (4096 + 8 * 8 * 131072)
tg_status tg_direct_fp64_noalloc(const double *src_pos_dev,
                                 const double *src_mass_dev,
                                 const double *src_eps_dev, int64_t ns,
                                 const double *tgt_pos_dev,
                                 const double *tgt_eps_dev, int64_t nt,
                                 const int64_t *src_seg_host,
                                 const int64_t *tgt_seg_host, int32_t nseg,
                                 int32_t self_pairs, int32_t accumulate,
                                 int32_t softening, double *acc_dev,
                                 double *pot_dev, void *stream);

/* ---- leapfrog (kick-drift-kick) and block time-steps ------------------
 * kick: v += a h for the listed particles (all n when active_idx_dev is
 * NULL; then n_active_dev is ignored and n gives the count).  h = dt / 2,
 * or with level_dev != NULL, h = (dt * 2^-level_i) / 2 with dt = dt_max.
 * If skip_at_k0 != 0 and k_dev[0] == 0 the kick is skipped (the closing
 * half-kick of the first block step). */
tg_status tg_kick(tg_ctx *ctx, double *vel_dev, const double *acc_dev,
                  int64_t n, const int32_t *active_idx_dev,
                  const int32_t *n_active_dev, const uint8_t *level_dev,
                  double dt, const int64_t *k_dev, int32_t skip_at_k0);

/* drift: x += v dt for all n particles. */
tg_status tg_drift(tg_ctx *ctx, double *pos_dev, const double *vel_dev,
                   int64_t n, double dt);

/* Block levels of the listed particles at substep k_dev[0]: the smallest l
 * in 0..nlev-1 with dt_max 2^-l <= tau_i sqrt(eps_i/|a_i|), decided as
 * (dt_l^2)^2 |a|^2 <= tau4eps2_dev[i] = (tau_i^2)^2 eps_i^2, else nlev-1;
 * then raised to the smallest level whose step divides k. */
tg_status tg_levels(tg_ctx *ctx, const double *acc_dev,
                    const double *tau4eps2_dev, int64_t n,
                    const int32_t *active_idx_dev,
                    const int32_t *n_active_dev, double dt_max, int32_t nlev,
                    const int64_t *k_dev, uint8_t *level_dev);

/* As tg_levels, with the velocity criterion dt_vel = tau_vel eps / |v| as
 * well (a reading of the VINE criterion the paper sets tau_vel for, Sec. 3):
 * a level is admissible only if also dt_l^2 |v|^2 <= tau2eps2v_dev[i] =
 * tau_vel,i^2 eps_i^2.  vel_dev [n][3] and tau2eps2v_dev [n] are both given
 * or both NULL (NULL: tg_levels). */
tg_status tg_levels_v(tg_ctx *ctx, const double *acc_dev, const double *vel_dev,
                      const double *tau4eps2_dev, const double *tau2eps2v_dev,
                      int64_t n, const int32_t *active_idx_dev,
                      const int32_t *n_active_dev, double dt_max, int32_t nlev,
                      const int64_t *k_dev, uint8_t *level_dev);

/* Indices (ascending) of the particles active at substep k_dev[0] + k_add:
 * (k mod 2^(nlev-1-level_i)) == 0.  Writes idx_dev[0..m) and n_out_dev[0]=m. */
tg_status tg_active_set(tg_ctx *ctx, const uint8_t *level_dev, int64_t n,
                        int32_t nlev, const int64_t *k_dev, int32_t k_add,
                        int32_t *idx_dev, int32_t *n_out_dev);

/* k_dev[0] += inc (device-side substep counter for replayed graphs). */
tg_status tg_counter_add(tg_ctx *ctx, int64_t *k_dev, int64_t inc);

/* ---- direct forces inside the walk: SMBHs as external point masses ----
 * Register n_ext point masses (device arrays pos [n_ext][3], mass, eps) whose
 * FP64 Plummer force, pair softening max(eps, eps_ext), every later
 * tg_tree_forces adds to each target of the same system (seg_host [n_sys+1]
 * ascending offsets into the externals; NULL with n_sys = 1 means all).
 * The arrays are read at walk time, so new positions need no new call.
 * n_ext = 0 clears them.  n_ext <= 1024.  Errors: TG_EINVAL, TG_ESTATE (a
 * new segment table during graph capture). */
tg_status tg_set_external(tg_ctx *ctx, const double *pos_dev,
                          const double *mass_dev, const double *eps_dev,
                          int32_t n_ext, const int64_t *seg_host, int32_t n_sys);

/* ---- chain coupling (Sec. 2, the hybrid method) ------------------------
 * The stars near an SMBH that the regularised chain integrates ("members",
 * at most 256, owned and advanced by the caller's chain integrator) act on
 * the tree particles, and feel them, through these calls.  All arrays are
 * device memory in the caller's order unless marked host. */
typedef struct {
  const double *pos;          /* [n][3] tree particles (stars) */
  const double *mass;         /* [n] */
  int64_t n;                  /* 0..max_particles */
  const uint8_t *exclude;     /* [n] nonzero: not coupled (ghost members); NULL: none */
  const double *member_pos;   /* [nc][3] chain members, global frame */
  const double *member_mass;  /* [nc] */
  int32_t nc;                 /* 1..256 */
  double com[3];              /* host: the chain's centre of mass R */
  double m_chain;             /* host: the chain's mass M (sum of member masses), > 0 */
  double r_crit, gamma_crit;  /* Eq. 2: r_crit = min(r_chain, r_chain,0) >= 0, gamma_crit > 0 */
  double eps_pm;              /* Plummer softening of perturber-member pairs (0: Newtonian) */
  int32_t *pert_idx;          /* [pert_cap] out: perturbers, ascending */
  int32_t pert_cap;
  int32_t *n_pert;            /* [1] out: perturber count (may exceed pert_cap) */
} tg_chain;

/* Perturbers by the tidal criterion (Eq. 2): star j perturbs the chain iff
 * |x_j - R| < ((2 / gamma_crit) (m_j / M))^(1/3) r_crit, decided without
 * roots as (r2 r2) r2 < (k k) rc6, k = (2 / (gamma_crit M)) m_j,
 * rc6 = (r_crit^2 r_crit^2) r_crit^2, r2 = (dx dx + dy dy) + dz dz, every
 * operation rounded separately.  Excluded stars are never perturbers.
 * Writes the ascending list (at most pert_cap entries) and the count; a
 * count above pert_cap sets TG_ERR_CHAIN (tg_sync: TG_ECAPACITY).
 * Errors: TG_EINVAL. */
tg_status tg_perturbers(tg_ctx *ctx, const tg_chain *chain);

/* Selects the perturbers (as tg_perturbers), then adds the coupling forces:
 *  - acc_dev / pot_dev ([n][3], [n] or NULL) of each listed star
 *    (active_idx_dev / n_active_dev as in tg_tree_forces, NULL = all), if not
 *    excluded: a perturber gets the force of every member (pair softening
 *    eps_pm), any other star the Newtonian force of the chain particle (mass
 *    M at R), which stands for the chain in the tree (Sec. 2);
 *  - member_acc_dev ([nc][3], overwritten): the force of the perturbers on
 *    each member (the chain integration's external perturbation);
 *  - com_acc_dev ([3], overwritten): the force on the chain particle, the
 *    Newtonian force of every non-perturber, non-excluded star plus the
 *    correction of Eq. 3, (1 / M) sum_i m_i member_acc_i.
 * Sums are compensated where they run over stars; deterministic.  acc is
 * added to (call after the tree forces of the same positions).
 * Errors: TG_EINVAL. */
tg_status tg_chain_forces(tg_ctx *ctx, const tg_chain *chain,
                          const int32_t *active_idx_dev, const int32_t *n_active_dev,
                          double *acc_dev, double *pot_dev, double *com_acc_dev,
                          double *member_acc_dev);

/* Several chains at once (the extension to several distant SMBHs that the
 * paper names as its next step, Sec. 7), READING: every chain couples to
 * the stars exactly as tg_chain_forces does for one, with the same star
 * arrays and one exclusion mask that holds the ghost members of all chains;
 * a star may perturb several chains.  The chain particles feel each other
 * as Newtonian point masses (M_d at R_d), added to their com_acc; members
 * feel other chains only through their chain particle.
 *   chains: host [n_chains] (1..16), sharing pos, mass, n and exclude, each
 *     with its own perturber list;
 *   com_acc_dev: [n_chains][3] overwritten;
 *   member_acc_dev: [sum nc][3] overwritten, the chains' members in order;
 *   acc_dev / pot_dev / active list as in tg_chain_forces (added to).
 * Errors: TG_EINVAL (also for two chains with the same centre). */
tg_status tg_chains_forces(tg_ctx *ctx, const tg_chain *chains, int32_t n_chains,
                           const int32_t *active_idx_dev, const int32_t *n_active_dev,
                           double *acc_dev, double *pot_dev, double *com_acc_dev,
                           double *member_acc_dev);

/* The perturbers of the last tg_perturbers / tg_chain_forces on this chain
 * (pert_idx, n_pert), relative to the chain particle and predicted to first
 * order in time for the chain integration (Sec. 2: perturber positions are
 * predicted relative to the chain particle at each chain force evaluation):
 * row k < min(n_pert, pert_cap), j = pert_idx[k]:
 *   out_pos[k] = (x_j + v_j dt) - (R + V dt),  out_vel[k] = v_j - V,
 *   out_mass[k] = m_j (out_mass may be NULL),
 * V = com_vel (host [3]), R + V dt formed on the host; each operation rounded
 * separately.  vel_dev: [n][3] star velocities; outputs [pert_cap][3] device.
 * Rows beyond the count are untouched; a listed index outside [0, n) (a
 * list not selected from these stars) gives a NaN row.  Errors: TG_EINVAL. */
tg_status tg_predict_perturbers(tg_ctx *ctx, const tg_chain *chain, const double *vel_dev,
                                const double com_vel[3], double dt, double *out_pos_dev,
                                double *out_vel_dev, double *out_mass_dev);

/* Stars within radius r of center (host [3]): |x - c|^2 < r r, the chain
 * start around an SMBH (r_chain,0) and absorption into the chain (Eq. 4,
 * r_chain about R).  Ascending indices (at most cap) and the count in
 * n_out_dev[0]; a count above cap sets TG_ERR_CHAIN.  Errors: TG_EINVAL. */
tg_status tg_select_within(tg_ctx *ctx, const double *pos_dev, int64_t n,
                           const uint8_t *exclude_dev, const double center[3], double r,
                           int32_t *idx_dev, int32_t cap, int32_t *n_out_dev);

/* ---- AR-chain integrator (host, FP64; Sec. 2) --------------------------
 * The chain members are integrated in the chain's centre-of-mass frame by
 * algorithmic regularization: the logarithmic-Hamiltonian time-transformed
 * leapfrog (Mikkola & Tanikawa 1999; Preto & Tremaine 1999) with
 * Bulirsch-Stoer extrapolation (Mikkola & Aarseth 2002), which follows
 * close and colliding encounters without softening.  The integrated
 * variables are the chain vectors (Sec. 2: the chain of inter-particle
 * vectors, Mikkola & Aarseth 1990, 1993): with the members ordered along a
 * chain c[0..n-1], X_k = x_c[k+1] - x_c[k] and W_k = v_c[k+1] - v_c[k].
 * Pairs one or two links apart take their separation from the chain
 * vectors, so a close pair keeps its digits wherever it sits; the chain is
 * built by the members' mutual forces (Sec. 2: sorted by gravitational
 * force, not distance): the strongest pair first, then at either end the
 * member pulled hardest by that end.  It is rebuilt before every
 * extrapolated step from sums of the old chain vectors.  All arrays are
 * HOST memory; nothing here touches the GPU. */
typedef struct {
  int32_t n;                  /* members, 2..256 */
  double *x, *v;              /* [n][3] centre-of-mass frame (in/out) */
  const double *m;            /* [n] > 0 */
  double t;                   /* physical time (in/out) */
  double B;                   /* binding energy U - T plus the perturbers' work (in/out; set by init) */
  double ds;                  /* fictitious step suggestion (in/out; <= 0 before init: chosen) */
  /* Optional chain state kept between calls (NULL: none).  With chain_valid
   * nonzero, init, advance and energy start from chain / cx / cv instead
   * of x, v (which are then outputs only); every call that has the arrays
   * writes them and sets chain_valid.  A caller that changes x, v (new
   * members) clears chain_valid. */
  int32_t *chain;             /* [n] member indices in chain order */
  double *cx, *cv;            /* [n-1][3] chain vectors X_k, W_k */
  int32_t chain_valid;
} tg_archain;

/* Perturbers as point masses moved to first order, y(t) = x + v (t - t0),
 * relative to the chain's centre of mass (e.g. from tg_predict_perturbers
 * with dt = 0); the members feel their tidal part (the mean acceleration is
 * removed, as the centre of mass is the tree's chain particle). */
typedef struct {
  int32_t np;
  const double *x, *v, *m;    /* [np][3], [np][3], [np] */
  double t0;
} tg_archain_perturbers;

/* Sets B = U - T (and ds if <= 0).  Errors: TG_EINVAL (n, masses, G,
 * coincident members). */
tg_status tg_archain_init(tg_archain *chain, double G);

/* Advances the members by physical time dt (>= 0) to relative accuracy tol
 * per extrapolated step; perturbers may be NULL.  The last step is searched
 * so that t ends at t + dt.  *steps_out (may be NULL) gets the number of
 * extrapolated steps.  Errors: TG_EINVAL, TG_EINTERNAL (step underflow). */
tg_status tg_archain_advance(tg_archain *chain, double G, double dt, double tol,
                             const tg_archain_perturbers *perturbers, int64_t *steps_out);

/* Relative energy bookkeeping error (T - U + B) / U of the chain (0 when the
 * integration and the work of the perturbers balance exactly). */
tg_status tg_archain_energy(const tg_archain *chain, double G, double *err_out);

/* Chain membership after a chain step (host; Sec. 2, Eq. 4 and 5; the
 * absorption-first rule of Sec. 4).  READING:
 *  - absorption (Eq. 4): perturber p joins if |px_p|^2 < r_chain^2, px
 *    relative to the chain's centre of mass (e.g. tg_predict_perturbers
 *    with dt = 0), r_chain the largest member distance in the last chain
 *    step;
 *  - escape (Eq. 5): member i leaves if |x_i|^2 > (gamma r_chain0)^2 and
 *    x_i . v_i > 0 (it recedes; the paper takes gamma = 1.5);
 *  - while some perturber joins, escapes wait unless r_chain > 1.05 gamma
 *    r_chain0;
 *  - the chain ends if fewer than two members would remain, or if the
 *    designated massive member leaves and no other massive member stays;
 *    otherwise the most massive remaining massive member (ties: the lowest
 *    index) takes over as the chain's centre particle.
 * Squares and dot products are summed x, y, z in order with every operation
 * rounded on its own.  All arrays are HOST memory; the caller applies the
 * result (ghost flags, masses, frames). */
typedef struct {
  int32_t n;                  /* members, 1..256 */
  const double *x, *v;        /* [n][3] relative to the centre of mass */
  const double *m;            /* [n] */
  const uint8_t *massive;     /* [n] nonzero: a designated massive particle (SMBH) */
  int32_t designated;         /* the member that is the chain's centre particle */
  double r_chain, r_chain0, gamma;
  int32_t np;                 /* perturbers */
  const double *px;           /* [np][3] relative to the centre of mass */
} tg_membership_in;

typedef struct {
  int32_t *absorb;            /* [np] out: rows of px that join, ascending */
  int32_t n_absorb;
  int32_t *escape;            /* [n] out: members that leave, ascending */
  int32_t n_escape;
  int32_t terminate;          /* 1: the chain ends (all members back to the tree) */
  int32_t designated;         /* the centre particle afterwards, -1 when it ends */
} tg_membership_out;

tg_status tg_chain_membership(const tg_membership_in *in, tg_membership_out *out);

/* ---- whole steps (every stage above in one call; capturable) ---------- */
typedef struct {
  double *pos, *vel, *acc, *pot;   /* stars [n][3], pot [n] may be NULL */
  const double *mass;              /* [n] */
  int64_t n;
  const int64_t *sys_off;          /* host [n_sys+1], NULL for one system */
  int32_t n_sys;
  double *bh_pos, *bh_vel, *bh_acc, *bh_pot;   /* SMBHs [n_bh][3]; pot may be NULL */
  const double *bh_mass, *bh_eps;              /* [n_bh] */
  int32_t n_bh;
  const int64_t *bh_seg;           /* host [n_sys+1]: SMBHs of each system */
  double eps, theta;               /* star softening, opening angle (see tg_set_mac) */
  const uint8_t *frozen;           /* [n] nonzero: star held still in the steps (a ghost chain
                                      member, Sec. 2: not advanced and never active, so it
                                      sets no time-step; it stays a source of its tiny
                                      mass); NULL: none */
} tg_system;

/* Forces for the listed stars (all when active_idx_dev is NULL): tree +
 * FP64 SMBH terms, and the FP64 forces on every SMBH from the stars and the
 * other SMBHs of its system (Sec. 2: the perturber/chain force hand-off). */
tg_status tg_forces(tg_ctx *ctx, const tg_system *sys,
                    const int32_t *active_idx_dev, const int32_t *n_active_dev);

/* One kick-drift-kick step of length dt for stars and SMBHs (acc must hold
 * the forces of the current positions, e.g. from tg_forces). */
tg_status tg_step_kdk(tg_ctx *ctx, const tg_system *sys, double dt);

/* One drift-kick-drift step (the paper's tree step, Sec. 2 step 6): x += v
 * dt/2, forces at the half step, v += a dt, x += v dt/2, stars and SMBHs.
 * acc holds the half-step forces afterwards. */
tg_status tg_step_dkd(tg_ctx *ctx, const tg_system *sys, double dt);

typedef struct {
  uint8_t *level;                  /* [n] block level of each star */
  const double *tau4eps2;          /* [n] (tau^2)^2 eps^2 per star */
  int32_t *active_idx;             /* [n] scratch: active stars */
  int32_t *n_active;               /* [1] */
  int64_t *k;                      /* [1] substep counter (units of the smallest step) */
  double dt_max;                   /* step of level 0 */
  int32_t nlev;                    /* levels 0..nlev-1; smallest step dt_max 2^-(nlev-1) */
  const double *tau2eps2v;         /* [n] tau_vel^2 eps^2 per star (velocity criterion), or NULL */
  int32_t rebuild_every;           /* > 1: rebuild the tree at substeps k that are multiples of
                                      it and refit it in between (tg_refit_tree); 0, 1: rebuild
                                      at every substep with active stars */
} tg_blocks;

/* One substep of the smallest step: closing half kicks of the stars whose
 * step ends at k (none at k = 0), new levels, opening half kicks, drift of
 * everything, k += 1, forces for the stars active at the new k.  SMBHs take
 * the smallest step every substep.  All counts live on the device, so one
 * captured substep can be replayed. */
tg_status tg_step_block(tg_ctx *ctx, const tg_system *sys, const tg_blocks *blocks);

/* n_sub substeps with the results of n_sub tg_step_block calls, bit for
 * bit, for callers that drive block steps from the host.  Levels change only
 * for active stars, so after each substep the finest level held by a star
 * that is not frozen fixes the next substep at which any star is active
 * (Sec. 2: forces only for the active particles).  The substeps before it
 * run as the SMBHs' kicks and drift, the stars' drift and the SMBH sums,
 * without the tree's launches.  Reads two device words after each substep
 * that has active stars and waits for the stream there, so it cannot be
 * graph-captured (TG_ESTATE during a capture).  n_idle (may be NULL)
 * receives the number of substeps run in the short form.  On return
 * active_idx / n_active hold the active set at the final k, as after
 * tg_step_block. */
tg_status tg_step_blocks(tg_ctx *ctx, const tg_system *sys, const tg_blocks *blocks,
                         int64_t n_sub, int64_t *n_idle);

/* ---- HIP graphs over any sequence of the calls above ------------------ */
typedef struct tg_graph tg_graph;
tg_status tg_graph_begin(tg_ctx *ctx);
tg_status tg_graph_end(tg_ctx *ctx, tg_graph **out);
/* A graph replays the captured kernels with the pointers, sizes and
 * system layout they had, on its context's buffers: launch it only while
 * the context lives (destroying it afterwards is fine).  The context's
 * device tables that a graph reads (system offsets and sort tiles,
 * direct-sum segment tables, external segments) are overwritten by a later
 * eager call with a new layout (a tg_build_tree with other offsets, a
 * segment table that evicts one of the 8 slots, tg_set_external with new
 * segments); tg_graph_launch then returns TG_ESTATE without launching
 * anything, and the step must be captured again. */
tg_status tg_graph_launch(tg_graph *g, void *stream);
void tg_graph_destroy(tg_graph *g);

/* ---- tree inspection (device pointers valid until the next build) ------ */
typedef struct {
  int64_t n, n_nodes, n_groups;
  int32_t n_sys;
  const uint64_t *skeys;     /* [n] sorted keys (42 levels: the first 21 digits) */
  const uint64_t *skeys_lo;  /* [n] 42 levels: the last 21 digits of the sorted keys; else NULL */
  const uint32_t *perm;      /* [n] sorted rank -> caller index */
  const uint8_t *level;      /* [n_nodes] */
  const uint8_t *nchild;     /* [n_nodes] */
  const uint32_t *first;     /* [n_nodes] first sorted particle */
  const uint32_t *count;     /* [n_nodes] */
  const uint32_t *child;     /* [n_nodes] first child id (0 for leaves) */
  const uint32_t *parent;    /* [n_nodes] (0xffffffff for roots) */
  const double *cube;        /* [n_sys][4] lo x, y, z, side */
  const double *com;         /* [n_nodes][4] com x, y, z, side^2 */
  const double *mom;         /* [n_nodes][8] M, Sxx, Syy, Szz, Sxy, Sxz, Syz, 0 */
  const uint32_t *groups;    /* [n_groups][4] first, count, node, system */
} tg_tree_view;

/* Synchronises the stream to read the counts. */
tg_status tg_get_tree(tg_ctx *ctx, tg_tree_view *out);

/* ---- autotuning (n_L, n_G, resident waves) -----------------------------
 * Times build + moments + forces on the given particles for every candidate
 * (leaf sizes x group sizes x waves per CU, 0-terminated lists; NULL = the
 * built-in lists), keeps the fastest in the context and reports it in
 * best[3] = {leaf_size, group_size, waves_per_cu} and *best_ms.  times (may
 * be NULL): host array, one entry per candidate in list order (leaf
 * outermost, waves innermost), the fastest of `repeats` timed runs after
 * one warm-up run, in ms. */
tg_status tg_autotune(tg_ctx *ctx, const double *pos_dev,
                      const double *mass_dev, int64_t n,
                      const int64_t *sys_off_host, int32_t n_sys, double eps,
                      double theta, const int32_t *leaf_list,
                      const int32_t *group_list, const int32_t *waves_list,
                      int32_t repeats, int32_t best[3], double *best_ms,
                      double *times);

/* ---- measurement ---------------------------------------------------------
 * With profiling on, every tg_tree_forces outside graph capture records a
 * pair of HIP events on the context's stream around its walk kernel (the
 * group walk with its P2P/P2M sums).  tg_get_profile waits for them and
 * returns the summed kernel time in ms and the number of walks since
 * profiling was last switched on. */
tg_status tg_set_profiling(tg_ctx *ctx, int32_t on);
tg_status tg_get_profile(tg_ctx *ctx, double *walk_ms, int64_t *n_walks);

/* Wait for the stream; return TG_EDATA / TG_ECAPACITY if the device set an
 * error bit since the last tg_sync (bits in *bits if non-NULL), then clear. */
tg_status tg_sync(tg_ctx *ctx, uint32_t *bits);

const char *tg_last_error(void);

/* Library build description (arch, flags), static string. */
const char *tg_version(void);

/* ---- the hybrid step (Sec. 2): tree stars + one regularised chain -------
 * A host driver over the calls above for a system with one SMBH, global
 * kick-drift-kick steps of length dt, in the order of the paper's step list
 * (Sec. 2, steps (1)-(8)).  READING of the hybrid recipe:
 *  - without a chain: one tg_step_kdk; then the stars within r_chain0 of the
 *    SMBH (tg_select_within) start a chain with it (step (8));
 *  - members are integrated by the AR-chain in the chain's centre-of-mass
 *    frame; their stars stay in the arrays as ghosts with no further
 *    advancement: mass times ghost_mass, excluded from the coupling, never
 *    kicked or drifted, their position and velocity those they had when
 *    they joined (the SMBH's arrays get the member's global coordinates,
 *    for reference only: the SMBH is not a tree particle);
 *  - a step: the opening half kick of the stars and of the chain particle
 *    (mass M at R, velocity V; no softening; its force a_com from
 *    tg_chain_forces, with Eq. 3); the chain step (3): the members cross dt
 *    in tg_archain_advance with the perturbers of the last coupling moving
 *    on the straight lines of this step's drift (tg_predict_perturbers,
 *    dt = 0); the drift; the tree forces (6b) without the SMBH, queued on
 *    the GPU while the AR-chain advances on the host (they do not depend on
 *    the chain: the ghosts stay where they joined); tg_chain_forces with
 *    the advanced members; the closing half kick;
 *  - then, chain and tree at the same time, tg_chain_membership (steps
 *    (4)-(5)): absorbed stars become ghosts, escaped ones get their mass
 *    and global coordinates back, a chain that ends returns everything; the
 *    centre of mass is re-formed and the forces are evaluated again.
 * The driver owns the system while it lives: it writes the stars' masses
 * (ghosts), the rows of stars that leave the chain and the SMBH's arrays,
 * and synchronises the stream every step, so its calls cannot be
 * graph-captured.  tg_hybrid_create allocates the driver's own device
 * buffers and pinned host staging (freed by tg_hybrid_destroy); the
 * AR-chain's host threads start at its first threaded batch and live until
 * the process ends.
 * Errors: TG_EINVAL (arguments; the system needs exactly one SMBH),
 * TG_ECAPACITY (perturbers beyond pert_cap, members beyond 256). */
typedef struct tg_hybrid tg_hybrid;

typedef struct {
  double r_chain0;            /* chain start radius about the SMBH, > 0 */
  double gamma_crit;          /* Eq. 2, > 0 (the paper: 1e-4 ... ) */
  double gamma_esc;           /* Eq. 5, > 0 (the paper: 1.5) */
  double tol;                 /* AR-chain tolerance per extrapolated step, > 0 */
  double ghost_mass;          /* ghost mass factor, in (0, 1) */
  int32_t pert_cap;           /* perturber list capacity, >= 1 */
} tg_hybrid_config;

typedef struct {
  int32_t active;             /* 1 while a chain exists */
  int32_t n_members;          /* including the SMBH */
  int32_t n_perturbers;       /* of the last coupling */
  double com[3], com_vel[3];  /* the chain particle */
  double m_chain, r_chain;    /* mass; largest member distance from the centre */
  double energy_error;        /* the AR-chain's bookkeeping error */
  int64_t steps, starts, absorbed, escaped, ended;
  double archain_seconds;     /* host wall time inside the AR-chain, all steps */
  double step_seconds;        /* host wall time inside the step calls, all steps */
} tg_hybrid_state;

tg_status tg_hybrid_create(tg_ctx *ctx, const tg_system *sys, const tg_hybrid_config *cfg,
                           tg_hybrid **out);
/* Evaluates the forces of the current state (and may start a chain): call
 * once before the first step. */
tg_status tg_hybrid_begin(tg_hybrid *h);
tg_status tg_hybrid_step(tg_hybrid *h, double dt);
/* One block substep (tg_blocks as for tg_step_block) of the same scheme:
 * the chain particle sits on the finest level (kicked and drifted every
 * substep, its force formed every substep), ghosts are frozen (never
 * active), the members cross each substep in the AR-chain, forces go to the
 * stars active at the new k only (tree without the SMBH, then the
 * coupling).  At a hand-off every velocity is brought to the substep's
 * time first: the chain particle's by its pending closing half kick; a
 * star joins (and a chain starts with it) only at a substep where its own
 * step ends, with its pending closing half kick; stars that leave go to
 * the finest level, get their forces at once and are stored half a kick
 * back (W - a dt_min / 2), as are the re-formed chain particle and a freed
 * SMBH, so the next substep's closing half kicks bring them into step.
 * Without a chain: tg_step_block, then the chain start test. */
tg_status tg_hybrid_step_block(tg_hybrid *h, const tg_blocks *blocks);
/* members_out (host [n_members] or NULL): star index of each member, -1 for
 * the SMBH; member x/v (host [n_members][3] or NULL): centre-of-mass frame. */
tg_status tg_hybrid_state_get(const tg_hybrid *h, tg_hybrid_state *st, int32_t *members_out,
                              double *member_x, double *member_v);
/* Destroy the driver before its context (it synchronises the context's
 * stream); NULL is ignored. */
void tg_hybrid_destroy(tg_hybrid *h);

#ifdef __cplusplus
}
#endif
#endif /* TG_H */
