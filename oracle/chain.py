"""Plain CPU oracle of the chain coupling (TEST INFRASTRUCTURE ONLY).

Nothing in the product library imports this module; only the tests, the
smoke check and the benchmark's CPU leg do.  It shares no code with the HIP
path.

What it computes (Sec. 2, the hybrid method):

* Perturbers, Eq. 2: tree particle j perturbs the chain iff
      r_j < ((2 / gamma_crit) (m_j / M_chain))^(1/3) r_crit,
  r_j its distance to the chain's centre of mass.  READING: decided without
  roots, both sides cubed and squared,
      (r2 r2) r2 < (k k) rc6,   r2 = (dx dx + dy dy) + dz dz,
      k = c m_j,  c = 2 / (gamma_crit M_chain),  rc6 = (rc2 rc2) rc2,
      rc2 = r_crit r_crit,
  every operation rounded on its own, so that the decision is reproducible.
  Particles with a set exclusion flag (ghosts) are never selected.
* Radius selection (the chain start, r_j,BH < r_chain,0, and absorption,
  Eq. 4, r_j,CoM < r_chain): r2 < r r.
* Coupling forces on the tree particles (READING of the resolved-chain
  paragraph): every listed, non-excluded star feels the chain as its
  centre-of-mass particle, a point mass M at R, or, if it is a perturber,
  as the resolved members; pairs with the chain are unsoftened by default
  (Sec. 3, softening paragraph), or Plummer-softened with eps_pm.
* Prediction of the perturbers for the chain integration (the paper
  predicts their positions relative to the chain particle to first order
  at each chain force evaluation): for perturber j and a time offset dt,
      x_rel = (x_j + v_j dt) - (R + V dt),   v_rel = v_j - V,
  each operation rounded on its own (R + V dt formed first, per axis).
* Force on the chain particle: the (direct) force of every non-perturber
  star on the point R, plus the correction of Eq. 3,
      a_CoM,corr = (1 / M) sum_i m_i a_i,
  a_i the force of the perturbers on member i (also returned: the AR-chain
  integrates the members with it as external perturbation).
Sums in long double.
"""
from __future__ import annotations

import numpy as np

LD = np.longdouble


def tidal_constants(m_chain: float, r_crit: float, gamma_crit: float):
    """c = 2 / (gamma_crit M_chain) and rc6 = (rc2 rc2) rc2 (host doubles)."""
    c = 2.0 / (float(gamma_crit) * float(m_chain))
    rc2 = float(r_crit) * float(r_crit)
    return c, (rc2 * rc2) * rc2


def _r2(pos, com):
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    dx = pos[:, 0] - float(com[0])
    dy = pos[:, 1] - float(com[1])
    dz = pos[:, 2] - float(com[2])
    return (dx * dx + dy * dy) + dz * dz


def perturbers(pos, mass, com, m_chain, r_crit, gamma_crit, exclude=None):
    """Ascending indices of the perturbers (Eq. 2, cubed and squared form)."""
    c, rc6 = tidal_constants(m_chain, r_crit, gamma_crit)
    r2 = _r2(pos, com)
    k = c * np.asarray(mass, np.float64)
    sel = (r2 * r2) * r2 < (k * k) * rc6
    if exclude is not None:
        sel &= ~np.asarray(exclude, bool)
    return np.nonzero(sel)[0].astype(np.int32)


def within(pos, center, r, exclude=None):
    """Ascending indices with |x - center|^2 < r r."""
    sel = _r2(pos, center) < float(r) * float(r)
    if exclude is not None:
        sel &= ~np.asarray(exclude, bool)
    return np.nonzero(sel)[0].astype(np.int32)


def predict(pos, vel, mass, pert, com, com_vel, dt):
    """Perturbers relative to the chain particle, predicted by dt:
    (x_rel [k, 3], v_rel [k, 3], m [k]) for the listed perturbers."""
    P = np.asarray(pert, np.int64)
    x = np.asarray(pos, np.float64).reshape(-1, 3)[P]
    v = np.asarray(vel, np.float64).reshape(-1, 3)[P]
    R = np.asarray(com, np.float64)
    V = np.asarray(com_vel, np.float64)
    Rp = R + V * float(dt)
    xr = (x + v * float(dt)) - Rp[None, :]
    vr = v - V[None, :]
    return xr, vr, np.asarray(mass, np.float64)[P]


def _field(xs, ms, xt, e2, G):
    """Force and potential of the sources (xs [k][3], ms [k]) on each target
    (xt [t][3]), long double: a_t = sum_s G m_s (x_s - x_t) / (r^2 + e2)^(3/2),
    phi_t = -sum_s G m_s / (r^2 + e2)^(1/2), sources taken in order."""
    xs = np.asarray(xs, np.float64).reshape(-1, 3).astype(LD)
    ms = np.asarray(ms, np.float64).astype(LD)
    xt = np.asarray(xt, np.float64).reshape(-1, 3).astype(LD)
    a = np.zeros(xt.shape, LD)
    p = np.zeros(xt.shape[0], LD)
    for s in range(xs.shape[0]):
        d = xs[s][None, :] - xt
        r2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2] + LD(e2)
        D1 = LD(1) / np.sqrt(r2)
        gm = LD(G) * ms[s]
        a += (gm * D1 * D1 * D1)[:, None] * d
        p -= gm * D1
    return a, p


def _on_point(xs, ms, xt, G):
    """Newtonian force of many sources on one point, long double sum."""
    xs = np.asarray(xs, np.float64).reshape(-1, 3).astype(LD)
    d = xs - np.asarray(xt, np.float64).astype(LD)[None, :]
    r2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
    D1 = LD(1) / np.sqrt(r2)
    w = LD(G) * np.asarray(ms, np.float64).astype(LD) * D1 * D1 * D1
    return (w[:, None] * d).sum(0)


def coupling(pos, mass, targets, com, m_chain, mpos, mmass, pert, eps_pm=0.0,
             exclude=None, G=1.0):
    """Coupling terms (long double, returned as float64).

    targets: star indices that get their chain term (listed, non-excluded).
    pert: the perturber indices (from :func:`perturbers`).
    Returns (acc_add [len(targets), 3], pot_add [len(targets)],
             a_com [3], a_members [Nc, 3]).
    """
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    mass = np.asarray(mass, np.float64)
    mpos = np.asarray(mpos, np.float64).reshape(-1, 3)
    mmass = np.asarray(mmass, np.float64)
    e2 = float(eps_pm) * float(eps_pm)
    is_p = np.zeros(pos.shape[0], bool)
    is_p[np.asarray(pert, np.int64)] = True
    ex = np.zeros(pos.shape[0], bool) if exclude is None else np.asarray(exclude, bool)
    R = np.asarray(com, np.float64).reshape(1, 3)
    tg = np.asarray(targets, np.int64)
    acc = np.zeros((tg.size, 3))
    pot = np.zeros(tg.size)
    # perturbers: the resolved members; others: the chain particle
    rp = np.nonzero(~ex[tg] & is_p[tg])[0]
    rn = np.nonzero(~ex[tg] & ~is_p[tg])[0]
    a, p = _field(mpos, mmass, pos[tg[rp]], e2, G)
    acc[rp], pot[rp] = a.astype(np.float64), p.astype(np.float64)
    a, p = _field(R, [m_chain], pos[tg[rn]], 0.0, G)
    acc[rn], pot[rn] = a.astype(np.float64), p.astype(np.float64)
    # the chain particle: non-perturber, non-excluded stars, Newtonian
    keep = np.nonzero(~is_p & ~ex)[0]
    a_com = _on_point(pos[keep], mass[keep], R[0], G)
    # members: the perturbers' force, then Eq. 3
    P = np.asarray(pert, np.int64)
    am, _ = _field(pos[P], mass[P], mpos, e2, G)
    corr = np.zeros(3, LD)
    for i in range(mpos.shape[0]):
        corr += LD(mmass[i]) * am[i]
    a_com = a_com + corr / LD(m_chain)
    return acc, pot, np.asarray(a_com, np.float64), np.asarray(am, np.float64)


def chains_coupling(pos, mass, targets, chains, exclude=None, G=1.0):
    """Several chains (READING of the extension to several distant SMBHs the
    paper names as its next step, Sec. 7): every chain couples to the stars
    as one chain does (:func:`coupling`), with the same exclusion mask, which
    holds the ghost members of all chains; a star may perturb several chains.
    The chain particles feel each other as Newtonian point masses.

    chains: list of dicts with com, m_chain, mpos, mmass, r_crit, gamma_crit
    and optionally eps_pm.  Returns (acc_add, pot_add, a_com [K, 3],
    a_members [sum nc, 3], perturber lists).
    """
    tg = np.asarray(targets, np.int64)
    acc = np.zeros((tg.size, 3), LD)
    pot = np.zeros(tg.size, LD)
    coms, mems, perts = [], [], []
    for ch in chains:
        P = perturbers(pos, mass, ch["com"], ch["m_chain"], ch["r_crit"], ch["gamma_crit"],
                       exclude)
        a, p, ac, am = coupling(pos, mass, tg, ch["com"], ch["m_chain"], ch["mpos"],
                                ch["mmass"], P, ch.get("eps_pm", 0.0), exclude, G)
        acc += a.astype(LD)
        pot += p.astype(LD)
        coms.append(ac.astype(LD))
        mems.append(am)
        perts.append(P)
    K = len(chains)
    for a in range(K):
        Ra = np.asarray(chains[a]["com"], np.float64)
        for d in range(K):
            if d != a:
                coms[a] = coms[a] + _on_point(np.asarray(chains[d]["com"], np.float64),
                                              [chains[d]["m_chain"]], Ra, G)
    return (acc.astype(np.float64), pot.astype(np.float64),
            np.array([c.astype(np.float64) for c in coms]),
            np.concatenate(mems), perts)


def membership(mx, mv, mm, massive, designated, r_chain, r_chain0, gamma, px):
    """Membership update after a chain step (Sec. 2, Eq. 4 and 5, and the
    priority rule of Sec. 4), READING:

    * absorption (Eq. 4): perturber p joins if |x_p - R|^2 < r_chain^2, with
      r_chain the chain radius (largest member distance from the centre of
      mass in the last chain step);
    * escape (Eq. 5): member i leaves if |x_i|^2 > r_escape^2, r_escape =
      gamma r_chain,0, and it recedes, x_i . v_i > 0;
    * while a perturber is absorbed, escapes wait unless r_chain exceeds
      1.05 r_escape;
    * the chain ends if fewer than two members would remain, or if the
      designated massive particle leaves and no other massive member stays;
      otherwise the most massive remaining massive member (ties: the lowest
      index) becomes the designated one.
    Squares and dot products are summed x, y, z in that order, each
    operation rounded on its own.  mx, mv: members relative to the centre of
    mass; px: perturbers relative to it.  Returns a dict with ``absorb``
    (perturber rows), ``escape`` (member indices), ``terminate`` and
    ``designated`` (-1 when the chain ends).
    """
    mx = np.asarray(mx, np.float64).reshape(-1, 3)
    mv = np.asarray(mv, np.float64).reshape(-1, 3)
    px = np.asarray(px, np.float64).reshape(-1, 3)
    n = mx.shape[0]
    rc2 = float(r_chain) * float(r_chain)
    p2 = (px[:, 0] * px[:, 0] + px[:, 1] * px[:, 1]) + px[:, 2] * px[:, 2]
    absorb = np.nonzero(p2 < rc2)[0].astype(np.int32)
    r_esc = float(gamma) * float(r_chain0)
    m2 = (mx[:, 0] * mx[:, 0] + mx[:, 1] * mx[:, 1]) + mx[:, 2] * mx[:, 2]
    rv = (mx[:, 0] * mv[:, 0] + mx[:, 1] * mv[:, 1]) + mx[:, 2] * mv[:, 2]
    escape = np.nonzero((m2 > r_esc * r_esc) & (rv > 0.0))[0].astype(np.int32)
    if absorb.size and escape.size and not (float(r_chain) > 1.05 * r_esc):
        escape = escape[:0]
    new_d = int(designated)
    terminate = False
    if new_d in set(escape.tolist()):
        left = [i for i in range(n) if massive[i] and i not in set(escape.tolist())]
        if left:
            new_d = max(left, key=lambda i: (float(mm[i]), -i))
        else:
            terminate = True
    if n - escape.size + absorb.size < 2:
        terminate = True
    if terminate:
        new_d = -1
    return {"absorb": absorb, "escape": escape, "terminate": terminate, "designated": new_d}
