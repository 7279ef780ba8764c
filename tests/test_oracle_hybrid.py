"""Pins for the hybrid oracle (``oracle.hybrid``), with no product code.

* With no star near the SMBH the hybrid step is the tree's step:
  ``Hybrid.step`` equals ``steps.kdk_step`` and ``Hybrid.step_block`` equals
  ``steps.block_substep``, bit for bit.
* Hand-built events at predicted steps: an SMBH with two light stars on
  Kepler orbits (one bound, one hyperbolic).  The chain starts at the first
  step end with the bound star inside r_chain0 (Sec. 2, step (8)), the
  hyperbolic star is absorbed at the first step end at which it is closer
  to the centre of mass than the chain radius (Eq. 4) and escapes at the
  first step end beyond gamma r_chain0 while moving away (Eq. 5).  The step
  ends are predicted from the two-body solutions alone.
* Momentum of the stars and the chain particle is conserved (opening angle
  0, so the tree forces are pairwise) over steps with chain starts,
  absorptions and escapes, within rounding and the ghosts' tiny masses.
* Energy of an SMBH and one star whose eccentric orbit crosses r_chain0
  (a chain starts near pericentre and ends when the star escapes) falls as
  dt^2 over an orbit, in global steps and in block substeps (dt_max halved,
  tau scaled with it).  A hand-off with velocities half a kick apart leaves
  an O(dt) error and makes it fall only as dt.
"""
import copy

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from oracle import hybrid as ohyb
from oracle import steps as osteps
from paper_1507_01009_amd import ics


def kepler_state(q, e, tp, t, rot=0.0, incl=0.0, M=1.0):
    """Position and velocity at time t on a Kepler orbit about a fixed mass
    M (G = 1): pericentre distance q, eccentricity e, pericentre passage at
    tp; the orbit lies in the x-y plane with its pericentre rotated by rot,
    then the plane is tilted by incl about x."""
    if e > 1.0:
        a = q / (e - 1.0)
        n = np.sqrt(M / a ** 3)
        H = brentq(lambda H: e * np.sinh(H) - H - n * (t - tp), -60.0, 60.0)
        x, y = a * (e - np.cosh(H)), a * np.sqrt(e * e - 1.0) * np.sinh(H)
        Hd = n / (e * np.cosh(H) - 1.0)
        vx, vy = -a * np.sinh(H) * Hd, a * np.sqrt(e * e - 1.0) * np.cosh(H) * Hd
    else:
        a = q / (1.0 - e)
        n = np.sqrt(M / a ** 3)
        Mn = n * (t - tp)
        E = brentq(lambda E: E - e * np.sin(E) - Mn, Mn - 2.0, Mn + 2.0)
        x, y = a * (np.cos(E) - e), a * np.sqrt(1.0 - e * e) * np.sin(E)
        Ed = n / (1.0 - e * np.cos(E))
        vx, vy = -a * np.sin(E) * Ed, a * np.sqrt(1.0 - e * e) * np.cos(E) * Ed
    c, s = np.cos(rot), np.sin(rot)
    p = np.array([c * x - s * y, s * x + c * y, 0.0])
    v = np.array([c * vx - s * vy, s * vx + c * vy, 0.0])
    ci, si = np.cos(incl), np.sin(incl)
    T = np.array([[1.0, 0.0, 0.0], [0.0, ci, -si], [0.0, si, ci]])
    return T @ p, T @ v


def _state(pos, vel, mass, eps, theta=0.5, M=1.0, bh_pos=None, bh_vel=None):
    n = len(pos)
    return osteps.State(np.array(pos, float), np.array(vel, float), np.array(mass, float), eps,
                        theta, np.array([0, n], np.int64),
                        np.zeros((1, 3)) if bh_pos is None else np.array(bh_pos, float).reshape(1, 3),
                        np.zeros((1, 3)) if bh_vel is None else np.array(bh_vel, float).reshape(1, 3),
                        np.array([M]), np.array([eps]), np.array([0, 1], np.int64))


def _cusp(n=1500, seed=5, m_bh=0.01):
    p, v, m = ics.dehnen(n, 1.5, seed)
    return p, v, m, m_bh


# ------------------------------------------------------------ no chain
def test_without_a_chain_the_step_is_the_tree_step_bitwise():
    p, v, m, mbh = _cusp(1200, 3)
    a = _state(p, v, m, 0.01, M=mbh)
    b = copy.deepcopy(a)
    h = ohyb.Hybrid(a, r_chain0=1e-12)
    h.begin()
    osteps.forces(b)
    for _ in range(4):
        h.step(1e-3)
        osteps.kdk_step(b, 1e-3)
    assert not h.active and h.starts == 0
    for f in ("pos", "vel", "acc", "pot", "bh_pos", "bh_vel", "bh_acc"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    # block substeps
    c = _state(p, v, m, 0.01, M=mbh)
    d = copy.deepcopy(c)
    h = ohyb.Hybrid(c, r_chain0=1e-12)
    h.begin()
    osteps.forces(d)
    lc, ld = np.zeros(1200, np.uint8), np.zeros(1200, np.uint8)
    t4 = np.full(1200, 0.3 ** 4 * 0.01 ** 2)
    kc = kd = 0
    for _ in range(12):
        kc = h.step_block(lc, t4, kc, 0.25, 6)
        kd, _ = osteps.block_substep(d, ld, t4, kd, 0.25, 6)
    assert kc == kd == 12 and np.array_equal(lc, ld) and len(set(lc.tolist())) > 1
    for f in ("pos", "vel", "acc", "bh_pos", "bh_vel"):
        assert np.array_equal(getattr(c, f), getattr(d, f)), f


# ------------------------------------------- events at predicted steps
# SMBH of mass 1 at rest at the origin; stars of 1e-9 (they hardly move it).
R0, GAMMA = 0.1, 1.5
QA, EA = 0.04, 0.529                              # bound: apocentre 0.13 < gamma r_chain0
QB, EB, TPB, ROTB, INCB = 0.05, 1.2, 0.10, 2.0, 0.9   # hyperbolic


def _tpA():
    a = QA / (1.0 - EA)
    return np.pi * np.sqrt(a ** 3)                # at apocentre at t = 0


def _predicted(dt, nsteps):
    """First step ends of: A inside r_chain0 (chain start); then B closer
    than A, the farthest member (absorption); then B beyond gamma r_chain0
    moving away (escape)."""
    rA = lambda t: np.linalg.norm(kepler_state(QA, EA, _tpA(), t)[0])
    def B(t):
        return kepler_state(QB, EB, TPB, t, ROTB, INCB)
    ks = ka = ke = None
    for k in range(1, nsteps + 1):
        t = k * dt
        if ks is None:
            if rA(t) < R0:
                ks = k
            continue
        pb, vb = B(t)
        if ka is None:
            if np.linalg.norm(pb) < rA(t):
                ka = k
            continue
        if np.linalg.norm(pb) > GAMMA * R0 and np.dot(pb, vb) > 0.0:
            ke = k
            break
    return ks, ka, ke


def test_chain_start_absorption_and_escape_at_predicted_steps():
    dt, nsteps = 1e-3, 160
    ks, ka, ke = _predicted(dt, nsteps)
    assert ks is not None and ka is not None and ke is not None and ks < ka < ke
    pA, vA = kepler_state(QA, EA, _tpA(), 0.0)
    pB, vB = kepler_state(QB, EB, TPB, 0.0, ROTB, INCB)
    st = _state([pA, pB], [vA, vB], [1e-9, 1e-9], 1e-7)
    h = ohyb.Hybrid(st, R0, gamma_crit=1e-12, gamma_esc=GAMMA)
    h.begin()
    assert not h.active
    events = []
    prev = (0, 0, 0, 0)
    for k in range(1, nsteps + 1):
        h.step(dt)
        cur = (h.starts, h.absorbed, h.escaped, h.ended)
        if cur != prev:
            events.append((k, cur, list(h.star)))
        prev = cur
    assert events == [(ks, (1, 0, 0, 0), [-1, 0]),
                      (ka, (1, 1, 0, 0), [-1, 0, 1]),
                      (ke, (1, 1, 1, 0), [-1, 0])], (events, (ks, ka, ke))
    # B is back in the tree with its full mass, in the global frame on its
    # Kepler orbit (to the leapfrog's error of its tree phases)
    assert st.mass[1] == 1e-9 and not h.excl[1]
    assert h.excl[0] and st.mass[0] == pytest.approx(1e-19)
    pb, _ = kepler_state(QB, EB, TPB, nsteps * dt, ROTB, INCB)
    assert np.linalg.norm(st.pos[1] - pb) < 1e-3 * np.linalg.norm(pb)


def test_a_ghost_is_not_advanced_in_the_tree():
    """The bound star's row keeps the position and velocity it had when the
    chain started, however long the chain lasts."""
    dt = 1e-3
    pA, vA = kepler_state(QA, EA, _tpA(), 0.0)
    pB, vB = kepler_state(QB, EB, TPB, 0.0, ROTB, INCB)
    st = _state([pA, pB], [vA, vB], [1e-9, 1e-9], 1e-7)
    h = ohyb.Hybrid(st, R0, gamma_crit=1e-12, gamma_esc=GAMMA)
    h.begin()
    row = None
    for k in range(1, 120):
        h.step(dt)
        if h.active and row is None:
            row = (st.pos[0].copy(), st.vel[0].copy())
    assert row is not None and h.active and 0 in h.star
    assert np.array_equal(st.pos[0], row[0]) and np.array_equal(st.vel[0], row[1])
    # while the member itself has moved on (global frame)
    X, _ = h._globals()
    assert np.linalg.norm(X[h.star.index(0)] - row[0]) > 0.01


# ---------------------------------------------------------- momentum
def _momentum(h):
    st = h.st
    free = ~h.excl
    P = (st.mass[free, None] * st.vel[free]).sum(0)
    scale = (st.mass[free] * np.linalg.norm(st.vel[free], axis=1)).sum()
    if h.active:
        P = P + h.M * h.V
        scale += h.M * np.linalg.norm(h.V) + (h.m * np.linalg.norm(h.v, axis=1)).sum()
    else:
        P = P + st.bh_mass[0] * st.bh_vel[0]
        scale += st.bh_mass[0] * np.linalg.norm(st.bh_vel[0])
    return P, scale


def test_momentum_conserved_through_chain_events():
    p, v, m, mbh = _cusp(1500, 9, 0.01)
    st = _state(p, v, m, 1e-3, theta=0.0, M=mbh)
    h = ohyb.Hybrid(st, r_chain0=0.1, gamma_crit=1e-4, gamma_esc=1.5)
    h.begin()
    assert h.active
    P0, s0 = _momentum(h)
    worst = 0.0
    for _ in range(25):
        h.step(4e-3)
        P, s = _momentum(h)
        worst = max(worst, np.linalg.norm(P - P0) / s0)
    assert h.absorbed >= 10 and h.escaped >= 2, (h.absorbed, h.escaped)
    assert worst < 1e-11, worst


# ------------------------------------------------------------- energy
def _energy(h):
    """Kinetic + potential energy with every velocity in step (global steps,
    or block substeps at a synchronisation point after the pending closing
    kicks)."""
    st = h.st
    if h.active:
        x0, x1 = h.x[0], h.x[1]
        kin = 0.5 * h.M * np.dot(h.V, h.V) + 0.5 * (h.m * np.sum(h.v * h.v, 1)).sum()
        return kin - h.G * h.m[0] * h.m[1] / np.linalg.norm(x0 - x1)
    kin = 0.5 * st.mass[0] * np.dot(st.vel[0], st.vel[0])
    kin += 0.5 * st.bh_mass[0] * np.dot(st.bh_vel[0], st.bh_vel[0])
    return kin + st.mass[0] * st.pot[0]


def _pair(e=0.9, a=1.0, m=1e-3, eps=1e-6):
    """SMBH of 1 and a star of m on an ellipse, the star at apocentre, in
    the centre-of-mass frame."""
    M = 1.0
    mu = M + m
    ra = a * (1.0 + e)
    va = np.sqrt(mu * (1.0 - e) / ra)
    st = _state([[ra * M / mu, 0.0, 0.0]], [[0.0, va * M / mu, 0.0]], [m], eps, M=M,
                bh_pos=[-ra * m / mu, 0.0, 0.0], bh_vel=[0.0, -va * m / mu, 0.0])
    return st


def test_energy_through_a_chain_passage_falls_as_dt_squared_global_steps():
    T = 2.0 * np.pi                          # one orbit: apocentre to apocentre
    errs = []
    for dt in (4e-3, 2e-3, 1e-3):
        st = _pair()
        h = ohyb.Hybrid(st, r_chain0=0.3, gamma_crit=1e-4, gamma_esc=1.5)
        h.begin()
        e0 = _energy(h)
        for _ in range(int(round(T / dt))):
            h.step(dt)
        assert h.starts == 1 and h.ended == 1 and not h.active
        errs.append(abs(_energy(h) - e0) / abs(e0))
    assert 3.0 < errs[0] / errs[1] < 5.5 and 3.0 < errs[1] / errs[2] < 5.5, errs


def test_energy_through_a_chain_passage_falls_as_dt_squared_block_substeps():
    nlev = 5
    per = 2 ** (nlev - 1)
    T = 2.0 * np.pi
    errs = []
    for dt_max in (0.016, 0.008, 0.004):
        st = _pair()
        h = ohyb.Hybrid(st, r_chain0=0.3, gamma_crit=1e-4, gamma_esc=1.5)
        h.begin()
        e0 = _energy(h)
        level = np.zeros(1, np.uint8)
        # tau sqrt(eps) scaled with dt_max: the same level pattern
        t4 = np.array([(0.6 * dt_max) ** 4])
        nsub = int(round(T / (dt_max / per) / per)) * per
        k = 0
        for _ in range(nsub):
            k = h.step_block(level, t4, k, dt_max, nlev)
        assert h.starts == 1 and h.ended == 1 and not h.active
        s = copy.deepcopy(st)                # the pending closing half kicks
        oracle.kick(s.vel, s.acc, dt_max, idx=np.array([0], np.int32), level=level)
        oracle.kick(s.bh_vel, s.bh_acc, dt_max / per)
        h2 = copy.copy(h)
        h2.st = s
        errs.append(abs(_energy(h2) - e0) / abs(e0))
    assert 3.0 < errs[0] / errs[1] < 5.5 and 3.0 < errs[1] / errs[2] < 5.5, errs
