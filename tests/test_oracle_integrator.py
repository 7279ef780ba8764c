"""Pins for the oracle's leapfrog (KDK), block-step levels and SMBH pairs.

References: a Kepler two-body orbit (energy error falls as dt^2, the
paper's tau^2 scaling in its time-step study), time reversibility of the
symmetric leapfrog, and the reduction of block steps on a single level to
the global-step leapfrog, bit for bit.
"""
import numpy as np
import pytest

import oracle


def _kepler_step(x, v, m, eps, dt, n):
    """n KDK steps of two bodies using the oracle's pair forces."""
    acc, _ = oracle.direct_pairs(x, m, eps, x, eps, self_pairs=True)
    for _ in range(n):
        oracle.kick(v, acc, dt)
        oracle.drift(x, v, dt)
        acc, _ = oracle.direct_pairs(x, m, eps, x, eps, self_pairs=True)
        oracle.kick(v, acc, dt)
    return x, v


def _energy(x, v, m, eps):
    _, pot = oracle.direct_pairs(x, m, eps, x, eps, self_pairs=True)
    return 0.5 * np.sum(m * np.sum(v * v, 1)) + 0.5 * np.sum(m * pot)


def _binary():
    m = np.array([0.6, 0.4])
    x = np.array([[-0.4, 0.0, 0.0], [0.6, 0.0, 0.0]])
    vt = np.sqrt(1.0 / 1.0) * 0.8           # sub-circular: eccentric orbit
    v = np.array([[0.0, -0.4 * vt, 0.0], [0.0, 0.6 * vt, 0.0]])
    return x, v, m


def test_kepler_energy_error_scales_dt_squared():
    errs = []
    for dt in (0.02, 0.01, 0.005):
        x, v, m = _binary()
        e0 = _energy(x, v, m, 0.0)
        x, v = _kepler_step(x, v, m, 0.0, dt, int(round(6.0 / dt)))
        errs.append(abs(_energy(x, v, m, 0.0) - e0) / abs(e0))
    assert 3.0 < errs[0] / errs[1] < 5.5
    assert 3.0 < errs[1] / errs[2] < 5.5


def test_leapfrog_time_reversible():
    x, v, m = _binary()
    x0, v0 = x.copy(), v.copy()
    x, v = _kepler_step(x, v, m, 0.01, 0.01, 200)
    v *= -1.0
    x, v = _kepler_step(x, v, m, 0.01, 0.01, 200)
    v *= -1.0
    assert np.allclose(x, x0, atol=1e-11) and np.allclose(v, v0, atol=1e-11)


def test_direct_pairs_softening_is_pair_max():
    s = np.array([[0.0, 0.0, 0.0]])
    t = np.array([[0.3, 0.4, 0.0]])
    a, p = oracle.direct_pairs(s, np.array([2.0]), np.array([0.1]), t, np.array([0.2]))
    r2 = 0.25 + 0.04
    assert p[0] == pytest.approx(-2.0 / np.sqrt(r2), rel=1e-15)
    assert np.allclose(a[0], -2.0 * t[0] / r2 ** 1.5, rtol=1e-15)


def test_levels_thresholds():
    nlev, dtmax = 8, 2.0 ** -6
    tau, eps = 0.3, 0.01
    # choose |a| so that dt = tau sqrt(eps/|a|) sits just either side of dt_l
    acc, want = [], []
    for l in range(nlev):
        dl = dtmax * 2.0 ** -l
        amag = tau * tau * eps / (dl * dl)
        for f, lev in ((1.0 - 1e-9, l), (1.0 + 1e-9, min(l + 1, nlev - 1))):
            acc.append([amag * f, 0.0, 0.0])
            want.append(lev)
    acc = np.array(acc)
    level = np.zeros(len(acc), np.uint8)
    oracle.levels(acc, np.full(len(acc), tau ** 4 * eps ** 2), level, dtmax, nlev, 0)
    assert list(level) == want
    # at substep k = 2 only levels with step dividing 2 are allowed
    level[:] = 7
    oracle.levels(np.zeros((len(acc), 3)), np.ones(len(acc)), level, dtmax, nlev, 2)
    assert np.all(level == 6)


def test_active_sets():
    level = np.array([0, 7, 6, 3, 7], np.uint8)
    assert list(oracle.active_at(level, 8, 0)) == [0, 1, 2, 3, 4]
    assert list(oracle.active_at(level, 8, 1)) == [1, 4]
    assert list(oracle.active_at(level, 8, 2)) == [1, 2, 4]
    assert list(oracle.active_at(level, 8, 16)) == [1, 2, 3, 4]
    assert list(oracle.active_at(level, 8, 128)) == [0, 1, 2, 3, 4]


def _block_run(x, v, m, eps, level_const, nlev, dtmax, nsub):
    """Block-step KDK with every particle pinned to one level."""
    n = x.shape[0]
    level = np.full(n, level_const, np.uint8)
    dtmin = dtmax * 2.0 ** -(nlev - 1)
    acc, _ = oracle.direct_pairs(x, m, eps, x, eps, self_pairs=True)
    for k in range(nsub):
        act = oracle.active_at(level, nlev, k)
        if k > 0:
            oracle.kick(v, acc, dtmax, idx=act, level=level)      # closing
        oracle.kick(v, acc, dtmax, idx=act, level=level)          # opening
        oracle.drift(x, v, dtmin)
        nxt = oracle.active_at(level, nlev, k + 1)
        if nxt.size:
            a2, _ = oracle.direct_pairs(x, m, eps, x, eps, self_pairs=True)
            acc[nxt] = a2[nxt]
    act = oracle.active_at(level, nlev, nsub)
    oracle.kick(v, acc, dtmax, idx=act, level=level)
    return x, v


def test_block_steps_on_one_level_equal_global_kdk_bitwise():
    nlev, dtmax = 8, 2.0 ** -6
    x, v, m = _binary()
    xb, vb = _block_run(x.copy(), v.copy(), m, 0.01, 7, nlev, dtmax, 16)
    xg, vg = _kepler_step(x.copy(), v.copy(), m, 0.01, dtmax * 2.0 ** -7, 16)
    assert np.array_equal(xb, xg) and np.array_equal(vb, vg)


def test_levels_velocity_criterion_thresholds():
    """dt_vel = tau_vel eps / |v| just either side of every dt_l; zero
    acceleration, so the velocity alone decides."""
    nlev, dtmax = 8, 2.0 ** -6
    tau, eps = 0.3, 0.01
    vel, want = [], []
    for l in range(nlev):
        dl = dtmax * 2.0 ** -l
        vmag = tau * eps / dl
        for f, lev in ((1.0 - 1e-9, l), (1.0 + 1e-9, min(l + 1, nlev - 1))):
            vel.append([0.0, vmag * f, 0.0])
            want.append(lev)
    vel = np.array(vel)
    n = len(vel)
    level = np.zeros(n, np.uint8)
    oracle.levels(np.zeros((n, 3)), np.ones(n), level, dtmax, nlev, 0, vel=vel,
                  tau2eps2v=np.full(n, tau ** 2 * eps ** 2))
    assert list(level) == want


def test_levels_take_the_stricter_criterion():
    nlev, dtmax, tau, eps = 8, 2.0 ** -6, 0.3, 0.01
    dl3 = dtmax * 2.0 ** -3
    acc = np.array([[tau * tau * eps / dl3 ** 2 * 0.999, 0.0, 0.0]] * 2)   # level 3 by |a|
    vel = np.array([[0.0, 0.0, tau * eps / (dtmax * 2.0 ** -5) * 0.999],    # level 5 by |v|
                    [0.0, 0.0, tau * eps / (dtmax * 2.0 ** -1) * 0.999]])   # level 1 by |v|
    level = np.zeros(2, np.uint8)
    oracle.levels(acc, np.full(2, tau ** 4 * eps ** 2), level, dtmax, nlev, 0, vel=vel,
                  tau2eps2v=np.full(2, tau ** 2 * eps ** 2))
    assert list(level) == [5, 3]


def _kepler_dkd(x, v, m, eps, dt, n):
    for _ in range(n):
        oracle.drift(x, v, 0.5 * dt)
        acc, _ = oracle.direct_pairs(x, m, eps, x, eps, self_pairs=True)
        oracle.kick(v, acc, 2.0 * dt)
        oracle.drift(x, v, 0.5 * dt)
    return x, v


def test_dkd_energy_error_scales_dt_squared_and_is_reversible():
    errs = []
    for dt in (0.02, 0.01, 0.005):
        x, v, m = _binary()
        e0 = _energy(x, v, m, 0.0)
        x, v = _kepler_dkd(x, v, m, 0.0, dt, int(round(6.0 / dt)))
        errs.append(abs(_energy(x, v, m, 0.0) - e0) / abs(e0))
    assert 3.0 < errs[0] / errs[1] < 5.5 and 3.0 < errs[1] / errs[2] < 5.5
    x, v, m = _binary()
    x0, v0 = x.copy(), v.copy()
    x, v = _kepler_dkd(x, v, m, 0.01, 0.01, 200)
    v *= -1.0
    x, v = _kepler_dkd(x, v, m, 0.01, 0.01, 200)
    v *= -1.0
    assert np.allclose(x, x0, atol=1e-11) and np.allclose(v, v0, atol=1e-11)


def test_frozen_stars_stay_put_and_still_pull():
    """Ghost chain members (Sec. 2) are held still in every step type and
    never become active, but remain sources: with the ghosts given zero
    velocity and put on the coarsest level, freezing them changes nothing
    for the other stars in a KDK step, and a ghost's pull is felt."""
    from oracle import steps as osteps
    from paper_1507_01009_amd import ics
    w = ics.hernquist_c2(n=3000)
    frozen = np.zeros(3000, bool)
    frozen[::50] = True

    def state(fr, vel_zero=False):
        vel = w.vel.copy()
        if vel_zero:
            vel[frozen] = 0.0
        st = osteps.State(w.pos.copy(), vel, w.mass.copy(), w.eps, w.theta,
                          w.sys_off.copy(), w.bh_pos.reshape(-1, 3).copy(),
                          w.bh_vel.reshape(-1, 3).copy(), w.bh_mass.copy(), w.bh_eps.copy(),
                          np.array([0, 1], np.int64), frozen=fr)
        osteps.forces(st)
        return st

    a = state(frozen)
    p0, v0 = a.pos.copy(), a.vel.copy()
    osteps.kdk_step(a, 1e-3)
    osteps.dkd_step(a, 1e-3)
    assert np.array_equal(a.pos[frozen], p0[frozen]) and np.array_equal(a.vel[frozen], v0[frozen])
    assert not np.array_equal(a.pos[~frozen], p0[~frozen])
    # the same step without freezing, ghosts at rest: the other stars' first
    # drift is identical (their later kicks then feel the ghosts' new places)
    b, c = state(frozen, True), state(None, True)
    osteps.kdk_step(b, 1e-3)
    osteps.kdk_step(c, 1e-3)
    assert np.array_equal(b.pos[~frozen], c.pos[~frozen])
    assert not np.array_equal(b.pos[frozen], c.pos[frozen])
    # block steps: frozen stars are never active and keep their level
    lev = np.zeros(3000, np.uint8)
    t4 = np.full(3000, 1e-12)
    d = state(frozen)
    k, act = osteps.block_substep(d, lev, t4, 0, 2.0 ** -6, 4)
    assert act.size > 0 and not np.any(frozen[act])
    assert np.all(lev[frozen] == 0) and np.any(lev[~frozen] > 0)
    # frozen stars stay sources: the forces do not depend on the mask
    assert np.array_equal(state(frozen).acc, state(None).acc)
