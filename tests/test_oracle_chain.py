"""Pins for the oracle's chain coupling (Sec. 2: perturbers by the tidal
criterion Eq. 2, absorption radius Eq. 4, the resolved-chain forces and the
centre-of-mass correction Eq. 3).

Independent references: the cube-root form of Eq. 2 as printed; its closed-
form radius for equal masses; a one-member chain, whose resolved force is
the point-mass force; Newton's third law between the chain and its
perturbers (momentum conservation across the two sums); the vanishing
dipole about the centre of mass (resolved and point forces agree to second
order in size / distance).
"""
import numpy as np
import pytest

from oracle import chain


def _cloud(n, seed):
    rng = np.random.default_rng(seed)
    pos = rng.normal(size=(n, 3)) * np.exp(rng.uniform(-4, 1, (n, 1)))
    mass = np.exp(rng.uniform(np.log(1e-7), np.log(1e-3), n))
    return pos, mass


def _chain(seed, nc=5, size=1e-3):
    rng = np.random.default_rng(seed)
    mpos = rng.normal(size=(nc, 3)) * size + np.array([0.01, -0.02, 0.005])
    mmass = rng.uniform(1e-5, 1e-4, nc)
    mmass[0] = 0.01            # the SMBH
    M = 0.0
    R = np.zeros(3)
    for i in range(nc):
        M += mmass[i]
        R += mmass[i] * mpos[i]
    return mpos, mmass, R / M, M


def test_tidal_rule_matches_the_cube_root_form():
    pos, mass = _cloud(200000, 1)
    M, rc, gam = 0.0101, 0.02, 1e-4
    com = np.array([0.01, -0.02, 0.005])
    got = set(chain.perturbers(pos, mass, com, M, rc, gam).tolist())
    r = np.linalg.norm(pos - com, axis=1)
    rad = np.cbrt(2.0 / gam * mass / M) * rc
    want = set(np.nonzero(r < rad)[0].tolist())
    assert len(want) > 100
    for j in got ^ want:
        assert abs(r[j] - rad[j]) <= 1e-14 * rad[j], j


@pytest.mark.parametrize("gam", [1e-4, 1e-5])
def test_tidal_radius_closed_form(gam):
    M, rc, m = 0.02, 0.01, 1e-5
    rstar = (2.0 / gam * m / M) ** (1.0 / 3.0) * rc
    f = np.array([0.5, 1 - 1e-9, 1 + 1e-9, 2.0, 0.0])
    d = np.array([1.0, 2.0, -3.0]) / np.sqrt(14.0)
    com = np.array([0.3, 0.1, -0.2])
    pos = com + f[:, None] * rstar * d
    got = chain.perturbers(pos, np.full(5, m), com, M, rc, gam).tolist()
    assert got == [0, 1, 4]
    ex = np.array([0, 0, 0, 0, 1], bool)
    assert chain.perturbers(pos, np.full(5, m), com, M, rc, gam, exclude=ex).tolist() == [0, 1]


def test_radius_selection():
    pos, _ = _cloud(50000, 2)
    c = np.array([0.1, 0.0, -0.1])
    got = chain.within(pos, c, 0.3)
    r = np.linalg.norm(pos - c, axis=1)
    assert set(got.tolist()) ^ set(np.nonzero(r < 0.3)[0].tolist()) <= set(
        np.nonzero(np.abs(r - 0.3) < 1e-15)[0].tolist())
    assert np.all(np.diff(got) > 0)


def test_one_member_chain_is_a_point_mass():
    pos, mass = _cloud(3000, 3)
    R = np.array([0.01, -0.02, 0.005])
    M = 0.01
    pert = chain.perturbers(pos, mass, R, M, 0.02, 1e-4)
    assert pert.size > 10
    acc, pot, a_com, am = chain.coupling(pos, mass, np.arange(3000), R, M, R[None], [M], pert)
    d = pos - R
    r = np.linalg.norm(d, axis=1)
    want_star = -M * d / r[:, None] ** 3
    assert np.allclose(acc, want_star, rtol=1e-13, atol=0)
    assert np.allclose(pot, -M / r, rtol=1e-13, atol=0)
    # the chain particle feels every star, perturbers through Eq. 3
    want_com = (mass[:, None] * d / r[:, None] ** 3).sum(0)
    assert np.allclose(a_com, want_com, rtol=1e-12, atol=0)
    assert np.allclose(am[0], (mass[pert, None] * d[pert] / r[pert, None] ** 3).sum(0), rtol=1e-12)


@pytest.mark.parametrize("eps_pm", [0.0, 1e-4])
def test_chain_and_perturbers_conserve_momentum(eps_pm):
    pos, mass = _cloud(5000, 4)
    mpos, mmass, R, M = _chain(5)
    pert = chain.perturbers(pos, mass, R, M, 0.02, 1e-4)
    assert pert.size > 10
    acc, _, a_com, am = chain.coupling(pos, mass, pert, R, M, mpos, mmass, pert,
                                       eps_pm=eps_pm)
    on_pert = (mass[pert, None] * acc).sum(0)
    on_chain = (mmass[:, None] * am).sum(0)
    scale = np.abs(mass[pert, None] * acc).sum(0)
    assert np.all(np.abs(on_pert + on_chain) <= 1e-13 * scale)
    # Eq. 3 in the chain particle's force: a_com minus the non-perturbers'
    # point force is the mass-weighted member average
    keep = np.setdiff1d(np.arange(5000), pert)
    d = pos[keep] - R
    r = np.linalg.norm(d, axis=1)
    rest = (mass[keep, None] * d / r[:, None] ** 3).sum(0)
    assert np.allclose(a_com - rest, on_chain / M, rtol=1e-10, atol=0)


def test_resolved_chain_approaches_the_point_mass_far_away():
    mpos, mmass, R, M = _chain(6, nc=8, size=1e-3)
    errs = []
    for dist in (1e-2, 1e-1, 1.0):
        star = (R + dist * np.array([0.6, 0.0, 0.8]))[None]
        res, _, _, _ = chain.coupling(star, [1e-8], [0], R, M, mpos, mmass, [0])
        pt, _, _, _ = chain.coupling(star, [1e-8], [0], R, M, mpos, mmass, [])
        errs.append(np.linalg.norm(res - pt) / np.linalg.norm(pt))
    # no dipole about the centre of mass: the error falls as (size / r)^2
    assert errs[1] < errs[0] / 50 and errs[2] < errs[1] / 50


def test_excluded_stars_get_nothing_and_give_nothing():
    pos, mass = _cloud(2000, 7)
    mpos, mmass, R, M = _chain(8)
    ex = np.zeros(2000, bool)
    ex[::7] = True
    pert = chain.perturbers(pos, mass, R, M, 0.02, 1e-4, exclude=ex)
    assert not np.any(ex[pert])
    acc, pot, a_com, _ = chain.coupling(pos, mass, np.arange(2000), R, M, mpos, mmass,
                                        pert, exclude=ex)
    assert np.all(acc[ex] == 0) and np.all(pot[ex] == 0)
    pos2 = pos.copy()
    pos2[ex] += 1e-3        # moving excluded stars changes nothing
    _, _, a_com2, _ = chain.coupling(pos2, mass, np.arange(2000), R, M, mpos, mmass,
                                     pert, exclude=ex)
    assert np.array_equal(a_com, a_com2)


def test_prediction_is_first_order_and_relative():
    pos, mass = _cloud(4000, 9)
    rng = np.random.default_rng(10)
    vel = rng.normal(size=(4000, 3))
    mpos, mmass, R, M = _chain(11)
    V = np.array([0.1, -0.2, 0.05])
    pert = chain.perturbers(pos, mass, R, M, 0.02, 1e-4)
    xr0, vr0, m0 = chain.predict(pos, vel, mass, pert, R, V, 0.0)
    assert np.array_equal(xr0, pos[pert] - R) and np.array_equal(m0, mass[pert])
    assert np.allclose(vr0, vel[pert] - V, rtol=0, atol=1e-15)
    # a straight line: the relative position moves with the relative velocity
    xr1, vr1, _ = chain.predict(pos, vel, mass, pert, R, V, 1e-3)
    assert np.allclose(xr1, xr0 + 1e-3 * vr0, rtol=0, atol=1e-14)
    assert np.array_equal(vr1, vr0)


def _two_chains(seed):
    """A cloud with two SMBH chains 0.5 apart; the members are ghosts in the
    star arrays (excluded), as in the hybrid scheme."""
    rng = np.random.default_rng(seed)
    pos, mass = _cloud(6000, seed)
    chains, ghost = [], np.zeros(0, np.int64)
    for k, c in enumerate((np.array([0.25, 0.0, 0.0]), np.array([-0.25, 0.05, 0.0]))):
        # the chain's members are the SMBH plus the stars nearest to it
        near = np.argsort(np.linalg.norm(pos - c, axis=1))[:4]
        mpos = np.concatenate([c[None, :], pos[near]])
        mmass = np.concatenate([[0.01], mass[near]])
        M = mmass.sum()
        R = (mmass[:, None] * mpos).sum(0) / M
        chains.append({"com": R, "m_chain": M, "mpos": mpos, "mmass": mmass,
                       "r_crit": 0.05, "gamma_crit": 1e-4})
        ghost = np.concatenate([ghost, near])
    excl = np.zeros(pos.shape[0], bool)
    excl[ghost] = True
    return pos, mass, chains, excl


@pytest.mark.parametrize("seed", [3, 8])
def test_several_chains_conserve_momentum(seed):
    """Newton's third law across every sum: stars and chains, perturbers and
    members, chain particles with each other."""
    pos, mass, chains, excl = _two_chains(seed)
    tg = np.nonzero(~excl)[0]
    acc, pot, a_com, am, perts = chain.chains_coupling(pos, mass, tg, chains, excl)
    assert all(p.size > 5 for p in perts)
    tot = (mass[tg, None] * acc).sum(0)
    for k, ch in enumerate(chains):
        tot = tot + ch["m_chain"] * a_com[k]
    scale = np.abs(mass[tg, None] * acc).sum(0)
    assert np.all(np.abs(tot) <= 1e-12 * scale)
    assert am.shape == (sum(c["mpos"].shape[0] for c in chains), 3)


def test_one_chain_of_several_is_the_single_chain():
    pos, mass, chains, excl = _two_chains(5)
    tg = np.nonzero(~excl)[0]
    acc, pot, a_com, am, perts = chain.chains_coupling(pos, mass, tg, chains[:1], excl)
    c = chains[0]
    P = chain.perturbers(pos, mass, c["com"], c["m_chain"], c["r_crit"], c["gamma_crit"], excl)
    a1, p1, ac1, am1 = chain.coupling(pos, mass, tg, c["com"], c["m_chain"], c["mpos"],
                                      c["mmass"], P, 0.0, excl)
    assert np.array_equal(perts[0], P)
    assert np.allclose(acc, a1, rtol=1e-15, atol=0) and np.allclose(a_com[0], ac1, rtol=1e-15)
    # with two, chain 0's particle also feels chain 1 as a point mass
    acc2, _, a_com2, _, _ = chain.chains_coupling(pos, mass, tg, chains, excl)
    d = chains[1]["com"] - c["com"]
    pull = chains[1]["m_chain"] * d / np.linalg.norm(d) ** 3
    a_one_other = chain.chains_coupling(pos, mass, tg, chains[1:], excl)[2][0]
    assert np.allclose(a_com2[0], ac1 + pull, rtol=1e-12, atol=0)
    assert np.allclose(a_com2[1] - a_one_other,
                       -c["m_chain"] * d / np.linalg.norm(d) ** 3, rtol=1e-12, atol=0)


def _members(n=6, seed=1):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 3)) * 0.01
    v = rng.normal(size=(n, 3))
    m = np.concatenate([[0.01], rng.uniform(1e-5, 1e-4, n - 1)])
    massive = np.zeros(n, bool)
    massive[0] = True
    return x, v, m, massive


def test_membership_escape_needs_distance_and_recession():
    x, v, m, mas = _members()
    x[2] = [0.05, 0.0, 0.0]; v[2] = [1.0, 0.0, 0.0]      # far and receding: escapes
    x[3] = [0.0, 0.05, 0.0]; v[3] = [0.0, -1.0, 0.0]     # far, approaching: stays
    x[4] = [0.0, 0.0, 0.02]; v[4] = [0.0, 0.0, 1.0]      # receding inside r_escape: stays
    r = chain.membership(x, v, m, mas, 0, 0.03, 0.02, 1.5, np.zeros((0, 3)))
    assert r["escape"].tolist() == [2] and r["absorb"].size == 0
    assert not r["terminate"] and r["designated"] == 0


def test_membership_absorption_inside_the_chain_radius_only():
    x, v, m, mas = _members()
    px = np.array([[0.029, 0, 0], [0, 0.031, 0], [0.02, 0.02, 0.0], [0, 0, -0.0299999]])
    r = chain.membership(x, v, m, mas, 0, 0.03, 0.02, 1.5, px)
    assert r["absorb"].tolist() == [0, 2, 3]          # |(.02,.02,0)| = .0283 < .03


def test_membership_absorption_delays_escape_until_five_percent():
    x, v, m, mas = _members()
    x[2] = [0.05, 0.0, 0.0]; v[2] = [1.0, 0.0, 0.0]
    px = np.array([[0.001, 0.0, 0.0]])
    r_esc = 1.5 * 0.02
    for r_chain, escapes in ((1.04 * r_esc, []), (1.06 * r_esc, [2])):
        r = chain.membership(x, v, m, mas, 0, r_chain, 0.02, 1.5, px)
        assert r["absorb"].tolist() == [0] and r["escape"].tolist() == escapes


def test_membership_termination_and_a_new_designated_particle():
    x, v, m, mas = _members(3)
    x[:] = [[0.05, 0, 0], [0.06, 0, 0], [0.001, 0, 0]]
    v[:] = [[1, 0, 0], [1, 0, 0], [0, 0, 0]]
    # two of three leave: one member would remain
    r = chain.membership(x, v, m, mas, 0, 0.03, 0.02, 1.5, np.zeros((0, 3)))
    assert r["terminate"] and r["designated"] == -1
    # the designated SMBH leaves; a second, heavier SMBH stays and takes over
    x, v, m, mas = _members(5)
    x[0] = [0.05, 0, 0]; v[0] = [1, 0, 0]
    mas[3] = mas[4] = True
    m[3], m[4] = 0.004, 0.006
    r = chain.membership(x, v, m, mas, 0, 0.03, 0.02, 1.5, np.zeros((0, 3)))
    assert not r["terminate"] and r["designated"] == 4 and r["escape"].tolist() == [0]
    # no other massive member: the chain ends
    mas[3] = mas[4] = False
    r = chain.membership(x, v, m, mas, 0, 0.03, 0.02, 1.5, np.zeros((0, 3)))
    assert r["terminate"] and r["designated"] == -1
