"""The host AR-chain integrator (tg_archain_*, FP64, no GPU needed).

References independent of the integrator: the exact Kepler solution
(eccentric and near-radial two-body orbits, where an unregularized scheme
fails), energy conservation, time reversibility, and a high-order
Runge-Kutta integration (scipy DOP853 at rtol 1e-13) of the same
perturbed few-body equations on a well-separated configuration.
"""
import numpy as np
import pytest

from paper_1507_01009_amd import binding as B


def _kepler(m1, m2, a, e, t):
    """CoM-frame positions and velocities of a two-body orbit that starts at
    apocentre at t = 0 (x axis), by Kepler's equation."""
    mu = m1 + m2
    n = np.sqrt(mu / a ** 3)
    M = np.pi + n * t
    E = M.copy() if np.ndim(M) else M
    for _ in range(100):
        E = E - (E - e * np.sin(E) - M) / (1 - e * np.cos(E))
    r = np.array([a * (np.cos(E) - e), a * np.sqrt(1 - e * e) * np.sin(E), 0.0])
    Edot = n / (1 - e * np.cos(E))
    v = np.array([-a * np.sin(E) * Edot, a * np.sqrt(1 - e * e) * np.cos(E) * Edot, 0.0])
    x = np.stack([-m2 / mu * r, m1 / mu * r])
    w = np.stack([-m2 / mu * v, m1 / mu * v])
    return x, w


@pytest.mark.parametrize("e", [0.0, 0.9, 0.999, 0.99999])
def test_kepler_orbit_exact(e):
    m = np.array([1.0, 1e-3])
    x0, v0 = _kepler(m[0], m[1], 1.0, e, 0.0)
    ch = B.ARChain(x0, v0, m)
    T = 2 * np.pi / np.sqrt(m.sum())
    for k, t in enumerate((0.37 * T, 1.0 * T, 2.5 * T)):
        ch.advance(t - ch.t, tol=1e-13)
        x, v = _kepler(m[0], m[1], 1.0, e, t)
        assert abs(ch.t - t) <= 1e-13 * t
        rel = ch.x[1] - ch.x[0]
        want = x[1] - x[0]
        assert np.linalg.norm(rel - want) <= 1e-8 * (1 + e) * 1.0, (e, k)
    assert abs(ch.energy_error()) < 1e-11


@pytest.mark.parametrize("e", [0.5, 0.99])
def test_many_short_advances_land_on_their_end_times(e):
    """Sixty calls over one period: every call ends with the search for its
    last step, closed in physical time where the gap is short against the
    pair's crossing time (and refused near pericentre where it is not); the
    orbit still follows Kepler's solution and each call ends on its time."""
    m = np.array([1.0, 1e-3])
    x0, v0 = _kepler(m[0], m[1], 1.0, e, 0.0)
    ch = B.ARChain(x0, v0, m)
    T = 2 * np.pi / np.sqrt(m.sum())
    for k in range(1, 61):
        t = k * T / 60
        ch.advance(t - ch.t, tol=1e-13)
        assert ch.t == t or abs(ch.t - t) <= 1e-15 * t
    x, v = _kepler(m[0], m[1], 1.0, e, ch.t)
    assert np.linalg.norm((ch.x[1] - ch.x[0]) - (x[1] - x[0])) <= 1e-8
    assert np.linalg.norm((ch.v[1] - ch.v[0]) - (v[1] - v[0])) <= 1e-7
    assert abs(ch.energy_error()) < 1e-11


def _cluster(seed, n=6):
    rng = np.random.default_rng(seed)
    m = np.concatenate([[1.0], rng.uniform(1e-4, 1e-3, n - 1)])
    x = np.concatenate([[[0, 0, 0]], rng.normal(size=(n - 1, 3)) * 0.3])
    # near-circular speeds about the heavy body, randomly tilted
    v = np.zeros((n, 3))
    for i in range(1, n):
        r = np.linalg.norm(x[i])
        t = np.cross(x[i], rng.normal(size=3))
        v[i] = t / np.linalg.norm(t) * np.sqrt(1.0 / r) * rng.uniform(0.7, 1.1)
    M = m.sum()
    x -= (m[:, None] * x).sum(0) / M
    v -= (m[:, None] * v).sum(0) / M
    return x, v, m


def test_energy_conservation_and_reversibility():
    x0, v0, m = _cluster(1)
    ch = B.ARChain(x0, v0, m)
    ch.advance(20.0, tol=1e-12)          # ~100 inner orbits
    assert abs(ch.energy_error()) < 1e-10
    # back and forth over a stretch shorter than the few-body Lyapunov time
    ch = B.ARChain(x0, v0, m)
    ch.advance(2.0, tol=1e-13)
    ch.v *= -1.0
    ch.reset_from_xv()                   # the state is taken from x, v again
    ch.advance(2.0, tol=1e-13)
    ch.v *= -1.0
    assert np.allclose(ch.x, x0, atol=1e-9) and np.allclose(ch.v, v0, atol=1e-9)


def _rhs(m, pm, py, pw):
    def f(t, s):
        n = m.size
        x = s[:3 * n].reshape(n, 3)
        v = s[3 * n:].reshape(n, 3)
        a = np.zeros((n, 3))
        for i in range(n):
            for j in range(n):
                if i != j:
                    d = x[j] - x[i]
                    a[i] += m[j] * d / np.linalg.norm(d) ** 3
        fx = np.zeros((n, 3))
        for p in range(pm.size):
            y = py[p] + pw[p] * t
            d = y[None, :] - x
            fx += pm[p] * d / (np.linalg.norm(d, axis=1) ** 3)[:, None]
        fx -= (m[:, None] * fx).sum(0) / m.sum()
        return np.concatenate([v.ravel(), (a + fx).ravel()])
    return f


def test_perturbed_chain_matches_runge_kutta():
    from scipy.integrate import solve_ivp
    x0, v0, m = _cluster(2, n=4)
    rng = np.random.default_rng(3)
    py = rng.normal(size=(5, 3)) * 3.0
    pw = rng.normal(size=(5, 3)) * 0.05
    pm = rng.uniform(1e-3, 1e-2, 5)
    ch = B.ARChain(x0, v0, m)
    ch.advance(3.0, tol=1e-13, px=py, pv=pw, pm=pm, t0=0.0)
    sol = solve_ivp(_rhs(m, pm, py, pw), (0.0, 3.0), np.concatenate([x0.ravel(), v0.ravel()]),
                    method="DOP853", rtol=1e-13, atol=1e-15)
    xe = sol.y[:12, -1].reshape(4, 3)
    ve = sol.y[12:, -1].reshape(4, 3)
    assert np.allclose(ch.x, xe, rtol=0, atol=1e-9)
    assert np.allclose(ch.v, ve, rtol=0, atol=1e-8)
    # the binding energy carries the perturbers' work: the bookkeeping closes
    assert abs(ch.energy_error()) < 1e-10
    # and the perturbation mattered
    free = B.ARChain(x0, v0, m)
    free.advance(3.0, tol=1e-13)
    assert np.abs(free.x - ch.x).max() > 1e-6


def test_argument_errors():
    with pytest.raises(B.TGError):
        B.ARChain(np.zeros((1, 3)), np.zeros((1, 3)), [1.0])
    with pytest.raises(B.TGError):
        B.ARChain(np.zeros((2, 3)), np.zeros((2, 3)), [1.0, 1.0])   # coincident
    with pytest.raises(B.TGError):
        B.ARChain([[0, 0, 0], [1, 0, 0]], np.zeros((2, 3)), [1.0, -1.0])
    ch = B.ARChain([[0, 0, 0], [1, 0, 0]], [[0, 0, 0], [0, 1, 0]], [1.0, 1e-3])
    with pytest.raises(B.TGError):
        ch.advance(-1.0)


def test_chain_is_ordered_by_force():
    """Sec. 2: the chain is sorted by gravitational force, not distance.
    A tight binary (1, 2) at distance 1 from a heavy body 0, and a light
    body 3 at 0.3 on the other side of it: the binary is the strongest
    pair; body 0 is pulled hardest by the binary's nearer member (1), so it
    joins at that end; body 3 then joins at body 0's end.  The chain is
    3-0-1-2 (or the same read backwards)."""
    m = np.array([1.0, 1e-3, 1e-3, 1e-6])
    x = np.array([[0.0, 0, 0], [1.0 - 5e-4, 0, 0], [1.0 + 5e-4, 0, 0], [-0.3, 0, 0]])
    v = np.zeros((4, 3))
    v[1, 1], v[2, 1] = -0.5, 0.5
    ch = B.ARChain(x, v, m)
    assert ch.chain.tolist() in ([3, 0, 1, 2], [2, 1, 0, 3])
    # chain vectors are the links: X_k = x_chain[k+1] - x_chain[k]
    assert np.allclose(ch.cx, x[ch.chain[1:]] - x[ch.chain[:-1]], rtol=0, atol=1e-15)


def test_tight_binary_far_from_the_centre_of_mass_keeps_its_digits():
    """A circular binary of two 1e-3 masses with separation 1e-5 orbits a
    unit mass at distance 1: its members sit 1e5 binary separations from the
    centre of mass.  Over 200 binary orbits (20 calls, the chain state kept
    between them) the energy bookkeeping stays within 1e-11 and the
    separation, read from the binary's chain vector, within 1e-10.  In
    centre-of-mass coordinates the same integration loses 1e-16 of the
    members' distance per operation, 1e-11 of the separation; it ended at
    1.4e-8 (energy) and 3.0e-8 (separation)."""
    a, D, mb = 1e-5, 1.0, 1e-3
    Vb = np.sqrt((1.0 + 2 * mb) / D)
    vb = np.sqrt(2 * mb / a) / 2
    x = np.array([[0, 0, 0], [D, -a / 2, 0], [D, a / 2, 0]], float)
    v = np.array([[0, 0, 0], [vb, Vb, 0], [-vb, Vb, 0.0]])
    m = np.array([1.0, mb, mb])
    x -= (m[:, None] * x).sum(0) / m.sum()
    v -= (m[:, None] * v).sum(0) / m.sum()
    P = 2 * np.pi * np.sqrt(a ** 3 / (2 * mb))
    ch = B.ARChain(x, v, m)
    for _ in range(20):
        ch.advance(10 * P, tol=1e-13)
    link = [k for k in range(2) if {int(ch.chain[k]), int(ch.chain[k + 1])} == {1, 2}]
    assert len(link) == 1
    sep = np.linalg.norm(ch.cx[link[0]])
    assert abs(sep / a - 1.0) < 1e-10, sep / a - 1.0
    assert abs(ch.energy_error()) < 1e-11, ch.energy_error()
