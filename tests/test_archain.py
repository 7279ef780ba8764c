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
