"""Pins for the oracle's cubic-spline softening (the tree's alternative to
Plummer softening, Sec. 2; the kernel of Monaghan & Lattanzio 1985 with
support 2h as used for gravity by Hernquist & Katz 1989).

References independent of the oracle's formulas: the kernel's mass density
(normalised here by quadrature), from which Poisson's equation and the
central potential follow; finite differences of the derivative chain;
continuity at the kernel's breakpoints; Newtonian values beyond 2h; the
convergence order of the multipole expansion against a sum of particle
terms; theta = 0 against the direct sum; momentum conservation.
"""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle
from paper_1507_01009_amd import ics


def W(u):
    """Monaghan-Lattanzio cubic spline density of a unit mass, h = 1."""
    u = abs(u)
    if u < 1.0:
        return (1.0 - 1.5 * u * u + 0.75 * u ** 3) / np.pi
    if u < 2.0:
        return 0.25 * (2.0 - u) ** 3 / np.pi
    return 0.0


def test_kernel_density_is_normalised():
    m = quad(lambda r: 4 * np.pi * r * r * W(r), 0, 2, points=[1.0], epsabs=1e-14)[0]
    assert abs(m - 1.0) < 1e-12


@pytest.mark.parametrize("h", [1.0, 0.01, 3.7e-4])
def test_poisson_equation_gives_the_kernel_density(h):
    # laplacian of psi = r^2 psi_2 - 3 psi_1; -(that) / 4 pi = density
    for u in np.r_[np.linspace(0.01, 1.99, 199), 2.5, 4.0]:
        p = oracle.spline_psi(u * h, h)
        rho = -((u * h) ** 2 * p[2] - 3 * p[1]) / (4 * np.pi)
        assert abs(rho * h ** 3 - W(u)) <= 1e-12 * (1.0 + abs(W(u))) * 10, u


@pytest.mark.parametrize("h", [1.0, 0.02])
def test_central_potential_from_the_density(h):
    # potential at the centre of a spherical distribution: 4 pi int rho r dr
    phi0 = quad(lambda r: 4 * np.pi * r * W(r), 0, 2, points=[1.0], epsabs=1e-14)[0]
    assert abs(oracle.spline_psi(0.0, h)[0] * h - phi0) < 1e-12
    assert abs(phi0 - 7.0 / 5.0) < 1e-12


def test_derivative_chain_by_finite_differences():
    h = 0.3
    for u in np.r_[np.linspace(0.05, 0.95, 19), np.linspace(1.05, 1.95, 19), 2.3, 3.1]:
        r = u * h
        d = 1e-6 * h
        lo, hi = oracle.spline_psi(r - d, h), oracle.spline_psi(r + d, h)
        p = oracle.spline_psi(r, h)
        for k in range(3):
            num = -(hi[k] - lo[k]) / (2 * d) / r
            assert abs(num - p[k + 1]) <= 1e-6 * abs(p[k + 1]), (u, k)


@pytest.mark.parametrize("ub", [1.0, 2.0])
def test_continuous_at_the_breakpoints(ub):
    h = 0.7
    a = oracle.spline_psi(ub * h * (1 - 1e-13), h)
    b = oracle.spline_psi(ub * h * (1 + 1e-13), h)
    assert np.allclose(a, b, rtol=1e-11, atol=0)


def test_newtonian_beyond_twice_h():
    h = 0.01
    for r in (0.02, 0.025, 0.3, 7.0):
        p = oracle.spline_psi(r, h)
        assert np.allclose(p, [1 / r, 1 / r ** 3, 3 / r ** 5, 15 / r ** 7], rtol=1e-14)
    a, ph = oracle.p2p_single([0.0, 0.0, 0.0], 2.0, [0.0, 0.03, 0.0], h, softening="spline")
    assert np.allclose(a, [0.0, -2.0 / 0.03 ** 2, 0.0], rtol=1e-14) and abs(ph + 2 / 0.03) < 1e-12


def test_pair_force_inside_the_kernel():
    h = 0.5
    for u in (0.0, 0.3, 1.2, 1.99):
        x = np.array([0.0, 0.0, u * h])
        a, ph = oracle.p2p_single([0.0, 0.0, 0.0], 1.0, x, h, softening="spline")
        p = oracle.spline_psi(u * h, h)
        assert np.allclose(a, -p[1] * x, rtol=1e-14, atol=0)
        assert abs(ph + p[0]) < 1e-14
    # coincident particles: finite potential 7/(5h), no force
    a, ph = oracle.p2p_single([1.0, 2.0, 3.0], 1.0, [1.0, 2.0, 3.0], h, softening="spline")
    assert np.all(a == 0.0) and abs(ph + 1.4 / h) < 1e-14


def _cluster(b, sym, seed=3):
    rng = np.random.default_rng(seed)
    if sym:
        d = rng.normal(size=(4, 3))
        pts = np.concatenate([d, -d]) * b
        m = np.ones(8) / 8
    else:
        pts = rng.normal(size=(3, 3)) * b
        m = np.array([0.5, 0.3, 0.2])
    c = (m[:, None] * pts).sum(0) / m.sum()
    pts -= c
    return pts, m


def _cell(pts, m):
    S = np.einsum("i,ij,ik->jk", m, pts, pts)
    return np.array([m.sum(), 0, 0, 0, S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[0, 2], S[1, 2]])


@pytest.mark.parametrize("u", [0.5, 1.5, 3.0])
@pytest.mark.parametrize("sym,order", [(True, 16.0), (False, 8.0)])
def test_multipole_converges_against_particle_sums(u, sym, order):
    """The expansion is exact to second order, so its error against the
    particle sum shrinks by 2^3 (asymmetric) or 2^4 (symmetric: no octupole)
    per halving of the cluster, inside and outside the kernel."""
    h = 1.0
    x = np.array([0.3, -0.5, 0.8])
    x = x / np.linalg.norm(x) * u * h
    errs = []
    for b in (0.02, 0.01, 0.005):
        pts, m = _cluster(b, sym)
        ref_a = np.zeros(3)
        ref_p = 0.0
        for j in range(m.size):
            a, p = oracle.p2p_single(pts[j], m[j], x, h, softening="spline")
            ref_a += a
            ref_p += p
        a, p = oracle.p2m_single(_cell(pts, m), x, h, softening="spline")
        errs.append(np.linalg.norm(a - ref_a) / np.linalg.norm(ref_a))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 0.75 * order < r1 < 1.3 * order and 0.75 * order < r2 < 1.3 * order, errs


def test_multipole_beyond_the_kernel_is_the_newtonian_one():
    pts, m = _cluster(0.05, False)
    cell = _cell(pts, m)
    x = np.array([0.4, 0.2, -0.3])
    a_s, p_s = oracle.p2m_single(cell, x, 0.1, softening="spline")
    a_n, p_n = oracle.p2m_single(cell, x, 0.0)       # Plummer with eps = 0: Newton
    assert np.allclose(a_s, a_n, rtol=1e-13) and abs(p_s - p_n) < 1e-13 * abs(p_n)


def test_theta_zero_is_the_direct_sum_and_momentum_is_conserved():
    pos, _, m = ics.plummer(3000, 11)
    eps = 0.05                                        # many pairs inside 2h
    ev = oracle.tree_forces(pos, m, eps, 0.0, softening="spline")
    acc, pot = oracle.direct(pos, m, eps, softening="spline")
    assert ev.n_p2m == 0
    assert np.max(np.linalg.norm(ev.acc - acc, axis=1) / np.linalg.norm(acc, axis=1)) < 1e-12
    assert np.max(np.abs(ev.pot - pot) / np.abs(pot)) < 1e-12
    ptot = (m[:, None] * acc).sum(0)
    assert np.linalg.norm(ptot) < 1e-14 * np.abs(m[:, None] * acc).sum()
    # and the spline is not Plummer: inside the kernel the pair is stiffer
    accp, _ = oracle.direct(pos, m, eps)
    assert np.median(np.linalg.norm(acc - accp, axis=1) / np.linalg.norm(accp, axis=1)) > 1e-3


def test_tree_error_at_theta_half_is_that_of_the_expansion():
    pos, _, m = ics.dehnen(20000, 1.0, 77)
    eps = 0.01
    ev = oracle.tree_forces(pos, m, eps, 0.5, softening="spline")
    tg = np.arange(0, 20000, 97)
    acc, _ = oracle.direct(pos, m, eps, targets=tg, softening="spline")
    e = np.linalg.norm(ev.acc[tg] - acc, axis=1) / np.linalg.norm(acc, axis=1)
    evp = oracle.tree_forces(pos, m, eps, 0.5)
    accp, _ = oracle.direct(pos, m, eps, targets=tg)
    ep = np.linalg.norm(evp.acc[tg] - accp, axis=1) / np.linalg.norm(accp, axis=1)
    assert np.median(e) < 2 * np.median(ep) and np.median(e) < 1e-3
    assert (ev.n_p2p, ev.n_p2m) == (evp.n_p2p, evp.n_p2m)      # lists do not depend on it


def test_smbh_pairs_take_the_larger_softening():
    a, p = oracle.direct_pairs([[0.0, 0.0, 0.0]], [0.01], [0.05], [[0.03, 0.0, 0.0]], [0.001],
                               softening="spline")
    ps = oracle.spline_psi(0.03, 0.05)
    assert np.allclose(a[0], [-0.01 * ps[1] * 0.03, 0, 0], rtol=1e-14)
    assert abs(p[0] + 0.01 * ps[0]) < 1e-16
    # zero softening on both sides: Newtonian
    a, p = oracle.direct_pairs([[0.0, 0.0, 0.0]], [1.0], [0.0], [[0.0, 0.5, 0.0]], [0.0],
                               softening="spline")
    assert np.allclose(a[0], [0, -4.0, 0], rtol=1e-14) and abs(p[0] + 2.0) < 1e-14
