"""Seeded synthetic initial conditions (the paper's workloads).

This module only draws particles; it holds none of the tree-gravity
arithmetic, and both the HIP path and the CPU oracle take their inputs from
it.  Units: G = M = scale radius = 1 (Sec. 3 of the paper).

* Plummer sphere: the classic inverse-CDF radius and rejection-sampled speed
  from the isotropic distribution function f(E) ~ (-E)^(7/2).
* Dehnen gamma-models, gamma in {0.5, 1, 1.5}; gamma = 1 is the Hernquist
  sphere the paper uses (rho ~ r^-1 inside, r^-4 outside; Sec. 3).  Radii by
  inverting M(r) = (r/(1+r))^(3-gamma) with the enclosed-mass fraction drawn
  below 0.99 (keeps the outermost particles near a few hundred scale radii
  so that 21-bit keys resolve the centre); speeds by inverse-CDF sampling of
  the isotropic Eddington distribution function of the untruncated model.
* Equal stellar masses 1/N; positions and velocities recentred on the
  centre of mass.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1507010090


# --------------------------------------------------------------------------
# Dehnen model closed forms (G = M = a = 1)
# --------------------------------------------------------------------------
def dehnen_mass(r, gamma):
    r = np.asarray(r, np.float64)
    return (r / (1.0 + r)) ** (3.0 - gamma)


def dehnen_density(r, gamma):
    r = np.asarray(r, np.float64)
    return (3.0 - gamma) / (4.0 * np.pi) * r ** (-gamma) * (1.0 + r) ** (gamma - 4.0)


def dehnen_psi(r, gamma):
    """Relative potential Psi = -Phi > 0."""
    r = np.asarray(r, np.float64)
    if gamma == 2.0:
        return np.log1p(1.0 / r)
    return (1.0 - (r / (1.0 + r)) ** (2.0 - gamma)) / (2.0 - gamma)


def dehnen_r_of_psi(psi, gamma):
    psi = np.asarray(psi, np.float64)
    y = (1.0 - (2.0 - gamma) * psi) ** (1.0 / (2.0 - gamma))
    return y / (1.0 - y)


def dehnen_vcirc(r, gamma, extra_mass=0.0):
    r = np.asarray(r, np.float64)
    return np.sqrt((dehnen_mass(r, gamma) + extra_mass) / r)


def dehnen_half_mass_radius(gamma):
    y = 0.5 ** (1.0 / (3.0 - gamma))
    return y / (1.0 - y)


def _d2rho_dpsi2(r, gamma):
    """d^2 rho / d Psi^2 at radius r (chain rule through r)."""
    rho = dehnen_density(r, gamma)
    g1 = -gamma / r + (gamma - 4.0) / (1.0 + r)
    g1p = gamma / r ** 2 - (gamma - 4.0) / (1.0 + r) ** 2
    rho1 = rho * g1
    rho2 = rho * (g1 * g1 + g1p)
    M = dehnen_mass(r, gamma)
    psi1 = -M / r ** 2
    psi2 = -(4.0 * np.pi * rho - 2.0 * M / r ** 3)
    return (rho2 * psi1 - rho1 * psi2) / psi1 ** 3


@dataclass
class EddingtonDF:
    """Isotropic f(E) of a Dehnen model, tabulated in log E."""
    gamma: float
    logE: np.ndarray = field(default=None)
    logf: np.ndarray = field(default=None)

    def __post_init__(self):
        g = self.gamma
        psi0 = 1.0 / (2.0 - g)
        # E grid from far outside to very near the centre
        rgrid = np.logspace(-5.5, 5.5, 1400)
        E = dehnen_psi(rgrid, g)[::-1]
        E = E[(E > 0) & (E < psi0)]
        # f(E) = 1/(sqrt(8) pi^2) int_0^E rho''(Psi) dPsi / sqrt(E - Psi)
        # (the boundary term vanishes since d rho/d Psi -> 0 as Psi -> 0).
        # Psi = E (1 - u^2), u = w^2 cluster nodes where Psi -> E.
        xw, ww = np.polynomial.legendre.leggauss(160)
        w = 0.5 * (xw + 1.0)
        wt = 0.5 * ww
        u = w * w
        du = 2.0 * w * wt
        f = np.empty_like(E)
        for k, e in enumerate(E):
            psi = e * (1.0 - u * u)
            r = dehnen_r_of_psi(psi, g)
            val = _d2rho_dpsi2(r, g)
            f[k] = 2.0 * math.sqrt(e) * np.sum(val * du)
        f /= math.sqrt(8.0) * np.pi ** 2
        ok = f > 0
        self.logE = np.log(E[ok])
        self.logf = np.log(f[ok])

    def __call__(self, E):
        E = np.asarray(E, np.float64)
        out = np.zeros_like(E)
        m = E > 0
        out[m] = np.exp(np.interp(np.log(E[m]), self.logE, self.logf))
        return out


def hernquist_df_exact(E):
    """Closed-form isotropic Hernquist DF (Hernquist 1990), G = M = a = 1."""
    q = np.sqrt(np.asarray(E, np.float64))
    s = 1.0 - q * q
    return (1.0 / (math.sqrt(2.0) * (2.0 * np.pi) ** 3) / s ** 2.5 *
            (3.0 * np.arcsin(q) + q * np.sqrt(s) * (1.0 - 2.0 * q * q) *
             (8.0 * q ** 4 - 8.0 * q * q - 3.0)))


_DF_CACHE: dict = {}


def _df(gamma):
    if gamma not in _DF_CACHE:
        _DF_CACHE[gamma] = EddingtonDF(gamma)
    return _DF_CACHE[gamma]


def _isotropic(rng, n):
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    sth = np.sqrt(1.0 - cth * cth)
    return np.stack([sth * np.cos(phi), sth * np.sin(phi), cth], 1)


def _recentre(pos, vel):
    pos -= pos.mean(0)
    vel -= vel.mean(0)
    return pos, vel


def plummer(n, seed):
    """Equal-mass Plummer sphere, G = M = a = 1 (no truncation)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.uniform(0.0, 1.0, n)
    X = np.clip(X, 1e-300, 1.0 - 1e-16)
    r = (X ** (-2.0 / 3.0) - 1.0) ** -0.5
    pos = r[:, None] * _isotropic(rng, n)
    # speed fraction q by rejection on q^2 (1 - q^2)^(7/2) (max ~0.092)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        a = rng.uniform(0.0, 1.0, todo.size)
        b = rng.uniform(0.0, 0.1, todo.size)
        ok = b < a * a * (1.0 - a * a) ** 3.5
        q[todo[ok]] = a[ok]
        todo = todo[~ok]
    v = q * math.sqrt(2.0) * (1.0 + r * r) ** -0.25
    vel = v[:, None] * _isotropic(rng, n)
    pos, vel = _recentre(pos, vel)
    return pos, vel, np.full(n, 1.0 / n)


def dehnen(n, gamma, seed, mass_fraction=0.99, chunk=1 << 18):
    """Equal-mass Dehnen gamma-model, truncated in enclosed-mass fraction."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.uniform(0.0, mass_fraction, n)
    X = np.maximum(X, 1e-300)
    y = X ** (1.0 / (3.0 - gamma))
    r = y / (1.0 - y)
    pos = r[:, None] * _isotropic(rng, n)
    df = _df(gamma)
    psi = dehnen_psi(r, gamma)
    K = 128
    u = (np.arange(K) + 0.5) / K
    speed = np.empty(n)
    U = rng.uniform(0.0, 1.0, n)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        ps = psi[a:b, None]
        p = u[None, :] ** 2 * df(ps * (1.0 - u[None, :] ** 2))
        cdf = np.cumsum(p, 1)
        cdf /= cdf[:, -1:]
        # inverse CDF on the midpoint grid, linear between nodes
        idx = (cdf < U[a:b, None]).sum(1)
        idx = np.minimum(idx, K - 1)
        lo = np.where(idx > 0, cdf[np.arange(b - a), np.maximum(idx - 1, 0)], 0.0)
        hi = cdf[np.arange(b - a), idx]
        frac = np.where(hi > lo, (U[a:b] - lo) / np.maximum(hi - lo, 1e-300), 0.5)
        uu = (idx + frac) / K
        speed[a:b] = uu * np.sqrt(2.0 * psi[a:b])
    vel = speed[:, None] * _isotropic(rng, n)
    pos, vel = _recentre(pos, vel)
    return pos, vel, np.full(n, 1.0 / n)


def clump_in_halo(n, seed, width=1e-7, centre=(1.25, -2.5, 3.75)):
    """A wide Gaussian cloud (dispersion 100) holding a tight Gaussian clump
    (dispersion ``width``) of half the particles at ``centre``: a cell side
    of 2^-21 of the cube does not split the clump, 2^-42 does."""
    rng = np.random.Generator(np.random.PCG64(seed))
    wide = rng.normal(size=(n // 2, 3)) * 100.0
    clump = np.asarray(centre, np.float64) + rng.normal(size=(n - n // 2, 3)) * width
    return np.concatenate([wide, clump])


# --------------------------------------------------------------------------
# The five workloads (sizes and parameters of the benchmark configurations)
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    pos: np.ndarray          # [N, 3] stars
    vel: np.ndarray
    mass: np.ndarray
    eps: float
    theta: float
    sys_off: np.ndarray      # int64 [S+1]
    bh_pos: np.ndarray       # [nbh, 3]
    bh_vel: np.ndarray
    bh_mass: np.ndarray
    bh_eps: np.ndarray
    bh_sys: np.ndarray       # int32 [nbh] system of each SMBH
    params: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.pos.shape[0]


def _one_bh(m=0.01, eps=0.01):
    return (np.zeros((1, 3)), np.zeros((1, 3)), np.array([m]), np.array([eps]))


def plummer_c1(n=4096, seed=None):
    """Equal-mass Plummer sphere, eps = 0.01, theta = 0.5, no SMBH."""
    seed = SEED_BASE + 1 if seed is None else seed
    pos, vel, m = plummer(n, seed)
    z = np.zeros((0, 3))
    return Workload("plummer_n%d" % n, pos, vel, m, 0.01, 0.5,
                    np.array([0, n], np.int64), z, z, np.zeros(0), np.zeros(0),
                    np.zeros(0, np.int32), {"leaf_size": 8})


def hernquist_c2(n=131072, seed=None):
    """Hernquist sphere + one SMBH 0.01 at rest at the origin."""
    seed = SEED_BASE + 2 if seed is None else seed
    pos, vel, m = dehnen(n, 1.0, seed)
    bp, bv, bm, be = _one_bh(0.01, 0.01)
    return Workload("hernquist_n%d_bh" % n, pos, vel, m, 0.01, 0.5,
                    np.array([0, n], np.int64), bp, bv, bm, be,
                    np.zeros(1, np.int32), {"dt": 1e-3, "steps": 100})


def cusp_c3(n=1048576, seed=None):
    """Dehnen gamma = 1.5, eps* = 1e-3, SMBH binary 2 x 0.005 at +-0.005 on x.

    Circular binary: each SMBH moves along +-y with
    v = sqrt(r (G m_other / d^2 + G M*(<r) / r^2)), r = d/2.
    """
    seed = SEED_BASE + 3 if seed is None else seed
    pos, vel, m = dehnen(n, 1.5, seed)
    d, mb = 0.01, 0.005
    r = d / 2
    v = math.sqrt(r * (mb / d ** 2 + float(dehnen_mass(r, 1.5)) / r ** 2))
    bp = np.array([[r, 0, 0], [-r, 0, 0]], np.float64)
    bv = np.array([[0, v, 0], [0, -v, 0]], np.float64)
    return Workload("dehnen1.5_n%d_bhbinary" % n, pos, vel, m, 1e-3, 0.5,
                    np.array([0, n], np.int64), bp, bv, np.array([mb, mb]),
                    np.array([1e-3, 1e-3]), np.zeros(2, np.int32), {})


def hernquist_c4(n=4194304, seed=None):
    """Hernquist, block steps: 8 levels, dt_max = 2^-6, 1000 substeps."""
    seed = SEED_BASE + 4 if seed is None else seed
    pos, vel, m = dehnen(n, 1.0, seed)
    bp, bv, bm, be = _one_bh(0.01, 0.01)
    return Workload("hernquist_n%d_blocksteps" % n, pos, vel, m, 0.01, 0.5,
                    np.array([0, n], np.int64), bp, bv, bm, be,
                    np.zeros(1, np.int32),
                    {"nlev": 8, "dt_max": 2.0 ** -6, "substeps": 1000,
                     "tau_star": 0.3, "tau_bh": 0.003})


def batch_c5(S=32, nmin=1 << 14, nmax=1 << 19, seed=None):
    """S independent realisations, N log-uniform, gamma cycling 0.5, 1, 1.5;
    one SMBH 0.01 at each origin.  Systems are concatenated."""
    seed = SEED_BASE + 5 if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), S))).astype(np.int64)
    gammas = [(0.5, 1.0, 1.5)[r % 3] for r in range(S)]
    P, V, M = [], [], []
    for r in range(S):
        p, v, m = dehnen(int(ns[r]), gammas[r], seed + 1000 * (r + 1))
        P.append(p); V.append(v); M.append(m)
    off = np.zeros(S + 1, np.int64)
    off[1:] = np.cumsum(ns)
    bp = np.zeros((S, 3)); bv = np.zeros((S, 3))
    return Workload("batch%d_n%d" % (S, int(off[-1])), np.concatenate(P),
                    np.concatenate(V), np.concatenate(M), 0.01, 0.5, off, bp,
                    bv, np.full(S, 0.01), np.full(S, 0.01),
                    np.arange(S, dtype=np.int32),
                    {"gammas": gammas, "dt": 1e-3})
