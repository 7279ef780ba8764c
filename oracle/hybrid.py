"""Plain CPU oracle of the hybrid step (TEST INFRASTRUCTURE ONLY).

Nothing in the product library imports this module; only the tests use it.
It composes the oracle's own pieces in the order of the hybrid recipe of
Sec. 2 (steps (1)-(8)), with one SMBH as the designated massive particle.

Readings of Sec. 2 that this module fixes:

* Ghosts.  A star that joins the chain stays in the tree's arrays as a
  ghost with no further advancement: its position and velocity stay those
  it had when it joined, its mass is multiplied by ``ghost_mass``, it is
  never kicked, drifted or active (it sets no time-step) and it is left
  out of the coupling.  When it leaves, its mass and its position and
  velocity in the global frame (R + x, V + v) are restored.  The SMBH is not
  a tree particle; while it is a member its arrays get R + x, V + v for
  reference only.
* The chain particle (mass M at the members' centre of mass R, velocity V)
  is a tree particle without softening: the stars that are not perturbers
  feel it as a point mass, the perturbers (Eq. 2) feel the resolved
  members, and its force is the non-perturbers' pull plus Eq. 3.
* Order of a step.  The chain step (3) comes before the tree forces (6b):
  the members cross the step with the perturbers of the last coupling
  moving relative to the chain particle on straight lines, with the
  velocities the tree's drift gives them in this step (after the opening
  half kick), their mean force removed (it acts on the chain particle
  through Eq. 3).  The tree step (6) is the leapfrog in its kick-drift-kick
  form: opening half kick, drift, forces (6b) with the members at their new
  positions about the drifted chain particle, closing half kick.  The
  membership check (4)-(5) then runs at the end of the step, when the chain
  and the tree are at the same time; after a change the centre of mass is
  re-formed from the members' global coordinates and the forces are
  evaluated again.  A chain that ends returns every member; a new one may
  start in the same step (8).
* Block substeps.  The chain particle is on the finest level and takes
  closing and opening half kicks every substep; the members cross every
  substep.  Forces go to the stars active at the new substep counter.  At
  a hand-off every velocity is brought to the same time first: the chain
  particle's by its pending closing half kick, a joining star's by its own
  (a star joins, and a chain starts with it, only at a substep where its
  own step ends); stars that leave go to the finest level and, once their
  forces exist, are stored half a kick back (W - a dt_min / 2), as is the
  new chain particle (V - a_com dt_min / 2) and an SMBH set free, so that
  the next substep's closing half kicks bring them into step.

The members are integrated by a high-order Runge-Kutta method (scipy's
DOP853 at rtol 1e-13), not by the regularised chain, so that the
comparison with the product also checks its AR-chain.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import solve_ivp

import oracle
from oracle import chain as ochain
from oracle import steps as osteps


def _members_rhs(m, px, pv, pm, G):
    """Members' mutual Newtonian forces plus the tidal part of the
    perturbers' pull (perturbers at px + pv t, relative to the chain
    particle)."""
    n = m.size

    def f(t, s):
        x = s[:3 * n].reshape(n, 3)
        v = s[3 * n:].reshape(n, 3)
        d = x[None, :, :] - x[:, None, :]              # d[i, j] = x_j - x_i
        r = np.linalg.norm(d, axis=2)
        np.fill_diagonal(r, np.inf)                    # no self pull
        a = G * ((m[None, :] / r ** 3)[:, :, None] * d).sum(1)
        fx = np.zeros((n, 3))
        for p in range(pm.size):
            y = px[p] + pv[p] * t
            d = y[None, :] - x
            fx += G * pm[p] * d / (np.linalg.norm(d, axis=1) ** 3)[:, None]
        if pm.size:
            fx -= (m[:, None] * fx).sum(0) / m.sum()
        return np.concatenate([v.ravel(), (a + fx).ravel()])
    return f


class Hybrid:
    def __init__(self, st: osteps.State, r_chain0, gamma_crit=1e-4, gamma_esc=1.5,
                 ghost_mass=1e-10, G=1.0):
        assert st.bh_mass.shape[0] == 1 and st.sys_off.shape[0] == 2
        self.st = st
        self.r_chain0, self.gamma_crit, self.gamma_esc = r_chain0, gamma_crit, gamma_esc
        self.ghost_mass, self.G = ghost_mass, G
        self.active = False
        self.star = []                      # -1 for the SMBH
        self.m = np.zeros(0)
        self.x = self.v = np.zeros((0, 3))
        self.R = np.zeros(3)
        self.V = np.zeros(3)
        self.M = 0.0
        self.r_chain = 0.0
        self.a_com = np.zeros(3)
        self.pert = np.zeros(0, np.int32)
        self.excl = np.zeros(st.pos.shape[0], bool)
        st.frozen = self.excl              # ghosts: never kicked, drifted or active
        self.starts = self.absorbed = self.escaped = self.ended = 0

    # -- chain bookkeeping
    def _reform(self, X, W):
        M = 0.0
        R = np.zeros(3)
        V = np.zeros(3)
        for i in range(self.m.size):
            M += self.m[i]
            R += self.m[i] * X[i]
            V += self.m[i] * W[i]
        self.R, self.V, self.M = R / M, V / M, M
        self.x = X - self.R
        self.v = W - self.V

    def _globals(self, V=None):
        V = self.V if V is None else V
        return self.R + self.x, V + self.v

    def _radius(self):
        return float(np.sqrt(max(((a[0] * a[0] + a[1] * a[1]) + a[2] * a[2]) for a in self.x)))

    def _write_smbh(self, V=None):
        """The SMBH member's global coordinates into its arrays (it is not a
        tree particle: reference only)."""
        X, W = self._globals(V)
        for i, s in enumerate(self.star):
            if s < 0:
                self.st.bh_pos[0] = X[i]
                self.st.bh_vel[0] = W[i]

    def _ghost(self, ids, mass):
        for s, mm in zip(ids, mass):
            self.st.mass[s] = mm * self.ghost_mass
            self.excl[s] = True

    def _restore(self, rows, X, W, mass):
        for s, x, w, mm in zip(rows, X, W, mass):
            self.st.pos[s] = x
            self.st.vel[s] = w
            self.st.mass[s] = mm
            self.excl[s] = False

    def _leave(self, leaves, V):
        """Members listed in `leaves` back to the tree with their global
        coordinates (velocities relative to V); returns the star rows."""
        X, W = self._globals(V)
        back = [i for i in sorted(leaves) if self.star[i] >= 0]
        rows = [self.star[i] for i in back]
        self._restore(rows, X[back], W[back], self.m[back])
        for i in leaves:
            if self.star[i] < 0:
                self.st.bh_pos[0] = X[i]
                self.st.bh_vel[0] = W[i]
        self.escaped += len(rows)
        return rows

    def _end(self):
        self.active = False
        self.star, self.m = [], np.zeros(0)
        self.x = self.v = np.zeros((0, 3))
        self.pert = np.zeros(0, np.int32)
        self.a_com = np.zeros(3)
        self.ended += 1

    # -- forces
    def forces(self, rows=None):
        """Forces of the listed stars (all if None).  Without a chain: the
        tree and the SMBH terms (and the SMBH's force).  With a chain: the
        tree without the SMBH (ghosts at their frozen places), then the
        coupling for the same stars; the chain particle's force and the
        perturber list from all stars."""
        st = self.st
        n = st.pos.shape[0]
        rows = np.arange(n) if rows is None else np.asarray(rows, np.int64)
        if not self.active:
            osteps.forces(st, None if rows.size == n else rows)
            return
        if rows.size:
            ev = oracle.tree_forces(st.pos, st.mass, st.eps, st.theta, st.leaf_size,
                                    st.group_size, active=None if rows.size == n else rows,
                                    softening=st.softening)
            st.acc[rows] = ev.acc[rows]
            st.pot[rows] = ev.pot[rows]
        X, _ = self._globals()
        r_crit = min(self.r_chain, self.r_chain0)
        self.pert = ochain.perturbers(st.pos, st.mass, self.R, self.M, r_crit, self.gamma_crit,
                                      self.excl)
        a, p, ac, _ = ochain.coupling(st.pos, st.mass, rows, self.R, self.M, X, self.m,
                                      self.pert, 0.0, self.excl, self.G)
        if rows.size:
            st.acc[rows] += a
            st.pot[rows] += p
        self.a_com = ac

    def _chain_step(self, dt, V_drift):
        """(3): the members over dt, the perturbers of the last coupling on
        the straight lines of this step's drift relative to the chain
        particle (which drifts with V_drift)."""
        px, pv, pm = ochain.predict(self.st.pos, self.st.vel, self.st.mass, self.pert, self.R,
                                    V_drift, 0.0)
        n = self.m.size
        sol = solve_ivp(_members_rhs(self.m, px, pv, pm, self.G), (0.0, dt),
                        np.concatenate([self.x.ravel(), self.v.ravel()]), method="DOP853",
                        rtol=1e-13, atol=1e-18)
        self.x = sol.y[:3 * n, -1].reshape(n, 3)
        self.v = sol.y[3 * n:, -1].reshape(n, 3)
        self.r_chain = self._radius()

    def _form(self, ids, X, W, mass):
        """A new chain: the SMBH (member 0, global X[0], W[0]) and the listed
        stars, which become ghosts."""
        self.star = [-1] + list(ids)
        self.m = np.concatenate([self.st.bh_mass[:1], mass])
        self._reform(X, W)
        self.r_chain = self._radius()
        self._ghost(ids, mass)
        self.active = True
        self.starts += 1

    # -- global steps
    def _maybe_start(self):
        """(8): stars within r_chain0 of the SMBH start a chain with it
        (SMBH first, then the stars in ascending order)."""
        st = self.st
        ids = ochain.within(st.pos, st.bh_pos[0], self.r_chain0).tolist()
        if not ids:
            return
        X = np.concatenate([st.bh_pos[:1], st.pos[ids]])
        W = np.concatenate([st.bh_vel[:1], st.vel[ids]])
        self._form(ids, X, W, st.mass[ids].copy())
        self.forces()

    def begin(self):
        self.forces()
        if not self.active:
            self._maybe_start()

    def _membership(self):
        """(4)-(5) at the end of a step (positions and velocities in step)."""
        st = self.st
        px = st.pos[self.pert] - self.R
        massive = np.array([s < 0 for s in self.star])
        r = ochain.membership(self.x, self.v, self.m, massive, 0, self.r_chain, self.r_chain0,
                              self.gamma_esc, px)
        if not r["terminate"] and r["absorb"].size == 0 and r["escape"].size == 0:
            return
        n = len(self.star)
        leaves = set(range(n)) if r["terminate"] else set(r["escape"].tolist())
        X, W = self._globals()
        self._leave(leaves, self.V)
        if r["terminate"]:
            self._end()
            self.forces()
            return
        keep = [i for i in range(n) if i not in leaves]
        join = [int(self.pert[a]) for a in r["absorb"]]
        jm = st.mass[join].copy()
        self.star = [self.star[i] for i in keep] + join
        self.m = np.concatenate([self.m[keep], jm])
        self._reform(np.concatenate([X[keep], st.pos[join]]),
                     np.concatenate([W[keep], st.vel[join]]))
        self.r_chain = self._radius()
        self._ghost(join, jm)
        self.absorbed += len(join)
        self.forces()

    def step(self, dt):
        """One global step of dt."""
        st = self.st
        if not self.active:
            osteps.kdk_step(st, dt)
            self._maybe_start()
            return
        # (6) opening half kick of the stars (not the ghosts) and of the chain particle
        osteps._kick_stars(st, dt)
        V_half = self.V + self.a_com * (0.5 * dt)
        # (3) the chain step
        self._chain_step(dt, V_half)
        # (6) drift; (6b) forces with the members about the drifted chain particle
        osteps._drift_stars(st, dt)
        self.R = self.R + V_half * dt
        self.V = V_half
        self.forces()
        # (6c) closing half kick
        osteps._kick_stars(st, dt)
        self.V = self.V + self.a_com * (0.5 * dt)
        self._write_smbh()
        # (4)-(5), then (8)
        self._membership()
        if not self.active:
            self._maybe_start()

    # -- block substeps
    def _active_now(self, rows, level, nlev, k):
        """Which of the listed stars have a step ending at substep k."""
        rows = np.asarray(rows, np.int64)
        per = (1 << (nlev - 1 - level[rows].astype(np.int64)))
        return (k % per) == 0

    def _sync_vel(self, rows, level, dt_max):
        """Velocities of stars at the end of their own step: the pending
        closing half kick with their current force."""
        rows = np.asarray(rows, np.int64)
        v = self.st.vel[rows].copy()
        if rows.size:
            oracle.kick(v, self.st.acc[rows], dt_max, level=level[rows])
        return v

    def _half_back(self, rows, level, nlev, dt_max):
        """Stars that start on the finest level: stored half a kick back so
        the next substep's closing half kick brings them into step."""
        rows = np.asarray(rows, np.int32)
        if rows.size:
            level[rows] = nlev - 1
            oracle.kick(self.st.vel, self.st.acc, -dt_max, idx=rows, level=level)

    def _start_block(self, level, nlev, k, dt_max):
        """(8) at substep k: stars within r_chain0 of the SMBH whose own step
        ends at k start a chain with it, all velocities in step."""
        st = self.st
        ids = ochain.within(st.pos, st.bh_pos[0], self.r_chain0)
        ids = ids[self._active_now(ids, level, nlev, k)].tolist() if ids.size else []
        if not ids:
            return
        dt_min = dt_max * 2.0 ** -(nlev - 1)
        bv = st.bh_vel[:1].copy()
        oracle.kick(bv, st.bh_acc[:1], dt_min)          # the SMBH's closing half kick
        X = np.concatenate([st.bh_pos[:1], st.pos[ids]])
        W = np.concatenate([bv, self._sync_vel(ids, level, dt_max)])
        self._form(ids, X, W, st.mass[ids].copy())
        self.forces(np.zeros(0, np.int64))
        self.V = self.V - self.a_com * (0.5 * dt_min)

    def _membership_block(self, level, nlev, k, dt_max):
        """(4)-(5) at substep k with every velocity in step: absorption only
        of perturbers whose own step ends at k."""
        st = self.st
        dt_min = dt_max * 2.0 ** -(nlev - 1)
        Vs = self.V + self.a_com * (0.5 * dt_min)        # the chain particle's closing half kick
        cand = np.asarray(self.pert, np.int64)
        cand = cand[self._active_now(cand, level, nlev, k)] if cand.size else cand
        px = st.pos[cand] - self.R
        massive = np.array([s < 0 for s in self.star])
        r = ochain.membership(self.x, self.v, self.m, massive, 0, self.r_chain, self.r_chain0,
                              self.gamma_esc, px)
        if not r["terminate"] and r["absorb"].size == 0 and r["escape"].size == 0:
            return
        n = len(self.star)
        leaves = set(range(n)) if r["terminate"] else set(r["escape"].tolist())
        X, W = self._globals(Vs)
        back = self._leave(leaves, Vs)
        if r["terminate"]:
            self._end()
            self.forces(np.asarray(back, np.int64))
            self._half_back(back, level, nlev, dt_max)
            oracle.kick(st.bh_vel, st.bh_acc, -dt_min)   # the free SMBH, half a kick back
            return
        keep = [i for i in range(n) if i not in leaves]
        join = [int(cand[a]) for a in r["absorb"]]
        jm = st.mass[join].copy()
        self.star = [self.star[i] for i in keep] + join
        self.m = np.concatenate([self.m[keep], jm])
        self._reform(np.concatenate([X[keep], st.pos[join]]),
                     np.concatenate([W[keep], self._sync_vel(join, level, dt_max)]))
        self.r_chain = self._radius()
        self._ghost(join, jm)
        self.absorbed += len(join)
        self.forces(np.asarray(back, np.int64))
        self._half_back(back, level, nlev, dt_max)
        self.V = self.V - self.a_com * (0.5 * dt_min)

    def step_block(self, level, t4e2, k, dt_max, nlev):
        """One substep at counter k; returns k + 1."""
        st = self.st
        if not self.active:
            k, _ = osteps.block_substep(st, level, t4e2, k, dt_max, nlev)
            self._start_block(level, nlev, k, dt_max)
            return k
        dt = dt_max * 2.0 ** -(nlev - 1)
        # (1), (6): the stars' closing kicks, levels and opening kicks
        act = osteps._active(st, level, nlev, k)
        if k > 0:
            oracle.kick(st.vel, st.acc, dt_max, idx=act, level=level)
        oracle.levels(st.acc, t4e2, level, dt_max, nlev, k, idx=act)
        oracle.kick(st.vel, st.acc, dt_max, idx=act, level=level)
        # the chain particle on the finest level: closing (not at k = 0) and
        # opening half kicks with its last force
        if k != 0:
            self.V = self.V + self.a_com * (0.5 * dt)
        self.V = self.V + self.a_com * (0.5 * dt)
        # (3) the chain step over the substep
        self._chain_step(dt, self.V)
        # drift; forces of the stars active at the new k
        osteps._drift_stars(st, dt)
        self.R = self.R + self.V * dt
        k += 1
        self.forces(osteps._active(st, level, nlev, k).astype(np.int64))
        self._write_smbh(self.V + self.a_com * (0.5 * dt))
        # (4)-(5), then (8)
        self._membership_block(level, nlev, k, dt_max)
        if not self.active:
            self._start_block(level, nlev, k, dt_max)
        return k
