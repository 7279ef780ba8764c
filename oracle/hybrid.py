"""Plain CPU oracle of the hybrid step (TEST INFRASTRUCTURE ONLY).

Nothing in the product library imports this module; only the tests use it.
It composes the oracle's own pieces in the order of the hybrid recipe
(Sec. 2), read as global kick-drift-kick steps with one SMBH:

* no chain: one KDK step of stars and SMBH (:func:`oracle.steps.kdk_step`);
  then the stars within r_chain0 of the SMBH start a chain with it;
* with a chain: the members (SMBH first, then stars in ascending order) are
  integrated in the chain's centre-of-mass frame; their stars stay in the
  arrays as ghosts (mass times ghost_mass, excluded from the coupling) and
  get the members' global coordinates after every stage that moves them;
* block substeps (:meth:`Hybrid.step_block`): the stars' part of
  :func:`oracle.steps.block_substep` with the ghosts frozen, the chain
  particle on the finest level (closing and opening half kicks with its last
  force, then the drift), the members over the substep, forces for the stars
  active at the new k only (tree without the SMBH, then the coupling for the
  same stars; the chain particle's force from all stars), membership; stars
  that leave the chain go to the finest level and get their forces at once;
* a step: half kick of every star and of the chain particle (its force from
  the coupling, Eq. 3 included); the perturbers of the last coupling taken
  relative to the chain particle; drift of every star and of the chain
  particle; tree forces without the SMBH, with the ghosts carried by the
  chain particle (R plus the members' offsets from the start of the step);
  the members over the whole step with those perturbers moving on straight
  lines (their tidal part, the mean force removed), here by a high-order
  Runge-Kutta integration (scipy DOP853), not the regularised chain; ghosts
  rewritten; the coupling with the members' new positions;
  second half kick; ghosts rewritten; membership (Eq. 4, Eq. 5); after a
  change the centre of mass is re-formed and the forces evaluated again; a
  chain that ends returns every member, and a new one may start.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import solve_ivp

import oracle
from oracle import chain as ochain
from oracle import steps as osteps


def _members_rhs(m, px, pv, pm, G):
    n = m.size

    def f(t, s):
        x = s[:3 * n].reshape(n, 3)
        v = s[3 * n:].reshape(n, 3)
        a = np.zeros((n, 3))
        for i in range(n):
            for j in range(n):
                if i != j:
                    d = x[j] - x[i]
                    a[i] += G * m[j] * d / np.linalg.norm(d) ** 3
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
        st.frozen = self.excl              # ghosts are held still in block substeps
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

    def _globals(self):
        return self.R + self.x, self.V + self.v

    def _radius(self):
        return float(np.sqrt(max(((a[0] * a[0] + a[1] * a[1]) + a[2] * a[2]) for a in self.x)))

    def _write(self):
        X, W = self._globals()
        for i, s in enumerate(self.star):
            if s < 0:
                self.st.bh_pos[0] = X[i]
                self.st.bh_vel[0] = W[i]
            else:
                self.st.pos[s] = X[i]
                self.st.vel[s] = W[i]

    def _ghosts(self, ids, mass, ghost):
        for s, mm in zip(ids, mass):
            self.st.mass[s] = mm * self.ghost_mass if ghost else mm
            self.excl[s] = ghost

    # -- forces
    def forces(self):
        st = self.st
        if not self.active:
            osteps.forces(st)
            return
        self._write()
        ev = oracle.tree_forces(st.pos, st.mass, st.eps, st.theta, st.leaf_size, st.group_size,
                                softening=st.softening)
        st.acc[:] = ev.acc
        st.pot[:] = ev.pot
        X, _ = self._globals()
        r_crit = min(self.r_chain, self.r_chain0)
        self.pert = ochain.perturbers(st.pos, st.mass, self.R, self.M, r_crit, self.gamma_crit,
                                      self.excl)
        n = st.pos.shape[0]
        a, p, ac, _ = ochain.coupling(st.pos, st.mass, np.arange(n), self.R, self.M, X, self.m,
                                      self.pert, 0.0, self.excl, self.G)
        st.acc += a
        st.pot += p
        self.a_com = ac

    def _perturbers(self):
        return ochain.predict(self.st.pos, self.st.vel, self.st.mass, self.pert, self.R, self.V,
                              0.0)

    def _maybe_start(self):
        st = self.st
        ids = ochain.within(st.pos, st.bh_pos[0], self.r_chain0).tolist()
        if not ids:
            return
        self.star = [-1] + ids
        self.m = np.concatenate([st.bh_mass[:1], st.mass[ids]])
        X = np.concatenate([st.bh_pos[:1], st.pos[ids]])
        W = np.concatenate([st.bh_vel[:1], st.vel[ids]])
        self._reform(X, W)
        self.r_chain = self._radius()
        self._ghosts(ids, self.m[1:], True)
        self.active = True
        self.starts += 1
        self.forces()

    def begin(self):
        self.forces()
        if not self.active:
            self._maybe_start()

    def _membership(self):
        px, _, _ = self._perturbers()
        massive = np.array([s < 0 for s in self.star])
        r = ochain.membership(self.x, self.v, self.m, massive, 0, self.r_chain, self.r_chain0,
                              self.gamma_esc, px)
        if not r["terminate"] and r["absorb"].size == 0 and r["escape"].size == 0:
            return
        X, W = self._globals()
        leaves = set(range(len(self.star))) if r["terminate"] else set(r["escape"].tolist())
        back = [(self.star[i], self.m[i]) for i in sorted(leaves) if self.star[i] >= 0]
        keep = [i for i in range(len(self.star)) if i not in leaves]
        self._write()
        self._ghosts([b[0] for b in back], [b[1] for b in back], False)
        self.escaped += len(back)
        if r["terminate"]:
            self.active = False
            self.star, self.m = [], np.zeros(0)
            self.x = self.v = np.zeros((0, 3))
            self.pert = np.zeros(0, np.int32)
            self.ended += 1
            self.forces()
            return
        join = [int(self.pert[a]) for a in r["absorb"]]
        st = self.st
        jm = st.mass[join].copy()
        self.star = [self.star[i] for i in keep] + join
        m = np.concatenate([self.m[keep], jm])
        X = np.concatenate([X[keep], st.pos[join]])
        W = np.concatenate([W[keep], st.vel[join]])
        self.m = m
        self._reform(X, W)
        self.r_chain = self._radius()
        self._ghosts(join, jm, True)
        self.absorbed += len(join)
        self.forces()

    def step(self, dt):
        st = self.st
        if not self.active:
            osteps.kdk_step(st, dt)
            self._maybe_start()
            return
        oracle.kick(st.vel, st.acc, dt)
        self.V = self.V + self.a_com * (0.5 * dt)
        px, pv, pm = self._perturbers()
        oracle.drift(st.pos, st.vel, dt)
        self.R = self.R + self.V * dt
        # tree forces with the ghosts carried by the chain particle (R plus
        # the members' offsets from the start of the step)
        self._write()
        ev = oracle.tree_forces(st.pos, st.mass, st.eps, st.theta, st.leaf_size, st.group_size,
                                softening=st.softening)
        st.acc[:] = ev.acc
        st.pot[:] = ev.pot
        n = self.m.size
        sol = solve_ivp(_members_rhs(self.m, px, pv, pm, self.G), (0.0, dt),
                        np.concatenate([self.x.ravel(), self.v.ravel()]), method="DOP853",
                        rtol=1e-13, atol=1e-18)
        self.x = sol.y[:3 * n, -1].reshape(n, 3)
        self.v = sol.y[3 * n:, -1].reshape(n, 3)
        self.r_chain = self._radius()
        # the coupling with the members' new positions
        self._write()
        X, _ = self._globals()
        r_crit = min(self.r_chain, self.r_chain0)
        self.pert = ochain.perturbers(st.pos, st.mass, self.R, self.M, r_crit, self.gamma_crit,
                                      self.excl)
        a, p, ac, _ = ochain.coupling(st.pos, st.mass, np.arange(st.pos.shape[0]), self.R,
                                      self.M, X, self.m, self.pert, 0.0, self.excl, self.G)
        st.acc += a
        st.pot += p
        self.a_com = ac
        oracle.kick(st.vel, st.acc, dt)
        self.V = self.V + self.a_com * (0.5 * dt)
        self._write()
        self._membership()
        if not self.active:
            self._maybe_start()

    # -- block substeps
    def _forces_list(self, rows):
        st = self.st
        rows = np.asarray(rows, np.int64)
        if not self.active:
            osteps.forces(st, rows)
            return
        self._write()
        if rows.size:
            ev = oracle.tree_forces(st.pos, st.mass, st.eps, st.theta, st.leaf_size,
                                    st.group_size, active=rows, softening=st.softening)
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

    def _start_block(self):
        st = self.st
        ids = ochain.within(st.pos, st.bh_pos[0], self.r_chain0).tolist()
        if not ids:
            return
        self.star = [-1] + ids
        self.m = np.concatenate([st.bh_mass[:1], st.mass[ids]])
        X = np.concatenate([st.bh_pos[:1], st.pos[ids]])
        W = np.concatenate([st.bh_vel[:1], st.vel[ids]])
        self._reform(X, W)
        self.r_chain = self._radius()
        self._ghosts(ids, self.m[1:], True)
        self.active = True
        self.starts += 1
        self._forces_list([])

    def _membership_block(self, level, nlev):
        px, _, _ = self._perturbers()
        massive = np.array([s < 0 for s in self.star])
        r = ochain.membership(self.x, self.v, self.m, massive, 0, self.r_chain, self.r_chain0,
                              self.gamma_esc, px)
        if not r["terminate"] and r["absorb"].size == 0 and r["escape"].size == 0:
            return
        X, W = self._globals()
        leaves = set(range(len(self.star))) if r["terminate"] else set(r["escape"].tolist())
        back = [(self.star[i], self.m[i]) for i in sorted(leaves) if self.star[i] >= 0]
        keep = [i for i in range(len(self.star)) if i not in leaves]
        self._write()
        self._ghosts([b[0] for b in back], [b[1] for b in back], False)
        self.escaped += len(back)
        back_ids = [b[0] for b in back]
        if r["terminate"]:
            self.active = False
            self.star, self.m = [], np.zeros(0)
            self.x = self.v = np.zeros((0, 3))
            self.pert = np.zeros(0, np.int32)
            self.ended += 1
        else:
            join = [int(self.pert[a]) for a in r["absorb"]]
            st = self.st
            jm = st.mass[join].copy()
            self.star = [self.star[i] for i in keep] + join
            self.m = np.concatenate([self.m[keep], jm])
            self._reform(np.concatenate([X[keep], st.pos[join]]),
                         np.concatenate([W[keep], st.vel[join]]))
            self.r_chain = self._radius()
            self._ghosts(join, jm, True)
            self.absorbed += len(join)
        level[back_ids] = nlev - 1
        self._forces_list(back_ids)

    def step_block(self, level, t4e2, k, dt_max, nlev):
        """One substep at counter k; returns k + 1."""
        st = self.st
        if not self.active:
            k, _ = osteps.block_substep(st, level, t4e2, k, dt_max, nlev)
            self._start_block()
            return k
        dt = dt_max * 2.0 ** -(nlev - 1)
        act = osteps._active(st, level, nlev, k)
        if k > 0:
            oracle.kick(st.vel, st.acc, dt_max, idx=act, level=level)
        oracle.levels(st.acc, t4e2, level, dt_max, nlev, k, idx=act)
        oracle.kick(st.vel, st.acc, dt_max, idx=act, level=level)
        if k != 0:
            self.V = self.V + self.a_com * (0.5 * dt)
        self.V = self.V + self.a_com * (0.5 * dt)
        px, pv, pm = self._perturbers()
        osteps._drift_stars(st, dt)
        k += 1
        self.R = self.R + self.V * dt
        # tree forces of the stars active at the new k, with the ghosts
        # carried by the chain particle
        rows = osteps._active(st, level, nlev, k).astype(np.int64)
        self._write()
        if rows.size:
            ev = oracle.tree_forces(st.pos, st.mass, st.eps, st.theta, st.leaf_size,
                                    st.group_size, active=rows, softening=st.softening)
            st.acc[rows] = ev.acc[rows]
            st.pot[rows] = ev.pot[rows]
        n = self.m.size
        sol = solve_ivp(_members_rhs(self.m, px, pv, pm, self.G), (0.0, dt),
                        np.concatenate([self.x.ravel(), self.v.ravel()]), method="DOP853",
                        rtol=1e-13, atol=1e-18)
        self.x = sol.y[:3 * n, -1].reshape(n, 3)
        self.v = sol.y[3 * n:, -1].reshape(n, 3)
        self.r_chain = self._radius()
        # the coupling for the same stars with the members' new positions
        self._write()
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
        self._membership_block(level, nlev)
        if self.active:
            self._write()
        else:
            self._start_block()
        return k
