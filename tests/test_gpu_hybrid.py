"""The hybrid step (tg_hybrid_*) against the oracle's hybrid run: the same
recipe composed of the oracle's pieces, with the chain members integrated
by a high-order Runge-Kutta method instead of the regularised chain.

Workload: a Dehnen gamma = 1.5 cusp of 16 384 stars with an SMBH of 0.01 at
rest at its centre, eps = 1e-3, theta = 0.5; r_chain0 = 0.04, gamma_crit =
1e-4, gamma_esc = 1.2, dt = 1e-3: the chain starts with 11 stars and both
absorbs and loses members within 22 steps.  Ghost members keep the state
they joined with, so only the stars outside the chain are compared.  Chain starts, absorptions and escapes
must agree event for event, the member lists exactly, and the stars, the
chain particle and the members to the accuracy of the two chain
integrations (1e-9 relative).
"""
import sys

import numpy as np
import pytest

from oracle import hybrid as ohybrid
from oracle import steps as osteps
from paper_1507_01009_amd import ics

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _workload(n=16384):
    pos, vel, m = ics.dehnen(n, 1.5, ics.SEED_BASE + 61)
    return ics.Workload("cusp_bh", pos, vel, m, 1e-3, 0.5, np.array([0, n]),
                        np.zeros((1, 3)), np.zeros((1, 3)), np.array([0.01]),
                        np.array([1e-3]), np.zeros(1, np.int32))


def _ostate(w):
    return osteps.State(w.pos.copy(), w.vel.copy(), w.mass.copy(), w.eps, w.theta,
                        w.sys_off.copy(), w.bh_pos.copy(), w.bh_vel.copy(), w.bh_mass.copy(),
                        w.bh_eps.copy(), np.array([0, 1], np.int64))


@pytest.mark.parametrize("steps", [22])
def test_hybrid_steps_match_the_oracle(steps):
    say("hybrid", steps)
    from paper_1507_01009_amd import binding as B
    from test_gpu_steps import Dev
    w = _workload()
    dt = 1e-3
    ctx = B.Context(w.n)
    d = Dev(ctx, w)
    hy = B.Hybrid(ctx, d.sys, r_chain0=0.04, gamma_esc=1.2)
    hy.begin()
    oh = ohybrid.Hybrid(_ostate(w), r_chain0=0.04, gamma_esc=1.2)
    oh.begin()
    s = hy.state()
    assert s["active"] and oh.active and s["members"].tolist() == oh.star
    for k in range(steps):
        hy.step(dt)
        oh.step(dt)
        s = hy.state()
        say("  step %d: members %d perturbers %d absorbed %d escaped %d" % (
            k, len(s["members"]), s["n_perturbers"], s["absorbed"], s["escaped"]))
        assert s["active"] == oh.active
        assert s["members"].tolist() == oh.star
        assert (s["starts"], s["absorbed"], s["escaped"], s["ended"]) == (
            oh.starts, oh.absorbed, oh.escaped, oh.ended)
        if s["active"]:
            assert s["n_perturbers"] == oh.pert.size
    assert s["absorbed"] > 0 and s["escaped"] > 0
    ctx.sync()
    h = d.host()
    st = oh.st
    live = ~oh.excl
    sc = np.abs(st.pos).max()
    assert np.max(np.abs(h["pos"][live] - st.pos[live])) <= 1e-9 * sc
    assert np.max(np.abs(h["vel"][live] - st.vel[live])) <= 1e-9 * np.abs(st.vel).max()
    assert np.allclose(h["mass"] if "mass" in h else d.mass.cpu().numpy(), st.mass, rtol=0, atol=0)
    if oh.active:
        assert np.allclose(s["com"], oh.R, rtol=0, atol=1e-12)
        assert np.allclose(s["com_vel"], oh.V, rtol=0, atol=1e-10)
        assert np.max(np.abs(s["x"] - oh.x)) <= 1e-9 * np.abs(oh.x).max()
        assert np.max(np.abs(s["v"] - oh.v)) <= 1e-8 * np.abs(oh.v).max()
        assert abs(s["energy_error"]) < 1e-9
    hy.close()


def test_hybrid_chain_ends_and_restarts():
    """r_chain0 = 0.02, gamma_esc = 1.0, dt = 2e-3 on the same cusp: the
    chain formed at the start ends after one step (its one star escapes),
    a new chain starts later and then absorbs and loses stars; every event,
    member list and the final state as in the oracle."""
    say("hybrid end and restart")
    from paper_1507_01009_amd import binding as B
    from test_gpu_steps import Dev
    w = _workload()
    dt = 2e-3
    ctx = B.Context(w.n)
    d = Dev(ctx, w)
    hy = B.Hybrid(ctx, d.sys, r_chain0=0.02, gamma_esc=1.0)
    hy.begin()
    oh = ohybrid.Hybrid(_ostate(w), r_chain0=0.02, gamma_esc=1.0)
    oh.begin()
    for k in range(40):
        hy.step(dt)
        oh.step(dt)
        s = hy.state()
        assert s["active"] == oh.active, k
        assert s["members"].tolist() == oh.star, k
        assert (s["starts"], s["absorbed"], s["escaped"], s["ended"]) == (
            oh.starts, oh.absorbed, oh.escaped, oh.ended), k
    say("  starts %d ended %d absorbed %d escaped %d" % (s["starts"], s["ended"], s["absorbed"],
                                                         s["escaped"]))
    assert s["ended"] >= 1 and s["starts"] >= 2 and s["absorbed"] > 0 and s["escaped"] > 0
    ctx.sync()
    h = d.host()
    st = oh.st
    live = ~oh.excl
    assert np.max(np.abs(h["pos"][live] - st.pos[live])) <= 1e-9 * np.abs(st.pos).max()
    assert np.max(np.abs(h["vel"][live] - st.vel[live])) <= 1e-9 * np.abs(st.vel).max()
    assert np.array_equal(d.mass.cpu().numpy(), st.mass)
    hy.close()


def test_hybrid_errors():
    say("hybrid errors")
    from paper_1507_01009_amd import binding as B
    from test_gpu_steps import Dev
    w = _workload(4096)
    ctx = B.Context(w.n)
    d = Dev(ctx, w)
    with pytest.raises(B.TGError):
        B.Hybrid(ctx, d.sys, r_chain0=0.0)
    with pytest.raises(B.TGError):
        B.Hybrid(ctx, d.sys, r_chain0=0.01, ghost_mass=1.0)
    hy = B.Hybrid(ctx, d.sys, r_chain0=0.01)
    with pytest.raises(B.TGError):
        hy.step(-1.0)
    hy.close()


def test_hybrid_block_substeps_match_the_oracle():
    """Block substeps (8 levels, dt_max = 2^-6) with the chain particle on
    the finest level: 130 substeps, with absorptions and escapes."""
    say("hybrid block")
    from paper_1507_01009_amd import binding as B
    from test_gpu_steps import Dev, _blocks
    w = _workload()
    nlev, dt_max, nsub = 8, 2.0 ** -6, 130
    ctx = B.Context(w.n)
    d = Dev(ctx, w)
    blk, keep = _blocks(ctx, w, nlev, dt_max)
    hy = B.Hybrid(ctx, d.sys, r_chain0=0.04, gamma_esc=1.2)
    hy.begin()
    oh = ohybrid.Hybrid(_ostate(w), r_chain0=0.04, gamma_esc=1.2)
    oh.begin()
    level = np.zeros(w.n, np.uint8)
    t4e2 = np.full(w.n, 0.3 ** 4 * w.eps ** 2)
    k = 0
    for i in range(nsub):
        hy.step_block(blk)
        k = oh.step_block(level, t4e2, k, dt_max, nlev)
        s = hy.state()
        assert s["members"].tolist() == oh.star, i
        assert (s["starts"], s["absorbed"], s["escaped"], s["ended"]) == (
            oh.starts, oh.absorbed, oh.escaped, oh.ended), i
    say("  absorbed %d escaped %d members %d" % (s["absorbed"], s["escaped"],
                                                 len(s["members"])))
    assert s["absorbed"] > 0 and s["escaped"] > 0
    ctx.sync()
    assert int(keep[4].item()) == k == nsub
    assert np.array_equal(keep[0].cpu().numpy()[~oh.excl], level[~oh.excl])
    h = d.host()
    st = oh.st
    live = ~oh.excl
    assert np.max(np.abs(h["pos"][live] - st.pos[live])) <= 1e-9 * np.abs(st.pos).max()
    assert np.max(np.abs(h["vel"][live] - st.vel[live])) <= 1e-9 * np.abs(st.vel).max()
    assert np.array_equal(d.mass.cpu().numpy(), st.mass)
    assert np.allclose(s["com"], oh.R, rtol=0, atol=1e-12)
    assert np.max(np.abs(s["x"] - oh.x)) <= 1e-9 * np.abs(oh.x).max()
    hy.close()


def test_hybrid_block_chain_ends_and_restarts():
    """Block substeps (8 levels, dt_max = 2^-6) with r_chain0 = 0.02 and
    gamma_esc = 1.0: the first chain ends at substep 16, its star returns
    on the finest level, and a new chain starts some 300 substeps later;
    events, member lists, levels and the final state as in the oracle."""
    say("hybrid block end and restart")
    from paper_1507_01009_amd import binding as B
    from test_gpu_steps import Dev, _blocks
    w = _workload()
    nlev, dt_max, nsub = 8, 2.0 ** -6, 360
    ctx = B.Context(w.n)
    d = Dev(ctx, w)
    blk, keep = _blocks(ctx, w, nlev, dt_max)
    hy = B.Hybrid(ctx, d.sys, r_chain0=0.02, gamma_esc=1.0)
    hy.begin()
    oh = ohybrid.Hybrid(_ostate(w), r_chain0=0.02, gamma_esc=1.0)
    oh.begin()
    level = np.zeros(w.n, np.uint8)
    t4e2 = np.full(w.n, 0.3 ** 4 * w.eps ** 2)
    k = 0
    for i in range(nsub):
        hy.step_block(blk)
        k = oh.step_block(level, t4e2, k, dt_max, nlev)
        s = hy.state()
        assert s["members"].tolist() == oh.star, i
        assert (s["starts"], s["absorbed"], s["escaped"], s["ended"]) == (
            oh.starts, oh.absorbed, oh.escaped, oh.ended), i
    say("  starts %d ended %d members %d" % (s["starts"], s["ended"], len(s["members"])))
    assert s["ended"] >= 1 and s["starts"] >= 2 and s["active"]
    ctx.sync()
    assert int(keep[4].item()) == k == nsub
    assert np.array_equal(keep[0].cpu().numpy()[~oh.excl], level[~oh.excl])
    h = d.host()
    st = oh.st
    live = ~oh.excl
    assert np.max(np.abs(h["pos"][live] - st.pos[live])) <= 1e-9 * np.abs(st.pos).max()
    assert np.max(np.abs(h["vel"][live] - st.vel[live])) <= 1e-9 * np.abs(st.vel).max()
    assert np.array_equal(d.mass.cpu().numpy(), st.mass)
    hy.close()


def test_context_close_closes_the_driver_first():
    """Closing the context while a driver lives closes the driver first (it
    uses the context's stream); closing the driver again is a no-op."""
    say("hybrid lifetime")
    from paper_1507_01009_amd import binding as B
    from test_gpu_steps import Dev
    w = _workload(4096)
    ctx = B.Context(w.n)
    d = Dev(ctx, w)
    hy = B.Hybrid(ctx, d.sys, r_chain0=0.04)
    hy.begin()
    ctx.close()
    assert not hy.h and not ctx.h
    hy.close()
