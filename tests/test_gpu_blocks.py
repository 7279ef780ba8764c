"""Block steps driven from the host (tg_step_blocks) and the tiled active
set (tg_active_set), through the C ABI.

tg_step_blocks must give the results of as many tg_step_block calls bit for
bit (positions, velocities, accelerations, potentials, levels, the substep
counter, the active set and the SMBH state), while it runs the substeps that
no star takes part in without the tree's launches.  It is also compared with
the oracle's block substeps.  The active set is compared with the oracle's
list on ragged sizes around the 1024-star tiles.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import steps as osteps
from paper_1507_01009_amd import ics
from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n", [1, 1023, 1024, 1025, 70001])
@pytest.mark.parametrize("k,k_add", [(0, 0), (6, 2), (127, 0), (-3, 1)])
def test_active_set_on_ragged_tiles(n, k, k_add):
    say("active set", n, k, k_add)
    import torch
    from paper_1507_01009_amd import binding as B
    rng = np.random.default_rng(n + 7 * abs(k))
    level = rng.integers(0, 10, n).astype(np.uint8)     # some beyond the finest
    ctx = B.Context(n)
    dl = to_dev(level)
    dk = to_dev(np.array([k], np.int64))
    idx = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    na = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.active_set(dl, 8, dk, idx, na, k_add=k_add)
    ctx.sync()
    ref = oracle.active_at(np.minimum(level, 7), 8, k + k_add)
    assert int(na.item()) == ref.size
    got = idx.cpu().numpy()
    assert np.array_equal(got[:ref.size], ref)
    assert np.all(got[ref.size:] == -7)                  # nothing written past the list


def test_active_set_empty_input():
    say("active set n=0")
    import torch
    from paper_1507_01009_amd import binding as B
    ctx = B.Context(16)
    na = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    idx = torch.zeros(16, dtype=torch.int32, device="cuda")
    dk = to_dev(np.array([0], np.int64))
    ctx.active_set(torch.zeros(0, dtype=torch.uint8, device="cuda"), 8, dk, idx, na)
    ctx.sync()
    assert int(na.item()) == 0


def _run(w, nlev, dt_max, nsub, driver, frozen=None, every=0, softening=None):
    import torch
    from paper_1507_01009_amd import binding as B
    from test_gpu_steps import Dev, _blocks
    ctx = B.Context(w.n, max_systems=w.sys_off.shape[0] - 1)
    if softening:
        ctx.set_softening(softening)
    d = Dev(ctx, w)
    keep_fz = None
    if frozen is not None:
        keep_fz = to_dev(frozen)
        d.sys.frozen = B._ptr(keep_fz)
    blk, keep = _blocks(ctx, w, nlev, dt_max)
    blk.rebuild_every = every
    ctx.forces(d.sys)
    n_idle = 0
    if driver:
        n_idle = ctx.step_blocks(d.sys, blk, nsub)
    else:
        for _ in range(nsub):
            ctx.step_block(d.sys, blk)
    ctx.sync()
    h = d.host()
    na = int(keep[3].item())
    h["level"] = keep[0].cpu().numpy()
    h["k"] = int(keep[4].item())
    h["n_active"] = na
    h["idx"] = keep[2].cpu().numpy()[:na]
    del keep_fz
    return h, n_idle


@pytest.mark.parametrize("case", ["paper_dt", "coarse_dt", "frozen_refit"])
def test_driver_equals_single_substeps_bitwise(case):
    say("driver bitwise", case)
    w = ics.hernquist_c4(n=16384)
    frozen, every = None, 0
    if case == "paper_dt":
        nlev, dt_max, nsub = 8, 2.0 ** -6, 300
    elif case == "coarse_dt":
        nlev, dt_max, nsub = 8, 0.25, 40
    else:
        nlev, dt_max, nsub = 8, 2.0 ** -6, 200
        frozen = np.zeros(w.n, np.uint8)
        frozen[::37] = 1
        every = 4
    a, _ = _run(w, nlev, dt_max, nsub, False, frozen, every)
    b, n_idle = _run(w, nlev, dt_max, nsub, True, frozen, every)
    say("  idle substeps %d of %d" % (n_idle, nsub))
    if case != "coarse_dt":
        assert n_idle > nsub // 2
    assert a["k"] == b["k"] == nsub
    assert a["n_active"] == b["n_active"]
    assert np.array_equal(a["idx"], b["idx"])
    for key in ("pos", "vel", "acc", "pot", "level", "bpos", "bvel", "bacc"):
        assert np.array_equal(a[key], b[key]), key


def test_driver_matches_oracle():
    say("driver vs oracle")
    w = ics.hernquist_c4(n=8192)
    nlev, dt_max, nsub = 8, 2.0 ** -6, 130
    h, n_idle = _run(w, nlev, dt_max, nsub, True)
    from test_gpu_steps import ostate
    st = ostate(w)
    osteps.forces(st)
    level = np.zeros(w.n, np.uint8)
    t4e2 = np.full(w.n, 0.3 ** 4 * w.eps ** 2)
    k, act = 0, None
    for _ in range(nsub):
        k, act = osteps.block_substep(st, level, t4e2, k, dt_max, nlev)
    assert n_idle > 0
    assert np.array_equal(h["level"], level)
    assert h["n_active"] == act.size and np.array_equal(h["idx"], act)
    assert np.max(np.abs(h["pos"] - st.pos)) <= 1e-12 * np.abs(st.pos).max()
    assert np.max(np.abs(h["vel"] - st.vel)) <= 1e-11 * np.abs(st.vel).max()
    assert np.max(np.abs(h["bpos"] - st.bh_pos)) <= 1e-14


@pytest.mark.parametrize("nsub", [0, 1, 2, 25])
def test_driver_with_every_star_frozen(nsub):
    """No star can become active: after the first substep every one runs in
    the short form; the stars stay put and the SMBH moves as with single
    substeps."""
    say("driver all frozen", nsub)
    w = ics.hernquist_c4(n=4096)
    frozen = np.ones(w.n, np.uint8)
    a, _ = _run(w, 8, 2.0 ** -6, nsub, False, frozen)
    b, n_idle = _run(w, 8, 2.0 ** -6, nsub, True, frozen)
    assert n_idle == max(0, nsub - 1)
    assert np.array_equal(b["pos"], w.pos) and np.array_equal(b["vel"], w.vel)
    assert b["k"] == nsub and b["n_active"] == 0
    for key in ("bpos", "bvel", "bacc", "acc"):
        assert np.array_equal(a[key], b[key]), key


def test_driver_errors():
    say("driver errors")
    import torch
    from paper_1507_01009_amd import binding as B
    from test_gpu_steps import Dev, _blocks
    w = ics.hernquist_c4(n=4096)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = B.Context(w.n, stream=s)
        d = Dev(ctx, w)
        blk, keep = _blocks(ctx, w, 8, 2.0 ** -6)
        ctx.forces(d.sys)
        ctx.sync()
        with pytest.raises(B.TGError) as e:
            ctx.step_blocks(d.sys, blk, -1)
        assert e.value.status == -1
        ctx.graph_begin()
        with pytest.raises(B.TGError) as e:
            ctx.step_blocks(d.sys, blk, 3)
        assert e.value.status == -5
        ctx.counter_add(keep[4])
        g = ctx.graph_end()
        g.launch(s)
        s.synchronize()
        assert int(keep[4].item()) == 1
        del g


@pytest.mark.parametrize("case", ["batch3", "spline"])
def test_driver_other_paths_bitwise(case):
    """Several systems (idle substeps take the separate drift and sums) and
    spline softening (the fused drift and sums with the spline kernel)."""
    say("driver", case)
    if case == "batch3":
        w = ics.batch_c5(S=3, nmin=6000, nmax=20000)
        soft = None
    else:
        w = ics.hernquist_c4(n=16384)
        soft = "spline"
    a, _ = _run(w, 8, 2.0 ** -6, 150, False, softening=soft)
    b, n_idle = _run(w, 8, 2.0 ** -6, 150, True, softening=soft)
    say("  idle substeps %d" % n_idle)
    assert n_idle > 0 and a["k"] == b["k"] == 150
    assert a["n_active"] == b["n_active"] and np.array_equal(a["idx"], b["idx"])
    for key in ("pos", "vel", "acc", "pot", "level", "bpos", "bvel", "bacc"):
        assert np.array_equal(a[key], b[key]), key
