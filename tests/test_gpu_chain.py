"""GPU parity of the chain coupling (through the C ABI) against the oracle.

Selections (perturbers by Eq. 2, radius selections) are index lists and
must be bit-exact; the coupling forces (stars, members, the chain particle
with the Eq. 3 correction) must agree to the FP64 bar, max relative error
<= 1e-12.  Workload: the Dehnen gamma = 1.5 cusp with its SMBH binary; the
chain holds both SMBHs and the stars nearest to the binary's centre, which
stay in the star arrays as excluded ghosts.
"""
import sys

import numpy as np
import pytest

from oracle import chain as ochain
from paper_1507_01009_amd import ics
from gpu_helpers import rel_err, to_dev

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
# r_crit per size: the inner cusp is sparse at small N
RC = {65536: 0.05, 262144: 0.03, 1048576: 0.01}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _setup(n, n_ghost=30):
    w = ics.cusp_c3(n=n)
    r = np.linalg.norm(w.pos, axis=1)
    ghosts = np.sort(np.argsort(r)[:n_ghost])
    mpos = np.concatenate([w.bh_pos, w.pos[ghosts]])
    mmass = np.concatenate([w.bh_mass, w.mass[ghosts]])
    M = 0.0
    S = np.zeros(3)
    for i in range(mmass.size):
        M += mmass[i]
        S += mmass[i] * mpos[i]
    excl = np.zeros(n, np.uint8)
    excl[ghosts] = 1
    return w, mpos, mmass, S / M, M, excl


def _dev_chain(ctx, w, mpos, mmass, R, M, excl, cap, r_crit=None, gam=1e-4, eps_pm=0.0,
               use_excl=True):
    import torch
    d = {"pos": to_dev(w.pos), "mass": to_dev(w.mass), "mpos": to_dev(mpos),
         "mmass": to_dev(mmass), "excl": to_dev(excl) if use_excl else None,
         "idx": torch.full((cap,), -1, dtype=torch.int32, device="cuda"),
         "np": torch.zeros(1, dtype=torch.int32, device="cuda")}
    r_crit = RC[w.n] if r_crit is None else r_crit
    d["ch"] = ctx.make_chain(d["pos"], d["mass"], d["mpos"], d["mmass"], R, M, r_crit, gam,
                             d["idx"], d["np"], eps_pm=eps_pm, exclude=d["excl"])
    return d


@pytest.mark.parametrize("n,use_excl,gam", [(65536, True, 1e-4), (1048576, True, 1e-4),
                                            (1048576, False, 1e-5), (262144, True, 1e-3)])
def test_perturbers_bit_exact(n, use_excl, gam):
    say("perturbers", n, use_excl, gam)
    from paper_1507_01009_amd import binding as B
    w, mpos, mmass, R, M, excl = _setup(n)
    ctx = B.Context(n)
    d = _dev_chain(ctx, w, mpos, mmass, R, M, excl, 8192, gam=gam, use_excl=use_excl)
    ctx.perturbers(d["ch"])
    ctx.sync()
    want = ochain.perturbers(w.pos, w.mass, R, M, RC[n], gam,
                             exclude=excl if use_excl else None)
    got_n = int(d["np"].cpu().numpy()[0])
    say("  perturbers %d" % want.size)
    assert want.size > 50 and got_n == want.size
    assert np.array_equal(d["idx"].cpu().numpy()[:got_n], want)


@pytest.mark.parametrize("n", [65536, 1048576])
def test_select_within_bit_exact(n):
    say("within", n)
    import torch
    from paper_1507_01009_amd import binding as B
    w, mpos, mmass, R, M, excl = _setup(n)
    ctx = B.Context(n)
    dpos, dex = to_dev(w.pos), to_dev(excl)
    idx = torch.full((20000,), -1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    for center, r, ex in ((w.bh_pos[0], RC[n], None), (R, 2 * RC[n], excl), (R, 0.0, None)):
        ctx.select_within(dpos, center, r, idx, cnt, exclude=None if ex is None else dex)
        ctx.sync()
        want = ochain.within(w.pos, center, r, exclude=ex)
        k = int(cnt.cpu().numpy()[0])
        say("  within %g: %d" % (r, want.size))
        assert k == want.size and (r == 0.0 or want.size > 0)
        assert np.array_equal(idx.cpu().numpy()[:k], want)


@pytest.mark.parametrize("n,eps_pm,every", [(262144, 0.0, 1), (262144, 1e-4, 3),
                                            (1048576, 0.0, 1)])
def test_chain_forces_match_oracle(n, eps_pm, every):
    say("chain forces", n, eps_pm, every)
    import torch
    from paper_1507_01009_amd import binding as B
    w, mpos, mmass, R, M, excl = _setup(n)
    ctx = B.Context(n)
    d = _dev_chain(ctx, w, mpos, mmass, R, M, excl, 8192, eps_pm=eps_pm)
    f64 = dict(dtype=torch.float64, device="cuda")
    acc = torch.zeros((n, 3), **f64)
    pot = torch.zeros(n, **f64)
    com_acc = torch.zeros(3, **f64)
    macc = torch.zeros((mmass.size, 3), **f64)
    act = None if every == 1 else np.arange(0, n, every, dtype=np.int32)
    didx = None if act is None else to_dev(act)
    dna = None if act is None else to_dev(np.array([act.size], np.int32))
    ctx.chain_forces(d["ch"], acc, com_acc, macc, pot=pot, active_idx=didx, n_active=dna)
    ctx.sync()
    pert = ochain.perturbers(w.pos, w.mass, R, M, RC[n], 1e-4, exclude=excl)
    say("  perturbers %d" % pert.size)
    tg = np.arange(n) if act is None else act
    a, p, a_com, am = ochain.coupling(w.pos, w.mass, tg, R, M, mpos, mmass, pert,
                                      eps_pm=eps_pm, exclude=excl)
    ga, gp = acc.cpu().numpy(), pot.cpu().numpy()
    live = tg[excl[tg] == 0]
    rows = np.nonzero(excl[tg] == 0)[0]
    e = rel_err(ga[live], a[rows])
    ep = np.abs(gp[live] - p[rows]) / np.abs(p[rows])
    say("  stars max %.3g pot %.3g" % (e.max(), ep.max()))
    assert e.max() <= FP64_TOL and ep.max() <= FP64_TOL
    untouched = np.setdiff1d(np.arange(n), live)
    assert np.all(ga[untouched] == 0) and np.all(gp[untouched] == 0)
    em = rel_err(macc.cpu().numpy(), am)
    ec = np.linalg.norm(com_acc.cpu().numpy() - a_com) / np.linalg.norm(a_com)
    say("  members max %.3g com %.3g" % (em.max(), ec))
    assert em.max() <= FP64_TOL and ec <= FP64_TOL


def test_capacity_and_errors():
    say("chain capacity")
    import torch
    from paper_1507_01009_amd import binding as B
    w, mpos, mmass, R, M, excl = _setup(65536)
    ctx = B.Context(65536)
    d = _dev_chain(ctx, w, mpos, mmass, R, M, excl, 10)
    ctx.perturbers(d["ch"])
    with pytest.raises(B.TGError) as e:
        ctx.sync()
    assert e.value.status == -4
    want = ochain.perturbers(w.pos, w.mass, R, M, RC[65536], 1e-4, exclude=excl)
    assert int(d["np"].cpu().numpy()[0]) == want.size
    assert np.array_equal(d["idx"].cpu().numpy(), want[:10])
    ctx.sync()
    bad = _dev_chain(ctx, w, mpos, mmass, R, M, excl, 10, gam=0.0)
    with pytest.raises(B.TGError) as e:
        ctx.perturbers(bad["ch"])
    assert e.value.status == -1
    bad = _dev_chain(ctx, w, mpos, mmass, R, -1.0, excl, 10)
    with pytest.raises(B.TGError) as e:
        ctx.perturbers(bad["ch"])
    assert e.value.status == -1
    f64 = dict(dtype=torch.float64, device="cuda")
    with pytest.raises(B.TGError) as e:
        ctx.chain_forces(d["ch"], torch.zeros((65536, 3), **f64), None,
                         torch.zeros((mmass.size, 3), **f64))
    assert e.value.status == -1
    # no stars: empty list, the chain particle feels only nothing
    empty = ctx.make_chain(d["pos"][:0], d["mass"][:0], d["mpos"], d["mmass"], R, M,
                           RC[65536], 1e-4, d["idx"], d["np"])
    com_acc = torch.full((3,), 7.0, **f64)
    macc = torch.full((mmass.size, 3), 7.0, **f64)
    ctx.chain_forces(empty, None, com_acc, macc)
    ctx.sync()
    assert int(d["np"].cpu().numpy()[0]) == 0
    assert np.all(com_acc.cpu().numpy() == 0) and np.all(macc.cpu().numpy() == 0)


@pytest.mark.parametrize("n,dt", [(262144, 0.0), (262144, 3e-4), (1048576, -2e-5)])
def test_prediction_bit_exact(n, dt):
    say("predict", n, dt)
    import torch
    from paper_1507_01009_amd import binding as B
    w, mpos, mmass, R, M, excl = _setup(n)
    ctx = B.Context(n)
    d = _dev_chain(ctx, w, mpos, mmass, R, M, excl, 8192)
    ctx.perturbers(d["ch"])
    V = np.array([0.03, -0.11, 0.007])
    f64 = dict(dtype=torch.float64, device="cuda")
    op = torch.full((8192, 3), 7.0, **f64)
    ov = torch.full((8192, 3), 7.0, **f64)
    om = torch.full((8192,), 7.0, **f64)
    ctx.predict_perturbers(d["ch"], to_dev(w.vel), V, dt, op, ov, om)
    ctx.sync()
    pert = ochain.perturbers(w.pos, w.mass, R, M, RC[n], 1e-4, exclude=excl)
    xr, vr, m = ochain.predict(w.pos, w.vel, w.mass, pert, R, V, dt)
    k = pert.size
    assert np.array_equal(op.cpu().numpy()[:k], xr)
    assert np.array_equal(ov.cpu().numpy()[:k], vr)
    assert np.array_equal(om.cpu().numpy()[:k], m)
    assert np.all(op.cpu().numpy()[k:] == 7.0)


def test_largest_chain_and_zero_capacity():
    say("chain 256 members")
    import torch
    from paper_1507_01009_amd import binding as B
    w, mpos, mmass, R, M, excl = _setup(65536, n_ghost=254)
    assert mmass.size == 256
    ctx = B.Context(65536)
    d = _dev_chain(ctx, w, mpos, mmass, R, M, excl, 8192)
    f64 = dict(dtype=torch.float64, device="cuda")
    acc = torch.zeros((65536, 3), **f64)
    com_acc = torch.zeros(3, **f64)
    macc = torch.zeros((256, 3), **f64)
    ctx.chain_forces(d["ch"], acc, com_acc, macc)
    ctx.sync()
    pert = ochain.perturbers(w.pos, w.mass, R, M, RC[65536], 1e-4, exclude=excl)
    a, _, a_com, am = ochain.coupling(w.pos, w.mass, np.arange(65536), R, M, mpos, mmass, pert,
                                      exclude=excl)
    live = np.nonzero(excl == 0)[0]
    assert rel_err(acc.cpu().numpy()[live], a[live]).max() <= FP64_TOL
    assert rel_err(macc.cpu().numpy(), am).max() <= FP64_TOL
    assert np.linalg.norm(com_acc.cpu().numpy() - a_com) <= FP64_TOL * np.linalg.norm(a_com)
    # no room for a single perturber: the count is still exact, the error is reported
    z = _dev_chain(ctx, w, mpos, mmass, R, M, excl, 1)
    z["ch"].pert_cap = 0
    ctx.perturbers(z["ch"])
    with pytest.raises(B.TGError) as e:
        ctx.sync()
    assert e.value.status == -4
    assert int(z["np"].cpu().numpy()[0]) == pert.size
    assert int(z["idx"].cpu().numpy()[0]) == -1
    bad = _dev_chain(ctx, w, np.zeros((257, 3)), np.full(257, 1e-6), R, M, excl, 10)
    with pytest.raises(B.TGError) as e:
        ctx.perturbers(bad["ch"])
    assert e.value.status == -1


def test_chain_step_round_trip():
    """Perturbers gathered on the GPU drive the host AR-chain exactly as the
    oracle's gather does; the chain's energy bookkeeping closes."""
    say("chain round trip")
    import torch
    from paper_1507_01009_amd import binding as B
    n = 262144
    w, mpos, mmass, R, M, excl = _setup(n)
    ghosts = np.nonzero(excl)[0]
    mvel = np.concatenate([w.bh_vel.reshape(-1, 3), w.vel[ghosts]])
    V = (mmass[:, None] * mvel).sum(0) / M
    ctx = B.Context(n)
    d = _dev_chain(ctx, w, mpos, mmass, R, M, excl, 8192)
    ctx.perturbers(d["ch"])
    f64 = dict(dtype=torch.float64, device="cuda")
    op, ov, om = (torch.zeros((8192, 3), **f64), torch.zeros((8192, 3), **f64),
                  torch.zeros(8192, **f64))
    ctx.predict_perturbers(d["ch"], to_dev(w.vel), V, 0.0, op, ov, om)
    ctx.sync()
    k = int(d["np"].cpu().numpy()[0])
    pert = ochain.perturbers(w.pos, w.mass, R, M, RC[n], 1e-4, exclude=excl)
    xr, vr, m = ochain.predict(w.pos, w.vel, w.mass, pert, R, V, 0.0)
    a = B.ARChain(mpos - R, mvel - V, mmass)
    a.advance(2e-4, px=op.cpu().numpy()[:k], pv=ov.cpu().numpy()[:k], pm=om.cpu().numpy()[:k])
    b = B.ARChain(mpos - R, mvel - V, mmass)
    b.advance(2e-4, px=xr, pv=vr, pm=m)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)
    assert abs(a.energy_error()) < 1e-10


def test_prediction_rejects_foreign_indices():
    """A perturber list that was not selected from these stars: indices
    outside [0, n) give NaN rows (the kernel checks every index)."""
    say("predict foreign list")
    import torch
    from paper_1507_01009_amd import binding as B
    w, mpos, mmass, R, M, excl = _setup(65536)
    ctx = B.Context(65536)
    d = _dev_chain(ctx, w, mpos, mmass, R, M, excl, 4)
    d["idx"].copy_(torch.tensor([3, -1, 65536, 70000], dtype=torch.int32))
    d["np"].fill_(4)
    f64 = dict(dtype=torch.float64, device="cuda")
    op, ov, om = (torch.zeros((4, 3), **f64), torch.zeros((4, 3), **f64), torch.zeros(4, **f64))
    ctx.predict_perturbers(d["ch"], to_dev(w.vel), [0.0, 0.0, 0.0], 0.0, op, ov, om)
    ctx.sync()
    p = op.cpu().numpy()
    assert np.array_equal(p[0], w.pos[3] - R) and np.all(np.isnan(p[1:]))
    assert np.all(np.isnan(om.cpu().numpy()[1:]))
