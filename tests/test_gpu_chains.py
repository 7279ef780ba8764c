"""GPU parity of several chains at once (tg_chains_forces) against the
oracle's several-chain coupling: two Dehnen cusps 1.0 apart, each with an
SMBH whose chain holds it and the 20 stars nearest to it (ghosts in the star
arrays).  Perturber lists bit-exact per chain; star terms, chain particles
(with their mutual pull) and member forces to the FP64 bar, 1e-12.
"""
import sys

import numpy as np
import pytest

from oracle import chain as ochain
from paper_1507_01009_amd import ics
from gpu_helpers import rel_err, to_dev

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _workload(n_each=65536, nc=21):
    parts, masses, chains = [], [], []
    ghosts = []
    for k, (c, seed) in enumerate(((np.array([0.5, 0.0, 0.0]), 31),
                                   (np.array([-0.5, 0.1, 0.0]), 32))):
        p, _, m = ics.dehnen(n_each, 1.5, ics.SEED_BASE + seed)
        p = p * 0.2 + c
        near = np.argsort(np.linalg.norm(p - c, axis=1))[:nc - 1]
        ghosts.append(near + k * n_each)
        mpos = np.concatenate([c[None, :], p[near]])
        mmass = np.concatenate([[0.01], m[near]])
        M, S = 0.0, np.zeros(3)
        for i in range(nc):
            M += mmass[i]
            S += mmass[i] * mpos[i]
        chains.append({"com": S / M, "m_chain": M, "mpos": mpos, "mmass": mmass,
                       "r_crit": 0.005, "gamma_crit": 1e-4})
        parts.append(p)
        masses.append(m)
    pos = np.concatenate(parts)
    mass = np.concatenate(masses)
    excl = np.zeros(pos.shape[0], np.uint8)
    excl[np.concatenate(ghosts)] = 1
    return pos, mass, chains, excl


def _run(ctx, pos, mass, chains, excl, active=None, cap=4096):
    import torch
    d = {"pos": to_dev(pos), "mass": to_dev(mass), "excl": to_dev(excl), "keep": []}
    chs = []
    for c in chains:
        mp, mm = to_dev(c["mpos"]), to_dev(c["mmass"])
        idx = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        npt = torch.zeros(1, dtype=torch.int32, device="cuda")
        d["keep"] += [mp, mm, idx, npt]
        chs.append(ctx.make_chain(d["pos"], d["mass"], mp, mm, c["com"], c["m_chain"],
                                  c["r_crit"], c["gamma_crit"], idx, npt, exclude=d["excl"]))
    n = pos.shape[0]
    acc = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    pot = torch.zeros(n, dtype=torch.float64, device="cuda")
    K = len(chains)
    com = torch.zeros((K, 3), dtype=torch.float64, device="cuda")
    mem = torch.zeros((sum(c["mmass"].size for c in chains), 3), dtype=torch.float64,
                      device="cuda")
    didx = dna = None
    if active is not None:
        didx = to_dev(active.astype(np.int32))
        dna = to_dev(np.array([active.size], np.int32))
    ctx.chains_forces(chs, acc, com, mem, pot, didx, dna)
    ctx.sync()
    perts = [d["keep"][4 * k + 2][:int(d["keep"][4 * k + 3].item())].cpu().numpy()
             for k in range(K)]
    return (acc.cpu().numpy(), pot.cpu().numpy(), com.cpu().numpy(), mem.cpu().numpy(),
            perts, chs, d)


@pytest.mark.parametrize("every", [1, 3])
def test_two_chains_match_oracle(every):
    say("two chains", every)
    from paper_1507_01009_amd import binding as B
    pos, mass, chains, excl = _workload()
    n = pos.shape[0]
    active = None if every == 1 else np.arange(0, n, every)
    ctx = B.Context(n)
    acc, pot, com, mem, perts, _, _ = _run(ctx, pos, mass, chains, excl, active)
    tg = np.arange(n) if active is None else active
    ra, rp, rc, rm, rperts = ochain.chains_coupling(pos, mass, tg, chains, excl.astype(bool))
    for k in range(2):
        say("  chain %d: %d perturbers" % (k, rperts[k].size))
        assert rperts[k].size > 5 and np.array_equal(perts[k], rperts[k])
    live = ~excl.astype(bool)[tg]
    assert rel_err(acc[tg][live], ra[live]).max() <= FP64_TOL
    assert np.max(np.abs(pot[tg][live] - rp[live]) / np.abs(rp[live])) <= FP64_TOL
    assert np.all(acc[tg][~live] == 0.0)
    assert rel_err(com, rc).max() <= FP64_TOL
    assert rel_err(mem, rm).max() <= FP64_TOL
    if active is not None:
        rest = np.setdiff1d(np.arange(n), active)
        assert np.all(acc[rest] == 0.0)


def test_one_chain_through_the_several_chains_call_is_tg_chain_forces():
    say("one of several")
    import torch
    from paper_1507_01009_amd import binding as B
    pos, mass, chains, excl = _workload(n_each=16384)
    ctx = B.Context(pos.shape[0])
    acc, pot, com, mem, perts, chs, d = _run(ctx, pos, mass, chains[:1], excl)
    acc1 = torch.zeros((pos.shape[0], 3), dtype=torch.float64, device="cuda")
    com1 = torch.zeros(3, dtype=torch.float64, device="cuda")
    mem1 = torch.zeros((chains[0]["mmass"].size, 3), dtype=torch.float64, device="cuda")
    ctx.chain_forces(chs[0], acc1, com1, mem1)
    ctx.sync()
    assert np.array_equal(acc, acc1.cpu().numpy())
    assert np.array_equal(com[0], com1.cpu().numpy()) and np.array_equal(mem, mem1.cpu().numpy())


def test_errors():
    say("several chains errors")
    import torch
    from paper_1507_01009_amd import binding as B
    pos, mass, chains, excl = _workload(n_each=4096)
    ctx = B.Context(pos.shape[0])
    _, _, _, _, _, chs, d = _run(ctx, pos, mass, chains, excl)
    acc = torch.zeros((pos.shape[0], 3), dtype=torch.float64, device="cuda")
    com = torch.zeros((17, 3), dtype=torch.float64, device="cuda")
    mem = torch.zeros((17 * 21, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(B.TGError):                     # same perturber list twice
        ctx.chains_forces([chs[0], chs[0]], acc, com, mem)
    other_mask = to_dev(np.zeros(pos.shape[0], np.uint8))
    bad = B.tg_chain.from_buffer_copy(chs[1])
    bad.exclude = B._ptr(other_mask)
    with pytest.raises(B.TGError):                     # a different mask
        ctx.chains_forces([chs[0], bad], acc, com, mem)
    with pytest.raises(B.TGError):                     # too many chains
        ctx.chains_forces([chs[0]] * 17, acc, com, mem)
    ctx.sync()
