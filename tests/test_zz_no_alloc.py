"""The allocation-free direct forces (tg_direct_fp64_noalloc, through the C
ABI) against tg_direct_fp64 on the same inputs: two calls in a row, the
second with a smaller input (segments, accumulation, spline softening),
then self pairs.  The kernels and the split of the sums are the same, so
the results must be equal bit for bit (well inside the FP64 bar of 1e-12).
Sizes beyond the scratch limit are refused on the host."""
import sys

import numpy as np
import pytest

from paper_1507_01009_amd import ics
from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _both(ctx, B, args, acc0=None, pot0=None, **kw):
    import torch
    (sp, sm, se, tp, te) = args
    nt = tp.shape[0]
    outs = []
    for which in ("ctx", "noalloc"):
        acc = (torch.zeros((nt, 3), dtype=torch.float64, device="cuda") if acc0 is None
               else to_dev(acc0))
        pot = (torch.zeros(nt, dtype=torch.float64, device="cuda") if pot0 is None
               else to_dev(pot0))
        if which == "ctx":
            ctx.set_softening(kw.get("softening", "plummer"))
            ctx.direct_fp64(sp, sm, se, tp, te, acc, pot, src_seg=kw.get("src_seg"),
                            tgt_seg=kw.get("tgt_seg"), self_pairs=kw.get("self_pairs", False),
                            accumulate=kw.get("accumulate", False))
            ctx.sync()
        else:
            soft = B.TG_SOFT_SPLINE if kw.get("softening") == "spline" else B.TG_SOFT_PLUMMER
            B.direct_fp64_noalloc(sp, sm, se, tp, te, acc, pot, src_seg=kw.get("src_seg"),
                                  tgt_seg=kw.get("tgt_seg"),
                                  self_pairs=kw.get("self_pairs", False),
                                  accumulate=kw.get("accumulate", False), softening=soft)
            torch.cuda.synchronize()
        outs.append((acc.cpu().numpy(), pot.cpu().numpy()))
    return outs


def test_noalloc_direct_equals_context_direct_twice_then_smaller():
    import torch
    from paper_1507_01009_amd import binding as B
    w = ics.cusp_c3(n=200000)
    ctx = B.Context(w.n)
    # call 1: every star on the two SMBHs (few-target path, 49 blocks each)
    say("noalloc call 1: 200000 sources -> 2 targets")
    a1 = (to_dev(w.pos), to_dev(w.mass), to_dev(np.full(w.n, w.eps)), to_dev(w.bh_pos),
          to_dev(w.bh_eps))
    (ra, rp), (na, np_) = _both(ctx, B, a1)
    assert np.array_equal(ra, na) and np.array_equal(rp, np_)
    assert np.all(np.isfinite(na)) and np.any(na != 0.0)
    # call 2, smaller: 3 segments of sources and targets, accumulating onto
    # given values, spline softening (chunked many-target path)
    say("noalloc call 2: 5000 sources / 300 targets in 3 segments, accumulate, spline")
    rng = np.random.default_rng(4)
    sp = rng.normal(size=(5000, 3))
    tp = rng.normal(size=(300, 3))
    sseg, tseg = np.array([0, 1200, 1201, 5000]), np.array([0, 100, 100, 300])
    a2 = (to_dev(sp), to_dev(rng.uniform(0.5, 1.5, 5000) / 5000), to_dev(rng.uniform(0.01, 0.1, 5000)),
          to_dev(tp), to_dev(rng.uniform(0.01, 0.1, 300)))
    acc0, pot0 = rng.normal(size=(300, 3)), rng.normal(size=300)
    (ra, rp), (na, np_) = _both(ctx, B, a2, acc0, pot0, src_seg=sseg, tgt_seg=tseg,
                                accumulate=True, softening="spline")
    assert np.array_equal(ra, na) and np.array_equal(rp, np_)
    assert not np.array_equal(na, acc0)
    # an empty target segment keeps its accumulated values
    assert np.array_equal(na[100:100], acc0[100:100])
    # call 3: self pairs on a small set
    say("noalloc call 3: 700 self pairs")
    x = to_dev(w.pos[:700])
    a3 = (x, to_dev(w.mass[:700]), to_dev(np.full(700, w.eps)), x, to_dev(np.full(700, w.eps)))
    (ra, rp), (na, np_) = _both(ctx, B, a3, self_pairs=True)
    assert np.array_equal(ra, na) and np.array_equal(rp, np_)
    ctx.close()
    del torch


def test_noalloc_refuses_beyond_its_limits_on_the_host():
    import torch
    from paper_1507_01009_amd import binding as B
    say("noalloc limits")
    z = torch.zeros((70, 3), dtype=torch.float64, device="cuda")
    e = torch.full((70,), 0.01, dtype=torch.float64, device="cuda")
    m = torch.full((70,), 1.0, dtype=torch.float64, device="cuda")
    acc = torch.zeros((70, 3), dtype=torch.float64, device="cuda")
    seg = np.arange(71)                         # 70 segments > TG_NOALLOC_MAX_SEG
    with pytest.raises(B.TGError) as err:
        B.direct_fp64_noalloc(z, m, e, z, e, acc, src_seg=seg, tgt_seg=seg)
    assert err.value.status == -4 and "TG_NOALLOC_MAX_SEG" in str(err.value)
    with pytest.raises(B.TGError) as err:
        B.direct_fp64_noalloc(z, m, e, z, e, acc, softening=7)
    assert err.value.status == -1
    torch.cuda.synchronize()
    assert torch.all(acc == 0.0)
