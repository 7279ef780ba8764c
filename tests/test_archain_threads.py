"""The AR-chain's extrapolation columns computed on host threads give the
same result, bit for bit, as one at a time (no GPU needed): a 70-member
chain with 60 perturbers advanced in two processes, TG_ARCHAIN_THREADS = 1
and 6.  The vector clones of the pair sums (baseline, AVX2 + FMA, AVX-512)
agree to 1e-10 relative on the same chain.  Two host threads advancing two
chains at once share the column threads and get their results alone."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import json, sys
import numpy as np
sys.path.insert(0, %r)
from paper_1507_01009_amd import binding as B
rng = np.random.default_rng(4)
n, npert = 70, 60
x = rng.normal(size=(n, 3)) * 0.01
m = rng.uniform(1e-5, 1e-4, n); m[0] = 0.01
v = np.zeros((n, 3))
for i in range(1, n):
    r = np.linalg.norm(x[i] - x[0]); t = np.cross(x[i] - x[0], rng.normal(size=3))
    v[i] = t / np.linalg.norm(t) * np.sqrt(0.01 / r)
x -= (m[:, None] * x).sum(0) / m.sum(); v -= (m[:, None] * v).sum(0) / m.sum()
px = rng.normal(size=(npert, 3)) * 0.05; pv = rng.normal(size=(npert, 3)) * 0.1
pm = rng.uniform(1e-5, 1e-4, npert)
ch = B.ARChain(x, v, m)
ch.advance(2e-4, tol=1e-12, px=px, pv=pv, pm=pm, t0=0.0)
print(json.dumps({"x": ch.x.tolist(), "v": ch.v.tolist(), "t": ch.t}))
""" % ROOT


def _run(threads):
    env = dict(os.environ, TG_ARCHAIN_THREADS=str(threads))
    out = subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True,
                         timeout=300, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_threaded_columns_are_bit_identical():
    a, b = _run(1), _run(6)
    assert a["t"] == b["t"]
    assert np.array_equal(np.array(a["x"]), np.array(b["x"]))
    assert np.array_equal(np.array(a["v"]), np.array(b["v"]))


def _run_isa(isa):
    env = dict(os.environ, TG_ARCHAIN_THREADS="1", TG_ARCHAIN_ISA=isa)
    out = subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True,
                         timeout=300, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_vector_clones_agree():
    """The pair sums compiled for AVX-512, AVX2 + FMA and the baseline
    round differently but agree to the integration's tolerance; a wrong
    clone (a dropped lane, a bad mask) would not."""
    ref = _run_isa("base")
    for isa in ("avx2", "auto"):
        b = _run_isa(isa)
        assert b["t"] == ref["t"]
        sx = np.abs(np.array(ref["x"])).max()
        sv = np.abs(np.array(ref["v"])).max()
        assert np.max(np.abs(np.array(b["x"]) - np.array(ref["x"]))) <= 1e-10 * sx
        assert np.max(np.abs(np.array(b["v"]) - np.array(ref["v"]))) <= 1e-10 * sv


POOL_SCRIPT = r"""
import json, sys, threading
import numpy as np
sys.path.insert(0, %r)
from paper_1507_01009_amd import binding as B

def chain(seed):
    rng = np.random.default_rng(seed)
    n, npert = 70, 60
    x = rng.normal(size=(n, 3)) * 0.01
    m = rng.uniform(1e-5, 1e-4, n); m[0] = 0.01
    v = np.zeros((n, 3))
    for i in range(1, n):
        r = np.linalg.norm(x[i] - x[0]); t = np.cross(x[i] - x[0], rng.normal(size=3))
        v[i] = t / np.linalg.norm(t) * np.sqrt(0.01 / r)
    x -= (m[:, None] * x).sum(0) / m.sum(); v -= (m[:, None] * v).sum(0) / m.sum()
    px = rng.normal(size=(npert, 3)) * 0.05; pv = rng.normal(size=(npert, 3)) * 0.1
    pm = rng.uniform(1e-5, 1e-4, npert)
    return B.ARChain(x, v, m), (px, pv, pm)

def run(seed, out):
    ch, (px, pv, pm) = chain(seed)
    for _ in range(3):
        ch.advance(5e-5, tol=1e-12, px=px, pv=pv, pm=pm, t0=ch.t)
    out[seed] = ch.x.copy()

alone = {}
for s in (11, 12):
    run(s, alone)
both = {}
th = [threading.Thread(target=run, args=(s, both)) for s in (11, 12)]
for t in th: t.start()
for t in th: t.join()
print(json.dumps({"same": all(np.array_equal(alone[s], both[s]) for s in (11, 12))}))
""" % ROOT


def test_concurrent_chains_share_the_pool():
    """Two host threads advancing different chains at once share the
    process's column threads (one batch at a time) and get the results of
    advancing each chain alone, bit for bit."""
    env = dict(os.environ, TG_ARCHAIN_THREADS="6")
    out = subprocess.run([sys.executable, "-c", POOL_SCRIPT], env=env, capture_output=True,
                         text=True, timeout=300, check=True)
    assert json.loads(out.stdout.strip().splitlines()[-1])["same"]
