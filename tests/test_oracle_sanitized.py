"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

bh_oracle.c is built with -fsanitize=address,undefined (recovery off) and
driven through its entry points on small inputs that reach its edges: empty
and one-particle systems in a batch, coincident particles (an over-full
leaf at the deepest level), 42-level keys, both opening tests, the spline
softening, refit sides, interaction lists, direct sums and the kick, drift
and level routines.  Any out-of-bounds access, use after free or undefined
operation aborts the subprocess, and the test fails with its report.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import numpy as np
import oracle
from paper_1507_01009_amd import ics
oracle.set_threads(2)
rng = np.random.default_rng(3)
p, _, m = ics.plummer(600, 21)
dup = np.repeat(np.array([[0.1, -0.2, 0.3]]), 40, axis=0)
pos = np.concatenate([p, dup, rng.normal(size=(1, 3)), np.zeros((0, 3)), rng.normal(size=(37, 3))])
n = pos.shape[0]
mass = np.full(n, 1.0 / n)
off = np.array([0, 640, 641, 641, n], np.int64)
for lv in (21, 42):
    t = oracle.build_tree(pos, off, 4, lv)
    sp, sm = oracle.sorted_arrays(t, pos, mass)
    mom = oracle.moments(t, sp, sm)
    g = oracle.groups(t, 16)
    ev = oracle.tree_forces(pos, mass, 1e-3, 0.5, 4, 16, sys_off=off, levels=lv)
    assert np.isfinite(ev.acc).all()
act = np.arange(0, n, 3)
ev = oracle.tree_forces(pos, mass, 1e-3, 0.0, 4, 16, active=act, sys_off=off)
acc_old = np.where(np.isfinite(ev.acc), ev.acc, 1.0)
acc_old[~np.isfinite(acc_old).all(axis=1)] = 1.0
ev2 = oracle.tree_forces(pos, mass, 1e-3, 0.5, 4, 16, sys_off=off, alpha=1e-3,
                         acc_old=np.ones((n, 3)))
ev3 = oracle.tree_forces(pos, mass, 1e-3, 0.5, 4, 16, sys_off=off, softening="spline")
t = oracle.build_tree(pos, off, 4)
moved = pos + 1e-3 * rng.normal(size=pos.shape)
ev4 = oracle.tree_forces(moved, mass, 1e-3, 0.5, 4, 16, sys_off=off, tree=t, refit=True)
L = oracle.walk_lists(ev.tree, ev.mom, ev.groups, ev.box, ev.sel, 0.5)
a, ph = oracle.direct(pos, mass, 1e-3, np.arange(0, n, 7), sys_off=off)
vel = rng.normal(size=(n, 3))
oracle.kick(vel, ev3.acc, 1e-3)
oracle.drift(moved, vel, 1e-3)
lev = np.zeros(n, np.uint8)
oracle.levels(ev3.acc, np.full(n, 1e-6), lev, 2.0 ** -6, 5, 0)
idx = oracle.active_at(lev, 5, 3)
print("sanitized oracle ran", n, len(L), len(idx), flush=True)
'''


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isfile(asan):
        pytest.skip("no ASan runtime for gcc")
    lib = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ)
    env.update({
        "TG_ORACLE_LIB": lib,
        "LD_PRELOAD": asan,
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "PYTHONPATH": ROOT + os.pathsep + env.get("PYTHONPATH", ""),
    })
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "sanitized oracle ran" in r.stdout, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
