"""The C ABI library loads without a GPU and exports every entry point that
include/tg.h declares (no compute calls here)."""
import ctypes
import os
import re
import shutil

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tg.h")
LIB = os.path.join(ROOT, "paper_1507_01009_amd", "libtg.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libtg():
    if not os.path.exists(LIB):
        if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
            pytest.skip("hipcc not available to build libtg.so")
        from paper_1507_01009_amd import build
        build.build()
    import torch  # noqa: F401  (bind to the HIP runtime torch ships)
    return ctypes.CDLL(LIB)


def test_header_declares_the_path():
    names = declared()
    for n in ("tg_create", "tg_build_tree", "tg_compute_moments", "tg_tree_forces",
              "tg_direct_fp64", "tg_kick", "tg_drift", "tg_levels", "tg_active_set",
              "tg_graph_begin", "tg_graph_end", "tg_graph_launch", "tg_walk_lists",
              "tg_get_tree", "tg_autotune", "tg_sync", "tg_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(libtg):
    missing = [n for n in declared() if not hasattr(libtg, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_1507_01009_amd import binding
    assert sorted(binding.EXPORTED) == declared()


def test_default_config_and_version(libtg):
    from paper_1507_01009_amd import binding as B
    cfg = B.tg_config()
    libtg.tg_default_config(ctypes.byref(cfg))
    assert (cfg.leaf_size, cfg.group_size, cfg.precision, cfg.G) == (8, 64, 0, 1.0)
    libtg.tg_version.restype = ctypes.c_char_p
    assert b"gfx950" in libtg.tg_version()


def test_create_rejects_bad_config_without_gpu(libtg):
    """Argument checks run on the host before any device call."""
    from paper_1507_01009_amd import binding as B
    cfg = B.tg_config()
    libtg.tg_default_config(ctypes.byref(cfg))
    cfg.group_size = 129
    h = ctypes.c_void_p()
    libtg.tg_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert libtg.tg_create(ctypes.byref(cfg), None, ctypes.byref(h)) == -1
    libtg.tg_last_error.restype = ctypes.c_char_p
    assert b"group_size" in libtg.tg_last_error()
