"""ctypes binding of libtg.so (include/tg.h): argument marshalling only.

Every call forwards device pointers from torch tensors (torch supplies HBM
and streams; all arithmetic runs in the library's HIP kernels).  There is no
fallback: if libtg.so is missing or no GPU is visible the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TG_LIB") or os.path.join(_HERE, "libtg.so")   # TG_LIB: a test build

TG_FP64, TG_MIXED = 0, 1
TG_SOFT_PLUMMER, TG_SOFT_SPLINE = 0, 1
ERR_NONFINITE, ERR_MASS, ERR_NODES, ERR_FRONTIER, ERR_LISTS = 1, 2, 4, 8, 16
STATUS = {0: "TG_OK", -1: "TG_EINVAL", -2: "TG_ENOMEM", -3: "TG_EHIP",
          -4: "TG_ECAPACITY", -5: "TG_ESTATE", -6: "TG_EDATA", -7: "TG_EINTERNAL"}


class TGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class tg_config(C.Structure):
    _fields_ = [("max_particles", C.c_int64), ("max_systems", C.c_int32),
                ("leaf_size", C.c_int32), ("group_size", C.c_int32),
                ("precision", C.c_int32), ("max_nodes", C.c_int64),
                ("frontier_cap", C.c_int32), ("waves_per_cu", C.c_int32),
                ("G", C.c_double), ("key_levels", C.c_int32)]


class tg_tree_view(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_nodes", C.c_int64), ("n_groups", C.c_int64),
                ("n_sys", C.c_int32),
                ("skeys", C.c_void_p), ("skeys_lo", C.c_void_p), ("perm", C.c_void_p),
                ("level", C.c_void_p),
                ("nchild", C.c_void_p), ("first", C.c_void_p), ("count", C.c_void_p),
                ("child", C.c_void_p), ("parent", C.c_void_p), ("cube", C.c_void_p),
                ("com", C.c_void_p), ("mom", C.c_void_p), ("groups", C.c_void_p)]


class tg_system(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("vel", C.c_void_p), ("acc", C.c_void_p),
                ("pot", C.c_void_p), ("mass", C.c_void_p), ("n", C.c_int64),
                ("sys_off", C.c_void_p), ("n_sys", C.c_int32),
                ("bh_pos", C.c_void_p), ("bh_vel", C.c_void_p), ("bh_acc", C.c_void_p),
                ("bh_pot", C.c_void_p), ("bh_mass", C.c_void_p), ("bh_eps", C.c_void_p),
                ("n_bh", C.c_int32), ("bh_seg", C.c_void_p), ("eps", C.c_double),
                ("theta", C.c_double), ("frozen", C.c_void_p)]


class tg_blocks(C.Structure):
    _fields_ = [("level", C.c_void_p), ("tau4eps2", C.c_void_p),
                ("active_idx", C.c_void_p), ("n_active", C.c_void_p), ("k", C.c_void_p),
                ("dt_max", C.c_double), ("nlev", C.c_int32), ("tau2eps2v", C.c_void_p),
                ("rebuild_every", C.c_int32)]


class tg_chain(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("mass", C.c_void_p), ("n", C.c_int64),
                ("exclude", C.c_void_p), ("member_pos", C.c_void_p),
                ("member_mass", C.c_void_p), ("nc", C.c_int32),
                ("com", C.c_double * 3), ("m_chain", C.c_double), ("r_crit", C.c_double),
                ("gamma_crit", C.c_double), ("eps_pm", C.c_double),
                ("pert_idx", C.c_void_p), ("pert_cap", C.c_int32), ("n_pert", C.c_void_p)]


class tg_membership_in(C.Structure):
    _fields_ = [("n", C.c_int32), ("x", C.c_void_p), ("v", C.c_void_p), ("m", C.c_void_p),
                ("massive", C.c_void_p), ("designated", C.c_int32), ("r_chain", C.c_double),
                ("r_chain0", C.c_double), ("gamma", C.c_double), ("np", C.c_int32),
                ("px", C.c_void_p)]


class tg_membership_out(C.Structure):
    _fields_ = [("absorb", C.c_void_p), ("n_absorb", C.c_int32), ("escape", C.c_void_p),
                ("n_escape", C.c_int32), ("terminate", C.c_int32), ("designated", C.c_int32)]


class tg_hybrid_config(C.Structure):
    _fields_ = [("r_chain0", C.c_double), ("gamma_crit", C.c_double), ("gamma_esc", C.c_double),
                ("tol", C.c_double), ("ghost_mass", C.c_double), ("pert_cap", C.c_int32)]


class tg_hybrid_state(C.Structure):
    _fields_ = [("active", C.c_int32), ("n_members", C.c_int32), ("n_perturbers", C.c_int32),
                ("com", C.c_double * 3), ("com_vel", C.c_double * 3), ("m_chain", C.c_double),
                ("r_chain", C.c_double), ("energy_error", C.c_double), ("steps", C.c_int64),
                ("starts", C.c_int64), ("absorbed", C.c_int64), ("escaped", C.c_int64),
                ("ended", C.c_int64), ("archain_seconds", C.c_double),
                ("step_seconds", C.c_double)]


class tg_archain(C.Structure):
    _fields_ = [("n", C.c_int32), ("x", C.c_void_p), ("v", C.c_void_p), ("m", C.c_void_p),
                ("t", C.c_double), ("B", C.c_double), ("ds", C.c_double),
                ("chain", C.c_void_p), ("cx", C.c_void_p), ("cv", C.c_void_p),
                ("chain_valid", C.c_int32)]


class tg_archain_perturbers(C.Structure):
    _fields_ = [("np", C.c_int32), ("x", C.c_void_p), ("v", C.c_void_p), ("m", C.c_void_p),
                ("t0", C.c_double)]


_lib = None


def lib():
    """Load libtg.so; raise if it was not built."""
    global _lib
    if _lib is None:
        # torch first: libtg.so then binds to the HIP runtime torch loaded
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError("libtg.so not built (run __graft_entry__.build() "
                              "or python paper_1507_01009_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        P, i64, i32, f64, st = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_int
        sigs = {
            "tg_default_config": (None, [P]),
            "tg_create": (st, [P, P, P]),
            "tg_destroy": (None, [P]),
            "tg_set_stream": (st, [P, P]),
            "tg_set_sizes": (st, [P, i32, i32]),
            "tg_build_tree": (st, [P, P, i64, P, i32]),
            "tg_compute_moments": (st, [P, P]),
            "tg_tree_forces": (st, [P, f64, f64, P, P, P, P]),
            "tg_get_counts": (st, [P, P]),
            "tg_reset_counts": (st, [P]),
            "tg_walk_lists": (st, [P, f64, P, P, P, i64, P, i64, P, P]),
            "tg_direct_fp64": (st, [P, P, P, P, i64, P, P, i64, P, P, i32, i32,
                                    i32, P, P]),
            "tg_direct_fp64_noalloc": (st, [P, P, P, i64, P, P, i64, P, P, i32, i32, i32,
                                            i32, P, P, P]),
            "tg_kick": (st, [P, P, P, i64, P, P, P, f64, P, i32]),
            "tg_drift": (st, [P, P, P, i64, f64]),
            "tg_levels": (st, [P, P, P, i64, P, P, f64, i32, P, P]),
            "tg_levels_v": (st, [P, P, P, P, P, i64, P, P, f64, i32, P, P]),
            "tg_active_set": (st, [P, P, i64, i32, P, i32, P, P]),
            "tg_counter_add": (st, [P, P, i64]),
            "tg_set_external": (st, [P, P, P, P, i32, P, i32]),
            "tg_set_mac": (st, [P, i32, f64, P]),
            "tg_refit_tree": (st, [P, P, P]),
            "tg_perturbers": (st, [P, P]),
            "tg_chain_forces": (st, [P, P, P, P, P, P, P, P]),
            "tg_chains_forces": (st, [P, P, i32, P, P, P, P, P, P]),
            "tg_select_within": (st, [P, P, i64, P, P, f64, P, i32, P]),
            "tg_predict_perturbers": (st, [P, P, P, P, f64, P, P, P]),
            "tg_archain_init": (st, [P, f64]),
            "tg_archain_advance": (st, [P, f64, f64, f64, P, P]),
            "tg_archain_energy": (st, [P, f64, P]),
            "tg_chain_membership": (st, [P, P]),
            "tg_hybrid_create": (st, [P, P, P, P]),
            "tg_hybrid_begin": (st, [P]),
            "tg_hybrid_step": (st, [P, f64]),
            "tg_hybrid_step_block": (st, [P, P]),
            "tg_hybrid_state_get": (st, [P, P, P, P, P]),
            "tg_hybrid_destroy": (None, [P]),
            "tg_set_softening": (st, [P, i32]),
            "tg_forces": (st, [P, P, P, P]),
            "tg_step_kdk": (st, [P, P, f64]),
            "tg_step_dkd": (st, [P, P, f64]),
            "tg_step_block": (st, [P, P, P]),
            "tg_step_blocks": (st, [P, P, P, i64, P]),
            "tg_graph_begin": (st, [P]),
            "tg_graph_end": (st, [P, P]),
            "tg_graph_launch": (st, [P, P]),
            "tg_graph_destroy": (None, [P]),
            "tg_get_tree": (st, [P, P]),
            "tg_autotune": (st, [P, P, P, i64, P, i32, f64, f64, P, P, P, i32,
                                 P, P, P]),
            "tg_set_profiling": (st, [P, i32]),
            "tg_get_profile": (st, [P, P, P]),
            "tg_sync": (st, [P, P]),
            "tg_last_error": (C.c_char_p, []),
            "tg_version": (C.c_char_p, []),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


EXPORTED = ("tg_default_config", "tg_create", "tg_destroy", "tg_set_stream",
            "tg_set_sizes", "tg_build_tree", "tg_compute_moments",
            "tg_tree_forces", "tg_get_counts", "tg_reset_counts", "tg_walk_lists",
            "tg_direct_fp64", "tg_direct_fp64_noalloc", "tg_kick", "tg_drift", "tg_levels", "tg_levels_v",
            "tg_active_set", "tg_counter_add", "tg_set_external", "tg_set_mac", "tg_set_softening",
            "tg_refit_tree",
            "tg_perturbers", "tg_chain_forces", "tg_chains_forces", "tg_select_within",
            "tg_predict_perturbers", "tg_archain_init", "tg_archain_advance",
            "tg_archain_energy", "tg_chain_membership", "tg_hybrid_create", "tg_hybrid_begin",
            "tg_hybrid_step", "tg_hybrid_step_block", "tg_hybrid_state_get", "tg_hybrid_destroy",
            "tg_forces",
            "tg_step_kdk", "tg_step_dkd", "tg_step_block", "tg_step_blocks", "tg_graph_begin",
            "tg_graph_end", "tg_graph_launch", "tg_graph_destroy",
            "tg_get_tree", "tg_autotune", "tg_set_profiling",
            "tg_get_profile", "tg_sync", "tg_last_error",
            "tg_version")


def _check(rc):
    if rc != 0:
        raise TGError(rc, lib().tg_last_error().decode())


def _ptr(t):
    """Device pointer of a torch tensor (None passes NULL)."""
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA/HIP tensors"
    return C.c_void_p(t.data_ptr())


def _i64_host(a):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=np.int64)
    return arr, arr.ctypes.data_as(C.c_void_p)


def direct_fp64_noalloc(src_pos, src_mass, src_eps, tgt_pos, tgt_eps, acc, pot=None,
                        src_seg=None, tgt_seg=None, self_pairs=False, accumulate=False,
                        softening=TG_SOFT_PLUMMER, stream=None):
    """tg_direct_fp64_noalloc on device tensors (no context; the library's
    fixed scratch array; torch's current stream unless one is given)."""
    sa, sp = _i64_host(src_seg)
    ta, tp = _i64_host(tgt_seg)
    nseg = 0 if sa is None else sa.shape[0] - 1
    _check(lib().tg_direct_fp64_noalloc(
        _ptr(src_pos), _ptr(src_mass), _ptr(src_eps), src_mass.shape[0], _ptr(tgt_pos),
        _ptr(tgt_eps), tgt_pos.shape[0], sp, tp, nseg, int(bool(self_pairs)),
        int(bool(accumulate)), int(softening), _ptr(acc), _ptr(pot), _stream_handle(stream)))


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class Graph:
    """A captured sequence of calls; it replays kernels on its context's
    buffers, so it keeps the context alive and refuses to launch once the
    context is closed."""

    def __init__(self, handle, ctx):
        self.h = handle
        self._ctx = ctx

    def launch(self, stream=None):
        if not getattr(self._ctx, "h", None):
            raise TGError(-5, "tg_graph_launch: the graph's context is closed")
        _check(lib().tg_graph_launch(self.h, _stream_handle(stream)))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.tg_graph_destroy(self.h)
            self.h = None


class Context:
    """One libtg context (tg_create ... tg_destroy) bound to a torch stream."""

    def __init__(self, max_particles, max_systems=1, leaf_size=8, group_size=64,
                 precision=TG_FP64, max_nodes=0, frontier_cap=0, waves_per_cu=0,
                 G=1.0, stream=None, key_levels=21):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libtg needs a visible MI355X (no CPU fallback)")
        L = lib()
        cfg = tg_config()
        L.tg_default_config(C.byref(cfg))
        cfg.max_particles = int(max_particles)
        cfg.max_systems = int(max_systems)
        cfg.leaf_size = int(leaf_size)
        cfg.group_size = int(group_size)
        cfg.precision = int(precision)
        cfg.max_nodes = int(max_nodes)
        cfg.frontier_cap = int(frontier_cap)
        cfg.waves_per_cu = int(waves_per_cu)
        cfg.G = float(G)
        cfg.key_levels = int(key_levels)
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = C.c_void_p()
        _check(L.tg_create(C.byref(cfg), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.cfg = cfg

    def close(self):
        # drivers built on this context go first (they use its stream)
        for d in list(getattr(self, "_deps", ())):
            d.close()
        if getattr(self, "h", None):
            lib().tg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- configuration
    def set_stream(self, stream):
        self.stream = stream
        _check(lib().tg_set_stream(self.h, C.c_void_p(stream.cuda_stream)))

    def set_sizes(self, leaf_size, group_size):
        _check(lib().tg_set_sizes(self.h, int(leaf_size), int(group_size)))

    # -- tree build and moments
    def build_tree(self, pos, sys_off=None):
        n = pos.shape[0]
        arr, p = _i64_host(sys_off)
        S = 1 if arr is None else arr.shape[0] - 1
        _check(lib().tg_build_tree(self.h, _ptr(pos), n, p, S))

    def compute_moments(self, mass):
        _check(lib().tg_compute_moments(self.h, _ptr(mass)))

    def tree_forces(self, eps, theta, acc, pot=None, active_idx=None, n_active=None):
        _check(lib().tg_tree_forces(self.h, float(eps), float(theta),
                                    _ptr(active_idx), _ptr(n_active), _ptr(acc),
                                    _ptr(pot)))

    def get_counts(self):
        out = np.zeros(8, np.int64)
        _check(lib().tg_get_counts(self.h, out.ctypes.data_as(C.c_void_p)))
        return {"n_p2p": int(out[0]), "n_p2m": int(out[1]),
                "n_targets": int(out[2]), "n_groups": int(out[3])}

    def get_cumulative_counts(self):
        out = np.zeros(8, np.int64)
        _check(lib().tg_get_counts(self.h, out.ctypes.data_as(C.c_void_p)))
        return {"n_p2p": int(out[4]), "n_p2m": int(out[5]),
                "n_targets": int(out[6]), "n_groups": int(out[7])}

    def reset_counts(self):
        _check(lib().tg_reset_counts(self.h))

    def refit_tree(self, pos, mass):
        """Moments and opening sizes of the last build for moved particles."""
        _check(lib().tg_refit_tree(self.h, _ptr(pos), _ptr(mass)))

    def set_mac(self, relative=False, alpha=0.0, acc_old=None):
        """Opening test of later walks: the opening angle (default), or the
        relative test with tolerance alpha and old accelerations acc_old
        ([N, 3] device, caller order; None = the system's acc in forces)."""
        _check(lib().tg_set_mac(self.h, 1 if relative else 0, float(alpha),
                                _ptr(acc_old)))

    def set_softening(self, kind):
        """Pair softening of later walks, SMBH terms and direct sums:
        "plummer" (default) or "spline" (cubic spline, h = eps)."""
        k = {"plummer": TG_SOFT_PLUMMER, "spline": TG_SOFT_SPLINE}.get(kind, kind)
        _check(lib().tg_set_softening(self.h, int(k)))

    def walk_lists(self, theta, active_idx=None, n_active=None):
        """(info [ng, 4] int64, ids uint32) as numpy; see tg_walk_lists."""
        import torch
        ng = C.c_int64()
        ni = C.c_int64()
        rc = lib().tg_walk_lists(self.h, float(theta), _ptr(active_idx), _ptr(n_active),
                                 None, 0, None, 0, C.byref(ng), C.byref(ni))
        if rc not in (0, -4):
            _check(rc)
        dev = self.stream.device if hasattr(self.stream, "device") else "cuda"
        info = torch.zeros((max(ng.value, 1), 4), dtype=torch.int64, device=dev)
        ids = torch.zeros(max(ni.value, 1), dtype=torch.int32, device=dev)
        _check(lib().tg_walk_lists(self.h, float(theta), _ptr(active_idx), _ptr(n_active),
                                   _ptr(info), info.shape[0], _ptr(ids), ids.shape[0],
                                   C.byref(ng), C.byref(ni)))
        return (info[:ng.value].cpu().numpy(),
                ids[:ni.value].cpu().numpy().view(np.uint32))

    # -- FP64 direct forces
    def direct_fp64(self, src_pos, src_mass, src_eps, tgt_pos, tgt_eps, acc, pot=None,
                    src_seg=None, tgt_seg=None, self_pairs=False, accumulate=False):
        sa, sp = _i64_host(src_seg)
        ta, tp = _i64_host(tgt_seg)
        nseg = 0 if sa is None else sa.shape[0] - 1
        _check(lib().tg_direct_fp64(self.h, _ptr(src_pos), _ptr(src_mass), _ptr(src_eps),
                                    src_mass.shape[0], _ptr(tgt_pos), _ptr(tgt_eps),
                                    tgt_pos.shape[0], sp, tp, nseg, int(bool(self_pairs)),
                                    int(bool(accumulate)), _ptr(acc), _ptr(pot)))

    # -- leapfrog and block steps
    def kick(self, vel, acc, dt, active_idx=None, n_active=None, level=None, k=None,
             skip_at_k0=False):
        _check(lib().tg_kick(self.h, _ptr(vel), _ptr(acc), vel.shape[0], _ptr(active_idx),
                             _ptr(n_active), _ptr(level), float(dt), _ptr(k),
                             int(bool(skip_at_k0))))

    def drift(self, pos, vel, dt):
        _check(lib().tg_drift(self.h, _ptr(pos), _ptr(vel), pos.shape[0], float(dt)))

    def levels(self, acc, tau4eps2, level, dt_max, nlev, k=None, active_idx=None,
               n_active=None, vel=None, tau2eps2v=None):
        """Block levels; with vel and tau2eps2v also the velocity criterion."""
        _check(lib().tg_levels_v(self.h, _ptr(acc), _ptr(vel), _ptr(tau4eps2),
                                 _ptr(tau2eps2v), acc.shape[0], _ptr(active_idx),
                                 _ptr(n_active), float(dt_max), int(nlev), _ptr(k),
                                 _ptr(level)))

    def active_set(self, level, nlev, k, idx, n_out, k_add=0):
        _check(lib().tg_active_set(self.h, _ptr(level), level.shape[0], int(nlev), _ptr(k),
                                   int(k_add), _ptr(idx), _ptr(n_out)))

    def counter_add(self, k, inc=1):
        _check(lib().tg_counter_add(self.h, _ptr(k), int(inc)))

    def set_external(self, pos, mass, eps, seg=None):
        """SMBHs as external point masses added to every later tree_forces."""
        arr, p = _i64_host(seg)
        nsys = 1 if arr is None else arr.shape[0] - 1
        n = 0 if mass is None else mass.shape[0]
        _check(lib().tg_set_external(self.h, _ptr(pos), _ptr(mass), _ptr(eps), n, p, nsys))

    # -- chain coupling
    def make_chain(self, pos, mass, member_pos, member_mass, com, m_chain, r_crit,
                   gamma_crit, pert_idx, n_pert, eps_pm=0.0, exclude=None):
        """A tg_chain over device tensors (kept alive by the caller); com and
        m_chain are host values."""
        ch = tg_chain()
        ch.pos, ch.mass, ch.n = _ptr(pos), _ptr(mass), pos.shape[0]
        ch.exclude = _ptr(exclude)
        ch.member_pos, ch.member_mass = _ptr(member_pos), _ptr(member_mass)
        ch.nc = member_mass.shape[0]
        for k in range(3):
            ch.com[k] = float(com[k])
        ch.m_chain, ch.r_crit, ch.gamma_crit = float(m_chain), float(r_crit), float(gamma_crit)
        ch.eps_pm = float(eps_pm)
        ch.pert_idx, ch.pert_cap, ch.n_pert = _ptr(pert_idx), pert_idx.shape[0], _ptr(n_pert)
        return ch

    def perturbers(self, chain):
        _check(lib().tg_perturbers(self.h, C.byref(chain)))

    def chain_forces(self, chain, acc, com_acc, member_acc, pot=None, active_idx=None,
                     n_active=None):
        _check(lib().tg_chain_forces(self.h, C.byref(chain), _ptr(active_idx), _ptr(n_active),
                                     _ptr(acc), _ptr(pot), _ptr(com_acc), _ptr(member_acc)))

    def chains_forces(self, chains, acc, com_acc, member_acc, pot=None, active_idx=None,
                      n_active=None):
        """Several chains (a list of tg_chain sharing the star arrays)."""
        arr = (tg_chain * len(chains))(*chains)
        _check(lib().tg_chains_forces(self.h, arr, len(chains), _ptr(active_idx),
                                      _ptr(n_active), _ptr(acc), _ptr(pot), _ptr(com_acc),
                                      _ptr(member_acc)))

    def predict_perturbers(self, chain, vel, com_vel, dt, out_pos, out_vel, out_mass=None):
        v3 = (C.c_double * 3)(*[float(x) for x in com_vel])
        _check(lib().tg_predict_perturbers(self.h, C.byref(chain), _ptr(vel), v3, float(dt),
                                           _ptr(out_pos), _ptr(out_vel), _ptr(out_mass)))

    def select_within(self, pos, center, r, idx, n_out, exclude=None):
        c3 = (C.c_double * 3)(*[float(x) for x in center])
        _check(lib().tg_select_within(self.h, _ptr(pos), pos.shape[0], _ptr(exclude), c3,
                                      float(r), _ptr(idx), idx.shape[0], _ptr(n_out)))

    # -- whole steps
    def make_system(self, pos, vel, acc, mass, eps, theta, pot=None, sys_off=None,
                    bh_pos=None, bh_vel=None, bh_acc=None, bh_mass=None, bh_eps=None,
                    bh_pot=None, bh_seg=None, frozen=None):
        """A tg_system describing device tensors (kept alive by the caller);
        frozen: uint8 [n] device mask of stars held still in the steps."""
        y = tg_system()
        y.pos, y.vel, y.acc, y.pot = (_ptr(pos), _ptr(vel), _ptr(acc), _ptr(pot))
        y.mass, y.n = _ptr(mass), pos.shape[0]
        so, sp = _i64_host(sys_off)
        y.sys_off, y.n_sys = sp, 1 if so is None else so.shape[0] - 1
        nb = 0 if bh_mass is None else bh_mass.shape[0]
        y.bh_pos, y.bh_vel, y.bh_acc = _ptr(bh_pos), _ptr(bh_vel), _ptr(bh_acc)
        y.bh_pot, y.bh_mass, y.bh_eps = _ptr(bh_pot), _ptr(bh_mass), _ptr(bh_eps)
        y.n_bh = nb
        bs, bp = _i64_host(bh_seg)
        y.bh_seg = bp
        y.eps, y.theta = float(eps), float(theta)
        y.frozen = _ptr(frozen)
        y._keep = (so, bs)   # host arrays must outlive the calls
        return y

    def forces(self, system, active_idx=None, n_active=None):
        _check(lib().tg_forces(self.h, C.byref(system), _ptr(active_idx), _ptr(n_active)))

    def step_kdk(self, system, dt):
        _check(lib().tg_step_kdk(self.h, C.byref(system), float(dt)))

    def step_dkd(self, system, dt):
        _check(lib().tg_step_dkd(self.h, C.byref(system), float(dt)))

    def make_blocks(self, level, tau4eps2, active_idx, n_active, k, dt_max, nlev,
                    tau2eps2v=None, rebuild_every=0):
        b = tg_blocks()
        b.level, b.tau4eps2 = _ptr(level), _ptr(tau4eps2)
        b.active_idx, b.n_active, b.k = _ptr(active_idx), _ptr(n_active), _ptr(k)
        b.dt_max, b.nlev = float(dt_max), int(nlev)
        b.tau2eps2v = _ptr(tau2eps2v)
        b.rebuild_every = int(rebuild_every)
        return b

    def step_block(self, system, blocks):
        _check(lib().tg_step_block(self.h, C.byref(system), C.byref(blocks)))

    def step_blocks(self, system, blocks, n_sub):
        """n_sub substeps; returns how many ran without the tree's launches."""
        n_idle = C.c_int64(0)
        _check(lib().tg_step_blocks(self.h, C.byref(system), C.byref(blocks), int(n_sub),
                                    C.byref(n_idle)))
        return n_idle.value

    # -- HIP graphs
    def graph_begin(self):
        _check(lib().tg_graph_begin(self.h))

    def graph_end(self):
        g = C.c_void_p()
        _check(lib().tg_graph_end(self.h, C.byref(g)))
        return Graph(g, self)

    # -- inspection
    def get_tree(self):
        v = tg_tree_view()
        _check(lib().tg_get_tree(self.h, C.byref(v)))
        return v

    def tree_arrays(self):
        """Copy the current tree to numpy (for parity checks)."""
        import torch
        v = self.get_tree()
        n, nn, ng, S = v.n, v.n_nodes, v.n_groups, v.n_sys

        torch.cuda.synchronize()

        def grab(ptr, count, dtype):
            out = np.zeros(count, dtype)
            if count:
                _memcpy_d2h(out.ctypes.data, ptr, out.nbytes)
            return out

        return {
            "skeys": grab(v.skeys, n, np.uint64), "perm": grab(v.perm, n, np.uint32),
            "skeys_lo": grab(v.skeys_lo, n, np.uint64) if v.skeys_lo else None,
            "level": grab(v.level, nn, np.uint8), "nchild": grab(v.nchild, nn, np.uint8),
            "first": grab(v.first, nn, np.uint32), "count": grab(v.count, nn, np.uint32),
            "child": grab(v.child, nn, np.uint32), "parent": grab(v.parent, nn, np.uint32),
            "cube": grab(v.cube, 4 * S, np.float64).reshape(S, 4),
            "com": grab(v.com, 4 * nn, np.float64).reshape(nn, 4),
            "mom": grab(v.mom, 8 * nn, np.float64).reshape(nn, 8),
            "groups": grab(v.groups, 4 * ng, np.uint32).reshape(ng, 4),
        }

    def autotune(self, pos, mass, eps, theta, sys_off=None, leaf_list=None,
                 group_list=None, waves_list=None, repeats=3):
        def lst(x):
            if x is None:
                return None, None
            a = np.array(list(x) + [0], np.int32)
            return a, a.ctypes.data_as(C.c_void_p)
        arr, p = _i64_host(sys_off)
        S = 1 if arr is None else arr.shape[0] - 1
        la, lp = lst(leaf_list)
        ga, gp = lst(group_list)
        wa, wp = lst(waves_list)
        best = np.zeros(3, np.int32)
        ms = C.c_double()
        nl = len(leaf_list) if leaf_list is not None else 4
        ng = len(group_list) if group_list is not None else 4
        nw = len(waves_list) if waves_list is not None else 3
        times = np.full(nl * ng * nw, np.nan)
        _check(lib().tg_autotune(self.h, _ptr(pos), _ptr(mass), pos.shape[0], p, S,
                                 float(eps), float(theta), lp, gp, wp, int(repeats),
                                 best.ctypes.data_as(C.c_void_p), C.byref(ms),
                                 times.ctypes.data_as(C.c_void_p)))
        return {"leaf_size": int(best[0]), "group_size": int(best[1]),
                "waves_per_cu": int(best[2]), "ms": ms.value, "times": times}

    def set_profiling(self, on=True):
        _check(lib().tg_set_profiling(self.h, int(bool(on))))

    def get_profile(self):
        """(summed walk-kernel ms, number of walks) since profiling was set."""
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().tg_get_profile(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def sync(self):
        bits = C.c_uint32()
        rc = lib().tg_sync(self.h, C.byref(bits))
        if rc != 0:
            raise TGError(rc, lib().tg_last_error().decode() + " (bits 0x%x)" % bits.value)
        return bits.value


_hip = None


def _memcpy_d2h(dst, src, nbytes):
    """Blocking device-to-host copy through the HIP runtime torch loaded."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so.7")
        _hip.hipMemcpy.restype = C.c_int
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    rc = _hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(src), C.c_size_t(nbytes), 2)
    if rc != 0:
        raise RuntimeError("hipMemcpy failed: %d" % rc)


def chain_membership(x, v, m, massive, designated, r_chain, r_chain0, gamma, px):
    """Host membership update after a chain step (tg_chain_membership);
    numpy in, dict out: absorb (perturber rows), escape (member indices),
    terminate, designated."""
    import numpy as np
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    v = np.ascontiguousarray(v, np.float64).reshape(-1, 3)
    m = np.ascontiguousarray(m, np.float64)
    mas = np.ascontiguousarray(massive, np.uint8)
    px = np.ascontiguousarray(px, np.float64).reshape(-1, 3)
    a = np.zeros(max(px.shape[0], 1), np.int32)
    e = np.zeros(max(x.shape[0], 1), np.int32)
    p = lambda arr: arr.ctypes.data_as(C.c_void_p)
    i = tg_membership_in(x.shape[0], p(x), p(v), p(m), p(mas), int(designated), float(r_chain),
                         float(r_chain0), float(gamma), px.shape[0], p(px) if px.size else None)
    o = tg_membership_out(p(a), 0, p(e), 0, 0, 0)
    _check(lib().tg_chain_membership(C.byref(i), C.byref(o)))
    return {"absorb": a[:o.n_absorb].copy(), "escape": e[:o.n_escape].copy(),
            "terminate": bool(o.terminate), "designated": int(o.designated)}


class Hybrid:
    """The hybrid step driver (tg_hybrid_*) over a context and a system with
    one SMBH; keep the system's tensors alive while it lives."""

    def __init__(self, ctx, system, r_chain0, gamma_crit=1e-4, gamma_esc=1.5, tol=1e-12,
                 ghost_mass=1e-10, pert_cap=8192):
        cfg = tg_hybrid_config(float(r_chain0), float(gamma_crit), float(gamma_esc), float(tol),
                               float(ghost_mass), int(pert_cap))
        self.h = C.c_void_p()
        self._sys = system
        self._ctx = ctx            # the context outlives the driver
        _check(lib().tg_hybrid_create(ctx.h, C.byref(system), C.byref(cfg), C.byref(self.h)))
        if not hasattr(ctx, "_deps"):
            ctx._deps = weakref.WeakSet()
        ctx._deps.add(self)

    def begin(self):
        _check(lib().tg_hybrid_begin(self.h))

    def step(self, dt):
        _check(lib().tg_hybrid_step(self.h, float(dt)))

    def step_block(self, blocks):
        _check(lib().tg_hybrid_step_block(self.h, C.byref(blocks)))

    def state(self):
        import numpy as np
        s = tg_hybrid_state()
        _check(lib().tg_hybrid_state_get(self.h, C.byref(s), None, None, None))
        n = s.n_members
        ids = np.zeros(max(n, 1), np.int32)
        x = np.zeros((max(n, 1), 3))
        v = np.zeros((max(n, 1), 3))
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        _check(lib().tg_hybrid_state_get(self.h, C.byref(s), p(ids), p(x), p(v)))
        return {"active": bool(s.active), "members": ids[:n].copy(), "x": x[:n].copy(),
                "v": v[:n].copy(), "n_perturbers": s.n_perturbers, "com": list(s.com),
                "com_vel": list(s.com_vel), "m_chain": s.m_chain, "r_chain": s.r_chain,
                "energy_error": s.energy_error, "steps": s.steps, "starts": s.starts,
                "absorbed": s.absorbed, "escaped": s.escaped, "ended": s.ended,
                "archain_seconds": s.archain_seconds, "step_seconds": s.step_seconds}

    def close(self):
        if getattr(self, "h", None):
            lib().tg_hybrid_destroy(self.h)
            self.h = None

    def __del__(self):
        if _lib is not None:
            self.close()


class ARChain:
    """Host AR-chain (tg_archain_*): members in the centre-of-mass frame,
    numpy float64 arrays owned by this object."""

    def __init__(self, x, v, m, t=0.0, G=1.0):
        self.x = np.ascontiguousarray(x, np.float64).reshape(-1, 3).copy()
        self.v = np.ascontiguousarray(v, np.float64).reshape(-1, 3).copy()
        self.m = np.ascontiguousarray(m, np.float64).copy()
        self.G = float(G)
        n = self.m.shape[0]
        # the chain state kept between calls (order and chain vectors)
        self.chain = np.zeros(max(n, 1), np.int32)
        self.cx = np.zeros((max(n - 1, 1), 3))
        self.cv = np.zeros((max(n - 1, 1), 3))
        self.s = tg_archain()
        self.s.n = n
        self.s.x = self.x.ctypes.data_as(C.c_void_p)
        self.s.v = self.v.ctypes.data_as(C.c_void_p)
        self.s.m = self.m.ctypes.data_as(C.c_void_p)
        self.s.t, self.s.B, self.s.ds = float(t), 0.0, 0.0
        self.s.chain = self.chain.ctypes.data_as(C.c_void_p)
        self.s.cx = self.cx.ctypes.data_as(C.c_void_p)
        self.s.cv = self.cv.ctypes.data_as(C.c_void_p)
        self.s.chain_valid = 0
        _check(lib().tg_archain_init(C.byref(self.s), self.G))

    def reset_from_xv(self):
        """Take x, v (centre-of-mass frame) as the state again (after they
        were changed by hand); the chain is rebuilt from them."""
        self.s.chain_valid = 0

    @property
    def t(self):
        return self.s.t

    def advance(self, dt, tol=1e-12, px=None, pv=None, pm=None, t0=None):
        p = None
        keep = None
        if pm is not None and len(pm):
            keep = [np.ascontiguousarray(a, np.float64) for a in (px, pv, pm)]
            p = tg_archain_perturbers()
            p.np = keep[2].shape[0]
            p.x, p.v, p.m = [a.ctypes.data_as(C.c_void_p) for a in keep]
            p.t0 = self.s.t if t0 is None else float(t0)
        steps = C.c_int64(0)
        _check(lib().tg_archain_advance(C.byref(self.s), self.G, float(dt), float(tol),
                                        C.byref(p) if p is not None else None, C.byref(steps)))
        return steps.value

    def energy_error(self):
        e = C.c_double(0.0)
        _check(lib().tg_archain_energy(C.byref(self.s), self.G, C.byref(e)))
        return e.value
