"""Shared helpers for the GPU parity tests: run the HIP path through the
C ABI (via the binding) and the CPU oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np

import oracle


def torch_dev():
    import torch
    return torch


def to_dev(a, dtype=None):
    torch = torch_dev()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_run(pos, mass, eps, theta, leaf_size=8, group_size=64, active=None,
            sys_off=None, precision=0, lists=False, ctx=None, pot=True,
            waves_per_cu=0, frontier_cap=0, max_nodes=0, alpha=None, acc_old=None,
            softening=None, key_levels=21):
    """Build + moments + forces on the GPU; returns a dict of numpy arrays.
    With alpha the walk uses the relative test against acc_old ([N, 3]);
    softening "spline" switches the pair softening for this run."""
    torch = torch_dev()
    from paper_1507_01009_amd import binding as B
    n = pos.shape[0]
    S = 1 if sys_off is None else len(sys_off) - 1
    own = ctx is None
    if own:
        ctx = B.Context(max(n, 1), max_systems=S, leaf_size=leaf_size,
                        group_size=group_size, precision=precision,
                        waves_per_cu=waves_per_cu, frontier_cap=frontier_cap,
                        max_nodes=max_nodes, key_levels=key_levels)
    dpos = to_dev(pos.reshape(-1, 3).astype(np.float64))
    dm = to_dev(mass.astype(np.float64))
    acc = torch.full((max(n, 1), 3), float("nan"), dtype=torch.float64, device="cuda")
    dpot = torch.full((max(n, 1),), float("nan"), dtype=torch.float64, device="cuda") if pot else None
    if active is not None:
        didx = to_dev(np.asarray(active, np.int32))
        dna = to_dev(np.array([len(active)], np.int32))
    else:
        didx = dna = None
    dold = None
    if alpha is not None:
        dold = to_dev(np.asarray(acc_old, np.float64).reshape(-1, 3))
        ctx.set_mac(True, alpha, dold)
    if softening is not None:
        ctx.set_softening(softening)
    ctx.build_tree(dpos, sys_off)
    ctx.compute_moments(dm)
    ctx.tree_forces(eps, theta, acc, dpot, didx, dna)
    ctx.sync()
    out = {"acc": acc.cpu().numpy()[:n], "pot": dpot.cpu().numpy()[:n] if pot else None,
           "counts": ctx.get_counts(), "tree": ctx.tree_arrays(), "ctx": ctx}
    if lists:
        out["lists"] = ctx.walk_lists(theta, didx, dna)
    if alpha is not None:
        ctx.set_mac(False)
    if softening is not None:
        ctx.set_softening("plummer")
    return out


def rel_err(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


def oracle_lists(ev, theta):
    """Oracle sorted lists for every evaluated group, keyed by group index
    (relative test when the evaluation used it)."""
    L = oracle.walk_lists(ev.tree, ev.mom, ev.groups, ev.box, ev.sel, theta,
                          rel=ev.rel, arel=ev.arel, side=ev.side)
    return {int(g): l for g, l in zip(ev.sel, L)}


def gpu_lists_by_group(info, ids):
    out = {}
    for g, off, nm, npp in info:
        m = np.sort(ids[off:off + nm])
        p = np.sort(ids[off + nm:off + nm + npp])
        out[int(g)] = (m, p)
    return out


def mac_margin(tree, mom, box, node, theta, side=None):
    """Relative distance of one opening decision from its threshold."""
    lev = int(tree.level[node])
    s = tree.cube[tree.sys[node], 3] * 2.0 ** -lev if side is None else side[node]
    c = mom[node, 1:4]
    lo, hi = box[:3], box[3:]
    m = np.maximum(np.maximum(lo - c, c - hi), 0.0)
    d2 = float(np.sum(m * m))
    return abs(s * s - theta * theta * d2) / (s * s)


def rel_margin(ev, k, node):
    """Relative distance of one relative-test decision from its threshold
    P^2 = A d^8 (the separation rule uses only exact cell geometry and the
    box, so only this part can differ between the two sides)."""
    box = ev.box[k]
    c = ev.mom[node, 1:4]
    m = np.maximum(np.maximum(box[:3] - c, c - box[3:]), 0.0)
    d2 = float(np.sum(m * m))
    P = ev.rel[node, 3]
    rhs = ev.arel[k] * d2 ** 4
    return abs(P * P - rhs) / max(P * P, 1e-300)
