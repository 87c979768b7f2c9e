"""Comparison of two grain states (oracle vs GPU) by global voxel.

A state is a dict with ``alive`` (G,), ``lo`` (G, 3), ``ext`` (G, 3) and ``phi``
(list of (ez, ey, ex) arrays or None).  Boxes may differ between the two sides;
values are compared on the union of both boxes through the periodic sampling
rule (a voxel outside a grain's box reads the fill value ``-W``).
"""
import numpy as np


def _sample(state, k, gx, gy, gz, n, fill):
    lo, ext = state["lo"][k], state["ext"][k]
    lx = np.mod(gx - lo[0], n[0])
    ly = np.mod(gy - lo[1], n[1])
    lz = np.mod(gz - lo[2], n[2])
    ok = (lx < ext[0]) & (ly < ext[1]) & (lz < ext[2])
    out = np.full(gx.shape, fill, dtype=np.float64)
    phi = state["phi"][k]
    out[ok] = phi[lz[ok], ly[ok], lx[ok]]
    return out


def _box_coords(state, k, n):
    lo, ext = state["lo"][k], state["ext"][k]
    z, y, x = np.meshgrid(np.arange(ext[2]), np.arange(ext[1]), np.arange(ext[0]), indexing="ij")
    return ((x + lo[0]) % n[0]).ravel(), ((y + lo[1]) % n[1]).ravel(), ((z + lo[2]) % n[2]).ravel()


def compare_states(a, b, n, W, band_only=False, grains=None):
    """Largest |phi_a - phi_b| over both boxes of every grain, and liveness mismatches.

    band_only: only voxels where either side has |phi| < W count.
    Returns dict(max_abs, alive_mismatch, worst_grain, box_mismatch).
    """
    n = tuple(int(v) for v in n)
    G = len(a["alive"])
    worst, wk = 0.0, -1
    alive_mis = int(np.sum(np.asarray(a["alive"], bool) != np.asarray(b["alive"], bool)))
    box_mis = 0
    ks = range(G) if grains is None else grains
    for k in ks:
        if not (a["alive"][k] and b["alive"][k]):
            continue
        if not (np.array_equal(a["lo"][k], b["lo"][k]) and np.array_equal(a["ext"][k], b["ext"][k])):
            box_mis += 1
        for s in (a, b):
            gx, gy, gz = _box_coords(s, k, n)
            va = _sample(a, k, gx, gy, gz, n, -W)
            vb = _sample(b, k, gx, gy, gz, n, -W)
            d = np.abs(va - vb)
            if band_only:
                d = d[(np.abs(va) < W) | (np.abs(vb) < W)]
            m = float(d.max()) if d.size else 0.0
            if m > worst:
                worst, wk = m, k
    return dict(max_abs=worst, alive_mismatch=alive_mis, worst_grain=wk, box_mismatch=box_mis)


def top2_gap(state, n, W):
    """Per voxel: gap between the largest and second largest grain value (global
    grid); +inf where fewer than two grains cover the voxel (no tie possible)."""
    n = tuple(int(v) for v in n)
    shape = (n[2], n[1], n[0])
    m1 = np.full(shape, -np.inf)
    m2 = np.full(shape, -np.inf)
    for k in range(len(state["alive"])):
        if not state["alive"][k]:
            continue
        gx, gy, gz = _box_coords(state, k, n)
        v = state["phi"][k].ravel()
        cur1 = m1[gz, gy, gx]
        cur2 = m2[gz, gy, gx]
        new1 = np.maximum(cur1, v)
        new2 = np.where(v > cur1, cur1, np.maximum(cur2, v))
        m1[gz, gy, gx] = new1
        m2[gz, gy, gx] = new2
    gap = np.full(shape, np.inf)
    two = np.isfinite(m2)
    gap[two] = m1[two] - m2[two]
    return gap


def interface_voxels(state):
    """Per grain: the voxels whose volume term clamp(phi + 1/2, 0, 1) lies
    strictly between 0 and 1 (|phi| < 1/2), the only ones where a change of
    phi changes the grain volume."""
    out = np.zeros(len(state["alive"]), np.int64)
    for k in range(len(state["alive"])):
        if state["alive"][k]:
            out[k] = int((np.abs(state["phi"][k]) < 0.5).sum())
    return out


def volume_bound(vol, iface, tol_phi):
    """Allowed |V_a - V_b| per grain between two states whose band values
    differ by at most tol_phi: each interface voxel moves its volume term by at
    most tol_phi, so the error is at most tol_phi * iface; grains above 0.5%
    of their volume per that bound keep the 0.5% relative bar."""
    return np.maximum(5e-3 * vol, tol_phi * iface)
