"""Comparison helpers for the GPU parity tests (per particle id, per cell)."""

import numpy as np

CHANNELS = ["rho", "J", "F", "eng"]


def min_image(d, n):
    return d - n * np.round(d / n)


def by_id(arr, ids):
    """Reorder the last axis of arr so that entry i belongs to particle id i."""
    out = np.empty_like(arr)
    out[..., ids.astype(np.int64)] = arr
    return out


def state_errors(gx, gu, gid, ox, ou, n, ndim, sigma=0.05):
    """Max position error (cells, minimum image) and max velocity error
    relative to max(|u|, sigma), per particle id."""
    gx = by_id(gx, gid)
    gu = by_id(gu, gid)
    ex = 0.0
    for a in range(ndim):
        ex = max(ex, float(np.abs(min_image(gx[a] - ox[a], n[a])).max(initial=0.0)))
    scale = np.maximum(np.sqrt((ou * ou).sum(axis=0)), sigma)
    eu = float((np.sqrt(((gu - ou) ** 2).sum(axis=0)) / scale).max(initial=0.0))
    return ex, eu


def state_error_stats(gx, gu, gid, ox, ou, n, ndim, sigma=0.05):
    gx = by_id(gx, gid)
    gu = by_id(gu, gid)
    dx = np.stack([min_image(gx[a] - ox[a], n[a]) for a in range(ndim)])
    du = gu - ou
    out = {}
    for a in range(ndim):
        out[f"x{a}"] = (float(np.abs(dx[a]).max()), float(np.sqrt(np.mean(dx[a] ** 2))))
    for a in range(3):
        rel = du[a] / np.maximum(np.abs(ou[a]), sigma)
        out[f"u{a}"] = (float(np.abs(rel).max()), float(np.sqrt(np.mean(rel ** 2))))
    return out


def _pairs(gm, om, am):
    for ch in CHANNELS:
        if ch not in gm or om.get(ch) is None:
            continue
        g, o, a = gm[ch], om[ch], am[ch]
        if isinstance(g, list):
            for k in range(3):
                yield f"{ch}{k}", g[k], o[k], a[k]
        else:
            yield ch, g, o, a


def moment_errors(gm, om, am):
    """Per channel: max |gpu - oracle| / A_c over cells (A_c = sum |mu| W),
    RMS of the same ratio, and max |diff| / max |oracle|."""
    out = {}
    for name, g, o, a in _pairs(gm, om, am):
        d = np.abs(g.reshape(o.shape) - o)
        ratio = np.where(a > 0, d / np.where(a > 0, a, 1.0), d)
        out[name] = (float(ratio.max()), float(np.sqrt(np.mean(ratio ** 2))),
                     float(d.max() / max(np.abs(o).max(), 1e-300)))
    return out


# Frozen bounds of the float32 form against the float64 oracle, (max, rms) per
# quantity: positions in cells, velocity components relative to
# max(|u|, sigma), deposits relative to A_c of the cell.  Each is twice the
# value measured on MI355X over every particle and cell of the 32^3
# turbulent box after 20 steps (run-based kernel, 8^3 tiles), rounded up:
#   x 1.84e-7 / 3.09e-8, u 2.12e-6 / 2.00e-7, rho 7.2e-8 / 1.8e-8,
#   J 2.34e-7 / 4.98e-8, F 4.36e-7 / 5.51e-8, eng 3.08e-7 / 4.99e-8.
# Twice, not more: the particle states are deterministic and the deposits
# differ between runs only by the float64 summation order (1e-16 of A_c), so
# a regression of the float32 arithmetic shows up as a breach; the factor two
# leaves room for other seeds and kernels of the same arithmetic.
FP32_BOUNDS = {
    "x": (3.7e-7, 6.2e-8),
    "u": (4.3e-6, 4.0e-7),
    "rho": (1.5e-7, 3.6e-8),
    "J": (4.7e-7, 1.0e-7),
    "F": (8.8e-7, 1.2e-7),
    "eng": (6.2e-7, 1.0e-7),
}


def check_fp32_table(states, moments):
    """Assert the error table (state_error_stats, moment_errors) is within
    FP32_BOUNDS; returns the breaches as a list (empty when all hold)."""
    bad = []
    for k, v in list(states.items()) + list(moments.items()):
        mx, rms = v[0], v[1]
        bmax, brms = FP32_BOUNDS[k.rstrip("012")]
        if not (mx <= bmax and rms <= brms):
            bad.append((k, mx, rms, bmax, brms))
    return bad
