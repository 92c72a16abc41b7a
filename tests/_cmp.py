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
