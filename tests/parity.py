"""Comparison of a GPU particle state / nodal statistics with the oracle's.

Tolerances (FP64): per-particle |dq| <= 1e-10 * scale_q with scale x, y: domain length,
U: max |<U>| (at least 1), omega: mean omega, psi: 1, w: max w; element ids equal except
for particles within 1e-12 of an edge of either candidate element (those and the other
particles of their elements are excluded); nodal statistics |ds| <= 1e-11 * max |s_ref|
per statistic, NaN matching NaN.
"""
import numpy as np

REL_PARTICLE = 1e-10
REL_STAT = 1e-11
EDGE_BAND = 1e-12


def edge_distances(frame, e, x, y):
    v = frame[e].reshape(-1, 3, 2)
    d = np.full(len(e), np.inf)
    for k in range(3):
        a, b = v[:, (k + 1) % 3], v[:, (k + 2) % 3]
        ex, ey = (b - a).T
        L = np.hypot(ex, ey)
        d = np.minimum(d, np.abs((x - a[:, 0]) * ey - (y - a[:, 1]) * ex) / L)
    return d


def compare_states(gpu, ref, frame, length, excluded_elems=None):
    """Returns (report dict, set of excluded elements)."""
    assert np.array_equal(gpu["pid"], ref["pid"]), "particle ids differ"
    excl = set() if excluded_elems is None else set(excluded_elems)
    diff_e = np.nonzero(gpu["elem"] != ref["elem"])[0]
    for i in diff_e:
        de = min(edge_distances(frame, np.array([ref["elem"][i]]), ref["x"][i:i + 1], ref["y"][i:i + 1])[0],
                 edge_distances(frame, np.array([gpu["elem"][i]]), gpu["x"][i:i + 1], gpu["y"][i:i + 1])[0])
        assert de < EDGE_BAND, f"element mismatch for pid {ref['pid'][i]} at distance {de}"
        excl.add(int(ref["elem"][i]))
        excl.add(int(gpu["elem"][i]))
    keep = ~np.isin(ref["elem"], list(excl)) & ~np.isin(gpu["elem"], list(excl))
    scale = dict(x=length, y=length, u=max(1.0, float(np.abs(ref["u"]).max())),
                 om=float(np.abs(ref["om"]).mean()), psi=1.0, w=float(np.abs(ref["w"]).max()))
    rep = {"n": int(len(ref["pid"])), "excluded_elems": len(excl), "compared": int(keep.sum())}
    for k, s in scale.items():
        d = np.abs(gpu[k][keep] - ref[k][keep])
        if k == "x":
            d = np.minimum(d, np.abs(d - length))     # same point across the periodic seam
        rep[k] = float(d.max() / s) if d.size else 0.0
        assert rep[k] <= REL_PARTICLE, f"{k}: relative difference {rep[k]:.3e}"
    return rep, excl


def compare_stats(gpu, ref, skip_nodes=None):
    g, r = gpu.copy(), ref.copy()
    if skip_nodes is not None and len(skip_nodes):
        g[list(skip_nodes)] = np.nan
        r[list(skip_nodes)] = np.nan
    nan_g, nan_r = np.isnan(g), np.isnan(r)
    skip = np.zeros(len(g), bool) if skip_nodes is None else np.isin(np.arange(len(g)), list(skip_nodes))
    assert np.array_equal(nan_g[~skip], nan_r[~skip]), "NaN pattern of the statistics differs"
    out = {}
    for q in range(r.shape[1]):
        ok = ~nan_r[:, q]
        if not ok.any():
            continue
        m = np.abs(r[ok, q]).max()
        d = np.abs(g[ok, q] - r[ok, q]).max()
        out[q] = float(d / m) if m > 0 else float(d)
        assert out[q] <= REL_STAT or d <= 1e-300, f"statistic {q}: relative difference {out[q]:.3e}"
    return out
