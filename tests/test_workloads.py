"""Synthetic workload generators: geometry and boundary bookkeeping of the meshes, and
the analytic fields they carry (inputs only; no method arithmetic here)."""
import math

import numpy as np
import pytest

from paper_1006_0532_amd import workloads as W


def _areas(mesh):
    P = mesh.xy[mesh.tri].copy()
    if mesh.period_x > 0:
        L = mesh.period_x
        w = (P[:, :, 0].max(1) - P[:, :, 0].min(1)) > 0.5 * L
        P[w, :, 0] = np.where(P[w, :, 0] < 0.5 * L, P[w, :, 0] + L, P[w, :, 0])
    return 0.5 * ((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
                  - (P[:, 2, 0] - P[:, 0, 0]) * (P[:, 1, 1] - P[:, 0, 1])), P


@pytest.mark.parametrize("nxh,nyc,nyv", [(4, 4, 4), (12, 10, 14)])
def test_cavity_mesh_geometry(nxh, nyc, nyv):
    m = W.cavity_mesh(nxh, nyc, nyv)
    a, P = _areas(m)
    assert m.n_elems == 2 * (3 * nxh * nyc + nxh * nyv)
    assert (a > 0).all()
    assert abs(a.sum() - 4.0) < 1e-12            # 3H x H channel + H x H cavity
    # boundary edges: free-slip top (3 nxh edges), no-slip street level (2 nxh), cavity
    # sides (2 nyv) and floor (nxh)
    k = m.edge_kind.ravel()
    assert (k == W.EDGE_SLIP).sum() == 3 * nxh
    assert (k == W.EDGE_WALL).sum() == 2 * nxh + 2 * nyv + nxh
    # every edge belongs to one element (boundary) or two (interior, incl. the seam)
    e = np.concatenate([np.sort(m.tri[:, [(j + 1) % 3, (j + 2) % 3]], 1) for j in range(3)])
    _, cnt = np.unique(e[:, 0].astype(np.int64) * m.n_nodes + e[:, 1], return_counts=True)
    assert set(cnt.tolist()) <= {1, 2}
    assert (cnt == 1).sum() == 6 * nxh + 2 * nyv
    # no node outside the domain, none inside the two solid blocks beside the cavity
    x, y = m.xy[:, 0], m.xy[:, 1]
    assert (x >= 0).all() and (x < 3.0).all() and (y >= 0).all() and (y <= 2.0).all()
    assert not ((y < 1.0 - 1e-14) & ((x < 1.0 - 1e-14) | (x > 2.0 + 1e-14))).any()


def test_cavity_mesh_is_locally_delaunay():
    """The diagonal chosen in each quad passes the empty-circumcircle test against the
    opposite vertex of its partner triangle."""
    m = W.cavity_mesh(10, 8, 8, jitter=0.2)
    a, P = _areas(m)
    tri = m.tri
    for t in range(0, m.n_elems, 2):
        p, q = P[t], P[t + 1]
        shared = set(tri[t].tolist()) & set(tri[t + 1].tolist())
        assert len(shared) == 2
        opp = [j for j in range(3) if tri[t + 1][j] not in shared][0]
        d = q[opp]
        # bring d into p's frame across the seam
        if abs(d[0] - p[:, 0].mean()) > 1.5:
            d = d + np.array([3.0 if d[0] < 1.5 else -3.0, 0.0])
        inc = W._incircle(p[0, 0], p[0, 1], p[1, 0], p[1, 1], p[2, 0], p[2, 1], d[0], d[1])
        assert inc <= 1e-12


def test_cavity_fields():
    m = W.cavity_mesh(16, 12, 12)
    f = W.cavity_fields(m)
    x, y = m.xy[:, 0], m.xy[:, 1]
    wall = np.zeros(m.n_nodes, bool)
    for k in range(3):
        sel = m.edge_kind[:, k] == W.EDGE_WALL
        wall[m.tri[sel, (k + 1) % 3]] = True
        wall[m.tri[sel, (k + 2) % 3]] = True
    assert np.all(f.mean_omega[wall] == 50.0)
    assert np.all(f.mean_omega >= 1.0)
    # no-slip walls and the street level: zero mean velocity
    assert np.abs(f.mean_u[wall]).max() < 1e-15
    # the recirculation is divergence-free: discrete check on the analytic stream function
    cav = y < 1.0
    xp, k = x[cav] - 1.0, math.pi
    assert np.allclose(f.mean_u[cav, 0], 0.1 * np.sin(k * xp) ** 2 * k * np.sin(2 * k * y[cav]))
    assert np.allclose(f.mean_u[cav, 1], -0.1 * k * np.sin(2 * k * xp) * np.sin(k * y[cav]) ** 2)
    top = np.isclose(y, 2.0)
    assert np.allclose(f.mean_u[top, 0], (0.1 / 0.41) * math.log(101.0))
    assert np.all(f.grad_p[y >= 1.0, 0] == -1.0) and np.all(f.grad_p[y < 1.0] == 0.0)


def test_channel_mesh_counts():
    m = W.channel_mesh(8, 6)
    a, _ = _areas(m)
    assert m.n_elems == 96 and (a > 0).all() and abs(a.sum() - 2 * 2 * math.pi) < 1e-12
    k = m.edge_kind.ravel()
    assert (k == W.EDGE_WALL).sum() == 16
