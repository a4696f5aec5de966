"""Oracle pins for the second estimator of Sec. 3.3 (element means averaged to the nodes,
Eqs. 35-36, with statistics used as element averages of the nodal values)."""
import numpy as np

import oracle as O
from paper_1006_0532_amd import workloads as W
from tests.common import frozen_fields


def _box(nx=4, ny=4):
    return W.channel_mesh(nx, ny, length=2.0, stretch=1.0, jitter=0.15, seed=4, periodic=False,
                          bottom=W.EDGE_SLIP, top=W.EDGE_SLIP)


def _random_state(mesh, per_elem, rng):
    """per_elem particles at random interior points of every element, random states."""
    P = mesh.xy[mesh.tri]
    b = rng.dirichlet([2.0, 2.0, 2.0], size=(mesh.n_elems, per_elem))
    pts = np.einsum("ekv,evd->ekd", b, P).reshape(-1, 2)
    n = len(pts)
    return dict(x=pts[:, 0].copy(), y=pts[:, 1].copy(), u=rng.normal(0.5, 0.3, (n, 3)),
                om=rng.gamma(4.0, 0.5, n), psi=rng.uniform(0, 1, n), w=rng.uniform(0.5, 1.5, n),
                pid=np.arange(n, dtype=np.uint64), elem=np.repeat(np.arange(mesh.n_elems, dtype=np.int32), per_elem))


def test_two_pass_estimator_by_brute_force():
    """Element means and central moments of every element, then plain averages over the
    elements around each node (empty elements left out), written out as loops."""
    rng = np.random.default_rng(12)
    mesh = _box()
    per = rng.integers(0, 4, mesh.n_elems)     # some empty elements
    st = _random_state(mesh, 3, rng)
    keep = np.concatenate([np.arange(3) < per[e] for e in range(mesh.n_elems)])
    st = {k: v[keep] for k, v in st.items()}
    st["pid"] = np.arange(len(st["x"]), dtype=np.uint64)
    g = O.Grid(mesh, frozen_fields(mesh), W.model_constants())
    e = O.Ensemble(g, W.init_desc(ppe=1, estimator=1))
    e.import_state(st, step=0, next_pid=len(st["x"]))
    got = e.stats()
    q5 = np.column_stack([st["u"], st["om"], st["psi"]])
    elem_stats = {}
    for el in range(mesh.n_elems):
        idx = [i for i in range(len(st["x"])) if st["elem"][i] == el]
        if not idx:
            continue
        w = st["w"][idx]
        m = (w[:, None] * q5[idx]).sum(0) / w.sum()
        d = q5[idx] - m
        pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2), (4, 4)]
        c = [float((w * d[:, a] * d[:, b]).sum() / w.sum()) for a, b in pairs]
        elem_stats[el] = (w.sum(), m, np.array(c))
    for n in range(mesh.n_nodes):
        around = [el for el in range(mesh.n_elems) if n in mesh.tri[el]]
        full = [el for el in around if el in elem_stats]
        Wn = sum(elem_stats[el][0] for el in full)
        assert abs(got[n, 0] - Wn) <= 1e-13 * max(1.0, Wn)
        if not full:
            assert np.all(np.isnan(got[n, 1:]))
            continue
        m = np.mean([elem_stats[el][1] for el in full], axis=0)
        c = np.mean([elem_stats[el][2] for el in full], axis=0)
        np.testing.assert_allclose(got[n, 1:6], m, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(got[n, 6:], c, rtol=1e-12, atol=1e-14)


def test_element_averaged_fields_in_the_velocity_update():
    """With G = 0, C0 eps = 0 and nu = 0, one step changes U_1 by -d<P>/dx dt: with a
    pressure gradient equal to x at the nodes, every particle of an element sees the
    average of its three nodal values, wherever it sits (P1 interpolation would give its
    own x)."""
    mesh = _box(6, 4)
    f = frozen_fields(mesh)
    f.grad_p[:, 0] = mesh.xy[:, 0]
    mo = W.model_constants(nu=0.0)
    dt = 1e-3
    for est in (0, 1):
        g = O.Grid(mesh, f, mo)
        e = O.Ensemble(g, W.init_desc(ppe=5, u_sigma=0.0, estimator=est))
        a = e.export()
        e.step(dt)
        b = e.export()
        du = b["u"][:, 0] - a["u"][:, 0]
        cx = mesh.xy[mesh.tri[a["elem"]], 0].mean(axis=1)
        expect = -(cx if est == 1 else a["x"]) * dt
        np.testing.assert_allclose(du, expect, rtol=1e-9, atol=1e-15)
