"""Oracle pin for the time step of Eq. (26) (Sec. 3.1): Delta t = CFL min_n sqrt(A_n) /
max_n ||<Z>_n||_2 with A_n the average area of the elements around node n and
Z = (U_1, U_2, U_3, omega, psi)."""
import math

import numpy as np

import oracle as O
from paper_1006_0532_amd import workloads as W

Z = (0.3, -0.4, 1.2, 2.0, 0.5)


def _uniform_state(mesh, per_elem=3):
    """per_elem identical particles in every element (inside, away from the edges)."""
    tri = mesh.tri
    P = mesh.xy[tri]
    if mesh.period_x > 0:
        L = mesh.period_x
        wrap = (P[:, :, 0].max(1) - P[:, :, 0].min(1)) > 0.5 * L
        P[wrap, :, 0] = np.where(P[wrap, :, 0] < 0.5 * L, P[wrap, :, 0] + L, P[wrap, :, 0])
    bary = np.array([[0.6, 0.2, 0.2], [0.2, 0.6, 0.2], [0.2, 0.2, 0.6]])[:per_elem]
    pts = np.einsum("kv,evd->ekd", bary, P).reshape(-1, 2)
    if mesh.period_x > 0:
        pts[:, 0] = np.mod(pts[:, 0], mesh.period_x)
    n = len(pts)
    return dict(x=pts[:, 0].copy(), y=pts[:, 1].copy(), u=np.tile(Z[:3], (n, 1)), om=np.full(n, Z[3]),
                psi=np.full(n, Z[4]), w=np.ones(n), pid=np.arange(n, dtype=np.uint64),
                elem=np.repeat(np.arange(mesh.n_elems, dtype=np.int32), per_elem))


def _ensemble(mesh):
    f = W.uniform_fields(mesh)
    g = O.Grid(mesh, f, W.model_constants())
    e = O.Ensemble(g, W.init_desc(ppe=1))
    st = _uniform_state(mesh)
    e.import_state(st, step=0, next_pid=len(st["x"]))
    return e


def test_regular_grid_closed_form():
    """Equal triangles of area (2/8)(2/6)/2 and one state everywhere."""
    mesh = W.channel_mesh(8, 6, length=2.0, stretch=1.0, jitter=0.0, random_diagonals=False,
                          bottom=W.EDGE_SLIP, top=W.EDGE_SLIP)
    e = _ensemble(mesh)
    expect = 0.7 * math.sqrt((2.0 / 8.0) * (2.0 / 6.0) / 2.0) / math.sqrt(sum(z * z for z in Z))
    assert abs(e.cfl_dt(0.7) - expect) < 1e-14 * expect
    assert abs(e.cfl_dt(0.35) - 0.5 * expect) < 1e-14 * expect


def test_stretched_grid_takes_the_smallest_node_area():
    """Geometric rows: the smallest average area is at the wall nodes, where every element
    around the node lies in the first row (area dx h0 / 2)."""
    nx, ny = 8, 10
    mesh = W.channel_mesh(nx, ny, length=2.0, stretch=20.0, jitter=0.0, random_diagonals=False,
                          bottom=W.EDGE_SLIP, top=W.EDGE_SLIP)
    ys = np.unique(mesh.xy[:, 1])
    h0 = ys[1] - ys[0]
    e = _ensemble(mesh)
    expect = 0.7 * math.sqrt((2.0 / nx) * h0 / 2.0) / math.sqrt(sum(z * z for z in Z))
    assert abs(e.cfl_dt(0.7) - expect) < 1e-13 * expect
