"""Pins of the oracle's grid layer: P1 shape functions (Eqs. 37-38, 44-45), element
gradients (Eqs. 39-40), the two-pass second derivative (Sec. 3.4), adjacency and
wall lines."""
import numpy as np
import pytest

import oracle as O
from paper_1006_0532_amd import workloads as W
from tests.common import box


@pytest.fixture(scope="module")
def chan():
    m, f, mo, _ = W.channel_small()
    return m, f, O.Grid(m, f, mo)


def test_areas_cover_domain(chan):
    m, f, g = chan
    ex = g.export()
    assert (ex["area"] > 0).all()
    assert abs(ex["area"].sum() - 4 * np.pi) < 1e-12


def test_vertex_and_centroid_coordinates(chan):
    m, f, g = chan
    fr = g.export()["frame"]
    rng = np.random.default_rng(1)
    for e in rng.integers(0, m.n_elems, 200):
        v = fr[e].reshape(3, 2)
        for k in range(3):
            lam = g.bary(e, *v[k])
            assert np.allclose(lam, np.eye(3)[k], atol=1e-13)
        lam = g.bary(e, *v.mean(0))
        assert np.allclose(lam, 1 / 3, atol=1e-13)


def test_linear_fields_interpolate_exactly(chan):
    """sum_k lambda_k q(v_k) = q(P) for linear q: pins the signs and the vertex roles of
    the two cross products of Eqs. (44)-(45) and the N^B complement."""
    m, f, g = chan
    fr = g.export()["frame"]
    rng = np.random.default_rng(2)
    for e in rng.integers(0, m.n_elems, 300):
        v = fr[e].reshape(3, 2)
        a, b = rng.uniform(0, 1, 2)
        if a + b > 1:
            a, b = 1 - a, 1 - b
        P = v[0] + a * (v[1] - v[0]) + b * (v[2] - v[0])
        lam = g.bary(e, *P)
        assert abs(lam.sum() - 1.0) < 4e-16 * 4
        for q in (lambda p: 0.3 + 1.7 * p[0] - 2.1 * p[1], lambda p: -5.0 * p[1], lambda p: p[0]):
            assert abs(sum(lam[k] * q(v[k]) for k in range(3)) - q(P)) < 1e-13
        assert (lam >= -1e-14).all()
        # outside points give a negative coordinate opposite the crossed edge
        Q = v[0] + 1.3 * (v[1] - v[0]) - 0.1 * (v[2] - v[0])
        assert g.bary(e, *Q).min() < 0


def test_gradients_of_linear_fields_exact():
    m = box(10, 12, jitter=0.1, length=3.0)
    f = W.uniform_fields(m)
    x, y = m.xy[:, 0], m.xy[:, 1]
    f.mean_u[:, 0] = 0.4 - 1.2 * y
    f.mean_u[:, 1] = 2.5 * y
    f.mean_u[:, 2] = -0.75 * y + 3
    g = O.Grid(m, f, W.model_constants())
    gu = g.export()["gradu"]
    assert np.abs(gu[:, 0]).max() < 1e-13 and np.abs(gu[:, 1] + 1.2).max() < 1e-13
    assert np.abs(gu[:, 2]).max() < 1e-13 and np.abs(gu[:, 3] - 2.5).max() < 1e-13
    assert np.abs(gu[:, 5] + 0.75).max() < 1e-13
    lap = g.export()["lapu"]
    assert np.abs(lap).max() < 1e-12


def test_gradient_x_linear_across_periodic_seam():
    """d/dx of a field linear in x is exact away from the seam and the element frames of
    the seam elements keep the gradient continuous."""
    m = box(12, 6, jitter=0.0, length=3.0)
    f = W.uniform_fields(m)
    f.mean_u[:, 1] = 0.5 * m.xy[:, 1] ** 2      # x-independent, periodic
    g = O.Grid(m, f, W.model_constants())
    gu = g.export()["gradu"]
    assert np.abs(gu[:, 2]).max() < 1e-13      # d/dx of a field independent of x


def test_two_pass_laplacian_exact_for_quadratics_on_regular_grid():
    """On a regular triangulation with one diagonal direction the two averaging passes of
    Sec. 3.4 reproduce the Laplacian of a quadratic exactly at interior nodes."""
    m = W.channel_mesh(16, 16, length=2.0, stretch=1.0, jitter=0.0, random_diagonals=False)
    f = W.uniform_fields(m)
    y = m.xy[:, 1]
    f.mean_u[:, 0] = y * y
    f.mean_u[:, 1] = 0.5 * y * y + 0.3 * y
    g = O.Grid(m, f, W.model_constants())
    lap = g.export()["lapu"]
    interior = np.abs(y) < 0.7
    assert np.abs(lap[interior, 0] - 2.0).max() < 1e-12
    assert np.abs(lap[interior, 1] - 1.0).max() < 1e-12


def test_neighbours_symmetric_and_kinds(chan):
    m, f, g = chan
    ex = g.export()
    nbr, kind = ex["nbr"], ex["kind"]
    for e in range(m.n_elems):
        for k in range(3):
            o = nbr[e, k]
            if o < 0:
                assert kind[e, k] == W.EDGE_WALL
                continue
            assert e in nbr[o]
            kb = list(nbr[o]).index(e)
            assert kind[e, k] == kind[o, kb]
    # 2 seam elements per row cross the seam; 40 wall edges on each wall
    assert (kind == W.EDGE_PERIODIC).sum() == 2 * 50
    assert (kind == W.EDGE_WALL).sum() == 80


def test_wall_lines_of_channel(chan):
    m, f, g = chan
    ex = g.export()
    wall = ex["wall"].astype(bool)
    wl = ex["wline"][wall]
    lower = wl[:, 1] < 0
    assert np.all(wl[lower, 1] == -1.0) and np.allclose(wl[lower, 2:], [0, 1], atol=1e-15)
    assert np.all(wl[~lower, 1] == 1.0) and np.allclose(wl[~lower, 2:], [0, -1], atol=1e-15)
    # wall elements are exactly those touching the first or last node row
    ncol = 40
    rows = m.tri // ncol
    expect = (rows.min(1) == 0) | (rows.max(1) == 50)
    assert np.array_equal(wall, expect)


def test_mesh_errors():
    m, f, mo, _ = W.channel_small(nx=6, ny=4)
    bad = W.Mesh(m.xy, m.tri[:, ::-1].copy(), m.edge_kind, m.period_x)
    with pytest.raises(ValueError, match="counter-clockwise"):
        O.Grid(bad, f, mo)
    k = m.edge_kind.copy()
    k[k == W.EDGE_WALL] = W.EDGE_INTERIOR
    with pytest.raises(ValueError, match="wall or slip"):
        O.Grid(W.Mesh(m.xy, m.tri, k, m.period_x), f, mo)
    f2 = W.channel_fields(m)
    f2.mean_omega[3] = np.nan
    with pytest.raises(ValueError, match="non-finite"):
        O.Grid(m, f2, mo)
