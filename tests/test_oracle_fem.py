"""Pins of the oracle's FEM solves (Sec. 3.2): P1 element matrices against their textbook
values, a manufactured Poisson solution converging at second order, the one-dimensional
closed form of Eq. (12) between two walls with the condition of Eq. (59), hand-worked
right-hand sides of Eqs. (12)-(15), and the discrete properties of the projection
(Eqs. 31, 33): weakly divergence-free corrected velocity at interior nodes, the closed form
of the stabilisation term, invariance under a constant pressure and a zero sum."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from oracle import fem
from paper_1006_0532_amd import workloads as W

MODEL = dict(nu=1e-4, CT=6.0)


def _grid(mesh):
    g = O.Grid(mesh, W.uniform_fields(mesh), W.model_constants())
    ex = g.export()
    return ex["frame"], ex["area"]


def _channel(nx, ny, **kw):
    kw.setdefault("stretch", 1.0)
    kw.setdefault("jitter", 0.0)
    return W.channel_mesh(nx, ny, length=2.0, random_diagonals=False, **kw)


def test_element_matrices_of_the_unit_right_triangle():
    frame = np.array([[0.0, 0.0, 1.0, 0.0, 0.0, 1.0]])
    area = np.array([0.5])
    K, M = fem.element_matrices(frame, area)
    assert np.allclose(K[0], 0.5 * np.array([[2, -1, -1], [-1, 1, 0], [-1, 0, 1]]))
    assert np.allclose(M[0], np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]]) / 24.0)


def _poisson_error(n):
    """-lap u = f on the periodic strip [0, 2) x [-1, 1] with zero normal gradient at the
    free-slip walls: u = cos(pi x) cos(pi y), f = 2 pi^2 u; solution with the exact mean."""
    mesh = _channel(2 * n, 2 * n, bottom=W.EDGE_SLIP, top=W.EDGE_SLIP, jitter=0.15, seed=n)
    frame, area = _grid(mesh)
    K, M = fem.element_matrices(frame, area)
    Kg, Mg = fem.assemble(mesh.tri, K, mesh.n_nodes), fem.assemble(mesh.tri, M, mesh.n_nodes)
    x, y = mesh.xy[:, 0], mesh.xy[:, 1]
    u = np.cos(math.pi * x) * np.cos(math.pi * y)
    b = Mg @ (2 * math.pi ** 2 * u)
    nn = mesh.n_nodes
    A = sp.bmat([[Kg, np.ones((nn, 1))], [np.ones((1, nn)), None]]).tocsc()
    uh = spla.spsolve(A, np.concatenate([b, [u.sum()]]))[:nn]
    return np.sqrt((Mg @ (uh - u) ** 2).sum() / (Mg @ u ** 2).sum())


def test_poisson_converges_at_second_order():
    e1, e2 = _poisson_error(6), _poisson_error(12)
    assert e2 < 0.03 and e1 / e2 > 3.3, (e1, e2)


def _uniform_stats(mesh, U=(0.0, 0.0, 0.0), om=2.0, R=(0.5, 0.4, 0.3, 0.0, 0.0, 0.0)):
    st = np.zeros((mesh.n_nodes, 13))
    st[:, 0] = 1.0
    st[:, 1:4] = U
    st[:, 4] = om
    st[:, 6:12] = R
    return st


def test_elliptic_relaxation_between_two_walls_matches_the_closed_form():
    """Uniform statistics without mean gradient: f_ij = (1 - C1)/2 k <omega> delta_ij; L is
    uniform per component (C_xi = 2.3 for wp_22, the wall normal being +-y); the walls
    impose wp_22 = -4.5 eps and zero elsewhere.  Then wp(y) = f + (w - f) cosh(y/L) /
    cosh(1/L), approached at second order."""
    c = fem.ELLIPTIC_CONSTANTS
    errs = []
    for n in (8, 16):
        mesh = _channel(4, 2 * n)
        frame, area = _grid(mesh)
        st = _uniform_stats(mesh, om=0.5)
        wp = fem.elliptic_relaxation(mesh, frame, area, st, MODEL)
        k = 0.5 * (0.5 + 0.4 + 0.3)
        eps = 0.5 * (k + MODEL["nu"] * 36.0 * 0.5)
        y = mesh.xy[:, 1]
        err = 0.0
        for i, cxi in ((0, 1.0), (1, 2.3), (2, 1.0)):
            L = c["CL"] * max(cxi * k ** 1.5 / eps, c["Ceta"] * (MODEL["nu"] ** 3 / eps) ** 0.25)
            f = 0.5 * (1 - c["C1"]) * k * 0.5
            w = -4.5 * eps if i == 1 else 0.0
            exact = f + (w - f) * np.cosh(y / L) / np.cosh(1.0 / L)
            err = max(err, np.abs(wp[:, i, i] - exact).max() / abs(f))
        off = wp.copy()
        for i in range(3):
            off[:, i, i] = 0
        assert np.abs(off).max() < 1e-12
        errs.append(err)
    assert errs[1] < 0.01 and errs[0] / errs[1] > 3.0, errs


def test_elliptic_rhs_by_hand():
    """Simple shear <U> = (S y, 0, 0) (exact nodal gradients on any grid).  Isotropic R:
    b = 0, A_v = 1, so f_12 = k (C2 + g5/3) S, f_21 = -k g5/3 S.  Anisotropic diagonal R:
    b_11 = R11/2k - 1/3, b_22 = R22/2k - 1/3 and
    f_12 = k S (C2 A_v + g5/3 + g5 b_11), f_21 = k S (-g5/3 - g5 b_22)."""
    c = fem.ELLIPTIC_CONSTANTS
    mesh = _channel(6, 6, jitter=0.2, seed=4)
    frame, area = _grid(mesh)
    S = 0.7
    for R in ((0.4, 0.4, 0.4), (0.6, 0.3, 0.2)):
        st = _uniform_stats(mesh, R=R + (0.0, 0.0, 0.0))
        st[:, 1] = S * mesh.xy[:, 1]
        f = fem.elliptic_rhs(mesh, frame, area, st, MODEL)
        k = 0.5 * sum(R)
        Av = min(1.0, c["Cv"] * R[0] * R[1] * R[2] / (2 * k / 3) ** 3)
        b11, b22 = R[0] / (2 * k) - 1 / 3, R[1] / (2 * k) - 1 / 3
        g5 = c["gamma5"]
        assert np.allclose(f[:, 0, 1], k * S * (c["C2"] * Av + g5 / 3 + g5 * b11), rtol=1e-10)
        assert np.allclose(f[:, 1, 0], k * S * (-g5 / 3 - g5 * b22), rtol=1e-10)
        assert np.allclose(f[:, 0, 0], 0.5 * (1 - c["C1"]) * k * 2.0, rtol=1e-10)
        assert np.allclose(f[:, 0, 2], 0.0, atol=1e-13) and np.allclose(f[:, 2, 1], 0.0, atol=1e-13)


def _projection_case(cp=0.0, seed=3):
    mesh = _channel(8, 10, bottom=W.EDGE_WALL, top=W.EDGE_WALL, jitter=0.2, seed=seed, stretch=4.0)
    frame, area = _grid(mesh)
    rng = np.random.default_rng(seed)
    st = _uniform_stats(mesh)
    x, y = mesh.xy[:, 0], mesh.xy[:, 1]
    st[:, 1] = (1 - y ** 2) * (1 + 0.3 * np.sin(math.pi * x))
    st[:, 2] = 0.2 * np.cos(math.pi * x) * (1 - y ** 2)
    p_prev = rng.normal(size=mesh.n_nodes)
    return mesh, frame, area, st, p_prev


def test_projection_makes_the_velocity_weakly_divergence_free():
    """C_p = 0: int grad N_a . U^{n+1} = 0 at every node off the walls, where U^{n+1} is
    the P1 <U>* minus (dt/rho) times the element gradient of dP (Eq. 31)."""
    mesh, frame, area, st, p_prev = _projection_case()
    dt, rho = 1e-3, 1.3
    dP, g = fem.pressure_projection(mesh, frame, area, st, p_prev, dt, cp=0.0, rho=rho)
    bx, by = fem.p1_gradients(frame, area)
    tri = mesh.tri
    ue = st[:, 1][tri].mean(1) - dt / rho * g[:, 0]       # element means of the P1 field
    ve = st[:, 2][tri].mean(1) - dt / rho * g[:, 1]
    wdiv = np.zeros(mesh.n_nodes)
    for a in range(3):
        np.add.at(wdiv, tri[:, a], area * (bx[:, a] * ue + by[:, a] * ve))
    interior = np.abs(mesh.xy[:, 1]) < 1 - 1e-12
    ref = np.abs(area[:, None] * bx * st[:, 1][tri]).max()
    assert np.abs(wdiv[interior]).max() < 1e-9 * ref
    assert abs(dP.sum()) < 1e-10 * np.abs(dP).max()


def test_projection_stabilisation_closed_form():
    """A divergence-free <U>* (uniform) leaves only the C_p term of Eq. (33):
    dP = -(C_p / dt) (P^n - mean P^n); adding a constant to P^n changes nothing."""
    mesh, frame, area, st, p_prev = _projection_case()
    st[:, 1] = 1.0
    st[:, 2] = 0.0
    dP, g = fem.pressure_projection(mesh, frame, area, st, p_prev, 1e-2, cp=1e-3)
    assert np.allclose(dP, -0.1 * (p_prev - p_prev.mean()), atol=1e-12)
    dP2, _ = fem.pressure_projection(mesh, frame, area, st, p_prev + 5.0, 1e-2, cp=1e-3)
    assert np.allclose(dP, dP2, atol=1e-12)


def test_missing_statistics_are_an_error():
    mesh = _channel(4, 4)
    frame, area = _grid(mesh)
    st = _uniform_stats(mesh)
    st[3, :] = np.nan
    with pytest.raises(ValueError):
        fem.elliptic_relaxation(mesh, frame, area, st, MODEL)
    with pytest.raises(ValueError):
        fem.pressure_projection(mesh, frame, area, st, np.zeros(mesh.n_nodes), 1e-3)
