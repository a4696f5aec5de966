"""Pins of the oracle's particle loop: position (Eq. 7), GLM velocity (Eqs. 10/27, 11),
turbulent frequency (Eq. 19), tracking (Sec. 3.6) and wall conditions (Sec. 3.8).

Each pin is fixed by mathematics outside the oracle: exact kinematics when noise and
forcing vanish, reflection geometry, brute-force point location, the variance of a
Wiener increment, the reflection principle of Brownian motion, and the exact
first/second-moment recursions of Euler-discretised Ornstein-Uhlenbeck and CIR
processes with frozen coefficients.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from paper_1006_0532_amd import workloads as W
from tests.common import box, edge_distance, frozen_fields


def _ens(mesh, fields, model, **init):
    g = O.Grid(mesh, fields, model)
    d = W.init_desc(**init)
    return g, O.Ensemble(g, d)


def test_frozen_motion_exact_periodic():
    """nu = 0, G = 0, C0 eps = 0, no forcing: X^n = X^0 + n U dt exactly (mod L)."""
    m = box(6, 6, length=3.0)
    f = frozen_fields(m, mean_u=(0.37, 0.0, 0.1))
    mo = W.model_constants(nu=0.0)
    g, E = _ens(m, f, mo, ppe=20, u_sigma=0.0, src_r=0.0)
    s0 = E.export()
    dt = 0.013
    X = s0["x"].copy()
    for n in range(40):
        E.step(dt)
        X = X + 0.37 * dt
    s = E.export()
    assert np.array_equal(s["pid"], s0["pid"])
    d = np.mod(s["x"] - X + 1.5, 3.0) - 1.5
    assert np.abs(d).max() < 1e-12
    assert np.array_equal(s["y"], s0["y"])
    # the interpolated coefficients cancel G only to rounding (partition of unity)
    assert np.abs(s["u"][:, 0] - 0.37).max() < 1e-14 and np.abs(s["u"][:, 2] - 0.1).max() < 1e-14
    fr = g.export()["frame"]
    for i in range(0, len(s["x"]), 7):
        e, xs = g.locate_brute(s["x"][i], s["y"][i])
        if edge_distance(fr, s["elem"][i], s["x"][i], s["y"][i]) > 1e-12:
            assert e == s["elem"][i] and xs == s["x"][i]


def _fold(Y):
    t = np.mod(Y + 1.0, 4.0)
    y = np.where(t <= 2.0, t - 1.0, 3.0 - t)
    sign = np.where(t <= 2.0, 1.0, -1.0)
    return y, sign


def test_free_slip_reflection_is_a_mirror():
    """Perfect reflection at free-slip walls y = -1, +1 (Sec. 4.2): the position follows
    the unfolded straight line folded into the channel, the normal velocity flips."""
    m = box(6, 8, length=3.0)
    f = frozen_fields(m, mean_u=(0.1, 0.9, 0.0))
    g, E = _ens(m, f, W.model_constants(nu=0.0), ppe=10, u_sigma=0.0, src_r=0.0)
    s0 = E.export()
    dt = 0.01
    Y = s0["y"].copy()
    for n in range(300):
        E.step(dt)
        Y = Y + 0.9 * dt
    s = E.export()
    y, sign = _fold(Y)
    assert np.abs(s["y"] - y).max() < 1e-11
    assert np.array_equal(np.sign(s["u"][:, 1]), sign)
    assert np.abs(np.abs(s["u"][:, 1]) - 0.9).max() < 1e-13
    assert E.counters()["reflections"] > 0


def test_no_slip_reflection_mirror_and_zero_velocity():
    """Trajectory (a) of Sec. 3.8: position mirrored across the wall, U = 0 (Eq. 56)."""
    m = box(6, 8, length=3.0, bottom=W.EDGE_WALL, top=W.EDGE_WALL)
    f = frozen_fields(m, mean_u=(0.0, -0.5, 0.0))
    g, E = _ens(m, f, W.model_constants(nu=0.0), ppe=10, u_sigma=0.0, src_r=0.0)
    s0 = E.export()
    dt = 0.02
    E.step(dt)
    s = E.export()
    ystar = s0["y"] - 0.5 * dt
    hit = ystar < -1.0
    assert hit.sum() > 0
    assert np.abs(s["y"][hit] - (-2.0 - ystar[hit])).max() < 1e-14
    assert np.all(s["u"][hit] == 0.0)
    assert np.abs(s["u"][~hit, 1] + 0.5).max() < 1e-14
    assert E.counters()["wall_a"] == hit.sum()
    assert E.counters()["wall_b"] == 0    # nu = 0: no trajectory (b)


def test_walk_agrees_with_brute_force_location():
    """Large steps force multi-element walks through a jittered grid with periodic and
    slip boundaries; every final host equals the brute-force search (closed test,
    lowest element id) except within 1e-12 of an edge."""
    m = box(5, 4, length=2.5, jitter=0.2, seed=5)
    f = frozen_fields(m, mean_u=(1.0, 0.5, 0.0))
    g, E = _ens(m, f, W.model_constants(nu=0.0), ppe=200, u_sigma=0.4, src_r=0.0)
    fr = g.export()["frame"]
    checked = 0
    for n in range(6):
        E.step(0.25)
        s = E.export()
        for i in range(len(s["x"])):
            x, y, e = s["x"][i], s["y"][i], s["elem"][i]
            lam = g.bary(e, x, y)
            assert lam.min() >= 0.0
            if edge_distance(fr, e, x, y) < 1e-12:
                continue
            eb, xs = g.locate_brute(x, y)
            assert eb == e and xs == x
            checked += 1
    c = E.counters()
    assert checked > 0.99 * 6 * len(s["x"])
    assert c["walk_steps"] > 2 * len(s["x"])          # walks of several elements
    assert c["reflections"] > 0


def test_diffusion_variance():
    """Eq. (7) with U = 0: the displacement over one step is (2 nu)^1/2 dW, variance 2 nu dt."""
    m = box(8, 8, length=2.0)
    nu, dt = 1.0e-3, 2.0e-3
    f = frozen_fields(m)
    g, E = _ens(m, f, W.model_constants(nu=nu), ppe=2000, u_sigma=0.0, src_r=0.0)
    s0 = E.export()
    E.step(dt)
    s = E.export()
    dx = np.mod(s["x"] - s0["x"] + 1.0, 2.0) - 1.0
    far = np.abs(s0["y"]) < 0.9
    dy = (s["y"] - s0["y"])[far]
    n = dx.size
    v = 2 * nu * dt
    assert abs(dx.mean()) < 5 * math.sqrt(v / n)
    assert abs(dx.var() - v) < 5 * v * math.sqrt(2.0 / n)
    assert abs(dy.var() - v) < 5 * v * math.sqrt(2.0 / dy.size)
    assert abs(np.corrcoef(dx[far], dy)[0, 1]) < 5 / math.sqrt(dy.size)


def _place(g, E, xs, ys, u, om):
    n = len(xs)
    el = np.empty(n, np.int32)
    xx = np.empty(n)
    for i in range(n):
        el[i], xx[i] = g.locate_brute(xs[i], ys[i])
        assert el[i] >= 0
    st = dict(x=xx, y=np.asarray(ys, float), u=np.tile(u, (n, 1)), om=np.full(n, om),
              psi=np.zeros(n), w=np.ones(n), pid=np.arange(n, dtype=np.uint64), elem=el)
    E.import_state(st, step=0, next_pid=n)


@pytest.mark.parametrize("z", [0.5, 1.0, 2.0])
def test_wall_event_probability_reflection_principle(z):
    """Trajectories (a) + (b) of Sec. 3.8 together fire with the probability that a
    Brownian path with variance 2 nu t started at distance d touches the wall within
    dt: 2 Phi(-d / (2 nu dt)^1/2) (reflection principle).  This fixes Eq. (53)."""
    m = box(8, 8, length=2.0, bottom=W.EDGE_WALL, top=W.EDGE_WALL)
    nu, dt = 1.0e-4, 1.0e-3
    f = frozen_fields(m)
    g, E = _ens(m, f, W.model_constants(nu=nu), ppe=1, u_sigma=0.0, src_r=0.0)
    N = 20000
    d = z * math.sqrt(2 * nu * dt)
    rng = np.random.default_rng(3)
    _place(g, E, rng.uniform(0, 2.0, N), np.full(N, -1.0 + d), (0.0, 0.0, 0.0), 1.0)
    E.step(dt)
    c = E.counters()
    p = 2 * stats.norm.cdf(-z)
    phat = (c["wall_a"] + c["wall_b"]) / N
    assert abs(phat - p) < 5 * math.sqrt(p * (1 - p) / N)
    pa = stats.norm.cdf(-z)
    assert abs(c["wall_a"] / N - pa) < 5 * math.sqrt(pa * (1 - pa) / N)


def test_glm_ou_moment_recursions():
    """Frozen uniform coefficients make every velocity component an Euler-discretised
    OU process (Eq. 27): m <- m + dt (a + g (m - U)), v <- (1 + g dt)^2 v + C0 eps dt,
    with g = (wp - eps/2)/k from Eq. (11) and eps from Eq. (18).  Free-slip reflection
    flips the sign of the zero-mean wall-normal component, which keeps its law."""
    m = box(20, 20, length=2.0)
    nu, dt, Om, r = 1.0e-4, 1.0e-3, 5.0, 0.0025
    wp = -0.1
    f = W.uniform_fields(m, grad_p=(-0.5, 0.0), wp=(wp,) * 3 + (0,) * 3, mean_u=(0.2, 0, 0),
                         mean_omega=Om, rey=(r,) * 3 + (0,) * 3)
    mo = W.model_constants(nu=nu)
    g, E = _ens(m, f, mo, ppe=150, u_sigma=0.1, src_r=0.0)
    k = 1.5 * r
    eps = Om * (k + nu * mo["CT"] ** 2 * Om)
    gg = (wp - 0.5 * eps) / k
    c0e = -2.0 * (3 * wp * r) / (3 * k)
    s = E.export()
    N = len(s["x"])
    mean = s["u"].mean(0)
    var = s["u"].var(0)
    a = np.array([0.5, 0.0, 0.0])
    ubar = np.array([0.2, 0.0, 0.0])
    for n in range(60):
        E.step(dt)
        mean = mean + dt * (a + gg * (mean - ubar))
        var = (1 + gg * dt) ** 2 * var + c0e * dt
    s = E.export()
    got_m, got_v = s["u"].mean(0), s["u"].var(0)
    for i in range(3):
        assert abs(got_m[i] - mean[i]) < 5 * math.sqrt(var[i] / N), i
        assert abs(got_v[i] - var[i]) < 5 * var[i] * math.sqrt(2.0 / N), i
    # continuous OU closed form, within the O(dt) Euler error plus sampling
    t = 60 * dt
    v_inf = c0e / (-2 * gg)
    v_t = v_inf + (0.01 - v_inf) * math.exp(2 * gg * t)
    assert abs(got_v[2] - v_t) < 0.05 * v_t


def test_frequency_cir_stationary_mean():
    """With frozen <omega> and S_omega, Euler of Eq. (19) keeps the linear mean recursion
    m <- m - C3 W (m - W) dt - S W m dt, whose fixed point is C3 W / (C3 + S)."""
    m = box(20, 20, length=2.0)
    nu, dt, Om = 1.0e-4, 1.0e-3, 10.0
    f = W.uniform_fields(m, mean_omega=Om)
    mo = W.model_constants(nu=nu)
    g, E = _ens(m, f, mo, ppe=150, u_sigma=0.01, src_r=0.0)
    S = mo["Cw2"]          # no mean shear: production is zero
    C3 = mo["C3"]
    s = E.export()
    N = len(s["x"])
    mean = s["om"].mean()
    steps = 150
    for n in range(steps):
        E.step(dt)
        mean = mean - C3 * Om * (mean - Om) * dt - S * Om * mean * dt
    s = E.export()
    assert abs(s["om"].mean() - mean) < 5 * math.sqrt(s["om"].var() / N)
    fixed = C3 * Om / (C3 + S)
    rho = 1 - (C3 + S) * Om * dt
    assert abs(mean - fixed) <= abs(rho) ** steps * 2.0 + 1e-12
    assert E.counters()["omega_reflections"] < 1e-4 * N * steps


def test_source_sets_scalar():
    m, f, mo, ini = W.channel_small()
    g, E = _ens(m, f, mo, ppe=50)
    s = E.export()
    d2 = (s["x"] - math.pi) ** 2 + s["y"] ** 2
    assert np.array_equal(s["psi"] == 1.0, d2 < 0.05 ** 2)
    assert np.all((s["psi"] == 0.0) | (s["psi"] == 1.0))
    E.step(1e-3)
    s = E.export()
    d2 = (s["x"] - math.pi) ** 2 + s["y"] ** 2
    assert E.counters()["source_hits"] == (d2 < 0.05 ** 2).sum()
    assert np.all((s["psi"] >= 0.0) & (s["psi"] <= 1.0))


def test_initial_distribution():
    """Set-up of Sec. 3.7: equal count per element, uniform inside each element,
    Gaussian velocity about the nodal mean, Gamma frequency (shape 4)."""
    m, f, mo, ini = W.channel_small()
    g, E = _ens(m, f, mo, ppe=50)
    s = E.export()
    assert np.array_equal(np.bincount(s["elem"], minlength=m.n_elems), np.full(m.n_elems, 50))
    assert np.array_equal(s["pid"], np.arange(m.n_elems * 50, dtype=np.uint64))
    assert np.array_equal(s["elem"], (s["pid"] // 50).astype(np.int32))
    sub = np.arange(0, len(s["x"]), 10)
    lam = np.array([g.bary(s["elem"][i], s["x"][i], s["y"][i]) for i in sub])
    assert lam.min() > -1e-13
    # barycentric coordinates of uniform points in a triangle: lambda_B ~ Beta(1, 2)
    assert stats.kstest(lam[:, 1], "beta", args=(1, 2)).pvalue > 1e-4
    nodes = m.tri[s["elem"][sub]]
    mu = np.einsum("pk,pkc->pc", lam, f.mean_u[nodes])
    omn = np.einsum("pk,pk->p", lam, f.mean_omega[nodes])
    du = s["u"][sub] - mu
    n = du.shape[0]
    assert np.abs(du.mean(0)).max() < 5 * 0.05 / math.sqrt(n)
    assert np.abs(du.std(0) - 0.05).max() < 5 * 0.05 * math.sqrt(0.5 / n)
    ratio = s["om"][sub] / omn            # Gamma(4, 1/4): mean 1, variance 1/4
    assert abs(ratio.mean() - 1) < 5 * math.sqrt(0.25 / n)
    assert stats.kstest(ratio, "gamma", args=(4.0, 0, 0.25)).pvalue > 1e-4
    assert np.all(s["w"] == 1.0)


def test_position_uses_start_of_step_velocity():
    """Forward Euler (Sec. 3.1) of Eq. (7): X^{n+1} = X^n + U^n dt, with the velocity of
    the start of the step even when the velocity itself changes during the step."""
    m = box(8, 8, length=3.0)
    f = W.uniform_fields(m, grad_p=(-3.0, 0.0), mean_u=(0.5, 0.0, 0.0), mean_omega=20.0)
    g, E = _ens(m, f, W.model_constants(nu=0.0), ppe=50, u_sigma=0.2, src_r=0.0)
    s0 = E.export()
    dt = 0.004
    E.step(dt)
    s = E.export()
    assert np.abs(s["u"] - s0["u"]).max() > 1e-3
    moved = np.abs(s0["y"] + s0["u"][:, 1] * dt) < 0.99
    dx = np.mod(s["x"] - (s0["x"] + s0["u"][:, 0] * dt) + 1.5, 3.0) - 1.5
    assert np.abs(dx[moved]).max() < 1e-14
    assert np.abs(s["y"] - (s0["y"] + s0["u"][:, 1] * dt))[moved].max() < 1e-15


def test_laplacian_drift_of_mean_velocity():
    """The 2 nu lap<U> dt drift of Eq. (27): with U^0 = <U>(X), G = 0 and C0 eps = 0 the
    mean increment of U_3 = c y^2 is 2 nu (2 c) dt at particles in interior elements of a
    regular grid (the two-pass Laplacian is exact there)."""
    m = W.channel_mesh(16, 16, length=2.0, stretch=1.0, jitter=0.0, random_diagonals=False,
                       bottom=W.EDGE_SLIP, top=W.EDGE_SLIP)
    nu, dt, c = 0.01, 0.05, 1.0
    om, r = 1.0, 0.5
    k = 1.5 * r
    eps = om * (k + nu * 36.0 * om)
    f = W.uniform_fields(m, wp=(0.5 * eps,) * 3 + (0,) * 3, mean_omega=om, rey=(r,) * 3 + (0,) * 3)
    f.mean_u[:, 2] = c * m.xy[:, 1] ** 2
    g, E = _ens(m, f, W.model_constants(nu=nu), ppe=400, u_sigma=0.0, src_r=0.0)
    s0 = E.export()
    E.step(dt)
    s = E.export()
    inner = np.abs(m.xy[m.tri[s0["elem"]], 1]).max(1) < 0.7
    du = (s["u"][:, 2] - s0["u"][:, 2])[inner]
    n = du.size
    expect = 2 * nu * 2 * c * dt
    # noise: (2 nu)^1/2 dU3/dy dW_y with |dU3/dy| <= 2 c 0.7
    sd = math.sqrt(2 * nu) * 2 * c * 0.7 * math.sqrt(dt)
    assert abs(du.mean() - expect) < 5 * sd / math.sqrt(n)
    assert expect > 10 * sd / math.sqrt(n)


def test_wiener_increments_shared_and_independent():
    """Eqs. (7) and (8) use the same dW (Sec. 2): the velocity and position increments
    covary by 2 nu dU1/dy dt; dW' of Eq. (10) is independent of dW."""
    m = W.channel_mesh(16, 16, length=2.0, stretch=1.0, jitter=0.0, random_diagonals=False,
                       bottom=W.EDGE_SLIP, top=W.EDGE_SLIP)
    nu, dt, a = 2e-3, 1e-3, 3.0
    f = W.uniform_fields(m, wp=(-0.1,) * 3 + (0,) * 3, mean_omega=5.0)
    f.mean_u[:, 0] = a * m.xy[:, 1]          # dU1/dy = a
    g, E = _ens(m, f, W.model_constants(nu=nu), ppe=400, u_sigma=0.0, src_r=0.0)
    s0 = E.export()
    E.step(dt)
    s = E.export()
    keep = np.abs(s0["y"]) < 0.9
    dX = (np.mod(s["x"] - s0["x"] - s0["u"][:, 0] * dt + 1.0, 2.0) - 1.0)[keep]
    dY = (s["y"] - s0["y"] - s0["u"][:, 1] * dt)[keep]
    dU = (s["u"] - s0["u"])[keep]
    n = dX.size
    cov = np.mean((dY - dY.mean()) * (dU[:, 0] - dU[:, 0].mean()))
    expect = 2 * nu * a * dt
    sd = math.sqrt(dY.var() * dU[:, 0].var() / n)
    assert abs(cov - expect) < 5 * sd and expect > 10 * sd
    for j in range(3):       # x-increment uncorrelated with every velocity increment
        assert abs(np.corrcoef(dX, dU[:, j])[0, 1]) < 5 / math.sqrt(n)
    assert abs(np.corrcoef(dU[:, 1], dU[:, 2])[0, 1]) < 5 / math.sqrt(n)


def test_reflection_in_rotated_rectangle():
    """Perfect reflection (Sec. 3.8) in a rectangle with free-slip sides, rotated by 30
    degrees: the result equals folding each coordinate of the straight path in the
    rectangle's own axes, with the matching velocity component reversed."""
    th = math.radians(30.0)
    Rm = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    base = W.channel_mesh(6, 6, length=2.0, stretch=1.0, jitter=0.1, periodic=False,
                          bottom=W.EDGE_SLIP, top=W.EDGE_SLIP, seed=9)
    m = W.Mesh(base.xy @ Rm.T, base.tri, base.edge_kind, 0.0)
    U = np.array([-0.9, 0.7])
    Ur = Rm @ U
    f = frozen_fields(m, mean_u=(Ur[0], Ur[1], 0.0))
    g, E = _ens(m, f, W.model_constants(nu=0.0), ppe=30, u_sigma=0.0, src_r=0.0)
    s0 = E.export()
    dt = 0.2
    E.step(dt)
    s = E.export()
    P0 = np.column_stack([s0["x"], s0["y"]]) @ Rm          # back to rectangle axes
    Q = P0 + U * dt

    def fold(v, lo, hi):
        L = hi - lo
        t = np.mod(v - lo, 2 * L)
        return np.where(t <= L, lo + t, lo + 2 * L - t), np.where(t <= L, 1.0, -1.0)

    fx, sx = fold(Q[:, 0], 0.0, 2.0)
    fy, sy = fold(Q[:, 1], -1.0, 1.0)
    got = np.column_stack([s["x"], s["y"]]) @ Rm
    assert np.abs(got[:, 0] - fx).max() < 1e-12 and np.abs(got[:, 1] - fy).max() < 1e-12
    gu = np.column_stack([s["u"][:, 0], s["u"][:, 1]]) @ Rm
    assert np.abs(gu[:, 0] - sx * U[0]).max() < 1e-12 and np.abs(gu[:, 1] - sy * U[1]).max() < 1e-12
    assert (sx < 0).sum() > 0 and (sy < 0).sum() > 0


def test_frequency_with_production():
    """Eq. (20): a uniform shear dU1/dy = a with <uv> = R12 gives production
    P = -R12 a, which shifts the source term S = C_w2 - C_w1 P / eps of Eq. (19)."""
    m = box(20, 20, length=2.0)
    nu, dt, Om, a = 1.0e-4, 1.0e-3, 2.0, -20.0
    R = (0.01, 0.01, 0.01, 0.008, 0.0, 0.0)
    f = W.uniform_fields(m, mean_omega=Om, rey=R)
    f.mean_u[:, 0] = a * m.xy[:, 1]
    mo = W.model_constants(nu=nu)
    g, E = _ens(m, f, mo, ppe=150, u_sigma=0.01, src_r=0.0)
    k = 0.015
    eps = Om * (k + nu * mo["CT"] ** 2 * Om)
    S = mo["Cw2"] - mo["Cw1"] * (-R[3] * a) / eps
    C3 = mo["C3"]
    s = E.export()
    N = len(s["x"])
    mean = s["om"].mean()
    for n in range(150):
        E.step(dt)
        mean = mean - C3 * Om * (mean - Om) * dt - S * Om * mean * dt
    s = E.export()
    assert abs(s["om"].mean() - mean) < 5 * math.sqrt(s["om"].var() / N)
