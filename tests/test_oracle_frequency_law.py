"""Pins of the oracle's turbulent-frequency diffusion (Eq. 19) and of the frequency drawn
after a no-slip wall event (Eq. 58).

With frozen <omega> = W and S_omega, Eq. (19) is a square-root (CIR) diffusion
    d omega = -(C3 + S) W omega dt + C3 W^2 dt + (2 C3 C4 W^2 omega)^1/2 dW.
Its forward-Euler step keeps two exact moment recursions (dW is independent of omega
and the drift is linear):
    m' = (1 - a dt) m + C3 W^2 dt,
    v' = (1 - a dt)^2 v + 2 C3 C4 W^2 dt E|omega|,      a = (C3 + S) W,
whose fixed point is the Euler stationary variance s^2 b / (a (2 - a dt)) with
s^2 = 2 C3 C4 W^2 and b = C3 W / (C3 + S).  The continuous process is stationary in
the Gamma law of shape 2 a b / s^2 = 1 / C4 and mean b (Feller), which small-dt Euler
paths keep.  The variance fixes the diffusion coefficient (its factor 2, the power of
<omega>, |omega|), which the mean recursion alone does not see.

Eq. (58) draws a new frequency after trajectory (a) or (b): Gamma with variance
C4 <omega>^2 about the nodal mean at the particle, i.e. shape 1/C4 and mean <omega>
interpolated at the post-reflection position.
"""
import math

import numpy as np
from scipy import stats

import oracle as O
from paper_1006_0532_amd import workloads as W
from tests.common import box


def _with_frequencies(E, om):
    """Keep the oracle's own positions, velocities and pids; replace the frequencies."""
    s = E.export()
    s["om"] = om
    E.import_state(s, step=E.step_index, next_pid=int(s["pid"].max()) + 1)


def _cir_setup(Om, ppe, seed):
    m = box(20, 20, length=2.0)
    f = W.uniform_fields(m, mean_omega=Om)       # no mean shear: production is zero
    mo = W.model_constants(nu=1.0e-4)
    g = O.Grid(m, f, mo)
    E = O.Ensemble(g, W.init_desc(ppe=ppe, u_sigma=0.01, src_r=0.0, seed=seed))
    C3, C4, S = mo["C3"], mo["C4"], mo["Cw2"]
    return g, E, C3, C4, S


def test_frequency_euler_variance_recursion():
    """Mean and variance of Euler's Eq. (19) follow the exact recursions from a
    non-stationary start, through the whole relaxation to the Euler stationary
    variance (5 sigma of the sample moments)."""
    Om, dt, steps = 10.0, 1.0e-3, 100
    g, E, C3, C4, S = _cir_setup(Om, 60, 0x5151)
    rng = np.random.default_rng(7)
    N = E.count()
    om0 = rng.gamma(2.0, 6.0, N)                 # mean 12, far from the fixed point 8.7
    _with_frequencies(E, om0)
    a = (C3 + S) * Om
    m, v = om0.mean(), om0.var()
    for _ in range(steps):
        E.step(dt)
        # E|omega| = E omega: a negative Euler value is reflected, and this test holds
        # such events below 1e-4 per particle-step (checked below)
        v = (1 - a * dt) ** 2 * v + 2 * C3 * C4 * Om * Om * dt * m
        m = (1 - a * dt) * m + C3 * Om * Om * dt
    om = E.export()["om"]
    got_m, got_v = om.mean(), om.var()
    m4 = np.mean((om - got_m) ** 4)
    assert abs(got_m - m) < 5 * math.sqrt(got_v / N)
    assert abs(got_v - v) < 5 * math.sqrt((m4 - got_v ** 2) / N)
    # after a t = 5.7 e-folds of the mean the recursion is close to its fixed point
    b = C3 * Om / (C3 + S)
    s2 = 2 * C3 * C4 * Om * Om
    assert abs(v / (s2 * b / (a * (2 - a * dt))) - 1) < 1e-2
    assert E.counters()["omega_reflections"] < 1e-4 * N * steps


def test_frequency_stationary_gamma_law():
    """Started in the stationary Gamma(1/C4, mean b) law (numpy's sampler), small-dt
    Euler of Eq. (19) stays in it: KS test after 2 a t = 5.7 e-folds, mean and the
    Euler stationary variance within 5 sigma."""
    Om, dt, steps = 10.0, 1.0e-4, 500
    g, E, C3, C4, S = _cir_setup(Om, 60, 0x5152)
    b = C3 * Om / (C3 + S)
    rng = np.random.default_rng(8)
    N = E.count()
    shape = 1.0 / C4
    _with_frequencies(E, rng.gamma(shape, b / shape, N))
    E.step(dt, steps)
    om = E.export()["om"]
    a = (C3 + S) * Om
    v_euler = 2 * C3 * C4 * Om * Om * b / (a * (2 - a * dt))
    m4 = np.mean((om - om.mean()) ** 4)
    assert abs(om.mean() - b) < 5 * math.sqrt(om.var() / N)
    assert abs(om.var() - v_euler) < 5 * math.sqrt((m4 - om.var() ** 2) / N)
    assert stats.kstest(om, "gamma", args=(shape, 0, b / shape)).pvalue > 1e-4


def test_wall_event_frequency_law():
    """Eq. (58) after trajectory (a): with nu = 0 and a frozen downward velocity, the
    particles that cross the no-slip wall y = -1 are mirrored (Sec. 3.8), take U = 0 and a
    frequency omega / <omega>(x_post) ~ Gamma(1/C4, scale C4), where <omega> = 6 + 4 y is
    linear (so P1 interpolation is exact) and x_post is the mirrored position."""
    m = box(10, 10, length=2.0, bottom=W.EDGE_WALL, top=W.EDGE_WALL, jitter=0.1, seed=4)
    mu = (0.3, -0.5, 0.0)
    f = W.uniform_fields(m, wp=(0.0,) * 6, mean_u=mu)
    f.mean_omega[:] = 6.0 + 4.0 * m.xy[:, 1]
    mo = W.model_constants(nu=0.0)
    g = O.Grid(m, f, mo)
    E = O.Ensemble(g, W.init_desc(ppe=500, u_sigma=0.0, src_r=0.0, seed=0x5858))
    s0 = E.export()
    dt = 0.2
    E.step(dt)
    s = E.export()
    assert np.array_equal(s["pid"], s0["pid"])
    ystar = s0["y"] + s0["u"][:, 1] * dt
    hit = ystar < -1.0
    n = int(hit.sum())
    assert n > 3000
    c = E.counters()
    assert c["wall_a"] == n and c["wall_b"] == 0
    assert np.abs(s["y"][hit] - (-2.0 - ystar[hit])).max() < 1e-13
    assert np.all(s["u"][hit] == 0.0)
    ratio = s["om"][hit] / (6.0 + 4.0 * s["y"][hit])
    C4 = mo["C4"]
    assert abs(ratio.mean() - 1.0) < 5 * math.sqrt(C4 / n)
    r4 = np.mean((ratio - ratio.mean()) ** 4)
    assert abs(ratio.var() - C4) < 5 * math.sqrt((r4 - ratio.var() ** 2) / n)
    assert stats.kstest(ratio, "gamma", args=(1.0 / C4, 0, C4)).pvalue > 1e-4
    # the draw does not depend on the frequency before the event, and its mean is taken at
    # the mirrored position: the ratio is uncorrelated with it (a mean taken at the start
    # of the step, y0 = -1.9 - y_post here, would make it fall with y_post)
    assert abs(np.corrcoef(ratio, s0["om"][hit])[0, 1]) < 5 / math.sqrt(n)
    assert abs(np.corrcoef(ratio, s["y"][hit])[0, 1]) < 5 / math.sqrt(n)
