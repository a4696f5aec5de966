"""Oracle pins for statistics feedback (Sec. 3.1, Table 1 order: a step uses the Eulerian
statistics of the step before) through the particle-redistribution test of Sec. 3.7:
Eq. (27) with G = -I, C0 eps = 2, nu = 0 and the fed-back mean alpha <U> is Eq. (47),
dU = -(U - alpha <U>) dt + sqrt(2) dW.  Forward Euler gives exact recursions for the
ensemble mean and variance (Eqs. 48-50), independent of the grid."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1006_0532_amd import workloads as W

DT, ALPHA = 0.01, 0.5


def _moments(st):
    w, u = st["w"], st["u"]
    m = (w[:, None] * u).sum(0) / w.sum()
    v = (w[:, None] * (u - m) ** 2).sum(0) / w.sum()
    return m, v


def test_feedback_of_a_zero_mean_clears_the_derived_fields():
    """alpha = 0 feeds a zero mean velocity back: every element gradient and nodal
    Laplacian of <U> is zero (Eqs. 39-40 and Sec. 3.4 applied to a zero field)."""
    mesh, f, mo, ini = W.redistribution_test(nx=6, ny=8, ppe=30)
    g = O.Grid(mesh, f, mo)
    e = O.Ensemble(g, ini)
    e.feedback(0.0)
    ex = g.export()
    assert np.all(ex["gradu"] == 0.0) and np.all(ex["lapu"] == 0.0)


def test_reynolds_stress_feedback_changes_the_relaxation():
    """With the Reynolds stresses fed back, k is the particles' (about 1.5 instead of the
    frozen 3), so G = (wp - eps/2)/k becomes about -1.5 I and the velocity variance relaxes
    towards a lower level than with the frozen R (G = -I)."""
    out = []
    for rey in (False, True):
        mesh, f, mo, ini = W.redistribution_test(ppe=60)
        g = O.Grid(mesh, f, mo)
        e = O.Ensemble(g, ini)
        e.feedback(ALPHA, feed_rey=rey)
        for n in range(30):
            e.step(DT)
            e.feedback(ALPHA, feed_rey=rey)
        out.append(_moments(e.export())[1][2])
    assert out[1] < out[0] - 0.05, out


@pytest.mark.parametrize("alpha", [ALPHA, 0.9])
def test_mean_follows_the_euler_recursion_of_eq49(alpha):
    """<U>_{n+1} = <U>_n (1 - (1 - alpha) dt): the fed-back nodal means interpolated to the
    particles average to alpha times the particle mean (partition of unity)."""
    mesh, f, mo, ini = W.redistribution_test(ppe=100)
    g = O.Grid(mesh, f, mo)
    e = O.Ensemble(g, ini)
    m0, v0 = _moments(e.export())
    e.feedback(alpha)
    N = e.count()
    for n in range(1, 41):
        e.step(DT)
        e.feedback(alpha)
    m, v = _moments(e.export())
    expect = m0 * (1.0 - (1.0 - alpha) * DT) ** 40
    sigma = math.sqrt(2.0 * DT * 40 / N) + 1e-4
    assert np.all(np.abs(m - expect) < 5 * sigma), (m, expect, sigma)
    # a different alpha would be far outside: the pin sees the scale of the feedback
    wrong = m0 * (1.0 - (1.0 - (alpha + 0.3)) * DT) ** 40
    assert abs(wrong[0] - m[0]) > 10 * sigma


def test_variance_follows_the_euler_recursion():
    """Fluctuations: var_{n+1} = (1 - dt)^2 var_n + 2 dt for the components the walls do not
    couple to the inhomogeneous transient (U1 along the strip, U3 out of plane)."""
    mesh, f, mo, ini = W.redistribution_test(ppe=100)
    g = O.Grid(mesh, f, mo)
    e = O.Ensemble(g, ini)
    m0, v0 = _moments(e.export())
    e.feedback(ALPHA)
    N = e.count()
    for n in range(40):
        e.step(DT)
        e.feedback(ALPHA)
    m, v = _moments(e.export())
    expect = v0.copy()
    for n in range(40):
        expect = (1.0 - DT) ** 2 * expect + 2.0 * DT
    sigma = math.sqrt(2.0 / N) * 1.5
    for q in (0, 2):
        assert abs(v[q] - expect[q]) < 5 * sigma, (q, v, expect)


@pytest.mark.slow
@pytest.mark.parametrize("method", ["control", "app_b"])
def test_redistribution_keeps_the_steady_state(method):
    """Sec. 3.7 with particles redistributed every step (n_min = ppe / 10, as in Fig. 4),
    by the per-element number control or by the global loop of App. B: the stretched
    strip relaxes to a homogeneous state; the spatial average of the nodal <u_i u_i>
    approaches the Euler steady state 1 / (1 - dt/2) (Eq. 48's delta_ij up to the time
    step) and the mean keeps decaying by Eq. (49)."""
    mesh, f, mo, ini = W.redistribution_test(ppe=100)
    g = O.Grid(mesh, f, mo)
    e = O.Ensemble(g, ini)
    m0, _ = _moments(e.export())
    e.feedback(ALPHA)
    moved = 0
    for n in range(300):
        e.step(DT)
        if method == "control":
            r = e.control(10, 400)
            moved += r["cloned"] + r["merged"]
        else:
            moved += e.redistribute(10)
        e.feedback(ALPHA)
    assert moved > 0
    st = e.stats()
    ok = ~np.isnan(st[:, 0])
    Wn = st[ok, 0]
    rbar = (Wn[:, None] * st[ok][:, 6:9]).sum(0) / Wn.sum()
    steady = 1.0 / (1.0 - DT / 2.0)
    assert np.all(np.abs(rbar - steady) < 0.05), rbar
    m, _ = _moments(e.export())
    assert abs(m[0] - m0[0] * (1.0 - (1.0 - ALPHA) * DT) ** 300) < 0.02
