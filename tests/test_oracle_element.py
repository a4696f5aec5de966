"""Pins of the oracle's per-element algorithms: adaptive velocity binning (Sec. 3.5,
App. A), IECM mixing (Eqs. 23-25), nodal statistics (Sec. 3.3) and particle-number
control (Sec. 3.7, App. B)."""
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1006_0532_amd import workloads as W
from tests.common import box

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _worked():
    rows = []
    for line in open(os.path.join(GOLD, "binning_worked_examples.txt")):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([int(t) for t in line.split()])
    return rows


@pytest.mark.parametrize("n,b1,b2,b3,m,groups", _worked())
def test_binning_worked_examples(n, b1, b2, b3, m, groups):
    rng = np.random.default_rng(n)
    u = rng.normal(size=(n, 3))
    cp, pos, b = O.bin_element(u, np.arange(n), (b1, b2, b3), m)
    assert cp == groups
    counts = np.bincount(b, minlength=cp)
    if n % groups == 0:
        assert np.all(counts == n // groups)


def _brute_bins(u, pid, bins, m):
    """Sort-and-divide of Sec. 3.5 by plain recursion on Python lists, with the group of
    the particle at position n among N equal to floor(C n / N) (App. A)."""
    n = len(pid)
    g, P, stop = [], 1, False
    for l in range(3):
        q = max(1, n // (m * P))
        gl = 1 if stop else min(bins[l], q)
        stop = stop or gl < bins[l]
        g.append(gl)
        P *= gl
    order = sorted(range(n), key=lambda i: (u[i][0], pid[i]))
    C = 1
    for l in range(1, 3):
        C *= g[l - 1]
        groups = {}
        for r, i in enumerate(order):
            groups.setdefault(C * r // n, []).append(i)
        order = []
        for t in sorted(groups):
            order += sorted(groups[t], key=lambda i: (u[i][l], pid[i]))
    Cp = P
    return Cp, {i: r for r, i in enumerate(order)}, {i: Cp * r // n for r, i in enumerate(order)}


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 31, 50, 97, 200, 413])
@pytest.mark.parametrize("bins", [(4, 2, 2), (4, 4, 2), (5, 5, 5), (1, 1, 1), (3, 1, 2)])
def test_binning_matches_brute_force(n, bins):
    rng = np.random.default_rng(n * 31 + bins[0])
    u = rng.normal(size=(n, 3))
    pid = rng.permutation(10 * n)[:n].astype(np.uint64)
    # ties on velocity components (clones carry identical velocities) break by pid
    if n > 4:
        u[1] = u[0]
        u[3, 1] = u[2, 1]
    cp, pos, b = O.bin_element(u, pid, bins, 2)
    cpb, posb, bb = _brute_bins(u.tolist(), pid.tolist(), bins, 2)
    assert cp == cpb
    assert [posb[i] for i in range(n)] == pos.tolist()
    assert [bb[i] for i in range(n)] == b.tolist()
    counts = np.bincount(b, minlength=cp)
    assert set(counts.tolist()) <= {n // cp, -(-n // cp)}
    assert counts.min() >= min(2, n) or cp == 1


def test_binning_independent_of_input_order():
    rng = np.random.default_rng(7)
    u = rng.normal(size=(120, 3))
    pid = np.arange(120, dtype=np.uint64)
    cp, pos, b = O.bin_element(u, pid, (4, 2, 2), 2)
    perm = rng.permutation(120)
    cp2, pos2, b2 = O.bin_element(u[perm], pid[perm], (4, 2, 2), 2)
    assert np.array_equal(pos2, pos[perm]) and np.array_equal(b2, b[perm])


# ------------------------------------------------------------------- IECM

def _mixing_setup(bins, ppe=60):
    m = box(6, 6, length=2.0)
    f = W.uniform_fields(m, mean_u=(0.3, 0.0, 0.0), mean_omega=4.0)
    mo = W.model_constants()
    g = O.Grid(m, f, mo)
    d = W.init_desc(ppe=ppe, bins=bins, src_x=1.0, src_y=0.0, src_r=0.35, src_continuous=0)
    return m, g, O.Ensemble(g, d)


@pytest.mark.parametrize("bins", [(4, 2, 2), (1, 1, 1), (5, 5, 5)])
def test_iecm_conserves_bin_means_and_bounds(bins):
    """IECM (Eq. 24) relaxes every particle towards the mean of its velocity bin with a
    common factor per element, so each bin's weighted scalar sum is unchanged and the
    scalar stays within the bin's range; with one bin it is IEM (Eq. 23)."""
    m, g, E = _mixing_setup(bins)
    pre = E.export()
    assert 0 < (pre["psi"] == 1).sum() < len(pre["psi"])
    dt = 0.05
    E.step(dt)
    post = E.export()
    assert np.array_equal(pre["pid"], post["pid"])
    for e in range(m.n_elems):
        sel = np.nonzero(post["elem"] == e)[0]
        if sel.size == 0:
            continue
        cp, pos, b = O.bin_element(post["u"][sel], post["pid"][sel], bins, 2)
        fmix = min(dt / E.tm(e), 1.0)
        for k in range(cp):
            ib = sel[b == k]
            w, p0, p1 = pre["w"][ib], pre["psi"][ib], post["psi"][ib]
            assert abs((w * p1).sum() - (w * p0).sum()) <= 1e-14 * max(1.0, abs((w * p0).sum())) * len(ib)
            assert p1.min() >= p0.min() - 1e-15 and p1.max() <= p0.max() + 1e-15
            mean = (w * p0).sum() / w.sum()
            assert np.allclose(p1, p0 - fmix * (p0 - mean), atol=1e-15)
        if cp == 1:
            assert bins == (1, 1, 1) or sel.size < 4


def test_micromixing_timescale_spot_values():
    """Eq. (25) at hand-computed points: with zero mean velocity the first branch is
    infinite and t_m = max(k/eps, C_T (nu/eps)^1/2)."""
    m = box(4, 4, length=2.0)
    f = W.uniform_fields(m, mean_u=(0.0, 0.0, 0.0), mean_omega=2.0, rey=(0.5,) * 3 + (0,) * 3)
    mo = W.model_constants()
    g = O.Grid(m, f, mo)
    E = O.Ensemble(g, W.init_desc(ppe=2, src_x=1.0, src_y=0.0))
    k, om, nu = 0.75, 2.0, mo["nu"]
    eps = om * (k + nu * 36.0 * om)
    assert abs(E.tm(0) - max(k / eps, 6.0 * math.sqrt(nu / eps))) < 1e-15
    # with a mean velocity: first branch C_s (r0^2/eps)^(1/3) + C_t d / U_c at the centroid
    f2 = W.uniform_fields(m, mean_u=(3.0, 4.0, 0.0), mean_omega=2.0, rey=(0.5,) * 3 + (0,) * 3)
    g2 = O.Grid(m, f2, mo)
    E2 = O.Ensemble(g2, W.init_desc(ppe=2, src_x=1.0, src_y=0.0, src_r=0.05))
    fr = g2.export()["frame"]
    for e in (0, 7, 20):
        c = fr[e].reshape(3, 2).mean(0)
        d = math.hypot(c[0] - 1.0, c[1])
        first = 0.02 * (0.05 ** 2 / eps) ** (1 / 3) + 0.7 * d / 5.0
        assert abs(E2.tm(e) - min(first, max(k / eps, 6.0 * math.sqrt(nu / eps)))) < 1e-14


# ------------------------------------------------------------------- statistics

def test_statistics_partition_of_unity_and_realizability():
    m, f, mo, ini = W.channel_small()
    g = O.Grid(m, f, mo)
    E = O.Ensemble(g, ini)
    E.step(1e-3, 2)
    st = E.stats()
    s = E.export()
    w = s["w"]
    q = np.column_stack([s["u"], s["om"], s["psi"]])
    # shape functions sum to one in every element: nodal weights add up to the total
    assert abs(st[:, 0].sum() - w.sum()) < 1e-12 * w.sum()
    for j in range(5):
        assert abs((st[:, 0] * st[:, 1 + j]).sum() - (w * q[:, j]).sum()) < 1e-11 * np.abs(w * q[:, j]).sum()
    R11, R22, R33, R12 = st[:, 6], st[:, 7], st[:, 8], st[:, 9]
    assert (R11 >= 0).all() and (R22 >= 0).all() and (R33 >= 0).all() and (st[:, 12] >= 0).all()
    assert (R12 ** 2 <= R11 * R22 * (1 + 1e-12) + 1e-30).all()


def test_statistics_of_constant_quantities_and_brute_force():
    m = box(4, 4, length=2.0)
    f = W.uniform_fields(m, mean_u=(0.25, 0.0, 0.0))
    g = O.Grid(m, f, W.model_constants())
    E = O.Ensemble(g, W.init_desc(ppe=12, u_sigma=0.0, src_r=0.0))
    st = E.stats()
    assert np.allclose(st[:, 1], 0.25, rtol=1e-15, atol=0) and np.all(st[:, 2] == 0)
    assert np.all(np.abs(st[:, 6]) < 1e-30)
    # brute force: every node from every particle with the node's shape-function value
    E.step(0.01)
    st = E.stats()
    s = E.export()
    lam = np.array([g.bary(e, x, y) for e, x, y in zip(s["elem"], s["x"], s["y"])])
    q = np.column_stack([s["u"], s["om"], s["psi"]])
    for nd in range(m.n_nodes):
        wl = np.zeros(len(s["x"]))
        for k in range(3):
            hit = m.tri[s["elem"], k] == nd
            wl[hit] = s["w"][hit] * lam[hit, k]
        W_ = wl.sum()
        M = (wl[:, None] * q).sum(0) / W_
        d = q - M
        assert abs(st[nd, 0] - W_) < 1e-13 * W_
        assert np.allclose(st[nd, 1:6], M, rtol=1e-12, atol=1e-15)
        assert abs(st[nd, 6] - (wl * d[:, 0] ** 2).sum() / W_) < 1e-13
        assert abs(st[nd, 9] - (wl * d[:, 0] * d[:, 1]).sum() / W_) < 1e-13
        assert abs(st[nd, 12] - (wl * d[:, 4] ** 2).sum() / W_) < 1e-13


# ------------------------------------------------------------------- number control

def _bins_of(state, sel, bins):
    return O.bin_element(state["u"][sel], state["pid"][sel], bins, 2)


def test_control_conserves_and_bounds_counts():
    """Per element: splitting halves a donor's weight and adds an identical particle;
    merging joins two particles of one bin into their weighted average.  Total weight
    and the weighted sums of U, omega and psi are conserved in every element and every
    velocity bin; counts move into [n_min, n_max] as far as the rules allow."""
    m = W.channel_mesh(10, 12, stretch=1.1 ** 5, seed=3)
    f = W.channel_fields(m)
    mo = W.model_constants()
    g = O.Grid(m, f, mo)
    E = O.Ensemble(g, W.init_desc(ppe=40, bins=(4, 2, 2), src_x=3.0, src_r=0.9, src_continuous=0))
    E.step(2e-3, 3)
    E.control(41, 10000)            # unequal weights before the merges below
    E.step(2e-3, 1)
    pre = E.export()
    assert len(np.unique(pre["w"])) > 1
    cnt = np.bincount(pre["elem"], minlength=m.n_elems)
    n_min, n_max = 41, 41
    assert (cnt < n_min).any() and (cnt > n_max).any()
    rep = E.control(n_min, n_max)
    post = E.export()
    cnt2 = np.bincount(post["elem"], minlength=m.n_elems)
    for e in range(m.n_elems):
        n = cnt[e]
        if n == 0:
            assert cnt2[e] == 0
        elif n < n_min:
            assert cnt2[e] == n + min(n_min - n, n)
        elif n > n_max:
            assert n_max <= cnt2[e] < n
        else:
            assert cnt2[e] == n
    assert rep["live"] == len(post["x"])
    assert len(np.unique(post["pid"])) == len(post["pid"])
    new = post["pid"][post["pid"] >= pre["pid"].max() + 1]
    assert np.array_equal(np.sort(new), np.arange(pre["pid"].max() + 1, pre["pid"].max() + 1 + rep["cloned"], dtype=np.uint64))
    # conservation per element and per bin (bins of the pre-control canonical order)
    post_by_pid = {int(p): i for i, p in enumerate(post["pid"])}
    for e in range(m.n_elems):
        sa = np.nonzero(pre["elem"] == e)[0]
        sb = np.nonzero(post["elem"] == e)[0]
        for q in ("w",):
            assert abs(pre[q][sa].sum() - post[q][sb].sum()) <= 1e-14 * pre[q][sa].sum()
        for q in ("psi", "om"):
            a = (pre["w"][sa] * pre[q][sa]).sum()
            b = (post["w"][sb] * post[q][sb]).sum()
            assert abs(a - b) <= 1e-13 * max(1.0, abs(a))
        a = (pre["w"][sa, None] * pre["u"][sa]).sum(0)
        b = (post["w"][sb, None] * post["u"][sb]).sum(0)
        assert np.allclose(a, b, rtol=1e-13, atol=1e-13)
        if cnt[e] > n_max:
            cp, pos, bb = _bins_of(pre, sa, (4, 2, 2))
            for k in range(cp):
                members = sa[bb == k]
                wsum_pre = pre["w"][members].sum()
                psi_pre = (pre["w"][members] * pre["psi"][members]).sum()
                surv = [post_by_pid[int(p)] for p in pre["pid"][members] if int(p) in post_by_pid]
                assert abs(post["w"][surv].sum() - wsum_pre) <= 1e-14 * wsum_pre
                assert abs((post["w"][surv] * post["psi"][surv]).sum() - psi_pre) <= 1e-13 * max(1, psi_pre)
    assert rep["merged"] > 0 and rep["cloned"] > 0


def test_control_clones_identical_and_weights_dyadic():
    m = box(4, 4, length=2.0)
    f = W.uniform_fields(m, mean_u=(0.2, 0.0, 0.0))
    g = O.Grid(m, f, W.model_constants())
    E = O.Ensemble(g, W.init_desc(ppe=5, src_r=0.0))
    pre = E.export()
    rep = E.control(8, 20)
    post = E.export()
    assert rep["cloned"] == 3 * m.n_elems
    n0 = len(pre["x"])
    clones = post["pid"] >= n0
    donors_w = post["w"][~clones]
    assert set(np.unique(post["w"]).tolist()) <= {0.5, 1.0}
    assert (donors_w == 0.5).sum() == clones.sum()
    for i in np.nonzero(clones)[0]:
        same = (post["x"] == post["x"][i]) & (post["y"] == post["y"][i]) & ~clones
        assert same.sum() == 1
        j = np.nonzero(same)[0][0]
        assert np.array_equal(post["u"][i], post["u"][j]) and post["w"][j] == 0.5
