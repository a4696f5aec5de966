"""GPU parity: the HIP path (through the C ABI) against the oracle on the same seeded
inputs, element by element and node by node."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_1006_0532_amd import workloads as W
from tests.common import box
from tests.parity import compare_states, compare_stats

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "a GPU is required"
    from paper_1006_0532_amd import pdfgpu
    pdfgpu.load()
    return pdfgpu


def _pair(gpu, mesh, fields, model, init, capacity=0):
    og = O.Grid(mesh, fields, model)
    oe = O.Ensemble(og, init)
    gg = gpu.Grid(mesh, fields, model)
    ge = gpu.Ensemble(gg, init, capacity=capacity)
    return og, oe, gg, ge


def _skip_nodes(mesh, excl):
    return set(mesh.tri[list(excl)].ravel().tolist()) if excl else set()


def _length(mesh):
    return mesh.period_x if mesh.period_x > 0 else float(np.ptp(mesh.xy[:, 0]))


def test_init_parity(gpu):
    _say("test_init_parity: channel_small")
    mesh, f, mo, ini = W.channel_small()
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    g, r = ge.export(), oe.export()
    assert np.array_equal(g["elem"], r["elem"])
    compare_states(g, r, frame, _length(mesh))
    compare_stats(ge.stats(), oe.stats())


def test_stats_mask_selects_columns(gpu):
    """pdf_stats with a stat_mask returns the selected columns of the full statistics in
    ascending order, bit for bit, to host and to device memory; empty and out-of-range
    masks are argument errors."""
    import torch
    _say("test_stats_mask_selects_columns")
    mesh, f, mo, ini = W.channel_small(nx=12, ny=10)
    ge = gpu.Ensemble(gpu.Grid(mesh, f, mo), ini)
    ge.step(1e-3, 2)
    full = ge.stats()
    assert full.shape == (mesh.n_nodes, gpu.PDF_NSTAT)
    rng = np.random.default_rng(5)
    masks = [1, 1 << 12, 0b1010101, gpu.PDF_STATS_ALL] + [int(m) for m in rng.integers(1, 1 << 13, 4)]
    for m in masks:
        cols = [j for j in range(gpu.PDF_NSTAT) if (m >> j) & 1]
        host = ge.stats(mask=m)
        assert np.array_equal(host, full[:, cols], equal_nan=True), m
        dev = torch.full((mesh.n_nodes, len(cols)), -7.0, dtype=torch.float64, device="cuda")
        ge.stats_device(dev.data_ptr(), mask=m)
        ge.sync()
        assert np.array_equal(dev.cpu().numpy(), full[:, cols], equal_nan=True), m
    for bad in (0, 1 << 13, gpu.PDF_STATS_ALL | (1 << 20)):
        with pytest.raises(gpu.PdfError):
            ge.stats(mask=bad)


@pytest.mark.parametrize("steps", [1, 20])
def test_channel_small_step_parity(gpu, steps):
    """Full step (advance, track, group, bin, mix, statistics) every step, 2e5 particles."""
    _say(f"test_channel_small_step_parity: {steps} steps")
    mesh, f, mo, ini = W.channel_small()
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    excl = set()
    for n in range(steps):
        oe.step(1e-3)
        ge.step(1e-3)
        rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
        compare_stats(ge.stats(), oe.stats(), _skip_nodes(mesh, excl))
    assert len(excl) <= 4
    assert ge.counters() == oe.counters()


def test_control_parity(gpu):
    """Number control after a few steps: splits and same-bin merges match the oracle."""
    _say("test_control_parity")
    mesh = W.channel_mesh(20, 24, stretch=1.1 ** 8, seed=21)
    f = W.channel_fields(mesh)
    mo = W.model_constants()
    ini = W.init_desc(ppe=40, bins=(4, 2, 2), src_x=3.0, src_r=0.4)
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    excl = set()
    for n in range(4):
        oe.step(2e-3)
        ge.step(2e-3)
        ro = oe.control(38, 42)
        rg = ge.control(38, 42)
        assert ro == {k: rg[k] for k in ro}, (ro, rg)
        assert rg["cloned"] > 0 and rg["merged"] > 0
        rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
    oe.step(2e-3)
    ge.step(2e-3)
    compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
    compare_stats(ge.stats(), oe.stats(), _skip_nodes(mesh, excl))


def test_control_sets_the_element_tiers(gpu):
    """200 per element merged down to at most 128 by control: the element pass then runs a
    first wavefront tier of two particles per lane (n <= 128) and the set-up tier of five
    for the elements the next step pushes above; both tiers are populated every step."""
    _say("test_control_sets_the_element_tiers")
    mesh = W.channel_mesh(10, 12, stretch=1.1 ** 8, seed=31)
    f = W.channel_fields(mesh)
    mo = W.model_constants()
    ini = W.init_desc(ppe=200, bins=(4, 2, 2), src_x=3.0, src_r=0.4)
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    excl = set()
    for n in range(4):
        oe.step(5e-3)
        ge.step(5e-3)
        ref = oe.export()
        rep, excl = compare_states(ge.export(), ref, frame, _length(mesh), excl)
        counts = np.bincount(ref["elem"], minlength=mesh.n_elems)
        if n > 0:
            assert (counts > 128).any() and (counts <= 128).any(), counts
        ro = oe.control(100, 128)
        rg = ge.control(100, 128)
        assert ro == {k: rg[k] for k in ro}, (ro, rg)
    oe.step(5e-3)
    ge.step(5e-3)
    rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
    compare_stats(ge.stats(), oe.stats(), _skip_nodes(mesh, excl))
    assert len(excl) <= 4


def _adversarial_velocities(st, seed=5):
    """Velocity sets that stress the element sort, by element id mod 5: all equal (ties
    by pid at every level); U1 of both signed zeros and the smallest subnormals; a
    Gaussian with one outlier a million times larger; U1 a run of consecutive doubles
    above 1; U1 half 0, half the smallest subnormal (a span whose reciprocal overflows)."""
    rng = np.random.default_rng(seed)
    u = st["u"].copy()
    tiny = np.nextafter(0.0, 1.0)
    for e in np.unique(st["elem"]):
        idx = np.nonzero(st["elem"] == e)[0]
        n = len(idx)
        kind = int(e) % 5
        if kind == 0:
            u[idx] = (0.25, -0.125, 0.5)
        elif kind == 1:
            u[idx, 0] = np.resize([-0.0, 0.0, tiny, -tiny, 1e-300, -1e-300], n)
            u[idx, 1:] = rng.normal(0.0, 0.05, (n, 2))
        elif kind == 2:
            u[idx] = rng.normal(0.0, 0.05, (n, 3))
            u[idx[n // 2], 0] = 1e6
        elif kind == 3:
            v = 1.0
            for j in rng.permutation(n):
                u[idx[j], 0] = v
                v = np.nextafter(v, 2.0)
            u[idx, 1] = np.resize([0.1, 0.2], n)
        else:
            u[idx, 0] = np.where(np.arange(n) % 2 == 0, 0.0, tiny)
    return u


@pytest.mark.parametrize("conditioning", [0, 1])
def test_element_sort_on_adversarial_velocities(gpu, conditioning):
    """Bins seen through number control (merges pair particles of one bin): imported
    states whose velocities tie, straddle zero, hold an outlier or span a few ulps give
    the oracle's merges, under the sort-and-divide bins and under Fox's projection."""
    _say(f"test_element_sort_on_adversarial_velocities conditioning={conditioning}")
    mesh = box(4, 4, length=2.0, jitter=0.1)
    f = W.uniform_fields(mesh, mean_u=(0.3, 0.1, 0.0), mean_omega=4.0)
    mo = W.model_constants()
    ini = W.init_desc(ppe=100, bins=(4, 2, 2), src_x=1.0, src_r=0.4, conditioning=conditioning)
    og = O.Grid(mesh, f, mo)
    st = O.Ensemble(og, ini).export()
    st["u"] = _adversarial_velocities(st)
    oe = O.Ensemble(og, ini)
    oe.import_state(st, step=0, next_pid=len(st["x"]))
    gg = gpu.Grid(mesh, f, mo)
    ge = gpu.Ensemble(gg, ini, capacity=200 * mesh.n_elems)
    ge.import_state(st, step=0, next_pid=len(st["x"]))
    frame = og.export()["frame"]
    ro, rg = oe.control(40, 60), ge.control(40, 60)
    assert ro == {k: rg[k] for k in ro}, (ro, rg)
    assert rg["merged"] > 0
    rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh))
    assert not excl


def test_walls_slip_and_multistep_walks(gpu):
    """Tiny jittered box with large steps: multi-element walks, free-slip reflections,
    periodic seam; element ids must equal the oracle's."""
    _say("test_walls_slip_and_multistep_walks")
    mesh = box(5, 4, length=2.5, jitter=0.2, seed=5)
    f = W.uniform_fields(mesh, mean_u=(1.0, 0.5, 0.0), mean_omega=3.0)
    mo = W.model_constants(nu=1e-3)
    ini = W.init_desc(ppe=200, u_sigma=0.4, src_x=1.0, src_r=0.3, bins=(3, 2, 1))
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    excl = set()
    for n in range(5):
        oe.step(0.05)
        ge.step(0.05)
        rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
    c = ge.counters()
    assert c["reflections"] > 0 and c["walk_steps"] > 0
    assert c == oe.counters()


def test_most_walks_reach_a_wall(gpu):
    """A strong wall-normal mean flow and large steps send more than 65 536 of 1.9e5
    particles across the free-slip top wall in one step, so the list of walks that reach a
    wall (advanced again by the full loop) is longer than one pass of that kernel's grid;
    states after every step, statistics and counters equal the oracle's."""
    _say("test_most_walks_reach_a_wall")
    mesh = box(20, 24, length=2.0, jitter=0.1, seed=17, bottom=W.EDGE_WALL, top=W.EDGE_SLIP)
    f = W.uniform_fields(mesh, mean_u=(0.3, 2.5, 0.0), mean_omega=2.0)
    mo = W.model_constants(nu=1e-4)
    ini = W.init_desc(ppe=200, u_sigma=0.3, src_x=1.0, src_r=0.3, bins=(3, 2, 1), seed=0x3A11)
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    excl = set()
    for dt in (0.35, 0.02, 0.02, 0.3):
        before = ge.counters()
        oe.step(dt)
        ge.step(dt)
        c = ge.counters()
        assert c == oe.counters()
        refl = c["reflections"] - before["reflections"]
        if dt > 0.1:
            assert refl > 65536, (dt, refl)
        rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
        _say(f"  dt {dt}: {refl} reflections; {rep}")
    skip = set(mesh.tri[list(excl)].ravel().tolist()) if excl else set()
    compare_stats(ge.stats(), oe.stats(), skip)


def test_no_slip_events(gpu):
    """Near-wall particles: trajectories (a) and (b) with Gamma frequency resampling."""
    _say("test_no_slip_events")
    mesh = W.channel_mesh(12, 16, length=2.0, stretch=1.1 ** 7, seed=8)
    f = W.channel_fields(mesh)
    # nu dt = 1e-7: explicit Euler of Eq. (27) stays stable at <omega> = 50 (|1 + G dt| < 1)
    mo = W.model_constants(nu=1e-4)
    ini = W.init_desc(ppe=60, src_r=0.0)
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    excl = set()
    for n in range(6):
        oe.step(1e-3)
        ge.step(1e-3)
        rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
    c = ge.counters()
    assert c["wall_a"] > 0 and c["wall_b"] > 0
    assert c == oe.counters()


def test_large_elements_use_global_scratch(gpu):
    """Elements above the on-chip limit take the global-memory path of the element pass."""
    _say("test_large_elements_use_global_scratch")
    mesh = box(4, 2, length=2.0, jitter=0.0)     # periodic meshes need elements < period/2 wide
    f = W.uniform_fields(mesh, mean_u=(0.2, 0.0, 0.0))
    mo = W.model_constants()
    ini = W.init_desc(ppe=2200, bins=(5, 5, 5), src_x=1.0, src_r=0.5)
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    for n in range(2):
        oe.step(1e-3)
        ge.step(1e-3)
        compare_states(ge.export(), oe.export(), frame, _length(mesh))
    compare_stats(ge.stats(), oe.stats())


def test_determinism_and_resume(gpu):
    """Bitwise-identical reruns; 6 steps == 3 + export/import + 3."""
    _say("test_determinism_and_resume")
    mesh, f, mo, ini = W.channel_small(nx=16, ny=20)
    gg = gpu.Grid(mesh, f, mo)
    a = gpu.Ensemble(gg, ini)
    a.step(1e-3, 6)
    b = gpu.Ensemble(gg, ini)
    b.step(1e-3, 6)
    sa, sb = a.export(), b.export()
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(a.stats(), b.stats(), equal_nan=True)
    c = gpu.Ensemble(gg, ini)
    c.step(1e-3, 3)
    snap = c.export()
    d = gpu.Ensemble(gg, ini)
    d.import_state(snap, step=3, next_pid=len(snap["x"]))
    d.step(1e-3, 3)
    sd = d.export()
    for k in sa:
        assert np.array_equal(sa[k], sd[k]), k


def test_error_paths(gpu):
    """A particle outside the domain is reported as lost; bad arguments are rejected."""
    _say("test_error_paths")
    mesh, f, mo, ini = W.channel_small(nx=8, ny=10)
    gg = gpu.Grid(mesh, f, mo)
    e = gpu.Ensemble(gg, ini)
    st = e.export()
    st["y"][0] = 50.0          # far outside the channel: more than four reflections needed
    e.import_state(st, step=0, next_pid=len(st["x"]))
    e.step(1e-3)
    with pytest.raises(gpu.PdfError) as ex:
        e.sync()
    assert ex.value.status == -6
    e2 = gpu.Ensemble(gg, ini)
    with pytest.raises(gpu.PdfError):
        e2.control(10, 5)
    with pytest.raises(gpu.PdfError):
        e2.step(-1.0)
    bad = W.Mesh(mesh.xy, mesh.tri[:, ::-1].copy(), mesh.edge_kind, mesh.period_x)
    with pytest.raises(gpu.PdfError) as ex:
        gpu.Grid(bad, f, mo)
    assert ex.value.status == -4


def test_capacity_error_keeps_the_state_consistent(gpu):
    """Number control asks for more clones than the capacity holds: PDF_E_CAPACITY, the
    clones that fit are written (a prefix of the clone order, contiguous new pids), none
    past the capacity, the donors of the missing ones keep their weight, so the total
    weight and the weighted sums are unchanged, and the live count is the slots used."""
    _say("test_capacity_error_keeps_the_state_consistent")
    mesh, f, mo, ini = W.channel_small(nx=8, ny=10)
    n0 = mesh.n_elems * ini["ppe"]
    cap = n0 + 800
    e = gpu.Ensemble(gpu.Grid(mesh, f, mo), ini, capacity=cap)
    e.step(1e-3)
    before = e.export()
    rep = e.control(60, 80, check=False)
    assert e.last_status == -5
    assert rep["cloned"] == 800 and rep["live"] == cap, rep
    assert e.count(check=False) == cap and e.last_status == -5
    after = e.export(check=False)
    assert e.last_status == -5
    assert len(after["pid"]) == cap
    assert len(np.unique(after["pid"])) == cap
    new = after["pid"] >= n0
    assert new.sum() == 800 and np.array_equal(np.sort(after["pid"][new]), np.arange(n0, n0 + 800))
    assert np.array_equal(after["pid"][~new], before["pid"])
    for k in ("w",):
        assert abs(after[k].sum() - before[k].sum()) <= 1e-12 * before[k].sum()
    wu = lambda st: (st["w"][:, None] * st["u"]).sum(0)
    assert np.abs(wu(after) - wu(before)).max() <= 1e-12 * np.abs(wu(before)).max()
    # every clone is a half-weight copy of a donor that now has half its weight
    halved = after["w"][~new] < before["w"]
    assert halved.sum() == 800 and np.all(after["w"][new] == 0.5)
    with pytest.raises(gpu.PdfError) as ex:
        e.sync()
    assert ex.value.status == -5


def test_nonfinite_inputs_are_rejected(gpu):
    """A NaN nodal field is refused by pdf_grid_create, and a NaN particle velocity by
    pdf_particles_import, both with PDF_E_NONFINITE."""
    _say("test_nonfinite_inputs_are_rejected")
    mesh, f, mo, ini = W.channel_small(nx=8, ny=10)
    for name in ("mean_u", "mean_omega", "grad_p", "wp", "rey"):
        bad = W.Fields(*[a.copy() for a in f.as_tuple()])
        arr = getattr(bad, name)
        arr.reshape(-1)[7] = np.nan
        with pytest.raises(gpu.PdfError) as ex:
            gpu.Grid(mesh, bad, mo)
        assert ex.value.status == -7, name
    e = gpu.Ensemble(gpu.Grid(mesh, f, mo), ini)
    st = e.export()
    st["u"][3, 1] = np.inf
    with pytest.raises(gpu.PdfError) as ex:
        e.import_state(st, step=0, next_pid=len(st["x"]))
    assert ex.value.status == -7


def test_elements_above_the_wavefront_limit(gpu):
    """An ensemble seeded with 40 per element holds at most 64 per wavefront; importing
    600 per element sends every element to the workgroup kernel's on-chip path."""
    _say("test_elements_above_the_wavefront_limit")
    mesh = box(4, 4, length=2.0, jitter=0.1)
    f = W.uniform_fields(mesh, mean_u=(0.3, 0.1, 0.0), mean_omega=4.0)
    mo = W.model_constants()
    big = W.init_desc(ppe=600, bins=(4, 4, 2), src_x=1.0, src_r=0.4)
    og = O.Grid(mesh, f, mo)
    oe = O.Ensemble(og, big)
    gg = gpu.Grid(mesh, f, mo)
    ge = gpu.Ensemble(gg, W.init_desc(ppe=40, bins=(4, 4, 2), src_x=1.0, src_r=0.4),
                      capacity=700 * mesh.n_elems)
    st = oe.export()
    ge.import_state(st, step=0, next_pid=len(st["x"]))
    frame = og.export()["frame"]
    compare_stats(ge.stats(), oe.stats())
    excl = set()
    for n in range(3):
        oe.step(1e-3)
        ge.step(1e-3)
        rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
    compare_stats(ge.stats(), oe.stats(), _skip_nodes(mesh, excl))
    ro, rg = oe.control(500, 550), ge.control(500, 550)
    assert ro == {k: rg[k] for k in ro}
    compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)


def test_one_particle_bins_and_many_bins(gpu):
    """min_per_bin = 1 (workgroup kernel) and a 5x5x5 request (many groups per level)."""
    _say("test_one_particle_bins_and_many_bins")
    mesh = box(6, 6, length=2.0)
    f = W.uniform_fields(mesh, mean_u=(0.3, 0.1, 0.0), mean_omega=4.0)
    mo = W.model_constants()
    for bins, m in [((5, 5, 5), 1), ((5, 5, 5), 2), ((8, 4, 4), 2)]:
        ini = W.init_desc(ppe=150, bins=bins, min_per_bin=m, src_x=1.0, src_r=0.4)
        og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
        frame = og.export()["frame"]
        excl = set()
        for n in range(3):
            oe.step(2e-3)
            ge.step(2e-3)
            rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
        compare_stats(ge.stats(), oe.stats(), _skip_nodes(mesh, excl))


@pytest.mark.slow
def test_channel_large_first_steps(gpu):
    """The benchmark workload at full size (400 000 triangles, 8e7 particles), in the
    benchmark's launch configuration (capacity 1.3 n0 + 1024, step + control(150, 250)):
    control reports every step, every particle and every node after 3 steps."""
    _say("test_channel_large_first_steps: channel 400x500, 200 per element")
    mesh = W.channel_mesh(400, 500)
    f = W.channel_fields(mesh)
    mo = W.model_constants()
    ini = W.init_desc(ppe=200, bins=(4, 2, 2))
    n0 = mesh.n_elems * 200
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini, capacity=int(1.3 * n0) + 1024)
    assert ge.count() == oe.count() == n0
    for n in range(3):
        oe.step(2e-4)
        ge.step(2e-4)
        ro, rg = oe.control(150, 250), ge.control(150, 250)
        _say(f"  step {n + 1}: {rg}")
        assert ro == {k: rg[k] for k in ro}, (ro, rg)
    frame = og.export()["frame"]
    rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh))
    _say(f"  particles: {rep}")
    assert len(excl) <= 8
    compare_stats(ge.stats(), oe.stats(), _skip_nodes(mesh, excl))
    assert ge.counters() == oe.counters()


def test_cavity_small_parity(gpu):
    """Street canyon (cavity corners, no-slip street level, free-slip top, periodic seam),
    10 steps with number control every other step."""
    _say("test_cavity_small_parity")
    mesh, f, mo, ini = W.cavity_small()
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    excl = set()
    for n in range(10):
        oe.step(1e-3)
        ge.step(1e-3)
        if n % 2 == 1:
            ro, rg = oe.control(40, 60), ge.control(40, 60)
            assert ro == {k: rg[k] for k in ro}, (ro, rg)
        rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
    compare_stats(ge.stats(), oe.stats(), _skip_nodes(mesh, excl))
    c = ge.counters()
    assert c["wall_a"] > 0 and c["reflections"] > 0 and c["source_hits"] > 0
    assert c == oe.counters()


@pytest.mark.parametrize("U", [(-1.0, 1.0), (1.0, 1.0)])
def test_concave_fallback_parity(gpu, U):
    """Concave-boundary fall-back of Sec. 3.6 (Fig. 2): a small street canyon with one
    re-entrant corner on the periodic seam, a frozen velocity that carries particles
    round a corner every step and long steps; the fall-back fires dozens of times a step
    (across the seam for U = (-1, 1)) and the GPU agrees with the oracle particle by
    particle, in its counters and in the statistics.  The fields keep C0 eps > 0: with it
    clamped to zero, every particle that left a no-slip wall at U = 0 would take the same
    deterministic velocity up to the last bit, and the velocity sorts of the binning would
    order such near-ties by rounding, which the two sides need not share."""
    _say(f"test_concave_fallback_parity U={U}")
    from tests.test_oracle_fallback import canyon_on_seam
    mesh = canyon_on_seam()
    f = W.uniform_fields(mesh, mean_u=(U[0], U[1], 0.0), mean_omega=1.0)
    mo = W.model_constants(nu=1.0e-4)
    ini = W.init_desc(ppe=300, u_sigma=0.02, src_x=0.5, src_y=0.5, src_r=0.1)
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    excl = set()
    for n in range(4):
        oe.step(0.05)
        ge.step(0.05)
        rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
    compare_stats(ge.stats(), oe.stats(), _skip_nodes(mesh, excl))
    c = ge.counters()
    assert c == oe.counters()
    assert c["fallbacks"] > 50 and c["wall_a"] > 0, c


@pytest.mark.parametrize("feed_rey", [False, True])
def test_statistics_feedback_parity(gpu, feed_rey):
    """Redistribution test of Sec. 3.7: the fed-back mean (alpha = 0.5) and optionally the
    fed-back Reynolds stresses drive the next step; number control every step."""
    _say(f"test_statistics_feedback_parity feed_rey={feed_rey}")
    mesh, f, mo, ini = W.redistribution_test(ppe=60)
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    oe.feedback(0.5, feed_rey)
    ge.set_feedback(True, 0.5, feed_rey)
    excl = set()
    for n in range(8):
        oe.step(0.01)
        ge.step(0.01)
        ro, rg = oe.control(10, 100), ge.control(10, 100)
        assert ro == {k: rg[k] for k in ro}, (ro, rg)
        oe.feedback(0.5, feed_rey)
        rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
    compare_stats(ge.stats(), oe.stats(), _skip_nodes(mesh, excl))
    assert len(excl) <= 4


def test_feedback_in_graph_replay_is_bitwise_eager(gpu):
    _say("test_feedback_in_graph_replay_is_bitwise_eager")
    mesh, f, mo, ini = W.redistribution_test(nx=10, ny=12, ppe=60)
    gg = gpu.Grid(mesh, f, mo)
    a, b = gpu.Ensemble(gg, ini), gpu.Ensemble(gg, ini)
    for e in (a, b):
        e.set_feedback(True, 0.5, True)
    b.set_options(use_graph=1)
    for chunk in (2, 3, 4):
        a.step(0.01, chunk)
        b.step(0.01, chunk)
        sa, sb = a.export(), b.export()
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), (chunk, k)
        assert np.array_equal(a.stats(), b.stats(), equal_nan=True)
    # the grid itself is untouched: a fresh ensemble without feedback equals the oracle's set-up
    c = gpu.Ensemble(gg, ini)
    og = O.Grid(mesh, f, mo)
    oc = O.Ensemble(og, ini)
    c.step(0.01)
    oc.step(0.01)
    compare_states(c.export(), oc.export(), og.export()["frame"], _length(mesh))


def test_cfl_time_step(gpu):
    """Eq. (26) from the GPU statistics: equal to the oracle's on the channel after some
    steps, and per problem in a batched ensemble."""
    _say("test_cfl_time_step")
    mesh, f, mo, ini = W.channel_small(nx=20, ny=24)
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    for n in range(3):
        oe.step(1e-3)
        ge.step(1e-3)
    a, b = ge.cfl_dt(0.7), oe.cfl_dt(0.7)
    assert b > 0 and abs(a - b) <= 1e-12 * b, (a, b)
    m2 = box(6, 6, length=2.0)
    f2 = W.uniform_fields(m2, mean_u=(0.5, 0.2, 0.0), mean_omega=2.0)
    g2 = gpu.Grid(m2, f2, mo)
    ini2 = W.init_desc(ppe=30, bins=(2, 2, 1), src_x=1.0, src_r=0.3, seed=77)
    bat = gpu.Ensemble([gg, g2], [ini, ini2])
    bat.step([1e-3, 2e-3], 2)
    for p, (m, ff, d, dt) in enumerate(((mesh, f, ini, 1e-3), (m2, f2, ini2, 2e-3))):
        dd = dict(d)
        dd["seed"] = int(d["seed"]) ^ (p << 32)
        o = O.Ensemble(O.Grid(m, ff, mo), dd)
        o.step(dt)
        o.step(dt)
        a, b = bat.cfl_dt(0.7, problem=p), o.cfl_dt(0.7)
        assert abs(a - b) <= 1e-12 * b, (p, a, b)


def test_element_estimator_parity(gpu):
    """Second estimator of Sec. 3.3 (element means averaged to the nodes, element-averaged
    fields), with number control and statistics feedback."""
    _say("test_element_estimator_parity")
    mesh = W.channel_mesh(20, 24, stretch=1.1 ** 8, seed=21)
    f = W.channel_fields(mesh)
    mo = W.model_constants()
    ini = W.init_desc(ppe=40, bins=(4, 2, 2), src_x=3.0, src_r=0.4, estimator=1)
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    compare_stats(ge.stats(), oe.stats())
    ge.set_feedback(True, 1.0, False)
    oe.feedback(1.0, False)
    excl = set()
    for n in range(6):
        oe.step(2e-3)
        ge.step(2e-3)
        ro, rg = oe.control(38, 42), ge.control(38, 42)
        assert ro == {k: rg[k] for k in ro}, (ro, rg)
        oe.feedback(1.0, False)
        rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
    compare_stats(ge.stats(), oe.stats(), _skip_nodes(mesh, excl))
    assert ge.cfl_dt(0.7) == pytest.approx(oe.cfl_dt(0.7), rel=1e-12)


@pytest.mark.parametrize("ppe,n_min,dt", [(20, 10, 0.02), (4, 2, 0.05)])
def test_redistribution_parity(gpu, ppe, n_min, dt):
    """Particle redistribution of App. B after every step of the Sec. 3.7 test (stretched
    strip, fed-back mean with alpha = 0.5): the same moves as the oracle, hence the same
    particles in every element; the second case empties elements (centroid placement)."""
    _say(f"test_redistribution_parity ppe={ppe} n_min={n_min}")
    mesh, f, mo, ini = W.redistribution_test(ppe=ppe)
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    oe.feedback(0.5, False)
    ge.set_feedback(True, 0.5, False)
    excl = set()
    total = 0
    for n in range(10):
        oe.step(dt)
        ge.step(dt)
        mo_, mg = oe.redistribute(n_min), ge.redistribute(n_min)
        assert mo_ == mg, (n, mo_, mg)
        total += mg
        if mg:
            with pytest.raises(gpu.PdfError):
                ge.redistribute(n_min)
        oe.feedback(0.5, False)
        rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
        assert not excl, n
    assert total > 100
    oe.step(dt)
    ge.step(dt)
    compare_states(ge.export(), oe.export(), frame, _length(mesh))
    compare_stats(ge.stats(), oe.stats())


def test_redistribution_batched(gpu):
    """Per-problem redistribution in a batched ensemble: every problem, then one problem
    only, each equal to its own oracle ensemble (key seed ^ problem << 32)."""
    _say("test_redistribution_batched")
    mo = W.model_constants(nu=0.0)
    cases = []
    for p, (nx, ny, ppe) in enumerate(((8, 12, 6), (10, 8, 5))):
        mesh, f, mo, ini = W.redistribution_test(nx=nx, ny=ny, ppe=ppe, seed=100 + p)
        cases.append((mesh, f, ini))
    grids = [gpu.Grid(m, f, mo) for m, f, _ in cases]
    bat = gpu.Ensemble(grids, [c[2] for c in cases])
    oes = []
    for p, (m, f, d) in enumerate(cases):
        dd = dict(d)
        dd["seed"] = int(d["seed"]) ^ (p << 32)
        oes.append((O.Ensemble(O.Grid(m, f, mo), dd), O.Grid(m, f, mo).export()["frame"], m))
    for n in range(4):
        bat.step([0.05, 0.05])
        for o, _, _ in oes:
            o.step(0.05)
        if n % 2 == 0:
            mg = bat.redistribute(3)
            mo_ = sum(o.redistribute(3) for o, _, _ in oes)
        else:
            mg = bat.redistribute(3, problem=1)
            mo_ = oes[1][0].redistribute(3)
        assert mg == mo_ and mg > 0, (n, mg, mo_)
        for p, (o, frame, m) in enumerate(oes):
            rep, excl = compare_states(bat.export(problem=p), o.export(), frame, _length(m))
            assert not excl


def test_redistribution_skewed_counts_parity(gpu):
    """App. B on element counts spread over many levels on both sides (empty elements,
    elements of more than 100 particles whose departures span several 32-slot words):
    the same moves as the oracle's serial loop, for two thresholds in a row."""
    _say("test_redistribution_skewed_counts_parity")
    mesh = box(6, 6, length=2.0, seed=23)
    f = W.uniform_fields(mesh, mean_u=(0.2, 0.0, 0.0), mean_omega=1.0)
    mo = W.model_constants(nu=1.0e-4)
    ini = W.init_desc(ppe=30, u_sigma=0.3, src_r=0.0, bins=(2, 2, 1), seed=0xABB)
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    st = oe.export()
    n, ne = len(st["x"]), mesh.n_elems
    rng = np.random.default_rng(41)
    wgt = np.array([(e % 7) ** 3 for e in range(ne)], float)
    cnt = rng.multinomial(n, wgt / wgt.sum())
    assert cnt.max() > 100 and (cnt == 0).sum() >= 8
    elem = np.repeat(np.arange(ne, dtype=np.int32), cnt)
    a, b = rng.random(n), rng.random(n)
    flip = a + b > 1.0
    a[flip], b[flip] = 1.0 - a[flip], 1.0 - b[flip]
    v = frame[elem].reshape(n, 3, 2)
    xy = v[:, 0] + a[:, None] * (v[:, 1] - v[:, 0]) + b[:, None] * (v[:, 2] - v[:, 0])
    st["x"], st["y"], st["elem"] = np.mod(xy[:, 0], mesh.period_x), xy[:, 1], elem
    nxt = int(st["pid"].max()) + 1
    oe.import_state(st, step=3, next_pid=nxt)
    ge.import_state(st, step=3, next_pid=nxt)
    compare_states(ge.export(), oe.export(), frame, _length(mesh))
    total = 0
    for n_min in (45, 70):
        mo_, mg = oe.redistribute(n_min), ge.redistribute(n_min)
        assert mo_ == mg and mg > 0, (n_min, mo_, mg)
        total += mg
        rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh))
        assert not excl
        oe.step(0.01)
        ge.step(0.01)
        compare_states(ge.export(), oe.export(), frame, _length(mesh))
    assert total > 1000


@pytest.mark.parametrize("nc", [5, 20])
def test_projection_conditioning_parity(gpu, nc):
    """Fox's projection (Eqs. 64-66) in place of the sort-and-divide bins, with number
    control: the same projected order, intervals and mixing as the oracle."""
    _say(f"test_projection_conditioning_parity nc={nc}")
    mesh = W.channel_mesh(20, 24, stretch=1.1 ** 8, seed=21)
    f = W.channel_fields(mesh)
    mo = W.model_constants()
    ini = W.init_desc(ppe=40, bins=(nc, 1, 1), src_x=3.0, src_r=0.4, conditioning=1)
    og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
    frame = og.export()["frame"]
    excl = set()
    for n in range(6):
        oe.step(2e-3)
        ge.step(2e-3)
        ro, rg = oe.control(38, 42), ge.control(38, 42)
        assert ro == {k: rg[k] for k in ro}, (ro, rg)
        rep, excl = compare_states(ge.export(), oe.export(), frame, _length(mesh), excl)
    assert not excl
    compare_stats(ge.stats(), oe.stats())


def test_projection_in_large_elements(gpu):
    """The workgroup kernel's projection: 600 per element (on chip) and 2200 per element
    (global scratch)."""
    _say("test_projection_in_large_elements")
    mo = W.model_constants()
    for nx, ny, ppe in ((4, 4, 600), (4, 2, 2200)):
        mesh = box(nx, ny, length=2.0, jitter=0.1 if ppe == 600 else 0.0)
        f = W.uniform_fields(mesh, mean_u=(0.3, 0.1, 0.0), mean_omega=4.0)
        ini = W.init_desc(ppe=ppe, bins=(5, 1, 1), src_x=1.0, src_r=0.5, conditioning=1)
        og, oe, gg, ge = _pair(gpu, mesh, f, mo, ini)
        frame = og.export()["frame"]
        for n in range(3):
            oe.step(1e-3)
            ge.step(1e-3)
            compare_states(ge.export(), oe.export(), frame, _length(mesh))
        compare_stats(ge.stats(), oe.stats())


def test_projection_and_bins_in_one_batched_ensemble(gpu):
    """Problems of one batched ensemble may condition differently: each equals its own
    oracle ensemble."""
    _say("test_projection_and_bins_in_one_batched_ensemble")
    mo = W.model_constants()
    m0 = W.channel_mesh(12, 10, seed=7)
    m1 = box(6, 6, length=2.0, jitter=0.2, seed=5)
    cases = [(m0, W.channel_fields(m0), W.init_desc(ppe=40, bins=(4, 2, 2), src_x=2.0, src_r=0.4, seed=101)),
             (m1, W.uniform_fields(m1, mean_u=(0.5, 0.2, 0.0), mean_omega=3.0),
              W.init_desc(ppe=90, bins=(6, 1, 1), src_x=1.0, src_r=0.5, seed=202, conditioning=1))]
    bat = gpu.Ensemble([gpu.Grid(m, f, mo) for m, f, _ in cases], [c[2] for c in cases])
    oes = []
    for p, (m, f, d) in enumerate(cases):
        dd = dict(d)
        dd["seed"] = int(d["seed"]) ^ (p << 32)
        og = O.Grid(m, f, mo)
        oes.append((O.Ensemble(og, dd), og.export()["frame"], m))
    for n in range(4):
        bat.step([1e-3, 2e-3])
        for (o, _, _), dt in zip(oes, (1e-3, 2e-3)):
            o.step(dt)
    for p, (o, frame, m) in enumerate(oes):
        rep, excl = compare_states(bat.export(problem=p), o.export(), frame, _length(m))
        assert not excl
        compare_stats(bat.stats(p), o.stats())
