"""Oracle pins for the particle redistribution of App. B.

The loop moves one particle at a time from the element holding the most particles to the
element holding the fewest, until the fewest reaches N_min or the counts are even (max -
min <= 1).  The pins check what that fixes independently of the random choices:
- hand-worked count sequences (ties to the lowest element index, the two stopping rules);
- with enough particles (N >= n_e N_min) the number of moves is the total deficit
  sum_e max(0, N_min - n_e), since no donor can fall below N_min;
- with too few particles the final counts are the even split floor/ceil(N / n_e);
- particle count, pids and total weight are unchanged, every moved particle carries the
  position and properties of a particle that was already in its new element, and an empty
  element receives its first particle at its centroid;
- the moving particle and the copied one are drawn uniformly (a biased pick fails a
  4-sigma bound on the mean of a rank-tagged attribute)."""
import numpy as np
import pytest

import oracle as O
from paper_1006_0532_amd import workloads as W


def _mesh(nx=4, ny=2):
    return W.channel_mesh(nx, ny, length=2.0, stretch=1.0, jitter=0.0, random_diagonals=False,
                          bottom=W.EDGE_SLIP, top=W.EDGE_SLIP)


def _grid(mesh):
    return O.Grid(mesh, W.uniform_fields(mesh), W.model_constants())


def _state(frame, counts, seed=1):
    """counts[e] particles strictly inside element e (element frame), random properties."""
    rng = np.random.default_rng(seed)
    elem = np.repeat(np.arange(len(counts), dtype=np.int32), counts)
    n = len(elem)
    lam = rng.uniform(0.05, 1.0, (n, 3))
    lam /= lam.sum(1, keepdims=True)
    F = frame[elem]
    x = (lam * F[:, 0::2]).sum(1)
    y = (lam * F[:, 1::2]).sum(1)
    return dict(x=x, y=y, u=rng.normal(size=(n, 3)), om=rng.gamma(4.0, 0.25, n), psi=rng.uniform(size=n),
                w=rng.uniform(0.5, 1.5, n), pid=rng.permutation(n).astype(np.uint64), elem=elem)


def _ensemble(counts, mesh=None, seed=1):
    mesh = mesh or _mesh()
    g = _grid(mesh)
    frame = g.export()["frame"]
    st = _state(frame, counts, seed)
    e = O.Ensemble(g, W.init_desc(ppe=1, seed=seed))
    e.import_state(st, step=3, next_pid=len(st["x"]))
    return e, st, frame


def _counts(e, ne):
    return np.bincount(e.export()["elem"], minlength=ne)


def test_hand_worked_sequence_with_empty_element():
    """Counts (5, 0, 1, 2, ...) with N_min = 2: e1 (empty) takes a particle of e0 at its
    centroid, then e1 (tie with e2, lower index) takes a copy of it, then e2 takes a copy
    of its own particle; three moves."""
    ne = _mesh().n_elems
    counts = np.full(ne, 2)
    counts[:3] = (5, 0, 1)
    e, st, frame = _ensemble(counts)
    assert e.redistribute(2) == 3
    got = e.export()
    c = np.bincount(got["elem"], minlength=ne)
    assert c[0] == 2 and c[1] == 2 and c[2] == 2 and (c[3:] == 2).all()
    cx, cy = frame[1, 0::2].mean(), frame[1, 1::2].mean()
    in1 = got["elem"] == 1
    assert np.all(got["x"][in1] == cx) and np.all(got["y"][in1] == cy)
    for k in ("om", "psi"):
        assert got[k][in1][0] == got[k][in1][1]
    assert np.all(got["u"][in1][0] == got["u"][in1][1])
    # the first mover kept its own properties: they are those of one of e0's particles
    src = np.flatnonzero(st["elem"] == 0)
    assert any(st["om"][i] == got["om"][in1][0] and st["psi"][i] == got["psi"][in1][0] for i in src)
    # e2: the copy duplicates e2's original particle
    in2 = np.flatnonzero(got["elem"] == 2)
    assert got["x"][in2[0]] == got["x"][in2[1]] and got["om"][in2[0]] == got["om"][in2[1]]


def test_stops_when_even_or_all_at_threshold():
    ne = _mesh().n_elems
    # all equal below the threshold: nothing to do
    e, _, _ = _ensemble(np.full(ne, 3))
    assert e.redistribute(10) == 0
    # counts differing by one: the printed loop would swap them forever, this one stops
    counts = np.full(ne, 3)
    counts[::2] = 4
    e, _, _ = _ensemble(counts)
    assert e.redistribute(10) == 0
    # already at the threshold
    e, _, _ = _ensemble(np.full(ne, 3))
    assert e.redistribute(3) == 0


def test_ties_go_to_lowest_index():
    """(2, 0, 0, 1, ...) with N_min = 1: the two empty elements tie and the lower index (e1)
    receives; after that max - min = 1 and the loop stops with e2 still empty.
    (2, 0, 2, 1, ...): e0 and e2 tie at the maximum and the lower index (e0) gives."""
    ne = _mesh().n_elems
    counts = np.ones(ne, int)
    counts[:3] = (2, 0, 0)
    e, _, _ = _ensemble(counts)
    assert e.redistribute(1) == 1
    assert tuple(_counts(e, ne)[:3]) == (1, 1, 0)
    counts[:3] = (2, 0, 2)
    e, _, _ = _ensemble(counts)
    assert e.redistribute(1) == 1
    assert tuple(_counts(e, ne)[:3]) == (1, 1, 2)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_moves_equal_total_deficit(seed):
    mesh = _mesh(6, 4)
    ne = mesh.n_elems
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, 30, ne)
    n_min = int(counts.sum() // ne) - 2
    deficit = int(np.maximum(0, n_min - counts).sum())
    e, st, _ = _ensemble(counts, mesh, seed)
    assert e.redistribute(n_min) == deficit
    c = _counts(e, ne)
    assert c.min() >= n_min and c.sum() == counts.sum()
    # elements that had at least N_min + 1 only gave, the others only received
    assert np.all(c[counts < n_min] == n_min)
    assert np.all((c <= counts) | (counts < n_min))


@pytest.mark.parametrize("seed", [4, 5])
def test_even_split_when_particles_are_short(seed):
    mesh = _mesh(6, 4)
    ne = mesh.n_elems
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, 12, ne)
    N = int(counts.sum())
    e, _, _ = _ensemble(counts, mesh, seed)
    e.redistribute(N // ne + 5)
    c = _counts(e, ne)
    lo = N // ne
    assert c.min() >= lo and c.max() <= lo + 1
    assert int((c == lo + 1).sum()) == N - lo * ne


def test_conservation_and_copies():
    mesh = _mesh(6, 4)
    ne = mesh.n_elems
    rng = np.random.default_rng(7)
    counts = rng.integers(0, 25, ne)
    counts[5] = 0
    e, st, frame = _ensemble(counts, mesh, 7)
    before = e.export()
    moves = e.redistribute(12)
    assert moves > 0
    after = e.export()
    assert np.array_equal(before["pid"], after["pid"])
    assert np.array_equal(before["w"], after["w"])            # weights travel with the particle
    assert abs(after["w"].sum() - before["w"].sum()) == 0.0
    moved = (before["elem"] != after["elem"]) | (before["x"] != after["x"])
    stay = ~moved
    key = lambda d, i: (d["x"][i], d["y"][i], *d["u"][i], d["om"][i], d["psi"][i])
    originals = {}
    for i in np.flatnonzero(stay):
        originals.setdefault(int(after["elem"][i]), set()).add(key(after, i))
    for i in np.flatnonzero(moved):
        el = int(after["elem"][i])
        if counts[el] == 0:
            cx, cy = frame[el, 0::2].mean(), frame[el, 1::2].mean()
            assert after["x"][i] == cx and after["y"][i] == cy
        else:
            assert key(after, i) in originals[el]
    # the oracle's grouping is rebuilt by the next step
    e.step(1e-4)
    assert e.count() == len(before["x"])


def test_draws_are_uniform():
    """One element of 4000 particles gives 8 to each of 119 elements of 8.  The
    canonical order sorts by U1 first, so a pick biased towards one end of it shows in the
    U1 tags: the weight (kept by the moving particle) is 1 + tanh(U1)/2 in the giving
    element, and psi is the U1 rank / 7 inside each receiving element (copied with the
    donor).  Both means must match their population's within 4 sigma."""
    mesh = _mesh(10, 6)
    ne = mesh.n_elems
    counts = np.full(ne, 8)
    counts[0] = 4000
    g = _grid(mesh)
    frame = g.export()["frame"]
    st = _state(frame, counts, 11)
    big = st["elem"] == 0
    st["w"][big] = 1.0 + 0.5 * np.tanh(st["u"][big, 0])
    for el in range(1, ne):
        ids = np.flatnonzero(st["elem"] == el)
        st["psi"][ids[np.argsort(st["u"][ids, 0])]] = np.arange(8) / 7.0
    e = O.Ensemble(g, W.init_desc(ppe=1, seed=11))
    e.import_state(st, step=0, next_pid=len(st["x"]))
    before = e.export()
    moves = e.redistribute(16)
    assert moves == 8 * (ne - 1)
    after = e.export()
    gave = (before["elem"] == 0) & (after["elem"] != 0)
    assert gave.sum() == moves
    wpop = before["w"][big[np.argsort(st["pid"], kind="stable")]]
    wm = after["w"][gave]
    assert abs(wm.mean() - wpop.mean()) < 4.0 * wpop.std() / np.sqrt(len(wm))
    # copied psi: per receiving element the copies form one correlated sample (copies of
    # copies), so the bound uses one sample per element
    per_el = np.array([after["psi"][gave & (after["elem"] == el)].mean() for el in range(1, ne)])
    assert abs(per_el.mean() - 0.5) < 4.0 * np.sqrt(np.var(np.arange(8) / 7.0) / (ne - 1))
