"""The level decomposition behind the device planner of App. B's redistribution.

App. B moves one particle at a time from the fullest element to the emptiest (ties to the
lowest index) until the emptiest holds n_min or the two differ by at most one.  The device
plans all moves at once from the claim that, while the loop runs, the giving side and the
receiving side never meet: move m is the m-th (level, element) pair of the receiving side
(levels lmin, lmin + 1, ...; at level l every element that started with at most l particles,
in index order) and of the giving side (levels hmax, hmax - 1, ...; at level h every element
that started with at least h), and only the slot choices inside one element depend on that
element's earlier moves.  This test checks the claim on random count vectors against a plain
transcription of the serial loop, with slot draws from a seeded stand-in for the random
numbers (the same draw for move m on both sides)."""
import random

import pytest


def serial_moves(c0, n_min, draw):
    """App. B's serial loop: the plan {slot: (position source, property source, element)};
    a centroid position is -(e + 1)."""
    ne = len(c0)
    start = [0]
    for c in c0:
        start.append(start[-1] + c)
    cnt = list(c0)
    if ne == 0 or min(cnt) >= n_min or max(cnt) - min(cnt) <= 1:
        return {}
    lists = {}

    def members(e):
        if e not in lists:
            lists[e] = list(range(start[e], start[e + 1]))
        return lists[e]

    moved = {}
    m = 0
    while True:
        recv = min(range(ne), key=lambda e: (cnt[e], e))
        top = max(cnt)
        give = min(e for e in range(ne) if cnt[e] == top)
        if cnt[recv] >= n_min or top - cnt[recv] <= 1:
            break
        u_give, u_take = draw(m)
        g = members(give)
        slot = g.pop(int(u_give * len(g)))
        t = members(recv)
        if t:
            src = t[int(u_take * len(t))]
            pos, prop = moved[src][:2] if src in moved else (src, src)
        else:
            pos, prop = -recv - 1, slot
        moved[slot] = (pos, prop, recv)
        t.append(slot)
        cnt[recv] += 1
        cnt[give] -= 1
        m += 1
    return moved


def level_moves(c0, n_min, draw):
    """The same plan from the level decomposition: the number of moves from a walk over
    levels, each side's move indices from (level, element) ranks, then the slot draws of each
    element in its own move order."""
    ne = len(c0)
    if ne == 0:
        return {}
    start = [0]
    for c in c0:
        start.append(start[-1] + c)
    lmin, hmax = min(c0), max(c0)
    if lmin >= n_min or hmax - lmin <= 1:
        return {}
    l, r, h, q, K = lmin, 0, hmax, 0, 0
    while not (l >= n_min or h - l <= 1):
        P = sum(1 for c in c0 if c <= l)
        Q = sum(1 for c in c0 if c >= h)
        k = min(P - r, Q - q)
        K, r, q = K + k, r + k, q + k
        if r == P:
            l, r = l + 1, 0
        if q == Q:
            h, q = h - 1, 0
    if K == 0:
        return {}

    def side(key, L):
        first = [0]
        for t in range(L):
            first.append(first[-1] + sum(1 for x in key if x <= t))
        out = {}
        for e in range(ne):
            out[e] = [(t, first[t] + sum(1 for e2 in range(e) if key[e2] <= t))
                      for t in range(key[e], L)]
            out[e] = [(t, m) for t, m in out[e] if m < K]
        return out

    takes = side([c - lmin for c in c0], l - lmin + 1)
    gives = side([hmax - c for c in c0], hmax - h + 1)
    slot_of = {}
    for e in range(ne):
        gone = [False] * c0[e]
        for t, m in gives[e]:
            size = hmax - t
            rank = int(draw(m)[0] * size)
            for j in range(c0[e]):
                if not gone[j]:
                    if rank == 0:
                        break
                    rank -= 1
            gone[j] = True
            slot_of[m] = start[e] + j
    plan = {}
    for e in range(ne):
        arrivals = []
        for t, m in takes[e]:
            size = lmin + t
            if size == 0:
                pos, prop = -e - 1, slot_of[m]
            else:
                d = int(draw(m)[1] * size)
                pos, prop = (start[e] + d,) * 2 if d < c0[e] else arrivals[d - c0[e]]
            arrivals.append((pos, prop))
            plan[slot_of[m]] = (pos, prop, e)
    return plan


@pytest.mark.parametrize("seed", range(6))
def test_level_decomposition_reproduces_the_serial_loop(seed):
    rng = random.Random(seed)
    cases = 0
    for _ in range(300):
        ne = rng.randint(1, 30)
        mode = rng.random()
        if mode < 0.4:
            c0 = [rng.choice([0, 0, 1, 2, rng.randint(0, 15), rng.randint(0, 40)]) for _ in range(ne)]
        else:
            c0 = [max(0, int(rng.gauss(12, 6))) for _ in range(ne)]
        n_min = rng.randint(0, 25)
        key = rng.random()

        def draw(m, key=key):
            d = random.Random(hash((key, m)))
            return d.random(), d.random()

        a = serial_moves(c0, n_min, draw)
        assert level_moves(c0, n_min, draw) == a, (c0, n_min)
        cases += bool(a)
    assert cases > 100
