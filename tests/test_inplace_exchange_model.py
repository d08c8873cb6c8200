"""A CPU model of one level of the in-place variant's exchange, as the GPU
kernels schedule it: work items start at every rank boundary that a tile
cuts on either side of the split point (back keys left of it ranked from the
left, front keys right of it ranked from the right end), an item lists the
keys of one tile per side from its two starts, and exchanges as many pairs
as the shorter list holds.  Items run one at a time in a random order (any
order the GPU may pick), and the model checks the claims the kernels rely
on: no two items start at the same rank, no item uses a key that another
item has already changed or writes a position twice, and the level ends as
the partition Algorithm 1 produces (front keys first) with the same keys."""
import random

import pytest


def exchange_level(keys, tile, rng, front_side):
    n = len(keys)
    front = [k == front_side for k in keys]
    orig = list(keys)
    nt = (n + tile - 1) // tile
    tcnt = [sum(front[j * tile:min(n, j * tile + tile)]) for j in range(nt)]
    pre = [sum(tcnt[:j]) for j in range(nt)]
    F = sum(tcnt)
    nl = (F + tile - 1) // tile
    a = [j * tile - pre[j] for j in range(nt)]     # back keys before tile j
    items = []
    for t in range(nt):
        lo, hi = t * tile, min(n, t * tile + tile)
        if lo < F:
            backs = [p for p in range(lo, min(hi, F)) if not front[p]]
            if backs:
                g = F - 1 - a[t]                   # front keys left of the partner
                i = max(x for x in range(nt) if pre[x] <= g)
                fr = [p for p in range(i * tile, min(n, i * tile + tile)) if front[p]]
                items.append((backs[0], fr[g - pre[i]], a[t]))
        if hi > F:
            fronts = [p for p in range(max(lo, F), hi) if front[p]]
            if fronts:
                r0 = F - pre[t] - tcnt[t]          # front keys after the tile
                jj = max(x for x in range(nl) if a[x] <= r0)
                if a[jj] == r0:
                    continue
                bk = [p for p in range(jj * tile, min(n, jj * tile + tile, F)) if not front[p]]
                items.append((bk[r0 - a[jj]], fronts[-1], r0))
    assert len({it[2] for it in items}) == len(items), "two items start at one rank"
    rng.shuffle(items)
    written = set()
    cur = list(keys)
    for ls, rs, _ in items:
        assert ls < F <= rs
        A = [p for p in range(ls, min((ls // tile + 1) * tile, F)) if cur[p] != front_side]
        B = [p for p in range(rs, max((rs // tile) * tile, F) - 1, -1) if cur[p] == front_side]
        m = min(len(A), len(B))
        for p in A[:m] + B[:m]:
            assert cur[p] == orig[p], "an item used a key another item changed"
            assert p not in written, "a position written twice"
        for pa, pb in zip(A[:m], B[:m]):
            written.update((pa, pb))
            cur[pa], cur[pb] = cur[pb], cur[pa]
    assert all(k == front_side for k in cur[:F]) and all(k != front_side for k in cur[F:])
    assert sorted(cur) == sorted(orig)


@pytest.mark.parametrize("seed", range(4))
def test_exchange_model(seed):
    rng = random.Random(seed)
    for _ in range(400):
        n = rng.randint(1, 260)
        p1 = rng.choice([rng.random(), 0.01, 0.99, 0.5])
        keys = [1 if rng.random() < p1 else 0 for _ in range(n)]
        exchange_level(keys, rng.choice([1, 2, 3, 8, 16, 64]), rng, rng.choice([0, 1]))
