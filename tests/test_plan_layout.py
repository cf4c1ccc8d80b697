"""Host logic of plans: the decomposition of a CSR layout into workgroup
items (sa_plan_layout, no GPU needed) covers every evaluation exactly once,
respects the item capacity, and names consistent fragment slots."""
import numpy as np
import pytest

from paper_1701_08547_amd import api


def _check(seg, shape):
    tile, items_per_lane, wpb = shape
    L = api.plan_layout(seg, shape)
    items, waves, splits = L["items"], L["waves"], L["splits"]
    n_var = len(seg) - 1
    cap = tile * wpb
    packed_of = np.full(n_var, -1)
    parts = {}
    for i, (kind, slot, v) in enumerate(items):
        if kind == 0:
            assert slot == -1
            total = 0
            prev_end = None
            for w in range(wpb):
                e0, e1, v0, v1 = waves[i, w]
                if prev_end is not None:
                    assert v0 == prev_end  # contiguous segment ranges over the waves
                prev_end = v1
                for u in range(v0, v1):
                    assert packed_of[u] == -1
                    packed_of[u] = i
                    size = seg[u + 1] - seg[u]
                    assert size <= tile
                    total += size
            assert total <= cap
        else:
            assert kind == 1
            parts.setdefault(v, []).append((i, slot))
            for w in range(wpb):
                e0, e1, v0, v1 = waves[i, w]
                assert v0 == v and v1 == v + 1
            size = waves[i, -1, 1] - waves[i, 0, 0]
            assert 0 < size <= cap
    for v in range(n_var):
        size = seg[v + 1] - seg[v]
        if v in parts:
            assert packed_of[v] == -1 and size > tile
            # wave parts tile the segment exactly, in order
            edges = []
            for i, _ in parts[v]:
                for w in range(wpb):
                    edges.append((waves[i, w, 0], waves[i, w, 1]))
            assert edges[0][0] == seg[v] and edges[-1][1] == seg[v + 1]
            for (a0, a1), (b0, b1) in zip(edges, edges[1:]):
                assert a1 == b0 and a0 <= a1
        else:
            assert packed_of[v] >= 0, v
    # fragment slots: exactly the segments cut into more than one item
    split_v = {int(s[0]): (int(s[1]), int(s[2])) for s in splits}
    used = set()
    for v, its in parts.items():
        slots = [s for _, s in its]
        if len(its) == 1:
            assert slots == [-1] and v not in split_v
        else:
            first, n = split_v[v]
            assert n == len(its) and slots == list(range(first, first + n))
            used.update(slots)
    assert len(used) == L["n_slots"] and (not used or max(used) == L["n_slots"] - 1)


SHAPES = [(256, 4, 4), (1024, 1, 8), (4096, 4, 4), (8192, 2, 16)]


@pytest.mark.parametrize("shape", SHAPES)
def test_random_layouts(shape):
    g = np.random.default_rng(sum(shape))
    for _ in range(10):
        n = int(g.integers(1, 300))
        sizes = np.where(g.random(n) < 0.1, 0, np.floor(np.exp(g.uniform(0, np.log(200000), n)))).astype(np.int64)
        seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        _check(seg, shape)


def test_c1_layout_needs_no_merge():
    """1,000 segments of 16,384 with tile 4,096 x 4 waves: one item per
    segment, no fragments."""
    seg = np.arange(1001, dtype=np.int64) * 16384
    L = api.plan_layout(seg, (4096, 4, 4))
    assert len(L["items"]) == 1000 and len(L["splits"]) == 0 and L["n_slots"] == 0
    _check(seg, (4096, 4, 4))


def test_all_empty_and_edge_layouts():
    for seg in ([0], [0, 0, 0, 0], [0, 1], [0, 0, 5, 5, 100000, 100000]):
        _check(np.array(seg, np.int64), (1024, 4, 4))


def test_invalid_offsets_rejected():
    for seg, n_evals in (([1, 5], 5), ([0, 5, 3], 3), ([0, 5], 6)):
        s = np.array(seg, np.int64)
        ni = api.ctypes.c_int64()
        rc = api.lib().sa_plan_layout(s.ctypes.data_as(api.ctypes.c_void_p), len(seg) - 1, n_evals, None,
                                      api.ctypes.byref(ni), None, None, None, None, None)
        assert rc == -1
    with pytest.raises(api.SAError):
        api.plan_layout(np.array([0, 10], np.int64), (1000, 4, 4))  # tile not a multiple of 256
    with pytest.raises(api.SAError):
        api.plan_layout(np.array([0, 10], np.int64), (1024, 3, 4))
