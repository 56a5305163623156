"""Pins of the oracle's reference light tree and initial cut (section 3,
section 3.1: LBVH over light positions; initial cut by breadth-first descent).
"""
import numpy as np
import pytest

from paper_1911_10217_amd import scenes


def _tri_at(points, size=1e-3):
    """Small triangles whose vertex sum is 3 * p + fixed offsets."""
    p = np.asarray(points, np.float64)
    v0 = p
    v1 = p + np.array([size, 0.0, 0.0])
    v2 = p + np.array([0.0, 0.0, size])
    return np.concatenate([v0, v1, v2], axis=1).astype(np.float32)


def _oracle(orc, tri, M=4, **kw):
    p = scenes.params_for(M=M, **kw)
    emit = np.ones((tri.shape[0], 3), np.float32)
    return orc.Oracle(p, tri, emit)


def _check_tree_invariants(t, N):
    first, last, left, right, parent = t["first"], t["last"], t["left"], t["right"], t["parent"]
    assert sorted(t["perm"].tolist()) == list(range(N))
    if N == 1:
        assert first[0] == 0 and last[0] == 0 and parent[0] == 0xFFFFFFFF
        return
    assert first[0] == 0 and last[0] == N - 1 and parent[0] == 0xFFFFFFFF
    seen = np.zeros(2 * N - 1, np.int64)
    for i in range(N - 1):
        l, r = left[i], right[i]
        seen[l] += 1
        seen[r] += 1
        assert parent[l] == i and parent[r] == i
        assert first[l] == first[i] and last[r] == last[i]
        assert last[l] + 1 == first[r]
        assert first[l] <= last[l] < first[r] <= last[r]
    # every node but the root is a child exactly once
    assert seen[0] == 0 and np.all(seen[1:] == 1)
    for j in range(N):
        assert first[N - 1 + j] == j and last[N - 1 + j] == j


def test_morton_axis_priority(orc):
    # vertex sums at the bounding-box corners; x is the most significant axis,
    # then y, then z, so the order is origin, +z, +y, +x
    tri = _tri_at([[1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, 0]])
    t = _oracle(orc, tri).tree()
    assert t["perm"].tolist() == [3, 2, 1, 0]


def test_morton_interleaving_bits(orc):
    # quantised (x, y, z) on a 1024 grid: a point at x-cell 1 has Morton code
    # 4, a point at z-cell 3 has code 9 (z bits 0 and 3), at y-cell 2 has 16:
    # the sorted order is therefore x1 (4), z3 (9), y2 (16).
    pts = np.array([[0, 2, 0], [0, 0, 3], [1, 0, 0], [1023, 1023, 1023], [0, 0, 0]], np.float64)
    # vertex sum = 3 * p + (size, 0, size); place p so that the sum hits cell centres
    tri = _tri_at((pts + 0.5) / 1024.0)
    t = _oracle(orc, tri).tree()
    order = t["perm"].tolist()
    assert order[0] == 4 and order[-1] == 3
    assert order[1:4] == [2, 1, 0]


def test_equal_positions_keep_input_order(orc):
    tri = _tri_at([[0.5, 0.5, 0.5]] * 6 + [[0.0, 0.0, 0.0]])
    t = _oracle(orc, tri).tree()
    assert t["perm"].tolist() == [6, 0, 1, 2, 3, 4, 5]
    _check_tree_invariants(t, 7)


def test_three_light_topology(orc):
    # x-cells 0, 1 and 1023: the root separates {0, 1} from {1023}; node ids:
    # root 0, its left child (internal, range [0,1]) takes id 1, its right
    # child is leaf 2 -> id N-1+2 = 4; node 1's children are leaves 2 and 3.
    xs = np.array([0.0, 1.0, 1023.0])
    lo, hi = 0.0, 1023.0
    pts = np.zeros((3, 3))
    pts[:, 0] = xs / 1023.0 * (1 - 1e-3)
    tri = _tri_at(pts)
    t = _oracle(orc, tri).tree()
    assert t["left"].tolist() == [1, 2] and t["right"].tolist() == [4, 3]
    assert t["first"][:2].tolist() == [0, 0] and t["last"][:2].tolist() == [2, 1]
    assert t["parent"].tolist() == [0xFFFFFFFF, 0, 1, 1, 0]


@pytest.mark.parametrize("N", [1, 2, 3, 5, 17, 1000])
def test_tree_invariants_random(orc, N):
    rng = np.random.default_rng(N)
    tri = rng.random((N, 9)).astype(np.float32)
    _check_tree_invariants(_oracle(orc, tri, M=min(4, N)).tree(), N)


def _line(N):
    # N = 2^k lights equally spaced along x: a perfectly balanced radix tree
    pts = np.zeros((N, 3))
    pts[:, 0] = (np.arange(N) + 0.25) / N
    pts[:, 1] = 0.5
    pts[:, 2] = 0.5
    rng = np.random.default_rng(0)
    return _tri_at(pts[rng.permutation(N)], size=1e-5)


@pytest.mark.parametrize("k", [1, 3, 6, 10])
def test_balanced_tree_closed_form(orc, k):
    N = 1 << k
    t = _oracle(orc, _line(N), M=1).tree()
    _check_tree_invariants(t, N)
    for i in range(N - 1):
        size = int(t["last"][i] - t["first"][i] + 1)
        assert size & (size - 1) == 0, "every subtree of a balanced tree holds 2^j lights"
        assert t["last"][t["left"][i]] - t["first"][i] + 1 == size // 2, "split in the middle"


def _ranges(o):
    node, end = o.template()
    t = o.tree()
    return [(int(t["first"][n]), int(t["last"][n])) for n in node], end


@pytest.mark.parametrize("M,expect", [
    (1, [(0, 15)]),
    (2, [(0, 7), (8, 15)]),
    (4, [(0, 3), (4, 7), (8, 11), (12, 15)]),
    (5, [(0, 1), (2, 3), (4, 7), (8, 11), (12, 15)]),
    (16, [(i, i) for i in range(16)]),
])
def test_initial_cut_breadth_first(orc, M, expect):
    o = _oracle(orc, _line(16), M=M)
    r, end = _ranges(o)
    assert r == expect
    assert end.tolist() == [b + 1 for _, b in expect]
    assert o.Meff == len(expect)


def test_initial_cut_more_slots_than_lights(orc):
    o = _oracle(orc, _line(4), M=16)
    r, end = _ranges(o)
    assert r == [(0, 0), (1, 1), (2, 2), (3, 3)] and o.Meff == 4


def test_initial_cut_partitions_lights(orc):
    s = scenes.make_tiny()
    o = orc.Oracle(s.params, s.tri, s.emit, s.boxes)
    node, end = o.template()
    assert o.Meff == 16
    assert np.all(np.diff(end.astype(np.int64)) > 0) and end[-1] == s.N
    t = o.tree()
    starts = np.concatenate([[0], end[:-1]])
    assert np.array_equal(t["first"][node], starts)


def test_emitter_records(orc):
    s = scenes.make_tiny(n_lights=64)
    o = orc.Oracle(s.params, s.tri, s.emit, s.boxes)
    t = o.tree()
    rec = t["rec"]
    tri = s.tri[t["perm"]].astype(np.float64)
    np.testing.assert_array_equal(rec[:, :9], s.tri[t["perm"]])
    np.testing.assert_array_equal(rec[:, 9:12], s.emit[t["perm"]])
    cr = np.cross(tri[:, 3:6] - tri[:, 0:3], tri[:, 6:9] - tri[:, 0:3])
    area = 0.5 * np.linalg.norm(cr, axis=1)
    np.testing.assert_allclose(rec[:, 12], area, rtol=1e-5)
    np.testing.assert_allclose(rec[:, 13:16], cr / np.linalg.norm(cr, axis=1, keepdims=True), atol=1e-5)
