"""Pins of the oracle's footprint-sized cells (section 3: position cells
sized from the footprint of the shading point, about a user-defined tile
for visible points).  Reading: each point carries the side f of its
footprint; its level is the smallest L below `footprint_levels` whose cell
edge base 2^L reaches tile * f (base: the grid's smallest cell edge), and at
level L each axis holds cells of 2^L finest cells.  Expected levels and
keys are written out by hand from that rule; the jittered lookup at a level
against closed-form neighbour frequencies; and the estimator stays
unbiased."""
import numpy as np
import pytest
from scipy import stats

from paper_1911_10217_amd import scenes

from test_oracle_estimator import _below_lights, _mean_and_se

SCENE = 3
TILE = 16.0


def _oracle(orc, n_points=4, dims=(64, 64, 64), levels=4, **kw):
    s = scenes.make_tiny(n_lights=64, n_points=n_points, n_boxes=0, M=8, spp=1, scene_id=SCENE,
                         grid_dims=dims, hashed=1, capacity=1 << 16, footprint_levels=levels,
                         footprint_tile=TILE, **kw)
    return s, orc.Oracle(s.params, s.tri, s.emit)


def _lins(o, pos, nrm, spp=1, frame=0, fp=None):
    pos = np.asarray(pos, np.float32)
    nrm = np.asarray(nrm, np.float32)
    if fp is not None:
        o.set_footprints(np.asarray(fp, np.float32))
    _, rec = o.frame(pos, nrm, spp, frame, records=True)
    k = rec["key"].astype(np.uint64)
    assert np.all((k >> np.uint64(32)) == SCENE)
    return (k & np.uint64(0xFFFFFFFF)).astype(np.int64)


UP = [0.0, 1.0, 0.0]


def test_levels_from_footprints_in_closed_form(orc):
    """64^3 cells on the unit cube: base 1/64.  tile * f equal to 2^L / 64
    is reached by level L exactly; a hair above needs level L + 1; 0 and
    tiny footprints give level 0; huge ones the coarsest level."""
    s, o = _oracle(orc, n_points=10)
    base = 1.0 / 64.0
    f = [0.0, 1e-9, base / TILE, 2 * base / TILE, 4 * base / TILE, 8 * base / TILE,
         np.nextafter(np.float32(base / TILE), np.float32(1)), np.nextafter(np.float32(2 * base / TILE), np.float32(1)),
         1e3, np.nextafter(np.float32(4 * base / TILE), np.float32(1))]
    o.set_footprints(np.array(f, np.float32))
    assert o.point_levels(10).tolist() == [0, 0, 0, 1, 2, 3, 1, 2, 3, 3]


def test_keys_at_each_level_in_closed_form(orc):
    """Level-major linear index: level L starts after all cells of the
    finer levels (64^3, 32^3, 16^3 of them) and numbers its own cells
    ix + dL (iy + dL iz) with dL = 64 / 2^L and i = floor(64 p) >> L."""
    s, o = _oracle(orc, n_points=4)
    base = 1.0 / 64.0
    p = np.array([[0.3, 0.5, 0.7]] * 4, np.float32)
    n = np.array([UP] * 4, np.float32)
    fp = np.array([0.0, 2 * base / TILE, 4 * base / TILE, 8 * base / TILE], np.float32)
    lins = _lins(o, p, n, fp=fp)
    first = [0, 64 ** 3, 64 ** 3 + 32 ** 3, 64 ** 3 + 32 ** 3 + 16 ** 3]
    want = []
    for L in range(4):
        dL = 64 >> L
        i = [int(np.floor(np.float32(c) * np.float32(64))) >> L for c in (0.3, 0.5, 0.7)]
        want.append(first[L] + i[0] + dL * (i[1] + dL * i[2]))
    assert lins.tolist() == want
    # level 3 by hand: cells of 1/8, point (0.3, 0.5, 0.7) in cell (2, 4, 5)
    assert want[3] == first[3] + 2 + 8 * (4 + 8 * 5)


def test_without_footprints_the_keys_are_the_position_cells(orc):
    s, o = _oracle(orc, n_points=200)
    rng = np.random.default_rng(2)
    pos = rng.random((200, 3)).astype(np.float32)
    n = np.tile(np.float32(UP), (200, 1))
    lin = _lins(o, pos, n)
    assert np.array_equal(lin.astype(np.uint64) | (np.uint64(SCENE) << np.uint64(32)), o.cell_keys(pos))
    # footprints of zero: level 0, the same keys
    assert np.array_equal(_lins(o, pos, n, fp=np.zeros(200)), lin)


def test_coarse_cells_group_whole_blocks_of_fine_cells(orc):
    """At level L two points share a cell exactly when their finest indices
    agree after dropping L bits; a non-cubic grid of 40 x 24 x 10 cells
    (base: the x edge) has ((d - 1) >> L) + 1 cells per axis at level L."""
    dims = (40, 24, 10)
    s, o = _oracle(orc, n_points=3000, dims=dims, levels=3)
    rng = np.random.default_rng(3)
    pos = rng.random((3000, 3)).astype(np.float32)
    n = np.tile(np.float32(UP), (3000, 1))
    base = 1.0 / 40.0
    L = rng.integers(0, 3, 3000)
    fp = (np.float32(base) * (2.0 ** L).astype(np.float32) / np.float32(TILE)).astype(np.float32)
    o.set_footprints(fp)
    assert np.array_equal(o.point_levels(3000), L)
    lins = _lins(o, pos, n)
    fine = np.stack([np.floor(pos[:, a] * np.float32(dims[a])).astype(np.int64) for a in range(3)], 1)
    first = [0]
    for lv in range(3):
        first.append(first[-1] + np.prod([((d - 1) >> lv) + 1 for d in dims]))
    dl = np.array([[((d - 1) >> lv) + 1 for d in dims] for lv in range(3)])
    i = fine >> L[:, None]
    want = np.array(first)[L] + i[:, 0] + dl[L, 0] * (i[:, 1] + dl[L, 1] * i[:, 2])
    assert np.array_equal(lins, want)
    assert first[3] == 40 * 24 * 10 + 20 * 12 * 5 + 10 * 6 * 3


def test_jitter_reaches_cells_of_the_points_level(orc):
    """Normal +y: the lookup moves by (cell of the level) * (xi0, 0, -xi1).
    From fractional position (0.2, 0.9) inside its level-2 cell (4 finest
    cells wide) it lands one level-2 cell lower in x with probability 0.3
    and one higher in z with 0.4."""
    s, o = _oracle(orc, n_points=1, jitter=1.0)
    cell = 4.0 / 64.0
    x = np.array([[(2 + 0.2) * cell, 0.5 * cell, (3 + 0.9) * cell]], np.float32)
    n = np.array([UP], np.float32)
    o.set_footprints(np.array([4.0 / 64.0 / TILE], np.float32))
    assert o.point_levels(1).tolist() == [2]
    lins = np.concatenate([_lins(o, x, n, 64, f) for f in range(40)])
    first2 = 64 ** 3 + 32 ** 3
    r = lins - first2
    ix, iy, iz = r % 16, (r // 16) % 16, r // 256
    assert np.all(iy == 0)
    cnt = np.array([np.sum((ix == a) & (iz == b)) for a, b in ((2, 3), (1, 3), (2, 4), (1, 4))])
    assert cnt.sum() == lins.size
    p = np.array([0.7 * 0.6, 0.3 * 0.6, 0.7 * 0.4, 0.3 * 0.4])
    assert stats.chisquare(cnt, p * lins.size).pvalue > 1e-4, cnt


def test_bad_footprints_and_levels_are_refused(orc):
    s, o = _oracle(orc)
    for bad in ([np.nan], [-1.0], [np.inf]):
        with pytest.raises(ValueError):
            o.set_footprints(np.array(bad, np.float32))
    with pytest.raises(ValueError):
        _oracle(orc, levels=17)
    with pytest.raises(ValueError):
        scenes_bad = scenes.make_tiny(n_lights=8, n_points=4, footprint_levels=3, footprint_tile=0.0)
        orc.Oracle(scenes_bad.params, scenes_bad.tri, scenes_bad.emit)


def test_estimator_unbiased_with_footprint_cells(orc):
    s = _below_lights(scenes.make_tiny(n_lights=96, n_points=24, n_boxes=0, M=8, spp=8, grid_dims=(64, 64, 64),
                                       hashed=1, capacity=4096, footprint_levels=5, footprint_tile=TILE,
                                       jitter=1.0))
    o = orc.Oracle(s.params, s.tri, s.emit)
    rng = np.random.default_rng(9)
    o.set_footprints((rng.random(s.P) * 16.0 / 64.0 / TILE).astype(np.float32))
    lv = o.point_levels(s.P)
    assert len(set(lv.tolist())) >= 4
    frames = o.run(s.pos, s.nrm, 8, 300)
    mean, se = _mean_and_se(frames[20:])
    truth = o.truth_unoccluded(s.pos, s.nrm)
    z = (mean - truth) / np.maximum(se, 1e-12)
    assert np.max(np.abs(z)) < 5.0, np.max(np.abs(z))
    assert abs(float(np.mean(z))) < 0.5


def test_level_keys_with_normal_bins(orc):
    """Normal bins sit above the level's position cells: 40 x 24 x 10 cells,
    2 x 2 normal bins, level 2 has 10 x 6 x 3 position cells; normal +z maps
    to the octahedral centre (1/2, 1/2), bin (1, 1)."""
    dims = (40, 24, 10)
    s, o = _oracle(orc, n_points=1, dims=dims, levels=3, normal_bits=1)
    p = np.array([[0.55, 0.3, 0.95]], np.float32)
    n = np.array([[0.0, 0.0, 1.0]], np.float32)
    lin = _lins(o, p, n, fp=[4.0 / 40.0 / TILE])
    first2 = (40 * 24 * 10 + 20 * 12 * 5) * 4
    ix, iy, iz = 22 >> 2, 7 >> 2, 9 >> 2
    assert lin.tolist() == [first2 + ix + 10 * (iy + 6 * (iz + 3 * (1 + 2 * 1)))]
