"""Pins of the oracle's 5-D cell keys (section 3: cells over position and
normal, located by jittered quantised coordinates): closed-form bins of the
octahedral normal map, its published inverse, the closed-form distribution
of the jittered lookup, and unbiasedness of the estimator with such cells."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_1911_10217_amd import scenes

from test_oracle_estimator import _below_lights, _mean_and_se

SCENE = 7  # scene id: keys carry it in their upper 32 bits


def _oracle(orc, n_points=4, **kw):
    s = scenes.make_tiny(n_lights=64, n_points=n_points, n_boxes=0, M=8, spp=1, scene_id=SCENE, **kw)
    return s, orc.Oracle(s.params, s.tri, s.emit)


def _keys(o, pos, nrm, spp, frame=0):
    _, rec = o.frame(np.asarray(pos, np.float32), np.asarray(nrm, np.float32), spp, frame, records=True)
    k = rec["key"].astype(np.uint64)
    assert np.all((k >> np.uint64(32)) == SCENE)
    return (k & np.uint64(0xFFFFFFFF)).astype(np.int64)


def _split(lin, dims, nb):
    # lin = ix + dx (iy + dy (iz + dz (qu + nb qv)))
    dx, dy, dz = dims
    ix, r = lin % dx, lin // dx
    iy, r = r % dy, r // dy
    iz, r = r % dz, r // dz
    return ix, iy, iz, r % nb, r // nb


def test_position_only_keys_unchanged(orc):
    s, o = _oracle(orc, n_points=64)
    lin = _keys(o, s.pos, s.nrm, 1)
    assert np.array_equal(lin.astype(np.uint64) | (np.uint64(SCENE) << np.uint64(32)), o.cell_keys(s.pos))


def test_axis_normals_land_in_closed_form_bins(orc):
    nb = 8
    s, o = _oracle(orc, normal_bits=3)
    # octahedral map: +z -> (1/2, 1/2); +-x -> u = 1 or 0 at v = 1/2;
    # +-y -> v = 1 or 0 at u = 1/2; -z folds onto the corner (1, 1)
    cases = {(0, 0, 1): (nb // 2, nb // 2), (1, 0, 0): (nb - 1, nb // 2), (-1, 0, 0): (0, nb // 2),
             (0, 1, 0): (nb // 2, nb - 1), (0, -1, 0): (nb // 2, 0), (0, 0, -1): (nb - 1, nb - 1)}
    n = np.array(list(cases), np.float32)
    pos = np.full((n.shape[0], 3), 0.3, np.float32)
    _, _, _, qu, qv = _split(_keys(o, pos, n, 1), s.params["grid_dims"], nb)
    assert list(zip(qu.tolist(), qv.tolist())) == list(cases.values())
    # opposite normals at one point get different cells: back-facing light
    # is learnt separately
    assert len(set((qu + nb * qv).tolist())) == len(cases)


def _oct_decode(u, v):
    # the published inverse of the octahedral map (Cigolle et al. 2014)
    x, y = 2.0 * u - 1.0, 2.0 * v - 1.0
    z = 1.0 - np.abs(x) - np.abs(y)
    lower = z < 0
    xf = np.where(lower, (1.0 - np.abs(y)) * np.sign(x), x)
    yf = np.where(lower, (1.0 - np.abs(x)) * np.sign(y), y)
    d = np.stack([xf, yf, z], 1)
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_bins_decode_near_their_normals(orc):
    nb = 16
    rng = np.random.default_rng(5)
    n = rng.normal(size=(3000, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    s, o = _oracle(orc, n_points=3000, normal_bits=4)
    pos = np.full((3000, 3), 0.3, np.float32)
    _, _, _, qu, qv = _split(_keys(o, pos, n, 1), s.params["grid_dims"], nb)
    c = _oct_decode((qu + 0.5) / nb, (qv + 0.5) / nb)
    ang = np.degrees(np.arccos(np.clip((c * n).sum(1), -1, 1)))
    # a bin spans at most ~2 * 180 / 16 degrees of arc along the folded edges
    assert ang.max() < 25.0, ang.max()
    assert np.median(ang) < 6.0
    # the map reaches most bins (the square's corners are thin slivers)
    assert len(set((qu + nb * qv).tolist())) > 0.8 * nb * nb


def test_position_jitter_closed_form_frequencies(orc):
    # normal +y: the tangent frame of Duff et al. gives t = +x, b = -z, so the
    # lookup moves by cell * (xi0, 0, -xi1) with xi uniform in [-1/2, 1/2).
    # From fractional position (0.2, 0.9) in its cell the lookup lands one
    # cell lower in x with probability 0.3 and one higher in z with 0.4.
    s, o = _oracle(orc, jitter=1.0)
    d = s.params["grid_dims"]
    cell = 1.0 / d[0]
    x = np.array([[(2 + 0.2) * cell, 0.5 * cell, (3 + 0.9) * cell]], np.float32)
    n = np.array([[0.0, 1.0, 0.0]], np.float32)
    spp = 64
    lins = np.concatenate([_keys(o, x, n, spp, f) for f in range(40)])
    ix, iy, iz, _, _ = _split(lins, d, 1)
    assert np.all(iy == 0)
    cnt = np.array([np.sum((ix == a) & (iz == b)) for a, b in ((2, 3), (1, 3), (2, 4), (1, 4))])
    assert cnt.sum() == lins.size
    p = np.array([0.7 * 0.6, 0.3 * 0.6, 0.7 * 0.4, 0.3 * 0.4])
    assert stats.chisquare(cnt, p * lins.size).pvalue > 1e-4, cnt


def test_normal_jitter_splits_a_boundary_normal_evenly(orc):
    # normal +z sits on the corner of four bins at (1/2, 1/2); a jitter of one
    # bin sends it to each with probability 1/4.  The point is at its cell's
    # centre, where a position jitter of one cell never leaves the cell.
    nb = 4
    s, o = _oracle(orc, normal_bits=2, jitter=1.0)
    d = s.params["grid_dims"]
    cell = 1.0 / d[0]
    x = np.array([[2.5 * cell, 3.5 * cell, 4.5 * cell]], np.float32)
    n = np.array([[0.0, 0.0, 1.0]], np.float32)
    lins = np.concatenate([_keys(o, x, n, 64, f) for f in range(40)])
    ix, iy, iz, qu, qv = _split(lins, d, nb)
    assert np.all(ix == 2) and np.all(iy == 3) and np.all(iz == 4)
    cnt = np.array([np.sum((qu == a) & (qv == b)) for a in (1, 2) for b in (1, 2)])
    assert cnt.sum() == lins.size
    assert stats.chisquare(cnt).pvalue > 1e-4, cnt


def test_estimator_unbiased_with_5d_jittered_cells(orc):
    s = _below_lights(scenes.make_tiny(n_lights=96, n_points=24, n_boxes=0, M=8, spp=8, normal_bits=2,
                                       jitter=1.0))
    o = orc.Oracle(s.params, s.tri, s.emit)
    frames = o.run(s.pos, s.nrm, 8, 300)
    mean, se = _mean_and_se(frames[20:])
    truth = o.truth_unoccluded(s.pos, s.nrm)
    z = (mean - truth) / np.maximum(se, 1e-12)
    assert np.max(np.abs(z)) < 5.0, np.max(np.abs(z))
    assert abs(float(np.mean(z))) < 0.5
    # more cells than position cells alone: normals and jitter split them
    assert o.num_cells() > len(set(o.cell_keys(s.pos).tolist()))
