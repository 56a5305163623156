"""Pins of the oracle's sampling, visibility and estimator against closed
forms, brute force and the definition of the integral it estimates
(section 3: sample a cluster from the cell's cdf, a light in it, compute its
contribution; the estimate is unbiased for the direct illumination)."""
import math

import numpy as np
import pytest

from paper_1911_10217_amd import scenes


def _scene(orc, tri, emit, boxes=None, **kw):
    p = scenes.params_for(**kw)
    return orc.Oracle(p, tri, emit, boxes)


# --------------------------------------------------------------------------
# cell location
# --------------------------------------------------------------------------
def test_cell_keys_hand_cases(orc):
    s = scenes.make_tiny(n_lights=8)
    o = orc.Oracle(s.params, s.tri, s.emit)
    pts = np.array([[0, 0, 0], [0.999, 0.999, 0.999], [1.0, 1.0, 1.0], [0.13, 0.26, 0.51],
                    [-5, 0.5, 7], [0.125, 0.0, 0.0]], np.float32)
    # 8^3 grid over [0,1]^3: key = ix + 8 (iy + 8 iz)
    want = [0, 7 + 8 * (7 + 8 * 7), 511, 1 + 8 * (2 + 8 * 4), 0 + 8 * (4 + 8 * 7), 1]
    assert o.cell_keys(pts).tolist() == want


def test_cell_keys_scene_id_in_high_bits(orc):
    s = scenes.make_tiny(n_lights=8)
    p = dict(s.params, scene_id=5)
    o = orc.Oracle(p, s.tri, s.emit)
    assert o.cell_keys(np.array([[0.9, 0.0, 0.0]], np.float32))[0] == (5 << 32) | 7


# --------------------------------------------------------------------------
# visibility (slab test over every box)
# --------------------------------------------------------------------------
def test_visibility_hand_cases(orc):
    box = np.array([[0.4, 0.4, 0.4, 0.6, 0.6, 0.6]], np.float32)
    s = scenes.make_tiny(n_lights=8)
    o = orc.Oracle(s.params, s.tri, s.emit, box)
    x = np.array([[0.1, 0.5, 0.5],   # straight through the box
                  [0.1, 0.9, 0.5],   # passes above
                  [0.1, 0.5, 0.5],   # stops before the box
                  [0.5, 0.5, 0.5],   # starts inside
                  [0.1, 0.6, 0.5],   # runs inside the top face's plane (dy = 0): closed slab, occluded
                  [0.5, 0.1, 0.5],   # axis-parallel (dx = dz = 0), through
                  [0.7, 0.1, 0.5],   # axis-parallel, outside the slab in x
                  [0.6, 0.5, 0.5]],  # starts on the +x face, leaves it
                 np.float32)
    y = np.array([[0.9, 0.5, 0.5], [0.9, 0.9, 0.5], [0.35, 0.5, 0.5], [0.5, 0.9, 0.5],
                  [0.9, 0.6, 0.5], [0.5, 0.9, 0.5], [0.7, 0.9, 0.5], [0.9, 0.5, 0.5]], np.float32)
    assert o.visible(x, y).tolist() == [0, 1, 1, 0, 0, 0, 1, 1]


def test_visibility_touching_an_edge_does_not_occlude(orc):
    # dyadic coordinates: the segment meets the box only along its edge
    # x = y = 0.75, where the entry and exit parameters are both exactly 0.5
    box = np.array([[0.25, 0.25, 0.25, 0.75, 0.75, 0.75]], np.float32)
    s = scenes.make_tiny(n_lights=8)
    o = orc.Oracle(s.params, s.tri, s.emit, box)
    x = np.array([[0.5, 1.0, 0.5], [0.5, 1.0, 0.5]], np.float32)
    y = np.array([[1.0, 0.5, 0.5], [1.0, 0.25, 0.5]], np.float32)
    assert o.visible(x, y).tolist() == [1, 0]


def test_visibility_brute_force_fp64(orc):
    # every segment agrees with an FP64 point sampling along it (spacing
    # 4e-4), except where growing or shrinking the boxes by 1e-3 changes the
    # sampled answer (the segment passes that close to a box boundary)
    rng = np.random.default_rng(5)
    boxes = scenes._random_boxes(rng, 48, 0.0, 1.0, 0.05, 0.25)
    s = scenes.make_tiny(n_lights=8)
    o = orc.Oracle(s.params, s.tri, s.emit, boxes)
    n = 400
    x = rng.random((n, 3)).astype(np.float32)
    y = rng.random((n, 3)).astype(np.float32)
    vis = o.visible(x, y)
    t = np.linspace(1e-4, 1 - 1e-4, 4001)
    pts = x[:, None, :].astype(np.float64) + t[None, :, None] * (y - x)[:, None, :].astype(np.float64)
    b = boxes.astype(np.float64)

    def blocked(delta):
        hit = np.zeros(n, bool)
        for bb in b:
            ins = np.all((pts > bb[:3] - delta) & (pts < bb[3:] + delta), axis=2)
            hit |= ins.any(axis=1)
        return hit

    shrunk, grown = blocked(-1e-3), blocked(1e-3)
    clear = shrunk == grown
    assert np.all(vis[clear] == (~grown[clear]).astype(np.uint8))
    assert clear.sum() > 300 and 30 < (~grown[clear]).sum() < clear.sum() - 30


# --------------------------------------------------------------------------
# sampling from a cell's table
# --------------------------------------------------------------------------
def _balanced_scene(orc, N, M, **kw):
    pts = np.zeros((N, 3))
    pts[:, 0] = (np.arange(N) + 0.25) / N
    pts[:, 1] = 0.95
    pts[:, 2] = 0.5
    tri = np.concatenate([pts, pts + [1e-2, 0, 0], pts + [0, 0, 1e-2]], axis=1).astype(np.float32)
    return _scene(orc, tri, np.ones((N, 3), np.float32), M=M, **kw)


def test_cluster_and_light_frequencies(orc):
    o = _balanced_scene(orc, 64, 8, eps=0.0)
    node, _ = o.template()
    Q = np.array([4, 0, 1, 2, 0.5, 8, 1, 3.5], np.float32)
    o.load_cell(0, node, Q)
    n = 40000
    pos = np.full((n, 3), 0.05, np.float32)
    nrm = np.tile(np.array([0, 1, 0], np.float32), (n, 1))
    _, rec = o.frame(pos, nrm, 1, 3, records=True)
    assert np.all(rec["ready"] == 1)
    counts = np.bincount(rec["slot"], minlength=8)
    p = Q.astype(np.float64) / Q.sum()
    assert counts[1] == 0 and counts[4] > 0  # zero-probability cluster never drawn
    m = p > 0
    chi2 = float((((counts - n * p) ** 2)[m] / (n * p)[m]).sum())
    assert chi2 < 30.0, chi2  # 6 dof
    # light is uniform inside its cluster (cluster 5 = lights 40..47)
    lights = rec["light"][rec["slot"] == 5]
    assert lights.min() >= 40 and lights.max() <= 47
    h = np.bincount(lights - 40, minlength=8)
    e = lights.size / 8
    assert float(((h - e) ** 2 / e).sum()) < 30.0
    # 1/p(l) = size(s) * C[M-1] / Q~[s]
    want = 8.0 * Q.sum() / Q[rec["slot"]]
    np.testing.assert_allclose(rec["inv_pdf"], want, rtol=1e-6)


def test_light_pdf_sums_to_one(orc):
    o = _balanced_scene(orc, 64, 8, eps=0.05)
    node, _ = o.template()
    rng = np.random.default_rng(1)
    o.load_cell(0, node, rng.random(8).astype(np.float32))
    n = 20000
    pos = np.full((n, 3), 0.05, np.float32)
    nrm = np.tile(np.array([0, 1, 0], np.float32), (n, 1))
    _, rec = o.frame(pos, nrm, 1, 0, records=True)
    p_light = {}
    for l, ip in zip(rec["light"], rec["inv_pdf"]):
        p_light[int(l)] = 1.0 / float(ip)
    # every light was drawn at least once and the distinct pdfs sum to one
    assert len(p_light) == 64
    assert abs(sum(p_light.values()) - 1.0) < 1e-5


def test_single_slot_cut_is_uniform_light_selection(orc):
    s = scenes.make_tiny(n_lights=100, n_points=64, M=1, spp=4)
    o = orc.Oracle(s.params, s.tri, s.emit, s.boxes)
    _, rec = o.frame(s.pos, s.nrm, 4, 0, records=True)
    assert np.all(rec["slot"] == 0) and np.all(rec["inv_pdf"] == 100.0)
    o.adapt()
    _, rec = o.frame(s.pos, s.nrm, 4, 1, records=True)
    assert np.all(rec["slot"] == 0)
    np.testing.assert_allclose(rec["inv_pdf"], 100.0, rtol=2e-7)  # (100 C)/Q~ with C = Q~


def test_fresh_cells_sample_uniform_clusters(orc):
    s = scenes.make_tiny(n_lights=256, n_points=256, M=16, spp=2)
    o = orc.Oracle(s.params, s.tri, s.emit, s.boxes)
    node, end = o.template()
    _, rec = o.frame(s.pos, s.nrm, 2, 0, records=True)
    assert np.all(rec["ready"] == 0)
    sizes = np.diff(np.concatenate([[0], end])).astype(np.float32)
    np.testing.assert_array_equal(rec["inv_pdf"], sizes[rec["slot"]] * 16.0)


# --------------------------------------------------------------------------
# closed forms for the integral
# --------------------------------------------------------------------------
def _corner_form_factor(a, b):
    # differential area below the corner of a parallel W x H rectangle at
    # height h, a = W/h, b = H/h (standard view-factor catalogue entry)
    A = math.sqrt(1 + a * a)
    B = math.sqrt(1 + b * b)
    return (a / A * math.atan(b / A) + b / B * math.atan(a / B)) / (2 * math.pi)


def test_polygon_formula_matches_rectangle_view_factor(orc):
    # a W x H rectangle (two triangles) at height h above a point under its
    # corner; int cos cos / r^2 dA = pi * F
    W, H, h = 0.7, 0.4, 0.3
    tri = np.array([[0, h, 0, W, h, 0, W, h, H], [0, h, 0, W, h, H, 0, h, H]], np.float32)
    emit = np.ones((2, 3), np.float32)
    o = _scene(orc, tri, emit, M=2, albedo=1.0)
    x = np.array([[0, 0, 0]], np.float32)
    n = np.array([[0, 1, 0]], np.float32)
    L = o.truth_unoccluded(x, n)[0, 0]
    # L = f_r * Le * pi F = (1/pi) * pi F = F
    want = _corner_form_factor(np.float32(W) / np.float32(h), np.float32(H) / np.float32(h))
    assert abs(L - want) < 1e-6 * want


def test_polygon_formula_clips_below_horizon(orc):
    # a vertical square straddling the tangent plane: only the upper half counts
    tri = np.array([[0.2, -0.5, 1, 0.2, 0.5, 1, -0.8, 0.5, 1],
                    [0.2, -0.5, 1, -0.8, 0.5, 1, -0.8, -0.5, 1]], np.float32)
    half = np.array([[0.2, 0.0, 1, 0.2, 0.5, 1, -0.8, 0.5, 1],
                     [0.2, 0.0, 1, -0.8, 0.5, 1, -0.8, 0.0, 1]], np.float32)
    x = np.array([[0, 0, 0]], np.float32)
    n = np.array([[0, 1, 0]], np.float32)
    a = _scene(orc, tri, np.ones((2, 3), np.float32), M=2).truth_unoccluded(x, n)[0, 0]
    b = _scene(orc, half, np.ones((2, 3), np.float32), M=2).truth_unoccluded(x, n)[0, 0]
    assert abs(a - b) < 1e-9 and a > 0


def test_closed_form_matches_fp64_integration(orc):
    s = scenes.make_tiny(n_lights=32, n_points=12, n_boxes=0)
    o = orc.Oracle(s.params, s.tri, s.emit)
    cf = o.truth_unoccluded(s.pos, s.nrm)
    mc = o.truth_mc(s.pos, s.nrm, ks=48)
    np.testing.assert_allclose(mc, cf, rtol=2e-3, atol=1e-4 * float(cf.max()))


# --------------------------------------------------------------------------
# unbiasedness of the learned estimator (z-tests against the truth)
# --------------------------------------------------------------------------
def _below_lights(s):
    # points inside the emitter band see a 1/r^2 singularity (an estimator of
    # infinite variance), where a z-test is meaningless: keep them below it.
    # A larger floor eps keeps the learned pdf's tails light enough for a
    # z-test over a few hundred frames.
    s.pos[:, 1] *= 0.8
    s.params["eps"] = 0.5
    return s


def _mean_and_se(frames):
    a = np.stack(frames).astype(np.float64)
    return a.mean(axis=0), a.std(axis=0, ddof=1) / math.sqrt(a.shape[0])


def test_estimator_unbiased_unoccluded(orc):
    s = _below_lights(scenes.make_tiny(n_lights=96, n_points=24, n_boxes=0, M=8, spp=8))
    o = orc.Oracle(s.params, s.tri, s.emit)
    frames = o.run(s.pos, s.nrm, 8, 300)
    mean, se = _mean_and_se(frames[20:])  # after the cuts have adapted
    truth = o.truth_unoccluded(s.pos, s.nrm)
    z = (mean - truth) / np.maximum(se, 1e-12)
    assert np.max(np.abs(z)) < 5.0, np.max(np.abs(z))
    assert abs(float(np.mean(z))) < 0.5
    # the learned tables changed the cuts and the cluster weights
    c = o.cells()
    node, _ = o.template()
    assert np.any(c["node"] != node[None, :])


def test_estimator_unbiased_with_occluders(orc):
    s = _below_lights(scenes.make_tiny(n_lights=48, n_points=16, n_boxes=24, M=8, spp=8))
    o = orc.Oracle(s.params, s.tri, s.emit, s.boxes)
    frames = o.run(s.pos, s.nrm, 8, 300)
    mean, se = _mean_and_se(frames[20:])
    reps = np.stack([o.truth_mc(s.pos, s.nrm, ks=12, replica=r) for r in range(4)])
    truth = reps.mean(axis=0)
    se_t = reps.std(axis=0, ddof=1) / 2.0
    z = (mean - truth) / np.maximum(np.sqrt(se ** 2 + se_t ** 2), 1e-12)
    lit = truth > 1e-9
    assert np.max(np.abs(z[lit])) < 5.0, np.max(np.abs(z[lit]))
    assert np.all(np.abs(mean[~lit]) < 1e-6)


def test_cluster_total_reward_also_unbiased(orc):
    s = _below_lights(scenes.make_tiny(n_lights=96, n_points=16, n_boxes=0, M=8, spp=8, reward_mode=1))
    o = orc.Oracle(s.params, s.tri, s.emit)
    frames = o.run(s.pos, s.nrm, 8, 150)
    mean, se = _mean_and_se(frames[20:])
    truth = o.truth_unoccluded(s.pos, s.nrm)
    z = (mean - truth) / np.maximum(se, 1e-12)
    assert np.max(np.abs(z)) < 5.0


@pytest.mark.parametrize("reward_mode", [0, 1])
def test_learning_reduces_variance_under_occlusion(orc, reward_mode):
    # a roof hides 7/8 of the lights from every point: the learned cuts move
    # the samples onto the visible lights (the paper's claim, qualitatively)
    rng = np.random.default_rng(2)
    N = 256
    cen = np.empty((N, 3))
    n_vis = N // 8
    cen[:n_vis, 0] = rng.uniform(0.0, 0.2, n_vis)
    cen[n_vis:, 0] = rng.uniform(0.5, 1.0, N - n_vis)
    cen[:, 1] = rng.uniform(0.9, 0.99, N)
    cen[:, 2] = rng.uniform(0.0, 1.0, N)
    v = cen[:, None, :] + rng.uniform(-0.01, 0.01, size=(N, 3, 3))
    tri = v.reshape(N, 9).astype(np.float32)
    emit = np.ones((N, 3), np.float32)
    roof = np.array([[0.3, 0.5, -1, 2.0, 0.6, 2.0]], np.float32)
    P = 32
    pos = np.stack([rng.uniform(0.0, 0.2, P), np.full(P, 0.1), rng.uniform(0, 1, P)], axis=1).astype(np.float32)
    nrm = np.tile(np.array([0, 1, 0], np.float32), (P, 1))
    kw = dict(M=16, grid_dims=(2, 2, 2), reward_mode=reward_mode)
    learn = _scene(orc, tri, emit, roof, **kw)
    plain = _scene(orc, tri, emit, roof, temporal=0, **kw)
    fl = np.stack(learn.run(pos, nrm, 4, 80)[20:])
    fp = np.stack(plain.run(pos, nrm, 4, 80)[20:])
    var_l = fl.var(axis=0).mean()
    var_p = fp.var(axis=0).mean()
    assert var_l < 0.5 * var_p, (var_l, var_p)
    # and both estimate the same image
    assert abs(fl.mean() / fp.mean() - 1.0) < 0.15


def test_sub_frames_unbiased_and_adapted_between_passes(orc):
    # a frame split into sub-frames (section 3): the mean of its passes is
    # unbiased against the closed-form radiance, and the cuts adapt after
    # every pass, so n sub-frames learn as much as n whole frames
    s = _below_lights(scenes.make_tiny(n_lights=96, n_points=24, n_boxes=0, M=8, spp=8))
    o = orc.Oracle(s.params, s.tri, s.emit)
    frames = [o.frame_sub(s.pos, s.nrm, 8, 4, f) for f in range(75)]
    mean, se = _mean_and_se(frames[5:])
    truth = o.truth_unoccluded(s.pos, s.nrm)
    z = (mean - truth) / np.maximum(se, 1e-12)
    assert np.max(np.abs(z)) < 5.0, np.max(np.abs(z))
    assert abs(float(np.mean(z))) < 0.5
    # one sub-frame is one frame of spp / n_sub samples; the whole frame is
    # their mean in pass order
    a = orc.Oracle(s.params, s.tri, s.emit)
    b = orc.Oracle(s.params, s.tri, s.emit)
    got = a.frame_sub(s.pos, s.nrm, 8, 2, 3)
    r0, _ = b.frame(s.pos, s.nrm, 4, 6)
    b.adapt()
    r1, _ = b.frame(s.pos, s.nrm, 4, 7)
    b.adapt()
    assert np.array_equal(got, (r0 + r1) * np.float32(0.5))
    ca, cb = a.cells(), b.cells()
    for k in ("key", "node", "Q", "C"):
        assert np.array_equal(ca[k], cb[k])
    # with a single sub-frame it is the plain frame
    c = orc.Oracle(s.params, s.tri, s.emit)
    d = orc.Oracle(s.params, s.tri, s.emit)
    r, _ = d.frame(s.pos, s.nrm, 8, 5)
    d.adapt()
    assert np.array_equal(c.frame_sub(s.pos, s.nrm, 8, 1, 5), r)
