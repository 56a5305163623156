"""Batched passes (one persistent kernel for several scenes, replayed from a
hipGraph) against the oracle: every scene of a batch gives, pass after pass,
the oracle's radiance and cell tables bit for bit, for every schedule the
autotuner may pick, for frames out of order with changing emission, and for
a scene at the batched workload's largest sizes (about 1M emitters and 2M
points, checked on sampled cells: cells learn independently, so the oracle
runs only their points)."""
import numpy as np
import pytest

import oracle
from paper_1911_10217_amd import scenes

pytestmark = pytest.mark.gpu

FRAMES = 5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _scenes():
    return [
        scenes.make_tiny(n_points=3000, spp=1, M=16),
        scenes.make_tiny(n_lights=2000, n_points=5003, spp=2, M=32, seed=scenes.SEED_BASE + 11, hashed=1,
                         capacity=4096),
        scenes.make_static(width=160, height=90, capacity=1 << 14),
        scenes.make_tiny(n_lights=7, n_points=700, n_boxes=5, spp=4, M=16, seed=scenes.SEED_BASE + 12),
    ]


@pytest.fixture(scope="module")
def small_batch():
    """The scenes, and each one's oracle run: radiance and cells after every
    pass of frames 0..FRAMES-1 from a fresh cell table."""
    sc = _scenes()
    runs = []
    for s in sc:
        o = oracle.Oracle(s.params, s.tri, s.emit, s.boxes)
        rads, cells = [], []
        for f in range(FRAMES):
            r, _ = o.frame(s.pos, s.nrm, s.params["spp"], f)
            o.adapt()
            rads.append(r)
            cells.append(o.cells())
        runs.append((rads, cells))
    return sc, runs


def _ctx(torch, s):
    from paper_1911_10217_amd import rlc
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ctx = rlc.Context(s.params)
    ctx.rlc_build_light_tree(t(s.tri), t(s.emit))
    ctx.rlc_set_occluders(t(s.boxes) if s.K else None)
    return ctx, t(s.pos), t(s.nrm)


def _assert_cells(g, o, where, keys=None):
    if keys is not None:
        gi = np.searchsorted(g["key"], keys)
        oi = np.searchsorted(o["key"], keys)
        assert np.array_equal(g["key"][gi], keys) and np.array_equal(o["key"][oi], keys), where
        g = {k: v[gi] for k, v in g.items()}
        o = {k: v[oi] for k, v in o.items()}
    assert np.array_equal(g["key"], o["key"]), (where, "cell sets differ")
    for k in ("ready", "node", "end", "Q", "Qt", "C", "sum", "cnt"):
        assert np.array_equal(g[k], o[k]), (where, k)


SCHEDULES = [
    dict(tile=256, blocks_per_cu=4, dynamic=0, cell_sorted=0),
    dict(tile=512, blocks_per_cu=8, dynamic=1, cell_sorted=0),
    dict(tile=1024, blocks_per_cu=16, dynamic=1, cell_sorted=1),
    dict(tile=2048, blocks_per_cu=4, dynamic=0, cell_sorted=1),
]


def test_batch_matches_oracle_every_schedule(torch, small_batch):
    """Every schedule, every pass: each scene's radiance (its spp is a power
    of two, so sums run in sample order) and its whole cell table equal the
    oracle's; the dumps between replays are eager work on the stream."""
    from paper_1911_10217_amd import rlc
    sc, runs = small_batch
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        side = [_ctx(torch, s) for s in sc]
        batch = rlc.Batch([(c, p, n, s.params["spp"]) for (c, p, n), s in zip(side, sc)], st)
        for sched in SCHEDULES:
            batch.rlc_batch_set_schedule(**sched)
            assert batch.rlc_batch_get_schedule() == sched
            for c, _, _ in side:
                c.rlc_reset_cells()
            for f in range(FRAMES):
                rads = batch.rlc_batch_frame(f)
                for i, (rads_o, cells_o) in enumerate(runs):
                    assert np.array_equal(rads[i].cpu().numpy(), rads_o[f]), (sched, f, i)
                    _assert_cells(side[i][0].rlc_dump_cells(), cells_o[f], (sched, f, i))
        batch.close()
        st.synchronize()


def test_batch_frames_out_of_order_and_emission_changes(torch):
    """Frames replayed out of order, the animated scene's emission set before
    each; a cut of more than 64 clusters over 5-D cells with jittered
    lookups.  Each scene equals the oracle run in the same order."""
    from paper_1911_10217_amd import rlc
    dyn = scenes.make_dynamic(n_points=2048, per_cluster=128, grid=2, n_bricks=256, M=16)
    tiny = scenes.make_tiny(n_points=1024, spp=1)
    wide = scenes.make_tiny(n_points=512, spp=1, M=128, normal_bits=2, jitter=1.0)
    sc = (dyn, tiny, wide)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        a = [_ctx(torch, s) for s in sc]
        orcs = [oracle.Oracle(s.params, s.tri, s.emit, s.boxes) for s in sc]
        batch = rlc.Batch([(c, p, n, 1) for c, p, n in a], st)
        for f in (0, 1, 2, 7, 8, 3):
            e = dyn.emission_at(f)
            a[0][0].rlc_set_emission(torch.from_numpy(e).cuda())
            orcs[0].set_emission(e)
            rads = batch.rlc_batch_frame(f)
            for i, (s, o) in enumerate(zip(sc, orcs)):
                ref, _ = o.frame(s.pos, s.nrm, 1, f)
                o.adapt()
                assert np.array_equal(rads[i].cpu().numpy(), ref), (f, i)
                _assert_cells(a[i][0].rlc_dump_cells(), o.cells(), (f, i))
        batch.close()


@pytest.mark.parametrize("n_scenes", [16, 17])
def test_batch_of_many_small_scenes(torch, n_scenes):
    """Batches at the edge of the 16-cell end-of-pass kernel (cells of up to
    16 scenes over one index space; cuts of 16, 32 and 64 clusters side by
    side, so the serial phase's lanes run cuts of different lengths; row
    pools of one stripe and of eight) and one scene past it, which takes the
    one-wave kernel scene after scene; one scene has few points and seven
    lights.  Every scene equals the oracle after every pass."""
    from paper_1911_10217_amd import rlc
    sc = []
    for i in range(n_scenes):
        M = (16, 32, 64)[i % 3]
        n_lights = 7 if i == 5 else 200 + 37 * i
        sc.append(scenes.make_tiny(n_lights=n_lights, n_points=64 if i == 5 else 400 + 50 * i, n_boxes=8, M=M,
                                   spp=1, seed=scenes.SEED_BASE + 100 + i, scene_id=i, hashed=1,
                                   capacity=8192 if i % 2 == 0 else 1024, max_cells=8192 if i % 2 == 0 else 512))
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        a = [_ctx(torch, s) for s in sc]
        orcs = [oracle.Oracle(s.params, s.tri, s.emit, s.boxes) for s in sc]
        batch = rlc.Batch([(c, p, n, 1) for c, p, n in a], st)
        for f in range(3):
            rads = batch.rlc_batch_frame(f)
            for i, (s, o) in enumerate(zip(sc, orcs)):
                ref, _ = o.frame(s.pos, s.nrm, 1, f)
                o.adapt()
                assert np.array_equal(rads[i].cpu().numpy(), ref), (n_scenes, f, i)
                _assert_cells(a[i][0].rlc_dump_cells(), o.cells(), (n_scenes, f, i))
        batch.close()
        for c, _, _ in a:
            c.close()


def test_batch_recaptures_after_rebuilds_and_guards_destroy(torch):
    """Rebuilding a scene's occluders or light tree frees the buffers the
    captured graph points at: the next batch pass captures again from the
    current ones (results equal the oracle restarted from a fresh table, as
    a tree rebuild resets the cells).  A context cannot be destroyed while a
    batch refers to it."""
    from paper_1911_10217_amd import rlc
    s = scenes.make_tiny(n_points=2000, spp=1, M=16)
    u = scenes.make_tiny(n_points=900, spp=1, M=16, seed=scenes.SEED_BASE + 13)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        (c0, p0, n0), (c1, p1, n1) = _ctx(torch, s), _ctx(torch, u)
        batch = rlc.Batch([(c0, p0, n0, 1), (c1, p1, n1, 1)], st)
        o = oracle.Oracle(s.params, s.tri, s.emit, s.boxes)
        for f in range(2):
            r = batch.rlc_batch_frame(f)
            ref, _ = o.frame(s.pos, s.nrm, 1, f)
            o.adapt()
            assert np.array_equal(r[0].cpu().numpy(), ref)
        # same boxes, new buffers: the cells keep learning
        c0.rlc_set_occluders(t(s.boxes))
        r = batch.rlc_batch_frame(2)
        ref, _ = o.frame(s.pos, s.nrm, 1, 2)
        o.adapt()
        assert np.array_equal(r[0].cpu().numpy(), ref)
        _assert_cells(c0.rlc_dump_cells(), o.cells(), "after occluders")
        # a new tree resets the cells
        c0.rlc_build_light_tree(t(s.tri), t(s.emit))
        o = oracle.Oracle(s.params, s.tri, s.emit, s.boxes)
        for f in (3, 4):
            r = batch.rlc_batch_frame(f)
            ref, _ = o.frame(s.pos, s.nrm, 1, f)
            o.adapt()
            assert np.array_equal(r[0].cpu().numpy(), ref), f
        _assert_cells(c0.rlc_dump_cells(), o.cells(), "after tree")
        with pytest.raises(rlc.RLCError) as e:
            c1.close()
        assert e.value.code == rlc.RLC_ESTATE
        c1.rlc_sync()  # still alive
        batch.close()
        c1.close()
        c0.close()


def test_batch_with_a_scene_of_the_largest_batched_sizes(torch, small_batch):
    """One batch holding a scene at the top of the batched workload's ranges
    (1,048,576 emitters in 256 clusters, 2,097,152 points, 8,192 boxes, cut
    size 32) and two small scenes.  The small ones are compared whole; the
    large one on sampled cells (the three most visited and 13 random ones),
    whose points the oracle runs: radiance at those points and their cells'
    tables bit for bit after every pass."""
    from paper_1911_10217_amd import rlc
    big = scenes.make_static(width=2048, height=1024, per_cluster=4096, n_boxes=8192, M=32,
                             capacity=1 << 16, scene_id=5, seed=scenes.SEED_BASE + 40)
    assert big.N == 1 << 20 and big.P == 1 << 21
    sc, runs = small_batch
    small = [0, 3]
    o_big = oracle.Oracle(big.params, big.tri, big.emit, big.boxes)
    keys = o_big.cell_keys(big.pos)
    uniq, counts = np.unique(keys, return_counts=True)
    rng = np.random.default_rng(8)
    pick = np.unique(np.concatenate([uniq[np.argsort(counts)[-3:]], rng.choice(uniq, 13, replace=False)]))
    sel = np.nonzero(np.isin(keys, pick))[0].astype(np.uint32)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        side = [_ctx(torch, big)] + [_ctx(torch, sc[i]) for i in small]
        spp = [1] + [sc[i].params["spp"] for i in small]
        batch = rlc.Batch([(c, p, n, k) for (c, p, n), k in zip(side, spp)], st)
        batch.rlc_batch_set_schedule(tile=1024, blocks_per_cu=8, dynamic=1, cell_sorted=1)
        for f in range(4):
            rads = batch.rlc_batch_frame(f)
            ref, _ = o_big.frame(big.pos[sel], big.nrm[sel], 1, f, pid=sel)
            o_big.adapt()
            assert np.array_equal(rads[0].cpu().numpy()[sel], ref), f
            for j, i in enumerate(small):
                assert np.array_equal(rads[1 + j].cpu().numpy(), runs[i][0][f]), (f, i)
                _assert_cells(side[1 + j][0].rlc_dump_cells(), runs[i][1][f], (f, i))
        _assert_cells(side[0][0].rlc_dump_cells(), o_big.cells(), "large scene", keys=pick)
        batch.close()


def test_autotune_picks_a_candidate_and_resets(torch, small_batch):
    from paper_1911_10217_amd import rlc
    sc, runs = small_batch
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        side = [_ctx(torch, s) for s in sc]
        batch = rlc.Batch([(c, p, n, s.params["spp"]) for (c, p, n), s in zip(side, sc)], st)
        best, cands = batch.rlc_batch_autotune(passes=2)
        assert len(cands) == 48 and all(ms > 0 for _, ms in cands)
        assert best == min(cands, key=lambda x: x[1])[0]
        assert batch.rlc_batch_get_schedule() == best
        # cells were reset: the next passes equal the oracle's from a fresh table
        for f in range(2):
            rads = batch.rlc_batch_frame(f)
            for i, (rads_o, cells_o) in enumerate(runs):
                assert np.array_equal(rads[i].cpu().numpy(), rads_o[f]), (f, i)
                _assert_cells(side[i][0].rlc_dump_cells(), cells_o[f], (f, i))
        batch.close()


def test_batch_rejects_default_stream(torch):
    from paper_1911_10217_amd import rlc
    s = scenes.make_tiny(n_points=256)
    c, p, n = _ctx(torch, s)
    with pytest.raises(rlc.RLCError):
        rlc.Batch([(c, p, n, 1)], torch.cuda.default_stream())
