"""Batched passes (one persistent kernel for several scenes, replayed from a
hipGraph) give exactly the results of running each scene on its own, which
the oracle parity tests pin; every schedule the autotuner may pick does."""
import numpy as np
import pytest

from paper_1911_10217_amd import scenes

pytestmark = pytest.mark.gpu


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


def _ctx(torch, s):
    from paper_1911_10217_amd import rlc
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ctx = rlc.Context(s.params)
    ctx.rlc_build_light_tree(t(s.tri), t(s.emit))
    ctx.rlc_set_occluders(t(s.boxes) if s.K else None)
    return ctx, t(s.pos), t(s.nrm)


SCHEDULES = [
    dict(tile=256, blocks_per_cu=4, dynamic=0, cell_sorted=0),
    dict(tile=512, blocks_per_cu=8, dynamic=1, cell_sorted=0),
    dict(tile=1024, blocks_per_cu=16, dynamic=1, cell_sorted=1),
    dict(tile=2048, blocks_per_cu=4, dynamic=0, cell_sorted=1),
]


def test_batch_equals_single_scenes(torch):
    from paper_1911_10217_amd import rlc
    sc = _scenes()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        batch_side = [_ctx(torch, s) for s in sc]
        single_side = [_ctx(torch, s) for s in sc]
        batch = rlc.Batch([(c, p, n, s.params["spp"]) for (c, p, n), s in zip(batch_side, sc)], st)
        for sched in SCHEDULES:
            batch.rlc_batch_set_schedule(**sched)
            assert batch.rlc_batch_get_schedule() == sched
            for (c, _, _), (d, _, _) in zip(batch_side, single_side):
                c.rlc_reset_cells()
                d.rlc_reset_cells()
            for f in range(5):
                rads = batch.rlc_batch_frame(f)
                for i, ((c, p, n), (d, pd, nd), s) in enumerate(zip(batch_side, single_side, sc)):
                    ref = d.rlc_frame(pd, nd, s.params["spp"], f)
                    assert torch.equal(rads[i], ref), (sched, f, i)
                # eager work between graph replays
                g = [c.rlc_dump_cells() for c, _, _ in batch_side]
                o = [d.rlc_dump_cells() for d, _, _ in single_side]
                for gi, oi in zip(g, o):
                    for k in gi:
                        assert np.array_equal(gi[k], oi[k]), (sched, f, k)
        batch.close()
        st.synchronize()


def test_batch_frames_out_of_order_and_emission_changes(torch):
    from paper_1911_10217_amd import rlc
    dyn = scenes.make_dynamic(n_points=2048, per_cluster=128, grid=2, n_bricks=256, M=16)
    tiny = scenes.make_tiny(n_points=1024, spp=1)
    # a cut of more than 64 clusters, over 5-D cells with jittered lookups
    wide = scenes.make_tiny(n_points=512, spp=1, M=128, normal_bits=2, jitter=1.0)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        a = [_ctx(torch, s) for s in (dyn, tiny, wide)]
        b = [_ctx(torch, s) for s in (dyn, tiny, wide)]
        batch = rlc.Batch([(c, p, n, 1) for c, p, n in a], st)
        for f in (0, 1, 2, 7, 8, 3):
            e = torch.from_numpy(dyn.emission_at(f)).cuda()
            a[0][0].rlc_set_emission(e)
            b[0][0].rlc_set_emission(e)
            rads = batch.rlc_batch_frame(f)
            for i, (d, pd, nd) in enumerate(b):
                assert torch.equal(rads[i], d.rlc_frame(pd, nd, 1, f)), (f, i)
        batch.close()


def test_autotune_picks_a_candidate_and_resets(torch):
    from paper_1911_10217_amd import rlc
    sc = _scenes()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        side = [_ctx(torch, s) for s in sc]
        batch = rlc.Batch([(c, p, n, s.params["spp"]) for (c, p, n), s in zip(side, sc)], st)
        best, cands = batch.rlc_batch_autotune(passes=2)
        assert len(cands) == 48 and all(ms > 0 for _, ms in cands)
        assert best == min(cands, key=lambda x: x[1])[0]
        assert batch.rlc_batch_get_schedule() == best
        # cells were reset: the next pass equals a fresh single-scene pass
        ref = [_ctx(torch, s) for s in sc]
        rads = batch.rlc_batch_frame(0)
        for i, ((d, pd, nd), s) in enumerate(zip(ref, sc)):
            assert torch.equal(rads[i], d.rlc_frame(pd, nd, s.params["spp"], 0))
        batch.close()


def test_batch_rejects_default_stream(torch):
    from paper_1911_10217_amd import rlc
    s = scenes.make_tiny(n_points=256)
    c, p, n = _ctx(torch, s)
    with pytest.raises(rlc.RLCError):
        rlc.Batch([(c, p, n, 1)], torch.cuda.default_stream())
