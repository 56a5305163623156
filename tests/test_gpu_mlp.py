"""The learned proposal on the GPU, through the C ABI, against the oracle.

The forward pass and the gradient are compared element by element with the
oracle's FP64 evaluation that rounds to BF16 where the kernels hold BF16
values: at least 99.9% of the entries within 1e-4 relative error (relative
to the entry, or to 1e-3 of the tensor's largest entry when that is
larger), and every entry within one BF16 rounding step (2^-8 relative): the
kernels sum in FP32 in another order, so a value that the oracle rounds to
BF16 next to a rounding boundary may land one BF16 step away.  Adam
training is compared per tensor.  The mixture pass is compared exactly
(cells) and to 1e-4 (radiance) with both sides reading the same cdf table,
an input of the test."""
import math

import numpy as np
import pytest

from paper_1911_10217_amd import scenes

pytestmark = pytest.mark.gpu

IN, H, OUT = 144, 64, 64


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for nin, nout in ((IN, H), (H, H), (H, H), (H, OUT)):
        parts.append(rng.normal(0, scale * math.sqrt(2.0 / nin), size=nout * nin))
        parts.append(rng.normal(0, 0.1, size=nout))
    return np.concatenate(parts).astype(np.float32)


def _tensors(params):
    off, out = 0, []
    for nin, nout in ((IN, H), (H, H), (H, H), (H, OUT)):
        out.append(("W", params[off:off + nin * nout]))
        off += nin * nout
        out.append(("b", params[off:off + nout]))
        off += nout
    return out


def _rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def _elementwise(gpu, ref, what, rtol=1e-4, frac=0.999, flip=2.0 ** -8, floor=1e-3):
    """|gpu - ref| <= rtol max(|ref|, floor max|ref|) for at least `frac` of
    the entries, and <= flip max(|ref|, floor max|ref|) for all of them."""
    a = np.asarray(gpu, np.float64).reshape(-1)
    b = np.asarray(ref, np.float64).reshape(-1)
    scale = np.maximum(np.abs(b), floor * np.abs(b).max())
    r = np.abs(a - b) / np.maximum(scale, 1e-300)
    assert (r <= rtol).mean() >= frac, (what, float((r <= rtol).mean()), float(r.max()))
    assert r.max() <= flip, (what, float(r.max()))


def _ctx(torch, s):
    from paper_1911_10217_amd import rlc
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ctx = rlc.Context(s.params)
    ctx.rlc_build_light_tree(t(s.tri), t(s.emit))
    ctx.rlc_set_occluders(t(s.boxes) if s.K else None)
    return ctx, t(s.pos), t(s.nrm)


def _encode(orc, s):
    p = s.params
    return orc.mlp_encode(s.pos, s.nrm, p["grid_lo"], p["grid_hi"])


@pytest.mark.parametrize("P", [1, 17, 1000])
def test_forward_matches_oracle(torch, orc, P):
    s = scenes.make_tiny(n_lights=300, n_points=P)
    ctx, pos, nrm = _ctx(torch, s)
    params = _rand_params(1)
    ctx.rlc_mlp_set_params(torch.from_numpy(params).cuda())
    cdf, z = ctx.rlc_mlp_forward(pos, nrm, cdf=True, logits=True)
    z = z.cpu().numpy()
    cdf = cdf.cpu().numpy()
    zo, qo = orc.mlp_forward(params.astype(np.float64), _encode(orc, s), bf16=True)
    _elementwise(z, zo, "logits")
    # the table is the running sum of the probabilities, ending at 1
    assert (np.diff(cdf, axis=1) >= 0).all()
    assert np.allclose(cdf[:, -1], 1.0, atol=2e-5)
    q = np.diff(np.concatenate([np.zeros((P, 1), np.float32), cdf], 1), axis=1)
    # differences of FP32 running sums: absolute error up to a few ulp of 1
    assert np.abs(q - qo).max() < 1e-5
    _elementwise(q, qo, "probabilities")


def test_gradient_matches_oracle(torch, orc):
    s = scenes.make_tiny(n_lights=300, n_points=500)
    ctx, pos, nrm = _ctx(torch, s)
    params = _rand_params(2)
    ctx.rlc_mlp_set_params(torch.from_numpy(params).cuda())
    rng = np.random.default_rng(3)
    n = 301  # four full blocks of 64 tuples and a ragged one
    pid = rng.integers(0, s.P, n).astype(np.int32)
    node = rng.integers(0, 64, n).astype(np.int32)
    w = rng.exponential(size=n).astype(np.float32)
    w[::7] = 0.0
    g = lambda a: torch.from_numpy(a).cuda()
    loss, grad = ctx.rlc_mlp_grad(pos, nrm, g(pid), g(node), g(w))
    grad = grad.cpu().numpy()
    x = _encode(orc, s)
    lo, go = orc.mlp_loss_grad(params.astype(np.float64), x[pid], node.astype(np.uint32), w.astype(np.float64),
                               bf16=True)
    assert loss == pytest.approx(lo, rel=1e-5)
    _elementwise(grad, go, "gradient")
    for i, ((kind, a), (_, b)) in enumerate(zip(_tensors(grad), _tensors(go))):
        _elementwise(a, b, "%s%d" % (kind, i // 2 + 1), frac=0.99)
    # no tuples, or only zero weights: zero gradient
    z = np.zeros(5, np.float32)
    loss0, g0 = ctx.rlc_mlp_grad(pos, nrm, g(pid[:5]), g(node[:5]), g(z))
    assert loss0 == 0.0 and not g0.cpu().numpy().any()


def test_gradient_rejects_bad_tuples(torch):
    from paper_1911_10217_amd import rlc
    s = scenes.make_tiny(n_lights=100, n_points=50)
    ctx, pos, nrm = _ctx(torch, s)
    ctx.rlc_mlp_init(7)
    g = lambda a: torch.tensor(a).cuda()
    with pytest.raises(rlc.RLCError):
        ctx.rlc_mlp_grad(pos, nrm, g(np.int32([0, 50])), g(np.int32([0, 1])), g(np.float32([1, 1])))
    with pytest.raises(rlc.RLCError):
        ctx.rlc_mlp_grad(pos, nrm, g(np.int32([0, 1])), g(np.int32([0, 64])), g(np.float32([1, 1])))
    # the context still works afterwards
    ctx.rlc_mlp_grad(pos, nrm, g(np.int32([0, 1])), g(np.int32([0, 63])), g(np.float32([1, 2])))


def test_training_matches_oracle(torch, orc):
    """Several epochs of shuffled minibatches with a ragged last batch: the
    same tuple order (Philox keys) and the same Adam steps on both sides."""
    s = scenes.make_tiny(n_lights=300, n_points=200)
    ctx, pos, nrm = _ctx(torch, s)
    params = _rand_params(4)
    ctx.rlc_mlp_set_params(torch.from_numpy(params).cuda())
    rng = np.random.default_rng(5)
    n = 700
    pid = rng.integers(0, s.P, n).astype(np.int32)
    node = (pid % 64).astype(np.int32)
    w = rng.exponential(size=n).astype(np.float32)
    g = lambda a: torch.from_numpy(a).cuda()
    loss = ctx.rlc_mlp_train(pos, nrm, g(pid), g(node), g(w), epochs=3, batch=256, lr=1e-3)
    got = ctx.rlc_mlp_get_params().cpu().numpy()
    po = params.astype(np.float64)
    m, v = np.zeros_like(po), np.zeros_like(po)
    step, lo = orc.mlp_train(po, m, v, 0, _encode(orc, s), pid.astype(np.uint32), node.astype(np.uint32),
                             w.astype(np.float64), epochs=3, batch=256, lr=1e-3, scene_id=s.params["scene_id"],
                             seed=s.params["seed"], bf16=True)
    assert step == 9
    assert loss == pytest.approx(lo, rel=2e-2)
    d_gpu = got.astype(np.float64) - params
    d_orc = po - params
    # Adam moves every weight by about lr per step; sign flips of tiny
    # gradients make single weights differ, the bulk must agree
    for (kind, a), (_, b) in zip(_tensors(d_gpu), _tensors(d_orc)):
        assert _rel_l2(a, b) < 0.1, kind
    assert np.mean(np.abs(d_gpu - d_orc) > 3e-3) < 0.02


@pytest.mark.parametrize("n", [1, 5, 16, 17, 700, 65537, 524288])
def test_epoch_order_matches_oracle(torch, orc, n):
    """The tuple order of training epochs, bit for bit: sizes that need no
    cycle walk (powers of four), sizes just past one, a ragged size, the
    learned workload's 524,288 tuples."""
    s = scenes.make_tiny(n_lights=64, n_points=16, scene_id=5)
    ctx, _, _ = _ctx(torch, s)
    for e in (0, 3):
        got = ctx.rlc_mlp_order(n, e).cpu().numpy().astype(np.uint32)
        want = orc.mlp_shuffle(n, e, s.params["scene_id"], s.params["seed"])
        assert np.array_equal(got, want), e


def test_training_is_deterministic_and_can_be_asynchronous(torch):
    s = scenes.make_tiny(n_lights=300, n_points=100)
    ctx, pos, nrm = _ctx(torch, s)
    rng = np.random.default_rng(9)
    n = 500
    g = lambda a: torch.from_numpy(a).cuda()
    pid = g(rng.integers(0, s.P, n).astype(np.int32))
    node = g(rng.integers(0, 64, n).astype(np.int32))
    w = g(rng.exponential(size=n).astype(np.float32))
    ctx.rlc_mlp_init(5)
    ctx.rlc_mlp_train(pos, nrm, pid, node, w, epochs=2, batch=128, lr=1e-2)
    a = ctx.rlc_mlp_get_params().cpu().numpy()
    ctx.rlc_mlp_init(5)
    assert ctx.rlc_mlp_train(pos, nrm, pid, node, w, epochs=2, batch=128, lr=1e-2, sync=False) is None
    ctx.rlc_sync()
    b = ctx.rlc_mlp_get_params().cpu().numpy()
    assert np.array_equal(a, b)
    # a bad tuple in an asynchronous call is reported by the next synchronising call
    from paper_1911_10217_amd import rlc
    bad = g(np.full(n, 64, np.int32))
    ctx.rlc_mlp_train(pos, nrm, pid, bad, w, epochs=1, batch=128, lr=1e-2, sync=False)
    with pytest.raises(rlc.RLCError):
        ctx.rlc_sync()
    ctx.rlc_sync()


def test_copy_params_from_a_context_on_another_stream(torch):
    """A network trained on a side stream serves a context on the main
    stream: the copy waits for the training without a host synchronisation
    and gives the same weights and the same forward pass."""
    from paper_1911_10217_amd import rlc
    s = scenes.make_tiny(n_lights=300, n_points=200)
    a, pos, nrm = _ctx(torch, s)
    rng = np.random.default_rng(8)
    n = 3000
    g = lambda x: torch.from_numpy(x).cuda()
    pid = g(rng.integers(0, s.P, n).astype(np.int32))
    node = g(rng.integers(0, 64, n).astype(np.int32))
    w = g(rng.exponential(size=n).astype(np.float32))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b, _, _ = _ctx(torch, s)
        b.rlc_mlp_init(7)
        b.rlc_mlp_train(pos, nrm, pid, node, w, epochs=3, batch=512, lr=1e-2, sync=False)
    with pytest.raises(rlc.RLCError) as e:
        a.rlc_mlp_copy_params(a)
    assert e.value.code == rlc.RLC_EINVAL
    a.rlc_mlp_copy_params(b)
    qa = a.rlc_mlp_forward(pos, nrm, cdf=True)[0]
    pa = a.rlc_mlp_get_params()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        pb = b.rlc_mlp_get_params()
        qb = b.rlc_mlp_forward(pos, nrm, cdf=True)[0]
    torch.cuda.synchronize()
    assert torch.equal(pa, pb) and torch.equal(qa, qb)
    fresh, _, _ = _ctx(torch, s)
    with pytest.raises(rlc.RLCError) as e:
        a.rlc_mlp_copy_params(fresh)
    assert e.value.code == rlc.RLC_ESTATE


def test_init_is_seeded_and_bounded(torch):
    s = scenes.make_tiny(n_lights=100, n_points=50)
    ctx, pos, nrm = _ctx(torch, s)
    ctx.rlc_mlp_init(11)
    a = ctx.rlc_mlp_get_params().cpu().numpy()
    ctx.rlc_mlp_init(11)
    b = ctx.rlc_mlp_get_params().cpu().numpy()
    ctx.rlc_mlp_init(12)
    c = ctx.rlc_mlp_get_params().cpu().numpy()
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    for (kind, t), nin in zip(_tensors(a), (IN, IN, H, H, H, H, H, H)):
        if kind == "b":
            assert not t.any()
        else:
            bound = math.sqrt(6.0 / nin)
            assert np.abs(t).max() <= bound and abs(t.mean()) < 0.05 * bound
            assert abs(t.std() - bound / math.sqrt(3)) < 0.05 * bound


def _cdf_input(P, seed, sharp=3.0):
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(P, 64)) * sharp
    q = np.exp(z - z.max(1, keepdims=True))
    return q / q.sum(1, keepdims=True)


@pytest.mark.parametrize("w", [0.5, 0.0, 0.9])
def test_mixture_frames_match_oracle(torch, orc, w):
    """w is the network's share; w = 0 is the plain method on both sides."""
    s = scenes.make_tiny(n_lights=500, n_points=1000, spp=4, M=16)
    ctx, pos, nrm = _ctx(torch, s)
    o = orc.Oracle(s.params, s.tri, s.emit, s.boxes)
    assert np.array_equal(ctx.rlc_mlp_fixed_cut()[1], o.fixed_cut()[1])
    cdf = orc.mlp_cdf(_cdf_input(s.P, 6))
    o.set_mixture(cdf, w)
    ctx.rlc_set_mixture(torch.from_numpy(cdf).cuda(), w)
    n = s.P * 4
    lp = torch.zeros(n, dtype=torch.int32, device="cuda")
    ln = torch.zeros(n, dtype=torch.int32, device="cuda")
    lw = torch.zeros(n, dtype=torch.float32, device="cuda")
    ctx.rlc_set_sample_log(lp, ln, lw)
    for f in range(4):
        rad = ctx.rlc_frame(pos, nrm, 4, f).cpu().numpy()
        ro, rec = o.frame(s.pos, s.nrm, 4, f, records=True)
        o.adapt()
        # the per-point sums run in sample order (spp a power of two): exact
        assert np.array_equal(rad, ro), f
        assert np.array_equal(ln.cpu().numpy(), rec["fnode"].astype(np.int32)), f
        assert np.array_equal(lp.cpu().numpy(), np.repeat(np.arange(s.P), 4)), f
        assert np.allclose(lw.cpu().numpy(), rec["weight"], rtol=1e-4, atol=1e-7), f
        g = ctx.rlc_dump_cells()
        c = o.cells()
        assert np.array_equal(g["key"], c["key"]) and np.array_equal(g["ready"], c["ready"]), f
        # a cell whose pass held no draws from its cut keeps sampling from the
        # initial cut; its table is compared once it has one
        r = g["ready"] == 1
        assert r.any()
        for k in ("node", "end", "Q", "Qt", "C"):
            assert np.array_equal(g[k][r], c[k][r]), (f, k)
    ctx.rlc_set_sample_log()
    ctx.rlc_set_mixture()


def test_mixture_split_calls_match_fused(torch, orc):
    """rlc_sample / rlc_shade / rlc_learn with the mixture: same draws as the
    oracle, and learning skips the proposal's draws."""
    s = scenes.make_tiny(n_lights=400, n_points=600, spp=2, M=16)
    ctx, pos, nrm = _ctx(torch, s)
    o = orc.Oracle(s.params, s.tri, s.emit, s.boxes)
    cdf = orc.mlp_cdf(_cdf_input(s.P, 8))
    o.set_mixture(cdf, 0.5)
    ctx.rlc_set_mixture(torch.from_numpy(cdf).cuda(), 0.5)
    smp = ctx.rlc_sample(pos, nrm, 2, 0)
    rad, contrib, reward = ctx.rlc_shade(pos, nrm, 2, smp)
    ctx.rlc_learn(smp, reward)
    ctx.rlc_adapt_cuts()
    ro, rec = o.frame(s.pos, s.nrm, 2, 0, records=True)
    o.adapt()
    assert np.array_equal(smp["light"].cpu().numpy(), rec["light"].astype(np.int32))
    assert np.array_equal(smp["comp"].cpu().numpy(), rec["comp"].astype(np.int32))
    assert np.allclose(smp["inv_pdf"].cpu().numpy(), rec["inv_pdf"], rtol=1e-6)
    assert np.allclose(rad.cpu().numpy(), ro, rtol=1e-4, atol=1e-7)
    g = ctx.rlc_dump_cells()
    c = o.cells()
    assert np.array_equal(g["ready"], c["ready"])
    r = g["ready"] == 1
    for k in ("node", "Q", "C"):
        assert np.array_equal(g[k][r], c[k][r]), k
    # learning without the component records is refused while mixing
    from paper_1911_10217_amd import rlc
    smp.pop("comp")
    with pytest.raises(rlc.RLCError):
        ctx.rlc_learn(smp, reward)


def test_mixture_rejects_short_tables(torch):
    from paper_1911_10217_amd import rlc
    s = scenes.make_tiny(n_lights=100, n_points=64, spp=1)
    ctx, pos, nrm = _ctx(torch, s)
    ctx.rlc_set_mixture(torch.ones((10, 64), device="cuda"), 0.5)
    with pytest.raises(rlc.RLCError):
        ctx.rlc_frame(pos, nrm, 1, 0)
    ctx.rlc_set_mixture()
    # the network alone (w = 1) may give a light density 0: refused
    for w in (1.0, 1.5, -0.1, float("nan")):
        with pytest.raises(rlc.RLCError):
            ctx.rlc_set_mixture(torch.ones((64, 64), device="cuda"), w)
    lp = torch.zeros(10, dtype=torch.int32, device="cuda")
    ctx.rlc_set_sample_log(lp, lp.clone(), torch.zeros(10, device="cuda"))
    with pytest.raises(rlc.RLCError):
        ctx.rlc_frame(pos, nrm, 1, 0)
    ctx.rlc_set_sample_log()
    ctx.rlc_frame(pos, nrm, 1, 0)


def _clean_scene():
    """Points in the lower half facing up, eps = 0.5: every light's
    contribution is smooth and every cluster keeps a sizeable probability,
    so a z-test over a few thousand samples per point is meaningful."""
    s = scenes.make_tiny(n_lights=256, n_points=256, spp=16, M=16, n_boxes=0, eps=0.5)
    s.pos[:, 1] *= 0.5
    s.nrm[:] = np.float32([0, 1, 0])
    return s


def _log_and_train(torch, ctx, pos, nrm, P, frames=4, spp=16):
    n = P * spp
    lp = torch.zeros(frames * n, dtype=torch.int32, device="cuda")
    ln = torch.zeros(frames * n, dtype=torch.int32, device="cuda")
    lw = torch.zeros(frames * n, dtype=torch.float32, device="cuda")
    for f in range(frames):
        ctx.rlc_set_sample_log(lp[f * n:(f + 1) * n], ln[f * n:(f + 1) * n], lw[f * n:(f + 1) * n])
        ctx.rlc_frame(pos, nrm, spp, f)
    ctx.rlc_set_sample_log()
    ctx.rlc_mlp_init(3)
    ctx.rlc_mlp_train(pos, nrm, lp, ln, lw, epochs=4, batch=1024, lr=3e-3)
    cdf, _ = ctx.rlc_mlp_forward(pos, nrm)
    return cdf


def _estimates(ctx, pos, nrm, P, frames, spp=16):
    est = np.zeros((frames, P, 3))
    for f in range(frames):
        est[f] = ctx.rlc_frame(pos, nrm, spp, 100 + f).cpu().numpy()
    return est


def test_trained_mixture_is_unbiased(torch, orc):
    """End to end on the GPU: log, train, forward, render with the mixture;
    the mean over frames agrees with the closed-form irradiance (no
    occluders) in z-tests per point and over the image."""
    s = _clean_scene()
    ctx, pos, nrm = _ctx(torch, s)
    cdf = _log_and_train(torch, ctx, pos, nrm, s.P)
    ctx.rlc_set_mixture(cdf, 0.5)
    frames = 128
    est = _estimates(ctx, pos, nrm, s.P, frames)
    truth = orc.Oracle(s.params, s.tri, s.emit).truth_unoccluded(s.pos, s.nrm)
    mean = est.mean(0)
    se = est.std(0) / math.sqrt(frames)
    ok = truth > 1e-6
    z = (mean - truth) / np.maximum(se, 1e-12)
    assert np.abs(z[ok]).max() < 6.0
    Z = (mean - truth)[ok].sum() / math.sqrt((se[ok] ** 2).sum())
    assert abs(Z) < 4.0


def test_trained_mixture_reduces_variance(torch):
    """What the network gains: at equal samples, after the same logged
    passes, the 50/50 mixture's per-point variance is below the plain
    method's."""
    s = _clean_scene()
    ctx, pos, nrm = _ctx(torch, s)
    cdf = _log_and_train(torch, ctx, pos, nrm, s.P)
    plain, ppos, pnrm = _ctx(torch, s)
    for f in range(4):
        plain.rlc_frame(ppos, pnrm, 16, f)
    ctx.rlc_set_mixture(cdf, 0.5)
    frames = 64
    vm = _estimates(ctx, pos, nrm, s.P, frames).var(0).sum(1)
    vp = _estimates(plain, ppos, pnrm, s.P, frames).var(0).sum(1)
    ok = vp > 0
    assert np.median(vm[ok] / vp[ok]) < 0.85
    assert vm.sum() < 0.85 * vp.sum()
