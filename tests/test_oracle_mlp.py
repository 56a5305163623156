"""Pins of the oracle's learned proposal: BF16 rounding, the sin/cos input
encoding, the 144-64-64-64-64 network's forward pass and gradient, Adam, the
training order, and the mixture of the learned distribution with the cell's
cut distribution (it must remain a proper, unbiased importance sampler).

The anchors are independent of the oracle's code: closed forms, central
finite differences, PyTorch's CPU float64 autograd and Adam, and
PyTorch's own float32 -> bfloat16 conversion."""
import math

import numpy as np
from scipy import stats
import pytest
import torch

from paper_1911_10217_amd import scenes

IN, H, OUT = 144, 64, 64


def _rand_params(rng, scale=1.0):
    """Kaiming-like random parameters in the oracle's flat layout."""
    parts = []
    for nin, nout in ((IN, H), (H, H), (H, H), (H, OUT)):
        parts.append(rng.normal(0, scale * math.sqrt(2.0 / nin), size=nout * nin))
        parts.append(rng.normal(0, 0.1, size=nout))
    return np.concatenate(parts)


def _torch_net(params):
    """The same network from PyTorch modules (float64), weights copied in."""
    p = torch.tensor(params, dtype=torch.float64)
    layers, off = [], 0
    for nin, nout in ((IN, H), (H, H), (H, H), (H, OUT)):
        W = p[off:off + nin * nout].reshape(nout, nin)
        off += nin * nout
        b = p[off:off + nout]
        off += nout
        lin = torch.nn.Linear(nin, nout, dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(W)
            lin.bias.copy_(b)
        layers += [lin, torch.nn.ReLU()]
    return torch.nn.Sequential(*layers[:-1])


def _flat_grad(net):
    out = []
    for m in net:
        if isinstance(m, torch.nn.Linear):
            out += [m.weight.grad.reshape(-1), m.bias.grad]
    return torch.cat(out).numpy()


# --------------------------------------------------------------------------
# BF16
# --------------------------------------------------------------------------
def test_bf16_round_matches_torch(orc):
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-30, 30, 5000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9 + 2 ** -30,
                         -(1.0 + 2 ** -8), 65504.0, 3.0e38, 1e-40]])
    ours = orc.bf16_round(a)
    want = torch.tensor(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, want)


def test_bf16_round_hand_cases(orc):
    r = orc.bf16_round([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.0 - 2 ** -7 - 2 ** -9])
    # ties go to the even mantissa; 2^-9 is below half an ulp at 1.0
    assert r.tolist() == [1.0, 1.0 + 2 ** -6, 1.0, -2.0 - 2 ** -6]


# --------------------------------------------------------------------------
# encoding
# --------------------------------------------------------------------------
def test_encoding_closed_forms(orc):
    lo, hi = [0.0, 0.0, 0.0], [1.0, 2.0, 4.0]
    # v = (0, 0.5, 0.25) and normal (0, 0, 1)
    x = orc.mlp_encode([[0.0, 1.0, 1.0]], [[0.0, 0.0, 1.0]], lo, hi)[0]
    assert x.shape == (144,)
    for k in range(12):
        # v = 0: sin 0, cos 1
        assert x[24 * 0 + 2 * k] == 0.0 and x[24 * 0 + 2 * k + 1] == 1.0
        # normal x = 0
        assert x[24 * 3 + 2 * k] == 0.0 and x[24 * 3 + 2 * k + 1] == 1.0
        # v = 1/2: sin(2^k pi / 2), cos(2^k pi / 2)
        s, c = [(1, 0), (0, -1)][k] if k < 2 else (0, 1)
        assert abs(x[24 * 1 + 2 * k] - s) < 1e-12 and abs(x[24 * 1 + 2 * k + 1] - c) < 1e-12
        # v = 1/4
        want = {0: (math.sqrt(0.5), math.sqrt(0.5)), 1: (1, 0), 2: (0, -1)}.get(k, (0, 1))
        assert abs(x[24 * 2 + 2 * k] - want[0]) < 1e-12 and abs(x[24 * 2 + 2 * k + 1] - want[1]) < 1e-12
        # normal z = 1: sin(2^k pi) = 0, cos = -1 for k = 0 and 1 above
        assert abs(x[24 * 5 + 2 * k]) < 1e-12
        assert x[24 * 5 + 2 * k + 1] == pytest.approx(-1.0 if k == 0 else 1.0, abs=1e-12)


def test_encoding_is_sin_cos_of_the_normalised_coordinates(orc):
    rng = np.random.default_rng(2)
    pos = rng.uniform(-1, 3, (50, 3)).astype(np.float32)
    nrm = rng.normal(size=(50, 3)).astype(np.float32)
    lo, hi = np.float32([-1, -1, -1]), np.float32([3, 3, 3])
    x = orc.mlp_encode(pos, nrm, lo, hi)
    v = np.concatenate([((pos - lo) / (hi - lo)).astype(np.float32), nrm], 1).astype(np.float64)
    for c in range(6):
        for k in range(12):
            # sin^2 + cos^2 = 1 and the doubling formula links neighbouring frequencies
            s, co = x[:, 24 * c + 2 * k], x[:, 24 * c + 2 * k + 1]
            assert np.allclose(s * s + co * co, 1.0, atol=1e-12)
            if k:
                s0, c0 = x[:, 24 * c + 2 * k - 2], x[:, 24 * c + 2 * k - 1]
                assert np.allclose(s, 2 * s0 * c0, atol=1e-9)
        assert np.allclose(x[:, 24 * c], np.sin(np.pi * v[:, c]), atol=1e-12)


# --------------------------------------------------------------------------
# forward
# --------------------------------------------------------------------------
def test_forward_matches_torch_float64(orc):
    rng = np.random.default_rng(3)
    params = _rand_params(rng)
    x = rng.normal(size=(37, IN))
    z, q = orc.mlp_forward(params, x)
    net = _torch_net(params)
    zt = net(torch.tensor(x)).detach().numpy()
    assert np.allclose(z, zt, rtol=1e-12, atol=1e-12)
    assert np.allclose(q, torch.softmax(torch.tensor(zt), 1).numpy(), rtol=1e-12, atol=1e-15)
    assert np.allclose(q.sum(1), 1.0, atol=1e-14)


def test_forward_zero_weights_gives_softmax_of_last_bias(orc):
    params = np.zeros(orc.mlp_nparam())
    b4 = np.linspace(-2, 3, OUT)
    params[-OUT:] = b4
    z, q = orc.mlp_forward(params, np.ones((2, IN)))
    e = np.exp(b4 - b4.max())
    assert np.allclose(z, b4[None]) and np.allclose(q, (e / e.sum())[None], rtol=1e-14)


def test_forward_bf16_mode_rounds_where_the_gpu_does(orc):
    rng = np.random.default_rng(4)
    params = _rand_params(rng)
    x = rng.uniform(-1, 1, size=(9, IN))
    z16, _ = orc.mlp_forward(params, x, bf16=True)
    # the same network with weights and input pre-rounded, activations rounded
    # after each ReLU, built from torch modules
    W = orc.bf16_round(params)
    net = _torch_net(np.where(_bias_mask(), params, W))
    h = torch.tensor(orc.bf16_round(x))
    for m in net:
        h = m(h)
        if isinstance(m, torch.nn.ReLU):
            h = torch.tensor(orc.bf16_round(h.detach().numpy()))
    assert np.allclose(z16, h.detach().numpy(), rtol=1e-12, atol=1e-12)
    z64, _ = orc.mlp_forward(params, x)
    assert np.linalg.norm(z16 - z64) < 3e-2 * np.linalg.norm(z64)


def _bias_mask():
    m = []
    for nin, nout in ((IN, H), (H, H), (H, H), (H, OUT)):
        m += [np.zeros(nin * nout, bool), np.ones(nout, bool)]
    return np.concatenate(m)


# --------------------------------------------------------------------------
# gradient
# --------------------------------------------------------------------------
def _batch(rng, n):
    x = rng.uniform(-1, 1, size=(n, IN))
    node = rng.integers(0, OUT, n).astype(np.uint32)
    w = rng.exponential(size=n)
    w[0] = 0.0
    return x, node, w


def test_gradient_matches_central_differences(orc):
    rng = np.random.default_rng(5)
    params = _rand_params(rng)
    x, node, w = _batch(rng, 5)
    L, g = orc.mlp_loss_grad(params, x, node, w)
    idx = np.concatenate([rng.choice(orc.mlp_nparam(), 300, replace=False),
                          np.arange(orc.mlp_nparam() - OUT, orc.mlp_nparam())])
    h = 1e-6
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (orc.mlp_loss_grad(pp, x, node, w)[0] - orc.mlp_loss_grad(pm, x, node, w)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_gradient_and_loss_match_torch_autograd(orc):
    rng = np.random.default_rng(6)
    params = _rand_params(rng)
    x, node, w = _batch(rng, 23)
    L, g = orc.mlp_loss_grad(params, x, node, w)
    net = _torch_net(params)
    z = net(torch.tensor(x))
    wt = torch.tensor(w)
    lt = -(wt * torch.log_softmax(z, 1)[torch.arange(23), torch.tensor(node.astype(np.int64))]).sum() / wt.sum()
    lt.backward()
    assert L == pytest.approx(lt.item(), rel=1e-12)
    assert np.allclose(g, _flat_grad(net), rtol=1e-10, atol=1e-13)


def test_gradient_of_zero_weight_batch_is_zero(orc):
    rng = np.random.default_rng(7)
    params = _rand_params(rng)
    x, node, _ = _batch(rng, 4)
    L, g = orc.mlp_loss_grad(params, x, node, np.zeros(4))
    assert L == 0.0 and not g.any()


def _bf16_t(t):
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


class _RoundValue(torch.autograd.Function):
    """Rounds values to BF16 on the way forward; gradient passes unchanged."""

    @staticmethod
    def forward(ctx, x):
        return _bf16_t(x)

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGrad(torch.autograd.Function):
    """Identity on the way forward; rounds the gradient to BF16 going back."""

    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return _bf16_t(g)


def test_gradient_bf16_mode_matches_torch_with_rounding_points(orc):
    """bf16 mode: BF16 weights and input; activations rounded after ReLU; the
    output gradient w_i (q - e_k) and each back-propagated pre-activation
    gradient rounded; built here from torch autograd with rounding nodes."""
    rng = np.random.default_rng(8)
    params = _rand_params(rng)
    x, node, w = _batch(rng, 64)
    L16, g16 = orc.mlp_loss_grad(params, x, node, w, bf16=True)
    Wr = np.where(_bias_mask(), params, orc.bf16_round(params))
    net = _torch_net(Wr)
    lins = [m for m in net if isinstance(m, torch.nn.Linear)]
    h = _bf16_t(torch.tensor(x))
    for i, lin in enumerate(lins):
        h = _RoundGrad.apply(lin(h))
        if i < 3:
            h = _RoundValue.apply(torch.relu(h))
    wt = torch.tensor(w)
    lu = -(wt * torch.log_softmax(h, 1)[torch.arange(64), torch.tensor(node.astype(np.int64))]).sum()
    lu.backward()
    want = np.concatenate([t.grad.reshape(-1).numpy() for lin in lins for t in (lin.weight, lin.bias)])
    assert np.allclose(g16, want / w.sum(), rtol=1e-9, atol=1e-15)
    assert L16 == pytest.approx(lu.item() / w.sum(), rel=1e-12)
    # the rounding costs accuracy mostly in the first layers, where the
    # batch gradient is a small difference of large per-tuple terms
    _, g64 = orc.mlp_loss_grad(params, x, node, w)
    last = slice(orc.mlp_nparam() - OUT * H - OUT, orc.mlp_nparam())
    assert np.linalg.norm(g16[last] - g64[last]) < 1e-2 * np.linalg.norm(g64[last])
    assert np.linalg.norm(g16 - g64) < 0.25 * np.linalg.norm(g64)


# --------------------------------------------------------------------------
# Adam, shuffle, training
# --------------------------------------------------------------------------
def test_adam_matches_torch(orc):
    rng = np.random.default_rng(9)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(4)]
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, 1):
        orc.mlp_adam(p, m, v, g, t, lr=1e-2)
    tp = torch.nn.Parameter(torch.tensor(p0))
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for g in grads:
        tp.grad = torch.tensor(g)
        opt.step()
    assert np.allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_adam_first_step_is_lr_times_sign(orc):
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    orc.mlp_adam(p, m, v, g, 1, lr=0.1)
    # m^ = g, v^ = g^2: the step is lr g / (|g| + eps)
    assert np.allclose(p, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 15, 16, 17, 63, 64, 65, 1000, 4096, 4097, 65537])
def test_shuffle_is_a_permutation_for_every_size(orc, n):
    """Sizes at, just below and just above powers of four (where the
    Feistel domain grows and the walk starts or stops being needed)."""
    perm = orc.mlp_shuffle(n, 3, 7, scenes.SEED_BASE + 5)
    assert np.array_equal(np.sort(perm), np.arange(n))


def test_shuffle_changes_with_epoch_scene_and_seed(orc):
    seed = scenes.SEED_BASE + 5
    base = orc.mlp_shuffle(1000, 3, 7, seed)
    for other in (orc.mlp_shuffle(1000, 4, 7, seed), orc.mlp_shuffle(1000, 3, 8, seed),
                  orc.mlp_shuffle(1000, 3, 7, seed + 1)):
        assert np.mean(other != base) > 0.9
    assert np.array_equal(base, orc.mlp_shuffle(1000, 3, 7, seed))


def test_shuffle_positions_are_uniform(orc):
    """Over epochs, the first two positions of a 10-tuple order (its domain
    has 16 values, so most maps walk) take every ordered pair of distinct
    tuples equally often, as a uniformly random order would."""
    n, epochs = 10, 9000
    first = np.empty((epochs, 2), np.int64)
    for e in range(epochs):
        first[e] = orc.mlp_shuffle(n, e, 1, scenes.SEED_BASE + 6)[:2]
    assert np.all(first[:, 0] != first[:, 1])
    cnt = np.bincount(first[:, 0] * n + first[:, 1], minlength=n * n).reshape(n, n)
    off = cnt[~np.eye(n, dtype=bool)]
    assert stats.chisquare(off).pvalue > 1e-4
    assert stats.chisquare(np.bincount(first[:, 0], minlength=n)).pvalue > 1e-4


def test_shuffle_moves_low_and_high_bits(orc):
    """With n = 4^5 no value walks; a round that left either half of the
    word in place would keep it: about 1/32 of the tuples keep their low
    (or high) 5 bits, and about one keeps its place."""
    n = 1024
    perm = orc.mlp_shuffle(n, 0, 2, scenes.SEED_BASE + 7).astype(np.int64)
    i = np.arange(n)
    assert np.mean((perm & 31) == (i & 31)) < 0.1
    assert np.mean((perm >> 5) == (i >> 5)) < 0.1
    assert np.sum(perm == i) < 8


def test_training_single_full_batch_is_one_adam_step(orc):
    rng = np.random.default_rng(10)
    params = _rand_params(rng)
    xall = rng.uniform(-1, 1, size=(40, IN))
    pid = rng.integers(0, 40, 30).astype(np.uint32)
    node = rng.integers(0, OUT, 30).astype(np.uint32)
    w = rng.exponential(size=30)
    p1, m1, v1 = params.copy(), np.zeros_like(params), np.zeros_like(params)
    step, _ = orc.mlp_train(p1, m1, v1, 0, xall, pid, node, w, epochs=1, batch=64)
    assert step == 1
    # the loss over a batch does not depend on the order of its tuples
    _, g = orc.mlp_loss_grad(params, xall[pid], node, w)
    p2, m2, v2 = params.copy(), np.zeros_like(params), np.zeros_like(params)
    orc.mlp_adam(p2, m2, v2, g, 1)
    assert np.allclose(p1, p2, rtol=1e-12, atol=1e-15)


def test_training_learns_a_position_dependent_target(orc):
    """Tuples whose node is a function of the position: the trained network
    puts most of its mass on the right node."""
    rng = np.random.default_rng(11)
    P = 256
    pos = rng.uniform(0, 1, (P, 3)).astype(np.float32)
    nrm = np.tile(np.float32([0, 1, 0]), (P, 1))
    xall = orc.mlp_encode(pos, nrm, [0, 0, 0], [1, 1, 1])
    target = (np.floor(pos[:, 0] * 4) + 4 * np.floor(pos[:, 2] * 4)).astype(np.uint32)
    pid = np.repeat(np.arange(P, dtype=np.uint32), 4)
    node = target[pid]
    w = np.ones(pid.size)
    params = _rand_params(rng, 0.5)
    m, v = np.zeros_like(params), np.zeros_like(params)
    _, q0 = orc.mlp_forward(params, xall)
    step, _ = orc.mlp_train(params, m, v, 0, xall, pid, node, w, epochs=30, batch=128, lr=3e-3)
    assert step == 30 * 8
    _, q = orc.mlp_forward(params, xall)
    assert q[np.arange(P), target].mean() > 0.5 > 4 * q0[np.arange(P), target].mean()


# --------------------------------------------------------------------------
# mixture sampling
# --------------------------------------------------------------------------
def _mix_scene(orc, n_lights=300, M=16, boxes=None):
    s = scenes.make_tiny(n_lights=n_lights, n_points=64, spp=1, M=M)
    o = orc.Oracle(s.params, s.tri, s.emit, s.boxes if boxes is None else boxes)
    return s, o


def _p_mix(o, cdf_row, Qt, C, end, w):
    """p(l) for every light of a cell with table (Qt, C, end) at one point."""
    N = o.N
    fnode, fend = o.fixed_cut()
    l = np.arange(N)
    s = np.searchsorted(end, l, side="right")
    size = np.diff(np.concatenate([[0], end]))[s]
    pt = Qt[s].astype(np.float64) / (size * float(C[-1]))
    k = np.searchsorted(fend, l, side="right")
    fsize = np.diff(np.concatenate([[0], fend]))[k]
    qk = np.diff(np.concatenate([[0.0], cdf_row[:len(fend)].astype(np.float64)]))[k]
    pm = qk / (fsize * float(cdf_row[len(fend) - 1]))
    return w * pt + (1 - w) * pm


def test_fixed_cut_is_the_breadth_first_cut_of_64(orc):
    s, o = _mix_scene(orc)
    node, end = o.fixed_cut()
    t = o.tree()
    assert len(node) == 64 and end[-1] == o.N
    first = t["first"][node]
    assert np.array_equal(first[1:], end[:-1]) and first[0] == 0
    # breadth-first: the internal nodes of the cut lie on two neighbouring
    # levels, and no leaf of the cut lies deeper than them
    depth = []
    for nd in node:
        d, x = 0, nd
        while t["parent"][x] != 0xFFFFFFFF:
            x, d = t["parent"][x], d + 1
        depth.append(d)
    depth = np.array(depth)
    leaf = node >= o.N - 1
    assert depth[~leaf].max() - depth[~leaf].min() <= 1
    assert (depth[leaf] <= depth[~leaf].max()).all()
    # a tree of fewer lights gives a cut of every leaf
    s2 = scenes.make_tiny(n_lights=40, n_points=8)
    o2 = orc.Oracle(s2.params, s2.tri, s2.emit)
    n2, e2 = o2.fixed_cut()
    assert len(n2) == 40 and np.array_equal(e2, np.arange(1, 41))


def _random_cdf(rng, P, sharp=3.0):
    z = rng.normal(size=(P, 64)) * sharp
    q = np.exp(z - z.max(1, keepdims=True))
    q /= q.sum(1, keepdims=True)
    return q


def test_mixture_pdf_sums_to_one_and_matches_draw_frequencies(orc):
    rng = np.random.default_rng(12)
    s, o = _mix_scene(orc, n_lights=300)
    q = _random_cdf(rng, 1)
    cdf = orc.mlp_cdf(q)
    # one point drawn many times: its cell keeps the initial table (no adapt)
    spp = 20000
    pos = np.float32([[0.3, 0.4, 0.6]])
    nrm = np.float32([[0, 1, 0]])
    o.set_mixture(cdf, 0.5)
    _, rec = o.frame(pos, nrm, spp, 0, records=True)
    tnode, tend = o.template()
    Qt = np.ones(len(tend), np.float32)
    C = np.cumsum(Qt).astype(np.float32)
    p = _p_mix(o, cdf[0], Qt, C, tend, 0.5)
    assert abs(p.sum() - 1.0) < 1e-6
    # every sample's 1/p is the mixture density of the light it drew
    assert np.allclose(1.0 / rec["inv_pdf"], p[rec["light"]], rtol=2e-6)
    # draw frequencies: chi-square over the fixed-cut nodes
    fend = o.fixed_cut()[1]
    k = np.searchsorted(fend, rec["light"], side="right")
    assert np.array_equal(k, rec["fnode"])
    pk = np.array([p[(np.arange(o.N) >= (fend[i - 1] if i else 0)) & (np.arange(o.N) < fend[i])].sum()
                   for i in range(len(fend))])
    obs = np.bincount(k, minlength=len(fend))
    exp = pk * spp
    keep = exp > 5
    chi2 = (((obs - exp) ** 2 / exp)[keep]).sum()
    dof = keep.sum() - 1
    assert chi2 < dof + 5 * math.sqrt(2 * dof)
    # about half the draws come from each component
    assert abs(rec["comp"].mean() - 0.5) < 0.02


def test_mixture_weight_zero_is_the_plain_method(orc):
    """w is the network's share: w = 0 turns the mixture off, so the draws,
    densities, radiance and cells are the plain method's, bit for bit."""
    rng = np.random.default_rng(13)
    s, o = _mix_scene(orc)
    s2, o2 = _mix_scene(orc)
    o.set_mixture(orc.mlp_cdf(_random_cdf(rng, s.P)), 0.0)
    r1, a = o.frame(s.pos, s.nrm, 4, 0, records=True)
    r2, b = o2.frame(s.pos, s.nrm, 4, 0, records=True)
    assert np.array_equal(a["light"], b["light"]) and not a["comp"].any()
    assert np.array_equal(a["inv_pdf"], b["inv_pdf"]) and np.array_equal(r1, r2)
    o.adapt()
    o2.adapt()
    ca, cb = o.cells(), o2.cells()
    assert all(np.array_equal(ca[k], cb[k]) for k in ("key", "node", "end", "Q", "Qt", "C"))


def test_mixture_weight_one_draws_only_inside_likely_nodes(orc):
    """w = 1, the network alone (the oracle accepts it to pin the proposal's
    own draws): only nodes of positive learned probability are drawn."""
    s, o = _mix_scene(orc)
    q = np.zeros((s.P, 64))
    q[:, 7] = 0.75
    q[:, 40] = 0.25
    o.set_mixture(orc.mlp_cdf(q), 1.0)
    _, rec = o.frame(s.pos, s.nrm, 8, 0, records=True)
    assert set(np.unique(rec["fnode"]).tolist()) == {7, 40} and rec["comp"].all()
    fend = o.fixed_cut()[1]
    size = np.diff(np.concatenate([[0], fend]))
    want = np.where(rec["fnode"] == 7, size[7] / 0.75, size[40] / 0.25)
    assert np.allclose(rec["inv_pdf"], want, rtol=1e-6)
    # draws of the learned component leave the cells' statistics untouched
    c = o.cells()
    assert not c["cnt"].any()


def test_training_weight_is_luminance_over_density(orc):
    rng = np.random.default_rng(14)
    s, o = _mix_scene(orc)
    o.set_mixture(orc.mlp_cdf(_random_cdf(rng, s.P)), 0.5)
    _, rec = o.frame(s.pos, s.nrm, 4, 0, records=True)
    c = rec["contrib"]
    want = ((c[:, 0] + c[:, 1]) + c[:, 2]) * rec["inv_pdf"]
    assert np.array_equal(rec["weight"], want.astype(np.float32))
    assert (rec["weight"] > 0).mean() > 0.3


@pytest.mark.slow
def test_mixture_estimate_is_unbiased(orc):
    """z-test of the mixture estimator against the closed-form irradiance
    (no occluders), with a deliberately poor learned distribution."""
    rng = np.random.default_rng(15)
    s = scenes.make_tiny(n_lights=200, n_points=48, spp=1, M=16)
    s.pos[:, 1] *= 0.8
    o = orc.Oracle(s.params, s.tri, s.emit, np.zeros((0, 6), np.float32))
    truth = o.truth_unoccluded(s.pos, s.nrm)
    o.set_mixture(orc.mlp_cdf(_random_cdf(rng, s.P, sharp=4.0)), 0.5)
    spp = 2048
    _, rec = o.frame(s.pos, s.nrm, spp, 0, records=True)
    est = (rec["contrib"] * rec["inv_pdf"][:, None]).reshape(s.P, spp, 3).astype(np.float64)
    mean = est.mean(1)
    se = est.std(1) / math.sqrt(spp)
    z = (mean - truth) / np.maximum(se, 1e-12)
    ok = truth > 1e-6
    assert np.abs(z[ok]).max() < 5.0
    assert abs(z[ok].mean()) < 4.0 / math.sqrt(ok.sum())
