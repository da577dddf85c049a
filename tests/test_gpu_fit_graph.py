"""Fitting control points through torch.autograd (C4), graph capture and the
autotuner."""
import math

import numpy as np
import pytest
import torch

import fa_inputs as fi
import oracle
from gpu_util import U32, mixed_batch, models, oracle_blocks, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fa():
    import paper_2409_00184_amd as fa
    assert torch.cuda.is_available()
    return fa


def _fit_case(fa, b, y, P0, res):
    m = models(b)
    plan = fa.Plan(m, res)
    ctrl = torch.as_tensor(P0, dtype=torch.float32, device="cuda").requires_grad_(True)
    yt = torch.as_tensor(y, device="cuda").reshape(b.nblocks, 1, *res)
    out = fa.FADecode.apply(ctrl, m, res, 1, plan)
    loss = ((out - yt) ** 2).mean()
    loss.backward()
    return m, ctrl.grad.detach().cpu().numpy().astype(np.float64), float(loss.detach())


def _oracle_grad(b, P0, y, res):
    """FP64: r = B P - y, grad = (2/M) B^T r, and the two rounding scales of
    an FP32 gradient: (2/M) B^T |r| (the adjoint's own sums) and
    (2/M) B^T (B |P|) (the decoded values' rounding, up to 64 u32 B|P| per
    voxel, carried through the residual); the value basis is non-negative,
    so B^T and B of non-negative vectors are their absolute sums."""
    ob = oracle_blocks(b, P0.astype(np.float64))
    f = oracle.decode_blocks(ob, res, 1)
    r = f - y.reshape(f.shape).astype(np.float64)
    M = r.size
    g = oracle.decode_adjoint(ob, res, r, 1) * (2.0 / M)
    ga = oracle.decode_adjoint(ob, res, np.abs(r), 1) * (2.0 / M)
    S = oracle.decode_blocks(oracle_blocks(b, np.abs(P0.astype(np.float64))), res, 1)
    gs = oracle.decode_adjoint(ob, res, S, 1) * (2.0 / M)
    return g, ga, float((r ** 2).mean()), f, gs


@pytest.mark.parametrize("nblocks,resn", [(6, 24), (256, 64)])
def test_fit_gradient_vs_oracle_and_fd(fa, nblocks, resn):
    """C4 shape at full size (256 blocks, 64^3 samples each, NCP* in
    {16,24,32}, cubic, k^-5/3 targets) and a small case: the autograd
    gradient (HIP adjoint) against the FP64 oracle gradient elementwise, and
    against FP64 central differences (h = 1e-3) on 64 seeded control points."""
    say("fit gradient", nblocks, resn)
    b, y = fi.config_c4(nblocks=nblocks, res=resn)
    res = (resn,) * 3
    g = fi.rng(61)
    P0 = (0.5 * g.normal(size=b.ctrl.size)).astype(np.float32)
    m, grad, loss = _fit_case(fa, b, y, P0, res)
    go, ga, lo, f, gs = _oracle_grad(b, P0, y, res)
    assert abs(loss - lo) <= 1e-5 * lo
    valid = np.zeros(b.ctrl.size, bool)
    for k in range(b.nblocks):
        o = int(b.ctrl_off[k])
        valid[o:o + int(np.prod(b.ncp[k]))] = True
    err = np.abs(grad - go)[valid]
    lim = 256 * U32 * ga[valid] + 64 * U32 * gs[valid] + 1e-30
    assert np.all(err <= lim), float((err / lim).max())
    # central differences of the FP64 loss on 64 seeded control points
    h = 1e-3
    picks = g.choice(np.flatnonzero(valid), 64, replace=False)
    ob = oracle_blocks(b, P0.astype(np.float64))
    M = y.size
    for e in picks:
        k = int(np.searchsorted(b.ctrl_off, e, side="right") - 1)
        sub = oracle.Blocks(ob.ncp[k:k + 1], ob.deg[k:k + 1], ob.knot_off[k:k + 1],
                            ob.ctrl_off[k:k + 1], ob.knots, ob.ctrl)
        yk = y[k].reshape(1, 1, *res).astype(np.float64)
        Lk = []
        for sgn in (1.0, -1.0):
            c = ob.ctrl.copy()
            c[e] += sgn * h
            fk = oracle.decode_blocks(sub.with_ctrl(c), res, 1)
            Lk.append(((fk - yk) ** 2).sum() / M)
        fd = (Lk[0] - Lk[1]) / (2 * h)
        assert abs(fd - grad[e]) <= 1e-4 * abs(fd) + 1e-3 * ga[e] + 1e-12, (e, fd, grad[e])


@pytest.mark.parametrize("nblocks,resn", [(6, 24), (256, 64)])
def test_fused_mse_gradient_vs_oracle(fa, nblocks, resn):
    """The fused loss (decode, fa_mse_grad, adjoint) gives the FP64 oracle's
    loss and gradient under the same bounds as the torch-composed loss, and
    agrees with that loss to FP32 rounding."""
    say("fused mse", nblocks, resn)
    b, y = fi.config_c4(nblocks=nblocks, res=resn)
    res = (resn,) * 3
    g = fi.rng(62)
    P0 = (0.5 * g.normal(size=b.ctrl.size)).astype(np.float32)
    m = models(b)
    plan = fa.Plan(m, res)
    ctrl = torch.as_tensor(P0, device="cuda").requires_grad_(True)
    yt = torch.as_tensor(y, device="cuda").reshape(b.nblocks, *res).contiguous()
    loss = fa.FAFitMSE.apply(ctrl, m, res, yt, plan)
    loss.backward()
    grad = ctrl.grad.detach().cpu().numpy().astype(np.float64)
    go, ga, lo, _, gs = _oracle_grad(b, P0, y, res)
    assert abs(float(loss.detach()) - lo) <= 1e-5 * lo
    valid = np.zeros(b.ctrl.size, bool)
    for k in range(b.nblocks):
        o = int(b.ctrl_off[k])
        valid[o:o + int(np.prod(b.ncp[k]))] = True
    err = np.abs(grad - go)[valid]
    lim = 256 * U32 * ga[valid] + 64 * U32 * gs[valid] + 1e-30
    assert np.all(err <= lim), float((err / lim).max())
    _, g2, l2 = _fit_case(fa, b, y, P0, res)
    assert abs(float(loss.detach()) - l2) <= 1e-5 * l2
    assert np.abs(grad - g2)[valid].max() <= 1e-5 * np.abs(g2[valid]).max()


@pytest.mark.parametrize("res,tune", [
    ((64, 64, 64), None),                       # default schedule
    ((23, 17, 41), (4, 4, 768, 0, 4096, 1)),    # ragged grid, ordinary stores
    ((40, 48, 70), (16, 8, 1 << 20, 0, 4096, 0)),  # z tiles, slab restaged in x chunks
])
def test_decode_residual_matches_decode_then_mse(fa, res, tune):
    """The fused value decode + residual equals fa_decode_blocks followed by
    fa_mse_grad bit for bit in the cotangent, and in sumsq up to the order
    of the FP64 sums (checked against an FP64 sum of the same residuals)."""
    say("decode residual", res, tune)
    b = mixed_batch(66, 9, ncp_lo=4, ncp_hi=32)
    m = models(b)
    g = fi.rng(67)
    y = torch.as_tensor(g.normal(size=(b.nblocks,) + res).astype(np.float32)).cuda()
    nvox = int(np.prod(res))
    scale = 2.0 / (b.nblocks * nvox)
    plan = fa.Plan(m, res, *tune) if tune else fa.Plan(m, res)
    grad, sumsq = fa.decode_residual(m, res, y, scale, plan=plan)
    f = fa.decode(m, res, 1, plan=plan)
    ref_g = torch.empty_like(y)
    ref_s = torch.empty(b.nblocks, dtype=torch.float64, device="cuda")
    st = fa.lib.fa_mse_grad(fa._ptr(f), fa._ptr(y), b.nblocks, nvox, scale, fa._ptr(ref_g),
                            fa._ptr(ref_s), fa._stream(None))
    assert st == 0
    torch.cuda.synchronize()
    assert torch.equal(grad, ref_g)
    # the residual as both kernels form it (one FP32 subtraction), squared
    # and summed in FP64
    r64 = (f.reshape(b.nblocks, -1) - y.reshape(b.nblocks, -1)).double()
    exact = (r64 * r64).sum(1)
    assert torch.allclose(sumsq, exact, rtol=1e-12, atol=0), (sumsq - exact).abs().max()
    assert torch.allclose(ref_s, exact, rtol=1e-12, atol=0)
    # the default order (no plan) gives the same values
    g2, s2 = fa.decode_residual(m, res, y, scale,
                                tune=fa.FATune(*tune) if tune else None)
    assert torch.equal(g2, grad) and torch.equal(s2, sumsq)


def test_fit_converges(fa):
    """A few Adam steps on C4-shaped blocks lower the loss steadily."""
    say("fit converges")
    b, y = fi.config_c4(nblocks=16, res=32)
    res = (32, 32, 32)
    m = models(b)
    plan = fa.Plan(m, res)
    ctrl = torch.zeros(b.ctrl.size, device="cuda", requires_grad=True)
    yt = torch.as_tensor(y, device="cuda").reshape(16, 1, *res)
    opt = torch.optim.Adam([ctrl], lr=0.05)
    losses = []
    for it in range(40):
        opt.zero_grad()
        loss = ((fa.FADecode.apply(ctrl, m, res, 1, plan) - yt) ** 2).mean()
        loss.backward()
        opt.step()
        losses.append(loss.item())
    assert losses[-1] < 0.5 * losses[0], losses[::8]


def test_graph_replay_matches_eager(fa):
    """Decode (planned, persistent), query and adjoint captured into one
    graph; every replay, with eager work and synchronisation in between,
    reproduces the eager results bit for bit."""
    say("graph replay")
    b = mixed_batch(62, 12, ncp_hi=24)
    m = models(b)
    res = (20, 33, 40)
    plan = fa.Plan(m, res, rows=4, waves=4, grid=37)
    out = torch.empty((b.nblocks, 4) + res, device="cuda")
    xyz = torch.rand(50000, 3, device="cuda")
    boc = torch.arange(12, dtype=torch.int32, device="cuda")
    q = torch.empty(50000, 4, device="cuda")
    gin = torch.randn((b.nblocks, 1) + res, device="cuda")
    G = torch.zeros_like(m.ctrl)

    def step():
        fa.decode(m, res, 15, plan=plan, out=out)
        fa.query(m, xyz, (3, 2, 2), (0, 0, 0), (1, 1, 1), boc, out=q)
        fa.decode_backward(m, res, gin, 1, grad_ctrl=G)

    inside = torch.zeros(G.numel(), dtype=torch.bool)
    for k in range(b.nblocks):
        o = int(b.ctrl_off[k])
        inside[o:o + int(np.prod(b.ncp[k]))] = True
    inside = inside.cuda()
    step()
    torch.cuda.synchronize()
    ref = (out.clone(), q.clone(), G.clone())
    graph, _ = fa.capture(step)
    for rep in range(5):
        out.fill_(float("nan"))
        q.zero_()
        G.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref[0]), ("decode", rep)
        assert torch.equal(q, ref[1]), ("query", rep)
        assert torch.equal(G[inside], ref[2][inside]), ("adjoint", rep)
        assert bool((G[~inside] == -1.0).all()), ("adjoint padding", rep)
        _ = (out * 2).sum().item()  # eager work between replays


@pytest.mark.parametrize("adam", ["capturable", "fused", "native"])
def test_captured_fit_step_matches_eager(fa, adam):
    """A whole fit iteration (decode, fused MSE, adjoint, capturable Adam:
    multi-kernel or fused) captured into one graph: every replay, with eager
    work and synchronisation in between, moves the lattice exactly as an
    eager iteration from the same state does (the eager one accumulates into
    a zeroed gradient, the graph sets it)."""
    say("captured fit step", adam)
    b = mixed_batch(64, 6, ncp_lo=4, ncp_hi=14)
    res = (24, 20, 28)
    g = fi.rng(65)
    y = torch.as_tensor(g.normal(size=(b.nblocks,) + res).astype(np.float32)).cuda()
    P0 = torch.as_tensor(0.1 * g.normal(size=b.ctrl.size).astype(np.float32)).cuda()
    runs = []
    for _ in range(2):
        m = models(b)
        ctrl = P0.clone().requires_grad_(True)
        if adam == "native":
            opt = fa.Adam([ctrl], lr=0.05)
        else:
            opt = torch.optim.Adam([ctrl], lr=0.05, capturable=True, fused=(adam == "fused"))
        runs.append((m, ctrl, opt, fa.Plan(m, res)))
    me, ce, oe, pe = runs[0]
    mg, cg, og, pg = runs[1]

    def eager():
        oe.zero_grad(set_to_none=False)
        loss = fa.FAFitMSE.apply(ce, me, res, y, pe)
        loss.backward()
        oe.step()
        return loss

    graph, loss_g = fa.capture_fit_step(cg, og, mg, res, y, pg, warmup=3)
    for _ in range(3):  # the capture's eager warm-up iterations
        eager()
    torch.cuda.synchronize()
    assert torch.equal(cg.detach(), ce.detach())
    for rep in range(4):
        graph.replay()
        torch.cuda.synchronize()
        le = eager()
        torch.cuda.synchronize()
        d = (cg.detach() - ce.detach()).abs().max().item()
        say("  replay", rep, "loss", float(loss_g.detach()), float(le.detach()), "max |ctrl diff|", d)
        assert torch.equal(cg.detach(), ce.detach()), ("ctrl", rep, d)
        assert float(loss_g.detach()) == float(le.detach()), ("loss", rep)
        _ = (ce.detach() * 2).sum().item()  # eager work between replays


def test_autotune_picks_valid_schedule(fa, tmp_path, monkeypatch):
    say("autotune")
    from paper_2409_00184_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(autotune, "TABLE", str(tmp_path / "no_table.json"))
    b = mixed_batch(63, 40, ncp_hi=32)
    m = models(b)
    res = (32, 32, 64)
    plan, report = autotune.tune(m, res, 15, "f32", candidates=autotune.CANDIDATES[:6])
    assert len(report) == 6 and (tmp_path / "tune.json").exists()
    a = fa.decode(m, res, 15, plan=plan)
    ref = fa.decode(m, res, 15)
    assert torch.equal(a, ref)
    plan2, rep2 = autotune.tune(m, res, 15, "f32")  # from the cache
    assert len(rep2) == 1 and plan2.tune.rows_per_item == plan.tune.rows_per_item


def test_autotune_interleaved_layout(fa, tmp_path, monkeypatch):
    """The autotuner times the interleaved-record layout through its own
    cache entry; its schedule decodes the same records as the default."""
    say("autotune interleaved")
    from paper_2409_00184_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(autotune, "TABLE", str(tmp_path / "no_table.json"))
    b = mixed_batch(64, 24, ncp_hi=32)
    m = models(b)
    res = (32, 24, 64)
    mk = 15 | fa.OUT_INTERLEAVED
    plan, report = autotune.tune(m, res, mk, "f32", candidates=autotune.CANDIDATES[:4])
    assert len(report) == 4
    assert autotune.signature(m, res, mk, "f32") != autotune.signature(m, res, 15, "f32")
    a = fa.decode(m, res, mk, plan=plan)
    assert a.shape == (b.nblocks,) + res + (4,)
    assert torch.equal(a, fa.decode(m, res, mk))
    assert torch.equal(a, fa.decode(m, res, 15).permute(0, 2, 3, 4, 1))


def test_fused_mse_backward_scale_and_fresh_gradients(fa):
    """FAFitMSE's backward multiplies the adjoint (written into a buffer
    kept on the micro-models) by the incoming gradient and returns a new
    tensor each time: a second backward with the loss scaled by 3 gives
    exactly 3x the first gradient, and neither gradient is the buffer."""
    say("fused mse backward scale")
    b = mixed_batch(68, 5, ncp_lo=4, ncp_hi=12)
    m = models(b)
    res = (9, 10, 12)
    g = fi.rng(69)
    y = torch.as_tensor(g.normal(size=(b.nblocks,) + res).astype(np.float32)).cuda()
    P0 = torch.as_tensor(g.normal(size=b.ctrl.size).astype(np.float32)).cuda()
    ctrl = P0.clone().requires_grad_(True)
    (g1,) = torch.autograd.grad(fa.FAFitMSE.apply(ctrl, m, res, y, None), ctrl)
    (g2,) = torch.autograd.grad(3.0 * fa.FAFitMSE.apply(ctrl, m, res, y, None), ctrl)
    assert torch.equal(g2, g1 * 3.0)
    buf = m._adjoint_buf
    assert len({g1.data_ptr(), g2.data_ptr(), buf.data_ptr()}) == 3
    # the buffer holds the unscaled adjoint of the last backward
    assert torch.equal(buf, g1)


@pytest.mark.parametrize("n", [1, 255, 256, 257, 5000])
def test_mse_loss_fixed_order(fa, n):
    """fa_mse_loss against the same FP64 additions done in numpy in the
    documented order (thread t adds blocks t, t + 256, ... in turn, then a
    binary tree over the 256 threads): bit for bit, and within one FP32 ulp
    of the plain sequential sum."""
    say("mse loss", n)
    g = np.random.Generator(np.random.PCG64(400 + n))
    ss = g.exponential(3.0, n) * 10.0 ** g.integers(-3, 4, n)
    count = float(n * 4096 + 7)
    got = fa.mse_loss(torch.as_tensor(ss, device="cuda"), count).item()
    part = np.zeros(256)
    for t in range(256):
        acc = 0.0
        for b in range(t, n, 256):
            acc = acc + ss[b]
        part[t] = acc
    h = 128
    while h:
        part[:h] = part[:h] + part[h:2 * h]
        h //= 2
    assert got == float(np.float32(part[0] / count))
    seq = float(np.float32(math.fsum(ss) / count))
    assert abs(got - seq) <= float(np.spacing(np.float32(seq)))


@pytest.mark.parametrize("n,offset,wd", [(4096 * 5 + 12, 0, 0.0), (4099, 0, 0.01), (1000, 1, 0.0),
                                         (3, 0, 0.0), (0, 0, 0.0)])
def test_native_adam_matches_torch(fa, n, offset, wd):
    """fa.Adam (fa_adam_step) against torch.optim.Adam on the same FP32
    parameters and gradients for K steps: 16-byte and 4-byte aligned arrays,
    lengths with a ragged tail, weight decay, an empty tensor.  Bound: each
    step rounds about ten FP32 operations per element, and the two sides
    compute 1 - b^t differently (FP32 pow here, FP64 there), so after K steps
    |p - p_torch| <= 32 K u32 (max |p| + lr)."""
    say("native adam", n, offset, wd)
    g = torch.Generator().manual_seed(71 + n)
    K, lr = 10, 0.05
    base = torch.randn(n + offset, generator=g)
    grads = [torch.randn(n, generator=g) for _ in range(K)]
    pa = base.cuda()[offset:] if offset else base.cuda()
    pa = torch.nn.Parameter(pa) if offset == 0 else pa.requires_grad_(True)
    pt = torch.nn.Parameter(base[offset:].clone().cuda())
    oa = fa.Adam([pa], lr=lr, betas=(0.9, 0.99), eps=1e-8, weight_decay=wd)
    ot = torch.optim.Adam([pt], lr=lr, betas=(0.9, 0.99), eps=1e-8, weight_decay=wd,
                          foreach=False)
    for k in range(K):
        pa.grad = grads[k].cuda()
        pt.grad = grads[k].cuda()
        oa.step()
        ot.step()
    torch.cuda.synchronize()
    if n == 0:
        return
    d = (pa.detach() - pt.detach()).abs().max().item()
    lim = 32 * K * 2.0 ** -24 * (pt.detach().abs().max().item() + lr)
    say("  max |diff|", d, "bound", lim)
    assert d <= lim
    st = oa.state[pa]["state"].cpu().numpy()
    assert st[0] == K
