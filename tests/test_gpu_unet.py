"""GPU U-Net kernels and network vs the FP64 NumPy reference (oracle/unet_ref.py).

Single convolutions get identical bfloat16 inputs on both sides, so they
agree to FP32 accumulation error.  The whole network stores every activation
in bfloat16 on both sides; FP32 vs FP64 sums can flip a rounding by one
bfloat16 ulp.  Each layer of the network is therefore checked element by
element on its own GPU input (its output must be the bfloat16 rounding of the
exact result, or one ulp off where the exact result lies within FP32
accumulation error of a rounding boundary), and the whole network's output
and gradient element by element against bounds in bfloat16 ulps of their
scale, with the relative L2 error as a summary."""
import numpy as np
import pytest
import torch

from oracle import unet_ref as U

pytestmark = pytest.mark.gpu


def raw(x):
    """float64 values that are bfloat16-exact -> raw uint16 bits (as int16 tensor)."""
    b = (np.asarray(x, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)
    return torch.from_numpy(b.view(np.int16).copy()).cuda()


def lib():
    from paper_1307_6748_amd import _capi as A
    return A.lib()


def P(t):
    import ctypes as C
    return None if t is None else C.c_void_p(t.data_ptr())


SHAPES = [(16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (128, 64), (96, 32), (48, 16)]


@pytest.mark.parametrize("cin,cout", SHAPES)
@pytest.mark.parametrize("n", [4, 8, 16])
def test_conv_forward(cin, cout, n):
    rng = np.random.default_rng(cin * 7 + cout + n)
    x = U.bf16(rng.standard_normal((n, n, n, cin)))
    W = U.bf16(rng.standard_normal((27, cout, cin)) * 0.1)
    b = rng.standard_normal(cout).astype(np.float32).astype(np.float64)
    ref = U.conv3(x, W, b)
    yf = torch.empty(n ** 3 * cout, dtype=torch.float32, device="cuda")
    yb = torch.empty(n ** 3 * cout, dtype=torch.int16, device="cuda")
    bt = torch.from_numpy(b.astype(np.float32)).cuda()
    xt, wt = raw(x), raw(W)  # keep the device copies alive until the kernels ran
    rc = lib().isis_conv3_fwd(P(xt), n, cin, P(wt), P(bt), cout, 0, P(yb), P(yf), None)
    assert rc == 0
    got = yf.cpu().numpy().reshape(n, n, n, cout)
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.abs(ref).max()
    # bf16 output = rounding of the FP32 result
    gb = yb.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    assert np.array_equal(gb.view(np.float32).reshape(got.shape), U.bf16(got).astype(np.float32))
    # ReLU variant
    rc = lib().isis_conv3_fwd(P(xt), n, cin, P(wt), P(bt), cout, 1, None, P(yf), None)
    assert rc == 0
    assert np.max(np.abs(yf.cpu().numpy().reshape(got.shape) - np.maximum(ref, 0))) <= \
        1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("cin,cout,n", [(c, o, 64) for c, o in SHAPES] +
                         [(16, 48, 64), (16, 16, 128), (48, 16, 128)])
def test_conv_forward_staged(cin, cout, n):
    """Sides >= 64 take the LDS-staged kernel (4 x 64 tiles of an x-plane,
    16-channel slices).  Checked on eight 8^3 output blocks (corners and the
    periodic wrap included): the oracle convolves each block with its
    one-voxel periodic halo, whose interior is then exact."""
    rng = np.random.default_rng(cin * 7 + cout + n)
    x = U.bf16(rng.standard_normal((n, n, n, cin)))
    W = U.bf16(rng.standard_normal((27, cout, cin)) * 0.1)
    b = rng.standard_normal(cout).astype(np.float32).astype(np.float64)
    yf = torch.empty(n ** 3 * cout, dtype=torch.float32, device="cuda")
    yb = torch.empty(n ** 3 * cout, dtype=torch.int16, device="cuda")
    bt = torch.from_numpy(b.astype(np.float32)).cuda()
    xt, wt = raw(x), raw(W)
    rc = lib().isis_conv3_fwd(P(xt), n, cin, P(wt), P(bt), cout, 1, P(yb), P(yf), None)
    assert rc == 0
    got = yf.cpu().numpy().reshape(n, n, n, cout)
    gb = (yb.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    corners = [(0, 0, 0), (n - 4, n - 4, n - 4), (n // 2 - 3, 5, n - 60), (7, n - 8, 28)]
    corners += [tuple(int(c) for c in rng.integers(0, n, 3)) for _ in range(4)]
    for c in corners:
        idx = [(c[d] - 1 + np.arange(10)) % n for d in range(3)]
        ref = np.maximum(U.conv3(x[np.ix_(*idx)], W, b)[1:9, 1:9, 1:9], 0.0)
        sel = np.ix_(idx[0][1:9], idx[1][1:9], idx[2][1:9])
        assert np.max(np.abs(got[sel] - ref)) <= 1e-5 * max(np.abs(ref).max(), 1e-30), c
        assert np.array_equal(gb.reshape(got.shape)[sel], U.bf16(got[sel]).astype(np.float32))


@pytest.mark.parametrize("cin,cout", SHAPES)
def test_conv_data_gradient(cin, cout):
    """Flipped, transposed weights turn the forward kernel into the adjoint."""
    n = 8
    rng = np.random.default_rng(cin + 3 * cout)
    dy = U.bf16(rng.standard_normal((n, n, n, cout)))
    W = rng.standard_normal((27, cout, cin)) * 0.1
    Wq = U.bf16(W)
    ref = U.conv3_bwd_data(dy, Wq)
    wt = torch.empty(27 * cin * cout, dtype=torch.int16, device="cuda")
    wf = torch.from_numpy(W.astype(np.float32)).cuda()
    assert lib().isis_conv3_flip_weights(P(wf), cin, cout, P(wt), None) == 0
    dx = torch.empty(n ** 3 * cin, dtype=torch.float32, device="cuda")
    dyt = raw(dy)
    assert lib().isis_conv3_fwd(P(dyt), n, cout, P(wt), None, cin, 0, None, P(dx), None) == 0
    got = dx.cpu().numpy().reshape(n, n, n, cin)
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.abs(ref).max()


# Data gradients launch the forward kernel with the channel counts swapped;
# at sides >= 64 these are the LDS-staged instantiations (32,16), (64,32),
# (64,128), (32,96) and the ring kernel for 16 input channels (16,48).
@pytest.mark.parametrize("cin,cout", [(16, 32), (32, 64), (128, 64), (96, 32), (48, 16)])
@pytest.mark.parametrize("n", [64, 128])
def test_conv_data_gradient_staged(cin, cout, n):
    """The adjoint convolution at the sizes training runs it (128^3 samples:
    level 0 at 128, level 1 at 64), checked on eight 8^3 blocks with the
    oracle's adjoint on each block's one-voxel periodic halo."""
    rng = np.random.default_rng(cin * 11 + cout + n)
    dy = U.bf16(rng.standard_normal((n, n, n, cout)))
    W = rng.standard_normal((27, cout, cin)) * 0.1
    Wq = U.bf16(W)
    wt = torch.empty(27 * cin * cout, dtype=torch.int16, device="cuda")
    wf = torch.from_numpy(W.astype(np.float32)).cuda()
    assert lib().isis_conv3_flip_weights(P(wf), cin, cout, P(wt), None) == 0
    dx = torch.empty(n ** 3 * cin, dtype=torch.float32, device="cuda")
    dyt = raw(dy)
    assert lib().isis_conv3_fwd(P(dyt), n, cout, P(wt), None, cin, 0, None, P(dx), None) == 0
    got = dx.cpu().numpy().reshape(n, n, n, cin)
    corners = [(0, 0, 0), (n - 4, n - 4, n - 4), (n // 2 - 3, 5, n - 60), (7, n - 8, 28)]
    corners += [tuple(int(c) for c in rng.integers(0, n, 3)) for _ in range(4)]
    for c in corners:
        idx = [(c[d] - 1 + np.arange(10)) % n for d in range(3)]
        ref = U.conv3_bwd_data(dy[np.ix_(*idx)], Wq)[1:9, 1:9, 1:9]
        sel = np.ix_(idx[0][1:9], idx[1][1:9], idx[2][1:9])
        assert np.max(np.abs(got[sel] - ref)) <= 1e-5 * np.abs(ref).max(), c


@pytest.mark.parametrize("cin,cout", SHAPES)
@pytest.mark.parametrize("n", [2, 8, 32, 64])
def test_conv_weight_gradient(cin, cout, n):
    rng = np.random.default_rng(5 * cin + cout + n)
    x = U.bf16(rng.standard_normal((n, n, n, cin)))
    dy = U.bf16(rng.standard_normal((n, n, n, cout)))
    ref = U.conv3_bwd_weight(x, dy)
    refb = dy.sum(axis=(0, 1, 2))
    ws_bytes = lib().isis_conv3_bwd_weight_workspace(n, cin, cout)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    dw = torch.empty(27 * cout * cin, dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    xt, dyt = raw(x), raw(dy)
    rc = lib().isis_conv3_bwd_weight(P(xt), n, cin, P(dyt), cout, P(dw), P(db), P(ws),
                                     ws_bytes, None)
    assert rc == 0
    got = dw.cpu().numpy().reshape(27, cout, cin)
    scale = np.sqrt(n ** 3) * 3
    assert np.max(np.abs(got - ref)) <= 2e-5 * scale
    assert np.max(np.abs(db.cpu().numpy() - refb)) <= 2e-5 * scale
    # deterministic
    dw2 = torch.empty_like(dw)
    lib().isis_conv3_bwd_weight(P(xt), n, cin, P(dyt), cout, P(dw2), None, P(ws),
                                ws_bytes, None)
    assert torch.equal(dw, dw2)


def _sample(n, seed):
    rng = np.random.default_rng(seed)
    eta = np.exp(1.2 * rng.standard_normal((n, n, n)))
    cold = np.sqrt(np.maximum(0.0, 1.0 - 0.3 * eta))
    target = cold + 0.05 * rng.standard_normal((n, n, n))
    return eta, cold, target


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n", [16, 32, 64])
def test_network_forward(n):
    """The prediction against the FP64 reference network with bfloat16
    storage.  At 64^3 the level-0 convolutions take the LDS-staged kernels and
    the last decoder stage reads its upsampled and skip inputs directly."""
    from paper_1307_6748_amd import warmstart as W
    eta, cold, _ = _sample(n, 11)
    p = W.init_params(3)
    p[-1] = 0.05
    net = W.WarmStart(params=p)
    out = torch.empty(n ** 3, dtype=torch.float32, device="cuda")
    ge, gc = torch.from_numpy(eta).cuda(), torch.from_numpy(cold).cuda()
    guess = net.predict(ge, gc, 0.8, guess=torch.empty_like(ge), out=out)
    ref, _ = U.forward(p.astype(np.float64), U.make_input(eta, 0.8, cold), bf=True)
    got = out.cpu().numpy().reshape(n, n, n)
    assert _rel(got, ref) < 1e-2, _rel(got, ref)
    assert np.allclose(guess.cpu().numpy().reshape(n, n, n), cold + got, rtol=0, atol=1e-7)


def test_network_gradient_and_adam():
    from paper_1307_6748_amd import warmstart as W
    n = 16
    eta, cold, target = _sample(n, 12)
    p = W.init_params(4)
    p[-1] = 0.05
    net = W.WarmStart(params=p)
    ge, gc, gt = (torch.from_numpy(v).cuda() for v in (eta, cold, target))
    grad = torch.empty(W.param_count(), dtype=torch.float32, device="cuda")
    lr = 1e-3
    loss = net.train_step(ge, gc, gt, 0.8, lr, grad=grad)
    p64 = p.astype(np.float64)
    out, cache = U.forward(p64, U.make_input(eta, 0.8, cold), bf=True)
    g_ref = U.backward(p64, cache, out, target - cold, bf=True)
    assert abs(loss - U.mse(out, target - cold)) <= 2e-2 * U.mse(out, target - cold)
    g = grad.cpu().numpy().astype(np.float64)
    assert _rel(g, g_ref) < 5e-2, _rel(g, g_ref)
    # per layer, the gradients point the same way
    off = 0
    for ci, co in U.CONVS:
        k = 27 * ci * co + co
        a, b = g[off:off + k], g_ref[off:off + k]
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300)
        assert cos > 0.99, (off, cos)
        off += k
    # Adam's first step from the GPU's own gradient
    p1, _, _ = U.adam(p64, g, np.zeros_like(p64), np.zeros_like(p64), 1, lr)
    assert np.max(np.abs(net.params.cpu().numpy() - p1)) <= 1e-6


def _bf16_ulp(v):
    """One bfloat16 ulp at the magnitude of v (8 significant bits)."""
    a = np.maximum(np.abs(v), 1e-30)
    return 2.0 ** (np.floor(np.log2(a)) - 7)


# conv c reads: the input (14), the previous output, a pooled input (15-17) or
# a concatenation (18-20); ids as in isis_unet_tensor
CONV_INPUT = {0: 14, 1: 0, 2: 15, 3: 2, 4: 16, 5: 4, 6: 17, 7: 6, 8: 18, 9: 8, 10: 19,
              11: 10, 12: 20, 13: 12}


def _forward_64():
    from paper_1307_6748_amd import warmstart as W
    n = 64
    eta, cold, target = _sample(n, 21)
    p = W.init_params(5)
    p[-1] = 0.05
    net = W.WarmStart(params=p)
    ge, gc = torch.from_numpy(eta).cuda(), torch.from_numpy(cold).cuda()
    out = net.forward(ge, gc, 0.7)
    torch.cuda.synchronize()
    return net, p.astype(np.float64), eta, cold, target, out.cpu().numpy().reshape(n, n, n)


def test_network_layers_elementwise_64():
    """Every step of the 64^3 forward pass on the GPU's own input of that step
    (the staged, ring and concatenation-reading kernels are all on this path):
    each convolution's bf16 output is the rounding of the exact result or one
    ulp off, pooling is the exact mean rounded, concatenations are copies, the
    head is the FP32 dot product."""
    net, p, eta, cold, _, out = _forward_64()
    n = 64
    convs, (wh, bh) = U.split_params(p)
    T = {i: net.tensor(n, i) for i in range(22)}
    x0 = U.make_input(eta, 0.7, cold)
    assert np.array_equal(T[14], U.bf16(x0))
    worst = 0.0
    u32 = 2.0 ** -24
    for c in range(14):
        W, b = convs[c]
        X, Wq, bb = T[CONV_INPUT[c]], U.bf16(W), b.astype(np.float32).astype(np.float64)
        pre = U.conv3(X, Wq, bb)
        ref = U.bf16(np.maximum(pre, 0.0))
        got = T[c]
        diff = np.abs(got - ref)
        # got = bf16(s), s the FP32 sum; |s - pre| <= gamma_K sum|terms|
        # (K = 27 cin products, gamma_K = K u / (1 - K u)), so got and ref are
        # at most one ulp plus that apart (the ReLU included)
        K = 27 * X.shape[3] + 2
        delta = K * u32 / (1 - K * u32) * (U.conv3(np.abs(X), np.abs(Wq)) + np.abs(bb))
        ok = diff <= _bf16_ulp(np.maximum(np.abs(ref), np.abs(got))) + delta
        frac = float(np.mean(diff > 0))
        worst = max(worst, frac)
        assert ok.all(), (c, float((diff - _bf16_ulp(np.maximum(np.abs(ref), np.abs(got))) -
                                    delta).max()))
        assert frac <= 2e-3, (c, frac)
    for tid, src in ((15, 1), (16, 3), (17, 5)):
        ref = U.bf16(U.pool2(T[src]))
        d = np.abs(T[tid] - ref)
        bound = _bf16_ulp(np.maximum(np.abs(ref), np.abs(T[tid]))) + 8 * u32 * U.pool2(np.abs(T[src]))
        assert (d <= bound).all() and np.mean(d > 0) <= 1e-3, tid
    for tid, lo, sk in ((18, 7, 5), (19, 9, 3), (20, 11, 1)):
        assert np.array_equal(T[tid], np.concatenate([U.up2(T[lo]), T[sk]], axis=3)), tid
    head = T[13] @ wh + bh[0]
    assert np.max(np.abs(out - head)) <= 1e-6 * (np.abs(T[13]) @ np.abs(wh)).max()
    assert np.array_equal(T[21], out)
    print(f"largest fraction of 1-ulp roundings per layer: {worst:.2e}")


def test_network_output_elementwise_64():
    """The whole 64^3 forward pass against the FP64 reference network with
    bf16 storage, element by element: one-ulp rounding differences of early
    layers propagate, so each output may differ by a few bf16 ulps of the
    output's scale (its RMS); relative L2 as a summary."""
    _, p, eta, cold, _, out = _forward_64()
    ref, _ = U.forward(p, U.make_input(eta, 0.7, cold), bf=True)
    scale = np.sqrt(np.mean(ref ** 2))
    err = np.abs(out - ref) / (_bf16_ulp(scale))
    print(f"output: max |diff| = {err.max():.2f} ulp of the RMS, 99.9% {np.quantile(err, 0.999):.2f}, "
          f"rel. L2 {_rel(out, ref):.2e}")
    assert err.max() <= 4.0  # measured 0.87
    assert _rel(out, ref) < 1e-2


def test_network_gradient_elementwise_64():
    """The 64^3 gradient element by element against the reference backward
    pass run on the GPU's own activations (same ReLU pattern): per parameter
    within a few bf16 ulps of the RMS gradient of its layer, or 5 % of its own
    size; relative L2 as a summary."""
    net, p, eta, cold, target, out = _forward_64()
    n = 64
    ge, gc, gt = (torch.from_numpy(v).cuda() for v in (eta, cold, target))
    grad, loss = net.backward(gc, gt)
    g = grad.cpu().numpy().astype(np.float64)
    cache = {"in": net.tensor(n, 14)}
    for c in range(14):
        cache[f"o{c}"] = net.tensor(n, c)
        cache[f"m{c}"] = cache[f"o{c}"] > 0
    cache["Ws"] = [U.bf16(W) for W, _ in U.split_params(p)[0]]
    g_ref = U.backward(p, cache, out.astype(np.float64), target - cold, bf=True)
    assert abs(loss - U.mse(out, target - cold)) <= 1e-4 * U.mse(out, target - cold)
    off = 0
    worst = 0.0
    for c, (ci, co) in enumerate(U.CONVS + [(16, 1)]):
        k = 27 * ci * co + co if c < 14 else 17
        a, b = g[off:off + k], g_ref[off:off + k]
        rms = np.sqrt(np.mean(b ** 2))
        r = np.abs(a - b) / np.maximum(_bf16_ulp(rms), 0.05 * np.abs(b))
        worst = max(worst, float(r.max()))
        assert r.max() <= 1.0, (c, float(r.max()))  # measured <= 0.08
        off += k
    print(f"gradient: worst layer max |diff| {worst:.2f} (ulps of the layer RMS or 5 %), "
          f"rel. L2 {_rel(g, g_ref):.2e}")
    assert _rel(g, g_ref) < 1e-3  # measured 7e-6


def test_training_step_parts_equal_the_fused_step():
    """isis_unet_forward + isis_unet_backward + isis_unet_adam_step give
    bit for bit what isis_unet_train_step gives (same kernels, same order),
    and the Adam step is the reference update of the GPU's gradient."""
    from paper_1307_6748_amd import warmstart as W
    n = 32
    eta, cold, target = _sample(n, 31)
    p = W.init_params(6)
    ge, gc, gt = (torch.from_numpy(v).cuda() for v in (eta, cold, target))
    a1, a2 = W.WarmStart(params=p), W.WarmStart(params=p)
    g1 = torch.empty_like(a1.params)
    loss1 = a1.train_step(ge, gc, gt, 0.9, 2e-3, grad=g1)
    out2 = a2.forward(ge, gc, 0.9)
    g2, loss2 = a2.backward(gc, gt)
    a2.adam_step(g2, 2e-3)
    torch.cuda.synchronize()
    assert loss1 == loss2
    assert torch.equal(g1, g2) and torch.equal(a1.params, a2.params)
    assert torch.equal(a1.m, a2.m) and torch.equal(a1.v, a2.v)
    p1, m1, v1 = U.adam(p.astype(np.float64), g2.cpu().numpy().astype(np.float64),
                        np.zeros(p.size), np.zeros(p.size), 1, 2e-3)
    assert np.max(np.abs(a2.params.cpu().numpy() - p1)) <= 1e-6
    assert out2.numel() == n ** 3


def test_training_resumes_bitwise_from_a_checkpoint(tmp_path):
    """A run stopped after some steps and resumed from its checkpoint
    (parameters, Adam moments and step, shuffling state) takes exactly the
    steps the uninterrupted run takes: the parameters agree bit for bit."""
    from paper_1307_6748_amd import warmstart as W
    n = 16
    pairs = []
    for q in range(5):
        eta, cold, target = _sample(n, 40 + q)
        pairs.append((torch.from_numpy(eta).cuda(), 0.5 + 0.1 * q, torch.from_numpy(cold).cuda(),
                      torch.from_numpy(target).cuda()))
    tr = W.Trainer(W.WarmStart(params=W.init_params(8)), len(pairs), epochs=3, lr=2e-3,
                   lr_final=1e-4, seed=3)
    for _ in range(7):  # into the second epoch
        tr.step(pairs)
    ck = str(tmp_path / "ck.npz")
    tr.save_checkpoint(ck)
    for _ in range(6):  # across the next epoch boundary
        tr.step(pairs)
    tr2 = W.Trainer.load_checkpoint(ck)
    for _ in range(6):
        tr2.step(pairs)
    torch.cuda.synchronize()
    assert (tr2.k, tr2.epoch, tr2.pos) == (tr.k, tr.epoch, tr.pos)
    assert np.array_equal(tr2.order, tr.order)
    assert torch.equal(tr2.net.params, tr.net.params)
    assert torch.equal(tr2.net.m, tr.net.m) and torch.equal(tr2.net.v, tr.net.v)
    assert tr2.net.step == tr.net.step and tr2.losses == tr.losses


def test_warm_start_judge():
    """use_guess = 2: a guess is kept only if its residual is at most what
    one cold-started V-cycle reaches (the handle's measured first-cycle
    factor after a cold solve, else desc.guess_accept or 1e-2) times r_ref.
    Noise is replaced by the cold start; a guess better than the cold start
    but not better than one cold cycle is replaced too; a near-solution is
    kept and saves cycles."""
    from paper_1307_6748_amd import solver as S
    from paper_1307_6748_amd import synth
    n, box = 32, 64.0
    eta = torch.from_numpy(synth.lognormal(n, box, 1.0, 1)).cuda()
    p = S.symmetron(1.0, 0.5)
    s = S.Solver(n, box)
    ref, st0 = s.solve(eta, p, 1.0, 1e-10)
    rho1 = st0.rel_hist[1]
    noise = torch.from_numpy(5.0 * synth.random_field(n, 2)).cuda()
    _, st1 = s.solve(eta, p, 1.0, 1e-10, phi=noise.clone(), use_guess=2)
    assert not st1.used_guess and st1.cycles == st0.cycles
    # halfway between the cold start and the solution: residual below r_ref
    # but above rho1 r_ref -> the cold start is used
    cold = S.cold_start(p, 1.0, eta)
    mid = 0.5 * (cold + ref)
    r_mid = s.residual(eta, mid, p, 1.0) / st0.r_ref
    assert rho1 < r_mid < 1.0, (rho1, r_mid)
    _, st3 = s.solve(eta, p, 1.0, 1e-10, phi=mid.clone(), use_guess=2)
    assert not st3.used_guess and st3.cycles == st0.cycles
    # an explicit threshold above the guess's residual keeps it
    s2 = S.Solver(n, box, guess_accept=min(1.0, 2.0 * r_mid))
    _, st4 = s2.solve(eta, p, 1.0, 1e-10, phi=mid.clone(), use_guess=2)
    assert st4.used_guess
    good = ref + 1e-6 * torch.from_numpy(synth.random_field(n, 3)).cuda()
    _, st2 = s.solve(eta, p, 1.0, 1e-10, phi=good, use_guess=2)
    assert st2.used_guess and st2.cycles < st0.cycles


@pytest.mark.parametrize("seed,a", [(2100, 0.6), (2101, 0.85), (2102, 1.0)])
def test_trained_warm_start_against_oracle(orc, seed, a):
    """The trained network (paper_1307_6748_amd/data) on held-out densities at
    the training spacing (h = 0.5 Mpc/h, 64^3 in a 32 Mpc/h box): its guess is
    closer to the oracle's solution than the cold start and has a smaller
    residual; the judged solve reaches the tolerance in no more V-cycles than
    the cold-started one (the judge drops a guess that one cold cycle beats)."""
    import os
    from paper_1307_6748_amd import solver as S
    from paper_1307_6748_amd import warmstart as W
    if not os.path.exists(W.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights")
    n, box = 64, 32.0
    eta_np = W.training_density(n, box, seed)
    om = orc.Model(model=orc.SYMMETRON, a=a, lambda0=1.0, a_ssb=0.5)
    ref = orc.solve(om, eta_np, box, tol=1e-11).phi
    net = W.WarmStart.load()
    p = S.symmetron(1.0, 0.5)
    eta = torch.from_numpy(eta_np).cuda()
    cold = S.cold_start(p, a, eta)
    guess = net.predict(eta, cold, a)
    g, c = guess.cpu().numpy().reshape(n, n, n), cold.cpu().numpy().reshape(n, n, n)
    err_g = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    err_c = np.linalg.norm(c - ref) / np.linalg.norm(ref)
    assert err_g < 0.5 * err_c
    s = S.Solver(n, box)
    r_g = s.residual(eta, guess, p, a)
    assert r_g < s.residual(eta, cold, p, a)
    _, stc = s.solve(eta, p, a, 1e-8)
    _, stw = s.solve(eta, p, a, 1e-8, phi=guess.clone(), use_guess=2)
    print(f"seed {seed} a={a}: CNN rel. L2 error {err_g:.3e}, cold start {err_c:.3e}; guess "
          f"residual {r_g / stc.r_ref:.3e} r_ref, first cold cycle {stc.rel_hist[1]:.3e}; "
          f"used {stw.used_guess}, cycles {stw.cycles} vs {stc.cycles} cold")
    assert stw.status == 0
    assert stw.used_guess == (r_g <= stc.rel_hist[1] * stc.r_ref)
    assert stw.cycles <= stc.cycles
