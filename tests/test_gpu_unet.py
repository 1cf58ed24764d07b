"""GPU U-Net kernels and network vs the FP64 NumPy reference (oracle/unet_ref.py).

Single convolutions get identical bfloat16 inputs on both sides, so they
agree to FP32 accumulation error.  The whole network stores every activation
in bfloat16 on both sides; FP32 vs FP64 sums can flip a rounding by one
bfloat16 ulp, which propagates, so network outputs and gradients are compared
in relative L2 norm at bfloat16-level tolerances."""
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


@pytest.mark.parametrize("cin,cout", SHAPES)
@pytest.mark.parametrize("n", [2, 8, 32])
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


def test_warm_start_judge():
    """use_guess = 2: a useless guess is replaced by the cold start; a good one
    is kept and saves cycles."""
    from paper_1307_6748_amd import solver as S
    from paper_1307_6748_amd import synth
    n, box = 32, 64.0
    eta = torch.from_numpy(synth.lognormal(n, box, 1.0, 1)).cuda()
    p = S.symmetron(1.0, 0.5)
    s = S.Solver(n, box)
    ref, st0 = s.solve(eta, p, 1.0, 1e-10)
    noise = torch.from_numpy(5.0 * synth.random_field(n, 2)).cuda()
    _, st1 = s.solve(eta, p, 1.0, 1e-10, phi=noise.clone(), use_guess=2)
    assert not st1.used_guess and st1.cycles == st0.cycles
    good = ref + 1e-6 * torch.from_numpy(synth.random_field(n, 3)).cuda()
    _, st2 = s.solve(eta, p, 1.0, 1e-10, phi=good, use_guess=2)
    assert st2.used_guess and st2.cycles < st0.cycles


@pytest.mark.parametrize("seed,a", [(2100, 0.6), (2101, 0.85), (2102, 1.0)])
def test_trained_warm_start_against_oracle(orc, seed, a):
    """The trained network (paper_1307_6748_amd/data) on held-out densities at
    the training spacing (h = 0.5 Mpc/h, 64^3 in a 32 Mpc/h box): its guess is
    closer to the oracle's solution than the cold start, has a smaller
    residual, and the judged solve reaches the tolerance."""
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
    print(f"seed {seed} a={a}: CNN rel. L2 error {err_g:.3e}, cold start {err_c:.3e}")
    assert err_g < 0.5 * err_c
    s = S.Solver(n, box)
    assert s.residual(eta, guess, p, a) < s.residual(eta, cold, p, a)
    _, stc = s.solve(eta, p, a, 1e-8)
    _, stw = s.solve(eta, p, a, 1e-8, phi=guess.clone(), use_guess=2)
    assert stw.status == 0 and stw.used_guess
    assert stw.cycles <= stc.cycles + 1
