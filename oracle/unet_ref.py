"""FP64 NumPy reference of the learned warm start (test infrastructure only).

A 3D U-Net maps (log density, expansion factor, cold-start field) to the
correction phi* - phi_cold of the scalar-field solve.  This module is the
plain, slow reference the GPU kernels are checked against; only the tests,
the smoke check and the CPU-baseline leg of the benchmark use it.  It shares
no code with the GPU library.

Network (4 levels, channels 16/32/64/64, 3x3x3 convolutions with periodic
padding, ReLU, 2x2x2 average pooling, nearest-neighbour upsampling, skip
connections by channel concatenation [upsampled, skip], 1x1x1 head):

    enc0: 16->16, 16->16          (input padded from 3 to 16 channels)
    enc1: pool, 16->32, 32->32
    enc2: pool, 32->64, 64->64
    bot:  pool, 64->64, 64->64
    dec2: up, cat(64+64), 128->64, 64->64
    dec1: up, cat(64+32), 96->32, 32->32
    dec0: up, cat(32+16), 48->16, 16->16
    head: 16->1 (1x1x1, no ReLU)

Tensors are channels-last [x][y][z][c].  A 3x3x3 convolution reads the input
at (i+di, j+dj, k+dk), tap index t = (di+1)*9 + (dj+1)*3 + (dk+1), and its
weights are stored W[t][cout][cin] followed by the bias b[cout]; the flat
parameter vector concatenates the 14 convolutions in the order above and
then the head (w[16], b[1]).  The same layout is used by the GPU library.

Inputs: channel 0 = log(eta)/2, channel 1 = a, channel 2 = phi_cold,
channels 3..15 = 0.

bf16=True emulates the GPU's storage precision: weights and every stored
activation / gradient tensor are rounded to bfloat16 (round to nearest even)
where the GPU stores them; sums are exact (FP64 here, FP32 on the GPU).
"""
from __future__ import annotations

import numpy as np

CONVS = [(16, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (64, 64), (64, 64),
         (128, 64), (64, 64), (96, 32), (32, 32), (48, 16), (16, 16)]
IN_CH = 16
HEAD_IN = 16


def param_count() -> int:
    return sum(27 * ci * co + co for ci, co in CONVS) + HEAD_IN + 1


def split_params(p):
    """Views (W[27,cout,cin], b[cout]) per convolution, then (w_head, b_head)."""
    out, off = [], 0
    for ci, co in CONVS:
        W = p[off: off + 27 * co * ci].reshape(27, co, ci)
        off += 27 * co * ci
        b = p[off: off + co]
        off += co
        out.append((W, b))
    wh = p[off: off + HEAD_IN]
    off += HEAD_IN
    bh = p[off: off + 1]
    return out, (wh, bh)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = np.where(np.isnan(f), u, r)  # NaN passes through
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def taps():
    return [(di, dj, dk) for di in (-1, 0, 1) for dj in (-1, 0, 1) for dk in (-1, 0, 1)]


def shifted(x, d):
    """y[i,j,k] = x[i+di, j+dj, k+dk] (periodic)."""
    return np.roll(x, shift=(-d[0], -d[1], -d[2]), axis=(0, 1, 2))


def conv3(x, W, b=None):
    """y[v, co] = sum_t sum_ci x[v + d_t, ci] W[t, co, ci] + b[co]."""
    y = np.zeros(x.shape[:3] + (W.shape[1],))
    for t, d in enumerate(taps()):
        y += shifted(x, d) @ W[t].T
    if b is not None:
        y += b
    return y


def conv3_bwd_data(dy, W):
    """Adjoint of conv3 in x: dx[v, ci] = sum_t sum_co dy[v - d_t, co] W[t, co, ci]."""
    dx = np.zeros(dy.shape[:3] + (W.shape[2],))
    for t, d in enumerate(taps()):
        dx += shifted(dy @ W[t], (-d[0], -d[1], -d[2]))
    return dx


def conv3_bwd_weight(x, dy):
    """dW[t, co, ci] = sum_v dy[v, co] x[v + d_t, ci]."""
    co, ci = dy.shape[3], x.shape[3]
    dW = np.zeros((27, co, ci))
    dyf = dy.reshape(-1, co)
    for t, d in enumerate(taps()):
        dW[t] = dyf.T @ shifted(x, d).reshape(-1, ci)
    return dW


def pool2(x):
    n0, n1, n2, c = x.shape
    return x.reshape(n0 // 2, 2, n1 // 2, 2, n2 // 2, 2, c).mean(axis=(1, 3, 5))


def pool2_bwd(dy):
    return up2(dy) / 8.0


def up2(x):
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def up2_bwd(dy):
    return 8.0 * pool2(dy)


def make_input(eta, a, phi_cold):
    n = eta.shape[0]
    x = np.zeros((n, n, n, IN_CH))
    x[..., 0] = np.log(eta) / 2.0
    x[..., 1] = a
    x[..., 2] = phi_cold
    return x


def forward(p, x, bf=False, masks=None):
    """Network output (n^3 field) and the cache the backward pass needs.

    masks (the "m{i}" entries of another call's cache) freezes the ReLU
    pattern: the network is then polynomial in the parameters, which makes
    finite-difference checks of the gradient exact up to O(eps^2)."""
    q = bf16 if bf else (lambda v: v)
    convs, (wh, bh) = split_params(np.asarray(p, dtype=np.float64))
    cache = {"in": q(x)}
    Ws = [q(W) for W, _ in convs]

    def cr(i, inp):
        pre = conv3(inp, Ws[i], convs[i][1])
        m = (pre > 0) if masks is None else masks[f"m{i}"]
        out = q(pre * m)
        cache[f"o{i}"] = out
        cache[f"m{i}"] = m
        return out

    h = cache["in"]
    h = cr(0, h)
    s0 = cr(1, h)
    h = cr(2, q(pool2(s0)))
    s1 = cr(3, h)
    h = cr(4, q(pool2(s1)))
    s2 = cr(5, h)
    h = cr(6, q(pool2(s2)))
    h = cr(7, h)
    h = cr(8, np.concatenate([up2(h), s2], axis=3))
    h = cr(9, h)
    h = cr(10, np.concatenate([up2(h), s1], axis=3))
    h = cr(11, h)
    h = cr(12, np.concatenate([up2(h), s0], axis=3))
    h = cr(13, h)
    out = h @ wh + bh[0]
    cache["Ws"] = Ws
    return out, cache


def mse(out, target):
    return float(np.mean((out - target) ** 2))


def backward(p, cache, out, target, bf=False):
    """Gradient of mse(out, target) with respect to the flat parameters."""
    q = bf16 if bf else (lambda v: v)
    convs, (wh, bh) = split_params(np.asarray(p, dtype=np.float64))
    Ws = cache["Ws"]
    g = np.zeros(param_count())
    gconv = [None] * 14
    nvox = out.size
    dout = 2.0 * (out - target) / nvox
    d13 = cache["o13"]
    g_wh = (d13.reshape(-1, HEAD_IN) * dout.reshape(-1, 1)).sum(axis=0)
    g_bh = dout.sum()
    dh = q(dout[..., None] * wh[None, None, None, :])

    def back(i, dh_out, inp):
        dpre = q(dh_out * cache[f"m{i}"])
        gconv[i] = (conv3_bwd_weight(inp, dpre), dpre.sum(axis=(0, 1, 2)))
        return q(conv3_bwd_data(dpre, Ws[i]))

    o = cache
    c12 = np.concatenate([up2(o["o11"]), o["o1"]], axis=3)
    c10 = np.concatenate([up2(o["o9"]), o["o3"]], axis=3)
    c8 = np.concatenate([up2(o["o7"]), o["o5"]], axis=3)
    dh = back(13, dh, o["o12"])
    dh = back(12, dh, c12)
    d_up, d_s0 = dh[..., :32], dh[..., 32:]
    dh = q(up2_bwd(d_up))
    dh = back(11, dh, o["o10"])
    dh = back(10, dh, c10)
    d_up, d_s1 = dh[..., :64], dh[..., 64:]
    dh = q(up2_bwd(d_up))
    dh = back(9, dh, o["o8"])
    dh = back(8, dh, c8)
    d_up, d_s2 = dh[..., :64], dh[..., 64:]
    dh = q(up2_bwd(d_up))
    dh = back(7, dh, o["o6"])
    dh = back(6, dh, q(pool2(o["o5"])))
    dh = q(d_s2 + q(pool2_bwd(dh)))
    dh = back(5, dh, o["o4"])
    dh = back(4, dh, q(pool2(o["o3"])))
    dh = q(d_s1 + q(pool2_bwd(dh)))
    dh = back(3, dh, o["o2"])
    dh = back(2, dh, q(pool2(o["o1"])))
    dh = q(d_s0 + q(pool2_bwd(dh)))
    dh = back(1, dh, o["o0"])
    back(0, dh, o["in"])
    off = 0
    for (ci, co), (dW, db) in zip(CONVS, gconv):
        g[off: off + 27 * co * ci] = dW.ravel()
        off += 27 * co * ci
        g[off: off + co] = db
        off += co
    g[off: off + HEAD_IN] = g_wh
    g[off + HEAD_IN] = g_bh
    return g


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; step >= 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (fan-in 27 cin), zero biases, small head."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in CONVS:
        parts.append(rng.standard_normal(27 * co * ci) * np.sqrt(2.0 / (27 * ci)))
        parts.append(np.zeros(co))
    parts.append(rng.standard_normal(HEAD_IN) * 0.01)
    parts.append(np.zeros(1))
    return np.concatenate(parts)
