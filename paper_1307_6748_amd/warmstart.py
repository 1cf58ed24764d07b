"""Learned warm start for the FAS solve: a BF16 3D U-Net on the GPU.

The network (see include/isis_mg.h) predicts phi* - phi_cold from
(log eta, a, phi_cold).  Training pairs (eta, a) -> phi* come from the FAS
solver itself; training and inference run in the library's kernels (forward,
backward, Adam); this module only marshals tensors and runs the loop.  The
solver remains the judge: Solver.solve(..., use_guess=2) falls back to the
cold start when the prediction's residual is not below the cold start's.
"""
from __future__ import annotations

import ctypes as C
import os
import time

import numpy as np
import torch

from . import _capi as A
from . import solver as S
from . import synth

# (cin, cout) of the 14 convolutions, in parameter order (see the header).
CONVS = [(16, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (64, 64), (64, 64),
         (128, 64), (64, 64), (96, 32), (32, 32), (48, 16), (16, 16)]

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "data", "unet_symmetron_128.npz")


def param_count() -> int:
    return int(A.lib().isis_unet_param_count())


def init_params(seed: int) -> np.ndarray:
    """He-normal convolution weights (fan-in 27 cin), zero biases, small head."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in CONVS:
        parts.append(rng.standard_normal(27 * co * ci) * np.sqrt(2.0 / (27 * ci)))
        parts.append(np.zeros(co))
    parts.append(rng.standard_normal(16) * 0.01)
    parts.append(np.zeros(1))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == param_count()
    return p


def _ok(rc: int):
    if rc != A.ISIS_OK:
        raise S.IsisError(rc, A.lib().isis_unet_last_error().decode())


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class WarmStart:
    """U-Net parameters (FP32, device) plus Adam state and workspaces."""

    def __init__(self, params: np.ndarray | None = None, seed: int = 0):
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        if p.size != param_count():
            raise ValueError(f"expected {param_count()} parameters, got {p.size}")
        self.params = torch.from_numpy(p.copy()).cuda()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._ws = {}

    def _workspace(self, n: int, training: bool) -> torch.Tensor:
        key = (n, training)
        if key not in self._ws:
            nbytes = A.lib().isis_unet_workspace_size(n, 1 if training else 0)
            if nbytes == 0:
                raise ValueError(f"grid {n}^3 not supported by the warm start")
            self._ws = {}  # keep one workspace at a time (they can be large)
            self._ws[key] = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        return self._ws[key]

    def predict(self, eta: torch.Tensor, cold: torch.Tensor, a: float,
                guess: torch.Tensor | None = None, out: torch.Tensor | None = None):
        """guess = cold + network(log eta, a, cold) (FP64); out = raw output (FP32)."""
        n = round(eta.numel() ** (1 / 3))
        ws = self._workspace(n, False)
        if guess is None and out is None:
            guess = torch.empty_like(eta)
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        _ok(A.lib().isis_unet_predict(_p(self.params), _p(eta), _p(cold), float(a), n, _p(guess),
                                      _p(out), _p(ws), ws.numel(), st))
        return guess if guess is not None else out

    def train_step(self, eta, cold, target, a: float, lr: float, grad=None) -> float:
        n = round(eta.numel() ** (1 / 3))
        ws = self._workspace(n, True)
        self.step += 1
        loss = C.c_float()
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        _ok(A.lib().isis_unet_train_step(_p(self.params), _p(self.m), _p(self.v), self.step,
                                         float(lr), _p(eta), _p(cold), _p(target), float(a), n,
                                         _p(ws), ws.numel(), C.byref(loss), _p(grad), st))
        return loss.value

    def save(self, path: str, **meta):
        os.makedirs(os.path.dirname(path), exist_ok=True)
        np.savez(path, params=self.params.cpu().numpy(), **meta)

    @staticmethod
    def load(path: str = DEFAULT_WEIGHTS) -> "WarmStart":
        with np.load(path, allow_pickle=False) as z:
            return WarmStart(params=z["params"])


# ---------------------------------------------------------------------------
# Training data and training loop (symmetron, a ~ U[0.5, 1]).
# ---------------------------------------------------------------------------

def training_density(n: int, box: float, seed: int, points_per_halo: int = 50_000) -> np.ndarray:
    """Lognormal (sigma_delta = 2) plus NFW haloes at the number density of the
    512^3 workload (400 per (256 Mpc/h)^3), seeded."""
    haloes = max(1, int(round(400 * (box / 256.0) ** 3)))
    return synth.lognormal_nfw(n, box, 2.0, seed, haloes, seed + 100_000,
                               points_per_halo=points_per_halo)


def make_pairs(n: int, box: float, seeds, model: S.ModelParams, a_seed: int = 7,
               tol: float = 1e-10, log=None):
    """(eta, a, phi_cold, phi*) on the GPU for each seed; a ~ U[0.5, 1]."""
    rng = np.random.default_rng(a_seed)
    solver = S.Solver(n, box, max_cycles=100)
    pairs = []
    for q, sd in enumerate(seeds):
        a = float(rng.uniform(0.5, 1.0))
        eta = torch.from_numpy(training_density(n, box, sd)).cuda()
        cold = S.cold_start(model, a, eta)
        phi, st = solver.solve(eta, model, a, tol)
        pairs.append((eta, a, cold, phi))
        if log and (q + 1) % 20 == 0:
            log(f"pair {q + 1}/{len(seeds)}: a={a:.3f} cycles={st.cycles}")
    return pairs


def train(net: WarmStart, pairs, epochs: int, lr: float = 1e-3, lr_final: float = 1e-4,
          seed: int = 0, log=None) -> list:
    """Adam over the pairs in shuffled order, lr decayed geometrically."""
    rng = np.random.default_rng(seed)
    total = epochs * len(pairs)
    losses = []
    k = 0
    t0 = time.time()
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        ep_loss = 0.0
        for idx in order:
            eta, a, cold, phi = pairs[idx]
            lr_k = lr * (lr_final / lr) ** (k / max(1, total - 1))
            ep_loss += net.train_step(eta, cold, phi, a, lr_k)
            k += 1
        losses.append(ep_loss / len(pairs))
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean loss {losses[-1]:.3e} ({time.time() - t0:.1f}s)")
    return losses
