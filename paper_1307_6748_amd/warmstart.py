"""Learned warm start for the FAS solve: a BF16 3D U-Net on the GPU.

The network (see include/isis_mg.h) predicts phi* - phi_cold from
(log eta, a, phi_cold).  Training pairs (eta, a) -> phi* come from the FAS
solver itself; training and inference run in the library's kernels (forward,
backward, Adam); this module only marshals tensors and runs the loop.  The
solver remains the judge: Solver.solve(..., use_guess=2) keeps the prediction
only if its residual is at most what one cold-started V-cycle reaches, so it
cannot cost a cycle.  Training can be checkpointed and resumed bit for bit
(parameters, Adam moments, step count and the shuffling state).
"""
from __future__ import annotations

import ctypes as C
import json
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

    def forward(self, eta: torch.Tensor, cold: torch.Tensor, a: float,
                out: torch.Tensor | None = None) -> torch.Tensor:
        """Network output (FP32) with every activation kept for backward()."""
        n = round(eta.numel() ** (1 / 3))
        ws = self._workspace(n, True)
        out = torch.empty(n ** 3, dtype=torch.float32, device="cuda") if out is None else out
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        _ok(A.lib().isis_unet_forward(_p(self.params), _p(eta), _p(cold), float(a), n, _p(out),
                                      _p(ws), ws.numel(), st))
        return out

    def backward(self, cold: torch.Tensor, target: torch.Tensor,
                 grad: torch.Tensor | None = None) -> tuple[torch.Tensor, float]:
        """Gradient of the loss after forward() (same grid); returns (grad, loss)."""
        n = round(cold.numel() ** (1 / 3))
        ws = self._workspace(n, True)
        grad = torch.empty_like(self.params) if grad is None else grad
        loss = C.c_float()
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        _ok(A.lib().isis_unet_backward(_p(self.params), _p(cold), _p(target), n, _p(ws),
                                       ws.numel(), _p(grad), C.byref(loss), st))
        return grad, loss.value

    def adam_step(self, grad: torch.Tensor, lr: float):
        """One Adam update of the parameters from grad."""
        self.step += 1
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        _ok(A.lib().isis_unet_adam_step(_p(self.params), _p(grad), _p(self.m), _p(self.v),
                                        self.params.numel(), self.step, float(lr), st))

    def tensor(self, n: int, tid: int) -> np.ndarray:
        """Activation tid of the last forward() on an n^3 grid (see
        isis_unet_tensor), as float64 [x][y][z][c] (the head output: [x][y][z])."""
        ws = self._workspace(n, True)
        ptr, vox, ch = C.c_void_p(), C.c_long(), C.c_int()
        _ok(A.lib().isis_unet_tensor(_p(ws), n, int(tid), C.byref(ptr), C.byref(vox),
                                     C.byref(ch)))
        off = ptr.value - ws.data_ptr()
        count = vox.value * ch.value
        torch.cuda.synchronize()
        if tid == 21:
            raw = ws[off: off + 4 * count].cpu().numpy().view(np.float32)
            return raw.astype(np.float64).reshape(n, n, n)
        raw = ws[off: off + 2 * count].cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        m = round(vox.value ** (1 / 3))
        return raw.view(np.float32).astype(np.float64).reshape(m, m, m, ch.value)

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
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
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


class Trainer:
    """Adam over the pairs in shuffled order with a geometrically decayed
    learning rate.  Its state (the network's parameters, Adam moments and step,
    the epoch, the position in the epoch's order, the order itself and the
    shuffling generator) can be saved and restored, so that a resumed run
    takes exactly the steps the uninterrupted run would have taken."""

    def __init__(self, net: WarmStart, npairs: int, epochs: int, lr: float = 1e-3,
                 lr_final: float = 1e-4, seed: int = 0):
        self.net, self.npairs, self.epochs = net, int(npairs), int(epochs)
        self.lr, self.lr_final = float(lr), float(lr_final)
        self.rng = np.random.default_rng(seed)
        self.epoch, self.pos, self.k = 0, 0, 0
        self.order = self.rng.permutation(self.npairs)
        self.ep_loss = 0.0
        self.losses: list = []

    def done(self) -> bool:
        return self.epoch >= self.epochs

    def lr_at(self, k: int) -> float:
        total = self.epochs * self.npairs
        return self.lr * (self.lr_final / self.lr) ** (k / max(1, total - 1))

    def step(self, pairs) -> float:
        """One training step on the next pair of the shuffled order."""
        eta, a, cold, phi = pairs[int(self.order[self.pos])]
        loss = self.net.train_step(eta, cold, phi, a, self.lr_at(self.k))
        self.k += 1
        self.pos += 1
        self.ep_loss += loss
        if self.pos == self.npairs:
            self.losses.append(self.ep_loss / self.npairs)
            self.epoch += 1
            self.pos, self.ep_loss = 0, 0.0
            self.order = self.rng.permutation(self.npairs)
        return loss

    def save_checkpoint(self, path: str):
        net = self.net
        state = dict(npairs=self.npairs, epochs=self.epochs, lr=self.lr, lr_final=self.lr_final,
                     epoch=self.epoch, pos=self.pos, k=self.k, ep_loss=self.ep_loss,
                     losses=self.losses, adam_step=net.step,
                     rng=self.rng.bit_generator.state)
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        np.savez(path, params=net.params.cpu().numpy(), adam_m=net.m.cpu().numpy(),
                 adam_v=net.v.cpu().numpy(), order=np.asarray(self.order, dtype=np.int64),
                 state=json.dumps(state))

    @staticmethod
    def load_checkpoint(path: str) -> "Trainer":
        with np.load(path, allow_pickle=False) as z:
            st = json.loads(str(z["state"]))
            net = WarmStart(params=z["params"])
            net.m.copy_(torch.from_numpy(z["adam_m"]).cuda())
            net.v.copy_(torch.from_numpy(z["adam_v"]).cuda())
            order = z["order"].copy()
        net.step = int(st["adam_step"])
        tr = Trainer(net, st["npairs"], st["epochs"], st["lr"], st["lr_final"])
        tr.rng.bit_generator.state = st["rng"]
        tr.epoch, tr.pos, tr.k = int(st["epoch"]), int(st["pos"]), int(st["k"])
        tr.ep_loss, tr.losses, tr.order = float(st["ep_loss"]), list(st["losses"]), order
        return tr


def train(net: WarmStart, pairs, epochs: int, lr: float = 1e-3, lr_final: float = 1e-4,
          seed: int = 0, log=None, checkpoint: str | None = None,
          trainer: Trainer | None = None) -> list:
    """Run a Trainer to the end (a new one, or `trainer` to resume); with
    `checkpoint`, its state is saved there after every epoch."""
    tr = trainer or Trainer(net, len(pairs), epochs, lr, lr_final, seed)
    t0 = time.time()
    while not tr.done():
        ep = tr.epoch
        tr.step(pairs)
        if tr.epoch != ep:
            if log:
                log(f"epoch {tr.epoch}/{tr.epochs}: mean loss {tr.losses[-1]:.3e} "
                    f"({time.time() - t0:.1f}s)")
            if checkpoint:
                tr.save_checkpoint(checkpoint)
    return tr.losses
