"""Python face of the GPU solver: torch tensors in, C ABI calls out.

PyTorch provides device memory and the stream; every step of the solve runs
in the HIP kernels of libisis_mg.so.  There is no CPU path.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import torch

from . import _capi as A


class IsisError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"isis_mg error {code}: {msg}")
        self.code = code


class NotConverged(IsisError):
    pass


class Diverged(IsisError):
    pass


def _raise(code: int, msg: str):
    if code == A.ISIS_ERR_NOT_CONVERGED:
        raise NotConverged(code, msg)
    if code == A.ISIS_ERR_DIVERGED:
        raise Diverged(code, msg)
    raise IsisError(code, msg)


@dataclass
class ModelParams:
    """Model parameters (lengths in comoving Mpc/h, c = 1)."""
    model: int = A.ISIS_SYMMETRON
    lambda0: float = 1.0
    a_ssb: float = 0.5
    beta: float = 1.0
    n: float = 1.0
    fR0_abs: float = 1e-5
    omega_m: float = 0.27
    omega_l: float = 0.73
    kappa: float = 1.0
    m2: float = 0.0
    cham_alpha: float = 1.0
    cham_mu: float = 1.0
    cham_n: float = 1.0
    paper_u: bool = False

    def c(self) -> A.ModelParamsC:
        return A.ModelParamsC(int(self.model), self.lambda0, self.a_ssb, self.beta, self.n,
                              self.fR0_abs, self.omega_m, self.omega_l, self.kappa, self.m2,
                              self.cham_alpha, self.cham_mu, self.cham_n, int(bool(self.paper_u)))


def symmetron(lambda0=1.0, a_ssb=0.5, beta=1.0, omega_m=0.27) -> ModelParams:
    """omega_m enters only the fifth force (force())."""
    return ModelParams(model=A.ISIS_SYMMETRON, lambda0=lambda0, a_ssb=a_ssb, beta=beta,
                       omega_m=omega_m)


def fofr(n=1.0, fR0_abs=1e-5, omega_m=0.27, omega_l=None, paper_u=False) -> ModelParams:
    """Hu-Sawicki f(R), Sec. 4.2.  The field is u = ln(f_R/f_R0), or with
    paper_u the paper's own u = ln(a^2 |f_R|) (f_R = -a^-2 e^u)."""
    ol = 1.0 - omega_m if omega_l is None else omega_l
    return ModelParams(model=A.ISIS_FR_HS, n=n, fR0_abs=fR0_abs, omega_m=omega_m, omega_l=ol,
                       paper_u=paper_u)


def chameleon(alpha=1.0, mu=1.0, n=1.0) -> ModelParams:
    """Chameleon of Sec. 6, lap phi = alpha eta - mu phi^-(1+n) in code units,
    solved for psi = ln phi (the field the solver returns; needs eta > 0)."""
    return ModelParams(model=A.ISIS_CHAMELEON, cham_alpha=alpha, cham_mu=mu, cham_n=n)


def linear(kappa=1.0, m2=0.0) -> ModelParams:
    return ModelParams(model=A.ISIS_LINEAR, kappa=kappa, m2=m2)


H0 = 1.0 / 2997.92458  # h/Mpc with c = 1


def newtonian(omega_m: float, a: float) -> ModelParams:
    """The Poisson equation of Sec. 3.1, lap Phi = 1.5 Omega_m H0^2 (eta - 1) / a,
    as the linear model (kappa = 1.5 Omega_m H0^2 / a, m2 = 0)."""
    return linear(kappa=1.5 * omega_m * H0 * H0 / a, m2=0.0)


@dataclass
class Stats:
    status: int
    cycles: int
    cycles_fp32: int
    r_ref: float
    r0: float
    rel_res: float
    rel_hist: list = field(default_factory=list)
    ms_total: float = 0.0
    cell_updates: float = 0.0
    used_guess: bool = False
    # finest-level sweep timing (profiling on): [FP64, FP32]
    fine_sweep_ms: list = field(default_factory=lambda: [0.0, 0.0])
    fine_sweep_launches: list = field(default_factory=lambda: [0, 0])
    fine_sweep_updates: list = field(default_factory=lambda: [0.0, 0.0])
    fine_sweep_bytes: list = field(default_factory=lambda: [0.0, 0.0])
    temporal_block: int = 0  # the temporal block the solve used
    rho_hist: list = field(default_factory=list)  # per-cycle factors, [0] = 0
    safeguard_hits: int = 0  # symmetron: updates with the safeguarded denominator
    ms_smooth: float = 0.0   # profiling on: smoothing on the finest level and sides >= 256
    restriction: int = 0     # defect restriction used: 0 mean, 1 full weighting,
                             # 2 full weighting in the first two cycles, then the mean
    judged_cycles: int = 0   # cycles after which the judge ran (FP64, or FP32: judged_fp32)
    # finest-level first post-smoothing pass with the prolongation fused in
    # (profiling on): [FP64, FP32]
    fine_prol_ms: list = field(default_factory=lambda: [0.0, 0.0])
    fine_prol_launches: list = field(default_factory=lambda: [0, 0])
    fine_prol_bytes: list = field(default_factory=lambda: [0.0, 0.0])
    nu_pre: int = 2          # smoothing sweeps per level the solve used
    nu_post: int = 2
    prolongation: int = 0    # prolongation used: 0 trilinear, 1 coefficient-weighted
    judged_fp32: int = 0     # judged cycles judged by the FP32 problem's own defect

    @staticmethod
    def from_c(status: int, s: A.StatsC) -> "Stats":
        return Stats(status, s.cycles, s.cycles_fp32, s.r_ref, s.r0, s.rel_res,
                     list(s.rel_hist[: s.cycles + 1]), s.ms_total, s.cell_updates,
                     bool(s.used_guess), list(s.fine_sweep_ms), list(s.fine_sweep_launches),
                     list(s.fine_sweep_updates), list(s.fine_sweep_bytes), s.temporal_block,
                     list(s.rho_hist[: s.cycles + 1]), int(s.safeguard_hits), s.ms_smooth,
                     s.restriction, s.judged_cycles, list(s.fine_prol_ms),
                     list(s.fine_prol_launches), list(s.fine_prol_bytes), s.nu_pre, s.nu_post,
                     s.prolongation, s.judged_fp32)


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _check_field(t: torch.Tensor, n: int, name: str, dtype=torch.float64):
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() != n ** 3:
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor with {n}^3 elements")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


PRECISIONS = {"fp64": A.ISIS_FP64, "mixed": A.ISIS_MIXED}


class Solver:
    """FAS multigrid solver for one grid size (one C-ABI handle).

    The workspace is a torch uint8 tensor on the current device; kernels run
    on the torch stream current at construction.  temporal_block = -1 (the
    default) lets the library pick the sweeps per HBM pass for each model;
    0, 1, 2 force one choice (see isis_mg_desc).  prolongation = -1 (the
    default) weights the prolongation by the flux coefficient e^u for f(R)
    and uses the trilinear one otherwise; 0 / 1 force trilinear / weighted
    (weighted: f(R) and the chameleon only).  restriction = -1 (the default)
    restricts the defect for f(R) by full weighting in the first two V-cycles
    and by the 8-child mean after them (full weighting throughout with the
    trilinear prolongation), by the mean for the others; 0 / 1 force the
    mean / full weighting.
    judge_skip: skip the judge on cycles predicted to stay above tol, and
    judge FP32 cycles predicted to stay far above it by the FP32 problem's
    own defect (see isis_mg_desc.judge_skip).  nu_post = -1 (the default): one
    post-smoothing sweep for the symmetron and the chameleon, two otherwise."""

    def __init__(self, N: int, box: float, nu_pre: int = 2, nu_post: int = -1,
                 nu_coarse: int = 32, max_cycles: int = 50, precision: str = "fp64",
                 temporal_block: int = -1, fp32_floor: float = 0.0, guess_accept: float = 0.0,
                 restriction: int = -1, judge_skip: bool = False, prolongation: int = -1):
        self.N, self.box = int(N), float(box)
        self._h = None
        lib = A.lib()
        d = A.DescC(self.N, self.box, nu_pre, nu_post, nu_coarse, max_cycles,
                    PRECISIONS[precision], float(fp32_floor), temporal_block, _stream(), None, 0,
                    float(guess_accept), int(restriction), int(bool(judge_skip)),
                    int(prolongation))
        nbytes = lib.isis_mg_workspace_size(C.byref(d))
        if nbytes == 0:
            raise ValueError("invalid solver description (N, box, nu_*, max_cycles, precision, "
                             "temporal_block)")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        d.workspace = C.c_void_p(self.workspace.data_ptr())
        d.workspace_bytes = nbytes
        h = C.c_void_p()
        rc = lib.isis_mg_create(C.byref(d), C.byref(h))
        if rc != A.ISIS_OK:
            _raise(rc, lib.isis_mg_last_error(None).decode())
        self._h = h
        self._desc = d

    def set_profiling(self, enable: bool = True):
        """Time the finest-level sweep launches with HIP events (see Stats)."""
        rc = A.lib().isis_mg_set_profiling(self._h, 1 if enable else 0)
        if rc != A.ISIS_OK:
            _raise(rc, self._err())

    def close(self):
        if self._h is not None:
            A.lib().isis_mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self) -> str:
        return A.lib().isis_mg_last_error(self._h).decode()

    def solve(self, eta: torch.Tensor, params: ModelParams, a: float, tol: float,
              phi: torch.Tensor | None = None, use_guess: bool = False,
              check: bool = True) -> tuple[torch.Tensor, Stats]:
        """Solve L(phi, eta) = 0.  If `phi` is given it receives the solution.
        use_guess: False/0 cold start; True/1 start from `phi`; 2 start from
        `phi` only if it cannot cost a V-cycle over the cold start (its
        residual is at most guess_accept, or the handle's measured first-cycle
        factor, times r_ref)."""
        _check_field(eta, self.N, "eta")
        if phi is None:
            phi = torch.empty_like(eta)
            use_guess = False
        _check_field(phi, self.N, "phi")
        st = A.StatsC()
        pc = params.c()
        rc = A.lib().isis_mg_solve(self._h, _ptr(eta), _ptr(phi), C.byref(pc), float(a),
                                   float(tol), int(use_guess), C.byref(st))
        stats = Stats.from_c(rc, st)
        if check and rc != A.ISIS_OK:
            _raise(rc, self._err())
        if rc in (A.ISIS_ERR_INVALID_ARG, A.ISIS_ERR_HIP, A.ISIS_ERR_UNSUPPORTED):
            _raise(rc, self._err())
        return phi, stats

    def residual(self, eta: torch.Tensor, phi: torch.Tensor, params: ModelParams, a: float,
                 out: torch.Tensor | None = None) -> float:
        _check_field(eta, self.N, "eta")
        _check_field(phi, self.N, "phi")
        if out is not None:
            _check_field(out, self.N, "out")
        rms = C.c_double()
        pc = params.c()
        rc = A.lib().isis_mg_residual(self._h, _ptr(eta), _ptr(phi), C.byref(pc), float(a),
                                      _ptr(out), C.byref(rms))
        if rc != A.ISIS_OK:
            _raise(rc, self._err())
        return rms.value


# ---------------------------------------------------------------------------
# Level operators (one V-cycle step each) on torch tensors, in place.
# ---------------------------------------------------------------------------

def _side(t: torch.Tensor) -> int:
    n = round(t.numel() ** (1.0 / 3.0))
    if n ** 3 != t.numel():
        raise ValueError("field is not cubic")
    return n


def _ok(rc: int):
    if rc != A.ISIS_OK:
        _raise(rc, A.lib().isis_mg_last_error(None).decode())


def halfsweep(params: ModelParams, a: float, h: float, phi, eta, sigma=None, colour: int = 0):
    n = _side(phi)
    for t, nm in ((phi, "phi"), (eta, "eta")):
        _check_field(t, n, nm)
    if sigma is not None:
        _check_field(sigma, n, "sigma")
    pc = params.c()
    _ok(A.lib().isis_op_halfsweep(C.byref(pc), float(a), n, float(h), _ptr(phi), _ptr(eta),
                                  _ptr(sigma), int(colour), _stream()))


def sweeps(params: ModelParams, a: float, h: float, phi, eta, sigma=None, count: int = 1,
           temporal_block: int = 0, tmp=None):
    n = _side(phi)
    _check_field(phi, n, "phi")
    _check_field(eta, n, "eta")
    if sigma is not None:
        _check_field(sigma, n, "sigma")
    tmp = torch.empty_like(phi) if tmp is None else tmp
    pc = params.c()
    _ok(A.lib().isis_op_sweeps(C.byref(pc), float(a), n, float(h), _ptr(phi), _ptr(tmp),
                               _ptr(eta), _ptr(sigma), int(count), int(temporal_block),
                               _stream()))


def prolong_sweeps(params: ModelParams, a: float, h: float, phi, eta, coarse, coarse_hat,
                   sigma=None, count: int = 1, temporal_block: int = 0, tmp=None):
    """phi += P(coarse - coarse_hat), then `count` sweeps, as the solver's
    post-smoothing step makes them (the correction inside the first fused
    pass where the sweeps are fused)."""
    n = _side(phi)
    _check_field(phi, n, "phi")
    _check_field(eta, n, "eta")
    _check_field(coarse, n // 2, "coarse")
    _check_field(coarse_hat, n // 2, "coarse_hat")
    if sigma is not None:
        _check_field(sigma, n, "sigma")
    tmp = torch.empty_like(phi) if tmp is None else tmp
    pc = params.c()
    _ok(A.lib().isis_op_prolong_sweeps(C.byref(pc), float(a), n, float(h), _ptr(phi), _ptr(tmp),
                                       _ptr(eta), _ptr(sigma), _ptr(coarse), _ptr(coarse_hat),
                                       int(count), int(temporal_block), _stream()))


def defect(params: ModelParams, a: float, h: float, phi, eta, sigma=None, out=None):
    n = _side(phi)
    _check_field(phi, n, "phi")
    _check_field(eta, n, "eta")
    out = torch.empty_like(phi) if out is None else out
    pc = params.c()
    _ok(A.lib().isis_op_defect(C.byref(pc), float(a), n, float(h), _ptr(phi), _ptr(eta),
                               _ptr(sigma), _ptr(out), _stream()))
    return out


def restrict(fine, out=None):
    n = _side(fine)
    _check_field(fine, n, "fine")
    out = torch.empty(fine.numel() // 8, dtype=fine.dtype, device=fine.device) if out is None else out
    _ok(A.lib().isis_op_restrict(n, _ptr(fine), _ptr(out), _stream()))
    return out


def fas_descend(params: ModelParams, a: float, h_fine: float, phi_f, eta_f, sigma_f, eta_c,
                full_weighting: bool = False):
    n = _side(phi_f)
    _check_field(phi_f, n, "phi_f")
    _check_field(eta_f, n, "eta_f")
    _check_field(eta_c, n // 2, "eta_c")
    mk = lambda: torch.empty_like(eta_c)  # noqa: E731
    phi_c, phihat_c, sigma_c, rr_c = mk(), mk(), mk(), mk()
    scratch = torch.empty_like(phi_f) if full_weighting else None
    pc = params.c()
    _ok(A.lib().isis_op_fas_descend(C.byref(pc), float(a), n, float(h_fine), _ptr(phi_f),
                                    _ptr(eta_f), _ptr(sigma_f), _ptr(eta_c), _ptr(phi_c),
                                    _ptr(phihat_c), _ptr(sigma_c), _ptr(rr_c), _ptr(scratch),
                                    _stream()))
    return phi_c, phihat_c, sigma_c


def restrict_fw(fine, out=None):
    """Full-weighting restriction (the adjoint of the prolongation over 8)."""
    n = _side(fine)
    _check_field(fine, n, "fine")
    out = torch.empty(fine.numel() // 8, dtype=fine.dtype, device=fine.device) if out is None else out
    _ok(A.lib().isis_op_restrict_fw(n, _ptr(fine), _ptr(out), _stream()))
    return out


def prolong_correct_w(fine, coarse, coarse_hat):
    """fine += P_b(coarse - coarse_hat), the coefficient-weighted prolongation
    (weights from b = e^coarse_hat; isis_op_prolong_correct_w), in place."""
    n = _side(fine)
    _check_field(fine, n, "fine")
    _check_field(coarse, n // 2, "coarse")
    _check_field(coarse_hat, n // 2, "coarse_hat")
    _ok(A.lib().isis_op_prolong_correct_w(n, _ptr(fine), _ptr(coarse), _ptr(coarse_hat),
                                          _stream()))


def prolong_correct(fine, coarse, coarse_hat):
    n = _side(fine)
    _check_field(fine, n, "fine")
    _check_field(coarse, n // 2, "coarse")
    _check_field(coarse_hat, n // 2, "coarse_hat")
    _ok(A.lib().isis_op_prolong_correct(n, _ptr(fine), _ptr(coarse), _ptr(coarse_hat), _stream()))


def coarse_solve(params: ModelParams, a: float, h: float, phi, eta, sigma=None, nu_c: int = 32):
    _check_field(phi, 4, "phi")
    _check_field(eta, 4, "eta")
    pc = params.c()
    _ok(A.lib().isis_op_coarse_solve(C.byref(pc), float(a), float(h), _ptr(phi), _ptr(eta),
                                     _ptr(sigma), int(nu_c), _stream()))


def cold_start(params: ModelParams, a: float, eta, out=None):
    out = torch.empty_like(eta) if out is None else out
    pc = params.c()
    _ok(A.lib().isis_op_cold_start(C.byref(pc), float(a), eta.numel(), _ptr(eta), _ptr(out),
                                   _stream()))
    return out


def force(params: ModelParams, a: float, box: float, field=None, potential=None, out=None):
    """Acceleration (fx, fy, fz) on the grid: -grad(potential) minus the
    scalar-field term of the model's geodesic equation (see isis_force)."""
    ref = field if field is not None else potential
    n = _side(ref)
    if out is None:
        out = tuple(torch.empty_like(ref) for _ in range(3))
    pc = params.c()
    _ok(A.lib().isis_force(C.byref(pc), float(a), n, float(box) / n, _ptr(field),
                           _ptr(potential), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _stream()))
    return out


# ---------------------------------------------------------------------------
# Refinement boundaries with masks (Sec. 3.3.1, 3.4.1) on an n^3 patch.
# ---------------------------------------------------------------------------

def masked_defect(params: ModelParams, a: float, h: float, phi, eta, mask, u_int, u_pre,
                  sigma=None, out=None):
    """L - sigma at the inside cells (mask > 0) with ghost values for masked
    neighbours; 0 elsewhere (see isis_op_masked_defect)."""
    n = _side(phi)
    for t, nm in ((phi, "phi"), (eta, "eta"), (mask, "mask"), (u_int, "u_int"), (u_pre, "u_pre")):
        _check_field(t, n, nm)
    out = torch.empty_like(phi) if out is None else out
    pc = params.c()
    _ok(A.lib().isis_op_masked_defect(C.byref(pc), float(a), n, float(h), _ptr(phi), _ptr(eta),
                                      _ptr(sigma), _ptr(mask), _ptr(u_int), _ptr(u_pre),
                                      _ptr(out), _stream()))
    return out


def masked_halfsweep(params: ModelParams, a: float, h: float, phi, eta, mask, u_int, u_pre,
                     sigma=None, colour: int = 0):
    n = _side(phi)
    for t, nm in ((phi, "phi"), (eta, "eta"), (mask, "mask"), (u_int, "u_int"), (u_pre, "u_pre")):
        _check_field(t, n, nm)
    pc = params.c()
    _ok(A.lib().isis_op_masked_halfsweep(C.byref(pc), float(a), n, float(h), _ptr(phi),
                                         _ptr(eta), _ptr(sigma), _ptr(mask), _ptr(u_int),
                                         _ptr(u_pre), int(colour), _stream()))


def patch_solve(params: ModelParams, a: float, h: float, phi, eta, mask, u_int, block: int = 4,
                max_sweeps: int = 10000, tol: float = 1e-10, check: bool = True):
    """Relaxation solve of a refinement patch in place (see isis_patch_solve);
    returns (status, sweeps, rms)."""
    n = _side(phi)
    for t, nm in ((phi, "phi"), (eta, "eta"), (mask, "mask"), (u_int, "u_int")):
        _check_field(t, n, nm)
    nbytes = A.lib().isis_patch_workspace_size(n)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=phi.device)
    sweeps, rms = C.c_int(), C.c_double()
    pc = params.c()
    rc = A.lib().isis_patch_solve(C.byref(pc), float(a), n, float(h), _ptr(phi), _ptr(eta),
                                  _ptr(mask), _ptr(u_int), int(block), int(max_sweeps),
                                  float(tol), _ptr(ws), nbytes, C.byref(sweeps), C.byref(rms),
                                  _stream())
    if rc in (A.ISIS_ERR_INVALID_ARG, A.ISIS_ERR_HIP) or (check and rc != A.ISIS_OK):
        _raise(rc, A.lib().isis_mg_last_error(None).decode())
    return rc, sweeps.value, rms.value
