"""FP64 CPU oracle for the FAS multigrid scalar-field solve (test infrastructure).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It loads ``liboracle.so`` compiled from
``isis_oracle.c`` (plain C, FP64, ``-ffp-contract=off``) and exposes it on
NumPy arrays.  Nothing here touches the GPU library, and the GPU library never
imports this.

Models and readings follow the paper (Llinares, Mota & Winther 2013):
Sec. 3.1 (Laplacian, V-cycle), Sec. 3.2 (FAS, Newton-Gauss-Seidel),
Sec. 3.3-3.4 (canonical and non-canonical discretisation), Sec. 4.1
(symmetron), Sec. 4.2 (Hu-Sawicki f(R)).  The readings of unspecified points
are listed in the header of ``isis_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "isis_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# A different build of the oracle (used by the mutation test, which plants
# mistakes in a copy of the source) can be loaded by setting ORACLE_LIB.
_LIB_OVERRIDE = os.environ.get("ORACLE_LIB")

SYMMETRON, FR_HS, LINEAR, CHAMELEON = 0, 1, 2, 3
OK, INVALID, NOT_CONVERGED, DIVERGED = 0, -1, -2, -3
MAX_HIST = 256


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, src, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


class _Model(C.Structure):
    _fields_ = [("model", C.c_int), ("a", C.c_double), ("lambda0", C.c_double),
                ("a_ssb", C.c_double), ("n", C.c_double), ("fR0_abs", C.c_double),
                ("omega_m", C.c_double), ("omega_l", C.c_double), ("kappa", C.c_double),
                ("m2", C.c_double), ("beta", C.c_double), ("cham_alpha", C.c_double),
                ("cham_mu", C.c_double), ("cham_n", C.c_double), ("paper_u", C.c_int)]


class _Cfg(C.Structure):
    _fields_ = [("nu_pre", C.c_int), ("nu_post", C.c_int), ("nu_coarse", C.c_int),
                ("max_cycles", C.c_int), ("restrict_fw", C.c_int), ("prolong_w", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("cycles", C.c_int), ("r_ref", C.c_double), ("r0", C.c_double),
                ("rel_hist", C.c_double * MAX_HIST), ("wall_s", C.c_double),
                ("guard_hits", C.c_longlong)]


@dataclass
class Model:
    """Model parameters.  Lengths in comoving Mpc/h, c = 1."""
    model: int = SYMMETRON
    a: float = 1.0
    lambda0: float = 1.0
    a_ssb: float = 0.5
    n: float = 1.0
    fR0_abs: float = 1e-5
    omega_m: float = 0.27
    omega_l: float = 0.73
    kappa: float = 1.0
    m2: float = 0.0
    beta: float = 1.0
    cham_alpha: float = 1.0  # chameleon: lap phi = alpha eta - mu phi^-(1+n), phi = e^psi
    cham_mu: float = 1.0
    cham_n: float = 1.0
    paper_u: bool = False    # f(R): field in the paper's u = ln(a^2 |f_R|)

    def _c(self) -> _Model:
        return _Model(int(self.model), self.a, self.lambda0, self.a_ssb, self.n, self.fR0_abs,
                      self.omega_m, self.omega_l, self.kappa, self.m2, self.beta,
                      self.cham_alpha, self.cham_mu, self.cham_n, int(bool(self.paper_u)))


@dataclass
class Cfg:
    nu_pre: int = 2
    # post-smoothing sweeps; None = per model, the GPU library's default: one
    # for the symmetron and the chameleon, two for the others
    nu_post: int | None = None
    nu_coarse: int = 32
    max_cycles: int = 50
    # restriction of the defect: False = mean of the 8 children, True = full
    # weighting, 2 = full weighting in the first two V-cycles of the solve and
    # the mean after them; None = per model, the choice the GPU library makes
    # by default (2 for f(R) with the weighted prolongation, True for f(R)
    # with the trilinear one, False otherwise)
    restrict_fw: bool | int | None = None
    # prolongation: False = trilinear, True = weighted by b = e^u (flux-form
    # models; see orc_prolong_correct_w); None = per model, the GPU
    # library's default (weighted for f(R), where it takes fewer V-cycles)
    prolong_w: bool | None = None

    def _c(self, model: int = SYMMETRON) -> _Cfg:
        pw = (model == FR_HS) if self.prolong_w is None else bool(self.prolong_w)
        if model not in (FR_HS, CHAMELEON):
            pw = False
        if self.restrict_fw is None:
            fw = (2 if pw else 1) if model == FR_HS else 0
        else:
            fw = 2 if self.restrict_fw == 2 else int(bool(self.restrict_fw))
        post = (1 if model in (SYMMETRON, CHAMELEON) else 2) if self.nu_post is None else self.nu_post
        return _Cfg(self.nu_pre, post, self.nu_coarse, self.max_cycles, int(fw), int(pw))


@dataclass
class Result:
    status: int
    phi: np.ndarray
    cycles: int
    r_ref: float
    r0: float
    rel_hist: np.ndarray = field(default_factory=lambda: np.zeros(0))
    wall_s: float = 0.0
    guard_hits: int = 0  # symmetron updates with the safeguarded denominator


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _LIB_OVERRIDE or _LIB
        if not _LIB_OVERRIDE and not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(path)
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.orc_source.argtypes = [C.POINTER(_Model), C.c_double, C.c_double,
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_defect.argtypes = [C.POINTER(_Model), C.c_int, C.c_double, dp, dp, C.c_void_p, dp]
        L.orc_newton_diag.argtypes = [C.POINTER(_Model), C.c_int, C.c_double, dp, dp, dp]
        L.orc_halfsweep.argtypes = [C.POINTER(_Model), C.c_int, C.c_double, dp, dp, C.c_void_p,
                                    C.c_int]
        L.orc_sweep.argtypes = [C.POINTER(_Model), C.c_int, C.c_double, dp, dp, C.c_void_p]
        L.orc_restrict.argtypes = [C.c_int, dp, dp]
        L.orc_restrict_fw.argtypes = [C.c_int, dp, dp]
        L.orc_prolong_correct.argtypes = [C.c_int, dp, dp, dp]
        L.orc_prolong_correct_w.argtypes = [C.c_int, dp, dp, dp]
        L.orc_cold_start.argtypes = [C.POINTER(_Model), C.c_long, dp, dp]
        L.orc_rms.argtypes = [C.c_int, dp]
        L.orc_rms.restype = C.c_double
        L.orc_num_levels.argtypes = [C.c_int]
        L.orc_masked_defect.argtypes = [C.POINTER(_Model), C.c_int, C.c_double, dp, dp, C.c_void_p,
                                        dp, dp, dp, dp]
        L.orc_masked_newton_diag.argtypes = [C.POINTER(_Model), C.c_int, C.c_double, dp, dp, dp,
                                             dp, dp, dp]
        L.orc_masked_halfsweep.argtypes = [C.POINTER(_Model), C.c_int, C.c_double, dp, dp,
                                           C.c_void_p, dp, dp, dp, C.c_int]
        L.orc_patch_solve.argtypes = [C.POINTER(_Model), C.c_int, C.c_double, dp, dp, dp, dp, C.c_int,
                                      C.c_int, C.c_double, C.POINTER(C.c_double)]
        L.orc_guard_hits.argtypes = [C.c_int]
        L.orc_guard_hits.restype = C.c_longlong
        L.orc_solve.argtypes = [C.POINTER(_Model), C.POINTER(_Cfg), C.c_int, C.c_double, dp,
                                dp, C.c_int, C.c_double, C.POINTER(_Stats)]
        L.orc_force.argtypes = [C.POINTER(_Model), C.c_int, C.c_double, dp, C.c_void_p, dp, dp,
                                dp]
        _lib = L
    return _lib


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr_or_null(x):
    if x is None:
        return None
    return x.ctypes.data_as(C.c_void_p)


def set_threads(n: int) -> None:
    """Set the OpenMP thread count of the oracle (results do not depend on it)."""
    os.environ["OMP_NUM_THREADS"] = str(n)
    try:
        C.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
    except OSError:
        pass


def source(m: Model, phi: float, eta: float) -> tuple[float, float]:
    """Pointwise S(phi, eta) and dS/dphi."""
    S, dS = C.c_double(), C.c_double()
    mc = m._c()
    lib().orc_source(C.byref(mc), float(phi), float(eta), C.byref(S), C.byref(dS))
    return S.value, dS.value


def defect(m: Model, h: float, phi, eta, sigma=None) -> np.ndarray:
    """L_h(phi, eta) - Sigma on a periodic n^3 grid."""
    phi, eta = _f64(phi), _f64(eta)
    n = phi.shape[0]
    out = np.empty_like(phi)
    sig = None if sigma is None else _f64(sigma)
    mc = m._c()
    lib().orc_defect(C.byref(mc), n, h, phi, eta, _ptr_or_null(sig), out)
    return out


def force(m: Model, h: float, field, potential=None):
    """Acceleration (fx, fy, fz) in super-comoving variables: -grad(potential)
    (if given) minus the scalar-field term of the model's geodesic equation
    (Sec. 4.1 symmetron, Sec. 4.2 f(R)), second-order central differences."""
    field = _f64(field)
    pot = None if potential is None else _f64(potential)
    fx, fy, fz = (np.empty_like(field) for _ in range(3))
    mc = m._c()
    lib().orc_force(C.byref(mc), field.shape[0], h, field, _ptr_or_null(pot), fx, fy, fz)
    return fx, fy, fz


def newton_diag(m: Model, h: float, phi, eta) -> np.ndarray:
    """The Newton denominator D_c the smoother divides by."""
    phi, eta = _f64(phi), _f64(eta)
    out = np.empty_like(phi)
    mc = m._c()
    lib().orc_newton_diag(C.byref(mc), phi.shape[0], h, phi, eta, out)
    return out


def halfsweep(m: Model, h: float, phi, eta, sigma=None, colour: int = 0) -> np.ndarray:
    """One colour of a red-black Newton-Gauss-Seidel sweep; returns a new array."""
    out = _f64(phi).copy()
    eta = _f64(eta)
    sig = None if sigma is None else _f64(sigma)
    mc = m._c()
    lib().orc_halfsweep(C.byref(mc), out.shape[0], h, out, eta, _ptr_or_null(sig), int(colour))
    return out


def sweep(m: Model, h: float, phi, eta, sigma=None, count: int = 1) -> np.ndarray:
    out = _f64(phi).copy()
    eta = _f64(eta)
    sig = None if sigma is None else _f64(sigma)
    mc = m._c()
    for _ in range(count):
        lib().orc_sweep(C.byref(mc), out.shape[0], h, out, eta, _ptr_or_null(sig))
    return out


def restrict(fine) -> np.ndarray:
    fine = _f64(fine)
    n = fine.shape[0]
    out = np.empty((n // 2,) * 3)
    lib().orc_restrict(n, fine, out)
    return out


def restrict_fw(fine) -> np.ndarray:
    """Full-weighting restriction, P^T / 8 (the defect's option)."""
    fine = _f64(fine)
    n = fine.shape[0]
    out = np.empty((n // 2,) * 3)
    lib().orc_restrict_fw(n, fine, out)
    return out


def prolong_correct(fine, coarse, coarse_hat) -> np.ndarray:
    out = _f64(fine).copy()
    lib().orc_prolong_correct(out.shape[0], out, _f64(coarse), _f64(coarse_hat))
    return out


def prolong_correct_w(fine, coarse, coarse_hat) -> np.ndarray:
    """fine + P_b(coarse - coarse_hat), weights from b = e^coarse_hat."""
    out = _f64(fine).copy()
    lib().orc_prolong_correct_w(out.shape[0], out, _f64(coarse), _f64(coarse_hat))
    return out


def cold_start(m: Model, eta) -> np.ndarray:
    eta = _f64(eta)
    out = np.empty_like(eta)
    mc = m._c()
    lib().orc_cold_start(C.byref(mc), eta.size, eta, out)
    return out


def masked_defect(m: Model, h: float, phi, eta, mask, u_int, u_pre, sigma=None) -> np.ndarray:
    """L - Sigma at the inside cells (mask > 0) of a refinement patch, with
    ghost values for masked neighbours (Sec. 3.3.1, 3.4.1); 0 elsewhere."""
    phi, eta, mask, u_int, u_pre = (_f64(x) for x in (phi, eta, mask, u_int, u_pre))
    out = np.empty_like(phi)
    sig = None if sigma is None else _f64(sigma)
    mc = m._c()
    lib().orc_masked_defect(C.byref(mc), phi.shape[0], h, phi, eta, _ptr_or_null(sig), mask,
                            u_int, u_pre, out)
    return out


def masked_newton_diag(m: Model, h: float, phi, eta, mask, u_int, u_pre) -> np.ndarray:
    phi, eta, mask, u_int, u_pre = (_f64(x) for x in (phi, eta, mask, u_int, u_pre))
    out = np.empty_like(phi)
    mc = m._c()
    lib().orc_masked_newton_diag(C.byref(mc), phi.shape[0], h, phi, eta, mask, u_int, u_pre, out)
    return out


def masked_halfsweep(m: Model, h: float, phi, eta, mask, u_int, u_pre, sigma=None,
                     colour: int = 0) -> np.ndarray:
    out = _f64(phi).copy()
    eta, mask, u_int, u_pre = (_f64(x) for x in (eta, mask, u_int, u_pre))
    sig = None if sigma is None else _f64(sigma)
    mc = m._c()
    lib().orc_masked_halfsweep(C.byref(mc), out.shape[0], h, out, eta, _ptr_or_null(sig), mask,
                               u_int, u_pre, int(colour))
    return out


def patch_solve(m: Model, h: float, phi0, eta, mask, u_int, block: int = 4,
                max_sweeps: int = 10000, tol: float = 1e-10):
    """Relaxation solve of a refinement patch (blocks of red-black sweeps, the
    boundary values reset from the field before each block).  Returns
    (phi, sweeps, rms) with rms the absolute RMS defect over inside cells."""
    phi = _f64(phi0).copy()
    eta, mask, u_int = (_f64(x) for x in (eta, mask, u_int))
    rms = C.c_double()
    mc = m._c()
    sw = lib().orc_patch_solve(C.byref(mc), phi.shape[0], h, phi, eta, mask, u_int, int(block),
                               int(max_sweeps), float(tol), C.byref(rms))
    if sw < 0:
        raise ValueError("oracle: invalid patch-solve arguments")
    return phi, int(sw), rms.value


def guard_hits(reset: bool = True) -> int:
    """Symmetron updates made with the safeguarded denominator since the last
    reset (halfsweep/sweep calls; a solve resets and reports its own)."""
    return int(lib().orc_guard_hits(1 if reset else 0))


def rms(r) -> float:
    r = _f64(r)
    return float(lib().orc_rms(r.shape[0], r))


def num_levels(n: int) -> int:
    return int(lib().orc_num_levels(int(n)))


def solve(m: Model, eta, box: float, tol: float = 1e-10, phi0=None, cfg: Cfg | None = None
          ) -> Result:
    """FAS V-cycles from phi0 (or the cold start) until rel. residual <= tol."""
    cfg = cfg or Cfg()
    eta = _f64(eta)
    n = eta.shape[0]
    phi = np.empty_like(eta) if phi0 is None else _f64(phi0).copy()
    st = _Stats()
    mc, cc = m._c(), cfg._c(m.model)
    s = lib().orc_solve(C.byref(mc), C.byref(cc), n, box, eta, phi, 0 if phi0 is None else 1,
                        tol, C.byref(st))
    if s == INVALID:
        raise ValueError("oracle: invalid arguments")
    hist = np.array(st.rel_hist[: st.cycles + 1])
    return Result(s, phi, st.cycles, st.r_ref, st.r0, hist, st.wall_s, int(st.guard_hits))


def vcycles(m: Model, eta, box: float, phi0, k: int, cfg: Cfg | None = None) -> Result:
    """Exactly k V-cycles from phi0 (no stop test)."""
    cfg = cfg or Cfg()
    c2 = Cfg(cfg.nu_pre, cfg.nu_post, cfg.nu_coarse, k, cfg.restrict_fw, cfg.prolong_w)
    return solve(m, eta, box, tol=0.0, phi0=phi0, cfg=c2)
