"""Model variants on the GPU against the oracle: the chameleon of Sec. 6
(solved for psi = ln phi with the non-canonical operator of Sec. 3.4) and
Hu-Sawicki f(R) in the paper's own variable u = ln(a^2 |f_R|) (Sec. 4.2).

The per-step kernels are covered for these models by test_gpu_ops (every
case of gpucase.H_CASES); here: whole solves in FP64 and mixed precision,
the equivalence of the two f(R) variables, and a 512^3 chameleon solve on the
benchmark's density checked by the oracle's own residual.
"""
import numpy as np
import pytest

from gpucase import cubic, dev, models

pytestmark = pytest.mark.gpu

VARIANTS = ["chameleon", "chameleon_n05", "fofr_paper_u"]


def _solver(n, box, **kw):
    from paper_1307_6748_amd import solver as S
    return S.Solver(n, box, **kw)


def _eta(n, box, seed):
    from paper_1307_6748_amd import synth
    return synth.lognormal(n, box, 2.0, seed)


@pytest.mark.parametrize("name", VARIANTS)
def test_variant_solve_fp64(orc, name):
    """64^3, lognormal sigma_delta = 2: same cycle count, per-cycle factors
    and converged field as the oracle's FAS solve."""
    om, sp, a = models(name)
    n, box = 64, 128.0
    eta = _eta(n, box, 31)
    ro = orc.solve(om, eta, box, tol=1e-10, cfg=orc.Cfg(max_cycles=60))
    phi, st = _solver(n, box, max_cycles=60).solve(dev(eta), sp, a, 1e-10)
    assert ro.status == 0 and st.status == 0 and st.cycles == ro.cycles
    g, o = np.asarray(st.rel_hist), np.asarray(ro.rel_hist)
    assert np.all(np.abs(g - o) <= 1e-5 * np.abs(o) + 1e-12)
    assert abs(st.r_ref - ro.r_ref) <= 1e-11 * ro.r_ref
    assert np.max(np.abs(cubic(phi, n) - ro.phi)) <= 1e-9 * np.abs(ro.phi).max()


@pytest.mark.parametrize("name", VARIANTS)
def test_variant_solve_mixed(orc, name):
    """Mixed precision (FP32 cycles in w = field/ln2 for these non-canonical
    models, FP64 judge and last cycle) reaches 1e-8, and its distance from the
    oracle's 1e-12 solution is within 1e-6 (relative L2) of the distance of
    the oracle's own FP64 solve stopped at 1e-8.  (For the n = -1/2
    chameleon, whose root spans ~11 decades on this density, any solve
    stopped at 1e-8 is ~1e-4 away; for the others ~1e-8.)"""
    om, sp, a = models(name)
    n, box = 64, 128.0
    eta = _eta(n, box, 32)
    ro = orc.solve(om, eta, box, tol=1e-12, cfg=orc.Cfg(max_cycles=80))
    r8 = orc.solve(om, eta, box, tol=1e-8, cfg=orc.Cfg(max_cycles=80))
    phi, st = _solver(n, box, precision="mixed", max_cycles=60).solve(dev(eta), sp, a, 1e-8)
    assert st.status == 0 and st.rel_res <= 1e-8 and st.cycles_fp32 >= 1
    got = cubic(phi, n)
    norm = np.linalg.norm(ro.phi)
    err = np.linalg.norm(got - ro.phi) / norm
    err_fp64 = np.linalg.norm(r8.phi - ro.phi) / norm
    assert err <= err_fp64 + 1e-6, (err, err_fp64)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_paper_variable_is_shifted_standard_variable(precision):
    """The solve in the paper's u equals the solve in ln(f_R/f_R0) plus
    ln(a^2 |f_R0|).  In FP64 the relative residuals of every cycle agree too
    (the two equations differ by the factor a^2 |f_R0|).  In mixed precision
    the FP32 phases differ: u_p = u + ln(a^2 |f_R0|) (about -12 here) carries
    about ten times the absolute FP32 rounding, so the cycle split differs."""
    from paper_1307_6748_amd import solver as S
    n, box, a, fr0 = 64, 128.0, 0.8, 1e-5
    eta = dev(_eta(n, box, 33))
    s = _solver(n, box, precision=precision, max_cycles=60)
    u, st = s.solve(eta, S.fofr(1.0, fr0, 0.27, 0.73), a, 1e-10)
    up, stp = s.solve(eta, S.fofr(1.0, fr0, 0.27, 0.73, paper_u=True), a, 1e-10)
    assert st.status == 0 and stp.status == 0
    if precision == "fp64":
        assert st.cycles == stp.cycles
        assert np.allclose(stp.rel_hist[:st.cycles + 1], st.rel_hist[:st.cycles + 1],
                           rtol=1e-4, atol=1e-13)
    c = np.log(a * a * fr0)
    tol = 1e-9 if precision == "fp64" else 1e-7
    assert np.max(np.abs(cubic(up, n) - cubic(u, n) - c)) <= tol * abs(c)


def test_chameleon_512_bench_density(orc):
    """512^3 benchmark density (lognormal sigma_delta = 2 + 400 NFW haloes),
    chameleon n = 1 in mixed precision, one sweep per pass (the benchmark's
    launch configuration): the oracle's own residual of the GPU field meets
    the tolerance and equals the reported one; phi = e^psi > 0 and the field
    is finite."""
    from paper_1307_6748_amd import solver as S
    from paper_1307_6748_amd import synth
    n, box = 512, 256.0
    eta = synth.lognormal_nfw(n, box, 2.0, 20, 400, 22, omega_m=0.27)
    sp = S.chameleon(alpha=1e-3, mu=1e-3, n=1.0)
    om = orc.Model(model=orc.CHAMELEON, cham_alpha=1e-3, cham_mu=1e-3, cham_n=1.0)
    s = _solver(n, box, precision="mixed", temporal_block=1, max_cycles=100)
    phi, st = s.solve(dev(eta), sp, 1.0, 1e-8)
    assert st.status == 0
    got = cubic(phi, n)
    del phi
    assert np.all(np.isfinite(got))
    h = box / n
    r = orc.rms(orc.defect(om, h, got, eta))
    r_ref = orc.rms(orc.defect(om, h, orc.cold_start(om, eta), eta))
    assert abs(r_ref - st.r_ref) <= 1e-9 * r_ref
    assert r / r_ref <= 1e-8 * 1.001
    assert abs(r / r_ref - st.rel_res) <= 1e-6 * st.rel_res


def test_chameleon_force_is_unsupported():
    import torch
    from paper_1307_6748_amd import solver as S
    n = 8
    x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(S.IsisError):
        S.force(S.chameleon(), 1.0, 8.0, field=x, potential=None)


def test_automatic_temporal_block_per_model():
    """temporal_block = -1: two sweeps per HBM pass for the canonical models
    (symmetron, linear), one for the non-canonical ones (f(R), chameleon);
    the stats report the choice, and each solve still converges."""
    from paper_1307_6748_amd import solver as S
    n, box = 64, 128.0
    eta = dev(_eta(n, box, 34))
    s = _solver(n, box, temporal_block=-1, max_cycles=60)
    for p, a, tb in ((S.symmetron(1.0, 0.5), 1.0, 2), (S.linear(1.3, 0.4), 1.0, 2),
                     (S.fofr(1.0, 1e-5, 0.27, 0.73), 1.0, 1), (S.chameleon(2.0, 3.0, 1.0), 1.0, 1)):
        _, st = s.solve(eta, p, a, 1e-8)
        assert st.status == 0 and st.temporal_block == tb
