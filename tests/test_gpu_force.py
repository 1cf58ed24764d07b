"""Force on the grid (isis_force) against the oracle, element by element, and
the linear-regime force ratios end to end on the GPU (solver + force)."""
import numpy as np
import pytest

from gpucase import cubic, dev, field_for, models

pytestmark = pytest.mark.gpu

H0 = 1.0 / 2997.92458


def _check(f_gpu, f_orc, n):
    for g, o in zip(f_gpu, f_orc):
        scale = max(np.abs(o).max(), 1e-300)
        assert np.max(np.abs(cubic(g, n) - o)) <= 1e-13 * scale


# 6, 12, 36: the per-cell kernel (not a multiple of 64); 64, 128: the tiled one
@pytest.mark.parametrize("name", ["symmetron_a1", "symmetron_a05", "fofr", "fofr_a07",
                                  "fofr_paper_u", "linear"])
@pytest.mark.parametrize("n", [6, 12, 36, 64, 128])
@pytest.mark.parametrize("with_pot", [False, True])
def test_force_matches_oracle(orc, name, n, with_pot):
    from paper_1307_6748_amd import solver as S
    om, sp, a = models(name)
    box = 1.5 * n
    phi = field_for(name, n, 11)
    pot = np.random.default_rng(12).standard_normal((n, n, n)) if with_pot else None
    if name == "linear" and not with_pot:
        pot = None
    ref = orc.force(om, box / n, phi, pot)
    got = S.force(sp, a, box, field=dev(phi), potential=None if pot is None else dev(pot))
    _check(got, ref, n)


def test_force_linear_without_field(orc):
    """The linear model has no scalar-field term: the field may be NULL."""
    from paper_1307_6748_amd import solver as S
    n, box = 64, 32.0
    pot = np.random.default_rng(3).standard_normal((n, n, n))
    om, sp, a = models("linear")
    got = S.force(sp, a, box, field=None, potential=dev(pot))
    _check(got, orc.force(om, box / n, np.zeros((n, n, n)), pot), n)


def test_force_full_size(orc):
    """512^3 (the benchmark grid) on a random f(R)-like field and potential."""
    from paper_1307_6748_amd import solver as S
    n, box = 512, 256.0
    om, sp, a = models("fofr")
    phi = field_for("fofr", n, 21)
    pot = np.random.default_rng(22).standard_normal((n, n, n))
    got = S.force(sp, a, box, field=dev(phi), potential=dev(pot))
    _check(got, orc.force(om, box / n, phi, pot), n)


def test_force_rejects_bad_arguments():
    import torch
    from paper_1307_6748_amd import solver as S
    x = torch.zeros(8 ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(S.IsisError):
        S.force(S.symmetron(omega_m=0.0), 1.0, 8.0, field=x)  # the symmetron force needs Omega_m
    with pytest.raises(S.IsisError):
        S.force(S.fofr(), 1.0, 8.0, field=None, potential=x)  # f(R) needs its field


@pytest.mark.parametrize("model", ["symmetron", "fofr"])
def test_linear_regime_force_ratio_on_gpu(model):
    """eta = 1 + eps sin(k x), solved on the GPU for the scalar field and for
    the Newtonian potential; the force ratio is the textbook one: symmetron
    2 beta^2 chi0^2, f(R) 1/3, times the Yukawa factor lambda/(lambda + m^2)."""
    import torch
    from paper_1307_6748_amd import solver as S
    n, box, mode, eps, a = 32, 64.0, 2, 1e-5, 1.0
    h = box / n
    k = 2 * np.pi * mode / box
    x = (np.arange(n) + 0.5) * h
    eta = 1.0 + eps * np.broadcast_to(np.sin(k * x)[:, None, None], (n, n, n))
    eta = np.ascontiguousarray(eta)
    lam = (2 - 2 * np.cos(k * h)) / h ** 2
    om = 0.27
    if model == "symmetron":
        beta, lam0, assb = 1.5, 4.0, 0.5
        p = S.symmetron(lambda0=lam0, a_ssb=assb, beta=beta, omega_m=om)
        A = (assb / a) ** 3
        expect = 2 * beta ** 2 * (1 - A) * lam / (lam + a ** 2 / lam0 ** 2 * (1 - A))
    else:
        fr0, ol = 1e-4, 0.73
        p = S.fofr(n=1.0, fR0_abs=fr0, omega_m=om, omega_l=ol)
        cL = 4 * ol / om
        eu0 = (a ** 3 * (1 + cL) / (1 + cL * a ** 3)) ** 2
        mu2 = om * H0 ** 2 / (a * fr0) * (1 + cL * a ** 3) / 2
        expect = (1 / 3) * eu0 * lam / (eu0 * lam + mu2)
    s = S.Solver(n, box, max_cycles=80)
    # (the cold start is almost exact here, so the round-off floor of the
    # relative residual is ~3e-9; 1e-8 of its residual is far below what the
    # 2e-3 ratio check needs)
    phi, _ = s.solve(dev(eta), p, a, 1e-8)
    pot, _ = s.solve(dev(eta), S.newtonian(om, a), a, 1e-8)
    f5 = cubic(S.force(p, a, box, field=phi)[0], n)
    fN = cubic(S.force(S.linear(), a, box, potential=(a * a) * pot)[0], n)
    sel = np.abs(fN) > 0.5 * np.abs(fN).max()
    ratio = f5[sel] / fN[sel]
    assert np.max(np.abs(ratio - expect)) < 2e-3 * expect
