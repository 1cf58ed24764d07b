"""GPU vs oracle, one V-cycle step at a time, element by element.

Every call goes through the C ABI (isis_op_*).  Sizes span several blocks
and include non-power-of-two grids (n = 6, 18, 36) so that the last block of
each grid-stride loop is ragged.  Tolerances: the GPU contracts a*b+c into
FMAs and uses its own exp/log, so results agree to a few ulps of the terms
that cancel (|phi| * 12/h^2 for the Laplacian), not bitwise.
"""
import numpy as np
import pytest

from gpucase import H_CASES, cubic, density, dev, field_for, models, sigma_for

pytestmark = pytest.mark.gpu

CASES = sorted(H_CASES)


def _scale(phi, h):
    return (np.abs(phi).max() + 1.0) * 12.0 / h ** 2


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("n", [6, 8, 18, 32])
@pytest.mark.parametrize("colour", [0, 1])
def test_halfsweep(orc, name, n, colour):
    from paper_1307_6748_amd import solver as S
    om, sp, a = models(name)
    h = 0.7
    phi = field_for(name, n, 1 + n)
    eta = density(n, 2 + n)
    sigma = sigma_for(name, n, 3 + n, 0.1)
    expect = orc.halfsweep(om, h, phi, eta, sigma, colour)
    gp = dev(phi)
    S.halfsweep(sp, a, h, gp, dev(eta), dev(sigma), colour)
    got = cubic(gp, n)
    assert np.max(np.abs(got - expect)) <= 1e-13 * (np.abs(expect).max() + 1.0)
    i, j, k = np.indices((n, n, n))
    other = ((i + j + k) % 2) != colour
    assert np.array_equal(got[other], phi[other])


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("n", [6, 16, 32])
def test_defect(orc, name, n):
    from paper_1307_6748_amd import solver as S
    om, sp, a = models(name)
    h = 1.3
    phi = field_for(name, n, 11)
    eta = density(n, 12)
    for sigma in (None, sigma_for(name, n, 13)):
        expect = orc.defect(om, h, phi, eta, sigma)
        got = cubic(S.defect(sp, a, h, dev(phi), dev(eta), None if sigma is None else dev(sigma)), n)
        tol = 1e-14 * (_scale(phi, h) + np.abs(expect).max())
        assert np.max(np.abs(got - expect)) <= tol


@pytest.mark.parametrize("n", [2, 8, 12, 36])
def test_restrict(orc, n):
    from paper_1307_6748_amd import solver as S
    f = np.random.default_rng(n).standard_normal((n, n, n))
    got = cubic(S.restrict(dev(f)), n // 2)
    assert np.max(np.abs(got - orc.restrict(f))) <= 1e-15 * np.abs(f).max()


# 128, 256: the LDS-staged kernel (coarse side a power of two, multiple of 64);
# 384: coarse side 192 is a multiple of 64 but not a power of two (pair kernel)
@pytest.mark.parametrize("n", [4, 8, 12, 36, 128, 256, 384])
def test_prolong_correct(orc, n):
    from paper_1307_6748_amd import solver as S
    rng = np.random.default_rng(n)
    fine = rng.standard_normal((n, n, n))
    c = rng.standard_normal((n // 2,) * 3)
    ch = rng.standard_normal((n // 2,) * 3)
    expect = orc.prolong_correct(fine, c, ch)
    g = dev(fine)
    S.prolong_correct(g, dev(c), dev(ch))
    assert np.max(np.abs(cubic(g, n) - expect)) <= 1e-14 * np.abs(expect).max()


# the weighted variants of the same three kernels (tiled at 128, 256; pairs
# elsewhere); coarse_hat spread over a wide range so that the weights span
# (0, 1/2), with a few cells far beyond the exponential's range
@pytest.mark.parametrize("n", [4, 8, 12, 36, 128, 256, 384])
def test_prolong_correct_w(orc, n):
    from paper_1307_6748_amd import solver as S
    rng = np.random.default_rng(100 + n)
    fine = rng.standard_normal((n, n, n))
    ch = 3.0 * rng.standard_normal((n // 2,) * 3)
    ch.flat[:: max(1, ch.size // 5)] += 800.0 * rng.choice([-1.0, 1.0], size=ch.flat[:: max(1, ch.size // 5)].size)
    c = ch + rng.standard_normal((n // 2,) * 3)
    expect = orc.prolong_correct_w(fine, c, ch)
    g = dev(fine)
    S.prolong_correct_w(g, dev(c), dev(ch))
    got = cubic(g, n)
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - expect)) <= 1e-14 * (np.abs(expect).max() + 1.0)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("n", [4, 12, 32, 64, 128])
@pytest.mark.parametrize("with_sigma", [False, True])
@pytest.mark.parametrize("fw", [False, True])
def test_fas_descend(orc, name, n, with_sigma, fw):
    """phi_c = phihat_c = R phi_f; sigma_c = L_c(R phi_f) - R'(L_f(phi_f) - sigma_f),
    R' the 8-child mean or full weighting.  At 64 and 128 the mean takes the
    LDS-tiled descent (2 and 4 coarse planes per workgroup), which forms
    sigma_c itself, one coarse plane behind, with the x-neighbours' means of
    the first and last plane of each workgroup summed from HBM."""
    from paper_1307_6748_amd import solver as S
    om, sp, a = models(name)
    h = 0.9
    phi = field_for(name, n, 21)
    eta = density(n, 22)
    sig = sigma_for(name, n, 23) if with_sigma else None
    eta_c = orc.restrict(eta)
    # oracle: the steps of the descent, as the oracle's V-cycle takes them
    phi_c = orc.restrict(phi)
    d = orc.defect(om, h, phi, eta, sig)
    rr = orc.restrict_fw(d) if fw else orc.restrict(d)
    sigma_c = orc.defect(om, 2 * h, phi_c, eta_c) - rr
    gphi_c, gphihat_c, gsigma_c = S.fas_descend(sp, a, h, dev(phi), dev(eta),
                                                None if sig is None else dev(sig), dev(eta_c),
                                                full_weighting=fw)
    nc = n // 2
    assert np.max(np.abs(cubic(gphi_c, nc) - phi_c)) <= 1e-15 * (np.abs(phi_c).max() + 1)
    assert np.array_equal(cubic(gphi_c, nc), cubic(gphihat_c, nc))
    tol = 1e-14 * (_scale(phi, h) + np.abs(sigma_c).max())
    assert np.max(np.abs(cubic(gsigma_c, nc) - sigma_c)) <= tol


@pytest.mark.parametrize("n", [2, 4, 6, 12, 64, 128, 256])
def test_restrict_fw(orc, n):
    """Full-weighting restriction vs the oracle: the per-cell kernel on small
    or non-power-of-two grids, the LDS-staged one from 64^3 (wrap included)."""
    from paper_1307_6748_amd import solver as S
    f = np.random.default_rng(n).standard_normal((n, n, n))
    ref = orc.restrict_fw(f)
    got = cubic(S.restrict_fw(dev(f)), n // 2)
    assert np.max(np.abs(got - ref)) <= 1e-15 * np.abs(f).max() * 4


@pytest.mark.parametrize("name", CASES)
def test_coarse_solve(orc, name):
    from paper_1307_6748_amd import solver as S
    om, sp, a = models(name)
    h = 8.0
    phi = field_for(name, 4, 31)
    eta = density(4, 32)
    sigma = sigma_for(name, 4, 33, 0.01)
    expect = orc.sweep(om, h, phi, eta, sigma, count=32)
    g = dev(phi)
    S.coarse_solve(sp, a, h, g, dev(eta), dev(sigma), 32)
    assert np.max(np.abs(cubic(g, 4) - expect)) <= 1e-12 * (np.abs(expect).max() + 1)


@pytest.mark.parametrize("name", CASES)
def test_cold_start(orc, name):
    from paper_1307_6748_amd import solver as S
    om, sp, a = models(name)
    eta = density(10, 41)
    eta[0, 0, :3] = [1.0, 8.0, 1e4]
    expect = orc.cold_start(om, eta)
    got = cubic(S.cold_start(sp, a, dev(eta)), 10)
    assert np.max(np.abs(got - expect)) <= 1e-14 * (np.abs(expect).max() + 1)


@pytest.mark.parametrize("name", ["symmetron_a1", "fofr", "linear", "chameleon", "fofr_paper_u"])
@pytest.mark.parametrize("n", [8, 32, 64])
@pytest.mark.parametrize("tb", [0, 1, 2])
def test_sweeps_production_path(orc, name, n, tb):
    """The solver's sweep path (fused / temporally blocked where available)
    equals the per-colour reference sweeps."""
    from paper_1307_6748_amd import solver as S
    om, sp, a = models(name)
    h = 0.5
    phi = field_for(name, n, 51)
    eta = density(n, 52)
    sigma = sigma_for(name, n, 53, 0.1)
    for count in (1, 2, 3):
        expect = orc.sweep(om, h, phi, eta, sigma, count=count)
        g = dev(phi)
        S.sweeps(sp, a, h, g, dev(eta), dev(sigma), count=count, temporal_block=tb)
        assert np.max(np.abs(cubic(g, n) - expect)) <= 1e-12 * (np.abs(expect).max() + 1)


@pytest.mark.parametrize("name", ["symmetron_a1", "fofr", "linear", "chameleon", "fofr_paper_u"])
@pytest.mark.parametrize("n", [8, 32, 64, 128])
@pytest.mark.parametrize("tb", [0, 1, 2])
def test_prolong_sweeps(orc, name, n, tb):
    """The solver's post-smoothing step: phi += P(coarse - coarse_hat), then
    `count` sweeps.  On the fused kernels (n >= 64, tb >= 1) the correction is
    applied inside the first pass to every value it loads, halo included,
    from a two-plane coarse ring; it must equal the oracle's prolongation
    followed by its sweeps (count 0: the prolongation alone)."""
    from paper_1307_6748_amd import solver as S
    om, sp, a = models(name)
    h = 0.5
    rng = np.random.default_rng(60 + n)
    phi = field_for(name, n, 61)
    eta = density(n, 62)
    sigma = sigma_for(name, n, 63, 0.1)
    coarse = field_for(name, n // 2, 64)
    coarse_hat = coarse + 0.05 * rng.standard_normal(coarse.shape)
    for count in (0, 1, 2, 3):
        expect = orc.sweep(om, h, orc.prolong_correct(phi, coarse, coarse_hat), eta, sigma,
                           count=count) if count else orc.prolong_correct(phi, coarse, coarse_hat)
        g = dev(phi)
        S.prolong_sweeps(sp, a, h, g, dev(eta), dev(coarse), dev(coarse_hat), sigma=dev(sigma),
                         count=count, temporal_block=tb)
        assert np.max(np.abs(cubic(g, n) - expect)) <= 1e-12 * (np.abs(expect).max() + 1), count
