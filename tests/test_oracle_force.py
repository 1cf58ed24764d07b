"""Pins of the oracle's force on the grid (the step after the solve in the
paper's pipeline: the geodesic equations of Sec. 4.1 and 4.2).

The gradient stencil, sign and axis mapping are pinned by the exact central
difference of a sine; the structure of the scalar-field terms (chi grad chi,
e^u grad u) by ratios against a plain gradient; and their coefficients by
physics: in the linear regime the symmetron's fifth force is 2 beta^2
chi0^2 times Newtonian gravity below its Compton wavelength (chi0^2 = 1 -
(a_ssb/a)^3), and the f(R) force is 1/3 of Newtonian gravity (gravity
enhanced by 4/3), each with the Yukawa suppression lambda / (lambda + m^2)
whose mass the linear-response pins fix."""
import numpy as np
import pytest

from paper_1307_6748_amd import synth

H0 = 1.0 / 2997.92458  # h/Mpc, c = 1


def _centres(n, box):
    return (np.arange(n) + 0.5) * (box / n)


def _along(v, axis, n):
    shape = [1, 1, 1]
    shape[axis] = n
    return np.ascontiguousarray(np.broadcast_to(v.reshape(shape), (n, n, n)))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_gradient_of_a_sine_is_the_exact_central_difference(orc, axis):
    """-grad(potential) with potential = sin(k x): the periodic central
    difference is exactly cos(k x) sin(k h) / h along the axis, zero across."""
    n, box, mode = 16, 32.0, 3
    h = box / n
    k = 2 * np.pi * mode / box
    x = _centres(n, box)
    pot = _along(np.sin(k * x), axis, n)
    m = orc.Model(model=orc.LINEAR, kappa=1.0)
    f = orc.force(m, h, np.zeros((n, n, n)), pot)
    expect = -_along(np.cos(k * x) * np.sin(k * h) / h, axis, n)
    for ax in range(3):
        if ax == axis:
            assert np.max(np.abs(f[ax] - expect)) < 1e-14
        else:
            assert np.max(np.abs(f[ax])) == 0.0


def test_gradient_is_second_order(orc):
    """Halving h cuts the error of the gradient of a smooth periodic field 4x."""
    errs = []
    box = 10.0
    m = orc.Model(model=orc.LINEAR, kappa=1.0)
    for n in (16, 32, 64):
        x = _centres(n, box)
        k = 2 * np.pi / box
        pot = _along(np.exp(np.sin(k * x)), 0, n)
        fx = orc.force(m, box / n, np.zeros((n, n, n)), pot)[0]
        exact = -_along(k * np.cos(k * x) * np.exp(np.sin(k * x)), 0, n)
        errs.append(np.max(np.abs(fx - exact)))
    assert 3.7 < errs[0] / errs[1] < 4.3 and 3.7 < errs[1] / errs[2] < 4.3


def test_constant_field_has_no_force(orc):
    n = 8
    for m in (orc.Model(model=orc.SYMMETRON), orc.Model(model=orc.FR_HS)):
        f = orc.force(m, 1.0, np.full((n, n, n), 0.7), np.full((n, n, n), 3.0))
        assert max(np.max(np.abs(c)) for c in f) == 0.0


def test_axis_permutation_equivariance(orc):
    rng = np.random.default_rng(3)
    n = 8
    phi = rng.random((n, n, n))
    m = orc.Model(model=orc.FR_HS, a=0.9)
    f = orc.force(m, 0.5, phi)
    g = orc.force(m, 0.5, np.ascontiguousarray(phi.transpose(1, 2, 0)))
    # field'(i,j,k) = field(j,k,i): the x-force of field' is the y-force of field
    assert np.allclose(g[0], f[1].transpose(1, 2, 0), rtol=0, atol=1e-300)
    assert np.allclose(g[1], f[2].transpose(1, 2, 0), rtol=0, atol=1e-300)
    assert np.allclose(g[2], f[0].transpose(1, 2, 0), rtol=0, atol=1e-300)


def test_scalar_terms_have_the_geodesic_structure(orc):
    """Symmetron: force proportional to chi grad chi; f(R): to e^u grad u --
    the ratio to the plain central difference of the field is chi times a
    constant, resp. e^u times a constant, at every cell."""
    rng = np.random.default_rng(4)
    n, h = 8, 0.5
    phi = 0.5 + rng.random((n, n, n))
    lin = orc.Model(model=orc.LINEAR)
    g = orc.force(lin, h, np.zeros((n, n, n)), phi)[0]  # -D phi
    mask = np.abs(g) > 1e-3
    fs = orc.force(orc.Model(model=orc.SYMMETRON, a=0.9, beta=1.3), h, phi)[0]
    c1 = fs[mask] / (phi[mask] * g[mask])
    assert np.ptp(c1) < 1e-12 * np.abs(c1).max() and c1[0] > 0
    ff = orc.force(orc.Model(model=orc.FR_HS, a=0.9), h, phi)[0]
    c2 = ff[mask] / (np.exp(phi[mask]) * g[mask])
    assert np.ptp(c2) < 1e-12 * np.abs(c2).max() and c2[0] > 0


def _linear_forces(orc, m, n, box, eps, mode, a):
    """Scalar-field force and Newtonian force for eta = 1 + eps sin(k x): the
    field from the oracle's nonlinear solve, the potential from its linear
    solve of the Poisson equation of Sec. 3.1 (lap Phi = 1.5 Omega_m H0^2
    (eta - 1) / a, Phi~ = a^2 Phi).  Returns both x-forces and lambda_k."""
    h = box / n
    k = 2 * np.pi * mode / box
    x = _centres(n, box)
    s = _along(np.sin(k * x), 0, n)
    eta = 1.0 + eps * s
    base = orc.cold_start(m, synth.uniform(n, 1.0))
    r = orc.solve(m, eta, box, tol=1e-13, phi0=base, cfg=orc.Cfg(max_cycles=80))
    f5 = orc.force(m, h, r.phi)[0]
    lin = orc.Model(model=orc.LINEAR, a=a, kappa=1.5 * m.omega_m * H0 ** 2 / a, m2=0.0)
    rp = orc.solve(lin, eta, box, tol=1e-13, cfg=orc.Cfg(max_cycles=80))
    fN = orc.force(lin, h, np.zeros((n, n, n)), a * a * rp.phi)[0]
    lam = (2 - 2 * np.cos(k * h)) / h ** 2
    return f5, fN, lam


@pytest.mark.parametrize("beta,a", [(1.0, 1.0), (0.5, 1.0), (2.0, 0.8)])
def test_symmetron_fifth_force_is_2beta2_gravity(orc, beta, a):
    lam0, assb = 4.0, 0.5
    m = orc.Model(model=orc.SYMMETRON, a=a, lambda0=lam0, a_ssb=assb, beta=beta, omega_m=0.27)
    f5, fN, lam = _linear_forces(orc, m, 32, 32.0, 1e-5, 2, a)
    A = (assb / a) ** 3
    chi0sq = 1 - A
    msq = a ** 2 / lam0 ** 2 * (1 - A)
    expect = 2 * beta ** 2 * chi0sq * lam / (lam + msq)
    sel = np.abs(fN) > 0.5 * np.abs(fN).max()
    ratio = f5[sel] / fN[sel]
    assert np.max(np.abs(ratio - expect)) < 1e-3 * expect


@pytest.mark.parametrize("a,nn", [(1.0, 1.0), (0.7, 1.0), (1.0, 2.0)])
def test_fofr_force_is_one_third_of_gravity(orc, a, nn):
    om, ol, fr0 = 0.27, 0.73, 1e-4
    m = orc.Model(model=orc.FR_HS, a=a, n=nn, fR0_abs=fr0, omega_m=om, omega_l=ol)
    f5, fN, lam = _linear_forces(orc, m, 32, 64.0, 1e-5, 2, a)
    cL = 4 * ol / om
    a3 = a ** 3
    eu0 = (a3 * (1 + cL) / (1 + cL * a3)) ** (nn + 1)  # background e^u: S(u0, eta=1) = 0
    Q = om * H0 ** 2 / (a * fr0)
    mu2 = Q * (1 + cL * a3) / (nn + 1)
    expect = (1.0 / 3.0) * eu0 * lam / (eu0 * lam + mu2)
    sel = np.abs(fN) > 0.5 * np.abs(fN).max()
    ratio = f5[sel] / fN[sel]
    assert np.max(np.abs(ratio - expect)) < 1e-3 * expect
