"""Pins of the oracle's refinement-boundary discretisation with masks
(Sec. 3.3.1 and 3.4.1): inside cells (mask > 0) are relaxed, masked
neighbours (mask <= 0) enter through ghost values
u_G = u^Int + (m_f / m_c)(u_c - u_c^Pre), and the Newton denominator gains the
ghosts' dependence on u_c.  Pinned by: reduction to the uniform operator when
nothing is masked; the ghost as the geometric construction (boundary at the
mask's zero crossing, linear extrapolation through it); exactness on linear
fields for any masks; the denominator against central differences; a planar
patch against a 1D Dirichlet solve; and a refined patch approaching the
uniform fine solution."""
import numpy as np
import pytest

from paper_1307_6748_amd import synth

MODELS = {
    "symmetron": dict(model=0, a=1.0, lambda0=1.0, a_ssb=0.5),
    "fofr": dict(model=1, a=1.0, n=1.0, fR0_abs=1e-5, omega_m=0.27, omega_l=0.73),
    "chameleon": dict(model=3, cham_alpha=2.0, cham_mu=3.0, cham_n=1.0),
    "linear": dict(model=2, kappa=1.3, m2=0.4),
}


def _field(name, n, seed):
    rng = np.random.default_rng(seed)
    if name == "symmetron":
        return 0.5 + 0.4 * rng.random((n, n, n))
    if name == "fofr":
        return -3.0 + 2.0 * rng.random((n, n, n))
    if name == "chameleon":
        return -1.0 + 2.0 * rng.random((n, n, n))
    return rng.standard_normal((n, n, n))


def _patch_mask(n, lo, hi, rng=None, frac=False):
    """1 inside the box [lo, hi)^3, -1 outside; with frac, random fractional
    values (inside (0.1, 1], outside [-1, 0], some exactly -1)."""
    idx = np.arange(n)
    ins = ((idx >= lo) & (idx < hi))
    inside = ins[:, None, None] & ins[None, :, None] & ins[None, None, :]
    m = np.where(inside, 1.0, -1.0)
    if frac:
        r = rng.random((n, n, n))
        m = np.where(inside, 0.1 + 0.9 * r, np.where(r < 0.3, -1.0, -r))
    return m


@pytest.mark.parametrize("name", sorted(MODELS))
def test_nothing_masked_is_the_uniform_operator(orc, name):
    n, h = 8, 0.7
    om = orc.Model(**MODELS[name])
    phi = _field(name, n, 1)
    eta = 0.2 + synth.random_field(n, 2, scale=2.0)
    sig = 0.1 * synth.random_field(n, 3)
    ones = np.ones((n, n, n))
    junk = synth.random_field(n, 4)  # u_int, u_pre: unused without masked neighbours
    assert np.array_equal(orc.masked_defect(om, h, phi, eta, ones, junk, junk, sig),
                          orc.defect(om, h, phi, eta, sig))
    assert np.array_equal(orc.masked_newton_diag(om, h, phi, eta, ones, junk, junk),
                          orc.newton_diag(om, h, phi, eta))
    for c in (0, 1):
        assert np.array_equal(orc.masked_halfsweep(om, h, phi, eta, ones, junk, junk, sig, c),
                              orc.halfsweep(om, h, phi, eta, sig, c))


def test_ghost_is_the_extrapolation_through_the_boundary(orc):
    """The boundary sits where the linear interpolation of the mask between
    the two centres crosses zero, at the fraction t = m_c / (m_c - m_f) of the
    way to the masked cell; the boundary value interpolates linearly between
    u_c^Pre and u_f^Int; the ghost extrapolates linearly from u_c through the
    boundary value to the masked cell's centre.  Read off the linear model's
    operator (L = lap u for kappa = m2 = 0) cell by cell."""
    n, h = 10, 0.5
    rng = np.random.default_rng(5)
    mask = _patch_mask(n, 2, 8, rng, frac=True)
    phi = rng.standard_normal((n, n, n))
    u_int = rng.standard_normal((n, n, n))
    u_pre = rng.standard_normal((n, n, n))
    om = orc.Model(model=orc.LINEAR, kappa=0.0, m2=0.0)
    got = orc.masked_defect(om, h, phi, np.ones_like(phi), mask, u_int, u_pre)
    want = np.zeros_like(phi)
    for i, j, k in zip(*np.nonzero(mask > 0)):
        acc = 0.0
        for d in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
            f = ((i + d[0]) % n, (j + d[1]) % n, (k + d[2]) % n)
            if mask[f] > 0:
                acc += phi[f]
                continue
            t = mask[i, j, k] / (mask[i, j, k] - mask[f])
            uI = u_pre[f] if mask[f] > -1.0 else u_int[f]
            u_b = u_pre[i, j, k] + t * (uI - u_pre[i, j, k])
            acc += phi[i, j, k] + (u_b - phi[i, j, k]) / t
        want[i, j, k] = (acc - 6.0 * phi[i, j, k]) / h ** 2
    assert np.max(np.abs(got - want)) <= 1e-11 * np.abs(want).max()


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_linear_fields_are_exact_with_any_masks(orc, seed):
    """A linear field with its boundary values set from itself (u^Pre = u,
    u^Int = the field): the ghost values are the field's own values, so the
    discrete Laplacian vanishes at every inside cell whatever the masks."""
    n, h = 12, 0.8
    rng = np.random.default_rng(seed)
    mask = _patch_mask(n, 3, 9, rng, frac=True)
    x = (np.arange(n) + 0.5) * h
    a, b, c, d = rng.standard_normal(4)
    u = d + a * x[:, None, None] + b * x[None, :, None] + c * x[None, None, :]
    om = orc.Model(model=orc.LINEAR, kappa=0.0, m2=0.0)
    L = orc.masked_defect(om, h, u, np.ones_like(u), mask, u, u)
    assert np.max(np.abs(L)) <= 1e-12 * np.abs(u).max() / h ** 2


@pytest.mark.parametrize("name", sorted(MODELS))
def test_masked_denominator_is_the_derivative(orc, name):
    """D_c = dL_c/du_c with u^Int and u^Pre held: central differences of the
    masked operator at inside cells next to masked neighbours (symmetron at
    dS/dchi > 0, where its safeguard is inactive)."""
    n, h = 10, 0.6
    rng = np.random.default_rng(11)
    mask = _patch_mask(n, 2, 8, rng, frac=True)
    om = orc.Model(**MODELS[name])
    phi = _field(name, n, 12)
    eta = 0.2 + synth.random_field(n, 13, scale=(1.0 if name == "symmetron" else 3.0))
    if name == "symmetron":  # A eta > 1 everywhere: dS/dchi > 0
        eta = 9.0 + eta
    u_int = phi + 0.3 * rng.standard_normal(phi.shape)
    u_pre = phi + 0.2 * rng.standard_normal(phi.shape)
    D = orc.masked_newton_diag(om, h, phi, eta, mask, u_int, u_pre)
    edge = [tuple(c) for c in np.argwhere(mask > 0)
            if min(c) == 2 or max(c) == 7][:40]
    assert len(edge) == 40
    eps = 1e-5
    for c in edge:
        up, um = phi.copy(), phi.copy()
        up[c] += eps
        um[c] -= eps
        fd = (orc.masked_defect(om, h, up, eta, mask, u_int, u_pre)[c] -
              orc.masked_defect(om, h, um, eta, mask, u_int, u_pre)[c]) / (2 * eps)
        assert abs(fd - D[c]) <= 1e-6 * abs(D[c]), (c, fd, D[c])


def test_planar_patch_is_a_1d_dirichlet_problem(orc):
    """A slab patch (inside for 3 <= i <= 12 along x, all y and z) of the
    linear problem with data varying along x only: the converged patch solve
    (u^Pre = u at the fixed point, so the ghost is u^Int) is the 1D problem
    (u_{i+1} + u_{i-1} - 2 u_i)/h^2 - m2 u_i = kappa (eta_i - 1) with the
    ghost values u^Int at i = 2 and i = 13 as Dirichlet data."""
    n, h, kappa, m2 = 16, 0.5, 1.3, 0.4
    lo, hi = 3, 13
    x = np.arange(n)
    mask1 = np.where((x >= lo) & (x < hi), 1.0, -1.0)
    mask = np.broadcast_to(mask1[:, None, None], (n, n, n)).copy()
    eta1 = 1.0 + 0.5 * np.sin(0.7 * x)
    eta = np.broadcast_to(eta1[:, None, None], (n, n, n)).copy()
    g1 = 0.3 * np.cos(0.4 * x) + 0.1 * x
    u_int = np.broadcast_to(g1[:, None, None], (n, n, n)).copy()
    om = orc.Model(model=orc.LINEAR, kappa=kappa, m2=m2)
    phi0 = np.zeros((n, n, n))
    phi, sweeps, rms = orc.patch_solve(om, h, phi0, eta, mask, u_int, block=3, tol=1e-12)
    assert rms <= 1e-12 and sweeps > 0
    # 1D tridiagonal system on the inside cells
    m = hi - lo
    A = np.zeros((m, m))
    rhs = kappa * (eta1[lo:hi] - 1.0) * h ** 2
    for q in range(m):
        A[q, q] = -2.0 - m2 * h ** 2
        if q > 0:
            A[q, q - 1] = 1.0
        if q < m - 1:
            A[q, q + 1] = 1.0
    rhs[0] -= g1[lo - 1]
    rhs[-1] -= g1[hi]
    u1 = np.linalg.solve(A, rhs)
    inside = phi[lo:hi]
    assert np.max(np.abs(inside - u1[:, None, None])) <= 1e-10 * np.abs(u1).max()
    # masked cells keep their values
    assert np.array_equal(phi[:lo], phi0[:lo]) and np.array_equal(phi[hi:], phi0[hi:])


def test_refined_patch_approaches_the_fine_solution(orc):
    """A static refinement (Sec. 3.3.1): the symmetron solved on a 16^3 coarse
    grid; a patch covering its central 8^3 cells at twice the resolution gets
    its outside values by trilinear interpolation of the coarse solution.  In
    the patch interior the patch solution is much closer to the uniform 32^3
    solution than the interpolated coarse one is."""
    box = 16.0
    om = orc.Model(model=orc.SYMMETRON, a=1.0, lambda0=1.0, a_ssb=0.5)
    eta_f = synth.lognormal(32, box, 1.0, 41)
    eta_c = orc.restrict(eta_f)
    coarse = orc.solve(om, eta_c, box, tol=1e-12).phi
    fine = orc.solve(om, eta_f, box, tol=1e-12).phi
    interp = orc.prolong_correct(np.zeros((32,) * 3), coarse, np.zeros((16,) * 3))
    # patch: fine cells 14..49 of the (periodic) 32^3 grid around the centre
    # would wrap; take fine cells 8..23 (inside) with two outside layers
    lo, hi, pad = 8, 24, 2
    sl = slice(lo - pad, hi + pad)
    npch = hi - lo + 2 * pad
    mask = _patch_mask(npch, pad, pad + (hi - lo))
    u_int = interp[sl, sl, sl]
    phi, sweeps, rms = orc.patch_solve(om, box / 32, u_int, eta_f[sl, sl, sl], mask, u_int,
                                       block=4, tol=1e-11)
    assert rms <= 1e-11
    core = slice(pad + 2, pad + (hi - lo) - 2)  # away from the patch boundary
    fine_core = fine[sl, sl, sl][core, core, core]
    e_patch = np.abs(phi[core, core, core] - fine_core).max()
    e_interp = np.abs(u_int[core, core, core] - fine_core).max()
    assert e_patch < 0.1 * e_interp, (e_patch, e_interp)  # measured 0.04


def test_chameleon_masked_steps_are_bounded(orc):
    """Chameleon with n = -1/2 on a lognormal density with sigma_delta = 2,
    patch cells started at zero, far from the local roots (which span about
    -8 .. 11): the masked half-sweep moves no cell by more than 2 (reading
    R15; unbounded Newton steps overflow here), and the patch solve reaches
    its tolerance with a finite field."""
    m = orc.Model(model=orc.CHAMELEON, cham_alpha=0.7, cham_mu=0.4, cham_n=-0.5)
    n, box = 16, 32.0
    eta = synth.lognormal(n, box, 2.0, 31)
    mask = _patch_mask(n, 2, 14)
    root = orc.cold_start(m, eta)
    u = np.zeros_like(eta)
    for c in (0, 1):
        v = orc.masked_halfsweep(m, box / n, u, eta, mask, root, root, colour=c)
        assert np.max(np.abs(v - u)) == 2.0
        u = v
    phi, sweeps, rms = orc.patch_solve(m, box / n, np.zeros_like(eta), eta, mask, root, block=4,
                                       tol=1e-10)
    assert rms <= 1e-10 and np.all(np.isfinite(phi))
