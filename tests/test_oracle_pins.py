"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, discrete eigenvalues, parameter definitions printed in the paper,
continuum limits, invariants and textbook special cases.  A dropped term, a
wrong sign, a wrong index or a transposed operand in the oracle fails at
least one of them.
"""
import numpy as np
import pytest

from paper_1307_6748_amd import synth

H0 = 1.0 / 2997.92458  # h/Mpc, c = 1


def lam_1d(m, n, h):
    """Eigenvalue of minus the periodic 1D second difference for mode m."""
    return (2.0 - 2.0 * np.cos(2.0 * np.pi * m / n)) / h ** 2


def lam_k(modes, n, h):
    return sum(lam_1d(m, n, h) for m in modes)


def cos_x(n, box, m):
    x = synth.cell_centres(n, box)
    return np.ascontiguousarray(np.broadcast_to(np.cos(2 * np.pi * m * x / box)[:, None, None],
                                                (n, n, n)))


# ---------------------------------------------------------------------------
# Operators
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("modes", [(1, 2, 3), (7, 1, 4), (8, 8, 8)])
def test_laplacian_eigenvector(orc, modes):
    """Sec. 3.1, discrete Laplacian: a product of sines at cell centres is an
    eigenvector with eigenvalue -sum_d (2 - 2 cos(2 pi m_d / N)) / h^2."""
    n, box = 16, 10.0
    h = box / n
    s = synth.sine_mode(n, box, modes)
    m = orc.Model(model=orc.LINEAR, kappa=0.0, m2=0.0)
    out = orc.defect(m, h, s, np.ones_like(s))
    expect = -lam_k(modes, n, h) * s
    assert np.max(np.abs(out - expect)) <= 1e-12 * lam_k(modes, n, h)


def test_linear_model_terms(orc):
    """LINEAR: L = lap(phi) - m2 phi - kappa (eta - 1)."""
    n, box = 16, 12.0
    h = box / n
    s = synth.sine_mode(n, box, (2, 1, 3))
    m = orc.Model(model=orc.LINEAR, kappa=2.5, m2=0.7)
    out = orc.defect(m, h, np.zeros_like(s), 1.0 + s)
    assert np.allclose(out, -2.5 * s, atol=1e-14, rtol=0)
    out = orc.defect(m, h, s, np.ones_like(s))
    assert np.allclose(out, -(lam_k((2, 1, 3), n, h) + 0.7) * s, atol=1e-13, rtol=0)


def test_flux_sum_vanishes(orc):
    """Fluxes telescope over the periodic box: sum_c (L_c + S_c) = 0 for both
    the canonical and the non-canonical operator (Sec. 3.4)."""
    n, box = 16, 32.0
    h = box / n
    u = synth.random_field(n, 3, scale=2.0, offset=-1.0)
    eta = synth.random_field(n, 4, scale=3.0, offset=0.1)
    for model in (orc.Model(model=orc.FR_HS), orc.Model(model=orc.SYMMETRON)):
        L = orc.defect(model, h, u, eta)
        S = np.array([orc.source(model, a, b)[0] for a, b in zip(u.ravel(), eta.ravel())])
        F = L.ravel() + S
        assert abs(F.sum()) <= 1e-12 * np.abs(F).sum()


@pytest.mark.parametrize("n", [16, 32, 64])
def test_flux_operator_continuum_limit(orc, n):
    """Non-canonical operator, Sec. 3.4: with b(u) = e^u the continuum
    div(e^u grad u) equals lap(e^u).  For e^u = 1 + 0.5 sin(2 pi x / B) this
    is -0.5 (2 pi / B)^2 sin(2 pi x / B); the arithmetic face averages must
    approach it at second order.  The pointwise source is removed with the
    oracle's own S (a uniform field has zero flux)."""
    box = 64.0
    h = box / n
    x = synth.cell_centres(n, box)
    e = 1.0 + 0.5 * np.sin(2 * np.pi * x / box)
    u = np.ascontiguousarray(np.broadcast_to(np.log(e)[:, None, None], (n, n, n)))
    eta = np.ones_like(u)
    m = orc.Model(model=orc.FR_HS)
    L = orc.defect(m, h, u, eta)[:, 0, 0]
    S = np.array([orc.source(m, v, 1.0)[0] for v in u[:, 0, 0]])
    F = L + S
    exact = -0.5 * (2 * np.pi / box) ** 2 * np.sin(2 * np.pi * x / box)
    err = np.max(np.abs(F - exact)) / np.max(np.abs(exact))
    # second order: err ~ C h^2 with C fixed by the profile
    assert err < 0.5 * (2 * np.pi * h / box) ** 2
    if n == 64:
        n2 = 32
        h2 = box / n2
        x2 = synth.cell_centres(n2, box)
        e2 = 1.0 + 0.5 * np.sin(2 * np.pi * x2 / box)
        u2 = np.ascontiguousarray(np.broadcast_to(np.log(e2)[:, None, None], (n2, n2, n2)))
        L2 = orc.defect(m, h2, u2, np.ones_like(u2))[:, 0, 0]
        S2 = np.array([orc.source(m, v, 1.0)[0] for v in u2[:, 0, 0]])
        ex2 = -0.5 * (2 * np.pi / box) ** 2 * np.sin(2 * np.pi * x2 / box)
        err2 = np.max(np.abs(L2 + S2 - ex2)) / np.max(np.abs(ex2))
        assert 3.6 < err2 / err < 4.4


def test_flux_operator_small_amplitude_is_laplacian(orc):
    """For u = eps s the non-canonical operator is the Laplacian to O(eps^2)."""
    n, box = 16, 40.0
    h = box / n
    s = synth.sine_mode(n, box, (1, 2, 1))
    m = orc.Model(model=orc.FR_HS)
    for eps in (1e-3, 1e-4):
        u = eps * s
        L = orc.defect(m, h, u, np.ones_like(u))
        S = np.array([orc.source(m, v, 1.0)[0] for v in u.ravel()]).reshape(u.shape)
        F = L + S
        rel = np.max(np.abs(F + lam_k((1, 2, 1), n, h) * u)) / np.max(np.abs(lam_k((1, 2, 1), n, h) * u))
        assert rel < 2 * eps


@pytest.mark.parametrize("model", ["symmetron", "fr", "linear", "chameleon", "fr_paper_u"])
def test_newton_denominator_is_jacobian_diagonal(orc, model):
    """Sec. 3.3 / 3.4 (eq. dbeq): the smoother's denominator equals dL_c/dphi_c
    (central finite difference of the oracle's own L) wherever the
    symmetron's safeguard is inactive."""
    n, box = 8, 8.0
    h = box / n
    rng = np.random.default_rng(5)
    if model == "symmetron":
        m = orc.Model(model=orc.SYMMETRON, a=1.0, lambda0=1.0, a_ssb=0.5)
        phi = 0.8 + 0.4 * rng.random((n, n, n))  # 3 phi^2 > 1 - A eta: dS >= 0
    elif model == "fr":
        m = orc.Model(model=orc.FR_HS, fR0_abs=1e-5)
        phi = -2.0 + 3.0 * rng.random((n, n, n))
    elif model == "chameleon":
        m = orc.Model(model=orc.CHAMELEON, cham_alpha=2.0, cham_mu=3.0, cham_n=0.5)
        phi = -1.0 + 2.0 * rng.random((n, n, n))
    elif model == "fr_paper_u":
        m = orc.Model(model=orc.FR_HS, fR0_abs=1e-5, n=2.0, a=0.7, paper_u=True)
        phi = np.log(0.49e-5) - 2.0 + 3.0 * rng.random((n, n, n))
    else:
        m = orc.Model(model=orc.LINEAR, kappa=1.0, m2=0.3)
        phi = rng.standard_normal((n, n, n))
    eta = 0.2 + 3.0 * rng.random((n, n, n))
    D = orc.newton_diag(m, h, phi, eta)
    for c in [(0, 0, 0), (3, 5, 7), (7, 7, 7), (2, 0, 6)]:
        d = 1e-6
        p1 = phi.copy(); p1[c] += d
        p2 = phi.copy(); p2[c] -= d
        fd = (orc.defect(m, h, p1, eta)[c] - orc.defect(m, h, p2, eta)[c]) / (2 * d)
        assert abs(fd - D[c]) <= 1e-6 * abs(D[c])


def test_symmetron_safeguard_denominator(orc):
    """Where dS/dchi < 0 the symmetron denominator is -6/h^2 - |dS/dchi|,
    i.e. it differs from the true derivative by 2 |dS/dchi|."""
    n, box = 8, 8.0
    h = box / n
    m = orc.Model(model=orc.SYMMETRON, a=1.0, lambda0=1.0, a_ssb=0.5)
    phi = np.full((n, n, n), 0.1)
    eta = np.full((n, n, n), 1.0)
    D = orc.newton_diag(m, h, phi, eta)
    c = (1, 2, 3)
    d = 1e-6
    p1 = phi.copy(); p1[c] += d
    p2 = phi.copy(); p2[c] -= d
    fd = (orc.defect(m, h, p1, eta)[c] - orc.defect(m, h, p2, eta)[c]) / (2 * d)
    # true derivative -6/h^2 - dS with dS < 0 here
    dS = -6.0 / h ** 2 - fd
    assert dS < 0
    assert abs(D[c] - (-6.0 / h ** 2 + dS)) <= 1e-6 * abs(D[c])


@pytest.mark.parametrize("model", ["symmetron", "fr"])
def test_newton_gauss_seidel_step_is_quadratic(orc, model):
    """Sec. 3.2: one Newton-Gauss-Seidel update solves its own cell's equation
    with quadratic error.  After the red half-sweep the residual left at red
    cells scales as the square of the perturbation."""
    n, box = 16, 32.0
    h = box / n
    eta = synth.lognormal(n, box, 1.0, 7)
    if model == "symmetron":
        m = orc.Model(model=orc.SYMMETRON, a=1.0, lambda0=1.0, a_ssb=0.5)
    else:
        m = orc.Model(model=orc.FR_HS, fR0_abs=1e-5)
    base = orc.solve(m, eta, box, tol=1e-12).phi
    noise = synth.random_field(n, 9, scale=2.0, offset=-1.0)
    i, j, k = np.indices((n, n, n))
    red = ((i + j + k) % 2) == 0
    res = []
    for d in (1e-2, 5e-3):
        phi = base + d * noise
        out = orc.halfsweep(m, h, phi, eta, None, 0)
        res.append(np.max(np.abs(orc.defect(m, h, out, eta)[red])))
    ratio = res[0] / res[1]
    assert 3.5 < ratio < 4.5


def test_linear_red_halfsweep_zeroes_red_residual(orc):
    """For a linear operator one Newton-GS update is exact: after the red
    half-sweep every red cell satisfies its equation."""
    n, box = 16, 16.0
    h = box / n
    m = orc.Model(model=orc.LINEAR, kappa=1.0, m2=0.5)
    eta = synth.random_field(n, 1, scale=2.0)
    phi = synth.random_field(n, 2)
    sigma = synth.random_field(n, 3)
    out = orc.halfsweep(m, h, phi, eta, sigma, 0)
    i, j, k = np.indices((n, n, n))
    red = ((i + j + k) % 2) == 0
    r = orc.defect(m, h, out, eta, sigma)
    assert np.max(np.abs(r[red])) < 1e-13
    assert np.array_equal(out[~red], phi[~red])  # black untouched


# ---------------------------------------------------------------------------
# Transfer operators
# ---------------------------------------------------------------------------

def test_restriction_mean_of_children(orc):
    n = 8
    f = np.arange(n ** 3, dtype=float).reshape(n, n, n)
    c = orc.restrict(f)
    # mean of 8 children of a linear function = value at the coarse centre
    I, J, K = np.indices((4, 4, 4))
    expect = ((2 * I + 0.5) * n + (2 * J + 0.5)) * n + (2 * K + 0.5)
    assert np.array_equal(c, expect)
    assert orc.restrict(np.full((8, 8, 8), 3.25)).tolist() == np.full((4, 4, 4), 3.25).tolist()


def test_prolongation_trilinear(orc):
    """Cell-centred trilinear interpolation: exact for linear functions away
    from the periodic seam, preserves constants and the mean, and is second
    order for smooth periodic data."""
    nc = 8
    nf = 16
    I, J, K = np.indices((nc, nc, nc)).astype(float)
    g = 1.5 * I - 0.25 * J + 2.0 * K
    out = orc.prolong_correct(np.zeros((nf,) * 3), g, np.zeros_like(g))
    i, j, k = np.indices((nf,) * 3).astype(float)
    # coarse cell I has centre at fine coordinate 2I + 1/2 (in fine cells)
    expect = 1.5 * (i / 2 - 0.25) - 0.25 * (j / 2 - 0.25) + 2.0 * (k / 2 - 0.25)
    inner = (slice(1, nf - 1),) * 3
    assert np.allclose(out[inner], expect[inner], atol=1e-13, rtol=0)
    c = np.full((nc,) * 3, 0.7)
    assert np.allclose(orc.prolong_correct(np.ones((nf,) * 3), c, np.zeros_like(c)), 1.7,
                       atol=1e-15, rtol=0)
    rnd = synth.random_field(nc, 11)
    p = orc.prolong_correct(np.zeros((nf,) * 3), rnd, np.zeros_like(rnd))
    assert abs(p.mean() - rnd.mean()) < 1e-14
    # the correction is P(coarse - coarse_hat)
    p2 = orc.prolong_correct(np.zeros((nf,) * 3), rnd + 2.0, np.full_like(rnd, 2.0))
    assert np.allclose(p, p2, atol=1e-14, rtol=0)
    errs = []
    for n_c in (8, 16):
        box = 1.0
        xc = synth.cell_centres(n_c, box)
        xf = synth.cell_centres(2 * n_c, box)
        sc = np.sin(2 * np.pi * xc)
        cc = np.ascontiguousarray(np.broadcast_to(sc[:, None, None], (n_c,) * 3))
        pf = orc.prolong_correct(np.zeros((2 * n_c,) * 3), cc, np.zeros_like(cc))[:, 0, 0]
        errs.append(np.max(np.abs(pf - np.sin(2 * np.pi * xf))))
    assert 3.5 < errs[0] / errs[1] < 4.5


# ---------------------------------------------------------------------------
# Closed forms of the models
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("a", [0.6, 0.8, 1.0])
@pytest.mark.parametrize("eta0", [0.1, 0.5, 2.0, 10.0])
def test_symmetron_homogeneous_root(orc, a, eta0):
    """Sec. 4.1, uniform density: chi = sqrt(max(0, 1 - (a_ssb/a)^3 eta))
    (the broken phase for low density, chi = 0 when screened)."""
    n, box = 8, 8.0
    m = orc.Model(model=orc.SYMMETRON, a=a, lambda0=1.0, a_ssb=0.5)
    eta = synth.uniform(n, eta0)
    v = 1.0 - (0.5 / a) ** 3 * eta0
    chi = np.sqrt(max(v, 0.0))
    guess = chi + 0.05 + 0.05 * synth.random_field(n, 3)
    r = orc.solve(m, eta, box, tol=0.0, phi0=guess, cfg=orc.Cfg(max_cycles=25))
    assert np.max(np.abs(r.phi - chi)) < 1e-10
    assert abs(orc.defect(m, box / n, np.full((n,) * 3, chi), eta)).max() < 1e-14
    if a == 1.0 and eta0 == 2.0:
        assert abs(chi - 0.8660254037844386) < 1e-15


def test_symmetron_z2_symmetry(orc):
    """chi -> -chi maps solutions to solutions; the iteration is odd."""
    w = synth.workload("small_symmetron")
    m = orc.Model(model=orc.SYMMETRON, a=1.0, lambda0=1.0, a_ssb=0.5)
    cold = orc.cold_start(m, w["eta"])
    r1 = orc.vcycles(m, w["eta"], w["box"], cold, 3)
    r2 = orc.vcycles(m, w["eta"], w["box"], -cold, 3)
    assert np.array_equal(r1.phi, -r2.phi)


def _mode_amplitude(field, s):
    return float((field * s).sum() / (s * s).sum())


def _response_mass(orc, m, n, box, eta0, eps, m1, m2):
    """Fit L'(phi) = -(lambda_k + mu^2) from responses to eta = eta0 (1 + eps cos)."""
    h = box / n
    amps = []
    for mode in (m1, m2):
        s = cos_x(n, box, mode)
        eta = eta0 * (1.0 + eps * s)
        base = orc.cold_start(m, synth.uniform(n, eta0))
        r = orc.solve(m, eta, box, tol=1e-12, phi0=base, cfg=orc.Cfg(max_cycles=60))
        amps.append(_mode_amplitude(r.phi - base, s) / eps)
    l1, l2 = lam_1d(m1, n, h), lam_1d(m2, n, h)
    A1, A2 = amps
    mu2 = (A2 * l2 - A1 * l1) / (A1 - A2)
    coef = -A1 * (l1 + mu2)
    return mu2, coef


def test_symmetron_vacuum_range_is_lambda0(orc):
    """Sec. 4.1: lambda0 is the range of the field at zero density and a_SSB is
    where the mean density restores the symmetry.  The Yukawa mass of small
    perturbations around the homogeneous root is linear in the density, equal
    to a^2/lambda0^2 (comoving) at eta = 0 and zero at eta = (a/a_ssb)^3."""
    a, lam0, assb = 0.8, 1.3, 0.5
    m = orc.Model(model=orc.SYMMETRON, a=a, lambda0=lam0, a_ssb=assb)
    etas = np.array([0.5, 1.0, 2.0])
    mus = np.array([_response_mass(orc, m, 16, 16.0, e, 1e-4, 1, 3)[0] for e in etas])
    slope, icpt = np.polyfit(etas, mus, 1)
    assert abs(icpt - a ** 2 / lam0 ** 2) < 1e-5 * a ** 2 / lam0 ** 2
    assert abs(-icpt / slope - (a / assb) ** 3) < 1e-5 * (a / assb) ** 3


@pytest.mark.parametrize("fr0,table", [(1e-4, 23.7), (1e-5, 7.5), (1e-6, 2.4)])
def test_fr_background_range_matches_paper_table(orc, fr0, table):
    """Sec. 4.2 and the model-parameter table of Sec. 6.1: with
    (Omega_m, Omega_L) = (0.267, 0.733) and n = 1 the range of the f(R)
    fifth force today is 23.7, 7.5 and 2.4 Mpc/h for |f_R0| = 1e-4, 1e-5,
    1e-6, and lambda = 3 sqrt((n+1)/(Omega_m + 4 Omega_L)) sqrt(|f_R0|/1e-6)
    Mpc/h (the 3 is c/H0 rounded to 3000 Mpc/h)."""
    m = orc.Model(model=orc.FR_HS, a=1.0, n=1.0, fR0_abs=fr0, omega_m=0.267, omega_l=0.733)
    box = {1e-4: 256.0, 1e-5: 64.0, 1e-6: 16.0}[fr0]
    mu2, coef = _response_mass(orc, m, 16, box, 1.0, 1e-4, 1, 2)
    rng_ = 1.0 / np.sqrt(mu2)
    assert abs(rng_ - table) <= 0.05 + 1e-3 * table
    formula = 3.0 * np.sqrt(2.0 / (0.267 + 4 * 0.733)) * np.sqrt(fr0 / 1e-6)
    assert abs(rng_ / formula - 2997.92458 / 3000.0) < 1e-5


@pytest.mark.parametrize("a", [1.0, 0.5])
def test_fr_linear_response_from_fR_equation(orc, a):
    """Sec. 4.2, equation for f_R, linearised by hand around its uniform
    background.  Its bracket vanishes at eta = 1 for
    (f_R0/f_R)^(1/(n+1)) = (a^-3 + cL)/(1 + cL), which fixes |f_R_bg|; the
    density term -(1/a) Omega_m H0^2 (eta - 1) and the derivative of the
    bracket then give, for u = ln(f_R/f_R0),
      lap(u) = Omega_m H0^2 / (a |f_R_bg|) delta_eta + mu^2 u,
      mu^2 = a^2 Omega_m H0^2 (a^-3 + cL) / ((n+1) |f_R_bg|)."""
    fr0, om, ol, nn = 1e-5, 0.27, 0.73, 1.0
    m = orc.Model(model=orc.FR_HS, a=a, n=nn, fR0_abs=fr0, omega_m=om, omega_l=ol)
    mu2, coef = _response_mass(orc, m, 16, 64.0, 1.0, 1e-4, 1, 2)
    cL = 4 * ol / om
    fbg = fr0 * ((1 + cL) / (a ** -3 + cL)) ** (nn + 1)
    coef_expect = om * H0 ** 2 / (a * fbg)
    mu2_expect = a ** 2 * om * H0 ** 2 * (a ** -3 + cL) / ((nn + 1) * fbg)
    assert abs(coef - coef_expect) < 1e-5 * coef_expect
    assert abs(mu2 - mu2_expect) < 1e-4 * mu2_expect


@pytest.mark.parametrize("eta0,a", [(1.0, 1.0), (10.0, 1.0), (1e3, 1.0), (0.1, 1.0), (1.0, 0.5)])
def test_fr_homogeneous_root(orc, eta0, a):
    """Sec. 4.2 at uniform density: u = -(n+1) ln[(eta a^-3 + cL)/(1 + cL)];
    f_R = f_R0 at eta = 1 today (the background minimum)."""
    om, ol = 0.27, 0.73
    m = orc.Model(model=orc.FR_HS, a=a, n=1.0, fR0_abs=1e-5, omega_m=om, omega_l=ol)
    n, box = 8, 16.0
    cL = 4 * ol / om
    u0 = -2.0 * np.log((eta0 / a ** 3 + cL) / (1 + cL))
    eta = synth.uniform(n, eta0)
    guess = u0 + 0.1 * synth.random_field(n, 2, offset=-0.5)
    r = orc.solve(m, eta, box, tol=0.0, phi0=guess, cfg=orc.Cfg(max_cycles=30))
    assert np.max(np.abs(r.phi - u0)) < 1e-10
    if eta0 == 1.0 and a == 1.0:
        assert abs(u0) < 1e-15
    if eta0 == 10.0:
        assert abs(u0 - (-1.132621)) < 5e-6
    if eta0 == 1e3:
        assert abs(u0 - (-8.898316)) < 5e-6


def test_symmetron_domain_wall_tanh(orc):
    """Planar symmetron domain walls (1D data in 3D): the continuum solution of
    chi'' = K (chi^3 - v^2 chi) with K = a^2 / (2 lambda0^2),
    v^2 = 1 - (a_ssb/a)^3 eta is v tanh(x / delta) with delta = 2 lambda0 / (a v).
    Two walls in a periodic box: the product of two tanh profiles, up to
    exp(-2 d / delta) tails.  The discrete solution converges at O(h^2)."""
    a, lam0, assb, eta0 = 1.0, 1.0, 0.5, 1.0
    m = orc.Model(model=orc.SYMMETRON, a=a, lambda0=lam0, a_ssb=assb)
    box = 32.0
    v = np.sqrt(1.0 - (assb / a) ** 3 * eta0)
    delta = 2 * lam0 / (a * v)
    x1, x2 = box / 4, 3 * box / 4
    errs = []
    for n in (32, 64):
        x = synth.cell_centres(n, box)
        prof = v * np.tanh((x - x1) / delta) * np.tanh((x2 - x) / delta)
        guess = np.ascontiguousarray(np.broadcast_to(prof[:, None, None], (n, n, n)))
        # Uniform density: r_ref = 0, so the tolerance is absolute.  The two
        # walls have a nearly free breathing mode (lattice-pinned), so the
        # residual levels off near 1e-9 instead of dropping geometrically.
        r = orc.solve(m, synth.uniform(n, eta0), box, tol=1e-12, phi0=guess,
                      cfg=orc.Cfg(max_cycles=12))
        assert r.r_ref == 0.0 and r.rel_hist[-1] < 2e-9
        got = r.phi[:, 0, 0]
        assert np.max(np.abs(r.phi - got[:, None, None])) < 1e-9  # 1D up to the stall
        errs.append(np.max(np.abs(got - prof)))
    assert errs[0] < 0.02
    assert 3.5 < errs[0] / errs[1] < 4.5


# ---------------------------------------------------------------------------
# The multigrid solve
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m2", [0.0, 0.3])
def test_linear_sine_exact_discrete_solution(orc, m2):
    """Sec. 3.1: FAS on the linear problem lap(phi) - m2 phi = kappa s with s a
    discrete eigenvector has the exact discrete solution
    phi = -kappa s / (lambda_k + m2)."""
    n, box, kappa = 32, 20.0, 1.7
    h = box / n
    modes = (1, 3, 2)
    s = synth.sine_mode(n, box, modes)
    m = orc.Model(model=orc.LINEAR, kappa=kappa, m2=m2)
    r = orc.solve(m, 1.0 + s, box, tol=1e-12)
    assert r.status == orc.OK
    exact = -kappa * s / (lam_k(modes, n, h) + m2)
    assert np.max(np.abs(r.phi - exact)) < 1e-11 * np.max(np.abs(exact))


def test_rms_and_r_ref_closed_form(orc):
    """The stop test's norm and reference residual (reading 12): RMS over the
    N^3 fine cells, r_ref = RMS of L_0 at the cold start.  For the linear model
    the cold start is phi = 0, so L_0 = -kappa (eta - 1); with eta - 1 = amp s,
    s a product of sines of modes 0 < m < N/2 at the cell centres, the mean of
    s^2 over the grid is exactly 1/8, hence r_ref = |kappa| amp 2^(-3/2).
    From the guess phi0 = c s, L_0 = -(c (lambda_k + m2) + kappa amp) s, so
    r0 = |c (lambda_k + m2) + kappa amp| 2^(-3/2) while r_ref does not move."""
    n, box, kappa, amp, m2 = 16, 24.0, -1.7, 0.3, 0.45
    h = box / n
    modes = (1, 3, 2)
    s = synth.sine_mode(n, box, modes)
    eta = 1.0 + amp * s
    m = orc.Model(model=orc.LINEAR, kappa=kappa, m2=m2)
    closed = abs(kappa) * amp * 2.0 ** -1.5
    r = orc.solve(m, eta, box, tol=1e-30, cfg=orc.Cfg(max_cycles=1))
    assert abs(r.r_ref - closed) <= 1e-13 * closed
    assert abs(r.r0 - closed) <= 1e-13 * closed      # cold start: r0 = r_ref
    assert abs(r.rel_hist[0] - 1.0) <= 1e-13
    c = 0.37
    r = orc.solve(m, eta, box, tol=1e-30, phi0=c * s, cfg=orc.Cfg(max_cycles=1))
    r0 = abs(c * (lam_k(modes, n, h) + m2) + kappa * amp) * 2.0 ** -1.5
    assert abs(r.r_ref - closed) <= 1e-13 * closed
    assert abs(r.r0 - r0) <= 1e-12 * r0
    assert abs(r.rel_hist[0] - r0 / closed) <= 1e-12 * r0 / closed
    # the norm itself: a constant field and a +-v checkerboard have RMS |v|
    assert orc.rms(np.full((8, 8, 8), -2.5)) == 2.5
    i, j, k = np.indices((8, 8, 8))
    assert abs(orc.rms(3.0 * (-1.0) ** (i + j + k)) - 3.0) <= 1e-15 * 3.0


def test_safeguard_count_is_the_number_of_negative_derivatives(orc):
    """Reading 14: the count of safeguarded updates.  In one red half-sweep
    every red cell is updated once from its own value before the sweep (cells
    of one colour never neighbour each other), so the count is the number of
    red cells with dS/dchi = K (A eta - 1 + 3 chi^2) < 0 at the input field.
    The linear model has no safeguard and counts nothing; a solve from the
    cold start at a uniform screened density counts nothing either."""
    n, box, a, lam, assb = 8, 16.0, 0.8, 1.0, 0.5
    K, A = a * a / (2 * lam * lam), (assb / a) ** 3
    phi = 0.4 * synth.random_field(n, 31)
    eta = 4.0 * synth.random_field(n, 32)
    m = orc.Model(model=orc.SYMMETRON, a=a, lambda0=lam, a_ssb=assb)
    i, j, k = np.indices((n, n, n))
    for colour in (0, 1):
        orc.guard_hits(reset=True)
        orc.halfsweep(m, box / n, phi, eta, colour=colour)
        dS = K * (A * eta - 1.0 + 3.0 * phi ** 2)
        want = int(np.sum((((i + j + k) & 1) == colour) & (dS < 0)))
        assert 0 < want < n ** 3 // 2
        assert orc.guard_hits() == want
    orc.guard_hits(reset=True)
    orc.halfsweep(orc.Model(model=orc.LINEAR, kappa=1.0, m2=0.1), box / n, phi, eta)
    assert orc.guard_hits() == 0
    r = orc.solve(m, np.full((n, n, n), 3.0 / A), box, tol=1e-10)  # A eta = 3: screened
    assert r.status == orc.OK and r.guard_hits == 0
    r = orc.solve(m, eta, box, tol=1e-10, phi0=phi)
    assert r.status == orc.OK and r.guard_hits > 0


def _mats_1d(n, h):
    D = np.zeros((n, n))
    for i in range(n):
        D[i, i] = -2.0
        D[i, (i - 1) % n] += 1.0
        D[i, (i + 1) % n] += 1.0
    return D / h ** 2


@pytest.mark.parametrize("fw", [False, True])
def test_fas_two_grid_equals_textbook_correction_scheme(orc, fw):
    """On a linear problem FAS is the linear correction scheme (Sec. 3.1):
    two levels (8^3 -> 4^3) with an exact coarse solve give
    phi <- S^nu2 (phi + P A_c^-1 R (b - A S^nu1 phi)), built here from dense
    matrices (A = lap - m2, P = trilinear, R = mean of 8 children, or with
    full weighting R = P^T / 8 for the defect -- reading 2's option; phi is
    restricted by the mean in both, which the linear scheme does not see)."""
    n, box, kappa, m2 = 8, 8.0, 1.0, 1.0
    h = box / n
    I1 = np.eye(n)
    D1 = _mats_1d(n, h)
    A = (np.kron(np.kron(D1, I1), I1) + np.kron(np.kron(I1, D1), I1) +
         np.kron(np.kron(I1, I1), D1)) - m2 * np.eye(n ** 3)
    nc = n // 2
    Ic = np.eye(nc)
    Dc = _mats_1d(nc, 2 * h)
    Ac = (np.kron(np.kron(Dc, Ic), Ic) + np.kron(np.kron(Ic, Dc), Ic) +
          np.kron(np.kron(Ic, Ic), Dc)) - m2 * np.eye(nc ** 3)
    R1 = np.zeros((nc, n))
    P1 = np.zeros((n, nc))
    for I in range(nc):
        R1[I, 2 * I] = R1[I, 2 * I + 1] = 0.5
    for i in range(n):
        p = i // 2
        q = (p + (1 if i % 2 else -1)) % nc
        P1[i, p] += 0.75
        P1[i, q] += 0.25
    if fw:
        R1 = P1.T / 2.0
    R = np.kron(np.kron(R1, R1), R1)
    P = np.kron(np.kron(P1, P1), P1)
    idx = np.indices((n, n, n)).reshape(3, -1)
    colour = idx.sum(axis=0) % 2
    eta = synth.random_field(n, 21, scale=2.0)
    b = kappa * (eta.ravel() - 1.0)
    phi = synth.random_field(n, 22).ravel()

    def gs(p):
        for c in (0, 1):
            msk = colour == c
            r = b - A @ p
            p = p + np.where(msk, r / np.diag(A), 0.0)
        return p

    x = phi.copy()
    for _ in range(2):
        x = gs(x)
    x = x + P @ np.linalg.solve(Ac, R @ (b - A @ x))
    for _ in range(2):
        x = gs(x)
    m = orc.Model(model=orc.LINEAR, kappa=kappa, m2=m2)
    r = orc.vcycles(m, eta, box, phi.reshape(n, n, n), 1, orc.Cfg(nu_coarse=400, restrict_fw=fw))
    assert np.max(np.abs(r.phi.ravel() - x)) < 1e-12 * np.max(np.abs(x))


def test_full_weighting_restriction(orc):
    """Reading 2's option, full weighting R = P^T / 8: adjoint of the
    prolongation (<R f, c> = <f, P c> / 8 for random fields), constants kept,
    totals preserved (sum of the coarse field = sum of the fine one / 8).  On
    a product of sines of wavenumbers k_d it returns the same product at the
    coarse centres times prod_d cos^3(k_d h / 2) (the 8-child mean: times
    prod_d cos(k_d h / 2))."""
    n, box = 16, 10.0
    h = box / n
    f = synth.random_field(n, 51, scale=2.0, offset=-1.0)
    c = synth.random_field(n // 2, 52, scale=2.0, offset=-1.0)
    Pc = orc.prolong_correct(np.zeros((n, n, n)), c, np.zeros((n // 2,) * 3))
    Rf = orc.restrict_fw(f)
    assert abs(np.sum(Rf * c) - np.sum(f * Pc) / 8.0) <= 1e-13 * np.sum(np.abs(f * Pc))
    assert np.max(np.abs(orc.restrict_fw(np.full((n, n, n), 3.7)) - 3.7)) <= 8 * 2.0 ** -52 * 3.7
    assert abs(np.sum(Rf) - np.sum(f) / 8.0) <= 1e-12 * np.sum(np.abs(f))
    modes = (1, 3, 2)
    s_f = synth.sine_mode(n, box, modes)
    s_c = synth.sine_mode(n // 2, box, modes)
    th = [np.pi * m * h / box for m in modes]  # k h / 2
    g_fw = np.prod([np.cos(t) ** 3 for t in th])
    g_mean = np.prod([np.cos(t) for t in th])
    assert np.max(np.abs(orc.restrict_fw(s_f) - g_fw * s_c)) <= 1e-14
    assert np.max(np.abs(orc.restrict(s_f) - g_mean * s_c)) <= 1e-14


def test_solution_does_not_depend_on_the_restriction(orc):
    """Reading 2: the restriction changes the convergence factors, not the
    discrete root: f(R) and symmetron solves with the mean and with full
    weighting of the defect agree to their tolerance."""
    w = synth.workload("small_symmetron", 16)
    for m in (orc.Model(model=orc.FR_HS, a=1.0, n=1.0, fR0_abs=1e-5, omega_m=0.27,
                        omega_l=0.73),
              orc.Model(model=orc.SYMMETRON, a=1.0, lambda0=1.0, a_ssb=0.5)):
        r0 = orc.solve(m, w["eta"], w["box"], tol=1e-13, cfg=orc.Cfg(restrict_fw=False))
        r1 = orc.solve(m, w["eta"], w["box"], tol=1e-13, cfg=orc.Cfg(restrict_fw=True))
        assert r0.status == orc.OK and r1.status == orc.OK
        assert np.max(np.abs(r1.phi - r0.phi)) <= 1e-10 * np.max(np.abs(r0.phi))
        assert not np.allclose(r0.rel_hist[1:3], r1.rel_hist[1:3], rtol=1e-3)


def test_fas_fixed_point(orc):
    """Sec. 3.2: at the discrete root the FAS coarse equation is solved by
    R phi itself (Sigma = L_c(R phi) - R[0]), so a V-cycle leaves the root
    unchanged."""
    w = synth.workload("small_symmetron")
    m = orc.Model(model=orc.SYMMETRON, a=1.0, lambda0=1.0, a_ssb=0.5)
    r = orc.solve(m, w["eta"], w["box"], tol=1e-13)
    r2 = orc.vcycles(m, w["eta"], w["box"], r.phi, 1)
    assert np.max(np.abs(r2.phi - r.phi)) < 1e-13


@pytest.mark.parametrize("m2", [0.0, 0.5])
def test_linear_convergence_factor_h_independent(orc, m2):
    """Multigrid invariant: the V(2,2) convergence factor on the linear problem
    is small and does not grow with resolution."""
    rhos = []
    for n in (16, 32, 64):
        box = float(n)
        eta = 1.0 + synth.random_field(n, 5, scale=1.0, offset=-0.5)
        eta += 1.0 - eta.mean()  # m2 = 0 needs a zero-mean source
        m = orc.Model(model=orc.LINEAR, kappa=1.0, m2=m2)
        r = orc.vcycles(m, eta, box, synth.random_field(n, 6), 6)
        h = r.rel_hist
        rhos.append(float(np.exp(np.mean(np.log(h[3:] / h[2:-1])))))
    assert max(rhos) < 0.15
    assert max(rhos) - min(rhos) < 0.05


def test_symmetron_solve_converges_fast(orc):
    """The 32^3 symmetron workload reaches 1e-10 in a few V-cycles."""
    w = synth.workload("small_symmetron")
    m = orc.Model(model=orc.SYMMETRON, a=1.0, lambda0=1.0, a_ssb=0.5)
    r = orc.solve(m, w["eta"], w["box"], tol=1e-10)
    assert r.status == orc.OK and r.cycles <= 6
    rho = r.rel_hist[1:] / r.rel_hist[:-1]
    assert np.all(rho < 0.05)
    assert np.all(r.phi > 0)  # positive branch selected by the cold start


def test_translation_equivariance(orc):
    """Shifting the density by one cell shifts the root (the colours swap, so
    only the iteration path differs)."""
    w = synth.workload("small_symmetron")
    m = orc.Model(model=orc.SYMMETRON, a=1.0, lambda0=1.0, a_ssb=0.5)
    r1 = orc.solve(m, w["eta"], w["box"], tol=1e-12)
    r2 = orc.solve(m, np.roll(w["eta"], 1, axis=0), w["box"], tol=1e-12)
    assert np.max(np.abs(np.roll(r1.phi, 1, axis=0) - r2.phi)) < 1e-11


def test_axis_permutation_equivariance(orc):
    w = synth.workload("small_symmetron")
    m = orc.Model(model=orc.SYMMETRON, a=1.0, lambda0=1.0, a_ssb=0.5)
    r1 = orc.solve(m, w["eta"], w["box"], tol=1e-12)
    eta_p = np.ascontiguousarray(np.transpose(w["eta"], (2, 0, 1)))
    r2 = orc.solve(m, eta_p, w["box"], tol=1e-12)
    assert np.max(np.abs(np.transpose(r1.phi, (2, 0, 1)) - r2.phi)) < 1e-12


def test_integral_constraint_at_root(orc):
    """At the root the fluxes telescope, so sum_c S(phi_c, eta_c) = 0."""
    w = synth.workload("fr_256", n=32)
    m = orc.Model(model=orc.FR_HS, fR0_abs=1e-5)
    r = orc.solve(m, w["eta"], w["box"], tol=1e-12)
    S = np.array([orc.source(m, p, e)[0] for p, e in zip(r.phi.ravel(), w["eta"].ravel())])
    assert abs(S.mean()) < 1e-9 * np.abs(S).mean()


def test_thread_count_independence(orc):
    w = synth.workload("fr_256", n=32)
    m = orc.Model(model=orc.FR_HS, fR0_abs=1e-5)
    orc.set_threads(1)
    r1 = orc.solve(m, w["eta"], w["box"], tol=1e-10)
    orc.set_threads(4)
    r2 = orc.solve(m, w["eta"], w["box"], tol=1e-10)
    assert np.array_equal(r1.phi, r2.phi)
    assert np.array_equal(r1.rel_hist, r2.rel_hist)


def test_invalid_arguments(orc):
    m = orc.Model()
    with pytest.raises(ValueError):
        orc.solve(m, np.ones((12, 12, 12)), 10.0)
    with pytest.raises(ValueError):
        orc.solve(m, np.ones((4, 4, 4)), 10.0)
    with pytest.raises(ValueError):
        orc.solve(orc.Model(a=0.0), np.ones((8, 8, 8)), 10.0)
    assert orc.num_levels(8) == 2 and orc.num_levels(512) == 8
