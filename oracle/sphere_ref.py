"""Radial reference solutions for the static top-hat sphere test of Sec. 5.1.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): the tests compare the
3D grid solutions of the GPU solver with these 1D solutions.  Nothing here
is shared with the GPU library.

A sphere of radius R and constant density sits in a uniform background; the
density jump is delta and the mean over the box B^3 is 1 (Sec. 5.1):
    eta_in = (1 + delta) / (1 + (4 pi / 3) delta (R / B)^3),
    eta_out = 1 / (1 + (4 pi / 3) delta (R / B)^3).
The field equations of Sec. 4.1 (symmetron) and Sec. 4.2 (f(R), in
u = ln(f_R / f_R0)) reduce in spherical symmetry to ODEs in r, solved here
two independent ways: scipy's collocation BVP solver, and a plain
finite-difference Newton iteration on a fine radial mesh (tests check that
the two agree).  Boundary conditions: regular at r = 0, the homogeneous
root of the background density at r_max (several field ranges from R).
"""
from __future__ import annotations

import numpy as np

H0 = 1.0 / 2997.92458  # h/Mpc, c = 1


def tophat(R: float, B: float, delta: float):
    norm = 1.0 + 4.0 * np.pi / 3.0 * delta * (R / B) ** 3
    return (1.0 + delta) / norm, 1.0 / norm


def grid_density(n: int, B: float, R: float, delta: float, sub: int = 4) -> np.ndarray:
    """Cell averages of the top-hat density (sphere at the box centre), from
    sub^3 sample points per cell; the cells cut by the surface get the
    volume-weighted mix of eta_in and eta_out."""
    eta_in, eta_out = tophat(R, B, delta)
    h = B / n
    off = (np.arange(sub) + 0.5) / sub * h
    x = np.arange(n) * h - B / 2.0  # cell low corners, centred box
    # nearest and farthest squared distance of each cell from the centre: the
    # cells wholly inside (all samples inside) get 1, those wholly outside 0,
    # and only the cells the surface cuts are sampled
    near = np.where(x > 0, x, np.where(x + h < 0, x + h, 0.0)) ** 2
    far = np.maximum(x ** 2, (x + h) ** 2)
    dmin = near[:, None, None] + near[None, :, None] + near[None, None, :]
    dmax = far[:, None, None] + far[None, :, None] + far[None, None, :]
    frac = (dmax < R * R).astype(np.float64)
    cut = np.argwhere((dmin < R * R) & ~(dmax < R * R))
    cnt = np.zeros(len(cut))
    for ox in off:
        dx2 = (x[cut[:, 0]] + ox) ** 2
        for oy in off:
            dxy = dx2 + (x[cut[:, 1]] + oy) ** 2
            for oz in off:
                cnt += (dxy + (x[cut[:, 2]] + oz) ** 2) < R * R
    frac[cut[:, 0], cut[:, 1], cut[:, 2]] = cnt / sub ** 3
    return eta_out + (eta_in - eta_out) * frac


def cell_radius(n: int, B: float) -> np.ndarray:
    c = (np.arange(n) + 0.5) * (B / n) - B / 2.0
    return np.sqrt(c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2)


# ---------------------------------------------------------------------------
# Models: right-hand side S(phi, eta), its derivative, and the flux b(phi)
# ---------------------------------------------------------------------------

def symmetron_model(a, lambda0, a_ssb):
    K = a * a / (2.0 * lambda0 ** 2)
    A = (a_ssb / a) ** 3

    def S(chi, eta):
        return K * ((A * eta - 1.0) * chi + chi ** 3)

    def dS(chi, eta):
        return K * (A * eta - 1.0 + 3.0 * chi ** 2)

    def root(eta):
        return np.sqrt(np.maximum(0.0, 1.0 - A * eta))

    return dict(S=S, dS=dS, b=lambda v: np.ones_like(v), db=lambda v: np.zeros_like(v),
                root=root)


def fofr_model(a, nexp, fR0_abs, omega_m, omega_l):
    Q = omega_m * H0 ** 2 / (a * fR0_abs)
    cL = 4.0 * omega_l / omega_m
    a3 = a ** 3

    def S(u, eta):
        return Q * (eta + cL * a3 - a3 * (1.0 + cL) * np.exp(-u / (nexp + 1.0)))

    def dS(u, eta):
        return Q * a3 * (1.0 + cL) * np.exp(-u / (nexp + 1.0)) / (nexp + 1.0)

    def root(eta):
        return -(nexp + 1.0) * np.log((eta / a3 + cL) / (1.0 + cL))

    return dict(S=S, dS=dS, b=np.exp, db=np.exp, root=root)


# ---------------------------------------------------------------------------
# Solver 1: scipy collocation
# ---------------------------------------------------------------------------

def solve_bvp_profile(model, R, B, delta, rmax, tol=1e-8, guess=None):
    """(1/r^2) d/dr (r^2 b(phi) dphi/dr) = S(phi, eta(r)) with y = (phi,
    r^2 b(phi) phi'), split at r = R (eta jumps there; phi and the flux are
    continuous).  guess: optional (r, phi) to start from (it selects the
    branch; the collocation solution is then the method's own).  Returns a
    callable profile phi(r)."""
    from scipy.integrate import solve_bvp

    eta_in, eta_out = tophat(R, B, delta)
    r0 = 1e-6 * R
    # piecewise problem on [r0, R] and [R, rmax] mapped onto s in [0, 1] each
    L1, L2 = R - r0, rmax - R

    def rhs(s, y):
        phi1, q1, phi2, q2 = y
        r1 = r0 + s * L1
        r2 = R + s * L2
        d1 = np.vstack([q1 / (r1 ** 2 * model["b"](phi1)), r1 ** 2 * model["S"](phi1, eta_in)]) * L1
        d2 = np.vstack([q2 / (r2 ** 2 * model["b"](phi2)), r2 ** 2 * model["S"](phi2, eta_out)]) * L2
        return np.vstack([d1, d2])

    root_out = float(model["root"](np.array(eta_out)))
    root_in = float(model["root"](np.array(eta_in)))

    def bc(ya, yb):
        return np.array([ya[1],                 # regular centre: flux 0
                         yb[0] - ya[2],         # phi continuous at R
                         yb[1] - ya[3],         # flux continuous at R
                         yb[2] - root_out])     # background at rmax

    s = np.linspace(0.0, 1.0, 2001)
    s = np.unique(np.concatenate([s, 1.0 - np.geomspace(1e-6, 1.0, 400), np.geomspace(1e-6, 1.0, 400)]))
    s = np.clip(s, 0.0, 1.0)
    s = np.unique(s)
    y0 = np.zeros((4, s.size))
    y0[0] = root_in
    y0[2] = root_out
    if guess is not None:
        gr, gp = guess
        r1, r2 = r0 + s * L1, R + s * L2
        y0[0] = np.interp(r1, gr, gp)
        y0[2] = np.interp(r2, gr, gp)
        gq = gr ** 2 * model["b"](gp) * np.gradient(gp, gr)
        y0[1] = np.interp(r1, gr, gq)
        y0[3] = np.interp(r2, gr, gq)
    sol = solve_bvp(rhs, bc, s, y0, tol=tol, max_nodes=2_000_000)
    if not sol.success:
        raise RuntimeError(f"solve_bvp: {sol.message}")

    def profile(r):
        r = np.asarray(r, dtype=float)
        out = np.empty_like(r)
        inside = r < R
        out[inside] = sol.sol(np.clip((r[inside] - r0) / L1, 0.0, 1.0))[0]
        out[~inside] = sol.sol(np.clip((r[~inside] - R) / L2, 0.0, 1.0))[2]
        return out

    return profile


# ---------------------------------------------------------------------------
# Solver 2: finite differences + Newton on a fine radial mesh
# ---------------------------------------------------------------------------

def solve_fd_profile(model, R, B, delta, rmax, m=20000, iters=200):
    """Cell-centred radial mesh (dr = rmax / m); flux form
    (r_{i+1/2}^2 b_{i+1/2} (phi_{i+1} - phi_i) - r_{i-1/2}^2 b_{i-1/2} (...)) /
    (r_i^2 dr^2) = S_i with b at faces the mean of the two cells, zero flux at
    r = 0 and phi = root(eta_out) beyond rmax.  Newton with a dense
    tridiagonal solve.  Returns (r, phi)."""
    from scipy.linalg import solve_banded

    eta_in, eta_out = tophat(R, B, delta)
    dr = rmax / m
    r = (np.arange(m) + 0.5) * dr
    # cell-averaged eta on the radial mesh (volume weights of the shell cut by R)
    lo, hi = r - dr / 2, r + dr / 2
    vin = np.clip(np.minimum(hi, R) ** 3 - lo ** 3, 0.0, None)
    frac = vin / (hi ** 3 - lo ** 3)
    eta = eta_out + (eta_in - eta_out) * frac
    phi = model["root"](eta).astype(float)
    ghost = float(model["root"](np.array(eta_out)))
    rf = np.arange(m + 1) * dr  # faces
    for _ in range(iters):
        pe = np.append(phi, ghost)
        bc_ = model["b"](pe)
        bf = 0.5 * (bc_[:-1] + bc_[1:])          # faces i+1/2, i = 0..m-1
        flux = rf[1:] ** 2 * bf * (pe[1:] - pe[:-1])  # through face i+1/2
        fin = np.concatenate([[0.0], flux[:-1]])       # through face i-1/2
        vol = r ** 2 * dr ** 2
        F = (flux - fin) / vol - model["S"](phi, eta)
        # Jacobian (tridiagonal): d flux_{i+1/2} / d phi_i, d phi_{i+1}
        dbi = 0.5 * model["db"](pe[:-1])
        dbn = 0.5 * model["db"](pe[1:])
        dflux_di = rf[1:] ** 2 * (dbi * (pe[1:] - pe[:-1]) - bf)
        dflux_dn = rf[1:] ** 2 * (dbn * (pe[1:] - pe[:-1]) + bf)
        diag = (dflux_di - np.concatenate([[0.0], dflux_dn[:-1]])) / vol - model["dS"](phi, eta)
        upper = dflux_dn[:-1] / vol[:-1]
        lower = -dflux_di[:-1] / vol[1:]   # row i+1, column i: face i+1/2
        ab = np.zeros((3, m))
        ab[0, 1:] = upper
        ab[1] = diag
        ab[2, :-1] = lower
        step = solve_banded((1, 1), ab, -F)
        phi = phi + step
        if np.max(np.abs(step)) < 1e-13 * (1.0 + np.max(np.abs(phi))):
            break
    else:
        raise RuntimeError("radial Newton did not converge")
    return r, phi
