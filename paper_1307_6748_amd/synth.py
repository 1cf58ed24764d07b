"""Seeded synthetic density fields for the scalar-field solve.

These stand in for the N-body density fields of the paper (CIC densities of
simulation particles, Sec. 5 and 6); no simulation data is used.  The module
holds only input generation (random numbers, FFT filtering, particle
sampling and cloud-in-cell deposit): none of the solver's arithmetic.  Both
the GPU library's tests and the CPU oracle's tests draw their inputs from
here.

Every generator returns ``eta``, the density in units of the mean (the
paper's eta of the symmetron equation and rho-tilde of the f(R) equation), as
a C-contiguous float64 array of shape (n, n, n) with index order [x][y][z].
"""
from __future__ import annotations

import hashlib

import numpy as np

RHO_CRIT = 2.775e11  # critical density, (Msun/h) / (Mpc/h)^3


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _kmag(n: int, box: float) -> np.ndarray:
    kx = np.fft.fftfreq(n, d=box / n) * 2.0 * np.pi
    kz = np.fft.rfftfreq(n, d=box / n) * 2.0 * np.pi
    return np.sqrt(kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2)


def gaussian_field(n: int, box: float, seed: int) -> np.ndarray:
    """Unit-variance Gaussian random field with power spectrum P(k) ~ k^-2.

    White noise from PCG64(seed) is filtered by 1/k in Fourier space (the
    k = 0 mode removed) and the result normalised to unit variance."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(w)
    del w
    k = _kmag(n, box)
    k[0, 0, 0] = 1.0
    wk /= k
    wk[0, 0, 0] = 0.0
    del k
    g = np.fft.irfftn(wk, s=(n, n, n), axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    return np.ascontiguousarray(g)


def lognormal(n: int, box: float, sigma_delta: float, seed: int) -> np.ndarray:
    """eta = exp(sigma_G G) / mean, sigma_G^2 = ln(1 + sigma_delta^2)."""
    sg = np.sqrt(np.log1p(sigma_delta ** 2))
    eta = np.exp(sg * gaussian_field(n, box, seed))
    eta /= eta.mean()
    return eta


def _nfw_radii(rng, count: int, c: float, r200: float) -> np.ndarray:
    """Radii drawn from an NFW mass profile truncated at r200 (inverse CDF)."""
    x = np.linspace(0.0, c, 4097)
    mu = np.log1p(x) - x / (1.0 + x)
    u = rng.random(count) * mu[-1]
    return np.interp(u, mu, x) * (r200 / c)


def nfw_density(n: int, box: float, count: int, seed: int, omega_m: float = 0.27,
                points_per_halo: int = 200_000) -> np.ndarray:
    """Density contrast rho_halo / rho_mean_m of `count` NFW haloes, CIC-deposited.

    Positions uniform in the box, log10 M uniform in [13, 15] (Msun/h),
    concentration uniform in [4, 10], truncated at R200 where
    M = (4 pi / 3) 200 rho_crit R200^3.  Each halo is sampled with
    `points_per_halo` equal-mass points at isotropic directions and deposited
    with periodic cloud-in-cell weights."""
    rng = np.random.default_rng(seed)
    h = box / n
    out = np.zeros((n, n, n))
    pos = rng.random((count, 3)) * box
    logm = rng.uniform(13.0, 15.0, count)
    conc = rng.uniform(4.0, 10.0, count)
    rho_m = omega_m * RHO_CRIT
    cell_vol = h ** 3
    for q in range(count):
        m = 10.0 ** logm[q]
        r200 = (3.0 * m / (4.0 * np.pi * 200.0 * RHO_CRIT)) ** (1.0 / 3.0)
        r = _nfw_radii(rng, points_per_halo, conc[q], r200)
        d = rng.standard_normal((points_per_halo, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        p = pos[q][None, :] + d * r[:, None]
        # CIC in a local sub-cube, then added to the periodic grid.
        s = p / h - 0.5
        base = np.floor(s).astype(np.int64)
        frac = s - base
        lo = base.min(axis=0)
        ext = base.max(axis=0) - lo + 2
        local = np.zeros(int(ext[0] * ext[1] * ext[2]))
        b = base - lo
        w = m / points_per_halo / cell_vol / rho_m
        for dx in (0, 1):
            wx = frac[:, 0] if dx else 1.0 - frac[:, 0]
            for dy in (0, 1):
                wy = frac[:, 1] if dy else 1.0 - frac[:, 1]
                for dz in (0, 1):
                    wz = frac[:, 2] if dz else 1.0 - frac[:, 2]
                    idx = ((b[:, 0] + dx) * ext[1] + (b[:, 1] + dy)) * ext[2] + (b[:, 2] + dz)
                    local += np.bincount(idx, weights=w * wx * wy * wz, minlength=local.size)
        local = local.reshape(tuple(int(e) for e in ext))
        ix = (np.arange(ext[0]) + lo[0]) % n
        iy = (np.arange(ext[1]) + lo[1]) % n
        iz = (np.arange(ext[2]) + lo[2]) % n
        # indices within one sub-cube are distinct (ext <= n), so += is safe
        out[np.ix_(ix, iy, iz)] += local
    return out


def lognormal_nfw(n: int, box: float, sigma_delta: float, seed_grf: int, haloes: int,
                  seed_haloes: int, omega_m: float = 0.27,
                  points_per_halo: int = 200_000) -> np.ndarray:
    """Lognormal background plus NFW haloes, renormalised to mean 1."""
    eta = lognormal(n, box, sigma_delta, seed_grf)
    if haloes > 0:
        eta += nfw_density(n, box, haloes, seed_haloes, omega_m, points_per_halo)
    eta /= eta.mean()
    return np.ascontiguousarray(eta)


def uniform(n: int, value: float) -> np.ndarray:
    return np.full((n, n, n), float(value))


def cell_centres(n: int, box: float) -> np.ndarray:
    return (np.arange(n) + 0.5) * (box / n)


def sine_mode(n: int, box: float, modes=(1, 2, 3)) -> np.ndarray:
    """Product of sines sin(2 pi m_d x_d / B) at cell centres."""
    x = cell_centres(n, box)
    sx = np.sin(2 * np.pi * modes[0] * x / box)
    sy = np.sin(2 * np.pi * modes[1] * x / box)
    sz = np.sin(2 * np.pi * modes[2] * x / box)
    return np.ascontiguousarray(sx[:, None, None] * sy[None, :, None] * sz[None, None, :])


def random_field(n: int, seed: int, scale: float = 1.0, offset: float = 0.0) -> np.ndarray:
    """Plain uniform random field (for operator and kernel tests)."""
    rng = np.random.default_rng(seed)
    return offset + scale * rng.random((n, n, n))


# Named workloads (sizes, boxes, seeds and density recipes).
def workload(name: str, n: int | None = None, points_per_halo: int = 200_000) -> dict:
    """Density field and metadata of a named workload.

    small_symmetron   32^3, box 64,  lognormal sigma_delta = 1, seed 1
    symmetron_256     256^3, box 256, lognormal sigma_delta = 3, seed 2
    fr_256            256^3, box 128, lognormal sigma_delta = 2 (seed 10) + 50 NFW (seed 11)
    large_512         512^3, box 256, lognormal sigma_delta = 2 (seed 20) + 400 NFW (seed 22)
    `n` overrides the grid size (the box is kept)."""
    if name == "small_symmetron":
        n = n or 32
        return dict(n=n, box=64.0, eta=lognormal(n, 64.0, 1.0, 1))
    if name == "symmetron_256":
        n = n or 256
        return dict(n=n, box=256.0, eta=lognormal(n, 256.0, 3.0, 2))
    if name == "fr_256":
        n = n or 256
        return dict(n=n, box=128.0,
                    eta=lognormal_nfw(n, 128.0, 2.0, 10, 50, 11, points_per_halo=points_per_halo))
    if name == "large_512":
        n = n or 512
        return dict(n=n, box=256.0,
                    eta=lognormal_nfw(n, 256.0, 2.0, 20, 400, 22,
                                      points_per_halo=points_per_halo))
    raise KeyError(name)
