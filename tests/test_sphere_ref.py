"""Pins of the radial references for the static top-hat sphere test (Sec.
5.1): two independent 1D solvers (collocation BVP and finite-difference
Newton) agree, the finite-difference one converges at second order, and a
sphere without a density jump gives the homogeneous root everywhere."""
import numpy as np
import pytest

from oracle import sphere_ref as SR


def test_tophat_has_unit_mean():
    R, B, delta = 3.0, 40.0, 5000.0
    ein, eout = SR.tophat(R, B, delta)
    vs = 4 * np.pi / 3 * R ** 3
    assert abs((ein * vs + eout * (B ** 3 - vs)) / B ** 3 - 1.0) < 1e-14
    assert abs((ein - eout) / eout - delta) < 1e-9 * delta
    eta = SR.grid_density(32, B, R, delta)
    assert abs(eta.mean() - 1.0) < 2e-2  # cell-averaged sphere on a coarse grid


@pytest.mark.parametrize("a", [1.0, 0.5])
def test_symmetron_two_solvers_agree(a):
    model = SR.symmetron_model(a, 1.0, 0.6)
    r, phi = SR.solve_fd_profile(model, 3.0, 40.0, 5000.0, 15.0, m=20000)
    prof = SR.solve_bvp_profile(model, 3.0, 40.0, 5000.0, 15.0, tol=1e-6, guess=(r, phi))
    sel = np.abs(r - 3.0) > 0.06
    assert np.max(np.abs(prof(r[sel]) - phi[sel])) < 2e-6
    # screened inside, the homogeneous root of the background far outside
    assert phi[0] < 1e-6
    assert abs(phi[-1] - model["root"](np.array(SR.tophat(3.0, 40.0, 5000.0)[1]))) < 1e-6


def test_fofr_fd_converges_to_the_bvp_at_second_order():
    model = SR.fofr_model(1.0, 1.0, 1e-6, 0.27, 0.73)
    R, B, rmax = 5.0, 100.0, 40.0
    r, u = SR.solve_fd_profile(model, R, B, 5000.0, rmax, m=20000)
    prof = SR.solve_bvp_profile(model, R, B, 5000.0, rmax, tol=1e-8, guess=(r, u))
    errs = []
    for m in (10000, 20000, 40000):
        r, u = SR.solve_fd_profile(model, R, B, 5000.0, rmax, m=m)
        sel = np.abs(r - R) > 0.1
        errs.append(np.max(np.abs(prof(r[sel]) - u[sel])))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_no_jump_gives_the_homogeneous_root():
    model = SR.symmetron_model(1.0, 1.0, 0.6)
    r, phi = SR.solve_fd_profile(model, 3.0, 40.0, 0.0, 15.0, m=2000)
    assert np.max(np.abs(phi - model["root"](np.array(1.0)))) < 1e-12
