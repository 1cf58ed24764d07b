"""Pins of the oracle's coefficient-weighted prolongation (reading R2's option
for the flux-form operators, Sec. 3.4; orc_prolong_correct_w).

The weights are pinned by what they are meant to do, not by retyping them:
with a uniform coefficient they are the trilinear stencil, they sum to one,
and across a jump of b along one axis the interpolated correction keeps the
flux b de/dx continuous through the face between the two coarse cells.
"""
import numpy as np

from oracle import oracle as orc


def _rng(seed):
    return np.random.default_rng(seed)


def test_uniform_coefficient_is_trilinear():
    rng = _rng(1)
    for n in (4, 8, 12):
        fine = rng.standard_normal((n, n, n))
        coarse = rng.standard_normal((n // 2,) * 3)
        hat = np.full((n // 2,) * 3, 0.37)
        got = orc.prolong_correct_w(fine, coarse + hat, hat)
        ref = orc.prolong_correct(fine, coarse + hat, hat)
        assert np.array_equal(got, ref)


def test_weights_sum_to_one():
    """A uniform correction c reaches every fine cell as c."""
    rng = _rng(2)
    n = 12
    fine = np.zeros((n, n, n))
    hat = 3.0 * rng.standard_normal((n // 2,) * 3)
    got = orc.prolong_correct_w(fine, hat + 0.25, hat)
    assert np.max(np.abs(got - 0.25)) <= 1e-15


def _step_case(axis, n, bp_log, bn_log, seed):
    """hat = bp_log on coarse planes 0 .. n/4-1 along `axis`, bn_log on the
    rest; the correction varies along `axis` only."""
    rng = _rng(seed)
    nc = n // 2
    prof_hat = np.where(np.arange(nc) < nc // 2, bp_log, bn_log)
    prof_e = rng.standard_normal(nc)
    shape = [1, 1, 1]
    shape[axis] = nc
    hat = np.broadcast_to(prof_hat.reshape(shape), (nc,) * 3).copy()
    e = np.broadcast_to(prof_e.reshape(shape), (nc,) * 3).copy()
    got = orc.prolong_correct_w(np.zeros((n,) * 3), hat + e, hat)
    line = np.moveaxis(got, axis, 0)[:, 1, 2]  # any transverse cell: all equal
    return prof_hat, prof_e, line


def test_flux_continuity_across_a_coefficient_jump():
    """Fine cell 2I+1 sits a quarter coarse spacing from its parent I (in b_P)
    towards I+1 (in b_N).  With the correction linear in each segment, the
    flux from I to the fine centre, from the fine centre to the face between
    I and I+1 (both in b_P, a quarter spacing each) and from the face to the
    centre of I+1 (in b_N, half a spacing) must agree."""
    n = 16
    for axis in range(3):
        for lp, ln in ((0.0, 2.3), (1.5, -4.0), (-0.7, -0.7)):
            hat, e, line = _step_case(axis, n, lp, ln, 10 + axis)
            nc = n // 2
            for I in (nc // 2 - 1, nc - 1):       # both jumps (the second wraps)
                J = (I + 1) % nc
                bP, bN = np.exp(hat[I]), np.exp(hat[J])
                ef = line[2 * I + 1]
                e_face = 2.0 * ef - e[I]          # from the equal fluxes in b_P
                f_in = bP * (ef - e[I]) / 0.25
                f_out = bN * (e[J] - e_face) / 0.5
                assert abs(f_in - f_out) <= 1e-12 * (abs(f_in) + abs(f_out) + 1.0), (axis, lp, ln)
                # the same from the other side: fine cell 2J on J's side of the face
                ef2 = line[(2 * J) % n]
                e_face2 = 2.0 * ef2 - e[J]
                g_in = bN * (e[J] - ef2) / 0.25
                g_out = bP * (e_face2 - e[I]) / 0.5
                assert abs(g_in - g_out) <= 1e-12 * (abs(g_in) + abs(g_out) + 1.0), (axis, lp, ln)


def test_away_from_the_jump_the_weights_are_trilinear():
    n = 16
    hat, e, line = _step_case(0, n, 0.4, 2.9, 20)
    nc = n // 2
    for I in (1, 2, nc // 2 + 1, nc // 2 + 2):    # parent and neighbour share b
        assert abs(line[2 * I + 1] - (0.75 * e[I] + 0.25 * e[I + 1])) <= 1e-14
        assert abs(line[2 * I] - (0.75 * e[I] + 0.25 * e[I - 1])) <= 1e-14


def test_extreme_contrast_stays_finite():
    """b ratios beyond the double range: the weight on the other cell goes to
    0 (it is far less conductive) or 1/2, with no overflow."""
    n = 8
    hat, e, line = _step_case(1, n, 0.0, -900.0, 30)
    assert np.all(np.isfinite(line))
    nc = n // 2
    I = nc // 2 - 1
    assert abs(line[2 * I + 1] - e[I]) <= 1e-14 * (abs(e[I]) + 1.0)  # towards the tiny b: weight 0
    hat, e, line = _step_case(1, n, 0.0, 900.0, 31)
    assert abs(line[2 * I + 1] - 0.5 * (e[I] + e[I + 1])) <= 1e-14 * (abs(e).max() + 1.0)


def test_fofr_solve_with_weighted_prolongation_reaches_the_root():
    """The option changes only how fast the cycles converge, not the fixed
    point: an f(R) solve with it meets a tight tolerance and agrees with the
    trilinear solve's field."""
    from paper_1307_6748_amd import synth
    m = orc.Model(model=orc.FR_HS, a=1.0, n=1.0, fR0_abs=1e-5, omega_m=0.27, omega_l=0.73)
    n, box = 32, 16.0
    eta = synth.lognormal(n, box, 2.0, 5)
    rw = orc.solve(m, eta, box, tol=1e-12, cfg=orc.Cfg(max_cycles=60, prolong_w=True))
    rt = orc.solve(m, eta, box, tol=1e-12, cfg=orc.Cfg(max_cycles=60, prolong_w=False))
    assert rw.status == orc.OK and rt.status == orc.OK
    assert np.max(np.abs(rw.phi - rt.phi)) <= 1e-8 * (np.abs(rt.phi).max() + 1.0)


def test_two_full_weighting_cycles_then_the_mean():
    """restrict_fw = 2 (f(R)'s default with the weighted prolongation) is two
    V-cycles with full weighting followed by cycles with the 8-child mean:
    the same field, bit for bit, as the two runs chained by hand."""
    from paper_1307_6748_amd import synth
    m = orc.Model(model=orc.FR_HS, a=1.0, n=1.0, fR0_abs=1e-5, omega_m=0.27, omega_l=0.73)
    n, box = 16, 8.0
    eta = synth.lognormal(n, box, 1.5, 6)
    cold = orc.cold_start(m, eta)
    both = orc.vcycles(m, eta, box, cold, 5, cfg=orc.Cfg(restrict_fw=2, prolong_w=True))
    first = orc.vcycles(m, eta, box, cold, 2, cfg=orc.Cfg(restrict_fw=True, prolong_w=True))
    rest = orc.vcycles(m, eta, box, first.phi, 3, cfg=orc.Cfg(restrict_fw=False, prolong_w=True))
    assert np.array_equal(both.phi, rest.phi)
    assert not np.array_equal(both.phi, orc.vcycles(m, eta, box, cold, 5,
                                                    cfg=orc.Cfg(restrict_fw=True, prolong_w=True)).phi)
    assert orc.Cfg()._c(orc.FR_HS).restrict_fw == 2
    assert orc.Cfg(prolong_w=False)._c(orc.FR_HS).restrict_fw == 1
