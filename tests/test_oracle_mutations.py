"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a temporary copy of the oracle's C source
(never in the oracle itself), builds it, and runs the pin suite against that
build in a subprocess.  The suite must fail for every planted mistake.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "isis_oracle.c")

MUTATIONS = {
    "jacobian_half_dropped": ("dflux += 0.5 * bc * (nb[f] - p) - bf;",
                              "dflux += bc * (nb[f] - p) - bf;"),
    "face_average_half_dropped": ("double bf = 0.5 * (bc + exp(nb[f]));",
                                  "double bf = (bc + exp(nb[f]));"),
    "flux_missing_inv_h2": ("return flux * ih2 - S;", "return flux - S;", 0),
    "symmetron_cubic_sign": ("*S = K * (A * eta * chi - chi + chi * chi * chi);",
                             "*S = K * (A * eta * chi - chi - chi * chi * chi);"),
    "symmetron_K_missing_a2": ("double K = m->a * m->a / (2.0 * m->lambda0 * m->lambda0);",
                               "double K = 1.0 / (2.0 * m->lambda0 * m->lambda0);"),
    "fr_cL_inverted": ("    double cL = 4.0 * m->omega_l / m->omega_m;\n    double a3",
                       "    double cL = 4.0 * m->omega_m / m->omega_l;\n    double a3"),
    "restriction_weight": ("coarse[cidx(nc, I, J, K)] = s / 8.0;",
                           "coarse[cidx(nc, I, J, K)] = s / 7.0;"),
    "prolongation_weights_swapped": ("const double w[2] = {0.75, 0.25};",
                                     "const double w[2] = {0.25, 0.75};"),
    "prolongation_no_phihat": ("(coarse[q] - coarse_hat[q])", "(coarse[q])", 0),
    # the coefficient-weighted prolongation
    "prolongation_w_no_phihat": ("(coarse[q] - coarse_hat[q])", "(coarse[q])", 1),
    "prolongation_w_sign": ("w[ax][1] = 1.0 / (2.0 * (1.0 + exp(up - un[ax])));",
                            "w[ax][1] = 1.0 / (2.0 * (1.0 + exp(un[ax] - up)));"),
    "prolongation_w_half_dropped": ("w[ax][1] = 1.0 / (2.0 * (1.0 + exp(up - un[ax])));",
                                    "w[ax][1] = 1.0 / (1.0 + exp(up - un[ax]));"),
    "prolongation_w_axis": ("coarse_hat[cidx(nc, I[0], J[1], K[0])],",
                            "coarse_hat[cidx(nc, I[0], J[0], K[1])],"),
    "fas_sigma_sign": ("c->sigma[q] -= c->work[q];", "c->sigma[q] += c->work[q];"),
    "laplacian_wrong_diagonal": ("double lap = (sum - 6.0 * p) * ih2;",
                                 "double lap = (sum - 5.0 * p) * ih2;", 0),
    "neighbour_index": ("nb[3] = phi[cidx(n, i, wrap(j + 1, n), k)];",
                        "nb[3] = phi[cidx(n, i, wrap(j - 1, n), k)];"),
    "force_difference_sign": ("return (f[cidx(n, ip, jp, kp)] - f[cidx(n, im, jm, km)]) / (2.0 * h);",
                              "return (f[cidx(n, im, jm, km)] - f[cidx(n, ip, jp, kp)]) / (2.0 * h);"),
    "force_fr_half_dropped": ("acc -= 0.5 * eup * cdiff(N, h, field, i, j, k, ax);",
                              "acc -= eup * cdiff(N, h, field, i, j, k, ax);"),
    "force_beta_not_squared": ("bl * bl /", "bl /"),
    "force_chi_tilde_missing_a": ("const double chit = m->a * field[c];",
                                  "const double chit = field[c];"),
    "force_axis_swap": ("if (ax == 1) { jp = wrap(j + 1, n); jm = wrap(j - 1, n); }",
                        "if (ax == 1) { kp = wrap(k + 1, n); km = wrap(k - 1, n); }"),
    "chameleon_exponent_missing_one": ("double e = exp(-(1.0 + m->cham_n) * psi);",
                                       "double e = exp(-m->cham_n * psi);"),
    "chameleon_potential_sign": ("*S = m->cham_alpha * eta - m->cham_mu * e;",
                                 "*S = m->cham_alpha * eta + m->cham_mu * e;"),
    "chameleon_derivative_factor": ("*dS = (1.0 + m->cham_n) * m->cham_mu * e;",
                                    "*dS = m->cham_mu * e;"),
    "chameleon_cold_start_exponent": (
        "phi[c] = log(m->cham_mu / (m->cham_alpha * eta[c])) / (1.0 + m->cham_n);",
        "phi[c] = log(m->cham_mu / (m->cham_alpha * eta[c]));"),
    "chameleon_canonical_laplacian_of_psi": (
        "if (m->model == ORC_FR_HS || m->model == ORC_CHAMELEON) {\n        /* Sec. 3.4",
        "if (m->model == ORC_FR_HS) {\n        /* Sec. 3.4"),
    "chameleon_step_unbounded": ("if (m->model == ORC_CHAMELEON) /* reading R15 */",
                                 "if (0) /* reading R15 */", 0),
    "rms_missing_sqrt": ("return sqrt(sumsq(nn, r) / (double)(nn * nn * nn));",
                         "return sumsq(nn, r) / (double)(nn * nn * nn);"),
    "rms_cell_count": ("return sqrt(sumsq(nn, r) / (double)(nn * nn * nn));",
                       "return sqrt(sumsq(nn, r) / (double)(nn * nn));"),
    "r_ref_not_normalised": ("double r_ref = orc_rms(n, lv[0].work);",
                             "double r_ref = sqrt(sumsq(n, lv[0].work));"),
    "full_weighting_weights": ("const double w[4] = {0.125, 0.375, 0.375, 0.125};",
                               "const double w[4] = {0.25, 0.25, 0.25, 0.25};"),
    "full_weighting_offset": ("fine[cidx(nf, wrap(2 * I - 1 + a, nf), wrap(2 * J - 1 + b, nf),",
                              "fine[cidx(nf, wrap(2 * I + a, nf), wrap(2 * J - 1 + b, nf),"),
    "full_weighting_not_used": ("    if (cfg->restrict_fw)\n        orc_restrict_fw(",
                                "    if (0)\n        orc_restrict_fw("),
    "amr_ghost_jacobian_dropped": (
        "            dflux += r[f] * (bf + 0.5 * bg * (v[f] - p)); /* ghost terms, Sec. 3.4.1 */\n",
        ""),
    "amr_canonical_ghost_jacobian_dropped": (
        "            *D = -6.0 * ih2 - fabs(dS) + g * ih2; /* reading R10 */",
        "            *D = -6.0 * ih2 - fabs(dS); /* reading R10 */"),
    "amr_int_ignored": ("const double uint_f = mask[q] > -1.0 ? u_pre[q] : u_int[q]; /* eq. bpsi */",
                        "const double uint_f = u_pre[q]; /* eq. bpsi */"),
    # the same mistakes in the masked operator and the masked half-sweep
    "amr_flux_missing_inv_h2": ("return flux * ih2 - S;", "return flux - S;", 1),
    "amr_laplacian_wrong_diagonal": ("double lap = (sum - 6.0 * p) * ih2;",
                                     "double lap = (sum - 5.0 * p) * ih2;", 1),
    "amr_chameleon_step_unbounded": ("if (m->model == ORC_CHAMELEON) /* reading R15 */",
                                     "if (0) /* reading R15 */", 1),
    "amr_ghost_sign": ("v[f] = uint_f + r[f] * (p - u_pre[c]); /* eq. ueq */",
                       "v[f] = uint_f - r[f] * (p - u_pre[c]); /* eq. ueq */"),
    "paper_u_a4_factor": ("- om * a * a * a * a * H2 * g * c * e +",
                          "- om * a * a * a * H2 * g * c * e +"),
    "paper_u_cold_shift_missing": ("if (m->paper_u) phi[c] += log(m->a * m->a * m->fR0_abs);",
                                   "if (m->paper_u) phi[c] += 0.0;"),
    "paper_u_force_factor": ("const double eup = m->paper_u ? exp(field[c])",
                             "const double eup = m->paper_u ? m->a * m->fR0_abs * exp(field[c])"),
}
PIN_FILES = ["test_oracle_pins.py", "test_oracle_force.py", "test_oracle_models.py",
             "test_oracle_newton.py", "test_oracle_amr.py", "test_oracle_prolong_w.py"]
# The pin file that catches a mutation runs first (the suite stops at its first
# failure); the other files follow, so every pin still gets its chance.
FIRST_FILE = {
    "force_": "test_oracle_force.py",
    "chameleon_": "test_oracle_models.py",
    "paper_u_": "test_oracle_models.py",
    "amr_": "test_oracle_amr.py",
    "prolongation_w_": "test_oracle_prolong_w.py",
}


def _pin_order(name):
    first = next((f for pre, f in FIRST_FILE.items() if name.startswith(pre)), PIN_FILES[0])
    return [first] + [f for f in PIN_FILES if f != first]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_fails_a_pin(tmp_path, name):
    from oracle import oracle as O
    old, new, *which = MUTATIONS[name]
    src = open(SRC).read()
    if which:  # a line that occurs in the uniform and the masked operator: one copy
        assert src.count(old) == 2, name
        at = src.index(old) if which[0] == 0 else src.index(old, src.index(old) + 1)
        src = src[:at] + new + src[at + len(old):]
    else:
        assert src.count(old) == 1, name
        src = src.replace(old, new)
    mut = tmp_path / "mutant.c"
    mut.write_text(src)
    so = str(tmp_path / "libmutant.so")
    O.build(force=True, src=str(mut), out=so)
    env = dict(os.environ, ORACLE_LIB=so, OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] +
                       [os.path.join(ROOT, "tests", f) for f in _pin_order(name)],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"{name}: pins did not fail\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout
