"""The pins hold the oracle to the paper and to mathematics, not to itself: a plausible
mistake planted in a copy of the oracle (a dropped factor, a flipped sign, the wrong
mean, a wrong branch) must make the pin written against it fail.

Each case copies the oracle package to a temporary directory, changes one expression
there, and runs the named pin tests in a subprocess that imports the copy (the test
configuration puts AMRFLD_PLANTED_ORACLE ahead of the repository).  The unchanged copy
must pass the same pins.  The oracle itself is never modified."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = "tests/test_oracle_pins.py::"

# name: (file, expression as written, planted mistake, pins that must catch it)
CASES = {
    "fine-to-coarse factor 2/3 dropped": (
        "fld_oracle.py", "C = (2.0 / 3.0) * harmonic_mean(K[leaves[m]], Kc[nb[m]]) * coef",
        "C = harmonic_mean(K[leaves[m]], Kc[nb[m]]) * coef",
        [PINS + "test_two_level_rows_match_hand_derivation"]),
    "stored inflow with the wrong sign": (
        "fld_oracle.py", "b[m] += w * C * E[nb[m]] + (1.0 - w) * Fin",
        "b[m] += w * C * E[nb[m]] - (1.0 - w) * Fin",
        [PINS + "test_neumann_interfaces_conserve_dirichlet_drifts"]),
    "Robin weight missing from the diagonal": (
        "fld_oracle.py", "diag[m] += w * C\n", "diag[m] += C\n",
        [PINS + "test_two_level_rows_match_hand_derivation"]),
    "flux register without the 2/3 factor": (
        "fld_oracle.py", "C = (2.0 / 3.0) * harmonic_mean(K[s], Kc[c]) * coef",
        "C = harmonic_mean(K[s], Kc[c]) * coef",
        [PINS + "test_heat_pulse_neumann_conserves_over_steps"]),
    "arithmetic instead of harmonic face mean": (
        "fld_oracle.py", "out[nz] = (2.0 * a * b)[nz] / s[nz]", "out[nz] = (0.5 * s)[nz]",
        [PINS + "test_face_mean_exact_for_layered_diffusivity"]),
    "held box face at a full cell": (
        "fld_oracle.py", "return 2.0 * harmonic_mean(Ki, Kb) * coef", "return harmonic_mean(Ki, Kb) * coef",
        ["tests/test_equilibrium_oracle.py::test_linear_profile_is_a_fixed_point"]),
    "coarse neighbour at dx instead of 3 dx / 2 in the gradient": (
        "fld_oracle.py", "h[m] = 1.5 * L.dx", "h[m] = L.dx",
        [PINS + "test_gradient_exact_for_single_axis_linear_field_on_amr"]),
    "LP limiter denominator with R instead of R^2": (
        "fld_oracle.py", "return (2.0 + R) / (6.0 + 3.0 * R + R * R)", "return (2.0 + R) / (6.0 + 3.0 * R + R)",
        [PINS + "test_lp_limiter_values_and_limits"]),
    "LP diffusivity without kappa_R": (
        "fld_oracle.py", "return self.c * lam / (rho * self.kappa_R)", "return self.c * lam / rho",
        [PINS + "test_lp_diffusivity_is_c_over_3_rho_kappa_in_the_diffusion_limit"]),
    "Minerbo upper branch with sqrt(1 + R)": (
        "fld_oracle.py", "high = 1.0 / (1.0 + R + np.sqrt(1.0 + 2.0 * R))", "high = 1.0 / (1.0 + R + np.sqrt(1.0 + R))",
        ["tests/test_variants_oracle.py::test_minerbo_exact_values"]),
    "restriction from one child": (
        "fld_oracle.py", "child_E.mean(axis=1)", "child_E[:, 0]",
        [PINS + "test_restriction_of_linear_field_is_parent_centre_value"]),
    "coupling source weighted by f instead of 1 - f": (
        "fld_oracle.py", "b += eta * (1.0 - f) * self.a * T ** 4", "b += eta * f * self.a * T ** 4",
        [PINS + "test_coupling_uniform_cell_matches_linearised_two_equation_backward_euler"]),
    "PCG beta inverted": (
        "fld_oracle.py", "beta = rho_new / rho\n", "beta = rho / rho_new\n",
        [PINS + "test_pcg_matches_cholesky_within_certificate"]),
    "theta step with the weights swapped": (
        "fld_oracle.py", "b1 - (1.0 - self.theta) * (D @ En)", "b1 - self.theta * (D @ En)",
        ["tests/test_variants_oracle.py::test_theta_step_is_the_dct_closed_form"]),
    "composite finer-face coupling A/4 instead of A/3": (
        "fld_oracle.py", "* coef / 3.0", "* coef / 4.0",
        ["tests/test_composite_oracle.py::test_composite_interface_entries_hand_derived"]),
    "patch Robin inflow weighted by w": (
        "patch_oracle.py", "b[face] += w * Cb * ghosts[d] + (1.0 - w) * fluxes[d]",
        "b[face] += w * Cb * ghosts[d] + w * fluxes[d]",
        ["tests/test_patch_oracle.py::test_neumann_inflow_enters_exactly"]),
}


def _run_pins(tmp_path, fname, old, new, pins):
    planted = tmp_path / "planted"
    shutil.copytree(os.path.join(ROOT, "oracle"), planted / "oracle",
                    ignore=shutil.ignore_patterns("__pycache__"))
    if old is not None:
        f = planted / "oracle" / fname
        src = f.read_text()
        assert src.count(old) == 1, f"expression not found once in {fname}: {old!r}"
        f.write_text(src.replace(old, new))
    env = dict(os.environ, AMRFLD_PLANTED_ORACLE=str(planted), PYTHONDONTWRITEBYTECODE="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        "--timeout", "120"] + pins, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def test_unplanted_copy_passes_every_targeted_pin(tmp_path):
    pins = sorted({p for case in CASES.values() for p in case[3]})
    rc, out = _run_pins(tmp_path, None, None, None, pins)
    assert rc == 0, out


@pytest.mark.parametrize("name", list(CASES))
def test_planted_mistake_fails_its_pin(tmp_path, name):
    fname, old, new, pins = CASES[name]
    rc, out = _run_pins(tmp_path, fname, old, new, pins)
    assert rc == 1, f"{name}: pins {pins} did not fail (exit {rc})\n{out}"
