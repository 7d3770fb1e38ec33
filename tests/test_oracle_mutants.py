"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each mutant patches one plausible error into the oracle (a dropped term, a wrong
sign, a transposed operand) and runs the pin tests; at least one must fail.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synthnet
import oracle.model as om
import oracle.reduction as orr
import test_oracle_model as tm
import test_oracle_reduction as tr

PINS = [
    lambda: tm.test_lossless_line_closed_form(),
    lambda: tm.test_injections_match_complex_phasors(0),
    lambda: tm.test_first_derivatives_complex_step("syn9", synthnet.case9(1)),
    lambda: tm.test_hessian_complex_step_of_gradient("syn12", synthnet.small(12, 18, 4, seed=4)),
    lambda: tr.test_kcond_is_inverse_of_kaug_inverse_uu_block("syn12", tr.NETS[2][1], 0),
    lambda: tr.test_condensed_solve_equals_augmented_solve("syn12", tr.NETS[2][1], 0.0),
    lambda: tr.test_sensitivity_is_derivative_of_power_flow("syn12", tr.NETS[2][1]),
    lambda: tr.test_kcond_is_reduced_lagrangian_hessian("syn12", tr.NETS[2][1]),
]


def _caught():
    for pin in PINS:
        try:
            pin()
        except (AssertionError, RuntimeError, ValueError, np.linalg.LinAlgError):
            return True
    return False


def test_unmutated_oracle_passes_every_pin():
    assert not _caught()


def _phi_dp_sign(kind, G, B, t):
    p, dp, ddp = _ORIG_PHI(kind, G, B, t)
    return p, (-dp if kind == "c" else dp), ddp


def _phi_value_sign(kind, G, B, t):
    c, s = np.cos(t), np.sin(t)
    if kind == "d":
        return G * s + B * c, G * c - B * s, -G * s - B * c
    return _ORIG_PHI(kind, G, B, t)


def _phi_ddp_dropped(kind, G, B, t):
    p, dp, ddp = _ORIG_PHI(kind, G, B, t)
    return p, dp, 0.0 * ddp


_ORIG_PHI = om.Model._phi
_ORIG_BLOCKS = orr.kkt_blocks
_ORIG_RHS = orr.condensed_rhs


def _blocks_no_sigx(model, x, u, lam, y, sig_x, sig_u, sig_s):
    B = _ORIG_BLOCKS(model, x, u, lam, y, sig_x, sig_u, sig_s)
    import scipy.sparse as sp
    B["K"] = (B["K"] - sp.diags(np.concatenate([0.0 * np.asarray(sig_u),
                                                np.asarray(sig_x)]))).tocsr()
    return B


def _blocks_transposed_gram(model, x, u, lam, y, sig_x, sig_u, sig_s):
    B = _ORIG_BLOCKS(model, x, u, lam, y, sig_x, sig_u, sig_s)
    import scipy.sparse as sp
    W, A = B["W"], B["A"]
    # A Sigma A^T has the wrong shape; the plausible slip is Sigma applied twice
    B["K"] = (W + sp.diags(np.concatenate([sig_u, sig_x]))
              + A.T @ sp.diags(np.asarray(sig_s) ** 2) @ A).tocsr()
    return B


def _rhs_wrong_sign(blocks, r, S=None, lu=None):
    nu, nx, m = blocks["nu"], blocks["nx"], blocks["m"]
    r1, r2, r3, r4, r5 = orr.unpack(r, nu, nx, m)
    r = np.concatenate([r1, r2, -r3, r4, r5])
    return _ORIG_RHS(blocks, r, S, lu)


def _lu_solve_no_transpose(lu, b, trans=0, **kw):
    return _ORIG_LU_SOLVE(lu, b, trans=0, **kw)


_ORIG_LU_SOLVE = sla.lu_solve


MUTANTS = {
    "phi_first_derivative_sign": (om.Model, "_phi", staticmethod(_phi_dp_sign)),
    "phi_q_value_sign_of_B": (om.Model, "_phi", staticmethod(_phi_value_sign)),
    "phi_second_derivative_dropped": (om.Model, "_phi", staticmethod(_phi_ddp_dropped)),
    "sigma_x_dropped_from_K": (orr, "kkt_blocks", _blocks_no_sigx),
    "sigma_s_squared_in_gram": (orr, "kkt_blocks", _blocks_transposed_gram),
    "rhs_r3_sign": (orr, "condensed_rhs", _rhs_wrong_sign),
    "adjoint_solve_not_transposed": (orr.sla, "lu_solve", _lu_solve_no_transpose),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    obj, attr, repl = MUTANTS[name]
    monkeypatch.setattr(obj, attr, repl)
    # the pin modules imported kkt_blocks etc. through the module object, so a
    # module-level patch is seen by them
    assert _caught(), f"mutant {name} survived every pin"


def test_charging_not_halved_is_caught(monkeypatch):
    orig_init = om.Model.__init__

    def init(self, net):
        orig_init(self, net)
        z = np.asarray(net.r) + 1j * np.asarray(net.x)
        self.y_ff = 1.0 / z + 1.0j * np.asarray(net.b)   # full b at each end
    monkeypatch.setattr(om.Model, "__init__", init)
    assert _caught()


# ---------------------------------------------------------------- sensitivity
import oracle.sensitivity as osn
import test_oracle_sensitivity as ts

SENS_PINS = [
    lambda: ts.test_load_jacobian_matches_residual_differences("syn5"),
    lambda: ts.test_sensitivity_matches_differences_of_barrier_solution("syn5", 1e-3),
    lambda: ts.test_objective_gradient_is_envelope("syn5"),
]
_ORIG_FP = osn.load_jacobian
_ORIG_C = osn.output_jacobian


def _fp_no_cost_term(ipm, w, s):
    Fp = _ORIG_FP(ipm, w, s)
    o = osn.offsets(ipm)
    Fp[o[0]:o[2], ipm.M.ref] = 0.0
    return Fp


def _fp_qg_rows_negated(ipm, w, s):
    Fp = _ORIG_FP(ipm, w, s)
    o = osn.offsets(ipm)
    Fp[o[4] + 1:o[4] + 1 + ipm.M.ng, :] *= -1.0
    return Fp


def _c_pg_ref_sign(ipm, w, s):
    C = _ORIG_C(ipm, w, s)
    o = osn.offsets(ipm)
    C[:, o[2]] *= -1.0
    return C


SENS_MUTANTS = {
    "cost_term_of_pd_ref_dropped": _fp_no_cost_term,
    "qg_load_rows_negated": _fp_qg_rows_negated,
    "pg_ref_output_sign": _c_pg_ref_sign,
}


@pytest.mark.parametrize("name", sorted(SENS_MUTANTS))
def test_sensitivity_mutant_is_caught(name, monkeypatch):
    attr = "load_jacobian" if name != "pg_ref_output_sign" else "output_jacobian"
    monkeypatch.setattr(osn, attr, SENS_MUTANTS[name])
    caught = False
    for pin in SENS_PINS:
        try:
            pin()
        except (AssertionError, np.linalg.LinAlgError):
            caught = True
            break
    assert caught, f"mutant {name} survived every pin"


def test_unmutated_sensitivity_passes_its_pins():
    for pin in SENS_PINS:
        pin()


# --------------------------------------------------------------------- RedLin
import oracle.redlin as orl
import test_oracle_redlin as trl

REDLIN_PINS = [
    lambda: trl.test_reduced_derivatives_match_differences("syn5"),
    lambda: trl.test_reduced_step_equals_condensed_forms("syn5"),
    lambda: trl.test_redlin_reaches_linred_optimum("syn5"),
]
_ORIG_DERIV = orl.RedLinIPM.derivatives


def _deriv_no_state_rows(self, u, x, y):
    D = _ORIG_DERIV(self, u, x, y)
    D["A_hat"] = D["A_hat"].copy()
    D["A_hat"][self.m:] = 0.0
    return D


def _deriv_adjoint_yx_sign(self, u, x, y):
    y2 = y.copy()
    y2[self.m:] *= -1.0
    D = _ORIG_DERIV(self, u, x, y2)
    D2 = _ORIG_DERIV(self, u, x, y)
    D2["lam"], D2["grad_lr"], D2["W_hat"] = D["lam"], D["grad_lr"], D["W_hat"]
    return D2


@pytest.mark.parametrize("name,fn", [("state_rows_dropped_from_A_hat", _deriv_no_state_rows),
                                     ("adjoint_state_multiplier_sign", _deriv_adjoint_yx_sign)])
def test_redlin_mutant_is_caught(name, fn, monkeypatch):
    monkeypatch.setattr(orl.RedLinIPM, "derivatives", fn)
    caught = False
    for pin in REDLIN_PINS:
        try:
            pin()
        except (AssertionError, RuntimeError, np.linalg.LinAlgError):
            caught = True
            break
    assert caught, f"mutant {name} survived every pin"
