"""Planted mistakes in the oracle: each fails at least one pin.

Every case copies one oracle module's source, plants one plausible slip by
an exact text substitution (the original text must occur exactly once, so a
later edit of the oracle that removes it fails this test loudly rather than
silently testing nothing), executes the copy as a separate module and runs
the pin checks of `oracle_pins` on it.  The pins are trustworthy only if
each such slip makes at least one of them fail.
"""

from __future__ import annotations

import importlib
import sys
import types

import pytest

import oracle_pins


def _mutant(modname: str, old: str, new: str):
    real = importlib.import_module(f"oracle.{modname}")
    with open(real.__file__) as fh:
        src = fh.read()
    assert src.count(old) == 1, f"planted text not found exactly once in oracle/{modname}.py: {old!r}"
    name = f"oracle._mutant_{modname}"
    mod = types.ModuleType(name)
    mod.__package__ = "oracle"
    mod.__file__ = real.__file__
    sys.modules[name] = mod   # dataclasses look their module up while the class is built
    try:
        exec(compile(src.replace(old, new), real.__file__ + " (mutant)", "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


def _fails(check, mod) -> bool:
    try:
        check(mod)
    except AssertionError:
        return True
    return False


# (module, original text, planted text, pins expected to catch it)
MUTATIONS = {
    "mr_step_conjugated": (
        "sap", "wr = dom.per_domain_sum(np.sum(np.conj(w) * r, axis=(1, 2)))",
        "wr = dom.per_domain_sum(np.sum(w * np.conj(r), axis=(1, 2)))",
        [oracle_pins.check_mr_least_squares, oracle_pins.check_mr_orthogonal_monotone]),
    "mr_step_scaled": (
        "sap", "omega[nz] = wr[nz] / ww[nz]", "omega[nz] = 0.9 * wr[nz] / ww[nz]",
        [oracle_pins.check_mr_least_squares, oracle_pins.check_mr_orthogonal_monotone]),
    "mr_residual_not_updated": (
        "sap", "r_new = r - om * w\n", "r_new = r + 0 * om * w\n",
        [oracle_pins.check_mr_orthogonal_monotone]),
    "restart_keeps_recursive_residual": (
        "krylov", "        R = B - A(X)\n        nA += 1\n        P = R.copy()\n",
        "        nA += 1\n        P = R.copy()\n",
        [oracle_pins.check_restart]),
    "zeta_sign": (
        "krylov", "zeta = np.vdot(Z, T) / np.vdot(Z, Z)", "zeta = -np.vdot(Z, T) / np.vdot(Z, Z)",
        [oracle_pins.check_block_invariants]),
    "rtv_transposed": (
        "krylov", "RtV = Rt.conj().T @ V\n            alpha = _lu_solve(RtV, Rt.conj().T @ R)            # 4.4",
        "RtV = (Rt.conj().T @ V).T\n            alpha = _lu_solve(RtV, Rt.conj().T @ R)            # 4.4",
        [oracle_pins.check_block_invariants]),
    "projectors_swapped": (
        "dirac", "_PM, _PP = _gamma.projectors()", "_PP, _PM = _gamma.projectors()",
        [oracle_pins.check_free_field_plane_wave]),
    "backward_phase_not_conjugated": (
        "dirac", "bw[tuple(sl)] *= np.conj(ph)", "bw[tuple(sl)] *= ph",
        [oracle_pins.check_free_field_plane_wave, oracle_pins.check_gamma5_hermiticity]),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_fails_a_pin(name):
    modname, old, new, checks = MUTATIONS[name]
    mod = _mutant(modname, old, new)
    caught = [c.__name__ for c in checks if _fails(c, mod)]
    assert caught, f"planted mistake {name!r} passed every pin it was aimed at"


@pytest.mark.parametrize("modname", ["sap", "krylov", "dirac"])
def test_unmutated_copy_passes(modname):
    # the harness itself: an unmodified copy passes the same pins
    mod = _mutant(modname, "import numpy as np\n", "import numpy as np\n")
    checks = {
        "sap": [oracle_pins.check_mr_least_squares, oracle_pins.check_mr_orthogonal_monotone],
        "krylov": [oracle_pins.check_block_invariants, oracle_pins.check_restart],
        "dirac": [oracle_pins.check_free_field_plane_wave, oracle_pins.check_gamma5_hermiticity],
    }[modname]
    for c in checks:
        c(mod)
