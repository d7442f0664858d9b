"""The block-CG oracle's pins must catch plausible mistakes.

Each case copies oracle/block_cg.py, plants one mistake (a wrong sign, a
wrong operand, a dropped pass or shift, a missing transpose), loads the copy
as a module and runs the pins of test_oracle_block.py against it; at least
one pin must fail.  CPU only.
"""
import importlib.util
import os

import pytest

import oracle
import test_oracle_block as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "block_cg.py")

MUTANTS = {
    "x_update_sign": ("        X += P @ alpha\n", "        X -= P @ alpha\n"),
    "residual_uses_p": ("        R -= Q @ alpha\n", "        R -= P @ alpha\n"),
    "beta_sign": ("        beta = -beta\n", ""),
    "beta_wrong_operand": ("beta = _spd_solve(PQ, live, Q.T @ Z)", "beta = _spd_solve(PQ, live, P.T @ Z)"),
    "alpha_wrong_operand": ("alpha = _spd_solve(PQ, live, P.T @ R)", "alpha = _spd_solve(PQ, live, Q.T @ R)"),
    "jacobi_multiplies": ("        dinv = 1.0 / d\n", "        dinv = d\n"),
    "no_shift": ("cholesky_drop(G + shift * np.eye(s), 0.0)", "cholesky_drop(G, 0.0)"),
    "one_cholqr_pass": ("    for _ in range(2):\n        L, keep = cholesky_drop(Wk.T @ Wk, tau)",
                        "    for _ in range(0):\n        L, keep = cholesky_drop(Wk.T @ Wk, tau)"),
    "factor_not_transposed": ("np.linalg.solve(L[np.ix_(idx, idx)], np.eye(idx.size)).T\n",
                              "np.linalg.solve(L[np.ix_(idx, idx)], np.eye(idx.size))\n"),
    "cholesky_update_sign": ("A[k + 1:, k + 1:] -= np.outer", "A[k + 1:, k + 1:] += np.outer"),
    "cholesky_keeps_dependent": ("        if not (d > tau):\n            continue", "        if not (d > 0.0):\n            continue"),
    "no_column_scaling": ("    W0 = W * D\n", "    W0 = W\n"),
}

PINS = [
    pins.test_cholesky_drop_factors_the_kept_columns,
    pins.test_orth_ill_conditioned_and_rank_deficient,
    lambda: pins.test_one_column_is_the_single_vector_iteration("jacobi"),
    lambda: pins.test_matches_cholesky(40, 5, 1e4),
    pins.test_finite_termination,
    pins.test_block_conjugacy_and_residual_orthogonality,
    pins.test_fewer_block_iterations_than_single_on_the_fem_system,
    pins.test_rank_deficient_right_hand_sides,
]


def _load(src_text, tmp_path, name):
    path = tmp_path / f"{name}.py"
    path.write_text(src_text)
    spec = importlib.util.spec_from_file_location(f"oracle._mutant_{name}", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _pins_pass(mod, monkeypatch) -> bool:
    with monkeypatch.context() as m:
        m.setattr(pins, "bc", mod)
        for pin in PINS:
            try:
                pin()
            except Exception:
                return False
    return True


def test_unmutated_copy_passes(tmp_path, monkeypatch):
    assert _pins_pass(_load(open(SRC).read(), tmp_path, "clean"), monkeypatch)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mod = _load(src.replace(old, new), tmp_path, name)
    assert not _pins_pass(mod, monkeypatch), f"mutant {name} passed every pin"
