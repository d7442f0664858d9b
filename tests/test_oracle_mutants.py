"""The oracle's pins must catch plausible mistakes.

Each case copies the oracle source, plants one mistake (a wrong sign, a
dropped term, a transposed operand, a wrong index, an off-by-one), compiles it
on the CPU, and checks that at least one pin rejects the mutant.  Nothing here
touches the GPU library.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import workloads as W

MUTANTS = {
    "spmv_wrong_index": ("val[k] * x[col[k]]", "val[k] * x[i]"),
    "spmv_drops_last_entry": ("k < rowptr[i + 1]; ++k) s +=", "k < rowptr[i + 1] - 1; ++k) s +="),
    "residual_sign": ("r[i] = r[i] - alpha * q[i]", "r[i] = r[i] + alpha * q[i]"),
    "x_update_sign": ("x[i] = x[i] + alpha * p[i]", "x[i] = x[i] - alpha * p[i]"),
    "alpha_inverted": ("alpha = rho / sigma", "alpha = sigma / rho"),
    "beta_inverted": ("beta = rho_new / rho", "beta = rho / rho_new"),
    "direction_drops_beta": ("p[i] = z[i] + beta * p[i]", "p[i] = z[i]"),
    "jacobi_multiplies": ("z[i] = r[i] / diag[i];\n        double rho_new", "z[i] = r[i] * diag[i];\n        double rho_new"),
    "initial_residual_sign": ("for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];\n    double rn",
                              "for (int i = 0; i < n; ++i) r[i] = r[i] - b[i];\n    double rn"),
    "norm_without_sqrt": ("rn = sqrt(oracle_dot(n, r, r, sum_mode));\n        if (hist)",
                          "rn = (oracle_dot(n, r, r, sum_mode));\n        if (hist)"),
    "p_dot_wrong_operand": ("sigma = oracle_dot(n, p, q, sum_mode)", "sigma = oracle_dot(n, q, q, sum_mode)"),
    # the single-reduction form
    "sr_sigma_wrong_vector": ("sigma = oracle_dot(n, p, sv, sum_mode);             /* sigma = p's */",
                              "sigma = oracle_dot(n, p, w, sum_mode);             /* sigma = p's */"),
    # Chronopoulos and Gear's scalar recurrence for p'Ap in place of p's: it
    # loses its sign after replacements near the attainable accuracy.
    "sr_sigma_scalar_recurrence": (
        "        }\n        sigma = oracle_dot(n, p, sv, sum_mode);             /* sigma = p's */",
        "            sigma = oracle_dot(n, w, u, sum_mode) - beta * gamma / alpha;\n            goto next;\n"
        "        }\n        sigma = oracle_dot(n, p, sv, sum_mode);\n    next:"),
    "sr_s_drops_beta": ("sv[i] = w[i] + beta * sv[i]", "sv[i] = w[i]"),
    "sr_residual_uses_w": ("r[i] = r[i] - alpha * sv[i]", "r[i] = r[i] - alpha * w[i]"),
    "sr_product_of_r": ("oracle_spmv(n, rowptr, col, val, u, w);             /* w = A u */",
                        "oracle_spmv(n, rowptr, col, val, r, w);             /* w = A u */"),
    "sr_gamma_stale": ("        gamma = gamma_new;\n", "        gamma = gamma;\n"),
    "sr_replacement_s_of_u": ("oracle_spmv(n, rowptr, col, val, p, sv);        /* s = A p, recomputed */",
                              "oracle_spmv(n, rowptr, col, val, u, sv);        /* s = A p, recomputed */"),
}

SINGLE_FORM = {k for k in MUTANTS if k.startswith("sr_")}


def _pins_pass(form: str = "standard") -> bool:
    """A compact subset of the oracle pins; True when every one holds."""
    try:
        rng = np.random.default_rng(0)
        a, b = W.problem(6, 1)
        d = a.to_dense()
        x = rng.standard_normal(a.n)
        if np.max(np.abs(oracle.spmv(a, x) - d @ x)) > 1e-12:
            return False
        xc = sla.cho_solve(sla.cho_factor(d), b)
        xs, info = oracle.pcg(a, b, tol=1e-10, form=form)
        if info["status"] != oracle.CONVERGED or np.linalg.norm(xs - xc) > 1e-6 * np.linalg.norm(xc):
            return False
        if np.linalg.norm(b - d @ xs) > 1e-10 * np.linalg.norm(b) * 1.0001:
            return False
        xs, info, hist, tr = oracle.pcg(a, b, tol=1e-10, history=True, trace=True, form=form)
        nb = np.linalg.norm(b)
        for k in range(6):
            if abs(hist[k] - np.linalg.norm(b - d @ tr[k, 0]) / nb) > 1e-10 * hist[0]:
                return False
        P = tr[:, 3]
        for i in range(1, 6):
            pap = P[i] @ d @ P[0] / np.sqrt((P[i] @ d @ P[i]) * (P[0] @ d @ P[0]))
            if not abs(pap) < 1e-8:
                return False
        n = 30
        u = rng.standard_normal(n)
        x, info = oracle.pcg(
            W.CSR(n, np.arange(0, n * n + 1, n, dtype=np.int32), np.tile(np.arange(n, dtype=np.int32), n),
                  (np.eye(n) + np.outer(u, u)).ravel()),
            rng.standard_normal(n), tol=1e-12, precond="none", form=form)
        if not (info["status"] == oracle.CONVERGED and info["iters"] == 2):
            return False
        if form == "single":
            # Systems that need residual replacements near the attainable
            # accuracy: the single-reduction form must converge alongside the
            # standard one (right-hand sides 20-29 include ones on which a
            # scalar recurrence for p'Ap loses its sign).
            a, _ = W.problem(16, 0)
            fam = W.amplitude_family(n=16, count=30)
            for b in fam.rhs(np.arange(20, 30)):
                _, i_s = oracle.pcg(a, b)
                _, i_r = oracle.pcg(a, b, form="single")
                if i_r["status"] != oracle.CONVERGED or abs(i_r["iters"] - i_s["iters"]) > 2:
                    return False
        return True
    except Exception:
        return False


@pytest.fixture
def swap_lib():
    saved = oracle._lib
    yield
    oracle._lib = saved


def _load_variant(src_text, tmp):
    import ctypes

    c = os.path.join(tmp, "m.c")
    so = os.path.join(tmp, "m.so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", c, "-o", so, "-lm"],
                   check=True)
    oracle._lib = None
    saved = oracle.LIB
    oracle.LIB = so
    try:
        oracle.lib()
    finally:
        oracle.LIB = saved


def test_unmutated_copy_passes(swap_lib):
    with open(oracle.SRC) as f:
        src = f.read()
    with tempfile.TemporaryDirectory() as tmp:
        _load_variant(src, tmp)
        assert _pins_pass("standard") and _pins_pass("single")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, swap_lib):
    with open(oracle.SRC) as f:
        src = f.read()
    old, new = MUTANTS[name]
    # Sites shared by both forms are mutated at their first occurrence, which is
    # in the standard form -- the form whose pins are then run.
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    if name in SINGLE_FORM:
        assert src.count(old) == 1, f"mutation site for {name} not unique"
    with tempfile.TemporaryDirectory() as tmp:
        _load_variant(src.replace(old, new, 1), tmp)
        form = "single" if name in SINGLE_FORM else "standard"
        assert not _pins_pass(form), f"pins did not catch {name}"
