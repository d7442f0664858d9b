import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


UNIT_ROUNDOFF = 2.0 ** -53


def tol_recomputed(n: int, tol: float = 1e-10) -> float:
    """Bound for a true relative residual that a test recomputes on the CPU.

    The GPU's products sum every row in stored order from separately rounded
    products, bitwise the CPU's sequential product (tested), so both sides
    form the same b_i - (A x)_i.  Only the two sums of n squares (||r||^2 and
    ||b||^2) run in other orders: each has relative error at most
    gamma_n = n u / (1 - n u), the square roots and the division add a few u.
    A solve whose own test passed at tol therefore recomputes to at most
    tol (1 + 2 gamma_n)(1 + 4 u) on the CPU.
    """
    u = UNIT_ROUNDOFF
    g = n * u / (1.0 - n * u)
    return tol * (1.0 + 2.0 * g) * (1.0 + 4.0 * u)


def mean_removed_relerr(x, xo) -> float:
    """||(x - mean x) - (xo - mean xo)|| / ||xo - mean xo||.

    The solutions of these Neumann-plus-small-mass systems are dominated by the
    constant mode (1'b / c per entry, with c = 1e-3), so a normwise error
    ||x - xo|| / ||xo|| barely sees the part of x that varies in space; this
    error measures that part alone.
    """
    import numpy as np

    x = np.asarray(x, dtype=np.float64)
    xo = np.asarray(xo, dtype=np.float64)
    d = xo - xo.mean()
    nd = np.linalg.norm(d)
    return float(np.linalg.norm((x - x.mean()) - d) / nd) if nd > 0 else float(np.linalg.norm(x - x.mean()))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def gpu_available() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def cuda():
    """The HIP device; GPU tests fail loudly (not skip) when the library is missing."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1107_0538_amd import capi

    capi.load()  # raises if the HIP library is not built
    return torch.device("cuda:0")
