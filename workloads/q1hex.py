"""Seeded synthetic finite-element systems that stand in for the paper's matrix.

The paper solves one SPD system from a finite-element model of an electrical
machine, stored in CSR with N = 132651 and NNZ = 3442951 (Section IV, and the
caption of Table I).  That matrix is not public.  This module builds a
structured stand-in with the same N and NNZ: a trilinear (Q1) hexahedral
discretisation of  -div(sigma grad u) + c u  on the unit cube with n nodes per
edge.  With no boundary rows removed, N = n**3 and the 27-point pattern gives
nnz = (3n - 2)**3, which at n = 51 equals the paper's N and NNZ exactly.

This module is input generation only.  It holds none of the solver's
arithmetic; both the oracle's tests and the GPU path's tests consume what it
returns.

Element matrices.  On a cube of side h the Q1 stiffness and mass entries
between two local nodes depend only on d, the number of coordinates in which
the two nodes differ (tensor products of the 1-D linear element):
    stiffness  h   * Khat(d),  Khat = (1/3, 0, -1/12, -1/12)
    mass       h^3 * Mhat(d),  Mhat(d) = (1/3)**(3-d) * (1/6)**d
An entry a_ij is the sum over the elements containing both nodes of
sigma_e * h * Khat(d) + c * h^3 * Mhat(d).  Each entry is formed once per
ordered pair, but the elements are always visited in ascending element
coordinates, so a_ij and a_ji are added in the same order and the matrix is
bitwise symmetric.

Node numbering: id = x + n*y + n*n*z (x fastest).  Element numbering: the
same with n-1 in place of n.  Randomness: numpy.random.default_rng(seed),
drawing the (n-1)**3 element log-coefficients first, then the right-hand side.
"""
from __future__ import annotations

import dataclasses

import numpy as np

KHAT = (1.0 / 3.0, 0.0, -1.0 / 12.0, -1.0 / 12.0)
MHAT = tuple((1.0 / 3.0) ** (3 - d) * (1.0 / 6.0) ** d for d in range(4))
MASS_COEF = 1e-3

# The 27 stencil offsets in ascending column order: dz outermost, dx innermost.
OFFSETS = tuple((dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1))


@dataclasses.dataclass
class CSR:
    """A square CSR matrix: int32 rowptr[n+1], int32 col[nnz], float64 val[nnz]."""

    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        for i in range(self.n):
            for k in range(self.rowptr[i], self.rowptr[i + 1]):
                a[i, self.col[k]] += self.val[k]
        return a


def pattern_size(n: int) -> tuple[int, int]:
    """(N, nnz) of the 27-point pattern on an n^3 grid with every node kept."""
    return n ** 3, (3 * n - 2) ** 3


def element_sigma(n: int, rng: np.random.Generator) -> np.ndarray:
    """sigma_e = exp(g_e), g_e ~ N(0,1) i.i.d., shape (n-1, n-1, n-1) as [ez, ey, ex]."""
    g = rng.standard_normal((n - 1) ** 3)
    return np.exp(g).reshape(n - 1, n - 1, n - 1)


def assemble(n: int, sigma: np.ndarray, c: float = MASS_COEF) -> CSR:
    """Assemble A = K_sigma + c*M on the n^3 grid (see the module docstring).

    sigma: element coefficients, shape (n-1, n-1, n-1) indexed [ez, ey, ex].
    """
    if n < 2:
        raise ValueError("need at least 2 nodes per edge")
    sigma = np.asarray(sigma, dtype=np.float64)
    if sigma.shape != (n - 1, n - 1, n - 1):
        raise ValueError("sigma must have shape (n-1, n-1, n-1)")
    h = 1.0 / (n - 1)
    # Pad so that element coordinate e maps to padded index e+1 and the
    # out-of-range coordinates -1 and n-1 read zero.
    sp = np.zeros((n + 1, n + 1, n + 1))
    sp[1:n, 1:n, 1:n] = sigma
    vp = np.zeros((n + 1, n + 1, n + 1))
    vp[1:n, 1:n, 1:n] = 1.0
    node = np.arange(n)

    def candidates(delta):
        # Padded element indices shared by node coordinate t and t + delta,
        # ascending in element coordinate.
        if delta == 0:
            return (node, node + 1)  # elements t-1 and t
        if delta == 1:
            return (node + 1,)  # element t
        return (node,)  # element t-1

    vals = np.empty((27, n, n, n))
    masks = np.empty((27, n, n, n), dtype=bool)
    inside = lambda d: (node + d >= 0) & (node + d < n)
    for o, (dz, dy, dx) in enumerate(OFFSETS):
        d = abs(dx) + abs(dy) + abs(dz)
        hk = h * KHAT[d]
        chm = c * h ** 3 * MHAT[d]
        acc = np.zeros((n, n, n))
        for iz in candidates(dz):
            for iy in candidates(dy):
                for ix in candidates(dx):
                    blk = np.ix_(iz, iy, ix)
                    acc = acc + (sp[blk] * hk + vp[blk] * chm)
        vals[o] = acc
        masks[o] = inside(dz)[:, None, None] & inside(dy)[None, :, None] & inside(dx)[None, None, :]
    # Row-major (node, offset) order gives rows in node order with ascending columns.
    vals = vals.reshape(27, -1).T
    masks = masks.reshape(27, -1).T
    ids = np.arange(n ** 3, dtype=np.int64)
    offs = np.array([dx + n * dy + n * n * dz for (dz, dy, dx) in OFFSETS], dtype=np.int64)
    counts = masks.sum(axis=1)
    rowptr = np.zeros(n ** 3 + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32")
    col = (ids[:, None] + offs[None, :])[masks].astype(np.int32)
    val = vals[masks]
    return CSR(n ** 3, rowptr.astype(np.int32), col, np.ascontiguousarray(val))


def q1hex(n: int, seed: int, c: float = MASS_COEF) -> tuple[CSR, np.random.Generator]:
    """The seeded sigma + mass system on an n^3 grid.

    Returns the matrix and the generator positioned after the sigma draw, so
    that the caller draws the right-hand side next.
    """
    rng = np.random.default_rng(seed)
    sigma = element_sigma(n, rng)
    return assemble(n, sigma, c), rng


def mass_matrix(n: int) -> CSR:
    """The consistent Q1 mass matrix on the unit cube (sigma = 0, c = 1)."""
    return assemble(n, np.zeros((n - 1, n - 1, n - 1)), 1.0)


def problem(n: int, seed: int = 0) -> tuple[CSR, np.ndarray]:
    """Matrix and right-hand side b ~ U[-1, 1]^N for one single-system workload."""
    a, rng = q1hex(n, seed)
    b = rng.uniform(-1.0, 1.0, a.n)
    return a, b


def batch_systems(count: int = 256, base_seed: int = 1000, lo: int = 12, hi: int = 48):
    """Independent systems of uneven size: system s draws n_s ~ U{lo..hi}, then sigma, then b."""
    out = []
    for s in range(count):
        rng = np.random.default_rng(base_seed + s)
        n = int(rng.integers(lo, hi + 1))
        a = assemble(n, element_sigma(n, rng))
        b = rng.uniform(-1.0, 1.0, a.n)
        out.append((n, a, b))
    return out


def multi_rhs(n_rows: int, s: int = 64, seed: int = 2) -> np.ndarray:
    """Row-major N x s block of right-hand sides, U[-1, 1]."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (n_rows, s))


def mass_1d(n: int) -> np.ndarray:
    """Dense 1-D linear-element mass matrix on [0, 1] with n nodes."""
    h = 1.0 / (n - 1)
    m = np.zeros((n, n))
    for e in range(n - 1):
        m[e, e] += h / 3.0
        m[e + 1, e + 1] += h / 3.0
        m[e, e + 1] += h / 6.0
        m[e + 1, e] += h / 6.0
    return m


def stiffness_1d(n: int) -> np.ndarray:
    """Dense 1-D linear-element stiffness matrix on [0, 1] with n nodes."""
    h = 1.0 / (n - 1)
    k = np.zeros((n, n))
    for e in range(n - 1):
        k[e, e] += 1.0 / h
        k[e + 1, e + 1] += 1.0 / h
        k[e, e + 1] -= 1.0 / h
        k[e + 1, e] -= 1.0 / h
    return k


@dataclasses.dataclass
class SourceFamily:
    """Right-hand sides made of Gaussian sources with fixed widths and amplitudes.

    Each right-hand side places `k` sources at centres theta (k x 3 in
    [0, 1]^3); f(p) = sum_k a_k exp(-|p - c_k|^2 / (2 w_k^2)) at the nodes and
    b = M f with the consistent Q1 mass matrix.  The widths w_k and amplitudes
    a_k are drawn once for the family and held fixed, so that the solution is
    a function of the centres alone.
    """

    n: int
    widths: np.ndarray
    amps: np.ndarray
    centres: np.ndarray  # (count, k, 3) as (x, y, z)

    @property
    def count(self) -> int:
        return self.centres.shape[0]

    def theta(self) -> np.ndarray:
        """Network inputs: the flattened centres, (count, 3k)."""
        return self.centres.reshape(self.count, -1).copy()

    def rhs(self, idx) -> np.ndarray:
        """Row-major (len(idx), N) block of right-hand sides b = M f.

        The Gaussian and the Q1 mass matrix both factor over the three axes
        (M = M1 (x) M1 (x) M1 on a tensor grid), so each source contributes the
        outer product of three 1-D vectors M1 g_axis.
        """
        idx = np.atleast_1d(np.asarray(idx))
        n = self.n
        t = np.linspace(0.0, 1.0, n)
        m1 = mass_1d(n)
        out = np.zeros((len(idx), n, n, n))
        for row, s in enumerate(idx):
            for k in range(self.widths.size):
                cx, cy, cz = self.centres[s, k]
                w2 = 2.0 * self.widths[k] ** 2
                gx = m1 @ np.exp(-((t - cx) ** 2) / w2)
                gy = m1 @ np.exp(-((t - cy) ** 2) / w2)
                gz = m1 @ np.exp(-((t - cz) ** 2) / w2)
                out[row] += self.amps[k] * (gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
        return out.reshape(len(idx), n ** 3)

    def source_field(self, s: int) -> np.ndarray:
        """f at the nodes for right-hand side s (used to pin rhs() against M f)."""
        n = self.n
        t = np.linspace(0.0, 1.0, n)
        z, y, x = np.meshgrid(t, t, t, indexing="ij")
        f = np.zeros((n, n, n))
        for k in range(self.widths.size):
            cx, cy, cz = self.centres[s, k]
            r2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
            f += self.amps[k] * np.exp(-r2 / (2.0 * self.widths[k] ** 2))
        return f.reshape(-1)


def source_family(n: int = 51, count: int = 2000, k: int = 8, seed: int = 3) -> SourceFamily:
    """Widths U[.02, .1] and amplitudes N(0, 1) first, then count x k centres U[0, 1]^3."""
    rng = np.random.default_rng(seed)
    widths = rng.uniform(0.02, 0.1, k)
    amps = rng.standard_normal(k)
    centres = rng.uniform(0.0, 1.0, (count, k, 3))
    return SourceFamily(n, widths, amps, centres)


@dataclasses.dataclass
class AmplitudeFamily:
    """Right-hand sides b = sum_k theta_k M g_k with k fixed Gaussian sources g_k.

    The solutions span exactly k directions and depend linearly on theta
    (the network input, U[0, 1]^k).  Their large smooth part makes the
    recurrence residual drift from the true one, so most solves need one or
    two residual replacements at tol = 1e-10.
    """

    base: SourceFamily
    amps: np.ndarray  # (count, k)

    @property
    def count(self) -> int:
        return self.amps.shape[0]

    def theta(self) -> np.ndarray:
        return self.amps.copy()

    def rhs(self, idx) -> np.ndarray:
        idx = np.atleast_1d(np.asarray(idx))
        k = self.base.widths.size
        basis = np.stack([dataclasses.replace(self.base, amps=np.eye(k)[j]).rhs(0)[0] for j in range(k)])
        return self.amps[idx] @ basis


def amplitude_family(n: int = 16, count: int = 400, k: int = 4, seed: int = 11) -> AmplitudeFamily:
    """k sources drawn as in source_family (count 1, seed), amplitudes U[0, 1] with seed + 1."""
    base = source_family(n=n, count=1, k=k, seed=seed)
    return AmplitudeFamily(base, np.random.default_rng(seed + 1).uniform(0.0, 1.0, (count, k)))
