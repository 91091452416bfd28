"""Seeded synthetic test problems for the shifted pipelined CG hot path.

This module only *describes* problems: an SPD operator (a Dirichlet stencil
or an assembled CSR matrix), a right-hand side b, an initial guess x0 and, for
manufactured problems, the exact solution.  It holds none of the solver's
arithmetic; the few places that need A*x_true to form b use library
primitives (``scipy.ndimage.convolve`` for stencils, ``scipy.sparse`` for CSR).
Both the oracle and the HIP path consume exactly the arrays built here.

Operators follow the paper's problem statement: A is a real SPD n-by-n matrix
(Section 2.1).  Stencils are the unscaled second-order finite-difference
Laplacians with homogeneous Dirichlet boundaries on the interior grid,
lexicographic order with x fastest; an optional constant diagonal shift c
gives A = L + c I.

Workloads (all seeded with ``numpy.random.default_rng(seed)``):
  * ``poisson2d_manufactured`` -- 2-D 5-point, x_true = 1/sqrt(n), b = A x_true.
  * ``lapl200``                 -- the paper's 2-D 200x200 model problem with
                                   b_j = 1/sqrt(n) (Section 5.1, Table 1).
  * ``poisson3d``               -- 3-D 7-point, x_true ~ U(-1, 1), b = A x_true.
  * ``paper_parallel_workload`` -- 2-D 1000x1000 Poisson, b = A * 1, x0 = 0
                                   (the strong-scaling problem of Section 5.2).
  * ``anisotropic_csr``         -- 2-D cell-centred diffusion with log-normal
                                   coefficients and 100:1 x/y anisotropy.
  * ``banded_csr``              -- random banded diagonally dominant SPD CSR.
  * ``batch_rectangles``        -- a batch of shifted 2-D Poisson rectangles.
  * ``arrival_stream``          -- Poisson-process arrivals of mixed requests.
  * ``diag_distinct`` / ``dense_spd`` -- tiny problems for exactness checks.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Operator", "Problem", "stencil2d", "stencil3d", "csr_operator",
    "poisson2d_manufactured", "lapl200", "poisson3d", "paper_parallel_workload",
    "anisotropic_csr", "banded_csr", "batch_rectangles", "arrival_stream",
    "diag_distinct", "dense_spd", "to_scipy",
]


@dataclasses.dataclass
class Operator:
    """An SPD operator.

    kind: ``"2d5"``, ``"3d7"`` or ``"csr"``.
    Stencils: grid ``nx, ny, nz`` (nz = 1 in 2-D), row = (diag + shift) at the
    centre and ``off`` at every existing neighbour.
    CSR: ``row_ptr`` (int64), ``col`` (int32), ``val`` (float64).  When
    ``fp32_exact`` is set every value is exactly representable in binary32,
    so FP32 and FP64 storage describe the same matrix.
    """
    kind: str
    n: int
    nx: int = 0
    ny: int = 0
    nz: int = 1
    diag: float = 0.0
    off: float = -1.0
    shift: float = 0.0
    row_ptr: Optional[np.ndarray] = None
    col: Optional[np.ndarray] = None
    val: Optional[np.ndarray] = None
    fp32_exact: bool = False

    @property
    def nnz(self) -> int:
        if self.kind == "csr":
            return int(self.row_ptr[-1])
        # each interior grid edge couples two unknowns
        if self.kind == "2d5":
            edges = (self.nx - 1) * self.ny + self.nx * (self.ny - 1)
        else:
            nx, ny, nz = self.nx, self.ny, self.nz
            edges = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
        return self.n + 2 * edges


@dataclasses.dataclass
class Problem:
    name: str
    op: Operator
    b: np.ndarray
    x0: np.ndarray
    x_true: Optional[np.ndarray] = None
    jacobi: bool = False
    sigma: float = 0.0        # shift for p-CG-sh (closed-form spectrum midpoint)
    rtol: float = 1e-10
    max_iter: int = 1000
    seed: int = 0
    meta: dict = dataclasses.field(default_factory=dict)


# --------------------------------------------------------------- operators

def stencil2d(nx: int, ny: Optional[int] = None, shift: float = 0.0) -> Operator:
    ny = nx if ny is None else ny
    return Operator("2d5", nx * ny, nx, ny, 1, 4.0, -1.0, float(shift))


def stencil3d(nx: int, ny: Optional[int] = None, nz: Optional[int] = None) -> Operator:
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return Operator("3d7", nx * ny * nz, nx, ny, nz, 6.0, -1.0, 0.0)


def csr_operator(row_ptr, col, val, fp32_exact=False) -> Operator:
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    return Operator("csr", len(row_ptr) - 1, row_ptr=row_ptr,
                    col=np.ascontiguousarray(col, dtype=np.int32),
                    val=np.ascontiguousarray(val, dtype=np.float64),
                    fp32_exact=fp32_exact)


def _stencil_kernel(op: Operator) -> np.ndarray:
    c = op.diag + op.shift
    if op.kind == "2d5":
        k = np.zeros((3, 3))
        k[1, 1] = c
        k[0, 1] = k[2, 1] = k[1, 0] = k[1, 2] = op.off
        return k
    k = np.zeros((3, 3, 3))
    k[1, 1, 1] = c
    for ax in range(3):
        for d in (0, 2):
            idx = [1, 1, 1]
            idx[ax] = d
            k[tuple(idx)] = op.off
    return k


def _grid_shape(op: Operator):
    return (op.ny, op.nx) if op.kind == "2d5" else (op.nz, op.ny, op.nx)


def to_scipy(op: Operator):
    """The operator as a scipy.sparse CSR matrix (Kronecker-sum construction
    for stencils: L = sum_d I x ... x T_d x ... x I)."""
    import scipy.sparse as sp
    if op.kind == "csr":
        return sp.csr_matrix((op.val, op.col, op.row_ptr), shape=(op.n, op.n))

    def T(m):
        return sp.diags([np.full(m - 1, op.off), np.zeros(m), np.full(m - 1, op.off)], [-1, 0, 1])

    dims = [op.nx, op.ny] + ([op.nz] if op.kind == "3d7" else [])
    L = sp.csr_matrix((op.n, op.n))
    for d, m in enumerate(dims):
        mats = [sp.identity(k) for k in dims]
        mats[d] = T(m)
        # x fastest: kron ordered slowest ... fastest
        K = mats[-1]
        for M in reversed(mats[:-1]):
            K = sp.kron(K, M)
        L = L + K
    L = L + sp.identity(op.n) * (op.diag + op.shift)
    return sp.csr_matrix(L)


def _matvec(op: Operator, x: np.ndarray) -> np.ndarray:
    """A x via library primitives (used only to build right-hand sides)."""
    if op.kind == "csr":
        return to_scipy(op) @ x
    from scipy import ndimage
    g = x.reshape(_grid_shape(op))
    return ndimage.convolve(g, _stencil_kernel(op), mode="constant", cval=0.0).ravel()


# ----------------------------------------------------------------- problems

def poisson2d_manufactured(N: int = 100) -> Problem:
    """2-D Poisson N x N, x_true = 1/sqrt(n), b = A x_true, x0 = 0,
    sigma = 4 (midpoint of the spectrum, lambda_min + lambda_max = 8)."""
    op = stencil2d(N)
    xt = np.full(op.n, 1.0 / math.sqrt(op.n))
    return Problem(f"poisson2d_{N}", op, _matvec(op, xt), np.zeros(op.n), xt,
                   sigma=4.0, rtol=1e-12, max_iter=2000)


def lapl200() -> Problem:
    """The lapl200 benchmark: 2-D Laplacian on a 200 x 200 grid (n = 40,000),
    b_j = 1/sqrt(n), x0 = 0, no preconditioner, sigma* = 4, 500 iterations
    (Section 5.1 and Table 1)."""
    op = stencil2d(200)
    b = np.full(op.n, 1.0 / math.sqrt(op.n))
    return Problem("lapl200", op, b, np.zeros(op.n), None, sigma=4.0,
                   rtol=1e-30, max_iter=500)


def poisson3d(N: int = 256, seed: int = 0, jacobi: bool = True, ny: Optional[int] = None,
              nz: Optional[int] = None) -> Problem:
    """3-D Poisson N^3 (or N x ny x nz), x_true ~ U(-1, 1), b = A x_true,
    x0 = 0, Jacobi, sigma = 1 (midpoint of spec(A M^-1) for the constant
    diagonal 6)."""
    op = stencil3d(N, ny, nz)
    rng = np.random.default_rng(seed)
    xt = rng.uniform(-1.0, 1.0, op.n)
    name = f"poisson3d_{N}" if ny is None and nz is None else f"poisson3d_{op.nx}x{op.ny}x{op.nz}"
    return Problem(name, op, _matvec(op, xt), np.zeros(op.n), xt,
                   jacobi=jacobi, sigma=1.0 if jacobi else 6.0, rtol=1e-10,
                   max_iter=5000, seed=seed)


def paper_parallel_workload(N: int = 1000) -> Problem:
    """2-D Poisson 1000 x 1000 without preconditioner (Section 5.2); the
    right-hand side is b = A * ones with x0 = 0; recursive tolerance 1e-6."""
    op = stencil2d(N)
    ones = np.ones(op.n)
    return Problem(f"paper_poisson2d_{N}", op, _matvec(op, ones), np.zeros(op.n), ones,
                   sigma=4.0, rtol=1e-6, max_iter=2500)


def _round_up_f32(v: np.ndarray) -> np.ndarray:
    f = v.astype(np.float32)
    low = f.astype(np.float64) < v
    f[low] = np.nextafter(f[low], np.float32(np.inf))
    return f.astype(np.float64)


def anisotropic_csr(N: int = 1024, seed: int = 0, sigma_log: float = 2.0,
                    x_aniso: float = 100.0) -> Problem:
    """2-D cell-centred anisotropic diffusion on an N x N grid.

    Cell coefficients c ~ exp(Normal(0, sigma_log^2)); an interior face takes
    the harmonic mean of its two cells, a boundary face takes its cell's value;
    x-faces are multiplied by ``x_aniso``.  Off-diagonals are -face and are
    rounded to binary32; each diagonal is the sum of the row's face values
    (boundary faces included, i.e. Dirichlet), rounded up to binary32, so the
    stored matrix stays symmetric, weakly diagonally dominant with strict
    dominance on the boundary rows -- hence SPD -- and is exactly the same
    matrix in FP32 and FP64 storage.  x_true ~ U(-1, 1), b = A x_true, Jacobi.
    """
    rng = np.random.default_rng(seed)
    c = np.exp(rng.normal(0.0, sigma_log, size=(N, N)))  # [y, x]
    hx = 2.0 * c[:, :-1] * c[:, 1:] / (c[:, :-1] + c[:, 1:]) * x_aniso  # face between x and x+1
    hy = 2.0 * c[:-1, :] * c[1:, :] / (c[:-1, :] + c[1:, :])            # face between y and y+1
    hx = hx.astype(np.float32).astype(np.float64)
    hy = hy.astype(np.float32).astype(np.float64)
    bx = (c * x_aniso).astype(np.float32).astype(np.float64)  # boundary faces in x
    by = c.astype(np.float32).astype(np.float64)              # boundary faces in y

    diag = np.zeros((N, N))
    diag[:, :-1] += hx
    diag[:, 1:] += hx
    diag[:-1, :] += hy
    diag[1:, :] += hy
    diag[:, 0] += bx[:, 0]
    diag[:, -1] += bx[:, -1]
    diag[0, :] += by[0, :]
    diag[-1, :] += by[-1, :]
    diag = _round_up_f32(diag)

    n = N * N
    idx = np.arange(n).reshape(N, N)
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [diag.ravel()]
    # west / east
    rows += [idx[:, 1:].ravel(), idx[:, :-1].ravel()]
    cols += [idx[:, :-1].ravel(), idx[:, 1:].ravel()]
    vals += [-hx.ravel(), -hx.ravel()]
    # south / north
    rows += [idx[1:, :].ravel(), idx[:-1, :].ravel()]
    cols += [idx[:-1, :].ravel(), idx[1:, :].ravel()]
    vals += [-hy.ravel(), -hy.ravel()]
    import scipy.sparse as sp
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A.sort_indices()
    op = csr_operator(A.indptr, A.indices, A.data, fp32_exact=True)
    xt = rng.uniform(-1.0, 1.0, n)
    return Problem(f"aniso_csr_{N}", op, A @ xt, np.zeros(n), xt, jacobi=True, sigma=1.0,
                   rtol=1e-10, max_iter=20000, seed=seed)


def banded_csr(n: int, seed: int = 0, half_band: int = 64, nnz_min: int = 7, nnz_max: int = 27) -> Problem:
    """Random banded SPD CSR: each row gets an odd target nnz in [7, 27] made of
    symmetric off-diagonal pairs at random offsets within the half-bandwidth;
    an off-diagonal is -w_ij with w_ij ~ U(0, 1]; the diagonal is
    sum_j w_ij (1 + margin), margin ~ U(0.01, 0.1).  Values are rounded to
    binary32 (diagonal rounded up), Jacobi, sigma = 1, x_true ~ U(-1, 1)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    hb = max(1, min(half_band, n - 1))
    pairs_per_row = (rng.integers(nnz_min, nnz_max + 1, n) | 1) // 2  # odd nnz -> (nnz-1)/2 pairs
    # row i proposes k_i = (nnz_i - 1)/2 entries (i, i+d) to its right; symmetry
    # mirrors the proposals of the rows above, so a row holds 1 + k_i + mean(k)
    # entries on average (about 17 for nnz_i odd in [7, 27])
    k = pairs_per_row
    tot = int(k.sum())
    ri = np.repeat(np.arange(n), k)
    d = rng.integers(1, hb + 1, tot)
    cj = ri + d
    keep = cj < n
    ri, cj = ri[keep], cj[keep]
    w = rng.uniform(0.0, 1.0, ri.size)
    w = 1.0 - w  # (0, 1]
    U = sp.coo_matrix((w, (ri, cj)), shape=(n, n)).tocsr()  # duplicates summed
    U.data = U.data.astype(np.float32).astype(np.float64)
    S = U + U.T
    rowsum = np.asarray(S.sum(axis=1)).ravel()
    margin = rng.uniform(0.01, 0.1, n)
    diag = _round_up_f32(rowsum * (1.0 + margin) + (rowsum == 0))
    A = (-S + sp.diags(diag)).tocsr()
    A.sort_indices()
    op = csr_operator(A.indptr, A.indices, A.data, fp32_exact=True)
    xt = rng.uniform(-1.0, 1.0, n)
    return Problem(f"banded_csr_{n}", op, A @ xt, np.zeros(n), xt, jacobi=True, sigma=1.0,
                   rtol=1e-8, max_iter=20000, seed=seed)


def batch_rectangles(count: int = 512, seed: int = 0, side_min: int = 32, side_max: int = 256,
                     shift_max: float = 0.1) -> list:
    """A batch of shifted 2-D Poisson rectangles: N_x, N_y ~ U{side_min..side_max},
    A_k = L + c_k I with c_k ~ U(0, shift_max), b_k ~ U(-1, 1), x0 = 0, no
    preconditioner, sigma_k = 4 + c_k (spectrum midpoint), tolerance 1e-8."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nx, ny = (int(v) for v in rng.integers(side_min, side_max + 1, 2))
        c = float(rng.uniform(0.0, shift_max))
        op = stencil2d(nx, ny, shift=c)
        b = rng.uniform(-1.0, 1.0, op.n)
        out.append(Problem(f"rect_{k}_{nx}x{ny}", op, b, np.zeros(op.n), None,
                           sigma=4.0 + c, rtol=1e-8, max_iter=20000, seed=seed))
    return out


def arrival_stream(count: int, rate_hz: float, seed: int = 0, log10_min: float = 3.0,
                   log10_max: float = 7.0) -> list:
    """Poisson-process arrivals: exponential inter-arrival times at ``rate_hz``;
    size n = round(10^U(log10_min, log10_max)); half 3-D 7-point cubes of side
    round(n^(1/3)) with Jacobi, half random banded CSR; sigma = 1, tolerance
    1e-8.  Returns a list of (arrival_time_s, Problem)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, count))
    out = []
    for k in range(count):
        n = int(round(10 ** rng.uniform(log10_min, log10_max)))
        sub = int(rng.integers(0, 2**31 - 1))
        if rng.uniform() < 0.5:
            side = max(2, int(round(n ** (1.0 / 3.0))))
            p = poisson3d(side, seed=sub)
            p.rtol, p.max_iter = 1e-8, 20000
        else:
            p = banded_csr(n, seed=sub)
        p.name = f"req{k}_{p.name}"
        out.append((float(t[k]), p))
    return out


def diag_distinct(k: int, n: int = 64, seed: int = 0) -> Problem:
    """Diagonal CSR matrix whose n diagonal entries take exactly k distinct
    values {1, ..., k} (each at least once, random multiplicities), and b with
    every component nonzero.  Exact CG terminates in k iterations."""
    rng = np.random.default_rng(seed)
    vals = np.concatenate([np.arange(1, k + 1), rng.integers(1, k + 1, n - k)]).astype(np.float64)
    rng.shuffle(vals)
    op = csr_operator(np.arange(n + 1), np.arange(n, dtype=np.int32), vals)
    b = rng.uniform(0.5, 1.5, n) * rng.choice([-1.0, 1.0], n)
    return Problem(f"diag{k}", op, b, np.zeros(n), b / vals, sigma=(1.0 + k) / 2.0,
                   rtol=1e-30, max_iter=k, seed=seed)


def dense_spd(n: int, cond: float = 1e3, seed: int = 0, spread: str = "linear") -> Problem:
    """Random dense SPD matrix Q diag(ev) Q^T stored as CSR, random b; the
    eigenvalues ev run from 1 to ``cond``, evenly spaced (``spread="linear"``,
    like a Laplacian's) or log-spaced (``"log"``)."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    if spread == "log":
        ev = np.logspace(0.0, math.log10(cond), n)
    else:
        ev = np.linspace(1.0, cond, n)
    A = (Q * ev) @ Q.T
    A = 0.5 * (A + A.T)
    rp = np.arange(0, n * n + 1, n)
    col = np.tile(np.arange(n, dtype=np.int32), n)
    op = csr_operator(rp, col, A.ravel())
    b = rng.normal(size=n)
    return Problem(f"dense_spd_{n}", op, b, np.zeros(n), None,
                   sigma=0.5 * (ev[0] + ev[-1]), rtol=1e-14, max_iter=4 * n, seed=seed)
