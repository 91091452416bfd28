"""Local rounding-error propagation analysis of shifted pipelined CG.

TEST INFRASTRUCTURE, NOT PRODUCT CODE (part of the oracle package).

Section 3.2 couples the gaps of r, s, w and z in the 4x4 system
pi_{i+1} = P_i(sigma) pi_i + eps_i with the local propagation matrix
P_i(sigma) built from the iteration's alpha_i and beta_i.  The products
P_{j,i}(sigma) = P_i ... P_j (j <= i; the identity for j > i) propagate the
local error of iteration j to iteration i, and
psi_i(sigma) = max over 1 <= j <= i of the spectral norm of P_{j,i}(sigma)
is the quantity minimised over sigma to pick the shift a posteriori from the
alpha/beta history of a p-CG run (Section 5.1).

Section 4 gives the variable-shift analogue P_i(sigma_{i-1}, sigma_i).

Parity status: psi itself is pinned (hand-computed one- and two-step
products, the reduction at sigma = 0, and psi_500(sigma*) of Section 5.1 on
lapl200).  The selection rule's ``slack`` (select_shift) is a reading of
Section 5.1's warning against large shifts whose value 2 was chosen so the
rule returns the published sigma* on lapl200: the slack rule is parity
unpinned.
"""
from __future__ import annotations

import numpy as np


def propagation_matrix(alpha: float, beta: float, sigma: float) -> np.ndarray:
    """P_i(sigma) of Section 3.2 for one iteration's alpha_i, beta_i."""
    a, b, s = alpha, beta, sigma
    return np.array([
        [1.0, -a * b, -a, 0.0],
        [0.0, b, 1.0, 0.0],
        [0.0, -a * b * s, 1.0 - a * s, -a * b],
        [0.0, 0.0, 0.0, b],
    ])


def propagation_matrix_variable(alpha: float, beta: float, sigma_prev: float, sigma: float) -> np.ndarray:
    """P_i(sigma_{i-1}, sigma_i) of Section 4.2 (variable shift)."""
    a, b, sp, ds = alpha, beta, sigma_prev, sigma - sigma_prev
    return np.array([
        [1.0, -a * b, -a, 0.0],
        [0.0, b, 1.0, 0.0],
        [0.0, -a * b * sp, 1.0 - a * sp, -a * b],
        [0.0, -b * ds, -ds, b],
    ])


def psi(alphas, betas, sigma: float, i: int | None = None) -> float:
    """psi_i(sigma) = max_{1<=j<=i} ||P_i(sigma) ... P_j(sigma)||_2.

    ``alphas[k]``, ``betas[k]`` are alpha_k, beta_k of iteration k (k = 0, 1, ...).
    ``i`` defaults to the last recorded iteration.
    """
    alphas = np.asarray(alphas, dtype=np.float64)
    betas = np.asarray(betas, dtype=np.float64)
    if i is None:
        i = len(alphas) - 1
    Q = np.eye(4)
    best = 0.0
    for j in range(i, 0, -1):        # P_{j,i} = P_{j+1,i} P_j
        Q = Q @ propagation_matrix(alphas[j], betas[j], sigma)
        best = max(best, float(np.linalg.norm(Q, 2)))
    return best


def psi_variable(alphas, betas, sigma_schedule, i: int | None = None) -> float:
    """psi_i with the variable-shift matrices P_k(sigma_{k-1}, sigma_k);
    ``sigma_schedule`` holds sigma_{-1}, sigma_0, ... and its last entry
    repeats."""
    alphas = np.asarray(alphas, dtype=np.float64)
    betas = np.asarray(betas, dtype=np.float64)
    sched = np.asarray(sigma_schedule, dtype=np.float64)
    if i is None:
        i = len(alphas) - 1

    def sig(k):  # sigma_k, k >= -1
        return sched[min(k + 1, len(sched) - 1)]

    Q = np.eye(4)
    best = 0.0
    for j in range(i, 0, -1):
        Q = Q @ propagation_matrix_variable(alphas[j], betas[j], sig(j - 1), sig(j))
        best = max(best, float(np.linalg.norm(Q, 2)))
    return best


def psi_history(alphas, betas, sigma: float) -> np.ndarray:
    """psi_i(sigma) for every i = 1 .. len(alphas) - 1 (the right panel of
    Fig. 2).  Quadratic in the number of iterations; fine for a few thousand."""
    return np.array([psi(alphas, betas, sigma, i) for i in range(1, len(alphas))])


def select_shift(alphas, betas, sigmas, i: int | None = None, slack: float = 1.0):
    """Evaluate psi_i on a grid of shifts (Fig. 1) and return (sigma*, values).

    sigma* is the smallest shift whose psi_i is within a factor ``slack`` of
    the smallest value on the grid: Section 5.1 picks a shift at which psi is
    (close to) minimal and warns that a too large shift may destroy
    convergence, and psi_i keeps falling slowly towards the top of the
    spectrum before it explodes there, so the smallest near-minimal shift is
    taken.  slack = 1 is the plain argmin with ties going to the smaller
    shift."""
    sig = np.asarray(sigmas, dtype=np.float64)
    vals = np.array([psi(alphas, betas, s, i) for s in sig])
    best = vals.min()
    ok = np.nonzero(vals <= slack * best)[0]
    k = int(ok[np.argmin(sig[ok])])
    return float(sig[k]), vals
