"""Dense matrix exponential by Pade scaling and squaring (oracle).

Test infrastructure (see the package docstring).

The paper evaluates the small exponential exp(h H_m) with MATLAB's expm
(Sec. 3.3, the discussion of Fig. 5), which is the scaling-and-squaring Pade
method of N. J. Higham, "The scaling and squaring method for the matrix
exponential revisited", SIAM J. Matrix Anal. Appl. 26(4), 2005. This module
follows that published method: choose the smallest diagonal Pade degree
m in {3, 5, 7, 9, 13} whose threshold theta_m bounds the 1-norm; otherwise
scale by 2^-s so that the 1-norm is at most theta_13, use degree 13, and
square s times. The numerator and denominator are summed from explicit powers
(plain, not the paper's or MATLAB's operation-saving split).
"""
from __future__ import annotations

from math import factorial

import numpy as np

# Higham (2005), Table 2.3: largest 1-norm for which the degree-m diagonal
# Pade approximant meets double-precision backward error.
THETA = {3: 1.495585217958292e-2, 5: 2.539398330063230e-1,
         7: 9.504178996162932e-1, 9: 2.097847961257068e0,
         13: 5.371920351148152e0}


def pade_coefficients(m: int) -> np.ndarray:
    """c_j of the [m/m] Pade numerator p(x) = sum_j c_j x^j of exp(x):
    c_j = (2m - j)! m! / ((2m)! j! (m - j)!). Denominator q(x) = p(-x)."""
    return np.array([factorial(2 * m - j) * factorial(m)
                     / (factorial(2 * m) * factorial(j) * factorial(m - j))
                     for j in range(m + 1)])


def pade(A: np.ndarray, m: int) -> np.ndarray:
    c = pade_coefficients(m)
    n = A.shape[0]
    P = np.zeros((n, n), dtype=A.dtype)
    Q = np.zeros((n, n), dtype=A.dtype)
    Ak = np.eye(n)
    for j in range(m + 1):
        if j > 0:
            Ak = Ak @ A
        P += c[j] * Ak
        Q += c[j] * ((-1) ** j) * Ak
    return np.linalg.solve(Q, P)


def expm(A: np.ndarray) -> np.ndarray:
    """e^A in float64, or complex128 for a complex A (the method is the same;
    complex input serves complex-step differentiation)."""
    A = np.asarray(A, dtype=np.complex128 if np.iscomplexobj(A) else np.float64)
    if A.size == 0:
        return A.copy()
    nrm = np.abs(A).sum(axis=0).max()
    for m in (3, 5, 7, 9):
        if nrm <= THETA[m]:
            return pade(A, m)
    s = 0
    if nrm > THETA[13]:
        s = int(np.ceil(np.log2(nrm / THETA[13])))
    R = pade(A / (2.0 ** s), 13)
    for _ in range(s):
        R = R @ R
    return R
