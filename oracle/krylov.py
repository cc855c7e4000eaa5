"""Right-preconditioned flexible GMRES (oracle; test infrastructure only).

The paper solves J B^{-1} z = b, B u = z (Section 2.1, equation
'right-preconditioned') with GMRES (Saad and Schultz, cited in Section 4).
Because the preconditioner here is a fixed linear V-cycle, FGMRES (Saad
1993) is used, which stores the preconditioned vectors Z and updates
x += Z y; it equals right-preconditioned GMRES in exact arithmetic.

Details: x0 = 0; classical Gram-Schmidt applied twice (CGS2); Givens
rotations on the (m+1) x m Hessenberg matrix; the inner loop stops when
|g_{j+1}| <= rtol ||b||; at the end of a cycle x += Z y and the true
residual b - A x decides convergence (relative to ||b||, no absolute
tolerance), otherwise the method restarts from it.  An Arnoldi step whose
new norm is <= 1e-14 times the norm before orthogonalisation is a lucky
breakdown.  The iteration count is the total number of Arnoldi steps over
all cycles.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np


@dataclass
class FGMRESResult:
    x: np.ndarray
    iterations: int
    relres: float
    converged: bool
    history: List[float] = field(default_factory=list)
    # the last cycle, for Arnoldi-relation checks
    V: np.ndarray = None
    Z: np.ndarray = None
    H: np.ndarray = None


def fgmres(A, b: np.ndarray, M: Callable[[np.ndarray], np.ndarray], restart: int = 30,
           rtol: float = 1e-8, max_it: int = 1000) -> FGMRESResult:
    n = b.shape[0]
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n)
    if bnorm == 0.0:
        return FGMRESResult(x, 0, 0.0, True)
    tol = rtol * bnorm
    its = 0
    history = []
    r = b.copy()
    beta = bnorm
    V = Z = H = None
    while True:
        m = restart
        V = np.zeros((n, m + 1))
        Z = np.zeros((n, m))
        H = np.zeros((m + 1, m))
        R = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k = 0
        for j in range(m):
            Z[:, j] = M(V[:, j])
            w = A @ Z[:, j]
            wnorm0 = np.linalg.norm(w)
            h = np.zeros(j + 1)
            for _ in range(2):  # CGS2
                c = V[:, : j + 1].T @ w
                w = w - V[:, : j + 1] @ c
                h += c
            hn = float(np.linalg.norm(w))
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            its += 1
            k = j + 1
            # apply the previous rotations, then a new one
            col = H[: j + 2, j].copy()
            for i in range(j):
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1]
                col[i] = t
            den = np.hypot(col[j], col[j + 1])
            cs[j] = col[j] / den
            sn[j] = col[j + 1] / den
            col[j] = den
            col[j + 1] = 0.0
            R[: j + 2, j] = col
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            history.append(abs(g[j + 1]) / bnorm)
            breakdown = hn <= 1e-14 * wnorm0
            if not breakdown:
                V[:, j + 1] = w / hn
            if abs(g[j + 1]) <= tol or breakdown or its >= max_it:
                break
        # x += Z y with R y = g
        y = np.linalg.solve(np.triu(R[:k, :k]), g[:k])
        x = x + Z[:, :k] @ y
        r = b - A @ x
        beta = float(np.linalg.norm(r))
        if beta <= tol or its >= max_it:
            return FGMRESResult(x, its, beta / bnorm, beta <= tol, history, V, Z, H)
