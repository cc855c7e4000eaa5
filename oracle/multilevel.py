"""The V-cycle of Algorithm 2 (oracle; test infrastructure only).

Algorithm 2 of the paper (Section 3.3), read as follows:
  * on every level i except the coarsest, z^(0) = 0 and `its` Richardson
    steps z <- z + B_i^{-1}(r_i - A_i z) are taken (its = 3, Section 4; the
    loop runs its times, since its output is z^(its));
  * the residual r_i - A_i z_i is carried to level i+1 by the fine-to-coarse
    operator, here P_i^T, or a fine-to-coarse interpolation R_i of its own
    when one is given (the paper's second MLS interpolation);
  * the coarsest level is solved directly (a dense LU), instead of being
    smoothed;
  * on the way up, z_i <- z_i + P_i z_{i+1}, followed by `its` more
    Richardson steps with the same smoother.
The coarse operators are rediscretised on each mesh (the algorithm asks for
the Jacobian of every level), with kappa taken at the coarse tetrahedra's
centroids.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .schwarz import RAS


@dataclass
class Level:
    A: sp.csr_matrix
    dmask: np.ndarray
    ras: Optional[RAS] = None  # None on the coarsest level
    P: Optional[sp.csr_matrix] = None  # maps level i+1 -> level i
    R: Optional[sp.csr_matrix] = None  # maps level i -> level i+1 (None: P^T)


class VCycle:
    def __init__(self, levels: List[Level], its: int = 3):
        self.levels = levels
        self.its = its
        Ac = levels[-1].A.toarray()
        self.coarse_lu = sla.lu_factor(Ac)

    def apply(self, v: np.ndarray) -> np.ndarray:
        L = len(self.levels)
        r = [None] * L
        z = [None] * L
        r[0] = v
        for i in range(L - 1):
            lev = self.levels[i]
            zi = np.zeros_like(r[i])
            for _ in range(self.its):
                zi = zi + lev.ras.apply(r[i] - lev.A @ zi)
            z[i] = zi
            t = r[i] - lev.A @ zi
            r[i + 1] = lev.P.T @ t if lev.R is None else lev.R @ t
        z[L - 1] = sla.lu_solve(self.coarse_lu, r[L - 1])
        for i in range(L - 2, -1, -1):
            lev = self.levels[i]
            zi = z[i] + lev.P @ z[i + 1]
            for _ in range(self.its):
                zi = zi + lev.ras.apply(r[i] - lev.A @ zi)
            z[i] = zi
        return z[0]

    __call__ = apply
