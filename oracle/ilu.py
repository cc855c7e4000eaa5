"""Incomplete LU factorisation with level of fill, ILU(k) (oracle; test
infrastructure only).

Section 4 of the paper replaces the exact subdomain solve of the RAS
smoother by ILU(p) (ILU(2) on the finest level and ILU(0) on the coarser
ones in the scaling runs).  The paper takes the factorisation from PETSc and
does not restate it; this is the textbook definition it refers to:

* level of fill: lev(i, j) = 0 where a_ij != 0 and infinity elsewhere; when
  row k eliminates entry (i, k), every (i, j) with j > k in row k's upper
  part gets lev(i, j) = min(lev(i, j), lev(i, k) + lev(k, j) + 1); the
  pattern of ILU(k) keeps the entries of level <= k (rows processed in
  order, the eliminations of a row in ascending column order);
* numeric factorisation (the i-k-j form of Gaussian elimination restricted
  to that pattern): for each row i and each k < i in its pattern, ascending,
  l_ik = a_ik / u_kk and a_ij -= l_ik u_kj for every j > k in both row k and
  row i's pattern; L is unit lower triangular, U upper triangular;
* apply: z = U^{-1} L^{-1} r by two sparse triangular solves.

Natural ordering (the subdomain's vertices in ascending global id), no
pivoting: the subdomain matrices are symmetric positive definite, and a zero
or negative pivot is an error.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def symbolic(A: sp.csr_matrix, fill: int):
    """Pattern of ILU(fill): list of sorted column arrays per row, and the
    level of every kept entry (same layout)."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    cols, levs = [], []
    for i in range(n):
        lev = {int(j): 0 for j in A.indices[A.indptr[i]:A.indptr[i + 1]]}
        lev.setdefault(i, 0)
        done = set()
        while True:
            # the smallest column k < i of row i not yet eliminated
            cand = [k for k in lev if k < i and k not in done]
            if not cand:
                break
            k = min(cand)
            done.add(k)
            lik = lev[k]
            if lik > fill:
                continue
            for j, lkj in zip(cols[k], levs[k]):
                if j <= k:
                    continue
                new = lik + lkj + 1
                if new <= fill and new < lev.get(j, fill + 1):
                    lev[j] = new
        keep = sorted(j for j, v in lev.items() if v <= fill)
        cols.append(np.array(keep, dtype=np.int64))
        levs.append(np.array([lev[j] for j in keep], dtype=np.int64))
    return cols, levs


def factor(A: sp.csr_matrix, cols):
    """Numeric ILU on the pattern `cols`: (L, U) with L unit lower (strict part
    stored) and U upper, as CSR matrices."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    rows = []
    for i in range(n):
        row = {int(j): 0.0 for j in cols[i]}
        for j, v in zip(A.indices[A.indptr[i]:A.indptr[i + 1]], A.data[A.indptr[i]:A.indptr[i + 1]]):
            if int(j) in row:
                row[int(j)] = float(v)
        for k in [c for c in sorted(row) if c < i]:
            ukk = rows[k][k]
            lik = row[k] / ukk
            row[k] = lik
            for j, ukj in rows[k].items():
                if j > k and j in row:
                    row[j] -= lik * ukj
        if not row[i] > 0:
            raise ZeroDivisionError(f"non-positive pivot in row {i}")
        rows.append(row)
    li, lj, lv, ui, uj, uv = [], [], [], [], [], []
    for i, row in enumerate(rows):
        for j, v in row.items():
            if j < i:
                li.append(i), lj.append(j), lv.append(v)
            else:
                ui.append(i), uj.append(j), uv.append(v)
    L = sp.csr_matrix((lv, (li, lj)), shape=(n, n)) + sp.identity(n, format="csr")
    U = sp.csr_matrix((uv, (ui, uj)), shape=(n, n))
    return L, U


class ILU:
    """z = (L U)^{-1} r for the ILU(fill) factors of A."""

    def __init__(self, A: sp.csr_matrix, fill: int):
        self.cols, self.levs = symbolic(A, fill)
        self.L, self.U = factor(A, self.cols)

    def solve(self, r: np.ndarray) -> np.ndarray:
        y = spla.spsolve_triangular(self.L, r, lower=True, unit_diagonal=True)
        return spla.spsolve_triangular(self.U, y, lower=False)
