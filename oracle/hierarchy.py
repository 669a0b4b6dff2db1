"""Oracle: Galerkin hierarchy and operator complexity (TEST INFRASTRUCTURE ONLY).

Paper Sec. 3.1: Galerkin coarse approximation H_c = R H P; operator complexity
eq. (operatorComplexity) = sum_l nnz(H^l) / nnz(H^1).
"""
import numpy as np
import scipy.sparse as sp

from .intergrid import coarse_dims, restriction, prolongation, scheme_families


class Hierarchy:
    """Operators A[l] (l = 0 finest), transfers R[l], P[l] between l and l+1."""

    def __init__(self, A0, n, levels, scheme, periodic=False):
        self.n = [tuple(n)]
        self.A = [sp.csr_matrix(A0)]
        self.R, self.P = [], []
        for l in range(levels - 1):
            nf = self.n[-1]
            nc = tuple(k // 2 for k in nf) if periodic else coarse_dims(nf)
            rf, pf = scheme_families(scheme, l)
            R = restriction(nf, rf, periodic)
            P = prolongation(nf, pf, periodic)
            self.R.append(R)
            self.P.append(P)
            self.A.append(sp.csr_matrix(R @ self.A[-1] @ P))
            self.n.append(nc)

    @property
    def levels(self):
        return len(self.A)


def pattern(A):
    """0/1 float matrix with the structural non-zeros of A."""
    B = sp.csr_matrix(A, copy=True)
    B.eliminate_zeros()
    B.data = np.ones_like(B.data, dtype=float)
    return B


def operator_complexity(A0, n, levels, scheme):
    """eq. (operatorComplexity), counted on sparsity patterns.

    Patterns are propagated with non-negative matrices (|R| pattern(H) |P|), so a
    structural non-zero is never lost to numerical cancellation.
    """
    A = pattern(A0)
    total = A.nnz
    nf = tuple(n)
    for l in range(levels - 1):
        rf, pf = scheme_families(scheme, l)
        R = pattern(restriction(nf, rf))
        P = pattern(prolongation(nf, pf))
        A = pattern(R @ A @ P)
        total += A.nnz
        nf = coarse_dims(nf)
    return total / pattern(A0).nnz
