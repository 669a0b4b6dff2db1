"""Oracle: additive Vanka smoother (TEST INFRASTRUCTURE ONLY).

Paper Sec. 3.2: patches X_i with injections V_i, patch matrices H_i = V_i H V_i^T,
local solves H_i e_i = V_i (q - H u), update u += W_i e_i; smoother error operator
eq. (smoother) S = I - w (sum_i V_i^T W_i H_i^{-1} V_i) H.
Paper Sec. 3.2 (list of patches): Element, Plus, RB and Full patches in 2D and 3D.
Paper Sec. 3.3: boundary patches = intersection of a whole patch with the domain
(every patch type except Element); W_i(j, j) = 1 / (number of patches containing j).

Patch offsets follow the ordering of the Fourier matrices Phi printed in Sec. 4.1
(eq. (4lfa), (5lfa), (skew5lfa)) for Element, Plus and RB; the Full patch is the
3^d box with x fastest.
"""
import numpy as np
import scipy.sparse as sp

from .discretization import grid_shape


def patch_offsets(kind, dim):
    """Member offsets of one patch relative to its anchor node."""
    if kind == "point":
        return [(0,) * dim]
    if dim == 2:
        if kind == "element":
            return [(0, 0), (1, 0), (0, 1), (1, 1)]
        if kind == "plus":
            return [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)]
        if kind == "rb":
            return [(-1, -1), (1, -1), (0, 0), (-1, 1), (1, 1)]
        if kind == "full":
            return [(dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    else:
        box = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
        if kind == "element":
            return [(dx, dy, dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
        if kind == "plus":
            return [o for o in box if sum(abs(v) for v in o) <= 1]
        if kind == "rb":
            # same red-black colour as the centre inside the 3^3 box
            return [o for o in box if sum(abs(v) for v in o) % 2 == 0]
        if kind == "full":
            return box
    raise ValueError((kind, dim))


def patch_index(n, kind):
    """idx[c, k] = linear index of member k of patch c, or -1 outside the domain.

    Every node anchors a (truncated) patch, except for the Element patch, which
    is anchored at every cell and has no boundary patches (Sec. 3.3).
    """
    n = tuple(n)
    D = len(n)
    offs = patch_offsets(kind, D)
    shape = grid_shape(n)
    coords = [c.ravel() for c in np.indices(shape)][::-1]  # x, y, z
    if kind == "element":
        keep = np.ones(coords[0].shape, dtype=bool)
        for d in range(D):
            keep &= coords[d] < n[d] - 1
        coords = [c[keep] for c in coords]
    P = coords[0].shape[0]
    idx = np.full((P, len(offs)), -1, dtype=np.int64)
    for k, o in enumerate(offs):
        ok = np.ones(P, dtype=bool)
        lin = np.zeros(P, dtype=np.int64)
        stride = 1
        for d in range(D):
            x = coords[d] + o[d]
            ok &= (x >= 0) & (x < n[d])
            lin += x * stride
            stride *= n[d]
        idx[ok, k] = lin[ok]
    return idx


def patch_counts(idx, N):
    """cnt[j] = number of patches containing node j."""
    valid = idx[idx >= 0]
    return np.bincount(valid, minlength=N).astype(float)


class AdditiveVanka:
    """Additive Vanka smoother for a sparse matrix A on an n-grid.

    apply(r) returns B r with B = sum_c V_c^T W_c A_c^{-1} V_c (the damping w is
    applied by the caller, eq. (smoother)).
    """

    def __init__(self, A, n, kind):
        A = sp.csr_matrix(A)
        self.n = tuple(n)
        self.N = A.shape[0]
        self.kind = kind
        self.idx = patch_index(n, kind)
        P, Np = self.idx.shape
        # patch matrices A_c = V_c A V_c^T; out-of-domain members padded by identity
        Ac = np.zeros((P, Np, Np), dtype=complex)
        for k in range(Np):
            for m in range(Np):
                ok = (self.idx[:, k] >= 0) & (self.idx[:, m] >= 0)
                if ok.any():
                    vals = A[self.idx[ok, k], self.idx[ok, m]]
                    Ac[ok, k, m] = np.asarray(vals).ravel()
            Ac[self.idx[:, k] < 0, k, k] = 1.0
        self.Ainv = np.linalg.inv(Ac)
        self.cnt = patch_counts(self.idx, self.N)
        self.weight = np.where(self.idx >= 0, 1.0 / self.cnt[np.maximum(self.idx, 0)], 0.0)

    def apply(self, r):
        r = np.asarray(r, dtype=complex)
        loc = np.where(self.idx >= 0, r[np.maximum(self.idx, 0)], 0.0)
        e = np.einsum("pkm,pm->pk", self.Ainv, loc)
        contrib = (self.weight * e)[self.idx >= 0]
        where = self.idx[self.idx >= 0]
        out = np.bincount(where, weights=contrib.real, minlength=self.N) \
            + 1j * np.bincount(where, weights=contrib.imag, minlength=self.N)
        return out

    def dense(self):
        """Dense B = sum_c V_c^T W_c A_c^{-1} V_c (small grids only)."""
        B = np.zeros((self.N, self.N), dtype=complex)
        for c in range(self.idx.shape[0]):
            mem = self.idx[c]
            ok = np.flatnonzero(mem >= 0)
            rows = mem[ok]
            B[np.ix_(rows, rows)] += (self.weight[c, ok][:, None]
                                      * self.Ainv[c][np.ix_(ok, ok)])
        return B


def smoother_error_operator(A, B, w):
    """Dense eq. (smoother): S = I - w B A."""
    A = A.toarray() if sp.issparse(A) else np.asarray(A)
    return np.eye(A.shape[0]) - w * (B @ A)

