"""Oracle: intergrid operators (TEST INFRASTRUCTURE ONLY).

Paper Sec. 3.1: full-weighting restriction eq. (biliniearIntergrid) = (1/16)[1 2 1;
2 4 2; 1 2 1], bicubic restriction eq. (bicubicIntergrid) = (1/256) outer([1 4 6 4 1]),
their 3D Kronecker analogues eq. (trilin), eq. (tricub); prolongation P = 2^d R^T
(the paper prints 4 R^T in 2D); the level-dependent scheme eq. (level1Intergrid),
eq. (levelDepIntergrid) and the mixed scheme.

Coarse node I sits on fine node 2I (nodal grid, n_c = (n_f - 1)/2 + 1).  Reading
where the paper is silent: at the boundary, stencil weights that point outside the
grid are dropped (no renormalisation).
"""
import numpy as np
import scipy.sparse as sp

from .discretization import kron_axis

#: 1D restriction weights (centre at index len//2).
R1D = {
    "linear": np.array([1.0, 2.0, 1.0]) / 4.0,
    "cubic": np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0,
}


def coarse_dims(n):
    for k in n:
        if (k - 1) % 2 != 0 or k < 3:
            raise ValueError(f"cannot coarsen {n}")
    return tuple((k - 1) // 2 + 1 for k in n)


def restrict1d(nf, family, periodic=False):
    """(n_c x n_f) 1D restriction, row I = weights centred at fine node 2I."""
    w = R1D[family]
    rho = len(w) // 2
    if periodic:
        nc = nf // 2
    else:
        nc = (nf - 1) // 2 + 1
    rows, cols, vals = [], [], []
    for I in range(nc):
        for t in range(-rho, rho + 1):
            j = 2 * I + t
            if periodic:
                j %= nf
            elif j < 0 or j >= nf:
                continue
            rows.append(I)
            cols.append(j)
            vals.append(w[t + rho])
    return sp.csr_matrix((vals, (rows, cols)), shape=(nc, nf))


def restriction(n, family, periodic=False):
    """d-dimensional restriction = Kronecker product of 1D ones."""
    return kron_axis([restrict1d(k, family, periodic) for k in n])


def prolongation(n, family, periodic=False):
    """P = 2^d R^T for the same family."""
    R = restriction(n, family, periodic)
    return sp.csr_matrix((2 ** len(n)) * R.T)


def scheme_families(scheme, level):
    """(R family, P family) between level and level+1 (level 0 = finest).

    'levdep' : cubic/cubic from the finest level, linear R / cubic P below it;
    'mixed'  : linear R / cubic P on every level;
    'cubic'  : cubic / cubic;  'linear': linear / linear.
    """
    if scheme == "levdep":
        return ("cubic", "cubic") if level == 0 else ("linear", "cubic")
    if scheme == "mixed":
        return ("linear", "cubic")
    if scheme == "cubic":
        return ("cubic", "cubic")
    if scheme == "linear":
        return ("linear", "linear")
    raise ValueError(scheme)
