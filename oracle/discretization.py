"""Oracle: the discrete acoustic Helmholtz operator (TEST INFRASTRUCTURE ONLY).

Paper Sec. 1, eq. (acousitcHelm): -Lap p - omega^2 kappa^2 (1 - i gamma/omega) p = q.
Paper Sec. 2.1: 2nd-order 5-point (2D) / 7-point (3D) stencil (mentioned as the
standard scheme) and the compact 4th-order stencils eq. (disc4thCompact),
eq. (disc4thCompact3D).  Paper Sec. 2.3 eq. (shift): the complex shift.

Grid convention: N cells per dimension -> N+1 nodes, all unknown, x_j = j h.
Arrays are numpy arrays of shape n[::-1] (x fastest), flattened in C order, so the
linear index of node (x, y[, z]) is x + nx*(y + ny*z).

Readings where the paper is silent:
  * absorbing layer: gamma_abc = amp*omega*sum_d ((W - s_d)/W)^2 for s_d < W, s_d
    the distance in cells to the nearer face along d, W = 20 cells (Sec. 5 says
    only "a layer of 20 grid cells of increasing attenuation");
  * first-order absorbing (Sommerfeld) closure du/dn = -i omega kappa u on the
    boundary nodes of the 2nd-order stencil, discretised by eliminating a ghost
    node, then each boundary row scaled by 1/2 per boundary direction so that H is
    complex symmetric;
  * attenuation enters as (1 - i gamma/omega) per eq. (acousitcHelm);
  * the shift is added with the same sign as the attenuation, H_s = H + i alpha
    omega^2 M (eq. (shift) prints a minus; with the plus sign H_s is the operator
    with extra attenuation, which is how Sec. 2.3 motivates it);
  * for the 2nd-order stencil M is the identity of the unscaled system, i.e. the
    diagonal row-scaling matrix S of the scaled system.
"""
import numpy as np
import scipy.sparse as sp


def grid_shape(n):
    """numpy array shape for node counts n = (nx, ny[, nz])."""
    return tuple(int(k) for k in reversed(n))


def kron_axis(factors):
    """Kronecker product of per-dimension factors [F_x, F_y, (F_z)], x fastest."""
    out = factors[0]
    for f in factors[1:]:
        out = sp.kron(f, out, format="csr")
    return sp.csr_matrix(out)


def axis_operator(n, d, T):
    """Operator T acting along dimension d, identity along the others."""
    facs = [sp.identity(k, format="csr", dtype=complex) for k in n]
    facs[d] = sp.csr_matrix(T, dtype=complex)
    return kron_axis(facs)


def boundary_flags(n):
    """List over dims of 0/1 arrays (flattened): node lies on a face normal to d."""
    shape = grid_shape(n)
    D = len(n)
    flags = []
    for d in range(D):
        idx = np.indices(shape)[D - 1 - d]
        flags.append(((idx == 0) | (idx == n[d] - 1)).astype(float).ravel())
    return flags


def face_distance(n):
    """Per-dim distance in cells to the nearer face, list of flattened arrays."""
    shape = grid_shape(n)
    D = len(n)
    out = []
    for d in range(D):
        idx = np.indices(shape)[D - 1 - d]
        out.append(np.minimum(idx, n[d] - 1 - idx).astype(float).ravel())
    return out


def sponge_gamma(n, omega, width=20, amp=1.0):
    """Absorbing-layer attenuation gamma_abc (flattened), reading of Sec. 5.

    Zero in the interior, rising quadratically to amp*omega per face at the boundary.
    """
    g = np.zeros(int(np.prod(n)))
    if width <= 0 or amp == 0.0:
        return g
    for s in face_distance(n):
        inside = s < width
        g[inside] += amp * omega * ((width - s[inside]) / width) ** 2
    return g


def beta(kappa, gamma, omega):
    """beta = omega^2 kappa^2 (1 - i gamma/omega), eq. (acousitcHelm), written as
    omega^2 kappa^2 - i omega kappa^2 gamma so that omega = 0 is allowed."""
    kappa = np.asarray(kappa, dtype=float).ravel()
    gamma = np.asarray(gamma, dtype=float).ravel()
    return omega ** 2 * kappa ** 2 - 1j * omega * kappa ** 2 * gamma


def lap1d(n, h, bc):
    """1D second-difference operator (-u_{j-1} + 2u_j - u_{j+1})/h^2.

    bc: 'dirichlet' - a missing neighbour counts as zero;
        'periodic'  - wraps around;
        'abc'       - ghost node eliminated with du/dn = -i omega kappa u: the end
                      rows become (2u_0 - 2u_1)/h^2 (the i omega kappa part is added
                      as a diagonal term by the caller).
    """
    T = sp.lil_matrix((n, n), dtype=complex)
    for j in range(n):
        T[j, j] = 2.0
        if j > 0:
            T[j, j - 1] = -1.0
        if j < n - 1:
            T[j, j + 1] = -1.0
    if bc == "periodic":
        T[0, n - 1] += -1.0
        T[n - 1, 0] += -1.0
    elif bc == "abc":
        T[0, 1] = -2.0
        T[n - 1, n - 2] = -2.0
    return sp.csr_matrix(T) / h ** 2


def fd2_operator(n, h, omega, kappa, gamma0, alpha=0.0, bc="abc",
                 sponge_width=20, sponge_amp=1.0):
    """2nd-order operator H (and the shifted H_s) on the nodal grid.

    Returns dict with csr matrices 'H', 'Hs', the mass matrix 'M' (diagonal) and the
    total attenuation 'gamma'.

    bc = 'abc'       : sponge layer + first-order absorbing closure + symmetrising
                       row scaling (the build's production boundary);
    bc = 'dirichlet' : no sponge, missing neighbours are zero (eigen-pins);
    bc = 'periodic'  : no sponge, wrap-around (LFA pins).
    """
    n = tuple(int(k) for k in n)
    D = len(n)
    N = int(np.prod(n))
    kappa = np.broadcast_to(np.asarray(kappa, dtype=float), grid_shape(n)).ravel()
    gamma0 = np.broadcast_to(np.asarray(gamma0, dtype=float), grid_shape(n)).ravel()
    if bc == "abc":
        gamma = gamma0 + sponge_gamma(n, omega, sponge_width, sponge_amp)
    else:
        gamma = gamma0.copy()
    H0 = sp.csr_matrix((N, N), dtype=complex)
    for d in range(D):
        H0 = H0 + axis_operator(n, d, lap1d(n[d], h, bc))
    diag = -beta(kappa, gamma, omega)
    if bc == "abc":
        flags = boundary_flags(n)
        nb = np.zeros(N)
        for f in flags:
            nb += f
        diag = diag + nb * 2j * omega * kappa / h
        s = np.ones(N)
        for f in flags:
            s *= np.where(f > 0, 0.5, 1.0)
    else:
        s = np.ones(N)
    H0 = H0 + sp.diags(diag)
    S = sp.diags(s)
    H = sp.csr_matrix(S @ H0)
    M = sp.csr_matrix(S.astype(complex))
    Hs = sp.csr_matrix(H + 1j * alpha * omega ** 2 * M)
    return {"H": H, "Hs": Hs, "M": M, "gamma": gamma, "scale": s}


# --- compact 4th-order stencils (Sec. 2.1) -------------------------------------

def compact4_stencils(dim, h):
    """Stencil dicts {offset: coefficient} for L and M of eq. (disc4thCompact[3D])."""
    L, M = {}, {}
    if dim == 2:
        Lw = np.array([[-1 / 6, -2 / 3, -1 / 6],
                       [-2 / 3, 10 / 3, -2 / 3],
                       [-1 / 6, -2 / 3, -1 / 6]]) / h ** 2
        Mw = np.array([[0, 1 / 12, 0], [1 / 12, 2 / 3, 1 / 12], [0, 1 / 12, 0]])
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if Lw[dy + 1, dx + 1] != 0:
                    L[(dx, dy)] = Lw[dy + 1, dx + 1]
                if Mw[dy + 1, dx + 1] != 0:
                    M[(dx, dy)] = Mw[dy + 1, dx + 1]
    else:
        outer = np.array([[0, 1, 0], [1, 2, 1], [0, 1, 0]], dtype=float)
        mid = np.array([[1, 2, 1], [2, -24, 2], [1, 2, 1]], dtype=float)
        Lw = -np.stack([outer, mid, outer]) / (6 * h ** 2)
        m_out = np.array([[0, 0, 0], [0, 1, 0], [0, 0, 0]], dtype=float)
        m_mid = np.array([[0, 1, 0], [1, 6, 1], [0, 1, 0]], dtype=float)
        Mw = np.stack([m_out, m_mid, m_out]) / 12.0
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if Lw[dz + 1, dy + 1, dx + 1] != 0:
                        L[(dx, dy, dz)] = Lw[dz + 1, dy + 1, dx + 1]
                    if Mw[dz + 1, dy + 1, dx + 1] != 0:
                        M[(dx, dy, dz)] = Mw[dz + 1, dy + 1, dx + 1]
    return L, M


def shift1d(n, t, periodic):
    """1D matrix with ones at (j, j+t): (S u)_j = u_{j+t}."""
    if periodic:
        rows = np.arange(n)
        cols = (rows + t) % n
    else:
        rows = np.arange(max(0, -t), min(n, n - t))
        cols = rows + t
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))


def stencil_matrix(n, stencil, periodic=False):
    """Sparse matrix of a constant stencil {offset: coef} (truncated or periodic)."""
    N = int(np.prod(n))
    A = sp.csr_matrix((N, N), dtype=complex)
    for off, c in stencil.items():
        facs = [shift1d(n[d], off[d], periodic) for d in range(len(n))]
        A = A + c * kron_axis(facs)
    return sp.csr_matrix(A)


def compact4_operator(n, h, omega, kappa, gamma0, alpha=0.0, bc="sponge",
                      sponge_width=20, sponge_amp=1.0):
    """Compact 4th-order operator H = L - M diag(beta), H_s = H + i alpha omega^2 M.

    bc = 'sponge'    : absorbing layer, stencil truncated at the boundary;
    bc = 'dirichlet' : truncated, no layer;  bc = 'periodic': wrap-around.
    Variable kappa enters as M diag(beta) (reading: the mass stencil acts on beta*u).
    """
    n = tuple(int(k) for k in n)
    kappa = np.broadcast_to(np.asarray(kappa, dtype=float), grid_shape(n)).ravel()
    gamma0 = np.broadcast_to(np.asarray(gamma0, dtype=float), grid_shape(n)).ravel()
    gamma = gamma0 + (sponge_gamma(n, omega, sponge_width, sponge_amp)
                      if bc == "sponge" else 0.0)
    Ls, Ms = compact4_stencils(len(n), h)
    per = bc == "periodic"
    L = stencil_matrix(n, Ls, per)
    M = stencil_matrix(n, Ms, per)
    H = sp.csr_matrix(L - M @ sp.diags(beta(kappa, gamma, omega)))
    Hs = sp.csr_matrix(H + 1j * alpha * omega ** 2 * M)
    return {"H": H, "Hs": Hs, "M": M, "gamma": gamma}


def operator(stencil, n, h, omega, kappa, gamma0, alpha=0.0, bc=None, **kw):
    """Dispatch on stencil = 'fd2' | 'compact4'."""
    if stencil == "fd2":
        return fd2_operator(n, h, omega, kappa, gamma0, alpha, bc or "abc", **kw)
    if stencil == "compact4":
        return compact4_operator(n, h, omega, kappa, gamma0, alpha, bc or "sponge", **kw)
    raise ValueError(stencil)
