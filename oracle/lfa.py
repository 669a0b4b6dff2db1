"""Oracle: local Fourier analysis (TEST INFRASTRUCTURE ONLY).

Paper Sec. 2.4: Definition "def_mu_loc" (smoothing factor over T^high), Definition
"def_rho_loc" (two-grid factor over T^low), Definition "def:4harmonics" (the space
of harmonics), eq. (symbolTG) (two-grid symbol).  Paper Sec. 4.1: Vanka smoother
symbol eq. (smoother_symbol), operator symbol eq. (Hsymbol), patch matrices and
Phi for the Element / Plus / RB patches eq. (4lfa), (5lfa), (skew5lfa); theta
sampled on 256 x 256 points of [-pi/2, 3pi/2)^2; Jacobi = 1 x 1 patch.
Paper Sec. 4.2: intergrid symbols, H_c = R H P on the harmonics.

Works in 2D and 3D.  Stencils are dicts {offset tuple: coefficient}.
"""
import itertools

import numpy as np

from .intergrid import R1D
from .vanka import patch_offsets


def fd2_stencil(dim, h, sigma, shift=0.0):
    """2nd-order stencil of H (or H_s with shift = alpha omega^2), M = identity."""
    st = {(0,) * dim: 2 * dim / h ** 2 - sigma + 1j * shift}
    for d in range(dim):
        for s in (-1, 1):
            o = [0] * dim
            o[d] = s
            st[tuple(o)] = -1.0 / h ** 2
    return st


def compact4_stencil(dim, h, sigma, shift=0.0):
    """Compact 4th-order stencil L - (sigma - i shift) M, eq. (disc4thCompact[3D])."""
    from .discretization import compact4_stencils
    L, M = compact4_stencils(dim, h)
    st = dict(L)
    for o, c in M.items():
        st[o] = st.get(o, 0.0) - (sigma - 1j * shift) * c
    return st


def compact4_abc(h, sigma):
    """The constants a, b, c of eq. (Hsymbol) (2D compact stencil)."""
    return (10 / (3 * h ** 2) - 2 * sigma / 3, -2 / (3 * h ** 2) - sigma / 12,
            -1 / (6 * h ** 2))


def symbol(stencil, theta):
    """Scalar symbol sum_o c_o exp(i theta . o); theta has shape (..., dim)."""
    theta = np.asarray(theta, dtype=float)
    out = np.zeros(theta.shape[:-1], dtype=complex)
    for o, c in stencil.items():
        out = out + c * np.exp(1j * (theta @ np.asarray(o, dtype=float)))
    return out


def patch_matrix(stencil, offsets):
    """H_i[k, m] = stencil coefficient at offset (o_m - o_k)."""
    N = len(offsets)
    Hi = np.zeros((N, N), dtype=complex)
    for k in range(N):
        for m in range(N):
            d = tuple(offsets[m][q] - offsets[k][q] for q in range(len(offsets[k])))
            Hi[k, m] = stencil.get(d, 0.0)
    return Hi


def vanka_symbol(stencil, patch, w, theta, dim=None):
    """eq. (smoother_symbol): S(theta) = 1 - w (V^T W Phi^H H_i^{-1} Phi V) H(theta),
    W = I/N (interior patch), V = ones."""
    theta = np.asarray(theta, dtype=float)
    dim = theta.shape[-1] if dim is None else dim
    offs = patch_offsets(patch, dim) if isinstance(patch, str) else list(patch)
    N = len(offs)
    Hinv = np.linalg.inv(patch_matrix(stencil, offs))
    O = np.asarray(offs, dtype=float)
    phi = np.exp(1j * (theta @ O.T))            # (..., N) = diagonal of Phi
    quad = np.einsum("...k,km,...m->...", np.conj(phi), Hinv, phi) / N
    return 1.0 - w * quad * symbol(stencil, theta)


def restriction_symbol(family, theta):
    """Tensor-product symbol of the 1D restriction weights, e.g. bilinear
    (1/4)(1+cos t1)(1+cos t2), bicubic (1/64)(3+4cos t1+cos 2t1)(...)."""
    w = R1D[family]
    rho = len(w) // 2
    theta = np.asarray(theta, dtype=float)
    out = np.ones(theta.shape[:-1], dtype=complex)
    for d in range(theta.shape[-1]):
        s = np.zeros(theta.shape[:-1], dtype=complex)
        for t in range(-rho, rho + 1):
            s = s + w[t + rho] * np.exp(1j * t * theta[..., d])
        out = out * s
    return out


def harmonics(theta):
    """The 2^d harmonics of theta (Definition "def:4harmonics"), shape (2^d, ..., dim)."""
    theta = np.asarray(theta, dtype=float)
    dim = theta.shape[-1]
    hs = []
    for shift in itertools.product((0.0, np.pi), repeat=dim):
        hs.append(theta + np.asarray(shift))
    return np.stack(hs)


def two_grid_symbol(stencil, patch, w, theta, rfam, pfam, nu1=1, nu2=1,
                    coarse_stencil=None):
    """eq. (symbolTG) on the 2^d-harmonic space, for an array of theta.

    The fine stencil is used for A_h; the coarse symbol is Galerkin:
    H_c = sum_h R(th_h) H(th_h) P(th_h), with P = 2^d R^T giving P(th_h) = R_P(th_h).
    Returns an array (..., 2^d, 2^d).
    """
    th = harmonics(theta)                          # (H, ..., dim)
    Hh = symbol(stencil, th)                       # (H, ...)
    Sh = vanka_symbol(stencil, patch, w, th)       # (H, ...)
    Rh = restriction_symbol(rfam, th)
    Ph = restriction_symbol(pfam, th)
    Hc = np.sum(Rh * Hh * Ph, axis=0)              # (...)
    nh = th.shape[0]
    Hh = np.moveaxis(Hh, 0, -1)
    Sh = np.moveaxis(Sh, 0, -1)
    Rh = np.moveaxis(Rh, 0, -1)
    Ph = np.moveaxis(Ph, 0, -1)
    eye = np.eye(nh)
    K = eye - (Ph[..., :, None] / Hc[..., None, None]) * (Rh * Hh)[..., None, :]
    S = Sh[..., :, None] * eye
    T = K
    for _ in range(nu1):
        T = T @ S
    for _ in range(nu2):
        T = S @ T
    return T


def theta_grid(npts=256, dim=2):
    """Samples theta_k = -pi/2 + 2 pi k / npts, k = 0..npts-1, per dimension."""
    t = -np.pi / 2 + 2 * np.pi * np.arange(npts) / npts
    grids = np.meshgrid(*([t] * dim), indexing="ij")
    return np.stack(grids, axis=-1)


def smoothing_factor(stencil, patch, w, npts=256, dim=2):
    """Definition "def_mu_loc": max |S(theta)| over T^high."""
    th = theta_grid(npts, dim)
    hi = ~np.all((th >= -np.pi / 2) & (th < np.pi / 2), axis=-1)
    return float(np.max(np.abs(vanka_symbol(stencil, patch, w, th[hi]))))


def two_grid_factor(stencil, patch, w, rfam="cubic", pfam="cubic", npts=256,
                    dim=2, nu1=1, nu2=1):
    """Definition "def_rho_loc": max spectral radius of TG(theta) over T^low.

    theta = 0 is dropped (the coarse symbol is singular there when sigma = 0).
    """
    th = theta_grid(npts, dim)
    lo = np.all((th >= -np.pi / 2) & (th < np.pi / 2), axis=-1)
    lo &= np.any(np.abs(th) > 1e-12, axis=-1)
    T = two_grid_symbol(stencil, patch, w, th[lo], rfam, pfam, nu1, nu2)
    ev = np.linalg.eigvals(T)
    return float(np.max(np.abs(ev)))
