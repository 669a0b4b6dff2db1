"""Pins of the oracle's local Fourier analysis (Sec. 2.4, Sec. 4)."""
import numpy as np
import pytest

from oracle import discretization as D
from oracle import hierarchy, lfa, vanka


def test_Hsymbol_matches_stencil():
    """eq. (Hsymbol) against the symbol of the printed stencil eq. (disc4thCompact)."""
    h, sigma = 1 / 100, 1234.5
    st = lfa.compact4_stencil(2, h, sigma)
    a, b, c = lfa.compact4_abc(h, sigma)
    th = np.random.default_rng(0).uniform(-np.pi, np.pi, size=(40, 2))
    c1, c2 = np.cos(th[:, 0]), np.cos(th[:, 1])
    assert np.allclose(lfa.symbol(st, th), a + 2 * b * c1 + 2 * b * c2 + 4 * c * c1 * c2)


@pytest.mark.parametrize("patch", ["point", "element", "plus", "rb"])
def test_fine_level_damping_is_the_lfa_optimum(paper, patch):
    """Table 'relaxParam' fine-level 2D dampings are the minimisers (0.01 grid) of
    the LFA smoothing factor (Definition 'def_mu_loc') for the compact stencil at
    10 points per wavelength (256^2 cells, omega = 51.2 pi, no shift)."""
    h = 1 / 256
    omega = 51.2 * np.pi
    st = lfa.compact4_stencil(2, h, omega ** 2)
    target = paper["damping_fine_2d"][patch]
    ws = np.round(np.arange(target - 0.05, target + 0.0501, 0.01), 2)
    mu = [lfa.smoothing_factor(st, patch, w, npts=256) for w in ws]
    best = ws[int(np.argmin(mu))]
    assert best == pytest.approx(target, abs=1e-9)


def test_two_grid_lfa_argmins():
    """Two-grid factor (Definition 'def_rho_loc', bicubic, nu1 = nu2 = 1): the
    minimisers over w agree with Table 'relaxParam' for Jacobi, Plus and RB.
    (For Element the two-grid minimiser is 0.87; the table's 0.97 is the
    smoothing-factor minimiser, pinned above.)"""
    h = 1 / 256
    st = lfa.compact4_stencil(2, h, (51.2 * np.pi) ** 2)
    for patch, target in (("point", 0.89), ("plus", 0.87), ("rb", 0.83)):
        ws = np.round(np.arange(target - 0.03, target + 0.0301, 0.01), 2)
        rho = [lfa.two_grid_factor(st, patch, w, npts=256) for w in ws]
        assert ws[int(np.argmin(rho))] == pytest.approx(target, abs=1e-9), patch


def test_two_grid_symbol_matches_periodic_operator():
    """P3: the two-grid error operator of eq. (2G) assembled on a periodic 16x16 grid
    maps span E(theta) to itself by the 4x4 symbol of eq. (symbolTG)."""
    nn = 16
    n = (nn, nn)
    h, sigma, w = 1 / nn, 60.0, 0.85
    st = lfa.compact4_stencil(2, h, sigma, shift=20.0)
    A = D.stencil_matrix(n, st, periodic=True)
    N = nn * nn
    for patch, (rf, pf) in (("rb", ("cubic", "cubic")), ("full", ("linear", "cubic"))):
        hy = hierarchy.Hierarchy(A, n, 2, "mixed" if rf == "linear" else "cubic", periodic=True)
        Ad = A.toarray()
        R, P = hy.R[0].toarray(), hy.P[0].toarray()
        Ac = R @ Ad @ P
        offs = vanka.patch_offsets(patch, 2)
        Ai = np.linalg.inv(lfa.patch_matrix(st, offs))
        B = np.zeros((N, N), dtype=complex)
        for p in range(N):
            x, y = p % nn, p // nn
            mem = [((x + o[0]) % nn) + nn * ((y + o[1]) % nn) for o in offs]
            for a, j in enumerate(mem):
                for b, k in enumerate(mem):
                    B[j, k] += Ai[a, b] / len(offs)
        S = np.eye(N) - w * B @ Ad
        TG = S @ (np.eye(N) - P @ np.linalg.solve(Ac, R @ Ad)) @ S
        th = np.array([2 * np.pi * 3 / nn, 2 * np.pi * 1 / nn])
        T4 = lfa.two_grid_symbol(st, patch, w, th[None, :], rf, pf)[0]
        harm = lfa.harmonics(th[None, :])[:, 0, :]
        yy, xx = np.meshgrid(np.arange(nn), np.arange(nn), indexing="ij")
        modes = np.stack([np.exp(1j * (t[0] * xx + t[1] * yy)).ravel() for t in harm], axis=1)
        assert np.allclose(TG @ modes, modes @ T4, atol=1e-10)
