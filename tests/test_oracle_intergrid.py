"""Pins of the oracle's intergrid operators and Galerkin hierarchy (Sec. 3.1)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import discretization as D
from oracle import hierarchy, intergrid, lfa


def test_restriction_symbols_match_printed_closed_forms():
    """Sec. 4.2 prints the bilinear and bicubic restriction symbols."""
    rng = np.random.default_rng(0)
    th = rng.uniform(-np.pi, np.pi, size=(50, 2))
    c1, c2 = np.cos(th[:, 0]), np.cos(th[:, 1])
    bil = 0.25 * (1 + c1) * (1 + c2)
    bic = (3 + 4 * c1 + np.cos(2 * th[:, 0])) * (3 + 4 * c2 + np.cos(2 * th[:, 1])) / 64
    assert np.allclose(lfa.restriction_symbol("linear", th), bil, atol=1e-14)
    assert np.allclose(lfa.restriction_symbol("cubic", th), bic, atol=1e-14)


def test_restriction_stencils_match_printed_matrices():
    """eq. (biliniearIntergrid) and eq. (bicubicIntergrid) as 2D stencils."""
    n = (9, 9)
    for fam, printed in [
        ("linear", np.array([[1, 2, 1], [2, 4, 2], [1, 2, 1]]) / 16),
        ("cubic", np.outer([1, 4, 6, 4, 1], [1, 4, 6, 4, 1]) / 256),
    ]:
        R = intergrid.restriction(n, fam).toarray()
        row = R[2 + 5 * 2].reshape(9, 9)                # coarse node (2, 2) -> fine (4, 4)
        r = printed.shape[0] // 2
        assert np.allclose(row[4 - r:4 + r + 1, 4 - r:4 + r + 1], printed)
        assert row.sum() == pytest.approx(1.0)


@pytest.mark.parametrize("fam", ["linear", "cubic"])
def test_prolongation_reproduces_linear_functions(fam):
    """P = 2^d R^T interpolates coarse linear data exactly away from the boundary."""
    n = (17, 17)
    P = intergrid.prolongation(n, fam)
    nc = intergrid.coarse_dims(n)
    Y, X = np.meshgrid(np.arange(nc[1]) * 2.0, np.arange(nc[0]) * 2.0, indexing="ij")
    yf, xf = np.meshgrid(np.arange(17.0), np.arange(17.0), indexing="ij")
    v = (3 * X - 2 * Y + 1).ravel()
    out = (P @ v).reshape(17, 17)
    ref = 3 * xf - 2 * yf + 1
    assert np.allclose(out[3:-3, 3:-3], ref[3:-3, 3:-3])


def test_restriction_of_fourier_mode_periodic():
    """On a periodic grid R maps the fine mode e^{i theta x} to R(theta) e^{i 2theta X}."""
    n = (16, 16)
    for fam in ("linear", "cubic"):
        R = intergrid.restriction(n, fam, periodic=True)
        th = np.array([2 * np.pi * 3 / 16, 2 * np.pi * 5 / 16])
        y, x = np.meshgrid(np.arange(16), np.arange(16), indexing="ij")
        mode = np.exp(1j * (th[0] * x + th[1] * y)).ravel()
        Y, X = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
        cmode = np.exp(1j * (2 * th[0] * X + 2 * th[1] * Y)).ravel()
        assert np.allclose(R @ mode, lfa.restriction_symbol(fam, th) * cmode)


def test_galerkin_coarse_correction_is_a_projection():
    """K = I - P A_c^{-1} R A with A_c = R A P satisfies K P = 0 and K^2 = K
    (eq. (2G), Galerkin coarse approximation of Sec. 3.1)."""
    n = (17, 17)
    rng = np.random.default_rng(2)
    kappa = rng.uniform(0.5, 1.0, size=(17, 17))
    ops = D.fd2_operator(n, 1 / 16, 12.0, kappa, 0.3, alpha=0.5, bc="abc", sponge_width=3)
    for scheme in ("levdep", "mixed", "linear"):
        hy = hierarchy.Hierarchy(ops["Hs"], n, 2, scheme)
        A = ops["Hs"].toarray()
        R, P = hy.R[0].toarray(), hy.P[0].toarray()
        Ac = R @ A @ P
        assert np.allclose(Ac, hy.A[1].toarray())
        K = np.eye(A.shape[0]) - P @ np.linalg.solve(Ac, R @ A)
        assert np.abs(K @ P).max() < 1e-10
        assert np.abs(K @ K - K).max() < 1e-10


def coarse_stencil_radius(A, n):
    """Largest |offset| per axis in the stencil of A on grid n."""
    A = sp.coo_matrix(A)
    ix, iy = A.row % n[0], A.row // n[0]
    jx, jy = A.col % n[0], A.col // n[0]
    return max(np.abs(ix - jx).max(), np.abs(iy - jy).max())


def test_stencil_growth_statements():
    """Sec. 3.1: bilinear keeps 3x3, bicubic grows to 5x5 on level 2 and 7x7 below,
    the mixed (and level-dependent) scheme never exceeds 5x5."""
    n = (65, 65)
    ops = D.compact4_operator(n, 1 / 64, 10.0, 1.0, 0.0, bc="dirichlet")
    expect = {"linear": [1, 1, 1, 1], "cubic": [1, 2, 3, 3], "mixed": [1, 2, 2, 2],
              "levdep": [1, 2, 2, 2]}
    for scheme, radii in expect.items():
        hy = hierarchy.Hierarchy(ops["H"], n, 4, scheme)
        got = [coarse_stencil_radius(hy.A[l], hy.n[l]) for l in range(4)]
        assert got == radii, scheme


@pytest.mark.slow
def test_operator_complexity_table(paper):
    """Table 'operator_complexity': 64^3 cells, compact 3D stencil, 2..5 levels."""
    table = paper["operator_complexity_64cube"]
    n = (65, 65, 65)
    L, M = D.compact4_stencils(3, 1 / 64)
    pat = {o: 1.0 for o in list(L) + list(M)}
    A0 = D.stencil_matrix(n, pat)
    for scheme in ("cubic", "levdep", "linear"):
        for i, levels in enumerate((2, 3, 4, 5)):
            oc = hierarchy.operator_complexity(A0, n, levels, scheme)
            assert round(oc, 3) == pytest.approx(table[scheme][i], abs=1e-9), (scheme, levels, oc)
