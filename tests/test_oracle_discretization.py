"""Pins of the oracle's discrete operator (Sec. 1 eq. (acousitcHelm), Sec. 2.1)."""
import numpy as np
import pytest

from oracle import discretization as D
from oracle import lfa


def sine_mode(n, k):
    """Discrete Dirichlet sine mode prod_d sin(k_d pi (j_d+1)/(n_d+1)), flattened."""
    vecs = [np.sin(k[d] * np.pi * (np.arange(n[d]) + 1) / (n[d] + 1)) for d in range(len(n))]
    out = vecs[0]
    for v in vecs[1:]:
        out = np.multiply.outer(v, out)
    return out.ravel()


@pytest.mark.parametrize("n", [(13, 11), (7, 6, 5)])
def test_fd2_sine_modes_are_exact_eigenvectors(n):
    h, omega = 0.1, 7.0
    kappa, gamma = 0.8, 0.3
    ops = D.fd2_operator(n, h, omega, kappa, gamma, alpha=0.0, bc="dirichlet")
    beta = omega ** 2 * kappa ** 2 * (1 - 1j * gamma / omega)
    rng = np.random.default_rng(0)
    for _ in range(5):
        k = [int(rng.integers(1, nd + 1)) for nd in n]
        v = sine_mode(n, k)
        th = [k[d] * np.pi / (n[d] + 1) for d in range(len(n))]
        lam = sum(2 - 2 * np.cos(t) for t in th) / h ** 2 - beta
        assert np.linalg.norm(ops["H"] @ v - lam * v) <= 1e-13 * abs(lam) * np.linalg.norm(v)


def test_compact4_sine_modes_match_eq_Hsymbol():
    n, h, omega, gamma = (12, 9), 0.05, 11.0, 0.0
    ops = D.compact4_operator(n, h, omega, 1.0, gamma, bc="dirichlet")
    sigma = omega ** 2
    a, b, c = lfa.compact4_abc(h, sigma)
    for k in [(1, 1), (3, 7), (12, 2), (6, 9)]:
        v = sine_mode(n, k)
        t1, t2 = k[0] * np.pi / 13, k[1] * np.pi / 10
        lam = a + 2 * b * np.cos(t1) + 2 * b * np.cos(t2) + 4 * c * np.cos(t1) * np.cos(t2)
        assert np.linalg.norm(ops["H"] @ v - lam * v) <= 1e-12 * abs(lam) * np.linalg.norm(v)


def test_compact4_3d_consistency():
    """The 3D compact L annihilates constants and maps x^2 (any axis) to -2 in the
    interior; M has unit row sum (consistency of eq. (disc4thCompact3D))."""
    n, h = (9, 8, 7), 0.25
    L, M = D.compact4_stencils(3, h)
    Lm = D.stencil_matrix(n, L)
    Mm = D.stencil_matrix(n, M)
    z, y, x = np.meshgrid(*(np.arange(k) * h for k in reversed(n)), indexing="ij")
    interior = np.zeros(z.shape, dtype=bool)
    interior[1:-1, 1:-1, 1:-1] = True
    interior = interior.ravel()
    assert np.allclose((Lm @ np.ones(Lm.shape[0]))[interior], 0, atol=1e-10)
    for f in (x, y, z):
        out = Lm @ (f ** 2).ravel()
        assert np.allclose(out[interior], -2.0, atol=1e-10)
    assert np.allclose((Mm @ np.ones(Mm.shape[0]))[interior], 1.0)
    assert sum(1 for c in L.values() if c != 0) == 19


@pytest.mark.parametrize("n", [(17, 13), (9, 7, 6)])
def test_abc_operator_green_identity(n):
    """With gamma = 0 and no layer, summing the scaled rows is the trapezoidal rule
    of int(-Lap u - k^2 u) = boundary flux: for u = 1 the imaginary part is
    omega * kappa * |boundary| / h^d and the real part -omega^2 kappa^2 |Omega| / h^d."""
    h, omega, kappa = 0.125, 3.0, 0.7
    ops = D.fd2_operator(n, h, omega, kappa, 0.0, alpha=0.0, bc="abc", sponge_width=0)
    one = np.ones(ops["H"].shape[0])
    total = one @ (ops["H"] @ one)
    ext = [(k - 1) * h for k in n]
    vol = np.prod(ext)
    if len(n) == 2:
        area = 2 * (ext[0] + ext[1])
    else:
        area = 2 * (ext[0] * ext[1] + ext[1] * ext[2] + ext[0] * ext[2])
    d = len(n)
    assert total.imag == pytest.approx(omega * kappa * area / h ** d, rel=1e-12)
    assert total.real == pytest.approx(-omega ** 2 * kappa ** 2 * vol / h ** d, rel=1e-12)


def test_abc_operator_neumann_part_and_symmetry():
    """omega = 0: the ghost-eliminated Laplacian annihilates constants; H is complex
    symmetric and its imaginary part is a non-negative diagonal."""
    n, h = (11, 9, 5), 0.1
    ops0 = D.fd2_operator(n, h, 0.0, 1.0, 0.0, bc="abc", sponge_width=0)
    assert np.abs(ops0["H"] @ np.ones(ops0["H"].shape[0])).max() < 1e-10
    rng = np.random.default_rng(1)
    kappa = rng.uniform(0.3, 1.0, size=tuple(reversed(n)))
    ops = D.fd2_operator(n, h, 9.0, kappa, 0.2, alpha=0.3, bc="abc", sponge_width=3)
    for key in ("H", "Hs"):
        A = ops[key]
        assert abs(A - A.T).max() < 1e-12 * abs(A).max()
        im = A.imag.tocsr()
        off = im - __import__("scipy.sparse", fromlist=["diags"]).diags(im.diagonal())
        assert abs(off).max() == 0
        assert im.diagonal().min() > 0


def test_sponge_profile():
    n = (61, 50)
    g = D.sponge_gamma(n, 10.0, width=20, amp=1.0).reshape(50, 61)
    assert g[25, 30] == 0.0                       # centre
    assert g[20:30, 20:41].max() == 0.0           # 20 cells away from every face
    row = g[25, :21]
    assert np.all(np.diff(row) < 0)               # rises towards the face
    assert g[25, 0] == pytest.approx(10.0)        # amp * omega on a face
    assert np.allclose(g, g[::-1, ::-1])          # symmetric layer


def test_shift_is_extra_attenuation():
    """H_s - H = i alpha omega^2 M, and H_s equals the operator with extra
    attenuation alpha*omega/kappa^2 in the interior (reading of eq. (shift))."""
    n, h, omega = (9, 9), 0.1, 5.0
    kappa = 0.9
    a = D.fd2_operator(n, h, omega, kappa, 0.0, alpha=0.2, bc="dirichlet")
    b = D.fd2_operator(n, h, omega, kappa, 0.2 * omega / kappa ** 2, alpha=0.0,
                       bc="dirichlet")
    assert abs(a["Hs"] - b["H"]).max() < 1e-12
