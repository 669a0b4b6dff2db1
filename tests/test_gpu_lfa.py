"""GPU: local Fourier analysis on the device (Sec. 2.4, Sec. 4) against the oracle's LFA,
and the LFA damping tuner reproducing the fine-level row of Table 'relaxParam'."""
import numpy as np
import pytest

from oracle import lfa

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2511_16808_amd import binding as B  # noqa: E402

PATCH = {"full": B.VH_PATCH_FULL, "point": B.VH_PATCH_POINT, "plus": B.VH_PATCH_PLUS,
         "rb": B.VH_PATCH_RB, "element": B.VH_PATCH_ELEMENT}
H2 = 1 / 256
SIGMA2 = (51.2 * np.pi) ** 2  # 10 points per wavelength at h = 1/256


def oracle_stencil(stencil, dim, h, sigma, shift):
    f = lfa.compact4_stencil if stencil == "compact4" else lfa.fd2_stencil
    return f(dim, h, sigma, shift)


def problem(stencil, dim, patch, h, sigma, shift=0.0, npts=256, fam="cubic"):
    return B.make_lfa_problem(
        dim=dim, stencil=B.VH_STENCIL_COMPACT4 if stencil == "compact4" else B.VH_STENCIL_FD2,
        patch=PATCH[patch], h=h, sigma=sigma, shift=shift, npts=npts,
        rfam=B.VH_IG_CUBIC if fam == "cubic" else B.VH_IG_LINEAR,
        pfam=B.VH_IG_CUBIC if fam == "cubic" else B.VH_IG_LINEAR)


@pytest.mark.parametrize("patch", ["point", "element", "plus", "rb", "full"])
@pytest.mark.parametrize("stencil,shift", [("compact4", 0.0), ("fd2", 0.3)])
def test_lfa_factors_2d(patch, stencil, shift):
    """mu to 1e-11 and rho to 1e-8 (relative) against the oracle, 2D, three dampings;
    the fd2 case carries a shift of 0.3 sigma in the operator."""
    ws = [0.6, 0.85, 1.0]
    npts = 128
    p = problem(stencil, 2, patch, H2, SIGMA2, shift * SIGMA2, npts=npts)
    mu, rho = B.vh_lfa_factors(p, ws)
    st = oracle_stencil(stencil, 2, H2, SIGMA2, shift * SIGMA2)
    for j, w in enumerate(ws):
        m = lfa.smoothing_factor(st, patch, w, npts=npts)
        r = lfa.two_grid_factor(st, patch, w, npts=npts)
        assert mu[j] == pytest.approx(m, rel=1e-11), (w, mu[j], m)
        assert rho[j] == pytest.approx(r, rel=1e-8), (w, rho[j], r)


@pytest.mark.parametrize("patch", ["element", "full", "plus", "point"])
@pytest.mark.parametrize("stencil", ["compact4", "fd2"])
def test_lfa_factors_3d(patch, stencil):
    """3D (8 harmonics, a degree-8 characteristic polynomial), trilinear transfers, 16^3
    samples, against the oracle."""
    h = 1 / 64
    sigma = (2 * np.pi / (10 * h)) ** 2
    ws = [0.5, 0.8]
    p = problem(stencil, 3, patch, h, sigma, npts=16, fam="linear")
    mu, rho = B.vh_lfa_factors(p, ws)
    st = oracle_stencil(stencil, 3, h, sigma, 0.0)
    for j, w in enumerate(ws):
        m = lfa.smoothing_factor(st, patch, w, npts=16, dim=3)
        r = lfa.two_grid_factor(st, patch, w, rfam="linear", pfam="linear", npts=16, dim=3)
        assert mu[j] == pytest.approx(m, rel=1e-11), (w, mu[j], m)
        assert rho[j] == pytest.approx(r, rel=1e-8), (w, rho[j], r)


@pytest.mark.parametrize("patch", ["point", "element", "plus", "rb"])
def test_lfa_tuner_reproduces_table_relaxparam_fine_row(paper, patch):
    """Table 'relaxParam', fine level, 2D: the smoothing-factor minimiser over w in
    [0.5, 1.3] (step 0.01), compact stencil at 10 points per wavelength, 256^2 samples."""
    ws = np.round(np.arange(0.5, 1.3001, 0.01), 2)
    p = problem("compact4", 2, patch, H2, SIGMA2, npts=256)
    w_best, f_best = B.vh_lfa_tune(p, 0, ws)
    assert w_best == pytest.approx(paper["damping_fine_2d"][patch], abs=1e-12)
    st = oracle_stencil("compact4", 2, H2, SIGMA2, 0.0)
    assert f_best == pytest.approx(lfa.smoothing_factor(st, patch, w_best, npts=256), rel=1e-11)


def test_lfa_two_grid_tuner_argmins():
    """The two-grid factor's minimisers for Jacobi, Plus and RB equal the table's values
    (the Element minimiser of the two-grid factor is 0.87, not the table's 0.97)."""
    ws = np.round(np.arange(0.7, 1.1001, 0.01), 2)
    for patch, target in (("point", 0.89), ("plus", 0.87), ("rb", 0.83), ("element", 0.87)):
        p = problem("compact4", 2, patch, H2, SIGMA2, npts=256)
        w_best, _ = B.vh_lfa_tune(p, 1, ws)
        assert w_best == pytest.approx(target, abs=1e-12), patch
