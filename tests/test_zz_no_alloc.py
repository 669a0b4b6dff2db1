"""GPU: the allocation-free entry point vh_lfa_factors_noalloc (its work arrays in a
static device array) against vh_lfa_factors, the allocating entry point with the same
kernels, on two calls in a row, the second on a smaller problem; both also against the
oracle's local Fourier analysis (Sec. 4, eq. (smoother_symbol), (symbolTG))."""
import numpy as np
import pytest

from oracle import lfa

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2511_16808_amd import binding as B  # noqa: E402


def _problem(dim, stencil, patch, h, sigma, shift, npts, fam):
    return B.make_lfa_problem(
        dim=dim, stencil=stencil, patch=patch, h=h, sigma=sigma, shift=shift, npts=npts,
        rfam=fam, pfam=fam, stream=torch.cuda.current_stream())


def _oracle(dim, stencil, patch, h, sigma, shift, npts, fam, ws):
    f = lfa.compact4_stencil if stencil == B.VH_STENCIL_COMPACT4 else lfa.fd2_stencil
    st = f(dim, h, sigma, shift)
    name = {B.VH_PATCH_FULL: "full", B.VH_PATCH_RB: "rb", B.VH_PATCH_ELEMENT: "element",
            B.VH_PATCH_PLUS: "plus", B.VH_PATCH_POINT: "point"}[patch]
    fam_name = "linear" if fam == B.VH_IG_LINEAR else "cubic"
    mu = [lfa.smoothing_factor(st, name, w, npts=npts, dim=dim) for w in ws]
    rho = [lfa.two_grid_factor(st, name, w, rfam=fam_name, pfam=fam_name, npts=npts, dim=dim)
           for w in ws]
    return mu, rho


CASES = [
    # first call: 2D Full patch, 5-point stencil with a shift, 128^2 samples, 5 dampings
    (2, B.VH_STENCIL_FD2, B.VH_PATCH_FULL, 1 / 256, (51.2 * np.pi) ** 2,
     0.3 * (51.2 * np.pi) ** 2, 128, B.VH_IG_CUBIC, [0.6, 0.8, 0.94, 1.0, 1.1]),
    # second call, smaller: 2D RB patch, compact stencil, 32^2 samples, 2 dampings
    (2, B.VH_STENCIL_COMPACT4, B.VH_PATCH_RB, 1 / 256, (51.2 * np.pi) ** 2, 0.0, 32,
     B.VH_IG_CUBIC, [0.83, 0.9]),
]


def test_noalloc_lfa_equals_the_allocating_entry_point_on_two_calls():
    print("noalloc LFA: two calls (128^2 x 5 dampings, then 32^2 x 2)", flush=True)
    for dim, stencil, patch, h, sigma, shift, npts, fam, ws in CASES:
        p = _problem(dim, stencil, patch, h, sigma, shift, npts, fam)
        mu_n, rho_n = B.vh_lfa_factors_noalloc(p, ws)
        mu_a, rho_a = B.vh_lfa_factors(p, ws)
        # the same kernels in the same launch shapes: the same bits
        assert mu_n == mu_a and rho_n == rho_a, (npts, mu_n, mu_a, rho_n, rho_a)
        mu_o, rho_o = _oracle(dim, stencil, patch, h, sigma, shift, npts, fam, ws)
        for j in range(len(ws)):
            assert mu_n[j] == pytest.approx(mu_o[j], rel=1e-11), (ws[j], mu_n[j], mu_o[j])
            assert rho_n[j] == pytest.approx(rho_o[j], rel=1e-8), (ws[j], rho_n[j], rho_o[j])


def test_noalloc_lfa_3d_and_one_factor_only():
    """3D Element patch, trilinear, 16^3 samples; then the smoothing factor alone after a
    call that left both factors in the shared array."""
    print("noalloc LFA: 3D 16^3, then mu only", flush=True)
    h = 1 / 64
    sigma = (2 * np.pi / (10 * h)) ** 2
    ws = [0.5, 0.8]
    args = (3, B.VH_STENCIL_FD2, B.VH_PATCH_ELEMENT, h, sigma, 0.0, 16, B.VH_IG_LINEAR)
    p = _problem(*args)
    mu_n, rho_n = B.vh_lfa_factors_noalloc(p, ws)
    mu_a, rho_a = B.vh_lfa_factors(p, ws)
    assert mu_n == mu_a and rho_n == rho_a
    mu_o, rho_o = _oracle(*args, ws)
    for j in range(len(ws)):
        assert mu_n[j] == pytest.approx(mu_o[j], rel=1e-11)
        assert rho_n[j] == pytest.approx(rho_o[j], rel=1e-8)
    p2 = _problem(2, B.VH_STENCIL_FD2, B.VH_PATCH_PLUS, 1 / 64, sigma, 0.0, 16, B.VH_IG_CUBIC)
    mu_only, none = B.vh_lfa_factors_noalloc(p2, [0.7], rho=False)
    assert none is None
    assert mu_only == B.vh_lfa_factors(p2, [0.7], rho=False)[0]


def test_noalloc_lfa_rejects_problems_beyond_its_scratch():
    p = _problem(3, B.VH_STENCIL_FD2, B.VH_PATCH_FULL, 1 / 64, 100.0, 0.0, 128, B.VH_IG_LINEAR)
    with pytest.raises(B.VhError) as e:
        B.vh_lfa_factors_noalloc(p, [1.0])
    assert e.value.status == B.VH_EINVAL and "allocation-free" in str(e.value)
