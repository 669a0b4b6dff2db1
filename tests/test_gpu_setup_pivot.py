"""GPU: patch inverses eliminated in the natural order without pivoting (the default,
vh_options.setup_pivot = 0, on levels whose patch matrices are complex symmetric with a
positive definite imaginary part) against partial pivoting (setup_pivot = 1), Sec. 3.2:
the inverses agree to rounding, and the level information reports which levels skipped
pivoting.  The oracle checks of the other GPU tests run the default."""
import numpy as np
import pytest

from tests.gpu_cases import Case, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2511_16808_amd import binding as B  # noqa: E402

# (id, case, expected setup_pivot flag per smoothed level under the default)
CASES = [
    # 2D level-dependent transfers: R = c P^T only between the two finest levels
    ("2d-levdep", dict(n=(65, 65), levels=4, alpha=0.3, medium="random", seed=2), [0, 0, 1]),
    ("2d-linear-small-shift", dict(n=(65, 97), levels=4, alpha=0.05, medium="layered", seed=3,
                                   intergrid="linear"), [0, 0, 0]),
    ("2d-dirichlet", dict(n=(33, 33), levels=3, alpha=0.5, bc="dirichlet", intergrid="cubic"),
     [0, 0]),
    ("3d-linear", dict(n=(17, 17, 25), levels=3, alpha=0.5, medium="random", seed=4), [0, 0]),
    # the compact stencil is not symmetric, and without a shift the imaginary part vanishes
    # away from the absorbing layer: partial pivoting
    ("2d-compact4", dict(n=(33, 33), levels=3, alpha=0.3, stencil="compact4", gamma0=0.0),
     [1, 1]),
    ("2d-no-shift", dict(n=(33, 33), levels=3, alpha=0.0, intergrid="linear"), [1, 1]),
]


@pytest.mark.parametrize("cid,kw,flags", CASES, ids=[c[0] for c in CASES])
def test_inverses_without_pivoting_match_partial_pivoting(cid, kw, flags):
    print(f"setup pivoting: {cid}", flush=True)
    case = Case(**kw)
    h0, h1 = case.gpu(setup_pivot=0), case.gpu(setup_pivot=1)
    try:
        for l in range(case.levels - 1):
            i0, i1 = B.vh_get_level_info(h0, l), B.vh_get_level_info(h1, l)
            assert i0["setup_pivot"] == flags[l] and i1["setup_pivot"] == 1, l
            Nl = int(np.prod(i0["n"][:case.dim]))
            E = i0["smoother_entries"]
            g0 = np.zeros((E, Nl), dtype=complex)
            g1 = np.zeros((E, Nl), dtype=complex)
            B.vh_export_level(h0, l, smoother=g0)
            B.vh_export_level(h1, l, smoother=g1)
            assert np.abs(g0 - g1).max() <= 1e-12 * np.abs(g1).max(), l
        v = torch.tensor(np.random.default_rng(5).standard_normal(case.N) + 0j, device="cuda")
        z0, z1 = torch.empty_like(v), torch.empty_like(v)
        B.vh_apply_vcycle(h0, v, z0)
        B.vh_apply_vcycle(h1, v, z1)
        assert rel(z0.cpu().numpy(), z1.cpu().numpy()) <= 1e-11
    finally:
        B.vh_destroy(h0)
        B.vh_destroy(h1)


def test_complex64_setup_without_pivoting_matches_the_oracle():
    """3D trilinear, complex64 storage: the no-pivot inverses rounded to complex64 give a
    V-cycle within 1e-5 of the oracle's FP64 one."""
    case = Case(n=(17, 17, 17), levels=3, alpha=0.5, medium="layered", seed=6, precision=1)
    ops, mg = case.oracle()
    hd = case.gpu()
    try:
        assert [B.vh_get_level_info(hd, l)["setup_pivot"] for l in range(2)] == [0, 0]
        v = np.random.default_rng(9).standard_normal(case.N) + 0j
        z = torch.empty(case.N, dtype=torch.complex128, device="cuda")
        B.vh_apply_vcycle(hd, torch.tensor(v, device="cuda"), z)
        assert rel(z.cpu().numpy(), mg.apply(v)) <= 1e-5
    finally:
        B.vh_destroy(hd)
