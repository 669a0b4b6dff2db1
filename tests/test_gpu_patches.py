"""GPU parity for the Element, Plus and RB patches (Sec. 3.2, 3.3) and the compact
4th-order stencil (eq. (disc4thCompact), (disc4thCompact3D)): every smoothing step and
V-cycle against the FP64 oracle, and the paper's own 2D configuration (compact stencil,
RB patch, level-dependent intergrid, GMRES(5)) against the oracle's iteration counts and
Table 'heterogeneous2D'."""
import numpy as np
import pytest

import synth
from oracle import krylov
from tests.gpu_cases import Case, rel, stencil_entries

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2511_16808_amd import binding as B  # noqa: E402

# damping of Table 'relaxParam' (2D columns; 3D Element and Plus columns, RB takes Plus)
DAMP = {2: {"element": [0.97, 0.66, 0.48, 0.88], "plus": [0.87, 0.57, 0.55, 0.74],
            "rb": [0.83, 0.5, 0.4, 0.65]},
        3: {"element": [1.1, 0.7, 0.45, 0.6], "plus": [0.92, 0.55, 0.45, 0.55],
            "rb": [0.92, 0.55, 0.45, 0.55]}}


def crandn(N, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(N) + 1j * r.standard_normal(N)


def gpu(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device="cuda")


def case(dim, patch, stencil="fd2", **kw):
    if dim == 2:
        base = dict(n=(65, 49), levels=3, alpha=0.3, medium="layered", seed=5, sponge_width=6)
    else:
        base = dict(n=(17, 25, 17), levels=3, alpha=0.5, medium="random", seed=6, sponge_width=4)
    base.update(kw)
    return Case(patch=patch, damping=DAMP[dim][patch], stencil=stencil, **base)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("patch", ["plus", "rb", "element"])
@pytest.mark.parametrize("stencil", ["fd2", "compact4"])
def test_smoother_and_vcycle(dim, patch, stencil):
    """FP64: one smoothing step per level to 1e-12, one V-cycle to 1e-10."""
    c = case(dim, patch, stencil)
    ops, mg = c.oracle()
    hd = c.gpu()
    try:
        assert B.vh_get_level_info(hd, 0)["smoother_entries"] == mg.smoothers[0].idx.shape[1] ** 2
        for l in range(c.levels - 1):
            N = int(np.prod(mg.h.n[l]))
            q, u = crandn(N, 10 + l), crandn(N, 20 + l)
            ug = gpu(u)
            B.vh_apply_smoother(hd, l, gpu(q), ug)
            assert rel(ug.cpu().numpy(), mg.relax(l, q, u)) <= 1e-12, l
        v = crandn(c.N, 7)
        z = torch.empty(c.N, dtype=torch.complex128, device="cuda")
        B.vh_apply_vcycle(hd, gpu(v), z)
        assert rel(z.cpu().numpy(), mg.apply(v)) <= 1e-10
    finally:
        B.vh_destroy(hd)


@pytest.mark.parametrize("dim", [2, 3])
def test_compact_fine_operator(dim):
    """The compact operator's stencil entries (3^d box) equal the oracle's to 1e-13,
    and the unshifted operator applies to 1e-13."""
    c = case(dim, "rb", "compact4")
    ops, mg = c.oracle()
    hd = c.gpu()
    try:
        info = B.vh_get_level_info(hd, 0)
        assert info["stencil_points"] == 3 ** dim
        coef = np.zeros((info["stencil_points"], c.N), dtype=complex)
        B.vh_export_level(hd, 0, coef=coef)
        ref = stencil_entries(ops["Hs"], c.n, info["offsets"])
        assert np.abs(coef - ref).max() <= 1e-13 * np.abs(ref).max()
        x = crandn(c.N, 1)
        y = torch.empty(c.N, dtype=torch.complex128, device="cuda")
        B.vh_apply_operator(hd, 0, 0, gpu(x), y)
        assert rel(y.cpu().numpy(), ops["H"] @ x) <= 1e-13
    finally:
        B.vh_destroy(hd)


@pytest.mark.parametrize("patch", ["rb", "element"])
def test_assembled_form_of_the_new_patches(patch):
    """The patch sum assembled into a 5^d-point stencil is the same operator."""
    c = case(2, patch, "compact4", smoother=B.VH_SMOOTHER_ASSEMBLED)
    ops, mg = c.oracle()
    hd = c.gpu()
    try:
        assert B.vh_get_level_info(hd, 0)["smoother_entries"] == 25
        v = crandn(c.N, 8)
        z = torch.empty(c.N, dtype=torch.complex128, device="cuda")
        B.vh_apply_vcycle(hd, gpu(v), z)
        assert rel(z.cpu().numpy(), mg.apply(v)) <= 1e-10
    finally:
        B.vh_destroy(hd)


@pytest.mark.parametrize("dim", [2, 3])
def test_batched_new_patches_complex64(dim):
    """Batched V-cycle (24 sources, complex64) per source against the oracle to 1e-5."""
    patch = "rb" if dim == 2 else "element"
    c = case(dim, patch, "compact4", precision=1)
    ops, mg = c.oracle()
    hd = c.gpu(batch=1)
    try:
        v = np.stack([crandn(c.N, 30 + s) for s in range(24)])
        z = torch.empty((24, c.N), dtype=torch.complex128, device="cuda")
        B.vh_apply_vcycle_batch(hd, 24, gpu(v), z)
        out = z.cpu().numpy()
        for s in (0, 11, 23):
            assert rel(out[s], mg.apply(v[s])) <= 1e-5, s
    finally:
        B.vh_destroy(hd)


@pytest.mark.parametrize("levels,alpha,paper_its,tol", [(2, 0.0, 6, 1), (3, 0.1, 12, None),
                                                        (4, 0.25, 34, 7)])
def test_paper_configuration_heterogeneous_2d(levels, alpha, paper_its, tol):
    """Table 'heterogeneous2D', 128^2 cells, linear kappa^2 in [0.25, 1], compact stencil,
    absorbing layer, gamma = 0, RB patch, level-dependent intergrid, V(1,1), GMRES(5):
    the GPU takes the oracle's iteration count (+-10 %).  At 2 and 4 levels that count is
    within the printed one (+-1, +-20 %, the oracle's own pins); at 3 levels the oracle
    takes 16 against the printed 12 (the layer profile is unpublished), so there only
    the GPU-oracle parity is asserted."""
    c = Case(n=(129, 129), levels=levels, alpha=alpha, medium="linear", patch="rb",
             damping=DAMP[2]["rb"], stencil="compact4", gamma0=0.0, restart=5)
    ops, mg = c.oracle()
    q = synth.point_source(c.n).ravel()
    hd = c.gpu()
    try:
        u = torch.empty(c.N, dtype=torch.complex128, device="cuda")
        st, stats = B.vh_solve(hd, gpu(q), 1, 1e-6, u)
        assert st == B.VH_OK
        assert np.linalg.norm(q - ops["H"] @ u.cpu().numpy()) / np.linalg.norm(q) <= 1e-6
    finally:
        B.vh_destroy(hd)
    _, info = krylov.fgmres(lambda v: ops["H"] @ v, mg.apply, q, 1e-6, 5, 1000)
    its = stats[0]["iterations"]
    assert abs(its - info["iterations"]) <= max(1, 0.1 * info["iterations"]), (its, info)
    if tol is not None:
        assert abs(its - paper_its) <= tol, (its, paper_its)
