"""GPU: W-cycles (Sec. 2.2) and the cubic intergrid on every level (eq. (bicubicIntergrid))
against the FP64 oracle, and the paper's Table 'const2D' reproduced on the GPU (compact
stencil, homogeneous medium, 4-level W(1,1), GMRES(5), every patch and intergrid)."""
import numpy as np
import pytest

import synth
from oracle import krylov
from tests.gpu_cases import Case, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2511_16808_amd import binding as B  # noqa: E402

DAMP2 = {"point": [0.89, 0.9, 0.3, 0.71], "element": [0.97, 0.66, 0.48, 0.88],
         "plus": [0.87, 0.57, 0.55, 0.74], "rb": [0.83, 0.5, 0.4, 0.65]}


def crandn(N, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(N) + 1j * r.standard_normal(N)


def gpu(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device="cuda")


@pytest.mark.parametrize("dim,intergrid,patch", [(2, "levdep", "full"), (2, "cubic", "rb"),
                                                 (2, "mixed", "element"), (3, "linear", "full")])
def test_w_cycle_fp64(dim, intergrid, patch):
    """One W(1,1) cycle (4 levels in 2D, 3 in 3D) to 1e-10; the cubic intergrid too."""
    if dim == 2:
        c = Case(n=(65, 65), levels=4, alpha=0.3, medium="layered", seed=2, sponge_width=6,
                 intergrid=intergrid, patch=patch, cycle="W",
                 damping=DAMP2.get(patch, [0.94, 1.2, 0.4, 0.6]))
    else:
        c = Case(n=(17, 17, 17), levels=3, alpha=0.5, medium="random", seed=3, sponge_width=4,
                 cycle="W")
    ops, mg = c.oracle()
    hd = c.gpu()
    try:
        v = crandn(c.N, 4)
        z = torch.empty(c.N, dtype=torch.complex128, device="cuda")
        B.vh_apply_vcycle(hd, gpu(v), z)
        assert rel(z.cpu().numpy(), mg.apply(v)) <= 1e-10
    finally:
        B.vh_destroy(hd)


def test_w_cycle_batched_complex64():
    c = Case(n=(65, 65), levels=4, alpha=0.3, medium="layered", seed=2, sponge_width=6,
             cycle="W", precision=1)
    ops, mg = c.oracle()
    hd = c.gpu(batch=1)
    try:
        v = np.stack([crandn(c.N, 40 + s) for s in range(20)])
        z = torch.empty((20, c.N), dtype=torch.complex128, device="cuda")
        B.vh_apply_vcycle_batch(hd, 20, gpu(v), z)
        out = z.cpu().numpy()
        for s in (0, 19):
            assert rel(out[s], mg.apply(v[s])) <= 1e-5
    finally:
        B.vh_destroy(hd)


CONST2D = [(p, sch) for p in ("point", "element", "plus", "rb") for sch in ("cubic", "mixed", "levdep")]


@pytest.mark.parametrize("patch,scheme", CONST2D)
def test_table_const2d_on_the_gpu(paper, patch, scheme):
    """Table 'const2D': 128^2 cells, omega = 25.6 pi, kappa = 1, gamma = 0, 20-cell layer,
    compact stencil, 4-level W(1,1), GMRES(5), Table 'relaxParam' damping, the printed
    shift of each patch.  The GPU's iteration count is the oracle's (+-10 %) and the
    printed one (+-20 %, the oracle's own pin: the layer profile is unpublished)."""
    row = paper["const2d_128"][patch]
    c = Case(n=(129, 129), levels=4, alpha=row["alpha"], medium="homogeneous", patch=patch,
             intergrid=scheme, damping=DAMP2[patch], stencil="compact4", gamma0=0.0,
             restart=5, cycle="W")
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
    assert abs(its - info["iterations"]) <= max(1, 0.1 * info["iterations"]), (its, info["iterations"])
    assert abs(its - row[scheme]) <= 0.2 * row[scheme], (its, row[scheme])


@pytest.mark.parametrize("levels", [3, 4, 5])
def test_operator_complexity_table_on_the_gpu(paper, levels):
    """Table 'operator_complexity', 64^3 cells, compact 3D stencil, trilinear Galerkin:
    the non-zeros of the GPU's level operators over those of the finest reproduce the
    printed complexity to its 3 decimals (the 4-level cell read as 1.205, the exact count,
    where 1.202 is printed).  The 2-level cell needs a 33^3 coarsest level, beyond the
    dense coarsest solve."""
    ref = paper["operator_complexity_64cube"]["linear"][levels - 2]
    c = Case(n=(65, 65, 65), levels=levels, alpha=0.5, medium="homogeneous", patch="element",
             stencil="compact4", intergrid="linear", gamma0=0.0, damping=[1.1, 0.7, 0.45, 0.6])
    hd = c.gpu()
    try:
        nnz = []
        for l in range(levels):
            info = B.vh_get_level_info(hd, l)
            N = int(np.prod(info["n"]))
            coef = np.zeros((info["stencil_points"], N), dtype=complex)
            B.vh_export_level(hd, l, coef=coef)
            nnz.append(int(np.count_nonzero(coef)))
        assert round(sum(nnz) / nnz[0], 3) == pytest.approx(ref, abs=5e-4), nnz
    finally:
        B.vh_destroy(hd)


@pytest.mark.parametrize("dim", [2, 3])
def test_combined_jacobi_fine_element_coarse(dim):
    """Sec. 5.5, Sec. 6 combined smoother (damped Jacobi on the fine level, Element-patch
    Vanka below, trilinear intergrid, compact stencil): every smoothing step to 1e-12 and
    the V-cycle to 1e-10 against the oracle with the same per-level patches."""
    if dim == 2:
        c = Case(n=(65, 49), levels=3, alpha=0.3, medium="layered", seed=5, sponge_width=6,
                 patch="element", fine_patch="point", intergrid="linear", stencil="compact4",
                 damping=[0.89, 0.66, 0.48])
    else:
        c = Case(n=(17, 25, 17), levels=3, alpha=0.5, medium="random", seed=6, sponge_width=4,
                 patch="element", fine_patch="point", intergrid="linear", stencil="compact4",
                 damping=[0.6, 0.7, 0.45])
    ops, mg = c.oracle()
    hd = c.gpu()
    try:
        assert B.vh_get_level_info(hd, 0)["smoother_entries"] == 1
        assert B.vh_get_level_info(hd, 1)["smoother_entries"] == (2 ** dim) ** 2
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


def test_combined_smoother_solve_3d():
    """3D 33^3, linear kappa^2 in [0.25, 1] (the model of Sec. 5.5), compact stencil,
    gamma = 0, layer, 3-level V(1,1), GMRES(5): the combined smoother's GPU iteration
    count equals the oracle's (+-10 %)."""
    c = Case(n=(33, 33, 33), levels=3, alpha=0.2, medium="linear", patch="element",
             fine_patch="point", intergrid="linear", stencil="compact4", gamma0=0.0,
             restart=5, damping=[0.6, 0.7, 0.45], sponge_width=8)
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
    assert abs(its - info["iterations"]) <= max(1, 0.1 * info["iterations"]), (its, info["iterations"])
