"""GPU parity: every stage of the HIP path against the FP64 oracle, element by element,
on the same seeded inputs (through the C ABI)."""
import numpy as np
import pytest

from tests.gpu_cases import Case, rel, stencil_entries

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2511_16808_amd import binding as B  # noqa: E402

# 2D: 65 x 129 nodes (ragged: N = 8385 is not a multiple of the block size);
# 3D: 17 x 33 x 17 nodes; both heterogeneous with the absorbing boundary.
CASES = {
    "2d": dict(n=(65, 129), levels=4, alpha=0.3, medium="layered", seed=3, sponge_width=6),
    "3d": dict(n=(17, 33, 17), levels=3, alpha=0.5, medium="random", seed=4, sponge_width=4),
}


def cplx_randn(N, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(N) + 1j * r.standard_normal(N)


def to_gpu(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device="cuda")


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    c = Case(**CASES[request.param])
    c.oracle()
    hd = c.gpu()
    yield c, hd
    B.vh_destroy(hd)


def test_fine_operator(case):
    c, hd = case
    ops, mg = c.oracle()
    info = B.vh_get_level_info(hd, 0)
    coef = np.zeros((info["stencil_points"], c.N), dtype=complex)
    B.vh_export_level(hd, 0, coef=coef)
    ref = stencil_entries(ops["Hs"], c.n, info["offsets"])
    assert np.abs(coef - ref).max() <= 1e-13 * np.abs(ref).max()
    x = cplx_randn(c.N, 1)
    y = torch.empty(c.N, dtype=torch.complex128, device="cuda")
    B.vh_apply_operator(hd, 0, 0, to_gpu(x), y)
    assert rel(y.cpu().numpy(), ops["H"] @ x) <= 1e-13


def test_galerkin_hierarchy(case):
    c, hd = case
    ops, mg = c.oracle()
    for l in range(1, c.levels):
        info = B.vh_get_level_info(hd, l)
        assert info["n"][:c.dim] == mg.h.n[l]
        coef = np.zeros((info["stencil_points"], int(np.prod(mg.h.n[l]))), dtype=complex)
        B.vh_export_level(hd, l, coef=coef)
        ref = stencil_entries(mg.h.A[l], mg.h.n[l], info["offsets"])
        # the GPU stencil must hold every structural non-zero of the Galerkin operator
        assert np.count_nonzero(np.abs(ref) > 0) == mg.h.A[l].count_nonzero()
        assert np.abs(coef - ref).max() <= 1e-12 * np.abs(ref).max(), l


def test_vanka_patch_inverses(case):
    """G[(a*Np+m)][i] = w_l / cnt_i * (A_{i - off_a})^{-1}[a][m]  (Sec. 3.2/3.3)."""
    c, hd = case
    ops, mg = c.oracle()
    for l in range(c.levels - 1):
        sm = mg.smoothers[l]
        n = mg.h.n[l]
        N = int(np.prod(n))
        Np = sm.idx.shape[1]
        info = B.vh_get_level_info(hd, l)
        assert info["smoother_entries"] == Np * Np
        G = np.zeros((Np * Np, N), dtype=complex)
        B.vh_export_level(hd, l, smoother=G)
        from oracle.vanka import patch_offsets
        offs = patch_offsets("full", c.dim)
        coords = [q.ravel() for q in np.indices(tuple(reversed(n)))][::-1]
        ref = np.zeros_like(G)
        for a, off in enumerate(offs):
            ok = np.ones(N, dtype=bool)
            cidx = np.zeros(N, dtype=np.int64)
            stride = 1
            for d in range(c.dim):
                x = coords[d] - off[d]
                ok &= (x >= 0) & (x < n[d])
                cidx += x * stride
                stride *= n[d]
            i = np.flatnonzero(ok)
            cc = cidx[i]
            w = mg.damping[l] / sm.cnt[i]
            for m in range(Np):
                ref[a * Np + m, i] = w * sm.Ainv[cc, a, m] * (sm.idx[cc, m] >= 0)
        assert np.abs(G - ref).max() <= 1e-11 * np.abs(ref).max(), l


def test_smoother_step(case):
    c, hd = case
    ops, mg = c.oracle()
    for l in range(c.levels - 1):
        N = int(np.prod(mg.h.n[l]))
        q = cplx_randn(N, 10 + l)
        u = cplx_randn(N, 20 + l)
        ug = to_gpu(u)
        B.vh_apply_smoother(hd, l, to_gpu(q), ug)
        ref = mg.relax(l, q, u)
        assert rel(ug.cpu().numpy(), ref) <= 1e-12, l


def test_coarsest_inverse(case):
    c, hd = case
    ops, mg = c.oracle()
    L = c.levels - 1
    Nc = int(np.prod(mg.h.n[L]))
    Dinv = np.zeros((Nc, Nc), dtype=complex)
    B.vh_export_level(hd, L, coarse_inv=Dinv)
    ref = np.linalg.inv(mg.h.A[L].toarray())
    assert rel(Dinv, ref) <= 1e-11


def test_vcycle_fp64(case):
    """One V(1,1) application, relative difference <= 1e-10."""
    c, hd = case
    ops, mg = c.oracle()
    for seed in (0, 1):
        v = cplx_randn(c.N, 100 + seed)
        z = torch.empty(c.N, dtype=torch.complex128, device="cuda")
        B.vh_apply_vcycle(hd, to_gpu(v), z)
        assert rel(z.cpu().numpy(), mg.apply(v)) <= 1e-10


@pytest.mark.parametrize("key", list(CASES))
def test_vcycle_c64(key):
    """complex64 preconditioner: relative difference to the FP64 oracle <= 1e-5."""
    c = Case(**CASES[key], precision=B.VH_PREC_C64)
    ops, mg = c.oracle()
    hd = c.gpu()
    try:
        v = cplx_randn(c.N, 7)
        z = torch.empty(c.N, dtype=torch.complex128, device="cuda")
        B.vh_apply_vcycle(hd, to_gpu(v), z)
        assert rel(z.cpu().numpy(), mg.apply(v)) <= 1e-5
    finally:
        B.vh_destroy(hd)


@pytest.mark.parametrize("key", list(CASES))
def test_vcycle_assembled_smoother(key):
    """The additive Vanka operator summed into a 5^d-point stencil is the same
    operator: the V-cycle still matches the oracle to 1e-10."""
    c = Case(**CASES[key], smoother=B.VH_SMOOTHER_ASSEMBLED)
    ops, mg = c.oracle()
    hd = c.gpu()
    try:
        assert B.vh_get_level_info(hd, 0)["smoother_entries"] == 5 ** c.dim
        v = cplx_randn(c.N, 8)
        z = torch.empty(c.N, dtype=torch.complex128, device="cuda")
        B.vh_apply_vcycle(hd, to_gpu(v), z)
        assert rel(z.cpu().numpy(), mg.apply(v)) <= 1e-10
    finally:
        B.vh_destroy(hd)


def test_vcycle_point_patch_and_nu():
    """Point patch (damped Jacobi, Sec. 4.1) and V(2,1)."""
    c = Case(n=(33, 65), levels=3, alpha=0.6, medium="random", seed=9, patch="point",
             damping=[0.7, 0.6], sponge_width=5, nu=(2, 1))
    ops, mg = c.oracle()
    hd = c.gpu()
    try:
        v = cplx_randn(c.N, 9)
        z = torch.empty(c.N, dtype=torch.complex128, device="cuda")
        B.vh_apply_vcycle(hd, to_gpu(v), z)
        assert rel(z.cpu().numpy(), mg.apply(v)) <= 1e-10
    finally:
        B.vh_destroy(hd)


def test_mixed_and_linear_intergrid_2d():
    for ig in ("mixed", "linear"):
        c = Case(n=(33, 33), levels=3, alpha=0.5, medium="random", seed=5, intergrid=ig,
                 sponge_width=4)
        ops, mg = c.oracle()
        hd = c.gpu()
        try:
            v = cplx_randn(c.N, 5)
            z = torch.empty(c.N, dtype=torch.complex128, device="cuda")
            B.vh_apply_vcycle(hd, to_gpu(v), z)
            assert rel(z.cpu().numpy(), mg.apply(v)) <= 1e-10, ig
        finally:
            B.vh_destroy(hd)


def test_operator_on_a_plane_of_two_million_nodes():
    """2049 x 1025 nodes (nx*ny >= 2^21, where the FP64-reciprocal node decode needs its
    downward correction) with a ragged last block: the fine operator applied on the GPU
    equals the oracle's to 1e-13, and so does one finest-level smoothing step of the
    symmetric assembled smoother against the full one."""
    kw = dict(n=(2049, 1025), levels=7, alpha=0.3, medium="random", seed=12, sponge_width=8)
    c = Case(**kw, smoother=B.VH_SMOOTHER_SYMMETRIC)
    ops = c.oracle_ops()
    hd = c.gpu()
    hf = Case(**kw, smoother=B.VH_SMOOTHER_ASSEMBLED).gpu()
    try:
        x = cplx_randn(c.N, 13)
        y = torch.empty(c.N, dtype=torch.complex128, device="cuda")
        B.vh_apply_operator(hd, 0, 0, to_gpu(x), y)
        assert rel(y.cpu().numpy(), ops["H"] @ x) <= 1e-13
        q = cplx_randn(c.N, 14)
        us, uf = to_gpu(x), to_gpu(x)
        B.vh_apply_smoother(hd, 0, to_gpu(q), us)
        B.vh_apply_smoother(hf, 0, to_gpu(q), uf)
        assert rel(us.cpu().numpy() - x, uf.cpu().numpy() - x) <= 1e-12
    finally:
        B.vh_destroy(hd)
        B.vh_destroy(hf)
