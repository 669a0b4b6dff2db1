"""GPU: the symmetric half of the assembled Full-patch smoother (VH_SMOOTHER_SYMMETRIC;
H_s complex symmetric, Sec. 3.1-3.3) against the oracle and against the full 5^d-point
stencil it replaces, through the C ABI."""
import numpy as np
import pytest

from tests.gpu_cases import Case, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2511_16808_amd import binding as B  # noqa: E402

SYM, FULL = B.VH_SMOOTHER_SYMMETRIC, B.VH_SMOOTHER_ASSEMBLED
# ragged tiles in x and y, planes below the first ones and Dirichlet rows included; the
# 2D level-dependent case keeps the full stencil below level 1 (mixed transfer)
CASES = {
    "2d_cubic": dict(n=(65, 129), levels=4, alpha=0.3, medium="layered", seed=3, sponge_width=6,
                     intergrid="cubic"),
    "2d_levdep": dict(n=(129, 65), levels=4, alpha=0.3, medium="random", seed=7, sponge_width=6),
    "3d": dict(n=(17, 33, 17), levels=3, alpha=0.5, medium="random", seed=4, sponge_width=4),
    "3d_dirichlet": dict(n=(33, 17, 21), levels=3, alpha=0.4, medium="random", seed=6,
                         bc="dirichlet", damping=[1.0, 0.8]),
    # several 16-plane chunks of the z walk, the last one short, on both smoothed levels
    "3d_chunks": dict(n=(41, 17, 37), levels=3, alpha=0.5, medium="layered", seed=5,
                      sponge_width=4),
}


def cplx_randn(N, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(N) + 1j * r.standard_normal(N)


def to_gpu(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device="cuda")


# 3D sweep forms (vh_options.sym_planes): the default choice (one plane per workgroup on
# these small grids), and the z walk of 2, 3, 5 or 16 planes (several chunks handing their
# mirrored sums on, a short last one)
WALKS = [("2d_cubic", 0), ("2d_levdep", 0), ("3d", 0), ("3d", 3), ("3d", 16),
         ("3d_dirichlet", 0), ("3d_dirichlet", 5), ("3d_chunks", 0), ("3d_chunks", 2),
         ("3d_chunks", 5), ("3d_chunks", 16)]


@pytest.mark.parametrize("key,planes", WALKS)
def test_symmetric_vcycle_matches_oracle(key, planes):
    """FP64 V-cycle with the symmetric half on every symmetric level: 1e-10 of the
    oracle, like the full stencil."""
    c = Case(**CASES[key], smoother=SYM)
    ops, mg = c.oracle()
    hd = c.gpu(sym_planes=planes)
    try:
        info = B.vh_get_level_info(hd, 0)
        assert info["smoother_entries"] == 5 ** c.dim
        # the default is one plane per workgroup on grids this small
        assert info["sym_planes"] == (planes if c.dim == 3 else 0)
        v = cplx_randn(c.N, 8)
        z = torch.empty(c.N, dtype=torch.complex128, device="cuda")
        B.vh_apply_vcycle(hd, to_gpu(v), z)
        assert rel(z.cpu().numpy(), mg.apply(v)) <= 1e-10
    finally:
        B.vh_destroy(hd)


@pytest.mark.parametrize("key,planes", WALKS)
@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 2e-6)])
def test_symmetric_sweep_equals_full_stencil(key, planes, precision, tol):
    """Every smoothed level: the exported stencil (rebuilt from the half) equals the full
    assembled one, and one smoothing step u + B(q - A u) agrees (FP64 to 1e-12, complex64
    to 2e-6, the rounding of the stored entries)."""
    c = Case(**CASES[key], precision=precision)
    hs = Case(**CASES[key], smoother=SYM, precision=precision).gpu(sym_planes=planes)
    hf = Case(**CASES[key], smoother=FULL, precision=precision).gpu()
    try:
        for l in range(c.levels - 1):
            info = B.vh_get_level_info(hf, l)
            Nl = int(np.prod(info["n"][:c.dim]))
            E = info["smoother_entries"]
            assert B.vh_get_level_info(hs, l)["smoother_entries"] == E
            es = np.zeros((E, Nl), dtype=complex)
            ef = np.zeros((E, Nl), dtype=complex)
            B.vh_export_level(hs, l, smoother=es)
            B.vh_export_level(hf, l, smoother=ef)
            assert np.abs(es - ef).max() <= tol * np.abs(ef).max(), l
            q = cplx_randn(Nl, 10 + l)
            u0 = cplx_randn(Nl, 20 + l)
            us, uf = to_gpu(u0), to_gpu(u0)
            B.vh_apply_smoother(hs, l, to_gpu(q), us)
            B.vh_apply_smoother(hf, l, to_gpu(q), uf)
            assert rel(us.cpu().numpy() - u0, uf.cpu().numpy() - u0) <= 4 * tol, l
    finally:
        B.vh_destroy(hs)
        B.vh_destroy(hf)


def test_symmetric_sample_matches_export():
    c = Case(**CASES["3d"], smoother=SYM)
    hd = c.gpu()
    try:
        E = 125
        full = np.zeros((E, c.N), dtype=complex)
        B.vh_export_level(hd, 0, smoother=full)
        nodes = np.array([0, 1, c.N - 1, 17 * 33 * 3 + 17 * 5 + 2, 4000], dtype=np.int64)
        s = B.vh_sample_level(hd, 0, 1, nodes, E)
        assert np.array_equal(s, full[:, nodes].T)
    finally:
        B.vh_destroy(hd)


def test_symmetric_solve_3d_complex64():
    """FGMRES with the complex64 preconditioner: the true residual reaches 1e-6 and the
    iteration count is within 1 of the full stencil's."""
    key = "3d"
    out = {}
    for sm in (SYM, FULL):
        c = Case(**CASES[key], smoother=sm, precision=1)
        ops, _ = c.oracle()
        hd = c.gpu()
        try:
            q = cplx_randn(c.N, 30)
            u = torch.empty(c.N, dtype=torch.complex128, device="cuda")
            st, stats = B.vh_solve(hd, to_gpu(q), 1, 1e-6, u)
            assert st == B.VH_OK
            un = u.cpu().numpy()
            assert np.linalg.norm(q - ops["H"] @ un) / np.linalg.norm(q) <= 1e-6
            out[sm] = stats[0]["iterations"]
        finally:
            B.vh_destroy(hd)
    assert abs(out[SYM] - out[FULL]) <= 1, out


def test_symmetric_rejects_batched_sweeps():
    c = Case(**CASES["3d"], smoother=SYM)
    hd = c.gpu()
    try:
        v = to_gpu(cplx_randn(2 * c.N, 1))
        z = torch.empty(2 * c.N, dtype=torch.complex128, device="cuda")
        with pytest.raises(B.VhError) as e:
            B.vh_apply_vcycle_batch(hd, 2, v, z)
        assert e.value.status == B.VH_EUNSUPPORTED
    finally:
        B.vh_destroy(hd)
