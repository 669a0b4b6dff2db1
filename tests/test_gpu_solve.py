"""GPU end-to-end: FGMRES(m) + V-cycle solves against the oracle (iteration count
within +-10%, true FP64 relative residual <= tol), and the edge cases of vh_solve."""
import numpy as np
import pytest

import synth
from oracle import krylov
from tests.gpu_cases import Case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2511_16808_amd import binding as B  # noqa: E402


def gpu_solve(c, q, tol=1e-6, **extra):
    hd = c.gpu(**extra)
    try:
        qg = torch.tensor(np.ascontiguousarray(q), dtype=torch.complex128, device="cuda")
        ug = torch.empty_like(qg)
        st, stats = B.vh_solve(hd, qg, qg.numel() // c.N, tol, ug)
        return st, stats, ug.cpu().numpy().reshape(-1, c.N)
    finally:
        B.vh_destroy(hd)


def oracle_solve(c, q, tol=1e-6, maxit=1000):
    ops, mg = c.oracle()
    return krylov.fgmres(lambda v: ops["H"] @ v, mg.apply, q, tol, c.restart, maxit)


def true_relres(c, q, u):
    ops, _ = c.oracle()
    return np.linalg.norm(q - ops["H"] @ u) / np.linalg.norm(q)


@pytest.mark.parametrize("precision", [0, 1])
def test_c1_homogeneous_129(precision):
    """128^2 cells, kappa = 1, 10 ppw, gamma = 0.01 omega, alpha = 0.1, 4-level V(1,1),
    Full 3x3 Vanka, FGMRES(20), point source at the centre."""
    c = Case(n=(129, 129), levels=4, alpha=0.1, medium="homogeneous", precision=precision)
    q = synth.point_source(c.n).ravel()
    _, info = oracle_solve(c, q)
    st, stats, u = gpu_solve(c, q)
    assert st == B.VH_OK and stats[0]["converged"]
    assert abs(stats[0]["iterations"] - info["iterations"]) <= max(1, 0.1 * info["iterations"])
    assert stats[0]["relres"] <= 1e-6
    assert true_relres(c, q, u[0]) <= 1e-6


def test_layered_2d_two_sources():
    c = Case(n=(129, 65), levels=3, alpha=0.3, medium="layered", seed=21, sponge_width=10)
    q = synth.random_sources(c.n, 2, seed=5, margin=12)
    st, stats, u = gpu_solve(c, q.ravel())
    for s in range(2):
        _, info = oracle_solve(c, q[s])
        assert abs(stats[s]["iterations"] - info["iterations"]) <= max(1, 0.1 * info["iterations"])
        assert true_relres(c, q[s], u[s]) <= 1e-6


@pytest.mark.parametrize("precision", [0, 1])
def test_3d_geophysical_small(precision):
    """33^3 nodes, depth-increasing medium with dipping layers and an inclusion,
    trilinear 3-level V(1,1), Full 3x3x3 Vanka, alpha = 0.5, FGMRES(30)."""
    c = Case(n=(33, 33, 33), levels=3, alpha=0.5, medium="layered", seed=3, restart=30,
             precision=precision, sponge_width=6)
    q = synth.point_source(c.n).ravel()
    _, info = oracle_solve(c, q)
    st, stats, u = gpu_solve(c, q)
    assert st == B.VH_OK
    assert abs(stats[0]["iterations"] - info["iterations"]) <= max(1, 0.1 * info["iterations"])
    assert true_relres(c, q, u[0]) <= 1e-6


def test_single_level_is_a_direct_solve():
    c = Case(n=(17, 17), levels=1, alpha=0.0, medium="random", seed=2, sponge_width=3)
    q = synth.point_source(c.n).ravel()
    st, stats, u = gpu_solve(c, q, tol=1e-10)
    assert st == B.VH_OK and stats[0]["iterations"] == 1
    assert true_relres(c, q, u[0]) <= 1e-10


def test_zero_rhs_and_errors():
    c = Case(n=(33, 33), levels=3, alpha=0.3, medium="random", seed=1, sponge_width=4)
    q = np.zeros(c.N, dtype=complex)
    st, stats, u = gpu_solve(c, q)
    assert st == B.VH_OK and stats[0]["iterations"] == 0 and np.all(u == 0)
    q = synth.point_source(c.n).ravel()
    st, stats, u = gpu_solve(c, q, maxit=1)
    assert st == B.VH_ENOCONV and stats[0]["iterations"] == 1 and not stats[0]["converged"]
    q[3] = np.nan
    with pytest.raises(B.VhError) as e:
        gpu_solve(c, q)
    assert e.value.status == B.VH_EBREAKDOWN


def test_restart_lengths_agree_with_oracle():
    """FGMRES(5) with several restarts: same count as the oracle's FGMRES(5)."""
    c = Case(n=(65, 65), levels=3, alpha=0.3, medium="layered", seed=8, restart=5,
             sponge_width=8)
    q = synth.point_source(c.n).ravel()
    _, info = oracle_solve(c, q)
    st, stats, u = gpu_solve(c, q)
    assert st == B.VH_OK and stats[0]["restarts"] >= 2
    assert abs(stats[0]["iterations"] - info["iterations"]) <= max(1, 0.1 * info["iterations"])
