"""GPU: the matrix-core form of the batched additive-Vanka sweep (vh_options.contraction),
2D Full patch, complex64 preconditioner, 16-64 sources.  Each source is checked against
the FP64 oracle (one smoothing step per level, one V-cycle, a solve), and the FP32 matrix
path against the vector-ALU batched path.

Tolerances.  FP32 products (MFMA_F32): the complex64 bound of 1e-5 per application.
Split BF16 (MFMA_BF16X3): each operand x is carried as hi + lo with hi = bf16(x) and
lo = bf16(x - hi), i.e. to 16 significant bits, so each product hi*hi + hi*lo + lo*hi
is within about 3 * 2^-17 ~ 2.3e-5 of the exact product (relative to |a||b|); with the
sums of 18 terms per output and the complex64 rounding around them the per-application
bound used is 5e-5 norm-wise for one smoothing step and 1e-4 for a V-cycle (whose levels
compound it).  Element-wise the bound of an output is 2.3e-5 times the sum of its terms'
magnitudes, which exceeds the output itself where the terms cancel, so the element-wise
measure of one step (largest error over largest output) is held to 1e-4."""
import numpy as np
import pytest

import synth
from oracle import krylov
from tests.gpu_cases import Case, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2511_16808_amd import binding as B  # noqa: E402

# 97 x 81 nodes: strips of 14 and 30 columns both leave a ragged last strip, and
# the rows split into ragged chunks; 3 levels (97x81, 49x41, 25x21 coarsest).
CASE = dict(n=(97, 81), levels=3, alpha=0.3, medium="layered", seed=12, sponge_width=8,
            precision=1)
TOL_STEP = {B.VH_CONTRACT_MFMA_F32: 1e-5, B.VH_CONTRACT_MFMA_BF16X3: 1e-4}
TOL_STEP_NORM = {B.VH_CONTRACT_MFMA_F32: 1e-5, B.VH_CONTRACT_MFMA_BF16X3: 5e-5}
TOL_CYCLE = {B.VH_CONTRACT_MFMA_F32: 1e-5, B.VH_CONTRACT_MFMA_BF16X3: 1e-4}
CONTRACTIONS = [B.VH_CONTRACT_MFMA_F32, B.VH_CONTRACT_MFMA_BF16X3]


def crandn(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def gpu(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex128, device="cuda")


@pytest.fixture(scope="module")
def case():
    c = Case(**CASE)
    c.oracle()
    return c


@pytest.mark.parametrize("contraction", CONTRACTIONS)
@pytest.mark.parametrize("nsrc", [16, 64])
def test_smoother_step_per_source(case, contraction, nsrc):
    ops, mg = case.oracle()
    hd = case.gpu(batch=1, contraction=contraction)
    try:
        for l in range(case.levels - 1):
            N = int(np.prod(mg.h.n[l]))
            q = crandn((nsrc, N), 100 + l)
            u = crandn((nsrc, N), 200 + l)
            ug = gpu(u)
            B.vh_apply_smoother_batch(hd, l, nsrc, gpu(q), ug)
            out = ug.cpu().numpy()
            refs = [mg.relax(l, q[s], u[s]) for s in range(nsrc)]
            errs = [rel(out[s], refs[s]) for s in range(nsrc)]
            assert max(errs) <= TOL_STEP[contraction], (l, max(errs))
            norm = max(np.linalg.norm(out[s] - refs[s]) / np.linalg.norm(refs[s])
                       for s in range(nsrc))
            assert norm <= TOL_STEP_NORM[contraction], (l, norm)
        info = B.vh_get_level_info(hd, 0)
        assert info["mfma_sources"] == nsrc and info["mfma_tile"] in (16, 32)
    finally:
        B.vh_destroy(hd)


@pytest.mark.parametrize("contraction", CONTRACTIONS)
def test_vcycle_per_source(case, contraction):
    ops, mg = case.oracle()
    nsrc = 40  # padded to a batch of 64
    hd = case.gpu(batch=1, contraction=contraction)
    try:
        v = crandn((nsrc, case.N), 7)
        z = torch.empty((nsrc, case.N), dtype=torch.complex128, device="cuda")
        B.vh_apply_vcycle_batch(hd, nsrc, gpu(v), z)
        out = z.cpu().numpy()
        errs = [rel(out[s], mg.apply(v[s])) for s in (0, 13, 39)]
        assert max(errs) <= TOL_CYCLE[contraction], max(errs)
    finally:
        B.vh_destroy(hd)


def test_fp32_matrix_path_matches_vector_path(case):
    """Same products in FP32 on the two units, summed in different orders: one smoothing
    step agrees to 1e-6 norm-wise; element-wise (largest difference over largest output)
    to 5e-6, since each output's rounding is bounded by 18 * 2^-24 times the sum of its
    terms' magnitudes, which exceeds the output where the terms cancel."""
    nsrc = 32
    N = case.N
    q = crandn((nsrc, N), 3)
    u = crandn((nsrc, N), 4)
    outs = []
    for contraction in (B.VH_CONTRACT_VALU, B.VH_CONTRACT_MFMA_F32):
        hd = case.gpu(batch=1, contraction=contraction)
        try:
            ug = gpu(u)
            B.vh_apply_smoother_batch(hd, 0, nsrc, gpu(q), ug)
            outs.append(ug.cpu().numpy())
        finally:
            B.vh_destroy(hd)
    assert np.linalg.norm(outs[1] - outs[0]) <= 1e-6 * np.linalg.norm(outs[0])
    assert rel(outs[1], outs[0]) <= 5e-6


@pytest.mark.parametrize("contraction", CONTRACTIONS)
def test_solve_64_sources(case, contraction):
    """Every sampled source reaches the FP64 tolerance; source 0 takes the oracle's
    iteration count within +-10 %; a second solve on the same handle gives the same
    bits (the tuned tiles are kept per handle)."""
    ops, mg = case.oracle()
    q = synth.random_sources(case.n, 64, seed=21, margin=9)
    hd = case.gpu(batch=1, contraction=contraction)
    try:
        qg = gpu(q.ravel())
        u1 = torch.empty_like(qg)
        st, stats = B.vh_solve(hd, qg, 64, 1e-6, u1)
        assert st == B.VH_OK
        u2 = torch.empty_like(qg)
        st, stats2 = B.vh_solve(hd, qg, 64, 1e-6, u2)
        assert torch.equal(u1, u2)
        un = u1.cpu().numpy().reshape(64, -1)
        for s in (0, 17, 63):
            assert np.linalg.norm(q[s] - ops["H"] @ un[s]) / np.linalg.norm(q[s]) <= 1e-6
        _, info = krylov.fgmres(lambda v: ops["H"] @ v, mg.apply, q[0], 1e-6, case.restart, 1000)
        assert abs(stats[0]["iterations"] - info["iterations"]) <= max(1, 0.1 * info["iterations"])
    finally:
        B.vh_destroy(hd)


def test_contraction_needs_the_supported_configuration():
    c = Case(n=(33, 33, 33), levels=3, alpha=0.5, medium="random", seed=1, sponge_width=4,
             precision=1)
    with pytest.raises(B.VhError):
        c.gpu(batch=1, contraction=B.VH_CONTRACT_MFMA_F32)
    c2 = Case(n=(33, 33), levels=3, alpha=0.3, medium="random", seed=1, sponge_width=4,
              precision=0)
    with pytest.raises(B.VhError):
        c2.gpu(batch=1, contraction=B.VH_CONTRACT_MFMA_BF16X3)
