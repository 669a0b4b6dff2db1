"""GPU: the residual formed inside the kernels that consume it (the 2D smoothing sweep and
the restriction, Sec. 2.2 two-grid cycle and Sec. 3.2 eq. (smoother)) gives the same bits
as the separate residual launches (vh_options.split_residual = 2 against 1), on every smoother form
and transfer family that takes it, with ping-pong runs of several smoothing steps and the
W-cycle; and the fused V-cycle still matches the oracle."""
import numpy as np
import pytest

from gpu_cases import Case, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2511_16808_amd import binding as B  # noqa: E402

SYM, ASM, PATCH = B.VH_SMOOTHER_SYMMETRIC, B.VH_SMOOTHER_ASSEMBLED, B.VH_SMOOTHER_PATCH

CASES = [
    # (id, case keyword arguments)
    ("2d-patch-levdep-f64", dict(n=(97, 97), levels=4)),
    ("2d-patch-levdep-c64", dict(n=(97, 97), levels=4, precision=1)),
    ("2d-assembled-c64", dict(n=(129, 65), levels=4, precision=1, smoother=ASM)),
    ("2d-symmetric-f64", dict(n=(129, 129), levels=4, smoother=SYM, intergrid="linear")),
    ("2d-symmetric-c64-nu22", dict(n=(129, 129), levels=4, precision=1, smoother=SYM,
                                   intergrid="linear", nu=(2, 2))),
    ("2d-point-element", dict(n=(97, 97), levels=4, patch="element", fine_patch="point",
                              damping=[0.6, 1.0, 1.0, 1.0])),
    ("2d-cubic-w-nu21", dict(n=(65, 65), levels=3, intergrid="cubic", cycle="W", nu=(2, 1))),
    ("2d-mixed-nu03", dict(n=(65, 97), levels=3, intergrid="mixed", nu=(0, 3))),
    ("3d-assembled-c64", dict(n=(33, 33, 33), levels=3, precision=1, smoother=ASM)),
    ("3d-patch-f64-w", dict(n=(17, 33, 17), levels=3, cycle="W")),
]


def vcycle(case, split, v):
    hd = case.gpu(split_residual=split)
    try:
        z = torch.empty_like(v)
        B.vh_apply_vcycle(hd, v, z)
        torch.cuda.synchronize()
        return z.cpu().numpy()
    finally:
        B.vh_destroy(hd)


@pytest.mark.parametrize("cid,kw", CASES, ids=[c[0] for c in CASES])
def test_fused_vcycle_is_bitwise_the_split_one(cid, kw):
    print(f"fused vs split V-cycle: {cid}", flush=True)
    case = Case(**kw)
    v = torch.tensor(np.random.default_rng(7).standard_normal(case.N) + 1j *
                     np.random.default_rng(8).standard_normal(case.N), device="cuda")
    zf = vcycle(case, 2, v)
    zs = vcycle(case, 1, v)
    assert np.all(np.isfinite(zf))
    assert np.array_equal(zf, zs)


@pytest.mark.parametrize("cid,kw", [CASES[3], CASES[5], CASES[6]],
                         ids=[CASES[k][0] for k in (3, 5, 6)])
def test_fused_vcycle_matches_the_oracle(cid, kw):
    case = Case(**kw)
    ops, mg = case.oracle()
    v = np.random.default_rng(3).standard_normal(case.N) + 0j
    z = vcycle(case, 2, torch.tensor(v, device="cuda"))
    assert rel(z, mg.apply(v)) <= 1e-10


@pytest.mark.parametrize("cid,kw", [CASES[0], CASES[4]], ids=[CASES[0][0], CASES[4][0]])
def test_fused_smoothing_step_hook(cid, kw):
    """vh_apply_smoother takes the fused step where the level has one: the same bits as
    the split step on every smoothed level."""
    case = Case(**kw)
    out = {}
    for split in (2, 1):
        hd = case.gpu(split_residual=split)
        try:
            res = []
            for lev in range(case.levels - 1):
                N = int(np.prod(B.vh_get_level_info(hd, lev)["n"]))
                rng = np.random.default_rng(lev)
                q = torch.tensor(rng.standard_normal(N) + 1j * rng.standard_normal(N), device="cuda")
                u = torch.tensor(rng.standard_normal(N) + 0j, device="cuda")
                B.vh_apply_smoother(hd, lev, q, u)
                res.append(u.cpu().numpy())
            out[split] = res
        finally:
            B.vh_destroy(hd)
    for a, b in zip(out[2], out[1]):
        assert np.array_equal(a, b)


def test_fused_solve_same_iterations_and_bits():
    case = Case(n=(129, 129), levels=4, precision=1, smoother=SYM, intergrid="linear",
                alpha=0.3, sponge_width=12)
    rng = np.random.default_rng(11)
    q = torch.tensor(rng.standard_normal(case.N) + 0j, device="cuda")
    res = {}
    for split in (2, 1, 0):
        hd = case.gpu(split_residual=split)
        try:
            u = torch.empty_like(q)
            st, stats = B.vh_solve(hd, q, 1, 1e-6, u)
            res[split] = (st, stats[0]["iterations"], u.cpu().numpy())
        finally:
            B.vh_destroy(hd)
    assert all(r[0] == B.VH_OK for r in res.values())
    assert res[2][1] == res[1][1] == res[0][1]
    assert np.array_equal(res[2][2], res[1][2]) and np.array_equal(res[0][2], res[1][2])


def test_level_info_reports_the_fusion_choice():
    case = Case(n=(129, 129), levels=4, smoother=SYM, intergrid="linear")
    for split, want in ((1, 0), (2, 1)):
        hd = case.gpu(split_residual=split)
        try:
            info = [B.vh_get_level_info(hd, l) for l in range(case.levels)]
        finally:
            B.vh_destroy(hd)
        assert all(i["fused_sweep"] == want and i["fused_restrict"] == want for i in info[:-1])
        assert info[-1]["fused_sweep"] == 0 and info[-1]["fused_restrict"] == 0
