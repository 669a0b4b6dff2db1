"""GPU parity at the full benchmark sizes, in the launch configuration bench.py times
(same workloads, options and entry points).  Where the oracle can hold the problem it
checks outputs directly (the 1025^2 V-cycle, every true residual); at 257^3, where its
FP64 hierarchy would need ~200 GB, it checks sampled finest-level patch inverses one
by one and the true residual with its FP64 operator."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import cycle, krylov  # noqa: E402
from oracle import discretization as D  # noqa: E402
from oracle import vanka  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import bench  # noqa: E402
from paper_2511_16808_amd import binding as B  # noqa: E402


def setup_workload(key, **over):
    w = dict(bench.WORKLOADS[key], key=key)
    n, h, omega, kappa, gamma, q = bench.make_medium(w)
    opt = B.make_options(precision=w["precision"], restart=w["restart"], damping=w["damping"],
                         intergrid=B.VH_IG_LEVDEP if w["dim"] == 2 else B.VH_IG_LINEAR,
                         batch=w.get("batch", 0), stream=torch.cuda.current_stream(), **over)
    kt = torch.tensor(kappa.ravel(), dtype=torch.float64, device="cuda")
    gt = torch.tensor(gamma.ravel(), dtype=torch.float64, device="cuda")
    hd = B.vh_setup(w["dim"], n, h, omega, kt, gt, w["alpha"], w["levels"], B.VH_PATCH_FULL, opt)
    return w, n, h, omega, kappa, gamma, q, hd


def true_relres(ops, q, u):
    return np.linalg.norm(q - ops["H"] @ u) / np.linalg.norm(q)


def sampled_nodes(n, seed):
    rng = np.random.default_rng(seed)
    # corners, faces, and planes on both sides of the slab edges of the assembled setup
    pts = [(0, 0, 0), (1, 128, 256), (256, 17, 3), (10, 20, 14), (11, 21, 15), (5, 9, 16),
           (200, 40, 17), (12, 22, 29), (13, 23, 30), (250, 250, 255), (3, 4, 240)]
    # both sides of the chunk edges of the symmetric sweep's z walk (8 or 24 planes), and the
    # x-tile edges of its 32 x 8 columns
    pts += [(31, 7, 23), (32, 8, 24), (255, 200, 47), (256, 201, 48), (96, 15, 239)]
    pts += [tuple(int(rng.integers(1, k - 1)) for k in n) for _ in range(8)]
    return pts


def patch_rows(Hs, n, damping, x, y, z):
    """FP64 rows of node (x, y, z) in the inverses of the (up to) 27 Full patches that
    contain it, weighted by damping / (number of such patches): ref[a*27 + m] for the
    patch whose member a is the node, member m the column."""
    nx, ny, nz = n
    offs = vanka.patch_offsets("full", 3)
    cnt = np.prod([3 - (c == 0) - (c == m - 1) for c, m in zip((x, y, z), n)])
    ref = np.zeros(729, dtype=complex)
    for a, oa in enumerate(offs):
        c = (x - oa[0], y - oa[1], z - oa[2])
        if not all(0 <= c[d] < n[d] for d in range(3)):
            continue
        mem = [(c[0] + o[0], c[1] + o[1], c[2] + o[2]) for o in offs]
        ok = [all(0 <= p[d] < n[d] for d in range(3)) for p in mem]
        idx = [p[0] + nx * (p[1] + ny * p[2]) for p, o in zip(mem, ok) if o]
        Ainv = np.linalg.inv(Hs[idx][:, idx].toarray())
        pos = [i for i, o in enumerate(ok) if o]
        arow = pos.index(a)
        for j, m in enumerate(pos):
            ref[a * 27 + m] = damping / cnt * Ainv[arow, j]
    return ref


@pytest.mark.parametrize("sm", ["patch", "symmetric"])
def test_c2_vcycle_and_solve_1025(sm):
    """1025^2 layered medium, 7-level V(1,1), complex128, with the per-patch inverses and
    with the symmetric half of the assembled stencil (bench.py's c2 configuration): one
    V-cycle equals the oracle's to 1e-10; the solve reaches a true FP64 residual <= 1e-6."""
    code = B.VH_SMOOTHER_PATCH if sm == "patch" else B.VH_SMOOTHER_SYMMETRIC
    w, n, h, omega, kappa, gamma, q, hd = setup_workload("c2", smoother=code)
    try:
        ops = D.fd2_operator(n, h, omega, kappa, gamma, w["alpha"])
        mg = cycle.Multigrid(ops["Hs"], n, w["levels"], "levdep", "full", w["damping"])
        v = np.random.default_rng(0).standard_normal(q.size) + 1j * np.random.default_rng(1).standard_normal(q.size)
        z = torch.empty(q.size, dtype=torch.complex128, device="cuda")
        B.vh_apply_vcycle(hd, torch.tensor(v, device="cuda"), z)
        zr = mg.apply(v)
        assert np.linalg.norm(z.cpu().numpy() - zr) <= 1e-10 * np.linalg.norm(zr)
        qt = torch.tensor(q, device="cuda")
        u = torch.empty_like(qt)
        st, stats = B.vh_solve(hd, qt, 1, 1e-6, u)
        assert st == B.VH_OK
        assert true_relres(ops, q, u.cpu().numpy()) <= 1e-6
    finally:
        B.vh_destroy(hd)


def test_c3_sampled_inverses_and_solve_257():
    """257^3, complex64 preconditioner: sampled finest-level patch inverses (27 patches
    per sampled node) equal the oracle's FP64 inverses rounded to complex64; the solve's
    true FP64 residual is <= 1e-6."""
    w, n, h, omega, kappa, gamma, q, hd = setup_workload("c3")
    try:
        ops = D.fd2_operator(n, h, omega, kappa, gamma, w["alpha"])
        nx, ny, nz = n
        pts = sampled_nodes(n, 3)
        nodes = np.array([x + nx * (y + ny * z) for x, y, z in pts], dtype=np.int64)
        G = B.vh_sample_level(hd, 0, 1, nodes, 729)
        Hs = ops["Hs"].tocsr()
        for k, (x, y, z) in enumerate(pts):
            ref = patch_rows(Hs, n, w["damping"][0], x, y, z)
            assert np.abs(G[k] - ref).max() <= 1e-6 * np.abs(ref).max(), (x, y, z)
        qt = torch.tensor(q, device="cuda")
        u = torch.empty_like(qt)
        st, stats = B.vh_solve(hd, qt, 1, 1e-6, u)
        assert st == B.VH_OK
        assert true_relres(ops, q, u.cpu().numpy()) <= 1e-6
    finally:
        B.vh_destroy(hd)


@pytest.mark.parametrize("sm", ["assembled", "symmetric"])
def test_c3_assembled_rows_and_solve_257(sm):
    """257^3 with the assembled smoother (built slab by slab), stored whole or as its
    symmetric half: sampled finest-level rows of the 125-point stencil equal the sums of
    the oracle's FP64 patch-inverse entries with the same offset, rounded to complex64;
    the solve's true FP64 residual is <= 1e-6."""
    code = B.VH_SMOOTHER_ASSEMBLED if sm == "assembled" else B.VH_SMOOTHER_SYMMETRIC
    w, n, h, omega, kappa, gamma, q, hd = setup_workload("c3", smoother=code)
    try:
        ops = D.fd2_operator(n, h, omega, kappa, gamma, w["alpha"])
        nx, ny, nz = n
        pts = sampled_nodes(n, 5)
        nodes = np.array([x + nx * (y + ny * z) for x, y, z in pts], dtype=np.int64)
        Bs = B.vh_sample_level(hd, 0, 1, nodes, 125)
        offs = vanka.patch_offsets("full", 3)
        box2 = [(dx, dy, dz) for dz in range(-2, 3) for dy in range(-2, 3) for dx in range(-2, 3)]
        Hs = ops["Hs"].tocsr()
        for k, (x, y, z) in enumerate(pts):
            rows = patch_rows(Hs, n, w["damping"][0], x, y, z)
            ref = np.zeros(125, dtype=complex)
            for a in range(27):
                for m in range(27):
                    d = tuple(offs[m][c] - offs[a][c] for c in range(3))
                    ref[box2.index(d)] += rows[a * 27 + m]
            assert np.abs(Bs[k] - ref).max() <= 1e-6 * np.abs(ref).max(), (x, y, z)
        # one finest-level smoothing step u + B (q - A u) through the library's sweep on
        # random data, checked at the sampled nodes against the oracle's FP64 patch rows
        # applied to the FP64 residual of the patch members
        rng = np.random.default_rng(11)
        N = nx * ny * nz
        qs = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        us = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        ug = torch.tensor(us, device="cuda")
        B.vh_apply_smoother(hd, 0, torch.tensor(qs, device="cuda"), ug)
        got = ug.cpu().numpy()[nodes]
        del ug
        r = qs - Hs @ us
        corr = np.zeros(len(pts), dtype=complex)
        for k, (x, y, z) in enumerate(pts):
            rows = patch_rows(Hs, n, w["damping"][0], x, y, z)
            for a in range(27):
                c = (x - offs[a][0], y - offs[a][1], z - offs[a][2])
                for m in range(27):
                    p = tuple(c[d] + offs[m][d] for d in range(3))
                    if rows[a * 27 + m] != 0:
                        corr[k] += rows[a * 27 + m] * r[p[0] + nx * (p[1] + ny * p[2])]
        ref = us[nodes] + corr
        scale = np.abs(corr).max()
        err = np.abs(got - ref)
        assert np.all(err <= 1e-5 * scale + 1e-6 * np.abs(us[nodes])), (err.max(), scale)
        qt = torch.tensor(q, device="cuda")
        u = torch.empty_like(qt)
        st, stats = B.vh_solve(hd, qt, 1, 1e-6, u)
        assert st == B.VH_OK
        assert true_relres(ops, q, u.cpu().numpy()) <= 1e-6
    finally:
        B.vh_destroy(hd)


def test_c4_batched_64_sources_513():
    """513^2, 64 sources batched through one hierarchy (complex64 preconditioner):
    every source's true FP64 residual <= 1e-6; the iteration counts of sources 0, 31 and
    63 (a source near each end and one in the middle of the row) within +-10 % of the
    oracle's FP64 FGMRES."""
    w, n, h, omega, kappa, gamma, q, hd = setup_workload("c4")
    try:
        qq = q.reshape(w["nsrc"], -1)
        qt = torch.tensor(q, device="cuda")
        u = torch.empty_like(qt)
        st, stats = B.vh_solve(hd, qt, w["nsrc"], 1e-6, u)
        assert st == B.VH_OK
        un = u.cpu().numpy().reshape(w["nsrc"], -1)
        ops = D.fd2_operator(n, h, omega, kappa, gamma, w["alpha"])
        for s in range(w["nsrc"]):
            assert true_relres(ops, qq[s], un[s]) <= 1e-6, s
        mg = cycle.Multigrid(ops["Hs"], n, w["levels"], "levdep", "full", w["damping"])
        for s in (0, 31, 63):
            print(f"oracle FGMRES, source {s}", flush=True)
            _, info = krylov.fgmres(lambda v: ops["H"] @ v, mg.apply, qq[s], 1e-6, w["restart"],
                                    1000)
            assert abs(stats[s]["iterations"] - info["iterations"]) <= \
                max(1, 0.1 * info["iterations"]), (s, stats[s]["iterations"], info["iterations"])
    finally:
        B.vh_destroy(hd)
