"""GPU: vh_footprint_bytes (used for admission by HBM footprint) bounds the device bytes
a handle actually holds at its peak, over setup and solve, for 2D and 3D hierarchies in
FP64 and complex64 with per-patch, assembled and symmetric smoothers and a batched
solve; and the solve statistics carry the setup time and the bytes moved."""
import numpy as np
import pytest

import synth
from tests.gpu_cases import Case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2511_16808_amd import binding as B  # noqa: E402

CASES = [
    # (n, levels, precision, smoother, nsrc, batch)
    ((129, 129), 4, 0, B.VH_SMOOTHER_PATCH, 1, 0),
    ((129, 129), 4, 1, B.VH_SMOOTHER_ASSEMBLED, 1, 0),
    ((257, 129), 4, 0, B.VH_SMOOTHER_SYMMETRIC, 1, 0),
    ((129, 129), 4, 1, B.VH_SMOOTHER_ASSEMBLED, 8, 1),
    ((33, 33, 33), 3, 1, B.VH_SMOOTHER_ASSEMBLED, 1, 0),
    ((33, 33, 33), 3, 0, B.VH_SMOOTHER_PATCH, 1, 0),
    ((65, 33, 33), 3, 1, B.VH_SMOOTHER_PATCH, 2, 1),
]


@pytest.mark.parametrize("n,levels,precision,smoother,nsrc,batch", CASES)
def test_footprint_bounds_the_peak(n, levels, precision, smoother, nsrc, batch):
    print(f"footprint case {n} levels {levels} prec {precision} smoother {smoother} "
          f"nsrc {nsrc} batch {batch}", flush=True)
    c = Case(n=n, levels=levels, alpha=0.3 if len(n) == 2 else 0.5, medium="layered", seed=4,
             precision=precision, smoother=smoother, sponge_width=6,
             restart=20 if len(n) == 2 else 30)
    a = c.gpu_args(batch=batch)
    fp = B.vh_footprint_bytes(c.dim, n, levels, a["patch"], nsrc, a["opt"])
    hd = B.vh_setup(c.dim, n, c.h, c.omega, a["kappa"], a["gamma"], c.alpha, levels, a["patch"],
                    a["opt"])
    try:
        q = synth.random_sources(n, nsrc, seed=9, margin=8).ravel()
        qg = torch.tensor(q, dtype=torch.complex128, device="cuda")
        ug = torch.empty_like(qg)
        st, stats = B.vh_solve(hd, qg, nsrc, 1e-6, ug)
        assert st == B.VH_OK
        in_use, peak = B.vh_get_memory(hd)
    finally:
        B.vh_destroy(hd)
    assert 0 < in_use <= peak <= fp, (in_use, peak, fp)
    assert fp <= 1.5 * peak, (peak, fp)
    for s in stats:
        assert s["setup_ms"] > 0
        # every source's solve reads at least its operator and basis once per iteration
        assert s["bytes_moved"] >= s["iterations"] * c.N * 16
