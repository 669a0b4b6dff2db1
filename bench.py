#!/usr/bin/env python3
"""Benchmark of the Vanka-smoothed shifted-Laplacian Helmholtz solver on one MI355X.

One step = one pass of the whole hot path over one synthetic input: vh_setup
(finest operator, Galerkin hierarchy, every patch inverse, coarsest inverse) and
vh_solve (FGMRES(m) preconditioned by V(1,1) cycles to true relative residual 1e-6)
from a medium and a source already resident in HBM, then vh_destroy.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3]

Prints ONE JSON line.  Workloads (synthetic media, seeded):
  c1  2D 129^2 nodes, homogeneous, 4 levels, complex128 (the oracle solves it in seconds)
  c2  2D 1025^2 layered medium, 7 levels, complex128
  c3  3D 257^3 geophysical medium, 6 levels, complex64 preconditioner / complex128 FGMRES
  c4  2D 513^2 layered medium, 64 sources sharing one hierarchy and every V-cycle sweep
  c5  serving mix of 2D/3D requests with Poisson arrivals through the request loop
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Helmholtz solves/s to rel.res 1e-6 (512^2, 256^3); V-cycle HBM GB/s; p50/p99 ms"
HBM_PEAK_GBPS = 8000.0

WORKLOADS = {
    "c1": dict(desc="2D homogeneous 129x129 nodes (128^2 cells), kappa=1, 10 ppw, gamma=0.01*omega, "
                    "ABC, shift 0.1, 4-level V(1,1), Full 3x3 Vanka, FGMRES(20), complex128",
               dim=2, n=(129, 129), levels=4, alpha=0.1, medium="homogeneous", seed=0,
               precision=0, restart=20, damping=[0.94, 1.2, 0.4, 0.6], smoother="symmetric",
               sample=dict(n=(129, 129), levels=4)),
    "c2": dict(desc="2D layered 1025x1025 nodes (1024^2 cells), 8-14 layers kappa in [0.25,1] + "
                    "5% smooth noise, 10 ppw at kappa_max, gamma=0.01*omega, ABC, shift 0.1, "
                    "7-level V(1,1), Full 3x3 Vanka, FGMRES(20), complex128",
               dim=2, n=(1025, 1025), levels=7, alpha=0.1, medium="layered_2d", seed=2,
               precision=0, restart=20, damping=[0.94, 1.2, 0.4, 0.6], smoother="symmetric",
               sample=dict(n=(1025, 1025), levels=7)),
    "c4": dict(desc="2D layered 513x513 nodes (512^2 cells), recipe of c2 with seed 4, 64 point "
                    "sources at row 2, columns 4+8k; one shared hierarchy, shift 0.2, 6-level "
                    "V(1,1), Full 3x3 Vanka, sources batched through every V-cycle sweep, "
                    "complex64 preconditioner, FGMRES(20) per source in complex128",
               dim=2, n=(513, 513), levels=6, alpha=0.2, medium="layered_2d", seed=4,
               precision=1, restart=20, damping=[0.94, 1.2, 0.4, 0.6], nsrc=64, batch=1,
               sample=dict(n=(513, 513), levels=6)),
    "c3": dict(desc="3D geophysical 257^3 nodes (256^3 cells), v in [1.5,4.5] km/s with dipping "
                    "layers and a 5 km/s ellipsoid, 10 ppw, gamma=0.01*omega, ABC, shift 0.5, "
                    "6-level trilinear V(1,1), Full 3x3x3 Vanka, complex64 preconditioner, "
                    "FGMRES(30) in complex128",
               dim=3, n=(257, 257, 257), levels=6, alpha=0.5, medium="geophysical_3d", seed=3,
               precision=1, restart=30, damping=[1.08, 0.5, 1.0, 0.4], smoother="symmetric",
               sample=dict(n=(65, 65, 65), levels=4)),
    "p2": dict(desc="the paper's own 2D configuration scaled to 1025x1025 nodes: kappa^2 linear in "
                    "depth over [0.25, 1] (Table heterogeneous2D model), 10 ppw at kappa_max, gamma = 0, "
                    "20-cell absorbing layer, compact 4th-order stencil, RB patch, level-dependent "
                    "intergrid, shift 0.25, 6-level V(1,1), GMRES(5), complex128",
               dim=2, n=(1025, 1025), levels=6, alpha=0.25, medium="linear", seed=0,
               precision=0, restart=5, damping=[0.83, 0.5, 0.4, 0.65], stencil="compact4",
               patch="rb", gamma0=0.0, sample=dict(n=(513, 513), levels=5)),
    "p3": dict(desc="the paper's own 3D configuration on the c3 medium: 257^3 nodes, compact "
                    "4th-order 19-point stencil, Element patch (per-patch inverses, 64 entries per "
                    "node), trilinear intergrid, gamma = 0, "
                    "20-cell absorbing layer, shift 0.4, 6-level V(1,1), complex64 preconditioner, "
                    "FGMRES(20) in complex128",
               dim=3, n=(257, 257, 257), levels=6, alpha=0.4, medium="geophysical_3d", seed=3,
               precision=1, restart=20, damping=[1.1, 0.7, 0.45, 0.6], stencil="compact4",
               patch="element", gamma0=0.0, smoother="patch", sample=dict(n=(65, 65, 65), levels=4)),
    "p3c": dict(desc="p3 with the paper's combined smoother (Sec. 5.5, Sec. 6): damped Jacobi on the "
                     "fine level, Element-patch Vanka on the coarser levels; 257^3 nodes, compact "
                     "stencil, trilinear, gamma = 0, shift 0.4, 6-level V(1,1), complex64 "
                     "preconditioner, FGMRES(20) in complex128",
                dim=3, n=(257, 257, 257), levels=6, alpha=0.4, medium="geophysical_3d", seed=3,
                precision=1, restart=20, damping=[0.6, 0.7, 0.45, 0.6], stencil="compact4",
                patch="element", fine_patch="point", gamma0=0.0, smoother="patch",
                sample=dict(n=(65, 65, 65), levels=4)),
}
DEFAULT_WORKLOAD = "c3"
PATCHES = {"full": 0, "point": 1, "plus": 3, "rb": 4, "element": 5}

SERVE_DESC = ("serving mix: Poisson arrivals; 70% 2D grids uniform over {257,513,1025,2049}^2 nodes, "
              "30% 3D over {97,129,193}^3; seeded layered media per request, 8-12 ppw, "
              "gamma=0.01*omega, ABC; 1-16 sources each (batched); complex64 preconditioner, "
              "FGMRES in complex128; admission by HBM footprint")


def serve_specs(count, seed, solves=None):
    """Seeded request mix: grid, levels, shift, restart, ppw and source count of each
    request (the media are generated later, one request at a time).  With `solves`, as
    many requests as it takes for their sources to reach that many solves."""
    import numpy as np
    rng = np.random.default_rng(seed)
    specs = []
    total = 0
    r = 0
    while (total < solves) if solves else (r < count):
        if rng.uniform() < 0.7:
            nn = int(rng.choice([257, 513, 1025, 2049]))
            n = (nn, nn)
            levels = {257: 5, 513: 6, 1025: 7, 2049: 8}[nn]
            shift, restart = 0.2, 20
        else:
            nn = int(rng.choice([97, 129, 193]))
            n = (nn, nn, nn)
            levels = {97: 4, 129: 5, 193: 5}[nn]
            shift, restart = 0.5, 30
        ppw = float(rng.uniform(8.0, 12.0))
        nsrc = int(rng.integers(1, 17))
        if solves:
            nsrc = min(nsrc, solves - total)
        specs.append(dict(r=r, n=n, levels=levels, shift=shift, restart=restart, ppw=ppw,
                          nsrc=nsrc))
        total += nsrc
        r += 1
    return specs


def serve_media(spec):
    """Seeded medium (c2 recipe in 2D, c3 recipe in 3D) and sources of one request."""
    import numpy as np
    import synth
    n, r = spec["n"], spec["r"]
    kappa = synth.layered_2d(n, 1000 + r) if len(n) == 2 else synth.geophysical_3d(n, 1000 + r)
    nn = n[0]
    h = 1.0 / (nn - 1)
    omega = synth.omega_for_ppw(h, spec["ppw"], float(kappa.max()))
    q = synth.random_sources(n, spec["nsrc"], seed=1000 + r, margin=min(22, nn // 4))
    return dict(spec, dim=len(n), h=h, omega=omega, kappa=kappa.ravel(),
                gamma=0.01 * omega * np.ones(kappa.size), q=q)


def serve_bench(args):
    """Serving workload: requests submitted at Poisson arrival times to one server.  A
    producer thread generates the media a few requests ahead of their arrival, and a
    fetcher thread collects the results in submission order while later requests arrive."""
    import queue
    import threading
    import numpy as np
    import torch
    from paper_2511_16808_amd import binding as B
    specs = serve_specs(args.requests, 5, args.solves)
    rng = np.random.default_rng(5)
    arrivals = np.cumsum(rng.exponential(1.0 / args.rate, size=len(specs)))
    arrivals -= arrivals[0]
    args.smoother = args.smoother or "assembled"
    smoother = B.VH_SMOOTHER_ASSEMBLED if args.smoother == "assembled" else B.VH_SMOOTHER_PATCH
    opts = {rs: B.make_options(precision=B.VH_PREC_C64, batch=1, restart=rs, smoother=smoother)
            for rs in (20, 30)}
    ready = queue.Queue(maxsize=4)

    def produce():
        for sp in specs:
            ready.put(serve_media(sp))
    threading.Thread(target=produce, daemon=True).start()
    torch.cuda.synchronize()
    srv = B.vh_server_create(int(args.budget_gib * (1 << 30)), args.slots)
    submitted = queue.Queue()
    results = []

    def fetch():
        while True:
            item = submitted.get()
            if item is None:
                return
            t, nsrc, N = item
            st, _, stats, lat, qm = B.vh_server_result(srv, t, N, nsrc, want_u=False)
            results.append((st, [x["iterations"] for x in stats], lat, qm, nsrc))
            if len(results) % 10 == 0:
                print(f"c5: {len(results)} of {len(specs)} requests done", file=sys.stderr,
                      flush=True)
    fetcher = threading.Thread(target=fetch)
    fetcher.start()
    t0 = time.perf_counter()
    late = 0.0
    for ta in arrivals:
        r = ready.get()
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        else:
            late = max(late, now - ta)
        t = B.vh_server_submit(srv, r["dim"], r["n"], r["h"], r["omega"], r["kappa"], r["gamma"],
                               r["shift"], r["levels"], B.VH_PATCH_FULL, r["q"], r["nsrc"], 1e-6,
                               opts[r["restart"]])
        submitted.put((t, r["nsrc"], int(np.prod(r["n"]))))
        del r
    submitted.put(None)
    fetcher.join()
    makespan = time.perf_counter() - t0
    info = B.vh_server_get_info(srv)
    B.vh_server_destroy(srv)
    lat = np.array([x[2] for x in results])
    qms = np.array([x[3] for x in results])
    its = [i for x in results for i in x[1]]
    nsol = sum(x[4] for x in results)
    ok = sum(int(x[0] == B.VH_OK) for x in results)
    out = {
        "metric": METRIC, "value": nsol / makespan, "unit": "solves/s", "n_gpus": 1,
        "steps": len(specs), "warmup": 0, "ms_per_step": 1e3 * makespan / len(specs),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64+c128",
        "data": "synthetic",
        "config": {"workload": "c5: " + SERVE_DESC, "requests": len(specs), "sources": nsol,
                   "arrival_rate_per_s": args.rate, "slots": args.slots,
                   "hbm_budget_gib": args.budget_gib, "smoother": args.smoother},
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "queue_p50_ms": float(np.percentile(qms, 50)),
        "queue_p99_ms": float(np.percentile(qms, 99)), "makespan_s": makespan,
        "max_submit_delay_s": late,
        "requests_ok": ok, "iterations_mean": float(np.mean(its)),
        "peak_running": info["peak_running"], "peak_in_use_gib": info["peak_in_use"] / 2 ** 30,
    }
    print(json.dumps(out))


def make_medium(w, n=None):
    import numpy as np
    import synth
    n = tuple(n or w["n"])
    if w["medium"] == "homogeneous":
        kappa = synth.homogeneous(n)
    elif w["medium"] == "linear":
        kappa = synth.linear_kappa2(n, 0.25, 1.0)
    elif w["medium"] == "layered_2d":
        kappa = synth.layered_2d(n, w["seed"])
    else:
        kappa = synth.geophysical_3d(n, w["seed"])
    h = 1.0 / (n[0] - 1)
    omega = synth.omega_for_ppw(h, 10.0, float(kappa.max()))
    gamma = w.get("gamma0", 0.01 * omega) * np.ones_like(kappa)
    nsrc = w.get("nsrc", 1)
    if nsrc == 1:
        q = synth.point_source(n).ravel()
    else:
        q = np.zeros((nsrc, int(np.prod(n))), dtype=complex)
        for k in range(nsrc):
            q[k] = synth.point_source(n, (4 + 8 * k, 2)).ravel()
        q = q.ravel()
    return n, h, omega, kappa, gamma, q


def kernel_sha(kernel):
    """Hash of the source text of one kernel template (from its declaration to the end
    of its body); counter-measured traffic is only reported for an unchanged kernel."""
    import hashlib
    fname = ("vh_mfma.hip" if kernel == "kb_sweep_mfma" else
             "vh_batch.hip" if kernel.startswith("kb_") else "vh_kernels.hip")
    src = open(os.path.join(ROOT, "paper_2511_16808_amd", "csrc", fname)).read()
    a = src.find(f"void {kernel}(")
    if a < 0:
        return None
    a = src.rfind("template", 0, a)
    b = src.find("\n}\n", a)
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def measured_traffic(key, kernel):
    """HBM bytes per launch of the dominant kernel from profiles/traffic.json (two
    calibrated rocprofv3 counter runs), or None if absent or taken on other code."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(key)
    if not rec or rec.get("kernel_sha") != kernel_sha(kernel):
        return None
    return rec["traffic"]


def vcycle_bytes(levels_info, dim, esz, smoother_entries, S=1):
    """Algorithmic HBM bytes of one V(1,1) cycle for S sources sharing it: every
    coefficient and smoother array read once per sweep, every vector of the S sources
    touched once per kernel."""
    total = 0
    L = len(levels_info)
    for l, info in enumerate(levels_info):
        N = 1
        for k in info["n"][:dim]:
            N *= k
        if l == L - 1:
            total += N * N * 16 + 2 * N * S * esz
            break
        Nc = 1
        for k in levels_info[l + 1]["n"][:dim]:
            Nc *= k
        K, E = info["stencil_points"], smoother_entries[l]
        if l == 0 and K == 2 * dim + 1:
            K = 1  # 5/7-point operator: only the centre entries are read (fixed off-diagonals)
        # a residual formed inside the sweep is neither stored nor read back (3 vectors
        # fewer); inside the restriction, 2 fewer
        vec = 15 - 3 * info.get("fused_sweep", 0) - 2 * info.get("fused_restrict", 0)
        total += N * esz * (2 * E + 2 * K) + N * S * esz * vec + Nc * S * esz * 2
    return total


def cpu_info():
    """CPU model (from /proc/cpuinfo) and os.cpu_count() of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_threads():
    """Threads for the multi-threaded oracle run: the host's CPU share for one GPU (the
    OMP_NUM_THREADS the environment sets, else the core count), at most 16."""
    env = os.environ.get("OMP_NUM_THREADS")
    n = int(env) if env and env.isdigit() else (os.cpu_count() or 1)
    return max(1, min(n, 16))


def _oracle_sample(key, sample_n, levels, threads, nsrc_sample=1):
    """Runs the FP64 oracle (setup + 2 FGMRES iterations per sampled source) in a child
    process with the given BLAS/OpenMP thread count; returns its timings."""
    code = f"""
import json, sys, time
sys.path.insert(0, {ROOT!r})
import numpy as np
from bench import WORKLOADS, make_medium
from oracle import discretization as D, cycle, krylov
w = WORKLOADS[{key!r}]
n, h, omega, kappa, gamma, q = make_medium(w, {tuple(sample_n)!r})
q = np.asarray(q).reshape(w.get('nsrc', 1), -1)
t0 = time.perf_counter()
ops = D.operator(w.get('stencil', 'fd2'), n, h, omega, kappa, gamma, w['alpha'])
patch = w.get('patch', 'full')
if w.get('fine_patch'):
    patch = [w['fine_patch']] + [patch] * ({levels} - 2)
mg = cycle.Multigrid(ops['Hs'], n, {levels}, 'levdep' if len(n) == 2 else 'linear',
                     patch, w['damping'])
t1 = time.perf_counter()
its = 2
picks = np.linspace(0, q.shape[0] - 1, {nsrc_sample}).round().astype(int)
for k in picks:
    krylov.fgmres(lambda v: ops['H'] @ v, mg.apply, q[k], 1e-30, w['restart'], its)
t2 = time.perf_counter()
print(json.dumps(dict(setup_s=t1 - t0, iter_s=(t2 - t1) / (its * len(picks)), N=int(np.prod(n)),
                      sources=[int(k) for k in picks])))
"""
    t = str(threads)
    env = dict(os.environ, OMP_NUM_THREADS=t, OPENBLAS_NUM_THREADS=t, MKL_NUM_THREADS=t)
    t0 = time.perf_counter()
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=600)
    wall = time.perf_counter() - t0
    if out.returncode != 0:
        return {"error": out.stderr[-400:]}
    r = json.loads(out.stdout.strip().splitlines()[-1])
    r["wall_s"] = wall
    return r


def cpu_baseline(w, gpu_iterations):
    """The FP64 oracle timed on this host on a reduced sample of the same recipe: setup +
    2 FGMRES iterations per sampled source, once single-threaded and once with the host's
    thread share, extrapolated linearly in nodes to the full grid and to the GPU's
    iteration count summed over the sources (one setup, then one solve per source).  The
    reported value is the faster of the two runs."""
    sample = w["sample"]
    nsrc = w.get("nsrc", 1)
    nsamp = min(nsrc, 4)
    model, ncpu = cpu_info()
    Nfull = 1
    for k in w["n"]:
        Nfull *= k
    runs = {}
    for threads in sorted({1, cpu_threads()}):
        r = _oracle_sample(w["key"], sample["n"], sample["levels"], threads, nsamp)
        if "error" in r:
            return r
        scale = Nfull / r["N"]
        t_solve = scale * (r["setup_s"] + gpu_iterations * r["iter_s"])
        runs[threads] = dict(value=nsrc / t_solve, setup_s=r["setup_s"], iter_s=r["iter_s"],
                             scale=scale, wall_s=r["wall_s"], sources=r["sources"])
    best = max(runs, key=lambda t: runs[t]["value"])
    rb = runs[best]
    return {
        "value": rb["value"], "unit": "solves/s", "cores": best, "kind": "oracle",
        "cpu_model": model, "cpu_count": ncpu,
        "threads": {str(t): {"value": x["value"], "setup_s": x["setup_s"], "iter_s": x["iter_s"]}
                    for t, x in runs.items()},
        "extrapolated": True,
        "sample": (f"oracle setup + 2 FGMRES iterations on the same recipe at "
                   f"{'x'.join(map(str, sample['n']))} nodes ({sample['levels']} levels)"
                   f"{', sources ' + str(rb['sources']) + ' of ' + str(nsrc) if nsrc > 1 else ''}, "
                   f"setup {rb['setup_s']:.1f}s, {rb['iter_s']:.2f}s/iteration, extrapolated "
                   f"x{rb['scale']:.1f} in nodes and to {gpu_iterations} iterations"
                   f"{' summed over ' + str(nsrc) + ' sources' if nsrc > 1 else ''}; "
                   f"runs at {', '.join(str(t) for t in runs)} thread(s), value from {best}; "
                   f"NumPy elementwise and SciPy sparse work is single-threaded; "
                   f"{sum(x['wall_s'] for x in runs.values()):.1f}s of CPU work"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS) + ["c5"])
    ap.add_argument("--requests", type=int, default=32, help="c5: number of requests")
    ap.add_argument("--solves", type=int, default=None,
                    help="c5: requests until their sources total this many solves "
                         "(overrides --requests)")
    ap.add_argument("--rate", type=float, default=2.0, help="c5: Poisson arrival rate (1/s)")
    ap.add_argument("--slots", type=int, default=4, help="c5: concurrent requests")
    ap.add_argument("--budget-gib", type=float, default=240.0, help="c5: HBM budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--c4-steps", type=int, default=5,
                    help="with the default workload: timed steps of the 64-source 513^2 "
                         "workload reported in the same line (0: skip)")
    ap.add_argument("--smoother", default=None, choices=["patch", "assembled", "symmetric"],
                    help="additive Vanka applied as stored patch inverses or as the same "
                         "operator assembled into a 5^d-point stencil (default: assembled, "
                         "unless the workload names its form)")
    ap.add_argument("--contraction", default="valu", choices=["valu", "mfma_f32", "mfma_bf16x3"],
                    help="batched per-patch smoother on the vector ALUs or the matrix cores "
                         "(implies --smoother patch)")
    ap.add_argument("--batch", type=int, default=None, choices=[0, 1],
                    help="override: sources one after another (0) or sharing each sweep (1)")
    ap.add_argument("--precision", default=None, choices=["c128", "c64"],
                    help="override the preconditioner precision")
    ap.add_argument("--sweep-tile", type=int, default=0,
                    help="64-source 2D walk variant (1..10; 0: timed per grid)")
    ap.add_argument("--sym-planes", type=int, default=0,
                    help="3D symmetric-half sweep: planes per workgroup (2..64; -1: one "
                         "plane per workgroup; 0: chosen from the grid)")
    ap.add_argument("--setup-pivot", type=int, default=0, choices=[0, 1],
                    help="1: partial pivoting in every patch inversion (0: none where the "
                         "patch matrices are complex symmetric with a positive definite "
                         "imaginary part)")
    ap.add_argument("--split-residual", action="store_true",
                    help="separate residual launches instead of the residual formed inside "
                         "the sweep and the restriction (same results)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(sharding across GPUs is not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2511_16808_amd import binding as B

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "c5":
        serve_bench(args)
        return
    if args.copy_probe_mib > 0:
        # one elementwise kernel that reads and writes exactly MiB << 20 bytes each
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    ceiling = copy_ceiling()
    out = run_workload(args.workload, args.steps, args.warmup, args.smoother, args.contraction,
                       args.batch, args.precision, not args.no_cpu_baseline,
                       args.split_residual, args.sweep_tile, args.sym_planes, args.setup_pivot)
    out["roofline"].update(ceiling_fields(out["roofline"], ceiling))
    if args.workload == DEFAULT_WORKLOAD and args.c4_steps > 0:
        # the 512^2 half of the metric: 64 sources through one hierarchy, timed after the
        # 256^3 steps (its own warm-up, steps, roofline and CPU baseline)
        c4 = run_workload("c4", args.c4_steps, 1, None, "valu", None, None,
                          not args.no_cpu_baseline, args.split_residual, args.sweep_tile)
        c4["roofline"].update(ceiling_fields(c4["roofline"], ceiling))
        out["c4"] = {k: c4[k] for k in ("metric", "value", "unit", "steps", "warmup",
                                        "ms_per_step", "dtype", "config", "iterations",
                                        "converged", "true_relres", "setup_ms", "solve_ms",
                                        "p50_ms", "p99_ms", "vcycle_ms", "vcycle_GBps",
                                        "vcycle_algorithmic_bytes", "bytes_moved_per_step",
                                        "solve_GBps", "c_f", "roofline", "cpu_baseline")
                     if k in c4}
    print(json.dumps(out))


def copy_ceiling(mib=2048, reps=5):
    """HBM rate a plain elementwise copy reaches on this GPU: out = in + 1 over `mib` MiB
    read and `mib` MiB written, timed with events on the current stream (best of reps)."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.add(src, 1.0, out=dst)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.add(src, 1.0, out=dst)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (mib << 20) / (best * 1e-3) / 1e9


def ceiling_fields(roof, ceiling):
    """The measured copy rate next to the spec peak, and the kernel's fraction of it."""
    if roof.get("unit") != "GB/s" or not ceiling:
        return {"copy_GBps": ceiling}
    return {"copy_GBps": ceiling,
            "frac_of_copy": (roof["achieved"] / ceiling) if roof.get("achieved") else None}


def run_workload(key, steps, warmup, smoother_name, contraction_name, batch_o, precision_o,
                 with_cpu, split=False, sweep_tile=0, sym_planes=0, setup_pivot=0):
    """Times `steps` whole passes (setup + solve + destroy) of one workload after `warmup`
    untimed ones; returns the JSON object of the benchmark line."""
    import numpy as np
    import torch
    from paper_2511_16808_amd import binding as B

    class _A:
        pass
    args = _A()
    args.workload, args.steps, args.warmup = key, steps, warmup
    args.smoother, args.contraction, args.batch, args.precision = (smoother_name, contraction_name,
                                                                    batch_o, precision_o)
    args.split_residual = split
    args.sweep_tile = sweep_tile
    w = dict(WORKLOADS[args.workload], key=args.workload)
    if args.smoother is None:
        args.smoother = w.get("smoother", "assembled")
    n, h, omega, kappa, gamma, q = make_medium(w)
    dim = w["dim"]
    N = int(np.prod(n))
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    kt = torch.tensor(kappa.ravel(), dtype=torch.float64, device=dev)
    gt = torch.tensor(gamma.ravel(), dtype=torch.float64, device=dev)
    qt = torch.tensor(q, dtype=torch.complex128, device=dev)
    ut = torch.empty_like(qt)
    contraction = {"valu": B.VH_CONTRACT_VALU, "mfma_f32": B.VH_CONTRACT_MFMA_F32,
                   "mfma_bf16x3": B.VH_CONTRACT_MFMA_BF16X3}[args.contraction]
    if contraction != B.VH_CONTRACT_VALU:
        args.smoother = "patch"  # the matrix-core sweep applies the stored patch inverses
    smoother = {"assembled": B.VH_SMOOTHER_ASSEMBLED, "symmetric": B.VH_SMOOTHER_SYMMETRIC,
                "patch": B.VH_SMOOTHER_PATCH}[args.smoother]
    nsrc = w.get("nsrc", 1)
    batch = w.get("batch", 0) if args.batch is None else args.batch
    precision = w["precision"] if args.precision is None else {"c128": 0, "c64": 1}[args.precision]
    patch = PATCHES[w.get("patch", "full")]
    stencil = B.VH_STENCIL_COMPACT4 if w.get("stencil") == "compact4" else B.VH_STENCIL_FD2
    opt = B.make_options(precision=precision, restart=w["restart"], damping=w["damping"],
                         intergrid=B.VH_IG_LEVDEP if dim == 2 else B.VH_IG_LINEAR, stencil=stencil,
                         smoother=smoother, stream=stream, timing=1, batch=batch,
                         contraction=contraction, split_residual=int(args.split_residual),
                         sweep_tile=args.sweep_tile, sym_planes=sym_planes,
                         setup_pivot=setup_pivot)
    if w.get("fine_patch"):
        opt.fine_patch = PATCHES[w["fine_patch"]]
    torch.cuda.synchronize()

    def step():
        t0 = time.perf_counter()
        hd = B.vh_setup(dim, n, h, omega, kt, gt, w["alpha"], w["levels"], patch, opt)
        t1 = time.perf_counter()
        st, stats = B.vh_solve(hd, qt, nsrc, 1e-6, ut)
        info = [B.vh_get_level_info(hd, l) for l in range(w["levels"])]
        B.vh_destroy(hd)
        t2 = time.perf_counter()
        return dict(status=st, stats=stats[0], all_stats=stats, setup_ms=1e3 * (t1 - t0),
                    step_ms=1e3 * (t2 - t0), info=info)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    last = runs[-1]
    st = last["stats"]
    esz = 16 if precision == 0 else 8
    its_all = [x["iterations"] for x in last["all_stats"]]
    S = 1
    while S < nsrc:
        S *= 2
    width = S if batch else 1   # sources per sweep launch
    info = last["info"]
    E = [i["smoother_entries"] for i in info]
    if args.smoother == "symmetric":
        # entries stored per node: the symmetric half (5^d + 1) / 2 on every level whose
        # operator is symmetric (3D trilinear: all; 2D level-dependent: the two finest)
        E = [(e + 1) // 2 if (dim == 3 or l < 2) else e for l, e in enumerate(E)]
    # dominant kernel: finest-level additive-Vanka sweep u += B r
    n_l = sum(r["stats"]["smooth1_launches"] for r in runs)
    ms_l = sum(r["stats"]["smooth1_ms"] for r in runs)
    fused0 = width == 1 and info[0].get("fused_sweep", 0) == 1
    if fused0:
        # u_out = u_in + B (q - A u_in): the smoother entries, the operator's coefficients
        # (the centre entries of the 5/7-point finest operator) and q, u_in, u_out
        K0 = 1 if info[0]["stencil_points"] == 2 * dim + 1 else info[0]["stencil_points"]
        bytes_per_launch = N * esz * (E[0] + K0 + 3)
    else:
        bytes_per_launch = N * esz * (E[0] + 3 * width)
    achieved = bytes_per_launch / (ms_l / n_l * 1e-3) / 1e9 if n_l else None
    if width == 1 and info[0].get("sym_planes", 0) > 0:
        kname = "k_vanka_sweep_sym3z"  # the 3D symmetric half walked along z
    elif width == 1:
        kname = "k_vanka_sweep_sym" if args.smoother == "symmetric" else "k_vanka_sweep"
    elif contraction != B.VH_CONTRACT_VALU and width >= 16:
        kname = "kb_sweep_mfma"
    elif dim == 2 and width == 64 and E[0] == 25:
        # the variant the tile tuner chose for the finest level (1: the LDS walk)
        kname = "kb_sweep2d_s64" if info[0].get("sweep_tile", 0) == 1 else "kb_walk2d_s64"
    elif dim == 2:
        kname = "kb_sweep2d_wide" if width >= 16 else "kb_sweep2d"
    else:
        kname = "kb_sweep"
    tkey = f"{args.workload}_{'batch_' + args.contraction if batch else args.smoother}"
    traffic = measured_traffic(tkey, kname)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBPS) if achieved else None}
    if kname == "kb_sweep_mfma":
        # the dense contraction: useful flop = 8 * 81 * S real flop per patch (complex 9x9
        # times 9xS); peak of the contraction's own dtype (dense, no sparsity)
        peak = 2500.0 if args.contraction == "mfma_bf16x3" else 157.3
        flops = 8.0 * 81 * width * N
        tf = flops / (ms_l / n_l * 1e-3) / 1e12 if n_l else None
        roof = {"bound": "mfma", "achieved": tf, "peak": peak, "unit": "TFLOP/s",
                "frac": (tf / peak) if tf else None, "hbm_GBps": achieved}
    vc_b = vcycle_bytes(info, dim, esz, E, width)
    vc_n = sum(r["stats"]["vcycles"] for r in runs)
    vc_ms = sum(r["stats"]["vcycle_ms"] for r in runs)
    lat = np.array([r["step_ms"] for r in runs])
    # algorithmic bytes of one step's solve (a batch of up to 64 sources reports its total
    # in each source's stats) and the solve's whole-kernel-sequence rate
    groups = last["all_stats"][::64] if batch else last["all_stats"]
    moved = float(sum(x["bytes_moved"] for x in groups))
    solve_ms = float(sum(x["solve_ms"] for x in groups))
    cfs = [x["c_f"] for x in last["all_stats"] if x["c_f"] == x["c_f"]]
    out = {
        "metric": METRIC,
        "value": nsrc * args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if precision == 0 else "c64+c128",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w['desc']}", "nodes": N, "levels": w["levels"],
                   "smoother": args.smoother, "sources": nsrc, "batched": bool(batch),
                   "contraction": args.contraction},
        "iterations": st["iterations"] if nsrc == 1 else
        {"mean": float(np.mean(its_all)), "min": int(min(its_all)), "max": int(max(its_all))},
        "converged": all(x["converged"] for x in last["all_stats"]) and
        all(r["status"] == 0 for r in runs),
        "true_relres": max(x["relres"] for x in last["all_stats"]),
        "setup_ms": float(np.median([r["setup_ms"] for r in runs])),
        "solve_ms": float(np.median([r["stats"]["solve_ms"] for r in runs])),
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "vcycle_ms": vc_ms / vc_n if vc_n else None,
        "vcycle_GBps": (vc_b / (vc_ms / vc_n * 1e-3) / 1e9) if vc_n else None,
        "vcycle_algorithmic_bytes": vc_b,
        "bytes_moved_per_step": moved,
        "solve_GBps": moved / (solve_ms * 1e-3) / 1e9 if solve_ms > 0 else None,
        "c_f": (float(np.mean(cfs)) if cfs else None),
        # per smoothed level: [residual formed in the sweep, in the restriction]
        "fused": [[i.get("fused_sweep", 0), i.get("fused_restrict", 0)] for i in info[:-1]],
        "roofline": {
            **roof,
            "kernel": ("finest-level additive Vanka sweep u += B (q - A u), residual formed "
                       "in the sweep" if fused0 else "finest-level additive Vanka sweep u += B r")
                      + f" ({kname}, {width} source(s)"
                      + (f", tile {info[0]['sweep_tile']}" if info[0].get("sweep_tile") else "") + ")",
            "traffic": traffic,
            "bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": ms_l / n_l if n_l else None,
            "launches": n_l,
        },
    }
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline(w, int(sum(its_all)))
    return out




if __name__ == "__main__":
    main()
