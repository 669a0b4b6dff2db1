"""Shared set-up for the GPU parity tests: one seeded problem, built once on the GPU
(through the C ABI) and once in the oracle, from the same synthetic inputs."""
import numpy as np
import scipy.sparse as sp

import synth
from oracle import cycle
from oracle import discretization as D


class Case:
    def __init__(self, n, levels, alpha=0.1, seed=0, medium="layered", ppw=10.0,
                 patch="full", precision=0, intergrid=None, damping=None, restart=20,
                 bc="abc", sponge_width=20, smoother=0, nu=(1, 1), stencil="fd2", gamma0=None,
                 cycle="V", fine_patch=None):
        self.n = tuple(n)
        self.dim = len(n)
        self.N = int(np.prod(n))
        self.h = 1.0 / (n[0] - 1)
        if medium == "layered" and self.dim == 2:
            self.kappa = synth.layered_2d(self.n, seed)
        elif medium == "layered":
            self.kappa = synth.geophysical_3d(self.n, seed)
        elif medium == "linear":
            self.kappa = synth.linear_kappa2(self.n, 0.25, 1.0)
        elif medium == "random":
            self.kappa = np.random.default_rng(seed).uniform(0.4, 1.0, size=tuple(reversed(n)))
        else:
            self.kappa = synth.homogeneous(self.n)
        self.omega = synth.omega_for_ppw(self.h, ppw, float(self.kappa.max()))
        g0 = 0.01 * self.omega if gamma0 is None else gamma0
        self.gamma = g0 * np.ones_like(self.kappa)
        self.stencil = stencil
        self.cycle = cycle
        self.fine_patch = fine_patch
        self.alpha = alpha
        self.levels = levels
        self.patch = patch
        self.precision = precision
        if intergrid is None:
            intergrid = "levdep" if self.dim == 2 else "linear"
        self.intergrid = intergrid
        if damping is None:
            damping = [0.94, 1.2, 0.4, 0.6] if self.dim == 2 else [1.08, 0.9, 0.6, 0.6]
        self.damping = list(damping)
        self.restart = restart
        self.bc = bc
        self.sponge_width = sponge_width
        self.smoother = smoother
        self.nu = nu
        self._oracle = None

    # ---- oracle side
    def oracle_ops(self):
        if self.stencil == "compact4":
            return D.compact4_operator(self.n, self.h, self.omega, self.kappa, self.gamma,
                                       self.alpha, bc="sponge" if self.bc == "abc" else "dirichlet",
                                       sponge_width=self.sponge_width)
        return D.fd2_operator(self.n, self.h, self.omega, self.kappa, self.gamma, self.alpha,
                              bc="abc" if self.bc == "abc" else "dirichlet",
                              sponge_width=self.sponge_width)

    def oracle(self):
        if self._oracle is None:
            ops = self.oracle_ops()
            patches = self.patch if self.fine_patch is None else \
                [self.fine_patch] + [self.patch] * (self.levels - 2)
            mg = cycle.Multigrid(ops["Hs"], self.n, self.levels, self.intergrid, patches,
                                 self.damping, nu1=self.nu[0], nu2=self.nu[1], cycle=self.cycle)
            self._oracle = (ops, mg)
        return self._oracle

    # ---- GPU side
    def gpu(self, **extra):
        from paper_2511_16808_amd import binding as B
        a = self.gpu_args(**extra)
        return B.vh_setup(self.dim, self.n, self.h, self.omega, a["kappa"], a["gamma"],
                          self.alpha, self.levels, a["patch"], a["opt"])

    def gpu_args(self, **extra):
        """kappa and gamma on the GPU, the patch code and the options of vh_setup."""
        import torch
        from paper_2511_16808_amd import binding as B
        ig = {"levdep": B.VH_IG_LEVDEP, "mixed": B.VH_IG_MIXED, "linear": B.VH_IG_LINEAR,
              "cubic": B.VH_IG_CUBIC}
        opt = B.make_options(precision=self.precision, restart=self.restart,
                             intergrid=ig[self.intergrid], damping=self.damping,
                             bc=B.VH_BC_ABC if self.bc == "abc" else B.VH_BC_DIRICHLET,
                             sponge_width=self.sponge_width, smoother=self.smoother,
                             nu1=self.nu[0], nu2=self.nu[1],
                             stencil=B.VH_STENCIL_COMPACT4 if self.stencil == "compact4"
                             else B.VH_STENCIL_FD2,
                             cycle=B.VH_CYCLE_W if self.cycle == "W" else B.VH_CYCLE_V,
                             stream=torch.cuda.current_stream(), **extra)
        kap = torch.tensor(self.kappa.ravel(), dtype=torch.float64, device="cuda")
        gam = torch.tensor(self.gamma.ravel(), dtype=torch.float64, device="cuda")
        kinds = {"full": B.VH_PATCH_FULL, "point": B.VH_PATCH_POINT, "plus": B.VH_PATCH_PLUS,
                 "rb": B.VH_PATCH_RB, "element": B.VH_PATCH_ELEMENT}
        patch = kinds[self.patch]
        if self.fine_patch is not None:
            opt.fine_patch = kinds[self.fine_patch]
        return {"kappa": kap, "gamma": gam, "patch": patch, "opt": opt}


def stencil_entries(A, n, offsets):
    """[K][N] array of A[i, i + off_k] (0 where the neighbour is outside the grid)."""
    A = sp.csr_matrix(A)
    dim = len(n)
    N = int(np.prod(n))
    coords = [c.ravel() for c in np.indices(tuple(reversed(n)))][::-1]
    out = np.zeros((len(offsets), N), dtype=complex)
    for k, off in enumerate(offsets):
        ok = np.ones(N, dtype=bool)
        j = np.zeros(N, dtype=np.int64)
        stride = 1
        for d in range(dim):
            x = coords[d] + off[d]
            ok &= (x >= 0) & (x < n[d])
            j += x * stride
            stride *= n[d]
        rows = np.flatnonzero(ok)
        out[k, rows] = np.asarray(A[rows, j[rows]]).ravel()
    return out


def rel(a, b):
    """Relative difference of a from b: the larger of the norm-wise ||a - b|| / ||b|| and
    the element-wise max |a_i - b_i| / max |b_i|, so that an error confined to a few
    nodes is not averaged away by the norm."""
    a, b = np.ravel(a), np.ravel(b)
    d = np.abs(a - b)
    norm = float(np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300))
    elem = float(d.max() / max(np.abs(b).max(), 1e-300)) if b.size else 0.0
    return max(norm, elem)
