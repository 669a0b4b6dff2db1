"""Object wrapper over the C ABI: owns one vh_handle and the torch tensors it needs."""
import torch

from . import binding as B


class HelmholtzSolver:
    """setup(grid, h, omega, kappa, gamma, shift, levels, patch) / solve(q, tol).

    kappa, gamma: float64 arrays (numpy or torch) of shape n[::-1] (x fastest);
    they are copied to the GPU once.  All work runs in libvh.so on `device`.
    """

    def __init__(self, n, h, omega, kappa, gamma=None, shift=0.1, levels=4,
                 patch=B.VH_PATCH_FULL, device="cuda:0", **options):
        if not torch.cuda.is_available():
            raise RuntimeError("HelmholtzSolver needs a GPU (HIP)")
        self.n = tuple(int(k) for k in n)
        self.dim = len(self.n)
        self.device = torch.device(device)
        self.N = 1
        for k in self.n:
            self.N *= k
        self.kappa = torch.as_tensor(kappa, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
        self.gamma = (None if gamma is None else
                      torch.as_tensor(gamma, dtype=torch.float64).reshape(-1).to(self.device).contiguous())
        if "stream" not in options:
            options["stream"] = torch.cuda.current_stream(self.device)
        self.options = B.make_options(**options)
        with torch.cuda.device(self.device):
            self.handle = B.vh_setup(self.dim, self.n, h, omega, self.kappa, self.gamma, shift,
                                     levels, patch, self.options)
        self.levels = levels

    def solve(self, q, tol=1e-6):
        """q: complex128 GPU tensor (nsrc, N) or (N,).  Returns (u, stats list)."""
        q = q.reshape(-1, self.N).contiguous()
        u = torch.empty_like(q)
        with torch.cuda.device(self.device):
            status, stats = B.vh_solve(self.handle, q, q.shape[0], tol, u)
        self.last_status = status
        return u, stats

    def vcycle(self, v):
        z = torch.empty_like(v)
        B.vh_apply_vcycle(self.handle, v.contiguous(), z)
        return z

    def apply(self, x, level=0, which=1):
        y = torch.empty_like(x)
        B.vh_apply_operator(self.handle, level, which, x.contiguous(), y)
        return y

    def close(self):
        if getattr(self, "handle", None) is not None:
            B.vh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
