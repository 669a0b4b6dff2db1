"""Oracle: multigrid cycles (TEST INFRASTRUCTURE ONLY).

Paper Sec. 2.2, Algorithm "Two-grid cycle": nu1 pre-relaxations, restricted
residual r_H = R(q - A u), coarse solve, u += P e_H, nu2 post-relaxations.  A
V-cycle replaces the coarse solve by one recursive cycle, a W-cycle by two.  The
coarsest system is solved directly (Sec. 1, Sec. 5.4 LU), here with
scipy.linalg.lu_factor.  Relaxation is the damped additive Vanka smoother of
eq. (smoother) with a damping w_l per level (Table "relaxParam").  The patch may be
one kind for every level or one per level: Sec. 5.5, Sec. 6 combine damped Jacobi (the
point patch) on the fine level with Element-patch Vanka on the coarser levels.
"""
import numpy as np
import scipy.linalg as sla

from .hierarchy import Hierarchy
from .vanka import AdditiveVanka


class Multigrid:
    """Multigrid preconditioner for the shifted operator A0 = H_s."""

    def __init__(self, A0, n, levels, scheme, patch, damping, nu1=1, nu2=1,
                 cycle="V", periodic=False):
        self.h = Hierarchy(A0, n, levels, scheme, periodic)
        self.nu1, self.nu2 = nu1, nu2
        self.cycle_type = cycle
        L = self.h.levels
        damping = list(damping)
        while len(damping) < L - 1:
            damping.append(damping[-1])
        self.damping = damping[: max(L - 1, 0)]
        patches = [patch] * max(L - 1, 0) if isinstance(patch, str) else list(patch)
        self.smoothers = [AdditiveVanka(self.h.A[l], self.h.n[l], patches[l])
                          for l in range(L - 1)]
        self.coarse_lu = sla.lu_factor(self.h.A[-1].toarray())

    @property
    def levels(self):
        return self.h.levels

    def relax(self, l, q, u):
        """One damped additive Vanka step: u + w_l B_l (q - A_l u)."""
        r = q - self.h.A[l] @ u
        return u + self.damping[l] * self.smoothers[l].apply(r)

    def cycle(self, l, q, u):
        """u <- Cycle(A_l, q, u)."""
        if l == self.levels - 1:
            return sla.lu_solve(self.coarse_lu, q)
        for _ in range(self.nu1):
            u = self.relax(l, q, u)
        rH = self.h.R[l] @ (q - self.h.A[l] @ u)
        eH = np.zeros(rH.shape[0], dtype=complex)
        visits = 2 if (self.cycle_type == "W" and l + 1 < self.levels - 1) else 1
        for _ in range(visits):
            eH = self.cycle(l + 1, rH, eH)
        u = u + self.h.P[l] @ eH
        for _ in range(self.nu2):
            u = self.relax(l, q, u)
        return u

    def apply(self, v):
        """Preconditioner M^{-1} v = one cycle from a zero initial guess."""
        v = np.asarray(v, dtype=complex)
        return self.cycle(0, v, np.zeros_like(v))
