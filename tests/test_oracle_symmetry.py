"""The property the symmetric smoother storage rests on, checked on the oracle: the
5/7-point H_s (absorbing rows scaled by 1/2 per boundary direction) is complex symmetric,
Galerkin levels built with R and P of one family stay symmetric (R = c P^T, Sec. 3.1),
and the additive Vanka operator of such a level (Sec. 3.2, 3.3) is B = D S with S
symmetric, D = diag(1/cnt_i).  A mixed transfer (linear R, cubic P) breaks it, which is
why the library keeps the full stencil below one.  The compact stencil in a
heterogeneous medium is not symmetric either."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import discretization as D
from oracle.hierarchy import Hierarchy
from oracle.vanka import AdditiveVanka


def asym(A):
    A = sp.csr_matrix(A)
    return abs(A - A.T).max() / abs(A).max()


def medium(n, seed):
    kappa = np.random.default_rng(seed).uniform(0.4, 1.0, size=tuple(reversed(n)))
    h = 1.0 / (n[0] - 1)
    omega = synth.omega_for_ppw(h, 10.0, float(kappa.max()))
    return h, omega, kappa, 0.01 * omega * np.ones_like(kappa)


@pytest.mark.parametrize("n,bc", [((17, 13), "abc"), ((9, 13, 9), "abc"), ((9, 9, 9), "dirichlet")])
def test_fd2_shifted_operator_and_same_family_galerkin_levels_are_symmetric(n, bc):
    h, omega, kappa, gamma = medium(n, 1)
    ops = D.fd2_operator(n, h, omega, kappa, gamma, 0.4, bc=bc, sponge_width=3)
    assert asym(ops["Hs"]) < 1e-15
    scheme = "linear" if len(n) == 3 else "cubic"
    hier = Hierarchy(ops["Hs"], n, 3, scheme, False)
    for l in range(1, hier.levels):
        assert asym(hier.A[l]) < 1e-14, l


def test_mixed_transfer_and_compact_stencil_are_not_symmetric():
    n = (17, 17)
    h, omega, kappa, gamma = medium(n, 2)
    ops = D.fd2_operator(n, h, omega, kappa, gamma, 0.4, bc="abc", sponge_width=3)
    assert asym(Hierarchy(ops["Hs"], n, 2, "mixed", False).A[1]) > 1e-3
    c4 = D.compact4_operator(n, h, omega, kappa, gamma, 0.4, bc="sponge", sponge_width=3)
    assert asym(c4["Hs"]) > 1e-3


@pytest.mark.parametrize("n", [(11, 9), (7, 6, 5)])
def test_vanka_operator_is_diagonal_times_symmetric(n):
    h, omega, kappa, gamma = medium(n, 3)
    ops = D.fd2_operator(n, h, omega, kappa, gamma, 0.4, bc="abc", sponge_width=2)
    sm = AdditiveVanka(ops["Hs"], n, "full")
    Bd = sm.dense()
    S = sm.cnt[:, None] * Bd  # D^{-1} B
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    # the same fails for a non-symmetric operator (planted: one off-diagonal changed)
    A = sp.lil_matrix(ops["Hs"])
    A[0, 1] = 2.0 * A[0, 1]
    Sb = AdditiveVanka(A.tocsr(), n, "full")
    Sx = Sb.cnt[:, None] * Sb.dense()
    assert np.abs(Sx - Sx.T).max() > 1e-6 * np.abs(Sx).max()
