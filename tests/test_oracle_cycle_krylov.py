"""Pins of the oracle's cycles (Algorithm 'Two-grid cycle', eq. (2G)) and of FGMRES."""
import numpy as np
import pytest

from oracle import cycle, krylov, lfa
from oracle import discretization as D
import synth


def small_problem(n=(9, 9), alpha=0.4, seed=7):
    rng = np.random.default_rng(seed)
    kappa = rng.uniform(0.5, 1.0, size=tuple(reversed(n)))
    return D.fd2_operator(n, 1 / (n[0] - 1), 18.0, kappa, 0.18, alpha=alpha, sponge_width=3)


def dense_of(op, N):
    return np.stack([op(e) for e in np.eye(N, dtype=complex)], axis=1)


def test_one_level_is_the_direct_solve():
    """P7: a 1-level 'cycle' is the coarsest direct solve, M^{-1} = H_s^{-1}."""
    ops = small_problem()
    mg = cycle.Multigrid(ops["Hs"], (9, 9), 1, "levdep", "full", [0.9])
    v = np.random.default_rng(0).standard_normal(81) + 0j
    assert np.allclose(mg.apply(v), np.linalg.solve(ops["Hs"].toarray(), v), rtol=1e-12)


def test_exact_preconditioner_converges_in_one_iteration():
    ops = small_problem(alpha=0.0)
    mg = cycle.Multigrid(ops["Hs"], (9, 9), 1, "levdep", "full", [0.9])
    q = synth.point_source((9, 9)).ravel()
    x, info = krylov.fgmres(lambda v: ops["H"] @ v, mg.apply, q, 1e-10, 20, 50)
    assert info["iterations"] == 1 and info["converged"]
    assert np.linalg.norm(q - ops["H"] @ x) <= 1e-10 * np.linalg.norm(q)


@pytest.mark.parametrize("nu", [(1, 1), (2, 1), (0, 2)])
def test_two_grid_error_operator(nu):
    """I - M^{-1} A_s equals eq. (2G): S^nu2 (I - P A_c^{-1} R A) S^nu1 with
    S = I - w B A (eq. (smoother)), B the dense additive-Vanka operator."""
    n = (9, 9)
    ops = small_problem(n)
    A = ops["Hs"].toarray()
    w = 0.8
    mg = cycle.Multigrid(ops["Hs"], n, 2, "levdep", "full", [w], nu1=nu[0], nu2=nu[1])
    M = dense_of(mg.apply, 81)
    B = mg.smoothers[0].dense()
    S = np.eye(81) - w * B @ A
    R, P = mg.h.R[0].toarray(), mg.h.P[0].toarray()
    K = np.eye(81) - P @ np.linalg.solve(R @ A @ P, R @ A)
    TG = np.linalg.matrix_power(S, nu[1]) @ K @ np.linalg.matrix_power(S, nu[0])
    assert np.allclose(np.eye(81) - M @ A, TG, atol=1e-10)


@pytest.mark.parametrize("ctype", ["V", "W"])
def test_three_level_cycle_recursion(ctype):
    """Three levels: the coarse solve of the two-grid operator is replaced by one (V)
    or two (W) cycles on level 2, i.e. A_c^{-1} -> (I - E^g) A_c^{-1} with E the
    level-2 two-grid error operator and g = 1 or 2 (Sec. 2.2)."""
    n = (17, 17)
    ops = small_problem(n, alpha=0.6)
    w = [0.9, 0.7]
    mg = cycle.Multigrid(ops["Hs"], n, 3, "levdep", "full", w, cycle=ctype)
    N = 289
    A0 = ops["Hs"].toarray()
    A1 = mg.h.A[1].toarray()
    A2 = mg.h.A[2].toarray()
    N1 = A1.shape[0]
    S0 = np.eye(N) - w[0] * mg.smoothers[0].dense() @ A0
    S1 = np.eye(N1) - w[1] * mg.smoothers[1].dense() @ A1
    R1, P1 = mg.h.R[1].toarray(), mg.h.P[1].toarray()
    E1 = S1 @ (np.eye(N1) - P1 @ np.linalg.solve(A2, R1 @ A1)) @ S1
    g = 2 if ctype == "W" else 1
    approx_inv = (np.eye(N1) - np.linalg.matrix_power(E1, g)) @ np.linalg.inv(A1)
    R0, P0 = mg.h.R[0].toarray(), mg.h.P[0].toarray()
    E0 = S0 @ (np.eye(N) - P0 @ approx_inv @ R0 @ A0) @ S0
    M = dense_of(mg.apply, N)
    assert np.allclose(np.eye(N) - M @ A0, E0, atol=1e-9)


def test_combined_jacobi_fine_vanka_coarse_cycle():
    """Sec. 5.5, Sec. 6: damped Jacobi on the fine level, Element-patch Vanka below.  The fine
    smoother is u + w D^{-1}(q - A u) with D the diagonal of A (written out here, not
    taken from the patch code); the level-1 smoother is the Element one; and the 3-level
    V-cycle error operator is eq. (2G) nested with those two smoothers."""
    n = (17, 17)
    ops = small_problem(n, alpha=0.6)
    w = [0.6, 0.7]
    mg = cycle.Multigrid(ops["Hs"], n, 3, "linear", ["point", "element"], w)
    ref = cycle.Multigrid(ops["Hs"], n, 3, "linear", "element", w)
    A0 = ops["Hs"].toarray()
    N = A0.shape[0]
    rng = np.random.default_rng(5)
    q = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    u = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    jac = u + w[0] * (q - A0 @ u) / np.diag(A0)
    assert np.allclose(mg.relax(0, q, u), jac, rtol=1e-13, atol=0)
    A1 = mg.h.A[1].toarray()
    assert np.allclose(mg.smoothers[1].dense(), ref.smoothers[1].dense(), rtol=1e-13, atol=0)
    A2 = mg.h.A[2].toarray()
    N1 = A1.shape[0]
    S0 = np.eye(N) - w[0] * np.diag(1.0 / np.diag(A0)) @ A0
    S1 = np.eye(N1) - w[1] * mg.smoothers[1].dense() @ A1
    R1, P1 = mg.h.R[1].toarray(), mg.h.P[1].toarray()
    E1 = S1 @ (np.eye(N1) - P1 @ np.linalg.solve(A2, R1 @ A1)) @ S1
    R0, P0 = mg.h.R[0].toarray(), mg.h.P[0].toarray()
    E0 = S0 @ (np.eye(N) - P0 @ (np.eye(N1) - E1) @ np.linalg.inv(A1) @ R0 @ A0) @ S0
    M = dense_of(mg.apply, N)
    assert np.allclose(np.eye(N) - M @ A0, E0, atol=1e-9)


def test_givens_rotation():
    rng = np.random.default_rng(1)
    for _ in range(10):
        a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        c, s = krylov.givens(a, b)
        G = np.array([[c, s], [-np.conj(s), c]])
        out = G @ np.array([a, b])
        assert abs(out[1]) < 1e-14 and np.allclose(G.conj().T @ G, np.eye(2))
    c, s = krylov.givens(0.0, 2.0 + 1j)
    assert c == 0.0 and s == 1.0


def test_fgmres_iterates_minimise_the_residual():
    """P8: without restart, the k-th FGMRES iterate minimises ||q - H x|| over
    x in M^{-1} K_k(H M^{-1}, q) (M fixed), checked by dense least squares."""
    n = (9, 9)
    ops = small_problem(n, alpha=0.5)
    mg = cycle.Multigrid(ops["Hs"], n, 2, "levdep", "full", [0.8])
    H = ops["H"].toarray()
    Minv = dense_of(mg.apply, 81)
    q = synth.point_source(n).ravel()
    K = [q]
    for k in range(1, 7):
        x, info = krylov.fgmres(lambda v: H @ v, mg.apply, q, 1e-30, 100, k)
        assert info["iterations"] == k
        basis, _ = np.linalg.qr(np.stack(K, axis=1))
        Y = Minv @ basis
        coef, *_ = np.linalg.lstsq(H @ Y, q, rcond=None)
        xref = Y @ coef
        assert np.linalg.norm(q - H @ x) == pytest.approx(np.linalg.norm(q - H @ xref), rel=1e-8)
        assert np.allclose(x, xref, rtol=1e-7, atol=1e-12)
        K.append(H @ Minv @ K[-1])


def test_fgmres_restart_converges_on_true_residual():
    ops = small_problem((17, 17), alpha=0.5)
    mg = cycle.Multigrid(ops["Hs"], (17, 17), 3, "levdep", "full", [0.9, 0.7])
    q = synth.point_source((17, 17)).ravel()
    x, info = krylov.fgmres(lambda v: ops["H"] @ v, mg.apply, q, 1e-8, 3, 500)
    assert info["converged"] and info["restarts"] >= 2
    assert np.linalg.norm(q - ops["H"] @ x) <= 1e-8 * np.linalg.norm(q)


@pytest.mark.slow
def test_table_const2d_w_cycle_iterations(paper):
    """Table 'const2D', 128^2 cells, omega = 25.6 pi, homogeneous, 4-level W(1,1),
    compact stencil, absorbing layer, GMRES(5), damping from Table 'relaxParam':
    every printed cell reproduced within +-20% (the layer profile is unpublished)."""
    n = (129, 129)
    h = 1 / 128
    omega = synth.omega_for_ppw(h, 10)
    q = synth.point_source(n).ravel()
    for patch, row in paper["const2d_128"].items():
        if patch.startswith("_"):
            continue
        ops = D.compact4_operator(n, h, omega, 1.0, 0.0, row["alpha"], "sponge")
        for scheme in ("cubic", "mixed", "levdep"):
            mg = cycle.Multigrid(ops["Hs"], n, 4, scheme, patch,
                                 paper["damping_2d"][patch], cycle="W")
            _, info = krylov.fgmres(lambda v: ops["H"] @ v, mg.apply, q, 1e-6, 5, 1000)
            assert abs(info["iterations"] - row[scheme]) <= 0.2 * row[scheme], \
                (patch, scheme, info["iterations"], row[scheme])


@pytest.mark.slow
def test_table_heterogeneous2d_two_level(paper):
    """Table 'heterogeneous2D': linear kappa^2 in [0.25, 1], 2-level V(1,1), RB,
    alpha = 0, GMRES(5) -> 6 iterations at 128^2 (+-1); 4-level alpha = 0.25 -> 34
    (+-20%)."""
    n = (129, 129)
    h = 1 / 128
    omega = synth.omega_for_ppw(h, 10)
    kappa = synth.linear_kappa2(n, 0.25, 1.0)
    q = synth.point_source(n).ravel()
    ref = paper["heterogeneous2d_linear_025"]["128"]
    for levels, alpha, target, tol in ((2, 0.0, ref[0], 1), (4, 0.25, ref[2], 0.2 * ref[2])):
        ops = D.compact4_operator(n, h, omega, kappa, 0.0, alpha, "sponge")
        mg = cycle.Multigrid(ops["Hs"], n, levels, "levdep", "rb", paper["damping_2d"]["rb"])
        _, info = krylov.fgmres(lambda v: ops["H"] @ v, mg.apply, q, 1e-6, 5, 1000)
        assert abs(info["iterations"] - target) <= tol, (levels, info["iterations"])


def test_stationary_iteration_residuals_are_powers_of_the_error_operator():
    """Sec. 5.1: x <- x + M^{-1}(q - A x) from x = 0 gives r^(k) = (I - A M^{-1})^k q;
    checked against dense matrix powers (M^{-1} assembled column by column), and the
    convergence factor of eq. (cf) against the same norms; an exact preconditioner
    stops after one cycle."""
    n = (9, 9)
    ops = small_problem(n)
    A = ops["Hs"].toarray()
    mg = cycle.Multigrid(ops["Hs"], n, 2, "levdep", "full", [0.8])
    Minv = dense_of(mg.apply, 81)
    q = np.random.default_rng(3).standard_normal(81) + 1j * np.random.default_rng(4).standard_normal(81)
    x, hist = krylov.stationary(lambda v: ops["Hs"] @ v, mg.apply, q, 6, 1e-14)
    E = np.eye(81) - A @ Minv
    ref = [np.linalg.norm(np.linalg.matrix_power(E, k) @ q) / np.linalg.norm(q)
           for k in range(len(hist))]
    assert len(hist) == 7
    assert np.allclose(hist, ref, rtol=1e-8, atol=0)
    # exact inverse: one cycle
    x, hist = krylov.stationary(lambda v: ops["Hs"] @ v,
                                lambda v: np.linalg.solve(A, v), q, 10, 1e-12)
    assert len(hist) == 2 and hist[1] <= 1e-12
    # divergence stops at 1e12
    x, hist = krylov.stationary(lambda v: ops["Hs"] @ v, lambda v: -50.0 * v, q, 400, 1e-12)
    assert hist[-1] > 1e12 and len(hist) < 400


def test_convergence_factor_of_a_history_with_a_geometric_tail():
    """eq. (cf) counted after a warm-up of w iterations: a residual history that is
    geometric with ratio rho from iteration w on has c_f = rho whatever its first w
    entries, and a history that only turns geometric one step later does not."""
    rho = 0.37
    head = [1.0, 0.52, 0.31, 0.17, 0.12, 0.1]          # iterations 0..5, not geometric
    hist = head + [0.1 * rho ** k for k in range(1, 12)]
    assert krylov.convergence_factor(hist, warmup=5) == pytest.approx(rho, rel=1e-13)
    # warm-up 3 reads ||r^(3)|| = 0.17 as the start: (0.1/0.17 rho^11)^(1/13)
    assert krylov.convergence_factor(hist, warmup=3) == pytest.approx(
        (0.1 / 0.17 * rho ** 11) ** (1 / 13), rel=1e-13)
    late = head + [0.1] + [0.1 * rho ** k for k in range(1, 11)]
    assert krylov.convergence_factor(late, warmup=5) == pytest.approx(rho ** (10 / 11), rel=1e-13)
    assert np.isnan(krylov.convergence_factor(hist[:6], warmup=5))


@pytest.mark.parametrize("patch", ["rb", "point", "element", "plus"])
def test_convergence_factor_against_two_grid_lfa(paper, patch):
    """P10 (Sec. 5.1): the 2-level cycle with bicubic transfers and no shift, used as a
    stationary solver on the compact-stencil problem at 10 points per wavelength with the
    absorbing layer, converges slightly faster than the two-grid LFA factor rho_loc.
    Error started random (the asymptotic experiment of Sec. 5.1), solved to 1e-9, c_f of
    eq. (cf) after 5 warm-up cycles; damping = the fine row of Table 'relaxParam'; 128^2
    cells (rho_loc depends only on omega h; 256^2 gives the same c_f to three digits).
    For the RB and Jacobi patches the LFA maximum lies at high frequencies and c_f is
    within 10 % below rho_loc.  For Element and Plus it lies on the resonance circle
    |theta| = omega h, whose propagating modes leave through the absorbing layer; there
    c_f stays below rho_loc and within 20 % below the LFA factor taken away from that
    circle (|theta| differing from omega h by more than 0.15)."""
    cells = 128
    n = (cells + 1, cells + 1)
    h = 1.0 / cells
    omega = 2 * np.pi / (10 * h)
    w = paper["damping_fine_2d"][patch]
    ops = D.compact4_operator(n, h, omega, 1.0, 0.0, 0.0, bc="sponge")
    rng = np.random.default_rng(7)
    y = rng.standard_normal(n[0] * n[1]) + 1j * rng.standard_normal(n[0] * n[1])
    mg = cycle.Multigrid(ops["Hs"], n, 2, "cubic", patch, [w])
    # error propagation from x = 0 towards y equals that of a random initial error
    x, hist = krylov.stationary(lambda v: ops["H"] @ v, mg.apply, ops["H"] @ y, 400, 1e-9)
    assert hist[-1] <= 1e-9 and len(hist) > 7
    cf = krylov.convergence_factor(hist, warmup=5)
    st = lfa.compact4_stencil(2, h, omega ** 2)
    th = lfa.theta_grid(256, 2)
    lo = np.all((th >= -np.pi / 2) & (th < np.pi / 2), axis=-1)
    lo &= np.any(np.abs(th) > 1e-12, axis=-1)
    rad = np.max(np.abs(np.linalg.eigvals(
        lfa.two_grid_symbol(st, patch, w, th[lo], "cubic", "cubic"))), axis=-1)
    rho = rad.max()
    assert rho == pytest.approx(lfa.two_grid_factor(st, patch, w, npts=256), rel=1e-14)
    assert cf <= rho
    if patch in ("rb", "point"):
        assert cf >= 0.9 * rho, (cf, rho)
    else:
        away = np.abs(np.linalg.norm(th[lo], axis=-1) - omega * h) > 0.15
        rho_away = rad[away].max()
        assert 0.8 * rho_away <= cf <= rho_away, (cf, rho_away, rho)
