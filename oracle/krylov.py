"""Oracle: right-preconditioned flexible GMRES(m) (TEST INFRASTRUCTURE ONLY).

Paper Sec. 2.3: the shifted operator, solved by multigrid, preconditions a Krylov
method such as flexible GMRES; Sec. 5: zero initial guess, stop at relative
residual < tol.  Readings (paper silent): modified Gram-Schmidt Arnoldi; complex
Givens rotation r = sqrt(|a|^2+|b|^2), c = |a|/r, s = (a/|a|) conj(b)/r (c = 0,
s = 1 when a = 0); convergence is declared only on the true residual ||q - H x||
recomputed at each restart; the iteration count is the number of preconditioner
applications summed over restarts.
"""
import numpy as np


def givens(a, b):
    """Rotation (c, s) with [c s; -conj(s) c] [a; b] = [r'; 0]."""
    if a == 0:
        return 0.0, 1.0 + 0j
    r = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    return abs(a) / r, (a / abs(a)) * np.conj(b) / r


def fgmres(matvec, precond, b, tol=1e-6, restart=20, maxit=1000, x0=None):
    """Solve matvec(x) = b.  Returns (x, info) with info = dict(iterations,
    converged, relres (true), history (estimated relres per iteration))."""
    b = np.asarray(b, dtype=complex)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=complex).copy()
    bnorm = np.linalg.norm(b)
    info = {"iterations": 0, "converged": False, "history": [], "restarts": 0}
    if bnorm == 0.0:
        info.update(converged=True, relres=0.0)
        return np.zeros_like(b), info
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    its = 0
    while True:
        if beta / bnorm <= tol:
            info.update(converged=True, relres=beta / bnorm, iterations=its)
            return x, info
        if its >= maxit:
            info.update(relres=beta / bnorm, iterations=its)
            return x, info
        m = restart
        V = np.zeros((m + 1, b.size), dtype=complex)
        Z = np.zeros((m, b.size), dtype=complex)
        Hm = np.zeros((m + 1, m), dtype=complex)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=complex)
        g = np.zeros(m + 1, dtype=complex)
        V[0] = r / beta
        g[0] = beta
        k = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            its += 1
            for i in range(j + 1):
                Hm[i, j] = np.vdot(V[i], w)
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            for i in range(j):
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -np.conj(sn[i]) * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            hn = Hm[j + 1, j]
            cs[j], sn[j] = givens(Hm[j, j], hn)
            Hm[j, j] = cs[j] * Hm[j, j] + sn[j] * hn
            Hm[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            info["history"].append(abs(g[j + 1]) / bnorm)
            if hn == 0.0:
                break
            V[j + 1] = w / hn
            if abs(g[j + 1]) / bnorm <= tol or its >= maxit:
                break
        y = np.zeros(k, dtype=complex)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - Hm[i, i + 1:k] @ y[i + 1:k]) / Hm[i, i]
        x = x + Z[:k].T @ y
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        info["restarts"] += 1


def convergence_factor(history, warmup=5):
    """eq. (cf): (||r_k|| / ||r_0||)^(1/k), counted after `warmup` iterations."""
    h = np.asarray(history, dtype=float)
    if h.size <= warmup + 1:
        return float("nan")
    k = h.size - 1 - warmup
    return float((h[-1] / h[warmup]) ** (1.0 / k))


def stationary(matvec, precond, b, maxit, tol):
    """The cycle as a stationary solver (Sec. 5.1): x <- x + M^{-1}(b - A x) from x = 0.
    Stops when ||r|| <= tol ||b||, when the residual exceeds 1e12 ||b|| (divergence) or
    after maxit cycles.  Returns (x, history) with history[k] = ||r^(k)|| / ||b||."""
    b = np.asarray(b, dtype=complex)
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, [0.0]
    hist = []
    for k in range(maxit + 1):
        r = b - matvec(x)
        rel = np.linalg.norm(r) / bnorm
        hist.append(rel)
        if not np.isfinite(rel) or rel <= tol or rel > 1e12 or k == maxit:
            break
        x = x + precond(r)
    return x, hist
