"""CPU: the identity behind the patch inversion without pivoting (Sec. 3.2 patch solves).
For a complex symmetric matrix eliminated in the natural order with the rotating-row
Gauss-Jordan tableau (unnormalised pivot rows, inverse columns appended), the pivot row at
step s is recovered from every row's leading entry: position (k - s) mod n holds a_k[0]
for a row k not yet used and -a_k[0] / d_k for a used row with pivot value d_k.  The
elimination written here follows that description; numpy's inverse checks the result."""
import numpy as np
import pytest


def rotating_row_inverse(A, pivot_row_from_columns):
    n = A.shape[0]
    rows = [A[k].astype(complex).copy() for k in range(n)]
    d = [None] * n
    worst = 0.0
    for s in range(n):
        p = rows[s].copy()
        if pivot_row_from_columns:
            q = np.empty(n, dtype=complex)
            for k in range(n):
                lead = rows[k][0]
                q[(k - s) % n] = lead if k >= s else -lead / d[k]
            worst = max(worst, np.abs(q - p).max() / np.abs(p).max())
            p = q
        new = []
        for k in range(n):
            r = rows[k]
            if k == s:
                d[k] = p[0]
                new.append(np.concatenate([r[1:], [1.0]]))
            else:
                c = -r[0] / p[0]
                new.append(np.concatenate([r[1:] + c * p[1:], [c]]))
        rows = new
    return np.array([rows[k] / d[k] for k in range(n)]), worst


@pytest.mark.parametrize("n,seed", [(9, 0), (27, 1), (27, 2), (8, 3)])
def test_pivot_row_from_leading_entries(n, seed):
    rng = np.random.default_rng(seed)
    # shifted-Laplacian-like: symmetric real part, positive definite imaginary part
    X = rng.standard_normal((n, n))
    B = X + X.T + 2.0 * np.eye(n)
    C = np.diag(rng.uniform(0.2, 1.0, n))
    A = B + 1j * C
    inv_ref = np.linalg.inv(A)
    inv_col, worst = rotating_row_inverse(A, True)
    inv_row, _ = rotating_row_inverse(A, False)
    assert worst <= 1e-12
    scale = np.abs(inv_ref).max()
    assert np.abs(inv_col - inv_ref).max() <= 1e-11 * scale
    assert np.abs(inv_row - inv_ref).max() <= 1e-11 * scale


def test_identity_needs_symmetry():
    """A non-symmetric matrix breaks the identity: the recovered row differs."""
    rng = np.random.default_rng(4)
    A = rng.standard_normal((9, 9)) + 1j * np.diag(rng.uniform(0.5, 1.0, 9)) + 4 * np.eye(9)
    _, worst = rotating_row_inverse(A, True)
    assert worst > 1e-3
