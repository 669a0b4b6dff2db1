"""Pins of the oracle's additive Vanka smoother (Sec. 3.2, 3.3, 4.1)."""
import numpy as np
import pytest

from oracle import discretization as D
from oracle import lfa, vanka


def test_patch_phases_match_printed_Phi(paper):
    for kind in ("element", "plus", "rb"):
        assert [list(o) for o in vanka.patch_offsets(kind, 2)] == paper["patch_phases"][kind]


def test_patch_matrices_match_printed_ones(paper):
    """eq. (4lfa), (5lfa), (skew5lfa): H_i in terms of a, b, c."""
    h, sigma = 1 / 64, 300.0
    st = lfa.compact4_stencil(2, h, sigma)
    a, b, c = lfa.compact4_abc(h, sigma)
    val = {"a": a, "b": b, "c": c, "0": 0.0}
    for kind in ("element", "plus", "rb"):
        Hi = lfa.patch_matrix(st, vanka.patch_offsets(kind, 2))
        ref = np.array([[val[e] for e in row] for row in paper["patch_matrices"][kind]])
        assert np.allclose(Hi, ref, rtol=1e-14, atol=0)


def test_patch_sizes_3d():
    """Sec. 3.2: 3D Element 8, Plus 7, RB 13, Full 27 vertices."""
    sizes = {k: len(vanka.patch_offsets(k, 3)) for k in ("element", "plus", "rb", "full")}
    assert sizes == {"element": 8, "plus": 7, "rb": 13, "full": 27}


def test_boundary_patch_sizes_and_interior_weights(paper):
    """Sec. 3.3: truncated boundary patch sizes; interior weight = 1/N."""
    n = (9, 8)
    for kind, sizes in paper["boundary_patch_sizes_2d"].items():
        if kind.startswith("_"):
            continue
        idx = vanka.patch_index(n, kind)
        size = (idx >= 0).sum(axis=1).reshape(8, 9)
        assert size[0, 0] == sizes["corner"] and size[-1, -1] == sizes["corner"]
        assert size[0, 4] == sizes["edge"] and size[4, 0] == sizes["edge"]
        assert size[4, 4] == sizes["interior"]
        cnt = vanka.patch_counts(idx, 72).reshape(8, 9)
        assert cnt[4, 4] == sizes["interior"]
    idx = vanka.patch_index(n, "element")
    assert idx.shape[0] == 8 * 7 and (idx >= 0).all()  # no boundary patches


def brute_force_B(A, n, kind):
    """Pure-Python sum over patches of V^T W A_c^{-1} V (tiny grids)."""
    A = A.toarray()
    N = A.shape[0]
    offs = vanka.patch_offsets(kind, len(n))
    members = []
    if kind == "element":
        anchors = [(x, y) for y in range(n[1] - 1) for x in range(n[0] - 1)]
    else:
        anchors = [(x, y) for y in range(n[1]) for x in range(n[0])]
    for (x, y) in anchors:
        mem = []
        for (dx, dy) in offs:
            if 0 <= x + dx < n[0] and 0 <= y + dy < n[1]:
                mem.append(x + dx + n[0] * (y + dy))
        members.append(mem)
    cnt = np.zeros(N)
    for mem in members:
        for j in mem:
            cnt[j] += 1
    B = np.zeros((N, N), dtype=complex)
    for mem in members:
        Ai = np.linalg.inv(A[np.ix_(mem, mem)])
        for a, j in enumerate(mem):
            for b, k in enumerate(mem):
                B[j, k] += Ai[a, b] / cnt[j]
    return B


@pytest.mark.parametrize("kind", ["full", "rb", "plus", "element", "point"])
def test_vanka_apply_matches_dense_and_brute_force(kind):
    n = (7, 6)
    rng = np.random.default_rng(3)
    kappa = rng.uniform(0.4, 1.0, size=(6, 7))
    ops = D.fd2_operator(n, 1 / 6, 14.0, kappa, 0.4, alpha=0.3, sponge_width=2)
    sm = vanka.AdditiveVanka(ops["Hs"], n, kind)
    B = sm.dense()
    Bref = brute_force_B(ops["Hs"], n, kind)
    assert np.abs(B - Bref).max() <= 1e-13 * np.abs(Bref).max()
    r = rng.standard_normal(42) + 1j * rng.standard_normal(42)
    assert np.allclose(sm.apply(r), B @ r, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("n", [(16, 16), (9, 13)])
def test_vanka_invariants_16x16(n):
    """Partition of unity sum_c V_c^T W_c V_c = I; D^{-1} B complex symmetric when
    H_s is (D = diag of the weights 1/cnt); heterogeneous medium with ABC."""
    rng = np.random.default_rng(4)
    kappa = rng.uniform(0.25, 1.0, size=tuple(reversed(n)))
    ops = D.fd2_operator(n, 1 / 15, 20.0, kappa, 0.2, alpha=0.1, sponge_width=4)
    sm = vanka.AdditiveVanka(ops["Hs"], n, "full")
    N = ops["Hs"].shape[0]
    pu = np.zeros(N)
    np.add.at(pu, sm.idx[sm.idx >= 0], sm.weight[sm.idx >= 0])
    assert np.allclose(pu, 1.0, atol=1e-15)
    B = sm.dense()
    C = sm.cnt[:, None] * B
    assert np.abs(C - C.T).max() <= 1e-13 * np.abs(C).max()


@pytest.mark.parametrize("kind,dim,nn", [("full", 2, 16), ("rb", 2, 16), ("element", 2, 16),
                                         ("plus", 2, 16), ("point", 2, 16), ("full", 3, 8)])
def test_periodic_smoother_acts_on_fourier_modes_by_symbol(kind, dim, nn):
    """P2: on a periodic constant-coefficient grid, S e^{i theta x} = S(theta) e^{i theta x}
    with S(theta) from eq. (smoother_symbol)."""
    n = (nn,) * dim
    h, sigma, w = 1 / nn, 30.0, 0.8
    st = lfa.compact4_stencil(dim, h, sigma) if dim == 2 else lfa.fd2_stencil(dim, h, sigma)
    A = D.stencil_matrix(n, st, periodic=True)
    N = A.shape[0]
    # periodic patches: every node anchors a whole patch (wrap-around)
    offs = vanka.patch_offsets(kind, dim)
    coords = np.indices(tuple(reversed(n))).reshape(dim, -1)[::-1]
    Ai = np.linalg.inv(lfa.patch_matrix(st, offs))
    Bm = np.zeros((N, N), dtype=complex)
    lin = lambda c: sum(int(c[d] % n[d]) * int(np.prod(n[:d])) for d in range(dim))
    for p in range(N):
        mem = [lin([coords[d][p] + o[d] for d in range(dim)]) for o in offs]
        for a, j in enumerate(mem):
            for b, k in enumerate(mem):
                Bm[j, k] += Ai[a, b] / len(offs)
    S = np.eye(N) - w * Bm @ A.toarray()
    rng = np.random.default_rng(5)
    for _ in range(4):
        k = rng.integers(0, nn, size=dim)
        th = 2 * np.pi * k / nn
        mode = np.exp(1j * (coords.T @ th))
        sym = lfa.vanka_symbol(st, kind, w, th[None, :])[0]
        assert np.allclose(S @ mode, sym * mode, atol=1e-11)


def test_jacobi_is_the_one_point_patch():
    """Sec. 4.1: the Jacobi symbol 1 - w H(theta)/a equals the 1x1 Vanka patch."""
    h, sigma, w = 1 / 32, 50.0, 0.7
    st = lfa.compact4_stencil(2, h, sigma)
    th = np.random.default_rng(6).uniform(-np.pi, np.pi, size=(20, 2))
    a = lfa.compact4_abc(h, sigma)[0]
    assert np.allclose(lfa.vanka_symbol(st, "point", w, th), 1 - w * lfa.symbol(st, th) / a)
