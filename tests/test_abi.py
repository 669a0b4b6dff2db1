"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and its
host-only logic (defaults, status strings, argument validation, footprint) works
without touching a GPU."""
import os
import re

import pytest

from paper_2511_16808_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "vh.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vh_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 13
    L = B.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(B._SIGNATURES), "binding and header disagree"


def test_defaults_and_status_strings():
    o = B.vh_options_default()
    assert (o.precision, o.restart, o.maxit, o.nu1, o.nu2) == (B.VH_PREC_FP64, 20, 1000, 1, 1)
    assert o.sponge_width == 20 and o.sponge_amp == 1.0 and o.intergrid == -1
    assert B.vh_status_string(B.VH_ENOCONV) == "not converged"
    assert B.vh_status_string(12345) == "unknown status"


@pytest.mark.parametrize("dim,n,levels,err", [
    (2, (129, 129), 9, "divisible"),        # 128 cells cannot be halved 8 times
    (2, (130, 129), 2, "divisible"),        # odd number of cells
    (2, (2, 129), 1, ">= 3 nodes"),
    (4, (9, 9), 1, "dim"),
    (2, (257, 257), 2, "coarsest level too large"),
])
def test_setup_rejects_bad_arguments_before_any_device_work(dim, n, levels, err):
    with pytest.raises(B.VhError) as e:
        B.vh_setup(dim, n, 1 / 128, 10.0, None, None, 0.1, levels, B.VH_PATCH_FULL)
    assert e.value.status == B.VH_EINVAL and err in str(e.value)


def test_symmetric_smoother_checks_ndamping_before_reading_damping():
    o = B.make_options(smoother=B.VH_SMOOTHER_SYMMETRIC)
    o.ndamping = 17
    with pytest.raises(B.VhError) as e:
        B.vh_setup(2, (33, 33), 1 / 32, 10.0, None, None, 0.1, 3, B.VH_PATCH_FULL, o)
    assert e.value.status == B.VH_EINVAL and "ndamping" in str(e.value)
    o = B.make_options(damping=[0.9, float("inf")])
    with pytest.raises(B.VhError) as e:
        B.vh_setup(2, (33, 33), 1 / 32, 10.0, None, None, 0.1, 3, B.VH_PATCH_FULL, o)
    assert e.value.status == B.VH_EINVAL and "finite" in str(e.value)


def test_solve_stats_layout_carries_setup_bytes_and_convergence_factor():
    names = [f for f, _ in B.vh_solve_stats._fields_]
    assert names[-3:] == ["setup_ms", "bytes_moved", "c_f"]
    text = open(os.path.join(ROOT, "include", "vh.h")).read()
    body = text[text.index("typedef struct vh_solve_stats"):text.index("} vh_solve_stats;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    decl = re.findall(r"\b(int|double)\s+([a-z0-9_]+)\s*;", body)
    assert [n for _, n in decl] == names
    ctypes_of = {"int": "c_int", "double": "c_double"}
    assert [ctypes_of[t] for t, _ in decl] == [ty.__name__ for _, ty in B.vh_solve_stats._fields_]
    assert B.lib().vh_get_memory(None, None, None) == B.VH_EINVAL


def test_footprint_counts_the_setup_peak_of_a_complex64_hierarchy():
    """With the complex64 preconditioner setup also holds the FP64 Galerkin operators of
    every level; the footprint is the larger of that and the solve peak."""
    n = (257, 257, 257)
    o = B.make_options(precision=B.VH_PREC_C64, restart=1, smoother=B.VH_SMOOTHER_ASSEMBLED)
    fp = B.vh_footprint_bytes(3, n, 6, B.VH_PATCH_FULL, 1, o)
    N = 257 ** 3
    a64 = 7 * N * 16 + 27 * 16 * sum((2 ** (8 - l) + 1) ** 3 for l in range(1, 6))
    stored = 7 * N * 8 + 7 * N * 16 + 2 * N * 16 + 125 * N * 8  # A, H, basis, smoother
    assert fp >= stored + a64


def test_setup_rejects_bad_options():
    for field, value in (("restart", 0), ("restart", 65), ("precision", 7), ("nu1", -1),
                         ("bc", 5), ("smoother", 3), ("sweep_tile", 11), ("sweep_tile", -1),
                         ("split_residual", 3), ("split_residual", -1), ("sym_planes", -2),
                         ("sym_planes", 1), ("sym_planes", 65), ("setup_pivot", 2), ("setup_pivot", -1)):
        o = B.make_options(**{field: value})
        with pytest.raises(B.VhError) as e:
            B.vh_setup(2, (33, 33), 1 / 32, 10.0, None, None, 0.1, 3, B.VH_PATCH_FULL, o)
        assert e.value.status == B.VH_EINVAL, field


def test_footprint_matches_the_layout():
    """C2-shaped 2D FP64 hierarchy: the per-patch inverses dominate (81 c128 per node)."""
    n = (1025, 1025)
    fp = B.vh_footprint_bytes(2, n, 7, B.VH_PATCH_FULL, 1)
    N = 1025 * 1025
    inv_fine = 81 * 16 * N
    assert inv_fine < fp < 2.6 * inv_fine
    o = B.make_options(precision=B.VH_PREC_C64)
    assert B.vh_footprint_bytes(2, n, 7, B.VH_PATCH_FULL, 1, o) < 0.62 * fp
    o = B.make_options(smoother=B.VH_SMOOTHER_ASSEMBLED)
    assert B.vh_footprint_bytes(2, n, 7, B.VH_PATCH_FULL, 1, o) < 0.6 * fp
    # the multi-source workspace grows with the group width (powers of two up to 64)
    ob = B.make_options(batch=1)
    f16 = B.vh_footprint_bytes(2, n, 7, B.VH_PATCH_FULL, 16, ob)
    f9 = B.vh_footprint_bytes(2, n, 7, B.VH_PATCH_FULL, 9, ob)
    f64 = B.vh_footprint_bytes(2, n, 7, B.VH_PATCH_FULL, 200, ob)
    assert fp < f9 == f16 < f64
    assert B.vh_footprint_bytes(2, (2, 5), 1, B.VH_PATCH_FULL, 1) == 0


def test_lfa_and_tuners_reject_bad_arguments_before_any_device_work():
    p = B.make_lfa_problem()
    assert (p.dim, p.npts, p.nu1, p.nu2, p.rfam) == (2, 256, 1, 1, B.VH_IG_CUBIC)
    for field, value in (("npts", 3), ("npts", 514), ("dim", 4), ("patch", 2), ("h", 0.0),
                         ("sigma", -1.0), ("rfam", B.VH_IG_LEVDEP), ("stencil", 7)):
        q = B.make_lfa_problem(**{field: value})
        with pytest.raises(B.VhError) as e:
            B.vh_lfa_factors(q, [0.8])
        assert e.value.status == B.VH_EINVAL, field
    with pytest.raises(B.VhError) as e:
        B.vh_lfa_factors(B.make_lfa_problem(dim=3, npts=130), [0.8])
    assert e.value.status == B.VH_EINVAL
    with pytest.raises(B.VhError) as e:
        B.vh_lfa_tune(p, 2, [0.8])
    assert e.value.status == B.VH_EINVAL
    with pytest.raises(B.VhError) as e:
        B.vh_lfa_factors(p, [float("nan")])
    assert e.value.status == B.VH_EINVAL
    with pytest.raises(B.VhError) as e:  # one level has nothing to tune
        B.vh_tune_damping(2, (33, 33), 1 / 32, 10.0, None, None, 0.1, 1, B.VH_PATCH_FULL,
                          None, None, 0, 0, 10, 1e-6, [0.8])
    assert e.value.status == B.VH_EINVAL
    st = B.lib().vh_tune_shift(2, None, 1.0, 1.0, None, None, 2, 0, None, None, 0, None, 0, 1,
                               1e-6, None, None)
    assert st == B.VH_EINVAL
    st = B.lib().vh_mg_iterate(None, 1, None, None, 0, 1, 1e-6, None, None)
    assert st == B.VH_EINVAL
    # the allocation-free LFA form refuses work arrays beyond its static scratch
    with pytest.raises(B.VhError) as e:
        B.vh_lfa_factors_noalloc(B.make_lfa_problem(dim=3, npts=128), [0.8])
    assert e.value.status == B.VH_EINVAL and "allocation-free" in str(e.value)
    with pytest.raises(B.VhError) as e:
        B.vh_lfa_factors_noalloc(p, [0.8], mu=False, rho=False)
    assert e.value.status == B.VH_EINVAL


def test_symmetric_smoother_rejects_what_it_does_not_cover():
    """The symmetric half needs the Full patch, the 5/7-point stencil, one source per sweep
    and damping > 0; refused before any device work."""
    cases = [(dict(stencil=B.VH_STENCIL_COMPACT4), B.VH_PATCH_FULL, B.VH_EUNSUPPORTED),
             (dict(batch=1), B.VH_PATCH_FULL, B.VH_EUNSUPPORTED),
             (dict(), B.VH_PATCH_RB, B.VH_EUNSUPPORTED),
             (dict(fine_patch=B.VH_PATCH_POINT), B.VH_PATCH_FULL, B.VH_EUNSUPPORTED),
             (dict(damping=[0.9, 0.0]), B.VH_PATCH_FULL, B.VH_EINVAL)]
    for extra, patch, status in cases:
        o = B.make_options(smoother=B.VH_SMOOTHER_SYMMETRIC, **extra)
        with pytest.raises(B.VhError) as e:
            B.vh_setup(2, (33, 33), 1 / 32, 10.0, None, None, 0.1, 3, patch, o)
        assert e.value.status == status, extra


def test_symmetric_footprint():
    """3D trilinear: every smoothed level stores 63 instead of 125 entries per node; 2D
    level-dependent transfers: only the two finest levels are symmetric."""
    n3 = (129, 129, 129)
    fa = B.vh_footprint_bytes(3, n3, 5, B.VH_PATCH_FULL, 1,
                              B.make_options(smoother=B.VH_SMOOTHER_ASSEMBLED))
    fs = B.vh_footprint_bytes(3, n3, 5, B.VH_PATCH_FULL, 1,
                              B.make_options(smoother=B.VH_SMOOTHER_SYMMETRIC))
    nxp = 160
    fine = 62 * 16 * nxp * 129 * 129  # entries saved on the finest level alone
    assert fa - fs > fine
    n2 = (257, 257)
    fa2 = B.vh_footprint_bytes(2, n2, 5, B.VH_PATCH_FULL, 1,
                               B.make_options(smoother=B.VH_SMOOTHER_ASSEMBLED))
    fs2 = B.vh_footprint_bytes(2, n2, 5, B.VH_PATCH_FULL, 1,
                               B.make_options(smoother=B.VH_SMOOTHER_SYMMETRIC))
    saved = 12 * 16 * (288 * 257 + 160 * 129)  # levels 0 and 1 only
    guards = 16 * ((2 + 2 * 288) + (2 + 2 * 160))  # zero entries before each half's first plane
    assert fa2 - fs2 == saved - guards
