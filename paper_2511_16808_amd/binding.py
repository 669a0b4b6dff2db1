"""ctypes binding of libvh.so (include/vh.h).  Argument marshalling only.

Function names mirror the C ABI.  Device arrays are passed as torch tensors on the
GPU (complex128 / float64, contiguous); the binding checks dtype, device and size
and hands the raw pointers to the library.  There is no fallback: if the library
is missing or the GPU is absent the calls raise.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvh.so")

VH_OK = 0
VH_EINVAL = -1
VH_ENOMEM = -2
VH_ENOCONV = -3
VH_EBREAKDOWN = -4
VH_EDEVICE = -5
VH_EUNSUPPORTED = -6

VH_PREC_FP64 = 0
VH_PREC_C64 = 1
VH_IG_LEVDEP = 0
VH_IG_MIXED = 1
VH_IG_LINEAR = 2
VH_IG_CUBIC = 3
VH_CYCLE_V = 0
VH_CYCLE_W = 1
VH_PATCH_FULL = 0
VH_PATCH_POINT = 1
VH_PATCH_PLUS = 3
VH_PATCH_RB = 4
VH_PATCH_ELEMENT = 5
VH_BC_ABC = 0
VH_BC_DIRICHLET = 1
VH_SMOOTHER_PATCH = 0
VH_SMOOTHER_ASSEMBLED = 1
VH_SMOOTHER_SYMMETRIC = 2
VH_STENCIL_FD2 = 0
VH_STENCIL_COMPACT4 = 1
VH_CONTRACT_VALU = 0
VH_CONTRACT_MFMA_F32 = 1
VH_CONTRACT_MFMA_BF16X3 = 2


class vh_options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int), ("restart", ctypes.c_int), ("maxit", ctypes.c_int),
        ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("intergrid", ctypes.c_int),
        ("bc", ctypes.c_int), ("sponge_width", ctypes.c_int), ("sponge_amp", ctypes.c_double),
        ("smoother", ctypes.c_int), ("ndamping", ctypes.c_int),
        ("damping", ctypes.c_double * 16), ("stream", ctypes.c_void_p), ("timing", ctypes.c_int),
        ("batch", ctypes.c_int), ("stencil", ctypes.c_int), ("fine_patch", ctypes.c_int),
        ("cycle", ctypes.c_int),
        ("contraction", ctypes.c_int), ("sweep_tile", ctypes.c_int), ("split_residual", ctypes.c_int),
        ("sym_planes", ctypes.c_int), ("setup_pivot", ctypes.c_int),
    ]


class vh_solve_stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
        ("relres", ctypes.c_double), ("relres_est", ctypes.c_double), ("solve_ms", ctypes.c_double),
        ("vcycles", ctypes.c_int), ("vcycle_ms", ctypes.c_double),
        ("smooth0_launches", ctypes.c_int), ("smooth0_ms", ctypes.c_double),
        ("smooth1_launches", ctypes.c_int), ("smooth1_ms", ctypes.c_double),
        ("setup_ms", ctypes.c_double), ("bytes_moved", ctypes.c_double), ("c_f", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vh_level_info(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3), ("stencil_points", ctypes.c_int),
        ("smoother_entries", ctypes.c_int), ("offsets", (ctypes.c_int * 3) * 125),
        ("bytes", ctypes.c_size_t), ("mfma_sources", ctypes.c_int), ("mfma_tile", ctypes.c_int),
        ("mfma_rows", ctypes.c_int), ("sweep_tile", ctypes.c_int), ("fused_sweep", ctypes.c_int),
        ("fused_restrict", ctypes.c_int), ("sym_planes", ctypes.c_int),
        ("setup_pivot", ctypes.c_int),
    ]


class vh_request(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
        ("omega", ctypes.c_double), ("kappa", ctypes.c_void_p), ("gamma", ctypes.c_void_p),
        ("shift", ctypes.c_double), ("levels", ctypes.c_int), ("patch", ctypes.c_int),
        ("q", ctypes.c_void_p), ("nsrc", ctypes.c_int), ("tol", ctypes.c_double),
        ("opt", ctypes.POINTER(vh_options)),
    ]


class vh_server_info(ctypes.Structure):
    _fields_ = [
        ("budget", ctypes.c_size_t), ("in_use", ctypes.c_size_t), ("peak_in_use", ctypes.c_size_t),
        ("running", ctypes.c_int), ("peak_running", ctypes.c_int), ("queued", ctypes.c_int),
        ("completed", ctypes.c_uint64),
    ]


class vh_lfa_problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("stencil", ctypes.c_int), ("patch", ctypes.c_int),
        ("h", ctypes.c_double), ("sigma", ctypes.c_double), ("shift", ctypes.c_double),
        ("rfam", ctypes.c_int), ("pfam", ctypes.c_int), ("npts", ctypes.c_int),
        ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("stream", ctypes.c_void_p),
    ]


class vh_cf_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("relres", ctypes.c_double), ("cf", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class VhError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"vh status {status}: {msg}")
        self.status = status


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double

_SIGNATURES = {
    "vh_options_default": (None, [ctypes.POINTER(vh_options)]),
    "vh_status_string": (ctypes.c_char_p, [_I]),
    "vh_last_error": (ctypes.c_char_p, []),
    "vh_setup": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(_I), _D, _D, _P, _P, _D, _I, _I,
                      ctypes.POINTER(vh_options)]),
    "vh_solve": (_I, [_P, _P, _I, _D, _P, ctypes.POINTER(vh_solve_stats)]),
    "vh_destroy": (_I, [_P]),
    "vh_num_levels": (_I, [_P]),
    "vh_get_memory": (_I, [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "vh_get_level_info": (_I, [_P, _I, ctypes.POINTER(vh_level_info)]),
    "vh_apply_operator": (_I, [_P, _I, _I, _P, _P]),
    "vh_apply_vcycle": (_I, [_P, _P, _P]),
    "vh_apply_smoother": (_I, [_P, _I, _P, _P]),
    "vh_apply_smoother_batch": (_I, [_P, _I, _I, _P, _P]),
    "vh_apply_vcycle_batch": (_I, [_P, _I, _P, _P]),
    "vh_export_level": (_I, [_P, _I, _P, _P, _P]),
    "vh_sample_level": (_I, [_P, _I, _I, _I, _P, _P]),
    "vh_footprint_bytes": (ctypes.c_size_t, [_I, ctypes.POINTER(_I), _I, _I, _I,
                                             ctypes.POINTER(vh_options)]),
    "vh_server_create": (_I, [ctypes.POINTER(_P), ctypes.c_size_t, _I]),
    "vh_server_submit": (_I, [_P, ctypes.POINTER(vh_request), ctypes.POINTER(ctypes.c_uint64)]),
    "vh_server_poll": (_I, [_P, ctypes.c_uint64, ctypes.POINTER(_I)]),
    "vh_server_wait": (_I, [_P, ctypes.c_uint64]),
    "vh_server_result": (_I, [_P, ctypes.c_uint64, _P, ctypes.POINTER(vh_solve_stats),
                              ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "vh_server_get_info": (_I, [_P, ctypes.POINTER(vh_server_info)]),
    "vh_server_destroy": (_I, [_P]),
    "vh_lfa_problem_default": (None, [ctypes.POINTER(vh_lfa_problem)]),
    "vh_lfa_factors": (_I, [ctypes.POINTER(vh_lfa_problem), _I, ctypes.POINTER(_D),
                            ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "vh_lfa_factors_noalloc": (_I, [ctypes.POINTER(vh_lfa_problem), _I, ctypes.POINTER(_D),
                                    ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "vh_lfa_tune": (_I, [ctypes.POINTER(vh_lfa_problem), _I, _I, ctypes.POINTER(_D),
                         ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "vh_mg_iterate": (_I, [_P, _I, _P, _P, _I, _I, _D, ctypes.POINTER(_D),
                           ctypes.POINTER(vh_cf_stats)]),
    "vh_tune_damping": (_I, [_I, ctypes.POINTER(_I), _D, _D, _P, _P, _D, _I, _I,
                             ctypes.POINTER(vh_options), _P, _I, _I, _I, _D, _I,
                             ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "vh_tune_shift": (_I, [_I, ctypes.POINTER(_I), _D, _D, _P, _P, _I, _I,
                           ctypes.POINTER(vh_options), _P, _I, ctypes.POINTER(_D), _I, _I, _D,
                           ctypes.POINTER(_D), ctypes.POINTER(_D)]),
}


def lib():
    """Loads libvh.so (built in-tree by paper_2511_16808_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2511_16808_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != VH_OK:
        raise VhError(status, lib().vh_last_error().decode())
    return status


def _ptr(t, dtype_name, numel=None):
    """Raw device pointer of a contiguous GPU tensor of the given dtype (None -> NULL)."""
    if t is None:
        return None
    import torch
    want = {"complex128": torch.complex128, "float64": torch.float64}[dtype_name]
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if t.dtype != want:
        raise ValueError(f"expected {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return t.data_ptr()


def vh_options_default():
    o = vh_options()
    lib().vh_options_default(ctypes.byref(o))
    return o


def vh_status_string(s):
    return lib().vh_status_string(s).decode()


def vh_last_error():
    return lib().vh_last_error().decode()


def vh_setup(dim, n, h, omega, kappa, gamma, shift, levels, patch, opt=None):
    """kappa, gamma: float64 GPU tensors of prod(n) nodes (gamma may be None)."""
    N = 1
    for k in n[:dim]:
        N *= int(k)
    arr = (_I * 3)(*(list(n) + [1] * (3 - len(n))))
    hd = _P()
    st = lib().vh_setup(ctypes.byref(hd), dim, arr, float(h), float(omega),
                        _ptr(kappa, "float64", N), _ptr(gamma, "float64", N), float(shift),
                        levels, patch, ctypes.byref(opt) if opt is not None else None)
    check(st)
    return hd


def _level_nodes(hd, level):
    """Node count of a level of the handle (from vh_get_level_info)."""
    info = vh_level_info()
    check(lib().vh_get_level_info(hd, level, ctypes.byref(info)))
    return info.n[0] * info.n[1] * info.n[2]


def vh_solve(hd, q, nsrc, tol, u, raise_on_noconv=False):
    """q, u: complex128 GPU tensors of nsrc*N.  Returns (status, [stats dicts])."""
    if nsrc < 1:
        raise ValueError("nsrc must be >= 1")
    n = nsrc * _level_nodes(hd, 0)
    stats = (vh_solve_stats * nsrc)()
    st = lib().vh_solve(hd, _ptr(q, "complex128", n), nsrc, float(tol), _ptr(u, "complex128", n),
                        stats)
    if st != VH_OK and (st != VH_ENOCONV or raise_on_noconv):
        check(st)
    return st, [s.as_dict() for s in stats]


def vh_destroy(hd):
    check(lib().vh_destroy(hd))


def vh_num_levels(hd):
    return lib().vh_num_levels(hd)


def vh_get_memory(hd):
    """(device bytes held now, peak since setup began)."""
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    check(lib().vh_get_memory(hd, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def vh_get_level_info(hd, level):
    info = vh_level_info()
    check(lib().vh_get_level_info(hd, level, ctypes.byref(info)))
    K = info.stencil_points
    return {
        "n": tuple(info.n), "stencil_points": K, "smoother_entries": info.smoother_entries,
        "offsets": [tuple(info.offsets[k]) for k in range(K)], "bytes": info.bytes,
        "mfma_sources": info.mfma_sources, "mfma_tile": info.mfma_tile,
        "mfma_rows": info.mfma_rows, "sweep_tile": info.sweep_tile,
        "fused_sweep": info.fused_sweep, "fused_restrict": info.fused_restrict,
        "sym_planes": info.sym_planes, "setup_pivot": info.setup_pivot,
    }


def vh_apply_operator(hd, level, which, x, y):
    n = _level_nodes(hd, level)
    check(lib().vh_apply_operator(hd, level, which, _ptr(x, "complex128", n),
                                  _ptr(y, "complex128", n)))


def vh_apply_vcycle(hd, v, z):
    n = _level_nodes(hd, 0)
    check(lib().vh_apply_vcycle(hd, _ptr(v, "complex128", n), _ptr(z, "complex128", n)))


def vh_apply_smoother(hd, level, q, u):
    n = _level_nodes(hd, level)
    check(lib().vh_apply_smoother(hd, level, _ptr(q, "complex128", n), _ptr(u, "complex128", n)))


def vh_apply_smoother_batch(hd, level, nsrc, q, u):
    n = nsrc * _level_nodes(hd, level)
    check(lib().vh_apply_smoother_batch(hd, level, nsrc, _ptr(q, "complex128", n),
                                        _ptr(u, "complex128", n)))


def vh_apply_vcycle_batch(hd, nsrc, v, z):
    n = nsrc * _level_nodes(hd, 0)
    check(lib().vh_apply_vcycle_batch(hd, nsrc, _ptr(v, "complex128", n),
                                      _ptr(z, "complex128", n)))


def vh_export_level(hd, level, coef=None, smoother=None, coarse_inv=None):
    """Host numpy complex128 output arrays (C-contiguous) or None."""
    def hp(a):
        if a is None:
            return None
        assert a.dtype.name == "complex128" and a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    check(lib().vh_export_level(hd, level, hp(coef), hp(smoother), hp(coarse_inv)))


def vh_sample_level(hd, level, which, nodes, width):
    """Entries of sampled nodes: host complex128 array (len(nodes), width)."""
    import numpy as np
    nd = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.zeros((nd.size, width), dtype=np.complex128)
    check(lib().vh_sample_level(hd, level, which, nd.size, nd.ctypes.data, out.ctypes.data))
    return out


def vh_footprint_bytes(dim, n, levels, patch, nsrc=1, opt=None):
    arr = (_I * 3)(*(list(n) + [1] * (3 - len(n))))
    return lib().vh_footprint_bytes(dim, arr, levels, patch, nsrc,
                                    ctypes.byref(opt) if opt is not None else None)


_tickets = {}  # (server, ticket) -> (N, nsrc) of the submitted request


def vh_server_create(hbm_budget, max_slots):
    srv = _P()
    check(lib().vh_server_create(ctypes.byref(srv), int(hbm_budget), int(max_slots)))
    return srv


def vh_server_submit(srv, dim, n, h, omega, kappa, gamma, shift, levels, patch, q, nsrc, tol,
                     opt=None):
    """kappa, gamma, q: host numpy arrays (float64, float64 or None, complex128 [nsrc][N]);
    they are copied by the server.  Returns the ticket."""
    import numpy as np
    k = np.ascontiguousarray(kappa, dtype=np.float64)
    g = None if gamma is None else np.ascontiguousarray(gamma, dtype=np.float64)
    qq = np.ascontiguousarray(q, dtype=np.complex128)
    N = 1
    for d in range(dim):
        N *= int(n[d])
    if k.size != N or (g is not None and g.size != N):
        raise ValueError(f"kappa and gamma need {N} nodes")
    if nsrc < 1 or qq.size != nsrc * N:
        raise ValueError(f"q needs nsrc * N = {nsrc * N} entries, got {qq.size}")
    req = vh_request()
    req.dim = dim
    for d in range(3):
        req.n[d] = int(n[d]) if d < dim else 1
    req.h, req.omega, req.shift, req.tol = float(h), float(omega), float(shift), float(tol)
    req.kappa = k.ctypes.data
    req.gamma = None if g is None else g.ctypes.data
    req.q = qq.ctypes.data
    req.levels, req.patch, req.nsrc = int(levels), int(patch), int(nsrc)
    req.opt = ctypes.pointer(opt) if opt is not None else None
    t = ctypes.c_uint64()
    check(lib().vh_server_submit(srv, ctypes.byref(req), ctypes.byref(t)))
    _tickets[(srv.value, t.value)] = (N, int(nsrc))
    return t.value


def vh_server_poll(srv, ticket):
    d = _I()
    check(lib().vh_server_poll(srv, ticket, ctypes.byref(d)))
    return bool(d.value)


def vh_server_wait(srv, ticket):
    check(lib().vh_server_wait(srv, ticket))


def vh_server_result(srv, ticket, N, nsrc, want_u=True):
    """Returns (status, u (nsrc, N) complex128 or None, [stats dicts], latency_ms, queue_ms).
    N and nsrc must be the request's (the output buffers are sized by them)."""
    import numpy as np
    rec = _tickets.get((srv.value, ticket))
    if rec is not None and rec != (int(N), int(nsrc)):
        raise ValueError(f"ticket {ticket} was submitted with (N, nsrc) = {rec}")
    _tickets.pop((srv.value, ticket), None)
    u = np.zeros((nsrc, N), dtype=np.complex128) if want_u else None
    stats = (vh_solve_stats * nsrc)()
    lat, qms = _D(), _D()
    st = lib().vh_server_result(srv, ticket, u.ctypes.data if want_u else None, stats,
                                ctypes.byref(lat), ctypes.byref(qms))
    if st not in (VH_OK, VH_ENOCONV):
        check(st)
    return st, u, [s.as_dict() for s in stats], lat.value, qms.value


def vh_server_get_info(srv):
    info = vh_server_info()
    check(lib().vh_server_get_info(srv, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in info._fields_}


def vh_server_destroy(srv):
    check(lib().vh_server_destroy(srv))


def make_lfa_problem(**kw):
    """vh_lfa_problem with the library's defaults, overridden by keyword arguments."""
    p = vh_lfa_problem()
    lib().vh_lfa_problem_default(ctypes.byref(p))
    for k, v in kw.items():
        if k == "stream":
            p.stream = v if isinstance(v, int) or v is None else v.cuda_stream
        else:
            setattr(p, k, v)
    return p


def _dvec(values):
    return (_D * len(values))(*[float(v) for v in values])


def vh_lfa_factors(p, w, mu=True, rho=True):
    """Returns (mu list or None, rho list or None) for the damping values w."""
    nw = len(w)
    m = (_D * nw)() if mu else None
    r = (_D * nw)() if rho else None
    check(lib().vh_lfa_factors(ctypes.byref(p), nw, _dvec(w), m, r))
    return (list(m) if mu else None), (list(r) if rho else None)


def vh_lfa_factors_noalloc(p, w, mu=True, rho=True):
    """vh_lfa_factors through the allocation-free entry point (static device scratch)."""
    nw = len(w)
    m = (_D * nw)() if mu else None
    r = (_D * nw)() if rho else None
    check(lib().vh_lfa_factors_noalloc(ctypes.byref(p), nw, _dvec(w), m, r))
    return (list(m) if mu else None), (list(r) if rho else None)


def vh_lfa_tune(p, objective, w):
    """Returns (w_best, f_best): objective 0 = mu, 1 = rho."""
    wb, fb = _D(), _D()
    check(lib().vh_lfa_tune(ctypes.byref(p), objective, len(w), _dvec(w), ctypes.byref(wb),
                            ctypes.byref(fb)))
    return wb.value, fb.value


def vh_mg_iterate(hd, which, q, x, warmup, maxit, tol):
    """q, x: complex128 GPU tensors.  Returns (stats dict, residual history list)."""
    hist = (_D * (maxit + 1))()
    st = vh_cf_stats()
    n = _level_nodes(hd, 0)
    check(lib().vh_mg_iterate(hd, which, _ptr(q, "complex128", n), _ptr(x, "complex128", n), warmup,
                              maxit, float(tol), hist, ctypes.byref(st)))
    return st.as_dict(), list(hist[:st.iterations + 1])


def vh_tune_damping(dim, n, h, omega, kappa, gamma, shift, levels, patch, opt, q, objective,
                    warmup, maxit, tol, w):
    """Returns (chosen damping per level, scores[level][candidate])."""
    arr = (_I * 3)(*(list(n) + [1] * (3 - len(n))))
    nl = levels - 1
    damp = (_D * nl)()
    scores = (_D * (nl * len(w)))()
    check(lib().vh_tune_damping(dim, arr, float(h), float(omega), _ptr(kappa, "float64"),
                                _ptr(gamma, "float64"), float(shift), levels, patch,
                                ctypes.byref(opt) if opt is not None else None,
                                _ptr(q, "complex128"), objective, warmup, maxit, float(tol),
                                len(w), _dvec(w), damp, scores))
    return list(damp), [list(scores[l * len(w):(l + 1) * len(w)]) for l in range(nl)]


def vh_tune_shift(dim, n, h, omega, kappa, gamma, levels, patch, opt, q, alphas, warmup, maxit,
                  tol):
    """Returns (status, chosen alpha or None, c_f per candidate)."""
    arr = (_I * 3)(*(list(n) + [1] * (3 - len(n))))
    a = _D()
    cfs = (_D * len(alphas))()
    st = lib().vh_tune_shift(dim, arr, float(h), float(omega), _ptr(kappa, "float64"),
                             _ptr(gamma, "float64"), levels, patch,
                             ctypes.byref(opt) if opt is not None else None,
                             _ptr(q, "complex128"), len(alphas), _dvec(alphas), warmup, maxit,
                             float(tol), ctypes.byref(a), cfs)
    if st not in (VH_OK, VH_ENOCONV):
        check(st)
    return st, (a.value if st == VH_OK else None), list(cfs)


def make_options(**kw):
    """vh_options with defaults, overridden by keyword arguments; `damping` may be a list,
    `stream` a torch.cuda.Stream or raw handle."""
    o = vh_options_default()
    for k, v in kw.items():
        if k == "damping":
            o.ndamping = len(v)
            for i, w in enumerate(v):
                o.damping[i] = float(w)
        elif k == "stream":
            o.stream = v if isinstance(v, int) or v is None else v.cuda_stream
        else:
            setattr(o, k, v)
    return o
