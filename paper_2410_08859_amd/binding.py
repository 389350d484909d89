"""ctypes binding of libdd_uot.so: the C ABI of include/dd_uot.h, same names.

Argument marshalling only: every step of the solver runs in the HIP library.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdd_uot.so")

OK, EINVAL, ENOMEM, EHIP, ESLOT, ESTATE = 0, -1, -2, -3, -4, -5
GW_GREEDY, GW_SAFE, GW_SWIFT, GW_STAGGERED, GW_LINE, GW_OPT = 0, 1, 2, 3, 4, 5
INIT_BLOCK, INIT_PRODUCT = 0, 1
HIST_FIELDS = ("theta", "e_cur", "e_greedy", "n_updated", "point_iters", "max_inner",
               "n_unconverged", "n_overflow", "inner_iters", "algo_bytes", "lse_terms",
               "fallbacks")

EXPORTED = (
    "dd_uot_default_config", "dd_uot_init", "dd_uot_init_batch", "dd_uot_set_eps",
    "dd_uot_iterate", "dd_uot_history", "dd_uot_score", "dd_uot_marginals",
    "dd_uot_basic_marginal", "dd_uot_potentials", "dd_uot_backward", "dd_uot_set_timing",
    "dd_uot_kernel_time", "dd_uot_cell_stats", "dd_uot_synchronize", "dd_uot_num_problems", "dd_uot_destroy",
    "dd_uot_last_error", "dd_uot_refine", "dd_uot_default_multiscale",
    "dd_uot_solve_multiscale", "dd_uot_init_moved", "dd_uot_init_batch_moved",
    "dd_uot_backward_ypos", "dd_uot_set_graph", "dd_uot_autotune",
    "dd_uot_interpolate_potential", "dd_uot_global_sinkhorn", "dd_uot_init_duals",
    "dd_uot_launch_caps", "dd_uot_set_polish", "dd_uot_get_state", "dd_uot_set_state",
    "dd_uot_set_err", "dd_uot_set_gang", "dd_uot_global_sinkhorn_noalloc", "dd_uot_autotune_gang",
)


class dduot_config(C.Structure):
    _fields_ = [
        ("n1", C.c_int32), ("n2", C.c_int32),
        ("h", C.c_double),
        ("lambda_", C.c_double), ("eps", C.c_double),
        ("cell", C.c_int32), ("precision", C.c_int32), ("getweights", C.c_int32),
        ("init", C.c_int32),
        ("sinkhorn_err", C.c_double),
        ("sinkhorn_max_iter", C.c_int32), ("fixed_inner_iters", C.c_int32),
        ("trunc", C.c_double), ("lenience", C.c_double),
        ("box_margin", C.c_int32), ("box_cap", C.c_int32),
        ("translate", C.c_int32), ("fast_cap", C.c_int32),
        ("balance", C.c_int32), ("support_only", C.c_int32),
    ]


class dduot_iter_stats(C.Structure):
    _fields_ = [
        ("half_iters", C.c_int32), ("n_safe", C.c_int32),
        ("inner_iters", C.c_int64), ("point_iters", C.c_int64),
        ("max_inner", C.c_int32), ("n_unconverged", C.c_int32), ("n_overflow", C.c_int32),
        ("n_cells", C.c_int32),
    ]


class dduot_score(C.Structure):
    _fields_ = [
        ("tracked", C.c_double), ("primal", C.c_double), ("dual", C.c_double),
        ("pd_gap", C.c_double), ("rel_pd_gap", C.c_double),
        ("l1_err_x", C.c_double), ("l1_err_y", C.c_double),
        ("mass_x", C.c_double), ("mass_y", C.c_double),
        ("half_iters", C.c_int64), ("overflow", C.c_int32),
        ("polish_iters", C.c_int32), ("dual_polished", C.c_double),
        ("primal_polished", C.c_double), ("rel_gap_polished", C.c_double),
        ("nnz", C.c_int64), ("n_safe", C.c_int64), ("n_unconverged", C.c_int64),
    ]


class dduot_multiscale(C.Structure):
    _fields_ = [
        ("levels", C.c_int32), ("coarse_cell", C.c_int32),
        ("eps_start_h2", C.c_double), ("eps_end_h2", C.c_double),
        ("halves_per_stage", C.c_int32), ("stage_max_halves", C.c_int32),
        ("stage_gap", C.c_double),
        ("coarse_max_iter", C.c_int32), ("final_max_halves", C.c_int32),
        ("check_every", C.c_int32),
        ("target_rel_gap", C.c_double),
        ("dd_from", C.c_int32), ("global_max_iter", C.c_int32),
        ("global_tol", C.c_double),
        ("coarse_box_cap", C.c_int32), ("coarse_lenience", C.c_double),
        ("verbose", C.c_int32), ("polish_iters", C.c_int32),
        ("final_err_ratio", C.c_double), ("final_err_min", C.c_double),
    ]


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the HIP library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not built; run paper_2410_08859_amd/build.py "
                           "first")
    # One HIP runtime per process: when PyTorch is installed its runtime
    # (same soname) is loaded first, so the library and torch share it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    P = C.POINTER
    dp = P(C.c_double)
    H = C.c_void_p
    sig = {
        "dd_uot_default_config": (None, [P(dduot_config)]),
        "dd_uot_init": (C.c_int, [P(dduot_config), dp, dp, C.c_void_p, P(H)]),
        "dd_uot_init_batch": (C.c_int, [C.c_int32, P(dduot_config), P(dp), P(dp), C.c_void_p, P(H)]),
        "dd_uot_set_eps": (C.c_int, [H, C.c_int32, C.c_double]),
        "dd_uot_iterate": (C.c_int, [H, C.c_int32, P(dduot_iter_stats)]),
        "dd_uot_history": (C.c_int, [H, C.c_int32, C.c_int32, dp]),
        "dd_uot_score": (C.c_int, [H, C.c_int32, P(dduot_score)]),
        "dd_uot_marginals": (C.c_int, [H, C.c_int32, dp, dp]),
        "dd_uot_basic_marginal": (C.c_int, [H, C.c_int32, C.c_int32, P(C.c_int32), dp, C.c_int64]),
        "dd_uot_potentials": (C.c_int, [H, C.c_int32, dp, dp]),
        "dd_uot_backward": (C.c_int, [H, C.c_int32, C.c_double, dp, dp]),
        "dd_uot_set_timing": (C.c_int, [H, C.c_int32]),
        "dd_uot_kernel_time": (C.c_int, [H, P(C.c_int64), dp, dp]),
        "dd_uot_cell_stats": (C.c_int, [H, C.c_int32, C.c_int32, P(C.c_int32), P(C.c_int32), dp]),
        "dd_uot_set_gang": (C.c_int, [H, C.c_int32, C.c_int32, P(C.c_int32)]),
        "dd_uot_autotune_gang": (C.c_int, [H, P(C.c_int32), P(C.c_int32), dp]),
        "dd_uot_global_sinkhorn_noalloc": (C.c_int, [P(dduot_config), dp, dp, dp, dp, C.c_int32,
                                                     C.c_double, C.c_void_p, P(C.c_int32), dp]),
        "dd_uot_synchronize": (C.c_int, [H]),
        "dd_uot_num_problems": (C.c_int32, [H]),
        "dd_uot_destroy": (None, [H]),
        "dd_uot_last_error": (C.c_char_p, []),
        "dd_uot_refine": (C.c_int, [H, P(dduot_config), dp, dp, C.c_void_p, P(H)]),
        "dd_uot_init_moved": (C.c_int, [P(dduot_config), dp, dp, dp, C.c_void_p, P(H)]),
        "dd_uot_init_batch_moved": (C.c_int, [C.c_int32, P(dduot_config), P(dp), P(dp), P(dp),
                                              C.c_void_p, P(H)]),
        "dd_uot_backward_ypos": (C.c_int, [H, C.c_int32, C.c_double, dp]),
        "dd_uot_set_graph": (C.c_int, [H, C.c_int32]),
        "dd_uot_set_polish": (C.c_int, [H, C.c_int32]),
        "dd_uot_set_err": (C.c_int, [H, C.c_int32, C.c_double]),
        "dd_uot_get_state": (C.c_int, [H, P(C.c_int32), dp, C.c_int64, P(C.c_int64), dp, dp, dp,
                                       P(C.c_int32), P(C.c_int64)]),
        "dd_uot_set_state": (C.c_int, [H, P(C.c_int32), dp, C.c_int64, dp, dp, dp, P(C.c_int32),
                                       C.c_int64, C.c_int32]),
        "dd_uot_autotune": (C.c_int, [H, P(C.c_int32), dp]),
        "dd_uot_default_multiscale": (None, [P(dduot_multiscale)]),
        "dd_uot_solve_multiscale": (C.c_int, [P(dduot_config), P(dduot_multiscale), dp, dp,
                                              C.c_void_p, P(H), dp, C.c_int32, P(C.c_int32)]),
        "dd_uot_interpolate_potential": (C.c_int, [dp, C.c_int32, C.c_int32, dp, C.c_void_p]),
        "dd_uot_global_sinkhorn": (C.c_int, [P(dduot_config), dp, dp, dp, dp, C.c_int32, C.c_double,
                                             C.c_void_p, P(C.c_int32), dp]),
        "dd_uot_init_duals": (C.c_int, [P(dduot_config), dp, dp, dp, dp, C.c_void_p, P(H)]),
        "dd_uot_launch_caps": (C.c_int, [H, P(C.c_int32), P(C.c_int32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class DDUOTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dd_uot error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc < 0:
        raise DDUOTError(rc, load().dd_uot_last_error().decode())
    return rc


def _is_tensor(a) -> bool:
    return hasattr(a, "data_ptr") and hasattr(a, "is_contiguous")


def _dptr(a):
    """double* of a NumPy array (host) or of a contiguous float64 torch
    tensor (host or device memory: the library tells them apart)."""
    if _is_tensor(a):
        return C.cast(C.c_void_p(a.data_ptr()), C.POINTER(C.c_double))
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _tensor_arg(a, n):
    import torch
    if a.dtype != torch.float64 or not a.is_contiguous() or a.numel() != n:
        raise ValueError("tensor arguments must be contiguous float64 with the grid's size")
    return a


def _out(n, given):
    """A given output buffer (NumPy array or tensor of n doubles), else a new array."""
    if given is None:
        return np.zeros(n)
    if _is_tensor(given):
        return _tensor_arg(given, n)
    if not (isinstance(given, np.ndarray) and given.dtype == np.float64 and given.flags.c_contiguous
            and given.size == n):
        raise ValueError("output arrays must be contiguous float64 with the grid's size")
    return given


def _shaped(a, n1, n2):
    return a.view(n1, n2) if _is_tensor(a) else a.reshape(n1, n2)


def dd_uot_default_config(**kw) -> dduot_config:
    cfg = dduot_config()
    load().dd_uot_default_config(C.byref(cfg))
    for k, v in kw.items():
        setattr(cfg, "lambda_" if k == "lam" else k, v)
    return cfg


def _grid(a, n1, n2):
    if _is_tensor(a):
        return _tensor_arg(a, n1 * n2)
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != n1 * n2:
        raise ValueError("marginal size does not match the grid")
    return a


def dd_uot_init(cfg: dduot_config, mu, nu, stream=None):
    mu = _grid(mu, cfg.n1, cfg.n2)
    nu = _grid(nu, cfg.n1, cfg.n2)
    h = C.c_void_p()
    _check(load().dd_uot_init(C.byref(cfg), _dptr(mu), _dptr(nu), stream, C.byref(h)))
    return h


def dd_uot_init_batch(cfgs, mus, nus, stream=None):
    n = len(cfgs)
    arr = (dduot_config * n)(*cfgs)
    mus = [_grid(m, c.n1, c.n2) for m, c in zip(mus, cfgs)]
    nus = [_grid(v, c.n1, c.n2) for v, c in zip(nus, cfgs)]
    pm = (C.POINTER(C.c_double) * n)(*[_dptr(m) for m in mus])
    pn = (C.POINTER(C.c_double) * n)(*[_dptr(v) for v in nus])
    h = C.c_void_p()
    _check(load().dd_uot_init_batch(n, arr, pm, pn, stream, C.byref(h)))
    return h


def dd_uot_set_eps(h, prob, eps):
    _check(load().dd_uot_set_eps(h, prob, eps))


def dd_uot_iterate(h, n_half_iters, stats=True):
    st = dduot_iter_stats() if stats else None
    _check(load().dd_uot_iterate(h, n_half_iters, C.byref(st) if st is not None else None))
    if st is None:
        return None
    return {f: getattr(st, f) for f, _ in dduot_iter_stats._fields_}


def dd_uot_history(h, prob, max_records=4096):
    out = np.zeros((max_records, len(HIST_FIELDS)))
    n = _check(load().dd_uot_history(h, prob, max_records, _dptr(out)))
    return out[:n]


def dd_uot_score(h, prob=0):
    s = dduot_score()
    _check(load().dd_uot_score(h, prob, C.byref(s)))
    return {f: getattr(s, f) for f, _ in dduot_score._fields_}


def dd_uot_marginals(h, prob, n1, n2, out=None):
    """(P_X, P_Y) of the state plan; `out`: two buffers to fill (arrays or
    float64 tensors, host or device)."""
    px = _out(n1 * n2, out[0] if out else None)
    py = _out(n1 * n2, out[1] if out else None)
    _check(load().dd_uot_marginals(h, prob, _dptr(px), _dptr(py)))
    return _shaped(px, n1, n2), _shaped(py, n1, n2)


def dd_uot_basic_marginal(h, prob, basic):
    box = (C.c_int32 * 4)()
    _check(load().dd_uot_basic_marginal(h, prob, basic, box, None, 0))
    o1, o2, l1, l2 = list(box)
    vals = np.zeros(max(l1 * l2, 1))
    _check(load().dd_uot_basic_marginal(h, prob, basic, box, _dptr(vals), vals.size))
    return (o1, o2, vals[: l1 * l2].reshape(l1, l2).copy())


def dd_uot_potentials(h, prob, n1, n2, beta=True):
    a = np.zeros(n1 * n2)
    b = np.zeros(n1 * n2) if beta else None
    _check(load().dd_uot_potentials(h, prob, _dptr(a), _dptr(b) if beta else None))
    return a.reshape(n1, n2), (b.reshape(n1, n2) if beta else None)


def dd_uot_backward(h, prob, n1, n2, gout=1.0, out=None):
    """gout * (dW/dmu, dW/dnu); `out`: two buffers to fill (arrays or float64
    tensors, host or device)."""
    dmu = _out(n1 * n2, out[0] if out else None)
    dnu = _out(n1 * n2, out[1] if out else None)
    _check(load().dd_uot_backward(h, prob, gout, _dptr(dmu), _dptr(dnu)))
    return _shaped(dmu, n1, n2), _shaped(dnu, n1, n2)


def dd_uot_set_timing(h, enable=True):
    _check(load().dd_uot_set_timing(h, 1 if enable else 0))


def dd_uot_kernel_time(h):
    n = C.c_int64()
    ms = C.c_double()
    by = C.c_double()
    _check(load().dd_uot_kernel_time(h, C.byref(n), C.byref(ms), C.byref(by)))
    return n.value, ms.value, by.value


def dd_uot_cell_stats(h, part):
    """Y-boxes (n, 4), inner iterations (n,) and terms (n,) of the cells of `part`."""
    lib = load()
    n = max(1, _check(lib.dd_uot_cell_stats(h, part, 1 << 30, None, None, None)))
    boxes = np.zeros((n, 4), np.int32)
    iters = np.zeros(n, np.int32)
    terms = np.zeros(n, np.float64)
    rc = lib.dd_uot_cell_stats(h, part, n, boxes.ctypes.data_as(C.POINTER(C.c_int32)),
                               iters.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(terms))
    _check(rc if rc < 0 else 0)
    return boxes, iters, terms


def dd_uot_synchronize(h):
    _check(load().dd_uot_synchronize(h))


def dd_uot_num_problems(h):
    return load().dd_uot_num_problems(h)


def dd_uot_destroy(h):
    if h:
        load().dd_uot_destroy(h)


def dd_uot_refine(coarse, cfg: dduot_config, mu, nu, stream=None):
    mu = _grid(mu, cfg.n1, cfg.n2)
    nu = _grid(nu, cfg.n1, cfg.n2)
    h = C.c_void_p()
    _check(load().dd_uot_refine(coarse, C.byref(cfg), _dptr(mu), _dptr(nu), stream, C.byref(h)))
    return h


def dd_uot_interpolate_potential(coarse, stream=None):
    """(n1c, n2c) potential -> (2 n1c, 2 n2c) on the device kernel."""
    a = np.ascontiguousarray(coarse, dtype=np.float64)
    if a.ndim != 2:
        raise ValueError("coarse potential must be 2-D")
    out = np.empty((2 * a.shape[0], 2 * a.shape[1]))
    _check(load().dd_uot_interpolate_potential(_dptr(a), a.shape[0], a.shape[1], _dptr(out), stream))
    return out


def dd_uot_global_sinkhorn(cfg: dduot_config, mu, nu, beta0=None, max_iter=1000, tol=0.0,
                           stream=None):
    """Returns dict(alpha, beta, iters, pd) (grids of the config's shape)."""
    mu = _grid(mu, cfg.n1, cfg.n2)
    nu = _grid(nu, cfg.n1, cfg.n2)
    beta = np.zeros((cfg.n1, cfg.n2)) if beta0 is None else \
        np.array(beta0, dtype=np.float64).reshape(cfg.n1, cfg.n2)
    alpha = np.empty((cfg.n1, cfg.n2))
    it = C.c_int32()
    pd = C.c_double()
    _check(load().dd_uot_global_sinkhorn(C.byref(cfg), _dptr(mu), _dptr(nu), _dptr(alpha),
                                         _dptr(beta), int(max_iter), float(tol), stream,
                                         C.byref(it), C.byref(pd)))
    return dict(alpha=alpha, beta=beta, iters=it.value, pd=pd.value)


def dd_uot_global_sinkhorn_noalloc(cfg: dduot_config, mu, nu, alpha, beta, max_iter=1000,
                                   tol=0.0, stream=None):
    """The global Sinkhorn on caller-owned device buffers (float64 tensors of
    n1*n2 entries: mu, nu in; alpha out; beta in and out); no allocation.
    Returns dict(iters, pd)."""
    n = cfg.n1 * cfg.n2
    for t in (mu, nu, alpha, beta):
        if not _is_tensor(t):
            raise ValueError("the no-allocation entry point takes device tensors")
        _tensor_arg(t, n)
    it = C.c_int32()
    pd = C.c_double()
    _check(load().dd_uot_global_sinkhorn_noalloc(C.byref(cfg), _dptr(mu), _dptr(nu), _dptr(alpha),
                                                 _dptr(beta), int(max_iter), float(tol), stream,
                                                 C.byref(it), C.byref(pd)))
    return dict(iters=it.value, pd=pd.value)


def dd_uot_init_duals(cfg: dduot_config, mu, nu, alpha, beta, stream=None):
    mu = _grid(mu, cfg.n1, cfg.n2)
    nu = _grid(nu, cfg.n1, cfg.n2)
    a = _grid(alpha, cfg.n1, cfg.n2)
    b = _grid(beta, cfg.n1, cfg.n2)
    h = C.c_void_p()
    _check(load().dd_uot_init_duals(C.byref(cfg), _dptr(mu), _dptr(nu), _dptr(a), _dptr(b), stream,
                                    C.byref(h)))
    return h


def dd_uot_launch_caps(h):
    """(fast tier box side, slot box side) of the cell-solve launches."""
    a, b = C.c_int32(), C.c_int32()
    _check(load().dd_uot_launch_caps(h, C.byref(a), C.byref(b)))
    return a.value, b.value


def dd_uot_default_multiscale(**kw) -> dduot_multiscale:
    m = dduot_multiscale()
    load().dd_uot_default_multiscale(C.byref(m))
    for k, v in kw.items():
        setattr(m, k, v)
    return m


def dd_uot_solve_multiscale(cfg: dduot_config, ms: dduot_multiscale, mu, nu, stream=None,
                            trace_cap=1024):
    """Returns (handle, trace) with trace rows (half-iterations, elapsed ms,
    certificate rel. gap, DD-plan rel. gap, polished rel. gap)."""
    mu = _grid(mu, cfg.n1, cfg.n2)
    nu = _grid(nu, cfg.n1, cfg.n2)
    h = C.c_void_p()
    tr = np.zeros(5 * trace_cap)
    n = C.c_int32()
    _check(load().dd_uot_solve_multiscale(C.byref(cfg), C.byref(ms), _dptr(mu), _dptr(nu), stream,
                                          C.byref(h), _dptr(tr), trace_cap, C.byref(n)))
    return h, tr[: 5 * n.value].reshape(-1, 5)


def dd_uot_init_moved(cfg: dduot_config, mu, nu, ypos, stream=None):
    """ypos: (n1, n2, 2) coordinates y' of the Y points."""
    mu = _grid(mu, cfg.n1, cfg.n2)
    nu = _grid(nu, cfg.n1, cfg.n2)
    yp = np.ascontiguousarray(ypos, dtype=np.float64)
    if yp.size != 2 * cfg.n1 * cfg.n2:
        raise ValueError("ypos must hold n1*n2*2 coordinates")
    h = C.c_void_p()
    _check(load().dd_uot_init_moved(C.byref(cfg), _dptr(mu), _dptr(nu), _dptr(yp), stream,
                                    C.byref(h)))
    return h


def dd_uot_init_batch_moved(cfgs, mus, nus, yposs, stream=None):
    n = len(cfgs)
    arr = (dduot_config * n)(*cfgs)
    mus = [_grid(m, c.n1, c.n2) for m, c in zip(mus, cfgs)]
    nus = [_grid(v, c.n1, c.n2) for v, c in zip(nus, cfgs)]
    yps = [np.ascontiguousarray(y, dtype=np.float64) for y in yposs]
    pm = (C.POINTER(C.c_double) * n)(*[_dptr(m) for m in mus])
    pn = (C.POINTER(C.c_double) * n)(*[_dptr(v) for v in nus])
    py = (C.POINTER(C.c_double) * n)(*[_dptr(y) for y in yps])
    h = C.c_void_p()
    _check(load().dd_uot_init_batch_moved(n, arr, pm, pn, py, stream, C.byref(h)))
    return h


def dd_uot_backward_ypos(h, prob, n1, n2, gout=1.0):
    out = np.zeros(2 * n1 * n2)
    _check(load().dd_uot_backward_ypos(h, prob, gout, _dptr(out)))
    return out.reshape(n1, n2, 2)


def dd_uot_set_gang(h, G, wgs_per_cu=2):
    """Gangs of G workgroups for the wide cells; returns (G in effect, workgroups)."""
    nwg = C.c_int32()
    g = _check(load().dd_uot_set_gang(h, G, wgs_per_cu, C.byref(nwg)))
    return g, nwg.value


def dd_uot_set_graph(h, enable=True):
    _check(load().dd_uot_set_graph(h, 1 if enable else 0))


def dd_uot_set_err(h, prob, err):
    _check(load().dd_uot_set_err(h, prob, err))


def dd_uot_set_polish(h, n_iters):
    _check(load().dd_uot_set_polish(h, n_iters))


def dd_uot_get_state(h, n1, n2, nbasic):
    """dict(boxes (nbasic, 4) int32, values, px, hbar, abar, warm, k)."""
    lib = load()
    nv = C.c_int64()
    _check(lib.dd_uot_get_state(h, None, None, 0, C.byref(nv), None, None, None, None, None))
    boxes = np.zeros(4 * nbasic, dtype=np.int32)
    vals = np.zeros(max(nv.value, 1))
    px, abar, hbar = np.zeros(n1 * n2), np.zeros(n1 * n2), np.zeros(nbasic)
    warm = np.zeros(nbasic, dtype=np.int32)
    k = C.c_int64()
    _check(lib.dd_uot_get_state(h, boxes.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(vals), vals.size,
                                C.byref(nv), _dptr(px), _dptr(hbar), _dptr(abar),
                                warm.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(k)))
    return dict(boxes=boxes.reshape(nbasic, 4), values=vals[: nv.value], px=px.reshape(n1, n2),
                hbar=hbar, abar=abar.reshape(n1, n2), warm=warm, k=k.value)


def dd_uot_set_state(h, state, force_greedy=False):
    boxes = np.ascontiguousarray(state["boxes"], dtype=np.int32).ravel()
    vals = np.ascontiguousarray(state["values"], dtype=np.float64)
    warm = np.ascontiguousarray(state["warm"], dtype=np.int32)
    px = np.ascontiguousarray(state["px"], dtype=np.float64).ravel()
    abar = np.ascontiguousarray(state["abar"], dtype=np.float64).ravel()
    hbar = np.ascontiguousarray(state["hbar"], dtype=np.float64)
    _check(load().dd_uot_set_state(h, boxes.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(vals),
                                   vals.size, _dptr(px), _dptr(hbar), _dptr(abar),
                                   warm.ctypes.data_as(C.POINTER(C.c_int32)), int(state["k"]),
                                   1 if force_greedy else 0))


def dd_uot_autotune_gang(h):
    """Returns (G, workgroups per CU chosen, [ms of one workgroup per wide cell,
    then of (2,2), (4,1), (4,2), (8,1), (8,2), (16,2); -1 = does not apply])."""
    g = C.c_int32()
    w = C.c_int32()
    ms = np.zeros(7)
    _check(load().dd_uot_autotune_gang(h, C.byref(g), C.byref(w), _dptr(ms)))
    return g.value, w.value, ms


def dd_uot_autotune(h):
    """Returns (threads per cell chosen, [ms for 64, 128, 256 threads; -1 = not admissible])."""
    c = C.c_int32()
    ms = np.zeros(3)
    _check(load().dd_uot_autotune(h, C.byref(c), _dptr(ms)))
    return c.value, ms
