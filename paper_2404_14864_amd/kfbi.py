"""Thin Python binding of the KFBI HIP library (include/kfbi.h).

Argument marshalling only: every function below forwards to the C entry
point of the same name in libkfbi.so, passing torch tensors as raw device
pointers and the current torch stream as the domain stream.  Nothing here
computes any part of the method; if the library is missing the import of
the functions fails loudly.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkfbi.so")

KFBI_OK, KFBI_EINVAL, KFBI_EDOMAIN, KFBI_ENOMEM, KFBI_ENOCONV, KFBI_EDEVICE, KFBI_ENOTSUP = range(7)
CURVES = {"disk": 0, "ellipse": 1, "star": 2}
KFBI_REAL, KFBI_COMPLEX = 0, 1
KFBI_PREC_FP64, KFBI_PREC_MIXED = 0, 1
KFBI_SOLVE_ASYNC = 1
KFBI_BATCH_NO_TUNE = 2
KFBI_SOLVE_RICHARDSON = 4
KFBI_HEAT, KFBI_WAVE, KFBI_SCHRODINGER = 0, 1, 2
KFBI_BC_DIRICHLET, KFBI_BC_NEUMANN = 0, 1
KFBI_SPLIT_STRANG, KFBI_SPLIT_GODUNOV = 0, 1


class KfbiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("kfbi error %d: %s" % (code, msg))
        self.code = code


class DomainDesc(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("M", ctypes.c_int32), ("Nb", ctypes.c_int32),
                ("kind", ctypes.c_int32), ("lobes", ctypes.c_int32),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("R", ctypes.c_double),
                ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("r0", ctypes.c_double), ("amp", ctypes.c_double),
                ("scalar", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class DomainInfo(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("Nb", ctypes.c_int32), ("L", ctypes.c_double),
                ("h", ctypes.c_double), ("n_inside", ctypes.c_int32),
                ("n_irregular", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("scalar", ctypes.c_int32), ("device_bytes", ctypes.c_uint64),
                ("device_bytes_max", ctypes.c_uint64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("fixed_iters", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("gamma", ctypes.c_double)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_resid", ctypes.c_double), ("refinements", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("device_ms", ctypes.c_double)]

    def as_dict(self):
        return {"iters": self.iters, "converged": bool(self.converged),
                "rel_resid": self.rel_resid, "refinements": self.refinements,
                "device_ms": self.device_ms}


class StepParams(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("theta", ctypes.c_double),
                ("diffusivity", ctypes.c_double), ("w", ctypes.c_double),
                ("v_grid", ctypes.c_void_p), ("v_gamma", ctypes.c_void_p),
                ("bc", ctypes.c_int32), ("split", ctypes.c_int32)]


class KernelProf(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


KERNELS = ("tridiag_sparse", "tridiag_dense", "dst", "idst", "eval_nodes", "corrections",
           "extract", "arnoldi")

_lib = None
_P = ctypes.c_void_p


def lib():
    """Load libkfbi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libkfbi.so not built; run python -m paper_2404_14864_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "kfbi_last_error": ([], ctypes.c_char_p),
        "kfbi_domain_create": ([ctypes.POINTER(DomainDesc), ctypes.POINTER(_P)], ctypes.c_int),
        "kfbi_domain_destroy": ([_P], ctypes.c_int),
        "kfbi_domain_get_info": ([_P, ctypes.POINTER(DomainInfo)], ctypes.c_int),
        "kfbi_domain_copy_classification": ([_P, _P], ctypes.c_int),
        "kfbi_domain_copy_boundary": ([_P, _P], ctypes.c_int),
        "kfbi_domain_copy_normals": ([_P, _P], ctypes.c_int),
        "kfbi_domain_copy_edges": ([_P, _P, _P], ctypes.c_int),
        "kfbi_grid_solve": ([_P, ctypes.c_double, ctypes.c_double, _P, _P], ctypes.c_int),
        "kfbi_grid_solve_noalloc": ([_P, ctypes.c_double, ctypes.c_double, _P, _P], ctypes.c_int),
        "kfbi_interface_apply": ([_P, ctypes.c_double, ctypes.c_double, _P, _P, _P, _P, _P], ctypes.c_int),
        "kfbi_helmholtz_solve": ([_P, ctypes.c_double, ctypes.c_double, _P, _P, _P, _P, _P,
                                  ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats)], ctypes.c_int),
        "kfbi_neumann_solve": ([_P, ctypes.c_double, ctypes.c_double, _P, _P, _P, _P, _P, _P,
                                ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats)], ctypes.c_int),
        "kfbi_stepper_create": ([_P, ctypes.c_int32, ctypes.POINTER(StepParams), ctypes.POINTER(_P)], ctypes.c_int),
        "kfbi_stepper_destroy": ([_P], ctypes.c_int),
        "kfbi_stepper_init": ([_P] + [_P] * 8, ctypes.c_int),
        "kfbi_step_heat": ([_P, _P, _P, _P, _P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats)], ctypes.c_int),
        "kfbi_step_wave": ([_P, _P, _P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats)], ctypes.c_int),
        "kfbi_step_schrodinger": ([_P, _P, _P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats)], ctypes.c_int),
        "kfbi_profile_enable": ([_P, ctypes.c_int32], ctypes.c_int),
        "kfbi_profile_read": ([_P, ctypes.POINTER(KernelProf)], ctypes.c_int),
        "kfbi_stepper_state_bytes": ([_P, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "kfbi_stepper_get_state": ([_P, _P, ctypes.c_uint64], ctypes.c_int),
        "kfbi_stepper_set_state": ([_P, _P, ctypes.c_uint64], ctypes.c_int),
        "kfbi_batch_create": ([ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(_P)], ctypes.c_int),
        "kfbi_batch_destroy": ([_P], ctypes.c_int),
        "kfbi_batch_helmholtz": ([_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                  ctypes.POINTER(_P), ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats)],
                                 ctypes.c_int),
        "kfbi_batch_step": ([_P, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(_P),
                             ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(SolveOpts),
                             ctypes.POINTER(SolveStats)], ctypes.c_int),
        "kfbi_batch_tuning": ([_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "kfbi_profile_replay": ([_P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


EXPORTED = ("kfbi_last_error", "kfbi_domain_create", "kfbi_domain_destroy", "kfbi_domain_get_info",
            "kfbi_domain_copy_classification", "kfbi_domain_copy_boundary", "kfbi_domain_copy_edges",
            "kfbi_grid_solve", "kfbi_interface_apply", "kfbi_helmholtz_solve", "kfbi_stepper_create",
            "kfbi_stepper_destroy", "kfbi_stepper_init", "kfbi_step_heat", "kfbi_step_wave",
            "kfbi_step_schrodinger", "kfbi_profile_enable", "kfbi_profile_read", "kfbi_profile_replay",
            "kfbi_stepper_state_bytes", "kfbi_stepper_get_state", "kfbi_stepper_set_state",
            "kfbi_batch_create", "kfbi_batch_destroy", "kfbi_batch_helmholtz", "kfbi_batch_tuning",
            "kfbi_batch_step", "kfbi_neumann_solve", "kfbi_domain_copy_normals", "kfbi_grid_solve_noalloc")


def kfbi_profile_enable(h, on=True):
    _check(lib().kfbi_profile_enable(h, 1 if on else 0))


def kfbi_profile_read(h):
    arr = (KernelProf * len(KERNELS))()
    _check(lib().kfbi_profile_read(h, arr))
    return {name: {"launches": int(arr[i].launches), "total_ms": arr[i].total_ms,
                   "bytes": arr[i].bytes} for i, name in enumerate(KERNELS)}


# ---- batches ---------------------------------------------------------------
def kfbi_batch_create(domains):
    """A batch of domain handles of one scalar type (all real or all
    complex) on one stream, solved together."""
    n = len(domains)
    arr = (_P * n)(*[d.value if isinstance(d, ctypes.c_void_p) else d for d in domains])
    out = _P()
    _check(lib().kfbi_batch_create(arr, n, ctypes.byref(out)))
    _BATCHES[out.value] = [_hv(d) for d in domains]
    return out


def kfbi_batch_destroy(b):
    _check(lib().kfbi_batch_destroy(b))
    _BATCHES.pop(_hv(b), None)


def _batch_doms(b, n):
    doms = _BATCHES.get(_hv(b))
    if doms is None:
        raise ValueError("unknown batch handle (not created by kfbi_batch_create, or destroyed)")
    if n != len(doms):
        raise ValueError("the batch has %d members; got %d entries" % (len(doms), n))
    return doms


def _member_ptrs(doms, lst, name, grid):
    if lst is None:
        return None
    if len(lst) != len(doms):
        raise ValueError("%s needs one entry per member (%d), got %d" % (name, len(doms), len(lst)))
    chk = _grid if grid else _gam
    return (_P * len(doms))(*[(chk(h, t, "%s[%d]" % (name, q)).value if t is not None else None)
                              for q, (h, t) in enumerate(zip(doms, lst))])


def kfbi_batch_helmholtz(b, kappas, f_grid, f_gamma, g_gamma, u_grid_out=None, phi_inout=None, opts=None):
    """Member q solves lap u - kappas[q] u = f_grid[q] with u = g_gamma[q] on
    Gamma; the arrays are lists of CUDA tensors of the batch's element type
    (float64, or complex128 for a batch of complex domains, whose kappas may
    be complex); u_grid_out and phi_inout may be None or contain None.
    Returns the per-member stats."""
    n = len(kappas)
    doms = _batch_doms(b, n)
    ks = [complex(k) for k in kappas]
    kap = (ctypes.c_double * n)(*[k.real for k in ks])
    kim = (ctypes.c_double * n)(*[k.imag for k in ks]) if any(k.imag != 0.0 for k in ks) else None
    stats = (SolveStats * n)()
    code = lib().kfbi_batch_helmholtz(b, kap, kim, _member_ptrs(doms, f_grid, "f_grid", True),
                                      _member_ptrs(doms, f_gamma, "f_gamma", False),
                                      _member_ptrs(doms, g_gamma, "g_gamma", False),
                                      _member_ptrs(doms, u_grid_out, "u_grid_out", True),
                                      _member_ptrs(doms, phi_inout, "phi_inout", False), _opts(opts), stats)
    _check(code, allow=(KFBI_ENOCONV,))
    return [stats[q].as_dict() for q in range(n)]


def kfbi_batch_step(b, steppers, g_next, u_out, active=None, src_grid=None, src_gamma=None, opts=None):
    """One time step of the active member steppers (heat or wave in a real
    batch, Schroedinger in a complex one; member q on the batch's domain q)
    with their solves batched.  g_next, u_out, src_grid, src_gamma: lists of
    CUDA tensors of the batch's element type (None entries for members not
    active or without sources); active: booleans (None: all).  Returns the
    per-member stats."""
    n = len(steppers)
    doms = _batch_doms(b, n)
    for q, x in enumerate(steppers):
        if _stepper_dom(x) != doms[q]:
            raise ValueError("steppers[%d] is not on the batch's member domain %d" % (q, q))
    if active is not None and len(active) != n:
        raise ValueError("active needs one entry per member (%d), got %d" % (n, len(active)))
    st = (_P * n)(*[_hv(x) for x in steppers])
    act = None if active is None else (ctypes.c_uint8 * n)(*[1 if a else 0 for a in active])
    stats = (SolveStats * n)()
    code = lib().kfbi_batch_step(b, st, act, _member_ptrs(doms, g_next, "g_next", False),
                                 _member_ptrs(doms, src_grid, "src_grid", True),
                                 _member_ptrs(doms, src_gamma, "src_gamma", False),
                                 _member_ptrs(doms, u_out, "u_out", True), _opts(opts), stats)
    _check(code, allow=(KFBI_ENOCONV,))
    return [stats[q].as_dict() for q in range(n)]


TUNING_KINDS = ("sparse64", "dense64", "sparse32")


def kfbi_batch_tuning(b):
    """Tridiagonal launch shape per class of equal M and solve kind:
    dicts {M, kind, modes_per_wg, staged, tuned, register_rows, us}."""
    n = ctypes.c_int32(0)
    _check(lib().kfbi_batch_tuning(b, 0, None, None, ctypes.byref(n)))
    rows = (ctypes.c_int32 * (6 * max(n.value, 1)))()
    us = (ctypes.c_double * max(n.value, 1))()
    _check(lib().kfbi_batch_tuning(b, n.value, rows, us, ctypes.byref(n)))
    out = []
    for r in range(n.value):
        M, kind, mb, st, tuned, reg = rows[6 * r:6 * r + 6]
        out.append({"M": M, "kind": TUNING_KINDS[kind], "modes_per_wg": mb, "staged": bool(st),
                    "tuned": bool(tuned), "register_rows": bool(reg), "us": us[r] if tuned else None})
    return out


def kfbi_profile_replay(h, kind, reps):
    """Average launch duration (ms) of `reps` back-to-back launches of one
    grid-solve kernel ("tridiag_sparse", "tridiag_dense" or "eval_nodes") and
    its algorithmic bytes per launch."""
    ms, by = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().kfbi_profile_replay(h, KERNELS.index(kind), int(reps), ctypes.byref(ms), ctypes.byref(by)))
    return ms.value, by.value


def _check(code, allow=()):
    if code != KFBI_OK and code not in allow:
        raise KfbiError(code, lib().kfbi_last_error().decode())
    return code


def _ptr(t, dtype=None, numel=None, name="array"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, got %d" % (name, numel, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


# What the wrappers know of the handles they created: every array argument is
# checked against its domain (element type and length) before the call, so a
# wrong dtype or a short tensor is refused on the host instead of being read
# or written past its end on the device.
_DOMAINS = {}    # domain handle value -> (M, Nb, complex?)
_STEPPERS = {}   # stepper handle value -> domain handle value
_BATCHES = {}    # batch handle value -> [domain handle values]


def _hv(h):
    return h.value if isinstance(h, ctypes.c_void_p) else h


def _meta(h):
    v = _hv(h)
    m = _DOMAINS.get(v)
    if m is None:
        info = DomainInfo()
        _check(lib().kfbi_domain_get_info(h, ctypes.byref(info)))
        m = (info.M, info.Nb, info.scalar == KFBI_COMPLEX)
        _DOMAINS[v] = m
    return m


def _stepper_dom(s):
    v = _hv(s)
    if v not in _STEPPERS:
        raise ValueError("unknown stepper handle (not created by kfbi_stepper_create, or destroyed)")
    return _STEPPERS[v]


def _grid(h, t, name):
    """A grid array ((M+1)^2 elements of the domain's type) or None."""
    M, _, c = _meta(h)
    return _ptr(t, torch.complex128 if c else torch.float64, (M + 1) * (M + 1), name)


def _gam(h, t, name):
    """A Gamma array (Nb elements of the domain's type) or None."""
    _, Nb, c = _meta(h)
    return _ptr(t, torch.complex128 if c else torch.float64, Nb, name)


def _opts(opts):
    if opts is None:
        return None
    o = SolveOpts(tol=opts.get("tol", 0.0), max_iter=opts.get("max_iter", 0),
                  restart=opts.get("restart", 0), fixed_iters=opts.get("fixed_iters", 0),
                  precision=opts.get("precision", -1),
                  flags=(KFBI_SOLVE_ASYNC if opts.get("async", False) else 0)
                  | (KFBI_BATCH_NO_TUNE if opts.get("no_tune", False) else 0)
                  | (KFBI_SOLVE_RICHARDSON if opts.get("solver", "gmres") == "richardson" else 0),
                  gamma=float(opts.get("gamma", 0.0)))
    return ctypes.byref(o)


# ---- domain ----------------------------------------------------------------
def kfbi_domain_create(desc, scalar=KFBI_REAL, precision=KFBI_PREC_FP64, stream=None):
    """desc: a workload descriptor dict (kind, cx, cy, R, a, b, r0, amp, lobes,
    L, M, Nb).  Returns an opaque domain handle."""
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    d = DomainDesc(L=desc["L"], M=desc["M"], Nb=desc["Nb"], kind=CURVES[desc["kind"]],
                   lobes=int(desc.get("lobes", 0)), cx=desc.get("cx", 0.0), cy=desc.get("cy", 0.0),
                   R=desc.get("R", 0.0), a=desc.get("a", 0.0), b=desc.get("b", 0.0),
                   r0=desc.get("r0", 0.0), amp=desc.get("amp", 0.0), scalar=scalar,
                   precision=precision, stream=ctypes.c_void_p(stream))
    h = _P()
    _check(lib().kfbi_domain_create(ctypes.byref(d), ctypes.byref(h)))
    _DOMAINS[h.value] = (desc["M"], desc["Nb"], scalar == KFBI_COMPLEX)
    return h


def kfbi_domain_destroy(h):
    _check(lib().kfbi_domain_destroy(h))
    _DOMAINS.pop(_hv(h), None)


def kfbi_domain_get_info(h):
    info = DomainInfo()
    _check(lib().kfbi_domain_get_info(h, ctypes.byref(info)))
    return {"M": info.M, "Nb": info.Nb, "L": info.L, "h": info.h, "n_inside": info.n_inside,
            "n_irregular": info.n_irregular, "n_edges": info.n_edges,
            "scalar": info.scalar, "device_bytes": int(info.device_bytes),
            "device_bytes_max": int(info.device_bytes_max)}


def kfbi_domain_copy_classification(h):
    import numpy as np
    info = kfbi_domain_get_info(h)
    out = np.zeros((info["M"] + 1) * (info["M"] + 1), dtype=np.uint8)
    _check(lib().kfbi_domain_copy_classification(h, out.ctypes.data_as(ctypes.c_void_p)))
    return out.reshape(info["M"] + 1, info["M"] + 1)


def kfbi_domain_copy_boundary(h):
    import numpy as np
    info = kfbi_domain_get_info(h)
    out = np.zeros(2 * info["Nb"], dtype=np.float64)
    _check(lib().kfbi_domain_copy_boundary(h, out.ctypes.data_as(ctypes.c_void_p)))
    return out[0::2].copy(), out[1::2].copy()


def kfbi_domain_copy_normals(h):
    import numpy as np
    info = kfbi_domain_get_info(h)
    out = np.zeros(2 * info["Nb"], dtype=np.float64)
    _check(lib().kfbi_domain_copy_normals(h, out.ctypes.data_as(ctypes.c_void_p)))
    return out[0::2].copy(), out[1::2].copy()


def kfbi_domain_copy_edges(h):
    import numpy as np
    info = kfbi_domain_get_info(h)
    n = info["n_edges"]
    pq = np.zeros(2 * n, dtype=np.int32)
    xyt = np.zeros(3 * n, dtype=np.float64)
    _check(lib().kfbi_domain_copy_edges(h, pq.ctypes.data_as(ctypes.c_void_p),
                                        xyt.ctypes.data_as(ctypes.c_void_p)))
    return pq.reshape(n, 2), xyt.reshape(n, 3)


# ---- solves ----------------------------------------------------------------
def kfbi_grid_solve(h, kappa, rhs, u_out):
    k = complex(kappa)
    if rhs is None or u_out is None:
        raise ValueError("rhs and u_out are required")
    _check(lib().kfbi_grid_solve(h, k.real, k.imag, _grid(h, rhs, "rhs"), _grid(h, u_out, "u_out")))


def kfbi_grid_solve_noalloc(h, kappa, rhs, u_out):
    """kfbi_grid_solve with its intermediates in the library's per-GPU
    scratch array (no device allocation in the call)."""
    k = complex(kappa)
    if rhs is None or u_out is None:
        raise ValueError("rhs and u_out are required")
    _check(lib().kfbi_grid_solve_noalloc(h, k.real, k.imag, _grid(h, rhs, "rhs"), _grid(h, u_out, "u_out")))


def kfbi_interface_apply(h, kappa, f_grid, f_gamma, phi, u_grid_out, uplus_out):
    k = complex(kappa)
    _check(lib().kfbi_interface_apply(h, k.real, k.imag, _grid(h, f_grid, "f_grid"), _gam(h, f_gamma, "f_gamma"),
                                      _gam(h, phi, "phi"), _grid(h, u_grid_out, "u_grid_out"),
                                      _gam(h, uplus_out, "uplus_out")))


def kfbi_helmholtz_solve(h, kappa, f_grid, f_gamma, g_gamma, u_grid_out, phi_inout=None, opts=None):
    k = complex(kappa)
    st = SolveStats()
    code = lib().kfbi_helmholtz_solve(h, k.real, k.imag, _grid(h, f_grid, "f_grid"), _gam(h, f_gamma, "f_gamma"),
                                      _gam(h, g_gamma, "g_gamma"), _grid(h, u_grid_out, "u_grid_out"),
                                      _gam(h, phi_inout, "phi_inout"), _opts(opts), ctypes.byref(st))
    _check(code, allow=(KFBI_ENOCONV,))
    return st.as_dict()


def kfbi_neumann_solve(h, kappa, f_grid, f_gamma, gn_gamma, u_grid_out, psi_inout=None, trace_out=None,
                       opts=None):
    """lap u - kappa u = f in Omega with du/dn = gn_gamma on Gamma; trace_out
    (optional) receives u's interior limit at the collocation points."""
    k = complex(kappa)
    st = SolveStats()
    code = lib().kfbi_neumann_solve(h, k.real, k.imag, _grid(h, f_grid, "f_grid"), _gam(h, f_gamma, "f_gamma"),
                                    _gam(h, gn_gamma, "gn_gamma"), _grid(h, u_grid_out, "u_grid_out"),
                                    _gam(h, psi_inout, "psi_inout"), _gam(h, trace_out, "trace_out"),
                                    _opts(opts), ctypes.byref(st))
    _check(code, allow=(KFBI_ENOCONV,))
    return st.as_dict()


# ---- steppers --------------------------------------------------------------
def kfbi_stepper_create(h, equation, tau, theta=0.25, diffusivity=1.0, w=0.0, v_grid=None, v_gamma=None,
                        bc=KFBI_BC_DIRICHLET, split=KFBI_SPLIT_STRANG):
    M, Nb, _ = _meta(h)
    p = StepParams(tau=tau, theta=theta, diffusivity=diffusivity, w=w,
                   v_grid=_ptr(v_grid, torch.float64, (M + 1) * (M + 1), "v_grid"),
                   v_gamma=_ptr(v_gamma, torch.float64, Nb, "v_gamma"), bc=bc, split=split)
    s = _P()
    _check(lib().kfbi_stepper_create(h, equation, ctypes.byref(p), ctypes.byref(s)))
    _STEPPERS[s.value] = _hv(h)
    return s


def kfbi_stepper_destroy(s):
    _check(lib().kfbi_stepper_destroy(s))
    _STEPPERS.pop(_hv(s), None)


def kfbi_stepper_state_bytes(s):
    n = ctypes.c_uint64(0)
    _check(lib().kfbi_stepper_state_bytes(s, ctypes.byref(n)))
    return int(n.value)


def kfbi_stepper_get_state(s, out=None):
    """Checkpoint: the stepper's state as a uint8 device tensor (opaque)."""
    n = kfbi_stepper_state_bytes(s)
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device="cuda")
    _check(lib().kfbi_stepper_get_state(s, _ptr(out, torch.uint8, None, "state"), out.numel()))
    return out


def kfbi_stepper_set_state(s, blob):
    """Restart from a blob written by kfbi_stepper_get_state."""
    _check(lib().kfbi_stepper_set_state(s, _ptr(blob, torch.uint8, None, "state"), blob.numel()))


def kfbi_stepper_init(s, u0, lap_u0, u0_gamma, lap_u0_gamma, uprev=None, lap_uprev=None,
                      uprev_gamma=None, lap_uprev_gamma=None):
    h = _stepper_dom(s)
    _check(lib().kfbi_stepper_init(s, _grid(h, u0, "u0"), _grid(h, lap_u0, "lap_u0"), _gam(h, u0_gamma, "u0_gamma"),
                                   _gam(h, lap_u0_gamma, "lap_u0_gamma"), _grid(h, uprev, "uprev"),
                                   _grid(h, lap_uprev, "lap_uprev"), _gam(h, uprev_gamma, "uprev_gamma"),
                                   _gam(h, lap_uprev_gamma, "lap_uprev_gamma")))


def kfbi_step_heat(s, g_next, src_grid, src_gamma, u_out, opts=None):
    st = SolveStats()
    h = _stepper_dom(s)
    _check(lib().kfbi_step_heat(s, _gam(h, g_next, "g_next"), _grid(h, src_grid, "src_grid"),
                                _gam(h, src_gamma, "src_gamma"), _grid(h, u_out, "u_out"),
                                _opts(opts), ctypes.byref(st)), allow=(KFBI_ENOCONV,))
    return st.as_dict()


def kfbi_step_wave(s, g_next, u_out, opts=None):
    st = SolveStats()
    h = _stepper_dom(s)
    _check(lib().kfbi_step_wave(s, _gam(h, g_next, "g_next"), _grid(h, u_out, "u_out"), _opts(opts),
                                ctypes.byref(st)), allow=(KFBI_ENOCONV,))
    return st.as_dict()


def kfbi_step_schrodinger(s, g_next, u_out, opts=None):
    st = SolveStats()
    h = _stepper_dom(s)
    _check(lib().kfbi_step_schrodinger(s, _gam(h, g_next, "g_next"), _grid(h, u_out, "u_out"), _opts(opts),
                                       ctypes.byref(st)), allow=(KFBI_ENOCONV,))
    return st.as_dict()
