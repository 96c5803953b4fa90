"""Python binding of libdpgmg (argument marshalling only).

Mirrors include/dpgmg.h call for call.  Every step of the solver runs in the
HIP library; this module only converts numpy arrays / torch tensors to
pointers.  It fails loudly when the library has not been built.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libdpgmg.so")

DPG_OK, DPG_EINVAL, DPG_ENOMEM, DPG_ENOTPD, DPG_ENOCONV, DPG_EBREAKDOWN, DPG_ESTATE, DPG_EDEVICE = \
    0, -1, -2, -3, -4, -5, -6, -7
DPG_FP64, DPG_MIXED = 0, 1
DPG_DEVICE_PTRS = 1
DPG_COLUMNWISE = 2
DPG_STORE_COARSE = 4
DPG_RECOMPUTE_PATCHES = 8
(X_ELEM_DOFS, X_MACRO_B, X_BLOCK_B, X_BLOCK_I, X_PATCHES, X_PROLONG, X_ELEM_S, X_ELEM_RHS,
 X_MACRO_M, X_COARSE_E, X_PATCH_INV, X_COARSEST, X_PROLONG_VAL, X_ASM_RHS) = range(1, 15)

_INT64_EXPORTS = {X_ELEM_DOFS, X_MACRO_B, X_BLOCK_B, X_BLOCK_I, X_PATCHES, X_PROLONG}
_DOUBLE_EXPORTS = {X_PROLONG_VAL}

SYMBOLS = ["dpg_default_options", "dpg_setup", "dpg_assemble", "dpg_build_hierarchy",
           "dpg_load_rhs", "dpg_solve", "dpg_get_fields", "dpg_info", "dpg_export",
           "dpg_profile", "dpg_kernel_stats", "dpg_last_error", "dpg_destroy",
           "dpg_release_setup", "dpg_solve_noalloc", "dpg_error_indicator",
           "dpg_boundary_points", "dpg_batch_open", "dpg_batch_add", "dpg_batch_step",
           "dpg_batch_take", "dpg_batch_close"]


class dpg_mesh(C.Structure):
    _fields_ = [("n", C.c_int32), ("origin", C.c_double * 3), ("side", C.c_double)]


class dpg_material(C.Structure):
    _fields_ = [("c", C.POINTER(C.c_double))]


class dpg_load(C.Structure):
    _fields_ = [("dir", C.c_double * 3), ("amp", C.c_double * 2), ("nsrc", C.c_int32),
                ("src", C.POINTER(C.c_double)), ("u0_qp", C.POINTER(C.c_double))]


class dpg_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("nu_pre", C.c_int32), ("nu_post", C.c_int32),
                ("nlevels", C.c_int32), ("maxit", C.c_int32), ("flags", C.c_int32),
                ("theta", C.c_double), ("hbm_budget", C.c_int64), ("stream", C.c_void_p),
                ("p_min", C.c_int32)]


class dpg_info_t(C.Structure):
    _fields_ = [("n_trace", C.c_int64), ("n_macro", C.c_int64), ("nlevels", C.c_int32),
                ("level_n", C.c_int32 * 16), ("level_ntrace", C.c_int64 * 16),
                ("level_nmacro", C.c_int64 * 16), ("resident_bytes", C.c_int64),
                ("n_test", C.c_int32), ("n_field", C.c_int32), ("n_tr", C.c_int32),
                ("setup_ms", C.c_double * 4), ("level_p", C.c_int32 * 16)]


class dpg_kstat(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("work", C.c_double)]


KERNEL_CLASSES = ["gram", "bmat", "load", "potrf", "trsm", "gemm", "macro_asm", "patch_gather",
                  "apply64", "apply32", "reduce", "condense", "expand", "transfer", "cg", "other",
                  "applyb64", "applyb32", "potrf_diag", "potrf_panel", "potrf_update",
                  "trsm_inv", "trsm_solve", "trsm_update"]
# kernel symbols behind each class (for matching a rocprofv3 trace)
KERNEL_SYMBOLS = {"gram": "k_gram", "bmat": "k_bmat", "load": "k_load", "potrf": "k_potrf",
                  "trsm": "k_trsm", "gemm": "k_gemm", "macro_asm": "k_macro_assemble",
                  "patch_gather": "k_patch_gather", "apply64": "k_units<double>",
                  "apply32": "k_strips<float>", "reduce": "k_reduce",
                  "applyb64": "k_rows_mfma64", "applyb32": "k_rows_mfma",
                  "potrf_diag": "k_potrf_diag", "potrf_panel": "k_potrf_panel",
                  "potrf_update": "k_potrf_update", "trsm_inv": "k_trsm_inv",
                  "trsm_solve": "k_trsm_solve", "trsm_update": "k_trsm_update"}


class DPGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdpgmg error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: run python -m paper_2304_01728_amd.build")
        L = C.CDLL(LIBPATH)
        vp = C.c_void_p
        L.dpg_default_options.argtypes = [C.POINTER(dpg_options)]
        L.dpg_default_options.restype = None
        L.dpg_setup.argtypes = [C.POINTER(dpg_mesh), C.c_int, C.c_int, C.c_double,
                                C.POINTER(dpg_material), C.POINTER(dpg_load), C.c_int,
                                C.POINTER(dpg_options), C.POINTER(vp)]
        L.dpg_setup.restype = C.c_int
        for name in ("dpg_assemble", "dpg_build_hierarchy", "dpg_release_setup"):
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = C.c_int
        L.dpg_load_rhs.argtypes = [vp, C.POINTER(dpg_load), C.c_int, vp]
        L.dpg_load_rhs.restype = C.c_int
        for name in ("dpg_solve", "dpg_solve_noalloc"):
            getattr(L, name).argtypes = [vp, vp, C.c_int, C.c_double, vp, vp, vp]
            getattr(L, name).restype = C.c_int
        L.dpg_get_fields.argtypes = [vp, vp, C.c_int, vp]
        L.dpg_get_fields.restype = C.c_int
        L.dpg_error_indicator.argtypes = [vp, vp, C.c_int, vp]
        L.dpg_error_indicator.restype = C.c_int
        L.dpg_info.argtypes = [vp, C.POINTER(dpg_info_t)]
        L.dpg_info.restype = C.c_int
        L.dpg_export.argtypes = [vp, C.c_int, C.c_int, vp, C.c_int64]
        L.dpg_export.restype = C.c_int64
        L.dpg_boundary_points.argtypes = [vp, vp, C.c_int64]
        L.dpg_boundary_points.restype = C.c_int64
        L.dpg_batch_open.argtypes = [vp, C.c_int]
        L.dpg_batch_add.argtypes = [vp, vp, C.c_int, C.c_double, vp]
        L.dpg_batch_step.argtypes = [vp, C.c_int, vp, vp]
        L.dpg_batch_take.argtypes = [vp, C.c_int, vp, vp, vp]
        L.dpg_batch_close.argtypes = [vp]
        for name in ("dpg_batch_open", "dpg_batch_add", "dpg_batch_step", "dpg_batch_take",
                     "dpg_batch_close"):
            getattr(L, name).restype = C.c_int
        L.dpg_profile.argtypes = [vp, C.c_int]
        L.dpg_profile.restype = C.c_int
        L.dpg_kernel_stats.argtypes = [vp, C.c_int, C.POINTER(dpg_kstat)]
        L.dpg_kernel_stats.restype = C.c_int
        L.dpg_last_error.argtypes = [vp]
        L.dpg_last_error.restype = C.c_char_p
        L.dpg_destroy.argtypes = [vp]
        L.dpg_destroy.restype = None
        _lib = L
    return _lib


def _check(ctx, code, allow=()):
    if code != DPG_OK and code not in allow:
        msg = lib().dpg_last_error(ctx).decode() if ctx else "setup failed"
        raise DPGError(code, msg)
    return code


def dpg_default_options(**kw):
    o = dpg_options()
    lib().dpg_default_options(C.byref(o))
    names = {f[0] for f in dpg_options._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"dpg_options has no field {k!r}")
        setattr(o, k, v)
    return o


def _loads(loads):
    """list of dicts {dir, amp, sources: [[x,y,z,sigma,re,im], ...], u0_qp: complex
    values at dpg_boundary_points} -> ctypes array."""
    arr = (dpg_load * max(1, len(loads)))()
    keep = []
    for i, ld in enumerate(loads):
        arr[i].dir[:] = list(np.asarray(ld.get("dir", (0.0, 0.0, 1.0)), dtype=float))
        amp = complex(ld.get("amp", 0.0))
        arr[i].amp[:] = [amp.real, amp.imag]
        src = np.ascontiguousarray(np.asarray(ld.get("sources", np.zeros((0, 6))), dtype=float))
        arr[i].nsrc = src.shape[0]
        if src.size:
            keep.append(src)
            arr[i].src = src.ctypes.data_as(C.POINTER(C.c_double))
        if ld.get("u0_qp") is not None:
            u0 = np.ascontiguousarray(np.asarray(ld["u0_qp"], dtype=np.complex128))
            keep.append(u0)
            arr[i].u0_qp = u0.ctypes.data_as(C.POINTER(C.c_double))
    return arr, keep


class Context:
    """Owner of a dpg_ctx handle (flags: the dpg_options.flags it was set up with)."""

    def __init__(self, handle, flags=0):
        self.h = handle
        self.flags = flags

    def close(self):
        if self.h:
            lib().dpg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dpg_setup(n, p, omega, loads, dp=1, side=1.0, origin=(0.0, 0.0, 0.0), c=None, options=None):
    mesh = dpg_mesh(n=n, side=side)
    mesh.origin[:] = list(origin)
    mat = None
    keepc = None
    if c is not None:
        keepc = np.ascontiguousarray(np.asarray(c, dtype=float))
        mat = dpg_material(c=keepc.ctypes.data_as(C.POINTER(C.c_double)))
    arr, keep = _loads(loads)
    opt = options if options is not None else dpg_default_options()
    h = C.c_void_p()
    code = lib().dpg_setup(C.byref(mesh), p, dp, omega, C.byref(mat) if mat else None, arr,
                           len(loads), C.byref(opt), C.byref(h))
    del keep, keepc
    if code != DPG_OK:
        raise DPGError(code, "dpg_setup failed")
    return Context(h.value, int(opt.flags))


def dpg_assemble(ctx):
    _check(ctx.h, lib().dpg_assemble(ctx.h))


def dpg_build_hierarchy(ctx):
    _check(ctx.h, lib().dpg_build_hierarchy(ctx.h))


def dpg_release_setup(ctx):
    _check(ctx.h, lib().dpg_release_setup(ctx.h))


def dpg_info(ctx):
    info = dpg_info_t()
    _check(ctx.h, lib().dpg_info(ctx.h, C.byref(info)))
    return info


def dpg_load_rhs(ctx, loads, want=True):
    arr, keep = _loads(loads)
    nT = dpg_info(ctx).n_trace
    out = np.zeros((len(loads), nT), dtype=np.complex128) if want else None
    _check(ctx.h, lib().dpg_load_rhs(ctx.h, arr, len(loads),
                                     out.ctypes.data if want else None))
    return out


def _device_arg(t, n, name):
    """Checks a torch tensor passed as a device pointer: complex128, contiguous,
    on a GPU, at least n entries.  Returns its address."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor with device=True")
    if t.dtype != torch.complex128 or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError(f"{name}: need a contiguous complex128 tensor on a GPU, got "
                         f"{t.dtype} on {t.device} (contiguous={t.is_contiguous()})")
    if t.numel() < n:
        raise ValueError(f"{name}: {t.numel()} entries, need nrhs x n_trace = {n}")
    return t.data_ptr()


def _solve(fn, ctx, rhs, nrhs, tol, x_out, device):
    nT = dpg_info(ctx).n_trace
    iters = np.zeros(nrhs, dtype=np.int32)
    rel = np.zeros(nrhs, dtype=np.float64)
    if device:
        if not ctx.flags & DPG_DEVICE_PTRS:
            raise ValueError("device=True needs a context set up with DPG_DEVICE_PTRS")
        rp = _device_arg(rhs, nrhs * nT, "rhs") if rhs is not None else None
        xp = _device_arg(x_out, nrhs * nT, "x_out") if x_out is not None else None
        x = x_out
    else:
        if ctx.flags & DPG_DEVICE_PTRS:
            raise ValueError("the context takes device pointers: pass device=True")
        if rhs is not None:
            rhs = np.ascontiguousarray(np.asarray(rhs, dtype=np.complex128).reshape(nrhs, nT))
        x = np.zeros((nrhs, nT), dtype=np.complex128) if x_out is None else x_out
        if x.dtype != np.complex128 or not x.flags.c_contiguous or x.size < nrhs * nT:
            raise ValueError("x_out: need a contiguous complex128 array of nrhs x n_trace")
        rp = rhs.ctypes.data if rhs is not None else None
        xp = x.ctypes.data
    code = fn(ctx.h, rp, nrhs, tol, xp, iters.ctypes.data, rel.ctypes.data)
    _check(ctx.h, code, allow=(DPG_ENOCONV,))
    return x, iters, rel, code


def dpg_solve(ctx, rhs=None, nrhs=1, tol=1e-8, x_out=None, device=False):
    """Solve; rhs: [nrhs, n_trace] complex128 (host) or None for the assembled
    loads.  With device=True, rhs / x_out are torch device tensors (complex128,
    contiguous) and the context must have been set up with DPG_DEVICE_PTRS.
    Returns (x, iters, relres, status)."""
    return _solve(lib().dpg_solve, ctx, rhs, nrhs, tol, x_out, device)


def dpg_solve_noalloc(ctx, rhs=None, nrhs=1, tol=1e-8, x_out=None, device=False):
    """dpg_solve column by column without any device allocation in the call
    (arguments and results as dpg_solve)."""
    return _solve(lib().dpg_solve_noalloc, ctx, rhs, nrhs, tol, x_out, device)


def dpg_get_fields(ctx, x):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    x = x.reshape(-1, x.shape[-1])
    info = dpg_info(ctx)
    nel = info.level_n[0] ** 3
    out = np.zeros((x.shape[0], nel, info.n_field), dtype=np.complex128)
    _check(ctx.h, lib().dpg_get_fields(ctx.h, x.ctypes.data, x.shape[0], out.ctypes.data))
    return out


def dpg_error_indicator(ctx, x):
    """eta_K^2 per element for trace solutions x [nrhs, n_trace] (host):
    returns [nrhs, n^3]."""
    if ctx.flags & DPG_DEVICE_PTRS:
        raise ValueError("the context takes device pointers; this wrapper passes host arrays")
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    x = x.reshape(-1, x.shape[-1])
    info = dpg_info(ctx)
    if x.shape[1] != info.n_trace:
        raise ValueError(f"x has {x.shape[1]} entries per column, need {info.n_trace}")
    nel = info.level_n[0] ** 3
    out = np.zeros((x.shape[0], nel), dtype=np.float64)
    _check(ctx.h, lib().dpg_error_indicator(ctx.h, x.ctypes.data, x.shape[0], out.ctypes.data))
    return out


def dpg_boundary_points(ctx):
    """[count, 3] coordinates of the boundary load points (the order u0_qp uses)."""
    n = lib().dpg_boundary_points(ctx.h, None, 0)
    if n < 0:
        _check(ctx.h, int(n))
    out = np.zeros((n, 3), dtype=np.float64)
    m = lib().dpg_boundary_points(ctx.h, out.ctypes.data, n)
    if m < 0:
        _check(ctx.h, int(m))
    return out


def dpg_batch_open(ctx, max_slots):
    _check(ctx.h, lib().dpg_batch_open(ctx.h, max_slots))
    ctx.batch_slots = max_slots


def dpg_batch_add(ctx, rhs=None, load_col=0, tol=1e-8):
    """Adds a right-hand side (host trace vector, or None for column load_col
    of the context's loads); returns its slot."""
    slot = C.c_int32()
    if rhs is not None:
        if ctx.flags & DPG_DEVICE_PTRS:
            rp = _device_arg(rhs, dpg_info(ctx).n_trace, "rhs")
        else:
            rhs = np.ascontiguousarray(np.asarray(rhs, dtype=np.complex128))
            if rhs.size != dpg_info(ctx).n_trace:
                raise ValueError("rhs must have n_trace entries")
            rp = rhs.ctypes.data
    else:
        rp = None
    _check(ctx.h, lib().dpg_batch_add(ctx.h, rp, load_col, tol, C.byref(slot)))
    return slot.value


def dpg_batch_step(ctx, max_iters):
    """Runs up to max_iters iterations; returns the finished slots not taken yet."""
    done = np.zeros(32, dtype=np.int32)
    nd = C.c_int32()
    _check(ctx.h, lib().dpg_batch_step(ctx.h, max_iters, done.ctypes.data, C.byref(nd)))
    return [int(v) for v in done[:nd.value]]


def dpg_batch_take(ctx, slot, x_out=None):
    """(x, iterations, relres, status) of a finished slot; frees it.  x is a
    host array unless the context takes device pointers (then x_out, a device
    tensor of n_trace complex128 entries, is required)."""
    it = C.c_int32()
    rr = C.c_double()
    if ctx.flags & DPG_DEVICE_PTRS:
        xp = _device_arg(x_out, dpg_info(ctx).n_trace, "x_out")
        x = x_out
    else:
        x = np.zeros(dpg_info(ctx).n_trace, dtype=np.complex128) if x_out is None else x_out
        xp = x.ctypes.data
    code = lib().dpg_batch_take(ctx.h, slot, xp, C.byref(it), C.byref(rr))
    _check(ctx.h, code, allow=(DPG_ENOCONV, DPG_EBREAKDOWN))
    return x, it.value, rr.value, code


def dpg_batch_close(ctx):
    _check(ctx.h, lib().dpg_batch_close(ctx.h))


def dpg_export(ctx, what, level=0):
    n = lib().dpg_export(ctx.h, what, level, None, 0)
    if n < 0:
        _check(ctx.h, int(n))
    if what in _INT64_EXPORTS:
        out = np.zeros(n, dtype=np.int64)
    elif what in _DOUBLE_EXPORTS:
        out = np.zeros(n, dtype=np.float64)
    else:
        out = np.zeros(n, dtype=np.complex128)
    m = lib().dpg_export(ctx.h, what, level, out.ctypes.data, n)
    if m < 0:
        _check(ctx.h, int(m))
    return out


def dpg_profile(ctx, enable=True):
    _check(ctx.h, lib().dpg_profile(ctx.h, 1 if enable else 0))


def dpg_kernel_stats(ctx):
    """{class name: (launches, total_ms, work)} for every class with launches."""
    out = {}
    for k, name in enumerate(KERNEL_CLASSES):
        st = dpg_kstat()
        _check(ctx.h, lib().dpg_kernel_stats(ctx.h, k, C.byref(st)))
        if st.launches:
            out[name] = (st.launches, st.total_ms, st.work)
    return out


def dpg_destroy(ctx):
    ctx.close()
