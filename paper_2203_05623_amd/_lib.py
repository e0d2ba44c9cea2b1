"""ctypes binding of libsth.so (the C-ABI declared in include/sth.h).

Argument marshalling only: every step of the Sternheimer path runs in the HIP
library.  Arrays may be numpy arrays (host) or torch CUDA tensors (device
pointers, ordered against torch's current stream).  The library must have
been built (``paper_2203_05623_amd.build.build()``); importing this module
without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsth.so")

STH_OK, STH_E_INVALID, STH_E_NOMEM, STH_E_AGAIN, STH_E_NOT_READY = 0, -1, -2, -3, -4
STH_E_DEVICE, STH_E_NOT_FOUND, STH_E_INTERNAL = -5, -6, -7
STH_PTR_HOST, STH_PTR_DEVICE = 0, 1
STH_FP64, STH_MIXED, STH_MIXED_BF16 = 0, 1, 2
SOLVE_CONVERGED, SOLVE_MAXIT, SOLVE_BREAKDOWN, SOLVE_NAN = 0, 1, 2, 3

EXPORTS = ["sth_create", "sth_destroy", "sth_set_system", "sth_release_system", "sth_apply_h",
           "sth_apply_h_noalloc",
           "sth_valence", "sth_submit_solves", "sth_poll", "sth_wait", "sth_fetch_drho",
           "sth_fetch_dpsi", "sth_fetch_stats", "sth_chi0_block", "sth_release_ticket",
           "sth_profile", "sth_profile_read", "sth_system_info_get", "sth_pdep", "sth_lanczos",
           "sth_last_error"]
PHASES = ["zfft_inv", "plane", "zfft_fwd", "gemm_ah_b", "reduce", "gemm_a_c", "cg", "rhs_retire"]


class sth_config(C.Structure):
    _fields_ = [("device", C.c_int), ("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int),
                ("check_every", C.c_int), ("max_queued", C.c_int)]


class sth_system_desc(C.Structure):
    _fields_ = [("L", C.c_double), ("n", C.c_int), ("npw", C.c_int),
                ("miller", C.POINTER(C.c_int32)), ("vloc_r", C.c_void_p), ("nproj", C.c_int),
                ("beta", C.c_void_p), ("dij", C.c_void_p), ("nv", C.c_int), ("psi_v", C.c_void_p),
                ("eps_v", C.c_void_p), ("spin_factor", C.c_double), ("ptr_kind", C.c_int),
                ("gamma_only", C.c_int)]


class sth_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int), ("precision", C.c_int),
                ("want_dpsi", C.c_int)]


class sth_ticket_info(C.Structure):
    _fields_ = [("state", C.c_int), ("n_total", C.c_int), ("n_finished", C.c_int),
                ("n_converged", C.c_int), ("max_rel_resid", C.c_double),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("cg_iterations", C.c_longlong), ("op_applications", C.c_longlong),
                ("op_applications_fp32", C.c_longlong), ("graph_replays", C.c_longlong),
                ("system_id", C.c_int), ("npert", C.c_int), ("nband", C.c_int)]


class sth_system_info(C.Structure):
    _fields_ = [("npw", C.c_int), ("nsticks", C.c_int), ("nslots", C.c_int), ("nv", C.c_int),
                ("nproj", C.c_int), ("fft_plan_fp64", C.c_int), ("fft_plan_fp32", C.c_int),
                ("gemm_kchunk", C.c_int), ("tune_ms", C.c_double * 48),
                ("tuned_from_cache", C.c_int), ("plane_kernel_fp64", C.c_int),
                ("plane_kernel_fp32", C.c_int), ("zfft_kernel_fp64", C.c_int),
                ("zfft_kernel_fp32", C.c_int), ("n", C.c_int), ("budget_used", C.c_size_t),
                ("budget_limit", C.c_size_t)]


class SthError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2203_05623_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    vp, i32, dbl, u64 = C.c_void_p, C.c_int32, C.c_double, C.c_uint64
    sig = {
        "sth_create": [C.POINTER(sth_config), C.POINTER(vp)],
        "sth_destroy": [vp],
        "sth_set_system": [vp, C.POINTER(sth_system_desc), vp, C.POINTER(i32)],
        "sth_release_system": [vp, i32],
        "sth_apply_h": [vp, i32, C.c_int, vp, vp, C.c_int, vp],
        "sth_valence": [vp, C.POINTER(sth_system_desc), C.c_int, dbl, C.c_int, vp, vp, C.c_int,
                        C.POINTER(dbl), C.POINTER(C.c_int)],
        "sth_submit_solves": [vp, i32, C.c_int, vp, C.c_int, C.POINTER(i32),
                              C.POINTER(sth_solve_opts), C.c_int, vp, C.POINTER(u64)],
        "sth_poll": [vp, u64, C.POINTER(sth_ticket_info)],
        "sth_wait": [vp, u64, dbl],
        "sth_fetch_drho": [vp, u64, vp, C.c_int, vp],
        "sth_fetch_dpsi": [vp, u64, vp, C.c_int, vp],
        "sth_fetch_stats": [vp, u64, vp, vp, vp, vp],
        "sth_chi0_block": [vp, u64, vp, vp, vp],
        "sth_release_ticket": [vp, u64],
        "sth_profile": [vp, C.c_int],
        "sth_profile_read": [vp, vp, vp, vp, vp],
        "sth_system_info_get": [vp, i32, C.POINTER(sth_system_info)],
        "sth_apply_h_noalloc": [vp, i32, C.c_int, vp, vp, vp],
        "sth_pdep": [vp, i32, C.c_int, C.c_int, dbl, C.c_int, dbl, C.c_int, vp, vp, C.c_int, vp,
                     C.POINTER(C.c_int), C.POINTER(dbl)],
        "sth_lanczos": [vp, i32, C.c_int, C.c_int, vp, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.sth_last_error.argtypes = []
    lib.sth_last_error.restype = C.c_char_p
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def _check(code):
    if code != STH_OK:
        raise SthError(code, lib().sth_last_error().decode())


# ------------------------------------------------------------------ marshalling helpers
def _is_torch(a):
    return type(a).__module__.startswith("torch")


_TORCH_DTYPES = {np.dtype(np.float64): "float64", np.dtype(np.complex128): "complex128",
                 np.dtype(np.int32): "int32"}


def _ptr(a, dtype, count=None, name="array", out=False):
    """(pointer, ptr_kind, keepalive) of a numpy array or a torch tensor.

    The library takes no lengths, so every array is checked here: a torch
    tensor (host or device) must have exactly `dtype`, be contiguous and hold
    `count` elements (complex128 counted as complex numbers); a numpy input is
    converted to a contiguous `dtype` copy, a numpy output must already be one
    (a copy would lose the result).  ValueError otherwise."""
    if a is None:
        return None, STH_PTR_HOST, None
    dt = np.dtype(dtype)
    if _is_torch(a):
        want = _TORCH_DTYPES[dt]
        got = str(a.dtype).replace("torch.", "")
        # complex data may arrive as a float64 view of (re, im) pairs
        if got == "float64" and want == "complex128":
            n = a.numel() // 2
        elif got != want:
            raise ValueError(f"{name}: tensor dtype {got}, expected {want}")
        else:
            n = a.numel()
        if not a.is_contiguous():
            raise ValueError(f"{name}: tensor must be contiguous")
        if count is not None and n != count:
            raise ValueError(f"{name}: {n} elements, expected {count}")
        if a.is_cuda:
            return a.data_ptr(), STH_PTR_DEVICE, a
        a = a.numpy()
        if got == "float64" and want == "complex128":
            a = a.view(np.complex128)
    if out:
        if not (isinstance(a, np.ndarray) and a.dtype == dt and a.flags.c_contiguous
                and a.flags.writeable):
            raise ValueError(f"{name}: output must be a writeable C-contiguous {dt} array")
        arr = a
    else:
        arr = np.ascontiguousarray(a, dtype=dt)
    if count is not None and arr.size != count:
        raise ValueError(f"{name}: {arr.size} elements, expected {count}")
    return arr.ctypes.data, STH_PTR_HOST, arr


def _stream(a=None):
    if a is not None and _is_torch(a) and a.is_cuda:
        import torch
        return torch.cuda.current_stream(a.device).cuda_stream
    return None


# ------------------------------------------------------------------ C-ABI functions
def sth_create(device=0, hbm_budget_bytes=0, max_slots=0, check_every=0, max_queued=0):
    cfg = sth_config(device, hbm_budget_bytes, max_slots, check_every, max_queued)
    h = C.c_void_p()
    _check(lib().sth_create(C.byref(cfg), C.byref(h)))
    return h


def sth_destroy(ctx):
    _check(lib().sth_destroy(ctx))


def _desc(L, n, miller, vloc_r, beta, dij, psi_v, eps_v, spin_factor):
    miller = np.ascontiguousarray(miller, dtype=np.int32).reshape(-1, 3)
    npw = len(miller)
    n = int(n)
    keep = [miller]
    kinds = set()

    def p(a, dt, count, name):
        ptr, kind, k = _ptr(a, dt, count, name)
        keep.append(k)
        if a is not None:
            kinds.add(kind)
        return ptr

    nproj = 0 if beta is None else int(beta.shape[0])
    nv = 0 if psi_v is None else int(psi_v.shape[0])
    d = sth_system_desc(
        L=float(L), n=n, npw=npw, miller=miller.ctypes.data_as(C.POINTER(C.c_int32)),
        vloc_r=p(vloc_r, np.float64, n ** 3, "vloc_r"), nproj=nproj,
        beta=p(beta, np.complex128, nproj * npw, "beta"),
        dij=p(dij, np.float64, nproj, "dij"), nv=nv,
        psi_v=p(psi_v, np.complex128, nv * npw, "psi_v"),
        eps_v=p(eps_v, np.float64, nv, "eps_v"), spin_factor=float(spin_factor),
        ptr_kind=STH_PTR_HOST)
    if nproj and dij is None:
        raise ValueError("dij is required with beta")
    if nv and eps_v is None:
        raise ValueError("eps_v is required with psi_v")
    if len(kinds) > 1:
        raise ValueError("system arrays must all be host arrays or all device tensors")
    d.ptr_kind = kinds.pop() if kinds else STH_PTR_HOST
    return d, keep


def sth_set_system(ctx, L, n, miller, vloc_r, beta, dij, psi_v, eps_v, spin_factor=2.0,
                   gamma_only=False):
    d, keep = _desc(L, n, miller, vloc_r, beta, dij, psi_v, eps_v, spin_factor)
    d.gamma_only = 1 if gamma_only else 0
    sid = C.c_int32()
    _check(lib().sth_set_system(ctx, C.byref(d), _stream(vloc_r), C.byref(sid)))
    del keep
    return sid.value


def sth_release_system(ctx, system_id):
    _check(lib().sth_release_system(ctx, system_id))


def sth_apply_h(ctx, system_id, c, out=None):
    """H c for c complex [nvec, npw] (numpy or torch); returns out."""
    npw = sth_system_info_get(ctx, system_id)["npw"]
    nvec = int(c.shape[0])
    if out is None:
        out = np.empty((nvec, npw), np.complex128) if not _is_torch(c) else c.clone()
    pin, kin, k1 = _ptr(c, np.complex128, nvec * npw, "c")
    pout, kout, k2 = _ptr(out, np.complex128, nvec * npw, "out", out=True)
    if kin != kout:
        raise ValueError("in and out must live on the same side")
    _check(lib().sth_apply_h(ctx, system_id, nvec, pin, pout, kin, _stream(c)))
    return out


def sth_apply_h_noalloc(ctx, system_id, c, out):
    """H c without allocation: c and out are torch CUDA tensors (complex128
    [nvec, npw], caller's order); enqueued on torch's current stream."""
    if not (_is_torch(c) and _is_torch(out)):
        raise ValueError("sth_apply_h_noalloc takes device (torch CUDA) tensors only")
    npw = sth_system_info_get(ctx, system_id)["npw"]
    nvec = int(c.shape[0])
    pin, _, k1 = _ptr(c, np.complex128, nvec * npw, "c")
    pout, _, k2 = _ptr(out, np.complex128, nvec * npw, "out", out=True)
    _check(lib().sth_apply_h_noalloc(ctx, system_id, nvec, pin, pout, _stream(c)))
    return out


def sth_valence(ctx, L, n, miller, vloc_r, beta, dij, nbands, tol=1e-10, maxit=0,
                spin_factor=2.0):
    d, keep = _desc(L, n, miller, vloc_r, beta, dij, None, None, spin_factor)
    npw = d.npw
    eps = np.empty(nbands)
    psi = np.empty((nbands, npw), np.complex128)
    res = C.c_double()
    its = C.c_int()
    _check(lib().sth_valence(ctx, C.byref(d), nbands, tol, maxit, eps.ctypes.data,
                             psi.ctypes.data, STH_PTR_HOST, C.byref(res), C.byref(its)))
    del keep
    return eps, psi, res.value, its.value


def sth_submit_solves(ctx, system_id, dv_r, bands, tol=1e-10, maxit=0, precision=STH_FP64,
                      want_dpsi=False):
    n = sth_system_info_get(ctx, system_id)["n"]
    npert = int(dv_r.shape[0])
    bands = np.ascontiguousarray(bands, dtype=np.int32).reshape(-1)
    pdv, kind, keep = _ptr(dv_r, np.float64, npert * n ** 3, "dv_r")
    opts = sth_solve_opts(float(tol), int(maxit), int(precision), int(bool(want_dpsi)))
    t = C.c_uint64()
    _check(lib().sth_submit_solves(ctx, system_id, npert, pdv, len(bands),
                                   bands.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(opts),
                                   kind, _stream(dv_r), C.byref(t)))
    del keep
    return t.value


def sth_poll(ctx, ticket):
    info = sth_ticket_info()
    _check(lib().sth_poll(ctx, ticket, C.byref(info)))
    return {k: getattr(info, k) for k, _ in sth_ticket_info._fields_}


def sth_wait(ctx, ticket, timeout_s=1e9):
    code = lib().sth_wait(ctx, ticket, float(timeout_s))
    if code == STH_E_NOT_READY:
        return False
    _check(code)
    return True


def _ticket_shape(ctx, ticket):
    info = sth_poll(ctx, ticket)
    sysinfo = sth_system_info_get(ctx, info["system_id"])
    return info["npert"], info["nband"], sysinfo["n"], sysinfo["npw"]


def sth_fetch_drho(ctx, ticket, out):
    npert, _, n, _ = _ticket_shape(ctx, ticket)
    p, kind, keep = _ptr(out, np.float64, npert * n ** 3, "drho", out=True)
    _check(lib().sth_fetch_drho(ctx, ticket, p, kind, _stream(out)))
    return out


def sth_fetch_dpsi(ctx, ticket, out):
    npert, nband, _, npw = _ticket_shape(ctx, ticket)
    p, kind, keep = _ptr(out, np.complex128, npert * nband * npw, "dpsi", out=True)
    _check(lib().sth_fetch_dpsi(ctx, ticket, p, kind, _stream(out)))
    return out


def sth_fetch_stats(ctx, ticket, n=None):
    """Per-solve (iterations, true relative residual, status, latency), each [npert * nband]."""
    npert, nband, _, _ = _ticket_shape(ctx, ticket)
    if n is not None and n != npert * nband:
        raise ValueError(f"ticket holds {npert * nband} solves, not {n}")
    n = npert * nband
    iters = np.empty(n, np.int32)
    resid = np.empty(n)
    status = np.empty(n, np.int32)
    lat = np.empty(n)
    _check(lib().sth_fetch_stats(ctx, ticket, iters.ctypes.data, resid.ctypes.data,
                                 status.ctypes.data, lat.ctypes.data))
    return iters, resid, status, lat


def sth_chi0_block(ctx, ticket, npert=None):
    np_, _, _, _ = _ticket_shape(ctx, ticket)
    if npert is not None and npert != np_:
        raise ValueError(f"ticket holds {np_} perturbations, not {npert}")
    npert = np_
    M = np.empty((npert, npert))
    S = np.empty((npert, npert))
    lam = np.empty(npert)
    _check(lib().sth_chi0_block(ctx, ticket, M.ctypes.data, S.ctypes.data, lam.ctypes.data))
    return M, S, lam


def sth_release_ticket(ctx, ticket):
    _check(lib().sth_release_ticket(ctx, ticket))


def sth_lanczos(ctx, system_id, band, phi, nsteps):
    """Lanczos chains of orbital `band` for the real grids phi [nphi, n, n, n]:
    (alpha, beta, d [nphi, nsteps], U [nphi, nsteps, nsteps], braket [nphi, nphi, nsteps])."""
    nphi = int(phi.shape[0])
    n = sth_system_info_get(ctx, system_id)["n"]
    p, kind, keep = _ptr(phi, np.float64, nphi * n ** 3, "phi")
    alpha = np.empty((nphi, nsteps))
    beta = np.empty((nphi, nsteps))
    d = np.empty((nphi, nsteps))
    U = np.empty((nphi, nsteps, nsteps))
    br = np.empty((nphi, nphi, nsteps), np.complex128)
    _check(lib().sth_lanczos(ctx, system_id, band, nphi, p, kind, nsteps, alpha.ctypes.data,
                             beta.ctypes.data, d.ctypes.data, U.ctypes.data, br.ctypes.data,
                             _stream(phi)))
    del keep
    return alpha, beta, d, U, br


def sth_pdep(ctx, system_id, n, npdep, nmax=0, tol=1e-6, maxit=100, solve_tol=1e-10,
             precision=STH_FP64, want_vectors=True):
    """(eigenvalues [npdep], eigenvectors [npdep, n, n, n] or None, iterations, max residual);
    n is the system's grid size (shape of the vectors); nmax 0 means 4 npdep."""
    if n != sth_system_info_get(ctx, system_id)["n"]:
        raise ValueError("n must be the system's grid size")
    eig = np.empty(npdep)
    vec = np.empty((npdep, n, n, n)) if want_vectors else None
    its = C.c_int()
    res = C.c_double()
    _check(lib().sth_pdep(ctx, system_id, npdep, nmax or 4 * npdep, tol, maxit, solve_tol,
                          precision, eig.ctypes.data, vec.ctypes.data if want_vectors else None,
                          STH_PTR_HOST, None, C.byref(its), C.byref(res)))
    return eig, vec, its.value, res.value


def sth_profile(ctx, enable=True):
    _check(lib().sth_profile(ctx, int(bool(enable))))


def sth_profile_read(ctx):
    """{phase: (ms, launches, algorithmic bytes, flops)}; resets the counters."""
    ms = np.zeros(8)
    n = np.zeros(8, np.int64)
    b = np.zeros(8)
    f = np.zeros(8)
    _check(lib().sth_profile_read(ctx, ms.ctypes.data, n.ctypes.data, b.ctypes.data,
                                  f.ctypes.data))
    return {PHASES[i]: (float(ms[i]), int(n[i]), float(b[i]), float(f[i])) for i in range(8)}


def sth_system_info_get(ctx, system_id):
    info = sth_system_info()
    _check(lib().sth_system_info_get(ctx, system_id, C.byref(info)))
    out = {k: getattr(info, k) for k, _ in sth_system_info._fields_}
    out["tune_ms"] = list(info.tune_ms)
    return out


def sth_last_error():
    return lib().sth_last_error().decode()
