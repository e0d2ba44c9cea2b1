"""GPU test of the allocation-free entry point sth_apply_h_noalloc through the C-ABI.

Its work space is one static device array per GPU.  The test calls it twice in
a row on the same context, the second time with fewer vectors, and compares
each result with the allocating entry point sth_apply_h (bit for bit: the same
kernels on the same per-column data) and with the oracle's H (1e-12 relative).
The 64-atom crystal (72^3 grid, 22,575 plane waves) needs about 1.9 MB of work
space per vector, so 70 vectors run as several chunks of the 64 MiB array.

The device buffers come from the HIP runtime the library itself links (bound
through ctypes), so that the test runs the entry point the way a caller in C
would, with one HIP runtime in the process.
"""
import ctypes as C
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

_H2D, _D2H = 1, 2   # hipMemcpyHostToDevice, hipMemcpyDeviceToHost


def _hip():
    import paper_2203_05623_amd as P
    P._lib.lib()   # the library (and with it its HIP runtime) is loaded
    hip = C.CDLL("libamdhip64.so.7", mode=os.RTLD_NOLOAD | os.RTLD_GLOBAL)
    hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip.hipFree.argtypes = [C.c_void_p]
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    hip.hipMemset.argtypes = [C.c_void_p, C.c_int, C.c_size_t]
    return hip


def _ok(code, what):
    assert code == 0, f"{what} returned HIP error {code}"


@pytest.mark.parametrize("name,sizes", [("cfg1", (37, 5)), ("cfg2", (70, 3))])
def test_apply_h_noalloc_matches_apply_h(name, sizes):
    import paper_2203_05623_amd as P
    hip = _hip()
    cfg = workloads.get_config(name)
    s = oracle.build_system(name)
    rng = np.random.default_rng(5)
    q, _ = np.linalg.qr(rng.standard_normal((s.npw, 4)) + 1j * rng.standard_normal((s.npw, 4)))
    psi = np.ascontiguousarray(q.T)
    ctx = P.sth_create(device=0, max_slots=64)
    bufs = []
    try:
        sid = P.sth_set_system(ctx, cfg.L, cfg.N, s.miller, s.vloc_r, s.beta, s.dij, psi,
                               np.arange(4.0))
        nbytes = max(sizes) * s.npw * 16
        for _ in range(2):
            p = C.c_void_p()
            _ok(hip.hipMalloc(C.byref(p), nbytes), "hipMalloc")
            bufs.append(p)
        din, dout = bufs
        for nvec in sizes:
            c = rng.standard_normal((nvec, s.npw)) + 1j * rng.standard_normal((nvec, s.npw))
            ref = P.sth_apply_h(ctx, sid, c)
            n = nvec * s.npw * 16
            _ok(hip.hipMemcpy(din, c.ctypes.data, n, _H2D), "hipMemcpy")
            _ok(hip.hipMemset(dout, 0xFF, n), "hipMemset")   # NaN pattern
            P._lib._check(P._lib.lib().sth_apply_h_noalloc(ctx, sid, nvec, din, dout, None))
            _ok(hip.hipDeviceSynchronize(), "hipDeviceSynchronize")
            got = np.empty_like(c)
            _ok(hip.hipMemcpy(got.ctypes.data, dout, n, _D2H), "hipMemcpy")
            assert np.array_equal(got, ref), f"{name} nvec={nvec}: differs from sth_apply_h"
            orc = oracle.apply_H(s, c)
            err = np.abs(got - orc).max() / np.abs(orc).max()
            print(f"{name} nvec={nvec}: equal to sth_apply_h, vs oracle {err:.2e}")
            assert err < 1e-12
        with pytest.raises(P.SthError) as e:
            P._lib._check(P._lib.lib().sth_apply_h_noalloc(ctx, sid, -1, None, None, None))
        assert e.value.code == P.STH_E_INVALID
    finally:
        for p in bufs:
            hip.hipFree(p)
        P.sth_destroy(ctx)
