"""Host-side checks of the HIP library that need no GPU: it is built, loads, and
exports every entry point declared in include/sth.h; the ctypes structures have
the C layout; calls without a device fail with an error code, not a crash."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))
HEADER = os.path.join(ROOT, "include", "sth.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:sth_status|const char\*)\s+(sth_\w+)\s*\(", text,
                                 re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2203_05623_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsth.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2203_05623_amd import _lib
    assert set(_declared()) == set(_lib.EXPORTS)


def test_struct_layouts_match_header(tmp_path):
    """Every field offset and struct size of the ctypes mirrors equals what a C
    compiler makes of include/sth.h (offsetof / sizeof printed by a small program
    built with gcc against the header)."""
    import shutil
    import subprocess
    from paper_2203_05623_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = [_lib.sth_config, _lib.sth_system_desc, _lib.sth_solve_opts,
               _lib.sth_ticket_info, _lib.sth_system_info]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "sth.h"',
             "int main(void) {"]
    want = []
    for st in structs:
        name = st.__name__
        lines.append(f'  printf("%zu\\n", sizeof({name}));')
        want.append(C.sizeof(st))
        for fname, _ in st._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({name}, {fname}));')
            want.append(getattr(st, fname).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert got == want
    assert C.sizeof(_lib.sth_config) == 32
    assert _lib.sth_system_desc.ptr_kind.offset == 88


def test_no_device_is_an_error_code(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2203_05623_amd import _lib
    with pytest.raises(_lib.SthError) as e:
        _lib.sth_create(device=0)
    assert e.value.code == _lib.STH_E_DEVICE
    assert lib.sth_last_error()


def test_binding_rejects_wrong_dtype_size_and_layout():
    """The C-ABI takes no lengths, so the binding checks every array before a pointer
    crosses it: exact element counts, the library's dtypes for tensors (whose
    pointers are passed as they are), and writeable contiguous outputs."""
    import numpy as np
    import torch
    from paper_2203_05623_amd import _lib
    ok = _lib._ptr(np.zeros(4, np.float32), np.float64, 4, "x")   # host input: converted copy
    assert ok[1] == _lib.STH_PTR_HOST and ok[2].dtype == np.float64
    with pytest.raises(ValueError, match="elements"):
        _lib._ptr(np.zeros(3), np.float64, 4, "x")
    with pytest.raises(ValueError, match="elements"):
        _lib._ptr(np.zeros(5, np.complex128), np.complex128, 4, "x")
    with pytest.raises(ValueError, match="output"):
        _lib._ptr(np.zeros((4, 4))[:, :2], np.float64, 8, "out", out=True)
    with pytest.raises(ValueError, match="output"):
        _lib._ptr(np.zeros(8, np.float32), np.float64, 8, "out", out=True)
    ro = np.zeros(8)
    ro.flags.writeable = False
    with pytest.raises(ValueError, match="output"):
        _lib._ptr(ro, np.float64, 8, "out", out=True)
    with pytest.raises(ValueError, match="dtype"):
        _lib._ptr(torch.zeros(4, dtype=torch.float32), np.float64, 4, "t")
    with pytest.raises(ValueError, match="dtype"):
        _lib._ptr(torch.zeros(4, dtype=torch.complex64), np.complex128, 4, "t")
    with pytest.raises(ValueError, match="contiguous"):
        _lib._ptr(torch.zeros(4, 4, dtype=torch.float64)[:, :2], np.float64, 8, "t")
    # a complex128 tensor and its float64 (re, im) view count the same complex numbers
    z = torch.zeros(3, dtype=torch.complex128)
    assert _lib._ptr(z, np.complex128, 3, "z")[1] == _lib.STH_PTR_HOST
    assert _lib._ptr(torch.view_as_real(z), np.complex128, 3, "z")[1] == _lib.STH_PTR_HOST
    with pytest.raises(ValueError, match="elements"):
        _lib._ptr(z, np.complex128, 4, "z")


def test_system_description_checks_shapes():
    """sth_set_system / sth_valence arguments are sized from n and the sphere."""
    import numpy as np
    from paper_2203_05623_amd import _lib
    miller = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0]], np.int32)
    n = 24
    v = np.zeros(n ** 3)
    beta = np.zeros((2, 3), np.complex128)
    psi = np.zeros((1, 3), np.complex128)
    d, _ = _lib._desc(10.0, n, miller, v, beta, np.zeros(2), psi, np.zeros(1), 2.0)
    assert (d.npw, d.nproj, d.nv) == (3, 2, 1)
    with pytest.raises(ValueError, match="vloc_r"):
        _lib._desc(10.0, n, miller, np.zeros(n ** 3 - 1), beta, np.zeros(2), psi, np.zeros(1), 2.0)
    with pytest.raises(ValueError, match="beta"):
        _lib._desc(10.0, n, miller, v, np.zeros((2, 4), np.complex128), np.zeros(2), psi,
                   np.zeros(1), 2.0)
    with pytest.raises(ValueError, match="dij"):
        _lib._desc(10.0, n, miller, v, beta, np.zeros(3), psi, np.zeros(1), 2.0)
    with pytest.raises(ValueError, match="psi_v"):
        _lib._desc(10.0, n, miller, v, beta, np.zeros(2), np.zeros((1, 2), np.complex128),
                   np.zeros(1), 2.0)
    with pytest.raises(ValueError, match="eps_v"):
        _lib._desc(10.0, n, miller, v, beta, np.zeros(2), psi, np.zeros(2), 2.0)
