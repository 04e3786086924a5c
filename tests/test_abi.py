"""The C-ABI library loads and exports every symbol include/pico.h declares;
argument validation happens on the host before any device work (no GPU
needed for these checks)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pico.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pico_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2605_09590_amd import pico as p
    if not os.path.exists(p.LIB_PATH):
        pytest.fail("libpico.so is not built (run __graft_entry__.build())")
    return p.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n


def test_binding_names_match_header():
    from paper_2605_09590_amd import pico as p
    for n in declared():
        assert hasattr(p, n), n


def _desc(p, **kw):
    d = p.pico_op_desc_t()
    d.ny, d.nx, d.ncoils = 64, 64, 4
    d.maps = 0x1000          # never dereferenced: validation fails first
    d.mask = 0x2000
    d.sampling = p.PICO_CART_1D
    d.cg_iters = 10
    d.probe_tile = 4
    d.power_iters = 15
    d.power_margin = 1.01
    for k, v in kw.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("kw,status", [
    ({"ny": 63}, 1), ({"ny": 100}, 1), ({"ncoils": 0}, 1), ({"ncoils": 65}, 1),
    ({"cg_iters": 0}, 1), ({"probe_tile": 0}, 1), ({"lambda_": -1.0}, 1),
    ({"maps": None}, 1), ({"recon": 7}, 4), ({"sampling": 2}, 1), ({"sampling": 9}, 4),
    ({"sampling": 1, "nx": 100}, 1),
    ({"lambda_": 0.1, "power_iters": 0}, 1),
])
def test_init_rejects_bad_descriptors(lib, kw, status):
    from paper_2605_09590_amd import pico as p
    d = _desc(p, **kw)
    h = ctypes.c_void_p(1234)
    st = lib.pico_init(ctypes.byref(d), None, ctypes.byref(h))
    assert st == status
    assert h.value is None
    assert len(lib.pico_last_error()) > 0


def test_init_rejects_non_spd_psi(lib):
    import numpy as np
    from paper_2605_09590_amd import pico as p
    d = _desc(p, ncoils=2)
    psi = np.array([[1.0, 2.0], [2.0, 1.0]], np.complex128).view(np.float64)
    d.psi = psi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p()
    assert lib.pico_init(ctypes.byref(d), None, ctypes.byref(h)) == 1
    assert b"positive definite" in lib.pico_last_error()


def test_null_handles(lib):
    from paper_2605_09590_amd import pico as p
    acc = p.pico_accum_t()
    assert lib.pico_noise_map(None, 0, 0, 1, 0, ctypes.byref(acc), None, None) == 1
    assert lib.pico_apply_cov(None, None, None, 1, None) == 1
    assert lib.pico_finalize(None, ctypes.byref(acc), None, None) == 1
    assert lib.pico_pmr_baseline(None, 0, 0, 1, ctypes.byref(acc), None, None) == 1
    lib.pico_destroy(None)
    import math
    assert math.isnan(lib.pico_lambda_abs(None))


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors have the size and field offsets the C compiler gives
    the structs of include/pico.h (a mismatch would misread fields silently)."""
    import shutil
    import subprocess
    from paper_2605_09590_amd import pico as p
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"pico_op_desc_t": p.pico_op_desc_t, "pico_accum_t": p.pico_accum_t,
               "pico_stats_t": p.pico_stats_t, "pico_request_info_t": p.pico_request_info_t}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "pico.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            cf = "lambda" if fname == "lambda_" else fname
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    for line in filter(None, out):
        cname, what, val = line.split()
        py = structs[cname]
        if what == "size":
            assert ctypes.sizeof(py) == int(val), cname
        else:
            assert getattr(py, what).offset == int(val), (cname, what)


def test_set_allocator_arguments(lib):
    # host-only: installing and removing callbacks touches no device
    from paper_2605_09590_amd import pico as p
    calls = []
    cb_a = p.ALLOC_FN(lambda n, ctx: calls.append(n) or None)
    cb_f = p.FREE_FN(lambda ptr, ctx: None)
    assert lib.pico_set_allocator(cb_a, p.FREE_FN(), None) == p.PICO_EINVAL
    assert "both callbacks" in p.pico_last_error()
    assert lib.pico_set_allocator(p.ALLOC_FN(), cb_f, None) == p.PICO_EINVAL
    assert lib.pico_set_allocator(cb_a, cb_f, None) == p.PICO_OK
    assert lib.pico_set_allocator(p.ALLOC_FN(), p.FREE_FN(), None) == p.PICO_OK
    p.pico_set_allocator(lambda n: 0, lambda ptr: None)
    p.pico_set_allocator()
    assert calls == []
