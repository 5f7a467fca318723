"""CPU-only checks of the C ABI: the library loads, exports every entry point
include/llgc.h declares, the ctypes struct layouts match the C header
(checked by compiling a probe with gcc), and argument validation that
returns before any device call."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "llgc.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(llgc_[a-z_]+)\s*\(", txt)))


def _lib():
    from paper_2410_00966_amd import llgc
    return llgc, llgc.load()


def test_library_exports_every_declared_symbol():
    llgc, L = _lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(llgc.EXPORTED)


def test_struct_layout_matches_header():
    llgc, _ = _lib()
    fields = {
        "llgc_grid": ("Grid", ["nx", "ny", "nz", "dx", "dy", "dz"]),
        "llgc_params": ("Params", [f for f, _ in llgc.Params._fields_]),
        "llgc_run_info": ("RunInfo", [f for f, _ in llgc.RunInfo._fields_]),
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>',
             f'#include "{HEADER}"', "int main(void) {"]
    for cname, (_, fl) in fields.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f in fl:
            lines.append(f'printf("{cname}.{f} %zu\\n", '
                         f'offsetof({cname}, {f}));')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-o", exe, src], check=True)
        out = subprocess.run([exe], capture_output=True, text=True,
                             check=True).stdout
    got = dict(l.rsplit(" ", 1) for l in out.strip().splitlines())
    for cname, (pyname, fl) in fields.items():
        cls = getattr(llgc, pyname)
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f in fl:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, f


def test_create_rejects_bad_arguments_without_a_device():
    llgc, L = _lib()
    h = ctypes.c_void_p()
    assert L.llgc_create(None, None, ctypes.byref(h)) == -1
    g = llgc.Grid(0, 4, 1, 1e-9, 1e-9, 1e-9)
    assert L.llgc_create(ctypes.byref(g), None, ctypes.byref(h)) == -1
    g = llgc.Grid(4, 4, 1, -1e-9, 1e-9, 1e-9)
    assert L.llgc_create(ctypes.byref(g), None, ctypes.byref(h)) == -1
    g = llgc.Grid(4, 4, 5, 1e-9, 1e-9, 1e-9)
    assert L.llgc_create(ctypes.byref(g), None, ctypes.byref(h)) == -7
    g = llgc.Grid(4096, 4, 1, 1e-9, 1e-9, 1e-9)
    assert L.llgc_create(ctypes.byref(g), None, ctypes.byref(h)) == -7
    assert L.llgc_destroy(None) == 0
    assert L.llgc_last_error(None) == b"null context"
    assert L.llgc_cavity_enabled(None) == -1


def test_sim_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2410_00966_amd import inputs as I
    from paper_2410_00966_amd.llgc import Sim
    p, _, _ = I.c1_small()
    with pytest.raises(RuntimeError):
        Sim(p)


def test_batch_and_plan_entry_points_reject_bad_arguments():
    llgc, L = _lib()
    h = ctypes.c_void_p()
    g = llgc.Grid(16, 16, 1, 1e-9, 1e-9, 1e-9)
    # unknown plan flag; batch plan outside its size range
    assert L.llgc_create_ex(ctypes.byref(g), None, 2, ctypes.byref(h)) == -1
    big = llgc.Grid(200, 16, 1, 1e-9, 1e-9, 1e-9)
    assert L.llgc_create_ex(ctypes.byref(big), None, llgc.PLAN_BATCH,
                            ctypes.byref(h)) == -7
    one = llgc.Grid(1, 16, 1, 1e-9, 1e-9, 1e-9)
    assert L.llgc_create_ex(ctypes.byref(one), None, llgc.PLAN_BATCH,
                            ctypes.byref(h)) == -7
    assert L.llgc_batch_create(None, 1, None, ctypes.byref(h)) == -1
    grids = (llgc.Grid * 1)(g)
    assert L.llgc_batch_create(grids, 0, None, ctypes.byref(h)) == -1
    assert L.llgc_batch_destroy(None) == 0
    assert L.llgc_batch_last_error(None) == b"null batch"
    assert L.llgc_batch_instance(None, 0) is None
    assert L.llgc_batch_run(None, 0, 0.0, 0, None, 0, None, None, None) == -1


def test_autotune_rejects_null_context():
    llgc, L = _lib()
    k = ctypes.c_int32(-1)
    assert L.llgc_autotune(None, 5, ctypes.byref(k)) == -1
    assert k.value == -1
