"""The C ABI library loads, exports every function include/snn.h declares, and the
Python binding's structures match the header's layout (checked by compiling the header
with gcc).  No compute call: runs without a GPU."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_1912_07423_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "snn.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(snn_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = L.load()
    declared = _declared_functions()
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(L.SIGNATURES) == declared


def test_exported_symbols_match_header():
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines() if " T snn_" in ln})
    assert exported == _declared_functions()


STRUCTS = {"snn_population": L.Population, "snn_projection": L.Projection,
           "snn_params": L.Params, "snn_allocator": L.Allocator, "snn_info": L.Info,
           "snn_state": L.State, "snn_profile": L.Profile, "snn_batch_member": L.BatchMember,
           "snn_batch_tuning": L.BatchTuning, "snn_bptt_desc": L.BpttDesc,
           "snn_delivery_tuning": L.DeliveryTuning}


def test_struct_layouts_match_header():
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){"]
    for cname, py in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            cf = "from" if fname == "from_" else fname
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {cf}));')
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-std=c11", "-o", exe, src], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = dict(ln.rsplit(" ", 1) for ln in out.strip().splitlines())
    for cname, py in STRUCTS.items():
        assert int(got[f"{cname} size"]) == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, (cname, fname)


def test_last_error_is_a_string():
    assert isinstance(L.load().snn_last_error(None), bytes)


def test_null_arguments_rejected_without_gpu():
    lib = L.load()
    h = C.c_void_p()
    assert lib.snn_build_network(None, None, 0, None, 0, None, None, C.byref(h)) == L.SNN_E_INVALID
    assert b"null" in lib.snn_last_error(None)
    assert b"null" in lib.snn_last_error(h)  # the message is per thread, not per network
    assert lib.snn_run(None, 1) == L.SNN_E_INVALID
    assert lib.snn_get_info(None, None) == L.SNN_E_INVALID
    lib.snn_destroy(None)
    assert lib.snn_build_batch(None, 3, 16, None, None, C.byref(h)) == L.SNN_E_INVALID
    assert lib.snn_batch_run(None, 1) == L.SNN_E_INVALID
    assert lib.snn_batch_network(None, 0, C.byref(h)) == L.SNN_E_INVALID
    lib.snn_batch_destroy(None)
    assert lib.snn_bptt_create(None, None, None, None, None, None, None, C.byref(h)) == L.SNN_E_INVALID
    assert lib.snn_bptt_forward(None, None, None, None, None, None, None, None) == L.SNN_E_INVALID
    lib.snn_bptt_destroy(None)
