"""CPU checks of the C ABI library: it builds, loads, and exports every
function include/inc.h declares; without a GPU it reports INC_ERR_NO_DEVICE
instead of falling back to anything."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "inc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(inc_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1309_7963_amd import build

    build.build(force=False)
    return C.CDLL(build.LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ("inc_simulate", "inc_simulate_dev", "inc_ctx_create", "inc_ctx_destroy", "inc_strerror"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_knows_every_symbol():
    from paper_1309_7963_amd import _lib

    assert sorted(_lib.SYMBOLS) == declared_functions()


def test_error_strings(lib):
    lib.inc_strerror.restype = C.c_char_p
    for code in range(0, -9, -1):
        assert lib.inc_strerror(code) != b"unknown error"
    lib.inc_contract_version.restype = C.c_int
    assert lib.inc_contract_version() >= 1


def _has_gpu():
    try:
        import torch

        return torch.cuda.device_count() > 0
    except Exception:
        return False


@pytest.mark.skipif(_has_gpu(), reason="a GPU is present")
def test_no_device_is_an_error_not_a_fallback():
    import paper_1309_7963_amd as inc

    with pytest.raises(inc.IncError) as e:
        inc.Context([(16, 8)])
    assert e.value.code == inc.INC_ERR_NO_DEVICE


def test_argument_errors_before_device(lib):
    import paper_1309_7963_amd as inc
    from paper_1309_7963_amd import _lib

    L = _lib.load()
    h = C.c_void_p()
    arr = (_lib.Nucleus * 1)(_lib.Nucleus(16, 16))
    assert L.inc_ctx_create(arr, 1, None, C.byref(h)) == inc.INC_ERR_ARG
    arr = (_lib.Nucleus * 1)(_lib.Nucleus(16, 8))
    assert L.inc_ctx_create(arr, 0, None, C.byref(h)) == inc.INC_ERR_ARG
    assert L.inc_simulate_dev(None, None, None, None, 0) == inc.INC_ERR_ARG
    assert L.inc_evaporate_dev(None, None, None, None) == inc.INC_ERR_ARG
    x = _lib.Excited()
    x.n = 1
    assert L.inc_evaporate_dev(None, C.byref(x), None, None) == inc.INC_ERR_ARG
    nn, lo, hi = C.c_int(), C.c_float(), C.c_float()
    assert L.inc_ctx_xs_table(None, None, C.byref(nn), C.byref(lo), C.byref(hi)) == inc.INC_ERR_ARG
    nsec_r = C.c_ulonglong()
    noop = _lib.RING_CONSUMER(lambda chunk, user: None)
    assert L.inc_ring_simulate_to(None, None, None, None, noop, None, C.byref(nsec_r), None, 0, None) == inc.INC_ERR_ARG
    rh = C.c_void_p(1)
    assert L.inc_ring_create_device(None, 1 << 14, 1 << 12, C.byref(rh)) == inc.INC_ERR_ARG and not rh.value
    # option ranges are checked before the device is looked for
    for field, bad in (("fast_math", 2), ("same_stream", -1), ("stack_levels", 5), ("block_size", 96),
                       ("waves_per_cu", 33), ("kin_threshold", 65), ("start_threshold", 65), ("input_order", 2),
                       ("heavy_fragments", 2), ("photon_evaporation", 2)):
        o = _lib.Options()
        setattr(o, field, bad)
        assert L.inc_ctx_create(arr, 1, C.byref(o), C.byref(h)) == inc.INC_ERR_ARG, field
    nsec = C.c_size_t()
    e = (C.c_float * 1)(10.0)
    rc = L.inc_simulate(16, 8, e, 1, 1, None, None, None, None, None, None, None, None, 0, C.byref(nsec))
    assert rc == inc.INC_ERR_ARG


# struct name in include/inc.h -> ctypes mirror in the binding
STRUCTS = {
    "inc_nucleus": "Nucleus", "inc_options": "Options", "inc_output": "Output", "inc_batch": "Batch",
    "inc_excited": "Excited", "inc_request": "Request", "inc_host_output": "HostOutput",
    "inc_server_stats": "ServerStats", "inc_ring_stats": "RingStats", "inc_ring_chunk": "RingChunk",
}


def test_struct_layouts_match_header(tmp_path):
    # sizes and field offsets of every struct of the header, as the C
    # compiler lays them out, against the binding's ctypes mirrors (and the
    # residual record against its numpy dtype)
    import ctypes as C

    from paper_1309_7963_amd import _lib

    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "inc.h"', "int main(void) {"]
    for cname, pname in STRUCTS.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in getattr(_lib, pname)._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append('printf("inc_residual size %zu\\n", sizeof(inc_residual));')
    for f in _lib.RESIDUAL_DTYPE.names:
        lines.append('printf("inc_residual %s %%zu\\n", offsetof(inc_residual, %s));' % (f, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess

    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for ln in subprocess.check_output([str(exe)], text=True).splitlines():
        a, b, c = ln.split()
        got[(a, b)] = int(c)
    for cname, pname in STRUCTS.items():
        S = getattr(_lib, pname)
        assert got[(cname, "size")] == C.sizeof(S), cname
        for f, _ in S._fields_:
            assert got[(cname, f)] == getattr(S, f).offset, (cname, f)
    assert got[("inc_residual", "size")] == _lib.RESIDUAL_DTYPE.itemsize
    for f in _lib.RESIDUAL_DTYPE.names:
        assert got[("inc_residual", f)] == _lib.RESIDUAL_DTYPE.fields[f][1], f
