"""The C-ABI library: loads, exports every declared symbol, rejects bad
arguments on the host (no GPU needed for any of these)."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2305_03317_amd import sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sp_[a-z_]+)\s*\(", text)))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("sp_graph_upload", "sp_bc", "sp_bc_batch", "sp_stream_submit"):
        assert core in names


def test_library_exports_every_declared_symbol():
    L = sp.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    bound = {name for name, _, _ in sp.SIGNATURES}
    assert set(declared_functions()) == bound


def test_library_was_built_from_this_header():
    """A library built from another version of sp.h would exchange structs of
    another size with the binding (and overwrite host memory)."""
    from paper_2305_03317_amd import _build
    assert sp.lib().sp_header_hash() == _build.header_hash()


def test_status_strings_and_version():
    assert sp.sp_status_string(sp.SP_OK) == "ok"
    assert "1e300" in sp.sp_status_string(sp.SP_WARN_SIGMA_LARGE)
    for code in range(-7, 0):
        assert sp.sp_status_string(code) not in ("", "unknown error")
    assert sp.sp_version() >= 100


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """ctypes mirrors of the header's structs have the C sizes and offsets."""
    import subprocess
    structs = {"sp_batch_config": sp.sp_batch_config, "sp_stats": sp.sp_stats,
               "sp_server_config": sp.sp_server_config, "sp_server_stats": sp.sp_server_stats,
               "sp_kernel_profile": sp.sp_kernel_profile, "sp_sssp_config": sp.sp_sssp_config,
               "sp_sssp_stats": sp.sp_sssp_stats, "sp_pagerank_config": sp.sp_pagerank_config,
               "sp_pagerank_stats": sp.sp_pagerank_stats, "sp_tc_stats": sp.sp_tc_stats,
               "sp_tune_candidate": sp.sp_tune_candidate, "sp_tune_report": sp.sp_tune_report}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sp.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    out = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)], text=True).split("\n") if l)
    for name, cls in structs.items():
        assert int(out[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(out["%s.%s" % (name, f)]) == getattr(cls, f).offset, (name, f)


def test_upload_rejects_bad_arguments_before_touching_a_device():
    L = sp.lib()
    h = ctypes.c_void_p()
    assert L.sp_graph_upload(-1, 0, None, None, 0, None, ctypes.byref(h)) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_graph_upload(3, 4, None, None, 0, None, ctypes.byref(h)) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_graph_upload(3, 0, None, None, 0x80, None, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert "bad arguments" in sp.sp_last_error()


def test_null_graph_rejected():
    L = sp.lib()
    assert L.sp_bc(None, None, 0, None, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_bc_batch(None, None, 0, None, None, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_graph_info(None, None, None, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_graph_release(None) == sp.SP_OK
    assert L.sp_get_last_stats(None) == sp.SP_ERR_INVALID_ARGUMENT


def test_no_device_is_reported_not_crashed():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import numpy as np
    L = sp.lib()
    rp = np.array([0, 1, 2], np.int32)
    ci = np.array([1, 0], np.int32)
    h = ctypes.c_void_p()
    st = L.sp_graph_upload(2, 2, rp.ctypes.data, ci.ctypes.data, 0, None, ctypes.byref(h))
    assert st in (sp.SP_ERR_NOT_SUPPORTED, sp.SP_ERR_DEVICE)


def test_server_calls_reject_bad_arguments_on_the_host():
    L = sp.lib()
    assert L.sp_server_create(None, None) == sp.SP_ERR_INVALID_ARGUMENT
    bad = sp.sp_server_config()
    bad.max_batch = 65
    h = ctypes.c_void_p()
    assert L.sp_server_create(ctypes.byref(bad), ctypes.byref(h)) == sp.SP_ERR_INVALID_ARGUMENT
    bad.max_batch = 0
    bad.reserved[1] = 3
    assert L.sp_server_create(ctypes.byref(bad), ctypes.byref(h)) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_server_add_graph(None, None, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_stream_submit(None, 0, None, 0, None, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_request_wait(None, 0, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_request_poll(None, None, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_request_cancel(None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_request_release(None) == sp.SP_OK
    assert L.sp_server_destroy(None) == sp.SP_OK
    assert L.sp_autotune(None, None, 0, None, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_autotune_get_last_report(None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_graph_fingerprint(None, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_graph_set_tuned(None, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_tune_cache_clear() == sp.SP_OK
    rep = sp.sp_autotune_get_last_report()   # nothing tuned on this thread yet
    assert rep["n_candidates"] == 0 and rep["candidates"] == []
    n = ctypes.c_int32()
    assert L.sp_profile_read(None, 4, ctypes.byref(n)) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_profile_enable(0) == sp.SP_OK
    assert L.sp_profile_enable(8) == sp.SP_ERR_INVALID_ARGUMENT


def test_sssp_calls_reject_bad_arguments_on_the_host():
    L = sp.lib()
    assert L.sp_graph_set_weights(None, None, 0, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_sssp(None, 0, None, None, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_sssp_get_last_stats(None) == sp.SP_ERR_INVALID_ARGUMENT
    assert {"SP_SSSP_AUTO", "SP_SSSP_PUSH", "SP_SSSP_PULL"} <= set(dir(sp))
    assert L.sp_pagerank(None, 1e-6, 0.85, 10, None, None, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_pagerank_get_last_stats(None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_triangle_count(None, None, None, None) == sp.SP_ERR_INVALID_ARGUMENT
    assert L.sp_tc_get_last_stats(None) == sp.SP_ERR_INVALID_ARGUMENT


def test_header_constants_match_binding():
    """Every #define in include/sp.h that the binding mirrors has the same value."""
    import re
    text = open(os.path.join(ROOT, "include", "sp.h")).read()
    defs = dict((k, int(v.rstrip("u"), 0)) for k, v in
                re.findall(r"#define\s+(SP_\w+)\s+\(?(-?(?:0x)?[0-9a-fA-F]+u?)\)?", text))
    mirrored = [k for k in defs if hasattr(sp, k)]
    assert {"SP_OK", "SP_PTR_DEVICE", "SP_VALIDATE", "SP_PROFILE_TIMES", "SP_PROFILE_COUNTS"} <= set(mirrored)
    for k in mirrored:
        assert getattr(sp, k) == defs[k], k


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No CPU fallback: without the built library every call raises."""
    monkeypatch.setattr(sp, "_lib", None)
    monkeypatch.setattr(sp, "LIB_PATH", str(tmp_path / "libsp.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        sp.lib()
    with pytest.raises(RuntimeError):
        sp.sp_graph_upload(np.array([0, 0], dtype=np.int32), np.array([], dtype=np.int32))
