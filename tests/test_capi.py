"""The C-ABI library loads, exports every function include/compton.h declares,
and fails cleanly (no compute call) where no GPU is present."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "compton.h")
LIB = os.path.join(ROOT, "paper_2206_02937_amd", "libcompton.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return sorted(set(re.findall(r"\b(cs_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["cs_create", "cs_destroy", "cs_last_error", "cs_compton_step", "cs_sample_plain"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libcompton.so is not built (python -m paper_2206_02937_amd.build)")
    L = C.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_struct_sizes_match_header():
    from paper_2206_02937_amd import compton

    assert C.sizeof(compton.Species) == 40
    assert compton.STATS_BYTES == 128
    # cs_tune_result: n, best, then four arrays of CS_TUNE_MAX (16) 4-byte values
    assert C.sizeof(compton.TuneResult) == 8 + 4 * 16 * 4
    assert [f[0] for f in compton.TuneResult._fields_] == ["n", "best", "strategy", "chunks_per_block",
                                                          "pairs_per_lane", "ms"]


def test_null_context_and_create_errors():
    from paper_2206_02937_amd import compton

    L = compton.lib()
    assert L.cs_destroy(None) == compton.CS_ERR_INVALID_ARG
    assert L.cs_sync(None, None) == compton.CS_ERR_INVALID_ARG
    sp = compton.Species(None, None, None, None, 0)
    assert L.cs_compton_step(None, 0, sp, sp, None, None, 0, 0.1, 1.0, 0, 0, 0, None, None, None) == \
        compton.CS_ERR_INVALID_ARG
    assert L.cs_compton_step_noalloc(None, 0, sp, sp, None, None, 0, 0.1, 1.0, 0, 0, 0, None, None, None) == \
        compton.CS_ERR_INVALID_ARG
    assert L.cs_ntc_graph_create(None, 0, sp, sp, None, None, 0, 0.1, 1.0, 0, 1, None, None, None) == \
        compton.CS_ERR_INVALID_ARG
    assert L.cs_create(None, 0) == compton.CS_ERR_INVALID_ARG
    assert b"NULL" in L.cs_last_error(None)
    import torch

    if not torch.cuda.is_available():
        h = C.c_void_p()
        rc = L.cs_create(C.byref(h), 0)
        assert rc == compton.CS_ERR_HIP and not h.value
        assert len(L.cs_last_error(None)) > 0


def test_library_exports_nothing_else():
    """Built with hidden visibility: the dynamic symbol table holds exactly the
    declared entry points (no internal C++ symbols leak)."""
    import subprocess

    if not os.path.exists(LIB):
        pytest.fail("libcompton.so is not built (python -m paper_2206_02937_amd.build)")
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines() if " T " in ln})
    assert exported == declared_functions()
