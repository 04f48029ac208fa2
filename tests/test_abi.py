"""The C ABI: libgbs.so loads and exports every function include/gbs.h declares
(no compute calls; runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gbs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gbs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gbs_create", "gbs_destroy", "gbs_set_model", "gbs_set_covariance",
                     "gbs_prob_exact", "gbs_prob_approx", "gbs_grad"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2106_01445_amd import gbs
    path = gbs.LIB_PATH
    if not os.path.exists(path):
        pytest.fail(f"{path} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(gbs.EXPORTS) == set(declared_functions())


def test_timing_groups_match_header():
    """The binding's timing buffers are sized from its group list; the library
    writes GBS_TIMING_GROUPS entries."""
    from paper_2106_01445_amd import gbs
    text = open(os.path.join(ROOT, "include", "gbs.h")).read()
    n = int(re.search(r"#define\s+GBS_TIMING_GROUPS\s+(\d+)", text).group(1))
    assert len(gbs.TIMING_GROUPS) == n


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2106_01445_amd import gbs
    saved = gbs._lib
    gbs._lib = None
    try:
        with pytest.raises(ImportError):
            gbs.load(str(tmp_path / "absent.so"))
    finally:
        gbs._lib = saved
