"""The C-ABI library loads and exports every entry point include/escape.h
declares (no GPU needed: no compute call is made here)."""
import ctypes
import os
import re

import pytest

import paper_1610_09411_amd as esc
from oracle import patterns as pat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "escape.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(esc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_functions():
    assert _declared() == sorted(esc.ABI_FUNCTIONS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(esc.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_params_struct_matches_header():
    """esc_params in the header and the binding's ctypes struct: same fields,
    same order, all int32 (the struct crosses the ABI by pointer)."""
    text = open(os.path.join(ROOT, "include", "escape.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*esc_params;", text).group(1)
    fields = re.findall(r"(\w+)\s+(\w+);", body)
    assert fields and all(t == "int32_t" for t, _ in fields), fields
    assert [n for _, n in fields] == [n for n, _ in esc._Params._fields_]
    assert all(t is ctypes.c_int32 for _, t in esc._Params._fields_)
    assert ctypes.sizeof(esc._Params) == 4 * len(fields)


def test_strerror_and_invalid_arguments():
    assert esc.esc_strerror(esc.ESC_OK) == "ok"
    assert "range" in esc.esc_strerror(esc.ESC_ERANGE)
    lib = esc._load()
    assert lib.esc_inverse_matrix(6, None) == esc.ESC_EINVAL
    assert lib.esc_create(None, 0, 0) == esc.ESC_EINVAL


@pytest.mark.parametrize("k", [4, 5])
def test_library_inverse_matrix_equals_oracle(k):
    assert esc.esc_inverse_matrix(k) == [list(r) for r in pat.a_inverse(k)]


def test_library_inverse_matrix_equals_paper_fig_Ainv():
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_fig_Ainv.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append([int(x) for x in line.split()])
    lib5 = esc.esc_inverse_matrix(5)
    assert [r[:21] for r in lib5[:21]] == rows
