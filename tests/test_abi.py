"""CPU checks of the C-ABI library: it loads and exports what include/pd.h declares.

No compute call is made here (no GPU in this environment)."""
import ctypes
import os

import pytest

from paper_2108_07212_amd import pd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_declares_the_four_problem_calls():
    names = pd.header_functions()
    for n in ("pd_setup", "pd_step", "pd_forces", "pd_damage"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(pd.LIB_PATH), reason="libpd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(pd.LIB_PATH)
    missing = [n for n in pd.header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_refuses_a_missing_library(tmp_path):
    with pytest.raises(ImportError):
        pd._lib = None
        pd.load_library(str(tmp_path / "nope.so"))


def test_struct_layout_matches_header():
    """ctypes records mirror the C structs field by field (names and order)."""
    import re
    txt = open(pd.HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\} pd_problem;", txt, re.S).group(1)
    fields = re.findall(r"([A-Za-z_0-9]+)\s*(?:,|;)", body.replace("*", " "))
    assert fields == [f for f, _ in pd.Problem._fields_]
    body = re.search(r"typedef struct \{([^{}]*)\} pd_tuning;", txt, re.S).group(1)
    fields = re.findall(r"([A-Za-z_0-9]+)\s*(?:,|;)", body)
    assert fields == [f for f, _ in pd.Tuning._fields_]
