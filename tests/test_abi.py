"""CPU-side checks of the C ABI: the library loads and exports every declared entry point
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "adelia.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*\*?\s+\**([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_hot_path_calls():
    names = declared_functions()
    for n in ["bta_factor", "bta_factor_batched", "bta_logdet", "bta_solve", "bta_selinv",
              "inla_objective", "inla_grad", "inla_grad_batched", "inla_fd_grad", "inla_hessian",
              "inla_fd_hessian"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2605_06392_amd._lib import LIB_PATH, SIGNATURES
    if not os.path.exists(LIB_PATH):
        pytest.fail("libadelia.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    for name in SIGNATURES:
        assert name in declared_functions(), name
