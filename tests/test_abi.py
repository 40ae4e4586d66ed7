"""The C-ABI library loads without a GPU and exports every function include/*.h declares."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))
LIB = os.path.join(ROOT, "paper_2205_08941_amd", "libbsm.so")


def declared_functions():
    text = "\n".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = "\n".join(l for l in text.splitlines() if not l.lstrip().startswith("typedef"))
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\([^;]*\)\s*;", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for n in ["bsm_create_pattern", "bsm_multiply_truncate", "bsm_trace_product", "lnv_step",
              "hotelling_inverse", "bsm_mlp_train", "bsm_pair_descriptors", "lnv_state_reset_guess"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libbsm.so is not built (run python paper_2205_08941_amd/build.py)")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    import paper_2205_08941_amd as bsm
    assert set(declared_functions()) <= set(bsm.EXPORTS)


def test_error_message_without_gpu_is_an_error_code():
    # with no GPU, creating a context must fail with a status code, not crash
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    lib = ctypes.CDLL(LIB)
    h = ctypes.c_void_p()
    code = lib.bsm_ctx_create(0, None, None, None, None, ctypes.byref(h))
    assert code < 0
