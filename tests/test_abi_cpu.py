"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every function include/lbm.h declares, its lattice tables match the
oracle's, and invalid arguments are rejected before anything is enqueued."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


@pytest.fixture(scope="module")
def lbm():
    from paper_2403_18466_amd import lbm as m
    if not os.path.exists(m.LIB_PATH):
        pytest.fail("liblbm_hip.so is not built (python -m paper_2403_18466_amd.build)")
    m.load_library()
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lbm):
    names = declared_functions()
    assert len(names) >= 16
    lib = ctypes.CDLL(lbm.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(lbm.EXPORTS) == names


def test_tables_match_oracle(lbm):
    for lat in ("D2Q9", "D3Q19"):
        c, w = lbm.lbm_lattice_tables(lat)
        oc, ow = oracle.tables(lat)
        assert np.array_equal(np.array(c), oc)
        assert np.array_equal(np.array(w), ow)


@pytest.mark.parametrize("field,value,status", [
    ("tau", 0.5, 1), ("tau", float("nan"), 1), ("nx", 0, 1), ("batch", 0, 1),
    ("nz", 2, 1), ("hidden", 48, 2), ("rho0", -1.0, 1), ("force_kind", 7, 1),
    ("force_kind", 2, 1),  # three-component force on D2Q9
])
def test_create_rejects_invalid_config(lbm, field, value, status):
    cfg = lbm.Config(nx=16, ny=16, hidden=32, mlp_prec="bf16")
    setattr(cfg, field, value)
    lib = lbm.load_library()
    c = cfg.c_struct()
    ctx = ctypes.c_void_p()
    st = lib.lbm_create(ctypes.byref(c), ctypes.byref(ctx))
    assert st == status
    assert ctx.value is None
    assert lib.lbm_last_error().decode()


def test_create_rejects_oversized_grid(lbm):
    cfg = lbm.Config(nx=65536, ny=65536)
    lib = lbm.load_library()
    c = cfg.c_struct()
    ctx = ctypes.c_void_p()
    assert lib.lbm_create(ctypes.byref(c), ctypes.byref(ctx)) == lbm.LBM_ERR_INVALID
    assert "2^30" in lib.lbm_last_error().decode()


def test_null_arguments_rejected(lbm):
    lib = lbm.load_library()
    assert lib.lbm_create(None, None) == lbm.LBM_ERR_INVALID
    assert lib.lbm_init(None, None, None, None, None) == lbm.LBM_ERR_INVALID
    assert lib.lbm_step(None, None, None, None, 1, None) == lbm.LBM_ERR_INVALID
    assert lib.lbm_adam(None, None, None, None, 4, 1e-3, 0.9, 0.999, 1e-8, 0.0, 1, None) == \
        lbm.LBM_ERR_INVALID
    assert lib.lbm_box_filter(None, None, 1, 1, 4, 4, 1, 2, None) == lbm.LBM_ERR_INVALID
    assert lib.lbm_status_str(3) == b"LBM_ERR_HIP"
    assert lib.lbm_destroy(None) == lbm.LBM_OK
    assert lib.lbm_state_elems(None) == 0


def test_product_path_does_not_import_oracle():
    """The library package never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2403_18466_amd")
    bad = re.compile(r"^\s*(import\s+oracle|from\s+oracle\b)|liblbm_oracle|lbm_oracle\.c", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not bad.search(text), f
