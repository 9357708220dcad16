"""The C-ABI library loads without a GPU and exports every function that
include/dpf.h declares; host-only contexts reject device work cleanly."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2605_10511_amd import dpf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dpf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dpf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("dpf_column_encode", "dpf_hash_build", "dpf_plan_build", "dpf_execute", "dpf_result_get"):
        assert n in names


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(dpf.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(_declared()) <= set(dpf.exported_names())


def test_host_only_context_rejects_device_work():
    ctx = dpf.Context(-1)
    info = ctx.info()
    assert info.device == -1
    with pytest.raises(dpf.DpfError) as e:
        dpf.Column(ctx, np.arange(10, dtype=np.int64), placement="HBM")
    assert e.value.code == dpf.DPF_ERR_INVALID_ARG
    col = dpf.Column(ctx, np.arange(10, dtype=np.int64), placement="HOST")
    with pytest.raises(dpf.DpfError):
        dpf.Hash(ctx, {"k": col}, "k", [], [])
    with pytest.raises(dpf.DpfError):
        dpf.Plan(ctx, {"k": col}, {"filters": [], "probes": [], "group_by": [], "aggs": [{"op": "COUNT"}]}, [])


def test_null_arguments_are_errors_not_crashes():
    lib = dpf.load()
    assert lib.dpf_ctx_create(-1, None, None) == dpf.DPF_ERR_INVALID_ARG
    assert lib.dpf_column_info(None, None) == dpf.DPF_ERR_INVALID_ARG
    assert lib.dpf_execute(None, 1, None, None, None, None) == dpf.DPF_ERR_INVALID_ARG
    assert lib.dpf_plan_blocks(None, None, None) == dpf.DPF_ERR_INVALID_ARG
    assert lib.dpf_plan_footprint(None, None) == dpf.DPF_ERR_INVALID_ARG
    assert b"NULL" in lib.dpf_last_error()


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2605_10511_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f
