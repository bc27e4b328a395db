"""Host-side checks of the C interface: the library loads without a GPU,
exports every entry point include/gx.h declares, and its host-built
acceptance tables equal the oracle's exact-decimal ones."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_19163_amd", "libgx.so")


def declared():
    src = open(os.path.join(ROOT, "include", "gx.h")).read()
    return sorted(set(re.findall(r"^(?:gx_status|const char \*|void)\s*\*?\s*(gx_[a-z_]+)\s*\(",
                                 src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2603_19163_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "gx_solve" in names and "gx_instance_upload" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    from paper_2603_19163_amd import gx
    assert set(declared()) <= set(gx.EXPORTED)
    for name in declared():
        assert callable(getattr(gx, name))


def test_exp_tables_match_oracle():
    from paper_2603_19163_amd import gx
    hi, lo = gx.gx_exp_tables()
    src = open(os.path.join(ROOT, "oracle", "exp_tables.h")).read()
    nums = [int(x) for x in re.findall(r"(\d+)u", src)]
    assert list(hi) == nums[:16] and list(lo) == nums[16:]


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2603_19163_amd import gx
    with pytest.raises(gx.GxError):
        gx.gx_create(0)
