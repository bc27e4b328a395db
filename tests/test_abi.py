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


def _c_layout(header, typedefs):
    """sizeof and field offsets of C structs, from a program gcc builds here."""
    import subprocess
    import tempfile
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{header}"', "int main(void) {"]
    for tname, fields in typedefs.items():
        lines.append(f'  printf("{tname} %zu\\n", sizeof({tname}));')
        for f in fields:
            lines.append(f'  printf("{tname}.{f} %zu\\n", offsetof({tname}, {f}));')
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(src, "w").write("\n".join(lines))
        subprocess.check_call(["gcc", "-std=c99", "-o", exe, src])
        out = subprocess.check_output([exe], text=True)
    return dict(l.rsplit(" ", 1) for l in out.splitlines())


def _py_layout(cls):
    d = {cls.__name__: str(ctypes.sizeof(cls))}
    for name, _ in cls._fields_:
        d[f"{cls.__name__}.{name}"] = str(getattr(cls, name).offset)
    return d


def test_binding_structs_match_the_header():
    from paper_2603_19163_amd import gx
    classes = [gx.gx_instance_desc, gx.gx_solve_params, gx.gx_device_info, gx.gx_job_info,
               gx.gx_server_cfg, gx.gx_server_stats, gx.gx_state_scalars, gx.gx_run_stats, gx.gx_sol_aos, gx.gx_peaks]
    c = _c_layout(os.path.join(ROOT, "include", "gx.h"),
                  {k.__name__: [f for f, _ in k._fields_] for k in classes})
    for k in classes:
        for key, val in _py_layout(k).items():
            assert c[key] == val, (key, c[key], val)


def test_numpy_records_match_the_structs():
    import oracle
    from paper_2603_19163_amd import gx
    assert gx.SOL_AOS.itemsize == ctypes.sizeof(gx.gx_sol_aos) == oracle.SOL_AOS.itemsize == 192
    for name, _ in gx.gx_sol_aos._fields_:
        assert gx.SOL_AOS.fields[name][1] == getattr(gx.gx_sol_aos, name).offset
        assert oracle.SOL_AOS.fields[name][1] == getattr(gx.gx_sol_aos, name).offset


def test_oracle_binding_structs_match_its_header():
    import oracle
    pairs = {"or_inst_desc": oracle._Desc, "or_params": oracle._Params, "or_state": oracle._State}
    c = _c_layout(os.path.join(ROOT, "oracle", "oracle.h"), {t: [f for f, _ in k._fields_] for t, k in pairs.items()})
    for t, k in pairs.items():
        py = _py_layout(k)
        assert c[t] == py[k.__name__], t
        for f, _ in k._fields_:
            assert c[f"{t}.{f}"] == py[f"{k.__name__}.{f}"], (t, f)
