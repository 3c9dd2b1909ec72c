"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, and host-side validation rejects malformed input before any device
call (no GPU is needed for these)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2009_12457_amd as bb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bbtc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bbtc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "bbtc_partition" in names and "bbtc_count" in names
    lib = ctypes.CDLL(bb.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(bb._SIGS), "binding and header disagree"


def test_struct_sizes_match_header_layout():
    assert ctypes.sizeof(bb.bbtc_csr) == 40
    assert ctypes.sizeof(bb.bbtc_options) == 48
    assert bb.bbtc_options.device_budget_bytes.offset == 32 and bb.bbtc_options.bound_min_deg.offset == 40
    assert bb.bbtc_options.dense.offset == 44
    assert ctypes.sizeof(bb.bbtc_task) == 24


def test_every_struct_matches_the_c_layout(tmp_path):
    """Size and field offsets of every struct the binding passes, against the
    C compiler's layout of include/bbtc.h (a binding struct shorter than the
    C one would let the library write past a Python-owned buffer)."""
    structs = {"bbtc_csr": bb.bbtc_csr, "bbtc_options": bb.bbtc_options, "bbtc_stats": bb.bbtc_stats,
               "bbtc_hybrid_stats": bb.bbtc_hybrid_stats, "bbtc_tables": bb.bbtc_tables}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bbtc.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name}.{f} %zu\\n", offsetof({name}, {f.rstrip("_")}));')
    lines.append('  printf("bbtc_task %zu\\n", sizeof(bbtc_task));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)
    assert int(got["bbtc_task"]) == bb.TASK_DTYPE.itemsize


def test_options_default():
    o = bb.bbtc_options_default()
    assert (o.p, o.mode, o.cut_mode, o.wave_min, o.hash_min, o.device_budget_bytes, o.bound_min_deg,
            o.dense) == (0,) * 8


def _expect_einval(n, rowptr, colidx, **opts):
    with pytest.raises(bb.BbtcError) as ei:
        bb.bbtc_partition(n, np.asarray(rowptr, np.int64), np.asarray(colidx, np.int32),
                          options=bb.bbtc_options_default(**opts))
    assert ei.value.status == bb.BBTC_EINVAL, str(ei.value)
    return str(ei.value)


def test_host_validation_rejects_malformed_csr():
    assert "self-loop" in _expect_einval(3, [0, 2, 3, 4], [0, 1, 0, 0])
    assert "symmetric" in _expect_einval(3, [0, 1, 2, 2], [1, 2])
    assert "increasing" in _expect_einval(3, [0, 2, 3, 4], [2, 1, 0, 0])
    assert "increasing" in _expect_einval(3, [0, 2, 3, 4], [1, 1, 0, 0])  # duplicate
    assert "range" in _expect_einval(3, [0, 1, 2, 2], [1, 7])
    assert "rowptr" in _expect_einval(3, [1, 1, 2, 2], [1, 0])
    assert "rowptr[n]" in _expect_einval(3, [0, 1, 2, 3], [1, 0])
    assert "non-decreasing" in _expect_einval(3, [0, 2, 1, 2], [1, 0])


def test_option_and_size_checks():
    rp, ci = [0, 1, 2, 2], [1, 0]
    assert "p must" in _expect_einval(3, rp, ci, p=4)      # p > n
    assert "p must" in _expect_einval(3, rp, ci, p=-1)
    assert "p must" in _expect_einval(3000, np.zeros(3001), [], p=2049)  # above the supported maximum
    assert "cut_mode" in _expect_einval(3, rp, ci, cut_mode=7)
    assert "mode" in _expect_einval(3, rp, ci, mode=9)
    assert "negative" in _expect_einval(3, rp, ci, wave_min=-3)
    assert "dense" in _expect_einval(3, rp, ci, dense=2)
    assert "n must" in _expect_einval(0, [0], [])
    assert "even" in _expect_einval(2, [0, 1, 1], [1])


def test_rowptr_bits_check():
    g = bb.bbtc_csr(n=2, nnz=2, rowptr=None, rowptr_bits=16, flags=0, colidx=None)
    h = ctypes.c_void_p()
    st = bb._lib.bbtc_partition(ctypes.byref(g), None, None, ctypes.byref(h))
    assert st == bb.BBTC_EINVAL and not h.value


def test_count_on_missing_plan_is_estate():
    st = bb._lib.bbtc_count(None, None, None, None)
    assert st == bb.BBTC_ESTATE


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the package before torch must not load a second HIP runtime:
    the library has to recognise torch's device pointers and streams."""
    import subprocess
    import sys
    code = ("import paper_2009_12457_amd\nimport torch\n"
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr
    libs = eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs
