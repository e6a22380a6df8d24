"""C-ABI checks that need no GPU: the library loads, exports every symbol
the public header declares, and its host-side argument logic works."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dashsvd.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dashsvd_\w+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ["dashsvd_create", "dashsvd_run", "dashsvd_get_USV", "dashsvd_destroy",
              "dashsvd_get_info", "dashsvd_status_string"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2404_09276_amd import dashsvd as d
    L = d.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    # and the binding's list covers the header
    assert set(_declared()) <= set(d.EXPORTS) | {"dashsvd_mlp_train_step"}


def test_status_strings():
    from paper_2404_09276_amd import dashsvd as d
    L = d.lib()
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6):
        s = L.dashsvd_status_string(code).decode()
        assert s and s != "unknown status"
    assert L.dashsvd_status_string(99).decode() == "unknown status"


def test_workspace_size_and_argument_checks_host_only():
    """dashsvd_workspace_size runs the driver's sizing pass without touching
    a device; invalid arguments are rejected with ERR_INVALID_ARG."""
    import synth
    from paper_2404_09276_amd import dashsvd as d
    A = synth.config_small()
    ws = d.workspace_size(A, 20, 10, "fp32")
    # at least the panels: Y (2000 x 32) + Q + C (1500 x 32), 4 bytes each
    assert ws > 4 * 32 * (2000 + 2 * 1500)
    ws64 = d.workspace_size(A, 20, 10, "fp64")
    assert ws64 > ws
    with pytest.raises(d.DashSVDError) as e:
        d.workspace_size(A, 20, 0, "fp32")  # oversampling 0
    assert e.value.status == d.ERR_INVALID_ARG
    with pytest.raises(d.DashSVDError):
        d.workspace_size(A, 1400, 200, "fp32")  # l > min(m, n)
    with pytest.raises(d.DashSVDError):
        d.workspace_size(A, 150, 20, "fp32")  # l > MAX_L


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2404_09276_amd import dashsvd as d
    with pytest.raises(d.DashSVDError) as e:
        d.DashSVD()
    assert e.value.status == d.ERR_HIP


def test_binding_refuses_missing_library(tmp_path, monkeypatch):
    from paper_2404_09276_amd import dashsvd as d
    monkeypatch.setattr(d, "_lib", None)
    monkeypatch.setattr(d, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError):
        d.lib()


def test_workspace_size_batched_host_only():
    """The batched form's sizing pass (the layout its run carves out of the
    workspace) runs host-only, grows with the batch, and rejects what the
    batched form does not take."""
    import synth
    from paper_2404_09276_amd import dashsvd as d
    mats = synth.batched_zipf(6, rows=(1000, 3000), seed=77)
    w6 = d.workspace_size_batched(mats, 8, 4, "fp32")
    w3 = d.workspace_size_batched(mats[:3], 8, 4, "fp32")
    assert w6 > w3 > 0
    assert d.workspace_size_batched(mats, 8, 4, "bf16") != w6
    with pytest.raises(d.DashSVDError) as e:
        d.workspace_size_batched(mats, 40, 30, "fp32")  # l above the batched limit
    assert e.value.status == d.ERR_INVALID_ARG
    wide = synth.uniform_csr(300, 700, 5000, seed=3)
    with pytest.raises(d.DashSVDError):
        d.workspace_size_batched(mats[:2] + [wide], 8, 4, "fp32")


_LAYOUT_C = r"""
#include <stddef.h>
#include <stdio.h>
#include "dashsvd.h"
#define F(T, f) printf("%s.%s %zu %zu\n", #T, #f, offsetof(T, f), sizeof(((T *)0)->f));
#define S(T) printf("%s %zu\n", #T, sizeof(T));
int main(void) {
  S(dashsvd_csr) S(dashsvd_options) S(dashsvd_info) S(dashsvd_metrics)
  %FIELDS%
  return 0;
}
"""


def test_struct_layout_matches_header(tmp_path):
    """The ctypes structures of the binding have the size and the field
    offsets of the C structures in include/dashsvd.h, as gcc lays them out:
    a field added, moved or resized on one side of the ABI only fails here
    instead of corrupting a run."""
    import ctypes as C
    import subprocess
    from paper_2404_09276_amd import dashsvd as d
    structs = {"dashsvd_csr": d._Csr, "dashsvd_options": d._Options, "dashsvd_info": d._Info,
               "dashsvd_metrics": d._Metrics}
    fields = "\n  ".join(f"F({cn}, {f[0]})" for cn, py in structs.items() for f in py._fields_)
    src = tmp_path / "layout.c"
    src.write_text(_LAYOUT_C.replace("%FIELDS%", fields))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {}
    for line in out:
        if line:
            parts = line.split()
            got[parts[0]] = tuple(int(x) for x in parts[1:])
    for cn, py in structs.items():
        assert got[cn] == (C.sizeof(py),), cn
        for f in py._fields_:
            desc = getattr(py, f[0])
            assert got[f"{cn}.{f[0]}"] == (desc.offset, desc.size), (cn, f[0])
