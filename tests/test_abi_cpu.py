"""The C ABI without a GPU: the library loads, exports every declared entry
point, lays out fbs_params as the header does, and rejects bad parameters on
the host before touching a device."""
import ctypes
import math
import os
import re
import subprocess

import pytest

from paper_1807_02044_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fbs.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fbs_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    lib = L.lib()
    decl = _declared()
    assert set(decl) == set(L.EXPORTS), (decl, L.EXPORTS)
    for name in decl:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (fbs_\w+)", out))
    assert set(decl) <= exported


def test_params_layout_matches_header(tmp_path):
    src = tmp_path / "off.c"
    fields = [f for f, _ in L.FbsParams._fields_]
    body = "".join(f'printf("%zu ", offsetof(fbs_params, {f}));' for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "fbs.h"\n'
                   f'int main(void){{{body} printf("%zu", sizeof(fbs_params)); return 0;}}\n')
    exe = tmp_path / "off"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True,
                                          text=True).stdout.split()]
    want = [getattr(L.FbsParams, f).offset for f in fields] + [ctypes.sizeof(L.FbsParams)]
    assert got == want


def _ok():
    return L.make_params(64, 48, 1, 0, 15, 4, 4.0, 10.0, 40.0)


@pytest.mark.parametrize("field,value,status", [
    ("width", 0, L.FBS_E_INVALID),
    ("height", -3, L.FBS_E_INVALID),
    ("width", 70000, L.FBS_E_UNSUPPORTED),
    ("channels", 2, L.FBS_E_INVALID),
    ("row_stride", 63, L.FBS_E_INVALID),
    ("d_min", -1, L.FBS_E_INVALID),
    ("d_max", 64, L.FBS_E_INVALID),
    ("radius", -1, L.FBS_E_INVALID),
    ("radius", L.FBS_MAX_RADIUS + 1, L.FBS_E_UNSUPPORTED),
    ("sigma_s", 0.0, L.FBS_E_INVALID),
    ("sigma_r", float("nan"), L.FBS_E_INVALID),
    ("cost_cap", 0.0, L.FBS_E_INVALID),
    ("cost_type", 7, L.FBS_E_INVALID),
    ("flags", 0x100, L.FBS_E_INVALID),
])
def test_validate_rejects(field, value, status):
    p = _ok()
    setattr(p, field, value)
    assert L.fbs_validate(p) == status
    assert L.fbs_last_error() != ""


def test_validate_accepts_limits():
    p = _ok()
    assert L.fbs_validate(p) == L.FBS_OK
    p.sigma_s = p.sigma_r = math.inf          # uniform weights
    p.radius = L.FBS_MAX_RADIUS
    assert L.fbs_validate(p) == L.FBS_OK
    p = L.make_params(2000, 8, 1, 0, L.FBS_MAX_DISP - 1, 0, 1.0, 1.0)
    assert L.fbs_validate(p) == L.FBS_OK
    p.d_max = L.FBS_MAX_DISP
    assert L.fbs_validate(p) == L.FBS_E_UNSUPPORTED


def test_ncc_rules_and_workspace():
    p = _ok()
    assert L.fbs_workspace_bytes(p) == 0
    p.cost_type = L.FBS_COST_NCC
    assert L.fbs_workspace_bytes(p) == 16 * 64 * 48
    p.ncc_radius = L.FBS_MAX_NCC_RADIUS + 1
    assert L.fbs_validate(p) == L.FBS_E_UNSUPPORTED
    p.ncc_radius = 1
    p.channels, p.row_stride = 3, 192
    assert L.fbs_validate(p) == L.FBS_E_UNSUPPORTED


def test_invalid_call_raises_before_device_work():
    p = _ok()
    p.d_max = 99
    with pytest.raises(L.FbsError) as e:
        L.fbs_run(p, 0x1000, 0x2000, 0x3000, 0x4000, None, None, 0)
    assert e.value.status == L.FBS_E_INVALID
    p = _ok()
    p.cost_type = L.FBS_COST_NCC
    with pytest.raises(L.FbsError) as e:
        L.fbs_run(p, 0x1000, 0x2000, 0x3000, 0x4000, None, None, 0)
    assert e.value.status == L.FBS_E_WORKSPACE
    with pytest.raises(L.FbsError) as e:
        L.fbs_cost(_ok(), 0x1000, 0x2000, 0x3002, None, 0)   # misaligned float volume
    assert e.value.status == L.FBS_E_INVALID


def test_status_strings_and_version():
    assert L.fbs_status_str(0) == "ok"
    assert L.fbs_status_str(L.FBS_E_HIP) == "HIP error"
    assert re.match(r"\d+\.\d+\.\d+", L.fbs_version())


def test_header_constants_match_binding():
    """Every #define and enum value of include/fbs.h has the same value in the binding."""
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "fbs.h")).read()
    found = dict(re.findall(r"#define\s+(FBS_\w+)\s+(0x[0-9a-fA-F]+|\d+)u?\b", hdr))
    found.update(re.findall(r"\b(FBS_\w+)\s*=\s*(-?\d+)", hdr))
    assert len(found) >= 12
    for name, val in found.items():
        assert hasattr(L, name), name
        assert getattr(L, name) == int(val, 0), name
