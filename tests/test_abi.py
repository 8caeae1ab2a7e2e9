"""The C-ABI library loads and exports every entry point that
include/mstruct.h declares; host-side argument checks reject bad calls
without touching a GPU.  CPU only (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mstruct.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mstruct_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_2402_17580_amd as ms
    if not os.path.exists(ms.LIB_PATH):
        pytest.fail("libmstruct.so is not built; run __graft_entry__.build()")
    return ms.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("mstruct_init", "mstruct_step", "mstruct_fused_scan_steps", "mstruct_temperature",
                 "mstruct_mlp_train_step", "mstruct_mlp_forward", "mstruct_mlp_grad"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_binding_covers_every_symbol():
    import paper_2402_17580_amd as ms
    assert sorted(ms.EXPORTS) == _declared()


def test_status_strings(L):
    for code in (0, -1, -2, -3, -4, -5):
        assert L.mstruct_status_string(code)
    assert L.mstruct_status_string(12345) == b"unknown status"
    assert L.mstruct_last_error(None) == b"null context"


def test_null_context_rejected_without_device(L):
    p = ctypes.c_void_p()
    assert L.mstruct_init(None, 0, None) == -1
    assert L.mstruct_destroy(None) == -1
    assert L.mstruct_step(None, None, None, 1e-6, None, None) == -1
    assert L.mstruct_step_implicit(None, None, None, 1e-3, 0.01, 50, None, None, None) == -1
    assert L.mstruct_implicit_unconverged(None, None, 0, None) == -1
    assert L.mstruct_set_option(None, 1, 0) == -1
    assert L.mstruct_wave_counts(None, None, 0, None) == -1
    assert L.mstruct_step_f64(None, None, None, 1e-6, None, 0, None) == -1
    assert L.mstruct_temperature(None, None, None, 0.0, None, None) == -1
    assert L.mstruct_fused_scan_steps(None, None, None, 0.0, 1e-6, 1, 1, 0, None, None) == -1
    assert L.mstruct_gather(None, None, None, 0, None, None) == -1
    assert L.mstruct_check_invariants(None, None, None, 0.0, None, None) == -1
    assert L.mstruct_correct(None, None, None, None) == -1
    assert L.mstruct_mlp_set_params(None, None, None, None, None, None) == -1
    assert L.mstruct_mlp_get_params(None, None) == -1
    assert L.mstruct_mlp_forward(None, None, 0, None, None) == -1
    assert L.mstruct_mlp_grad(None, None, None, 0, None, None, None) == -1
    assert L.mstruct_mlp_train_step(None, None, None, 0, 0.0, None, None) == -1


def test_product_path_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_2402_17580_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", txt, re.M), f
                assert "mstruct_oracle" not in txt and "liborc" not in txt, f


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures of the binding have the sizes and field offsets
    that a C compiler gives the header's structs."""
    import shutil
    import subprocess

    import paper_2402_17580_amd as ms
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"mstruct_phases": ms.PhasesC, "mstruct_phases_f64": ms.PhasesF64C, "mstruct_params": ms.ParamsC}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mstruct.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[f"{cname} size"]) == ctypes.sizeof(py)
        for f, _ in py._fields_:
            assert int(got[f"{cname} {f}"]) == getattr(py, f).offset, (cname, f)


def test_default_params_are_the_paper_tables(L):
    """mstruct_default_params (host only) returns Tables 1-3 and T_as,reg as
    typed from the paper, and the default readings; mstruct_init rejects
    other constants and unknown readings before touching a device."""
    import json

    import paper_2402_17580_amd as ms
    want = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_constants.json")))
    p = ms.default_params()
    pairs = {"T_solidus": "T_s", "T_liquidus": "T_l", "T_ambient": "T_inf", "T_alpha_s_start": "T_as_start",
             "T_alpha_s_end": "T_as_end", "T_alpha_m_start": "T_am_start", "k_alpha_eq": "k_alpha_eq",
             "k_alpha_m_eq": "k_am_eq", "c_alpha_s": "c_as", "c_beta": "c_beta", "k1": "k1", "k2": "k2", "k3": "k3",
             "f": "f", "T_alpha_s_reg": "T_as_reg"}
    for field, key in pairs.items():
        assert getattr(p, field) == want[key], field
    assert p.correction_T == 0 and p.martensite_mode == 0
    h = ctypes.c_void_p()
    q = ms.default_params()
    q.k1 = 0.3
    assert L.mstruct_init(ctypes.byref(q), 0, ctypes.byref(h)) == -4
    q = ms.default_params()
    q.martensite_mode = 2
    assert L.mstruct_init(ctypes.byref(q), 0, ctypes.byref(h)) == -1
    assert L.mstruct_default_params(None) == -1
