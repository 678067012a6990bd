"""Host-side checks of the HIP library (no GPU needed): it loads and exports
every entry point that include/hd.h declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(hd_[a-z0-9_]+)\s*\(", src))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("hd_build_bvh", "hd_free_bvh", "hd_bound", "hd_status_str"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2406_10357_amd as hd
    lib = hd.load_library()
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    import paper_2406_10357_amd as hd
    lib = hd.load_library()
    for s in range(6):
        assert lib.hd_status_str(s)


def test_product_path_fails_loudly_without_library(tmp_path):
    import paper_2406_10357_amd as hd
    with pytest.raises(RuntimeError):
        hd._lib, saved = None, hd._lib
        try:
            hd.load_library(str(tmp_path / "missing.so"))
        finally:
            hd._lib = saved


def test_binding_structs_match_the_header(tmp_path):
    """Every field of hd_options, hd_stats and hd_round_record sits at the same
    offset in the ctypes binding as in the C header (compiled here)."""
    import ctypes as C
    import subprocess
    import paper_2406_10357_amd as hd
    structs = {"hd_options": hd.Options, "hd_stats": hd.Stats, "hd_round_record": hd.RoundRecord}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    for row in filter(None, out):
        cname, field, val = row.split()
        py = structs[cname]
        want = C.sizeof(py) if field == "size" else getattr(py, field).offset
        assert int(val) == want, (cname, field, int(val), want)


def test_default_options_and_binding_defaults_agree():
    """hd_default_options sets the documented defaults (FP32 with the FP64
    recheck, cascade order 1234, a budget of 1e7, every other field zero),
    and make_options() with no arguments reproduces them field by field."""
    import ctypes as C
    import paper_2406_10357_amd as hd
    lib = hd.load_library()
    o = hd.Options()
    C.memset(C.byref(o), 0xAB, C.sizeof(o))  # garbage first: every field must be set
    lib.hd_default_options(C.byref(o))
    want = {"precision": hd.PREC_FP32_RECHECK, "order": 1234, "budget_m": 1e7}
    for f, _ in hd.Options._fields_:
        v = getattr(o, f)
        if f in want:
            assert v == want[f], (f, v)
        else:
            assert not v, (f, v)
    m = hd.make_options()
    for f, _ in hd.Options._fields_:
        assert getattr(m, f) == getattr(o, f), f
