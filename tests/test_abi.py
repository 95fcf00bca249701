"""Host-side checks of the C ABI: the library builds, loads without a GPU and
exports every function its headers declare; host-only calls behave."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_2503_10380_amd as cp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    return set(re.findall(r"CPPPL_API\s+[\w\s\*]+?\b(cpppl_\w+)\s*\(", text))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(cp.LIB_PATH):
        from paper_2503_10380_amd import build
        build.build()
    return cp.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared("cpppl.h") | _declared("cpppl_testing.h")
    assert len(names) >= 30
    out = subprocess.run(["nm", "-D", "--defined-only", cp.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = sorted(names - exported)
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)
    # nothing else leaks out of the library under the cpppl_ prefix
    assert {e for e in exported if e.startswith("cpppl_")} == names


def test_binding_covers_header(lib):
    assert set(cp.header_symbols()) == _declared("cpppl.h")


def test_workspace_size_host_only(lib):
    size = C.c_size_t()
    d = cp.Dims(4, 16, 48, 32)
    assert lib.cpppl_workspace_size(C.byref(d), cp.FP64, C.byref(size)) == 0
    s64 = size.value
    assert lib.cpppl_workspace_size(C.byref(d), cp.BF16, C.byref(size)) == 0
    assert size.value > s64 > 0
    bad = cp.Dims(4, 0, 48, 32)
    assert lib.cpppl_workspace_size(C.byref(bad), cp.FP64, C.byref(size)) == -1
    big = cp.Dims(4, 16, 48, 5000)
    assert lib.cpppl_workspace_size(C.byref(big), cp.FP64, C.byref(size)) == -1
    assert lib.cpppl_workspace_size(C.byref(d), 7, C.byref(size)) == -1
    c3 = cp.Dims(32, 256, 768, 1024)
    assert lib.cpppl_workspace_size(C.byref(c3), cp.BF16, C.byref(size)) == 0
    assert size.value < 16 * 2 ** 30  # C3 fits comfortably in one GPU's HBM
    # FP8 needs v % 8 == 0; singles reserve room for tau, t1, D_vo and Dbar
    assert lib.cpppl_workspace_size(C.byref(d), cp.FP8, C.byref(size)) == 0
    assert lib.cpppl_workspace_size(C.byref(cp.Dims(4, 12, 48, 32)), cp.FP8, C.byref(size)) == -1
    for prec in (cp.FP64, cp.BF16, cp.FP8):
        lib.cpppl_workspace_size(C.byref(d), prec, C.byref(size))
        plain = size.value
        lib.cpppl_workspace_size(C.byref(cp.Dims(4, 16, 48, 32, 1)), prec, C.byref(size))
        assert size.value > plain


def test_status_strings_and_null_handling(lib):
    assert lib.cpppl_status_str(0) == b"ok"
    assert lib.cpppl_status_str(-5).startswith(b"normal equations")
    assert lib.cpppl_destroy(None) == -1
    assert lib.cpppl_als(None, None, None) == -1
    d = cp.Dims(4, 16, 48, 32)
    assert lib.cpppl_ws_in_dim(C.byref(d)) == 2 * (2 * 4 + 2 * 16) + 1
    assert lib.cpppl_ws_out_dim(C.byref(d)) == 2 * 4 + 2 * 16


def test_library_built_from_these_sources(lib):
    """The library carries the hash of the sources it was built from, and the
    binding refuses one whose hash differs from the tree's."""
    from paper_2503_10380_amd import build
    assert lib.cpppl_build_hash().decode() == build.source_hash()
    assert len(build.source_hash()) == 64


_CTYPES = {"int": C.c_int, "double": C.c_double, "int64_t": C.c_int64, "double*": C.POINTER(C.c_double)}


def _struct_fields(name):
    """(type, field) pairs of `typedef struct { ... } name;` in cpppl.h, in order."""
    text = open(os.path.join(ROOT, "include", "cpppl.h")).read()
    end = text.index("} " + name + ";")
    body = text[text.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        m = re.match(r"(int64_t|int|double)\s*(\*?)\s*(.+)", decl)
        base, star, names = m.group(1), m.group(2), m.group(3)
        for part in names.split(","):
            part = part.strip()
            ptr = star or part.startswith("*")
            fname = part.lstrip("*").strip()
            arr = re.match(r"(\w+)\[(\d+)\]", fname)
            if arr:
                out.append((_CTYPES[base] * int(arr.group(2)), arr.group(1)))
            else:
                out.append((_CTYPES[base + ("*" if ptr else "")], fname))
    return out


@pytest.mark.parametrize("cname,pyname", [("cpppl_als_opts", "AlsOpts"),
                                          ("cpppl_als_report", "AlsReport"),
                                          ("cpppl_dims", "Dims")])
def test_binding_structs_match_header(cname, pyname):
    """Field names, order and types of the binding's ctypes structures are the
    header's (so the library and the binding agree on the layout)."""
    want = _struct_fields(cname)
    got = getattr(cp, pyname)._fields_
    assert [f for _, f in want] == [f for f, _ in got]
    for (wt, wf), (gf, gt) in zip(want, got):
        assert C.sizeof(wt) == C.sizeof(gt), wf
        assert getattr(wt, "_type_", None) == getattr(gt, "_type_", None), wf
    assert "energy_hist" in [f for f, _ in cp.AlsReport._fields_]
