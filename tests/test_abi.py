"""C ABI: the library loads, exports every function the header declares, and
rejects bad arguments on the host (no GPU needed for these paths)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "gfbp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gfbp_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("gfbp_code_build", "gfbp_code_free", "gfbp_decode_batch", "gfbp_workspace_size", "gfbp_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_cs_0605069_amd as gfbp

    L = gfbp.lib()
    for name in _declared():
        assert hasattr(L, name), f"{name} declared in gfbp.h but not exported"
    assert set(gfbp.EXPORTS) <= set(_declared())
    assert gfbp.version().startswith("gfbp")


def _desc(gfbp, q=4, n=6, m=3, rows=((0, 1, 2), (2, 3, 4), (4, 5, 0)), coef=None, poly=0):
    rp = np.zeros(m + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([c for r in rows for c in r], dtype=np.int32)
    cf = np.ones(len(col), dtype=np.uint8) if coef is None else np.asarray(coef, dtype=np.uint8)
    keep = (rp, col, cf)
    return gfbp.CodeDesc(q, poly, n, m, 0, rp.ctypes.data, col.ctypes.data, cf.ctypes.data), keep


@pytest.mark.parametrize("bad,status", [
    (dict(q=3), -2), (dict(q=128), -2), (dict(q=4, poly=0b101), -1),
    (dict(coef=[1, 1, 4, 1, 1, 1, 1, 1, 1]), -1), (dict(coef=[1, 0, 1, 1, 1, 1, 1, 1, 1]), -1),
    (dict(rows=((0, 1, 1), (2, 3, 4), (4, 5, 0))), -1), (dict(rows=((0, 1, 9), (2, 3, 4), (4, 5, 0))), -1),
])
def test_code_build_rejects_bad_descriptions(bad, status):
    import paper_cs_0605069_amd as gfbp

    d, keep = _desc(gfbp, **bad)
    h = ctypes.c_void_p()
    assert gfbp.lib().gfbp_code_build(ctypes.byref(d), ctypes.byref(h)) == status
    assert h.value is None
    assert gfbp.last_error() != ""


def test_null_arguments():
    import paper_cs_0605069_amd as gfbp

    L = gfbp.lib()
    assert L.gfbp_code_build(None, None) == -1
    assert L.gfbp_decode_batch(None, None, None, None, 0, None) == -1
    assert L.gfbp_workspace_size(None, 10, 0, 0) == 0
    assert L.gfbp_batch_workspace_size(None, None) == 0
    assert L.gfbp_tune_persistent(None, None, None, None, 0, None, 1, None, None) == -1
    assert L.gfbp_code_free(None) == 0
    r = ctypes.c_double(0.0)
    assert L.gfbp_stream_copy_rate(None, None, 16, 1, None, ctypes.byref(r)) == -1
    # host-side argument checks (no device memory is touched): sizes, alignment, overlap
    assert L.gfbp_stream_copy_rate(0x10000, 0x20000, 24, 1, None, ctypes.byref(r)) == -1
    assert L.gfbp_stream_copy_rate(0x10000, 0x20000, 16, 0, None, ctypes.byref(r)) == -1
    assert L.gfbp_stream_copy_rate(0x10008, 0x20000, 16, 1, None, ctypes.byref(r)) == -1
    assert L.gfbp_stream_copy_rate(0x10000, 0x10010, 64, 1, None, ctypes.byref(r)) == -1


@pytest.mark.parametrize("field,value", [("visit_order", [0, 1, 2, 3, 4, 4]), ("visit_order", [0, 1, 2, 3, 4, 6]),
                                         ("source_cols", [1, 1]), ("source_cols", [0, 7])])
def test_code_build_rejects_bad_orders(field, value):
    """A visiting order that is not a permutation of the columns, or a
    source chain with a repeated or out-of-range column, is refused before
    any device work."""
    import paper_cs_0605069_amd as gfbp

    d, keep = _desc(gfbp)
    d.n_info = 2
    arr = np.asarray(value, dtype=np.int32)
    setattr(d, field, arr.ctypes.data)
    h = ctypes.c_void_p()
    assert gfbp.lib().gfbp_code_build(ctypes.byref(d), ctypes.byref(h)) == -1
    assert h.value is None and field.split("_")[0] in gfbp.last_error()


def _header_defines():
    txt = open(os.path.join(ROOT, "include", "gfbp.h")).read()
    return {k: int(v) for k, v in re.findall(r"#define (GFBP_[A-Z0-9_]+) \(?(-?\d+)\)?", txt)}


def _header_struct(name):
    txt = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "gfbp.h")).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + ";", txt).group(1)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        first, *rest = decl.split(",")
        names.append(re.findall(r"(\w+)\s*(?:\[[^\]]*\])?$", first.strip())[0])
        names += [r.strip().lstrip("*").strip() for r in rest]
    return names


def test_binding_constants_match_the_header():
    import paper_cs_0605069_amd as gfbp

    d = _header_defines()
    for name, val in d.items():
        short = name[len("GFBP_"):]
        if hasattr(gfbp, short):
            assert getattr(gfbp, short) == val, name
    for short in ("OPT_SUS_STRICT", "OPT_NO_COMPACT", "OPT_STEP_GRAPHS", "OPT_PRIOR_IN_SWEEP", "OPT_PERSISTENT", "PUS",
                  "SUS", "CH_BSC", "CH_BEC", "CH_BIAWGN", "CH_LIKELIHOOD", "PRIOR_UNIFORM", "PRIOR_MARKOV",
                  "PRIOR_STATIC", "EVIDENCE_SYMBOL", "EVIDENCE_MN"):
        assert "GFBP_" + short in d and getattr(gfbp, short) == d["GFBP_" + short], short


@pytest.mark.parametrize("cname,pyname", [("gfbp_code_desc", "CodeDesc"), ("gfbp_code_info", "CodeInfo"),
                                          ("gfbp_batch", "Batch"), ("gfbp_result", "Result"),
                                          ("gfbp_session_desc", "SessionDesc"), ("gfbp_frames", "FramesIn"),
                                          ("gfbp_retired", "Retired"), ("gfbp_kernel_stats", "KernelStats")])
def test_binding_structs_match_the_header(cname, pyname):
    """The ctypes mirrors list the header's fields in the header's order."""
    import paper_cs_0605069_amd as gfbp

    assert [f[0] for f in getattr(gfbp, pyname)._fields_] == _header_struct(cname)
