"""The C ABI library on the CPU: it loads, exports every declared symbol, and
its host-side logic (code ingestion, schedule, validation, workspace sizing)
behaves as documented.  No call here touches a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2004_09084_amd import qcmet as Q
from paper_2004_09084_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "qcmet.h")).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(qm_\w+)\s*\(", txt, flags=re.M)))


def test_every_declared_symbol_is_exported():
    syms = declared_symbols()
    assert "qm_decode" in syms and "qm_code_create" in syms
    L = ctypes.CDLL(Q.LIB_PATH)
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(Q.EXPORTED) == syms


def test_abi_version():
    assert Q.qm_abi_version() == 1


@pytest.mark.parametrize("spec", [W.RATE01_SMALL, W.RATE01, W.RATE005, W.RATE002], ids=lambda s: s.name)
def test_code_info_and_default_schedule_match_oracle(spec):
    H = W.make_code(spec, 0)
    c = Q.Code(H, spec.Z)
    info = c.info
    assert (info.mb, info.nb, info.Z) == (spec.mb, spec.nb, spec.Z)
    assert info.n == spec.n and info.m == spec.m
    assert info.n_deg1_cols == spec.mb
    assert info.n_type1_cols == spec.ncol1
    assert info.n_type1_entries == int((H[:, :spec.ncol1] >= 0).sum())
    assert info.edges == int((H >= 0).sum()) * spec.Z
    gp, rows = c.schedule()
    gpo, rowso = oracle.greedy_schedule(H)
    assert np.array_equal(gp, gpo) and np.array_equal(rows, rowso)
    assert info.G == len(gp) - 1


def test_schedule_roundtrip_and_conflicts():
    H = np.array([[1, -1, -1], [2, 0, 0], [-1, 2, 1]], dtype=np.int32)   # Eq. (m2)
    c = Q.Code(H, 4)
    gp, rows = c.schedule()
    assert gp.tolist() == [0, 2, 3] and rows.tolist() == [0, 2, 1]
    c.set_schedule([0, 1, 2, 3], [2, 1, 0])
    gp, rows = c.schedule()
    assert gp.tolist() == [0, 1, 2, 3] and rows.tolist() == [2, 1, 0]
    with pytest.raises(Q.QMError) as e:
        c.set_schedule([0, 2, 3], [0, 1, 2])         # rows 0 and 1 share column 0
    assert e.value.code == Q.QM_ERR_SCHEDULE_CONFLICT
    with pytest.raises(Q.QMError) as e:
        c.set_schedule([0, 1, 2, 3], [0, 0, 1])      # not a permutation
    assert e.value.code == Q.QM_ERR_INVALID_ARG
    with pytest.raises(Q.QMError) as e:
        c.set_schedule([0, 1, 3], [0, 2])             # wrong length / end
    assert e.value.code in (Q.QM_ERR_INVALID_ARG,)


def test_invalid_codes_are_rejected():
    with pytest.raises(Q.QMError) as e:
        Q.Code(np.array([[0, 5]], dtype=np.int32), 4)            # shift >= Z
    assert e.value.code == Q.QM_ERR_INVALID_ARG
    with pytest.raises(Q.QMError) as e:
        Q.Code(np.array([[0, -2]], dtype=np.int32), 4)           # below -1
    assert e.value.code == Q.QM_ERR_INVALID_ARG
    # two degree-1 columns in one row
    with pytest.raises(Q.QMError) as e:
        Q.Code(np.array([[0, 1, 2], [0, -1, -1]], dtype=np.int32), 4)
    assert e.value.code == Q.QM_ERR_UNSUPPORTED
    # more than 16 entries in degree>=2 columns in one row
    with pytest.raises(Q.QMError) as e:
        Q.Code(np.zeros((2, 17), dtype=np.int32), 4)
    assert e.value.code == Q.QM_ERR_UNSUPPORTED
    with pytest.raises(Q.QMError):
        Q.qm_code_create(np.zeros((0, 3), dtype=np.int32), 4)


def test_decoder_create_and_workspace_size():
    spec = W.RATE01_SMALL
    H = W.make_code(spec, 0)
    c = Q.Code(H, spec.Z)
    nent = int((H[:, :5] >= 0).sum())
    for F, Fpad in ((1, 1), (4, 4), (5, 8), (64, 64), (100, 128), (128, 128)):
        for fl, msg in ((0, 4), (Q.QM_MSG_FP16, 2)):
            d = Q.qm_decoder_create([c.handle], [F], fl)
            nbytes = Q.qm_decoder_workspace_bytes(d)
            need = Fpad * (spec.n * 4 + nent * spec.Z * msg + spec.m * 4 + spec.m + 4)
            assert need <= nbytes <= need + 7 * 256 + 256 + 64 * 256 * 45, (F, fl)
            Q.qm_decoder_destroy(d)
    with pytest.raises(Q.QMError):
        Q.qm_decoder_create([c.handle], [-1], 0)
    with pytest.raises(Q.QMError):
        Q.qm_decoder_create([c.handle], [4], 0x100)


def test_tuning_validation():
    H = W.make_code(W.RATE01_SMALL, 0)
    c = Q.Code(H, 64)
    d = Q.qm_decoder_create([c.handle], [8], 0)
    t0 = Q.qm_decoder_get_tuning(d)
    assert t0["resident_cap"] == 10 and t0["lds_resident"] == 2   # the library's defaults
    Q.qm_decoder_set_tuning(d, frames_per_tile=8, block=128, merge=0)
    t = Q.qm_decoder_get_tuning(d)
    assert t["frames_per_tile"] == 8 and t["block"] == 128 and t["merge"] == 0
    for bad in (dict(frames_per_tile=3), dict(frames_per_tile=128), dict(block=100), dict(block=512),
                dict(frames_per_lane=3), dict(resident_cap=1), dict(resident_cap=2), dict(resident_cap=65),
                dict(resident_cap=-1), dict(frames_per_batch=-1), dict(lds_resident=3), dict(lds_resident=-1)):
        with pytest.raises(Q.QMError) as e:
            Q.qm_decoder_set_tuning(d, **bad)
        assert e.value.code == Q.QM_ERR_INVALID_ARG
    with pytest.raises(Q.QMError) as e:
        Q.qm_decoder_set_tuning(d, frames_per_lane=4)
    assert e.value.code == Q.QM_ERR_UNSUPPORTED
    Q.qm_decoder_destroy(d)


def test_decode_without_workspace_fails_before_any_device_work():
    H = W.make_code(W.RATE01_SMALL, 0)
    c = Q.Code(H, 64)
    d = Q.qm_decoder_create([c.handle], [4], 0)
    rc = Q.lib().qm_decode(d, ctypes.c_void_p(256), ctypes.c_void_p(256), 1, ctypes.c_void_p(256), None,
                           ctypes.c_void_p(256), None)
    assert rc == Q.QM_ERR_NO_WORKSPACE
    assert b"workspace" in Q.lib().qm_last_error()
    Q.qm_decoder_destroy(d)


def _header_struct_fields(name):
    """(field, C type) pairs of `typedef struct { ... } name;` in the header,
    in declaration order (comments removed; `T a, b;` gives two fields)."""
    txt = open(os.path.join(ROOT, "include", "qcmet.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", txt)
    assert m, name
    out = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        out += [(n.strip(), ctype) for n in names.split(",")]
    return out


@pytest.mark.parametrize("name,cls", [("qm_code_info", Q.qm_code_info), ("qm_tuning", Q.qm_tuning),
                                      ("qm_profile", Q.qm_profile)])
def test_binding_structs_match_header(name, cls):
    # the ctypes mirrors of the header's structs: same fields, order and types
    ctypes_of = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double,
                 "uint32_t": ctypes.c_uint32}
    hdr = _header_struct_fields(name)
    got = [(f, t) for f, t in cls._fields_]
    assert [f for f, _ in hdr] == [f for f, _ in got], name
    for (f, ct), (_, pt) in zip(hdr, got):
        assert ctypes_of[ct] is pt, (name, f, ct, pt)
