"""CPU checks of the C ABI: the library loads, exports every declared entry
point, host-side scheme data agrees with the oracle, and argument errors
that are decided before any device work return the documented codes."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import schemes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfet.h")

B = pytest.importorskip("paper_1102_5071_amd.binding")


def _lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libcfet.so is not built (run python -m paper_1102_5071_amd.build)")
    return B.load()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"CFET_API\s+[\w\s\*]+?\b(cfet_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("cfet_create", "cfet_propagate", "cfet_gradient", "cfet_stats", "cfet_destroy",
                 "cfet_apply", "cfet_last_error", "cfet_tridiag_expm"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert lib.cfet_version() == 1


def test_scheme_enum_matches_header():
    text = open(HEADER).read()
    enum = dict((k, int(v)) for k, v in re.findall(r"(CFET_CF\w+)\s*=\s*(\d+)", text))
    names = {"CF2:1": "CFET_CF2_1", "CF4:2": "CFET_CF4_2", "CF4:3": "CFET_CF4_3",
             "CF4:3Opt": "CFET_CF4_3OPT", "CF6:4": "CFET_CF6_4", "CF6:5": "CFET_CF6_5",
             "CF6:5b": "CFET_CF6_5B", "CF6:6": "CFET_CF6_6", "CF6:5Imp": "CFET_CF6_5IMP",
             "CF6:5Opt": "CFET_CF6_5OPT", "CF6:6Opt": "CFET_CF6_6OPT", "CF8:11": "CFET_CF8_11"}
    for k, v in names.items():
        assert B.SCHEMES[k] == enum[v]


@pytest.mark.parametrize("name", list(S.SCHEMES))
def test_library_scheme_weights_match_oracle(name):
    _lib()
    x, g = B.scheme_info(name)
    xo, go = S.gl_weights(S.scheme(name))
    assert np.allclose(x, xo, atol=1e-16, rtol=0)
    assert g.shape == go.shape
    # independent evaluations (explicit polynomials vs recurrence): a few ulps
    assert np.allclose(g, go, atol=1e-15, rtol=0)


def test_dt_choice_struct_layout():
    # the binding's mirror of cfet_dt_choice: 9 doubles/int64 then 6 int32
    assert ctypes.sizeof(B._DtChoice) == 96
    assert B._DtChoice.order.offset == 72 and B._DtChoice.rounds.offset == 92


def test_batch_stats_struct_layout():
    # the binding's mirror of cfet_batch_stats_t: the launch layout fields,
    # then 12 create-time timings (3 block sizes x 4 rows per lane)
    assert ctypes.sizeof(B._BatchStats) == 168
    assert B._BatchStats.block_threads.offset == 68 and B._BatchStats.tune_us.offset == 72
    assert B._BatchStats.tune_us.size == 96


def test_host_side_argument_errors():
    lib = _lib()
    assert lib.cfet_scheme_info(99, None, None, None, None) == 1
    assert lib.cfet_scheme_info(-1, None, None, None, None) == 1
    assert lib.cfet_create(None, 1, None, None, 0, None) == 1
    out = ctypes.c_void_p()
    assert lib.cfet_create(None, 1, None, None, 0, ctypes.byref(out)) == 1
    assert lib.cfet_create(None, 0, None, None, 0, ctypes.byref(out)) == 1
    assert lib.cfet_create(None, 8, None, None, 0, ctypes.byref(out)) == 1
    assert out.value is None
    assert lib.cfet_tridiag_expm(None, None, 0, 0.1, None, None, None) == 1
    assert lib.cfet_tridiag_expm(None, None, 65, 0.1, None, None, None) == 1
    assert lib.cfet_propagate(None, None, 0.0, 0.1, 1, 1, 4, None) == 1
    assert lib.cfet_propagate_static(None, None, 0.0, 0.1, 1, 1, 4, None) == 1
    assert lib.cfet_propagate_chebyshev(None, None, 0.0, 0.1, 1, 1, 1e-12, None) == 1
    assert lib.cfet_select_dt(None, None, 0.0, 1.0, 10, 1, 2.5, 1, 8, 5.0, 1e-8, 1, 0, None,
                              None) == 1
    assert lib.cfet_stats(None, None) == 1
    assert lib.cfet_destroy(None) == 1
    assert b"null" in lib.cfet_last_error(None)


def _csr(n, diag):
    rp = np.arange(n + 1, dtype=np.int64)
    col = np.arange(n, dtype=np.int32)
    val = np.asarray(diag, dtype=np.complex128)
    return rp, col, val


def test_batch_host_side_argument_errors():
    lib = _lib()
    out = ctypes.c_void_p()
    assert lib.cfet_batch_create(0, None, 1, None, 0, ctypes.byref(out)) == 1
    assert lib.cfet_batch_create(1, None, 1, None, 0, None) == 1
    keep = []
    rp, col, val = _csr(4, [1, 2, 3, 4])
    rp2, col2, val2 = _csr(8, np.ones(8))
    keep += [rp, col, val, rp2, col2, val2]
    ops = (B._CSR * 2)(B._CSR(4, 4, rp.ctypes.data, col.ctypes.data, val.ctypes.data),
                       B._CSR(8, 8, rp2.ctypes.data, col2.ctypes.data, val2.ctypes.data))
    inst = (B._Instance * 1)()
    inst[0].h0 = 0
    inst[0].nterms = 1
    inst[0].hk[0] = 1          # dimension 8 against H0 of dimension 4
    inst[0].fk[0] = B._Drive(0, 1.0, 1.0, 0.0, 0.0, 0.0, 1.0, 0, None, None)
    assert lib.cfet_batch_create(2, ops, 1, inst, 0, ctypes.byref(out)) == 1
    assert b"same n" in lib.cfet_batch_last_error(None)
    inst[0].hk[0] = 5          # out of range
    assert lib.cfet_batch_create(2, ops, 1, inst, 0, ctypes.byref(out)) == 1
    inst[0].hk[0] = 0
    inst[0].nterms = 8         # too many terms
    assert lib.cfet_batch_create(2, ops, 1, inst, 0, ctypes.byref(out)) == 1
    inst[0].nterms = 1
    inst[0].fk[0] = B._Drive(9, 1.0, 1.0, 0.0, 0.0, 0.0, 1.0, 0, None, None)  # bad drive kind
    assert lib.cfet_batch_create(2, ops, 1, inst, 0, ctypes.byref(out)) == 1
    bad = val.copy()
    bad[2] = np.nan
    keep.append(bad)
    ops[0] = B._CSR(4, 4, rp.ctypes.data, col.ctypes.data, bad.ctypes.data)
    assert lib.cfet_batch_create(2, ops, 1, inst, 0, ctypes.byref(out)) == 4
    assert out.value is None
    assert lib.cfet_batch_propagate(None, None, 0.0, 0.1, 1, 1, 4, 0.0, None) == 1
    assert lib.cfet_batch_stats(None, None) == 1
    assert lib.cfet_batch_set_layout(None, 256, 8) == 1
    assert lib.cfet_batch_instance_matvecs(None, None) == 1
    assert lib.cfet_batch_destroy(None) == 0


def test_batch_struct_layout():
    # cfet_instance: 9 int32 then 7 cfet_drive (80 bytes each, 8-byte aligned)
    assert ctypes.sizeof(B._Drive) == 80
    assert ctypes.sizeof(B._Instance) == 40 + 7 * 80


def test_stats_struct_layout():
    # cfet_stats_t: 4 int64, 4 int32, double, int64, double, 4 double, 2 int32,
    # int64 (the library static-asserts the same size)
    assert ctypes.sizeof(B._Stats) == 120
    assert B._Stats.matrix_bytes.offset == 112
