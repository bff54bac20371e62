"""The C ABI library loads without a GPU and exports every entry point the
header declares; argument checks that need no device behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "heqg.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(heqg_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2406_13221_amd import heqg
    return heqg.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared()
    assert len(names) >= 35
    for n in names:
        assert hasattr(L, n), n


def test_binding_covers_the_header(L):
    from paper_2406_13221_amd import heqg
    assert sorted(heqg.EXPORTS) == declared()


def test_param_validation_without_device(L):
    from paper_2406_13221_amd import heqg
    qb = (ctypes.c_int * 3)(40, 40, 40)
    bad = heqg.Params(11, 3, qb, 2, 60, 2, 40)            # log2N below the supported range
    assert L.heqg_ctx_tables_bytes(ctypes.byref(bad)) == 0
    assert b"log2N" in L.heqg_last_error()
    ok = heqg.Params(12, 3, qb, 2, 60, 2, 40)
    n = L.heqg_ctx_tables_bytes(ctypes.byref(ok))
    assert n >= 5 * 4096 * 16 * 2
    small_p = heqg.Params(12, 3, qb, 1, 60, 1, 40)        # alpha = 3 > n_p = 1
    assert L.heqg_ctx_tables_bytes(ctypes.byref(small_p)) == 0
    h = ctypes.c_void_p()
    assert L.heqg_ctx_create(ctypes.byref(ok), None, 0, ctypes.byref(h)) == heqg.ERR_ARG


def test_null_arguments_are_rejected(L):
    from paper_2406_13221_amd import heqg
    assert L.heqg_encode(None, None, 0, 1.0, None) == heqg.ERR_ARG
    assert L.heqg_add(None, None, None, None, None) == heqg.ERR_ARG
    assert L.heqg_nag_qg_step(None, None, None, None, None, None, None, None, 1, None, 0, None) == heqg.ERR_ARG
    assert L.heqg_keys_bytes(None, 3) == 0


def test_profiling_classes_without_device(L):
    # nothing sampled: zeros; a class outside 0..2 is an error
    assert L.heqg_prof_start(4) == 0
    a, n = ctypes.c_double(1.0), ctypes.c_int64(1)
    r, sr, op = ctypes.c_double(1.0), ctypes.c_double(1.0), ctypes.c_double(1.0)
    for k in range(3):
        assert L.heqg_prof_stop(k, ctypes.byref(a), ctypes.byref(n), ctypes.byref(r), ctypes.byref(sr),
                                ctypes.byref(op)) == 0
        assert (a.value, n.value, r.value, sr.value, op.value) == (0.0, 0, 0.0, 0.0, 0.0)
    assert L.heqg_prof_stop(3, None, None, None, None, None) == -1
    assert L.heqg_prof_stop(-1, None, None, None, None, None) == -1
