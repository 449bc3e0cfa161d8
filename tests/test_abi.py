"""The C-ABI library loads on the host and exports every symbol the header declares;
argument checks that return before any device work behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spgemm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spgemm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1804_01698_amd import binding
    return binding._lib


def test_header_declares_the_four_phase_calls():
    names = _declared()
    for n in ("spgemm_plan", "spgemm_symbolic", "spgemm_numeric", "spgemm_free"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_and_free_null(lib):
    assert lib.spgemm_strerror(0) == b"ok"
    assert b"shape" in lib.spgemm_strerror(-2)
    assert lib.spgemm_free(None) == 0


def test_host_side_argument_errors(lib):
    from paper_1804_01698_amd import binding as b
    A = b._Csr(4, 5, 0, 1, None, None)
    B = b._Csr(6, 3, 0, 1, None, None)          # 5 != 6: shape mismatch
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t(0)
    st = lib.spgemm_plan(ctypes.byref(h), 1, ctypes.byref(A), ctypes.byref(B), 0, 0,
                         ctypes.c_void_p(1), None, ctypes.byref(ws), None)
    assert st == -2 and not h.value
    st = lib.spgemm_plan(None, 1, ctypes.byref(A), ctypes.byref(A), 0, 0, None, None, ctypes.byref(ws), None)
    assert st == -1
    B2 = b._Csr(5, 3, 0, 1, None, None)
    st = lib.spgemm_plan(ctypes.byref(h), 1, ctypes.byref(A), ctypes.byref(B2), 7, 0,
                         ctypes.c_void_p(1), None, ctypes.byref(ws), None)
    assert st == -1                               # bad dtype
    st = lib.spgemm_plan(ctypes.byref(h), 1, ctypes.byref(A), ctypes.byref(B2), 0, 1 << 9,
                         ctypes.c_void_p(1), None, ctypes.byref(ws), None)
    assert st == -1                               # unknown flag
    bad = b._config_struct(dict(b.default_config(), sym_max=[64] * 9))
    st = lib.spgemm_plan(ctypes.byref(h), 1, ctypes.byref(A), ctypes.byref(B2), 0, 0,
                         ctypes.c_void_p(1), None, ctypes.byref(ws), ctypes.byref(bad))
    assert st == -1 and not h.value               # invalid config, rejected before any device work
    heap = b._config_struct(dict(b.default_config(), heap=1))
    st = lib.spgemm_plan(ctypes.byref(h), 1, ctypes.byref(A), ctypes.byref(B2), 0, 0,
                         ctypes.c_void_p(1), None, ctypes.byref(ws), ctypes.byref(heap))
    assert st == -1 and not h.value               # the heap merge needs sorted output
    assert lib.spgemm_symbolic_static(None, None, None) == -1
    assert b"static scratch" in lib.spgemm_strerror(-11)
    assert lib.spgemm_symbolic(None, None, None, None) == -1
    assert lib.spgemm_stream_copy(None, None, 15, None) == -1
    one = ctypes.c_void_p(8)                      # never dereferenced: every call below is rejected first
    assert lib.spgemm_stanza_read(None, 64, one, 1, 0, one, one, None) == -1        # no array
    assert lib.spgemm_stanza_read(one, 12, one, 1, 0, one, one, None) == -1         # not whole words
    assert lib.spgemm_stanza_read(one, 64, one, 1, 25, one, one, None) == -1        # stanza too long
    assert lib.spgemm_stanza_read(one, 64, one, -1, 0, one, one, None) == -1        # negative count
    assert lib.spgemm_stanza_read(one, 64, None, 1, 0, one, one, None) == -1        # no starts
    assert lib.spgemm_stanza_read(one, 64, one, 1, 0, None, one, None) == -1        # no sum
    assert lib.spgemm_stanza_read(one, 64, one, 1 << 40, 0, one, one, None) == -5   # count overflows


def test_plan_scratch_bytes(lib):
    from paper_1804_01698_amd import binding as b
    arr = (b._Csr * 2)(b._Csr(1000, 10, 0, 1, None, None), b._Csr(0, 10, 0, 1, None, None))
    n = lib.spgemm_plan_scratch_bytes(2, arr)
    assert n >= 1000 * 4 and n % 256 == 0                 # header + row flop
    arr2 = (b._Csr * 2)(b._Csr(1000, 10, 700, 1, None, None), b._Csr(0, 10, 0, 1, None, None))
    # 700 entries: at most 21 rows longer than 32 entries (one 256-byte slot
    # for their list), none longer than 4096
    assert lib.spgemm_plan_scratch_bytes(2, arr2) == n + 256
    arr3 = (b._Csr * 2)(b._Csr(1000, 10, 1 << 20, 1, None, None), b._Csr(0, 10, 0, 1, None, None))
    # lists: every row may be longer than 32 entries, 255 rows longer than 4096
    assert lib.spgemm_plan_scratch_bytes(2, arr3) == n + 4096 + 1024
    assert lib.spgemm_plan_scratch_bytes(0, arr) == 0


def test_config_rules(lib):
    """spgemm_config: defaults fill each table at most half; limits must be
    positive, non-decreasing, within their table and end at the heavy-row
    boundary (checked on the host)."""
    from paper_1804_01698_amd import binding as b
    d = b.default_config()
    sym_t = [64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384]
    num_t = [64, 128, 256, 512, 1024, 2048, 4096, 8192, 11264]
    assert d["hash_mul"] % 2 == 1
    assert d["sym_max"][8] == 8448 and d["num_max"][8] == 8448
    assert all(2 * x <= t for x, t in zip(d["sym_max"][:8], sym_t[:8]))
    assert all(2 * x <= t for x, t in zip(d["num_max"][:8], num_t[:8]))
    assert b.config_ok(d)
    full = dict(d, sym_max=sym_t[:8] + [8448], num_max=num_t[:8] + [8448])
    assert b.config_ok(full)                                      # tables filled to the brim
    assert b.config_ok(dict(d, hash_mul=0))                       # degenerate hash is allowed
    assert d["bucket_slots"] == 4
    assert all(b.config_ok(dict(d, bucket_slots=w)) for w in (4, 8, 16))   # HashVector-style chunks
    assert not any(b.config_ok(dict(d, bucket_slots=w)) for w in (0, 2, 12, 32))
    assert not b.config_ok(dict(d, sym_max=[65] + d["sym_max"][1:]))          # above the 64-key table
    assert not b.config_ok(dict(d, num_max=d["num_max"][:8] + [8000]))        # must end at 8448
    assert not b.config_ok(dict(d, sym_max=[32, 16] + d["sym_max"][2:]))      # decreasing
    assert not b.config_ok(dict(d, num_max=[0] + d["num_max"][1:]))           # not positive
