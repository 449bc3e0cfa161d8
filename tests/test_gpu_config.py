"""Plan configurations on the GPU: results stay exact under the worst hash
(every key to one bucket), with every table filled to the brim and with the
emptiest tables; the autotuner's table drives exact products."""
import sys

import numpy as np
import pytest

import oracle
from synth import erdos_renyi_fixed_degree, random_sparse, rmat, with_values

from _compare import assert_matches

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_01698_amd as sp
    return sp


def _run(sp, A, B, srt, cfg):
    import torch
    dA, dB = sp.DeviceCSR.from_host(A), sp.DeviceCSR.from_host(B)
    p = sp.Plan([dA], [dB], sorted_output=srt, config=cfg)
    p.symbolic()
    C = p.numeric()[0]
    torch.cuda.synchronize()
    st = p.stats(0)
    p.close()
    assert st["status"] == 0 and st["probe_overflow"] == 0
    return C


CASES = [
    ("er", lambda: (erdos_renyi_fixed_degree(2048, 12, 1), None)),
    ("rmat", lambda: (rmat(11, 8, 2), None)),
    ("i64", lambda: (random_sparse(300, 300, 0.05, 3, values="i64"), random_sparse(300, 400, 0.05, 4, values="i64"))),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("srt", [True, False])
def test_degenerate_hash_is_exact(sp, name, make, srt):
    _note(f"case degenerate hash {name} sorted={srt}")
    A, B = make()
    B = A if B is None else B
    cfg = dict(sp.default_config(), hash_mul=0)
    assert_matches(_run(sp, A, B, srt, cfg), oracle.spgemm(A, B, sorted_output=srt), srt)


@pytest.mark.parametrize("slots", [8, 16])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("srt", [True, False])
def test_wide_buckets_are_exact(sp, slots, name, make, srt):
    # the HashVector-style chunks (Section 4.2.2): 8- and 16-slot buckets at the
    # default hash, at full tables and under the worst hash (every key to the
    # first bucket, so probes run through whole chunks and on to the next)
    _note(f"case wide buckets {slots} {name} sorted={srt}")
    from paper_1804_01698_amd import autotune as at
    A, B = make()
    B = A if B is None else B
    ref = oracle.spgemm(A, B, sorted_output=srt)
    for cfg in (dict(sp.default_config(), bucket_slots=slots),
                dict(at.make_config(1.0, 1.0, at.HASH_MULS[1]), bucket_slots=slots),
                dict(sp.default_config(), hash_mul=0, bucket_slots=slots)):
        assert_matches(_run(sp, A, B, srt, cfg), ref, srt)


@pytest.mark.parametrize("load", [0.25, 1.0])
@pytest.mark.parametrize("srt", [True, False])
def test_table_loads_are_exact(sp, load, srt):
    from paper_1804_01698_amd import autotune as at
    _note(f"case table load {load} sorted={srt}")
    A = rmat(12, 16, 5)
    cfg = at.make_config(load, load, at.HASH_MULS[2])
    assert_matches(_run(sp, A, A, srt, cfg), oracle.spgemm(A, A, sorted_output=srt), srt)


def test_autotune_small_table(sp, tmp_path):
    from paper_1804_01698_amd import autotune as at
    _note("case autotune small")
    classes = {}
    for A, srt in ((erdos_renyi_fixed_degree(4096, 16, 1), False), (rmat(11, 16, 1), True)):
        classes[at.classify(A, srt)] = (A, A, srt)
    path = str(tmp_path / "tuned.json")
    table = at.tune(sp, classes, path=path, top=3, reps=1)
    t = at.load(path)
    assert set(t["classes"]) == set(classes)
    for key, (A, B, srt) in classes.items():
        v = t["classes"][key]
        assert sp.config_ok(v["config"]) and v["ms"] <= v["default_ms"] + 1e-9
        cfg = at.config_for(t, A, srt)
        assert_matches(_run(sp, A, B, srt, cfg), oracle.spgemm(A, B, sorted_output=srt), srt)
    assert table["device"]
