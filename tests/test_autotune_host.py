"""Host-side parts of the autotuner: input classes, candidate limits, the
Eq. 2-style prior and the table loader."""
import json

import numpy as np
import pytest

from paper_1804_01698_amd import autotune as at
from paper_1804_01698_amd import binding as b
from synth import erdos_renyi_fixed_degree, random_sparse, rmat


def test_classes_follow_table4_axes():
    er = erdos_renyi_fixed_degree(4096, 4, 1)
    rm = rmat(12, 16, 1)
    assert at.classify(er, True) == "uniform-sparse-sorted"
    assert at.classify(rm, False) == "skewed-dense-unsorted"


@pytest.mark.parametrize("load", at.LOADS)
def test_candidate_limits_are_valid_configs(load):
    cfg = at.make_config(load, load, at.HASH_MULS[0])
    assert b.config_ok(cfg)
    assert cfg["sym_max"][8] == 8448 and cfg["num_max"][8] == 8448
    assert all(x <= t for x, t in zip(cfg["sym_max"], at.SYM_TABLE))


def test_default_config_is_the_half_load_candidate():
    d = b.default_config()
    c = at.make_config(0.5, 0.5, d["hash_mul"])
    assert c["sym_max"][:8] == d["sym_max"][:8] and c["num_max"][:8] == d["num_max"][:8]


def test_heap_arm_is_a_valid_config():
    d = b.default_config()
    assert d["heap"] == 0
    assert b.config_ok(dict(d, heap=1))
    assert not b.config_ok(dict(d, heap=2))


def test_prior_prefers_emptier_tables_for_probing_but_charges_table_size():
    rng = np.random.default_rng(0)
    flop = rng.integers(200, 256, 1000)
    key = flop.copy()
    nnz = flop.copy()                     # no compression: every product a new key
    c25 = at.prior_cost(flop, key, nnz, at.make_config(0.25, 0.25, 1), False)
    c100 = at.prior_cost(flop, key, nnz, at.make_config(1.0, 1.0, 1), False)
    assert c100 > c25                     # near-full tables: probes dominate
    nnz_small = np.maximum(flop // 16, 1)  # high compression: tables sized by x are mostly empty
    d25 = at.prior_cost(flop, key, nnz_small, at.make_config(0.25, 0.25, 1), False)
    d100 = at.prior_cost(flop, key, nnz_small, at.make_config(1.0, 1.0, 1), False)
    assert d100 < d25
    assert at._probes(np.array([0.0]))[0] == pytest.approx(1.0)


def test_table_roundtrip(tmp_path):
    cfg = at.make_config(0.75, 0.5, at.HASH_MULS[1])
    table = {"device": "x", "created": "t", "classes": {"skewed-dense-sorted": {"config": cfg, "ms": 1.0}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(table))
    t = at.load(str(p))
    assert at.config_for(t, rmat(12, 16, 1), True) == cfg
    assert at.config_for(t, rmat(12, 16, 1), False) is None
    assert at.config_for(None, rmat(12, 16, 1), True) is None
    bad = dict(table, classes={"k": {"config": dict(cfg, sym_max=[1, 2])}})
    p.write_text(json.dumps(bad))
    with pytest.raises(ValueError):
        at.load(str(p))
