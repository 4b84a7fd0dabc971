"""The stored full-size digests (tests/golden/fullsize_*.json) agree with the
script that writes them from the oracle (tests/golden/make_fullsize_digests.py):
one fixture per configuration, with the sizes, seeds, quantizer and chunking
that the script uses, so the GPU test compares what the script computed."""
from __future__ import annotations

import json
import re
import sys
from pathlib import Path

import pytest

GOLDEN = Path(__file__).resolve().parent / "golden"
sys.path.insert(0, str(GOLDEN))

import make_fullsize_digests as M  # noqa: E402
from workload import gen  # noqa: E402

HEX = re.compile(r"^[0-9a-f]{64}$")


@pytest.mark.parametrize("name", sorted(M.CONFIGS))
def test_fixture_matches_its_configuration(name):
    path = GOLDEN / f"fullsize_{name}.json"
    assert path.exists(), f"{path.name}: run make_fullsize_digests.py --config {name}"
    doc = json.loads(path.read_text())
    nbits, nodes, length, seed, stride = M.CONFIGS[name]
    w = doc["workload"]
    assert (w["nbits"], w["nodes"], w["length"], w["key_seed"]) == (nbits, nodes, length, seed)
    qp = gen.Q_PLAIN
    assert w["quantizer"] == {"log2_scale": qp.log2_scale, "offset": qp.offset,
                              "delta": qp.delta}
    assert doc["stride"] == stride and doc["chunk"] == M.CHUNK
    assert length % stride == 0
    assert doc["samples"] == nodes * length // stride == M.CHUNK * len(doc["digests"])
    per_node = length // stride
    if nodes > 1:
        assert doc["agg_chunk"] == min(M.CHUNK, per_node)
        assert len(doc["agg_digests"]) * doc["agg_chunk"] == per_node
    else:
        assert doc["agg_digests"] == []
    assert all(HEX.match(d) for d in doc["digests"] + doc["agg_digests"])
    flag = "" if name == M.DEFAULT else f" --config {name}"
    assert doc["written_by"] == f"python tests/golden/make_fullsize_digests.py{flag} (oracle/ only)"


def test_batch_fixture_matches_its_configuration():
    path = GOLDEN / f"fullsize_{M.BATCH}.json"
    assert path.exists(), f"{path.name}: run make_fullsize_digests.py --config {M.BATCH}"
    doc = json.loads(path.read_text())
    w = doc["workload"]
    assert (w["seed"], w["nodes"], w["key_bits"]) == (M.B_SEED, M.B_NODES, list(M.B_KEY_BITS))
    assert w["lengths"] == gen.log_uniform_lengths(M.B_SEED, M.B_NODES, M.B_LO, M.B_HI)
    qp = gen.Q_PLAIN
    assert w["quantizer"] == {"log2_scale": qp.log2_scale, "offset": qp.offset,
                              "delta": qp.delta}
    assert doc["stride"] == M.B_STRIDE
    assert len(doc["node_digests"]) == M.B_NODES and len(doc["agg_digests"]) == len(M.B_KEY_BITS)
    assert all(HEX.match(d) for d in doc["node_digests"] + doc["agg_digests"])
    assert doc["written_by"] == (f"python tests/golden/make_fullsize_digests.py --config {M.BATCH} "
                                 "(oracle/ only)")


def test_no_fixture_without_a_configuration():
    names = {p.name[len("fullsize_"):-len(".json")] for p in GOLDEN.glob("fullsize_*.json")}
    assert names == set(M.CONFIGS) | {M.BATCH}
