"""Host logic of bench.py (CPU): the roofline figures it reports, worked out
by hand, and the rule that a committed HBM traffic record (FETCH_SIZE /
WRITE_SIZE) counts only for the kernel sources and the workload it was taken
on."""
from __future__ import annotations

import json
import shutil
from pathlib import Path

import bench


def test_matrix_instructions_per_product_match_the_counters():
    """The count bench derives from the band geometry equals SQ_INSTS_MFMA per
    Montgomery product and wavefront measured at 2048-, 3072- and 4096-bit keys
    (n^2 of 4096, 6144 and 8192 bits)."""
    assert [bench.mfma_per_product(b) for b in (4096, 6144, 8192)] == [85, 147, 248]


def test_roofline_mfma_by_hand():
    # 524288 encryptions of 2371 Montgomery products each in 1.5 s, 2048-bit key:
    # 2 d^2 byte multiply-accumulates per product, d = 512 bytes of n^2, two
    # int8 operations each, against 5.0e15 int8 operations per second
    r = bench.roofline_mfma(2048, 2371, 524288, 1.5)
    ops = 2 * 524288 * 2371 * 2 * 512 * 512 / 1.5
    issued = 2 * 524288 * 2371 * 85 * 16 * 16 * 64 / 1.5
    assert r["peak"] == 5000.0
    assert r["achieved"] == round(ops / 1e12, 1)
    assert r["frac"] == round(ops / 5.0e15, 4)
    assert r["issued_frac"] == round(issued / 5.0e15, 4)
    assert r["mfma_per_product"] == 85


def test_roofline_valu_by_hand():
    # one v_mad_u64_u32 per lane per clock: 256 CUs x 64 lanes x 2.4 GHz
    r = bench.roofline_valu(256 * 64 * 2.4e9, 1.0)
    assert r["peak"] == 39.322 and r["frac"] == 1.0
    assert bench.roofline_valu(256 * 64 * 2.4e9, 4.0)["frac"] == 0.25


def test_traffic_record_counts_only_for_its_sources_and_workload(tmp_path, monkeypatch):
    real_root = Path(bench.ROOT)
    for kernel, (rec_name, sources) in bench.TRAFFIC.items():
        root = tmp_path / kernel
        csrc = root / "paper_2601_14980_amd" / "csrc"
        csrc.mkdir(parents=True)
        (root / "profiles").mkdir()
        for name in sources:
            shutil.copy(real_root / "paper_2601_14980_amd" / "csrc" / name, csrc / name)
        monkeypatch.setattr(bench, "ROOT", str(root))
        rec = root / "profiles" / rec_name
        assert bench.measured_traffic(kernel, 524288) is None  # no record
        rec.write_text(json.dumps({"source_sha256": bench.kernel_source_hash(kernel),
                                   "elements": 524288, "hbm_bytes_per_launch": 123456789}))
        assert bench.measured_traffic(kernel, 524288) == 123456789
        assert bench.measured_traffic(kernel, 524287) is None  # another workload
        src = csrc / sources[-1]
        src.write_bytes(src.read_bytes() + b"\n")  # a changed source
        assert bench.measured_traffic(kernel, 524288) is None


def test_committed_traffic_records_name_their_kernels_sources():
    """Each committed record carries the hash of the sources it was taken on
    and the counters it scales; whether it still matches them decides only
    whether bench reports it."""
    for kernel, (rec_name, sources) in bench.TRAFFIC.items():
        rec = json.loads((Path(bench.ROOT) / "profiles" / rec_name).read_text())
        assert len(rec["source_sha256"]) == 64 and rec["elements"] == 524288
        assert rec["hbm_bytes_per_launch"] > rec["algorithmic_bytes_per_launch"] > 0
        for name in sources:
            assert (Path(bench.ROOT) / "paper_2601_14980_amd" / "csrc" / name).exists()
