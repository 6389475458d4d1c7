"""CPU checks of the benchmark's cost model and bookkeeping: algorithmic
bytes per key (a probe reads one 128-byte bucket, Section VII-F), the
radix-pass count the library plans, the two-level iceberg geometry, and the
reading of the recorded counter traffic."""
import json

import pytest

import bench
import datagen


def test_query_bytes_are_key_value_flag_plus_one_line_per_probe():
    p = {"insert": 1.109, "pos": 1.109, "neg": 1.81, "mix": 1.459}
    b = bench.algorithmic_bytes(p)
    assert b["find_pos"] == pytest.approx(4 + 4 + 1 + 128 * 1.109)
    assert b["find_neg"] == pytest.approx(9 + 128 * 1.81)
    assert b["find_mix"] == pytest.approx(9 + 128 * 1.459)
    # concurrent build: the pair, then per probe a bucket read and one slot atomic
    assert b["build"] == pytest.approx(8 + 1.109 * (128 + bench.WRITE_GRANULE))


def test_partitioned_build_bytes_at_the_headline_size():
    """2^28 pairs at LF 0.9: two passes, 16 slots x 18,641,352 buckets, the
    reported eviction statistics -> 77.5 bytes per pair."""
    n, m = 1 << 28, 18641352
    stats = {"passes": bench.partition_passes(m, 16), "slots_per_key": m * 16 / n,
             "evicted_per_key": 0.0568, "overflow_probes_per_key": 0.1025}
    assert stats["passes"] == 2
    b = bench.algorithmic_bytes({"insert": 1.1, "pos": 1, "neg": 2, "mix": 1.5}, stats)
    expect = 2 * (4 + 8 + 8) + 8 + 8 * m * 16 / n + 16 * 0.0568 + 0.1025 * (128 + 64)
    assert b["build"] == pytest.approx(expect)
    assert b["build"] == pytest.approx(77.5, abs=0.05)
    # padding that completes lines: a first-pass pair moves 20 B (written,
    # counted, read), a second-pass pair 16 B (written, read by the placement)
    padded = dict(stats, pad1_per_key=0.034, pad2_per_key=0.067)
    b2 = bench.algorithmic_bytes({"insert": 1.1, "pos": 1, "neg": 2, "mix": 1.5}, padded)
    assert b2["build"] == pytest.approx(expect + 20 * 0.034 + 16 * 0.067)


@pytest.mark.parametrize("n,lf,b,passes", [
    (1 << 20, 0.9, 16, 1),          # 72,818 buckets: 143 bins of 512
    (1 << 28, 0.9, 16, 2),          # 36,409 bins
    (1 << 22, 0.9, 16, 1),          # 291,272 buckets: 569 bins
    (1 << 23, 0.9, 16, 2),          # 1,138 bins
    (300000, 0.8, 1, 1),            # one-slot buckets: bins of 4,096 slots
    (4_000_037, 0.8, 1, 2),
])
def test_partition_pass_count(n, lf, b, passes):
    m = -(-datagen.capacity_for(n, lf) // b)
    assert bench.partition_passes(m, b) == passes


def test_two_level_iceberg_geometry():
    """The secondary level holds 1/8 of the primary's slots in 8-slot buckets
    and the load factor counts both levels."""
    n, lf = 1 << 27, 0.86
    m, m2 = bench.scheme_geometry("iht", n, lf, 16, 8)
    assert m2 == m * 16 // 8 // 8
    total = m * 16 + m2 * 8
    assert n / total == pytest.approx(lf, abs=0.001)
    assert bench.scheme_geometry("bcht", n, lf, 16, 0) == (-(-datagen.capacity_for(n, lf) // 16), 0)


def test_recorded_traffic_requires_matching_kernel_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"kernels_sha256_16": "0123456789abcdef", "n": 1 << 28, "build": 1, "find_neg": 2}
    (prof / "bcht_2e28_lf090_hbm_traffic.md").write_text(
        "# summary\n\nTRAFFIC " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0123456789abcdef")
    assert bench.recorded_traffic() == rec
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "fedcba9876543210")
    assert bench.recorded_traffic() is None


def test_kernel_source_sha_ignores_comments_not_code(tmp_path, monkeypatch):
    """The traffic record's key follows the code of the kernel and launch
    sources: a comment edit keeps it, a code edit changes it."""
    csrc = tmp_path / "paper_2108_07232_amd" / "csrc"
    csrc.mkdir(parents=True)
    names = ("bht_hash.hpp", "bht_kernels.hpp", "bht_partition.hpp", "bht.hip")
    for nm in names:
        (csrc / nm).write_text("int f() { return 4; }  // lanes\n/* block\n comment */\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.kernel_source_sha()
    (csrc / "bht.hip").write_text("// new words\n\nint f() { return 4; }  // other words\n")
    assert bench.kernel_source_sha() == base
    (csrc / "bht.hip").write_text("int f() { return 8; }\n")
    assert bench.kernel_source_sha() != base


def test_committed_traffic_line_parses():
    """The committed summary carries one machine-readable line with the
    figures the benchmark reports."""
    path = bench.os.path.join(bench.ROOT, "profiles", "bcht_2e28_lf090_hbm_traffic.md")
    lines = [l for l in open(path) if l.startswith("TRAFFIC ")]
    assert len(lines) == 1
    rec = json.loads(lines[0][len("TRAFFIC "):])
    assert rec["n"] == 1 << 28
    for k in ("build", "find_pos", "find_neg", "find_mix"):
        assert rec[k] > 0
    assert len(rec["kernels_sha256_16"]) == 16
