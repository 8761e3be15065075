"""bench.py's host-side helpers (no GPU): the lookup of counter traffic.

`roofline.traffic` may only carry a figure taken on the kernel sources being
measured and, where the record names them, with the same launch options."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.fixture
def traffic_root(tmp_path, monkeypatch):
    """A copy of the repository layout that bench.py reads: the kernel sources
    (for the hash) and a profiles/traffic.json the test writes."""
    csrc = tmp_path / "paper_1505_04086_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.ROUND_KERNEL_SOURCES:
        (csrc / f).write_bytes(open(os.path.join(ROOT, "paper_1505_04086_amd", "csrc", f), "rb").read())
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))

    def write(rec):
        (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    return tmp_path, write


def _record(single_hash, batched_hash):
    return {"source_hashes": {"mesh3d": single_hash, "batched": batched_hash},
            "workloads": {
                "mesh3d": {"round0_first_fit": {"bytes_per_launch": 111}},
                "batched": {"batched_round0_first_fit": [
                    {"bytes_per_launch": 222, "options": {"chunk": 0, "small_cutoff": -1}},
                    {"bytes_per_launch": 333, "options": {"chunk": 4, "small_cutoff": -1}}]}}}


def test_traffic_for_current_sources(traffic_root):
    root, write = traffic_root
    write(_record(bench.kernel_source_hash("mesh3d"), bench.kernel_source_hash("batched")))
    assert bench.load_traffic("mesh3d", "round0_first_fit") == 111
    # an entry without options matches whatever options the run used
    assert bench.load_traffic("mesh3d", "round0_first_fit", {"chunk": 2}) == 111
    # entries with options match only the same options
    assert bench.load_traffic("batched", "batched_round0_first_fit", {"small_cutoff": -1, "chunk": 0}) == 222
    assert bench.load_traffic("batched", "batched_round0_first_fit", {"chunk": 4, "small_cutoff": -1}) == 333
    assert bench.load_traffic("batched", "batched_round0_first_fit", {"chunk": 8, "small_cutoff": -1}) is None
    assert bench.load_traffic("batched", "batched_round0_first_fit", None) is None
    assert bench.load_traffic("rmat", "round0_first_fit") is None


def test_traffic_dropped_when_code_changes(traffic_root):
    root, write = traffic_root
    write(_record(bench.kernel_source_hash("mesh3d"), bench.kernel_source_hash("batched")))
    opts = {"chunk": 4, "small_cutoff": -1}
    csrc = root / "paper_1505_04086_amd" / "csrc"
    # comments and blank lines are not code: the counters stay valid
    f = csrc / bench.SINGLE_KERNEL_SOURCES[0]
    f.write_bytes(f.read_bytes() + b"\n// a comment\n/* another\n one */\n\n")
    assert bench.load_traffic("mesh3d", "round0_first_fit") == 111
    # a batch-only source: the batch's counters go, the single graph's stay
    b = csrc / "batch.hpp"
    b.write_bytes(b.read_bytes() + b"static int batch_probe;\n")
    assert bench.load_traffic("batched", "batched_round0_first_fit", opts) is None
    assert bench.load_traffic("mesh3d", "round0_first_fit") == 111
    # a shared source: both go
    f.write_bytes(f.read_bytes() + b"static int edited_probe;\n")
    assert bench.load_traffic("mesh3d", "round0_first_fit") is None


def test_code_only_keeps_strings():
    src = b'int a; // c1\n/* block\n comment */ const char *s = "x//y /* z */";\n\n  // only\nint c;\n'
    assert bench._code_only(src) == b'int a;\n const char *s = "x//y /* z */";\nint c;'


def test_traffic_missing_or_unreadable(traffic_root):
    root, write = traffic_root
    assert bench.load_traffic("mesh3d", "round0_first_fit") is None
    (root / "profiles" / "traffic.json").write_text("{not json")
    assert bench.load_traffic("mesh3d", "round0_first_fit") is None


def test_committed_traffic_record_shape():
    """The committed record: per-launch byte counts that follow from its own
    counters and calibration (FETCH_SIZE x fetch factor + WRITE_SIZE x write
    factor, in KiB)."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    cal = rec["calibration"]
    n = 0
    for kernels in rec["workloads"].values():
        for ent in kernels.values():
            for e in (ent if isinstance(ent, list) else [ent]):
                want = e["fetch_kib"] * 1024 * cal["fetch_factor"] + e["write_kib"] * 1024 * cal["write_factor"]
                assert abs(e["bytes_per_launch"] - want) <= 1024 * (cal["fetch_factor"] + cal["write_factor"])
                n += 1
    assert n >= 5
