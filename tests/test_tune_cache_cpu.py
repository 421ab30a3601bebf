"""The autotuner's cache (stap_tune_lookup / stap_tune_record, host only):
entries keyed by (architecture, p, q, r_b bound, precision) round-trip through
the JSON file named by KSTAP_TUNE_CACHE, are read back when another writer
changes the file, and bad entries are refused."""
import json
import os

import pytest

import paper_1604_03622_amd as kstap


@pytest.fixture
def cache_file(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("KSTAP_TUNE_CACHE", str(path))
    return path


def test_record_writes_the_file_and_lookup_reads_it(cache_file):
    assert kstap.tune_lookup(3, 16, 4, "fp32", arch="gfx950-test-a") is None
    kstap.tune_record(3, 16, 4, 64, 2, "fp32", ms=12.5, arch="gfx950-test-a")
    kstap.tune_record(3, 12, 6, 32, 1, "bf16x3", ms=3.0, arch="gfx950-test-a")
    data = json.loads(cache_file.read_text())
    assert data["format"] == "kstap-tune-1"
    keys = {(e["arch"], e["p"], e["q"], e["rb_bound"], e["precision"]): (e["pix_per_item"], e["grid_mult"])
            for e in data["entries"]}
    assert keys[("gfx950-test-a", 3, 16, 4, 0)] == (64, 2)
    assert keys[("gfx950-test-a", 3, 12, 8, 1)] == (32, 1)     # r_b = 6 maps to the bound 8
    assert kstap.tune_lookup(3, 16, 3, "fp32", arch="gfx950-test-a") == dict(pix_per_item=64, grid_mult=2)
    assert kstap.tune_lookup(3, 16, 4, "bf16x3", arch="gfx950-test-a") is None
    assert kstap.tune_lookup(3, 16, 4, "fp32", arch="gfx942-test") is None


def test_entries_written_by_another_process_are_read_back(cache_file):
    kstap.tune_record(3, 8, 3, 16, 1, "fp32", arch="gfx950-test-b")
    data = json.loads(cache_file.read_text())
    data["entries"].append(dict(arch="gfx950-test-b", p=3, q=8, rb_bound=8, precision=1, pix_per_item=128,
                                grid_mult=4, ms=1.0))
    os.utime(cache_file, ns=(1, 1))      # a different modification time than the library's own write
    cache_file.write_text(json.dumps(data))
    assert kstap.tune_lookup(3, 8, 7, "bf16x3", arch="gfx950-test-b") == dict(pix_per_item=128, grid_mult=4)
    assert kstap.tune_lookup(3, 8, 3, "fp32", arch="gfx950-test-b") == dict(pix_per_item=16, grid_mult=1)


def test_bad_entries_are_refused(cache_file):
    with pytest.raises(kstap.StapError):
        kstap.tune_record(3, 16, 4, 24, 1, arch="gfx950-test-c")       # not a multiple of the 16-position chain
    with pytest.raises(kstap.StapError):
        kstap.tune_record(3, 16, 4, 32, 0, arch="gfx950-test-c")
    assert kstap.tune_lookup(3, 16, 4, arch="gfx950-test-c") is None


def test_malformed_file_is_ignored(cache_file):
    cache_file.write_text("{not json")
    assert kstap.tune_lookup(3, 16, 4, arch="gfx950-test-d") is None
    kstap.tune_record(3, 16, 4, 32, 2, arch="gfx950-test-d")          # and replaced by a good one
    assert json.loads(cache_file.read_text())["entries"]
