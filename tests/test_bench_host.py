"""bench.py host logic: the measured-traffic figure is taken from the committed
counter summary only while the fused kernel's sources are the profiled ones."""
import os

import bench


def test_traffic_none_when_sources_differ(tmp_path, monkeypatch):
    other = tmp_path / "ttc.hip"
    other.write_text("// not the profiled kernel\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(other)])
    assert bench.profiled_traffic() is None


def test_traffic_none_without_profile(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.profiled_traffic() is None


def test_traffic_parsed_when_hash_matches(tmp_path, monkeypatch):
    import hashlib

    src = tmp_path / "k.hip"
    src.write_text("kernel\n")
    prof = tmp_path / "p.md"
    prof.write_text("text\n```\nkernel_source_sha256 = %s\ntraffic_bytes_per_launch = 1234\n```\n"
                    % hashlib.sha256(b"kernel\n").hexdigest())
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    assert bench.profiled_traffic() == 1234


def test_gpus_above_one_exits_with_message(monkeypatch, capsys):
    import pytest

    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
