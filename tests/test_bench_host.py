"""Host-side logic of bench.py: the traffic record is used only while the
kernel's source, and every local header it includes, is unchanged."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _tree(tmp_path, header_text):
    src = tmp_path / "csrc"
    src.mkdir()
    (src / "k.hip").write_text('#include "core.h"\n#include <hip/hip_runtime.h>\nkernel body\n')
    (src / "core.h").write_text('#include "base.h"\n' + header_text)
    (src / "base.h").write_text("base\n")
    return "csrc/k.hip"


def test_source_hash_follows_local_includes(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rel = _tree(tmp_path, "one\n")
    h0 = bench.kernel_source_sha(rel)
    assert len(h0) == 16 and h0 == bench.kernel_source_sha(rel)
    (tmp_path / "csrc" / "base.h").write_text("base changed\n")   # two includes down
    h1 = bench.kernel_source_sha(rel)
    assert h1 != h0
    (tmp_path / "csrc" / "core.h").write_text('#include "base.h"\ntwo\n')
    assert bench.kernel_source_sha(rel) not in (h0, h1)


def test_traffic_record_dropped_when_source_changes(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rel = _tree(tmp_path, "one\n")
    (tmp_path / "profiles").mkdir()
    rec = {"stencil_r2c": {"source": rel, "source_sha": bench.kernel_source_sha(rel),
                           "bytes_per_launch": 1234}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.traffic_for("stencil_r2c") == 1234
    assert bench.traffic_for("solve_s") is None
    (tmp_path / "csrc" / "core.h").write_text('#include "base.h"\nedited\n')
    assert bench.traffic_for("stencil_r2c") is None

