"""Host-side checks of bench.py's measurement bookkeeping (no GPU): the
profiled HBM traffic is reported only for the launch options and the kernel
code it was measured with, and the code digest ignores comments."""
import importlib.util
import os
import shutil

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


TUNED = {"threads_per_vertex": 0, "mode": 0, "max_rounds": 0, "frontier_cap": 0, "table_cap": 0,
         "types_per_lane": 1, "headers": 0, "time_window": 7200, "threads_per_query": 768, "query_order": 1}


def _profile_fields(path):
    fields = {}
    for line in open(path):
        line = line.strip().lstrip("-* ").strip()
        for k in ("launch_key", "traffic_bytes_per_launch", "kernel_source_sha256"):
            if line.startswith(k + ":"):
                fields[k] = line.split(":", 1)[1].strip()
    return fields


@pytest.mark.parametrize("name", ["mixed", "city-50k", "region-500k"])
def test_committed_profiles_match_the_kernel_code(name):
    b = _bench()
    path = os.path.join(ROOT, "profiles", f"k_relax_{name}.md")
    f = _profile_fields(path)
    assert f["kernel_source_sha256"] == b.kernel_source_digest(), "profile taken on other kernel code"
    assert b.profiled_traffic(path, f["launch_key"]) == int(f["traffic_bytes_per_launch"])


def test_traffic_only_for_the_profiled_launch_options():
    b = _bench()
    path = os.path.join(ROOT, "profiles", "k_relax_mixed.md")
    key = b.launch_key(TUNED)
    assert key == _profile_fields(path)["launch_key"]
    assert b.profiled_traffic(path, key) is not None
    other = dict(TUNED, time_window=3600)
    assert b.profiled_traffic(path, b.launch_key(other)) is None
    assert b.profiled_traffic(os.path.join(ROOT, "profiles", "no_such_profile.md"), key) is None


def test_digest_ignores_comments_but_not_code(tmp_path, monkeypatch):
    b = _bench()
    src = os.path.join(ROOT, "paper_1912_00966_amd", "csrc")
    fake = tmp_path / "paper_1912_00966_amd" / "csrc"
    fake.mkdir(parents=True)
    for n in b.KERNEL_SOURCES:
        shutil.copy(os.path.join(src, n), fake / n)
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    base = b.kernel_source_digest()
    assert base == _bench().kernel_source_digest()
    target = fake / b.KERNEL_SOURCES[0]
    text = target.read_text()
    target.write_text("// a new comment line\n" + text.replace("\n", "\n\n", 3) + "/* trailing\n block */\n")
    assert b.kernel_source_digest() == base
    target.write_text(text + "\nstatic const int added_for_test = 1;\n")
    assert b.kernel_source_digest() != base
