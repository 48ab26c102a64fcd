"""Host-side behaviour of bench.py that needs no GPU: the one-GPU guard, and the rule that
counter-derived figures (HBM traffic, vector issue) are reported only for the workload and
kernel sources they were measured on."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_figures_follow_workload_and_sources(monkeypatch):
    b = _bench()
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    args = b.parse()
    for k in ("k_render_bwd", "k_render_fwd"):
        # counter figures taken on the current sources (the rule, not the stored values)
        monkeypatch.setitem(b.COUNTERS, k, dict(b.COUNTERS[k], src=b.kernel_source_hash(k)))
        t = b.measured_traffic(k, args)
        assert t is not None and t > 0
        issue = b.measured_issue(k, args, 1.0)
        assert issue is not None and issue["issue_ms"] > 0
    # another workload than the one the counters were taken on: no figure
    monkeypatch.setattr(sys, "argv", ["bench.py", "--window", "4"])
    other = b.parse()
    assert b.measured_traffic("k_render_bwd", other) is None
    assert b.measured_issue("k_render_bwd", other, 1.0) is None
    # changed kernel sources: no figure
    monkeypatch.setitem(b.COUNTERS, "k_render_bwd", dict(b.COUNTERS["k_render_bwd"], src="0" * 16))
    assert b.measured_traffic("k_render_bwd", args) is None
    assert b.measured_issue("k_render_bwd", args, 1.0) is None
