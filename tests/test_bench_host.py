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


def _fake_dbs(tmp_path, kernels):
    """rocprofv3-like databases: a kernel trace and three counter passes."""
    import sqlite3
    trace = str(tmp_path / "trace.db")
    db = sqlite3.connect(trace)
    db.execute("create table kernels (name text, start integer, end integer)")
    for name, us, _ in kernels:
        for i in range(3):
            db.execute("insert into kernels values (?, ?, ?)", (name, 1000 * i, 1000 * i + int(us * 1000)))
    db.commit()
    dbs = {}
    for kind in ("read", "write", "sq"):
        path = str(tmp_path / f"{kind}.db")
        db = sqlite3.connect(path)
        db.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
        for name, _, counters in kernels:
            for c, v in counters.get(kind, {}).items():
                db.execute("insert into counters_collection values (?, ?, ?)", (name, c, v))
        db.commit()
        dbs[kind] = path
    return trace, dbs


def test_profile_summary_counts_bytes_by_request_size(tmp_path, monkeypatch):
    b = _bench()
    bwd = "void sof::k_render_bwd<16, 8, false>(sof::RenderBwdArgs)"
    copy = "sof::k_peak_copy(HIP_vector_type<float, 4u> const*, HIP_vector_type<float, 4u>*, long)"
    mib = 1
    n128 = (1 << 20) // 128
    kernels = [
        (bwd, 4000.0, {"read": {"TCC_EA0_RDREQ_32B": 10, "TCC_EA0_RDREQ_64B": 20, "TCC_EA0_RDREQ_128B": 30,
                                "TCC_EA0_RDREQ": 60},
                       "write": {"TCC_EA0_WRREQ": 7, "TCC_EA0_WRREQ_64B": 5},
                       "sq": {"SQ_INSTS_VALU": 1.2e9, "SQ_LDS_BANK_CONFLICT": 42}}),
        (copy, 300.0, {"read": {"TCC_EA0_RDREQ_128B": n128, "TCC_EA0_RDREQ": n128},
                       "write": {"TCC_EA0_WRREQ": (1 << 20) // 64, "TCC_EA0_WRREQ_64B": (1 << 20) // 64}}),
    ]
    trace, dbs = _fake_dbs(tmp_path, kernels)
    out = str(tmp_path / "summary.txt")
    monkeypatch.setattr(sys, "argv", ["bench.py", "--summarize", out, "--trace-db", trace, "--read-db", dbs["read"],
                                      "--write-db", dbs["write"], "--sq-db", dbs["sq"], "--calib-copy-mib", str(mib),
                                      "--header", "test summary"])
    args = b.parse()
    b.summarize(args)
    text = open(out).read()
    assert "1.0000 x its size (reads) and 1.0000 x (writes)" in text
    rec = b.read_profile(out)
    r = rec["k_render_bwd<16, 8, false>"]
    assert float(r["read_bytes"]) == 32 * 10 + 64 * 20 + 128 * 30
    assert float(r["write_bytes"]) == 64 * 5 + 32 * 2
    assert float(r["avg_us"]) == 4000.0
    assert r["src"] == b.kernel_source_hash("k_render_bwd<16, 8, false>")
    assert "k_peak_copy" not in rec                      # the reference copy is not a kernel of the method


def test_counter_figures_follow_workload_and_sources(tmp_path, monkeypatch):
    b = _bench()
    k = "k_render_bwd<16, 8, false>"
    line = "\t".join(f"{a}={v}" for a, v in dict(kernel=k, src=b.kernel_source_hash(k), avg_us="4000", read_bytes="1e9",
                                                 write_bytes="2e8", valu="2e9", hbm_frac="0.03", issue_frac="0.8",
                                                 lds_bank_conflict="0").items())
    path = tmp_path / "p.txt"
    path.write_text("header\n" + line + "\n")
    prof = b.read_profile(str(path))
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    args = b.parse()
    assert b.counter_figures(k, args, prof)["read_bytes"] == "1e9"
    # another workload than the one the counters were taken on: no figure
    monkeypatch.setattr(sys, "argv", ["bench.py", "--window", "4"])
    assert b.counter_figures(k, b.parse(), prof) is None
    # changed kernel sources: no figure
    prof[k]["src"] = "0" * 16
    assert b.counter_figures(k, args, prof) is None


def test_default_profiles_merge_with_the_step_summary_last(tmp_path, monkeypatch):
    """A kernel in both default summaries takes the step summary's line (read last)."""
    b = _bench()
    k = "k_project<3>"

    def line(us):
        return "\t".join(f"{a}={v}" for a, v in dict(kernel=k, src=b.kernel_source_hash(k), avg_us=us, read_bytes="1",
                                                     write_bytes="1", valu="1", hbm_frac="0.1", issue_frac="0.1",
                                                     lds_bank_conflict="0").items())
    query, step = tmp_path / "query.txt", tmp_path / "step.txt"
    query.write_text("header\n" + line("7900") + "\n")
    step.write_text("header\n" + line("57") + "\n")
    monkeypatch.setattr(b, "PROFILES", [str(query), str(step)])
    assert b.read_profile()[k]["avg_us"] == "57"
    monkeypatch.setattr(b, "PROFILES", [str(query), str(tmp_path / "missing.txt")])
    assert b.read_profile()[k]["avg_us"] == "7900"          # a missing summary is skipped
