"""Host-side logic of bench.py (CPU only): kernel-name parsing for the profile summaries, the
copy-calibrated traffic arithmetic on synthetic counter files, the kernel-hash gate, the algorithmic
byte model, and the one-GPU guard."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

STEP = "void lbm::(anonymous namespace)::step_kernel<{m}, 0, false, false, {bc}, {mrt}, {rows}, {cst}>(lbm::StepArgs)"
COPY = "lbm::(anonymous namespace)::copy_kernel(float __vector(4) const*, float __vector(4)*, long)"


def test_kernel_label():
    assert bench._kernel_label(STEP.format(m=2, bc=0, mrt="false", rows=1, cst="false")) == ("step", "f32", 0, False, False)
    assert bench._kernel_label(STEP.format(m=0, bc=0, mrt="false", rows=0, cst="false"))[1] == "f64"
    assert bench._kernel_label(STEP.format(m=3, bc=0, mrt="false", rows=1, cst="true"))[1] == "f16s"  # cached stores
    # boundary and MRT-R variants are not the periodic benchmark kernels
    assert bench._kernel_label(STEP.format(m=2, bc=1, mrt="false", rows=0, cst="false")) is None
    assert bench._kernel_label(STEP.format(m=2, bc=0, mrt="true", rows=0, cst="false")) is None
    assert bench._kernel_label(COPY) == ("copy",)
    # the two alternating steps of a one-buffer (in-place) instance
    for ip in (1, 2):
        name = STEP.format(m=2, bc=0, mrt="false", rows=1, cst="true").replace(">(", f", {ip}>(")
        assert bench._kernel_label(name) == ("step", "f32", 0, False, False)
    # 3D kernels: velocities, mode, aux, has_k, has_s, walk, cached stores
    k3 = "void lbm::(anonymous namespace)::step3_kernel<27, 3, 0, false, false, 1, true, 0>(lbm::StepArgs)"
    assert bench._kernel3_label(k3) == ("d3q27", "f16s")
    assert bench._kernel3_label(k3.replace("true, 0>", "true, 2>")) == ("d3q27", "f16s")  # an in-place step
    assert bench._kernel3_label(k3.replace("false, false", "true, false")) is None
    assert bench._kernel_label("void lbm::(anonymous namespace)::macros_kernel<2>(lbm::MacroArgs)") is None


def test_bytes_per_lup_model():
    # 9 populations in + 9 out, 2 velocity components (+ kappa field when D varies)
    assert bench.bytes_per_lup("f64", False) == 160 and bench.bytes_per_lup("f64", True) == 168
    assert bench.bytes_per_lup("f32", False) == 80 and bench.bytes_per_lup("f32", True) == 84
    assert bench.bytes_per_lup("f64s_f32m", False) == 152
    assert bench.bytes_per_lup("f16s", False) == 44


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_scales_counters_by_the_copy_kernel(tmp_path):
    """Synthetic counter files: the copy kernel reads half its bytes on FETCH_SIZE; a step kernel
    whose counters read exactly its algorithmic bytes at that scale must come out at ratio 1."""
    n = 2048
    alg = n * n * bench.bytes_per_lup("f32", False)
    copy_kib = 2 * 1024 * 1024  # 2 GiB moved each way
    run = tmp_path / "run"
    _write_csv(str(run / "trace" / "t_kernel_stats.csv"), ["Name", "Calls", "TotalDurationNs", "AverageNs"],
               [[STEP.format(m=2, bc=0, mrt="false", rows=1, cst="false"), 10, 570000, 57000], [COPY, 2, 1300000, 650000]])
    write_kib = 0.5 * alg / 1024                     # any split of alg into writes and reads ...
    fetch_kib = 0.5 * (alg - write_kib * 1024) / 1024  # ... with the reads seen at the copy's 0.5 scale
    for counter, step_val, copy_val in (("FETCH_SIZE", fetch_kib, 0.5 * copy_kib), ("WRITE_SIZE", write_kib, copy_kib)):
        _write_csv(str(run / f"pmc_{counter.lower()}_{n}" / "p_counter_collection.csv"),
                   ["Kernel_Name", "Counter_Name", "Counter_Value"],
                   [[STEP.format(m=2, bc=0, mrt="false", rows=1, cst="false"), counter, step_val]] * 3 + [[COPY, counter, copy_val]])
    pmc = {(c, n): str(run / f"pmc_{c.lower()}_{n}") for c in ("FETCH_SIZE", "WRITE_SIZE")}
    out = tmp_path / "out"
    bench.summarize_profiles({n: str(run / "trace")}, pmc, str(out), {n: "cmd"}, ["c1", "c2"])
    d = json.load(open(out / "step_kernel_pmc.json"))
    e = d["entries"][f"f32_{n}"]
    assert abs(e["fetch_scale"] - 0.5) < 1e-12 and abs(e["write_scale"] - 1.0) < 1e-12
    assert abs(e["traffic_over_algorithmic"] - 1.0) < 1e-12
    assert d["kernel_hash"] == bench.kernel_hash()
    trace = open(out / "step_kernel_trace_2048.md").read()
    assert "57.00" in trace
    # MLUPS and GB/s follow from the average duration: 2048^2 nodes in 57 us, 80 B per node
    assert f"| {n * n / 57e-6 / 1e6:.0f} | {n * n / 57e-6 * 80 / 1e9:.0f} |" in trace


def test_roofline_bound_follows_where_the_state_lives():
    assert bench.roofline_bound(0) == "hbm"
    assert bench.roofline_bound(1) == "infinity_cache"
    assert bench.roofline_bound(2) == "infinity_cache"
    # the cached copy is not mistaken for the calibration copy
    assert bench._kernel_label("lbm::(anonymous namespace)::copy_cached_kernel(float __vector(4) const*, "
                               "float __vector(4)*, long)") is None


def test_traffic_is_withheld_when_the_kernel_changed(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "step_kernel_pmc.json").write_text(json.dumps(
        {"kernel_hash": "0000", "entries": {"f32_2048": {"bytes_per_launch": 1.0}}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_hash", lambda: "1111")
    assert bench.traffic_from_profile("f32", 2048) is None
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0000")
    assert bench.traffic_from_profile("f32", 2048) == 1.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


STEP3 = "void lbm::(anonymous namespace)::step3_kernel<{q}, {m}, 0, false, false>(lbm::StepArgs)"


def test_kernel3_label_and_bytes():
    assert bench._kernel3_label(STEP3.format(q=19, m=2)) == ("d3q19", "f32")
    assert bench._kernel3_label(STEP3.format(q=27, m=0)) == ("d3q27", "f64")
    assert bench._kernel3_label(STEP3.format(q=27, m=0).replace("false, false", "true, false")) is None
    assert bench._kernel3_label(COPY) == ("copy",)
    assert bench._kernel_label(STEP3.format(q=19, m=2)) is None  # not a D2Q9 kernel
    assert bench.bytes_per_lup3(19, "f32") == 164 and bench.bytes_per_lup3(19, "f64") == 328
    assert bench.bytes_per_lup3(27, "f32") == 228 and bench.bytes_per_lup3(27, "f64") == 456
    assert bench.bytes_per_lup3(19, "f16s") == 88


def test_summarize3_scales_counters_by_the_copy_kernel(tmp_path):
    n = 64
    run = tmp_path / "run"
    _write_csv(str(run / "trace3" / "t_kernel_stats.csv"), ["Name", "Calls", "TotalDurationNs", "AverageNs"],
               [[STEP3.format(q=27, m=2), 100, 1000000, 10000]])
    copy_kib = 2 * 1024 * 1024
    alg = n ** 3 * bench.bytes_per_lup3(27, "f32")
    pmc = {}
    for counter, scale in (("FETCH_SIZE", 0.5), ("WRITE_SIZE", 1.0)):
        d = run / f"pmc3_{counter.lower()}"
        _write_csv(str(d / "p_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"],
                   [[STEP3.format(q=27, m=2), counter, scale * alg / 2 / 1024]] * 3 + [[COPY, counter, scale * copy_kib]])
        pmc[counter] = str(d)
    out = tmp_path / "out"
    out.mkdir()
    e = bench.summarize_profiles3(str(run / "trace3"), pmc, str(out), n, "cmd", ["c"])
    assert abs(e["d3q27_f32"]["traffic_over_algorithmic"] - 1.0) < 1e-12
    assert "| d3q27 | f32 |" in open(out / f"step3_kernel_traffic_{n}.md").read()
    assert "10.00" in open(out / f"step3_kernel_trace_{n}.md").read()
