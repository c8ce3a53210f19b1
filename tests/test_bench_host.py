"""Host-side checks of bench.py: the one-GPU guard, the hardware-queue default and the committed counter
tables it reads (HBM bytes per launch, VALU instructions per chain step).
CPU only: nothing here launches a kernel."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rows(name, width):
    for line in open(os.path.join(ROOT, "profiles", name)):
        f = line.split()
        if line.startswith("#") or not f:
            continue
        assert len(f) == width, line
        yield f


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_hbm_traffic_rows_add_up():
    # traffic_bytes = (FETCH_SIZE x f + WRITE_SIZE x w) x 1024, counters in KiB, with the copy calibration's
    # factors f and w that the table's header states
    import re
    head = open(os.path.join(ROOT, "profiles", "hbm_traffic.txt")).read()
    f = float(re.search(r"x ([0-9.]+) \(FETCH_SIZE\)", head).group(1))
    w = float(re.search(r"x ([0-9.]+) \(WRITE_SIZE\)", head).group(1))
    assert 1.5 < f < 2.5 and 0.5 < w < 1.5
    rows = list(_rows("hbm_traffic.txt", 6))
    assert {r[0] for r in rows} >= {"rf_n1024_int16", "unbiased_n8192_f32"}
    for r in rows:
        assert abs(int(r[5]) - (float(r[3]) * f + float(r[4]) * w) * 1024) <= 1


def test_valu_rows_divide_out_and_gate_on_the_kernel_source():
    rows = list(_rows("valu_issue.txt", 6))
    assert {r[0] for r in rows} >= {"rf_n1024_int16", "unbiased_n8192_f32"}
    for r in rows:
        assert abs(float(r[3]) / float(r[4]) - float(r[5])) < 0.1
        tile = tuple(int(v) for v in r[1].split("x"))
        got = bench._valu_per_chain_step(r[0], tile)
        # reported exactly when the row was counted on the current kernel source
        assert (got is not None) == any(q[0] == r[0] and q[1] == r[1] and q[2] == _current_sha() for q in rows)
        # another tile runs other code
        assert bench._valu_per_chain_step(r[0], (tile[0] * 2, tile[1])) is None


def test_issue_peak():
    # 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per SIMD every 4 cycles
    assert bench.VALU_ISSUE_PEAK == 6.144e11


def _current_sha():
    # the step kernel's source (the VALU rows are step-kernel runs)
    import hashlib
    src = os.path.join(ROOT, "paper_2210_10513_amd", "csrc", "pns_step.h")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def test_window_kernel_rows_hash_both_sources():
    import hashlib
    h = hashlib.sha256()
    for name in ("pns_step.h", "pns_wave.h"):
        h.update(open(os.path.join(ROOT, "paper_2210_10513_amd", "csrc", name), "rb").read())
    assert bench._kernel_sha(True) == h.hexdigest()[:16]
    assert bench._kernel_sha() == _current_sha() != bench._kernel_sha(True)


def test_cpu_baseline_child_reports_one_core_and_all_cores():
    """The oracle leg runs in a child process that never touches the GPU and
    reports the CPU model, one core and one process per core."""
    import json
    spec = json.dumps({"workload": "rf_n1024_int16", "budget_s": 0.3})
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-baseline", spec],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["value"] > 0 and out["cpu_model"]
    if "all_cores" in out:
        assert out["all_cores"]["cores"] > 1 and out["all_cores"]["value"] > 0


def test_hardware_queue_default_follows_the_launch_form(monkeypatch):
    """Twelve queues for launches queued directly (one per class stream and
    the context's stream), eight for graph replays, and an explicit
    --hw-queues wins."""
    import bench
    for argv, want in ((["bench.py"], "12"), (["bench.py", "--launch", "graph"], "8"),
                       (["bench.py", "--launch=graph"], "8"), (["bench.py", "--launch", "graph", "--hw-queues", "6"], "6"),
                       (["bench.py", "--hw-queues=10"], "10")):
        monkeypatch.setattr(sys, "argv", argv)
        assert bench._hw_queues_arg() == want, argv


def test_batch_issue_roofline_adds_the_classes_committed_rows():
    """The batch's VALU issue figure is the sum over launch classes of the
    committed VALU instructions per chain step times the class's chain steps,
    over the step time; a class without a row for its current kernel source
    gives no figure."""
    rows = [f for f in _rows("valu_issue.txt", 6) if f[0].startswith("batched64_class_")]
    assert rows
    classes = []
    for f in rows[:3]:
        key = f[0][len("batched64_class_"):]
        tile, flav, chains, nr = key.split("_")
        n0, n1 = nr[1:].split("-")
        classes.append({"tile": tile, "flavour": int(flav[1:]), "chains": int(chains[1:]), "N_min": int(n0),
                        "N_max": int(n1)})
    r = bench._batch_issue_roofline(classes, 1000, 0.5)
    if r is None:  # rows of an older kernel source: nothing to check against
        return
    want = sum(bench._valu_per_chain_step(bench._class_key(c), tuple(int(v) for v in c["tile"].split("x")),
                                          c["flavour"] == 5) * c["chains"] * 1000 for c in classes)
    assert abs(r["valu_per_step"] - want) <= 1e-9 * want
    assert abs(r["achieved"] - want / 0.5) <= 1e-9 * want / 0.5
    assert abs(r["frac"] - r["achieved"] / bench.VALU_ISSUE_PEAK) < 1e-12
    unknown = dict(classes[0], chains=classes[0]["chains"] + 1)
    assert bench._batch_issue_roofline(classes + [unknown], 1000, 0.5) is None
