"""Host-side checks of the benchmark's contract and of the committed profiles.

They need no GPU: ``bench.py`` refuses more than one GPU before it touches a
device, and the HBM traffic it reports comes from a committed summary of PMC
counters that is valid only for the executor sources it was taken on.
"""
import importlib.util
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def _bench():
    spec = importlib.util.spec_from_file_location("bench_contract_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line for a run that did not happen


def test_traffic_summary_is_for_the_current_executor_sources():
    b = _bench()
    with open(b.TRAFFIC_FILE) as f:
        t = json.load(f)
    assert t["kernel"] == "k_part_pipe<256>"
    # a stale summary would make the bench line report traffic as null
    assert t["source_hash"] == b.kernel_source_hash()
    assert b.measured_traffic("k_part_pipe<256>") == t["traffic_bytes_per_launch"]
    assert b.measured_traffic("k_tpl") is None


def test_traffic_is_the_calibrated_sum_of_the_two_counters():
    with open(os.path.join(PROFILES, "traffic.json")) as f:
        t = json.load(f)
    # FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; each is scaled by
    # what the same counter reads for a plain copy of known size
    kib = t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]
    assert abs(kib * 1024 - t["traffic_bytes_per_launch"]) <= 1e-5 * t["traffic_bytes_per_launch"]
    # a copy reads each byte once and writes it once; on this chip the fetch
    # counter reports half of a copy's reads, the write counter all of them
    assert 1.9 < t["fetch_scale"] < 2.1 and 0.95 < t["write_scale"] < 1.05


def test_profile_summaries_give_commands_over_committed_files():
    mds = sorted(f for f in os.listdir(PROFILES) if f.endswith(".md"))
    assert mds, "no profile summaries"
    for name in mds:
        with open(os.path.join(PROFILES, name)) as f:
            text = f.read()
        cmds = re.findall(r"```\n(.*?)\n```", text, re.S)
        assert cmds, f"{name}: no command"
        for c in cmds:
            assert "rocprofv3" in c, f"{name}: {c}"
            assert "_work" not in c, f"{name}: command runs an uncommitted file"
            for script in re.findall(r"\$REPO/([\w./-]+\.py)", c):
                assert os.path.exists(os.path.join(ROOT, script)), f"{name}: {script} missing"
        # a summary is text: a few KB, nothing that runs
        assert len(text) < 16 * 1024, name
