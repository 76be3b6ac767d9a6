"""Host-side checks of bench.py: the one-GPU contract of its command line, the
operation census that prices a launch, and the traffic record's validity
rules (no GPU needed)."""
import os
import subprocess
import sys
import types

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("extra,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused(extra, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *extra], capture_output=True, text=True,
                       env=e, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_census_prices_each_unit_of_work():
    # One photon: 6 steps, 4 interactions (so 2 boundary steps), leaving
    # through the +z image; a second photon killed by roulette.
    s = np.zeros(20)
    s[14], s[9], s[10], s[11] = 6.0, 4.0, 2.0, 1.0
    s[5] = 0.9                                     # all exit weight through +z
    c = {u: bench.unit_slots(u) for u in bench.CENSUS}
    expect = 6 * c["step"] + 4 * c["interaction"] + 2 * c["boundary"] + 1 * c["imaged_exit"]
    assert bench.census_slots(s) == pytest.approx(expect)
    # The same exit through a face without an image costs the cheap exit.
    s[5], s[0] = 0.0, 0.9
    assert bench.census_slots(s) == pytest.approx(expect - c["imaged_exit"] + c["other_exit"])


def test_census_classes_and_peak():
    # Half-rate instructions take two full-rate slots, transcendentals four;
    # a step is dominated by Philox's 20 products and 20 three-input XORs.
    assert bench.SLOTS_PER_CLASS == {"full": 1, "half": 2, "trans": 4}
    assert bench.CENSUS["step"]["half"] >= 40
    assert bench.unit_slots("step") == 15 + 2 * 47 + 4 * 4
    # The peak is the published FP32 vector rate in fused multiply-adds.
    assert bench.PEAK_SLOTS_PER_S == pytest.approx(157.3e12 / 2, rel=1e-3)


def test_traffic_record_applies_only_to_its_tally_path_and_sources(monkeypatch):
    log_args = types.SimpleNamespace(atomic_tally=False)
    atomic_args = types.SimpleNamespace(atomic_tally=True)
    rec = dict(bench.TRAFFIC)
    rec["sources_sha256"] = bench.walk_sources_digest()
    monkeypatch.setattr(bench, "TRAFFIC", rec)
    v = bench.measured_traffic(log_args if rec["tally"] == "log" else atomic_args)
    assert v == pytest.approx(1024.0 * (rec["fetch_kib"] * rec["fetch_factor"] + rec["write_kib"] * rec["write_factor"]))
    assert bench.measured_traffic(atomic_args if rec["tally"] == "log" else log_args) is None
    monkeypatch.setattr(bench, "TRAFFIC", dict(rec, sources_sha256="0" * 64))
    assert bench.measured_traffic(log_args) is None and bench.measured_traffic(atomic_args) is None


def test_code_digest_ignores_comments_and_whitespace_only():
    base = "int f(int a) {\n    return a + 1;   // one more\n}\n/* note */\n"
    same = "int f(int a) { return a + 1; }  // edited comment\n/* another\n note */"
    changed = "int f(int a) {\n    return a + 2;   // one more\n}\n"
    assert bench.code_digest(base) == bench.code_digest(same)
    assert bench.code_digest(base) != bench.code_digest(changed)
