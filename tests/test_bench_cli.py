"""bench.py host logic (no GPU): the one-GPU guard, the rule that measured
HBM bytes are reported only for the kernel sources they were taken from, and
that the profile summaries name those same sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_are_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_the_profiled_kernel_sources(monkeypatch):
    import bench
    digest = bench.kernel_digest()
    assert len(digest) == 16
    monkeypatch.setattr(bench, "COUNTER_DIGEST", digest)
    monkeypatch.setattr(bench, "COUNTER_TRAFFIC", {"1/256/0": 402902697})
    assert bench.measured_traffic("1/256/0") == 402902697
    assert bench.measured_traffic("2/256/0") is None
    monkeypatch.setattr(bench, "COUNTER_DIGEST", "0" * 16)
    assert bench.measured_traffic("1/256/0") is None
    monkeypatch.setattr(bench, "COUNTER_DIGEST", None)
    assert bench.measured_traffic("1/256/0") is None


def test_profiles_name_the_digest_the_counters_hold():
    # every profile summary that states the kernel sources it was taken
    # from states the digest under which bench.py reports the counted bytes
    import re
    import bench
    pdir = os.path.join(ROOT, "profiles")
    found = {}
    for name in sorted(os.listdir(pdir)):
        text = open(os.path.join(pdir, name)).read()
        for d in re.findall(r"digest\s+([0-9a-f]{16})", text):
            found.setdefault(d, []).append(name)
    assert found, "no profile states its kernel sources digest"
    assert set(found) == {bench.COUNTER_DIGEST}, found
