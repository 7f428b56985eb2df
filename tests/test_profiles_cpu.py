"""The rocprofv3 summaries under profiles/ and the bench's use of them: a
summary that states HBM traffic names its kernel, workload and the digest of
the kernel sources it was taken on, and the bench reports that figure for
exactly that kernel, workload and digest (else null)."""
import importlib.util
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def summaries():
    out = []
    for name in sorted(os.listdir(PROFILES)):
        if name.endswith(".md"):
            text = open(os.path.join(PROFILES, name)).read()
            keys = {k: v.strip() for k, v in re.findall(r"^- (\w+): (.+)$", text, re.M)}
            out.append((name, text, keys))
    return out


def test_every_summary_gives_its_commands():
    found = summaries()
    assert found, "no rocprofv3 summaries under profiles/"
    for name, text, _ in found:
        assert "rocprofv3 " in text, name
        # commands run committed files only
        assert "_work/" not in text, name


def test_traffic_entries_are_complete_and_found_by_the_bench():
    bench = load_bench()
    with_traffic = [(n, k) for n, _, k in summaries() if "traffic_kernel" in k]
    assert with_traffic, "no summary states the headline kernel's traffic"
    for name, k in with_traffic:
        for key in ("traffic_workload", "source_digest", "traffic_bytes_per_launch"):
            assert key in k, (name, key)
        assert re.fullmatch(r"[0-9a-f]{16}", k["source_digest"]), name
        t = float(k["traffic_bytes_per_launch"])
        assert t > 0, name
        got = bench.traffic_from_profiles(k["traffic_kernel"], k["traffic_workload"], k["source_digest"])
        assert got == t, (name, got, t)
        # another digest (kernel sources changed since) or workload: no figure
        assert bench.traffic_from_profiles(k["traffic_kernel"], k["traffic_workload"], "0" * 16) is None
        assert bench.traffic_from_profiles(k["traffic_kernel"], k["traffic_workload"] + "-x",
                                           k["source_digest"]) is None


def test_source_digest_format():
    bench = load_bench()
    d = bench.source_digest()
    assert re.fullmatch(r"[0-9a-f]{16}", d)
    assert d == bench.source_digest()
