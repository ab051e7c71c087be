"""The committed rocprofv3 summaries cover the kernels bench.py's roofline names:
the counter summary lists the headline step's calls (so the roofline's traffic
is not silently null) and the kernel-trace summary gives their durations."""
import importlib.util
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


MASK = "lane per particle, forward records accepted-pair bit masks per stencil row, adjoint replays them"


def test_counters_cover_the_headline_calls():
    bench = load_bench()
    for direction in ("fwd", "bwd"):
        names = bench.profile_names(MASK, direction)
        assert names, direction
        traffic = bench.counted_traffic(names)
        assert traffic is not None and traffic > 0, (direction, names)
    # the calibration line is present and states the copy's factors
    text = open(bench.COUNTERS).read()
    assert re.search(r"bytes fetched = [0-9.]+ x FETCH_SIZE", text)
    assert "command:" in text


def test_kernel_trace_lists_the_headline_kernels():
    path = os.path.join(ROOT, "profiles", "spring_cube_n1048576_kernel_stats.txt")
    text = open(path).read()
    bench = load_bench()
    for direction in ("fwd", "bwd"):
        for name in bench.profile_names(MASK, direction):
            rows = [line for line in text.splitlines() if line.startswith(name)]
            assert rows, name
            avg_us = float(rows[0][len(name):].split()[2])
            assert 1.0 < avg_us < 10000.0, (name, avg_us)
