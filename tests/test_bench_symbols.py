"""bench.py names each timed kernel by the instantiation the march launches and
looks up its counted HBM bytes (roofline.traffic) in the committed rocprofv3
summaries by that name: the names must be the profiler's, template arguments
included (the line-row kernel's chunk capacity among them), or the traffic
figure of the bench line would be null."""
import json
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _profiled(name):
    with open(os.path.join(ROOT, "profiles", name)) as fh:
        kernels = json.load(fh)["kernels"]
    return [k[5:] if k.startswith("void ") else k for k in kernels]


@pytest.mark.parametrize("summary, L, n, radix", [
    ("pmc_nig2048_m.json", 3072, 2048, (4, 4, 16, 4)),   # the headline: 2048^2 on L = 3072
    ("pmc_fv512.json", 1024, 512, (16, 4, 4, 4)),
])
@pytest.mark.parametrize("mixed", [False, True])
def test_bench_kernel_names_are_the_profiled_ones(summary, L, n, radix, mixed):
    names = _profiled(summary)
    for cls in ("line_rows", "cols", "rows_inv"):
        sym = bench.kernel_symbol(cls, L, mixed, 3, radix, n)
        assert any(k.startswith(sym + "(") for k in names), (cls, sym)


def test_line_rows_capacity_rule():
    # the smallest of E, 3E/2 and 2E that holds the longest chunk ceil(n / (L / E / 2))
    assert bench.line_rows_capacity(2048, 3072, 16) == 24      # chunks of 22
    assert bench.line_rows_capacity(1536, 3072, 16) == 16      # chunks of 16
    assert bench.line_rows_capacity(3000, 3072, 16) == 32      # chunks of 32
    assert bench.line_rows_capacity(512, 1024, 4) == 4         # chunks of 4
    assert bench.line_rows_capacity(1024, 1536, 4) == 6        # chunks of 6
