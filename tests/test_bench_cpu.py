"""Host logic of the benchmark: the committed rocprofv3 summaries are read
back only for the kernel sources they were taken with."""
import importlib.util
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _recorded_digest(name):
    text = open(os.path.join(ROOT, "profiles", name)).read()
    return re.search(r"`([0-9a-f]{64})`", text).group(1), text


def test_traffic_summary_parsed_only_for_its_sources(bench, monkeypatch):
    digest, text = _recorded_digest("hbm_traffic_TP4096_order4_fp16x2x6_m16.md")
    row = re.search(r"^\| `k_legendre_tab<[^`]*>` \| \d+ \| [\d.]+ \| [\d.]+ \| ([\d.e+]+) \|$", text, re.M)
    monkeypatch.setattr(bench, "sources_digest", lambda: digest)
    assert bench.measured_traffic("TP4096", "fp16x2:6+m16", "k_legendre_tab") == float(row.group(1))
    assert bench.measured_traffic("TP4096", "fp16x2:5", "k_legendre_tab") is None  # no summary
    assert bench.measured_traffic("TP4096", "fp16x2:6+m16", "k_no_such_kernel") is None
    monkeypatch.setattr(bench, "sources_digest", lambda: "0" * 64)
    assert bench.measured_traffic("TP4096", "fp16x2:6+m16", "k_legendre_tab") is None


def test_form_names(bench):
    """Form strings of --forms: precision, realizations per pass, +m16."""
    assert bench.parse_form("fp16x2:6+m16") == ("fp16x2", 6, True)
    assert bench.parse_form("fp32") == ("fp32", 1, False)
    assert bench.form_name(("fp16x2", 6, True)) == "fp16x2:6+m16"
    assert bench.form_name(("bf16", 1, False)) == "bf16"
    with pytest.raises(ValueError):
        bench.parse_form("fp16x2:6+x")


def test_mfma_summary_parsed_only_for_its_sources(bench, monkeypatch):
    digest, text = _recorded_digest("mfma_TP4096_order4.md")
    monkeypatch.setattr(bench, "sources_digest", lambda: digest)
    for form, kernel in [("fp16x2:6+m16", "k_legendre_tab"), ("fp16:6", "k_legendre_tab"), ("fp32", "k_legendre_mfma")]:
        row = re.search(r"^\| " + re.escape(form) + r" \| `" + kernel + r"<[^`]*>` \| \d+ \| [\d.]+ \| [\d.]+ \| ([\d.]+) \|",
                        text, re.M)
        got = bench.measured_mfma_busy("TP4096", form, kernel)
        assert got == float(row.group(1)) and 0.0 < got <= 100.0
    assert bench.measured_mfma_busy("TP4096", "fp16x2:6+m16", "k_legendre_mfma") is None
    monkeypatch.setattr(bench, "sources_digest", lambda: "0" * 64)
    assert bench.measured_mfma_busy("TP4096", "fp16x2:6+m16", "k_legendre_tab") is None
