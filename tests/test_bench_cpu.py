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


def test_sweep_sample_is_shared_by_every_grid(bench):
    """The sweep's sky positions: (ring, column) on the oversampling-1 grid of
    lmax + 1 rings and 2 lmax columns, distinct, off the pole rings; the
    same angles are (g ring, g column) on the grid of oversampling g."""
    import math

    import numpy as np

    lmax = 64
    R, C = bench.sweep_sample(lmax)
    assert R.size == C.size == 16 * 32
    assert R.min() >= 1 and R.max() <= lmax - 1 and C.min() >= 0 and C.max() < 2 * lmax
    assert len(set(zip(R.tolist(), C.tolist()))) == R.size
    for g in (1, 2, 3):
        th1, th_g = math.pi * R / lmax, math.pi * (g * R) / (g * lmax)
        ph1, ph_g = 2 * math.pi * C / (2 * lmax), 2 * math.pi * (g * C) / (2 * g * lmax)
        assert np.allclose(th1, th_g) and np.allclose(ph1, ph_g)


def test_sweep_fastest_settings(bench):
    """For each lmax and target, the fastest row within the target; None
    where no row reaches it."""
    rows = [{"lmax": 8, "oversampling": 1, "order": o, "form": "fp32", "ms_per_map": 1.0 + o,
             "rel_rms_err_max": 10.0 ** (-o)} for o in range(1, 5)]
    rows.append({"lmax": 8, "oversampling": 2, "order": 2, "form": "fp32", "ms_per_map": 3.5,
                 "rel_rms_err_max": 1e-4})
    best = {b["target"]: b["row"] for b in bench.sweep_best(rows, targets=(1e-2, 1e-4, 1e-6))}
    assert best[1e-2]["order"] == 2 and best[1e-2]["oversampling"] == 1
    assert best[1e-4]["oversampling"] == 2 and best[1e-4]["ms_per_map"] == 3.5
    assert best[1e-6] is None


def test_sweep_fastest_settings_per_potential_band_limit(bench):
    """Rows of a potential with its own band limit form their own table rows."""
    rows = [{"lmax": 8, "lmax_phi": lp, "oversampling": 2, "order": 3, "form": "fp32", "ms_per_map": t,
             "rel_rms_err_max": 1e-3} for lp, t in ((8, 1.0), (16, 2.0))]
    best = bench.sweep_best(rows, targets=(1e-2,))
    assert [(b["lmax_phi"], b["row"]["ms_per_map"]) for b in best] == [(8, 1.0), (16, 2.0)]


def test_spectra_helpers_match_the_oracle(bench, oracle):
    """The benchmark's C_l, bins and l* rule against the oracle's (step 9)."""
    import numpy as np

    rng = np.random.default_rng(8)
    lmax = 160
    alm = rng.standard_normal((lmax + 1) * (lmax + 2) // 2) + 1j * rng.standard_normal((lmax + 1) * (lmax + 2) // 2)
    np.testing.assert_allclose(bench.spectra_cl(alm, lmax), oracle.cl_from_alm(alm, lmax), rtol=1e-14)
    cl = rng.random(lmax + 1)
    c1, m1 = bench.spectra_bins(cl)
    c2, m2 = oracle.bin_cl(cl)
    np.testing.assert_array_equal(c1, c2)
    np.testing.assert_allclose(m1, m2, rtol=1e-15)
    for _ in range(20):
        e = rng.normal(0.004, 0.003, size=(4, len(c1))) * np.linspace(0.5, 3.0, len(c1))
        assert bench.spectra_ell_star(c1, e) == oracle.ell_star(c1, e)
