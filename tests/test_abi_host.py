"""Host-side checks of librpca that need no GPU: the shared library loads and
exports every entry point that include/rpca.h declares, the defaults equal
the oracle's constants, the host-only index sampler behaves, and context
creation fails cleanly without a device."""
import ctypes
import pathlib
import re

import numpy as np
import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
LIB = ROOT / "paper_1108_5359_amd" / "librpca.so"


def _declared():
    text = (ROOT / "include" / "rpca.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rpca_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def R():
    if not LIB.exists():
        pytest.fail("librpca.so is not built (run __graft_entry__.build())")
    import paper_1108_5359_amd.rpca as R
    return R


def test_every_declared_symbol_is_exported(R):
    names = _declared()
    assert {"rpca_seed", "rpca_filter_cols", "rpca_filter_rows", "rpca_reconstruct",
            "rpca_solve"} <= set(names)
    lib = ctypes.CDLL(str(LIB))
    for name in names:
        assert hasattr(lib, name), name


def test_defaults_equal_the_oracle_constants(R):
    import oracle
    o = R.rpca_opts_default()
    a, s = oracle.Alg1Params(), oracle.SeedParams()
    assert (o.filt_eps, o.filt_rho, o.filt_beta0_scale, o.filt_beta_max_scale, o.filt_max_iter) == \
        (a.eps, a.rho, a.beta0_scale, a.beta_max_scale, a.max_iter)
    assert (o.seed_tol, o.seed_rho, o.seed_mu0_scale, o.seed_mu_max_scale, o.seed_max_iter,
            o.seed_rank_floor) == (s.tol, s.rho, s.mu0_scale, s.mu_max_scale, s.max_iter,
                                   s.rank_floor)
    assert o.os_r == o.os_c == 10 and o.seed_lambda == 0.0


def test_sampler_properties(R):
    for seed in range(20):
        rows, cols = R.rpca_sample_indices(1000, 800, 100, 90, seed)
        assert rows.size == 100 and cols.size == 90
        assert (np.diff(rows) > 0).all() and (np.diff(cols) > 0).all()
        assert rows.min() >= 0 and rows.max() < 1000 and cols.max() < 800
    a = R.rpca_sample_indices(1000, 800, 100, 90, 7)
    b = R.rpca_sample_indices(1000, 800, 100, 90, 7)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    rows, _ = R.rpca_sample_indices(10, 10, 10, 10, 3)
    assert np.array_equal(rows, np.arange(10))          # p = m takes everything


def test_sampler_is_uniform(R):
    # Each of 50 rows is drawn with probability 10/50: chi-square over 4000 draws.
    counts = np.zeros(50)
    draws = 4000
    for seed in range(draws):
        rows, _ = R.rpca_sample_indices(50, 5, 10, 1, seed)
        counts[rows] += 1
    expected = draws * 10 / 50
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 100.0          # 49 dof: mean 49, P(chi2 > 100) < 1e-4


def test_sampler_rejects_bad_sizes(R):
    with pytest.raises(R.RpcaError):
        R.rpca_sample_indices(10, 10, 11, 1, 0)
    with pytest.raises(R.RpcaError):
        R.rpca_sample_indices(10, 10, 0, 1, 0)


def test_status_strings(R):
    assert R.rpca_status_string(R.RPCA_ERR_ARG) == "RPCA_ERR_ARG"
    assert R.rpca_status_string(R.RPCA_WARN_RANK) == "RPCA_WARN_RANK"


def test_context_without_device_fails_cleanly(R):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(R.RpcaError) as e:
        R.Context(0)
    assert e.value.status == R.RPCA_ERR_DEVICE


def test_committed_tuning_applies_to_the_library(R):
    # The autotuner's results file: every tuned field is a field of
    # rpca_batch_tuning, each value lies in the grid the tuner searched, and
    # the tuned choice was at least as fast as the defaults it was timed against.
    import json
    from paper_1108_5359_amd import autotune
    tuned = autotune.load()
    assert tuned, "tuning_mi355x.json holds no batch_tuning"
    t = R.rpca_batch_tuning_default(**tuned)
    for k, v in tuned.items():
        assert getattr(t, k) == v
    assert (tuned["lane_split2_p"], tuned["lane_split4_p"]) in [tuple(x) for x in autotune.GRID["lane_split"]]
    for k in ("filter_waves_per_cu", "order", "recon_cols_per_wave", "recon_waves_per_cu"):
        assert tuned[k] in autotune.GRID[k], k
    doc = json.loads(autotune.DEFAULT_OUT.read_text())
    assert doc["best_ms"] <= doc["default_ms"]
