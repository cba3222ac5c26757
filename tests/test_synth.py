"""The seeded input generator: the device (torch) version of the counter hash
gives the same bits as the numpy version, and the generators honour the
workload recipe (support rate, value law, factor scale)."""
import numpy as np
import pytest
import torch

import synth


def test_torch_hash_equals_numpy_hash():
    idx = np.array([0, 1, 2, 3, 12345, 2**40 + 17, 2**62 + 5, 99_999_999_999], dtype=np.int64)
    for seed, stream in [(1, 1), (7, 2), (123456789, 1)]:
        a = synth.hash_uniform(seed, stream, idx.astype(np.uint64))
        b = synth.hash_uniform_torch(seed, stream, torch.from_numpy(idx)).numpy()
        assert np.array_equal(a, b)


def test_device_generator_matches_host_generator_on_cpu():
    # Same factors, same support and values; M can differ only by the last
    # bit of a few entries (FP64 dot products summed in another order).
    kw = dict(factor_std=0.05, sparsity=0.1, values="unif11", seed=5)
    host = synth.lowrank_plus_sparse(300, 200, 4, exact_count=False, **kw)
    Mt, A0, B0 = synth.lowrank_plus_sparse_device(300, 200, 4, device="cpu", block_cols=64, **kw)
    assert np.array_equal(A0, host.A0) and np.array_equal(B0, host.B0)
    Md = Mt.numpy().T
    diff = np.abs(Md.astype(np.float64) - host.M.astype(np.float64))
    assert (diff <= np.spacing(np.abs(host.M)).astype(np.float64)).all()
    assert (diff > 0).mean() < 1e-3


def test_support_rate_and_values():
    pr = synth.lowrank_plus_sparse(400, 300, 3, factor_std=1e-3, sparsity=0.1, values="pm1", seed=2)
    rate = pr.support.mean()
    assert abs(rate - 0.1) < 4 * np.sqrt(0.1 * 0.9 / pr.support.size)
    S = pr.M.astype(np.float64) - pr.L0()
    assert np.allclose(np.abs(S[pr.support]), 1.0, atol=1e-2)
    assert np.abs(S[~pr.support]).max() < 1e-6
    pr2 = synth.lowrank_plus_sparse(200, 200, 2, factor_std=1e-3, sparsity=0.05, values="pm1",
                                    seed=3, exact_count=True)
    assert pr2.support.sum() == 2000


def test_union_fraction_is_exact():
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(20):
        m, n = int(rng.integers(5, 60)), int(rng.integers(5, 60))
        rects = []
        for _ in range(int(rng.integers(0, 6))):
            i0 = int(rng.integers(0, m)); j0 = int(rng.integers(0, n))
            rects.append((i0, int(rng.integers(i0 + 1, m + 1)), j0, int(rng.integers(j0 + 1, n + 1))))
        mask = np.zeros((m, n), dtype=bool)
        for i0, i1, j0, j1 in rects:
            mask[i0:i1, j0:j1] = True
        assert synth.union_fraction(rects, m, n) == pytest.approx(mask.mean(), abs=1e-15)


def test_batch_specs_follow_the_recipe():
    specs = synth.batch_specs(40, 2, m=(300, 2000), n=(100, 400), r=(1, 8), rho=(0.05, 0.15))
    assert [s.seed for s in specs] == sorted(set(s.seed for s in specs))   # distinct
    for s in specs:
        assert 300 <= s.m <= 2000 and 100 <= s.n <= 400 and 1 <= s.r <= 8
        assert 0.05 <= s.rho <= 0.15
        f = synth.union_fraction(s.rects, s.m, s.n)
        assert f >= s.rho
        # the last rectangle is the one that crossed rho
        assert synth.union_fraction(s.rects[:-1], s.m, s.n) < s.rho
        for i0, i1, j0, j1 in s.rects:
            assert 0 <= i0 < i1 <= s.m and 0 <= j0 < j1 <= s.n
            assert max(1, -(-s.m // 50)) <= i1 - i0 <= max(1, s.m // 10)
            assert max(1, -(-s.n // 20)) <= j1 - j0 <= max(1, s.n // 5)
    assert synth.batch_specs(3, 2, m=(300, 2000), n=(100, 400))[0] == \
        synth.batch_specs(3, 2, m=(300, 2000), n=(100, 400))[0]


def test_batch_job_host_and_device_agree():
    import torch
    for s in synth.batch_specs(3, 4, m=(200, 700), n=(100, 160)):
        P = synth.batch_job_host(s)
        Mt, A0, B0 = synth.batch_job_device(s, device="cpu")
        assert np.array_equal(Mt.numpy().T, P.M)
        assert P.support.mean() >= s.rho
        S0 = P.M.astype(np.float64) - (A0 @ B0.T)
        assert np.all(np.abs(S0[~P.support]) < 1e-6)
        assert np.all((S0[P.support] > -1e-6) & (S0[P.support] < 1 + 1e-6))   # U[0, 1] values


def test_checkerboard_is_rank_two_plus_impulsive_noise():
    pr = synth.checkerboard(300, 240, 30, 0.10, seed=4)
    C = pr.L0()
    assert np.linalg.matrix_rank(C) == 2
    assert set(np.unique(C)) == {0.0, 1.0}
    assert C[0, 0] == 0 and C[0, 30] == 1 and C[30, 30] == 0
    S0 = pr.M.astype(np.float64) - C
    assert np.array_equal(S0 != 0, pr.support)
    hit_rate = (pr.M != C.astype(np.float32)).mean()
    assert 0.03 < hit_rate < 0.07          # half of the 10% hits change the pixel
    assert set(np.unique(pr.M)) == {0.0, 1.0}
