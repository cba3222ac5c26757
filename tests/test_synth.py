"""The seeded input generator: the device (torch) version of the counter hash
gives the same bits as the numpy version, and the generators honour the
workload recipe (support rate, value law, factor scale)."""
import numpy as np
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
