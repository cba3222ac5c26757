"""GPU parity of target-rank estimation (Sec. 3.6): the library's loop over
its FP64 seed solver, through the C ABI, against the FP64 oracle's loop on the
same matrix and the same row / column orders.  The ranks are integers decided
in FP64 on both sides and must agree exactly, round by round."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_util import REL_TOL, dev_i64, dev_matrix, host_matrix, relF, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1108_5359_amd.rpca as R
    return R


@pytest.fixture(scope="module")
def ctx(R):
    c = R.Context(0)
    yield c
    c.close()


def _orders(m, n, seed):
    rng = np.random.default_rng(seed)
    return rng.permutation(m).astype(np.int64), rng.permutation(n).astype(np.int64)


CASES = {
    # name: (matrix factory, r0, order seed)
    "rank12_r0_2": (lambda: synth.lowrank_plus_sparse(1000, 1000, 12, factor_std=np.sqrt(1e-3),
                                                      sparsity=0.05, values="pm1", seed=7).M, 2, 4),
    "rank12_r0_6": (lambda: synth.lowrank_plus_sparse(1000, 1000, 12, factor_std=np.sqrt(1e-3),
                                                      sparsity=0.05, values="pm1", seed=7).M, 6, 4),
    "c1_draw4": (lambda: synth.config_problem("c1", seed=4).M, 10, 4),
    "c1_draw2_r0_3": (lambda: synth.config_problem("c1", seed=2).M, 3, 11),
    "gaussian_full_rank": (lambda: np.asfortranarray(
        np.random.default_rng(1).standard_normal((400, 300)).astype(np.float32)), 2, 2),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_estimate_rank_matches_oracle(R, ctx, name):
    make, r0, oseed = CASES[name]
    M = make()
    m, n = M.shape
    ro, co = _orders(m, n, oseed)
    ref = oracle.estimate_rank(M, r0, ro, co)
    say(f"estimate_rank {name}: oracle ranks={ref.ranks} sizes={ref.sizes} "
        f"accepted={ref.accepted} cv={ref.cv_rank}")
    st, info = R.rpca_estimate_rank(ctx, dev_matrix(M), m, n, m, r0, R.rpca_opts_default(), ro, co,
                                    True)
    k = info.rounds
    got_ranks = list(info.ranks[:k])
    got_sizes = [(info.ps[i], info.qs[i]) for i in range(k)]
    say(f"  library: status={R.rpca_status_string(st)} ranks={got_ranks} sizes={got_sizes} "
        f"accepted={info.accepted} cv={info.cv_rank}")
    assert got_ranks == ref.ranks and got_sizes == ref.sizes
    assert bool(info.accepted) == ref.accepted and info.r_est == ref.r_est
    assert info.cv_rank == ref.cv_rank
    assert (info.p, info.q) == (ref.p, ref.q)
    if ref.accepted and ref.cv_rank in (-1, ref.r_est):
        assert st == R.RPCA_OK
    else:
        assert st == R.RPCA_WARN_RANK


def test_accepted_seed_completes_like_the_oracle(R, ctx):
    # The accepted block and rank feed Algorithm 2 unchanged: the factored
    # solve on the block's sorted indices matches the oracle's solve on them.
    import torch
    pr = synth.lowrank_plus_sparse(1000, 1000, 12, factor_std=np.sqrt(1e-3), sparsity=0.05,
                                   values="pm1", seed=7)
    ro, co = _orders(1000, 1000, 4)
    st, info = R.rpca_estimate_rank(ctx, dev_matrix(pr.M), 1000, 1000, 1000, 2,
                                    R.rpca_opts_default(), ro, co, False)
    assert st == R.RPCA_OK and info.r_est == 12
    I, J = np.sort(ro[:info.p]), np.sort(co[:info.q])
    ref = oracle.solve(pr.M, info.r_est, I, J)
    assert oracle.relerr(ref.L, pr.L0()) <= 1e-6
    Md = dev_matrix(pr.M)
    r, p, q = info.r_est, info.p, info.q
    U = torch.zeros((r, p), dtype=torch.float64, device="cuda")
    sg = torch.zeros(r, dtype=torch.float64, device="cuda")
    V = torch.zeros((r, q), dtype=torch.float64, device="cuda")
    Qt = torch.zeros(r * (1000 - q), dtype=torch.float32, device="cuda")
    Pt = torch.zeros(r * (1000 - p), dtype=torch.float32, device="cuda")
    dI, dJ = dev_i64(I), dev_i64(J)
    st, fi = R.rpca_solve_factored(ctx, Md, 1000, 1000, 1000, r, R.rpca_opts_default(), dI, p, dJ, q,
                                   U, sg, V, Qt, None, Pt, None)
    assert st == R.RPCA_OK and fi.r_used == r
    L = torch.empty_like(Md)
    S = torch.empty_like(Md)
    R.rpca_reconstruct(ctx, Md, 1000, 1000, 1000, dI, p, dJ, q, U, sg, V, r, Qt, Pt, L, 1000, S, 1000)
    torch.cuda.synchronize()
    assert relF(host_matrix(L, 1000), ref.L) <= REL_TOL
    assert relF(host_matrix(S, 1000), ref.S) <= REL_TOL


def test_estimate_rank_argument_errors(R, ctx):
    M = synth.config_problem("c1", seed=1).M
    Md = dev_matrix(M)
    ro, co = _orders(1000, 1000, 1)
    bad = ro.copy()
    bad[5] = bad[6]                                   # not a permutation
    o = R.rpca_opts_default()
    for args in [(bad, co, 10), (ro, co, 0), (ro, co, 51)]:    # r0 = 51: block beyond m / 2
        with pytest.raises(R.RpcaError) as e:
            R.rpca_estimate_rank(ctx, Md, 1000, 1000, 1000, args[2], o, args[0], args[1], True)
        assert e.value.status == R.RPCA_ERR_ARG
