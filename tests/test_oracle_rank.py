"""Pins for the FP64 reference of target-rank estimation (Sec. 3.6, eqs.
rank_test and rank_test1): the estimate must be the true rank of synthetic
low-rank data, reached by growing blocks, and the loop must stop on data that
are not low rank."""
import numpy as np
import pytest

import oracle
import synth


def _orders(m, n, seed):
    rng = np.random.default_rng(seed)
    return rng.permutation(m), rng.permutation(n)


def test_exact_low_rank_is_accepted_at_once():
    # No corruption: the seed block of a rank-5 matrix has rank 5 (PCP keeps
    # an incoherent low-rank block whole), so a guess of 5 passes eq. rank_test
    # in one round.
    pr = synth.lowrank_plus_sparse(400, 300, 5, factor_std=0.05, sparsity=0.0, seed=3)
    ro, co = _orders(400, 300, 3)
    e = oracle.estimate_rank(pr.M, 5, ro, co)
    assert e.accepted and e.r_est == 5 and e.ranks == [5] and e.sizes == [(50, 50)]
    assert e.cv_rank == 5


@pytest.mark.parametrize("r0", [2, 6])
def test_low_guess_grows_to_the_true_rank(r0):
    # Rank 12 with 5% +-1 corruptions: a low guess gives a block too small for
    # the data's rank, the loop grows it by eq. rank_test and ends at 12.
    pr = synth.lowrank_plus_sparse(1000, 1000, 12, factor_std=np.sqrt(1e-3), sparsity=0.05,
                                   values="pm1", seed=7)
    ro, co = _orders(1000, 1000, 4)
    e = oracle.estimate_rank(pr.M, r0, ro, co)
    assert e.accepted and e.r_est == 12
    assert len(e.ranks) >= 2 and e.sizes[0] == (10 * r0, 10 * r0)
    # every grown block is os * (rank found in the round before)
    for k in range(1, len(e.sizes)):
        assert e.sizes[k] == (10 * e.ranks[k - 1], 10 * e.ranks[k - 1])
        assert e.ranks[k - 1] * 10 > e.sizes[k - 1][0]      # it grew because rank_test failed
    assert e.p >= 10 * e.r_est and e.q >= 10 * e.r_est       # eq. rank_test on the last one
    assert e.cv_rank == 12


def test_full_rank_data_stop_at_half_size():
    # i.i.d. Gaussian entries: every block is full rank, so the block would
    # have to grow beyond half of M (eq. rank_test1) and the loop stops.
    G = np.asfortranarray(np.random.default_rng(1).standard_normal((400, 400)).astype(np.float32))
    ro, co = _orders(400, 400, 2)
    e = oracle.estimate_rank(G, 2, ro, co)
    assert not e.accepted and e.cv_rank == -1
    p_next = 10 * e.ranks[-1]
    assert p_next > 200                                     # the next block exceeds m / 2
    assert all(p <= 200 and q <= 200 for p, q in e.sizes)   # no block solved beyond it


def test_blocks_are_nested_prefixes():
    # The blocks are prefixes of the orders, taken as sets: reversing the
    # order inside the first block's prefix changes nothing.
    pr = synth.lowrank_plus_sparse(600, 600, 4, factor_std=np.sqrt(1 / 600), sparsity=0.05,
                                   values="pm1", seed=9)
    ro, co = _orders(600, 600, 5)
    e = oracle.estimate_rank(pr.M, 4, ro, co, cross_validate=False)
    assert e.accepted and e.r_est == 4
    ro2 = ro.copy()
    ro2[:40] = ro2[:40][::-1]                                # same set, other order
    e2 = oracle.estimate_rank(pr.M, 4, ro2, co, cross_validate=False)
    assert e2.ranks == e.ranks and e2.sizes == e.sizes
