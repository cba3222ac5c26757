"""The two FP32 forms of the l1 filtering kernel (opts.filter_form):

* tile form (1): one wave per 16 regressions, the whole of each regression
  in that wave;
* split form (2): one workgroup of four waves per 16 regressions, each wave a
  quarter of the 16-element tiles, the partial w = A^T g summed through LDS
  and the stopping test of a step taken one step later.

Both compute Algorithm 1 on the same inputs, so each is held to the oracle's
tolerance on its own (relative Frobenius 1e-5 through the blocks U Q~ and
P~^T V^T, and on L and S); the iteration counts, which FP32 rounding decides
near the stopping threshold, are compared through their means.  Cases: the
oracle-sized workload, every split tile class from p = 64 (one tile per wave) to p = 300 (five),
ragged shapes, zero regressions, the iteration cap and a few steps against
the oracle's same steps, repeated regressions, both sides in one launch
against each side alone (bitwise), a chunked launch (device range) of the
overlapped form.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_util import REL_TOL, dev_f64_colmajor, dev_i64, dev_matrix, host_matrix, relF, say
from test_gpu_parity import (R, _filter_cols_gpu, _filter_rows_gpu, _solve_gpu, case,  # noqa: F401
                             ctx, small_case)

pytestmark = pytest.mark.gpu

FORMS = (1, 2)


def _opts(R, form, **kw):
    return R.rpca_opts_default(filter_form=form, **kw)


@pytest.mark.parametrize("seed", [1, 2])
def test_both_forms_match_the_oracle_c1(R, ctx, seed):
    pr, r, I, J, res = case("c1", seed)
    Jc, Ic = oracle.complement(J, pr.n), oracle.complement(I, pr.m)
    k = res.U.shape[1]
    its = {}
    for form in FORMS:
        say(f"forms c1 seed={seed} form={form}")
        st, Qt, itc = _filter_cols_gpu(R, ctx, pr, I, Jc, res.U, k, opts=_opts(R, form))
        assert st == R.RPCA_OK and np.isfinite(Qt).all()
        assert relF(res.U @ Qt, res.U @ res.Qt) <= REL_TOL
        st, Pt, itr = _filter_rows_gpu(R, ctx, pr, J, Ic, res.V, k, opts=_opts(R, form))
        assert st == R.RPCA_OK
        assert relF(Pt.T @ res.V.T, res.Pt.T @ res.V.T) <= REL_TOL
        assert (itc > 0).all() and (itr > 0).all()
        assert abs(itc.mean() - res.col_iters.mean()) <= 0.1 * res.col_iters.mean()
        its[form] = np.concatenate([itc, itr])
    # FP32 rounding near the stopping threshold decides single counts (in
    # either form: the two differ on about a quarter of the regressions, by up
    # to a few tens of steps), so only the means are held together
    assert abs(its[1].mean() - its[2].mean()) <= 0.05 * its[1].mean()


# p = 64 .. 300: PT = 4 (one element tile per wave), 5, 7, 10, 13, 16, 19 (five
# on the heaviest wave); r up to 30 (two rank tiles); padded leading dimension
@pytest.mark.parametrize("m,n,r,ld_pad", [
    (700, 640, 6, 0),       # p = 60 -> PT = 4
    (517, 333, 7, 5),       # p = 70 -> PT = 5, ld = m + 5
    (800, 900, 11, 0),      # p = 110 -> PT = 7
    (450, 460, 13, 4),      # p = 130 -> PT = 10
    (1300, 1100, 20, 0),    # p = 200 -> PT = 13 (the benchmark's class)
    (2000, 1500, 25, 0),    # p = 250 -> PT = 16, two rank tiles
    (2100, 1900, 30, 3),    # p = 300 -> PT = 19
])
def test_split_form_solve_ragged(R, ctx, m, n, r, ld_pad):
    pr, I, J, res = small_case(m, n, r, 0.05, 7 + r)
    out = {}
    for form in FORMS:
        say(f"forms solve m={m} n={n} r={r} ld={m + ld_pad} form={form}")
        st, info, L, S = _solve_gpu(R, ctx, pr, r, I, J, ld=m + ld_pad, opts=_opts(R, form))
        assert st >= 0, ctx.last_error()
        Lh, Sh = host_matrix(L, m), host_matrix(S, m)
        assert np.isfinite(Lh).all() and np.isfinite(Sh).all()
        assert relF(Lh, res.L) <= REL_TOL and relF(Sh, res.S) <= REL_TOL
        assert info.filt_not_converged == 0
        out[form] = info.filt_iters_total
    # the mean iteration counts of the two forms agree (single counts are
    # decided by rounding near the stopping threshold)
    assert abs(out[1] - out[2]) <= 0.05 * out[1]


def test_split_form_zero_regressions_cap_and_repeats(R, ctx):
    pr, r, I, J, res = case("c1", 1)
    Jc = oracle.complement(J, pr.n)
    M0 = pr.M.copy(order="F")
    M0[np.ix_(I, Jc[:5])] = 0.0          # five all-zero regressions
    pr0 = synth.Problem(M=M0, A0=pr.A0, B0=pr.B0, support=None, m=pr.m, n=pr.n, r=r, seed=0)
    say("split form: zero columns")
    st, Qt, it = _filter_cols_gpu(R, ctx, pr0, I, Jc, res.U, 10, opts=_opts(R, 2))
    assert st == R.RPCA_OK
    assert (it[:5] == 0).all() and not Qt[:, :5].any()
    for cap in (1, 3, 9):
        # the stopping test of the last step is still taken: the count is
        # -cap (not converged) for every regression, and z after cap steps
        # is the oracle's after cap steps (a refresh falls inside cap = 9)
        say(f"split form: max_iter={cap}")
        st, Qt, it = _filter_cols_gpu(R, ctx, pr, I, Jc[:37], res.U, 10,
                                      opts=_opts(R, 2, filt_max_iter=cap))
        Zo, Ko = oracle.alg1_batch(pr.M[np.ix_(I, Jc[:37])].astype(np.float64), res.U,
                                   oracle.Alg1Params(max_iter=cap))
        assert np.array_equal(it, Ko), (it, Ko)
        assert relF(res.U @ Qt, res.U @ Zo) <= REL_TOL
    cols = np.array([999, 3, 3, 500, 17] * 7)      # repeats, 35 regressions over 3 tiles
    st, Qt, it = _filter_cols_gpu(R, ctx, pr, I, cols, res.U, 10, opts=_opts(R, 2))
    Zo, Ko = oracle.alg1_batch(pr.M[np.ix_(I, cols)].astype(np.float64), res.U)
    assert relF(res.U @ Qt, res.U @ Zo) <= REL_TOL
    for a in range(5):
        for b in range(a + 5, 35, 5):
            assert np.array_equal(Qt[:, a], Qt[:, b])     # same regression, same bits


@pytest.mark.parametrize("form", FORMS)
def test_fused_sides_equal_separate_launches(R, ctx, form):
    # One launch of both sides (the row regressions take the first
    # workgroups) gives every regression the bits and the step count that
    # its own side's launch gives it.
    import torch
    pr, r, I, J, res = case("c1", 1)
    k = res.U.shape[1]
    m, n = pr.m, pr.n
    Ic, Jc = oracle.complement(I, m), oracle.complement(J, n)
    Md = dev_matrix(pr.M)
    L = torch.empty_like(Md)
    S = torch.empty_like(Md)
    Qt = torch.zeros((len(Jc), k), device="cuda")
    Pt = torch.zeros((len(Ic), k), device="cuda")
    kc = torch.zeros(len(Jc), dtype=torch.int32, device="cuda")
    kr = torch.zeros(len(Ic), dtype=torch.int32, device="cuda")
    say(f"fused sides, form {form}")
    st = R.rpca_filter_complete(ctx, Md, m, n, m, dev_i64(I), len(I), dev_i64(J), len(J), dev_i64(Jc),
                                dev_i64(Ic), dev_f64_colmajor(res.U),
                                torch.as_tensor(res.sigma).cuda(), dev_f64_colmajor(res.V), k,
                                _opts(R, form), Qt, kc, Pt, kr, L, m, S, m)
    torch.cuda.synchronize()
    assert st == R.RPCA_OK, ctx.last_error()
    say(f"separate sides, form {form}")
    st_c, Qs, ks_c = _filter_cols_gpu(R, ctx, pr, I, Jc, res.U, k, _opts(R, form))
    st_r, Ps, ks_r = _filter_rows_gpu(R, ctx, pr, J, Ic, res.V, k, _opts(R, form))
    assert st_c == R.RPCA_OK and st_r == R.RPCA_OK
    assert np.array_equal(Qt.double().cpu().numpy().T, Qs)
    assert np.array_equal(Pt.double().cpu().numpy().T, Ps)
    assert np.array_equal(kc.cpu().numpy(), ks_c) and np.array_equal(kr.cpu().numpy(), ks_r)


@pytest.mark.parametrize("chunks", [3, 16])
def test_split_form_in_the_overlapped_form(R, ctx, chunks):
    # column slabs read their regression range from the device
    import torch
    pr, r, I, J, res = case("c1", 2)
    k = res.U.shape[1]
    m, n = pr.m, pr.n
    Ic, Jc = oracle.complement(I, m), oracle.complement(J, n)
    outs = []
    for ov in (0, chunks):
        Md = dev_matrix(pr.M)
        L = torch.empty_like(Md)
        S = torch.empty_like(Md)
        Qt = torch.zeros((len(Jc), k), device="cuda")
        Pt = torch.zeros((len(Ic), k), device="cuda")
        kc = torch.zeros(len(Jc), dtype=torch.int32, device="cuda")
        kr = torch.zeros(len(Ic), dtype=torch.int32, device="cuda")
        say(f"split form overlapped chunks={ov}")
        R.rpca_filter_complete(ctx, Md, m, n, m, dev_i64(I), len(I), dev_i64(J), len(J), dev_i64(Jc),
                               dev_i64(Ic), dev_f64_colmajor(res.U),
                               torch.as_tensor(res.sigma).cuda(), dev_f64_colmajor(res.V), k,
                               _opts(R, 2, overlap_chunks=ov), Qt, kc, Pt, kr, L, m, S, m)
        torch.cuda.synchronize()
        outs.append((host_matrix(L, m), host_matrix(S, m), kc.cpu().numpy(), kr.cpu().numpy()))
    (L0, S0, kc0, kr0), (L1, S1, kc1, kr1) = outs
    assert np.array_equal(L0, L1) and np.array_equal(S0, S1)
    assert np.array_equal(kc0, kc1) and np.array_equal(kr0, kr1)
    assert relF(L1, res.L) <= REL_TOL and relF(S1, res.S) <= REL_TOL


def test_filter_form_option_is_checked(R, ctx):
    pr, r, I, J, res = case("c1", 1)
    import torch
    Md = dev_matrix(pr.M)
    L = torch.empty_like(Md)
    S = torch.empty_like(Md)
    with pytest.raises(R.RpcaError) as e:
        R.rpca_solve(ctx, Md, pr.m, pr.n, pr.m, r, R.rpca_opts_default(filter_form=3),
                     dev_i64(I), dev_i64(J), L, pr.m, S, pr.m)
    assert e.value.status == R.RPCA_ERR_ARG
