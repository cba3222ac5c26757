"""GPU parity: the HIP library, called through its C ABI, against the FP64
oracle on the same seeded inputs.

Tolerance (stated for this method): relative Frobenius error <= 1e-5 on L and
S; the filter steps are compared through the blocks they define
(``U Q~ = L^c`` and ``P~^T V^T = L^r``) with the same bound; the support of S
must agree away from the threshold.  Integer outputs that FP arithmetic
decides (iteration counts) are compared statistically only.
"""
from __future__ import annotations

import functools

import numpy as np
import pytest

import oracle
import synth
from gpu_util import (REL_TOL, dev_f64_colmajor, dev_i64, dev_matrix, host_matrix, relF, say,
                      support_mismatch)

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


@functools.lru_cache(maxsize=None)
def case(name: str, seed: int, **kw):
    pr = synth.config_problem(name, seed=seed, **kw)
    r = synth.CONFIGS[name]["r"]
    I, J = synth.seed_indices(pr.m, pr.n, 10 * r, 10 * r, seed=seed)
    res = oracle.solve(pr.M, r, I, J, assemble=(pr.m * pr.n <= 4_000_000))
    return pr, r, I, J, res


@functools.lru_cache(maxsize=None)
def small_case(m, n, r, sparsity, seed):
    pr = synth.lowrank_plus_sparse(m, n, r, factor_std=np.sqrt(1.0 / max(m, n)),
                                   sparsity=sparsity, values="pm1", seed=seed)
    I, J = synth.seed_indices(m, n, 10 * r, 10 * r, seed=seed)
    res = oracle.solve(pr.M, r, I, J)
    return pr, I, J, res


def _filter_cols_gpu(R, ctx, pr, I, cols, U, r, opts=None, ld=None):
    import torch
    opts = opts or R.rpca_opts_default()
    ld = ld or pr.m
    Md = dev_matrix(pr.M, ld)
    Qt = torch.full((len(cols), r), float("nan"), dtype=torch.float32, device="cuda")
    it = torch.zeros(len(cols), dtype=torch.int32, device="cuda")
    st = R.rpca_filter_cols(ctx, Md, pr.m, pr.n, ld, dev_i64(I), len(I), dev_i64(cols), len(cols),
                            dev_f64_colmajor(U), r, opts, Qt, it)
    torch.cuda.synchronize()
    return st, Qt.double().cpu().numpy().T, it.cpu().numpy()


def _filter_rows_gpu(R, ctx, pr, J, rows, V, r, opts=None, ld=None):
    import torch
    opts = opts or R.rpca_opts_default()
    ld = ld or pr.m
    Md = dev_matrix(pr.M, ld)
    Pt = torch.full((len(rows), r), float("nan"), dtype=torch.float32, device="cuda")
    it = torch.zeros(len(rows), dtype=torch.int32, device="cuda")
    st = R.rpca_filter_rows(ctx, Md, pr.m, pr.n, ld, dev_i64(J), len(J), dev_i64(rows), len(rows),
                            dev_f64_colmajor(V), r, opts, Pt, it)
    torch.cuda.synchronize()
    return st, Pt.double().cpu().numpy().T, it.cpu().numpy()


def _solve_gpu(R, ctx, pr, r, I=None, J=None, ld=None, opts=None):
    import torch
    opts = opts or R.rpca_opts_default()
    ld = ld or pr.m
    Md = dev_matrix(pr.M, ld)
    L = torch.full((pr.n, ld), float("nan"), dtype=torch.float32, device="cuda")
    S = torch.full((pr.n, ld), float("nan"), dtype=torch.float32, device="cuda")
    st, info = R.rpca_solve(ctx, Md, pr.m, pr.n, ld, r, opts,
                            None if I is None else dev_i64(I), None if J is None else dev_i64(J),
                            L, ld, S, ld)
    torch.cuda.synchronize()
    return st, info, L, S


# ----------------------------------------------------------------- steps 3, 4
@pytest.mark.parametrize("seed", [1, 2])
def test_filter_cols_matches_oracle_c1(R, ctx, seed):
    pr, r, I, J, res = case("c1", seed)
    Jc = oracle.complement(J, pr.n)
    say(f"filter_cols c1 seed={seed} p={len(I)} nc={len(Jc)} r={res.U.shape[1]}")
    st, Qt, it = _filter_cols_gpu(R, ctx, pr, I, Jc, res.U, res.U.shape[1])
    assert st == R.RPCA_OK
    assert np.isfinite(Qt).all()
    assert relF(res.U @ Qt, res.U @ res.Qt) <= REL_TOL
    assert (it > 0).all()
    assert abs(it.mean() - res.col_iters.mean()) <= 0.1 * res.col_iters.mean()


@pytest.mark.parametrize("seed", [1, 2])
def test_filter_rows_matches_oracle_c1(R, ctx, seed):
    pr, r, I, J, res = case("c1", seed)
    Ic = oracle.complement(I, pr.m)
    say(f"filter_rows c1 seed={seed} q={len(J)} nr={len(Ic)}")
    st, Pt, it = _filter_rows_gpu(R, ctx, pr, J, Ic, res.V, res.V.shape[1])
    assert st == R.RPCA_OK
    assert relF(Pt.T @ res.V.T, res.Pt.T @ res.V.T) <= REL_TOL
    assert (it > 0).all()
    assert abs(it.mean() - res.row_iters.mean()) <= 0.1 * res.row_iters.mean()


# ----------------------------------------------------------------- step 5
def test_reconstruct_matches_oracle_c1(R, ctx):
    import torch
    pr, r, I, J, res = case("c1", 1)
    say("reconstruct c1 seed=1")
    k = res.U.shape[1]
    Md = dev_matrix(pr.M)
    L = torch.full((pr.n, pr.m), float("nan"), dtype=torch.float32, device="cuda")
    S = torch.full_like(L, float("nan"))
    Qt = torch.as_tensor(np.ascontiguousarray(res.Qt.T, dtype=np.float32)).cuda()
    Pt = torch.as_tensor(np.ascontiguousarray(res.Pt.T, dtype=np.float32)).cuda()
    st = R.rpca_reconstruct(ctx, Md, pr.m, pr.n, pr.m, dev_i64(I), len(I), dev_i64(J), len(J),
                            dev_f64_colmajor(res.U), torch.as_tensor(res.sigma).cuda(),
                            dev_f64_colmajor(res.V), k, Qt, Pt, L, pr.m, S, pr.m)
    torch.cuda.synchronize()
    assert st == R.RPCA_OK
    Lh, Sh = host_matrix(L, pr.m), host_matrix(S, pr.m)
    # the oracle's L from FP32-rounded Q~, P~ (what the kernel receives)
    Lref, Sref = oracle.complete(pr.M, I, J, res.U, res.sigma, res.V,
                                 res.Qt.astype(np.float32).astype(np.float64),
                                 res.Pt.astype(np.float32).astype(np.float64))
    assert relF(Lh, Lref) <= 1e-6
    assert relF(Sh, Sref) <= 1e-6
    # S is M - L computed in FP32 from the same L
    assert np.array_equal(Sh, (pr.M.astype(np.float32) - Lh.astype(np.float32)).astype(np.float64))


@pytest.mark.parametrize("m,n,r,p,q,ld_pad", [
    (1500, 1100, 36, 360, 360, 0),     # R4 = 36: contiguous column ranges per wave
    (1300, 1700, 50, 500, 500, 4),     # R4 = 52, ld % 4 == 0 with padding
    (1031, 777, 64, 640, 640, 3),      # R4 = 64, odd ld: element-wise layout
    (999, 1234, 29, 290, 290, 0),      # R4 = 32: the column sweep, ragged m
])
def test_reconstruct_high_rank(R, ctx, m, n, r, p, q, ld_pad):
    # step 5 alone on arbitrary factors (orthonormal U, V; decreasing sigma;
    # FP32-valued Q~, P~) against the oracle's four-block completion
    import torch
    rng = np.random.Generator(np.random.PCG64([m, n, r]))
    I = np.sort(rng.choice(m, p, replace=False))
    J = np.sort(rng.choice(n, q, replace=False))
    U = np.linalg.qr(rng.standard_normal((p, r)))[0]
    V = np.linalg.qr(rng.standard_normal((q, r)))[0]
    sigma = np.sort(rng.uniform(0.5, 2.0, r))[::-1].copy()
    Qt = rng.standard_normal((r, n - q)).astype(np.float32).astype(np.float64)
    Pt = rng.standard_normal((r, m - p)).astype(np.float32).astype(np.float64)
    M = np.asfortranarray(rng.standard_normal((m, n)).astype(np.float32))
    ld = m + ld_pad
    say(f"reconstruct m={m} n={n} r={r} ld={ld}")
    Md = dev_matrix(M, ld)
    L = torch.full((n, ld), float("nan"), dtype=torch.float32, device="cuda")
    S = torch.full_like(L, float("nan"))
    st = R.rpca_reconstruct(ctx, Md, m, n, ld, dev_i64(I), p, dev_i64(J), q, dev_f64_colmajor(U),
                            torch.as_tensor(sigma).cuda(), dev_f64_colmajor(V), r,
                            torch.as_tensor(np.ascontiguousarray(Qt.T, dtype=np.float32)).cuda(),
                            torch.as_tensor(np.ascontiguousarray(Pt.T, dtype=np.float32)).cuda(),
                            L, ld, S, ld)
    torch.cuda.synchronize()
    assert st == R.RPCA_OK
    Lh, Sh = host_matrix(L, m), host_matrix(S, m)
    Lref, Sref = oracle.complete(M, I, J, U, sigma, V, Qt, Pt)
    assert relF(Lh, Lref) <= 1e-6 and relF(Sh, Sref) <= 1e-6
    assert np.array_equal(Sh, (M - Lh.astype(np.float32)).astype(np.float64))
    if ld_pad:
        assert torch_isnan_all(L[:, m:]) and torch_isnan_all(S[:, m:])


# ----------------------------------------------------------------- steps 1-5
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_solve_matches_oracle_c1(R, ctx, seed):
    pr, r, I, J, res = case("c1", seed)
    say(f"solve c1 seed={seed}")
    st, info, L, S = _solve_gpu(R, ctx, pr, r, I, J)
    assert st == R.RPCA_OK, ctx.last_error()
    assert info.r_used == 10 and info.seed_converged == 1
    Lh, Sh = host_matrix(L, pr.m), host_matrix(S, pr.m)
    say(f"ERR c1 fp32 seed={seed} relL={relF(Lh, res.L):.3e} relS={relF(Sh, res.S):.3e} "
        f"relL0={relF(Lh, pr.L0()):.3e}")
    assert relF(Lh, res.L) <= REL_TOL
    assert relF(Sh, res.S) <= REL_TOL
    assert support_mismatch(Sh, res.S, float(np.abs(pr.M).max())) == 0
    # exact recovery, as the oracle (spec gate is on the oracle)
    assert relF(Lh, pr.L0()) <= 1e-5


def test_solve_matches_oracle_c2_sampled(R, ctx):
    # m = n = 10000, r = 20: the workload the benchmark times.  The oracle
    # gives every regression; L is compared on 200000 sampled entries.
    pr, r, I, J, res = case("c2", 1)
    say("solve c2 seed=1 (full size)")
    st, info, L, S = _solve_gpu(R, ctx, pr, r, I, J)
    assert st == R.RPCA_OK, ctx.last_error()
    assert info.r_used == 20
    rng = np.random.default_rng(0)
    rows = rng.integers(0, pr.m, 200000)
    cols = rng.integers(0, pr.n, 200000)
    Lref = oracle.complete_entries(rows, cols, I, J, pr.m, pr.n, res.U, res.sigma, res.V, res.Qt,
                                   res.Pt)
    import torch
    lin = torch.as_tensor(cols * pr.m + rows).cuda()
    Lg = L.reshape(-1)[lin].double().cpu().numpy()
    Sg = S.reshape(-1)[lin].double().cpu().numpy()
    Mv = pr.M[rows, cols].astype(np.float64)
    Sref = Mv - Lref
    assert relF(Lg, Lref) <= REL_TOL
    assert relF(Sg, Sref) <= REL_TOL
    assert support_mismatch(Sg, Sref, float(np.abs(pr.M).max())) == 0
    # mean iteration count within 10% of the oracle's (FP32 vs FP64 stopping test)
    its = info.filt_iters_total / (len(res.col_iters) + len(res.row_iters))
    k_or = np.concatenate([res.col_iters, res.row_iters]).mean()
    assert abs(its - k_or) <= 0.1 * k_or
    assert info.filt_not_converged == 0


def test_filter_every_regression_c2(R, ctx):
    # m = n = 10000, r = 20: all 9800 column and 9800 row regressions of the
    # benchmarked workload, each against the oracle's through the block it
    # defines (U q~_j = L[I_s, j], p~_i^T V^T = L[i, J_s]), per regression and
    # over the whole block
    pr, r, I, J, res = case("c2", 1)
    k = res.U.shape[1]
    Jc, Ic = oracle.complement(J, pr.n), oracle.complement(I, pr.m)
    say("filter c2 every regression")
    st, Qt, itc = _filter_cols_gpu(R, ctx, pr, I, Jc, res.U, k)
    assert st == R.RPCA_OK and (itc > 0).all()
    Lc, Lc_ref = res.U @ Qt, res.U @ res.Qt
    assert relF(Lc, Lc_ref) <= REL_TOL
    per = np.linalg.norm(Lc - Lc_ref, axis=0) / np.linalg.norm(Lc_ref, axis=0)
    assert per.max() <= 10 * REL_TOL, (per.argmax(), per.max())
    st, Pt, itr = _filter_rows_gpu(R, ctx, pr, J, Ic, res.V, k)
    assert st == R.RPCA_OK and (itr > 0).all()
    Lr, Lr_ref = Pt.T @ res.V.T, res.Pt.T @ res.V.T
    assert relF(Lr, Lr_ref) <= REL_TOL
    per = np.linalg.norm(Lr - Lr_ref, axis=1) / np.linalg.norm(Lr_ref, axis=1)
    assert per.max() <= 10 * REL_TOL, (per.argmax(), per.max())
    say(f"  relF(L^c)={relF(Lc, Lc_ref):.2e} relF(L^r)={relF(Lr, Lr_ref):.2e}")


def test_seed_matches_oracle(R, ctx):
    import torch
    pr, r, I, J, res = case("c1", 2)
    say("seed c1 seed=2")
    p, q = len(I), len(J)
    U = torch.zeros((r, p), dtype=torch.float64, device="cuda")
    sg = torch.zeros(r, dtype=torch.float64, device="cuda")
    V = torch.zeros((r, q), dtype=torch.float64, device="cuda")
    st, ru, its = R.rpca_seed(ctx, dev_matrix(pr.M), pr.m, pr.n, pr.m, dev_i64(I), p, dev_i64(J),
                              q, r, R.rpca_opts_default(), U, sg, V)
    assert st == R.RPCA_OK and ru == res.seed.rank == 10
    assert abs(its - res.seed.iters) <= 1
    Uh, sh, Vh = U.cpu().numpy().T, sg.cpu().numpy(), V.cpu().numpy().T
    Ls = (Uh * sh) @ Vh.T
    assert relF(Ls, res.seed.L) <= 1e-9
    assert np.allclose(Uh.T @ Uh, np.eye(r), atol=1e-12)


# ----------------------------------------------------------------- edge cases
@pytest.mark.parametrize("m,n,r,ld_pad", [
    (333, 517, 3, 0),       # p = 30: one partial 16-row tile pair, ragged everything
    (517, 333, 7, 5),       # p = 70, ld = m + 5 (unaligned: scalar completion path)
    (1200, 700, 1, 3),      # r = 1, p = 10 < 16
    (450, 460, 13, 4),      # p = 130 (PT = 10), ld % 4 == 0 with padding
    (2000, 1500, 25, 0),    # r = 25 (two rank tiles), p = 250 (PT = 16)
])
def test_ragged_shapes(R, ctx, m, n, r, ld_pad):
    pr, I, J, res = small_case(m, n, r, 0.05, 7 + r)
    say(f"solve ragged m={m} n={n} r={r} ld={m + ld_pad}")
    st, info, L, S = _solve_gpu(R, ctx, pr, r, I, J, ld=m + ld_pad)
    assert st >= 0, ctx.last_error()
    assert info.r_used == res.U.shape[1]
    Lh, Sh = host_matrix(L, m), host_matrix(S, m)
    assert np.isfinite(Lh).all() and np.isfinite(Sh).all()
    assert relF(Lh, res.L) <= REL_TOL
    assert relF(Sh, res.S) <= REL_TOL
    # padding rows between m and ld are not written
    if ld_pad:
        assert torch_isnan_all(L[:, m:])


def torch_isnan_all(t):
    import torch
    return bool(torch.isnan(t).all().item())


def test_zero_columns_and_iteration_cap(R, ctx):
    pr, r, I, J, res = case("c1", 1)
    Jc = oracle.complement(J, pr.n)
    M0 = pr.M.copy(order="F")
    M0[np.ix_(I, Jc[:5])] = 0.0          # five all-zero regressions
    pr0 = synth.Problem(M=M0, A0=pr.A0, B0=pr.B0, support=None, m=pr.m, n=pr.n, r=r, seed=0)
    say("filter_cols zero columns")
    st, Qt, it = _filter_cols_gpu(R, ctx, pr0, I, Jc, res.U, 10)
    assert st == R.RPCA_OK
    assert (it[:5] == 0).all() and not Qt[:, :5].any()
    say("filter_cols max_iter=1")
    st, Qt, it = _filter_cols_gpu(R, ctx, pr, I, Jc[:37], res.U, 10,
                                  opts=R.rpca_opts_default(filt_max_iter=1))
    assert (it == -1).all()
    # the single step agrees with the oracle's single step
    Zo, Ko = oracle.alg1_batch(pr.M[np.ix_(I, Jc[:37])].astype(np.float64), res.U,
                               oracle.Alg1Params(max_iter=1))
    assert (Ko == -1).all()
    assert relF(res.U @ Qt, res.U @ Zo) <= REL_TOL


def test_filter_empty_and_subset(R, ctx):
    import torch
    pr, r, I, J, res = case("c1", 1)
    say("filter_cols nc=0 and arbitrary column subset")
    st = R.rpca_filter_cols(ctx, dev_matrix(pr.M), pr.m, pr.n, pr.m, dev_i64(I), len(I),
                            dev_i64([0]), 0, dev_f64_colmajor(res.U), 10, R.rpca_opts_default(),
                            torch.zeros(1, device="cuda"), None)
    assert st == R.RPCA_OK
    cols = np.array([999, 3, 3, 500, 17])           # any columns, repeats allowed
    st, Qt, it = _filter_cols_gpu(R, ctx, pr, I, cols, res.U, 10)
    Zo, Ko = oracle.alg1_batch(pr.M[np.ix_(I, cols)].astype(np.float64), res.U)
    assert relF(res.U @ Qt, res.U @ Zo) <= REL_TOL
    assert np.array_equal(Qt[:, 1], Qt[:, 2])


def test_determinism(R, ctx):
    pr, r, I, J, res = case("c1", 3)
    say("solve twice, bitwise")
    _, _, L1, S1 = _solve_gpu(R, ctx, pr, r, I, J)
    _, _, L2, S2 = _solve_gpu(R, ctx, pr, r, I, J)
    assert bool((L1 == L2).all().item()) and bool((S1 == S2).all().item())


def test_library_sampling_solve(R, ctx):
    # rpca_solve with NULL indices draws them itself; the oracle gets the
    # same draw from the host-side sampler.
    pr, r, I, J, res = case("c1", 1)
    opts = R.rpca_opts_default(rng_seed=12345)
    I2, J2 = R.rpca_sample_indices(pr.m, pr.n, 100, 100, 12345)
    say("solve c1 with library sampling")
    st, info, L, S = _solve_gpu(R, ctx, pr, r, opts=opts)
    ref = oracle.solve(pr.M, r, I2, J2)
    if ref.seed.rank == 10:
        assert st == R.RPCA_OK
        assert relF(host_matrix(L, pr.m), ref.L) <= REL_TOL
    else:
        assert st == R.RPCA_WARN_RANK


def test_argument_errors(R, ctx):
    import torch
    pr, r, I, J, res = case("c1", 1)
    Md = dev_matrix(pr.M)
    L = torch.zeros_like(Md)
    S = torch.zeros_like(Md)
    o = R.rpca_opts_default()
    say("argument errors")
    with pytest.raises(R.RpcaError) as e:        # ld < m
        R.rpca_solve(ctx, Md, pr.m, pr.n, pr.m - 1, r, o, None, None, L, pr.m, S, pr.m)
    assert e.value.status == R.RPCA_ERR_ARG
    with pytest.raises(R.RpcaError) as e:        # unsorted seed rows
        R.rpca_solve(ctx, Md, pr.m, pr.n, pr.m, r, o, dev_i64(I[::-1].copy()), dev_i64(J), L, pr.m,
                     S, pr.m)
    assert e.value.status == R.RPCA_ERR_ARG
    with pytest.raises(R.RpcaError) as e:        # seed larger than M
        R.rpca_solve(ctx, Md, pr.m, pr.n, pr.m, 200, o, None, None, L, pr.m, S, pr.m)
    assert e.value.status == R.RPCA_ERR_ARG
    with pytest.raises(R.RpcaError) as e:        # L aliases S
        R.rpca_solve(ctx, Md, pr.m, pr.n, pr.m, r, o, None, None, L, pr.m, L, pr.m)
    assert e.value.status == R.RPCA_ERR_ARG
    with pytest.raises(R.RpcaError) as e:        # bad constants
        R.rpca_solve(ctx, Md, pr.m, pr.n, pr.m, r, R.rpca_opts_default(filt_rho=0.5), None, None,
                     L, pr.m, S, pr.m)
    assert e.value.status == R.RPCA_ERR_ARG
    Mbad = Md.clone()
    Mbad[J[0], I[0]] = float("nan")               # NaN inside the seed block
    with pytest.raises(R.RpcaError) as e:
        R.rpca_solve(ctx, Mbad, pr.m, pr.n, pr.m, r, o, dev_i64(I), dev_i64(J), L, pr.m, S, pr.m)
    assert e.value.status == R.RPCA_ERR_NUMERIC


@pytest.mark.parametrize("precision", [0, 1])
def test_nonfinite_regression_input(R, ctx, precision):
    # NaN in M[I_s, j] (read by column regression j only) and +Inf in M[i, J_s]
    # (row regression i only): those regressions report RPCA_ITERS_NONFINITE
    # and a NaN output; every other regression is untouched; rpca_solve
    # returns RPCA_ERR_NUMERIC
    import torch
    pr, r, I, J, res = case("c1", 1)
    Jc, Ic = oracle.complement(J, pr.n), oracle.complement(I, pr.m)
    M2 = pr.M.copy(order="F")
    M2[I[3], Jc[5]] = np.nan
    M2[Ic[7], J[2]] = np.inf
    pr2 = synth.Problem(M=M2, A0=pr.A0, B0=pr.B0, support=None, m=pr.m, n=pr.n, r=r, seed=0)
    o = R.rpca_opts_default(precision=precision)
    say(f"non-finite regression inputs precision={precision}")
    st, Qt, itc = _filter_cols_gpu(R, ctx, pr2, I, Jc, res.U, 10, opts=o)
    assert itc[5] == R.RPCA_ITERS_NONFINITE and np.isnan(Qt[:, 5]).all()
    keep = np.arange(len(Jc)) != 5
    assert (itc[keep] > 0).all() and np.isfinite(Qt[:, keep]).all()
    assert relF(res.U @ Qt[:, keep], res.U @ res.Qt[:, keep]) <= REL_TOL
    st, Pt, itr = _filter_rows_gpu(R, ctx, pr2, J, Ic, res.V, 10, opts=o)
    assert itr[7] == R.RPCA_ITERS_NONFINITE and np.isnan(Pt[:, 7]).all()
    keep = np.arange(len(Ic)) != 7
    assert (itr[keep] > 0).all()
    assert relF(Pt[:, keep].T @ res.V.T, res.Pt[:, keep].T @ res.V.T) <= REL_TOL
    Md = dev_matrix(M2)
    L = torch.zeros_like(Md)
    S = torch.zeros_like(Md)
    with pytest.raises(R.RpcaError) as e:
        R.rpca_solve(ctx, Md, pr.m, pr.n, pr.m, r, o, dev_i64(I), dev_i64(J), L, pr.m, S, pr.m)
    assert e.value.status == R.RPCA_ERR_NUMERIC
    assert "non-finite" in ctx.last_error()
