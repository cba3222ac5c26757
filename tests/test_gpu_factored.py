"""GPU parity of the factored output (Algorithm 2 stopped before the m x n
completion, Sec. 3.4) and of online column filtering (new columns filtered
against the fitted U and completed alone, Sec. 3.2 / Sec. 4.3), through the C
ABI, against the FP64 oracle.

Tolerance: relative Frobenius error <= 1e-5 on every block the factors define
(``U Sigma V^T``, ``U Q~``, ``P~^T V^T``) and on L and S of the new columns;
supports of S agree away from the threshold.  Factors themselves are never
compared (singular vectors are defined up to sign and rotation).
"""
from __future__ import annotations

import functools

import numpy as np
import pytest

import oracle
import synth
from gpu_util import REL_TOL, dev_i64, dev_matrix, host_matrix, relF, say, support_mismatch

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
def appended(m, n, nnew, r, seed):
    """One low-rank-plus-sparse model over n + nnew columns: the first n are
    fitted, the last nnew arrive afterwards."""
    pr = synth.lowrank_plus_sparse(m, n + nnew, r, factor_std=np.sqrt(1.0 / max(m, n)),
                                   sparsity=0.10, values="pm1", seed=seed)
    M0 = np.asfortranarray(pr.M[:, :n])
    Mnew = np.asfortranarray(pr.M[:, n:])
    I, J = synth.seed_indices(m, n, 10 * r, 10 * r, seed=seed)
    fit = oracle.solve(M0, r, I, J)
    return pr, M0, Mnew, I, J, fit


def _factored_gpu(R, ctx, M, I, J, r, ld=None, opts=None):
    import torch
    m, n = M.shape
    ld = ld or m
    p, q = len(I), len(J)
    Md = dev_matrix(M, ld)
    U = torch.full((r, p), float("nan"), dtype=torch.float64, device="cuda")
    sg = torch.full((r,), float("nan"), dtype=torch.float64, device="cuda")
    V = torch.full((r, q), float("nan"), dtype=torch.float64, device="cuda")
    Qt = torch.full((r * (n - q),), float("nan"), dtype=torch.float32, device="cuda")
    Pt = torch.full((r * (m - p),), float("nan"), dtype=torch.float32, device="cuda")
    kc = torch.zeros(n - q, dtype=torch.int32, device="cuda")
    kr = torch.zeros(m - p, dtype=torch.int32, device="cuda")
    dI, dJ = dev_i64(I), dev_i64(J)
    st, info = R.rpca_solve_factored(ctx, Md, m, n, ld, r, opts or R.rpca_opts_default(), dI, p, dJ,
                                     q, U, sg, V, Qt, kc, Pt, kr)
    torch.cuda.synchronize()
    return dict(st=st, info=info, Md=Md, ld=ld, dI=dI, dJ=dJ, U=U, sg=sg, V=V, Qt=Qt, Pt=Pt,
                kc=kc, kr=kr)


def _host_factors(g, p, q, m, n):
    ru = g["info"].r_used
    U = g["U"].cpu().numpy().T[:, :ru]
    sg = g["sg"].cpu().numpy()[:ru]
    V = g["V"].cpu().numpy().T[:, :ru]
    Qt = g["Qt"][: ru * (n - q)].view(n - q, ru).double().cpu().numpy().T
    Pt = g["Pt"][: ru * (m - p)].view(m - p, ru).double().cpu().numpy().T
    return ru, U, sg, V, Qt, Pt


@pytest.mark.parametrize("seed", [1, 2])
def test_solve_factored_matches_oracle(R, ctx, seed):
    pr, M0, Mnew, I, J, fit = appended(1000, 1000, 200, 10, seed)
    m, n = M0.shape
    say(f"solve_factored m=n={m} r=10 seed={seed}")
    g = _factored_gpu(R, ctx, M0, I, J, 10)
    assert g["st"] == R.RPCA_OK, R.rpca_status_string(g["st"])
    ru, U, sg, V, Qt, Pt = _host_factors(g, len(I), len(J), m, n)
    assert ru == fit.U.shape[1]
    assert relF((U * sg) @ V.T, (fit.U * fit.sigma) @ fit.V.T) <= 1e-9
    assert relF(U @ Qt, fit.U @ fit.Qt) <= REL_TOL
    assert relF(Pt.T @ V.T, fit.Pt.T @ fit.V.T) <= REL_TOL
    # columns beyond the rank used are zero; iteration counts are positive
    assert np.all(g["U"].cpu().numpy()[ru:] == 0) and np.all(g["sg"].cpu().numpy()[ru:] == 0)
    assert (g["kc"].cpu().numpy() > 0).all() and (g["kr"].cpu().numpy() > 0).all()
    assert g["info"].t_reconstruct_ms == 0.0
    # the factors complete to the oracle's L and S through rpca_reconstruct
    import torch
    L = torch.empty_like(g["Md"])
    S = torch.empty_like(g["Md"])
    R.rpca_reconstruct(ctx, g["Md"], m, n, g["ld"], g["dI"], len(I), g["dJ"], len(J), g["U"], g["sg"],
                       g["V"], ru, g["Qt"], g["Pt"], L, g["ld"], S, g["ld"])
    torch.cuda.synchronize()
    Lh, Sh = host_matrix(L, m), host_matrix(S, m)
    assert relF(Lh, fit.L) <= REL_TOL and relF(Sh, fit.S) <= REL_TOL
    assert support_mismatch(Sh, fit.S, float(np.abs(M0).max())) == 0


def test_solve_factored_rank_below_target(R, ctx):
    # target rank above the data's: the seed's rank is used, the outputs are
    # packed with that leading dimension and the status says so
    pr, M0, Mnew, I, J, fit = appended(1000, 1000, 200, 10, 1)
    Ib, Jb = synth.seed_indices(1000, 1000, 120, 120, seed=5)
    ref = oracle.solve(M0, 12, Ib, Jb, assemble=False)
    g = _factored_gpu(R, ctx, M0, Ib, Jb, 12)
    say(f"solve_factored r=12 on rank-10 data: status={R.rpca_status_string(g['st'])} "
        f"r_used={g['info'].r_used} oracle rank={ref.U.shape[1]}")
    assert g["st"] == R.RPCA_WARN_RANK
    ru, U, sg, V, Qt, Pt = _host_factors(g, 120, 120, 1000, 1000)
    assert ru == ref.U.shape[1] == 10
    assert relF(U @ Qt, ref.U @ ref.Qt) <= REL_TOL
    assert relF(Pt.T @ V.T, ref.Pt.T @ ref.V.T) <= REL_TOL


@pytest.mark.parametrize("nnew,ld_pad", [(200, 0), (37, 3), (1, 0)])
def test_filter_new_cols_matches_oracle(R, ctx, nnew, ld_pad):
    import torch
    pr, M0, Mnew_all, I, J, fit = appended(1000, 1000, 200, 10, 1)
    m, n = M0.shape
    Mnew = np.asfortranarray(Mnew_all[:, :nnew])
    # expected: the oracle's own fit, its filtering of the new columns, eq. l1s'
    Qn, kn = oracle.filter_cols(Mnew, I, np.arange(nnew), fit.U)
    Lr, Sr = oracle.complete_new_cols(Mnew, I, fit.U, fit.sigma, fit.Pt, Qn)
    g = _factored_gpu(R, ctx, M0, I, J, 10)
    ru = g["info"].r_used
    ld = m + ld_pad
    say(f"filter_new_cols nnew={nnew} ld={ld} r_used={ru}")
    Mn = dev_matrix(Mnew, ld)
    Qn_d = torch.full((nnew, ru), float("nan"), dtype=torch.float32, device="cuda")
    it = torch.zeros(nnew, dtype=torch.int32, device="cuda")
    L = torch.full((nnew, ld), float("nan"), dtype=torch.float32, device="cuda")
    S = torch.full((nnew, ld), float("nan"), dtype=torch.float32, device="cuda")
    st = R.rpca_filter_new_cols(ctx, Mn, m, nnew, ld, g["dI"], len(I), g["U"], g["sg"], ru, g["Pt"],
                                R.rpca_opts_default(), Qn_d, it, L, ld, S, ld)
    torch.cuda.synchronize()
    assert st == R.RPCA_OK
    Lh, Sh = host_matrix(L, m), host_matrix(S, m)
    assert relF(Lh, Lr) <= REL_TOL and relF(Sh, Sr) <= REL_TOL
    assert support_mismatch(Sh, Sr, float(np.abs(pr.M).max())) == 0
    U = g["U"].cpu().numpy().T[:, :ru]
    assert relF(U @ Qn_d.double().cpu().numpy().T, fit.U @ Qn) <= REL_TOL
    assert (it.cpu().numpy() > 0).all()
    # the padding rows of L and S are not written
    if ld_pad:
        assert torch.isnan(L[:, m:]).all() and torch.isnan(S[:, m:]).all()
    # and the new columns are as close to the underlying low-rank model as the
    # oracle's (this draw's seed block is near PCP's recovery boundary: the
    # oracle itself is ~3e-4 from L0 here)
    L0 = pr.L0()[:, n:n + nnew]
    assert relF(Lh, L0) <= oracle.relerr(Lr, L0) + REL_TOL


def test_filter_new_cols_flags_nonfinite_columns(R, ctx):
    import torch
    pr, M0, Mnew_all, I, J, fit = appended(1000, 1000, 200, 10, 1)
    m = M0.shape[0]
    Mnew = np.array(Mnew_all[:, :40], order="F")
    Mnew[I[3], 7] = np.nan                 # a seed row of column 7
    Mnew[oracle.complement(I, m)[0], 9] = np.inf     # a non-seed row of column 9
    g = _factored_gpu(R, ctx, M0, I, J, 10)
    ru = g["info"].r_used
    Mn = dev_matrix(Mnew)
    Qn_d = torch.zeros((40, ru), dtype=torch.float32, device="cuda")
    it = torch.zeros(40, dtype=torch.int32, device="cuda")
    L = torch.empty_like(Mn)
    S = torch.empty_like(Mn)
    st = R.rpca_filter_new_cols(ctx, Mn, m, 40, m, g["dI"], len(I), g["U"], g["sg"], ru, g["Pt"],
                                R.rpca_opts_default(), Qn_d, it, L, m, S, m)
    torch.cuda.synchronize()
    assert st == R.RPCA_OK
    its = it.cpu().numpy()
    assert its[7] == R.RPCA_ITERS_NONFINITE
    assert np.all(its[np.arange(40) != 7] > 0)
    Lh = host_matrix(L, m)
    assert np.isnan(Lh[:, 7]).all()
    assert np.isfinite(np.delete(Lh, 7, axis=1)).all()


def test_filter_new_cols_argument_errors(R, ctx):
    import torch
    pr, M0, Mnew_all, I, J, fit = appended(1000, 1000, 200, 10, 1)
    m = M0.shape[0]
    g = _factored_gpu(R, ctx, M0, I, J, 10)
    Mn = dev_matrix(np.asfortranarray(Mnew_all[:, :8]))
    Qn_d = torch.zeros((8, 10), dtype=torch.float32, device="cuda")
    L = torch.empty_like(Mn)
    o = R.rpca_opts_default()
    with pytest.raises(R.RpcaError) as e:        # L and S the same buffer
        R.rpca_filter_new_cols(ctx, Mn, m, 8, m, g["dI"], len(I), g["U"], g["sg"], 10, g["Pt"], o,
                               Qn_d, None, L, m, L, m)
    assert e.value.status == R.RPCA_ERR_ARG
    with pytest.raises(R.RpcaError) as e:        # leading dimension below m
        R.rpca_filter_new_cols(ctx, Mn, m, 8, m - 1, g["dI"], len(I), g["U"], g["sg"], 10, g["Pt"],
                               o, Qn_d, None, L, m, torch.empty_like(Mn), m)
    assert e.value.status == R.RPCA_ERR_ARG
    with pytest.raises(R.RpcaError) as e:        # rank above the seed size
        R.rpca_filter_new_cols(ctx, Mn, m, 8, m, g["dI"], len(I), g["U"], g["sg"], len(I) + 1,
                               g["Pt"], o, Qn_d, None, L, m, torch.empty_like(Mn), m)
    assert e.value.status == R.RPCA_ERR_ARG
