"""FP32 form beyond the FP32 tile classes (p > 304, opts.precision = 0): the
quarter-tile shape (four waves per 16-regression tile, persistent
workgroups) with both contractions of Alg. 1 on FP32 MFMA, against the FP64
oracle at the same tolerance as every other form (relative Frobenius 1e-5 on
L^c = U Q~, L^r = P~^T V^T, L and S)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_util import REL_TOL, dev_f64_colmajor, dev_i64, dev_matrix, host_matrix, relF, say, support_mismatch
from test_gpu_parity import R, _filter_cols_gpu, _filter_rows_gpu, ctx, small_case  # noqa: F401

pytestmark = pytest.mark.gpu

FORM_QUARTER32 = 3      # rpca_filter_form: FP32 quarter-tile form


def _fp32(R):
    return R.rpca_opts_default(precision=0)


# p = 310, 410, 500 (tile classes 26, 26, 32; rank classes 8, 11 -> 13, 13):
# ragged tile counts leave some workgroups one tile fewer than others
@pytest.mark.parametrize("m,n,r", [(2300, 2111, 31), (2600, 2333, 41), (2700, 2517, 50)])
def test_fp32_quarter_solve_matches_oracle(R, ctx, m, n, r):
    import torch
    pr, I, J, res = small_case(m, n, r, 0.05, 7 + r)
    p = 10 * r
    assert R.rpca_filter_form(ctx, p, r, (m - p) + (n - p), _fp32(R)) == FORM_QUARTER32
    say(f"fp32 quarter-tile solve m={m} n={n} r={r} p={p}")
    Md = dev_matrix(pr.M)
    L = torch.full_like(Md, float("nan"))
    S = torch.full_like(Md, float("nan"))
    st, info = R.rpca_solve(ctx, Md, m, n, m, r, _fp32(R), dev_i64(I), dev_i64(J), L, m, S, m)
    torch.cuda.synchronize()
    assert st >= 0, ctx.last_error()
    assert info.filt_not_converged == 0
    Lh, Sh = host_matrix(L, m), host_matrix(S, m)
    eL, eS = relF(Lh, res.L), relF(Sh, res.S)
    its = info.filt_iters_total / ((m - p) + (n - p))
    k_or = np.concatenate([res.col_iters, res.row_iters]).mean()
    say(f"ERR fp32 quarter m={m} r={r} relL={eL:.3e} relS={eS:.3e} mean steps {its:.2f} "
        f"(oracle {k_or:.2f})")
    assert eL <= REL_TOL and eS <= REL_TOL
    assert support_mismatch(Sh, res.S, float(np.abs(pr.M).max())) == 0


def test_fp32_quarter_filter_every_regression(R, ctx):
    # every column and row regression of a p = 410 problem against the
    # oracle's own Alg. 1 results (the seed's U, V), through rpca_filter (both
    # families in one launch)
    import torch
    m, n, r = 2600, 2333, 41
    pr, I, J, res = small_case(m, n, r, 0.05, 7 + r)
    Jc, Ic = oracle.complement(J, n), oracle.complement(I, m)
    k = res.U.shape[1]
    say(f"fp32 quarter-tile rpca_filter p={10 * r} r={k}")
    Md = dev_matrix(pr.M)
    Qt = torch.full((len(Jc), k), float("nan"), device="cuda")
    Pt = torch.full((len(Ic), k), float("nan"), device="cuda")
    kc = torch.zeros(len(Jc), dtype=torch.int32, device="cuda")
    kr = torch.zeros(len(Ic), dtype=torch.int32, device="cuda")
    st = R.rpca_filter(ctx, Md, m, n, m, dev_i64(I), len(I), dev_i64(J), len(J), dev_i64(Jc), len(Jc),
                       dev_i64(Ic), len(Ic), dev_f64_colmajor(res.U), dev_f64_colmajor(res.V), k, _fp32(R),
                       Qt, kc, Pt, kr)
    torch.cuda.synchronize()
    assert st == R.RPCA_OK, ctx.last_error()
    Qh, Ph = Qt.double().cpu().numpy().T, Pt.double().cpu().numpy().T
    eq = relF(res.U @ Qh, res.U @ res.Qt)
    ep = relF(Ph.T @ res.V.T, res.Pt.T @ res.V.T)
    # per regression as well: the worst column of U Q~ against the oracle's
    cw = np.linalg.norm(res.U @ (Qh - res.Qt), axis=0) / np.maximum(np.linalg.norm(res.U @ res.Qt, axis=0),
                                                                     1e-30)
    say(f"ERR fp32 quarter filter relLc={eq:.3e} relLr={ep:.3e} worst column {cw.max():.3e}")
    assert eq <= REL_TOL and ep <= REL_TOL
    assert (kc.cpu().numpy() > 0).all() and (kr.cpu().numpy() > 0).all()


# rank classes at the ends (r = 1: one K-step; r = 62: sixteen, where two
# tiles' exchange buffers no longer fit next to the FP32 basis in LDS and a
# workgroup serves one tile).  The basis is an orthonormal basis of the true
# factor on the seed rows (columns), so each regression recovers its
# coefficients from x = U z* + sparse corruption; the FP64 oracle runs
# Algorithm 1 on the same inputs.
@pytest.mark.parametrize("m,n,r,p", [(1500, 1400, 1, 400), (1400, 1300, 62, 480), (1300, 1250, 7, 512)])
def test_fp32_quarter_rank_classes(R, ctx, m, n, r, p):
    pr = synth.lowrank_plus_sparse(m, n, r, factor_std=np.sqrt(1.0 / max(m, n)), sparsity=0.05,
                                   values="pm1", seed=21 + r)
    I, J = synth.seed_indices(m, n, p, p, seed=21 + r)
    Jc, Ic = oracle.complement(J, n), oracle.complement(I, m)
    U, _ = np.linalg.qr(pr.A0[I])
    V, _ = np.linalg.qr(pr.B0[J])
    assert R.rpca_filter_form(ctx, p, r, len(Jc), _fp32(R)) == FORM_QUARTER32
    say(f"fp32 quarter-tile rank class: p = q = {p}, r = {r}")
    st, Qt, itc = _filter_cols_gpu(R, ctx, pr, I, Jc, U, r, opts=_fp32(R))
    assert st == R.RPCA_OK, ctx.last_error()
    Zc, _ = oracle.alg1_batch(pr.M[np.ix_(I, Jc)].astype(np.float64), U)
    ec = relF(U @ Qt, U @ Zc)
    st, Pt, itr = _filter_rows_gpu(R, ctx, pr, J, Ic, V, r, opts=_fp32(R))
    assert st == R.RPCA_OK, ctx.last_error()
    Zr, _ = oracle.alg1_batch(pr.M[np.ix_(Ic, J)].T.astype(np.float64), V)
    er = relF(V @ Pt, V @ Zr)
    say(f"ERR fp32 quarter p={p} r={r} relLc={ec:.3e} relLr={er:.3e}")
    assert ec <= REL_TOL and er <= REL_TOL
    assert (itc > 0).all() and (itr > 0).all()


def test_fp32_quarter_nonfinite_and_bad_index(R, ctx):
    # p = 500: NaN in M[I_s, j] (column regression j only), +Inf in M[i, J_s]
    # (row regression i only), a column index past n: those report
    # RPCA_ITERS_NONFINITE / RPCA_ITERS_BAD_INDEX, every other regression is
    # the oracle's
    m, n, r = 2700, 2517, 50
    pr, I, J, res = small_case(m, n, r, 0.05, 7 + r)
    Jc, Ic = oracle.complement(J, n), oracle.complement(I, m)
    M2 = pr.M.copy(order="F")
    M2[I[3], Jc[5]] = np.nan
    M2[Ic[7], J[2]] = np.inf
    pr2 = synth.Problem(M=M2, A0=pr.A0, B0=pr.B0, support=None, m=m, n=n, r=r, seed=0)
    cols = Jc.copy()
    cols[9] = n + 5
    k = res.U.shape[1]
    say("fp32 quarter-tile non-finite and bad-index regressions")
    st, Qt, itc = _filter_cols_gpu(R, ctx, pr2, I, cols, res.U, k, opts=_fp32(R))
    assert itc[5] == R.RPCA_ITERS_NONFINITE and np.isnan(Qt[:, 5]).all()
    assert itc[9] == R.RPCA_ITERS_BAD_INDEX
    keep = (np.arange(len(Jc)) != 5) & (np.arange(len(Jc)) != 9)
    assert (itc[keep] > 0).all() and np.isfinite(Qt[:, keep]).all()
    assert relF(res.U @ Qt[:, keep], res.U @ res.Qt[:, keep]) <= REL_TOL
    st, Pt, itr = _filter_rows_gpu(R, ctx, pr2, J, Ic, res.V, k, opts=_fp32(R))
    assert itr[7] == R.RPCA_ITERS_NONFINITE and np.isnan(Pt[:, 7]).all()
    keep = np.arange(len(Ic)) != 7
    assert (itr[keep] > 0).all()
    assert relF(Pt[:, keep].T @ res.V.T, res.Pt[:, keep].T @ res.V.T) <= REL_TOL


def test_fp32_c3_full_size_sampled(R, ctx):
    # m = n = 50000, r = 50, 5% U[-1,1] corruptions, 500 x 500 seed, FP32
    # form: the whole matrix is solved on the GPU; the oracle recomputes the
    # seed and a sample of 300 column and 300 row regressions, and L, S are
    # compared on the entries those determine (plus seed-block entries)
    import torch
    m = n = 50000
    r, p = 50, 500
    say("fp32 c3: generating 50000 x 50000 on the device")
    Md, A0, B0 = synth.lowrank_plus_sparse_device(m, n, r, factor_std=np.sqrt(2e-5), sparsity=0.05,
                                                  values="unif11", seed=1, device="cuda")
    I, J = synth.seed_indices(m, n, p, p, seed=1)
    L = torch.empty_like(Md)
    S = torch.empty_like(Md)
    say("fp32 c3: solve")
    st, info = R.rpca_solve(ctx, Md, m, n, m, r, _fp32(R), dev_i64(I), dev_i64(J), L, m, S, m)
    torch.cuda.synchronize()
    assert st == R.RPCA_OK, ctx.last_error()
    assert info.r_used == r and info.filt_not_converged == 0
    say(f"fp32 c3: t_seed {info.t_seed_ms:.0f} ms, filter {info.t_filter_ms:.3f} ms, "
        f"completion {info.t_reconstruct_ms:.3f} ms")
    dI, dJ = dev_i64(I), dev_i64(J)
    Ms = Md[dJ][:, dI].double().cpu().numpy().T                 # M[I, J]
    sd = oracle.seed_pcp(Ms)
    assert sd.rank == r
    rng = np.random.default_rng(5)
    Ic, Jc = oracle.complement(I, m), oracle.complement(J, n)
    cs = np.sort(rng.choice(len(Jc), 300, replace=False))
    rs = np.sort(rng.choice(len(Ic), 300, replace=False))
    Xc = Md[dev_i64(Jc[cs])][:, dI].double().cpu().numpy().T      # p x 300
    Xr = Md[dJ][:, dev_i64(Ic[rs])].double().cpu().numpy()        # q x 300
    Qs, kq = oracle.alg1_batch(Xc, sd.U)
    Ps, kp = oracle.alg1_batch(Xr, sd.V)
    Qt = np.zeros((r, len(Jc)))
    Pt = np.zeros((r, len(Ic)))
    Qt[:, cs] = Qs
    Pt[:, rs] = Ps
    rows = np.concatenate([rng.choice(Ic[rs], 3000), rng.choice(I, 500)])
    cols = np.concatenate([rng.choice(Jc[cs], 2000), rng.choice(J, 1500)])
    rng.shuffle(cols)
    Lref = oracle.complete_entries(rows, cols, I, J, m, n, sd.U, sd.sigma, sd.V, Qt, Pt)
    lin = torch.as_tensor(cols.astype(np.int64) * m + rows.astype(np.int64)).cuda()
    Lg = L.reshape(-1)[lin].double().cpu().numpy()
    Sg = S.reshape(-1)[lin].double().cpu().numpy()
    Mv = Md.reshape(-1)[lin].double().cpu().numpy()
    eL, eS = relF(Lg, Lref), relF(Sg, Mv - Lref)
    say(f"ERR fp32 c3 sampled relL={eL:.3e} relS={eS:.3e}")
    assert eL <= REL_TOL and eS <= REL_TOL
    L0 = (A0[rows] * B0[cols]).sum(1)
    assert relF(Lg, L0) <= 1e-5


# Enough regressions (10 000 on one side) that every tile slot serves a long
# sequence and refills its columns: the same seven regressions repeated over
# the sequence land in different columns and start at different refill points,
# and must give the same bits and step counts each time; zero regressions stop
# at once (count 0, z = 0) and free their column; with an iteration cap every
# regression stops at the cap (count -cap, z = the oracle's after cap steps).
@pytest.mark.parametrize("precision", [0, 1])
def test_quarter_refill_repeats_zeros_caps(R, ctx, precision):
    m, n, r = 2600, 2333, 41
    pr, I, J, res = small_case(m, n, r, 0.05, 48)
    Jc = oracle.complement(J, n)
    k = res.U.shape[1]
    o = R.rpca_opts_default(precision=precision)
    pick = Jc[[5, 99, 400, 800, 1200, 1500, 1900]]
    cols = np.tile(pick, 1429)                        # 10 003 regressions
    zero = np.arange(3, cols.size, 977)               # some of them all-zero
    M0 = pr.M.copy(order="F")
    zcol = np.setdiff1d(Jc, pick)[:zero.size]
    M0[np.ix_(I, zcol)] = 0.0
    cols[zero] = zcol
    pr0 = synth.Problem(M=M0, A0=pr.A0, B0=pr.B0, support=None, m=m, n=n, r=r, seed=0)
    say(f"quarter-tile refill: repeats, zeros (precision={precision})")
    st, Qt, it = _filter_cols_gpu(R, ctx, pr0, I, cols, res.U, k, opts=o)
    assert st == R.RPCA_OK, ctx.last_error()
    assert (it[zero] == 0).all() and not Qt[:, zero].any()
    rep = np.setdiff1d(np.arange(cols.size), zero)
    first = {}
    for i in rep:
        a = first.setdefault(int(cols[i]), i)
        assert it[i] == it[a] and np.array_equal(Qt[:, i], Qt[:, a]), (i, a)
    Zo, Ko = oracle.alg1_batch(pr.M[np.ix_(I, pick)].astype(np.float64), res.U)
    Qp = np.stack([Qt[:, first[int(c)]] for c in pick], axis=1)
    assert relF(res.U @ Qp, res.U @ Zo) <= REL_TOL
    if precision == 0:
        base = Jc[:1200]
        capcols = np.tile(base, 9)                    # 10 800 regressions
        for cap in (1, 3, 9, 12):                   # below every step count of these regressions
            say(f"quarter-tile refill: max_iter={cap}")
            st, Qt, it = _filter_cols_gpu(R, ctx, pr, I, capcols, res.U, k,
                                          opts=R.rpca_opts_default(precision=0, filt_max_iter=cap))
            assert st == R.RPCA_OK, ctx.last_error()
            Zo, Ko = oracle.alg1_batch(pr.M[np.ix_(I, base)].astype(np.float64), res.U,
                                       oracle.Alg1Params(max_iter=cap))
            assert (Ko == -cap).all()
            assert np.array_equal(it, np.tile(Ko, 9)), cap
            for rpt in range(9):
                sl = slice(rpt * base.size, (rpt + 1) * base.size)
                assert relF(res.U @ Qt[:, sl], res.U @ Zo) <= REL_TOL, (cap, rpt)


def test_form_table_and_size_limit(R, ctx):
    # which kernel a call takes, by p and precision form; p = 513 is beyond
    # every built class and is refused before any launch
    import torch
    f = lambda p, r, prec: R.rpca_filter_form(ctx, p, r, 20000, R.rpca_opts_default(precision=prec))
    assert f(304, 20, 0) in (1, 2) and f(305, 20, 0) == FORM_QUARTER32
    assert f(512, 64, 0) == FORM_QUARTER32 and f(410, 1, 0) == FORM_QUARTER32
    assert f(500, 50, 1) == 0 and f(300, 30, 1) == 0
    assert f(40, 4, 1) in (1, 2)                      # below 48 elements the precision form stays FP32
    m, n, r, p = 700, 300, 5, 513
    pr = synth.lowrank_plus_sparse(m, n, r, factor_std=np.sqrt(1.0 / m), sparsity=0.05, values="pm1", seed=3)
    I, J = synth.seed_indices(m, n, p, 50, seed=3)
    U, _ = np.linalg.qr(pr.A0[I])
    cols = oracle.complement(J, n)[:10]
    for prec in (0, 1):
        say(f"filter beyond the classes: p = {p}, precision = {prec}")
        with pytest.raises(R.RpcaError) as e:
            _filter_cols_gpu(R, ctx, pr, I, cols, U, r, opts=R.rpca_opts_default(precision=prec))
        assert e.value.status == R.RPCA_ERR_UNSUPPORTED
