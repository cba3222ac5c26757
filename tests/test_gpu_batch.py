"""Batched form on the GPU (rpca_batch_*): many independent problems of uneven
sizes, every one compared with the FP64 oracle run on that problem alone
(Algorithm 2 per job; relative Frobenius 1e-5 on L and S, identical support
of S away from the threshold).

The jobs are shaped like video background modelling (pixels x frames, block
corruptions) and cover every path of the batch: lane-form regressions of
both class groups (p <= 40 and p = 50..80), the 16-regression tile form
(p > 80), mixed sides (lane columns, tile rows), completion in the batched
launch (r <= 8) and alone (r > 8), padded and odd leading dimensions, a job
whose seed takes every row, and a job with no regressions at all.

Seed tolerance.  With the block foregrounds of these jobs the seed PCP stops
at seed_tol = 1e-9 (relative residual) while its L^s is still ~3e-5 away from
the ALM fixed point, so two FP64 runs of it that differ only in rounding (the
GPU's and the oracle's SVDs) end ~1e-6 apart, and Sigma^{-1} of the
completion amplifies that.  Both sides therefore run the seed to its FP64
fixed point (seed_tol = 1e-12, identical on both sides): the comparison then
measures steps 3-5 and a converged seed, not where a stopping test fired."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_util import REL_TOL, dev_i64, relF, say, support_mismatch
from test_gpu_parity import R, ctx  # noqa: F401  (fixtures)

pytestmark = pytest.mark.gpu


def _edge_spec(m, n, r, seed, rho=0.08):
    rng = np.random.Generator(np.random.PCG64([seed, 7]))
    return synth.BatchJobSpec(m=m, n=n, r=r, rho=rho,
                              rects=synth.block_rectangles(rng, m, n, rho), seed=seed)


def _small_jobs():
    """(spec, p, q, ldm, ldl) of the small parity batch."""
    jobs = [(s, 10 * s.r, 10 * s.r, s.m, s.m)
            for s in synth.batch_specs(10, 11, m=(300, 3000), n=(100, 400), r=(1, 8))]
    jobs += [
        (_edge_spec(700, 450, 10, 901), 100, 100, 700, 700),    # tile form, completion alone
        (_edge_spec(900, 500, 6, 902), 60, 100, 900, 900),      # lane columns, tile rows
        (_edge_spec(1001, 333, 3, 903), 30, 30, 1004, 1003),    # padded / odd leading dims
        (_edge_spec(40, 300, 4, 904), 40, 40, 40, 40),          # seed takes every row
        (_edge_spec(50, 50, 5, 905), 50, 50, 50, 50),           # no regressions
        (_edge_spec(2500, 120, 8, 906), 80, 80, 2500, 2500),    # largest lane class
    ]
    return jobs


SEED_TOL = 1e-12
_CACHE = {}


def _opts(R):
    return R.rpca_opts_default(seed_tol=SEED_TOL)


def _small_batch_reference():
    if "small" not in _CACHE:
        out = []
        for spec, p, q, ldm, ldl in _small_jobs():
            P = synth.batch_job_host(spec)
            I, J = synth.seed_indices(spec.m, spec.n, p, q, seed=spec.seed)
            res = oracle.solve(P.M, spec.r, I, J, seed_params=oracle.SeedParams(tol=SEED_TOL))
            out.append((spec, p, q, ldm, ldl, P, I, J, res))
        _CACHE["small"] = out
    return _CACHE["small"]


def _upload(P, ldm):
    import torch
    Mt = torch.full((P.n, ldm), float("nan"), dtype=torch.float32, device="cuda")
    Mt[:, :P.m] = torch.from_numpy(np.ascontiguousarray(P.M.T)).cuda()
    return Mt


def _build(R, ctx, ref, tuning=None):
    import torch
    keep, jobs = [], []
    for spec, p, q, ldm, ldl, P, I, J, res in ref:
        Md = _upload(P, ldm)
        L = torch.full((P.n, ldl), float("nan"), dtype=torch.float32, device="cuda")
        S = torch.full((P.n, ldl), float("nan"), dtype=torch.float32, device="cuda")
        dI, dJ = dev_i64(I), dev_i64(J)
        keep.append((Md, L, S, dI, dJ))
        jobs.append(R.job(Md, P.m, P.n, ldm, spec.r, dI, p, dJ, q, L, ldl, S, ldl))
    b = R.Batch(ctx, jobs, _opts(R), tuning)
    return b, keep


def _check_job(k, ref_k, L, S):
    spec, p, q, ldm, ldl, P, I, J, res = ref_k
    Lh = L[:, :P.m].double().cpu().numpy().T
    Sh = S[:, :P.m].double().cpu().numpy().T
    eL, eS = relF(Lh, res.L), relF(Sh, res.S)
    assert eL <= REL_TOL and eS <= REL_TOL, (k, spec.m, spec.n, spec.r, p, q, eL, eS)
    assert support_mismatch(Sh, res.S, float(np.abs(P.M).max())) == 0, k


def test_batch_matches_oracle_per_job(R, ctx):
    import torch
    ref = _small_batch_reference()
    say(f"batch parity: {len(ref)} jobs")
    b, keep = _build(R, ctx, ref)
    st = R.rpca_batch_seed(b)
    assert st >= 0, ctx.last_error()
    R.rpca_batch_run(b)
    torch.cuda.synchronize()
    for k, (Md, L, S, dI, dJ) in enumerate(keep):
        spec, p, q, ldm, ldl, P, I, J, res = ref[k]
        st, info = R.rpca_batch_job_info(b, k)
        assert info.r_used == min(res.seed.rank, spec.r)
        _check_job(k, ref[k], L, S)
        # iteration counts within one of the oracle's (FP32 vs FP64 stopping test)
        if info.filt_iters_total:
            kor = np.concatenate([res.col_iters, res.row_iters])
            assert abs(info.filt_iters_max - int(np.abs(kor).max())) <= 2, k
        assert info.filt_not_converged == 0
    b.close()


def test_batch_large_p_fp32_jobs(R, ctx):
    # jobs beyond the FP32 tile classes in one batch (p = 410 and 500: the
    # FP32 quarter-tile form on both sides of each) next to a lane-form job,
    # each against the oracle run on that job alone (the random low-rank +
    # sparse problems of the single-problem tests, whose seeds reach their
    # rank at the default tolerance on both sides)
    import torch
    from test_gpu_parity import small_case
    cases = [(2600, 2333, 41, 48, 2600), (2700, 2517, 50, 57, 2703), (900, 400, 5, 12, 900)]
    keep, jobs, ref = [], [], []
    for m, n, r, seed, ldm in cases:
        pr, I, J, res = small_case(m, n, r, 0.05, seed)
        Md = _upload(pr, ldm)
        L = torch.full((n, ldm), float("nan"), dtype=torch.float32, device="cuda")
        S = torch.full((n, ldm), float("nan"), dtype=torch.float32, device="cuda")
        dI, dJ = dev_i64(I), dev_i64(J)
        keep.append((Md, L, S, dI, dJ))
        jobs.append(R.job(Md, m, n, ldm, r, dI, len(I), dJ, len(J), L, ldm, S, ldm))
        ref.append((pr, r, res))
    say(f"batch with large-p FP32 jobs: {[(m, n, r, 10 * r) for m, n, r, _, _ in cases]}")
    b = R.Batch(ctx, jobs, R.rpca_opts_default(), None)
    st = R.rpca_batch_seed(b)
    assert st >= 0, ctx.last_error()
    R.rpca_batch_run(b)
    torch.cuda.synchronize()
    for k, (Md, L, S, dI, dJ) in enumerate(keep):
        pr, r, res = ref[k]
        st, info = R.rpca_batch_job_info(b, k)
        assert info.r_used == min(res.seed.rank, r) and info.filt_not_converged == 0
        Lh = L[:, :pr.m].double().cpu().numpy().T
        Sh = S[:, :pr.m].double().cpu().numpy().T
        eL, eS = relF(Lh, res.L), relF(Sh, res.S)
        say(f"ERR batch large-p job {k} relL={eL:.3e} relS={eS:.3e}")
        assert eL <= REL_TOL and eS <= REL_TOL, (k, eL, eS)
        assert support_mismatch(Sh, res.S, float(np.abs(pr.M).max())) == 0, k
    b.close()


def test_batch_graph_replays_are_bitwise_equal(R, ctx):
    import torch
    ref = _small_batch_reference()[9:]
    b, keep = _build(R, ctx, ref, R.rpca_batch_tuning_default(graph=1))
    R.rpca_batch_seed(b)
    outs = []
    for run in range(4):           # eager, capture + replay, replay, replay
        say(f"batch graph run {run}")
        for Md, L, S, dI, dJ in keep:
            L.fill_(float("nan"))
            S.fill_(float("nan"))
        torch.cuda.synchronize()
        R.rpca_batch_run(b)
        torch.cuda.synchronize()
        outs.append([(L.clone(), S.clone()) for Md, L, S, dI, dJ in keep])
        x = torch.randn(1 << 20, device="cuda").sum().item()   # unrelated eager work between runs
        assert np.isfinite(x)
    for run in range(1, 4):
        for k in range(len(keep)):
            m = ref[k][5].m                      # the padding rows stay NaN
            assert torch.equal(outs[run][k][0][:, :m], outs[0][k][0][:, :m]), (run, k)
            assert torch.equal(outs[run][k][1][:, :m], outs[0][k][1][:, :m]), (run, k)
    for k in range(len(keep)):
        _check_job(k, ref[k], *outs[3][k])
    b.close()


@pytest.mark.parametrize("tuning", [dict(order=1), dict(filter_waves_per_cu=1, recon_cols_per_wave=3),
                                    dict(lane_max_p=0), dict(lane_max_r=4, graph=0),
                                    dict(lane_split2_p=0, lane_split4_p=0),
                                    dict(lane_split2_p=32, lane_split4_p=32),
                                    dict(lane_split2_p=8, lane_split4_p=64)])
def test_batch_tunings_agree(R, ctx, tuning):
    # every launch shape and form choice gives the oracle's answer
    import torch
    ref = _small_batch_reference()[8:]          # both class groups, tile form, edge jobs
    say(f"batch tuning {tuning}")
    b, keep = _build(R, ctx, ref, R.rpca_batch_tuning_default(**tuning))
    R.rpca_batch_seed(b)
    R.rpca_batch_run(b)
    torch.cuda.synchronize()
    for k, (Md, L, S, dI, dJ) in enumerate(keep):
        _check_job(k, ref[k], L, S)
    b.close()


def test_batch_argument_errors(R, ctx):
    import torch
    ref = _small_batch_reference()[:1]
    spec, p, q, ldm, ldl, P, I, J, res = ref[0]
    Md = _upload(P, ldm)
    L = torch.empty((P.n, ldl), device="cuda")
    S = torch.empty((P.n, ldl), device="cuda")
    dI, dJ = dev_i64(I), dev_i64(J)
    o = _opts(R)

    def create(**kw):
        a = dict(M=Md, m=P.m, n=P.n, ldm=ldm, r=spec.r, seed_rows=dI, p=p, seed_cols=dJ, q=q,
                 L=L, ldl=ldl, S=S, lds=ldl)
        a.update(kw)
        return R.Batch(ctx, [R.job(**a)], o)

    for bad in (dict(r=0), dict(r=p + 1), dict(ldm=P.m - 1), dict(S=L), dict(p=P.m + 1),
                dict(seed_rows=dev_i64(I[::-1].copy()))):
        with pytest.raises(R.RpcaError) as e:
            create(**bad)
        assert e.value.status == R.RPCA_ERR_ARG, bad
        assert "batch job 0" in ctx.last_error()
    b = create()
    with pytest.raises(R.RpcaError) as e:     # run before seed
        R.rpca_batch_run(b)
    assert e.value.status == R.RPCA_ERR_ARG
    with pytest.raises(R.RpcaError):
        R.rpca_batch_job_info(b, 5)
    b.close()
    for bad in (dict(lane_max_p=81), dict(lane_split2_p=33), dict(lane_split2_p=20, lane_split4_p=10),
                dict(lane_split4_p=65), dict(order=2)):
        with pytest.raises(R.RpcaError) as e:
            R.Batch(ctx, [R.job(Md, P.m, P.n, ldm, spec.r, dI, p, dJ, q, L, ldl, S, ldl)], o,
                    R.rpca_batch_tuning_default(**bad))
        assert e.value.status == R.RPCA_ERR_ARG, bad


@pytest.mark.parametrize("m,n,r,p,q,seed", [(600, 500, 3, 30, 30, 1), (700, 900, 5, 50, 70, 2),
                                           (800, 400, 8, 80, 64, 3), (500, 700, 2, 40, 20, 4)])
def test_batched_seed_solver_matches_oracle(R, ctx, m, n, r, p, q, seed):
    # Well-conditioned seed blocks (Bernoulli +-1 corruptions, default
    # tolerances): the batched seed solver (one workgroup per problem, Jacobi
    # SVD) reaches the oracle's rank, iteration count and L^s; the one-by-one
    # route on the same batch agrees too.
    import torch
    pr = synth.lowrank_plus_sparse(m, n, r, factor_std=np.sqrt(1.0 / max(m, n)), sparsity=0.1,
                                   values="pm1", seed=seed)
    I, J = synth.seed_indices(m, n, p, q, seed=seed)
    sd = oracle.seed_pcp(pr.M[np.ix_(I, J)].astype(np.float64))
    kk = min(sd.rank, r)
    Ls_ref = (sd.U[:, :kk] * sd.sigma[:kk]) @ sd.V[:, :kk].T
    Md = _upload(pr, m)
    L = torch.empty_like(Md)
    S = torch.empty_like(Md)
    dI, dJ = dev_i64(I), dev_i64(J)
    for batched in (1, 0):
        say(f"seed solver m={m} n={n} r={r} p={p} q={q} batched={batched}")
        b = R.Batch(ctx, [R.job(Md, m, n, m, r, dI, p, dJ, q, L, m, S, m)], R.rpca_opts_default(),
                    R.rpca_batch_tuning_default(seed_batched=batched))
        st = R.rpca_batch_seed(b)
        st, info = R.rpca_batch_job_info(b, 0)
        assert info.r_used == kk and info.seed_iters == sd.iters, (info.r_used, info.seed_iters, sd.iters)
        U = torch.zeros((r, p), dtype=torch.float64, device="cuda")
        sg = torch.zeros(r, dtype=torch.float64, device="cuda")
        V = torch.zeros((r, q), dtype=torch.float64, device="cuda")
        R.rpca_batch_job_factors(b, 0, U, sg, V)
        Uh, sh, Vh = U.cpu().numpy().T, sg.cpu().numpy(), V.cpu().numpy().T
        Ls = (Uh * sh) @ Vh.T
        # the one-by-one route takes singular vectors from the eigenvectors of
        # the Gram matrix, which squares the spectrum (measured: up to 2e-8)
        assert relF(Ls, Ls_ref) <= (1e-9 if batched else 1e-7), relF(Ls, Ls_ref)
        assert np.allclose(Uh.T @ Uh, np.diag((sh > 0).astype(float)), atol=1e-12)
        assert np.allclose(Vh.T @ Vh, np.diag((sh > 0).astype(float)), atol=1e-12)
        assert np.all(np.diff(sh[:kk]) <= 0)
        b.close()
