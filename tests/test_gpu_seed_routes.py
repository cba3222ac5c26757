"""GPU parity of the seed PCP (Sec. 3.1, eq. SPCP) on every route of the
library's FP64 seed solver, against the oracle's inexact ALM with a full
LAPACK SVD in each step:

* the device-resident subspace-iteration solver (blocks above 6400 entries up
  to 512 x 512; seed_route = 2),
* the eigen-decomposition route (seed_route = 1, and the automatic choice for
  one such block alone),
* the batched form's seed launch on blocks of several sizes at once (the
  automatic choice there: LDS Jacobi for the small block, one subspace
  launch for the others).

Compared: the rank, the ALM step count (within one step) and L^s = U Sigma V^T
(relative Frobenius; never the factors themselves, which are defined up to
sign), and the route the library reports it took: the subspace solver holds
at most 72 directions, so it completes where the iterate never keeps more
than 64 singular values above the threshold and otherwise reports a
fallback to the eigen route.  The first ALM step, whose input is a multiple
of M^s (S_0 = 0, Y_0 proportional to M^s), keeps every singular value above
about 0.44 sigma_1 (69 of the 200 x 200 block's, 107 of the 500 x 500 one's)
and the later ones at most about the final rank, so the larger of the two
decides.  Ritz values never exceed the singular values they approximate, so
a peak of 64 or less never falls back; one of 68 or more does.  On blocks whose PCP recovers L^s the subspace route agrees with the
oracle to rounding (1e-9 asserted); the eigen route squares the spectrum and
is held to 1e-7.  Seed times are printed (``SEED`` lines).
"""
from __future__ import annotations

import functools
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev_i64, dev_matrix, relF, say

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


# (p, q, r, magnitude of the full matrix the block comes from, corruption rate, seed)
BLOCKS = {
    "c1_100": (100, 100, 10, 1000, 0.10, 1),
    "c2_200": (200, 200, 20, 10000, 0.10, 2),
    "c5C_300": (300, 300, 30, 20000, 0.10, 3),
    "c3_500": (500, 500, 50, 50000, 0.05, 4),
    "tall_250x120": (250, 120, 12, 5000, 0.08, 5),
    "wide_96x300": (96, 300, 9, 5000, 0.08, 6),
}


@functools.lru_cache(maxsize=None)
def block(name):
    p, q, r, big, rho, seed = BLOCKS[name]
    pr = synth.lowrank_plus_sparse(p, q, r, factor_std=np.sqrt(1.0 / big), sparsity=rho,
                                   values="pm1" if name != "c3_500" else "unif11", seed=seed)
    sd = oracle.seed_pcp(pr.M.astype(np.float64))
    return pr, r, sd


def first_svt_rank(M):
    """Singular values above the threshold in the first ALM step of the seed
    PCP (S_0 = 0, Y_0 = M / max(||M||_2, ||M||_inf / lam), tau = 1 / mu_0)."""
    M = np.asarray(M, dtype=np.float64)
    lam = 1.0 / np.sqrt(max(M.shape))
    s = np.linalg.svd(M, compute_uv=False)
    mu0 = 1.25 / s[0]
    y0 = 1.0 / max(s[0], np.abs(M).max() / lam)
    return int(np.sum(s * (1.0 + y0 / mu0) > 1.0 / mu0))


def expected_route(R, M, route, final_rank):
    """The route rpca_seed should report; None where either is right (a
    peak rank of 65 to 67, where convergence order decides)."""
    if route == 1:
        return R.RPCA_SEED_ROUTE_EIGEN
    peak = max(first_svt_rank(M), final_rank)
    if peak <= 64:
        return R.RPCA_SEED_ROUTE_SUBSPACE
    return R.RPCA_SEED_ROUTE_FELL_BACK if peak >= 68 else None


def _seed(R, ctx, pr, r, route):
    import torch
    p, q = pr.m, pr.n
    U = torch.zeros((r, p), dtype=torch.float64, device="cuda")
    sg = torch.zeros(r, dtype=torch.float64, device="cuda")
    V = torch.zeros((r, q), dtype=torch.float64, device="cuda")
    Md = dev_matrix(pr.M)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, ru, its = R.rpca_seed(ctx, Md, p, q, p, dev_i64(np.arange(p)), p, dev_i64(np.arange(q)), q, r,
                              R.rpca_opts_default(seed_route=route), U, sg, V)
    ms = (time.perf_counter() - t0) * 1e3
    Uh, sh, Vh = U.cpu().numpy().T, sg.cpu().numpy(), V.cpu().numpy().T
    return st, ru, its, (Uh * sh) @ Vh.T, Uh, sh, ms


@pytest.mark.parametrize("name", sorted(BLOCKS))
@pytest.mark.parametrize("route", [2, 1])
def test_seed_route_matches_oracle(R, ctx, name, route):
    pr, r, sd = block(name)
    k = min(sd.rank, r)
    Ls_ref = (sd.U[:, :k] * sd.sigma[:k]) @ sd.V[:, :k].T
    _seed(R, ctx, pr, r, route)                                   # warm-up (code objects, workspace)
    st, ru, its, Ls, Uh, sh, ms = _seed(R, ctx, pr, r, route)
    taken = R.rpca_last_seed_route(ctx)
    e = relF(Ls, Ls_ref)
    say(f"SEED {name} route={route} p={pr.m} q={pr.n} status={R.rpca_status_string(st)} rank={ru}/"
        f"{sd.rank} iters={its}/{sd.iters} relF(L^s)={e:.2e} t={ms:.1f} ms taken={taken} "
        f"first-step rank={first_svt_rank(pr.M)}")
    want = expected_route(R, pr.M, route, sd.rank)
    assert want is None or taken == want
    assert st >= 0
    assert ru == k
    assert abs(its - sd.iters) <= 1
    assert e <= (1e-9 if taken == R.RPCA_SEED_ROUTE_SUBSPACE else 1e-7)
    assert np.allclose(Uh[:, :k].T @ Uh[:, :k], np.eye(k), atol=1e-10)
    assert np.all(np.diff(sh[:k]) <= 0) and np.all(sh[k:] == 0)


def test_batched_seeds_of_several_sizes(R, ctx):
    # One batch with seed blocks of 50^2 (LDS Jacobi), 100^2 and 300^2
    # (subspace iteration, one launch) and 200 x 160: each job's L^s against
    # the oracle's seed PCP of its block.
    import torch
    specs = [(600, 600, 5, 50, 50), (2000, 500, 10, 100, 100), (3000, 3000, 30, 300, 300),
             (1500, 1200, 16, 200, 160)]
    keep, jobs, refs = [], [], []
    for k, (m, n, r, p, q) in enumerate(specs):
        pr = synth.lowrank_plus_sparse(m, n, r, factor_std=np.sqrt(1.0 / max(m, n)), sparsity=0.1,
                                       values="pm1", seed=40 + k)
        I, J = synth.seed_indices(m, n, p, q, seed=40 + k)
        sd = oracle.seed_pcp(pr.M[np.ix_(I, J)].astype(np.float64))
        refs.append((pr, I, J, r, sd))
        Md = dev_matrix(pr.M)
        L = torch.empty_like(Md)
        S = torch.empty_like(Md)
        dI, dJ = dev_i64(I), dev_i64(J)
        keep.append((Md, L, S, dI, dJ))
        jobs.append(R.job(Md, m, n, m, r, dI, p, dJ, q, L, m, S, m))
    b = R.Batch(ctx, jobs, R.rpca_opts_default())
    t0 = time.perf_counter()
    R.rpca_batch_seed(b)
    say(f"SEED batch of {len(jobs)} blocks: {1e3 * (time.perf_counter() - t0):.1f} ms")
    for k, (pr, I, J, r, sd) in enumerate(refs):
        p, q = len(I), len(J)
        U = torch.zeros((r, p), dtype=torch.float64, device="cuda")
        sg = torch.zeros(r, dtype=torch.float64, device="cuda")
        V = torch.zeros((r, q), dtype=torch.float64, device="cuda")
        R.rpca_batch_job_factors(b, k, U, sg, V)
        st, info = R.rpca_batch_job_info(b, k)
        Ms = pr.M[np.ix_(I, J)]
        want = (R.RPCA_SEED_ROUTE_LDS_JACOBI if p * q <= 6400
                else expected_route(R, Ms, 2, sd.rank))
        kk = min(sd.rank, r)
        Ls = (U.cpu().numpy().T * sg.cpu().numpy()) @ V.cpu().numpy()
        Ls_ref = (sd.U[:, :kk] * sd.sigma[:kk]) @ sd.V[:, :kk].T
        e = relF(Ls, Ls_ref)
        say(f"SEED batch job {k} p={p} q={q} rank={info.r_used}/{sd.rank} iters={info.seed_iters}/"
            f"{sd.iters} relF(L^s)={e:.2e} route={info.seed_route} first-step rank={first_svt_rank(Ms)}")
        assert info.r_used == kk and abs(info.seed_iters - sd.iters) <= 1
        assert want is None or info.seed_route == want
        assert e <= (1e-7 if info.seed_route == R.RPCA_SEED_ROUTE_FELL_BACK else 1e-9)
    b.close()


def _seed_block(R, ctx, Mblk, r, route):
    """rpca_seed on the whole block (identity seed indices); status, rank,
    iterations, L^s."""
    import torch
    p, q = Mblk.shape
    Md = dev_matrix(np.asfortranarray(Mblk.astype(np.float32)))
    U = torch.zeros((r, p), dtype=torch.float64, device="cuda")
    sg = torch.zeros(r, dtype=torch.float64, device="cuda")
    V = torch.zeros((r, q), dtype=torch.float64, device="cuda")
    st, ru, its = R.rpca_seed(ctx, Md, p, q, p, dev_i64(np.arange(p)), p, dev_i64(np.arange(q)), q, r,
                              R.rpca_opts_default(seed_route=route), U, sg, V)
    Uh, sh, Vh = U.cpu().numpy().T, sg.cpu().numpy(), V.cpu().numpy().T
    return st, ru, its, (Uh * sh) @ Vh.T, R.rpca_last_seed_route(ctx)


def _against_oracle(R, name, Mblk, st, ru, its, Ls, taken, r, tol):
    sd = oracle.seed_pcp(Mblk.astype(np.float32).astype(np.float64))
    want = expected_route(R, Mblk, 2, sd.rank)
    k = min(sd.rank, r)
    Ls_ref = (sd.U[:, :k] * sd.sigma[:k]) @ sd.V[:, :k].T
    e = relF(Ls, Ls_ref)
    say(f"SEED {name} p={Mblk.shape[0]} q={Mblk.shape[1]} rank={ru}/{sd.rank} iters={its}/{sd.iters} "
        f"relF(L^s)={e:.2e} route={taken}")
    assert want is None or taken == want
    assert st >= 0 and ru == k and abs(its - sd.iters) <= 1
    assert e <= tol


def test_subspace_route_falls_back_past_its_widest_basis(R, ctx):
    # A 200 x 200 block of rank 90 with few corruptions: the iterate keeps
    # more than the 72 directions the subspace solver holds, so it reports a
    # fallback and the eigen route finishes (held to that route's 1e-7).
    pr = synth.lowrank_plus_sparse(200, 200, 90, factor_std=0.1, sparsity=0.02, values="pm1", seed=11)
    st, ru, its, Ls, taken = _seed_block(R, ctx, pr.M, 120, 2)
    _against_oracle(R, "fallback_rank90", pr.M, st, ru, its, Ls, taken, 120, 1e-7)
    assert ru > 64 and taken == R.RPCA_SEED_ROUTE_FELL_BACK


@pytest.mark.parametrize("shape", [(512, 81), (81, 512)])
def test_subspace_route_at_its_size_limits(R, ctx, shape):
    p, q = shape
    pr = synth.lowrank_plus_sparse(p, q, 8, factor_std=np.sqrt(1.0 / 5000), sparsity=0.08, values="pm1",
                                   seed=12 + p)
    st, ru, its, Ls, taken = _seed_block(R, ctx, pr.M, 8, 2)
    _against_oracle(R, f"limit_{p}x{q}", pr.M, st, ru, its, Ls, taken, 8, 1e-9)


def test_subspace_route_rank_one(R, ctx):
    # the basis starts 16 wide for a rank-1 block
    pr = synth.lowrank_plus_sparse(120, 150, 1, factor_std=0.05, sparsity=0.1, values="pm1", seed=13)
    st, ru, its, Ls, taken = _seed_block(R, ctx, pr.M, 1, 2)
    _against_oracle(R, "rank1_120x150", pr.M, st, ru, its, Ls, taken, 1, 1e-9)


@pytest.mark.parametrize("case", ["zero", "nan"])
def test_subspace_route_error_paths(R, ctx, case):
    Mblk = np.zeros((120, 110), dtype=np.float32)
    if case == "nan":
        Mblk = synth.lowrank_plus_sparse(120, 110, 4, factor_std=0.05, sparsity=0.1, values="pm1",
                                         seed=14).M.copy()
        Mblk[17, 33] = np.nan
    with pytest.raises(R.RpcaError) as ei:
        _seed_block(R, ctx, Mblk, 4, 2)
    want = R.RPCA_ERR_SEED if case == "zero" else R.RPCA_ERR_NUMERIC
    say(f"SEED error path {case}: {ei.value}")
    assert ei.value.status == want


def test_batched_eigen_route_seeds_side_by_side(R, ctx):
    # Four 120 x 120 seed blocks with seed_route = 1: all take the eigen route,
    # which a batch runs on helper contexts side by side.  Each job against
    # the oracle, and bit for bit against the same job alone in a batch (one
    # block: no helpers), so the result does not depend on the batch.
    import torch
    specs = [(1200, 1000, 12, 120, 120, 60 + k) for k in range(4)]
    built = []
    for m, n, r, p, q, sd_seed in specs:
        pr = synth.lowrank_plus_sparse(m, n, r, factor_std=np.sqrt(1.0 / max(m, n)), sparsity=0.1,
                                       values="pm1", seed=sd_seed)
        I, J = synth.seed_indices(m, n, p, q, seed=sd_seed)
        Md = dev_matrix(pr.M)
        built.append((pr, I, J, r, Md, dev_i64(I), dev_i64(J)))
    opts = R.rpca_opts_default(seed_route=1)

    def run(items):
        keep, jobs = [], []
        for pr, I, J, r, Md, dI, dJ in items:
            L = torch.empty_like(Md)
            S = torch.empty_like(Md)
            keep.append((L, S))
            jobs.append(R.job(Md, pr.m, pr.n, pr.m, r, dI, len(I), dJ, len(J), L, pr.m, S, pr.m))
        b = R.Batch(ctx, jobs, opts)
        R.rpca_batch_seed(b)
        out = []
        for k, (pr, I, J, r, Md, dI, dJ) in enumerate(items):
            U = torch.zeros((r, len(I)), dtype=torch.float64, device="cuda")
            sg = torch.zeros(r, dtype=torch.float64, device="cuda")
            V = torch.zeros((r, len(J)), dtype=torch.float64, device="cuda")
            R.rpca_batch_job_factors(b, k, U, sg, V)
            st, info = R.rpca_batch_job_info(b, k)
            out.append((U.cpu().numpy(), sg.cpu().numpy(), V.cpu().numpy(), info.seed_route, info.r_used,
                        info.seed_iters))
        b.close()
        return out

    together = run(built)
    for k, (pr, I, J, r, Md, dI, dJ) in enumerate(built):
        Uh, sh, Vh, route, ru, its = together[k]
        sd = oracle.seed_pcp(pr.M[np.ix_(I, J)].astype(np.float64))
        kk = min(sd.rank, r)
        Ls = (Uh.T * sh) @ Vh
        Ls_ref = (sd.U[:, :kk] * sd.sigma[:kk]) @ sd.V[:, :kk].T
        e = relF(Ls, Ls_ref)
        say(f"SEED eigen side by side job {k}: rank={ru}/{sd.rank} iters={its}/{sd.iters} relF(L^s)={e:.2e} "
            f"route={route}")
        assert route == R.RPCA_SEED_ROUTE_EIGEN
        assert ru == kk and abs(its - sd.iters) <= 1 and e <= 1e-7
        alone = run([built[k]])[0]
        assert np.array_equal(alone[0], Uh) and np.array_equal(alone[1], sh) and np.array_equal(alone[2], Vh)
