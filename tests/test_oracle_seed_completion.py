"""Pins for the FP64 reference of the seed PCP (eq. SPCP), the completion
(eqs. l1s / l1s') and Algorithm 2 end to end."""
import json
import pathlib

import numpy as np
import pytest

import oracle
import synth

GOLDEN = pathlib.Path(__file__).parent / "golden"


# ----------------------------------------------------------------- SVT
def test_svt_golden():
    d = json.loads((GOLDEN / "svt_diag.json").read_text())
    for c in d["cases"]:
        A, *_ = oracle.svt(np.array(c["W"]), c["eta"])
        assert np.allclose(A, np.array(c["A"]), atol=1e-14)


def test_svt_is_the_nuclear_prox():
    # Optimality of A = SVT_eta(W) for eta||A||_* + 1/2||A - W||^2:
    # (W - A)/eta = U V^T + R with U^T R = 0, R V = 0 and ||R||_2 <= 1.
    rng = np.random.default_rng(1)
    for (m, n) in [(6, 4), (10, 10), (30, 12)]:
        W = rng.standard_normal((m, n))
        s = np.linalg.svd(W, compute_uv=False)
        eta = float(np.median(s))
        A, U, sk, Vt = oracle.svt(W, eta)
        G = (W - A) / eta
        R = G - U @ Vt
        assert np.abs(U.T @ R).max() <= 1e-12
        assert np.abs(R @ Vt.T).max() <= 1e-12
        assert np.linalg.norm(R, 2) <= 1 + 1e-12
        # and it beats random perturbations
        f = lambda B: eta * np.linalg.svd(B, compute_uv=False).sum() + 0.5 * np.linalg.norm(B - W) ** 2
        f0 = f(A)
        for _ in range(20):
            assert f(A + 1e-3 * rng.standard_normal(A.shape)) >= f0


# ----------------------------------------------------------------- PCP / seed
def test_pcp_large_lambda_keeps_everything_low_rank():
    # If lam >= ||U V^T||_inf (M = U S V^T full rank), Y = U V^T certifies
    # L = M, S = 0 as the PCP optimum.
    rng = np.random.default_rng(2)
    M = rng.standard_normal((20, 15))
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    lam = 2.0 * np.abs(U @ Vt).max()
    res = oracle.pcp_ialm(M, lam, oracle.SeedParams(tol=1e-12, max_iter=3000))
    assert np.abs(res.S).max() <= 1e-8
    assert oracle.relerr(res.L, M) <= 1e-8


def test_pcp_small_lambda_keeps_everything_sparse():
    # If ||lam sgn(M)||_2 <= 1 (M with no zero entry), Y = lam sgn(M)
    # certifies L = 0, S = M.
    rng = np.random.default_rng(3)
    M = rng.standard_normal((20, 15))
    lam = 0.5 / np.linalg.norm(np.sign(M), 2)
    res = oracle.pcp_ialm(M, lam, oracle.SeedParams(tol=1e-12, max_iter=3000))
    assert np.abs(res.L).max() <= 1e-8 * np.abs(M).max()
    assert oracle.relerr(res.S, M) <= 1e-8


def test_seed_exact_recovery_and_kkt():
    # Well inside PCP's recovery region: rank 5 of 200, 5% corruptions.
    pr = synth.lowrank_plus_sparse(200, 200, 5, factor_std=np.sqrt(1 / 200), sparsity=0.05,
                                   values="pm1", seed=4, exact_count=True)
    Ms = pr.M.astype(np.float64)
    res = oracle.seed_pcp(Ms)
    assert res.converged and res.rank == 5
    assert oracle.relerr(res.L, pr.L0()) <= 1e-6
    # factors reproduce L^s and are orthonormal
    assert np.allclose(res.U.T @ res.U, np.eye(5), atol=1e-12)
    assert np.allclose(res.V.T @ res.V, np.eye(5), atol=1e-12)
    assert oracle.relerr((res.U * res.sigma) @ res.V.T, res.L) <= 1e-12
    kkt = oracle.pcp_kkt(Ms, res.L, res.S, res.Y, res.lam, res.YL)
    assert kkt["orth"] <= 1e-8 and kkt["spec"] <= 1 + 1e-8
    assert kkt["on_support"] <= 1e-8 and kkt["off_support"] <= 1e-8
    assert kkt["gap"] <= 1e-2


# ----------------------------------------------------------------- completion
def test_nystrom_golden():
    d = json.loads((GOLDEN / "nystrom_rank1.json").read_text())
    L0 = np.array(d["L0"])
    L, S = oracle.complete(L0, d["seed_rows"], d["seed_cols"], np.array(d["U"]),
                           np.array(d["sigma"]), np.array(d["V"]), np.array(d["Qt"]),
                           np.array(d["Pt"]))
    assert np.array_equal(L[1:, 1:], np.array(d["L_complement"]))
    assert np.array_equal(L, L0) and not S.any()


def test_nystrom_identity_against_pinv():
    # eq. l1s' (P~^T Sigma^-1 Q~) equals eq. l1s (L^r (L^s)^+ L^c) with the
    # pseudo-inverse from LAPACK.
    rng = np.random.default_rng(5)
    m, n, r = 60, 50, 4
    L0 = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    I = np.sort(rng.choice(m, 12, replace=False))
    J = np.sort(rng.choice(n, 10, replace=False))
    Ic, Jc = oracle.complement(I, m), oracle.complement(J, n)
    Ls = L0[np.ix_(I, J)]
    U, s, Vt = np.linalg.svd(Ls, full_matrices=False)
    U, s, V = U[:, :r], s[:r], Vt[:r].T
    Qt = U.T @ L0[np.ix_(I, Jc)]
    Pt = V.T @ L0[np.ix_(Ic, J)].T
    L, S = oracle.complete(L0, I, J, U, s, V, Qt, Pt)
    ref = L0[np.ix_(Ic, J)] @ np.linalg.pinv(Ls) @ L0[np.ix_(I, Jc)]
    assert oracle.relerr(L[np.ix_(Ic, Jc)], ref) <= 1e-11
    # CUR identity on exact rank-r data: the whole matrix comes back
    assert oracle.relerr(L, L0) <= 1e-11
    assert np.abs(S).max() <= 1e-11 * np.abs(L0).max()
    # entry-by-entry evaluation agrees with the assembled blocks
    rows = rng.integers(0, m, 200)
    cols = rng.integers(0, n, 200)
    e = oracle.complete_entries(rows, cols, I, J, m, n, U, s, V, Qt, Pt)
    assert np.allclose(e, L[rows, cols], rtol=1e-12, atol=1e-12)


# ----------------------------------------------------------------- end to end
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_c1_exact_recovery(seed):
    # m = n = 1000, r = 10, 10% +-1 corruptions, 100 x 100 seed.
    pr = synth.config_problem("c1", seed=seed)
    I, J = synth.seed_indices(1000, 1000, 100, 100, seed=seed)
    res = oracle.solve(pr.M, 10, I, J)
    assert res.seed.rank == 10
    assert (res.col_iters > 0).all() and (res.row_iters > 0).all()
    assert oracle.relerr(res.L, pr.L0()) <= 1e-6
    assert np.array_equal(res.S, pr.M.astype(np.float64) - res.L)
    # the support of S is that of S0
    tau = 1e-3 * np.abs(pr.M).max()
    assert np.array_equal(np.abs(res.S) > tau, pr.support)


def test_c1_seed_failure_is_visible_as_rank_mismatch():
    # At c1 the 100 x 100 seed sits close to PCP's recovery boundary; draw 4
    # is one where the seed PCP does not recover L^s, and the rank of the
    # recovered seed exceeds the target rank.
    pr = synth.config_problem("c1", seed=4)
    I, J = synth.seed_indices(1000, 1000, 100, 100, seed=4)
    sd = oracle.seed_pcp(pr.M[np.ix_(I, J)].astype(np.float64))
    assert sd.rank != 10


@pytest.mark.slow
def test_c1_agrees_with_full_matrix_pcp():
    # The full PCP with lam = 1/sqrt(1000) on all of M reaches the same L.
    pr = synth.config_problem("c1", seed=1)
    I, J = synth.seed_indices(1000, 1000, 100, 100, seed=1)
    res = oracle.solve(pr.M, 10, I, J)
    full = oracle.pcp_ialm(pr.M.astype(np.float64), 1 / np.sqrt(1000), oracle.SeedParams(tol=1e-9))
    assert full.rank == 10
    assert oracle.relerr(res.L, full.L) <= 1e-6


def test_generator_matches_table1_magnitudes():
    # Table 1: with N(0,1) factors ||L0||_* is close to r*m (39546 for
    # m = 2000, r = 20); the support count is exact.
    pr = synth.lowrank_plus_sparse(2000, 2000, 20, factor_std=1.0, sparsity=0.01,
                                   values="unif500", seed=1, exact_count=True)
    nuc = np.linalg.svd(pr.L0(), compute_uv=False).sum()
    assert abs(nuc - 40000) / 40000 <= 0.02
    assert pr.support.sum() == 40000


# ----------------------------------------------------------------- new columns (online filtering)
def _appended_problem(seed):
    # one low-rank model for 1200 columns: the first 1000 are fitted, the last
    # 200 arrive afterwards (c1 shapes and corruption law)
    pr = synth.lowrank_plus_sparse(1000, 1200, 10, factor_std=np.sqrt(1.0 / 1000), sparsity=0.10,
                                   values="pm1", seed=seed, exact_count=True)
    return pr, pr.M[:, :1000], np.asfortranarray(pr.M[:, 1000:])


@pytest.mark.parametrize("seed", [1, 2])
def test_new_columns_recover_the_low_rank_part(seed):
    # The paper's exact recoverability (Sec. 3.5): with the seed recovered,
    # each new column's filtering returns the true coefficients, so the
    # completed columns equal L0's new columns and S their corruptions.
    pr, M0, Mnew = _appended_problem(seed)
    I, J = synth.seed_indices(1000, 1000, 100, 100, seed=seed)
    fit = oracle.solve(M0, 10, I, J, assemble=False)
    assert fit.seed.rank == 10
    Qn, kn = oracle.filter_cols(Mnew, I, np.arange(200), fit.U)
    assert (kn > 0).all()
    L, S = oracle.complete_new_cols(Mnew, I, fit.U, fit.sigma, fit.Pt, Qn)
    L0 = pr.L0()[:, 1000:]
    assert oracle.relerr(L, L0) <= 1e-6
    tau = 1e-3 * np.abs(pr.M).max()
    assert np.array_equal(np.abs(S) > tau, pr.support[:, 1000:])


def test_new_columns_match_the_whole_matrix_fit():
    # Filtering a column later gives what the fit of the whole matrix gives
    # it: with the seed columns among the first 1000, the last 200 columns of
    # the 1200-column solve are non-seed columns completed by eq. l1s'.
    pr, M0, Mnew = _appended_problem(3)
    I, J = synth.seed_indices(1000, 1000, 100, 100, seed=3)
    fit = oracle.solve(M0, 10, I, J, assemble=False)
    Qn, _ = oracle.filter_cols(Mnew, I, np.arange(200), fit.U)
    L, S = oracle.complete_new_cols(Mnew, I, fit.U, fit.sigma, fit.Pt, Qn)
    whole = oracle.solve(pr.M, 10, I, J)
    assert np.abs(whole.L[:, 1000:] - L).max() <= 1e-12 * np.abs(L).max()
    # a planted mistake (Sigma instead of Sigma^-1 on the Nystrom rows) is seen
    Lbad = L.copy()
    Ic = oracle.complement(I, 1000)
    Lbad[Ic, :] = (fit.Pt.T * fit.sigma) @ Qn
    assert oracle.relerr(Lbad, pr.L0()[:, 1000:]) > 1e-2
