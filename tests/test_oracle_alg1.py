"""Pins for the FP64 reference of Algorithm 1 (the l1 regression of eq. l1g).

Each test checks the reference against something it does not compute itself:
a hand-worked fixture, an exhaustive search, a closed form, or an invariant
that the mathematics fixes.
"""
import json
import pathlib

import numpy as np
import pytest

import oracle

GOLDEN = pathlib.Path(__file__).parent / "golden"


# Fixed-step setting used to pin the iteration itself: the stopping test is
# switched off (eps = 0 runs exactly max_iter steps) and beta stays bounded, so
# sum 1/beta_k diverges and the ADM converges to the LAD optimum.
PIN = oracle.Alg1Params(eps=0.0, rho=1.1, beta_max_scale=10.0, max_iter=20000)


def _orth(p, r, rng):
    Q, _ = np.linalg.qr(rng.standard_normal((p, r)))
    return Q


def test_soft_threshold_golden():
    d = json.loads((GOLDEN / "soft_threshold.json").read_text())
    for t, tau, want in d["cases"]:
        assert oracle.soft_threshold(t, tau) == want


def test_soft_threshold_is_the_l1_prox():
    # S_tau(t) must minimise tau|x| + (x - t)^2 / 2: compare with a fine grid.
    rng = np.random.default_rng(3)
    grid = np.linspace(-6, 6, 240001)
    for _ in range(40):
        t, tau = rng.uniform(-5, 5), rng.uniform(0.01, 3)
        f = tau * np.abs(grid) + 0.5 * (grid - t) ** 2
        assert abs(oracle.soft_threshold(t, tau) - grid[np.argmin(f)]) <= 1e-4


def test_rank1_golden_weighted_median():
    d = json.loads((GOLDEN / "lad_rank1.json").read_text())
    for case in d["cases"]:
        a = np.array(case["A"])
        A = (a / np.linalg.norm(a))[:, None]
        x = np.array(case["x"])
        z, e, y, K = oracle.alg1(x, A, PIN)
        assert abs(z[0] - case["z"]) <= 1e-7 * max(1.0, abs(case["z"]))
        assert abs(np.abs(x - A[:, 0] * z[0]).sum() - case["value"]) <= 1e-7 * case["value"]


def test_rank1_random_weighted_median():
    # r = 1: argmin_z sum |x_i - a_i z| is the weighted median of x_i / a_i
    # with weights |a_i| (rescaled by ||a||).
    rng = np.random.default_rng(11)
    for p in (5, 8, 13, 30):
        a = rng.standard_normal(p)
        a /= np.linalg.norm(a)
        x = rng.standard_normal(p) * 0.1
        x[rng.choice(p, p // 4, replace=False)] += rng.choice([-5.0, 5.0], p // 4)
        lo, hi = oracle.weighted_median(x / a, np.abs(a))
        z, _, _, K = oracle.alg1(x, a[:, None], PIN)
        assert lo - 1e-9 <= z[0] <= hi + 1e-9


@pytest.mark.parametrize("p,r", [(6, 1), (8, 2), (10, 2), (12, 3), (9, 3)])
def test_matches_bruteforce_lad(p, r):
    # Exhaustive vertex enumeration of the LAD linear program on tiny sizes.
    rng = np.random.default_rng(100 + 7 * p + r)
    for trial in range(6):
        A = _orth(p, r, rng)
        z0 = rng.standard_normal(r)
        x = A @ z0 + 0.05 * rng.standard_normal(p)
        bad = rng.choice(p, max(1, p // 5), replace=False)
        x[bad] += rng.uniform(-4, 4, bad.size)
        best, sols = oracle.lad_bruteforce(x, A)
        z, e, y, K = oracle.alg1(x, A, PIN)
        f = np.abs(x - A @ z).sum()
        assert f <= best * (1 + 1e-10) + 1e-12
        if len(sols) == 1:
            assert np.allclose(z, sols[0], rtol=1e-8, atol=1e-9)


def test_stopping_rule_sees_primal_feasibility_only():
    # Algorithm 1 stops on ||X - AZ - E||_inf alone.  On a 3-point problem every
    # entry is clipped after a few steps, Y stops changing, the residual is
    # exactly 0 and the loop ends although Z has not reached the optimum (z = 3
    # for the second hand-worked case).  In the regime of l1 filtering (p >> r,
    # sparse corruption) clean entries stay unclipped and this does not occur.
    a = np.array([1.0, 2.0, 2.0])
    x = np.array([3.0, 2.0, -4.0])
    z, e, y, K = oracle.alg1(x, (a / 3.0)[:, None])
    assert 0 < K < 10 and abs(z[0] - 3.0) > 0.5
    assert np.abs(x - (a / 3.0) * z[0] - e).max() <= 1e-15 * 8


def test_no_corruption_returns_projection():
    # x = A z0 exactly: the minimum is 0 at z0 = A^T x and e = 0.
    rng = np.random.default_rng(5)
    for p, r in [(20, 3), (100, 10), (200, 20)]:
        A = _orth(p, r, rng)
        z0 = rng.standard_normal(r)
        x = A @ z0
        z, e, y, K = oracle.alg1(x, A)
        assert K > 0
        assert np.allclose(z, z0, rtol=0, atol=1e-9 * np.abs(z0).max())
        assert np.abs(e).max() <= 1e-8 * np.abs(x).max()


def test_exact_recovery_of_sparse_corruption():
    # Sec. 3.5: with few corrupted entries the regression recovers z0 exactly.
    rng = np.random.default_rng(7)
    p, r = 200, 20
    A = _orth(p, r, rng)
    for _ in range(5):
        z0 = rng.standard_normal(r) * 0.01
        s = np.zeros(p)
        idx = rng.choice(p, 20, replace=False)
        s[idx] = rng.choice([-1.0, 1.0], 20)
        x = A @ z0 + s
        z, e, y, K = oracle.alg1(x, A)
        assert K > 0
        assert np.linalg.norm(z - z0) <= 1e-7 * np.linalg.norm(z0)
        # e recovers the corruption
        assert np.abs(e - s).max() <= 1e-7


def test_dual_invariants_and_kkt():
    # A^T Y_k = 0 for every k >= 1 (Step 2 makes it so when A^T A = I), at any
    # stopping point.  Run to convergence, y certifies optimality of the LAD
    # problem: |y| <= 1 and y = sgn(e) where e is nonzero.
    rng = np.random.default_rng(9)
    p, r = 120, 12
    A = _orth(p, r, rng)
    for _ in range(5):
        x = A @ rng.standard_normal(r) * 0.01
        idx = rng.choice(p, 15, replace=False)
        x[idx] += rng.uniform(-1, 1, 15)
        z, e, y, K = oracle.alg1(x, A)
        assert np.abs(A.T @ y).max() <= 1e-10
        z, e, y, K = oracle.alg1(x, A, PIN)
        stat, feas, comp = oracle.lad_kkt(x, A, z, e, y, tol=1e-9)
        assert stat <= 1e-10
        assert feas <= 1e-9
        assert comp <= 1e-9


def test_rotation_invariance():
    # Replacing A by A Q (Q orthogonal) maps every iterate Z -> Q^T Z and leaves
    # E and Y unchanged, so results compared through A z are basis-free.
    rng = np.random.default_rng(13)
    p, r = 80, 8
    A = _orth(p, r, rng)
    Q = _orth(r, r, rng)
    x = A @ rng.standard_normal(r)
    x[rng.choice(p, 10, replace=False)] += 3.0
    z1, e1, y1, K1 = oracle.alg1(x, A)
    z2, e2, y2, K2 = oracle.alg1(x, A @ Q)
    assert K1 == K2
    assert np.allclose(Q @ z2, z1, atol=1e-12 * np.abs(x).max() * 100)
    assert np.allclose(e1, e2, atol=1e-10)
    assert np.allclose(y1, y2, atol=1e-8)


def test_literal_and_clip_forms_agree():
    # The clip rewrite must reproduce the literal iteration; with the stopping
    # test disabled (eps = 0) both run exactly max_iter steps.
    rng = np.random.default_rng(17)
    prm = oracle.Alg1Params(eps=0.0, max_iter=40)
    for p, r in [(50, 5), (200, 20)]:
        A = _orth(p, r, rng)
        x = A @ rng.standard_normal(r) * 0.01
        x[rng.choice(p, p // 10, replace=False)] += rng.choice([-1.0, 1.0], p // 10)
        z1, e1, y1, K1 = oracle.alg1(x, A, prm, form="literal")
        z2, e2, y2, K2 = oracle.alg1(x, A, prm, form="clip")
        assert K1 == K2 == -40
        assert np.abs(z1 - z2).max() <= 1e-12 * max(1.0, np.abs(z1).max()) * 10
        assert np.abs(e1 - e2).max() <= 1e-11
        assert np.abs(y1 - y2).max() <= 1e-9
    # with the default stopping test they take the same number of steps
    A = _orth(200, 20, rng)
    X = A @ rng.standard_normal((20, 64)) * 0.01
    X[rng.random(X.shape) < 0.1] += 1.0
    Z1, K1 = oracle.alg1_batch(X, A, form="literal")
    Z2, K2 = oracle.alg1_batch(X, A, form="clip")
    assert (np.abs(K1 - K2) <= 1).all()
    assert np.linalg.norm(A @ (Z1 - Z2)) <= 1e-6 * np.linalg.norm(A @ Z1)


def test_padding_is_exact():
    # Zero rows appended to (x, A) and zero columns appended to A change
    # nothing: the extra z entries stay 0 and the rest is identical.
    rng = np.random.default_rng(19)
    p, r = 37, 5
    A = _orth(p, r, rng)
    x = A @ rng.standard_normal(r)
    x[rng.choice(p, 5, replace=False)] += 2.0
    z, e, y, K = oracle.alg1(x, A)
    Ap = np.zeros((48, 8))
    Ap[:p, :r] = A
    xp = np.zeros(48)
    xp[:p] = x
    zp, ep, yp, Kp = oracle.alg1(xp, Ap)
    assert K == Kp
    assert np.array_equal(zp[r:], np.zeros(3))
    assert np.allclose(zp[:r], z, rtol=0, atol=1e-13)
    assert np.array_equal(ep[p:], np.zeros(48 - p))


def test_edge_cases():
    rng = np.random.default_rng(23)
    A = _orth(30, 3, rng)
    z, e, y, K = oracle.alg1(np.zeros(30), A)
    assert K == 0 and not z.any() and not e.any()
    x = A @ np.ones(3)
    x[0] += 10
    z, e, y, K = oracle.alg1(x, A, oracle.Alg1Params(max_iter=1))
    assert K == -1          # not converged after one step: flagged negative
    Z, K = oracle.alg1_batch(np.zeros((30, 0)), A)
    assert Z.shape == (3, 0) and K.shape == (0,)


def test_batch_equals_single():
    rng = np.random.default_rng(29)
    p, r = 60, 6
    A = _orth(p, r, rng)
    X = A @ rng.standard_normal((r, 33))
    X[rng.random(X.shape) < 0.1] -= 2.0
    Z, K = oracle.alg1_batch(X, A, nthreads=3)
    for j in range(X.shape[1]):
        z, _, _, k = oracle.alg1(X[:, j], A)
        assert k == K[j]
        assert np.array_equal(z, Z[:, j])


def test_scale_equivariance():
    # Scaling x by c > 0 scales z and e by c, leaves y and the iteration count
    # unchanged: beta_0 scales by 1/c and the stopping test is relative to
    # ||x||_inf.
    rng = np.random.default_rng(31)
    p, r = 100, 10
    A = _orth(p, r, rng)
    x = A @ rng.standard_normal(r) * 0.01
    x[rng.choice(p, 10, replace=False)] += 1.0
    z, e, y, K = oracle.alg1(x, A)
    for c in (1e-3, 1e3):
        zc, ec, yc, Kc = oracle.alg1(c * x, A)
        assert Kc == K
        assert np.allclose(zc, c * z, rtol=1e-9, atol=1e-12 * c)
        assert np.allclose(yc, y, atol=1e-7)
