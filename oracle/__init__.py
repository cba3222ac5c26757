"""FP64 CPU reference ("oracle") for l1 filtering -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  The GPU library (``paper_1108_5359_amd``) never imports, links
or runs anything here, and this package never imports the GPU library: the
two share no code.  The only module both read is ``synth`` (seeded inputs).

It follows Liu, Lin, Wei, Su, "Solving Principal Component Pursuit in Linear
Time via l1 Filtering" step by step (Algorithm 2):

1. seed rows/columns are inputs (drawn by the caller, Sec. 3.1);
2. the seed PCP (eq. SPCP) by the inexact augmented Lagrange multiplier /
   alternating direction method with singular value thresholding
   (Sec. 2, eqs. Proxy and SVT; the paper defers the pseudo-code to its
   reference on ALM, so the reading used is spelled out in ``seed_pcp``);
3. column l1 filtering (eq. l1c') and 4. row l1 filtering (eq. l1r'), each
   regression solved by Algorithm 1 (the C file ``alg1.c``);
5. the Nystrom completion of the remaining block (eq. l1s') and
   ``S = M - L`` (Algorithm 2, output).

Library primitives used as single steps: ``numpy.linalg.svd`` (LAPACK) for the
SVD inside singular value thresholding, and matrix products.
"""
from __future__ import annotations

import ctypes
import dataclasses
import itertools
import os
import pathlib
import subprocess

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
_LIB_PATH = _HERE / "_liboracle.so"
_lib = None


def build(force: bool = False) -> pathlib.Path:
    """Compile ``alg1.c`` with gcc (OpenMP, -O2, IEEE semantics kept)."""
    if force or not _LIB_PATH.exists() or _LIB_PATH.stat().st_mtime < (_HERE / "alg1.c").stat().st_mtime:
        tmp = _LIB_PATH.with_suffix(".so.tmp")
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99",
               str(_HERE / "alg1.c"), "-o", str(tmp), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            build()
        lib = ctypes.CDLL(str(_LIB_PATH))
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        sig = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double,
               ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp, dp]
        for name in ("oracle_alg1", "oracle_alg1_clip"):
            f = getattr(lib, name)
            f.argtypes = sig
            f.restype = ctypes.c_int
        lib.oracle_alg1_batch.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int64, dp, ctypes.c_int,
            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
            dp, dp, dp, ip, ctypes.c_int, ctypes.c_int]
        lib.oracle_alg1_batch.restype = None
        lib.oracle_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------------------
# Parameters (readings of what the paper leaves open)
# ---------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Alg1Params:
    """Constants of Algorithm 1: ``eps > 0, rho > 1, beta_bar >> beta_0 > 0``.

    The paper fixes none of the values.  Reading: per regression,
    ``beta_0 = beta0_scale / ||x||_2`` and ``beta_bar = beta_max_scale*beta_0``.
    """

    eps: float = 1e-9
    rho: float = 1.5
    beta0_scale: float = 1.25
    beta_max_scale: float = 1e10
    max_iter: int = 500


@dataclasses.dataclass(frozen=True)
class SeedParams:
    """Constants of the seed PCP solved by inexact ALM (eq. SPCP).

    ``lam <= 0`` means ``1/sqrt(max(p, q))`` (Sec. 3.1).  The stopping test is
    ``||M - L - S||_F / ||M||_F < tol`` (Sec. 4.1).  ``rank_floor`` drops
    thresholded singular values below ``rank_floor * sigma_1``.
    """

    lam: float = 0.0
    tol: float = 1e-9
    rho: float = 1.5
    mu0_scale: float = 1.25
    mu_max_scale: float = 1e7
    max_iter: int = 500
    rank_floor: float = 1e-6


# ---------------------------------------------------------------------------
# Elementary operators
# ---------------------------------------------------------------------------
def soft_threshold(t, tau):
    """S_tau(t) = sgn(t) max(|t| - tau, 0)  (Sec. 2, after eq. SVT)."""
    t = np.asarray(t, dtype=np.float64)
    return np.sign(t) * np.maximum(np.abs(t) - tau, 0.0)


def svt(W: np.ndarray, tau: float):
    """Singular value thresholding, the closed-form minimiser of
    ``tau ||A||_* + 1/2 ||A - W||_F^2`` (eqs. Proxy and SVT).

    Returns ``(A, U_k, s_k, Vt_k)`` where ``s_k = sigma_i - tau`` over the
    singular values of W above tau.
    """
    U, s, Vt = np.linalg.svd(W, full_matrices=False)
    keep = s > tau
    Uk, sk, Vtk = U[:, keep], s[keep] - tau, Vt[keep]
    return (Uk * sk) @ Vtk, Uk, sk, Vtk


# ---------------------------------------------------------------------------
# Algorithm 1 (one regression, or many independent ones)
# ---------------------------------------------------------------------------
def alg1(x: np.ndarray, A: np.ndarray, params: Alg1Params = Alg1Params(), form: str = "literal"):
    """Solve ``min ||e||_1 s.t. x = A z + e`` (A^T A = I) by Algorithm 1.

    Returns ``(z, e, y, K)``; ``K < 0`` flags a regression that did not meet
    the stopping test within ``max_iter`` iterations.
    """
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    A = np.asfortranarray(A, dtype=np.float64)
    p, r = A.shape
    assert x.shape[0] == p and params.max_iter >= 1 and 0 <= params.eps < 1
    z = np.zeros(r)
    e = np.zeros(p)
    y = np.zeros(p)
    f = lib.oracle_alg1 if form == "literal" else lib.oracle_alg1_clip
    K = f(p, r, _dptr(x), _dptr(A), p, params.eps, params.rho, params.beta0_scale,
          params.beta_max_scale, params.max_iter, _dptr(z), _dptr(e), _dptr(y))
    return z, e, y, int(K)


def alg1_batch(X: np.ndarray, A: np.ndarray, params: Alg1Params = Alg1Params(),
               form: str = "literal", nthreads: int = 0, keep_dual: bool = False):
    """Algorithm 1 on every column of X (p x nreg), independently.

    Returns ``Z`` (r x nreg), ``K`` (nreg) and, if ``keep_dual``, ``E``, ``Y``.
    """
    lib = _load()
    X = np.asfortranarray(X, dtype=np.float64)
    A = np.asfortranarray(A, dtype=np.float64)
    p, nreg = X.shape
    r = A.shape[1]
    assert A.shape[0] == p and params.max_iter >= 1 and 0 <= params.eps < 1
    Z = np.zeros((r, nreg), order="F")
    K = np.zeros(nreg, dtype=np.int32)
    E = np.zeros((p, nreg), order="F") if keep_dual else None
    Y = np.zeros((p, nreg), order="F") if keep_dual else None
    if nreg:
        lib.oracle_alg1_batch(
            p, r, nreg, _dptr(X), p, _dptr(A), p, params.eps, params.rho,
            params.beta0_scale, params.beta_max_scale, params.max_iter, _dptr(Z),
            _dptr(E) if keep_dual else None, _dptr(Y) if keep_dual else None,
            K.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), int(nthreads),
            0 if form == "literal" else 1)
    if keep_dual:
        return Z, K, E, Y
    return Z, K


def num_threads(requested: int = 0) -> int:
    return int(_load().oracle_num_threads(int(requested)))


# ---------------------------------------------------------------------------
# Seed PCP (eq. SPCP) by inexact ALM / ADM
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class SeedResult:
    U: np.ndarray       # p x r'
    sigma: np.ndarray   # r'
    V: np.ndarray       # q x r'
    rank: int
    iters: int
    converged: bool
    L: np.ndarray
    S: np.ndarray
    Y: np.ndarray       # multiplier after the last step (certifies S)
    YL: np.ndarray      # Y_k + mu_k (M - L_{k+1} - S_k) (certifies L)
    mu_last: float
    lam: float


def pcp_ialm(M: np.ndarray, lam: float, params: SeedParams = SeedParams()) -> SeedResult:
    """PCP ``min ||L||_* + lam ||S||_1 s.t. M = L + S`` (eq. PCP) by the
    inexact ALM.  Reading of the omitted pseudo-code (low-rank step first):

        Y_0 = M / max(||M||_2, ||M||_inf / lam),  S_0 = 0,
        mu_0 = mu0_scale / ||M||_2,  mu_bar = mu_max_scale * mu_0;
        L_{k+1} = SVT_{1/mu_k}(M - S_k + Y_k / mu_k)
        S_{k+1} = S_{lam/mu_k}(M - L_{k+1} + Y_k / mu_k)
        Y_{k+1} = Y_k + mu_k (M - L_{k+1} - S_{k+1})
        mu_{k+1} = min(rho mu_k, mu_bar)
    until ``||M - L - S||_F / ||M||_F < tol``.  The factors come from the
    final SVT (Sec. 3.2): ``U, V`` its singular vectors and
    ``Sigma = sigma - 1/mu``.
    """
    M = np.asarray(M, dtype=np.float64)
    norm2 = np.linalg.norm(M, 2)
    normF = np.linalg.norm(M)
    Y = M / max(norm2, np.abs(M).max() / lam)
    S = np.zeros_like(M)
    mu = params.mu0_scale / norm2
    mu_bar = params.mu_max_scale * mu
    converged = False
    k = 0
    L = np.zeros_like(M)
    Uk = np.zeros((M.shape[0], 0))
    sk = np.zeros(0)
    Vtk = np.zeros((0, M.shape[1]))
    mu_used = mu
    YL = Y
    for k in range(1, params.max_iter + 1):
        L, Uk, sk, Vtk = svt(M - S + Y / mu, 1.0 / mu)
        YL = Y + mu * (M - L - S)
        S = soft_threshold(M - L + Y / mu, lam / mu)
        Z = M - L - S
        Y = Y + mu * Z
        mu_used = mu
        mu = min(params.rho * mu, mu_bar)
        if np.linalg.norm(Z) / normF < params.tol:
            converged = True
            break
    if sk.size:
        keep = sk > params.rank_floor * sk[0]
        Uk, sk, Vtk = Uk[:, keep], sk[keep], Vtk[keep]
    return SeedResult(U=Uk, sigma=sk, V=Vtk.T.copy(), rank=int(sk.size), iters=k,
                      converged=converged, L=L, S=S, Y=Y, YL=YL, mu_last=mu_used, lam=lam)


def seed_pcp(Ms: np.ndarray, params: SeedParams = SeedParams()) -> SeedResult:
    """Seed matrix recovery (Sec. 3.1, eq. SPCP) on the (p x q) sample
    ``M^s``, with ``lambda~ = 1/sqrt(max(p, q))`` unless given."""
    p, q = Ms.shape
    lam = params.lam if params.lam > 0 else 1.0 / np.sqrt(max(p, q))
    return pcp_ialm(Ms, lam, params)


# ---------------------------------------------------------------------------
# l1 filtering (eqs. l1c', l1r') and completion (eq. l1s')
# ---------------------------------------------------------------------------
def complement(idx: np.ndarray, size: int) -> np.ndarray:
    mask = np.ones(size, dtype=bool)
    mask[idx] = False
    return np.nonzero(mask)[0].astype(np.int64)


def filter_cols(M: np.ndarray, seed_rows, cols, U: np.ndarray, params: Alg1Params = Alg1Params(),
                nthreads: int = 0):
    """Column filtering (eq. l1c'): for each column j in ``cols`` regress
    ``M[I_s, j]`` on ``U^s``.  Returns ``Qt`` (r x len(cols)) and counts."""
    X = np.asarray(M[np.ix_(np.asarray(seed_rows), np.asarray(cols))], dtype=np.float64)
    return alg1_batch(X, U, params, nthreads=nthreads)


def filter_rows(M: np.ndarray, seed_cols, rows, V: np.ndarray, params: Alg1Params = Alg1Params(),
                nthreads: int = 0):
    """Row filtering (eq. l1r'): ``M^r = P~^T V^T + S^r`` transposes to
    ``(M^r)^T = V P~ + (S^r)^T``, so each row i in ``rows`` regresses
    ``M[i, J_s]^T`` on ``V^s``.  Returns ``Pt`` (r x len(rows)) and counts."""
    X = np.asarray(M[np.ix_(np.asarray(rows), np.asarray(seed_cols))], dtype=np.float64).T
    return alg1_batch(X, V, params, nthreads=nthreads)


def complete(M, seed_rows, seed_cols, U, sigma, V, Qt, Pt):
    """Assemble L block by block (eqs. partition, row-column-recovery, l1s')
    and return ``(L, S = M - L)`` (Algorithm 2, output)::

        L[I_s, J_s] = U Sigma V^T           (the seed L^s)
        L[I_s, J_c] = U Q~                  (L^c)
        L[I_c, J_s] = P~^T V^T              (L^r)
        L[I_c, J_c] = P~^T Sigma^{-1} Q~    (eq. l1s')
    """
    m, n = M.shape
    I = np.asarray(seed_rows)
    J = np.asarray(seed_cols)
    Ic = complement(I, m)
    Jc = complement(J, n)
    L = np.zeros((m, n))
    L[np.ix_(I, J)] = (U * sigma) @ V.T
    L[np.ix_(I, Jc)] = U @ Qt
    L[np.ix_(Ic, J)] = Pt.T @ V.T
    L[np.ix_(Ic, Jc)] = (Pt.T / sigma) @ Qt
    S = np.asarray(M, dtype=np.float64) - L
    return L, S


def complete_entries(rows, cols, seed_rows, seed_cols, m, n, U, sigma, V, Qt, Pt):
    """Entries ``L[rows[k], cols[k]]`` from the same four block formulas,
    one entry at a time (for matrices too large to assemble)."""
    I = np.asarray(seed_rows)
    J = np.asarray(seed_cols)
    pos_I = -np.ones(m, dtype=np.int64)
    pos_I[I] = np.arange(I.size)
    pos_J = -np.ones(n, dtype=np.int64)
    pos_J[J] = np.arange(J.size)
    Ic = complement(I, m)
    Jc = complement(J, n)
    pos_Ic = -np.ones(m, dtype=np.int64)
    pos_Ic[Ic] = np.arange(Ic.size)
    pos_Jc = -np.ones(n, dtype=np.int64)
    pos_Jc[Jc] = np.arange(Jc.size)
    out = np.empty(len(rows))
    for k, (i, j) in enumerate(zip(rows, cols)):
        if pos_I[i] >= 0 and pos_J[j] >= 0:
            out[k] = np.dot(U[pos_I[i]] * sigma, V[pos_J[j]])
        elif pos_I[i] >= 0:
            out[k] = np.dot(U[pos_I[i]], Qt[:, pos_Jc[j]])
        elif pos_J[j] >= 0:
            out[k] = np.dot(Pt[:, pos_Ic[i]], V[pos_J[j]])
        else:
            out[k] = np.dot(Pt[:, pos_Ic[i]] / sigma, Qt[:, pos_Jc[j]])
    return out


def complete_new_cols(Mnew: np.ndarray, seed_rows, U, sigma, Pt, Qt_new):
    """L and S of columns that arrive after a fit (Sec. 3.2): every new column
    j is a non-seed column, so by eq. l1c' its seed rows are ``U q~_j`` and by
    eq. l1s' its other rows are ``P~^T Sigma^{-1} q~_j``, where ``q~_j`` is
    the column filtering of ``Mnew[seed_rows, j]`` against U (Algorithm 1;
    ``filter_cols``) and ``P~`` the fit's row filtering over the sorted
    complement of the seed rows.  ``S = Mnew - L``."""
    m = Mnew.shape[0]
    I = np.asarray(seed_rows)
    Ic = complement(I, m)
    L = np.zeros(Mnew.shape)
    L[I, :] = U @ Qt_new
    L[Ic, :] = (Pt.T / sigma) @ Qt_new
    S = np.asarray(Mnew, dtype=np.float64) - L
    return L, S


@dataclasses.dataclass
class RankEstimate:
    r_est: int          # rank of the last seed solved
    accepted: bool      # eq. rank_test held (False: stopped by eq. rank_test1)
    ranks: list         # r' of each round
    sizes: list         # (p, q) of each round
    cv_rank: int        # rank of the cross-validation block, -1 if not run

    @property
    def p(self):
        return self.sizes[-1][0]

    @property
    def q(self):
        return self.sizes[-1][1]


def estimate_rank(M: np.ndarray, r0: int, row_order, col_order, os_r: int = 10, os_c: int = 10,
                  cross_validate: bool = True, params: SeedParams = SeedParams(),
                  max_rounds: int = 16) -> RankEstimate:
    """Target-rank estimation of Sec. 3.6.

    Solve the seed PCP on a (os_r r_k) x (os_c r_k) block and take the rank r'
    of its L^s.  Accept when m'/r' >= os_r and n'/r' >= os_c (eq. rank_test);
    otherwise grow the block to (os_r r') x (os_c r') and repeat, unless that
    block exceeds half of M in either direction (eq. rank_test1), where the
    loop stops unaccepted.  Readings: the blocks are prefixes of the given
    row / column orders (so each contains the previous one; its indices are
    the prefix, sorted); the cross-validation block is the next disjoint
    block of the accepted size, solved only when it fits.
    """
    m, n = M.shape
    row_order = np.asarray(row_order, dtype=np.int64)
    col_order = np.asarray(col_order, dtype=np.int64)

    def rank_of(r_first, p, c_first, q):
        I = np.sort(row_order[r_first:r_first + p])
        J = np.sort(col_order[c_first:c_first + q])
        return seed_pcp(np.asarray(M[np.ix_(I, J)], dtype=np.float64), params).rank

    p, q = os_r * r0, os_c * r0
    ranks, sizes = [], []
    accepted = False
    for _ in range(max_rounds):
        rk = rank_of(0, p, 0, q)
        ranks.append(rk)
        sizes.append((p, q))
        if rk == 0:
            break
        if p / rk >= os_r and q / rk >= os_c:        # eq. rank_test
            accepted = True
            break
        p2, q2 = os_r * rk, os_c * rk
        if max(p2 / m, q2 / n) > 0.5:                # eq. rank_test1
            break
        p, q = p2, q2
    cv = -1
    if accepted and cross_validate and 2 * p <= m and 2 * q <= n:
        cv = rank_of(p, p, q, q)
    return RankEstimate(r_est=ranks[-1], accepted=accepted, ranks=ranks, sizes=sizes, cv_rank=cv)


@dataclasses.dataclass
class SolveResult:
    L: np.ndarray | None
    S: np.ndarray | None
    seed: SeedResult
    U: np.ndarray       # seed factors actually used (at most r columns)
    sigma: np.ndarray
    V: np.ndarray
    Qt: np.ndarray
    Pt: np.ndarray
    col_iters: np.ndarray
    row_iters: np.ndarray
    seed_rows: np.ndarray
    seed_cols: np.ndarray


def solve(M: np.ndarray, r: int, seed_rows, seed_cols, seed_params: SeedParams = SeedParams(),
          alg1_params: Alg1Params = Alg1Params(), nthreads: int = 0, assemble: bool = True) -> SolveResult:
    """Algorithm 2 end to end on ``M`` (m x n) with given seed indices.

    ``r`` is the target rank; the seed size is ``len(seed_rows) x
    len(seed_cols)`` (normally ``10r x 10r``).  The rank actually used is the
    rank of the recovered seed ``L^s``.
    """
    m, n = M.shape
    I = np.asarray(seed_rows, dtype=np.int64)
    J = np.asarray(seed_cols, dtype=np.int64)
    Ms = np.asarray(M[np.ix_(I, J)], dtype=np.float64)
    seed = seed_pcp(Ms, seed_params)
    # Reading: the target rank r is known (Sec. 3.6 opens with that
    # assumption); a seed of larger rank keeps its r leading components.
    k = min(seed.rank, r)
    U, sigma, V = seed.U[:, :k], seed.sigma[:k], seed.V[:, :k]
    Jc = complement(J, n)
    Ic = complement(I, m)
    Qt, kc = filter_cols(M, I, Jc, U, alg1_params, nthreads)
    Pt, kr = filter_rows(M, J, Ic, V, alg1_params, nthreads)
    L = S = None
    if assemble:
        L, S = complete(M, I, J, U, sigma, V, Qt, Pt)
    return SolveResult(L=L, S=S, seed=seed, U=U, sigma=sigma, V=V, Qt=Qt, Pt=Pt,
                       col_iters=kc, row_iters=kr, seed_rows=I, seed_cols=J)


# ---------------------------------------------------------------------------
# Independent checks used to pin the above
# ---------------------------------------------------------------------------
def lad_bruteforce(x: np.ndarray, A: np.ndarray, tol: float = 1e-12):
    """Exact ``min_z ||x - A z||_1`` for tiny problems by enumeration.

    A least-absolute-deviations fit with a full-column-rank A has an optimal
    solution that interpolates r of the points (a vertex of the linear
    program), so the minimum over all r-subsets T with ``A_T`` invertible of
    ``||x - A A_T^{-1} x_T||_1`` is the optimum.  Returns the optimal value
    and the list of distinct minimisers found.
    """
    p, r = A.shape
    best = np.inf
    sols = []
    for T in itertools.combinations(range(p), r):
        AT = A[list(T)]
        if abs(np.linalg.det(AT)) < 1e-12:
            continue
        z = np.linalg.solve(AT, x[list(T)])
        f = np.abs(x - A @ z).sum()
        if f < best - tol * max(1.0, abs(best) if np.isfinite(best) else 1.0):
            best, sols = f, [z]
        elif abs(f - best) <= tol * max(1.0, abs(best)):
            if not any(np.allclose(z, s, rtol=1e-9, atol=1e-12) for s in sols):
                sols.append(z)
    return best, sols


def weighted_median(values: np.ndarray, weights: np.ndarray) -> tuple[float, float]:
    """The interval of minimisers of ``sum_i w_i |v_i - t|`` (w_i > 0): the
    weighted median(s).  Returns (low, high); low == high when unique."""
    order = np.argsort(values, kind="stable")
    v = np.asarray(values)[order]
    w = np.asarray(weights)[order]
    total = w.sum()
    c = np.cumsum(w)
    k = int(np.searchsorted(c, total / 2.0))
    if np.isclose(c[k], total / 2.0, rtol=1e-14, atol=0) and k + 1 < v.size:
        return float(v[k]), float(v[k + 1])
    return float(v[k]), float(v[k])


def lad_kkt(x, A, z, e, y, tol):
    """Optimality residuals of ``min ||e||_1 s.t. x = A z + e`` at (z, e, y):
    stationarity ``A^T y = 0``, dual feasibility ``|y| <= 1``, and
    ``y_i = sgn(e_i)`` where ``|e_i| > tol``.  Returns the three maxima."""
    stat = np.abs(A.T @ y).max() if A.shape[1] else 0.0
    feas = max(0.0, np.abs(y).max() - 1.0)
    big = np.abs(e) > tol
    comp = np.abs(y[big] - np.sign(e[big])).max() if big.any() else 0.0
    return float(stat), float(feas), float(comp)


def pcp_kkt(M, L, S, Y, lam, YL=None):
    """Optimality residuals of PCP at (L, S):
    ``YL - U V^T`` must be orthogonal to U and V with spectral norm <= 1
    (subgradient of the nuclear norm at L), ``Y = lam sgn(S)`` on the support
    of S and ``|Y| <= lam`` off it (subgradient of lam ||.||_1 at S).  At a
    solution one multiplier serves both, so ``gap = ||YL - Y||_F / ||Y||_F``
    measures how far the pair is from optimal.  ``YL`` defaults to ``Y``."""
    if YL is None:
        YL = Y
    U, s, Vt = np.linalg.svd(L, full_matrices=False)
    keep = s > 1e-9 * max(s[0], 1e-300)
    U, Vt = U[:, keep], Vt[keep]
    W = YL - U @ Vt
    orth = max(np.abs(U.T @ W).max(), np.abs(W @ Vt.T).max())
    spec = np.linalg.norm(W, 2)
    supp = np.abs(S) > 1e-7 * np.abs(M).max()
    on = np.abs(Y[supp] - lam * np.sign(S[supp])).max() / lam if supp.any() else 0.0
    off = max(0.0, np.abs(Y[~supp]).max() / lam - 1.0) if (~supp).any() else 0.0
    gap = np.linalg.norm(YL - Y) / np.linalg.norm(Y)
    return dict(orth=float(orth), spec=float(spec), on_support=float(on), off_support=float(off),
                gap=float(gap))


def relerr(A, B) -> float:
    """``||A - B||_F / ||B||_F``."""
    return float(np.linalg.norm(np.asarray(A) - np.asarray(B)) / np.linalg.norm(np.asarray(B)))
