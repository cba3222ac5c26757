"""Seeded synthetic inputs shaped like the workloads of the l1-filtering paper.

This module only draws random numbers and lays them out in memory.  It holds
none of the method's arithmetic, so both the FP64 reference under ``oracle/``
and the GPU library read exactly the bytes it produces and nothing else is
shared between them.

Recipe (paper, Sec. 4.1, synthetic data): ``M = L0 + S0`` where ``L0 = A B^T``
is a product of two thin matrices with i.i.d. zero-mean Gaussian entries and
``S0`` is sparse with a uniformly random support.  ``M`` is rounded once to
FP32 and stored column-major (``M[i, j]`` at ``i + j*ld``), the BLAS
convention, so a row-major ``(n, m)`` tensor holds the same bytes.

Two ways of drawing the support are offered:

* ``exact_count=True``: exactly ``round(sparsity*m*n)`` positions drawn without
  replacement (the paper's generator fixes the number of nonzeros);
* otherwise each entry is corrupted independently with probability
  ``sparsity``, decided by a counter-based hash of the entry's linear index, so
  that any block of ``M`` can be regenerated on its own, in any order.

The hash is SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), written out from its published definition.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "Problem",
    "lowrank_plus_sparse_device",
    "hash_uniform_torch",
    "lowrank_plus_sparse",
    "seed_indices",
    "splitmix64",
    "hash_uniform",
    "CONFIGS",
    "config_problem",
    "BATCH_C4",
    "BatchJobSpec",
    "batch_specs",
    "block_rectangles",
    "union_fraction",
    "batch_job_host",
    "batch_job_device",
]

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to the state ``x`` (uint64 array)."""
    with np.errstate(over="ignore"):
        z = (np.asarray(x, dtype=np.uint64) + _GOLDEN).astype(np.uint64)
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
        return z ^ (z >> np.uint64(31))


def hash_uniform(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) keyed by (seed, stream, linear index)."""
    key = splitmix64(np.uint64((seed * 0x100000001B3 + stream) & 0xFFFFFFFFFFFFFFFF))
    with np.errstate(over="ignore"):
        h = splitmix64(np.asarray(idx, dtype=np.uint64) * _GOLDEN ^ key)
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


@dataclasses.dataclass
class Problem:
    """One synthetic instance.  ``M`` is FP32, Fortran-ordered, shape (m, n)."""

    M: np.ndarray
    A0: np.ndarray  # m x r, float64
    B0: np.ndarray  # n x r, float64
    support: np.ndarray | None  # bool (m, n) Fortran, or None if not kept
    m: int
    n: int
    r: int
    seed: int

    def L0(self) -> np.ndarray:
        return self.A0 @ self.B0.T

    def M_rowmajor_nm(self) -> np.ndarray:
        """The same bytes as ``M`` viewed as a C-ordered (n, m) array."""
        return self.M.T


def lowrank_plus_sparse(
    m: int,
    n: int,
    r: int,
    *,
    factor_std: float,
    sparsity: float,
    values: str = "pm1",
    seed: int = 1,
    exact_count: bool = False,
    keep_support: bool = True,
    block_cols: int = 1024,
) -> Problem:
    """Draw ``M = fl32(A B^T + S0)``.

    ``values``: ``"pm1"`` (+-1 with equal probability), ``"unif11"`` (uniform
    in [-1, 1]), ``"unif01"`` (uniform in [0, 1]) or ``"unif500"`` (uniform in
    [-500, 500], the paper's Table 1 recipe).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    A0 = rng.standard_normal((m, r)) * factor_std
    B0 = rng.standard_normal((n, r)) * factor_std
    M = np.empty((m, n), dtype=np.float32, order="F")
    support = np.zeros((m, n), dtype=bool, order="F") if keep_support else None

    if exact_count:
        k = int(round(sparsity * m * n))
        pos = rng.choice(m * n, size=k, replace=False)  # column-major linear index
        vals = _draw_values(rng.random(k), values)
        S_lin = np.zeros(m * n)
        S_lin[pos] = vals
        S0 = S_lin.reshape((m, n), order="F")
        for j0 in range(0, n, block_cols):
            j1 = min(n, j0 + block_cols)
            M[:, j0:j1] = (A0 @ B0[j0:j1].T + S0[:, j0:j1]).astype(np.float32)
        if support is not None:
            support.reshape(-1, order="F")[pos] = True
    else:
        for j0 in range(0, n, block_cols):
            j1 = min(n, j0 + block_cols)
            lin = (np.arange(j0, j1, dtype=np.uint64)[None, :] * np.uint64(m)
                   + np.arange(m, dtype=np.uint64)[:, None])
            hit = hash_uniform(seed, 1, lin) < sparsity
            vals = _draw_values(hash_uniform(seed, 2, lin), values)
            blk = A0 @ B0[j0:j1].T
            blk += np.where(hit, vals, 0.0)
            M[:, j0:j1] = blk.astype(np.float32)
            if support is not None:
                support[:, j0:j1] = hit
    return Problem(M=M, A0=A0, B0=B0, support=support, m=m, n=n, r=r, seed=seed)


def _draw_values(u: np.ndarray, values: str) -> np.ndarray:
    if values == "pm1":
        return np.where(u < 0.5, -1.0, 1.0)
    if values == "unif11":
        return 2.0 * u - 1.0
    if values == "unif01":
        return u
    if values == "unif500":
        return 1000.0 * u - 500.0
    raise ValueError(f"unknown value law {values!r}")


def seed_indices(m: int, n: int, p: int, q: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Seed rows (p of m) and seed columns (q of n): uniform without
    replacement, returned sorted ascending as int64."""
    rng = np.random.Generator(np.random.PCG64([seed, 0x5EED]))
    I = np.sort(rng.choice(m, size=p, replace=False)).astype(np.int64)
    J = np.sort(rng.choice(n, size=q, replace=False)).astype(np.int64)
    return I, J


# The five workloads.  Factor variance and corruption law follow each
# workload's description; the seed block is 10r x 10r.
CONFIGS = {
    "c1": dict(m=1000, n=1000, r=10, factor_std=np.sqrt(1.0 / 1000), sparsity=0.10,
               values="pm1", exact_count=True),
    "c2": dict(m=10000, n=10000, r=20, factor_std=np.sqrt(1.0 / 10000), sparsity=0.10,
               values="pm1", exact_count=False),
    "c3": dict(m=50000, n=50000, r=50, factor_std=np.sqrt(1.0 / 50000), sparsity=0.05,
               values="unif11", exact_count=False),
}


def config_problem(name: str, seed: int = 1, **overrides) -> Problem:
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    return lowrank_plus_sparse(seed=seed, **cfg)


# ---------------------------------------------------------------------------
# The same generator on a torch device, for matrices too large for the host
# (m = n = 50000: 10 GB in FP32).  The factors are drawn on the host exactly
# as above; the support and values use the same SplitMix64 counter hash
# (int64 arithmetic wraps like uint64; right shifts are made logical).
# ---------------------------------------------------------------------------
def _i64(x: int) -> int:
    x &= 0xFFFFFFFFFFFFFFFF
    return x - (1 << 64) if x >= (1 << 63) else x


def _lsr(z, k: int):
    return (z >> k) & ((1 << (64 - k)) - 1)


def _splitmix64_torch(x):
    z = x + _i64(0x9E3779B97F4A7C15)
    z = (z ^ _lsr(z, 30)) * _i64(0xBF58476D1CE4E5B9)
    z = (z ^ _lsr(z, 27)) * _i64(0x94D049BB133111EB)
    return z ^ _lsr(z, 31)


def hash_uniform_torch(seed: int, stream: int, idx):
    """torch version of :func:`hash_uniform` (idx: int64 tensor); equal bits."""
    import torch
    key = int(splitmix64(np.uint64((seed * 0x100000001B3 + stream) & 0xFFFFFFFFFFFFFFFF)))
    h = _splitmix64_torch((idx * _i64(0x9E3779B97F4A7C15)) ^ _i64(key))
    return _lsr(h, 11).to(torch.float64) * (1.0 / 9007199254740992.0)


def lowrank_plus_sparse_device(m: int, n: int, r: int, *, factor_std: float, sparsity: float,
                               values: str = "pm1", seed: int = 1, device="cuda",
                               block_cols: int = 512):
    """Bernoulli-support version of :func:`lowrank_plus_sparse` built on a
    torch device.  Returns ``(Mt, A0, B0)``: ``Mt`` is the (n, m) row-major
    FP32 tensor holding column-major M; ``A0``, ``B0`` are the host factors."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    A0 = rng.standard_normal((m, r)) * factor_std
    B0 = rng.standard_normal((n, r)) * factor_std
    Ad = torch.from_numpy(A0).to(device)
    Bd = torch.from_numpy(B0).to(device)
    Mt = torch.empty((n, m), dtype=torch.float32, device=device)
    rows = torch.arange(m, dtype=torch.int64, device=device)
    for j0 in range(0, n, block_cols):
        j1 = min(n, j0 + block_cols)
        lin = torch.arange(j0, j1, dtype=torch.int64, device=device)[:, None] * m + rows[None, :]
        hit = hash_uniform_torch(seed, 1, lin) < sparsity
        u = hash_uniform_torch(seed, 2, lin)
        if values == "pm1":
            vals = torch.where(u < 0.5, -1.0, 1.0)
        elif values == "unif11":
            vals = 2.0 * u - 1.0
        elif values == "unif01":
            vals = u
        elif values == "unif500":
            vals = 1000.0 * u - 500.0
        else:
            raise ValueError(values)
        blk = Bd[j0:j1] @ Ad.T
        blk += torch.where(hit, vals, torch.zeros_like(vals))
        Mt[j0:j1] = blk.to(torch.float32)
        del lin, hit, u, vals, blk
    return Mt, A0, B0


# ---------------------------------------------------------------------------
# Batches of independent problems shaped like video background modelling
# (pixels x frames, low rank plus block-shaped foreground).  Each job draws
# m, n, r, a corruption fraction rho and a list of rectangles on the host
# (PCG64); the entries of M are then a pure function of the job's seed, so
# the host and the device paint identical matrices.
#
# Corruptions (block reading): rectangles of height ~ U[m/50, m/10] and width
# ~ U[n/20, n/5] at uniform positions are added until their union covers at
# least rho of the matrix; every entry of the union gets a value U[0, 1]
# keyed by the entry's column-major linear index.
# ---------------------------------------------------------------------------
BATCH_C4 = dict(njobs=256, m=(2048, 76800), n=(100, 1000), r=(1, 8), rho=(0.05, 0.15), os=10)


@dataclasses.dataclass
class BatchJobSpec:
    m: int
    n: int
    r: int
    rho: float
    rects: list          # (i0, i1, j0, j1), half-open
    seed: int            # factors, values and seed indices

    @property
    def p(self) -> int:
        return BATCH_C4["os"] * self.r

    @property
    def q(self) -> int:
        return BATCH_C4["os"] * self.r


def union_fraction(rects, m: int, n: int) -> float:
    """Exact area of the union of half-open rectangles, over m*n
    (coordinate compression: the union is constant on the compressed cells)."""
    if not rects:
        return 0.0
    ys = sorted({0, m, *[r[0] for r in rects], *[r[1] for r in rects]})
    xs = sorted({0, n, *[r[2] for r in rects], *[r[3] for r in rects]})
    yi = {v: k for k, v in enumerate(ys)}
    xi = {v: k for k, v in enumerate(xs)}
    cov = np.zeros((len(ys) - 1, len(xs) - 1), dtype=bool)
    for i0, i1, j0, j1 in rects:
        cov[yi[i0]:yi[i1], xi[j0]:xi[j1]] = True
    h = np.diff(np.asarray(ys, dtype=np.float64))
    w = np.diff(np.asarray(xs, dtype=np.float64))
    return float((h[:, None] * w[None, :] * cov).sum() / (float(m) * n))


def block_rectangles(rng: np.random.Generator, m: int, n: int, rho: float) -> list:
    rects = []
    hmin, hmax = max(1, -(-m // 50)), max(1, m // 10)
    wmin, wmax = max(1, -(-n // 20)), max(1, n // 5)
    while union_fraction(rects, m, n) < rho:
        h = int(rng.integers(hmin, max(hmin, hmax) + 1))
        w = int(rng.integers(wmin, max(wmin, wmax) + 1))
        i0 = int(rng.integers(0, m - h + 1))
        j0 = int(rng.integers(0, n - w + 1))
        rects.append((i0, i0 + h, j0, j0 + w))
    return rects


def batch_specs(njobs: int = 256, seed: int = 1, m=(2048, 76800), n=(100, 1000), r=(1, 8),
                rho=(0.05, 0.15)) -> list:
    """Job shapes and corruption rectangles (uniform integer ranges, inclusive)."""
    rng = np.random.Generator(np.random.PCG64([seed, 0xBA7C4]))
    specs = []
    for j in range(njobs):
        mj = int(rng.integers(m[0], m[1] + 1))
        nj = int(rng.integers(n[0], n[1] + 1))
        rj = int(rng.integers(r[0], r[1] + 1))
        rhoj = float(rng.uniform(rho[0], rho[1]))
        rects = block_rectangles(rng, mj, nj, rhoj)
        specs.append(BatchJobSpec(m=mj, n=nj, r=rj, rho=rhoj, rects=rects,
                                  seed=(seed << 20) + j + 1))
    return specs


def _job_factors(spec: BatchJobSpec):
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    std = np.sqrt(1.0 / spec.m)
    return rng.standard_normal((spec.m, spec.r)) * std, rng.standard_normal((spec.n, spec.r)) * std


def batch_job_host(spec: BatchJobSpec, keep_support: bool = True) -> Problem:
    """M = fl32(A B^T + S0) of one job on the host (Fortran order)."""
    A0, B0 = _job_factors(spec)
    m, n = spec.m, spec.n
    S0 = np.zeros((m, n), order="F")
    support = np.zeros((m, n), dtype=bool, order="F")
    for i0, i1, j0, j1 in spec.rects:
        support[i0:i1, j0:j1] = True
    jj, ii = np.nonzero(support.T)                     # column-major order
    lin = jj.astype(np.uint64) * np.uint64(m) + ii.astype(np.uint64)
    S0[ii, jj] = hash_uniform(spec.seed, 2, lin)
    M = np.asfortranarray((A0 @ B0.T + S0).astype(np.float32))
    return Problem(M=M, A0=A0, B0=B0, support=support if keep_support else None, m=m, n=n,
                   r=spec.r, seed=spec.seed)


def batch_job_device(spec: BatchJobSpec, device="cuda", out=None):
    """The same matrix built on a torch device: returns ``(Mt, A0, B0)`` with
    ``Mt`` the (n, m) FP32 tensor holding column-major M (or written into
    ``out`` of that shape)."""
    import torch
    A0, B0 = _job_factors(spec)
    m, n = spec.m, spec.n
    Ad = torch.from_numpy(A0).to(device)
    Bd = torch.from_numpy(B0).to(device)
    L64 = Bd @ Ad.T                                       # (n, m) FP64, column-major M
    mask = torch.zeros((n, m), dtype=torch.bool, device=device)
    for i0, i1, j0, j1 in spec.rects:
        mask[j0:j1, i0:i1] = True
    lin = mask.view(-1).nonzero().squeeze(1)              # = j m + i, M's linear index
    L64.view(-1)[lin] += hash_uniform_torch(spec.seed, 2, lin)
    del mask, lin
    Mt = out if out is not None else torch.empty((n, m), dtype=torch.float32, device=device)
    Mt.copy_(L64)
    del L64
    return Mt, A0, B0


# ---------------------------------------------------------------------------
# A deterministic rank-2 low-rank part: the m x n "checkerboard" image of the
# paper's deterministic test (square cells of `cell` pixels, values 0 and 1:
# C[i, j] = (floor(i / cell) + floor(j / cell)) mod 2, which is
# a_i (1 - b_j) + (1 - a_i) b_j with 0/1 vectors a, b, hence rank 2), with a
# fraction of its pixels replaced by impulsive noise: a uniformly random
# support (counter hash of the linear index, as above), each hit pixel set
# to 0 or 1 with equal probability.  S0 = noisy - C is zero where the noise
# value equals the pixel's own value.
# ---------------------------------------------------------------------------
def checkerboard(m: int, n: int, cell: int, noise: float, seed: int = 1) -> Problem:
    i = np.arange(m)[:, None] // cell
    j = np.arange(n)[None, :] // cell
    C = ((i + j) % 2).astype(np.float64)
    lin = (np.arange(n, dtype=np.uint64)[None, :] * np.uint64(m)
           + np.arange(m, dtype=np.uint64)[:, None])
    hit = hash_uniform(seed, 1, lin) < noise
    val = (hash_uniform(seed, 2, lin) < 0.5).astype(np.float64)
    M = np.asfortranarray(np.where(hit, val, C).astype(np.float32))
    a = (np.arange(m) // cell % 2).astype(np.float64)
    b = (np.arange(n) // cell % 2).astype(np.float64)
    # C = A0 B0^T with A0 = [a, 1 - a], B0 = [1 - b, b]
    A0 = np.stack([a, 1.0 - a], axis=1)
    B0 = np.stack([1.0 - b, b], axis=1)
    return Problem(M=M, A0=A0, B0=B0, support=np.asfortranarray(hit & (val != C)), m=m, n=n, r=2,
                   seed=seed)
