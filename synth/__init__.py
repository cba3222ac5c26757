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
