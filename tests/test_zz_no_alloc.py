"""The no-allocation completion (rpca_reconstruct_noalloc) against
rpca_reconstruct: same kernels, so L and S must agree bit for bit.  Two
calls in a row on one device share the library's fixed scratch array; the
second, smaller call must not see anything of the first.  Sizes beyond the
scratch are refused before anything is enqueued."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import dev_f64_colmajor, dev_i64, dev_matrix, say

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


def _factors(m, n, r, seed):
    rng = np.random.Generator(np.random.PCG64([m, n, r, seed]))
    p, q = 10 * r, 10 * r
    I = np.sort(rng.choice(m, p, replace=False))
    J = np.sort(rng.choice(n, q, replace=False))
    U = np.linalg.qr(rng.standard_normal((p, r)))[0]
    V = np.linalg.qr(rng.standard_normal((q, r)))[0]
    sigma = np.sort(rng.uniform(0.5, 2.0, r))[::-1].copy()
    Qt = rng.standard_normal((r, n - q)).astype(np.float32)
    Pt = rng.standard_normal((r, m - p)).astype(np.float32)
    M = np.asfortranarray(rng.standard_normal((m, n)).astype(np.float32))
    return M, I, J, U, sigma, V, Qt, Pt


def _run(R, ctx, fn, m, n, r, seed, ld_pad=0):
    import torch
    M, I, J, U, sigma, V, Qt, Pt = _factors(m, n, r, seed)
    ld = m + ld_pad
    Md = dev_matrix(M, ld)
    L = torch.full((n, ld), float("nan"), dtype=torch.float32, device="cuda")
    S = torch.full_like(L, float("nan"))
    st = fn(ctx, Md, m, n, ld, dev_i64(I), len(I), dev_i64(J), len(J), dev_f64_colmajor(U),
            torch.as_tensor(sigma).cuda(), dev_f64_colmajor(V), r,
            torch.as_tensor(np.ascontiguousarray(Qt.T)).cuda(),
            torch.as_tensor(np.ascontiguousarray(Pt.T)).cuda(), L, ld, S, ld)
    torch.cuda.synchronize()
    return st, L, S


def _same(a, b):
    import torch
    return bool(((a == b) | (torch.isnan(a) & torch.isnan(b))).all().item())


def test_noalloc_equals_reconstruct_two_calls(R, ctx):
    # the first call fills 92% of the scratch ((120000 + 1000) * 4 * 64
    # bytes); the second is smaller (rank 7, odd leading dimension)
    import torch
    cases = [(120000, 1000, 64, 1, 0), (900, 700, 7, 2, 3)]
    for (m, n, r, seed, pad) in cases:
        say(f"noalloc m={m} n={n} r={r} ld+{pad}")
        st1, L1, S1 = _run(R, ctx, R.rpca_reconstruct, m, n, r, seed, pad)
        st2, L2, S2 = _run(R, ctx, R.rpca_reconstruct_noalloc, m, n, r, seed, pad)
        assert st1 == R.RPCA_OK and st2 == R.RPCA_OK
        assert _same(L1, L2) and _same(S1, S2)
        assert not bool(torch.isnan(L2[:, :m]).any().item())


def test_noalloc_refuses_sizes_beyond_its_scratch(R, ctx):
    import torch
    # (m + n) * 4 * ceil4(r) = (2100000 + 1) * 16 bytes > 32 MiB: refused on
    # the host; the buffers are real and of the stated sizes all the same
    m, n, r = 2_100_000, 1, 1
    say("noalloc size check")
    Md = torch.zeros((n, m), dtype=torch.float32, device="cuda")
    L = torch.zeros_like(Md)
    S = torch.zeros_like(Md)
    one = dev_i64([0])
    U = torch.ones((1, 1), dtype=torch.float64, device="cuda")
    sg = torch.ones(1, dtype=torch.float64, device="cuda")
    Pt = torch.zeros((m - 1, 1), dtype=torch.float32, device="cuda")
    with pytest.raises(R.RpcaError) as e:
        R.rpca_reconstruct_noalloc(ctx, Md, m, n, m, one, 1, one, 1, U, sg, U, 1,
                                   torch.zeros(1, device="cuda"), Pt, L, m, S, m)
    assert e.value.status == R.RPCA_ERR_ARG
    assert "scratch" in ctx.last_error()
    torch.cuda.synchronize()
