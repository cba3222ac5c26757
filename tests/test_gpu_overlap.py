"""Steps 3-5 with the completion overlapped with the filter
(rpca_filter_complete, opts.overlap_chunks > 0) give exactly what
rpca_filter followed by rpca_reconstruct gives (bit for bit: every regression
and every element of L, S is computed by the same code; only the order of the
launches and the stream they run on change), and therefore the oracle's
result within the stated 1e-5.  Cases: the oracle-sized workload in both
precision forms, the precision form's quarter-tile kernel (p = 300), chunk
counts from 1 to 16, the FP32 quarter-tile kernel (p = 410), the full-size
plain workload, ragged shapes with padded leading dimensions, slabs with no
column regressions, a seed taking every row."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_util import (REL_TOL, dev_f64_colmajor, dev_i64, dev_matrix, host_matrix, relF, say,
                      support_mismatch)
from test_gpu_parity import R, case, ctx, small_case  # noqa: F401  (fixtures and cached cases)

pytestmark = pytest.mark.gpu


def _run_both(R, ctx, pr, I, J, U, sigma, V, r, chunks, precision, ld=None):
    import torch
    m, n = pr.m, pr.n
    ld = ld or m
    Ic, Jc = oracle.complement(I, m), oracle.complement(J, n)
    Md = dev_matrix(pr.M, ld)
    dI, dJ, dIc, dJc = dev_i64(I), dev_i64(J), dev_i64(Ic), dev_i64(Jc)
    dU, dsg, dV = dev_f64_colmajor(U), torch.as_tensor(np.asarray(sigma, dtype=np.float64)).cuda(), dev_f64_colmajor(V)
    out = []
    for mode in ("sequential", "overlapped"):
        L = torch.full((n, ld), float("nan"), device="cuda")
        S = torch.full((n, ld), float("nan"), device="cuda")
        Qt = torch.full((max(len(Jc), 1), r), float("nan"), device="cuda")
        Pt = torch.full((max(len(Ic), 1), r), float("nan"), device="cuda")
        kc = torch.zeros(max(len(Jc), 1), dtype=torch.int32, device="cuda")
        kr = torch.zeros(max(len(Ic), 1), dtype=torch.int32, device="cuda")
        o = R.rpca_opts_default(precision=precision, overlap_chunks=chunks if mode == "overlapped" else 0)
        if mode == "sequential":
            R.rpca_filter(ctx, Md, m, n, ld, dI, len(I), dJ, len(J), dJc, len(Jc), dIc, len(Ic), dU, dV,
                          r, o, Qt, kc, Pt, kr)
            R.rpca_reconstruct(ctx, Md, m, n, ld, dI, len(I), dJ, len(J), dU, dsg, dV, r, Qt, Pt, L, ld,
                               S, ld)
        else:
            R.rpca_filter_complete(ctx, Md, m, n, ld, dI, len(I), dJ, len(J), dJc, dIc, dU, dsg, dV, r,
                                   o, Qt, kc, Pt, kr, L, ld, S, ld)
        torch.cuda.synchronize()
        out.append((L, S, Qt, Pt, kc, kr))
    (L1, S1, Q1, P1, kc1, kr1), (L2, S2, Q2, P2, kc2, kr2) = out

    def same(a, b):        # bitwise, NaN placeholders (empty sides) included
        return bool(((a == b) | (torch.isnan(a) & torch.isnan(b))).all())

    assert same(L1[:, :m], L2[:, :m]) and same(S1[:, :m], S2[:, :m])
    assert same(Q1, Q2) and same(P1, P2)
    assert torch.equal(kc1, kc2) and torch.equal(kr1, kr2)
    return host_matrix(L2, m), host_matrix(S2, m)


@pytest.mark.parametrize("seed,chunks,precision", [(1, 4, 0), (2, 1, 0), (1, 16, 0), (3, 5, 1), (1, 7, 1)])
def test_overlapped_equals_sequential_c1(R, ctx, seed, chunks, precision):
    pr, r, I, J, res = case("c1", seed)
    k = res.U.shape[1]
    say(f"overlap c1 seed={seed} chunks={chunks} precision={precision}")
    Lh, Sh = _run_both(R, ctx, pr, I, J, res.U, res.sigma, res.V, k, chunks, precision)
    assert relF(Lh, res.L) <= REL_TOL and relF(Sh, res.S) <= REL_TOL


def test_overlapped_equals_sequential_c2_full_size(R, ctx):
    # m = n = 10000: the two forms agree bit for bit (checked in _run_both);
    # the overlapped result against the oracle on 200000 sampled entries
    pr, r, I, J, res = case("c2", 1)
    k = res.U.shape[1]
    say("overlap c2 full size")
    Lh, Sh = _run_both(R, ctx, pr, I, J, res.U, res.sigma, res.V, k, 4, 0)
    rng = np.random.default_rng(1)
    rows = rng.integers(0, pr.m, 200000)
    cols = rng.integers(0, pr.n, 200000)
    Lref = oracle.complete_entries(rows, cols, I, J, pr.m, pr.n, res.U, res.sigma, res.V, res.Qt,
                                   res.Pt)
    Sref = pr.M[rows, cols].astype(np.float64) - Lref
    assert relF(Lh[rows, cols], Lref) <= REL_TOL
    assert relF(Sh[rows, cols], Sref) <= REL_TOL
    assert support_mismatch(Sh[rows, cols], Sref, float(np.abs(pr.M).max())) == 0


@pytest.mark.parametrize("m,n,r,ld_pad,chunks", [(333, 517, 3, 5, 4), (1200, 700, 1, 0, 9),
                                                 (517, 333, 7, 3, 16), (800, 103, 10, 0, 16),
                                                 (60, 300, 6, 0, 3)])
def test_overlapped_ragged(R, ctx, m, n, r, ld_pad, chunks):
    # (800, 103, 10): q = 100 of 103 columns are seed columns, most slabs hold
    # no column regression; (60, 300, 6): the seed takes every row
    pr, I, J, res = small_case(m, n, r, 0.05, 11 + r)
    k = res.U.shape[1]
    say(f"overlap ragged m={m} n={n} r={r} ld+{ld_pad} chunks={chunks}")
    Lh, Sh = _run_both(R, ctx, pr, I, J, res.U, res.sigma, res.V, k, chunks, 0, ld=m + ld_pad)
    assert relF(Lh, res.L) <= REL_TOL and relF(Sh, res.S) <= REL_TOL


@pytest.mark.parametrize("chunks", [3, 8])
def test_overlapped_quarter_tile_precision(R, ctx, chunks):
    # p = q = 300 (class PT = 19): the precision form's quarter-tile kernel
    # (persistent, two tiles per workgroup) reading its regression range from
    # the device in every column slab; the results are those of one launch
    pr, I, J, res = small_case(2100, 1900, 30, 0.05, 37)
    k = res.U.shape[1]
    say(f"overlap quarter-tile precision form chunks={chunks}")
    Lh, Sh = _run_both(R, ctx, pr, I, J, res.U, res.sigma, res.V, k, chunks, 1)
    assert relF(Lh, res.L) <= REL_TOL and relF(Sh, res.S) <= REL_TOL


@pytest.mark.parametrize("chunks,ld_pad", [(3, 0), (6, 7)])
def test_overlapped_quarter_tile_fp32(R, ctx, chunks, ld_pad):
    # p = q = 410 (class PT = 26) in the FP32 form: the quarter-tile kernel
    # with FP32 contractions, reading its regression range from the device in
    # every column slab, with and without a padded leading dimension
    pr, I, J, res = small_case(2600, 2333, 41, 0.05, 48)
    k = res.U.shape[1]
    say(f"overlap quarter-tile FP32 form chunks={chunks} ld+{ld_pad}")
    Lh, Sh = _run_both(R, ctx, pr, I, J, res.U, res.sigma, res.V, k, chunks, 0, ld=pr.m + ld_pad)
    assert relF(Lh, res.L) <= REL_TOL and relF(Sh, res.S) <= REL_TOL


def test_overlap_option_is_checked(R, ctx):
    pr, r, I, J, res = case("c1", 1)
    import torch
    Md = dev_matrix(pr.M)
    L = torch.empty_like(Md)
    S = torch.empty_like(Md)
    with pytest.raises(R.RpcaError) as e:
        R.rpca_solve(ctx, Md, pr.m, pr.n, pr.m, r, R.rpca_opts_default(overlap_chunks=17),
                     dev_i64(I), dev_i64(J), L, pr.m, S, pr.m)
    assert e.value.status == R.RPCA_ERR_ARG
