"""Served form on the GPU (rpca_server_*): a request loop with admission by
HBM footprint and continuous batching across worker threads.

* Each request's L and S are the same served alone (one worker, one request
  at a time) and in a mix (three workers, batches of up to four, all
  requests queued at once), within the stated tolerance (and, since every
  regression, seed and completion is computed the same way whatever batch
  it is in, bit for bit).
* Every served result matches the FP64 oracle run on that request alone
  (relative Frobenius 1e-5 on L and S; seeds run to their FP64 fixed point on
  both sides, see test_gpu_batch).
* The admitted footprint never exceeds the budget, admission is in arrival
  order, and a bad request fails alone.

The mix has the three request classes of the serving workload at reduced
size: small squares (lane form, batched seed), tall skinny matrices with
p = 60 (lane form split over lanes) and squares with p = q = 120 (tile form,
precision form, seed one by one)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_util import REL_TOL, dev_i64, relF, say, support_mismatch
from test_gpu_parity import R, ctx  # noqa: F401  (fixtures)

pytestmark = pytest.mark.gpu

SEED_TOL = 1e-12

# (m, n, r, sparsity) of the mix: the serving classes at reduced size
_CLASSES = [(600, 600, 3, 0.1), (3000, 250, 6, 0.1), (1500, 1500, 12, 0.1)]


def _mix(nreq=10, seed=5):
    rng = np.random.Generator(np.random.PCG64([seed, 0x5E7]))
    out = []
    for k in range(nreq):
        c = int(rng.choice(3, p=[0.6, 0.3, 0.1])) if k >= 3 else k
        m, n, r, sp = _CLASSES[c]
        s = 100 + k
        pr = synth.lowrank_plus_sparse(m, n, r, factor_std=np.sqrt(1.0 / max(m, n)), sparsity=sp,
                                       values="pm1", seed=s)
        I, J = synth.seed_indices(m, n, 10 * r, 10 * r, seed=s)
        out.append((pr, r, I, J))
    return out


_CACHE = {}


def _reference():
    if "mix" not in _CACHE:
        mix = _mix()
        refs = [oracle.solve(pr.M, r, I, J, seed_params=oracle.SeedParams(tol=SEED_TOL))
                for pr, r, I, J in mix]
        _CACHE["mix"] = (mix, refs)
    return _CACHE["mix"]


def _opts(R):
    return R.rpca_opts_default(seed_tol=SEED_TOL, precision=1)


def _buffers(mix):
    import torch
    bufs = []
    for pr, r, I, J in mix:
        Md = torch.from_numpy(np.ascontiguousarray(pr.M.T)).cuda()
        L = torch.full_like(Md, float("nan"))
        S = torch.full_like(Md, float("nan"))
        bufs.append((Md, L, S, dev_i64(I), dev_i64(J)))
    torch.cuda.synchronize()
    return bufs


def _job(R, item, buf):
    pr, r, I, J = item
    Md, L, S, dI, dJ = buf
    return R.job(Md, pr.m, pr.n, pr.m, r, dI, len(I), dJ, len(J), L, pr.m, S, pr.m)


def _serve(R, mix, bufs, workers, max_batch, one_at_a_time, budget=200e9):
    srv = R.Server(_opts(R), None, R.rpca_server_opts_default(workers=workers, max_batch=max_batch,
                                                             hbm_budget_bytes=budget))
    infos = []
    if one_at_a_time:
        for item, buf in zip(mix, bufs):
            infos.append(srv.wait(srv.submit(_job(R, item, buf))))
    else:
        tickets = [srv.submit(_job(R, item, buf)) for item, buf in zip(mix, bufs)]
        infos = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    return infos, stats


def test_served_results_are_the_same_alone_and_in_the_mix(R, ctx):
    mix, refs = _reference()
    say(f"serving: {len(mix)} requests alone")
    alone = _buffers(mix)
    infos_a, _ = _serve(R, mix, alone, workers=1, max_batch=1, one_at_a_time=True)
    say("serving: the same requests in a mix")
    mixed = _buffers(mix)
    infos_m, stats = _serve(R, mix, mixed, workers=3, max_batch=4, one_at_a_time=False)
    assert stats.completed == len(mix) and stats.failed == 0
    assert max(i.batch_size for i in infos_m) > 1            # they did share batches
    identical = 0
    for k, (a, b) in enumerate(zip(alone, mixed)):
        m = mix[k][0].m
        La, Sa = a[1][:, :m].double().cpu().numpy(), a[2][:, :m].double().cpu().numpy()
        Lb, Sb = b[1][:, :m].double().cpu().numpy(), b[2][:, :m].double().cpu().numpy()
        assert relF(Lb, La) <= REL_TOL and relF(Sb, Sa) <= REL_TOL, k
        identical += int(np.array_equal(La, Lb) and np.array_equal(Sa, Sb))
    say(f"serving: {identical} of {len(mix)} results bitwise identical alone and in the mix")
    assert identical == len(mix)


def test_served_results_match_the_oracle(R, ctx):
    mix, refs = _reference()
    bufs = _buffers(mix)
    infos, stats = _serve(R, mix, bufs, workers=3, max_batch=4, one_at_a_time=False)
    for k, ((pr, r, I, J), res, buf, inf) in enumerate(zip(mix, refs, bufs, infos)):
        Lh = buf[1].double().cpu().numpy().T
        Sh = buf[2].double().cpu().numpy().T
        assert inf.status >= 0 and inf.info.r_used == min(res.seed.rank, r)
        assert relF(Lh, res.L) <= REL_TOL and relF(Sh, res.S) <= REL_TOL, (k, relF(Lh, res.L))
        assert support_mismatch(Sh, res.S, float(np.abs(pr.M).max())) == 0, k
        assert inf.t_submit_ms <= inf.t_admit_ms <= inf.t_done_ms


def test_admission_respects_the_budget_and_arrival_order(R, ctx):
    mix, refs = _reference()
    bufs = _buffers(mix)
    fp = [12 * pr.m * pr.n for pr, r, I, J in mix]
    budget = 1.5 * max(fp)
    infos, stats = _serve(R, mix, bufs, workers=3, max_batch=4, one_at_a_time=False, budget=budget)
    say(f"serving: budget {budget / 1e6:.0f} MB, peak admitted {stats.peak_inflight_bytes / 1e6:.0f} MB, "
        f"{stats.batches} batches")
    assert stats.completed == len(mix) and stats.failed == 0
    # a request larger than the budget is admitted alone; otherwise the sum fits
    assert stats.peak_inflight_bytes <= max(budget, max(fp) * 1.2)
    admits = [i.t_admit_ms for i in infos]
    assert admits == sorted(admits)                            # FIFO admission
    for k, (res, buf) in enumerate(zip(refs, bufs)):
        assert relF(buf[1].double().cpu().numpy().T, res.L) <= REL_TOL, k


def test_a_bad_request_fails_alone(R, ctx):
    mix, refs = _reference()
    mix4 = mix[:4]
    bufs = _buffers(mix4)
    pr, r, I, J = mix4[1]
    bad = list(bufs[1])
    bad[3] = dev_i64(I[::-1].copy())                          # unsorted seed rows
    bufs[1] = tuple(bad)
    srv = R.Server(_opts(R), None, R.rpca_server_opts_default(workers=1, max_batch=4))
    tickets = [srv.submit(_job(R, item, buf)) for item, buf in zip(mix4, bufs)]
    infos = [srv.wait(t, check=False) for t in tickets]
    srv.close()
    assert infos[1].status == R.RPCA_ERR_ARG
    for k in (0, 2, 3):
        assert infos[k].status >= 0
        assert relF(bufs[k][1].double().cpu().numpy().T, refs[k].L) <= REL_TOL, k
    with pytest.raises(R.RpcaError):
        R.Server(_opts(R), None, R.rpca_server_opts_default(workers=0))
