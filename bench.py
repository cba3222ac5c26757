"""Benchmark: l1-filter solves/s on one MI355X.

Default workload (``--config c2``, the plain FP32 form): M = L0 + S0 with
m = n = 10000, rank r = 20 (Gaussian factors N(0, 1/10000)), 10% +-1
corruptions at uniformly random positions, seed block 200 x 200 at random
rows/columns.  One "step" is the whole hot path of l1 filtering over that
matrix: the 9800 column and 9800 row l1 regressions (Algorithm 1, one fused
launch) and the completion of L and S = M - L over all 10^8 entries.  The
seed PCP (a separate support stage) runs once before the timed region and is
reported as ``t_seed_ms``.  Inputs are resident in HBM when timing starts.
The precision form (FP16 contractions + FP32 refinement) is timed on the same
matrix and reported under ``detail.precision_form`` with its difference from
the FP32 result.

``--config c3``: m = n = 50000, r = 50, N(0, 2e-5) factors, 5% corruptions
uniform in [-1, 1], 500 x 500 seed, precision form (M: 10 GB).

``--config c5``: the served form.  A Poisson stream of requests drawn from a
mix (60% m = n = 2000, r = 5; 30% m = 20000 x n = 500, r = 10; 10% m = n =
20000, r = 30; N(0, 1/max(m, n)) factors, 10% +-1 corruptions, 10r x 10r
seeds, precision form) goes through the request loop (rpca_server_*, HBM
budget 200 GB).  Inputs are synthesised on the device before the clock runs
(a pool of instances per class that requests reuse).  Reported: the plain
GPU form's rate (rpca_solve on one request after another), the server's
rate at saturation (``value``), and p50 / p99 latency at 50%, 80%, 100% and
200% of the plain rate.

``--config c4``: the batched form, 256 independent problems shaped like video
background modelling (m ~ U{2048..76800} pixels, n ~ U{100..1000} frames,
r ~ U{1..8}, N(0, 1/m) factors, 5-15% block foregrounds U[0, 1], 10r x 10r
seeds; M: 22 GB).  One step is one ``rpca_batch_run``: every regression of
every problem in the persistent filter kernels, then every completion.

Prints ONE JSON line.  ``value`` = (column + row regressions) per second of
step time.  ``roofline`` describes the dominant kernel: algorithmic bytes or
flops per launch over its mean duration measured with HIP events on the launch
stream.  ``cpu_baseline`` times the FP64 reference (oracle) on a bounded
sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import pathlib
import sys
import time

import numpy as np

ROOT = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, GB/s
PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix
PEAK_FP16_MFMA_TFLOPS = 2500.0  # MI355X dense FP16/BF16 matrix

WORKLOADS = {
    "c2": dict(m=10000, n=10000, r=20, factor_std=np.sqrt(1e-4), sparsity=0.10, values="pm1",
               precision=0,
               text="plain form: m=n=10000, r=20, N(0,1e-4) factors, 10% +-1 corruptions, 200x200 "
                    "seed, 9800 column + 9800 row regressions of length 200, L and S over all 1e8 "
                    "entries"),
    "c3": dict(m=50000, n=50000, r=50, factor_std=np.sqrt(2e-5), sparsity=0.05, values="unif11",
               precision=1,
               text="precision form: m=n=50000, r=50, N(0,2e-5) factors, 5% U[-1,1] corruptions, "
                    "500x500 seed (FP64), 49500 column + 49500 row regressions of length 500 with "
                    "FP16 MFMA contractions and FP32 refinement, L and S over all 2.5e9 entries"),
}


BATCH = {"c4": dict(njobs=256, precision=0,
                   text="batched form: 256 problems, m ~ U{2048..76800}, n ~ U{100..1000}, "
                        "r ~ U{1..8}, N(0,1/m) factors, 5-15% U[0,1] block foregrounds, 10r x 10r "
                        "seeds; ~1.0e7 regressions of length 10-80; L and S over 5.6e9 entries")}


SERVE = {"c5": dict(classes=[("A", 2000, 2000, 5, 0.6, 6), ("B", 20000, 500, 10, 0.3, 4),
                            ("C", 20000, 20000, 30, 0.1, 2)],
                   sparsity=0.10, values="pm1", budget=200e9, precision=1,
                   text="served form: Poisson requests, 60% 2000x2000 r=5, 30% 20000x500 r=10, "
                        "10% 20000x20000 r=30, N(0,1/max(m,n)) factors, 10% +-1 corruptions, 10r x 10r "
                        "seeds, precision form, HBM budget 200 GB")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        h.update((ROOT / p).read_bytes())
    return h.hexdigest()[:16]


# filter kernel forms (rpca_filter_form): names, kernels, counter summary keys
FORM_NAMES = {0: "fp16", 1: "tile", 2: "split"}
FORM_KERNELS = {0: "l1_filter_kernel_f16 / _f16q (fp16 MFMA; the latter above p = 256)",
                1: "l1_filter_kernel (fp32 MFMA, tile form)",
                2: "l1_filter_split_kernel (fp32 MFMA, split form)"}
FORM_KEYS = {0: "l1_filter", 1: "l1_filter", 2: "l1_filter_split"}


def counter_traffic(kernel_key: str, digest: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when there is none or the kernel source changed since."""
    f = ROOT / "profiles" / f"{kernel_key}_counters.json"
    if not f.exists():
        return None
    d = json.loads(f.read_text())
    if d.get("source_digest") != digest:
        return None
    return d.get("hbm_bytes_per_launch")


class Workload:
    """Device-resident inputs and outputs of one l1-filtering run."""

    def __init__(self, name, seed, R, torch):
        import synth
        w = WORKLOADS[name]
        self.name, self.R, self.torch = name, R, torch
        self.m, self.n, self.r = w["m"], w["n"], w["r"]
        self.p = self.q = 10 * self.r
        dev = torch.device("cuda:0")
        self.dev = dev
        log(f"bench: generating {name}: m=n={self.m} r={self.r} (seed {seed})")
        self.Md, self.A0, self.B0 = synth.lowrank_plus_sparse_device(
            self.m, self.n, self.r, factor_std=w["factor_std"], sparsity=w["sparsity"],
            values=w["values"], seed=seed, device=dev)
        self.I, self.J = synth.seed_indices(self.m, self.n, self.p, self.q, seed=seed)
        self.Ic = np.setdiff1d(np.arange(self.m), self.I)
        self.Jc = np.setdiff1d(np.arange(self.n), self.J)
        self.nc, self.mr = len(self.Jc), len(self.Ic)
        T = lambda a: torch.as_tensor(a).to(dev)
        self.dI, self.dJ, self.dIc, self.dJc = T(self.I), T(self.J), T(self.Ic), T(self.Jc)
        r, p, q = self.r, self.p, self.q
        self.U = torch.zeros((r, p), dtype=torch.float64, device=dev)
        self.sg = torch.zeros(r, dtype=torch.float64, device=dev)
        self.V = torch.zeros((r, q), dtype=torch.float64, device=dev)
        self.Qt = torch.empty((self.nc, r), dtype=torch.float32, device=dev)
        self.Pt = torch.empty((self.mr, r), dtype=torch.float32, device=dev)
        self.kc = torch.empty(self.nc, dtype=torch.int32, device=dev)
        self.kr = torch.empty(self.mr, dtype=torch.int32, device=dev)
        self.L = torch.empty_like(self.Md)
        self.S = torch.empty_like(self.Md)
        self.ctx = R.Context(0)

    def seed(self):
        R, torch = self.R, self.torch
        t0 = time.perf_counter()
        st, self.r_used, self.seed_iters = R.rpca_seed(
            self.ctx, self.Md, self.m, self.n, self.m, self.dI, self.p, self.dJ, self.q, self.r,
            R.rpca_opts_default(), self.U, self.sg, self.V)
        torch.cuda.synchronize()
        self.t_seed_ms = (time.perf_counter() - t0) * 1e3
        log(f"bench: seed status={R.rpca_status_string(st)} r_used={self.r_used} "
            f"iters={self.seed_iters} t={self.t_seed_ms:.1f} ms")

    def step_overlapped(self, opts, stream):
        """Steps 3-5 in one call, the completion overlapped with the filter."""
        self.R.rpca_filter_complete(self.ctx, self.Md, self.m, self.n, self.m, self.dI, self.p,
                                    self.dJ, self.q, self.dJc, self.dIc, self.U, self.sg, self.V,
                                    self.r_used, opts, self.Qt, self.kc, self.Pt, self.kr, self.L,
                                    self.m, self.S, self.m, stream)

    def step(self, opts, stream, evs=None):
        """Steps 3-5 as two calls (filter, then completion), events around each."""
        R = self.R
        if evs:
            evs[0].record(stream)
        R.rpca_filter(self.ctx, self.Md, self.m, self.n, self.m, self.dI, self.p, self.dJ, self.q,
                      self.dJc, self.nc, self.dIc, self.mr, self.U, self.V, self.r_used, opts,
                      self.Qt, self.kc, self.Pt, self.kr, stream)
        if evs:
            evs[1].record(stream)
        R.rpca_reconstruct(self.ctx, self.Md, self.m, self.n, self.m, self.dI, self.p, self.dJ,
                           self.q, self.U, self.sg, self.V, self.r_used, self.Qt, self.Pt, self.L,
                           self.m, self.S, self.m, stream)
        if evs:
            evs[2].record(stream)

    def timed(self, opts, steps, warmup):
        """Headline: `steps` overlapped steps between two synchronisations.
        Then as many sequential steps with events around each kernel launch
        (the per-kernel durations of the roofline)."""
        torch = self.torch
        stream = torch.cuda.current_stream()
        overlap = opts.overlap_chunks > 0
        for _ in range(warmup):
            (self.step_overlapped if overlap else self.step)(opts, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            (self.step_overlapped if overlap else self.step)(opts, stream)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        for k in range(steps):
            self.step(opts, stream, events[k])
        torch.cuda.synchronize()
        filt_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in events]))
        recon_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in events]))
        K = np.abs(np.concatenate([self.kc.cpu().numpy(), self.kr.cpu().numpy()]).astype(np.int64))
        unconv = int((np.concatenate([self.kc.cpu().numpy(), self.kr.cpu().numpy()]) < 0).sum())
        return elapsed, filt_ms, recon_ms, K, unconv


class BatchWorkload:
    """Device-resident batch of independent problems (the c4 recipe)."""

    def __init__(self, name, seed, R, torch, tuning=None):
        import synth
        w = BATCH[name]
        self.name, self.R, self.torch = name, R, torch
        dev = torch.device("cuda:0")
        self.dev = dev
        self.specs = synth.batch_specs(w["njobs"], seed)
        log(f"bench: generating {name}: {len(self.specs)} problems")
        self.keep, jobs = [], []
        t0 = time.perf_counter()
        for s in self.specs:
            Md, _, _ = synth.batch_job_device(s, device=dev)
            I, J = synth.seed_indices(s.m, s.n, s.p, s.q, seed=s.seed)
            dI, dJ = torch.as_tensor(I).to(dev), torch.as_tensor(J).to(dev)
            L = torch.empty_like(Md)
            S = torch.empty_like(Md)
            self.keep.append((Md, L, S, dI, dJ, I, J))
            jobs.append(R.job(Md, s.m, s.n, s.m, s.r, dI, s.p, dJ, s.q, L, s.m, S, s.m))
        torch.cuda.synchronize()
        log(f"bench: generated in {time.perf_counter() - t0:.1f} s")
        self.ctx = R.Context(0)
        self.tuning = tuning if tuning is not None else R.rpca_batch_tuning_default()
        self.tuning_source = "library defaults" if tuning is None else "autotuner"
        self.batch = R.Batch(self.ctx, jobs, R.rpca_opts_default(precision=w["precision"]),
                             self.tuning)
        self.regs = sum((s.m - s.p) + (s.n - s.q) for s in self.specs)
        self.elems = sum(s.m * s.n for s in self.specs)
        self.filter_elems = sum((s.m - s.p) * s.q + (s.n - s.q) * s.p for s in self.specs)

    def seed(self):
        R = self.R
        t0 = time.perf_counter()
        st = R.rpca_batch_seed(self.batch)
        self.t_seed_ms = (time.perf_counter() - t0) * 1e3
        self.infos = [R.rpca_batch_job_info(self.batch, k)[1] for k in range(len(self.specs))]
        ranks = [i.r_used for i in self.infos]
        log(f"bench: batch seed status={R.rpca_status_string(st)} t={self.t_seed_ms:.0f} ms "
            f"r_used mean {np.mean(ranks):.2f}")

    def timed(self, steps, warmup):
        torch, R = self.torch, self.R
        stream = torch.cuda.current_stream()
        for _ in range(warmup):
            R.rpca_batch_run(self.batch, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            R.rpca_batch_run(self.batch, stream)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        # phase times (filter / completion) from the batch's own events, one
        # synchronized run at a time
        fs, rs = [], []
        for _ in range(max(3, min(steps, 10))):
            R.rpca_batch_run(self.batch, stream)
            info = R.rpca_batch_job_info(self.batch, 0)[1]
            fs.append(info.t_filter_ms)
            rs.append(info.t_reconstruct_ms)
        infos = [R.rpca_batch_job_info(self.batch, k)[1] for k in range(len(self.specs))]
        return elapsed, float(np.mean(fs)), float(np.mean(rs)), infos


def calibrate_copy(torch, dev):
    """A plain elementwise pass reading 1 GiB and writing 1 GiB (one kernel
    per call), for scaling the FETCH_SIZE / WRITE_SIZE counters of a
    profiled run to bytes."""
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        torch.add(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst


def main_batch(args, R, torch):
    from paper_1108_5359_amd import autotune
    tuned = None if args.no_tuned else autotune.load()
    tuning = R.rpca_batch_tuning_default(**tuned) if tuned else None
    wl = BatchWorkload(args.config, args.seed, R, torch, tuning)
    wl.seed()
    if args.calibrate_copy:
        calibrate_copy(torch, wl.dev)
    elapsed, filt_ms, recon_ms, infos = wl.timed(args.steps, args.warmup)
    ms_per_step = elapsed * 1e3 / args.steps
    value = wl.regs * args.steps / elapsed
    iters_total = sum(i.filt_iters_total for i in infos)
    unconv = sum(i.filt_not_converged for i in infos)
    log(f"bench: {wl.name} {ms_per_step:.3f} ms/step  filter {filt_ms:.3f} ms  completion "
        f"{recon_ms:.3f} ms  K mean {iters_total / wl.regs:.1f}  unconverged {unconv}")
    recon_bytes = 12.0 * wl.elems
    recon_gbs = recon_bytes / (recon_ms * 1e-3) / 1e9
    # filter: algorithmic flops of both contractions per iteration (4 p r per
    # regression); per-regression iteration counts are summed per side
    filt_flops = 0.0
    for s, i in zip(wl.specs, infos):
        filt_flops += 4.0 * s.p * i.r_used * i.filt_iters_total
    filt_tflops = filt_flops / (filt_ms * 1e-3) / 1e12
    digest = source_digest(["paper_1108_5359_amd/csrc/recon_kernel.h",
                            "paper_1108_5359_amd/csrc/batch.hip"])
    if recon_ms >= filt_ms:
        roofline = {"bound": "hbm", "kernel": "batch_reconstruct (+ batch_assemble)",
                    "achieved": round(recon_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(recon_gbs / PEAK_HBM_GBS, 4),
                    "traffic": counter_traffic(f"batch_reconstruct_{args.config}", digest)}
    else:
        roofline = {"bound": "mfma", "kernel": "lane_filter_kernel (fp32 4x4x1 MFMA)",
                    "achieved": round(filt_tflops, 3), "peak": PEAK_FP32_MFMA_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(filt_tflops / PEAK_FP32_MFMA_TFLOPS, 4),
                    "traffic": counter_traffic(f"lane_filter_{args.config}", digest)}
    detail = {"overlap_chunks": args.overlap_chunks,
              "filter_ms": round(filt_ms, 4), "reconstruct_ms": round(recon_ms, 4),
              "sequential_ms_per_step": round(filt_ms + recon_ms, 4),
              "reconstruct_gbs": round(recon_gbs, 1),
              "filter_tflops_contraction": round(filt_tflops, 3),
              "iters_mean": round(iters_total / wl.regs, 2),
              "iters_max": int(max(i.filt_iters_max for i in infos)), "unconverged": int(unconv),
              "t_seed_ms": round(wl.t_seed_ms, 1), "jobs": len(wl.specs),
              "tuning": wl.tuning.as_dict(), "tuning_source": wl.tuning_source}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_batch(wl, args.cpu_sample if args.cpu_sample is not None else 6,
                                 args.cpu_seconds)
    out = {
        "metric": "l1-filter solves/s (column + row l1 regressions, with completion of L and S)",
        "value": round(value, 1),
        "unit": "regressions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": BATCH[args.config]["text"], "name": args.config,
                   "problems": len(wl.specs), "regressions": wl.regs,
                   "elements": wl.elems},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(out), flush=True)
    wl.batch.close()
    wl.ctx.close()


def cpu_baseline_batch(wl, njobs, seconds):
    """The FP64 oracle as it stands on the host cores: Algorithm 2 (seed,
    every column and row regression, completion) on the problems of the batch
    in order, from host copies of their M: at least ``njobs`` of them, and on
    until ``seconds`` of oracle time have been spent (or every problem is
    done)."""
    import oracle
    oracle.build()
    threads = oracle.num_threads(0)
    regs, t, k = 0, 0.0, 0
    while k < len(wl.specs) and (k < njobs or t < seconds):
        s = wl.specs[k]
        Md, L, S, dI, dJ, I, J = wl.keep[k]
        Mh = np.asfortranarray(Md.cpu().numpy().T)
        t0 = time.perf_counter()
        oracle.solve(Mh, s.r, I, J)
        t += time.perf_counter() - t0
        regs += (s.m - s.p) + (s.n - s.q)
        k += 1
    njobs = k
    log(f"bench: cpu oracle {regs} regressions ({njobs} problems) in {t:.2f} s, threads {threads}")
    return {"value": round(regs / t, 1), "unit": "regressions/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the first {njobs} problems of the batch, whole (seed, {regs} column + row "
                      f"regressions, completion), FP64",
            "seconds": round(t, 2)}


def main_serve(args, R, torch):
    import threading
    import synth
    w = SERVE[args.config]
    dev = torch.device("cuda:0")
    rng = np.random.Generator(np.random.PCG64([args.seed, 0xC5]))
    # a pool of device-resident instances per class
    pool = {}
    t0 = time.perf_counter()
    for name, m, n, r, frac, count in w["classes"]:
        pool[name] = []
        for k in range(count):
            s = 1000 * args.seed + 10 * len(pool) + k
            Md, _, _ = synth.lowrank_plus_sparse_device(m, n, r, factor_std=np.sqrt(1.0 / max(m, n)),
                                                        sparsity=w["sparsity"], values=w["values"],
                                                        seed=s, device=dev)
            I, J = synth.seed_indices(m, n, 10 * r, 10 * r, seed=s)
            pool[name].append((Md, m, n, r, torch.as_tensor(I).to(dev), torch.as_tensor(J).to(dev)))
    torch.cuda.synchronize()
    log(f"bench: generated the request pool in {time.perf_counter() - t0:.1f} s")
    names = [c[0] for c in w["classes"]]
    fracs = np.array([c[4] for c in w["classes"]])
    counters = {nm: 0 for nm in names}

    def draw(nreq):
        reqs = []
        for _ in range(nreq):
            nm = names[int(rng.choice(len(names), p=fracs))]
            inst = pool[nm][counters[nm] % len(pool[nm])]
            counters[nm] += 1
            reqs.append((nm, inst))
        return reqs

    opts = R.rpca_opts_default(precision=w["precision"])
    # plain GPU form: rpca_solve on one request after another
    ctx = R.Context(0)
    plain_reqs = draw(args.plain_requests)
    lat_plain = {nm: [] for nm in names}
    for nm, (Md, m, n, r, dI, dJ) in plain_reqs[:3]:           # warm-up
        L = torch.empty_like(Md)
        S = torch.empty_like(Md)
        R.rpca_solve(ctx, Md, m, n, m, r, opts, dI, dJ, L, m, S, m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for nm, (Md, m, n, r, dI, dJ) in plain_reqs:
        t1 = time.perf_counter()
        L = torch.empty_like(Md)
        S = torch.empty_like(Md)
        R.rpca_solve(ctx, Md, m, n, m, r, opts, dI, dJ, L, m, S, m)
        lat_plain[nm].append((time.perf_counter() - t1) * 1e3)
        del L, S
    plain_s = time.perf_counter() - t0
    plain_rate = len(plain_reqs) / plain_s
    log(f"bench: plain form {plain_rate:.2f} solves/s over {len(plain_reqs)} requests")

    srv = R.Server(opts, None, R.rpca_server_opts_default(hbm_budget_bytes=w["budget"],
                                                          workers=args.workers,
                                                          max_batch=args.max_batch))

    def run_stream(reqs, qps):
        """Submit at Poisson arrival times (qps = None: all at once); wait for all."""
        gaps = rng.exponential(1.0 / qps, len(reqs)) if qps else np.zeros(len(reqs))
        arrivals = np.cumsum(gaps)
        tickets, bufs = [None] * len(reqs), [None] * len(reqs)
        infos = [None] * len(reqs)
        done = threading.Event()

        def waiter():
            for k in range(len(reqs)):
                while tickets[k] is None:
                    time.sleep(0.0002)
                infos[k] = srv.wait(tickets[k], check=False)
                bufs[k] = None                                   # outputs no longer needed
            done.set()

        th = threading.Thread(target=waiter)
        th.start()
        t_start = time.perf_counter()
        for k, (nm, (Md, m, n, r, dI, dJ)) in enumerate(reqs):
            delay = t_start + arrivals[k] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            L = torch.empty_like(Md)
            S = torch.empty_like(Md)
            bufs[k] = (L, S)
            tickets[k] = srv.submit(R.job(Md, m, n, m, r, dI, 10 * r, dJ, 10 * r, L, m, S, m))
        done.wait()
        th.join()
        lat = np.array([i.t_done_ms - i.t_submit_ms for i in infos])
        span = (max(i.t_done_ms for i in infos) - min(i.t_submit_ms for i in infos)) / 1e3
        by_class = {}
        for nm in names:
            sel = [x for (c, _), x in zip(reqs, lat) if c == nm]
            if sel:
                by_class[nm] = {"n": len(sel), "p50_ms": round(float(np.percentile(sel, 50)), 2),
                                "p99_ms": round(float(np.percentile(sel, 99)), 2)}
        failed = sum(1 for i in infos if i.status < 0)
        return {"offered_qps": round(qps, 3) if qps else None,
                "achieved_solves_per_s": round(len(reqs) / span, 3),
                "p50_ms": round(float(np.percentile(lat, 50)), 2),
                "p99_ms": round(float(np.percentile(lat, 99)), 2),
                "mean_batch": round(float(np.mean([i.batch_size for i in infos])), 2),
                "failed": failed, "by_class": by_class}, infos, reqs

    run_stream(draw(6), None)                                      # warm-up of the workers
    sat, sat_infos, sat_reqs = run_stream(draw(args.requests), None)
    log(f"bench: server at saturation {sat['achieved_solves_per_s']:.2f} solves/s "
        f"(mean batch {sat['mean_batch']})")
    levels = []
    for f in (0.5, 0.8, 1.0, 2.0):
        res, _, _ = run_stream(draw(args.requests), f * plain_rate)
        res["load"] = f"{int(f * 100)}% of the plain rate"
        levels.append(res)
        log(f"bench: {res['load']}: {res['achieved_solves_per_s']:.2f} solves/s, p50 "
            f"{res['p50_ms']:.1f} ms, p99 {res['p99_ms']:.1f} ms, mean batch {res['mean_batch']}")
    st = srv.stats()
    srv.close()

    # roofline of the completion over the saturation run's batches (one record
    # per batch: requests of a batch finish at the same instant)
    batches = {}
    for (nm, (Md, m, n, r, dI, dJ)), i in zip(sat_reqs, sat_infos):
        b = batches.setdefault(round(i.t_done_ms, 6), [0.0, i.info.t_reconstruct_ms])
        b[0] += 12.0 * m * n
    rb = sum(v[0] for v in batches.values())
    rt = sum(v[1] for v in batches.values()) * 1e-3
    recon_gbs = rb / rt / 1e9 if rt > 0 else 0.0
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        Md, m, n, r, dI, dJ = pool["A"][0]
        Mh = np.asfortranarray(Md.cpu().numpy().T)
        I, J = dI.cpu().numpy(), dJ.cpu().numpy()
        t0 = time.perf_counter()
        ns = 0
        while ns < 3 or time.perf_counter() - t0 < args.cpu_seconds:
            oracle.solve(Mh, r, I, J)
            ns += 1
        tc = time.perf_counter() - t0
        cpu = {"value": round(ns / tc, 3), "unit": "solves/s", "cores": oracle.num_threads(0),
               "kind": "oracle",
               "sample": f"{ns} solves of a class-A request (2000 x 2000, r = 5): seed, every "
                         "column and row regression, completion, FP64", "seconds": round(tc, 2)}
    out = {
        "metric": "served PCP solves/s (request mix, p50/p99 latency)",
        "value": sat["achieved_solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": 6,
        "ms_per_step": round(1e3 / sat["achieved_solves_per_s"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 data, f16 contractions / f32 state (p >= 48), f64 seed",
        "data": "synthetic",
        "config": {"workload": w["text"], "name": args.config, "workers": args.workers,
                   "max_batch": args.max_batch, "requests_per_level": args.requests},
        "roofline": {"bound": "hbm", "kernel": "completion of the served batches",
                     "achieved": round(recon_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(recon_gbs / PEAK_HBM_GBS, 4), "traffic": None},
        "cpu_baseline": cpu,
        "detail": {"plain_solves_per_s": round(plain_rate, 3),
                   "served_vs_plain": round(sat["achieved_solves_per_s"] / plain_rate, 3),
                   "plain_latency_ms": {nm: round(float(np.median(v)), 2) for nm, v in lat_plain.items() if v},
                   "saturation": sat, "levels": levels, "server": st.as_dict()},
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS) + sorted(BATCH) + sorted(SERVE))
    ap.add_argument("--requests", type=int, default=60, help="served form: requests per load level")
    ap.add_argument("--plain-requests", type=int, default=20,
                    help="served form: requests of the plain-rate measurement")
    ap.add_argument("--workers", type=int, default=3, help="served form: worker threads")
    ap.add_argument("--no-tuned", action="store_true",
                    help="batched form: library defaults instead of the autotuner's results")
    ap.add_argument("--max-batch", type=int, default=64, help="served form: requests per batch")
    ap.add_argument("--precision", type=int, default=None, help="0 = FP32, 1 = FP16 + refinement")
    ap.add_argument("--overlap-chunks", type=int, default=0,
                    help="column slabs of the overlapped filter + completion (0 = one after the other)")
    ap.add_argument("--filter-form", type=int, default=0,
                    help="FP32 filter kernel: 0 = automatic, 1 = tile form, 2 = split form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip timing the other precision form")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="regressions in the CPU baseline sample (0 = all; default: all at c2, "
                         "8000 at c3)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU baseline: repeat the sample (or take further problems of a batch) "
                         "until this much oracle time has been spent")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy (for scaling the "
                         "FETCH_SIZE / WRITE_SIZE counters of a profiled run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the method shards by regressions and row blocks, see the design notes",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1108_5359_amd.rpca as R

    if args.config in BATCH:
        return main_batch(args, R, torch)
    if args.config in SERVE:
        return main_serve(args, R, torch)
    wl = Workload(args.config, args.seed, R, torch)
    wl.seed()
    precision = WORKLOADS[args.config]["precision"] if args.precision is None else args.precision
    opts = R.rpca_opts_default(precision=precision, overlap_chunks=args.overlap_chunks,
                               filter_form=args.filter_form)
    form = R.rpca_filter_form(wl.ctx, wl.p, wl.r_used, wl.nc + wl.mr, opts)

    if args.calibrate_copy:
        calibrate_copy(torch, wl.dev)

    elapsed, filt_ms, recon_ms, K, unconv = wl.timed(opts, args.steps, args.warmup)
    ms_per_step = elapsed * 1e3 / args.steps
    regs = wl.nc + wl.mr
    value = regs * args.steps / elapsed
    log(f"bench: precision={precision} form={FORM_NAMES[form]} overlap_chunks={args.overlap_chunks} "
        f"{ms_per_step:.3f} ms/step "
        f"(kernels one after the other: filter {filt_ms:.3f} ms + reconstruct {recon_ms:.3f} ms)  "
        f"K mean {K.mean():.1f} max {K.max()} unconverged {unconv}")

    # Algorithmic work per launch: the filter's two contractions per iteration
    # (A^T g and A w: 4 p r flops per regression), the completion's 12 bytes
    # per element (read M, write L, write S).
    filt_flops = float(4.0 * wl.p * wl.r_used * K.sum())
    recon_bytes = float(12.0 * wl.m * wl.n)
    filt_tflops = filt_flops / (filt_ms * 1e-3) / 1e12
    recon_gbs = recon_bytes / (recon_ms * 1e-3) / 1e9
    if filt_ms >= recon_ms:
        digest = source_digest(["paper_1108_5359_amd/csrc/filter_kernel.h"])
        peak = PEAK_FP16_MFMA_TFLOPS if form == 0 else PEAK_FP32_MFMA_TFLOPS
        roofline = {"bound": "mfma", "kernel": FORM_KERNELS[form],
                    "achieved": round(filt_tflops, 3), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(filt_tflops / peak, 4),
                    "traffic": counter_traffic(f"{FORM_KEYS[form]}_{args.config}", digest)}
    else:
        digest = source_digest(["paper_1108_5359_amd/csrc/reconstruct.hip",
                                "paper_1108_5359_amd/csrc/recon_kernel.h"])
        roofline = {"bound": "hbm", "kernel": "reconstruct_kernel (+ assemble_factors)",
                    "achieved": round(recon_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(recon_gbs / PEAK_HBM_GBS, 4),
                    "traffic": counter_traffic(f"reconstruct_{args.config}", digest)}

    detail = {"overlap_chunks": args.overlap_chunks, "filter_form": FORM_NAMES[form],
              "filter_ms": round(filt_ms, 4), "reconstruct_ms": round(recon_ms, 4),
              "sequential_ms_per_step": round(filt_ms + recon_ms, 4),
              "filter_tflops_contraction": round(filt_tflops, 3),
              "reconstruct_gbs": round(recon_gbs, 1), "iters_mean": round(float(K.mean()), 2),
              "iters_max": int(K.max()), "unconverged": unconv,
              "t_seed_ms": round(wl.t_seed_ms, 1), "seed_iters": wl.seed_iters,
              "r_used": wl.r_used, "precision": precision}

    if not args.no_compare:
        # the other precision form on the same matrix, and how far apart they are
        Q0 = wl.Qt.clone()
        P0 = wl.Pt.clone()
        other = 1 - precision
        key = "precision_form" if other == 1 else "plain_fp32_form"
        try:
            e2, f2, r2, K2, u2 = wl.timed(R.rpca_opts_default(precision=other,
                                                              overlap_chunks=args.overlap_chunks),
                                          args.steps, 1)
        except R.RpcaError as err:
            detail[key] = {"unsupported": str(err)}
            e2 = None
    if not args.no_compare and e2 is not None:
        Uh = wl.U.cpu().numpy()          # (r, p) = U^T
        Vh = wl.V.cpu().numpy()
        dq = np.linalg.norm((wl.Qt.double() - Q0.double()).cpu().numpy() @ Uh)
        nq = np.linalg.norm(Q0.double().cpu().numpy() @ Uh)
        dp = np.linalg.norm((wl.Pt.double() - P0.double()).cpu().numpy() @ Vh)
        np_ = np.linalg.norm(P0.double().cpu().numpy() @ Vh)
        detail[key] = {"value": round(regs * args.steps / e2, 1),
                       "ms_per_step": round(e2 * 1e3 / args.steps, 4), "filter_ms": round(f2, 4),
                       "reconstruct_ms": round(r2, 4), "iters_mean": round(float(K2.mean()), 2),
                       "unconverged": u2,
                       "relF_vs_headline_form": round(float(np.hypot(dq, dp) / np.hypot(nq, np_)), 10)}
        log(f"bench: precision={other} {e2 * 1e3 / args.steps:.3f} ms/step  filter {f2:.3f} ms")
        wl.timed(opts, 1, 0)        # leave the headline form's outputs in place

    if not args.no_compare and form in (1, 2):
        # the other FP32 kernel form on the same matrix
        other_form = 3 - form
        o2 = R.rpca_opts_default(precision=precision, overlap_chunks=args.overlap_chunks,
                                 filter_form=other_form)
        if R.rpca_filter_form(wl.ctx, wl.p, wl.r_used, wl.nc + wl.mr, o2) == other_form:
            e3, f3, r3, K3, u3 = wl.timed(o2, args.steps, 1)
            detail[f"{FORM_NAMES[other_form]}_form"] = {
                "ms_per_step": round(e3 * 1e3 / args.steps, 4), "filter_ms": round(f3, 4),
                "iters_mean": round(float(K3.mean()), 2), "unconverged": u3}
            log(f"bench: form={FORM_NAMES[other_form]} {e3 * 1e3 / args.steps:.3f} ms/step  filter {f3:.3f} ms")
            wl.timed(opts, 1, 0)

    cpu = None
    if not args.no_cpu_baseline:
        sample = args.cpu_sample if args.cpu_sample is not None else (0 if args.config == "c2" else 8000)
        cpu = cpu_baseline(wl, sample, args.cpu_seconds)

    out = {
        "metric": "l1-filter solves/s (column + row l1 regressions, with completion of L and S)",
        "value": round(value, 1),
        "unit": "regressions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if precision == 0 else "f16 contractions / f32 state",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config]["text"], "name": args.config,
                   "m": wl.m, "n": wl.n, "r": wl.r, "seed_block": [wl.p, wl.q],
                   "regressions": regs},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(out), flush=True)
    wl.ctx.close()


def cpu_baseline(wl, sample, seconds):
    """The FP64 oracle as it stands on the host cores: Algorithm 1 (literal
    form, OpenMP over regressions) on a sample of the column and row
    regressions of the same matrix with the same seed factors, plus (for the
    full sample at m*n <= 1e8) the four-block completion and S = M - L; the
    pass is repeated until ``seconds`` of oracle time have been spent."""
    import oracle
    oracle.build()
    torch = wl.torch
    threads = oracle.num_threads(0)
    nreg = wl.nc + wl.mr
    if sample and sample < nreg:
        cols = wl.Jc[: sample // 2]
        rows = wl.Ic[: sample - sample // 2]
    else:
        cols, rows = wl.Jc, wl.Ic
    U = wl.U.cpu().numpy().T
    V = wl.V.cpu().numpy().T
    sigma = wl.sg.cpu().numpy()
    ru = wl.r_used
    U, V, sigma = U[:, :ru], V[:, :ru], sigma[:ru]
    # host copies of the regression inputs (column-major M: Md[j, i] = M[i, j])
    Xc = wl.Md[torch.as_tensor(cols).to(wl.dev)][:, torch.as_tensor(wl.I).to(wl.dev)]
    Xc = Xc.double().cpu().numpy().T                       # p x len(cols)
    Xr = wl.Md[torch.as_tensor(wl.J).to(wl.dev)][:, torch.as_tensor(rows).to(wl.dev)]
    Xr = Xr.double().cpu().numpy()                          # q x len(rows)
    full = len(cols) == wl.nc and len(rows) == wl.mr and wl.m * wl.n <= 100_000_000
    Mh = wl.Md.cpu().numpy().T if full else None
    t_f = t_c = 0.0
    passes = 0
    while passes == 0 or t_f + t_c < seconds:
        t0 = time.perf_counter()
        Qt, _ = oracle.alg1_batch(Xc, U)
        Pt, _ = oracle.alg1_batch(Xr, V)
        t_f += time.perf_counter() - t0
        if full:
            t0 = time.perf_counter()
            oracle.complete(Mh, wl.I, wl.J, U, sigma, V, Qt, Pt)
            t_c += time.perf_counter() - t0
        passes += 1
    t = t_f + t_c
    log(f"bench: cpu oracle {passes} x {len(cols) + len(rows)} regressions in {t_f:.2f} s, "
        f"completion {t_c:.2f} s, threads {threads}")
    return {"value": round(passes * (len(cols) + len(rows)) / t, 1), "unit": "regressions/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{len(cols)} column + {len(rows)} row regressions of the same matrix "
                      f"(FP64, Algorithm 1 literal form)"
                      f"{' + completion of all entries' if full else ' (no completion)'}"
                      f", {passes} pass{'es' if passes > 1 else ''}",
            "seconds": round(t, 2)}


if __name__ == "__main__":
    main()
