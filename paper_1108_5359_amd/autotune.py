"""Autotuner of the batched form's launch shapes (``rpca_batch_tuning``).

Searches, on a device-resident batch shaped like the target workload, the
choices the library leaves open:

* ``lane_split2_p`` / ``lane_split4_p``: above which seed size a regression
  of the lane form runs on 2 / 4 lanes (fewer registers per lane, more waves,
  partial sums shuffled between lanes);
* ``filter_waves_per_cu``: size of the persistent filter grid;
* ``order``: work queue costliest side first, or problem order;
* ``recon_cols_per_wave``: columns streamed by one wave of the batched
  completion (the completion grid);
* ``recon_waves_per_cu``: most completion waves resident per CU (through
  their LDS reservation).

Coordinate descent over these grids from the library's defaults, each
candidate timed as the median of ``--reps`` runs of ``rpca_batch_run`` after
one warm-up run (the seed runs once per candidate plan and is not timed).
The result, with every measurement, is written as JSON; ``bench.py`` applies
it to the batched workload when the file exists.

Run on the GPU:  python -m paper_1108_5359_amd.autotune --out paper_1108_5359_amd/tuning_mi355x.json
"""
from __future__ import annotations

import argparse
import json
import pathlib
import sys
import time

import numpy as np

HERE = pathlib.Path(__file__).resolve().parent
ROOT = HERE.parent
DEFAULT_OUT = HERE / "tuning_mi355x.json"

GRID = {
    "lane_split": [(32, 64), (16, 64), (24, 48), (32, 48), (16, 32), (0, 64), (0, 0)],
    "filter_waves_per_cu": [4, 6, 8, 12, 16],
    "order": [0, 1],
    "recon_cols_per_wave": [8, 16, 32, 64, 128, 256],
    "recon_waves_per_cu": [0, 2, 3, 4, 6, 8],
}


def load(path=DEFAULT_OUT):
    """The tuned ``rpca_batch_tuning`` fields from a results file, or None."""
    p = pathlib.Path(path)
    if not p.exists():
        return None
    return json.loads(p.read_text()).get("batch_tuning")


def _make_batch(R, torch, ctx, specs, keep, tuning):
    jobs = [R.job(Md, s.m, s.n, s.m, s.r, dI, s.p, dJ, s.q, L, s.m, S, s.m)
            for s, (Md, L, S, dI, dJ) in zip(specs, keep)]
    b = R.Batch(ctx, jobs, R.rpca_opts_default(), tuning)
    R.rpca_batch_seed(b)
    return b


def _time(R, torch, b, reps):
    stream = torch.cuda.current_stream()
    R.rpca_batch_run(b, stream)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        R.rpca_batch_run(b, stream)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts))


def tune(njobs=256, seed=11, reps=5, rounds=2, log=print):
    import torch

    sys.path.insert(0, str(ROOT))
    import synth
    import paper_1108_5359_amd.rpca as R

    dev = torch.device("cuda:0")
    specs = synth.batch_specs(njobs, seed)
    keep = []
    for s in specs:
        Md, _, _ = synth.batch_job_device(s, device=dev)
        I, J = synth.seed_indices(s.m, s.n, s.p, s.q, seed=s.seed)
        keep.append((Md, torch.empty_like(Md), torch.empty_like(Md), torch.as_tensor(I).to(dev),
                     torch.as_tensor(J).to(dev)))
    torch.cuda.synchronize()
    ctx = R.Context(0)
    best = R.rpca_batch_tuning_default()
    measured = []

    def evaluate(t):
        b = _make_batch(R, torch, ctx, specs, keep, t)
        ms = _time(R, torch, b, reps)
        b.close()
        measured.append({"tuning": t.as_dict(), "ms": round(ms, 4)})
        log(f"autotune: {t.as_dict()} -> {ms:.3f} ms")
        return ms

    best_ms = evaluate(best)
    for rnd in range(rounds):
        improved = False
        for key, values in GRID.items():
            for v in values:
                cand = R.rpca_batch_tuning(*[getattr(best, f) for f, _ in best._fields_])
                if key == "lane_split":
                    if (cand.lane_split2_p, cand.lane_split4_p) == v:
                        continue
                    cand.lane_split2_p, cand.lane_split4_p = v
                else:
                    if getattr(cand, key) == v:
                        continue
                    setattr(cand, key, v)
                ms = evaluate(cand)
                if ms < best_ms * 0.99:
                    best, best_ms, improved = cand, ms, True
        if not improved:
            break
    ctx.close()
    props = torch.cuda.get_device_properties(0)
    return {
        "device": props.name,
        "compute_units": props.multi_processor_count,
        "workload": f"batched form: {njobs} problems from synth.batch_specs(seed={seed}) "
                    "(video-shaped, p = 10r <= 80)",
        "metric": "median ms of rpca_batch_run (steps 3-5 of every problem)",
        "batch_tuning": best.as_dict(),
        "best_ms": round(best_ms, 4),
        "default_ms": measured[0]["ms"],
        "measurements": measured,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--jobs", type=int, default=256)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--rounds", type=int, default=2)
    ap.add_argument("--out", default=str(DEFAULT_OUT))
    args = ap.parse_args()
    res = tune(args.jobs, args.seed, args.reps, args.rounds,
               log=lambda *a: print(*a, file=sys.stderr, flush=True))
    pathlib.Path(args.out).write_text(json.dumps(res, indent=1) + "\n")
    print(json.dumps({"batch_tuning": res["batch_tuning"], "best_ms": res["best_ms"],
                      "default_ms": res["default_ms"]}))


if __name__ == "__main__":
    main()
