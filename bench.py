"""Benchmark of the 3D space-order-8 acoustic wave sweep on one MI355X.

One bench step = one whole run of the headline workload: the 3D so-8
isotropic acoustic wave on a 512^3 interior (halo 4), layered velocity,
Ricker source at the centre, 400 leapfrog steps, FP32 fields, inputs resident
in HBM.  value = grid-point updates per second (GPts/s) over the timed steps.

Also reported on the same GPU (`variants`):
  * 16-bit storage (bf16 / f16, FP32 arithmetic) of the same workload;
  * the 3D so-4 heat sweep, 512^3, 50 steps;
  * 32 independent shots of uneven sizes 128^3..384^3, 200 steps, in one
    launch per step (one graph), against 32 sequential plain runs;
  * the checkpointed misfit gradient (256^3, 500 steps, 64 receivers,
    checkpoints every 25 steps) against the plain forward of the same model.
`parity` compares the headline run with the FP64 oracle over all 400 steps,
and `cpu_baseline` is that same oracle run's time on all host threads (the
oracle compiled -O3 -march=native on the host; and, labelled as such, on one
thread for two steps).  `roofline` prices each point update at the plain
sweep's algorithmic bytes (u^n, u^{n-1}, beta read, u^{n+1} written: 16 B in
FP32), times the updates of one launch of the dominant kernel.
`runs` holds the median and minimum of the timed runs and the first run's
time, which includes capturing the run's graph.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GPts/s + % of HBM peak, 3D so-8 wave; batched & adjoint vs plain, same GPU"
COUNTERS = os.path.join(ROOT, "profiles", "counters.json")
CSRC = os.path.join(ROOT, "paper_2404_02218_amd", "csrc")
# the stored traffic is tied to the sources the headline's kernels compile
# from: the translation units of the plain and temporally blocked FP32 sweeps,
# every header they include and the build script that holds their compiler
# flags (the host runtime and the other kernels do not change what these
# kernels move)
KERNEL_SOURCES = [os.path.join(CSRC, f) for f in
                  ("zmarch_tb.hip", "zmarch_f32.hip", "zmarch_tb.hpp", "zmarch.hpp", "kernels.hpp", "device.hpp")] + \
                 [os.path.join(ROOT, "paper_2404_02218_amd", "build.py")]


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
    ap.add_argument("--only-heat", action="store_true",
                    help="the 3D so-4 heat leg only, --variant and --heat-steps apply (profiling)")
    ap.add_argument("--heat-steps", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--variant", default="-1",
                    help="force a kernel variant, by number or by name (else tune)")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"],
                    help="storage dtype of the headline leg (profiling of the 16-bit kernels)")
    ap.add_argument("--leg", default=None,
                    choices=["pw", "pw_loop", "slab", "faces", "absorbing", "heat2d", "batch", "adjoint",
                             "precision"],
                    help="run one secondary leg only and print its JSON (profiling)")
    ap.add_argument("--batch-steps", type=int, default=200, help="leapfrog steps of the batched-shots leg")
    ap.add_argument("--batch-variant", default=None,
                    help="batched-shots leg: run this variant only (no tuning, no sequential runs; profiling)")
    ap.add_argument("--adjoint-steps", type=int, default=500, help="leapfrog steps of the gradient leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 1 GiB device copies (for counter scaling)")
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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(variant_name: str):
    """HBM bytes per launch of the headline kernel from the committed counter
    summary, if it was taken from the current kernel source and variant."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    e = c.get("wave3d_so8_512", {}).get(variant_name)
    if not e:
        return None
    return e.get("hbm_bytes_per_launch")


def stream_copy_gbs(nbytes=1 << 30, reps=10):
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    with Timer() as t:
        for _ in range(reps):
            b.copy_(a)
    return 2.0 * nbytes * reps / (t.ms * 1e-3) / 1e9


def launch_model(vname, nsteps, es, storage):
    """The dominant kernel of a wave run: (temporally blocked?, launches per
    run, the kernel's own bytes per launch per interior point, its name).
    Plain sweep: one launch per step reads u^n, u^{n-1}, beta and writes
    u^{n+1} (4 fields).  Depth-2 temporal blocking: one launch per two steps
    reads the same 3 fields and writes u^{n+1} and u^{n+2} (5 fields); the
    runtime runs an even number of such passes and plain sweeps for the
    remaining steps (none for 400 steps).  The roofline itself prices every
    point update at the plain sweep's 4 fields (the algorithmic bytes of one
    update), so a launch of two steps counts 8 fields."""
    if vname.startswith("tb2_"):
        passes = nsteps // 2 - ((nsteps // 2) & 1)
        return True, passes + (nsteps - 2 * passes), 5 * es, f"k_tb2<{storage}>"
    return False, nsteps, 4 * es, f"k_zmarch<wave, r=4, {storage}>"


def resolve_variant(plan, spec) -> int:
    """The plan's variant number for `spec`: a number, or a variant name
    (names stay the same when variants are added); -1 for none."""
    spec = str(spec)
    try:
        return int(spec)
    except ValueError:
        pass
    names = {plan.variant_name(v): v for v in range(plan.variant_count())}
    if spec not in names:
        raise SystemExit(f"unknown variant {spec!r}; this plan has {sorted(names)}")
    return names[spec]


def wave_setup(S, W, n, nsteps, dtype, variant):
    import torch
    P = W.wave3d_c3(n=n, nsteps=nsteps)
    dn = {S.F32: "f32", S.BF16: "bf16", S.F16: "f16"}[dtype]
    plan = S.Plan(S.WAVE2, P.shape, 4, S.second_derivative_weights(8), halo=4, dtype=dtype)
    f = [plan.field() for _ in range(3)]
    f[2].load(W.embed(W.round_to_storage(P.beta, dn), 4))
    amp = torch.from_numpy(P.src_amp).cuda()
    variant = resolve_variant(plan, variant)
    if variant >= 0:
        plan.variant = variant
    else:
        plan.tune(f, reps=3)
    return P, plan, f, amp


def time_wave(plan, f, amp, P, steps, warmup, per_run=None):
    """Mean ms per run over `steps` timed runs (after `warmup` untimed ones).
    per_run, if a dict, receives the first warm-up run's wall time (which
    includes capturing and instantiating the run's graph) and the median and
    minimum of the timed runs, each bracketed by its own events."""
    import torch

    def one():
        f[0].storage.zero_()
        f[1].storage.zero_()
        plan.run(f, P.nsteps, src=P.src, src_amp=amp)

    for k in range(warmup):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one()
        torch.cuda.synchronize()
        if k == 0 and per_run is not None:
            per_run["first_run_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    with Timer() as t:
        for k in range(steps):
            ev[k].record()
            one()
        ev[steps].record()
    if per_run is not None:
        runs = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(steps))
        per_run["median_ms"] = round(float(np.median(runs)), 3)
        per_run["min_ms"] = round(runs[0], 3)
    return t.ms / steps


def native_oracle():
    """Build the FP64 oracle with -O3 -march=native for this host (the
    in-tree build is for any x86-64 host) and load it; returns its path."""
    import tempfile

    import oracle
    from oracle.build import build
    path = os.path.join(tempfile.mkdtemp(prefix="oracle_native_"), "liboracle_native.so")
    build(native=True, out=path)
    oracle.use_library(path)
    return path


def headline_oracle_run(S, W, plan, f, n, nsteps, final_timed, every=20):
    """The headline run once more, on the GPU and in the FP64 oracle, in
    segments of `every` steps (an even count, so the oracle's levels stay in
    place): the error over the run (max over the levels at every segment end
    of |gpu - oracle| over max |oracle|), the GPU's final levels against the
    timed run's (bitwise), and the oracle's time on all host threads, which
    is the CPU baseline of the full configuration."""
    import torch

    import oracle
    threads = len(os.sched_getaffinity(0))
    os.environ["OMP_NUM_THREADS"] = str(threads)
    lib = native_oracle()
    P = W.wave3d_c3(n=n, nsteps=nsteps)
    bb = np.ascontiguousarray(W.embed(W.round_to_storage(P.beta, "f32"), 4))
    a = np.zeros_like(bb)
    b = np.zeros_like(bb)
    c = oracle.fd_weights_float(8)
    f[0].zero()
    f[1].zero()
    num = den = 0.0
    secs = 0.0
    for t0 in range(0, nsteps, every):
        k = min(every, nsteps - t0)
        amp = np.ascontiguousarray(P.src_amp[t0:t0 + k])
        plan.run(f, k, src=P.src, src_amp=torch.from_numpy(amp).cuda())
        torch.cuda.synchronize()
        got = f[0].interior(4)
        t = time.perf_counter()
        oracle.wave_run(a, b, bb, 4, 4, c, k, src=P.src, src_amp=amp, inplace=True)
        secs += time.perf_counter() - t
        ref = W.interior_of(a, 4)
        num = max(num, float(np.max(np.abs(got - ref))))
        den = max(den, float(np.max(np.abs(ref))))
        del got
    final = float(np.max(np.abs(f[0].interior(4) - W.interior_of(a, 4)))) / float(np.max(np.abs(W.interior_of(a, 4))))
    same = bool(torch.equal(f[0].storage, final_timed[0]) and torch.equal(f[1].storage, final_timed[1]))
    parity = {"error": num / den, "bound": 1e-5, "within_bound": bool(num / den <= 1e-5),
              "final_level_error": final, "snapshot_every": every,
              "metric": "max over the levels every 20 steps of |gpu - oracle| / max of |oracle|",
              "segmented_run_bitwise_equal_to_timed_run": same,
              "oracle": "FP64 C, OpenMP over z, -O3 -march=native on this host, fed the FP32-rounded beta"}
    cpu = {"value": round(float(n) ** 3 * nsteps / secs / 1e9, 4), "unit": "GPts/s", "cores": threads,
           "kind": "oracle",
           "sample": f"the full headline configuration: FP64 oracle (C, OpenMP over z, -O3 -march=native "
                     f"on this host), so-8 wave {n}^3 interior, all {nsteps} leapfrog steps in segments of "
                     f"{every}, {secs:.1f} s; the same run is the parity reference",
           "library": os.path.basename(lib)}
    # one thread, two steps (labelled as such), and the host it ran on
    try:
        gomp = C.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        P1 = W.wave3d_c3(n=n, nsteps=2)
        z = np.zeros_like(bb)
        t0 = time.perf_counter()
        oracle.wave_run(z, z.copy(), bb, 4, 4, c, 2, src=P1.src, src_amp=P1.src_amp)
        d1 = time.perf_counter() - t0
        gomp.omp_set_num_threads(threads)
        cpu["single_thread"] = {"value": round(float(n) ** 3 * 2 / d1 / 1e9, 4), "unit": "GPts/s",
                                "sample": f"the same oracle on one thread, first 2 steps, {d1:.1f} s"}
    except OSError:
        pass
    cpu["host"] = host_cpu()
    log(f"[bench] headline vs FP64 oracle over the run: {num / den:.3e} (final level {final:.3e}); "
        f"oracle {secs:.1f} s on {threads} threads = {cpu['value']} GPts/s; bitwise == timed run: {same}")
    return parity, cpu


def host_cpu():
    """CPU model and socket count from /proc/cpuinfo."""
    model, sockets = None, set()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                key, _, val = line.partition(":")
                key = key.strip()
                if key == "model name" and model is None:
                    model = val.strip()
                elif key == "physical id":
                    sockets.add(val.strip())
    except OSError:
        pass
    return {"model": model, "sockets": len(sockets) or None, "affinity_cores": len(os.sched_getaffinity(0))}


def bench_batch(S, W, steps, nsteps=200, only_variant=None):
    """32 uneven shots in one graph (the tuned batch variant: fused launches
    over all shots, or every shot with its own tuned plan in four concurrent
    branches) vs 32 sequential tuned runs."""
    import torch
    B = W.batch_c4(nsteps=nsteps)
    shapes = [s.shape for s in B.shots]
    bp = S.BatchPlan(shapes, 4, S.second_derivative_weights(8))
    fields, amps = [], []
    for i, sh in enumerate(B.shots):
        f = [bp.field(i) for _ in range(3)]
        f[2].load(W.embed(W.round_to_storage(sh.beta, "f32"), 4))
        fields.append(f)
        amps.append(torch.from_numpy(sh.src_amp).cuda())
    srcs = [sh.src for sh in B.shots]
    if only_variant is not None:
        bp.variant = {bp.variant_name(v): v for v in range(1, bp.variant_count())}[only_variant]
        for f in fields:
            f[0].storage.zero_()
            f[1].storage.zero_()
        bp.run(fields, B.nsteps, srcs, amps)
        with Timer() as t:
            for _ in range(steps):
                for f in fields:
                    f[0].storage.zero_()
                    f[1].storage.zero_()
                bp.run(fields, B.nsteps, srcs, amps)
        pts = float(sum(np.prod(s) for s in shapes)) * B.nsteps
        return {"variant": only_variant, "leapfrog_steps": B.nsteps, "ms_per_run": round(t.ms / steps, 3),
                "GPts_s": round(pts / (t.ms / steps * 1e-3) / 1e9, 2)}
    bp.tune(fields, reps=2)

    def run_batch():
        for f in fields:
            f[0].storage.zero_()
            f[1].storage.zero_()
        bp.run(fields, B.nsteps, srcs, amps)

    run_batch()
    with Timer() as t:
        for _ in range(steps):
            run_batch()
    ms_b = t.ms / steps
    tuned = bp.variant
    # whole runs of the other candidate forms, for the record
    names = {bp.variant_name(v): v for v in range(1, bp.variant_count())}
    per_variant = {bp.variant_name(tuned): round(ms_b, 2)}
    for name in ("shots_concurrent_4", "tb2_64x32_t768_zc128", "tb2_64x32_t768_zc256", "zmarch_64x16_t256_zc32_nt",
                 "zmarch_64x16_t256_zc128_nt", "zmarch_64x16_t256_zc256_nt", "persistent_zmarch_64x16_t256_zc32_nt",
                 "persistent_zmarch_64x16_t256_zc128_nt", "persistent_zmarch_64x16_t256_zc256_nt"):
        if name in names and name not in per_variant:
            bp.variant = names[name]
            run_batch()
            with Timer() as t:
                for _ in range(steps):
                    run_batch()
            per_variant[name] = round(t.ms / steps, 2)
    bp.variant = tuned
    # sequential plain runs on the same fields' data
    plans = []
    for i, sh in enumerate(B.shots):
        p = S.Plan(S.WAVE2, sh.shape, 4, S.second_derivative_weights(8), halo=4)
        g = [p.field() for _ in range(3)]
        g[2].storage.copy_(fields[i][2].storage)
        p.tune(g, reps=2)
        plans.append((p, g))

    def run_seq():
        for i, (p, g) in enumerate(plans):
            g[0].storage.zero_()
            g[1].storage.zero_()
            p.run(g, B.nsteps, src=srcs[i], src_amp=amps[i])

    run_seq()
    with Timer() as t:
        for _ in range(steps):
            run_seq()
    ms_s = t.ms / steps
    run_batch()
    same = all(torch.equal(fields[i][0].storage, plans[i][1][0].storage) for i in range(len(plans)))
    pts = float(sum(np.prod(s) for s in shapes)) * B.nsteps
    return {"shots": len(shapes), "points": int(sum(np.prod(s) for s in shapes)),
            "leapfrog_steps": B.nsteps, "GPts_s": round(pts / (ms_b * 1e-3) / 1e9, 2),
            "ms_per_run": round(ms_b, 2), "sequential_GPts_s": round(pts / (ms_s * 1e-3) / 1e9, 2),
            "sequential_ms": round(ms_s, 2), "batched_vs_sequential": round(ms_s / ms_b, 3),
            "bitwise_equal_to_sequential": bool(same),
            "variant": bp.variant_name(bp.variant), "ms_per_run_by_variant": per_variant,
            "sequential_variants": sorted({p.variant_name(p.variant) for p, _ in plans})}


def bench_heat3d(S, W, steps, variant=-1, nsteps=50):
    """3D 13-point heat (so-4), 512^3, alpha = 0.05, Dirichlet zero halo of 2."""
    H = W.heat3d_c2(nsteps=nsteps)
    hp = S.Plan(S.HEAT, H.shape, 2, S.heat_weights(4, H.alpha), halo=2)
    hf = [hp.field() for _ in range(2)]
    hf[0].load(W.embed(W.round_to_storage(H.u0, "f32"), 2))
    variant = resolve_variant(hp, variant)
    if variant >= 0:
        hp.variant = variant
    else:
        hp.tune(hf, reps=3)
    hp.run(hf, H.nsteps)
    with Timer() as t:
        for _ in range(steps):
            hp.run(hf, H.nsteps)
    hms = t.ms / steps
    npts = float(np.prod(H.shape))
    hg = npts * H.nsteps / (hms * 1e-3) / 1e9
    hvn = hp.variant_name(hp.variant)
    # launches: a tb2 pass reads u^n and writes u^{n+2} (8 B per point for
    # two steps); a plain sweep moves 8 B per point for one step
    _, hl, _, _ = launch_model(hvn, H.nsteps, 4, "f32")
    hown = 8.0 * npts * hl / (hms * 1e-3) / 1e9
    log(f"[bench] heat {hvn}: {hms:.3f} ms per run, {hg:.1f} GPts/s, {hg * 8:.0f} GB/s algorithmic "
        f"(8 B per update), {hown:.0f} GB/s of the kernel's own bytes")
    return {"GPts_s": round(hg, 2), "ms_per_run": round(hms, 3), "steps": H.nsteps, "variant": hvn,
            "launches_per_run": hl, "algorithmic_bytes_per_update": 8,
            "algorithmic_GBps": round(hg * 8, 1), "frac_hbm": round(hg * 8 / HBM_PEAK_GBS, 4),
            "kernel_own_GBps": round(hown, 1)}


def bench_pw(S, W, steps, n=512, variant=-1):
    """The flux-form C-grid advection of (u, v, w) as a 60-term stencil
    program (3 inputs, 3 outputs, diagonal offsets), 512^3 interior (the
    134M-point size of the paper's PW advection runs), random velocity,
    zero halo.  One program apply per step; `variant` >= 0 times that variant
    alone (profiling), else every compiled one."""
    import torch
    from paper_2404_02218_amd.program import Program, pw_advection_terms
    shape = (n, n, n)
    prog = Program(shape, 1, 3, 3, pw_advection_terms(1.0, 1.0, 1.0))
    gen = torch.Generator(device="cuda").manual_seed(W.SEED_BASE + 6)
    ins = [prog.field() for _ in range(3)]
    for f in ins:
        f.view[1:-1, 1:-1, 1:-1] = torch.rand(shape, generator=gen, device="cuda") - 0.5
    outs = [prog.field() for _ in range(3)]
    variant = resolve_variant(prog, variant)
    # the compiled forms (the generic kernel, variant 1, is a cross-check):
    # 64 x 16 tiles, the tight ring, 64 x 32 tiles; the fastest is reported
    per_variant = {}
    for v in [variant] if variant >= 0 else [x for x in (0, 2, 3) if x < prog.variant_count()]:
        prog.variant = v
        prog.apply_program(outs, ins)
        with Timer() as t:
            for _ in range(steps):
                prog.apply_program(outs, ins)
        per_variant[v] = t.ms / steps
    prog.variant = min(per_variant, key=per_variant.get)
    ms = per_variant[prog.variant]
    pts = float(n) ** 3
    gbs = 24.0 * pts / (ms * 1e-3) / 1e9
    log(f"[bench] pw advection {n}^3: {ms:.3f} ms, {pts / (ms * 1e-3) / 1e9:.1f} GPts/s, {prog.variant_name(prog.variant)}"
        f" (" + ", ".join(f"{prog.variant_name(v)} {m:.3f} ms" for v, m in per_variant.items()) + ")")
    return {"interior": list(shape), "terms": len(prog.terms), "GPts_s": round(pts / (ms * 1e-3) / 1e9, 2),
            "ms_per_apply": round(ms, 3), "algorithmic_GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_per_point": 24, "variant": prog.variant_name(prog.variant),
            "ms_per_variant": {prog.variant_name(v): round(m, 3) for v, m in per_variant.items()},
            "kernel": "stencil_program (compiled with the 60 terms as constants)"}


def bench_pw_loop(S, W, iters, n=512):
    """A forward-Euler loop of the PW advection at 512^3 on one periodic rank:
    per half-iteration one 60-term program (tendencies of u, v, w) and three
    2-term updates into the other velocity set.  Halos are refreshed by
    packing and unpacking box exchanges on the device, once with the pruned
    schedule (stencil_schedule: each velocity once, in the 8 directions PW
    reads it; tendencies never) and once exchanging all 26 boxes of every
    input before every apply."""
    import torch
    from paper_2404_02218_amd.program import Act, Program, pw_advection_terms, schedule, select
    shape = (n, n, n)
    pw = Program(shape, 1, 3, 3, pw_advection_terms(1.0, 1.0, 1.0))
    upd = Program(shape, 1, 2, 1, [(0, 1.0, [(0, (0, 0, 0))]), (0, 0.01, [(1, (0, 0, 0))])])
    steps = []
    for a, b in (((0, 1, 2), (6, 7, 8)), ((6, 7, 8), (0, 1, 2))):
        steps.append((pw, list(a), [3, 4, 5]))
        steps += [(upd, [a[c], 3 + c], [b[c]]) for c in range(3)]
    gen = torch.Generator(device="cuda").manual_seed(W.SEED_BASE + 7)
    fields = [pw.field() for _ in range(9)]
    for f in fields[:3]:
        f.view[1:-1, 1:-1, 1:-1] = torch.rand(shape, generator=gen, device="cuda") - 0.5
    ex = pw.exchanges([1, 1, 1], [0, 0, 0], periodic=True, box=True)
    buf = torch.empty(pw.exchange_elems(ex), dtype=torch.float32, device="cuda")
    full = (1 << 27) - 1 - (1 << 13)
    naive = []
    for k, (_, ins, _) in enumerate(steps):
        naive += [Act("exchange", k, f, full) for f in ins] + [Act("apply", k, -1, 0)]
    out = {"interior": list(shape), "fields": 9, "steps_per_iteration": len(steps)}
    for name, (pro, body) in (("scheduled", schedule(steps, 9, loop=True)), ("exchange_all", ([], naive))):
        plan = []       # boxes resolved before timing
        elems = 0
        for a in body:
            if a.kind == "exchange":
                sel = select(ex, a.dirs, 3)
                part = [[x for x in ex if tuple(x.to[:3]) == tuple(-t for t in e.to[:3])][0] for e in sel]
                plan.append(("x", fields[a.field], sel, part))
                elems += pw.exchange_elems(sel)
            else:
                prog, ins, outs = steps[a.step]
                plan.append(("a", prog, [fields[f] for f in outs], [fields[f] for f in ins]))

        def run():
            for it in plan:
                if it[0] == "x":
                    pw.pack(it[1], it[3], buf)
                    pw.unpack(it[1], it[2], buf)
                else:
                    it[1].apply_program(it[2], it[3])
        for a in pro:
            sel = select(ex, a.dirs, 3)
            part = [[x for x in ex if tuple(x.to[:3]) == tuple(-t for t in e.to[:3])][0] for e in sel]
            pw.pack(fields[a.field], part, buf)
            pw.unpack(fields[a.field], sel, buf)
        run()
        with Timer() as t:
            for _ in range(iters):
                run()
        ms = t.ms / iters
        log(f"[bench] pw loop {name}: {ms:.3f} ms per iteration, {elems * 4 / 2**20:.1f} MiB exchanged")
        out[name] = {"ms_per_iteration": round(ms, 3), "exchanges_per_iteration":
                     sum(1 for a in body if a.kind == "exchange"),
                     "exchanged_MiB_per_iteration": round(elems * 4 / 2 ** 20, 2)}
    out["speedup"] = round(out["exchange_all"]["ms_per_iteration"] / out["scheduled"]["ms_per_iteration"], 3)
    del fields, buf
    return out


def bench_absorbing(S, W, steps, n=512, width=40, gmax=0.1):
    """The headline so-8 wave (512^3, 400 steps, FP32) with a 40-point
    absorbing layer on every face (quadratic profile, gamma up to 0.1 per
    axis), its source moved off the grid by (0.5, 0.5, 0.5) cells and 64
    receivers off the grid on a line 8 cells deep (stencil_run_interp).  The
    undamped on-grid run at the same variant is timed beside it."""
    import torch
    P = W.wave3d_c3(n=n, nsteps=400)
    plan = S.Plan(S.WAVE2, P.shape, 4, S.second_derivative_weights(8), halo=4)
    f = [plan.field() for _ in range(3)]
    f[2].load(W.embed(W.round_to_storage(P.beta, "f32"), 4))
    plan.set_damping(W.damping_profiles(P.shape, width, gmax))
    plan.tune(f, reps=3)
    src = np.minimum(P.src.astype(np.float64) + 0.5, n - 1)
    rec = np.minimum(W.receiver_line(n, 64, depth=8).astype(np.float64) + np.array([0.25, 0.5, 0.375]), n - 1)
    amp = torch.from_numpy(P.src_amp).cuda()
    tr = torch.zeros((P.nsteps, len(rec)), dtype=torch.float64, device="cuda")

    def timed(run):
        run()
        with Timer() as t:
            for _ in range(steps):
                run()
        return t.ms / steps

    def damped():
        f[0].storage.zero_()
        f[1].storage.zero_()
        plan.run_interp(f, P.nsteps, src=src, src_amp=amp, rec=rec, rec_trace=tr)

    ms = timed(damped)
    vname = plan.variant_name(plan.variant)
    v = plan.variant
    plan.set_damping(None)
    plan.variant = v

    def plain():
        f[0].storage.zero_()
        f[1].storage.zero_()
        plan.run(f, P.nsteps, src=P.src, src_amp=amp)

    ms0 = timed(plain)
    pts = float(n) ** 3 * P.nsteps
    log(f"[bench] absorbing layer + off-grid points: {ms:.1f} ms ({pts / (ms * 1e-3) / 1e9:.1f} GPts/s), "
        f"undamped on-grid {ms0:.1f} ms, {vname}")
    del f
    return {"interior": [n] * 3, "steps": P.nsteps, "layer_width": width, "gamma_max_per_axis": gmax,
            "receivers": len(rec), "GPts_s": round(pts / (ms * 1e-3) / 1e9, 2), "ms_per_run": round(ms, 2),
            "variant": vname, "undamped_ongrid_GPts_s": round(pts / (ms0 * 1e-3) / 1e9, 2),
            "vs_undamped_same_variant": round(ms0 / ms, 3)}


def bench_precision(S, W, n=512, nsteps=400, every=25):
    """Error of the headline workload (so-8 wave, n^3, nsteps steps, Ricker at
    the centre, zero start) against the FP64 oracle for FP32, BF16 and FP16
    storage, the oracle fed the same storage-rounded velocity term.  Both
    advance in segments of `every` steps; the error is max over the snapshots
    (every `every` steps and the last) of |gpu - oracle|, over max over the
    snapshots of |oracle| (a pointwise relative error is ill-posed at the
    wavefield's zeros, and the final level alone is divided by an amplitude
    that has decayed as the wave spread); the final level's own ratio is
    reported beside it.  About 40 s of host time per storage type at 512^3."""
    import torch

    import oracle
    P = W.wave3d_c3(n=n, nsteps=nsteps)
    c = oracle.fd_weights_float(8)
    out = {"interior": [n] * 3, "steps": nsteps, "snapshot_every": every,
           "metric": "max over snapshots |gpu - oracle| / max over snapshots |oracle|"}
    for dn in ("f32", "bf16", "f16"):
        plan = S.Plan(S.WAVE2, P.shape, 4, S.second_derivative_weights(8), halo=4, dtype=S.DTYPES[dn])
        f = [plan.field() for _ in range(3)]
        beta = W.round_to_storage(P.beta, dn)
        f[2].load(W.embed(beta, 4))
        bb = W.embed(beta, 4)
        a = np.zeros(tuple(s + 8 for s in P.shape))
        b = np.zeros_like(a)
        num = den = 0.0
        secs = 0.0
        for t0 in range(0, nsteps, every):
            k = min(every, nsteps - t0)
            amp = P.src_amp[t0:t0 + k]
            plan.run(f, k, src=P.src, src_amp=torch.from_numpy(np.ascontiguousarray(amp)).cuda())
            torch.cuda.synchronize()
            got = f[0].interior(4)
            t = time.perf_counter()
            a, b, _ = oracle.wave_run(a, b, bb, 4, 4, c, k, src=P.src, src_amp=amp)
            secs += time.perf_counter() - t
            ref = W.interior_of(a, 4)
            d = float(np.max(np.abs(got - ref)))
            m = float(np.max(np.abs(ref)))
            num, den = max(num, d), max(den, m)
        final = d / m
        log(f"[bench] precision {dn}: {num / den:.3e} over snapshots, final level {final:.3e} "
            f"(oracle {secs:.1f} s)")
        out[dn] = {"error": num / den, "final_level_error": final, "variant": plan.variant_name(plan.variant),
                   "oracle_s": round(secs, 1)}
        del f, a, b
        torch.cuda.empty_cache()
    return out


def bench_heat2d(S, W, steps):
    """2D 5-point heat, 256^2, Dirichlet zero halo, 100 steps: a field of
    260 KiB stays in L2, so launches, not HBM bandwidth, set the time.  The
    multi-step kernels take 4-16 steps per launch in LDS; the whole run is one
    graph.  The plain one-sweep-per-launch kernel is timed beside it."""
    H = W.heat2d_c1()
    plan = S.Plan(S.HEAT, H.shape, 1, S.heat_weights(2, H.alpha), halo=1)
    f = [plan.field() for _ in range(2)]
    u0 = W.embed(W.round_to_storage(H.u0, "f32"), 1)
    f[0].load(u0)
    # launch-bound: pick the variant by timing whole runs (a single launch's
    # kernel time leaves out the launches it saves)
    whole = {}
    for v in range(plan.variant_count()):
        plan.variant = v
        plan.run(f, H.nsteps)
        with Timer() as tv:
            for _ in range(steps):
                plan.run(f, H.nsteps)
        whole[v] = tv.ms / steps
    ms0 = whole[0]
    plan.variant = min(whole, key=whole.get)
    plan.run(f, H.nsteps)
    with Timer() as t:
        for _ in range(steps):
            plan.run(f, H.nsteps)
    ms = t.ms / steps
    pts = float(np.prod(H.shape)) * H.nsteps
    return {"interior": list(H.shape), "steps": H.nsteps, "GPts_s": round(pts / (ms * 1e-3) / 1e9, 2),
            "ms_per_run": round(ms, 4), "us_per_step": round(ms * 1e3 / H.nsteps, 2),
            "bound": "launch latency (field resident in L2)", "variant": plan.variant_name(plan.variant),
            "one_sweep_per_launch_us_per_step": round(ms0 * 1e3 / H.nsteps, 2)}


def bench_slab_share(S, W, steps):
    """One GPU's share of the 512^3 wave split over 8 GPUs as z-slabs: a
    64 x 512 x 512 interior (the slab z = 224..287 of the headline model, with
    its source).  Every step first refreshes the two 4-plane z halos of u^n by
    packing the faces and unpacking them into the halos (this slab's own
    faces stand in for its neighbours'), then sweeps once.  The 400 steps of
    pack, unpack and sweep are captured in one graph; the sweep alone over
    the same slab is timed beside it."""
    import torch
    P = W.wave3d_c3(nsteps=400)
    z0, nz = 224, 64
    shape = (nz, 512, 512)
    plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4)
    f = [plan.field() for _ in range(3)]
    f[2].load(W.embed(W.round_to_storage(P.beta[z0:z0 + nz], "f32"), 4))
    src = np.array([[P.src[0][0] - z0, P.src[0][1], P.src[0][2]]])
    amp = torch.from_numpy(P.src_amp).cuda()
    ex = plan.exchanges([8, 1, 1], [3, 0, 0])
    buf = torch.empty(plan.exchange_elems(ex), dtype=torch.float32, device="cuda")
    n = P.nsteps

    def exchange_and_sweep():
        for t in range(n):
            plan.pack(f[0], ex, buf)
            plan.unpack(f[0], ex, buf)
            plan.run(f, 1, src=src, src_amp=amp[t:t + 1])

    def reset():
        f[0].storage.zero_()
        f[1].storage.zero_()

    reset()
    exchange_and_sweep()
    torch.cuda.synchronize()
    eager = f[0].storage.clone()
    mode = "graph"
    try:
        g = torch.cuda.CUDAGraph()
        reset()
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            exchange_and_sweep()
        replays_equal = True
        for _ in range(2):
            reset()
            g.replay()
            torch.cuda.synchronize()
            replays_equal &= bool(torch.equal(f[0].storage, eager))
        run_once = g.replay
    except Exception as e:  # capture unsupported: time the eager loop
        log(f"[bench] slab graph capture failed ({e}); timing eager launches")
        mode, replays_equal, run_once = "eager", None, exchange_and_sweep
    with Timer() as t:
        for _ in range(steps):
            reset()
            run_once()
    ms_x = t.ms / steps
    plan.tune(f, reps=2)
    reset()
    plan.run(f, n, src=src, src_amp=amp)
    with Timer() as t:
        for _ in range(steps):
            reset()
            plan.run(f, n, src=src, src_amp=amp)
    ms_s = t.ms / steps
    pts = float(np.prod(shape)) * n
    face_mib = plan.exchange_elems(ex) * 4 / 2 ** 20
    return {"interior": list(shape), "steps": n, "launches": mode,
            "GPts_s_with_exchange": round(pts / (ms_x * 1e-3) / 1e9, 2), "ms_with_exchange": round(ms_x, 2),
            "GPts_s_sweep_only": round(pts / (ms_s * 1e-3) / 1e9, 2), "ms_sweep_only": round(ms_s, 2),
            "sweep_only_variant": plan.variant_name(plan.variant),
            "exchange_us_per_step": round((ms_x - ms_s) * 1e3 / n, 2),
            "faces_MiB_per_step": round(face_mib, 2), "graph_replays_equal_eager": replays_equal}


def bench_faces(S, W, reps=20):
    """Pack and unpack throughput of the halo faces of a 512^3 FP32 field
    (halo 4): the z faces are contiguous planes, the y faces 2 KiB row runs,
    the x faces 16-byte runs.  Bytes = elements x 4 B read + written."""
    import torch
    plan = S.Plan(S.WAVE2, (512, 512, 512), 4, S.second_derivative_weights(8), halo=4)
    f = plan.field()
    allx = plan.exchanges([1, 1, 1], [0, 0, 0], periodic=True)
    out = {}
    for d, name in enumerate(("z", "y", "x")):
        ex = [e for e in allx if e.size[d] == 4]
        buf = torch.empty(plan.exchange_elems(ex), dtype=torch.float32, device="cuda")
        nb = 2.0 * plan.exchange_elems(ex) * 4
        plan.pack(f, ex, buf)
        with Timer() as t:
            for _ in range(reps):
                plan.pack(f, ex, buf)
        pk = nb / (t.ms / reps * 1e-3) / 1e9
        with Timer() as t:
            for _ in range(reps):
                plan.unpack(f, ex, buf)
        up = nb / (t.ms / reps * 1e-3) / 1e9
        out[f"{name}_faces"] = {"MiB": round(plan.exchange_elems(ex) * 4 / 2 ** 20, 2),
                                "pack_GBps": round(pk, 1), "unpack_GBps": round(up, 1)}
    return out


def bench_adjoint(S, W, steps, nsteps=500):
    """Checkpointed gradient of J = 1/2 |d|^2 (the adjoint's work does not
    depend on the residual values) vs the plain forward of the same model."""
    import torch
    P = W.inversion_c5(nsteps=nsteps)
    n, N, k = P.shape[0], P.nsteps, P.checkpoint_every
    plan = S.Plan(S.WAVE2, P.shape, 4, S.second_derivative_weights(8), halo=4)
    f = [plan.field() for _ in range(3)]
    m0 = P.m0
    beta = W.round_to_storage(P.dt * P.dt / (P.h * P.h * m0), "f32")
    f[2].load(W.embed(beta, 4))
    amp = torch.from_numpy((P.dt ** 2 / m0[tuple(P.src[0])] * P.wavelet).reshape(-1, 1)).cuda()
    nrec = len(P.rec)
    tr = torch.zeros((N, nrec), dtype=torch.float64, device="cuda")
    scale = torch.from_numpy(np.array([P.dt ** 2 / m0[tuple(p)] for p in P.rec])).cuda()
    grad = torch.zeros(P.shape, dtype=torch.float64, device="cuda")
    ws = torch.empty(plan.adjoint_workspace_bytes(N, k), dtype=torch.uint8, device="cuda")
    plan.tune(f, reps=3)

    def fwd():
        f[0].storage.zero_()
        f[1].storage.zero_()
        plan.run(f, N, src=P.src, src_amp=amp, rec=P.rec, rec_trace=tr)

    def gradient():
        f[0].storage.zero_()
        f[1].storage.zero_()
        plan.forward_ckpt(f, N, k, ws, src=P.src, src_amp=amp, rec=P.rec, rec_trace=tr)
        plan.adjoint(f[2], N, k, ws, tr, P.rec, scale, P.dt, grad, src=P.src, src_amp=amp)

    fwd()
    with Timer() as t:
        for _ in range(steps):
            fwd()
    ms_f = t.ms / steps
    gradient()
    with Timer() as t:
        for _ in range(steps):
            gradient()
    ms_g = t.ms / steps
    pts = float(n) ** 3 * N
    last = N - (N - 1) // k * k   # steps in the last checkpoint segment
    return {"interior": list(P.shape), "leapfrog_steps": N, "receivers": nrec, "checkpoint_every": k,
            "forward_GPts_s": round(pts / (ms_f * 1e-3) / 1e9, 2), "forward_ms": round(ms_f, 2),
            "gradient_GPts_s": round(pts / (ms_g * 1e-3) / 1e9, 2), "gradient_ms": round(ms_g, 2),
            "gradient_vs_forward_time": round(ms_g / ms_f, 3),
            "workspace_GB": round(ws.numel() / 1e9, 2),
            # checkpointed forward 16 B (20 B in its last segment, which
            # also writes the second differences), recompute with second
            # differences 20 B in every other segment, adjoint in pairs of
            # steps 24 B (16 + 32 per pair)
            "bytes_per_gradient_update": round(16 + 24 + (4 * last + 20 * (N - last)) / N, 2),
            "misfit": "J = 1/2 |d|^2 (d_obs = 0); timing only, parity is in the tests",
            "variant": plan.variant_name(plan.variant)}


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
    if args.leg:
        legs = {"pw": lambda: bench_pw(S, W, max(1, args.steps), variant=args.variant),
                "pw_loop": lambda: bench_pw_loop(S, W, max(1, args.steps)),
                "slab": lambda: bench_slab_share(S, W, max(1, args.steps)),
                "faces": lambda: bench_faces(S, W),
                "absorbing": lambda: bench_absorbing(S, W, max(1, args.steps)),
                "heat2d": lambda: bench_heat2d(S, W, max(1, args.steps)),
                "batch": lambda: bench_batch(S, W, max(1, args.steps), args.batch_steps, args.batch_variant),
                "adjoint": lambda: bench_adjoint(S, W, max(1, args.steps), args.adjoint_steps),
                "precision": lambda: bench_precision(S, W)}
        res = {args.leg: legs[args.leg]()}
        if args.copy_calibration:
            res["stream_copy_GBps"] = round(stream_copy_gbs(), 1)
        print(json.dumps(res), flush=True)
        return
    if args.only_heat:
        out = {"heat3d_so4": bench_heat3d(S, W, args.steps, args.variant, args.heat_steps)}
        if args.copy_calibration:
            out["stream_copy_GBps"] = round(stream_copy_gbs(), 1)
        print(json.dumps(out), flush=True)
        return

    log(f"[bench] headline: so-8 wave {n}^3 x {nsteps} steps, {args.storage} storage")
    P, plan, f, amp = wave_setup(S, W, n, nsteps, S.DTYPES[args.storage], args.variant)
    es = 4 if args.storage == "f32" else 2
    vname = plan.variant_name(plan.variant)
    log(f"[bench] variant {vname}")
    per_run = {}
    ms = time_wave(plan, f, amp, P, args.steps, args.warmup, per_run)
    gpts = pts / (ms * 1e-3) / 1e9
    tb, launches, own_bpl, kname = launch_model(vname, nsteps, es, args.storage)
    steps_per_launch = 2 if tb else 1
    kern_ms = ms / launches
    # algorithmic bytes of one launch: the plain sweep's 4 fields per point
    # update, times the updates one launch makes
    bpl = 4 * es * steps_per_launch
    achieved = float(bpl) * n ** 3 / (kern_ms * 1e-3) / 1e9
    own = float(own_bpl) * n ** 3 / (kern_ms * 1e-3) / 1e9
    log(f"[bench] {ms:.2f} ms per run, {kern_ms * 1e3:.1f} us per launch, {gpts:.1f} GPts/s, "
        f"{achieved:.0f} GB/s algorithmic ({4 * es} B per update), {own:.0f} GB/s of the kernel's own bytes")
    traffic = stored_traffic(vname) if (n == 512 and args.storage == "f32") else None
    out = {
        "metric": METRIC, "value": round(gpts, 3), "unit": "GPts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.storage,
        "data": "synthetic",
        "runs": dict(per_run, note="ms per step: median and min of the timed runs (each bracketed by "
                                   "its own events); first_run_ms: the first warm-up run, which captures "
                                   "and instantiates the run's graph"),
        "config": {"workload": f"wave3d_so8_{n}^3_{nsteps}steps", "interior": [n, n, n], "halo": 4,
                   "radius": 4, "leapfrog_steps": nsteps, "storage": args.storage, "variant": vname,
                   "source": "Ricker 10 Hz at the centre, layered velocity 1.5-4.5 km/s +-5%"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": kname, "algorithmic_bytes_per_launch": bpl * n ** 3,
                     "algorithmic_bytes_per_update": 4 * es,
                     "points_per_launch": n ** 3, "steps_per_launch": steps_per_launch,
                     "launches_per_run": launches, "avg_launch_us": round(kern_ms * 1e3, 2),
                     "kernel_own_bytes_per_launch": own_bpl * n ** 3,
                     "kernel_own_GBps": round(own, 1), "kernel_own_frac": round(own / HBM_PEAK_GBS, 4)},
    }
    if traffic:
        out["roofline"]["traffic_GBps"] = round(traffic / (kern_ms * 1e-3) / 1e9, 1)
    if not args.no_cpu and not args.only_main:
        log("[bench] headline run against the FP64 oracle (also the CPU baseline)")
        final_timed = [f[0].storage.clone(), f[1].storage.clone()]
        out["parity"], cpu = headline_oracle_run(S, W, plan, f, n, nsteps, final_timed)
        del final_timed
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
            vn2 = plan2.variant_name(plan2.variant)
            _, l2, b2, k2 = launch_model(vn2, nsteps, 2, name)
            a2 = 8.0 * pts / (ms2 * 1e-3) / 1e9
            o2 = float(b2) * n ** 3 / (ms2 / l2 * 1e-3) / 1e9
            extras[f"wave_{name}"] = {
                "GPts_s": round(g2, 2), "ms_per_run": round(ms2, 2), "variant": vn2, "kernel": k2,
                "algorithmic_bytes_per_update": 8,
                "algorithmic_GBps": round(a2, 1), "frac_hbm": round(a2 / HBM_PEAK_GBS, 4),
                "kernel_own_GBps": round(o2, 1), "vs_fp32": round(g2 / gpts, 3)}
            del f2
            torch.cuda.empty_cache()
        log("[bench] heat so-4 512^3 x 50")
        extras["heat3d_so4"] = bench_heat3d(S, W, 3, args.variant)
        torch.cuda.empty_cache()
        log("[bench] heat 2D 256^2 x 100")
        extras["heat2d_so2"] = bench_heat2d(S, W, 20)
        log("[bench] one GPU's z-slab share with halo exchange")
        extras["slab_share_exchange"] = bench_slab_share(S, W, max(1, args.steps // 2))
        torch.cuda.empty_cache()
        log("[bench] face pack/unpack")
        extras["halo_faces"] = bench_faces(S, W)
        torch.cuda.empty_cache()
        log("[bench] pw advection program")
        extras["pw_advection_program"] = bench_pw(S, W, 10)
        torch.cuda.empty_cache()
        log("[bench] absorbing layer with off-grid source and receivers")
        extras["wave_absorbing_offgrid"] = bench_absorbing(S, W, max(1, args.steps // 2))
        torch.cuda.empty_cache()
        log("[bench] pw advection loop with scheduled exchanges")
        extras["pw_advection_loop_exchanges"] = bench_pw_loop(S, W, 5)
        torch.cuda.empty_cache()
        if not args.no_batch:
            log("[bench] batched shots")
            extras["batched_shots"] = bench_batch(S, W, max(1, args.steps // 2))
            torch.cuda.empty_cache()
        if not args.no_adjoint:
            log("[bench] checkpointed gradient")
            extras["adjoint_gradient"] = bench_adjoint(S, W, max(1, args.steps // 2))
            torch.cuda.empty_cache()
        out["variants"] = extras

    if not args.no_cpu and not args.only_main:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
