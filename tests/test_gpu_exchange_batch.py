"""GPU parity of halo pack/unpack, the emulated multi-rank decomposition,
batched shots, and 16-bit storage, through the C ABI."""
import numpy as np
import pytest

import oracle
import paper_2404_02218_amd as S
import workloads as W
from _helpers import gpu_wave, oracle_wave, rel_err, torch_f64, wave_inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [S.F32, S.BF16])
def test_pack_unpack_match_oracle_bitwise(device, dtype):
    import torch
    shape, halo, r = (18, 23, 41), 4, 4
    rng = np.random.default_rng(91)
    buf = W.round_to_storage(rng.standard_normal(tuple(n + 2 * halo for n in shape)),
                             "f32" if dtype == S.F32 else "bf16")
    plan = S.Plan(S.WAVE2, shape, r, S.second_derivative_weights(8), halo=halo, dtype=dtype)
    f = plan.field().load(buf)
    ex = plan.exchanges([1, 1, 1], [0, 0, 0], periodic=True)
    n = plan.exchange_elems(ex)
    tdt = f.storage.dtype
    dev_buf = torch.zeros(n, dtype=tdt, device=device)
    plan.pack(f, ex, dev_buf)
    torch.cuda.synchronize()
    oex = oracle.exchanges(list(shape), halo, r, [1, 1, 1], [0, 0, 0], True)
    ref = oracle.pack(buf, halo, oex)
    assert np.array_equal(dev_buf.to(torch.float64).cpu().numpy(), ref)
    # unpack a fresh buffer into a zero field
    newbuf = W.round_to_storage(rng.standard_normal(n), "f32" if dtype == S.F32 else "bf16")
    g = plan.field()
    plan.unpack(g, ex, torch_f64(newbuf, device).to(tdt))
    torch.cuda.synchronize()
    want = oracle.unpack(np.zeros_like(buf), halo, oex, newbuf)
    assert np.array_equal(g.to_numpy(), want)


def test_periodic_run_matches_oracle(device):
    shape = (20, 26, 36)
    u0, um1, beta = wave_inputs(shape, seed=95)
    plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4, bc=S.BC_PERIODIC)
    a, b, _ = gpu_wave(plan, u0, um1, beta, 25)
    ra, rb, _ = oracle_wave(u0, um1, beta, 4, 4, 25, periodic=True)
    assert rel_err(a, ra) <= 1e-5 and rel_err(b, rb) <= 1e-5


@pytest.mark.parametrize("parts,periodic", [((2, 2, 1), False), ((1, 3, 2), True)])
def test_decomposed_equals_monolithic_on_gpu(device, parts, periodic):
    """Subdomains with their own halos exchange faces every step through
    pack -> device copy -> unpack; the result is bitwise the monolithic run."""
    import torch
    r = 4
    loc = (16, 12, 20)
    shape = tuple(l * p for l, p in zip(loc, parts))
    u0, um1, beta = wave_inputs(shape, seed=97)
    bc = S.BC_PERIODIC if periodic else S.BC_DIRICHLET0
    mono = S.Plan(S.WAVE2, shape, r, S.second_derivative_weights(8), halo=r, bc=bc)
    ma, mb, _ = gpu_wave(mono, u0, um1, beta, 6)
    plan = S.Plan(S.WAVE2, loc, r, S.second_derivative_weights(8), halo=r)
    coords = [(i, j, k) for i in range(parts[0]) for j in range(parts[1]) for k in range(parts[2])]

    def sl(co):
        return tuple(slice(co[d] * loc[d], (co[d] + 1) * loc[d]) for d in range(3))

    F = {}
    for co in coords:
        f = [plan.field() for _ in range(3)]
        f[0].load(W.embed(u0[sl(co)], r))
        f[1].load(W.embed(um1[sl(co)], r))
        f[2].load(W.embed(beta[sl(co)], r))
        F[co] = f
    EX = {co: plan.exchanges(parts, co, periodic) for co in coords}
    for _ in range(6):
        bufs = {}
        for co in coords:
            n = plan.exchange_elems(EX[co])
            bufs[co] = torch.zeros(max(n, 1), dtype=torch.float32, device=device)
            plan.pack(F[co][0], EX[co], bufs[co])
        for co in coords:
            recv = []
            for e in EX[co]:
                nb = tuple((co[d] + e.to[d]) % parts[d] for d in range(3))
                k = next(i for i, f in enumerate(EX[nb]) if all(f.to[d] == -e.to[d] for d in range(3)))
                o = sum(plan.exchange_elems([f]) for f in EX[nb][:k])
                recv.append(bufs[nb][o:o + plan.exchange_elems([e])])
            if recv:
                plan.unpack(F[co][0], EX[co], torch.cat(recv))
        for co in coords:
            plan.run(F[co], 1)
    torch.cuda.synchronize()
    out = np.zeros(shape)
    for co in coords:
        out[sl(co)] = F[co][0].interior(r)
    assert np.array_equal(out, ma)


@pytest.mark.parametrize("steps,dtype", [(17, S.F32), (14, S.F32), (17, S.BF16), (14, S.F16)])
def test_batched_equals_sequential_bitwise(device, steps, dtype):
    # plain batched variants and the temporally blocked ones (tb2_*: two-step
    # passes over all shots, plain batched sweeps for the remaining steps),
    # for FP32 and 16-bit storage
    import torch
    shapes = [(20, 33, 45), (37, 16, 70), (28, 28, 28), (9, 40, 12), (40, 70, 130)]
    bp = S.BatchPlan(shapes, 4, S.second_derivative_weights(8), dtype=dtype)
    tb = [v for v in range(bp.variant_count()) if bp.variant_name(v).startswith("tb2_")]
    assert len(tb) == 3
    conc = [v for v in range(bp.variant_count()) if bp.variant_name(v).startswith("shots_concurrent")]
    assert len(conc) == 1
    pers = [v for v in range(bp.variant_count()) if bp.variant_name(v).startswith("persistent_")]
    assert len(pers) == 4
    fields, srcs, amps, recs, trs, ins = [], [], [], [], [], []
    for i, sh in enumerate(shapes):
        u0, um1, beta = wave_inputs(sh, seed=100 + i, dtype=dtype)
        ins.append((u0, um1, beta))
        f = [bp.field(i) for _ in range(3)]
        for fld, a in zip(f, (u0, um1, beta)):
            fld.load(W.embed(a, 4))
        fields.append(f)
        srcs.append(np.array([[s // 2 for s in sh]]))
        amps.append(torch_f64(np.random.default_rng(200 + i).standard_normal((steps, 1)), device))
        recs.append(np.array([[1, 2, 3], [s - 1 for s in sh]][: 1 + i % 2]))
        trs.append(torch.zeros((steps, len(recs[-1])), dtype=torch.float64, device=device))
    for v in (1, 5, 9, *tb, *pers, *conc):
        bp.variant = v
        for i in range(len(shapes)):
            for fld, a in zip(fields[i], ins[i]):
                fld.load(W.embed(a, 4))
        bp.run(fields, steps, srcs, amps, recs, trs)
        torch.cuda.synchronize()
        for i, sh in enumerate(shapes):
            plan = S.Plan(S.WAVE2, sh, 4, S.second_derivative_weights(8), halo=4, dtype=dtype)
            a, b, tr = gpu_wave(plan, *ins[i], steps, src=srcs[i], amp=amps[i].cpu().numpy(),
                                rec=recs[i])
            assert np.array_equal(fields[i][0].interior(4), a), (v, i)
            assert np.array_equal(fields[i][1].interior(4), b), (v, i)
            assert np.array_equal(trs[i].cpu().numpy(), tr), (v, i)


def test_persistent_batch_barrier_gives_up_and_reports(device, monkeypatch):
    """The persistent batched sweep's grid barrier waits a bounded number of
    polls.  Forced to zero from the host, the first workgroup to arrive gives
    up, every other one leaves at its next barrier, the run reports the error
    instead of returning fields, and a later run with the default bound gives
    the sequential runs' bits again."""
    import torch
    shapes = [(20, 33, 45), (28, 28, 28)]
    steps = 6
    bp = S.BatchPlan(shapes, 4, S.second_derivative_weights(8))
    v = next(v for v in range(bp.variant_count()) if bp.variant_name(v).startswith("persistent_"))
    bp.variant = v
    ins = [wave_inputs(sh, seed=300 + i) for i, sh in enumerate(shapes)]
    fields = [[bp.field(i) for _ in range(3)] for i in range(len(shapes))]

    def load():
        for f, x in zip(fields, ins):
            for fld, a in zip(f, x):
                fld.load(W.embed(a, 4))

    load()
    monkeypatch.setenv("STENCIL_BARRIER_POLLS", "0")
    with pytest.raises(S.StencilError, match="grid barrier"):
        bp.run(fields, steps)
    monkeypatch.delenv("STENCIL_BARRIER_POLLS")
    fields = [[bp.field(i) for _ in range(3)] for i in range(len(shapes))]
    load()
    bp.run(fields, steps)
    torch.cuda.synchronize()
    for i, sh in enumerate(shapes):
        plan = S.Plan(S.WAVE2, sh, 4, S.second_derivative_weights(8), halo=4)
        a, b, _ = gpu_wave(plan, *ins[i], steps)
        assert np.array_equal(fields[i][0].interior(4), a), i
        assert np.array_equal(fields[i][1].interior(4), b), i


def test_concurrent_batch_with_tuned_shot_plans(device, monkeypatch):
    """The concurrent batch variant forced through the environment: tuning
    then tunes each shot's own plan (forced to the temporally blocked sweep,
    each taking a slice of the batch's workspace), and two runs in a row (the
    second replays the captured graph of four branches) give every shot the
    bits of its own sequential run."""
    import torch
    # the batch takes the concurrent variant, and every shot's own plan the
    # temporally blocked sweep (a slice of the batch's workspace each)
    monkeypatch.setenv("STENCIL_FORCE_VARIANT", "shots_concurrent_4,tb2_64x32_t768_zc64")
    shapes = [(64, 64, 64), (20, 33, 45), (48, 100, 70), (9, 40, 12), (33, 70, 130), (16, 16, 16)]
    bp = S.BatchPlan(shapes, 4, S.second_derivative_weights(8))
    steps = 12
    fields, srcs, amps, recs, trs, ins = [], [], [], [], [], []
    for i, sh in enumerate(shapes):
        u0, um1, beta = wave_inputs(sh, seed=150 + i)
        ins.append((u0, um1, beta))
        f = [bp.field(i) for _ in range(3)]
        for fld, a in zip(f, (u0, um1, beta)):
            fld.load(W.embed(a, 4))
        fields.append(f)
        srcs.append(np.array([[s // 2 for s in sh], [1, 1, 1]]))
        amps.append(torch_f64(np.random.default_rng(250 + i).standard_normal((steps, 2)), device))
        recs.append(np.array([[s - 2 for s in sh]]))
        trs.append(torch.zeros((steps, 1), dtype=torch.float64, device=device))
    bp.tune(fields, reps=1)
    assert bp.variant_name(bp.variant) == "shots_concurrent_4"
    fb = [(bp.layouts[i].bytes + 255) // 256 * 256 for i in range(len(shapes))]
    from paper_2404_02218_amd import _abi
    import ctypes as C
    need = C.c_size_t()
    _abi.call("stencil_run_workspace", bp._h, C.byref(need))
    assert need.value == 2 * sum(fb)
    refs = []
    for i, sh in enumerate(shapes):
        plan = S.Plan(S.WAVE2, sh, 4, S.second_derivative_weights(8), halo=4)
        refs.append(gpu_wave(plan, *ins[i], steps, src=srcs[i], amp=amps[i].cpu().numpy(), rec=recs[i], variant=2))
    for rep in range(2):
        for i in range(len(shapes)):
            for fld, a in zip(fields[i], ins[i]):
                fld.load(W.embed(a, 4))
            trs[i].zero_()
        bp.run(fields, steps, srcs, amps, recs, trs)
        torch.cuda.synchronize()
        for i in range(len(shapes)):
            a, b, tr = refs[i]
            assert np.array_equal(fields[i][0].interior(4), a), (rep, i)
            assert np.array_equal(fields[i][1].interior(4), b), (rep, i)
            assert np.array_equal(trs[i].cpu().numpy(), tr), (rep, i)


@pytest.mark.parametrize("dtype,name,bound", [(S.BF16, "bf16", 5e-2), (S.F16, "f16", 2e-2)])
def test_wave_16bit_storage_error_vs_oracle(device, dtype, name, bound):
    shape = (32, 40, 72)
    u0, um1, beta = wave_inputs(shape, seed=111, dtype=dtype)
    src = np.array([[16, 20, 36]])
    amp = W.round_to_storage(np.random.default_rng(112).standard_normal((50, 1)), "f64")
    plan = S.Plan(S.WAVE2, shape, 4, S.second_derivative_weights(8), halo=4, dtype=dtype)
    base = gpu_wave(plan, u0, um1, beta, 50, src=src, amp=amp, variant=0)
    ra, _, _ = oracle_wave(u0, um1, beta, 4, 4, 50, src=src, amp=amp)
    err = rel_err(base[0], ra)
    print(f"{name} storage, 50 steps: error vs FP64 oracle {err:.3e}")
    assert err <= bound
    for v in (1, 6, 16):
        got = gpu_wave(plan, u0, um1, beta, 50, src=src, amp=amp, variant=v)
        assert np.array_equal(got[0], base[0])
