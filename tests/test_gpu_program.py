"""GPU parity of stencil programs (stencil_program_apply) and of the box
exchanges (faces, edges and corners) against the FP64 oracle.

Error bound: an output is a sum of at most T terms, each one or two FP32
products of FP32 values, accumulated in FP32 in program order by fused
multiply-adds (at most two roundings per term), so
|gpu - exact| <= (T + 2) 2^-24 * M at every point, where M is the same
program evaluated with |coefficients| and |inputs| (computed by the oracle).
The oracle's own error is ~1e-16 M."""
import itertools

import numpy as np
import pytest

import oracle
import paper_2404_02218_amd as S
import workloads as W
from paper_2404_02218_amd.program import Program, pw_advection_terms

pytestmark = pytest.mark.gpu


def _rand_program(rng, nin, nout, nterms, r, ndim):
    terms = []
    for _ in range(nterms):
        nfac = int(rng.integers(1, 3))
        facs = [(int(rng.integers(0, nin)), tuple(int(x) for x in rng.integers(-r, r + 1, size=ndim)))
                for _ in range(nfac)]
        terms.append((int(rng.integers(0, nout)), float(rng.standard_normal()), facs))
    return terms


def _embed(a, h):
    return np.pad(a, h)


def _run(prog, arrays, variant=0):
    import torch
    prog.variant = variant
    ins = []
    for a in arrays:
        f = prog.field()
        f.load(a)
        ins.append(f)
    outs = [prog.field() for _ in range(prog.nout)]
    prog.apply_program(outs, ins)
    torch.cuda.synchronize()
    return [o.to_numpy() for o in outs]


def _bound(terms, arrays, h, nout):
    absterms = [(o, abs(c), facs) for o, c, facs in terms]
    mag = oracle.program([np.abs(a) for a in arrays], h, nout, absterms)
    per_out = [sum(1 for o, _, _ in terms if o == k) for k in range(nout)]
    return [(n + 2) * 2.0 ** -24 * m + 1e-30 for n, m in zip(per_out, mag)]


@pytest.mark.parametrize("shape,h,r", [((13, 40, 70), 2, 2), ((9, 17, 130), 2, 1), ((1, 5, 7), 2, 2),
                                       ((50, 77), 2, 2), ((3, 64, 64), 1, 1)])
def test_random_programs_meet_the_fp32_bound(device, shape, h, r):
    rng = np.random.default_rng(hash(shape) % 2 ** 31)
    ndim = len(shape)
    terms = _rand_program(rng, 3, 2, 30, r, ndim)
    arrays = [W.round_to_storage(_embed(rng.standard_normal(shape), h), "f32") for _ in range(3)]
    prog = Program(shape, h, 3, 2, terms)
    got = _run(prog, arrays)
    # the compiled kernels (variants 0, 2 and 3) and the generic one (1) compute the same bits
    for v in range(1, prog.variant_count()):
        for a, b in zip(got, _run(prog, arrays, variant=v)):
            assert np.array_equal(a, b), v
    ref = oracle.program(arrays, h, 2, terms)
    bnd = _bound(terms, arrays, h, 2)
    I = (slice(h, -h),) * ndim
    for g, rf, b in zip(got, ref, bnd):
        assert np.all(np.abs(g[I] - rf[I]) <= b[I])
        # interior only: the outputs' halos are untouched (zero)
        m = np.ones(g.shape, dtype=bool)
        m[I] = False
        assert not np.any(g[m])


@pytest.mark.parametrize("shape", [(24, 40, 70), (16, 33, 64), (5, 7, 9)])
def test_pw_advection_program_matches_the_oracle_scheme(device, shape):
    """The product's 60-term expansion on the GPU against the oracle's direct
    C-grid formulas, on a periodic velocity (halos filled by wrapping)."""
    rng = np.random.default_rng(sum(shape))
    dx, dy, dz = 0.8, 1.1, 0.6
    vel = [W.round_to_storage(np.pad(rng.standard_normal(shape), 1, mode="wrap"), "f32") for _ in range(3)]
    terms = pw_advection_terms(dx, dy, dz)
    prog = Program(shape, 1, 3, 3, terms)
    got = _run(prog, vel)
    assert prog.variant_count() == 4
    for v in range(1, 4):
        for a, b in zip(got, _run(prog, vel, variant=v)):
            assert np.array_equal(a, b), v
    ref = oracle.pw_advection(*vel, 1, dx, dy, dz)
    bnd = _bound(terms, vel, 1, 3)
    I = (slice(1, -1),) * 3
    for g, rf, b in zip(got, ref, bnd):
        assert np.all(np.abs(g[I] - rf[I]) <= b[I])
        assert np.max(np.abs(rf[I])) > 0.1


def test_tuning_a_program_keeps_a_compiled_variant_and_its_bits(device):
    """stencil_tune on a program plan (fields: inputs, then outputs) times
    the compiled variants on the caller's fields and keeps one of them; the
    outputs then hold the program's result, the bits of every variant."""
    shape = (20, 70, 130)
    rng = np.random.default_rng(77)
    vel = [W.round_to_storage(np.pad(rng.standard_normal(shape), 1, mode="wrap"), "f32") for _ in range(3)]
    prog = Program(shape, 1, 3, 3, pw_advection_terms(1.0, 1.0, 1.0))
    want = _run(prog, vel, variant=0)
    ins = [prog.field() for _ in range(3)]
    for f, a in zip(ins, vel):
        f.load(a)
    outs = [prog.field() for _ in range(3)]
    v = prog.tune(ins + outs, reps=3)
    assert v in (0, 2, 3) and v == prog.variant
    import torch
    torch.cuda.synchronize()
    for o, w in zip(outs, want):
        assert np.array_equal(o.to_numpy(), w)
    for a, b in zip(_run(prog, vel, variant=v), want):
        assert np.array_equal(a, b)


def test_pw_advection_periodic_decomposition_equals_monolithic(device):
    """2 x 2 x 1 subdomains whose halos (faces, edges, corners) are filled by
    packing the neighbours' send boxes and unpacking them, on the GPU; the
    subdomain results equal the whole-domain run with a periodic
    self-exchange, bit for bit."""
    import torch
    shape, grid = (12, 32, 64), [2, 2, 1]
    sub = tuple(s // g for s, g in zip(shape, grid))
    rng = np.random.default_rng(77)
    whole = [W.round_to_storage(rng.standard_normal(shape), "f32") for _ in range(3)]
    terms = pw_advection_terms(1.0, 1.0, 1.0)
    mono = Program(shape, 1, 3, 3, terms)
    mf = []
    for a in whole:
        f = mono.field()
        f.load(_embed(a, 1))
        ex = mono.exchanges([1, 1, 1], [0, 0, 0], periodic=True, box=True)
        assert len(ex) == 26
        # a periodic self-exchange: the receive box of direction d takes the
        # send box of direction -d (what the neighbour on side d sends back)
        send = [[x for x in ex if tuple(x.to[:3]) == tuple(-t for t in e.to[:3])][0] for e in ex]
        buf = torch.empty(mono.exchange_elems(ex), dtype=torch.float32, device=device)
        mono.pack(f, send, buf)
        mono.unpack(f, ex, buf)
        mf.append(f)
    mo = [mono.field() for _ in range(3)]
    mono.apply_program(mo, mf)
    torch.cuda.synchronize()
    mono_out = [o.to_numpy()[(slice(1, -1),) * 3] for o in mo]

    prog = Program(sub, 1, 3, 3, terms)
    fields = {}
    for co in itertools.product(*[range(g) for g in grid]):
        sl = tuple(slice(c * n, (c + 1) * n) for c, n in zip(co, sub))
        fs = []
        for a in whole:
            f = prog.field()
            f.load(_embed(a[sl], 1))
            fs.append(f)
        fields[co] = fs
    for co in fields:
        for k in range(3):
            for e in prog.exchanges(grid, co, periodic=True, box=True):
                nb = tuple((c + t) % g for c, t, g in zip(co, e.to[:3], grid))
                back = [x for x in prog.exchanges(grid, nb, periodic=True, box=True)
                        if tuple(x.to[:3]) == tuple(-t for t in e.to[:3])][0]
                buf = torch.empty(prog.exchange_elems([e]), dtype=torch.float32, device=device)
                prog.pack(fields[nb][k], [back], buf)
                prog.unpack(fields[co][k], [e], buf)
    for co, fs in fields.items():
        outs = [prog.field() for _ in range(3)]
        prog.apply_program(outs, fs)
        torch.cuda.synchronize()
        sl = tuple(slice(c * n, (c + 1) * n) for c, n in zip(co, sub))
        for o, m in zip(outs, mono_out):
            assert np.array_equal(o.to_numpy()[(slice(1, -1),) * 3], m[sl]), co


def _advect_steps(shape, dt):
    """Forward-Euler loop of the PW advection as a step list over 9 fields:
    velocities (0, 1, 2) and (6, 7, 8), tendencies (3, 4, 5); each iteration
    advances (0,1,2) -> (6,7,8) -> (0,1,2)."""
    pw = Program(shape, 1, 3, 3, pw_advection_terms(1.0, 1.0, 1.0))
    upd = Program(shape, 1, 2, 1, [(0, 1.0, [(0, (0, 0, 0))]), (0, dt, [(1, (0, 0, 0))])])
    steps = []
    for a, b in (((0, 1, 2), (6, 7, 8)), ((6, 7, 8), (0, 1, 2))):
        steps.append((pw, list(a), [3, 4, 5]))
        for c in range(3):
            steps.append((upd, [a[c], 3 + c], [b[c]]))
    return pw, steps


def _run_schedule(pw, steps, fields, pro, body, iters, device):
    """Execute a schedule on the GPU: exchanges as a periodic self-exchange
    of the selected boxes (pack the partners' send boxes, unpack them)."""
    import torch
    from paper_2404_02218_amd.program import select
    ex = pw.exchanges([1, 1, 1], [0, 0, 0], periodic=True, box=True)
    buf = torch.empty(pw.exchange_elems(ex), dtype=torch.float32, device=device)
    moved = 0

    def run(acts):
        nonlocal moved
        for a in acts:
            if a.kind == "exchange":
                sel = select(ex, a.dirs, 3)
                partner = [[x for x in ex if tuple(x.to[:3]) == tuple(-t for t in e.to[:3])][0] for e in sel]
                pw.pack(fields[a.field], partner, buf)
                pw.unpack(fields[a.field], sel, buf)
                moved += pw.exchange_elems(sel)
            else:
                prog, ins, outs = steps[a.step]
                prog.apply_program([fields[f] for f in outs], [fields[f] for f in ins])
    run(pro)
    for _ in range(iters):
        run(body)
    torch.cuda.synchronize()
    return moved


def test_scheduled_exchanges_equal_exchanging_everything(device):
    """The pruned schedule (8 of 26 boxes per velocity, tendencies never
    exchanged) gives the same bits as exchanging every box of every input
    before every apply."""
    from paper_2404_02218_amd.program import Act, schedule
    shape = (12, 20, 36)
    pw, steps = _advect_steps(shape, 0.05)
    rng = np.random.default_rng(91)
    init = [W.round_to_storage(rng.standard_normal(shape), "f32") for _ in range(3)]
    results, moved = [], []
    full = (1 << 27) - 1 - (1 << 13)
    naive = [[], []]
    for k, (_, ins, _) in enumerate(steps):
        naive[1] += [Act("exchange", k, f, full) for f in ins] + [Act("apply", k, -1, 0)]
    for pro, body in (schedule(steps, 9, loop=True), naive):
        fields = [pw.field() for _ in range(9)]
        for f, a in zip(fields, init):
            f.load(_embed(a, 1))
        moved.append(_run_schedule(pw, steps, fields, pro, body, 3, device))
        results.append([f.to_numpy() for f in fields[:3]])
    for a, b in zip(*results):
        assert np.array_equal(a[(slice(1, -1),) * 3], b[(slice(1, -1),) * 3])
        assert np.isfinite(a).all()
    # pruned: per half-iteration each velocity once, in the directions PW
    # reads it (faces and two edges); naive: 9 inputs x all 26 boxes
    from paper_2404_02218_amd.program import select
    ex = pw.exchanges([1, 1, 1], [0, 0, 0], periodic=True, box=True)
    per_half = sum(pw.exchange_elems(select(ex, pw.halo_dirs(f), 3)) for f in range(3))
    assert moved[0] == 3 * 2 * per_half
    assert moved[1] == 3 * 2 * 9 * pw.exchange_elems(ex)


def test_compiled_program_in_a_captured_graph(device):
    """After a first apply (which loads the code object), a program apply can
    be captured in a HIP graph; every replay, with the inputs changed by eager
    work in between, equals an eager apply."""
    import torch
    shape = (20, 33, 70)
    prog = Program(shape, 1, 3, 3, pw_advection_terms(0.9, 1.1, 1.3))
    rng = np.random.default_rng(31)
    ins = [prog.field() for _ in range(3)]
    for f in ins:
        f.load(W.round_to_storage(np.pad(rng.standard_normal(shape), 1, mode="wrap"), "f32"))
    outs = [prog.field() for _ in range(3)]
    ref = [prog.field() for _ in range(3)]
    prog.apply_program(outs, ins)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        prog.apply_program(outs, ins)
    for k in range(4):
        for f in ins:
            f.view.mul_(1.0 + 0.25 * k)       # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        prog.apply_program(ref, ins)
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert np.array_equal(a.to_numpy(), b.to_numpy()), k
