"""Exchange scheduling (stencil_program_halo_dirs, stencil_schedule) checked
on the CPU with the FP64 oracle executing the schedules.

Halos start as NaN and an apply leaves its outputs' halos NaN (an apply
writes interiors only, so after it the halo is stale): a read of a stale halo
value then shows up as a NaN in an output.  A schedule is correct when no
NaN appears and every result equals the naive schedule's (every input
exchanged in all directions before every apply, the paper's swap before
every load); it is minimal when dropping any one direction of any exchange
lets a NaN through."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2404_02218_amd.program import Program, dir_code, pw_advection_terms, schedule


def _brute_dirs(terms, field, shape):
    """Directions d (codes) of the halo boxes that the reads of `field` land
    in, by visiting every interior point."""
    nd = len(shape)
    out = set()
    for _, _, facs in terms:
        for f, off in facs:
            if f != field:
                continue
            for i in itertools.product(*[range(n) for n in shape]):
                d = tuple(-1 if i[a] + off[a] < 0 else (1 if i[a] + off[a] >= shape[a] else 0) for a in range(nd))
                if any(d):
                    out.add(dir_code(d, nd))
    return sum(1 << c for c in out)


def test_halo_dirs_equal_brute_force():
    rng = np.random.default_rng(3)
    for shape in [(5, 6, 7), (3, 1, 9), (6, 8), (2, 3, 2)]:
        nd = len(shape)
        terms = [(0, 1.0, [(int(rng.integers(0, 3)), tuple(int(x) for x in rng.integers(-2, 3, size=nd)))
                           for _ in range(int(rng.integers(1, 3)))]) for _ in range(12)]
        p = Program(shape, 2, 3, 1, terms)
        for f in range(3):
            assert p.halo_dirs(f) == _brute_dirs(terms, f, shape), (shape, f)
    # PW advection: u is read across the x, y, z faces and the edges (y+, x-) and (z+, x-)
    p = Program((6, 7, 8), 1, 3, 3, pw_advection_terms(1.0, 1.0, 1.0))
    faces = {dir_code(d, 3) for d in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]}
    u_dirs = faces | {dir_code((0, 1, -1), 3), dir_code((1, 0, -1), 3)}
    assert p.halo_dirs(0) == sum(1 << c for c in u_dirs)


def _star(nin_field=0):
    return [(0, -6.0, [(nin_field, (0, 0, 0))])] + [
        (0, 1.0, [(nin_field, tuple(s if a == ax else 0 for a in range(3)))]) for ax in range(3) for s in (-1, 1)]


def test_schedule_examples():
    shape = (5, 6, 7)
    star = Program(shape, 1, 1, 1, _star())
    F = star.halo_dirs(0)
    # ping-pong: each field is exchanged once per write, nothing hoisted
    pro, body = schedule([(star, [0], [1]), (star, [1], [0])], 2)
    assert pro == []
    assert [(a.kind, a.step, a.field, a.dirs) for a in body] == [
        ("exchange", 0, 0, F), ("apply", 0, -1, 0), ("exchange", 1, 1, F), ("apply", 1, -1, 0)]
    # a coefficient field read at offsets and never written: hoisted
    coef = Program(shape, 1, 2, 1, [(0, 1.0, [(0, (0, 0, 1)), (1, (0, 0, -1))])])
    pro, body = schedule([(coef, [0, 2], [1]), (coef, [1, 2], [0])], 3)
    assert [(a.field, a.dirs) for a in pro] == [(2, coef.halo_dirs(1))]
    assert [a.field for a in body if a.kind == "exchange"] == [0, 1]
    # two reads of an unchanged field: one exchange with the union of both
    xp = Program(shape, 1, 1, 1, [(0, 1.0, [(0, (0, 0, 1))])])
    ym = Program(shape, 1, 1, 1, [(0, 1.0, [(0, (0, -1, 0))])])
    pro, body = schedule([(xp, [0], [1]), (ym, [0], [2])], 3, loop=False)
    ex = [a for a in body if a.kind == "exchange"]
    assert len(ex) == 1 and ex[0].dirs == xp.halo_dirs(0) | ym.halo_dirs(0)
    # A is read at +x before its write (step 0), written (step 1), and read at
    # -y after it (step 2): one exchange after the write, widened to the +x
    # read of the next iteration, and a prologue exchange of +x only
    pro, body = schedule([(xp, [0], [1]), (xp, [1], [0]), (ym, [0], [2])], 3)
    assert [(a.field, a.dirs) for a in pro] == [(0, xp.halo_dirs(0))]
    assert [(a.kind, a.step, a.field, a.dirs) for a in body] == [
        ("apply", 0, -1, 0), ("exchange", 1, 1, xp.halo_dirs(0)), ("apply", 1, -1, 0),
        ("exchange", 2, 0, xp.halo_dirs(0) | ym.halo_dirs(0)), ("apply", 2, -1, 0)]


def _self_exchange(a, h, shape, dirs):
    """Refresh the halo boxes of `a` in `dirs` from its own interior (one
    periodic rank: direction d receives what the partner sends towards -d)."""
    ex = oracle.exchanges(list(shape), h, h, [1] * len(shape), [0] * len(shape), periodic=True, box=True)
    nd = len(shape)
    for e in ex:
        if dirs >> dir_code(e.to[:nd], nd) & 1:
            partner = [x for x in ex if tuple(x.to[:nd]) == tuple(-t for t in e.to[:nd])][0]
            a = oracle.unpack(a, h, [e], oracle.pack(a, h, [partner]))
    return a


def _execute(steps, fields, h, shape, pro, body, iters, drop=None):
    """Run prologue + iters x body with the oracle; return the fields and
    every apply's outputs.  drop = (list, index, bit) removes one direction."""
    fields = [f.copy() for f in fields]
    I = (slice(h, -h),) * len(shape)
    outs_seen = []

    def run(acts, which):
        for i, a in enumerate(acts):
            if a.kind == "exchange":
                d = a.dirs
                if drop is not None and drop[0] == which and drop[1] == i:
                    d &= ~(1 << drop[2])
                fields[a.field] = _self_exchange(fields[a.field], h, shape, d)
            else:
                prog, ins, outs = steps[a.step]
                res = oracle.program([fields[f] for f in ins], h, len(outs), prog.terms)
                for f, r in zip(outs, res):
                    g = np.full_like(r, np.nan)
                    g[I] = r[I]
                    fields[f] = g
                    outs_seen.append(g[I])
    run(pro, "pro")
    for _ in range(iters):
        run(body, "body")
    return fields, outs_seen


def _naive(steps, nd):
    full = sum(1 << c for c in range(3 ** nd)) & ~(1 << (3 ** nd // 2))
    from paper_2404_02218_amd.program import Act
    body = []
    for k, (prog, ins, outs) in enumerate(steps):
        for f in sorted(set(ins)):
            body.append(Act("exchange", k, f, full))
        body.append(Act("apply", k, -1, 0))
    return [], body


@pytest.mark.parametrize("seed,loop", [(1, True), (2, True), (3, False), (4, True), (5, False)])
def test_random_schedules_are_correct_and_minimal(seed, loop):
    rng = np.random.default_rng(seed)
    shape, h, nfields = (4, 5, 6), 1, 4
    steps = []
    for _ in range(int(rng.integers(2, 5))):
        nin, nout = int(rng.integers(1, 3)), int(rng.integers(1, 3))
        ins = [int(x) for x in rng.choice(nfields, size=nin, replace=False)]
        free = [f for f in range(nfields) if f not in ins]
        outs = [int(x) for x in rng.choice(free, size=nout, replace=False)]
        terms = [(int(rng.integers(0, nout)), float(rng.uniform(0.5, 1.0)) * float(rng.choice([-1, 1])),
                  [(int(rng.integers(0, nin)), tuple(int(x) for x in rng.integers(-1, 2, size=3)))
                   for _ in range(int(rng.integers(1, 3)))]) for _ in range(6)]
        for o in range(nout):                       # every output gets a term
            terms.append((o, 0.5, [(int(rng.integers(0, nin)), (0, 0, 0))]))
        steps.append((Program(shape, h, nin, nout, terms), ins, outs))
    init = []
    for _ in range(nfields):
        a = np.full(tuple(n + 2 * h for n in shape), np.nan)
        a[(slice(h, -h),) * 3] = rng.uniform(-1, 1, size=shape)
        init.append(a)
    iters = 3 if loop else 1
    pro, body = schedule(steps, nfields, loop=loop)
    if not loop:
        assert pro == []
    got, seen = _execute(steps, init, h, shape, pro, body, iters)
    ref, _ = _execute(steps, init, h, shape, *_naive(steps, 3), iters)
    I = (slice(h, -h),) * 3
    assert not any(np.isnan(s).any() for s in seen)
    for g, r, a in zip(got, ref, init):
        assert np.array_equal(g[I], r[I], equal_nan=True)
    # no more exchanges than one per field before the first write plus one
    # per write of a field
    writes = sum(len(o) for _, _, o in steps)
    assert len(pro) + sum(a.kind == "exchange" for a in body) <= nfields + writes
    # minimal: every direction of every exchange is needed
    for which, acts in (("pro", pro), ("body", body)):
        for i, a in enumerate(acts):
            if a.kind != "exchange":
                continue
            assert a.dirs
            for b in range(27):
                if a.dirs >> b & 1:
                    _, seen2 = _execute(steps, init, h, shape, pro, body, iters, drop=(which, i, b))
                    assert any(np.isnan(s).any() for s in seen2), (which, i, b)


def test_schedule_validates():
    from paper_2404_02218_amd import StencilError
    shape = (5, 6, 7)
    star = Program(shape, 1, 1, 1, _star())
    with pytest.raises(StencilError):
        schedule([(star, [0], [0])], 2)             # output is an input
    with pytest.raises(StencilError):
        schedule([(star, [0], [5])], 2)             # id out of range
    flat = Program((6, 7), 1, 1, 1, [(0, 1.0, [(0, (0, 1))])])
    with pytest.raises(StencilError) as e:
        schedule([(star, [0], [1]), (flat, [1], [0])], 2)
    assert e.value.status == -5
    assert schedule([], 1) == ([], [])
