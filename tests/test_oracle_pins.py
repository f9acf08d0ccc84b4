"""Pins of the FP64 oracle against facts that do not come from the oracle
itself: textbook weights, closed-form Fourier-mode decay and plane-wave
dispersion, the light cone, a dense Kronecker-sum formulation, exact
rational evaluation, the paper's printed exchange declarations, the
decomposed == monolithic identity, and the adjoint's dot-product,
finite-difference and Taylor tests.  CPU only."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# finite-difference weights
# ---------------------------------------------------------------------------

def test_weights_match_textbook_tables():
    # centred second-difference weights, standard tables (Fornberg 1988)
    assert oracle.fd_weights(2) == [Fraction(-2), Fraction(1)]
    assert oracle.fd_weights(4) == [Fraction(-5, 2), Fraction(4, 3), Fraction(-1, 12)]
    assert oracle.fd_weights(8) == [Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5),
                                    Fraction(8, 315), Fraction(-1, 560)]


@pytest.mark.parametrize("so", [2, 4, 6, 8])
def test_weights_symbol_accuracy_order(so):
    # S(theta) = theta^2 + O(theta^(so+2)): halving theta shrinks the error 2^(so+2)x
    c = oracle.fd_weights(so)
    e1 = abs(oracle.symbol(c, 0.4) - 0.16)
    e2 = abs(oracle.symbol(c, 0.2) - 0.04)
    assert e1 > 0
    assert 0.8 * 2 ** (so + 2) < e1 / e2 < 1.2 * 2 ** (so + 2)


# ---------------------------------------------------------------------------
# heat: closed forms
# ---------------------------------------------------------------------------

def test_heat_dirichlet_sine_mode_2d_so2():
    n, alpha, steps = 30, 0.2, 40
    p, q = 3, 5
    i = np.arange(1, n + 1)
    mode = np.outer(np.sin(math.pi * p * i / (n + 1)), np.sin(math.pi * q * i / (n + 1)))
    g = 1 - 4 * alpha * (math.sin(math.pi * p / (2 * (n + 1))) ** 2
                         + math.sin(math.pi * q / (2 * (n + 1))) ** 2)
    c = [alpha * x for x in oracle.fd_weights_float(2)]
    out = oracle.heat_run(W.embed(mode, 1), 1, 1, c, steps)
    np.testing.assert_allclose(W.interior_of(out, 1), g ** steps * mode, rtol=0, atol=1e-14)
    # the Dirichlet halo is never written
    assert np.all(out[0, :] == 0) and np.all(out[:, -1] == 0)


def test_heat_periodic_fourier_mode_3d_so4():
    shape, alpha, steps = (12, 10, 16), 0.05, 25
    m = (1, 2, 3)
    k = [2 * math.pi * m[d] / shape[d] for d in range(3)]
    z, y, x = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    mode = np.cos(k[0] * z + k[1] * y + k[2] * x + 0.3)
    c4 = oracle.fd_weights(4)
    g = 1 - alpha * sum(oracle.symbol(c4, kd) for kd in k)
    c = [alpha * float(x) for x in c4]
    out = oracle.heat_run(W.embed(mode, 2), 2, 2, c, steps, periodic=True)
    np.testing.assert_allclose(W.interior_of(out, 2), g ** steps * mode, rtol=0, atol=1e-13)


def test_constant_field_is_invariant_periodic():
    c = [0.05 * float(x) for x in oracle.fd_weights(4)]
    u = np.full((9, 8, 7), 3.25)
    out = oracle.heat_run(W.embed(u, 2), 2, 2, c, 10, periodic=True)
    np.testing.assert_allclose(W.interior_of(out, 2), 3.25, rtol=1e-14)
    c8 = oracle.fd_weights_float(8)
    b = np.full((9 + 8, 8 + 8, 7 + 8), 0.03)
    a, _, _ = oracle.wave_run(W.embed(u, 4), W.embed(u, 4), b, 4, 4, c8, 12, periodic=True)
    np.testing.assert_allclose(W.interior_of(a, 4), 3.25, rtol=1e-13)


# ---------------------------------------------------------------------------
# wave: exact discrete dispersion, light cone, stability reading
# ---------------------------------------------------------------------------

def test_wave_plane_wave_exact_discrete_dispersion_so8():
    shape, steps = (16, 12, 20), 50
    m = (1, -2, 3)
    k = [2 * math.pi * m[d] / shape[d] for d in range(3)]
    c8 = oracle.fd_weights(8)
    courant = 0.2
    s = sum(oracle.symbol(c8, kd) for kd in k)
    wdt = 2 * math.asin(math.sqrt(courant ** 2 * s / 4.0))
    z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    phase = k[0] * z + k[1] * y + k[2] * x
    u0 = np.cos(phase)
    um1 = np.cos(phase + wdt)
    beta = np.full(tuple(n + 8 for n in shape), courant ** 2)
    a, b, _ = oracle.wave_run(W.embed(u0, 4), W.embed(um1, 4), beta, 4, 4,
                              [float(v) for v in c8], steps, periodic=True)
    np.testing.assert_allclose(W.interior_of(a, 4), np.cos(phase - steps * wdt), atol=1e-12)
    np.testing.assert_allclose(W.interior_of(b, 4), np.cos(phase - (steps - 1) * wdt),
                               atol=1e-12)


@pytest.mark.parametrize("steps", [1, 3, 6])
def test_wave_light_cone_is_exact(steps):
    shape, r = (24, 22, 40), 4
    s = np.array([11, 9, 14])
    rng = np.random.default_rng(5)
    beta = W.embed(rng.uniform(0.01, 0.05, shape), r)
    amp = rng.uniform(0.5, 1.5, (steps, 1))
    a, _, _ = oracle.wave_run(np.zeros_like(beta), np.zeros_like(beta), beta, r, r,
                              oracle.fd_weights_float(8), steps, src=[s], src_amp=amp)
    u = W.interior_of(a, r)
    z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    hops = (np.ceil(np.abs(z - s[0]) / r) + np.ceil(np.abs(y - s[1]) / r)
            + np.ceil(np.abs(x - s[2]) / r))
    assert np.all(u[hops > steps - 1] == 0.0)
    # and the cone is reached: the farthest point along an axis is non-zero
    tip = s.copy()
    tip[2] += r * (steps - 1)
    assert u[tuple(tip)] != 0.0


def _wave_energy_growth(courant_fraction, steps=120):
    shape = (14, 14, 14)
    rng = np.random.default_rng(11)
    u0 = W.embed(rng.standard_normal(shape), 4)
    c8 = oracle.fd_weights(8)
    s_max = oracle.symbol(c8, math.pi)
    # Courant number v dt / h as a fraction of the stability limit 2 / sqrt(3 S_max)
    cr = courant_fraction * 2.0 / math.sqrt(3 * s_max)
    beta = np.full(u0.shape, cr ** 2)
    a, _, _ = oracle.wave_run(u0, u0, beta, 4, 4, [float(v) for v in c8], steps)
    return np.abs(a).max() / np.abs(u0).max()


def test_wave_stability_reading_of_cfl():
    # half the stability limit stays bounded; a literal Courant number 0.5
    # (1.10x the limit for the 3D so-8 star) blows up
    assert _wave_energy_growth(0.5) < 10.0
    c8 = oracle.fd_weights(8)
    literal = 0.5 / (2.0 / math.sqrt(3 * oracle.symbol(c8, math.pi)))
    assert literal > 1.0
    assert _wave_energy_growth(literal) > 1e6
    assert abs(oracle.symbol(c8, math.pi) - W.S8_SYMBOL_MAX) < 1e-12


# ---------------------------------------------------------------------------
# brute force: dense Kronecker-sum operator, exact rationals
# ---------------------------------------------------------------------------

def _dense_operator(shape, c):
    """L = sum_d I x .. x A_d x .. x I with A_d[i, j] = c_|i-j| (zero halo)."""
    mats = []
    for n in shape:
        a = np.zeros((n, n))
        for i in range(n):
            for j in range(n):
                k = abs(i - j)
                if k < len(c):
                    a[i, j] = float(c[k])
        mats.append(a)
    total = None
    for d in range(len(shape)):
        term = np.ones((1, 1))
        for e in range(len(shape)):
            term = np.kron(term, mats[e] if e == d else np.eye(shape[e]))
        total = term if total is None else total + term
    return total


@pytest.mark.parametrize("shape,so", [((7, 6), 2), ((5, 6, 4), 4), ((6, 5, 7), 8), ((11,), 8)])
def test_heat_matches_dense_matrix_power(shape, so):
    r = so // 2
    rng = np.random.default_rng(1)
    u0 = rng.random(shape)
    c = [0.03 * float(x) for x in oracle.fd_weights(so)]
    L = _dense_operator(shape, c)
    steps = 5
    ref = np.linalg.matrix_power(np.eye(L.shape[0]) + L, steps) @ u0.reshape(-1)
    out = oracle.heat_run(W.embed(u0, r), r, r, c, steps)
    np.testing.assert_allclose(W.interior_of(out, r).reshape(-1), ref, rtol=1e-13, atol=1e-15)


def test_wave_matches_dense_companion_recurrence():
    shape, so, steps = (5, 6, 7), 8, 7
    r = so // 2
    rng = np.random.default_rng(2)
    beta_i = rng.uniform(0.01, 0.04, shape)
    u0 = rng.standard_normal(shape)
    um1 = rng.standard_normal(shape)
    c = oracle.fd_weights_float(so)
    L = _dense_operator(shape, c)
    B = np.diag(beta_i.reshape(-1))
    n = L.shape[0]
    a, b = u0.reshape(-1).copy(), um1.reshape(-1).copy()
    src = (2, 3, 4)
    flat = np.ravel_multi_index(src, shape)
    amp = rng.standard_normal(steps)
    trace = []
    for t in range(steps):
        new = (2 * np.eye(n) + B @ L) @ a - b
        new[flat] += amp[t]
        trace.append(new[flat])
        a, b = new, a
    out_a, out_b, tr = oracle.wave_run(W.embed(u0, r), W.embed(um1, r), W.embed(beta_i, r), r,
                                       r, c, steps, src=[src], src_amp=amp.reshape(-1, 1),
                                       rec=[src])
    np.testing.assert_allclose(W.interior_of(out_a, r).reshape(-1), a, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(W.interior_of(out_b, r).reshape(-1), b, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(tr[:, 0], trace, rtol=1e-12, atol=1e-13)


def test_1d_three_point_jacobi_exact_rationals():
    # the paper's 1D example: a 128-point field, 126 interior + 1 halo each side
    n, steps = 126, 6
    alpha = Fraction(1, 4)
    rng = np.random.default_rng(3)
    u0 = [Fraction(int(v), 1024) for v in rng.integers(0, 1024, n)]
    u = [Fraction(0)] + u0 + [Fraction(0)]
    for _ in range(steps):
        u = [Fraction(0)] + [u[i] + alpha * (u[i - 1] - 2 * u[i] + u[i + 1])
                             for i in range(1, n + 1)] + [Fraction(0)]
    c = [float(alpha * x) for x in oracle.fd_weights(2)]
    out = oracle.heat_run(np.array([0.0] + [float(v) for v in u0] + [0.0]), 1, 1, c, steps)
    assert out.shape == (128,)
    assert [Fraction(v) for v in out] == u  # dyadic inputs: FP64 is exact here


# ---------------------------------------------------------------------------
# exchange declarations and pack / unpack
# ---------------------------------------------------------------------------

def test_exchange_generator_reproduces_paper_example():
    with open(os.path.join(GOLDEN, "dmp_exchange_example.json")) as f:
        g = json.load(f)
    ex = oracle.exchanges(g["interior"], g["halo"], g["radius"], g["grid"], [0, 0],
                          periodic=True)
    decl = [e.as_dict(2) for e in ex]
    axis1 = [d for d in decl if d["to"][0] == 0]
    assert axis1 == g["printed_exchanges"]
    assert [s + 2 * g["halo"] for s in g["interior"]] == g["buffer_shape"]
    # the implied first-axis pair, and no corner boxes anywhere
    assert len(decl) == 4
    for d in decl:
        assert sum(1 for s, n in zip(d["size"], g["interior"]) if s != n) == 1


def test_exchange_missing_neighbour_is_skipped():
    ex = oracle.exchanges([10, 12, 14], 4, 4, [2, 1, 3], [0, 0, 2])
    tos = sorted(tuple(e.to[:3]) for e in ex)
    assert tos == [(0, 0, -1), (1, 0, 0)]


def _decomposed_run(kind, u_glob, beta_glob, parts, periodic, steps, r, c):
    """Split the interior into parts[0] x parts[1] x parts[2] boxes with their
    own halos, exchange faces through pack/unpack every step, sweep each."""
    shape = u_glob.shape
    loc = [shape[d] // parts[d] for d in range(3)]
    assert all(loc[d] * parts[d] == shape[d] for d in range(3))
    coords = [(i, j, k) for i in range(parts[0]) for j in range(parts[1]) for k in range(parts[2])]

    def sl(co):
        return tuple(slice(co[d] * loc[d], (co[d] + 1) * loc[d]) for d in range(3))

    u = {co: W.embed(u_glob[sl(co)], r) for co in coords}
    um1 = {co: W.embed(u_glob[sl(co)], r) for co in coords}
    beta = {co: W.embed(beta_glob[sl(co)], r) for co in coords} if beta_glob is not None else None
    ex = {co: oracle.exchanges(loc, r, r, parts, co, periodic) for co in coords}
    for _ in range(steps):
        bufs = {co: oracle.pack(u[co], r, ex[co]) for co in coords}
        for co in coords:
            off = 0
            for e in ex[co]:
                n = oracle.exchange_elems(e, 3)
                nb = tuple((co[d] + e.to[d]) % parts[d] for d in range(3))
                # partner's exchange that sends towards us
                k = next(i for i, f in enumerate(ex[nb])
                         if all(f.to[d] == -e.to[d] for d in range(3)))
                o2 = sum(oracle.exchange_elems(f, 3) for f in ex[nb][:k])
                u[co] = oracle.unpack(u[co], r, [e], bufs[nb][o2:o2 + n])
                off += n
        for co in coords:
            if kind == "heat":
                u[co] = oracle.heat_run(u[co], r, r, c, 1)
            else:
                a, b, _ = oracle.wave_run(u[co], um1[co], beta[co], r, r, c, 1)
                u[co], um1[co] = a, b
    out = np.zeros(shape)
    for co in coords:
        out[sl(co)] = W.interior_of(u[co], r)
    return out


@pytest.mark.parametrize("periodic", [False, True])
def test_decomposed_equals_monolithic_bitwise(periodic):
    rng = np.random.default_rng(7)
    shape, r = (12, 10, 16), 2
    u0 = rng.random(shape)
    c = [0.05 * float(x) for x in oracle.fd_weights(4)]
    mono = W.interior_of(oracle.heat_run(W.embed(u0, r), r, r, c, 6, periodic=periodic), r)
    dec = _decomposed_run("heat", u0, None, (2, 1, 2), periodic, 6, r, c)
    assert np.array_equal(mono, dec)


def test_decomposed_wave_equals_monolithic_bitwise():
    rng = np.random.default_rng(8)
    shape, r = (16, 8, 12), 4
    u0 = rng.standard_normal(shape)
    beta = rng.uniform(0.01, 0.04, shape)
    c = oracle.fd_weights_float(8)
    a, _, _ = oracle.wave_run(W.embed(u0, r), W.embed(u0, r), W.embed(beta, r), r, r, c, 5)
    dec = _decomposed_run("wave", u0, beta, (2, 2, 3), False, 5, r, c)
    assert np.array_equal(W.interior_of(a, r), dec)


# ---------------------------------------------------------------------------
# adjoint and gradient
# ---------------------------------------------------------------------------

def test_adjoint_dot_product():
    rng = np.random.default_rng(9)
    shape, r, steps = (10, 9, 11), 4, 30
    beta_i = rng.uniform(0.01, 0.04, shape)
    beta = W.embed(beta_i, r)
    c = oracle.fd_weights_float(8)
    srcs = np.array([[2, 3, 4], [5, 5, 5], [7, 1, 9]])
    recs = np.array([[1, 1, 1], [8, 7, 2], [4, 4, 8], [5, 5, 5]])
    a = rng.standard_normal((steps, len(srcs)))
    res = rng.standard_normal((steps, len(recs)))
    z = np.zeros_like(beta)
    _, _, d = oracle.wave_run(z, z, beta, r, r, c, steps, src=srcs, src_amp=a, rec=recs)
    lhs = float(np.sum(d * res))
    w = np.array([beta_i[tuple(p)] for p in recs])
    lam = oracle.wave_adjoint(beta, r, r, c, steps, recs, w, res, srcs)
    bs = np.array([beta_i[tuple(p)] for p in srcs])
    rhs = float(np.sum(a * lam / bs))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def _misfit_problem(shape=(14, 13, 15), steps=70, seed=12):
    rng = np.random.default_rng(seed)
    h = 10.0
    v0 = W.layered_velocity(rng, shape)
    vt = v0 * (1 + 0.05 * rng.uniform(-1, 1, shape))
    dt = W.wave_dt(max(v0.max(), vt.max()) * 1.06, h)
    src = np.array([[3, shape[1] // 2, shape[2] // 2]])
    rec = np.array([[2, shape[1] // 2, x] for x in range(2, shape[2] - 2, 3)])
    w = W.ricker(np.arange(steps) * dt, f0=40.0)
    return dict(h=h, dt=dt, m0=1 / v0 ** 2, mt=1 / vt ** 2, src=src, rec=rec, w=w,
                steps=steps, r=4, c=oracle.fd_weights_float(8))


def _J_and_grad(P, m, dobs):
    r, dt, h = P["r"], P["dt"], P["h"]
    beta = W.embed(dt * dt / (h * h * m), r)
    amp = (dt * dt / m[tuple(P["src"][0])] * P["w"]).reshape(-1, 1)
    rec_w = np.array([dt * dt / m[tuple(p)] for p in P["rec"]])
    return oracle.wave_gradient(beta, r, r, P["c"], P["steps"], P["src"], amp, P["rec"], dobs,
                                rec_w, -1.0 / (dt * dt))


def test_gradient_matches_central_differences_and_taylor():
    P = _misfit_problem()
    nrec = len(P["rec"])
    dobs0 = np.zeros((P["steps"], nrec))
    dobs, _, _ = _J_and_grad(P, P["mt"], dobs0)
    _, J0, g = _J_and_grad(P, P["m0"], dobs)
    assert J0 > 0
    rng = np.random.default_rng(13)
    dm = rng.standard_normal(P["m0"].shape) * P["m0"] * 0.01
    gdm = float(np.sum(g * dm))
    eps = 1e-3
    _, Jp, _ = _J_and_grad(P, P["m0"] + eps * dm, dobs)
    _, Jm, _ = _J_and_grad(P, P["m0"] - eps * dm, dobs)
    fd = (Jp - Jm) / (2 * eps)
    assert abs(fd - gdm) <= 1e-6 * abs(gdm)
    # Taylor: the first-order remainder decays quadratically
    rem = []
    for e in (4e-2, 2e-2, 1e-2):
        _, Je, _ = _J_and_grad(P, P["m0"] + e * dm, dobs)
        rem.append(abs(Je - J0 - e * gdm))
    assert 3.0 < rem[0] / rem[1] < 5.0 and 3.0 < rem[1] / rem[2] < 5.0


def test_gradient_of_pointwise_perturbation():
    # one-point perturbations, including at the source and at a receiver
    P = _misfit_problem(shape=(10, 9, 11), steps=50, seed=14)
    nrec = len(P["rec"])
    dobs, _, _ = _J_and_grad(P, P["mt"], np.zeros((P["steps"], nrec)))
    _, _, g = _J_and_grad(P, P["m0"], dobs)
    for pt in [tuple(P["src"][0]), tuple(P["rec"][1]), (5, 4, 5)]:
        dm = np.zeros_like(P["m0"])
        dm[pt] = P["m0"][pt] * 1e-4
        _, Jp, _ = _J_and_grad(P, P["m0"] + dm, dobs)
        _, Jm, _ = _J_and_grad(P, P["m0"] - dm, dobs)
        fd = (Jp - Jm) / 2
        assert abs(fd - g[pt] * dm[pt]) <= 1e-5 * abs(fd) + 1e-30


# ---------------------------------------------------------------- programs
# The program interpreter and the C-grid advection are pinned to exact
# integer arithmetic, to the star operator (pinned above), and to the
# conservation laws of the flux-form advection.

def _wrap(a, h=1):
    return np.pad(a, h, mode="wrap")


def _divergence_free(shape, seed, dx, dy, dz):
    """A C-grid velocity that is the discrete curl of a random periodic
    vector potential, so its discrete divergence vanishes."""
    rng = np.random.default_rng(seed)
    A1, A2, A3 = (rng.standard_normal(shape) for _ in range(3))
    back = lambda a, ax: np.roll(a, 1, axis=ax)  # a at index - 1 along ax (periodic)
    u = (A3 - back(A3, 1)) / dy - (A2 - back(A2, 0)) / dz
    v = (A1 - back(A1, 0)) / dz - (A3 - back(A3, 2)) / dx
    w = (A2 - back(A2, 2)) / dx - (A1 - back(A1, 1)) / dy
    div = (u - back(u, 2)) / dx + (v - back(v, 1)) / dy + (w - back(w, 0)) / dz
    assert np.abs(div).max() < 1e-12
    return u, v, w


@pytest.mark.parametrize("shape,seed", [((6, 7, 8), 1), ((5, 9, 4), 2), ((8, 8, 8), 3)])
def test_advection_conserves_momentum_and_kinetic_energy(shape, seed):
    dx, dy, dz = 1.0, 1.3, 0.7
    u, v, w = _divergence_free(shape, seed, dx, dy, dz)
    su, sv, sw = oracle.pw_advection(_wrap(u), _wrap(v), _wrap(w), 1, dx, dy, dz)
    I = (slice(1, -1),) * 3
    scale = np.abs(su[I]).sum() + np.abs(sv[I]).sum() + np.abs(sw[I]).sum()
    assert scale > 1.0
    # flux form: each momentum component's total is unchanged
    for s in (su, sv, sw):
        assert abs(s[I].sum()) <= 1e-13 * scale
    # centred fluxes of a divergence-free flow do no work: kinetic energy conserved
    E = (u * su[I] + v * sv[I] + w * sw[I]).sum()
    assert abs(E) <= 1e-13 * float((np.abs(u * su[I]) + np.abs(v * sv[I]) + np.abs(w * sw[I])).sum())
    # a flow that is not divergence-free does change the energy (the pin can fail)
    rng = np.random.default_rng(seed + 10)
    u2 = u + 0.3 * rng.standard_normal(shape)
    su2, sv2, sw2 = oracle.pw_advection(_wrap(u2), _wrap(v), _wrap(w), 1, dx, dy, dz)
    E2 = (u2 * su2[I] + v * sv2[I] + w * sw2[I]).sum()
    assert abs(E2) > 1e-6 * scale


def test_advection_exact_on_a_linear_flow_and_zero_on_a_uniform_one():
    # u = a x (x = face position), v = w = 0: the x flux term gives
    # -d(u^2)/dx = -2 a u exactly for centred averages of a linear field
    n, a, dx = 9, 0.37, 0.5
    x = (np.arange(-1, n + 1) + 0.5) * dx
    u = np.broadcast_to(a * x, (n + 2, n + 2, n + 2)).copy()
    z = np.zeros_like(u)
    su, sv, sw = oracle.pw_advection(u, z, z, 1, dx, 1.0, 1.0)
    I = (slice(1, -1),) * 3
    assert np.allclose(su[I], -2 * a * u[I], rtol=0, atol=1e-12)
    assert np.all(sv[I] == 0) and np.all(sw[I] == 0)
    c = np.full((n + 2,) * 3, 1.7)
    s = oracle.pw_advection(c, -0.4 * np.ones_like(c), 2.1 * np.ones_like(c), 1, 0.3, 0.6, 0.9)
    assert all(np.abs(q[I]).max() < 1e-12 for q in s)


def test_program_interpreter_is_exact_on_integers():
    # integer inputs and coefficients: every product and sum is exact in FP64,
    # so the oracle must equal a plain integer evaluation written here
    rng = np.random.default_rng(7)
    shape, h = (4, 5, 6), 2
    ins = [rng.integers(-9, 10, size=tuple(n + 2 * h for n in shape)).astype(np.float64) for _ in range(3)]
    terms = []
    for _ in range(25):
        nfac = int(rng.integers(1, 3))
        facs = [(int(rng.integers(0, 3)), tuple(int(x) for x in rng.integers(-2, 3, size=3))) for _ in range(nfac)]
        terms.append((int(rng.integers(0, 2)), float(rng.integers(-5, 6)), facs))
    outs = oracle.program(ins, h, 2, terms)
    ref = [np.zeros_like(ins[0]) for _ in range(2)]
    for z in range(h, h + shape[0]):
        for y in range(h, h + shape[1]):
            for x in range(h, h + shape[2]):
                for o, c, facs in terms:
                    val = int(c)
                    for f, (dz, dy, dxx) in facs:
                        val *= int(ins[f][z + dz, y + dy, x + dxx])
                    ref[o][z, y, x] += val
    for a, b in zip(outs, ref):
        assert np.array_equal(a, b)


def test_program_of_the_star_equals_the_star_operator():
    c = oracle.fd_weights_float(8)
    shape, h = (7, 8, 9), 4
    u = np.random.default_rng(8).standard_normal(tuple(n + 2 * h for n in shape))
    terms = [(0, 3 * c[0], [(0, (0, 0, 0))])]
    for k in range(1, 5):
        for ax in range(3):
            for s in (-1, 1):
                off = [0, 0, 0]
                off[ax] = s * k
                terms.append((0, c[k], [(0, tuple(off))]))
    got = oracle.program([u], h, 1, terms)[0]
    ref = oracle.star(u, h, 4, c)
    I = (slice(h, -h),) * 3
    assert np.max(np.abs(got[I] - ref[I])) <= 1e-13 * np.max(np.abs(ref[I]))


def test_box_exchanges_cover_every_neighbour_direction():
    shape, h, r = [10, 12, 14], 3, 2
    ex = oracle.exchanges(shape, h, r, [1, 1, 1], [0, 0, 0], periodic=True, box=True)
    assert len(ex) == 26
    dirs = [tuple(e.to[:3]) for e in ex]
    assert len(set(dirs)) == 26 and (0, 0, 0) not in dirs
    assert dirs == sorted(dirs)                      # C order of the direction
    faces = oracle.exchanges(shape, h, r, [1, 1, 1], [0, 0, 0], periodic=True)
    byd = {tuple(e.to[:3]): e.as_dict(3) for e in ex}
    for f in faces:                                  # face entries equal the star's
        assert byd[tuple(f.to[:3])] == f.as_dict(3)
    corner = byd[(1, -1, 1)]
    assert corner == {"at": [h + 10, h - r, h + 14], "size": [r, r, r], "src_offset": [-r, r, -r],
                      "to": [1, -1, 1]}
    # a corner rank of a non-periodic 2D grid: 2 faces and 1 corner
    ex2 = oracle.exchanges([8, 8], 1, 1, [2, 2], [0, 0], box=True)
    assert sorted(tuple(e.to[:2]) for e in ex2) == [(0, 1), (1, 0), (1, 1)]


def test_box_exchange_decomposition_equals_monolithic_program():
    # a periodic 2 x 2 x 1 split of a diagonal-reading program, halos filled
    # by pack/unpack of the box exchanges, equals the whole-domain program
    shape, h = (6, 8, 10), 1
    rng = np.random.default_rng(9)
    terms = [(0, 0.5, [(0, (0, 1, -1)), (1, (1, 0, 1))]), (0, -1.25, [(1, (-1, -1, 0))]),
             (1, 2.0, [(0, (1, 1, 1))]), (1, 0.75, [(1, (0, 0, 0)), (0, (-1, 0, 1))])]
    whole = [rng.standard_normal(shape) for _ in range(2)]
    ref = oracle.program([_wrap(a) for a in whole], h, 2, terms)
    grid = [2, 2, 1]
    sub = [s // g for s, g in zip(shape, grid)]
    import itertools
    for co in itertools.product(*[range(g) for g in grid]):
        sl = tuple(slice(c * n, (c + 1) * n) for c, n in zip(co, sub))
        fields = []
        for a in whole:
            f = np.zeros(tuple(n + 2 * h for n in sub))
            f[(slice(h, -h),) * 3] = a[sl]
            # the neighbours' faces, edges and corners arrive via their packs
            for e in oracle.exchanges(sub, h, 1, grid, co, periodic=True, box=True):
                nb = [(c + t) % g for c, t, g in zip(co, e.to[:3], grid)]
                nsl = tuple(slice(c * n, (c + 1) * n) for c, n in zip(nb, sub))
                nf = np.zeros_like(f)
                nf[(slice(h, -h),) * 3] = a[nsl]
                partner = [x for x in oracle.exchanges(sub, h, 1, grid, nb, periodic=True, box=True)
                           if tuple(x.to[:3]) == tuple(-t for t in e.to[:3])][0]
                f = oracle.unpack(f, h, [e], oracle.pack(nf, h, [partner]))
            fields.append(f)
        got = oracle.program(fields, h, 2, terms)
        for g_, r_ in zip(got, ref):
            assert np.array_equal(g_[(slice(h, -h),) * 3], r_[(slice(h, -h),) * 3][sl])


@pytest.mark.parametrize("shape", [(5, 6, 7), (4, 9), (11,), (1, 6, 5)])
def test_interp_weights_reproduce_affine_functions(shape):
    # multilinear weights: non-negative, summing to 1, exact on every affine
    # function, and a single unit weight at a grid point
    rng = np.random.default_rng(len(shape) + shape[0])
    nd = len(shape)
    hi = np.array(shape, dtype=np.float64) - 1
    pos = rng.uniform(0, 1, size=(40, nd)) * hi
    pos[0] = hi                                  # the upper corner of the grid
    pos[1] = 0
    pos[2] = np.floor(pos[2])                    # a grid point
    corners, w = oracle.interp(shape, pos)
    assert (w >= 0).all() and np.allclose(w.sum(1), 1, rtol=0, atol=1e-15)
    assert (corners >= 0).all() and (corners <= hi.astype(np.int64)).all()
    for _ in range(3):
        a, b = rng.standard_normal(nd), rng.standard_normal()
        f = lambda x: x @ a + b
        got = (w * f(corners.astype(np.float64))).sum(1)
        assert np.allclose(got, f(pos), rtol=0, atol=1e-12)
    for k in (0, 1, 2):
        on = w[k] == 1.0
        assert on.sum() == 1 and np.array_equal(corners[k][on][0], pos[k].astype(np.int64))
    # every corner lies within one cell of the position
    assert (np.abs(corners - pos[:, None, :]) <= 1 + 1e-12).all()


def test_damped_wave_satisfies_the_discrete_energy_identity():
    # (u+ - 2u + u-) + g (u+ - u-) = beta L u with L symmetric (zero halo):
    # E^{n+1/2} - E^{n-1/2} = -sum (g / beta) (u+ - u-)^2, where
    # E^{n+1/2} = sum (u^{n+1} - u^n)^2 / beta - <u^{n+1}, L u^n>.  A wrong
    # sign of g, or (1 - g) and (1 + g) swapped, breaks it.
    shape, h, r = (14, 15, 16), 4, 4
    c = oracle.fd_weights_float(8)
    rng = np.random.default_rng(21)
    I = (slice(h, -h),) * 3
    pad = lambda a: np.pad(a, h)
    beta = pad(rng.uniform(0.02, 0.06, size=shape))
    prof = [np.where(np.minimum(np.arange(n), np.arange(n)[::-1]) < 4,
                     0.3 * ((4 - np.minimum(np.arange(n), np.arange(n)[::-1])) / 4.0) ** 2, 0.0) for n in shape]
    gamma = pad(prof[0][:, None, None] + prof[1][None, :, None] + prof[2][None, None, :])
    u = [pad(rng.standard_normal(shape)), None]
    u[1] = u[0] + 0.01 * pad(rng.standard_normal(shape))   # (u^{-1}, u^0)
    levels = [u[0].copy(), u[1].copy()]                       # u^{-1}, u^0, u^1, ...
    a, b = u[1], u[0]
    for _ in range(6):
        a, b, _ = oracle.wave_run_damped(a, b, beta, gamma, h, r, c, 1)
        levels.append(a.copy())
    L = lambda x: oracle.star(x, h, r, c)

    def energy(un1, un):
        return float(((un1 - un)[I] ** 2 / beta[I]).sum() - (un1[I] * L(un)[I]).sum())
    scale = float((levels[1][I] ** 2 / beta[I]).sum())
    for n in range(2, len(levels)):
        up, uc, um = levels[n], levels[n - 1], levels[n - 2]
        diss = float((gamma[I] / beta[I] * (up - um)[I] ** 2).sum())
        assert diss > 0
        assert abs(energy(up, uc) - energy(uc, um) + diss) <= 1e-11 * scale
    # no damping: the same run as the undamped oracle, bit for bit
    z = np.zeros_like(gamma)
    d = oracle.wave_run_damped(u[1], u[0], beta, z, h, r, c, 5)
    p = oracle.wave_run(u[1], u[0], beta, h, r, c, 5)
    assert all(np.array_equal(x, y) for x, y in zip(d[:2], p[:2]))
