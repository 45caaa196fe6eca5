"""Pins for the FP64 oracle: each test checks it against something other than
itself -- exact rational arithmetic, closed-form solutions, the RK4 stability
polynomial, convergence order, symmetries, the safe-zone bound of Eq. (4) and
the decoding of stored precisions.  A dropped term, a wrong stage time, a wrong
sign or a transposed index in the oracle fails at least one of them.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from bto_inputs import fields, quant


# ---------------------------------------------------------------------------
# Exact rational brute force on a 4^3 grid (dyadic data): every floor and
# inside decision is exact, so flags/exit steps must agree exactly and the
# FP64 end positions to rounding.
# ---------------------------------------------------------------------------
def _rk4_fraction(grids, n, times, x0, N):
    def tri(g, p):
        cell = [min(math.floor(p[d]), n[d] - 2) for d in range(3)]
        f = [p[d] - cell[d] for d in range(3)]
        v = [Fraction(0)] * 3
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    w = (f[0] if a else 1 - f[0]) * (f[1] if b else 1 - f[1]) * (f[2] if c else 1 - f[2])
                    val = g[cell[2] + c][cell[1] + b][cell[0] + a]
                    for r in range(3):
                        v[r] += w * val[r]
        return v

    def S(p, s, th):
        if th == 0:
            return tri(grids[s], p)
        if th == 1:
            return tri(grids[s + 1], p)
        a, b = tri(grids[s], p), tri(grids[s + 1], p)
        return [(1 - th) * a[r] + th * b[r] for r in range(3)]

    def inside(p):
        return all(0 <= p[d] <= n[d] - 1 for d in range(3))

    x = list(x0)
    if not inside(x):
        return x, 1, 0
    for s in range(N):
        h = times[s + 1] - times[s]
        k1 = S(x, s, 0)
        ys = []
        ks = [k1]
        coef = [Fraction(1, 2), Fraction(1, 2), Fraction(1)]
        th = [Fraction(1, 2), Fraction(1, 2), 1]
        dead = False
        for st in range(3):
            y = [x[d] + coef[st] * h * ks[-1][d] for d in range(3)]
            if not inside(y):
                dead = True
                break
            ks.append(S(y, s, th[st]))
        if dead:
            return x, 1, s
        xn = [x[d] + h / 6 * (ks[0][d] + 2 * ks[1][d] + 2 * ks[2][d] + ks[3][d]) for d in range(3)]
        if not inside(xn):
            return x, 1, s
        x = xn
    return x, 0, N


def test_exact_rational_bruteforce_4cube():
    rng = np.random.default_rng(11)
    n = (4, 4, 4)
    N = 2  # exact denominators grow like a cube per stage: keep the run short
    ncyc = N + 1
    ints = rng.integers(-192, 193, size=(ncyc, 4, 4, 4, 3))
    grids_f = [[[[[Fraction(int(v), 64) for v in ints[c, k, j, i]] for i in range(4)] for j in range(4)]
                for k in range(4)] for c in range(ncyc)]
    grids64 = [ints[c].astype(np.float64) / 64.0 for c in range(ncyc)]
    times_f = [Fraction(s, 8) for s in range(ncyc)]
    times = np.array([float(t) for t in times_f])
    seeds_f = [[Fraction(int(a), 8) for a in rng.integers(0, 25, size=3)] for _ in range(60)]
    seeds_f += [[Fraction(0), Fraction(3), Fraction(3, 2)], [Fraction(3), Fraction(3), Fraction(3)]]
    seeds = np.array([[float(v) for v in s] for s in seeds_f])
    F = oracle.Field(n, grids64)
    r = oracle.flowmap(F, times, seeds, N)
    n_term = 0
    for p, s in enumerate(seeds_f):
        x, flag, ex = _rk4_fraction(grids_f, n, times_f, s, N)
        assert r["flag"][p] == flag, p
        assert r["exit"][p] == ex, p
        np.testing.assert_allclose(r["end"][p], [float(v) for v in x], rtol=0, atol=1e-13)
        n_term += flag == 1
    assert 0 < n_term < len(seeds_f)  # both outcomes exercised


# ---------------------------------------------------------------------------
# Trilinear sampler: exact on trilinear polynomials, linear in time.
# ---------------------------------------------------------------------------
def _poly_eval(cf, p):
    v = np.zeros(3)
    g = np.zeros((3, 3))
    for d in range(3):
        for a in range(2):
            for b in range(2):
                for c in range(2):
                    m = cf[d, a, b, c]
                    v[d] += m * p[0] ** a * p[1] ** b * p[2] ** c
                    g[d, 0] += m * a * p[1] ** b * p[2] ** c
                    g[d, 1] += m * b * p[0] ** a * p[2] ** c
                    g[d, 2] += m * c * p[0] ** a * p[1] ** b
    return v, g


def test_sampler_reproduces_trilinear_polynomials_and_time_lerp():
    rng = np.random.default_rng(3)
    n = (7, 5, 6)
    cfs = [rng.standard_normal((3, 2, 2, 2)) for _ in range(2)]
    s = fields.trilinear_polynomial(n, cfs, [0.0, 1.0])
    F = oracle.Field(n, s.grids("f64"))
    pts = rng.uniform(0, 1, size=(50, 3)) * (np.array(n) - 1)
    pts = np.vstack([pts, [[6, 4, 5], [0, 0, 0], [6, 0, 2.5], [3.0, 2.0, 1.0]]])
    for th in (0.0, 0.5, 1.0):
        for p in pts:
            v, G = oracle.sample(F, s.times, 0, th, p)
            v0, g0 = _poly_eval(cfs[0], p)
            v1, g1 = _poly_eval(cfs[1], p)
            np.testing.assert_allclose(v, (1 - th) * v0 + th * v1, atol=1e-12)
            np.testing.assert_allclose(G, (1 - th) * g0 + th * g1, atol=1e-12)


def test_stored_precisions_decode_exactly():
    rng = np.random.default_rng(5)
    n = (3, 4, 5)
    g = rng.standard_normal((5, 4, 3, 3)) * 7
    for dt in ("f32", "f16", "bf16"):
        q = quant.quantize(g, dt)
        F = oracle.Field(n, [q, q], dtype=dt)
        exact = quant.promote(q, dt)
        for (k, j, i) in [(0, 0, 0), (4, 3, 2), (2, 1, 1), (3, 2, 0)]:
            v, _ = oracle.sample(F, [0.0, 1.0], 0, 0.0, [i, j, k])
            assert np.array_equal(v, exact[k, j, i]), dt


# ---------------------------------------------------------------------------
# Closed forms for the RK4 tableau, the stage times and the cycle indexing.
# ---------------------------------------------------------------------------
def test_uniform_flow_nonuniform_steps_exact_and_exit_step():
    rng = np.random.default_rng(7)
    n = (20, 20, 20)
    N = 30
    times = np.concatenate([[0.25], 0.25 + np.cumsum(rng.uniform(0.1, 0.5, N))])
    u = np.array([0.7, -0.3, 0.45])
    s = fields.uniform_flow(n, u, times)
    F = oracle.Field(n, s.grids("f64"))
    seeds = oracle.seed_lattice(n, 3)
    r = oracle.flowmap(F, times, seeds, N)
    checked = 0
    for p, x0 in enumerate(seeds):
        traj = x0[None, :] + u[None, :] * (times[1:, None] - times[0])
        out = ~np.all((traj >= 0) & (traj <= 19), axis=1)
        # distance of each closed-form step end to the nearest face: skip ties
        if np.min(np.minimum(np.abs(traj), np.abs(19 - traj))) < 1e-9:
            continue
        checked += 1
        if out.any():
            e = int(np.argmax(out))
            assert r["flag"][p] == oracle.TERMINATED and r["exit"][p] == e
            expect = x0 + u * (times[e] - times[0])
        else:
            assert r["flag"][p] == oracle.VALID and r["exit"][p] == N
            expect = x0 + u * (times[N] - times[0])
        np.testing.assert_allclose(r["end"][p], expect, atol=1e-11)
    assert checked > 200 and (r["flag"] == 1).any() and (r["flag"] == 0).any()


def test_linear_vs_frozen_time_interpolation_closed_form():
    n = (30, 30, 30)
    N = 12
    times = np.linspace(0.0, 3.0, N + 1)
    us = np.array([[0.5 + 0.1 * c, -0.2 + 0.05 * c * c / N, 0.3 * math.cos(c)] for c in range(N + 1)])
    nx, ny, nz = n
    grids = [np.broadcast_to(us[c], (nz, ny, nx, 3)).copy() for c in range(N + 1)]
    F = oracle.Field(n, grids)
    seeds = np.array([[10.0, 12.0, 14.0], [15.5, 15.5, 15.5]])
    h = np.diff(times)
    lin = seeds + (h[:, None] * 0.5 * (us[:-1] + us[1:])).sum(0)
    fro = seeds + (h[:, None] * us[:-1]).sum(0)
    r_l = oracle.flowmap(F, times, seeds, N, mode=oracle.LINEAR)
    r_f = oracle.flowmap(F, times, seeds, N, mode=oracle.FROZEN)
    np.testing.assert_allclose(r_l["end"], lin, atol=1e-12)
    np.testing.assert_allclose(r_f["end"], fro, atol=1e-12)


def test_time_polynomial_drift_exact():
    """u = b0 + b1 t is linear in time, so linear time interpolation is exact
    and RK4 (Simpson in time) integrates it exactly: x(T) = x0 + b0 T + b1 T^2/2."""
    n = (40, 40, 40)
    N = 9
    times = np.array([0.0, 0.3, 0.5, 0.9, 1.0, 1.6, 2.0, 2.1, 2.7, 3.0])
    b0 = np.array([0.9, -0.4, 0.2])
    b1 = np.array([-0.3, 0.5, 0.6])
    nx, ny, nz = n
    grids = [np.broadcast_to(b0 + b1 * t, (nz, ny, nx, 3)).copy() for t in times]
    F = oracle.Field(n, grids)
    seeds = np.array([[12.0, 20.0, 5.0], [20.25, 20.5, 20.75]])
    r = oracle.flowmap(F, times, seeds, N)
    T0, T1 = times[0], times[-1]
    expect = seeds + b0 * (T1 - T0) + b1 * (T1 ** 2 - T0 ** 2) / 2
    np.testing.assert_allclose(r["end"], expect, atol=1e-12)


def test_solid_body_rotation_matches_rk4_amplification_factor():
    n = (16, 16, 6)
    c = (7.5, 7.5)
    Omega, w = 0.5, 0.05
    N = 40
    h = 0.125
    times = np.arange(N + 1) * h
    s = fields.solid_body_rotation(n, Omega, c, w, times)
    F = oracle.Field(n, s.grids("f64"))
    rng = np.random.default_rng(2)
    r0 = rng.uniform(0.5, 6.0, 30)
    ph = rng.uniform(0, 2 * math.pi, 30)
    seeds = np.stack([c[0] + r0 * np.cos(ph), c[1] + r0 * np.sin(ph), np.full(30, 1.5)], axis=1)
    res = oracle.flowmap(F, times, seeds, N)
    th = Omega * h
    z = 1j * th
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    # textbook modulus of the RK4 amplification factor on the imaginary axis
    assert abs(abs(R) ** 2 - (1 - th ** 6 / 72 + th ** 8 / 576)) < 1e-15
    zc = (seeds[:, 0] - c[0]) + 1j * (seeds[:, 1] - c[1])
    zN = zc * R ** N
    assert np.all(res["flag"] == 0)
    np.testing.assert_allclose(res["end"][:, 0], c[0] + zN.real, atol=1e-11)
    np.testing.assert_allclose(res["end"][:, 1], c[1] + zN.imag, atol=1e-11)
    np.testing.assert_allclose(res["end"][:, 2], 1.5 + w * N * h, atol=1e-12)
    # and the continuous solution within the RK4 global error bound
    ang = Omega * N * h
    zex = zc * np.exp(1j * ang)
    assert np.max(np.abs(zN - zex)) < 6.0 * N * th ** 5 / 120 * 2


def test_rk4_fourth_order_on_time_dependent_affine_flow():
    """u = A(t) x + b(t) with A, b linear in t: trilinear sampling and linear
    time interpolation are exact, so the oracle is RK4 on the true ODE; halving
    h must cut the error by ~16."""
    from scipy.integrate import solve_ivp

    rng = np.random.default_rng(9)
    A0 = rng.uniform(-0.3, 0.3, (3, 3))
    A1 = rng.uniform(-0.2, 0.2, (3, 3))
    b0 = rng.uniform(-0.5, 0.5, 3)
    b1 = rng.uniform(-0.5, 0.5, 3)
    n = (64, 64, 64)
    T = 2.0
    x0 = np.array([31.3, 30.7, 32.1])
    c0 = np.array([32.0, 32.0, 32.0])

    def rhs(t, x):
        return (A0 + t * A1) @ (x - c0) + b0 + t * b1

    ref = solve_ivp(rhs, (0, T), x0, method="DOP853", rtol=1e-13, atol=1e-13).y[:, -1]
    errs = []
    for N in (8, 16, 32):
        times = np.linspace(0.0, T, N + 1)
        mats = [A0 + t * A1 for t in times]
        vecs = [b0 + t * b1 - (A0 + t * A1) @ c0 for t in times]
        s = fields.affine_time_linear(n, mats, vecs, times)
        F = oracle.Field(n, s.grids("f64"))
        r = oracle.flowmap(F, times, x0[None], N)
        assert r["flag"][0] == 0
        errs.append(np.linalg.norm(r["end"][0] - ref))
    for a, b in zip(errs, errs[1:]):
        assert 12.0 < a / b < 20.0, errs


def test_abc_shear_special_case_is_trapezoid_rule():
    """B = C = 0: w = 0 and u, v depend on z only, so seeds on grid planes
    z = k move on straight lines: x(T) = x0 + A sin(Z0) sum h (s_n + s_n+1)/2."""
    n = (24, 24, 24)
    N = 20
    s = fields.abc_noise(n, N + 1, 0.05, A=math.sqrt(3), B=0.0, C=0.0, sigma=0.0)
    F = oracle.Field(n, s.grids("f64"))
    seeds = np.array([[6.25, 7.5, float(k)] for k in range(0, 24, 3)])
    r = oracle.flowmap(F, s.times, seeds, N)
    sv = 1 + 0.1 * np.sin(s.times)
    integ = (np.diff(s.times) * 0.5 * (sv[:-1] + sv[1:])).sum()
    Z = 2 * math.pi * seeds[:, 2] / 256
    A = math.sqrt(3)
    assert np.all(r["flag"] == 0)
    np.testing.assert_allclose(r["end"][:, 0], seeds[:, 0] + A * np.sin(Z) * integ, atol=1e-12)
    np.testing.assert_allclose(r["end"][:, 1], seeds[:, 1] + A * np.cos(Z) * integ, atol=1e-12)
    np.testing.assert_allclose(r["end"][:, 2], seeds[:, 2], atol=0)


def test_double_gyre_vertical_motion_closed_form():
    """w = 3.2 sin(pi z/32) cells/time decouples: z(t) = (64/pi) atan(tan(pi z0/64) e^{0.1 pi t}).
    The grid-sampled oracle must agree within the linear-interpolation bound
    (1/8) max|w''| grown by Gronwall over T = 5: about 0.05 cells."""
    s = fields.double_gyre()
    F = oracle.Field(s.n, s.grids("f64"))
    seeds = oracle.seed_lattice(s.n, 2)
    r = oracle.flowmap(F, s.times, seeds, 50)
    ok = r["flag"] == 0
    T = s.times[50]
    z = (64 / math.pi) * np.arctan(np.tan(math.pi * seeds[ok, 2] / 64) * math.exp(0.1 * math.pi * T))
    err = np.abs(r["end"][ok, 2] - z)
    eps = 3.2 * (math.pi / 32) ** 2 / 8
    L = 3.2 * math.pi / 32
    assert err.max() < eps * (math.exp(L * T) - 1) / L
    assert 0.15 < (r["flag"] == 1).mean() < 0.35


def test_axis_permutation_symmetry():
    """Swapping the x and z axes of grid, components and seeds swaps the
    results (catches transposed indices or components)."""
    s = fields.abc_noise((20, 20, 20), 11, 0.05, sigma=0.02, seed=4)
    gs = s.grids("f64")
    gp = [np.ascontiguousarray(g.transpose(2, 1, 0, 3)[..., ::-1]) for g in gs]
    n = (20, 20, 20)
    seeds = oracle.seed_lattice(n, 3)
    r = oracle.flowmap(oracle.Field(n, gs), s.times, seeds, 10)
    rp = oracle.flowmap(oracle.Field(n, gp), s.times, seeds[:, ::-1], 10)
    amb = r["margin"] < 1e-9
    assert np.array_equal(r["flag"][~amb], rp["flag"][~amb])
    np.testing.assert_allclose(r["end"], rp["end"][:, ::-1], atol=1e-12)

    # and a non-cubic block with a different extent per axis
    n2 = (12, 17, 9)
    s2 = fields.abc_noise(n2, 6, 0.05, sigma=0.02, seed=5)
    g2 = s2.grids("f64")
    g2p = [np.ascontiguousarray(g.transpose(2, 1, 0, 3)[..., ::-1]) for g in g2]
    sd = oracle.seed_lattice(n2, 2)
    a = oracle.flowmap(oracle.Field(n2, g2), s2.times, sd, 5)
    b = oracle.flowmap(oracle.Field(n2[::-1], g2p), s2.times, sd[:, ::-1], 5)
    assert np.array_equal(a["flag"], b["flag"]) and np.array_equal(a["exit"], b["exit"])
    np.testing.assert_allclose(a["end"], b["end"][:, ::-1], atol=1e-12)


@pytest.mark.parametrize("which", ["double_gyre", "abc"])
def test_safe_zone_invariant_eq4(which):
    """Eq. (4): a seed farther from every face than the largest distance a
    particle can travel in the interval cannot be terminated."""
    if which == "double_gyre":
        s = fields.double_gyre()
        N = 8
    else:
        s = fields.abc_noise((40, 40, 40), 31, 0.05, sigma=0.01, seed=6)
        N = 30
    gs = s.grids("f64")
    F = oracle.Field(s.n, gs)
    seeds = oracle.seed_lattice(s.n, 1)
    r = oracle.flowmap(F, s.times, seeds, N)
    vmax = [np.sqrt((g * g).sum(-1)).max() for g in gs]
    reach = sum((s.times[c + 1] - s.times[c]) * max(vmax[c], vmax[c + 1]) for c in range(N))
    nn = np.array(s.n) - 1
    dist = np.minimum(seeds, nn - seeds).min(axis=1)
    safe = dist > reach
    assert safe.any() and (r["flag"][~safe] == 1).any()
    assert np.all(r["flag"][safe] == 0)
    assert np.all(r["exit"][safe] == N)


def test_seed_lattice_definition():
    s = oracle.seed_lattice((32, 32, 32), 2)
    assert s.shape == (4096, 3)
    assert np.array_equal(s[1], [2.5, 0.5, 0.5]) and np.array_equal(s[16], [0.5, 2.5, 0.5])
    s4 = oracle.seed_lattice((128, 128, 128), 4)
    assert s4.shape == (32768, 3) and s4[0, 0] == 1.5 and s4[-1, 2] == 125.5
    s1 = oracle.seed_lattice((5, 6, 7), 1)
    assert s1.shape == (210, 3) and s1[0, 0] == 0.0 and s1[-1].tolist() == [4, 5, 6]
    s3 = oracle.seed_lattice((10, 11, 12), 3)
    assert s3.shape == (3 * 4 * 4, 3) and s3[0, 0] == 1.0 and s3[-1].tolist() == [7.0, 10.0, 10.0]


def test_seed_outside_block_is_terminated_at_step_zero():
    n = (8, 8, 8)
    s = fields.uniform_flow(n, [0.1, 0, 0], np.arange(4) * 0.1)
    F = oracle.Field(n, s.grids("f64"))
    seeds = np.array([[-0.5, 3, 3], [3, 3, 7.01], [3, 3, 7.0], [0, 0, 0]])
    r = oracle.flowmap(F, s.times, seeds, 3)
    assert r["flag"].tolist() == [1, 1, 0, 0]
    assert r["exit"].tolist() == [0, 0, 3, 3]


def test_nonfinite_velocity_flags_invalid():
    n = (10, 10, 10)
    s = fields.uniform_flow(n, [0.5, 0.0, 0.0], np.arange(6) * 0.2)
    gs = s.grids("f64")
    gs[2][5, 5, 5] = np.nan  # point (5, 5, 5) at cycle 2
    F = oracle.Field(n, gs)
    seeds = np.array([[4.0, 5.0, 5.0], [4.0, 2.0, 2.0]])
    r = oracle.flowmap(F, s.times, seeds, 5)
    assert r["flag"][0] == oracle.INVALID and r["flag"][1] == oracle.VALID
    # step 1 is the first to read cycle 2 (its stages 2-4), in cell (4, 5, 5)
    assert r["exit"][0] == 1
    assert np.all(np.isfinite(r["end"][0]))


# ---------------------------------------------------------------------------
# Exit point on the block surface (a terminated particle's last segment, from
# its last inside position to the first outside point, cut at the surface).
# ---------------------------------------------------------------------------
def test_exit_point_of_uniform_flow_is_the_line_face_crossing():
    rng = np.random.default_rng(11)
    n = (14, 12, 10)
    N = 25
    times = np.concatenate([[0.0], np.cumsum(rng.uniform(0.2, 0.6, N))])
    hi = np.array(n, dtype=float) - 1
    checked = 0
    for u in (np.array([0.9, -0.35, 0.2]), np.array([-0.4, 0.6, -0.75])):
        s = fields.uniform_flow(n, u, times)
        F = oracle.Field(n, s.grids("f64"))
        seeds = oracle.seed_lattice(n, 2)
        r = oracle.flowmap(F, times, seeds, N)
        for p, x0 in enumerate(seeds):
            # time at which the straight line x0 + u t leaves the box, per face
            t_face = np.where(u > 0, (hi - x0) / u, np.where(u < 0, -x0 / u, np.inf))
            t_star = t_face.min()
            if r["flag"][p] != oracle.TERMINATED:
                assert np.all(np.isnan(r["face"][p]))
                continue
            a = int(np.argmin(t_face))
            if np.sort(t_face)[1] - t_star < 1e-9:
                continue  # leaves through an edge: either face is right
            checked += 1
            np.testing.assert_allclose(r["face"][p], x0 + u * t_star, atol=1e-11)
            assert r["face"][p][a] == (hi[a] if u[a] > 0 else 0.0)
            assert r["face_cond"][p] == pytest.approx(np.abs(u).max() / abs(u[a]), rel=1e-12)
    assert checked > 300


def _rk4_rotation_stages(z, c3, Omega, h, w):
    """Classic RK4 stage points of dz/dt = i Omega z (complex, about the axis),
    vertical speed w: the three stage points and the step end."""
    k1 = 1j * Omega * z
    z2 = z + h / 2 * k1
    k2 = 1j * Omega * z2
    z3 = z + h / 2 * k2
    k3 = 1j * Omega * z3
    z4 = z + h * k3
    k4 = 1j * Omega * z4
    zn = z + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return [(z2, c3 + h / 2 * w), (z3, c3 + h / 2 * w), (z4, c3 + h * w), (zn, c3 + h * w)]


def test_exit_point_of_rotation_by_bisection_on_the_last_segment():
    n = (16, 16, 6)
    c = (5.5, 7.5)
    radii = (5.0, 7.2)
    Omega, w, h, N = 0.5, 0.0, 0.125, 60
    times = np.arange(N + 1) * h
    s = fields.solid_body_rotation(n, Omega, c, w, times)
    F = oracle.Field(n, s.grids("f64"))
    rng = np.random.default_rng(4)
    r0 = rng.uniform(radii[0], radii[1], 200)
    ph = rng.uniform(0, 2 * math.pi, 200)
    seeds = np.stack([c[0] + r0 * np.cos(ph), c[1] + r0 * np.sin(ph), np.full(200, 1.5)], axis=1)
    hi = np.array(n, dtype=float) - 1
    seeds = seeds[np.all((seeds >= 0) & (seeds <= hi), axis=1)]  # start inside the box
    res = oracle.flowmap(F, times, seeds, N)

    def inside(p):
        return bool(np.all(p >= 0) and np.all(p <= hi))

    kinds = []
    for p in range(len(seeds)):
        z = (seeds[p, 0] - c[0]) + 1j * (seeds[p, 1] - c[1])
        x = seeds[p].copy()
        out = None
        for st in range(N):
            for kind, (zz, zc) in enumerate(_rk4_rotation_stages(z, x[2], Omega, h, w)):
                q = np.array([c[0] + zz.real, c[1] + zz.imag, zc])
                if not inside(q):
                    out = q
                    break
            if out is not None:
                break
            zz, zc = _rk4_rotation_stages(z, x[2], Omega, h, w)[-1]
            z = zz
            x = np.array([c[0] + z.real, c[1] + z.imag, zc])
        if out is None:
            assert res["flag"][p] == oracle.VALID and np.all(np.isnan(res["face"][p]))
            continue
        if np.min(np.minimum(np.abs(out), np.abs(hi - out))) < 1e-9:
            continue  # outside point on a face to rounding: the event is a tie
        assert res["flag"][p] == oracle.TERMINATED and res["exit"][p] == st
        np.testing.assert_allclose(res["end"][p], x, atol=1e-10)
        lo_t, hi_t = 0.0, 1.0  # largest fraction of the segment still inside
        for _ in range(80):
            mid = 0.5 * (lo_t + hi_t)
            lo_t, hi_t = (mid, hi_t) if inside(x + mid * (out - x)) else (lo_t, mid)
        f = x + lo_t * (out - x)
        np.testing.assert_allclose(res["face"][p], f, atol=1e-9)
        # on the surface: one coordinate exactly on a face, all inside
        assert inside(res["face"][p])
        assert np.min(np.minimum(res["face"][p], hi - res["face"][p])) == 0.0
        kinds.append(kind)
    assert len(kinds) >= 15


def test_exit_point_when_only_the_step_end_leaves():
    """Two cycles, u_x = U everywhere; u_y = -a at cycle 0 and at cycle 1 for
    x <= 9, +B for x >= 10 (a ramp across the cell in between).  Seeds with
    x in [6, 7] and h U = 4 put the stage points y2, y3 at x + 2 (u_y = -a at
    both stage times) and y4 at x + 4 (u_y = B at theta = 1), so k = (U, -a),
    (U, -a), (U, -a), (U, B) exactly: every stage point moves down while the
    step end moves up by h (B - 5a) / 6 and leaves through the top face."""
    n = (16, 16, 4)
    U, a, B, h = 2.0, 0.1, 2.0, 2.0
    g0 = np.zeros((n[2], n[1], n[0], 3))
    g0[..., 0] = U
    g0[..., 1] = -a
    g1 = g0.copy()
    g1[:, :, 10:, 1] = B
    F = oracle.Field(n, [g0, g1])
    times = np.array([0.0, h])
    rng = np.random.default_rng(9)
    P = 200
    seeds = np.stack([rng.uniform(6.0, 7.0, P), rng.uniform(13.0, 15.0, P), rng.uniform(0.5, 2.5, P)], axis=1)
    r = oracle.flowmap(F, times, seeds, 1)
    dy = h * (B - 5 * a) / 6
    xn = seeds + np.array([h * U, dy, 0.0])
    leaves = xn[:, 1] > 15.0
    assert 30 < leaves.sum() < P - 30
    assert np.all(r["flag"][leaves] == oracle.TERMINATED) and np.all(r["exit"][leaves] == 0)
    np.testing.assert_allclose(r["end"][leaves], seeds[leaves], atol=0)
    tau = (15.0 - seeds[leaves, 1]) / dy
    np.testing.assert_allclose(r["face"][leaves], seeds[leaves] + tau[:, None] * (xn[leaves] - seeds[leaves]),
                               atol=1e-12)
    assert np.all(r["face"][leaves][:, 1] == 15.0)
    np.testing.assert_allclose(r["face_cond"][leaves], h * U / dy, rtol=1e-12)
    assert np.all(r["flag"][~leaves] == oracle.VALID) and np.all(np.isnan(r["face"][~leaves]))
    np.testing.assert_allclose(r["end"][~leaves], xn[~leaves], atol=1e-12)


def test_exit_point_absent_for_outside_seeds_and_invalid_particles():
    n = (10, 10, 10)
    s = fields.uniform_flow(n, [0.5, 0.0, 0.0], np.arange(6) * 0.2)
    gs = s.grids("f64")
    gs[2][5, 5, 5] = np.nan
    F = oracle.Field(n, gs)
    seeds = np.array([[4.0, 5.0, 5.0], [-0.5, 3.0, 3.0], [8.7, 2.0, 2.0]])
    r = oracle.flowmap(F, s.times, seeds, 5)
    assert r["flag"].tolist() == [oracle.INVALID, oracle.TERMINATED, oracle.TERMINATED]
    assert np.all(np.isnan(r["face"][:2])) and np.isnan(r["face_cond"][:2]).all()
    np.testing.assert_allclose(r["face"][2], [9.0, 2.0, 2.0], atol=1e-12)
