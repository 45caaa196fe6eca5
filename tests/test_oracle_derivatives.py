"""Pins for the oracle's derivatives: the forward tangent, the discrete adjoint
(seed and grid gradients) against FP64 central finite differences of the
oracle's own forward map (h = 1e-3), with entries whose +-h runs change any
flag, exit step or stage sampling cell excluded (the map is only piecewise
smooth across cell faces), plus closed forms for uniform flow.
"""

import numpy as np

import oracle
from bto_inputs import fields

H = 1e-3


def _setup():
    n = (24, 24, 24)
    N = 16
    s = fields.abc_noise(n, N + 1, 0.05, sigma=0.05, seed=8, global_n=64)
    gs = s.grids("f64")
    seeds = oracle.seed_lattice(n, 4)
    w = np.random.default_rng(3).standard_normal(seeds.shape)
    return n, N, s, gs, seeds, w


def _loss_parts(F, times, seeds, N, w):
    r = oracle.flowmap(F, times, seeds, N)
    valid = r["flag"] == 0
    L = (w * r["end"]).sum(1) * valid
    return L, r


def test_tangent_and_adjoint_match_central_fd_on_seeds():
    n, N, s, gs, seeds, w = _setup()
    F = oracle.Field(n, gs)
    base = oracle.flowmap(F, s.times, seeds, N, jac=True)
    g = oracle.adjoint(F, s.times, seeds, N, w)
    valid = base["flag"] == 0
    assert valid.sum() > 50
    # adjoint of the masked loss equals J^T w on valid particles, 0 elsewhere
    JTw = np.einsum("pij,pi->pj", base["jac"], w)
    np.testing.assert_allclose(g[valid], JTw[valid], rtol=1e-12, atol=1e-12)
    assert np.all(g[~valid] == 0)
    fd = np.zeros((len(seeds), 3, 3))
    ok = np.ones(len(seeds), bool)
    for d in range(3):
        e = np.zeros(3)
        e[d] = H
        rp = oracle.flowmap(F, s.times, seeds + e, N)
        rm = oracle.flowmap(F, s.times, seeds - e, N)
        same = (rp["sig"] == rm["sig"]) & (rp["sig"] == base["sig"]) & \
               (rp["flag"] == base["flag"]) & (rm["flag"] == base["flag"]) & \
               (rp["exit"] == base["exit"]) & (rm["exit"] == base["exit"])
        ok &= same
        fd[:, :, d] = (rp["end"] - rm["end"]) / (2 * H)
    sel = ok & valid
    assert sel.sum() > 20
    J = base["jac"][sel]
    err = np.linalg.norm(J - fd[sel]) / np.linalg.norm(fd[sel])
    assert err < 1e-4, err
    g_fd = np.einsum("pij,pi->pj", fd[sel], w[sel])
    err_g = np.linalg.norm(g[sel] - g_fd) / np.linalg.norm(g_fd)
    assert err_g < 1e-4, err_g
    # per-entry check with a floor of 1e-3 max|g_fd|
    floor = 1e-3 * np.abs(g_fd).max()
    assert np.all(np.abs(g[sel] - g_fd) <= 1e-4 * np.maximum(np.abs(g_fd), floor) + 1e-12)


def test_adjoint_grid_gradient_matches_fd_and_is_zero_off_trajectory():
    n, N, s, gs, seeds, w = _setup()
    seeds = seeds[::5]
    w = w[::5]
    F = oracle.Field(n, gs)
    g, gg = oracle.adjoint(F, s.times, seeds, N, w, grid_grad=True)
    base = oracle.flowmap(F, s.times, seeds, N)
    rng = np.random.default_rng(4)
    nz_idx = [tuple(ix) for ix in np.argwhere(np.stack(gg) != 0)]
    zero_idx = [tuple(ix) for ix in np.argwhere(np.stack(gg) == 0)]
    assert len(nz_idx) > 100
    picks = [nz_idx[i] for i in rng.choice(len(nz_idx), 60, replace=False)] + \
            [zero_idx[i] for i in rng.choice(len(zero_idx), 20, replace=False)]
    checked = 0
    for (c, k, j, i, comp) in picks:
        vals = []
        runs = []
        for sgn in (1, -1):
            gp = list(gs)
            gp[c] = gs[c].copy()
            gp[c][k, j, i, comp] += sgn * H
            Fp = oracle.Field(n, gp)
            L, r = _loss_parts(Fp, s.times, seeds, N, w)
            vals.append(L.sum())
            runs.append(r)
        if not all(np.array_equal(r["sig"], base["sig"]) and np.array_equal(r["flag"], base["flag"])
                   and np.array_equal(r["exit"], base["exit"]) for r in runs):
            continue
        checked += 1
        fd = (vals[0] - vals[1]) / (2 * H)
        an = gg[c][k, j, i, comp]
        if an == 0.0:
            assert abs(fd) < 1e-9
        else:
            assert abs(an - fd) <= 1e-4 * abs(fd) + 1e-9, (c, k, j, i, comp, an, fd)
    assert checked > 50


def test_uniform_flow_grid_gradient_closed_form():
    """Uniform flow: the sampler gradient is zero, so lambda stays equal to the
    cotangent and dL/dV_c[corner] = sum over stages of h b_s (time weight)
    (trilinear weight) lambda; the total over the grid of cycle c is
    lambda * (h_{c-1}/2 [c>0] + h_c/2 [c<N]) -- the trapezoid weights."""
    n = (12, 12, 12)
    N = 5
    times = np.array([0.0, 0.1, 0.25, 0.3, 0.45, 0.6])
    s = fields.uniform_flow(n, [0.3, 0.2, -0.1], times)
    F = oracle.Field(n, s.grids("f64"))
    seeds = np.array([[4.3, 5.1, 6.7]])
    lam = np.array([[0.7, -1.1, 0.4]])
    g, gg = oracle.adjoint(F, times, seeds, N, lam, grid_grad=True)
    np.testing.assert_allclose(g, lam, atol=1e-15)
    h = np.diff(times)
    for c in range(N + 1):
        wt = (h[c - 1] / 2 if c > 0 else 0.0) + (h[c] / 2 if c < N else 0.0)
        np.testing.assert_allclose(gg[c].reshape(-1, 3).sum(0), wt * lam[0], atol=1e-14)


def test_ftle_definition_on_known_singular_values():
    """sigma = ln(largest singular value of J) / |T| for J = Q1 diag(s) Q2 with
    orthogonal Q1, Q2 (and 0 for a rotation)."""
    rng = np.random.default_rng(11)
    Q1, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    Q2, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    s = np.array([0.3, 4.5, 1.7])
    J = (Q1 @ np.diag(s) @ Q2)[None]
    T = 2.5
    np.testing.assert_allclose(oracle.ftle(J, T), np.log(4.5) / T, rtol=1e-13)
    np.testing.assert_allclose(oracle.ftle(J, -T), np.log(4.5) / T, rtol=1e-13)
    np.testing.assert_allclose(oracle.ftle(Q1[None], T), 0.0, atol=1e-14)


def test_jacobian_and_ftle_of_hyperbolic_strain_closed_form():
    """Steady strain u = (a (x - c), -a (y - c), 0) is linear in space, so the
    trilinear sampler is exact and every RK4 step multiplies the offsets by
    the amplification factor R(+-a h) = 1 + z + z^2/2 + z^3/6 + z^4/24: the
    flow-map Jacobian is diag(R(a h)^N, R(-a h)^N, 1) and the FTLE is
    ln R(a h) / h, independent of the seed."""
    n = (33, 33, 9)
    c, a, h, N = 16.0, 0.2, 0.1, 25
    times = np.arange(N + 1) * h
    z_, y_, x_ = np.meshgrid(np.arange(n[2], dtype=float), np.arange(n[1], dtype=float),
                             np.arange(n[0], dtype=float), indexing="ij")
    g = np.stack([a * (x_ - c), -a * (y_ - c), np.zeros_like(x_)], axis=-1)
    F = oracle.Field(n, [g] * (N + 1))
    rng = np.random.default_rng(5)
    seeds = np.stack([c + rng.uniform(-5, 5, 40), c + rng.uniform(-10, 10, 40), rng.uniform(1, 7, 40)], axis=1)
    r = oracle.flowmap(F, times, seeds, N, jac=True)
    assert np.all(r["flag"] == 0)

    def R(z):
        return 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24

    gx, gy = R(a * h) ** N, R(-a * h) ** N
    np.testing.assert_allclose(r["end"][:, 0], c + (seeds[:, 0] - c) * gx, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["end"][:, 1], c + (seeds[:, 1] - c) * gy, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["end"][:, 2], seeds[:, 2], rtol=0, atol=1e-13)
    Jw = np.zeros((3, 3))
    Jw[0, 0], Jw[1, 1], Jw[2, 2] = gx, gy, 1.0
    np.testing.assert_allclose(r["jac"], np.broadcast_to(Jw, r["jac"].shape), rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.ftle(r["jac"], N * h), np.log(R(a * h)) / h, rtol=1e-12)
