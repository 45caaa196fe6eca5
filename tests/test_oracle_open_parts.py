"""Pins for the oracle parts that the parity harness leans on but that the
other pin modules leave open:

* the decoding of stored 16-bit grids, checked for every one of the 65,536
  binary16 and bfloat16 bit patterns (subnormals, signed zeros, infinities
  and NaNs included) against numpy's own conversions;
* the face margin that the parity comparison uses to set aside particles
  whose decisions are ties (every decision point's distance to the nearest
  face): on uniform flow every RK4 stage point lies on the straight path, so
  the margin is the smallest face distance over the seed and the tested stage
  and end points, in the tested order, which is written out here directly;
* the discrete adjoint in FROZEN time mode (every stage reads the grid of the
  step's first cycle): seed gradients and grid gradients against FP64 central
  finite differences of the oracle's forward map, and the grid of the last
  cycle, which no FROZEN step reads, receiving exactly nothing.
"""

import numpy as np

import oracle
from bto_inputs import fields

H = 1e-3


# ---------------------------------------------------------------------------
# Exhaustive 16-bit decoding.
# ---------------------------------------------------------------------------
def _all_patterns_field(dtype):
    bits = np.arange(1 << 16, dtype=np.uint16)
    padded = np.concatenate([bits, np.zeros(2, np.uint16)])  # 65,538 = 3 x 21,846 values
    n = (3641, 3, 2)                                           # 21,846 points
    arr = padded.reshape(n[2], n[1], n[0], 3)
    if dtype == "f16":
        arr = arr.view(np.float16)
    F = oracle.Field(n, [arr], dtype=dtype)
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    ijk = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    got = oracle.fetch(F, 0, ijk).ravel()[: 1 << 16]
    return bits, got


def _same_values(got, want):
    nan_g, nan_w = np.isnan(got), np.isnan(want)
    assert np.array_equal(nan_g, nan_w)
    ok = ~nan_w
    assert np.array_equal(got[ok], want[ok])
    # signed zeros and infinities keep their sign
    assert np.array_equal(np.signbit(got[ok]), np.signbit(want[ok]))


def test_binary16_decode_of_every_bit_pattern():
    bits, got = _all_patterns_field("f16")
    want = bits.view(np.float16).astype(np.float64)
    _same_values(got, want)
    # spot values from the binary16 definition (sign, 5-bit exponent, 10-bit fraction)
    assert got[0x0001] == 2.0 ** -24            # smallest subnormal
    assert got[0x03FF] == 1023 * 2.0 ** -24     # largest subnormal
    assert got[0x0400] == 2.0 ** -14            # smallest normal
    assert got[0x3C00] == 1.0 and got[0xC000] == -2.0
    assert got[0x7BFF] == 65504.0
    assert got[0x7C00] == np.inf and got[0xFC00] == -np.inf
    assert np.isnan(got[0x7C01]) and np.isnan(got[0xFE00])
    assert got[0x8000] == 0.0 and np.signbit(got[0x8000])


def test_bfloat16_decode_of_every_bit_pattern():
    bits, got = _all_patterns_field("bf16")
    with np.errstate(invalid="ignore"):
        want = (bits.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
    _same_values(got, want)
    # spot values from the bfloat16 definition (binary32 with the low 16 fraction bits dropped)
    assert got[0x0001] == 2.0 ** -133           # smallest subnormal
    assert got[0x0080] == 2.0 ** -126           # smallest normal
    assert got[0x3F80] == 1.0 and got[0xC040] == -3.0
    assert got[0x7F7F] == (2.0 - 2.0 ** -7) * 2.0 ** 127
    assert got[0x7F80] == np.inf and got[0xFF80] == -np.inf
    assert np.isnan(got[0x7F81]) and np.isnan(got[0xFFC0])
    assert got[0x8000] == 0.0 and np.signbit(got[0x8000])


# ---------------------------------------------------------------------------
# Face margin on uniform flow, in closed form.
# ---------------------------------------------------------------------------
def _face_dist(n, p):
    hi = np.asarray(n, dtype=np.float64) - 1.0
    return np.minimum(np.abs(p), np.abs(hi - p)).min(axis=-1)


def _inside(n, p):
    hi = np.asarray(n, dtype=np.float64) - 1.0
    return np.all((p >= 0.0) & (p <= hi), axis=-1)


def _margin_closed_form(n, u, times, seeds, N):
    """Every decision point of a uniform flow lies on x0 + u (t - t0): per step
    the stage points at t_s + h/2 (twice) and t_s + h, then the end point at
    t_s + h; the first point outside ends the particle and is itself counted."""
    x0 = np.asarray(seeds, dtype=np.float64)
    margin = _face_dist(n, x0)
    alive = _inside(n, x0)
    for s in range(N):
        t = times[s] - times[0]
        h = times[s + 1] - times[s]
        for tau in (t + 0.5 * h, t + 0.5 * h, t + h, t + h):
            p = x0 + np.outer(np.ones(len(x0)), u) * tau
            d = _face_dist(n, p)
            margin = np.where(alive, np.minimum(margin, d), margin)
            alive &= _inside(n, p)
    return margin


def test_face_margin_of_uniform_flow_closed_form():
    rng = np.random.default_rng(31)
    n = (14, 11, 9)
    N = 12
    times = np.concatenate([[0.3], 0.3 + np.cumsum(rng.uniform(0.1, 0.4, N))])
    for u in ([0.9, -0.35, 0.2], [-0.15, 0.05, -0.6], [0.0, 0.0, 0.0]):
        u = np.asarray(u)
        s = fields.uniform_flow(n, u, times)
        F = oracle.Field(n, s.grids("f64"))
        seeds = rng.uniform(-0.5, 1.2, size=(400, 3)) * (np.asarray(n) - 1)
        r = oracle.flowmap(F, times, seeds, N)
        want = _margin_closed_form(n, u, times, seeds, N)
        np.testing.assert_allclose(r["margin"], want, rtol=0, atol=1e-12)
    # margins set by a stage point (the first half step crosses x = 13 by 0.001
    # while the step's start is 0.249 inside), by the first outside end point,
    # and by the high face of y
    u = np.array([1.0, 0.0, 0.0])
    times = np.array([0.0, 0.5, 1.0, 1.5])
    s = fields.uniform_flow(n, u, times)
    F = oracle.Field(n, s.grids("f64"))
    seeds = np.array([[12.751, 5.0, 4.0],   # y2 of step 0 = 13.001: outside by 0.001
                      [11.551, 5.0, 4.0],   # the end of step 2 = 13.051 is the first outside point;
                                            # the nearest inside point is y2 of that step, 12.801
                      [3.0, 9.9995, 4.0]])  # 0.0005 below the y = 10 face all along
    r = oracle.flowmap(F, times, seeds, 3)
    want = _margin_closed_form(n, u, times, seeds, 3)
    np.testing.assert_allclose(r["margin"], want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["margin"], [0.001, 0.051, 0.0005], rtol=0, atol=1e-12)
    assert r["flag"].tolist() == [oracle.TERMINATED, oracle.TERMINATED, oracle.VALID]
    assert r["exit"].tolist() == [0, 2, 3]


# ---------------------------------------------------------------------------
# FROZEN-mode adjoint against FP64 central finite differences.
# ---------------------------------------------------------------------------
def _setup():
    n = (24, 24, 24)
    N = 16
    s = fields.abc_noise(n, N + 1, 0.05, sigma=0.05, seed=18, global_n=64)
    gs = s.grids("f64")
    seeds = oracle.seed_lattice(n, 4)
    w = np.random.default_rng(13).standard_normal(seeds.shape)
    return n, N, s, gs, seeds, w


def _same_path(runs, base):
    return all(np.array_equal(r["sig"], base["sig"]) and np.array_equal(r["flag"], base["flag"])
               and np.array_equal(r["exit"], base["exit"]) for r in runs)


def test_frozen_mode_seed_gradient_matches_central_fd():
    n, N, s, gs, seeds, w = _setup()
    F = oracle.Field(n, gs)
    fz = oracle.FROZEN
    base = oracle.flowmap(F, s.times, seeds, N, mode=fz, jac=True)
    g = oracle.adjoint(F, s.times, seeds, N, w, mode=fz)
    valid = base["flag"] == 0
    assert valid.sum() > 50
    np.testing.assert_allclose(g[valid], np.einsum("pij,pi->pj", base["jac"], w)[valid], rtol=1e-12, atol=1e-12)
    assert np.all(g[~valid] == 0)
    fd = np.zeros((len(seeds), 3, 3))
    ok = np.ones(len(seeds), bool)
    for d in range(3):
        e = np.zeros(3)
        e[d] = H
        rp = oracle.flowmap(F, s.times, seeds + e, N, mode=fz)
        rm = oracle.flowmap(F, s.times, seeds - e, N, mode=fz)
        ok &= (rp["sig"] == rm["sig"]) & (rp["sig"] == base["sig"]) & (rp["flag"] == base["flag"]) & \
              (rm["flag"] == base["flag"]) & (rp["exit"] == base["exit"]) & (rm["exit"] == base["exit"])
        fd[:, :, d] = (rp["end"] - rm["end"]) / (2 * H)
    sel = ok & valid
    assert sel.sum() > 20
    g_fd = np.einsum("pij,pi->pj", fd[sel], w[sel])
    assert np.linalg.norm(g[sel] - g_fd) / np.linalg.norm(g_fd) < 1e-4
    assert np.linalg.norm(base["jac"][sel] - fd[sel]) / np.linalg.norm(fd[sel]) < 1e-4
    # the FROZEN map differs from the LINEAR one, so this is not the LINEAR gradient again
    g_lin = oracle.adjoint(F, s.times, seeds, N, w)
    assert np.abs(g_lin[sel] - g[sel]).max() > 1e-3 * np.abs(g[sel]).max()


def test_frozen_mode_grid_gradient_matches_central_fd():
    n, N, s, gs, seeds, w = _setup()
    seeds, w = seeds[::5], w[::5]
    F = oracle.Field(n, gs)
    fz = oracle.FROZEN
    g, gg = oracle.adjoint(F, s.times, seeds, N, w, mode=fz, grid_grad=True)
    base = oracle.flowmap(F, s.times, seeds, N, mode=fz)
    # no FROZEN step reads the last cycle's grid
    assert np.all(gg[N] == 0)
    G = np.stack(gg)
    rng = np.random.default_rng(14)
    nz_idx = [tuple(ix) for ix in np.argwhere(G != 0)]
    zero_idx = [tuple(ix) for ix in np.argwhere(G == 0)]
    assert len(nz_idx) > 100
    last = [(N, 12, 12, 12, 0), (N, 5, 7, 9, 2)]
    picks = [nz_idx[i] for i in rng.choice(len(nz_idx), 50, replace=False)] + \
            [zero_idx[i] for i in rng.choice(len(zero_idx), 15, replace=False)] + last
    checked = 0
    for (c, k, j, i, comp) in picks:
        vals, runs = [], []
        for sgn in (1, -1):
            gp = list(gs)
            gp[c] = gs[c].copy()
            gp[c][k, j, i, comp] += sgn * H
            r = oracle.flowmap(oracle.Field(n, gp), s.times, seeds, N, mode=fz)
            vals.append(((w * r["end"]).sum(1) * (r["flag"] == 0)).sum())
            runs.append(r)
        if not _same_path(runs, base):
            continue
        checked += 1
        fd = (vals[0] - vals[1]) / (2 * H)
        an = G[c, k, j, i, comp]
        if an == 0.0:
            assert abs(fd) < 1e-9, (c, k, j, i, comp, fd)
        else:
            assert abs(an - fd) <= 1e-4 * abs(fd) + 1e-9, (c, k, j, i, comp, an, fd)
    assert checked > 45
