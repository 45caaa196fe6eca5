"""GPU adjoint (seed and grid gradients, Jacobian, FTLE) against the FP64
oracle: its discrete adjoint and tangent (same discrete derivative) and FP64
central finite differences of its forward map (h = 1e-3, entries whose +-h
runs change a flag, exit step or stage cell excluded)."""

import sys

import numpy as np
import pytest

import oracle
from bto_inputs import fields
from bto_inputs.workloads import WORKLOADS, loss_weights

pytestmark = pytest.mark.gpu
H = 1e-3


def _say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2004_02003_amd import _lib

    _lib.load()


def _dev(grids, dtype="f32"):
    from paper_2004_02003_amd import grid_to_device

    return [grid_to_device(g, dtype) for g in grids]


def _small():
    n = (24, 24, 24)
    N = 16
    s = fields.abc_noise(n, N + 1, 0.05, sigma=0.05, seed=8, global_n=64)
    gr = s.grids("f32")
    seeds = oracle.seed_lattice(n, 4)
    w = np.random.default_rng(3).standard_normal(seeds.shape)
    return n, N, s, gr, seeds, w


def _gpu_adjoint(n, gr, times, seeds, cot, ckpt, grid_grad=False, mode="linear"):
    import torch
    from paper_2004_02003_amd import Context

    dev = _dev(gr)
    with Context(n, len(seeds)) as ctx:
        ctx.seed_explicit(torch.as_tensor(seeds, dtype=torch.float64, device="cuda"))
        gg = [torch.zeros_like(g) for g in dev] if grid_grad else None
        status = torch.empty(len(seeds), dtype=torch.uint8, device="cuda")
        out = ctx.adjoint(dev, times, torch.as_tensor(cot, dtype=torch.float32, device="cuda").contiguous(),
                          grad_grids=gg, ckpt_every=ckpt, mode=mode, status=status)
        torch.cuda.synchronize()
        res = out.cpu().numpy(), status.cpu().numpy()
        if grid_grad:
            res = res + ([g.cpu().numpy() for g in gg],)
    return res


def test_seed_gradient_matches_oracle_adjoint_and_fd():
    n, N, s, gr, seeds, w = _small()
    _say("adjoint seed gradient 24^3, 16 steps")
    g, st = _gpu_adjoint(n, gr, s.times, seeds, w, ckpt=5)
    g = g[:, 0, :]
    F = oracle.Field(n, gr)
    base = oracle.flowmap(F, s.times, seeds, N)
    go = oracle.adjoint(F, s.times, seeds, N, w)
    ok = base["margin"] > 1e-6
    assert np.array_equal(st[ok], base["flag"][ok])
    valid = (base["flag"] == 0) & ok
    assert valid.sum() > 50
    err = np.linalg.norm(g[valid] - go[valid]) / np.linalg.norm(go[valid])
    assert err < 1e-5, err
    assert np.all(g[base["flag"] == 1] == 0)
    # against central FD of the FP64 forward
    fd = np.zeros_like(go)
    same = np.ones(len(seeds), bool)
    for d in range(3):
        e = np.zeros(3)
        e[d] = H
        rp = oracle.flowmap(F, s.times, seeds + e, N)
        rm = oracle.flowmap(F, s.times, seeds - e, N)
        same &= (rp["sig"] == base["sig"]) & (rm["sig"] == base["sig"]) & (rp["flag"] == 0) & (rm["flag"] == 0)
        fd[:, d] = ((w * rp["end"]).sum(1) - (w * rm["end"]).sum(1)) / (2 * H)
    sel = valid & same
    assert sel.sum() > 20
    rel = np.linalg.norm(g[sel] - fd[sel]) / np.linalg.norm(fd[sel])
    assert rel < 1e-4, rel


def test_checkpoint_interval_does_not_change_the_gradient():
    n, N, s, gr, seeds, w = _small()
    outs = []
    for k in (1, 3, 7, 16, 100):
        _say(f"adjoint ckpt_every={k}")
        outs.append(_gpu_adjoint(n, gr, s.times, seeds, w, ckpt=k)[0])
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_jacobian_matches_oracle_tangent_and_ftle():
    import torch
    from paper_2004_02003_amd import Context, jacobian_ftle

    n, N, s, gr, seeds, w = _small()
    _say("jacobian + ftle")
    dev = _dev(gr)
    with Context(n, len(seeds)) as ctx:
        J, sig, st = jacobian_ftle(ctx, torch.as_tensor(seeds, device="cuda"), dev, s.times, ckpt_every=4)
        torch.cuda.synchronize()
        J, sig, st = J.cpu().numpy(), sig.cpu().numpy(), st.cpu().numpy()
    o = oracle.flowmap(oracle.Field(n, gr), s.times, seeds, N, jac=True)
    valid = (o["flag"] == 0) & (o["margin"] > 1e-6)
    err = np.linalg.norm(J[valid] - o["jac"][valid]) / np.linalg.norm(o["jac"][valid])
    assert err < 1e-5, err
    T = s.times[N] - s.times[0]
    np.testing.assert_allclose(sig[valid], oracle.ftle(o["jac"][valid], T), rtol=1e-4, atol=1e-5)
    assert np.all(J[st != 0] == 0)


def test_grid_gradient_matches_oracle_dense_gradient():
    n, N, s, gr, seeds, w = _small()
    seeds, w = seeds[::3], w[::3]
    _say("adjoint grid gradient 24^3")
    g, st, gg = _gpu_adjoint(n, gr, s.times, seeds, w, ckpt=4, grid_grad=True)
    F = oracle.Field(n, gr)
    go, ggo = oracle.adjoint(F, s.times, seeds, N, w, grid_grad=True)
    base = oracle.flowmap(F, s.times, seeds, N)
    assert np.all(base["margin"] > 1e-6), "choose a case without face ties"
    A = np.stack(gg).astype(np.float64)
    B = np.stack(ggo)
    # entries no trajectory touches are exactly zero on both sides
    assert np.all(A[B == 0] == 0)
    err = np.linalg.norm(A - B) / np.linalg.norm(B)
    assert err < 1e-5, err


def test_frozen_mode_adjoint_matches_oracle():
    n, N, s, gr, seeds, w = _small()
    _say("adjoint frozen mode")
    g, st, gg = _gpu_adjoint(n, gr, s.times, seeds[::4], w[::4], ckpt=6, grid_grad=True, mode="frozen")
    F = oracle.Field(n, gr)
    go, ggo = oracle.adjoint(F, s.times, seeds[::4], N, w[::4], mode=oracle.FROZEN, grid_grad=True)
    base = oracle.flowmap(F, s.times, seeds[::4], N, mode=oracle.FROZEN)
    valid = (base["flag"] == 0) & (base["margin"] > 1e-6)
    err = np.linalg.norm(g[valid, 0] - go[valid]) / np.linalg.norm(go[valid])
    assert err < 1e-5, err
    errg = np.linalg.norm(np.stack(gg) - np.stack(ggo)) / np.linalg.norm(np.stack(ggo))
    assert errg < 1e-5, errg


def test_autograd_function_seed_and_grid_gradients():
    import torch
    from paper_2004_02003_amd import Context, advect_autograd

    n, N, s, gr, seeds, w = _small()
    _say("autograd")
    dev = [g.requires_grad_(True) for g in _dev(gr)]
    x0 = torch.as_tensor(seeds, device="cuda").requires_grad_(True)
    wt = torch.as_tensor(w, device="cuda")
    with Context(n, len(seeds)) as ctx:
        end, flag, ex = advect_autograd(ctx, x0, dev, s.times, ckpt_every=5)
        loss = (wt * end * (flag == 0).unsqueeze(1)).sum()
        loss.backward()
        torch.cuda.synchronize()
    F = oracle.Field(n, gr)
    go, ggo = oracle.adjoint(F, s.times, seeds, N, w, grid_grad=True)
    base = oracle.flowmap(F, s.times, seeds, N)
    valid = (base["flag"] == 0) & (base["margin"] > 1e-6)
    gx = x0.grad.cpu().numpy()
    assert np.linalg.norm(gx[valid] - go[valid]) / np.linalg.norm(go[valid]) < 1e-5
    A = np.stack([g.grad.cpu().numpy() for g in dev])
    assert np.linalg.norm(A - np.stack(ggo)) / np.linalg.norm(np.stack(ggo)) < 1e-4
    np.testing.assert_allclose(end.detach().cpu().numpy()[valid], base["end"][valid], atol=1e-5)


def test_abc_128_adjoint_workload_full_size():
    """The differentiation workload at full size: 32^3 seeds (stride 4) on the
    128^3 ABC field, 100 steps, checkpoints every 10; seed gradient of the
    seeded-weight loss on every seed against the oracle adjoint, plus the
    Jacobian on a subset against the oracle tangent."""
    import torch
    from paper_2004_02003_amd import Context, jacobian_ftle

    wl = WORKLOADS["abc_128_adjoint"]
    _say(f"{wl.name} full size")
    s = wl.make_field()
    gr = s.grids("f32")
    seeds = oracle.seed_lattice(wl.n, wl.stride)
    w = loss_weights(len(seeds), wl.extra["weight_seed"])
    dev = _dev(gr)
    with Context(wl.n, len(seeds)) as ctx:
        ctx.seed(wl.stride)
        cot = torch.as_tensor(w, dtype=torch.float32, device="cuda").contiguous()
        status = torch.empty(len(seeds), dtype=torch.uint8, device="cuda")
        g = ctx.adjoint(dev, s.times, cot, ckpt_every=wl.extra["ckpt_every"], status=status)
        sub = torch.as_tensor(seeds[::37], device="cuda")
        J, sig, stJ = jacobian_ftle(ctx, sub, dev, s.times, ckpt_every=wl.extra["ckpt_every"])
        torch.cuda.synchronize()
        g = g.cpu().numpy()[:, 0, :]
        st = status.cpu().numpy()
        J = J.cpu().numpy()
    F = oracle.Field(wl.n, gr)
    base = oracle.flowmap(F, s.times, seeds, wl.n_steps)
    go = oracle.adjoint(F, s.times, seeds, wl.n_steps, w)
    ok = base["margin"] > 1e-6
    assert np.array_equal(st[ok], base["flag"][ok])
    valid = (base["flag"] == 0) & ok
    err = np.linalg.norm(g[valid] - go[valid]) / np.linalg.norm(go[valid])
    _say(f"seed-gradient rel err {err:.2e} over {valid.sum()} seeds")
    assert err < 1e-5, err
    oj = oracle.flowmap(F, s.times, seeds[::37], wl.n_steps, jac=True)
    vj = (oj["flag"] == 0) & (oj["margin"] > 1e-6)
    errj = np.linalg.norm(J[vj] - oj["jac"][vj]) / np.linalg.norm(oj["jac"][vj])
    assert errj < 1e-5, errj


@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_adjoint_on_16bit_grids_matches_oracle(dt):
    """The adjoint reads 16-bit grids like the forward (converted exactly to
    FP32); the oracle runs on the same stored values."""
    import torch
    from paper_2004_02003_amd import Context

    n = (20, 18, 22)
    N = 12
    s = fields.abc_noise(n, N + 1, 0.05, sigma=0.05, seed=13, global_n=48)
    gr = s.grids(dt)
    seeds = oracle.seed_lattice(n, 3)
    w = np.random.default_rng(6).standard_normal(seeds.shape)
    _say(f"adjoint on {dt} grids")
    dev = _dev(gr, dt)
    with Context(n, len(seeds)) as ctx:
        ctx.seed_explicit(torch.as_tensor(seeds, device="cuda"))
        g = ctx.adjoint(dev, s.times, torch.as_tensor(w, dtype=torch.float32, device="cuda").contiguous(),
                        ckpt_every=5)
        torch.cuda.synchronize()
        g = g.cpu().numpy()[:, 0, :]
    F = oracle.Field(n, gr, dtype=dt)
    go = oracle.adjoint(F, s.times, seeds, N, w)
    base = oracle.flowmap(F, s.times, seeds, N)
    valid = (base["flag"] == 0) & (base["margin"] > 1e-6)
    assert valid.sum() > 20
    err = np.linalg.norm(g[valid] - go[valid]) / np.linalg.norm(go[valid])
    assert err < 1e-5, err


def test_jacobian_and_ftle_of_hyperbolic_strain_closed_form():
    """Steady strain u = (a (x - c), -a (y - c), 0): the flow-map Jacobian of
    RK4 is diag(R(a h)^N, R(-a h)^N, 1), R the RK4 amplification factor, and
    the FTLE is ln R(a h) / h for every seed (independent of the oracle)."""
    import torch
    from paper_2004_02003_amd import Context, jacobian_ftle

    n = (33, 33, 9)
    c, a, h, N = 16.0, 0.2, 0.1, 25
    times = np.arange(N + 1) * h
    z_, y_, x_ = np.meshgrid(np.arange(n[2], dtype=float), np.arange(n[1], dtype=float),
                             np.arange(n[0], dtype=float), indexing="ij")
    g = np.stack([a * (x_ - c), -a * (y_ - c), np.zeros_like(x_)], axis=-1).astype(np.float32)
    rng = np.random.default_rng(5)
    seeds = np.stack([c + rng.uniform(-5, 5, 200), c + rng.uniform(-10, 10, 200), rng.uniform(1, 7, 200)], axis=1)
    _say("jacobian of hyperbolic strain")
    dev = _dev([g] * (N + 1))
    with Context(n, len(seeds)) as ctx:
        J, sig, st = jacobian_ftle(ctx, torch.as_tensor(seeds, device="cuda"), dev, times, ckpt_every=10)
        torch.cuda.synchronize()
        J, sig, st = J.cpu().numpy(), sig.cpu().numpy(), st.cpu().numpy()

    def R(z):
        return 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24

    assert np.all(st == 0)
    Jw = np.diag([R(a * h) ** N, R(-a * h) ** N, 1.0])
    assert np.abs(J - Jw).max() < 1e-5
    np.testing.assert_allclose(sig, np.log(R(a * h)) / h, rtol=1e-5)


@pytest.mark.parametrize("shape", [{}, {"rebin_every": 3, "lanes_per_particle": 2, "steps_per_launch": 4}])
def test_recorded_checkpoints_give_the_recomputed_gradients(shape):
    """Checkpoints recorded by the advection (two streaming calls, launches cut
    at every 5th step; also with re-sorting every 3 steps, two lanes per
    particle and 4-step launches) give the same seed and grid gradients and
    flags as the adjoint's own recomputed forward; mismatched or incomplete
    records are refused."""
    import torch
    from paper_2004_02003_amd import BTOError, Context

    n, N, s, gr, seeds, w = _small()
    dev = _dev(gr)
    cot = torch.as_tensor(w, dtype=torch.float32, device="cuda").contiguous()
    o = oracle.flowmap(oracle.Field(n, gr), s.times, seeds, N)
    safe = o["margin"] > 1e-6
    _say(f"recorded checkpoints {shape}")
    with Context(n, len(seeds)) as ctx:
        ctx.set_tuning(ckpt_every=5, **shape)
        x0 = torch.as_tensor(seeds, dtype=torch.float64, device="cuda")
        ctx.seed_explicit(x0)
        ctx.advect(dev[:10], s.times[:10], record_ckpt=True)
        ctx.advect(dev[9:], s.times[9:], record_ckpt=True)
        fm = ctx.flowmap()
        st_r = torch.empty(len(seeds), dtype=torch.uint8, device="cuda")
        gg_r = [torch.zeros_like(g) for g in dev]
        g_r = ctx.adjoint(dev, s.times, cot, grad_grids=gg_r, ckpt_every=5, status=st_r, recorded=True)
        torch.cuda.synchronize()
        # a seed whose recomputation leaves the block though the advection
        # (rounding otherwise) kept it is dropped; only valid seeds can be
        srr, fmf = st_r.cpu().numpy(), fm["flag"].cpu().numpy()
        dropped = srr >= oracle.VALID + 3
        assert np.all(fmf[dropped] == 0) and dropped.mean() < 0.01
        assert np.array_equal(srr[~dropped], fmf[~dropped])
        with pytest.raises(BTOError):
            ctx.adjoint(dev, s.times, cot, ckpt_every=4, recorded=True)      # other spacing
        with pytest.raises(BTOError):
            ctx.adjoint(dev[:10], s.times[:10], cot, ckpt_every=5, recorded=True)  # other length
        # the adjoint's own forward from the seeds
        ctx.seed_explicit(x0)
        st_c = torch.empty(len(seeds), dtype=torch.uint8, device="cuda")
        gg_c = [torch.zeros_like(g) for g in dev]
        g_c = ctx.adjoint(dev, s.times, cot, grad_grids=gg_c, ckpt_every=5, status=st_c)
        torch.cuda.synchronize()
        with pytest.raises(BTOError):   # reseeded, nothing recorded since
            ctx.adjoint(dev, s.times, cot, ckpt_every=5, recorded=True)
        ctx.advect(dev, s.times)
        with pytest.raises(BTOError):   # advected without recording
            ctx.adjoint(dev, s.times, cot, ckpt_every=5, recorded=True)
        ctx.seed_explicit(x0)
        ctx.advect(dev[:10], s.times[:10], record_ckpt=True)
        ctx.set_tuning(ckpt_every=4)
        ctx.advect(dev[9:], s.times[9:], record_ckpt=True)
        with pytest.raises(BTOError):   # two spacings in one interval
            ctx.adjoint(dev, s.times, cot, ckpt_every=5, recorded=True)
    sr, sc = st_r.cpu().numpy(), st_c.cpu().numpy()
    keep = safe & (sr < 3)
    assert np.array_equal(sr[keep], sc[keep])
    ok = keep & (sr == 0)
    assert ok.sum() > 20
    a, b = g_r.cpu().numpy().reshape(-1, 3)[ok], g_c.cpu().numpy().reshape(-1, 3)[ok]
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-5
    if np.array_equal(sr, sc):  # grid gradients sum over every seed that stayed inside
        ga = np.concatenate([g.cpu().numpy().ravel() for g in gg_r])
        gb = np.concatenate([g.cpu().numpy().ravel() for g in gg_c])
        assert np.linalg.norm(ga - gb) / np.linalg.norm(gb) < 1e-5


def test_grid_gradient_is_deterministic_and_matches_the_atomic_path(monkeypatch):
    """The sorted reduction of the grid-gradient records gives bit-identical
    grids on repeated calls, and the same values as adding every flush with
    FP32 atomics (BTO_GRAD_ATOMICS=1) up to FP32 summation order."""
    n, N, s, gr, seeds, w = _small()
    _say("grid gradient: sorted reduction twice, then atomics")
    _, st1, g1 = _gpu_adjoint(n, gr, s.times, seeds, w, ckpt=4, grid_grad=True)
    _, st2, g2 = _gpu_adjoint(n, gr, s.times, seeds, w, ckpt=4, grid_grad=True)
    for a, b in zip(g1, g2):
        assert np.array_equal(a, b)
    monkeypatch.setenv("BTO_GRAD_ATOMICS", "1")
    _, st3, g3 = _gpu_adjoint(n, gr, s.times, seeds, w, ckpt=4, grid_grad=True)
    assert np.array_equal(st1, st3)
    ga = np.concatenate([g.ravel() for g in g1])
    gb = np.concatenate([g.ravel() for g in g3])
    assert np.abs(ga).max() > 0
    assert np.abs(ga - gb).max() <= 1e-6 * np.abs(gb).max()


def test_grid_gradient_when_records_overflow_into_atomics(monkeypatch):
    """A fast turbulent block (about 1.5 cells per step): most stages change
    cell, so a seed flushes more often than its 2 (N + 1) + 2 record slots and
    the rest of its flushes go to the grids with atomics.  The mixed result
    equals the all-atomic path to FP32 summation order and the oracle's dense
    gradient to the FP32 sampling error."""
    from bto_inputs import fields as F_

    n, N = 32, 20
    s = F_.turbulence(n, 16, 7, N + 1, 0.02, L=64, cfl=1.5)
    gr = s.grids("f32")
    seeds = oracle.seed_lattice((n, n, n), 4)
    w = np.random.default_rng(9).standard_normal(seeds.shape)
    _say("grid gradient, turbulent block, record overflow")
    _, st1, g1 = _gpu_adjoint((n, n, n), gr, s.times, seeds, w, ckpt=5, grid_grad=True)
    monkeypatch.setenv("BTO_GRAD_ATOMICS", "1")
    _, st2, g2 = _gpu_adjoint((n, n, n), gr, s.times, seeds, w, ckpt=5, grid_grad=True)
    assert np.array_equal(st1, st2)
    assert (st1 == 0).sum() > 50
    A = np.concatenate([g.ravel() for g in g1]).astype(np.float64)
    B = np.concatenate([g.ravel() for g in g2]).astype(np.float64)
    assert np.abs(A - B).max() <= 1e-5 * np.abs(B).max()
    go, ggo = oracle.adjoint(oracle.Field((n, n, n), gr), s.times, seeds, N, w, grid_grad=True)
    C = np.concatenate([g.ravel() for g in ggo])
    assert np.linalg.norm(A - C) / np.linalg.norm(C) < 1e-3


def test_grid_gradient_with_one_buffer_for_every_grid():
    """When every grid's gradient is the same buffer the library uses the
    atomic path, and the buffer receives the sum over all levels."""
    import torch
    from paper_2004_02003_amd import Context

    n, N, s, gr, seeds, w = _small()
    dev = _dev(gr)
    cot = torch.as_tensor(w, dtype=torch.float32, device="cuda").contiguous()
    _say("grid gradient into one shared buffer")
    with Context(n, len(seeds)) as ctx:
        x0 = torch.as_tensor(seeds, dtype=torch.float64, device="cuda")
        ctx.seed_explicit(x0)
        gg = [torch.zeros_like(g) for g in dev]
        ctx.adjoint(dev, s.times, cot, grad_grids=gg, ckpt_every=4)
        ctx.seed_explicit(x0)
        one = torch.zeros_like(dev[0])
        ctx.adjoint(dev, s.times, cot, grad_grids=[one] * len(dev), ckpt_every=4)
        torch.cuda.synchronize()
        total = torch.stack(gg).sum(0).cpu().numpy()
        got = one.cpu().numpy()
    assert np.abs(got - total).max() <= 1e-5 * np.abs(total).max()


def _recorded(ctx, dev, times, seeds, k):
    import torch

    ctx.set_tuning(ckpt_every=k)
    ctx.seed_explicit(torch.as_tensor(seeds, dtype=torch.float64, device="cuda"))
    ctx.advect(dev, times, record_ckpt=True)


@pytest.mark.parametrize("ncot", [1, 3])
def test_segment_by_segment_adjoint_equals_the_whole_interval(ncot):
    """The adjoint swept one checkpoint segment per call, each call given only
    its segment's grids (with a short last segment), gives the seed gradients
    of the whole-interval adjoint from the same recorded checkpoints bit for
    bit, its flags, and its grid gradients up to the order in which two
    segments' sums meet on their shared grid; calls out of order are refused."""
    import torch
    from paper_2004_02003_amd import BTOError, Context

    n, N, s, gr, seeds, w = _small()
    k = 5  # 16 steps: segments of 5, 5, 5, 1
    dev = _dev(gr)
    P = len(seeds)
    if ncot == 3:
        cot = torch.eye(3, dtype=torch.float32, device="cuda").expand(P, 3, 3).contiguous()
    else:
        cot = torch.as_tensor(w, dtype=torch.float32, device="cuda").contiguous().view(P, 1, 3)
    _say(f"segment adjoint, n_cot {ncot}")
    with Context(n, P) as ctx:
        _recorded(ctx, dev, s.times, seeds, k)
        st_w = torch.empty(P, dtype=torch.uint8, device="cuda")
        gg_w = [torch.zeros_like(g) for g in dev] if ncot == 1 else None
        g_w = ctx.adjoint(dev, s.times, cot, grad_grids=gg_w, ckpt_every=k, status=st_w, recorded=True)
        nseg = (N + k - 1) // k
        gg_s = [torch.zeros_like(g) for g in dev] if ncot == 1 else None
        g_s = torch.empty((P, ncot, 3), dtype=torch.float32, device="cuda")
        st_s = torch.empty(P, dtype=torch.uint8, device="cuda")
        with pytest.raises(BTOError):  # must start at the last segment
            ctx.adjoint_segment(nseg - 2, dev[(nseg - 2) * k:(nseg - 1) * k + 1], s.times[(nseg - 2) * k:(nseg - 1) * k + 1],
                                n_cot=ncot)
        for sg in range(nseg - 1, -1, -1):
            a, b = sg * k, min(sg * k + k, N)
            seg = [g.clone() for g in dev[a:b + 1]]  # only this segment's grids (copies)
            ctx.adjoint_segment(sg, seg, s.times[a:b + 1], cot=cot if sg == nseg - 1 else None, n_cot=ncot,
                                grad_seed=g_s if sg == 0 else None,
                                grad_grids=gg_s[a:b + 1] if gg_s is not None else None,
                                status=st_s if sg == 0 else None)
            del seg
        with pytest.raises(BTOError):  # the sequence has ended
            ctx.adjoint_segment(0, dev[:k + 1], s.times[:k + 1], n_cot=ncot, grad_seed=g_s)
        torch.cuda.synchronize()
    assert np.array_equal(st_s.cpu().numpy(), st_w.cpu().numpy())
    assert np.array_equal(g_s.cpu().numpy(), g_w.cpu().numpy())
    if ncot == 1:
        ga = np.concatenate([g.cpu().numpy().ravel() for g in gg_s])
        gb = np.concatenate([g.cpu().numpy().ravel() for g in gg_w])
        assert np.linalg.norm(ga - gb) / np.linalg.norm(gb) < 1e-6
        assert np.array_equal(ga == 0, gb == 0)


def test_adjoint_drops_seeds_whose_recomputation_contradicts_the_recorded_forward():
    """Checkpoints recorded on a slow uniform flow, the adjoint called on a
    fast one (a stand-in for a forward rounded otherwise): a seed whose
    recomputed steps leave the block is dropped (status BTO_ADJ_DROPPED, zero
    gradient rows, its grid records withdrawn even when the contradiction
    shows up only in an earlier segment, after a later one contributed),
    the others keep the closed-form gradients of uniform flow (dx_end/dx_0 = I;
    the grid gradient sums to the kept cotangents times the interval)."""
    import torch
    from paper_2004_02003_amd import Context, _lib

    n = (20, 20, 20)
    N, k, h = 4, 2, 0.5
    times = np.arange(N + 1) * h
    slow = fields.uniform_flow(n, np.array([-1.0, 0.0, 0.0]), times)
    fast = fields.uniform_flow(n, np.array([2.0, 0.0, 0.0]), times)
    # x0 = 17.25: the recorded checkpoints are 17.25 (step 0) and 16.25 (step 2);
    # from 16.25 two fast steps reach 18.25 (inside), from 17.25 they reach 19.25
    seeds = np.array([[5.0, 10.0, 10.0], [17.25, 10.3, 9.7], [17.25, 3.3, 12.1], [8.5, 4.5, 15.5],
                      [17.6, 7.0, 7.0], [2.0, 2.0, 2.0]])
    w = np.random.default_rng(11).standard_normal(seeds.shape)
    dslow, dfast = _dev(slow.grids("f32")), _dev(fast.grids("f32"))
    _say("adjoint drops contradicted seeds")
    with Context(n, len(seeds)) as ctx:
        _recorded(ctx, dslow, times, seeds, k)
        st = torch.empty(len(seeds), dtype=torch.uint8, device="cuda")
        gg = [torch.zeros_like(g) for g in dfast]
        g = ctx.adjoint(dfast, times, torch.as_tensor(w, dtype=torch.float32, device="cuda").contiguous(),
                        grad_grids=gg, ckpt_every=k, status=st, recorded=True)
        torch.cuda.synchronize()
        st, g = st.cpu().numpy(), g.cpu().numpy().reshape(-1, 3)
        gsum = sum(x.cpu().numpy().reshape(-1, 3).sum(axis=0) for x in gg)
    want_drop = np.array([False, True, True, False, True, False])
    assert np.array_equal(st == _lib.BTO_ADJ_DROPPED, want_drop), st
    assert np.all(st[~want_drop] == 0)
    assert np.all(g[want_drop] == 0)
    np.testing.assert_allclose(g[~want_drop], w[~want_drop], rtol=0, atol=1e-6)
    np.testing.assert_allclose(gsum, w[~want_drop].sum(axis=0) * (times[-1] - times[0]), rtol=1e-5, atol=1e-5)
