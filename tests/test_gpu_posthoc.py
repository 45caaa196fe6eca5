"""Post hoc side on the GPU through the C-ABI: lattice placement, the Eq. (1)
rebuild of terminated entries and the Eq. (5)/(6) accuracy metric against the
FP64 oracle (``oracle/reconstruct.py``), and the multi-block BTO accuracy
experiment (blocks advected independently vs the whole domain) end to end.

The rebuild is bit-exact: both sides evaluate Eq. (1) as written in FP64 (two
products, one sum, no contraction) from the same inputs.  The metric's sum is
reduced in a different order, so it agrees to a relative 1e-12."""

import sys

import numpy as np
import pytest

import oracle
from oracle import reconstruct as orc
from bto_inputs import fields

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2004_02003_amd import _lib

    _lib.load()


def _t(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("m", [(13, 7, 5), (1, 9, 4), (2, 2, 2), (40, 33, 17), (1, 1, 1), (200, 3, 2),
                               (3, 130, 2), (2, 3, 1024), (64, 64, 65)])
def test_reconstruct_bit_exact_against_oracle(m):
    from paper_2004_02003_amd import posthoc

    rng = np.random.default_rng(sum(m))
    P = int(np.prod(m))
    end = rng.normal(size=(P, 3)) * 10
    flag = np.where(rng.random(P) < 0.45, 1, 0).astype(np.uint8)
    flag[rng.random(P) < 0.05] = 2
    _say(f"reconstruct {m}")
    g_end = _t(end)
    st = posthoc.reconstruct_lattice(g_end, _t(flag), m)
    o_end, o_st = orc.reconstruct(end, flag == 0, m)
    assert np.array_equal(st.cpu().numpy(), o_st)
    assert np.array_equal(g_end.cpu().numpy(), o_end, equal_nan=True)


def test_reconstruct_edge_cases():
    from paper_2004_02003_amd import posthoc

    m = (6, 5, 4)
    P = int(np.prod(m))
    rng = np.random.default_rng(1)
    end = rng.normal(size=(P, 3))
    for name, flag in (("all valid", np.zeros(P, np.uint8)), ("none valid", np.ones(P, np.uint8)),
                       ("one valid", np.r_[np.zeros(1, np.uint8), np.ones(P - 1, np.uint8)])):
        _say(f"reconstruct edge: {name}")
        g = _t(end)
        st = posthoc.reconstruct_lattice(g, _t(flag), m).cpu().numpy()
        o_end, o_st = orc.reconstruct(end, flag == 0, m)
        assert np.array_equal(st, o_st), name
        assert np.array_equal(g.cpu().numpy(), o_end, equal_nan=True), name


def test_flowmap_error_against_oracle():
    from paper_2004_02003_amd import posthoc

    rng = np.random.default_rng(4)
    P = 100_003
    b = rng.normal(size=(P, 3))
    m = b + rng.normal(size=(P, 3)) * 0.01
    bs = rng.choice([0, 1, 2], size=P, p=[0.1, 0.6, 0.3]).astype(np.uint8)
    b[bs == 0] = np.nan
    mf = rng.choice([0, 1], size=P, p=[0.9, 0.1]).astype(np.uint8)
    _say("flowmap error 100003")
    r = posthoc.flowmap_error(_t(b), _t(bs), _t(m), _t(mf), cell=0.5)
    o = orc.flowmap_error(b, bs, m, mf, cell=0.5)
    assert r["n"] == o["n"] and r["uncovered"] == o["uncovered"]
    assert r["mean_l2"] == pytest.approx(o["mean_l2"], rel=1e-12)
    assert r["max_l2"] == pytest.approx(o["max_l2"], rel=1e-14)
    assert r["accuracy_pct"] == pytest.approx(o["accuracy_pct"], rel=1e-12)


def test_place_block_bit_exact():
    import torch
    from paper_2004_02003_amd import posthoc

    rng = np.random.default_rng(6)
    M = (10, 8, 6)
    dst = torch.full((int(np.prod(M)), 3), -1.0, dtype=torch.float64, device="cuda")
    dflag = torch.full((int(np.prod(M)),), 7, dtype=torch.uint8, device="cuda")
    ref = np.full((M[2], M[1], M[0], 3), -1.0)
    rflag = np.full((M[2], M[1], M[0]), 7, np.uint8)
    for mb, off, sh in (((5, 4, 3), (0, 0, 0), (0.0, 0.0, 0.0)), ((5, 4, 3), (5, 4, 3), (24.0, 16.5, -3.25)),
                        ((3, 2, 1), (7, 6, 5), (1e-3, 2.0, 3.0))):
        src = rng.normal(size=(int(np.prod(mb)), 3))
        sflag = rng.integers(0, 3, int(np.prod(mb))).astype(np.uint8)
        posthoc.place_block(_t(src), _t(sflag), mb, dst, dflag, M, off, shift=sh)
        ref[off[2]:off[2] + mb[2], off[1]:off[1] + mb[1], off[0]:off[0] + mb[0]] = \
            src.reshape(mb[2], mb[1], mb[0], 3) + np.array(sh)
        rflag[off[2]:off[2] + mb[2], off[1]:off[1] + mb[1], off[0]:off[0] + mb[0]] = sflag.reshape(mb[2], mb[1], mb[0])
    assert np.array_equal(dst.cpu().numpy(), ref.reshape(-1, 3))
    assert np.array_equal(dflag.cpu().numpy(), rflag.reshape(-1))
    from paper_2004_02003_amd import BTOError
    with pytest.raises(BTOError):
        posthoc.place_block(_t(src), _t(sflag), (3, 2, 1), dst, dflag, M, (8, 6, 5))  # does not fit
    with pytest.raises(BTOError):
        big = torch.zeros((1025 * 2, 3), dtype=torch.float64, device="cuda")
        posthoc.reconstruct_lattice(big, torch.zeros(2050, dtype=torch.uint8, device="cuda"), (1025, 2, 1))


def test_multiblock_bto_accuracy_end_to_end():
    """A 48^3-cell ABC domain cut into 2 x 2 x 2 blocks, seeds at 1:8, 20
    steps.  Each block's BTO flow map matches the oracle run on that block;
    the domain run matches the oracle on the domain; the rebuild and the
    accuracy metric match the oracle on the GPU's flow maps."""
    from paper_2004_02003_amd import grid_to_device, posthoc

    n, N, stride, blocks = 49, 20, 2, (2, 2, 2)
    s = fields.abc_noise(n, N + 1, 0.05, sigma=0.01, seed=5, global_n=48)
    gr = s.grids("f32")
    dev = [grid_to_device(g, "f32") for g in gr]
    _say("multi-block BTO 2x2x2 of 24^3 cells")
    b_end, b_flag, M = posthoc.run_blocks(dev, s.times, blocks, stride)
    m_end, m_flag, M2 = posthoc.run_domain(dev, s.times, stride)
    assert tuple(M) == tuple(M2) == (24, 24, 24)
    bE, bF = b_end.cpu().numpy(), b_flag.cpu().numpy()
    mE, mF = m_end.cpu().numpy(), m_flag.cpu().numpy()

    # oracle: each block on its own (BTO), and the domain as one block
    cells = 24
    mb = 12
    o_end = np.full((M[2], M[1], M[0], 3), np.nan)
    o_flag = np.zeros((M[2], M[1], M[0]), np.uint8)
    o_margin = np.zeros((M[2], M[1], M[0]))
    for bz in range(2):
        for by in range(2):
            for bx in range(2):
                o = (bx * cells, by * cells, bz * cells)
                sub = [g[o[2]:o[2] + cells + 1, o[1]:o[1] + cells + 1, o[0]:o[0] + cells + 1] for g in gr]
                r = oracle.flowmap(oracle.Field((cells + 1,) * 3, sub), s.times,
                                   oracle.seed_lattice((cells + 1,) * 3, stride), N)
                sl = (slice(bz * mb, bz * mb + mb), slice(by * mb, by * mb + mb), slice(bx * mb, bx * mb + mb))
                o_end[sl] = (r["end"] + np.array(o)).reshape(mb, mb, mb, 3)
                o_flag[sl] = r["flag"].reshape(mb, mb, mb)
                o_margin[sl] = r["margin"].reshape(mb, mb, mb)
    o_end, o_flag, o_margin = o_end.reshape(-1, 3), o_flag.reshape(-1), o_margin.reshape(-1)
    safe = o_margin >= 1e-6
    assert np.array_equal(bF[safe], o_flag[safe])
    ok = safe & (o_flag == 0)
    assert np.abs(bE[ok] - o_end[ok]).max() < 1e-5
    od = oracle.flowmap(oracle.Field((n, n, n), gr), s.times, oracle.seed_lattice((n, n, n), stride), N)
    dsafe = od["margin"] >= 1e-6
    assert np.array_equal(mF[dsafe], od["flag"][dsafe])
    dok = dsafe & (od["flag"] == 0)
    assert np.abs(mE[dok] - od["end"][dok]).max() < 1e-5

    frac_term = float((bF != 0).mean())
    assert 0.05 < frac_term < 0.6  # block boundaries cut many trajectories

    # rebuild (bit-exact vs the oracle on the same input) and metric
    st = posthoc.reconstruct_lattice(b_end, b_flag, M)
    o_rec, o_st = orc.reconstruct(bE, bF == 0, M)
    assert np.array_equal(st.cpu().numpy(), o_st)
    assert np.array_equal(b_end.cpu().numpy(), o_rec, equal_nan=True)
    acc = posthoc.flowmap_error(b_end, st, m_end, m_flag, cell=1.0)
    oacc = orc.flowmap_error(o_rec, o_st, mE, mF, cell=1.0)
    assert acc["n"] == oacc["n"] and acc["uncovered"] == oacc["uncovered"]
    assert acc["mean_l2"] == pytest.approx(oacc["mean_l2"], rel=1e-12)
    _say(f"terminated {frac_term:.3f}, rebuilt {(o_st == 2).mean():.3f}, accuracy {acc}")
    # valid BTO particles follow the communicating ones to FP32 sampling error
    known = (o_st == 1) & (mF == 0)
    assert np.abs(o_rec[known] - mE[known]).max() < 1e-4
    assert acc["accuracy_pct"] > 90.0
