"""The allocation-free accuracy metric through the C-ABI.

``bto_flowmap_error_static`` keeps its partial sums in a fixed device array
instead of allocating them.  On the same inputs it must return exactly what
``bto_flowmap_error`` returns (same kernels, same fixed reduction order), and
both must agree with the FP64 oracle of Eq. (5)/(6).  Two calls in a row, the
second on fewer entries than the first, check that the fixed array carries
nothing from one call into the next."""

import ctypes
import sys

import numpy as np
import pytest

from oracle import reconstruct as orc

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2004_02003_amd import _lib

    return _lib.load()


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    m_end = rng.normal(size=(n, 3)) * 20.0
    b_end = m_end + rng.normal(size=(n, 3)) * rng.choice([1e-3, 0.3, 4.0], size=(n, 1))
    m_flag = np.where(rng.random(n) < 0.2, 1, 0).astype(np.uint8)
    m_flag[rng.random(n) < 0.02] = 2
    b_state = rng.choice(np.array([0, 1, 2], dtype=np.uint8), size=n, p=[0.1, 0.7, 0.2])
    return b_end, b_state, m_end, m_flag


def _call(fn, n, dev, cell):
    import torch

    out = (ctypes.c_double * 5)()
    rc = fn(n, dev[0].data_ptr(), dev[1].data_ptr(), dev[2].data_ptr(), dev[3].data_ptr(), cell, out,
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, np.array(list(out))


@pytest.mark.parametrize("sizes", [(300_001, 4_097), (262_144, 1)])
def test_static_metric_equals_the_allocating_one(lib, sizes):
    import torch

    for k, n in enumerate(sizes):
        _say(f"flowmap_error_static n={n} (call {k + 1} of {len(sizes)})")
        host = _inputs(n, 17 + n)
        dev = [torch.as_tensor(np.ascontiguousarray(a), device="cuda") for a in host]
        rc_s, got = _call(lib.bto_flowmap_error_static, n, dev, 2.0)
        rc_a, ref = _call(lib.bto_flowmap_error, n, dev, 2.0)
        assert rc_s == 0 and rc_a == 0, (rc_s, rc_a)
        assert np.array_equal(got, ref), (got, ref)
        o = orc.flowmap_error(*host, cell=2.0)
        assert got[2] == o["n"] and got[3] == o["uncovered"]
        assert abs(got[1] - o["max_l2"]) <= 1e-12 * max(1.0, o["max_l2"])
        if o["n"]:
            assert abs(got[0] - o["mean_l2"]) <= 1e-12 * abs(o["mean_l2"])
            assert abs(got[4] - o["accuracy_pct"]) <= 1e-10 * max(1.0, abs(o["accuracy_pct"]))


def test_static_metric_rejects_bad_arguments(lib):
    from paper_2004_02003_amd import _lib

    out = (ctypes.c_double * 5)()
    assert lib.bto_flowmap_error_static(0, 1, 1, 1, 1, 1.0, out, None) == _lib.BTO_EINVAL
    assert lib.bto_flowmap_error_static(5, None, 1, 1, 1, 1.0, out, None) == _lib.BTO_EINVAL
    assert lib.bto_flowmap_error_static(5, 1, 1, 1, 1, 0.0, out, None) == _lib.BTO_EINVAL
