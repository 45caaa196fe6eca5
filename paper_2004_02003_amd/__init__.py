"""Per-block Boundary Termination Optimization (BTO) on AMD MI355X (gfx950).

Seeds a lattice of basis-flow particles in one block of a time-varying
velocity field, advances them with one RK4 step per cycle through hand-written
HIP kernels, terminates those that reach the block boundary, and writes the
interval's flow map (Sane et al., arXiv:2004.02003, Section 3.1).

``Context`` wraps the C-ABI declared in ``include/bto.h``; the library must be
built (``paper_2004_02003_amd/build.py``) -- there is no fallback path.
"""

from ._lib import BTOError, LIB_PATH  # noqa: F401


def __getattr__(name):
    # torch-dependent parts load on first use
    if name in ("Context", "grid_to_device"):
        from . import context
        return getattr(context, name)
    if name == "InSituDriver":
        from . import insitu
        return insitu.InSituDriver
    if name in ("BTOAdvectFn", "advect_autograd", "jacobian_ftle"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
