"""Helpers shared by the GPU parity tests: run the HIP path through the C-ABI
and the oracle on the same seeded inputs, and compare them."""

from __future__ import annotations

import numpy as np

import oracle

# Tolerances (cells): termination flags and exit steps must match exactly for
# every particle whose oracle decision points all stay at least MARGIN from a
# face; end positions within POS_TOL for FP32 arithmetic on the stored grid.
MARGIN = 1e-6
POS_TOL = 1e-5


def run_gpu(n, grids_dev, times, stride=None, seeds=None, mode="linear", chunks=None, origin=(0, 0, 0),
            spacing=(1, 1, 1), cap=None, tuning=None, record_exit=False):
    """Seed, advect (optionally in several calls), write the flow map (and
    with ``record_exit`` the exit points); returns numpy arrays in seed order
    plus the counters."""
    import torch
    from paper_2004_02003_amd import Context

    N = len(grids_dev) - 1
    if cap is None:
        cap = len(seeds) if seeds is not None else int(np.prod([(nd - 1 - (stride - 1) / 2) // stride + 1
                                                                for nd in n]))
    ctx = Context(n, max(int(cap), 1), origin=origin, spacing=spacing)
    try:
        if tuning:
            ctx.set_tuning(**tuning)
        if seeds is not None:
            ctx.seed_explicit(torch.as_tensor(np.ascontiguousarray(seeds, dtype=np.float64), device="cuda"))
        else:
            ctx.seed(stride)
        if chunks is None:
            chunks = [N]
        q = 0
        for k in chunks:
            ctx.advect(grids_dev[q:q + k + 1], times[q:q + k + 1], mode=mode, record_exit=record_exit)
            q += k
        assert q == N
        fm = ctx.flowmap(count_valid=True)
        if record_exit:
            fm["face"] = ctx.exit_points()
        st = ctx.stats()
        torch.cuda.synchronize()
        out = {k: v.cpu().numpy() for k, v in fm.items() if k != "n_valid"}
        out["n_valid"] = fm["n_valid"]
        out["stats"] = st
        return out
    finally:
        ctx.close()


# At most this fraction of the particles may be set aside as ties (oracle
# margin below MARGIN) before a comparison counts as failed: a face margin that
# came out too small would otherwise exclude everything and pass vacuously.
MAX_EXCLUDED = 0.01


def on_face(seeds, n):
    """Seeds (cell coordinates) lying exactly on a face of the block [0, n-1]^3."""
    s = np.asarray(seeds, dtype=np.float64).reshape(-1, 3)
    hi = np.asarray(n, dtype=np.float64) - 1.0
    return np.any((s == 0.0) | (s == hi), axis=1)


def compare(g, o, pos_tol=POS_TOL, margin=MARGIN, per_particle_tol=None, label="", max_excluded=MAX_EXCLUDED,
            seeds=None, n=None):
    """Assert parity of a GPU flow map ``g`` with an oracle result ``o``.

    Particles whose oracle decision points come within ``margin`` of a face
    are left out of the flag / exit-step / position checks; their fraction
    must stay at or below ``max_excluded``.  With ``seeds`` and ``n`` given,
    seeds placed exactly on a face (a lattice whose last points fall on the
    high face) must have margin 0, and their share is added to the
    allowance."""
    amb = o["margin"] < margin
    ok = ~amb
    excluded = float(amb.mean()) if amb.size else 0.0
    if seeds is not None:
        face = on_face(seeds, n)
        assert np.all(o["margin"][face] == 0.0), f"{label}: a seed on a face has a nonzero margin"
        max_excluded = max_excluded + float(face.mean())
    assert amb.size == 0 or ok.sum() > 0, f"{label}: every particle excluded as a tie"
    assert excluded <= max_excluded, f"{label}: {excluded:.2%} of the particles excluded as ties (> {max_excluded:.2%})"
    bad_flag = np.nonzero(ok & (g["flag"] != o["flag"]))[0]
    assert bad_flag.size == 0, f"{label}: flag mismatch at {bad_flag[:10]} (of {ok.sum()})"
    bad_exit = np.nonzero(ok & (g["exit"] != o["exit"]))[0]
    assert bad_exit.size == 0, f"{label}: exit-step mismatch at {bad_exit[:10]}"
    err = np.abs(g["end"] - o["end"]).max(axis=1)
    tol = pos_tol if per_particle_tol is None else np.maximum(pos_tol, per_particle_tol)
    bad = np.nonzero(ok & (err > tol))[0]
    assert bad.size == 0, (f"{label}: end position error {err[bad[:5]]} > tol at {bad[:5]}; "
                           f"max err {err[ok].max():.3e}")
    res = dict(n=len(err), ambiguous=int(amb.sum()), excluded_frac=excluded, max_err=float(err[ok].max()) if ok.any() else 0.0,
               mean_err=float(err[ok].mean()) if ok.any() else 0.0,
               terminated=float((o["flag"] == oracle.TERMINATED).mean()))
    if "face" in g and "face" in o:
        # exit points: present exactly where the oracle has one; errors in the
        # last inside and first outside points grow by the segment's factor
        has = ~np.isnan(o["face"][:, 0])
        gh = ~np.isnan(g["face"][:, 0])
        bad = np.nonzero(ok & (has != gh))[0]
        assert bad.size == 0, f"{label}: exit point presence differs at {bad[:10]}"
        sel = ok & has
        ferr = np.abs(g["face"] - o["face"]).max(axis=1)
        ftol = 2.0 * tol * np.maximum(1.0, np.nan_to_num(o["face_cond"], nan=1.0)) + 1e-6
        bad = np.nonzero(sel & (ferr > ftol))[0]
        assert bad.size == 0, (f"{label}: exit point error {ferr[bad[:5]]} > {np.broadcast_to(ftol, ferr.shape)[bad[:5]]}"
                               f" at {bad[:5]}")
        res["exit_points"] = int(sel.sum())
        res["exit_max_err"] = float(ferr[sel].max()) if sel.any() else 0.0
    return res


def oracle_lattice(field, times, n, stride, N, mode=oracle.LINEAR, ids=None, jac=False, nthreads=0):
    seeds = oracle.seed_lattice(n, stride)
    if ids is not None:
        seeds = seeds[ids]
    return seeds, oracle.flowmap(field, times, seeds, N, mode=mode, jac=jac, nthreads=nthreads)
