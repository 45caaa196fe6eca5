"""Post hoc reconstruction of a seed-lattice flow map and its accuracy metric,
in FP64 numpy (test infrastructure only: the product library never imports it).

Reconstruction (Section 3.2, theoretical error analysis): a particle that
reaches its block's boundary is terminated, so its flow-map value is unknown;
it is rebuilt from its known neighbours by the one-dimensional linear
interpolation of Eq. (1),

    L(x1) = (x1 - x0) / (x2 - x0) * f(x2) + (x2 - x1) / (x2 - x0) * f(x0),

applied per component, with x0 < x1 < x2 on one lattice line and f(x0),
f(x2) known.  Eq. (2) shows that interpolating later with such a rebuilt value
gives the same result as interpolating from the nearest existing neighbours.
The paper triangulates scattered basis flows (Delaunay, barycentric
coordinates); on the structured seed lattice used here the rebuild is taken
along lattice lines, one axis at a time (x, then y, then z): in the pass along
axis d every entry still unknown whose line holds known entries on both sides
takes Eq. (1) from the nearest ones (entries known at the start of the pass;
lattice positions are uniform, so the fractions are index fractions).  Entries
with no such pair on any axis stay unknown.

Accuracy (Section 4, accuracy metric): the total average L2 norm of Eq. (5)
between the reconstructed BTO flow map b and the communicating flow map m over
the particles p that the latter keeps, and Eq. (6),
Accuracy% = (C - L) / C * 100 with C the cell side length.
"""

from __future__ import annotations

import numpy as np

MISSING, KNOWN, REBUILT = 0, 1, 2


def fill_line(vals: np.ndarray, known: np.ndarray):
    """Eq. (1) along one lattice line: vals (m, 3), known (m,) bool.  Returns
    (new values, newly filled mask); entries without known neighbours on both
    sides are left as they are."""
    out = vals.copy()
    filled = np.zeros(len(known), dtype=bool)
    idx = np.nonzero(known)[0]
    for i0, i2 in zip(idx[:-1], idx[1:]):
        for i1 in range(i0 + 1, i2):
            a = (i1 - i0) / (i2 - i0)
            b = (i2 - i1) / (i2 - i0)
            out[i1] = a * vals[i2] + b * vals[i0]
            filled[i1] = True
    return out, filled


def reconstruct(end: np.ndarray, known: np.ndarray, m):
    """Rebuild unknown entries of a lattice flow map.

    end: (P, 3) end positions in lattice order (x fastest), P = m0*m1*m2;
    known: (P,) bool (valid particles).  Returns (values (P, 3), state (P,)
    uint8: MISSING / KNOWN / REBUILT); unknown entries that stay missing are NaN.
    """
    m0, m1, m2 = (int(v) for v in m)
    v = np.where(known[:, None], end, np.nan).reshape(m2, m1, m0, 3).copy()
    st = np.where(known, KNOWN, MISSING).astype(np.uint8).reshape(m2, m1, m0).copy()
    for axis in (2, 1, 0):  # array axes of x, y, z
        have = st != MISSING
        vt = np.moveaxis(v, axis, -2)        # (..., m_d, 3), views into v
        ht = np.moveaxis(have, axis, -1)     # (..., m_d)
        stt = np.moveaxis(st, axis, -1)
        for lead in np.ndindex(ht.shape[:-1]):
            line_known = ht[lead]
            if line_known.all() or line_known.sum() < 2:
                continue
            new, filled = fill_line(vt[lead], line_known)
            vt[lead][filled] = new[filled]
            stt[lead][filled] = REBUILT
    return v.reshape(-1, 3), st.reshape(-1)


def flowmap_error(b_end: np.ndarray, b_state: np.ndarray, m_end: np.ndarray, m_flag: np.ndarray,
                  cell: float = 1.0, valid_flag: int = 0):
    """Eq. (5) and Eq. (6): mean and maximum L2 distance between b and m over
    the particles m keeps (flag valid) that b covers, the accuracy percentage,
    and the number of such particles b leaves missing."""
    sel = (m_flag == valid_flag) & (b_state != MISSING)
    d = np.sqrt(((b_end[sel] - m_end[sel]) ** 2).sum(axis=1))
    L = float(d.mean()) if d.size else 0.0
    return dict(mean_l2=L, max_l2=float(d.max()) if d.size else 0.0, n=int(sel.sum()),
                uncovered=int(((m_flag == valid_flag) & (b_state == MISSING)).sum()),
                accuracy_pct=(cell - L) / cell * 100.0)
