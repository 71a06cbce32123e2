"""Edge placement error of a printed pattern against its target.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper scores masks by L2 and PVBand (Sec. II-C); edge placement error is
not defined there, so this reading is used for reports only: sample points
are taken every 10 nm along each straight edge of the (Manhattan) target,
starting 5 nm from the edge's ends; at each, the signed distance along the
outward normal from the target edge to the boundary of the printed pattern
is measured on the pixel grid (positive: the print extends beyond the
target), searched within +-40 nm (a sample with no boundary in that range
counts as 40 nm).
"""
from __future__ import annotations

import numpy as np


def _edges(Z):
    """Straight edge runs: (orientation, line, start, end, outward sign).

    Horizontal edges lie on the line between pixel rows line-1 and line;
    vertical edges between columns line-1 and line.  outward = +1 when the
    target is on the lower-index side of the line.
    """
    Z = np.asarray(Z, dtype=bool)
    N0, N1 = Z.shape
    out = []
    P = np.zeros((N0 + 2, N1 + 2), dtype=bool)
    P[1:-1, 1:-1] = Z
    for orient in ("h", "v"):
        A = P if orient == "h" else P.T
        n_lines = A.shape[0] - 1
        for line in range(1, n_lines + 1):
            above, below = A[line - 1, 1:-1], A[line, 1:-1]
            for sign, mask in ((+1, above & ~below), (-1, ~above & below)):
                idx = np.flatnonzero(mask)
                if idx.size == 0:
                    continue
                breaks = np.flatnonzero(np.diff(idx) > 1)
                starts = np.concatenate([[idx[0]], idx[breaks + 1]])
                ends = np.concatenate([idx[breaks], [idx[-1]]]) + 1
                for a, b in zip(starts, ends):
                    out.append((orient, line - 1, int(a), int(b), sign))
    return out


def epe(Z, printed, pitch_nm, step_nm=10.0, end_nm=5.0, search_nm=40.0):
    """Signed EPE samples (nm) of `printed` against target `Z` (both 0/1)."""
    Z = np.asarray(Z, dtype=bool)
    Pm = np.asarray(printed, dtype=bool)
    N0, N1 = Z.shape
    reach = int(np.ceil(search_nm / pitch_nm))
    vals = []
    for orient, line, a, b, sign in _edges(Z):
        length = (b - a) * pitch_nm
        pos = end_nm
        while pos <= length - end_nm + 1e-9:
            t = a + int(pos / pitch_nm)          # pixel along the edge holding the sample
            # k-th pixel outward (k >= 0) and inward (k < 0) across the line
            def pix(k):
                r = line + k if sign > 0 else line - 1 - k
                if orient == "h":
                    return Pm[r, t] if 0 <= r < N0 else False
                return Pm[t, r] if 0 <= r < N1 else False
            if pix(0):
                k = 0
                while k < reach and pix(k):
                    k += 1
                d = k
            elif not pix(-1):
                k = -1
                while k >= -reach and not pix(k):
                    k -= 1
                d = -reach if k < -reach else k + 1
            else:
                d = 0
            vals.append(float(np.clip(d * pitch_nm, -search_nm, search_nm)))
            pos += step_nm
    return np.asarray(vals)


def epe_summary(Z, printed, pitch_nm, limit_nm=15.0):
    v = epe(Z, printed, pitch_nm)
    if v.size == 0:
        return {"samples": 0, "mean_abs_nm": 0.0, "max_abs_nm": 0.0, "over_limit": 0}
    a = np.abs(v)
    return {"samples": int(v.size), "mean_abs_nm": float(a.mean()), "max_abs_nm": float(a.max()),
            "over_limit": int(np.count_nonzero(a > limit_nm))}
