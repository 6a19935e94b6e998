"""FP64 oracle of the training targets at continuous positions (Sec. 4.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 4.3 draws training pairs of continuous positions in the domain [-1,1]^3 and
samples the ensemble there by trilinear interpolation of the grid values; the
target is the dependence measure of the two interpolated sample vectors.

Readings where the paper is silent (the GPU path uses the same ones):
* the domain's -1 and +1 are the first and last vertex of an axis, so the data
  grid coordinate is c = (p + 1)/2 (n - 1); positions outside the domain are
  clamped to it and NaN coordinates map to -1;
* the cell is base = min(floor(c), n - 2) with fraction f = c - base, and the
  eight corners (dx,dy,dz) get weights prod(f or 1 - f), vertex index
  i + nx*(j + ny*k);
* a corner of weight zero does not contribute (a non-finite value there does
  not reach the sample);
* Pearson's r of two columns with zero variance is 0.
"""
from __future__ import annotations

import numpy as np


def data_cell(p, dims):
    """Corner vertex indices (n,8) and trilinear weights (n,8) of positions p (n,3)."""
    p = np.asarray(p, dtype=np.float64)
    n = np.asarray(dims, dtype=np.int64)
    c = (p + 1.0) * 0.5 * (n - 1)
    c = np.where(np.isnan(c), 0.0, np.clip(c, 0.0, n - 1))
    base = np.minimum(np.floor(c).astype(np.int64), n - 2)
    f = c - base
    v = np.empty((p.shape[0], 8), dtype=np.int64)
    w = np.empty((p.shape[0], 8), dtype=np.float64)
    for corner in range(8):
        d = np.array([corner & 1, (corner >> 1) & 1, (corner >> 2) & 1])
        q = base + d
        v[:, corner] = q[:, 0] + n[0] * (q[:, 1] + n[1] * q[:, 2])
        w[:, corner] = np.prod(np.where(d == 1, f, 1.0 - f), axis=1)
    return v, w


def interpolate_members(x, dims, p):
    """Interpolated local samples e(p) (N, n) from the member-major ensemble x[N][V]."""
    v, w = data_cell(p, dims)
    x = np.asarray(x)
    out = np.zeros((x.shape[0], v.shape[0]), dtype=np.float64)
    for corner in range(8):
        wc = w[:, corner][None, :]
        out += np.where(wc == 0.0, 0.0, wc * x[:, v[:, corner]].astype(np.float64))
    return out


def pearson(a, b) -> float:
    """Eq. (1) on FP64 sample vectors, two-pass; 0 if either variance is 0."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    da = a - a.mean()
    db = b - b.mean()
    saa, sbb = float(np.dot(da, da)), float(np.dot(db, db))
    if saa == 0.0 or sbb == 0.0:
        return 0.0
    return float(np.dot(da, db) / np.sqrt(saa * sbb))


def pearson_points(xa, xb, dims, pos):
    """Targets for position pairs pos (B,2,3): r(e^a(p1), e^b(p2)) of the
    member-major ensembles xa, xb [N][V]."""
    pos = np.asarray(pos, dtype=np.float64)
    ea = interpolate_members(xa, dims, pos[:, 0])
    eb = interpolate_members(xb, dims, pos[:, 1])
    return np.array([pearson(ea[:, i], eb[:, i]) for i in range(pos.shape[0])])


def interpolated_codes(x, dims, p):
    """KSG integer codes (N, n) of the interpolated columns at positions p (n,3)
    and per-column flags (nonfinite, constant): the min-max mapping onto
    [0, 2^23] of Sec. 3.2's codes (round-half-even of (a - lo) * (2^23 / (hi -
    lo)) in IEEE double) applied to the interpolated samples."""
    a = interpolate_members(x, dims, p)
    lo = np.min(a, axis=0)
    hi = np.max(a, axis=0)
    bad = ~np.all(np.isfinite(a), axis=0)
    flat = ~(hi > lo)
    codes = np.zeros(a.shape, dtype=np.int32)
    for i in range(a.shape[1]):
        if bad[i] or flat[i]:
            continue
        scale = 8388608.0 / (hi[i] - lo[i])
        codes[:, i] = np.rint((a[:, i] - lo[i]) * scale).astype(np.int32)
    return codes, bad, flat


def ksg_points(xa, xb, dims, pos, k, counts=False):
    """KSG MI (nats) between the interpolated samples at position pairs pos (B,2,3),
    with the estimator of oracle.direct on the interpolated columns' codes; 0 for a
    constant column, NaN for a non-finite one.  counts: (B, 2, N) nx, ny."""
    from oracle import direct
    pos = np.asarray(pos, dtype=np.float64)
    ca, bada, flata = interpolated_codes(xa, dims, pos[:, 0])
    cb, badb, flatb = interpolated_codes(xb, dims, pos[:, 1])
    B, N = pos.shape[0], ca.shape[0]
    out = np.empty(B)
    cnt = np.zeros((B, 2, N), dtype=np.int32)
    for b in range(B):
        if bada[b] or badb[b]:
            out[b] = np.nan
        elif flata[b] or flatb[b]:
            out[b] = 0.0
        else:
            out[b], cnt[b, 0], cnt[b, 1] = direct.ksg(ca[:, b], cb[:, b], k)
    return (out, cnt) if counts else out
