"""Pins of the FP64 oracle for training targets at continuous positions
(Sec. 4.3: the ensemble sampled by trilinear interpolation at positions in
[-1,1]^3, then Pearson's r of the two interpolated sample vectors)."""
import numpy as np

import gen
from oracle import direct
from oracle import points as pt

DIMS = (7, 5, 4)


def _grid_coords(dims):
    nx, ny, nz = dims
    v = np.arange(nx * ny * nz)
    return np.stack([v % nx, (v // nx) % ny, v // (nx * ny)], axis=1).astype(np.float64)


def test_weights_and_vertices():
    """Weights are a partition of unity; a vertex's position gives that vertex
    with weight one; the domain's corners are the grid's first and last vertex."""
    rng = np.random.default_rng(0)
    p = rng.uniform(-1, 1, (300, 3))
    v, w = pt.data_cell(p, DIMS)
    assert np.allclose(w.sum(1), 1.0, atol=1e-15) and np.all(w >= 0)
    V = DIMS[0] * DIMS[1] * DIMS[2]
    assert v.min() >= 0 and v.max() < V
    ijk = _grid_coords(DIMS)
    n = np.array(DIMS) - 1
    pv = 2.0 * ijk / n - 1.0
    v, w = pt.data_cell(pv, DIMS)
    k = np.argmax(w, axis=1)
    assert np.array_equal(v[np.arange(V), k], np.arange(V))
    assert np.allclose(w.max(1), 1.0, atol=1e-14)
    v, w = pt.data_cell(np.array([[-1.0, -1.0, -1.0], [1.0, 1.0, 1.0]]), DIMS)
    assert v[0, np.argmax(w[0])] == 0 and v[1, np.argmax(w[1])] == V - 1


def test_affine_ensemble_interpolates_exactly():
    """Members that are affine in the grid coordinates are reproduced exactly at
    any position: e(p)_m = alpha_m + beta_m . c with c = (p + 1)/2 (n - 1);
    outside the domain the clamped position's value comes back."""
    rng = np.random.default_rng(1)
    N = 9
    alpha = rng.standard_normal(N)
    beta = rng.standard_normal((N, 3))
    x = alpha[:, None] + beta @ _grid_coords(DIMS).T
    p = rng.uniform(-1, 1, (200, 3))
    c = (p + 1.0) / 2.0 * (np.array(DIMS) - 1)
    want = alpha[:, None] + beta @ c.T
    got = pt.interpolate_members(x, DIMS, p)
    assert np.max(np.abs(got - want)) < 1e-12
    q = p.copy()
    q[:, 2] = rng.uniform(1.0, 4.0, 200)
    q[:5, 0] = np.nan
    clamped = p.copy()
    clamped[:, 2] = 1.0
    clamped[:5, 0] = -1.0
    np.testing.assert_array_equal(pt.interpolate_members(x, DIMS, q),
                                  pt.interpolate_members(x, DIMS, clamped))


def test_pearson_special_cases():
    rng = np.random.default_rng(2)
    a = rng.standard_normal(500)
    assert abs(pt.pearson(a, 2 * a + 3) - 1.0) < 1e-14
    assert abs(pt.pearson(a, -0.5 * a + 1) + 1.0) < 1e-14
    assert pt.pearson(a, np.full(500, 2.5)) == 0.0
    b = rng.standard_normal(500)
    # the C oracle's Eq. (1) on the same float32 values
    a32, b32 = a.astype(np.float32), b.astype(np.float32)
    assert abs(pt.pearson(a32, b32) - direct.pearson(a32, b32)) < 1e-13
    # closed form for a 2-member sample: +-1
    assert pt.pearson([0.0, 1.0], [3.0, 7.0]) == 1.0


def test_targets_at_vertex_positions_are_vertex_targets():
    """Position pairs on grid vertices give the vertex-pair Pearson targets."""
    cfg = gen.CONFIGS["tiny"]
    x = gen.make_ensemble(cfg, device="cpu")[0].numpy()
    dims = (cfg.nx, cfg.ny, cfg.nz)
    pairs = gen.random_pairs(cfg.n_vertices, 40, seed=5)
    ijk = _grid_coords(dims)
    pos = 2.0 * ijk[pairs] / (np.array(dims) - 1) - 1.0
    got = pt.pearson_points(x, x, dims, pos)
    want = np.array([direct.pearson(x[:, a], x[:, b]) for a, b in pairs])
    assert np.max(np.abs(got - want)) < 1e-12


def test_midpoint_of_two_members_columns():
    """Halfway between two vertices along x the sample is their mean (weights
    1/2, 1/2), so r with either endpoint follows from the 2x2 covariance."""
    rng = np.random.default_rng(3)
    N = 64
    V = DIMS[0] * DIMS[1] * DIMS[2]
    x = rng.standard_normal((N, V))
    n = np.array(DIMS) - 1
    p0 = 2.0 * np.array([2, 1, 1]) / n - 1.0
    p1 = 2.0 * np.array([3, 1, 1]) / n - 1.0
    mid = (p0 + p1) / 2.0
    v0 = 2 + DIMS[0] * (1 + DIMS[1] * 1)
    a, b = x[:, v0], x[:, v0 + 1]
    e = pt.interpolate_members(x, DIMS, mid[None, :])[:, 0]
    assert np.max(np.abs(e - (a + b) / 2)) < 1e-15
    da, db = a - a.mean(), b - b.mean()
    saa, sbb, sab = da @ da, db @ db, da @ db
    want = (saa + sab) / np.sqrt(saa * (saa + 2 * sab + sbb))
    got = pt.pearson_points(x, x, DIMS, np.stack([p0, mid])[None])[0]
    assert abs(got - want) < 1e-13


def test_zero_weight_corner_does_not_contribute():
    """A non-finite value at a corner of weight zero does not reach the sample."""
    rng = np.random.default_rng(6)
    V = DIMS[0] * DIMS[1] * DIMS[2]
    x = rng.standard_normal((8, V))
    x[3, 1] = np.nan                     # vertex (1,0,0)
    p = np.array([[-1.0, -1.0, -1.0]])   # vertex 0; (1,0,0) is a corner of weight 0
    v, w = pt.data_cell(p, DIMS)
    assert 1 in v[0] and w[0][list(v[0]).index(1)] == 0.0
    np.testing.assert_array_equal(pt.interpolate_members(x, DIMS, p)[:, 0], x[:, 0])
    q = np.array([[2.0 / (DIMS[0] - 1) - 1.0 + 0.01, -1.0, -1.0]])
    assert np.isnan(pt.interpolate_members(x, DIMS, q)[3, 0])


def test_interpolated_codes_at_vertices_are_vertex_codes():
    """At a vertex's own position the interpolated column is the vertex column, so
    its codes are the C oracle's vertex codes and the KSG estimate is the vertex
    pair's; halfway between two vertices the codes follow from the mean column."""
    cfg = gen.CONFIGS["tiny"]
    x = gen.make_ensemble(cfg, device="cpu")[0].numpy()
    dims = (cfg.nx, cfg.ny, cfg.nz)
    pairs = gen.random_pairs(cfg.n_vertices, 12, seed=7)
    ijk = _grid_coords(dims)
    pos = (2.0 * ijk[pairs] / (np.array(dims) - 1) - 1.0)
    codes, bad, flat = pt.interpolated_codes(x, dims, pos[:, 0])
    assert not bad.any() and not flat.any()
    for i, v in enumerate(pairs[:, 0]):
        want, _ = direct.ksg_codes(x[:, v])
        assert np.array_equal(codes[:, i], want)
    got = pt.ksg_points(x, x, dims, pos, 4)
    want = np.array([direct.ksg_field(x[:, a], x[:, b:b + 1], 4)[0] for a, b in pairs])
    np.testing.assert_array_equal(got, want)
    # midpoint: the column is (x_a + x_b) / 2 exactly (weights 1/2 in FP64)
    v0 = 3 + cfg.nx * (2 + cfg.ny * 1)
    mid = 2.0 * (ijk[v0] + np.array([0.5, 0.0, 0.0])) / (np.array(dims) - 1) - 1.0
    m = 0.5 * x[:, v0].astype(np.float64) + 0.5 * x[:, v0 + 1].astype(np.float64)
    lo, hi = m.min(), m.max()
    want = np.rint((m - lo) * (8388608.0 / (hi - lo))).astype(np.int32)
    c, _, _ = pt.interpolated_codes(x, dims, mid[None, :])
    assert np.array_equal(c[:, 0], want)


def test_ksg_points_flags():
    """A constant interpolated column gives 0, a non-finite one NaN."""
    rng = np.random.default_rng(8)
    V = DIMS[0] * DIMS[1] * DIMS[2]
    x = rng.standard_normal((16, V))
    x[:, V - 1] = 1.5
    x[2, 0] = np.inf
    pos = np.array([[[1.0, 1.0, 1.0], [0.1, 0.2, 0.3]],
                    [[-1.0, -1.0, -1.0], [0.1, 0.2, 0.3]],
                    [[0.3, -0.2, 0.5], [0.1, 0.2, 0.3]]])
    out = pt.ksg_points(x, x, DIMS, pos, 3)
    assert out[0] == 0.0 and np.isnan(out[1]) and np.isfinite(out[2])
