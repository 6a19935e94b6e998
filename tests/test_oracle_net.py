"""Pins of the FP64 learned-field oracle (Sec. 4) against closed forms (no GPU).

* trilinear lookup (Sec. 4.2, dense levels): reproduces affine feature fields
  exactly, returns stored values at level vertices, weights sum to one, the
  boundary u = 1 lands on the last vertex; gather and scatter are adjoint;
* a hand-built network whose output has a closed form (asymmetric selections,
  so a transposed weight, a wrong feature slot or a missing ReLU fails);
* symmetry of the self field (Sec. 4.1) and the variable-swap identity of a
  two-encoder field (Sec. 6.4);
* the adjoint against central finite differences;
* the first Adam step in closed form.
"""
import math

import numpy as np
import pytest

import gen
from oracle import ndf_net as nn

DIMS = (5, 4, 3)
RES = [(2, 2, 2), (3, 3, 2), (4, 3, 3), (5, 4, 3)]


def _layout(width=128, n_enc=1, dims=DIMS, res=RES, grid_only=False, fourier=0):
    return gen.NetLayout(dims[0], dims[1], dims[2], tuple(res), 8, width, n_enc, 0, grid_only,
                         fourier)


def _net(flat, width=128, n_enc=1, dims=DIMS, res=RES, grid_only=False, fourier=0):
    return nn.Net(flat, dims, res, 8, width, n_enc, grid_only=grid_only, fourier=fourier)


def _cell_positions(R):
    rx, ry, rz = R
    c = np.arange(rx * ry * rz)
    x, y, z = c % rx, (c // rx) % ry, c // (rx * ry)
    return np.stack([x / (rx - 1), y / (ry - 1), z / (rz - 1)], axis=1)


def test_layout_parse_matches_generator():
    for n_enc in (1, 2):
        L = _layout(n_enc=n_enc)
        flat = gen.make_net_params(L)
        net = _net(flat, n_enc=n_enc)
        assert net.n_floats == L.n_floats
        for name, shape in L.tensors():
            if name.startswith("grid"):
                e, l = map(int, name[4:].split("_"))
                key = ("grid", e, l)
            elif name[-2] == "_":
                key = (name[:-2], int(name[-1]))
            else:
                key = name
            np.testing.assert_array_equal(net[key], L.view(flat, name))


def test_trilinear_affine_and_vertices():
    rng = np.random.default_rng(0)
    for R in RES + [(62, 88, 5)]:
        u = rng.uniform(0, 1, (500, 3))
        u[:5] = 1.0
        u[5:10] = 0.0
        idx, w = nn.trilinear(u, R)
        assert np.allclose(w.sum(1), 1.0, atol=1e-15)
        assert np.all(w >= 0)
        pos = _cell_positions(R)
        coef = rng.standard_normal(4)
        vals = coef[0] + pos @ coef[1:]
        interp = np.sum(w * vals[idx], axis=1)
        assert np.max(np.abs(interp - (coef[0] + u @ coef[1:]))) < 1e-12
        # at the level's own vertices the stored value comes back
        idx, w = nn.trilinear(pos, R)
        got = np.sum(w * vals[idx], axis=1)
        assert np.max(np.abs(got - vals)) < 1e-12
        # u = 1 on every axis is the last vertex with weight one
        idx, w = nn.trilinear(np.ones((1, 3)), R)
        assert idx[0, np.argmax(w[0])] == R[0] * R[1] * R[2] - 1 and w[0].max() == 1.0


def test_domain_positions_map_to_grid():
    """Continuous positions in the domain [-1,1]^3 (Sec. 4.3): -1 and +1 are the
    first and last vertex of an axis, so the trilinear features of an affine
    level field at p equal the affine function of u = (p + 1)/2 exactly, a vertex's
    position gives the vertex lookup's features, and positions outside the
    domain take the boundary's value."""
    rng = np.random.default_rng(4)
    np.testing.assert_array_equal(nn.domain_to_unit(np.array([[-1.0, 0.0, 1.0]])),
                                  [[0.0, 0.5, 1.0]])
    np.testing.assert_array_equal(nn.domain_to_unit(np.array([[-3.0, 2.5, np.nan]])),
                                  [[0.0, 1.0, 0.0]])
    L = _layout()
    net = _net(gen.make_net_params(L, grid_scale=1.0))
    coef = rng.standard_normal((4, 8))
    for l, R in enumerate(RES):
        pos = _cell_positions(R)
        net[("grid", 0, l)] = coef[0] + pos @ coef[1:]
    p = rng.uniform(-1, 1, (400, 3))
    h0 = nn.grid_encode(net, 0, nn.domain_to_unit(p))
    want = coef[0] + ((p + 1) / 2) @ coef[1:]
    for l in range(len(RES)):
        assert np.max(np.abs(h0[:, 8 * l:8 * l + 8] - want)) < 1e-12
    # vertex positions 2 i/(n - 1) - 1 reproduce the vertex lookup
    v = np.arange(DIMS[0] * DIMS[1] * DIMS[2])
    u_v = nn.vertex_positions(v, DIMS)
    p_v = 2.0 * u_v - 1.0
    np.testing.assert_allclose(nn.grid_encode(net, 0, nn.domain_to_unit(p_v)),
                               nn.grid_encode(net, 0, u_v), rtol=0, atol=1e-12)
    # outside the domain: the clamped boundary point
    q = rng.uniform(-1, 1, (50, 3))
    out = q.copy()
    out[:, 0] = rng.uniform(1.0, 3.0, 50)
    inside = q.copy()
    inside[:, 0] = 1.0
    np.testing.assert_array_equal(nn.grid_encode(net, 0, nn.domain_to_unit(out)),
                                  nn.grid_encode(net, 0, nn.domain_to_unit(inside)))


def test_field_points_at_vertices_is_the_field():
    """Phi(p_ref, p) at the positions of grid vertices equals the vertex field."""
    L = _layout(n_enc=2)
    net = _net(gen.make_net_params(L, seed=9, grid_scale=1.0, bias_scale=0.2), n_enc=2)
    V = DIMS[0] * DIMS[1] * DIMS[2]
    p_v = 2.0 * nn.vertex_positions(np.arange(V), DIMS) - 1.0
    for ref in (0, 17, V - 1):
        np.testing.assert_allclose(nn.field_points(net, ref, p_v), nn.field(net, ref),
                                   rtol=1e-12, atol=1e-12)


def test_gather_scatter_adjoint():
    rng = np.random.default_rng(1)
    L = _layout()
    net = _net(gen.make_net_params(L, grid_scale=1.0))
    u = rng.uniform(0, 1, (300, 3))
    G = net.zeros_like()
    for l in range(4):
        G[("grid", 0, l)] = rng.standard_normal(G[("grid", 0, l)].shape)
    y = rng.standard_normal((300, 32))
    probe = _net(G.flat)
    lhs = np.sum(nn.grid_encode(probe, 0, u) * y)
    S = net.zeros_like()
    nn.grid_scatter(net, 0, u, y, S)
    rhs = sum(np.sum(G[("grid", 0, l)] * S[("grid", 0, l)]) for l in range(4))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def hand_built_params(dims=DIMS, res=RES, noise_seed=3):
    """Parameters whose field is Phi(p1, p2) = Q(u1) Q(u2) + 1/8 with
    Q(u) = u_x + 6 u_y + 4.5 (see test_hand_built_network_closed_form)."""
    L = _layout(dims=dims, res=res)
    flat = np.zeros(L.n_floats)
    net = _net(flat, dims=dims, res=res)
    rng = np.random.default_rng(noise_seed)
    for l, R in enumerate(res):
        g = net[("grid", 0, l)]
        g[:] = rng.standard_normal(g.shape)          # unused slots hold noise
        pos = _cell_positions(R)
        if l == 0:
            g[:, 2] = pos[:, 0] + 2.0                 # A(u) = u_x + 2
        if l == 2:
            g[:, 5] = 3.0 * pos[:, 1] + 1.0           # B(u) = 3 u_y + 1
        if l == 3:
            g[:, 0] = pos[:, 2]                       # C(u) = u_z
    W1, b1 = net[("W1", 0)], net[("b1", 0)]
    W1[3, 2] = 1.0                                    # a1[3] = A
    W1[9, 21] = 2.0; b1[9] = 0.5                      # a1[9] = 2B + 1/2
    W1[100, 24] = -1.0; b1[100] = -5.0                # a1[100] < 0, cut by ReLU
    W2, b2 = net[("W2", 0)], net[("b2", 0)]
    W2[7, 3] = 1.0; W2[7, 9] = 1.0                    # a2[7] = A + 2B + 1/2 = Q
    W2[50, 100] = 3.0; b2[50] = 1.0                   # a2[50] = 1 only after ReLU
    W3, b3 = net[("W3", 0)], net[("b3", 0)]
    W3[11, 7] = 1.0                                   # lat[11] = Q
    W3[12, 50] = 1.0; b3[12] = -3.0                   # lat[12] = -2
    W4, b4 = net["W4"], net["b4"]
    W4[20, 11] = 1.0; W4[20, 12] = 0.25               # a4[20] = Q1 Q2 + 1
    W4[21, 12] = -1.0                                 # a4[21] = -4, cut by ReLU
    W5, b5 = net["W5"], net["b5"]
    W5[5, 20] = 2.0; W5[5, 21] = 7.0; b5[5] = 0.25    # a5[5] = 2 (Q1 Q2 + 1) + 1/4
    net["w6"][5] = 0.5
    net["b6"][0] = -1.0                               # y = Q1 Q2 + 1/8
    return net.flat.astype(np.float32)


def hand_built_value(v1, v2, dims=DIMS):
    u1 = nn.vertex_positions(v1, dims)
    u2 = nn.vertex_positions(v2, dims)
    q1 = u1[:, 0] + 6 * u1[:, 1] + 4.5
    q2 = u2[:, 0] + 6 * u2[:, 1] + 4.5
    return q1 * q2 + 0.125


def test_hand_built_network_closed_form():
    flat = hand_built_params()
    net = _net(flat)
    V = DIMS[0] * DIMS[1] * DIMS[2]
    v1, v2 = np.meshgrid(np.arange(V), np.arange(V))
    v1, v2 = v1.ravel(), v2.ravel()
    y, _ = nn.forward(net, v1, v2)
    assert np.max(np.abs(y - hand_built_value(v1, v2))) < 1e-12


def test_self_field_symmetric_exactly():
    L = _layout()
    net = _net(gen.make_net_params(L, grid_scale=0.5, bias_scale=0.1))
    pairs = gen.random_pairs(60, 500, seed=4)
    y12, _ = nn.forward(net, pairs[:, 0], pairs[:, 1])
    y21, _ = nn.forward(net, pairs[:, 1], pairs[:, 0])
    assert np.array_equal(y12, y21)


def test_two_encoder_swap_identity():
    # Phi_{nu mu}(p1, p2) = Phi_{mu nu}(p2, p1): swapping the encoders' parameters
    # and the positions leaves the value unchanged
    L = _layout(n_enc=2)
    flat = gen.make_net_params(L, grid_scale=0.5, bias_scale=0.1)
    net = _net(flat, n_enc=2)
    sw = _net(flat, n_enc=2)
    for key in list(net.slices):
        if isinstance(key, tuple) and key[0] != "grid":
            sw[(key[0], 1 - key[1])] = net[key]
        elif isinstance(key, tuple):
            sw[("grid", 1 - key[1], key[2])] = net[key]
    pairs = gen.random_pairs(60, 300, seed=6)
    y, _ = nn.forward(net, pairs[:, 0], pairs[:, 1])
    ys, _ = nn.forward(sw, pairs[:, 1], pairs[:, 0])
    assert np.max(np.abs(y - ys)) < 1e-13
    y_fwd, _ = nn.forward(net, pairs[:, 1], pairs[:, 0])
    assert np.max(np.abs(y - y_fwd)) > 1e-6           # the field itself is not symmetric


@pytest.mark.parametrize("n_enc,grid_only,fourier",
                         [(1, False, 0), (2, False, 0), (1, True, 0), (2, True, 0), (1, False, 12)])
def test_adjoint_vs_finite_differences(n_enc, grid_only, fourier):
    width = 16
    L = _layout(width=width, n_enc=n_enc, grid_only=grid_only, fourier=fourier)
    flat = gen.make_net_params(L, seed=9, grid_scale=0.5, bias_scale=0.2).astype(np.float64)
    net = _net(flat, width=width, n_enc=n_enc, grid_only=grid_only, fourier=fourier)
    pairs = gen.random_pairs(60, 64, seed=8)
    y, _ = nn.forward(net, pairs[:, 0], pairs[:, 1])
    t = y - 10.0                      # every residual positive: L = mean(y) + 10, smooth
    loss, g, _ = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], t)
    rng = np.random.default_rng(2)
    h = 1e-6
    for key in net.slices:
        o, shape = net.slices[key]
        n = int(np.prod(shape))
        d = np.zeros_like(flat)
        d[o:o + n] = rng.standard_normal(n)
        lp = nn.l1_loss(nn.forward(_net(flat + h * d, width=width, n_enc=n_enc,
                                        grid_only=grid_only, fourier=fourier),
                                   pairs[:, 0], pairs[:, 1])[0], t)
        lm = nn.l1_loss(nn.forward(_net(flat - h * d, width=width, n_enc=n_enc,
                                        grid_only=grid_only, fourier=fourier),
                                   pairs[:, 0], pairs[:, 1])[0], t)
        fd = (lp - lm) / (2 * h)
        an = float(np.dot(g.flat, d))
        assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)) + 1e-9, (key, fd, an)


def test_fourier_features_identities():
    """Fourier features (Sec. 4.2, Eq. 4) pinned by identities rather than by their
    formula: every (sin, cos) pair lies on the unit circle; each frequency is
    twice the previous one (double-angle formulas), with the same axis; the base
    frequency is pi (p_j = 1/2 gives (1, 0)); a change of one coordinate changes
    only that axis's raw column and features."""
    rng = np.random.default_rng(31)
    u = rng.random((50, 3))
    F = nn.fourier_features(u, 12)
    assert F.shape == (50, 3 + 72)
    np.testing.assert_allclose(F[:, :3], 2 * u - 1, atol=0)
    for i in range(12):
        for j in range(3):
            s_, c_ = F[:, 3 + 6 * i + 2 * j], F[:, 4 + 6 * i + 2 * j]
            np.testing.assert_allclose(s_ ** 2 + c_ ** 2, 1.0, atol=1e-12)
            if i < 11:
                s2, c2 = F[:, 3 + 6 * (i + 1) + 2 * j], F[:, 4 + 6 * (i + 1) + 2 * j]
                np.testing.assert_allclose(s2, 2 * s_ * c_, atol=1e-9)
                np.testing.assert_allclose(c2, c_ ** 2 - s_ ** 2, atol=1e-9)
    half = nn.fourier_features(np.array([[0.75, 0.75, 0.75]]), 1)[0]
    np.testing.assert_allclose(half[3:], [1, 0, 1, 0, 1, 0], atol=1e-15)
    for j in range(3):
        v = u.copy()
        v[:, j] = rng.random(50)
        G = nn.fourier_features(v, 12)
        changed = np.any(G != F, axis=0)
        cols = {j} | {3 + 6 * i + 2 * j + k for i in range(12) for k in (0, 1)}
        assert set(np.flatnonzero(changed)) == cols


def test_fourier_input_embedding_layout():
    """With L = 12 the encoder input is 112 wide: the 32 grid features, the raw
    position and 72 Fourier features, then five zero columns; a network whose W1
    reads only sin(2^3 pi p_y) gives that value through a closed form."""
    L = _layout(width=16, fourier=12)
    assert L.enc_in == 112
    flat = gen.make_net_params(L, seed=4, grid_scale=0.5)
    net = _net(flat, width=16, fourier=12)
    u = np.random.default_rng(6).random((40, 3))
    h0 = nn.input_embedding(net, 0, u)
    assert h0.shape == (40, 112)
    np.testing.assert_array_equal(h0[:, :32], nn.grid_encode(net, 0, u))
    np.testing.assert_array_equal(h0[:, 107:], 0)
    # W1 picks column 32 + 3 + 6 i + 2 j (i = 3, j = y), the encoder passes it on
    # through identities: latent[0] = relu(relu(sin)) for a positive sine
    net["W1", 0] = 0
    net["b1", 0] = 0
    W1 = net["W1", 0].copy()
    W1[0, 32 + 3 + 6 * 3 + 2 * 1] = 1.0
    net["W1", 0] = W1
    for k in ("W2", "W3"):
        net[k, 0] = np.eye(16)
        net[k.replace("W", "b"), 0] = 0
    enc = nn.encoder(net, 0, h0)
    want = np.maximum(np.sin(8 * np.pi * (2 * u[:, 1] - 1)), 0)
    np.testing.assert_allclose(enc["lat"][:, 0], want, atol=1e-15)


def test_l1_gradient_sign_convention():
    L = _layout(width=16)
    net = _net(gen.make_net_params(L, seed=3, grid_scale=0.5, bias_scale=0.2), width=16)
    pairs = gen.random_pairs(60, 8, seed=1)
    y, _ = nn.forward(net, pairs[:, 0], pairs[:, 1])
    _, g_lo, _ = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], y - 1.0)
    _, g_hi, _ = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], y + 1.0)
    np.testing.assert_allclose(g_lo.flat, -g_hi.flat, atol=1e-15)
    assert g_lo["b6"][0] == pytest.approx(1.0)        # d mean(y - t) / d b6


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    p = rng.standard_normal(1000)
    g = rng.standard_normal(1000) * 10.0 ** rng.uniform(-9, 1, 1000)
    lr = 3e-4
    p1, m, v = nn.adam_update(p, g, np.zeros(1000), np.zeros(1000), 1, lr)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)


# --------------------------------------------------------------- hash grids ----
RES_H = [(8, 8, 8), (16, 12, 8), (20, 16, 10), (24, 20, 12)]
DIMS_H = (24, 20, 12)


def test_hash_definition_values():
    """The spatial hash of Sec. 4.2's hash grids: xor of the corner coordinates
    times one prime per axis, the first prime 1, modulo 2^T.  Values worked by
    hand from the primes' hex forms 0x9E3779B1 and 0x30025795."""
    T = 10
    p = np.array([[5, 0, 0], [1029, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]])
    np.testing.assert_array_equal(nn.hash_cell(p, T), [5, 5, 0x1B1, 0x395, 0x225])
    assert nn.level_hashed((16, 12, 8), 10) and not nn.level_hashed((8, 8, 8), 10)
    assert nn.level_cells((16, 12, 8), 10) == 1024 and nn.level_cells((8, 8, 8), 10) == 512


def test_hashed_level_lookup_end_to_end():
    """Table entry i holding the value i in feature 0: at the position of a level
    vertex (weight one on that corner) the feature is the corner's hash; on a
    dense level it is the dense cell index."""
    T = 10
    L = gen.NetLayout(DIMS_H[0], DIMS_H[1], DIMS_H[2], tuple(RES_H), 8, 128, 1, T)
    net = nn.Net(gen.make_net_params(L), DIMS_H, RES_H, 8, 128, 1, T)
    for l, R in enumerate(RES_H):
        g = np.zeros((nn.level_cells(R, T), 8))
        g[:, 0] = np.arange(g.shape[0])
        net[("grid", 0, l)] = g
    rng = np.random.default_rng(3)
    for l, R in enumerate(RES_H):
        c = np.stack([rng.integers(0, r, 50) for r in R], axis=1)
        u = c / (np.array(R) - 1.0)
        h0 = nn.grid_encode(net, 0, u)[:, 8 * l]
        if nn.level_hashed(R, T):
            want = nn.hash_cell(c, T)
        else:
            want = c[:, 0] + R[0] * (c[:, 1] + R[1] * c[:, 2])
        np.testing.assert_allclose(h0, want, rtol=0, atol=1e-9)


def test_hashed_gather_scatter_adjoint_with_collisions():
    """The adjoint identity holds on hashed levels, where corners collide and
    their contributions add into one cell."""
    T = 9
    L = gen.NetLayout(DIMS_H[0], DIMS_H[1], DIMS_H[2], tuple(RES_H), 8, 128, 1, T)
    net = nn.Net(gen.make_net_params(L, grid_scale=1.0), DIMS_H, RES_H, 8, 128, 1, T)
    rng = np.random.default_rng(4)
    u = rng.uniform(0, 1, (400, 3))
    idx, _ = nn.trilinear(u, RES_H[3], T)
    assert len(np.unique(idx)) < len(np.unique(nn.trilinear(u, RES_H[3])[0]))  # collisions
    G = net.zeros_like()
    for l in range(4):
        G[("grid", 0, l)] = rng.standard_normal(G[("grid", 0, l)].shape)
    y = rng.standard_normal((400, 32))
    probe = nn.Net(G.flat, DIMS_H, RES_H, 8, 128, 1, T)
    lhs = np.sum(nn.grid_encode(probe, 0, u) * y)
    S = net.zeros_like()
    nn.grid_scatter(net, 0, u, y, S)
    rhs = sum(np.sum(G[("grid", 0, l)] * S[("grid", 0, l)]) for l in range(4))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_large_table_is_the_dense_grid():
    """A table at least as large as every level leaves every level dense: the same
    layout and the same field as T = 0."""
    L0 = gen.NetLayout(DIMS_H[0], DIMS_H[1], DIMS_H[2], tuple(RES_H), 8, 128, 2, 0)
    L1 = gen.NetLayout(DIMS_H[0], DIMS_H[1], DIMS_H[2], tuple(RES_H), 8, 128, 2, 13)
    assert L0.offsets() == L1.offsets()
    flat = gen.make_net_params(L0, grid_scale=1.0, bias_scale=0.1)
    a = nn.Net(flat, DIMS_H, RES_H, 8, 128, 2, 0)
    b = nn.Net(flat, DIMS_H, RES_H, 8, 128, 2, 13)
    np.testing.assert_array_equal(nn.field(a, 17), nn.field(b, 17))


# ------------------------------------------------------- operand rounding ----
def test_round_bf16_matches_library_and_ties_to_even():
    import torch
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-20, 20, 5000),
                        [0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8)]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).double().numpy()
    np.testing.assert_array_equal(nn.round_bf16(x), want)
    # halfway cases go to the even significand
    assert nn.round_bf16(1 + 2 ** -8) == 1.0
    assert nn.round_bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    hi_lo = nn.round_split_bf16(np.float32(np.pi))
    assert abs(hi_lo - np.float32(np.pi)) <= 2.0 ** -16 * np.pi


def test_round_e4m3_matches_library_on_its_range():
    import torch
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.uniform(-448, 448, 4000), rng.normal(size=4000) * 2.0 ** -7,
                        [0.0, 448.0, -448.0, 2 ** -6, 2 ** -9, 2 ** -10, 3 * 2 ** -10, 1.0625,
                         1.1875, 240.0, 232.0]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.float8_e4m3fn).double().numpy()
    np.testing.assert_array_equal(nn.round_e4m3(x), want)
    assert nn.round_e4m3(1.0625) == 1.0          # tie between 1 and 1.125: even
    assert nn.round_e4m3(1.1875) == 1.25         # tie between 1.125 and 1.25: even
    assert nn.round_e4m3(2 ** -10) == 0.0 and nn.round_e4m3(3 * 2 ** -10) == 2 ** -8
    assert nn.round_e4m3(1000.0) == 448.0        # saturates


def test_e4m3_block_scale():
    # smallest e with m / 2^e <= 448
    for m, e in [(448.0, 0), (448.0001, 1), (1.75, -8), (1.76, -7), (1.0, -8), (0.0, -126),
                 (1e-30, -108), (3.0e6, 13)]:
        got = int(nn.e4m3_scale_exp(m))
        assert got == e, (m, got, e)
        if m > 0 and e > -126:
            assert m / 2.0 ** e <= 448 < m / 2.0 ** (e - 1)
    rng = np.random.default_rng(5)
    a = rng.normal(size=(7, 64)) * 3.0
    q = nn.round_mx_e4m3(a)
    # scaling a block by a power of two scales its rounding exactly
    np.testing.assert_array_equal(nn.round_mx_e4m3(a * 2.0 ** 9), q * 2.0 ** 9)
    # values already on a block's E4M3 grid are kept
    np.testing.assert_array_equal(nn.round_mx_e4m3(q), q)
    # each block's largest magnitude lands within E4M3's relative spacing 2^-4
    b = np.abs(a).reshape(7, 2, 32).max(-1)
    bq = np.abs(q).reshape(7, 2, 32).max(-1)
    assert np.all(np.abs(bq - b) <= 2.0 ** -4 * b)


def test_calibration_vertices():
    v = nn.calibration_vertices(4, 100)
    np.testing.assert_array_equal(v, [12, 37, 62, 87])   # (2 i + 1) * 100 / 8
    v = nn.calibration_vertices(2048, 1_760_000)
    assert v[0] == 429 and v[-1] == 1_759_570 and np.all(np.diff(v) > 0)


def test_fp8_static_activation_scales():
    """Static E4M3 activation scales: s_l = 2^e with e the smallest exponent for
    which twice the calibrated maximum fits in 448 s_l, so no calibration input
    saturates; values beyond 448 s_l saturate.  Moving a power of two from W2 into
    W1 and b1 (ReLU is positively homogeneous) multiplies the first calibrated
    maximum by it, leaves the others, and leaves the emulated E4M3 field bit for
    bit as it was, which fails if a layer's scale is applied to another layer's
    input or the maxima are taken from the wrong activations."""
    cfg = gen.CONFIGS["tiny"]
    lay = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz)
    flat = gen.make_net_params(lay, seed=2329, grid_scale=0.5, bias_scale=0.1)
    dims = (cfg.nx, cfg.ny, cfg.nz)
    net = nn.Net(flat, dims, lay.res)
    M = nn.fp8_activation_maxima(net)
    assert np.all(M > 0)
    s = nn.fp8_activation_scales(M)
    assert np.all(2 * M <= 448 * s) and np.all(448 * s < 4 * M)
    ops = nn.fp8_inference_operands(net, M)
    x = np.array([0.0, 100 * s[1], 448 * s[1], 449 * s[1], -1e9])
    np.testing.assert_array_equal(ops.act(x, 3),
                                  [0.0, 96 * s[1], 448 * s[1], 448 * s[1], -448 * s[1]])
    k = 2.0 ** 3
    f2 = flat.copy()
    lay.view(f2, "W1_0")[:] *= k
    lay.view(f2, "b1_0")[:] *= k
    lay.view(f2, "W2_0")[:] /= k
    net2 = nn.Net(f2, dims, lay.res)
    M2 = nn.fp8_activation_maxima(net2)
    np.testing.assert_array_equal(M2, M * np.array([k, 1, 1, 1]))
    ref = cfg.ref_v
    y1 = nn.field(net, ref, rnd=ops)
    y2 = nn.field(net2, ref, rnd=nn.fp8_inference_operands(net2, M2))
    np.testing.assert_array_equal(y1, y2)
    # a different scale for layer 2 (the maxima of another layer) changes the field
    y3 = nn.field(net2, ref, rnd=nn.fp8_inference_operands(net2, M))
    assert not np.array_equal(y1, y3)
    # and the emulated error is an E4M3 error: well above BF16's, well below O(1)
    y = nn.field(net, ref)
    rel = np.linalg.norm(y1 - y) / np.linalg.norm(y)
    rel16 = np.linalg.norm(nn.field(net, ref, rnd=nn.bf16_inference_operands()) - y) / \
        np.linalg.norm(y)
    assert 2 * rel16 < rel < 0.2


def test_fp8_decoder_operands():
    """The cached-latent FP8 mode rounds the encoder exactly as the BF16 inference
    path (same latents bit for bit) and only the decoder to E4M3: its field error
    lies between the BF16 path's and the all-E4M3 path's."""
    cfg = gen.CONFIGS["tiny"]
    lay = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz)
    net = nn.Net(gen.make_net_params(lay, seed=2333, grid_scale=0.5, bias_scale=0.1),
                 (cfg.nx, cfg.ny, cfg.nz), lay.res)
    M = nn.fp8_activation_maxima(net)
    dec = nn.fp8_decoder_operands(net, M)
    b16 = nn.bf16_inference_operands()
    u = nn.vertex_positions(np.arange(cfg.n_vertices), (cfg.nx, cfg.ny, cfg.nz))
    h0 = nn.input_embedding(net, 0, u, b16)
    np.testing.assert_array_equal(nn.encoder(net, 0, h0, dec)["lat"],
                                  nn.encoder(net, 0, h0, b16)["lat"])
    y = nn.field(net, cfg.ref_v)
    err = {k: np.linalg.norm(nn.field(net, cfg.ref_v, rnd=o) - y) / np.linalg.norm(y)
           for k, o in (("bf16", b16), ("dec", dec), ("fp8", nn.fp8_inference_operands(net, M)))}
    assert err["bf16"] < err["dec"] < err["fp8"], err


def test_unrounded_operands_reproduce_the_fp64_oracle():
    """An Operands whose every rounding is the identity gives the plain FP64 network
    and gradients bit for bit, so the rounding hooks change no arithmetic."""
    ident = lambda x, layer=0: np.asarray(x, dtype=np.float64)  # noqa: E731
    I = nn.Operands(act=ident, weight=ident, grad=ident, latent=None)
    for n_enc in (1, 2):
        L = _layout(n_enc=n_enc)
        net = _net(gen.make_net_params(L, seed=9, grid_scale=0.5, bias_scale=0.1), n_enc=n_enc)
        V = DIMS[0] * DIMS[1] * DIMS[2]
        pairs = gen.random_pairs(V, 300, seed=3)
        t = np.linspace(-1, 1, 300)
        l0, g0, y0 = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], t)
        l1, g1, y1 = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], t, I)
        assert l0 == l1
        np.testing.assert_array_equal(y0, y1)
        np.testing.assert_array_equal(g0.flat, g1.flat)


def test_bf16_operand_rounding_floor():
    """The error that bf16 operands alone cause in the learned field's outputs and
    gradients (the floor a BF16 MFMA implementation is held to): forward outputs
    within a few 1e-3 relative L2, gradients within about 1e-1 per tensor.  Rounding
    the gradient operand contributes little (<= 5e-3); the forward weights and
    activations dominate, through the ReLU masks they flip and, for gradients that
    are sums of terms of both signs, through cancellation."""
    cfg = gen.CONFIGS["tiny"]
    lay = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz)
    net = nn.Net(gen.make_net_params(lay, seed=2321, grid_scale=0.5, bias_scale=0.1),
                 (cfg.nx, cfg.ny, cfg.nz), lay.res)
    pairs = gen.random_pairs(cfg.n_vertices, 2048, seed=12)
    y, _ = nn.forward(net, pairs[:, 0], pairs[:, 1])
    ye, _ = nn.forward(net, pairs[:, 0], pairs[:, 1], nn.Operands())
    rel_y = np.linalg.norm(ye - y) / np.linalg.norm(y)
    assert 1e-4 < rel_y < 1e-2
    s = np.where(np.random.default_rng(5).random(len(pairs)) < 0.5, -1.0, 1.0)
    t = y - s
    _, g0, _ = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], t)
    _, gb, _ = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], t, nn.Operands())
    ident = lambda x, layer=0: np.asarray(x, dtype=np.float64)  # noqa: E731
    _, gg, _ = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], t,
                                nn.Operands(act=ident, weight=ident))
    for name, _shape in lay.tensors():
        b = lay.view(g0.flat, name)
        nb = np.linalg.norm(b)
        if nb == 0:
            continue
        rel_all = np.linalg.norm(lay.view(gb.flat, name) - b) / nb
        rel_g = np.linalg.norm(lay.view(gg.flat, name) - b) / nb
        assert rel_all < 0.15, name
        assert rel_g < 5e-3, name


def test_grid_only_is_the_full_network_with_an_identity_encoder():
    """The grid-only network (encoder MLP omitted, Sec. 6.3) equals a full network
    whose encoder passes the grid features through unchanged: W1 = [I; -I; 0]
    (so h1 = [relu(h0), relu(-h0)]), W2 = I on those 64 units, W3 = [I, -I] into
    the first 32 latent units (relu(a) - relu(-a) = a exactly), and W4 of the
    full network = the grid-only W4 on those units.  Outputs and the gradients of
    the shared parameters (grids and decoder) agree."""
    width, K = 128, 32
    Lg = _layout(width=width, grid_only=True)
    Lf = _layout(width=width)
    fg = gen.make_net_params(Lg, seed=21, grid_scale=0.5, bias_scale=0.2).astype(np.float64)
    ng = _net(fg, width=width, grid_only=True)
    nf = _net(np.zeros(Lf.n_floats), width=width)
    for l in range(4):
        nf[("grid", 0, l)] = ng[("grid", 0, l)]
    W1 = np.zeros((width, K))
    W1[:K] = np.eye(K)
    W1[K:2 * K] = -np.eye(K)
    W2 = np.zeros((width, width))
    W2[:2 * K, :2 * K] = np.eye(2 * K)
    W3 = np.zeros((width, width))
    W3[:K, :K] = np.eye(K)
    W3[:K, K:2 * K] = -np.eye(K)
    W4 = np.zeros((width, width))
    W4[:, :K] = ng["W4"]
    nf[("W1", 0)], nf[("W2", 0)], nf[("W3", 0)], nf["W4"] = W1, W2, W3, W4
    for name in ("b4", "W5", "b5", "w6", "b6"):
        nf[name] = ng[name]
    V = DIMS[0] * DIMS[1] * DIMS[2]
    pairs = gen.random_pairs(V, 200, seed=4)
    yg, _ = nn.forward(ng, pairs[:, 0], pairs[:, 1])
    yf, _ = nn.forward(nf, pairs[:, 0], pairs[:, 1])
    np.testing.assert_allclose(yg, yf, rtol=1e-12, atol=1e-12)
    t = yg - 1.0
    _, gg, _ = nn.loss_and_grad(ng, pairs[:, 0], pairs[:, 1], t)
    _, gf, _ = nn.loss_and_grad(nf, pairs[:, 0], pairs[:, 1], t)
    for l in range(4):
        np.testing.assert_allclose(gg[("grid", 0, l)], gf[("grid", 0, l)], rtol=1e-9,
                                   atol=1e-12)
    np.testing.assert_allclose(gg["W4"], gf["W4"][:, :K], rtol=1e-9, atol=1e-12)
    for name in ("b4", "W5", "b5", "w6", "b6"):
        np.testing.assert_allclose(gg[name], gf[name], rtol=1e-9, atol=1e-12)
