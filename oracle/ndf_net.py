"""FP64 numpy oracle of the learned dependence field (Sec. 4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network (Sec. 4.1, Fig. 2): a position p is embedded by a multi-resolution
feature grid (Sec. 4.2; here dense levels, trilinear lookup), passed through an
encoder MLP to a latent vector; the latents of the two positions are merged by
element-wise multiplication and a decoder MLP maps the product to the dependence
value.  For a self field the two positions share one encoder and grid, so
Phi(p1, p2) = Phi(p2, p1) by construction (Sec. 4.1).  Training minimises the
mean L1 distance to the direct estimates over position pairs (Eq. 3, Sec. 4.3)
with Adam [KB14].

Readings where the paper is silent (the GPU path uses the same ones):
* grid vertex (i,j,k) sits at u = (i/(nx-1), j/(ny-1), k/(nz-1)) in [0,1]^3
  (the paper's p = 2u - 1 in [-1,1]^3, corners aligned);
* level l with sizes R: c = u*(R-1), base = clamp(floor(c), 0, R-2), f = c - base,
  eight corners (dx,dy,dz) weighted by prod(f or 1-f); cell = x + Rx*(y + Ry*z);
* hash grids (Sec. 4.2, T > 0): a level with more than 2^T dense cells is a table
  of 2^T cells indexed by the spatial hash of the encoding the paper uses
  (xor of x*1, y*2654435761, z*805459861, modulo 2^T); smaller levels stay dense
  (the paper's table is large enough that no level of its grids is hashed);
* encoder: 3 layers, ReLU after the first two, linear latent; decoder: two ReLU
  layers and a linear scalar output; weights row-major [out][in];
* Fourier features (Sec. 4.2, Eq. 4; fourier = L > 0): the encoder input is the
  grid features, then the raw position p = 2u - 1 (of the clamped u), then for
  i < L and j in (x, y, z) the pair sin(2^i pi p_j), cos(2^i pi p_j), zero-padded
  to a multiple of 16 inputs (L = 12: 32 + 3 + 72 + 5 = 112); the order of the
  concatenation is a layout choice, this one is the parameter blob's;
* grid-only network (the TensoRF-like ablation of Sec. 6.3, Fig. 6: the encoder
  MLP omitted, predictions from the input embedding alone): the latent of a
  position is its concatenated grid features, so the merge multiplies two
  L*F-vectors and the decoder's first layer is W4[width][L*F];
* L1 loss gradient uses sign(y - t) with sign(0) = 0.

The flat parameter layout is parsed here from its documented description (each
tensor at a multiple of 64 floats, order: per encoder its grid levels then
W1,b1,W2,b2,W3,b3; then W4,b4,W5,b5,w6,b6).
"""
from __future__ import annotations

import numpy as np

ALIGN = 64


def embed_width(grid_features, fourier):
    """Encoder inputs: the grid features, plus 3 raw coordinates and 6 L Fourier
    features padded to a multiple of 16 when fourier = L > 0."""
    if not fourier:
        return grid_features
    n = grid_features + 3 + 6 * fourier
    return (n + 15) // 16 * 16


class Net:
    """Named float64 views over a copy of a flat parameter vector."""

    def __init__(self, flat, dims, res, feats=8, width=128, n_enc=1, log2_hashmap=0,
                 grid_only=False, fourier=0):
        self.nx, self.ny, self.nz = dims
        self.res = [tuple(r) for r in res]
        self.T = log2_hashmap
        self.grid_only = grid_only
        self.fourier = fourier
        self.F = feats
        self.H = width
        self.n_enc = n_enc
        self.flat = np.array(flat, dtype=np.float64)
        self.slices = {}
        pos = 0
        L = len(self.res)

        def take(name, shape):
            nonlocal pos
            n = int(np.prod(shape))
            self.slices[name] = (pos, shape)
            pos += (n + ALIGN - 1) // ALIGN * ALIGN

        for e in range(n_enc):
            for l, R in enumerate(self.res):
                take(("grid", e, l), (level_cells(R, log2_hashmap), feats))
            if grid_only:
                continue
            take(("W1", e), (width, embed_width(L * feats, fourier)))
            take(("b1", e), (width,))
            take(("W2", e), (width, width))
            take(("b2", e), (width,))
            take(("W3", e), (width, width))
            take(("b3", e), (width,))
        w4_in = L * feats if grid_only else width
        for name, shape in (("W4", (width, w4_in)), ("b4", (width,)), ("W5", (width, width)),
                            ("b5", (width,)), ("w6", (width,)), ("b6", (1,))):
            take(name, shape)
        self.n_floats = pos
        assert self.flat.shape[0] == pos, (self.flat.shape, pos)

    def __getitem__(self, key):
        o, shape = self.slices[key]
        return self.flat[o:o + int(np.prod(shape))].reshape(shape)

    def __setitem__(self, key, value):
        o, shape = self.slices[key]
        self.flat[o:o + int(np.prod(shape))] = np.asarray(value, dtype=np.float64).reshape(-1)

    def zeros_like(self):
        g = Net.__new__(Net)
        g.__dict__.update(self.__dict__)
        g.flat = np.zeros_like(self.flat)
        return g


def vertex_positions(v, dims):
    """u in [0,1]^3 of grid vertices v = i + nx*(j + ny*k)."""
    nx, ny, nz = dims
    v = np.asarray(v, dtype=np.int64)
    i = v % nx
    j = (v // nx) % ny
    k = v // (nx * ny)
    return np.stack([i / (nx - 1), j / (ny - 1), k / (nz - 1)], axis=-1).astype(np.float64)


# Primes of the spatial hash of multi-resolution hash grids (Mueller et al. 2022),
# the encoding Sec. 4.2 builds on: one per axis, the first 1 so that x maps to itself.
HASH_PRIMES = (1, 2654435761, 805459861)


def level_hashed(R, T):
    """A level is a hash table of 2^T cells when T > 0 and its dense size exceeds it."""
    return T > 0 and int(np.prod(R)) > (1 << T)


def level_cells(R, T):
    return (1 << T) if level_hashed(R, T) else int(np.prod(R))


def hash_cell(p, T):
    """Spatial hash of integer corners p (n,3): xor over axes of p_a * prime_a,
    modulo 2^T (the primes' products taken modulo 2^64; the low T bits are those
    of the exact integers)."""
    p = np.asarray(p, dtype=np.uint64)
    h = np.zeros(p.shape[0], dtype=np.uint64)
    for a in range(3):
        h ^= p[:, a] * np.uint64(HASH_PRIMES[a])
    return (h & np.uint64((1 << T) - 1)).astype(np.int64)


def trilinear(u, R, T=0):
    """Corner cells (n,8) and weights (n,8) of positions u (n,3) on a level of size
    R; the cells are hashed when the level is a hash table (T > 0)."""
    hashed = level_hashed(R, T)
    R = np.asarray(R, dtype=np.int64)
    c = u * (R - 1)
    base = np.clip(np.floor(c), 0, R - 2).astype(np.int64)
    f = c - base
    idx = np.empty((u.shape[0], 8), dtype=np.int64)
    w = np.empty((u.shape[0], 8), dtype=np.float64)
    for corner in range(8):
        d = np.array([corner & 1, (corner >> 1) & 1, (corner >> 2) & 1])
        p = base + d
        idx[:, corner] = (hash_cell(p, T) if hashed
                          else p[:, 0] + R[0] * (p[:, 1] + R[1] * p[:, 2]))
        w[:, corner] = np.prod(np.where(d == 1, f, 1.0 - f), axis=1)
    return idx, w


def grid_encode(net, e, u, rnd=None):
    """Concatenated per-level trilinear features h0 (n, L*F)."""
    parts = []
    for l, R in enumerate(net.res):
        idx, w = trilinear(u, R, net.T)
        g = net[("grid", e, l)]
        if rnd is not None and rnd.grid is not None:
            g = rnd.grid(g)
        parts.append(np.einsum("nc,ncf->nf", w, g[idx]))
    return np.concatenate(parts, axis=1)


def fourier_features(u, L):
    """Raw positions and their Fourier features (Sec. 4.2, Eq. 4) for u in
    [0,1]^3 (n,3): p = 2u - 1, then sin and cos of omega_i p_j for omega_i =
    2^i pi, i < L, and the three axis-aligned unit vectors n_j."""
    p = 2.0 * np.asarray(u, dtype=np.float64) - 1.0
    cols = [p[:, 0], p[:, 1], p[:, 2]]
    for i in range(L):
        w = (2.0 ** i) * np.pi
        for j in range(3):
            cols.append(np.sin(w * p[:, j]))
            cols.append(np.cos(w * p[:, j]))
    return np.stack(cols, axis=1)


def input_embedding(net, e, u, rnd=None):
    """Encoder input h0 of positions u (n,3): the grid features, with Fourier
    features the raw positions and their Fourier features after them, zero-padded
    to the encoder's input width."""
    h0 = grid_encode(net, e, u, rnd)
    if not net.fourier:
        return h0
    ff = fourier_features(u, net.fourier)
    width = embed_width(h0.shape[1], net.fourier)
    pad = np.zeros((h0.shape[0], width - h0.shape[1] - ff.shape[1]))
    return np.concatenate([h0, ff, pad], axis=1)


def grid_scatter(net, e, u, dh0, grads):
    """Adjoint of grid_encode: add the gradient of h0 into the grid gradients."""
    F = net.F
    for l, R in enumerate(net.res):
        idx, w = trilinear(u, R, net.T)
        g = grads[("grid", e, l)]
        contrib = w[:, :, None] * dh0[:, None, l * F:(l + 1) * F]
        np.add.at(g, idx.reshape(-1), contrib.reshape(-1, F))


def relu(a):
    return np.maximum(a, 0.0)


# ----------------------------------------------------- operand rounding ----
# The network oracle is exact FP64.  To measure how much of a reduced-precision
# implementation's deviation from it is caused by rounding alone, every matrix
# product below takes an optional `rnd` (an Operands instance) that rounds the
# two factors as they enter the product and accumulates in FP64.  With
# rnd=None every product is the plain FP64 product.

def round_bf16(a):
    """Nearest bfloat16 (8 significand bits, ties to even) of float32(a), as float64."""
    x = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    b = x.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def round_split_bf16(a):
    """hi + lo with hi = bf16(a) and lo = bf16(a - hi): a float32 to about 16 bits."""
    a32 = np.asarray(a, dtype=np.float32).astype(np.float64)
    hi = round_bf16(a32)
    return hi + round_bf16(a32 - hi)


E4M3_MAX = 448.0  # largest finite OCP E4M3 value, 1.75 * 2^8


def round_e4m3(a):
    """Nearest OCP E4M3 value (3 significand bits, exponent bias 7, normals down to
    2^-6, subnormal spacing 2^-9; ties to even), saturated at +-448."""
    a = np.asarray(a, dtype=np.float64)
    mag = np.abs(a)
    _, ex = np.frexp(mag)                       # mag = f * 2^ex, f in [0.5, 1)
    e = np.maximum(ex - 1, -6)                  # exponent of the leading bit
    q = np.ldexp(1.0, e - 3)                    # spacing of E4M3 values there
    r = np.minimum(np.round(mag / q) * q, E4M3_MAX)  # np.round: half to even
    return np.where(mag == 0, 0.0, np.copysign(r, a))


def e4m3_scale_exp(m):
    """Smallest e with m / 2^e <= 448 for block maxima m >= 0 (2^-126 for m = 0):
    the power-of-two (E8M0) scale of a microscaling block."""
    m = np.asarray(m, dtype=np.float64)
    _, ex = np.frexp(np.where(m > 0, m, 1.0))
    e = ex - 1 - 8                              # 448 * 2^e >= m for e >= this + 1 at worst
    e = np.where(m > E4M3_MAX * np.ldexp(1.0, e), e + 1, e)
    return np.where(m > 0, np.maximum(e, -126), -126)


def round_mx_e4m3(a, block=32):
    """Microscaled E4M3 along the last axis: every run of `block` values shares the
    power-of-two scale 2^e of e4m3_scale_exp(its max |value|); each value becomes
    2^e * round_e4m3(value / 2^e)."""
    a = np.asarray(a, dtype=np.float64)
    k = a.shape[-1]
    assert k % block == 0
    b = a.reshape(a.shape[:-1] + (k // block, block))
    s = np.ldexp(1.0, e4m3_scale_exp(np.max(np.abs(b), axis=-1)))[..., None]
    return (round_e4m3(b / s) * s).reshape(a.shape)


class Operands:
    """Rounding of the factors of each product, per layer (1..3 encoder, 4..5
    decoder): act(x, layer) for activations entering a forward layer (rows are
    positions, the last axis is the layer's input), weight(W, layer) for W[out][in]
    (both directions), grad(g) for the gradient operand of the adjoint products
    and of the weight and bias gradients (and d2 in the head's weight gradient),
    latent(e) for the two latents before their product and grid(table) for the
    stored grid features (None: unrounded)."""

    def __init__(self, act=None, weight=None, grad=None, latent=None, grid=None):
        bf = lambda x, layer=0: round_bf16(x)  # noqa: E731
        self.act = act or bf
        self.weight = weight or bf
        self.grad = grad or (lambda x: round_bf16(x))
        self.latent = latent
        self.grid = grid


def bf16_inference_operands():
    """The learned-field inference path in BF16: bf16 grid features, every layer's
    operands bf16 and the latents rounded to bf16 before their product."""
    return Operands(latent=round_bf16, grid=round_bf16)


CAL_REFS = 32       # calibration set of the static E4M3 activation scales
CAL_QUERIES = 2048


def calibration_vertices(n, V):
    """n vertices spread evenly over [0, V): (2 i + 1) V / (2 n), i < n (floor)."""
    i = np.arange(n, dtype=np.int64)
    return ((2 * i + 1) * V) // (2 * n)


def fp8_activation_maxima(net):
    """Largest |input| of layers 2..5 (query encoder's h1 and h2, the latent
    product m, the decoder's d1) over the calibration set (CAL_REFS references
    x CAL_QUERIES queries), run through the BF16 inference operands and read
    as the BF16 values those layers pass on."""
    V = net.nx * net.ny * net.nz
    refs = calibration_vertices(CAL_REFS, V)
    qs = calibration_vertices(CAL_QUERIES, V)
    ops = bf16_inference_operands()
    m = np.zeros(4)
    for r in refs:
        _, c = forward(net, np.full(qs.shape, r, dtype=np.int64), qs, ops)
        for i, x in enumerate((c["B"]["h1"], c["B"]["h2"], c["m"], c["d1"])):
            m[i] = max(m[i], float(np.max(np.abs(round_bf16(x)))))
    return m


def fp8_activation_scales(maxima):
    """Static power-of-two scales 2^e of the layer inputs: e the smallest exponent
    with twice the calibrated maximum within E4M3's range (headroom for inputs
    beyond the calibration set, which saturate at +-448 2^e)."""
    return np.ldexp(1.0, e4m3_scale_exp(2.0 * np.asarray(maxima, dtype=np.float64)))


def fp8_inference_operands(net, maxima=None):
    """Inference with the first layer in BF16 and layers 2..5 in E4M3: weights
    microscaled (blocks of 32 inputs per output row), activations with one static
    scale s_l per layer input (fp8_activation_scales of the calibrated maxima):
    x -> s_l round_e4m3(x / s_l), saturating; bf16 grid features, FP32 latents
    (their rounding is far below E4M3's and is not emulated)."""
    s = fp8_activation_scales(fp8_activation_maxima(net) if maxima is None else maxima)

    def act(x, layer):
        if layer == 1:
            return round_bf16(x)
        return s[layer - 2] * round_e4m3(x / s[layer - 2])

    def weight(W, layer):
        return round_bf16(W) if layer == 1 else round_mx_e4m3(W)

    return Operands(act=act, weight=weight, grid=round_bf16)


def fp8_decoder_operands(net, maxima=None):
    """Many fields of one network at FP8 (the query latents cached): the encoder
    in BF16 as in bf16_inference_operands (bf16 latents), the decoder layers 4
    and 5 in E4M3 with the static input scales of fp8_inference_operands and
    microscaled weights."""
    s = fp8_activation_scales(fp8_activation_maxima(net) if maxima is None else maxima)

    def act(x, layer):
        if layer <= 3:
            return round_bf16(x)
        return s[layer - 2] * round_e4m3(x / s[layer - 2])

    def weight(W, layer):
        return round_bf16(W) if layer <= 3 else round_mx_e4m3(W)

    return Operands(act=act, weight=weight, latent=round_bf16, grid=round_bf16)


def _lin(x, W, layer, rnd):
    """x @ W.T with the operands rounded as rnd says for this layer."""
    if rnd is None:
        return x @ W.T
    return rnd.act(x, layer) @ rnd.weight(W, layer).T


def _adj(g, W, layer, rnd):
    """Data adjoint g @ W of a layer."""
    if rnd is None:
        return g @ W
    return rnd.grad(g) @ rnd.weight(W, layer)


def _bgrad(g, rnd):
    """Bias gradient sum_rows g: the weight gradient of a constant input 1, so its
    G operand is rounded like that of the layer's weight gradient."""
    if rnd is None:
        return g.sum(0)
    return rnd.grad(g).sum(0)


def _wgrad(g, x, layer, rnd):
    """Weight gradient g.T @ x of a layer."""
    if rnd is None:
        return g.T @ x
    return rnd.grad(g).T @ rnd.act(x, layer)


def encoder(net, e, h0, rnd=None):
    if net.grid_only:  # the encoder MLP omitted: the latent is the embedding itself
        return {"h0": h0, "lat": h0}
    a1 = _lin(h0, net[("W1", e)], 1, rnd) + net[("b1", e)]
    h1 = relu(a1)
    a2 = _lin(h1, net[("W2", e)], 2, rnd) + net[("b2", e)]
    h2 = relu(a2)
    lat = _lin(h2, net[("W3", e)], 3, rnd) + net[("b3", e)]
    return {"h0": h0, "a1": a1, "h1": h1, "a2": a2, "h2": h2, "lat": lat}


def _enc_index(net, side):
    return 0 if net.n_enc == 1 else side


def domain_to_unit(p):
    """u in [0,1]^3 of positions p (n,3) in the network's domain [-1,1]^3
    (Sec. 4.3): u = (p + 1)/2, coordinates outside the domain clamped to its
    boundary and NaN coordinates mapped to -1 (a reading: the paper only samples
    inside the domain)."""
    p = np.asarray(p, dtype=np.float64)
    u = np.clip((p + 1.0) / 2.0, 0.0, 1.0)
    return np.where(np.isnan(p), 0.0, u)


def forward(net, v1, v2, rnd=None):
    """Phi(p1, p2) for vertex pairs; returns (y, cache)."""
    dims = (net.nx, net.ny, net.nz)
    return forward_unit(net, vertex_positions(v1, dims), vertex_positions(v2, dims), rnd)


def forward_unit(net, u1, u2, rnd=None):
    """Phi(p1, p2) for positions given as u in [0,1]^3 (n,3); returns (y, cache)."""
    ea, eb = _enc_index(net, 0), _enc_index(net, 1)
    A = encoder(net, ea, input_embedding(net, ea, u1, rnd), rnd)
    B = encoder(net, eb, input_embedding(net, eb, u2, rnd), rnd)
    if rnd is not None and rnd.latent is not None:
        m = rnd.latent(A["lat"]) * rnd.latent(B["lat"])
    else:
        m = A["lat"] * B["lat"]
    a4 = _lin(m, net["W4"], 4, rnd) + net["b4"]
    d1 = relu(a4)
    a5 = _lin(d1, net["W5"], 5, rnd) + net["b5"]
    d2 = relu(a5)
    y = d2 @ net["w6"] + net["b6"][0]
    return y, {"u1": u1, "u2": u2, "A": A, "B": B, "m": m, "a4": a4, "d1": d1, "a5": a5,
               "d2": d2, "y": y}


def field(net, ref_v, dims_v=None, rnd=None):
    """phi(p) = Phi(p_ref, p) at every grid vertex (Sec. 5)."""
    V = net.nx * net.ny * net.nz
    v = np.arange(V, dtype=np.int64) if dims_v is None else np.asarray(dims_v)
    y, _ = forward(net, np.full(v.shape, ref_v, dtype=np.int64), v, rnd)
    return y


def field_points(net, ref_v, pos, rnd=None):
    """Phi(p_ref, p) at continuous positions pos (n,3) in [-1,1]^3, the positions a
    ray marcher samples (Sec. 5)."""
    u2 = domain_to_unit(pos)
    u1 = vertex_positions(np.full(u2.shape[0], ref_v, dtype=np.int64), (net.nx, net.ny, net.nz))
    y, _ = forward_unit(net, u1, u2, rnd)
    return y


def l1_loss(y, t):
    return float(np.mean(np.abs(y - t)))


def _encoder_backward(net, e, c, dlat, grads, rnd=None):
    if net.grid_only:
        return dlat
    grads[("W3", e)] += _wgrad(dlat, c["h2"], 3, rnd)
    grads[("b3", e)] += _bgrad(dlat, rnd)
    dh2 = _adj(dlat, net[("W3", e)], 3, rnd)
    da2 = dh2 * (c["a2"] > 0)
    grads[("W2", e)] += _wgrad(da2, c["h1"], 2, rnd)
    grads[("b2", e)] += _bgrad(da2, rnd)
    dh1 = _adj(da2, net[("W2", e)], 2, rnd)
    da1 = dh1 * (c["a1"] > 0)
    grads[("W1", e)] += _wgrad(da1, c["h0"], 1, rnd)
    grads[("b1", e)] += _bgrad(da1, rnd)
    return _adj(da1, net[("W1", e)], 1, rnd)


def loss_and_grad(net, v1, v2, t, rnd=None):
    """Mean L1 loss (Eq. 3 with d = L1) and its gradient w.r.t. every parameter."""
    dims = (net.nx, net.ny, net.nz)
    return loss_and_grad_unit(net, vertex_positions(v1, dims), vertex_positions(v2, dims), t,
                              rnd)


def loss_and_grad_points(net, pos, t, rnd=None):
    """loss_and_grad for pairs of continuous positions pos (B,2,3) in [-1,1]^3
    (the training pairs of Sec. 4.3)."""
    pos = np.asarray(pos, dtype=np.float64)
    return loss_and_grad_unit(net, domain_to_unit(pos[:, 0]), domain_to_unit(pos[:, 1]), t,
                              rnd)


def forward_points(net, pos, rnd=None):
    """Phi(p1, p2) for pairs of continuous positions pos (B,2,3)."""
    pos = np.asarray(pos, dtype=np.float64)
    y, _ = forward_unit(net, domain_to_unit(pos[:, 0]), domain_to_unit(pos[:, 1]), rnd)
    return y


def loss_and_grad_unit(net, u1, u2, t, rnd=None):
    """loss_and_grad for positions given as u in [0,1]^3."""
    t = np.asarray(t, dtype=np.float64)
    y, c = forward_unit(net, u1, u2, rnd)
    n = y.shape[0]
    gy = np.sign(y - t) / n
    g = net.zeros_like()
    # the head's weight gradient takes d2 as a gradient-product operand (the loss
    # gradient gy = +-1/n stays exact)
    g["w6"][:] += (c["d2"] if rnd is None else rnd.grad(c["d2"])).T @ gy
    g["b6"][:] += gy.sum()
    dd2 = gy[:, None] * net["w6"][None, :]
    da5 = dd2 * (c["a5"] > 0)
    g["W5"][:] += _wgrad(da5, c["d1"], 5, rnd)
    g["b5"][:] += _bgrad(da5, rnd)
    dd1 = _adj(da5, net["W5"], 5, rnd)
    da4 = dd1 * (c["a4"] > 0)
    g["W4"][:] += _wgrad(da4, c["m"], 4, rnd)
    g["b4"][:] += _bgrad(da4, rnd)
    dm = _adj(da4, net["W4"], 4, rnd)
    dla = dm * c["B"]["lat"]
    dlb = dm * c["A"]["lat"]
    ea, eb = _enc_index(net, 0), _enc_index(net, 1)
    dh0a = _encoder_backward(net, ea, c["A"], dla, g, rnd)
    dh0b = _encoder_backward(net, eb, c["B"], dlb, g, rnd)
    grid_scatter(net, ea, c["u1"], dh0a, g)
    grid_scatter(net, eb, c["u2"], dh0b, g)
    return l1_loss(y, t), g, y


def adam_update(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step [KB14] (bias-corrected, step counted from 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
