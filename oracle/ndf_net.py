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
* L1 loss gradient uses sign(y - t) with sign(0) = 0.

The flat parameter layout is parsed here from its documented description (each
tensor at a multiple of 64 floats, order: per encoder its grid levels then
W1,b1,W2,b2,W3,b3; then W4,b4,W5,b5,w6,b6).
"""
from __future__ import annotations

import numpy as np

ALIGN = 64


class Net:
    """Named float64 views over a copy of a flat parameter vector."""

    def __init__(self, flat, dims, res, feats=8, width=128, n_enc=1, log2_hashmap=0):
        self.nx, self.ny, self.nz = dims
        self.res = [tuple(r) for r in res]
        self.T = log2_hashmap
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
            take(("W1", e), (width, L * feats))
            take(("b1", e), (width,))
            take(("W2", e), (width, width))
            take(("b2", e), (width,))
            take(("W3", e), (width, width))
            take(("b3", e), (width,))
        for name, shape in (("W4", (width, width)), ("b4", (width,)), ("W5", (width, width)),
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


def grid_encode(net, e, u):
    """Concatenated per-level trilinear features h0 (n, L*F)."""
    parts = []
    for l, R in enumerate(net.res):
        idx, w = trilinear(u, R, net.T)
        g = net[("grid", e, l)]
        parts.append(np.einsum("nc,ncf->nf", w, g[idx]))
    return np.concatenate(parts, axis=1)


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


def encoder(net, e, h0):
    a1 = h0 @ net[("W1", e)].T + net[("b1", e)]
    h1 = relu(a1)
    a2 = h1 @ net[("W2", e)].T + net[("b2", e)]
    h2 = relu(a2)
    lat = h2 @ net[("W3", e)].T + net[("b3", e)]
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


def forward(net, v1, v2):
    """Phi(p1, p2) for vertex pairs; returns (y, cache)."""
    dims = (net.nx, net.ny, net.nz)
    return forward_unit(net, vertex_positions(v1, dims), vertex_positions(v2, dims))


def forward_unit(net, u1, u2):
    """Phi(p1, p2) for positions given as u in [0,1]^3 (n,3); returns (y, cache)."""
    ea, eb = _enc_index(net, 0), _enc_index(net, 1)
    A = encoder(net, ea, grid_encode(net, ea, u1))
    B = encoder(net, eb, grid_encode(net, eb, u2))
    m = A["lat"] * B["lat"]
    a4 = m @ net["W4"].T + net["b4"]
    d1 = relu(a4)
    a5 = d1 @ net["W5"].T + net["b5"]
    d2 = relu(a5)
    y = d2 @ net["w6"] + net["b6"][0]
    return y, {"u1": u1, "u2": u2, "A": A, "B": B, "m": m, "a4": a4, "d1": d1, "a5": a5,
               "d2": d2, "y": y}


def field(net, ref_v, dims_v=None):
    """phi(p) = Phi(p_ref, p) at every grid vertex (Sec. 5)."""
    V = net.nx * net.ny * net.nz
    v = np.arange(V, dtype=np.int64) if dims_v is None else np.asarray(dims_v)
    y, _ = forward(net, np.full(v.shape, ref_v, dtype=np.int64), v)
    return y


def field_points(net, ref_v, pos):
    """Phi(p_ref, p) at continuous positions pos (n,3) in [-1,1]^3, the positions a
    ray marcher samples (Sec. 5)."""
    u2 = domain_to_unit(pos)
    u1 = vertex_positions(np.full(u2.shape[0], ref_v, dtype=np.int64), (net.nx, net.ny, net.nz))
    y, _ = forward_unit(net, u1, u2)
    return y


def l1_loss(y, t):
    return float(np.mean(np.abs(y - t)))


def _encoder_backward(net, e, c, dlat, grads):
    grads[("W3", e)] += dlat.T @ c["h2"]
    grads[("b3", e)] += dlat.sum(0)
    dh2 = dlat @ net[("W3", e)]
    da2 = dh2 * (c["a2"] > 0)
    grads[("W2", e)] += da2.T @ c["h1"]
    grads[("b2", e)] += da2.sum(0)
    dh1 = da2 @ net[("W2", e)]
    da1 = dh1 * (c["a1"] > 0)
    grads[("W1", e)] += da1.T @ c["h0"]
    grads[("b1", e)] += da1.sum(0)
    return da1 @ net[("W1", e)]


def loss_and_grad(net, v1, v2, t):
    """Mean L1 loss (Eq. 3 with d = L1) and its gradient w.r.t. every parameter."""
    dims = (net.nx, net.ny, net.nz)
    return loss_and_grad_unit(net, vertex_positions(v1, dims), vertex_positions(v2, dims), t)


def loss_and_grad_points(net, pos, t):
    """loss_and_grad for pairs of continuous positions pos (B,2,3) in [-1,1]^3
    (the training pairs of Sec. 4.3)."""
    pos = np.asarray(pos, dtype=np.float64)
    return loss_and_grad_unit(net, domain_to_unit(pos[:, 0]), domain_to_unit(pos[:, 1]), t)


def forward_points(net, pos):
    """Phi(p1, p2) for pairs of continuous positions pos (B,2,3)."""
    pos = np.asarray(pos, dtype=np.float64)
    y, _ = forward_unit(net, domain_to_unit(pos[:, 0]), domain_to_unit(pos[:, 1]))
    return y


def loss_and_grad_unit(net, u1, u2, t):
    """loss_and_grad for positions given as u in [0,1]^3."""
    t = np.asarray(t, dtype=np.float64)
    y, c = forward_unit(net, u1, u2)
    n = y.shape[0]
    gy = np.sign(y - t) / n
    g = net.zeros_like()
    g["w6"][:] += c["d2"].T @ gy
    g["b6"][:] += gy.sum()
    dd2 = gy[:, None] * net["w6"][None, :]
    da5 = dd2 * (c["a5"] > 0)
    g["W5"][:] += da5.T @ c["d1"]
    g["b5"][:] += da5.sum(0)
    dd1 = da5 @ net["W5"]
    da4 = dd1 * (c["a4"] > 0)
    g["W4"][:] += da4.T @ c["m"]
    g["b4"][:] += da4.sum(0)
    dm = da4 @ net["W4"]
    dla = dm * c["B"]["lat"]
    dlb = dm * c["A"]["lat"]
    ea, eb = _enc_index(net, 0), _enc_index(net, 1)
    dh0a = _encoder_backward(net, ea, c["A"], dla, g)
    dh0b = _encoder_backward(net, eb, c["B"], dlb, g)
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
