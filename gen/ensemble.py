"""Seeded Gaussian-blob ensembles shaped like the paper's data (Sec. 3, Sec. 6.1).

Data model (Sec. 3): an ensemble of N members, each a scalar field per variable on
an nx*ny*nz grid.  Storage is member-major, ``x[var][member][v]`` in float32 with
``v = i + nx*(j + ny*k)``.

Member field (synthetic stand-in for the paper's weather ensemble, which is not
available):

  s_m(v) = sum_b a_mb * g_b(v),  g_b(i,j,k) = exp(-((i-cx)^2+(j-cy)^2)/(2 sh^2)
                                                 -(k-cz)^2/(2 sz^2))
  x_m(v) = f(s_m(v)) + eta,      f(s) = s + 0.3 s^2 where i < nx/2, else s,
                                 eta ~ N(0, 0.1^2) iid
  second variable (optional): y_m(v) = tanh(sum_b a_mb g'_b(v)) + eta',
                                 g' with both widths scaled by 1.5.

Blob centres are uniform over the index box, amplitudes a_mb ~ N(0,1) iid.

Small ensembles are generated in float64 numpy and rounded once to float32, so
they are bit-identical on every machine.  Paper-sized ensembles (7 GB per
variable) are generated with torch on the requested device in member chunks;
the oracle always consumes the very array the GPU path consumed.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math

import numpy as np

SEED_GEOMETRY = 2307
SEED_AMPLITUDE = 2308
SEED_NOISE = 2309
SEED_NOISE_VAR2 = 2310


@dataclass(frozen=True)
class EnsembleConfig:
    name: str
    n_members: int
    nx: int
    ny: int
    nz: int
    n_blobs: int
    sigma_h: tuple          # U[lo, hi] horizontal width (cells)
    sigma_z: tuple | None   # U[lo, hi] vertical width; None -> isotropic (= sigma_h draw)
    ref: tuple              # reference vertex (i, j, k)
    n_vars: int = 1
    noise_std: float = 0.1
    quad: float = 0.3
    var2_width_scale: float = 1.5

    @property
    def n_vertices(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def ref_v(self) -> int:
        i, j, k = self.ref
        return vertex_index(self, i, j, k)

    def with_members(self, n: int) -> "EnsembleConfig":
        return replace(self, n_members=n)


CONFIGS = {
    # 64 members on 16x16x8, 32 isotropic blobs of width U[1,5], ref (8,8,4)
    "tiny": EnsembleConfig("tiny", 64, 16, 16, 8, 32, (1.0, 5.0), None, (8, 8, 4)),
    # paper-shaped: 1000 members on 250x352x20, 256 blobs, sh U[3,30], sz U[1,4]
    "paper": EnsembleConfig("paper", 1000, 250, 352, 20, 256, (3.0, 30.0), (1.0, 4.0),
                            (125, 176, 10)),
    # paper-shaped with a second, dependent variable
    "paper2v": EnsembleConfig("paper2v", 1000, 250, 352, 20, 256, (3.0, 30.0), (1.0, 4.0),
                              (125, 176, 10), n_vars=2),
    # mid-size case for GPU parity: several tiles of every kernel plus ragged tails
    "mid": EnsembleConfig("mid", 200, 37, 29, 11, 48, (2.0, 8.0), (1.0, 3.0), (18, 14, 5)),
}


def vertex_index(cfg, i, j, k):
    return i + cfg.nx * (j + cfg.ny * k)


def vertex_coords(cfg, v):
    v = np.asarray(v, dtype=np.int64)
    i = v % cfg.nx
    j = (v // cfg.nx) % cfg.ny
    k = v // (cfg.nx * cfg.ny)
    return i, j, k


def blob_geometry(cfg: EnsembleConfig, seed: int = SEED_GEOMETRY):
    """Centres (J,3) in index units and widths (J,) horizontal / vertical."""
    rng = np.random.default_rng(seed)
    J = cfg.n_blobs
    c = np.stack([rng.uniform(0.0, cfg.nx - 1, J),
                  rng.uniform(0.0, cfg.ny - 1, J),
                  rng.uniform(0.0, cfg.nz - 1, J)], axis=1)
    sh = rng.uniform(cfg.sigma_h[0], cfg.sigma_h[1], J)
    if cfg.sigma_z is None:
        sz = sh.copy()
    else:
        sz = rng.uniform(cfg.sigma_z[0], cfg.sigma_z[1], J)
    return c, sh, sz


def amplitudes(cfg: EnsembleConfig, seed: int = SEED_AMPLITUDE):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((cfg.n_members, cfg.n_blobs))


def _profiles(cfg, c, sh, sz, scale=1.0):
    """Separable blob factors gx (J,nx), gy (J,ny), gz (J,nz), float64."""
    i = np.arange(cfg.nx, dtype=np.float64)
    j = np.arange(cfg.ny, dtype=np.float64)
    k = np.arange(cfg.nz, dtype=np.float64)
    sh = sh * scale
    sz = sz * scale
    gx = np.exp(-(i[None, :] - c[:, 0:1]) ** 2 / (2 * sh[:, None] ** 2))
    gy = np.exp(-(j[None, :] - c[:, 1:2]) ** 2 / (2 * sh[:, None] ** 2))
    gz = np.exp(-(k[None, :] - c[:, 2:3]) ** 2 / (2 * sz[:, None] ** 2))
    return gx, gy, gz


def _blob_matrix_np(cfg, scale=1.0):
    c, sh, sz = blob_geometry(cfg)
    gx, gy, gz = _profiles(cfg, c, sh, sz, scale)
    G = gz[:, :, None, None] * gy[:, None, :, None] * gx[:, None, None, :]
    return G.reshape(cfg.n_blobs, cfg.n_vertices)


def _transformed_mask(cfg):
    v = np.arange(cfg.n_vertices)
    return (v % cfg.nx) < (cfg.nx / 2.0)


def _make_small(cfg):
    G = _blob_matrix_np(cfg)
    A = amplitudes(cfg)
    s = A @ G
    quad = _transformed_mask(cfg)
    x = s + np.where(quad[None, :], cfg.quad * s * s, 0.0)
    rng = np.random.default_rng(SEED_NOISE)
    x = x + cfg.noise_std * rng.standard_normal(x.shape)
    out = [x.astype(np.float32)]
    if cfg.n_vars > 1:
        G2 = _blob_matrix_np(cfg, cfg.var2_width_scale)
        rng2 = np.random.default_rng(SEED_NOISE_VAR2)
        y = np.tanh(A @ G2) + cfg.noise_std * rng2.standard_normal(x.shape)
        out.append(y.astype(np.float32))
    return np.stack(out, axis=0)


def _make_large_torch(cfg, device, member_chunk=125):
    import torch
    c, sh, sz = blob_geometry(cfg)
    A = torch.from_numpy(amplitudes(cfg).astype(np.float32)).to(device)
    V = cfg.n_vertices

    def blob_matrix(scale):
        gx, gy, gz = _profiles(cfg, c, sh, sz, scale)
        gx = torch.from_numpy(gx.astype(np.float32)).to(device)
        gy = torch.from_numpy(gy.astype(np.float32)).to(device)
        gz = torch.from_numpy(gz.astype(np.float32)).to(device)
        return (gz[:, :, None, None] * gy[:, None, :, None] * gx[:, None, None, :]).reshape(
            cfg.n_blobs, V)

    quad = torch.from_numpy(_transformed_mask(cfg)).to(device)
    x = torch.empty((cfg.n_vars, cfg.n_members, V), dtype=torch.float32, device=device)
    G = blob_matrix(1.0)
    gen = torch.Generator(device=device)
    gen.manual_seed(SEED_NOISE)
    for m0 in range(0, cfg.n_members, member_chunk):
        m1 = min(cfg.n_members, m0 + member_chunk)
        s = A[m0:m1] @ G
        s = torch.where(quad[None, :], s + cfg.quad * s * s, s)
        s += cfg.noise_std * torch.randn(s.shape, generator=gen, device=device,
                                         dtype=torch.float32)
        x[0, m0:m1] = s
        del s
    del G
    if cfg.n_vars > 1:
        G2 = blob_matrix(cfg.var2_width_scale)
        gen.manual_seed(SEED_NOISE_VAR2)
        for m0 in range(0, cfg.n_members, member_chunk):
            m1 = min(cfg.n_members, m0 + member_chunk)
            y = torch.tanh(A[m0:m1] @ G2)
            y += cfg.noise_std * torch.randn(y.shape, generator=gen, device=device,
                                             dtype=torch.float32)
            x[1, m0:m1] = y
            del y
        del G2
    return x


SMALL_LIMIT = 64_000_000   # members * vertices generated exactly in float64 numpy


def make_ensemble(cfg, device="cpu", as_torch=True):
    """Return the ensemble ``x[n_vars][N][V]`` (float32).

    Small configs are generated in float64 numpy (machine-independent); paper-sized
    ones with torch on ``device``.
    """
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    if cfg.n_members * cfg.n_vertices <= SMALL_LIMIT:
        x = _make_small(cfg)
        if not as_torch:
            return x
        import torch
        return torch.from_numpy(x).to(device)
    if not as_torch:
        return _make_large_torch(cfg, "cpu").numpy()
    return _make_large_torch(cfg, device)


def population_cov(cfg, v, w):
    """Population covariance of variable 0 at vertices v and w (float64 arrays).

    With S(v,w) = sum_b g_b(v) g_b(w) (amplitudes are iid N(0,1)):
      linear at both            cov = S,           var = S + sigma^2
      quadratic at both         cov = S + 2 q^2 S^2 (Isserlis), var = S + 2 q^2 S^2 + sigma^2
      mixed                     cov = S   (odd moments vanish)
    """
    c, sh, sz = blob_geometry(cfg)
    gx, gy, gz = _profiles(cfg, c, sh, sz)
    iv, jv, kv = vertex_coords(cfg, v)
    iw, jw, kw = vertex_coords(cfg, w)
    gv = gx[:, iv] * gy[:, jv] * gz[:, kv]
    gw = gx[:, iw] * gy[:, jw] * gz[:, kw]
    S = np.sum(gv * gw, axis=0)
    qv = iv < cfg.nx / 2.0
    qw = iw < cfg.nx / 2.0
    both = qv & qw
    cov = S + np.where(both, 2 * cfg.quad ** 2 * S * S, 0.0)
    same = np.asarray(v) == np.asarray(w)
    cov = cov + np.where(same, cfg.noise_std ** 2, 0.0)
    return cov


def population_rho(cfg, v, w):
    v = np.asarray(v)
    w = np.asarray(w)
    cvw = population_cov(cfg, v, w)
    cvv = population_cov(cfg, v, v)
    cww = population_cov(cfg, w, w)
    return cvw / np.sqrt(cvv * cww)
