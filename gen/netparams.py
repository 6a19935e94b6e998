"""Network shape presets and seeded initial parameters for the learned field.

Flat FP32 parameter layout (the format the C library documents for
``ndf_net_param_bytes``): for each encoder e in 0..n_enc-1 (n_enc = 1 when the
reference and query share one encoder and grid, Sec. 4.1, else 2; a grid-only
network, the ablation of Sec. 6.3 with the encoder MLP omitted, has no W1..b3
and its W4 is float[H][L*F]):

    grid_e level l, l = 0..L-1 : float[cells_l][F]   cells_l = Rx*Ry*Rz, cell = x + Rx*(y + Ry*z),
                                 or cells_l = 2^T for a level hashed into a table of
                                 2^T cells (T = log2_hashmap > 0, Rx*Ry*Rz > 2^T)
    W1_e float[H][L*F], b1_e float[H]
    W2_e float[H][H],   b2_e float[H]
    W3_e float[H][H],   b3_e float[H]
then the shared decoder
    W4 float[H][H], b4 float[H], W5 float[H][H], b5 float[H], w6 float[H], b6 float[1]

Every tensor starts at a multiple of 64 floats; the gaps are zero.  Weight
matrices are row-major [out][in].
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np

ALIGN = 64


def level_resolutions(nx, ny, nz, n_levels=4):
    """Per-axis sizes growing geometrically from ~dims/4 to the data grid."""
    top = (nx, ny, nz)
    base = tuple(max(2, n // 4) for n in top)
    out = []
    for l in range(n_levels):
        t = l / (n_levels - 1)
        out.append(tuple(max(2, int(math.floor(b * (n / b) ** t + 0.5)))
                         for b, n in zip(base, top)))
    return out


@dataclass(frozen=True)
class NetLayout:
    nx: int
    ny: int
    nz: int
    res: tuple            # ((Rx,Ry,Rz),) * n_levels
    feats: int = 8
    width: int = 128
    n_enc: int = 1        # 1: shared encoder + grid (self field), 2: separate
    log2_hashmap: int = 0  # T > 0: levels larger than 2^T cells are hash tables of 2^T
    grid_only: bool = False  # encoder MLP omitted: the latent is the grid features
    fourier: int = 0      # L > 0: raw position and L Fourier frequencies appended to the
                          # encoder input, padded to a multiple of 16

    @staticmethod
    def for_grid(nx, ny, nz, n_levels=4, feats=8, width=128, n_enc=1, log2_hashmap=0,
                 grid_only=False, fourier=0):
        return NetLayout(nx, ny, nz, tuple(level_resolutions(nx, ny, nz, n_levels)),
                         feats, width, n_enc, log2_hashmap, grid_only, fourier)

    @property
    def enc_in(self):
        """Encoder input width: L*F grid features (+ 3 + 6 fourier, padded to 16)."""
        n = self.n_levels * self.feats
        if not self.fourier:
            return n
        return (n + 3 + 6 * self.fourier + 15) // 16 * 16

    def cells(self, l):
        rx, ry, rz = self.res[l]
        dense = rx * ry * rz
        T = self.log2_hashmap
        return (1 << T) if T and dense > (1 << T) else dense

    @property
    def n_levels(self):
        return len(self.res)

    def tensors(self):
        """[(name, shape)] in storage order."""
        H, F, L = self.width, self.feats, self.n_levels
        out = []
        for e in range(self.n_enc):
            for l in range(self.n_levels):
                out.append((f"grid{e}_{l}", (self.cells(l), F)))
            if not self.grid_only:
                out += [(f"W1_{e}", (H, self.enc_in)), (f"b1_{e}", (H,)),
                        (f"W2_{e}", (H, H)), (f"b2_{e}", (H,)),
                        (f"W3_{e}", (H, H)), (f"b3_{e}", (H,))]
        out += [("W4", (H, L * F if self.grid_only else H)), ("b4", (H,)), ("W5", (H, H)),
                ("b5", (H,)), ("w6", (H,)), ("b6", (1,))]
        return out

    def offsets(self):
        off = {}
        pos = 0
        for name, shape in self.tensors():
            off[name] = (pos, shape)
            n = int(np.prod(shape))
            pos += (n + ALIGN - 1) // ALIGN * ALIGN
        return off, pos

    @property
    def n_floats(self):
        return self.offsets()[1]

    def view(self, flat, name):
        off, _ = self.offsets()
        o, shape = off[name]
        return flat[o:o + int(np.prod(shape))].reshape(shape)


SEED_NET = 2320


def make_net_params(layout: NetLayout, seed: int = SEED_NET, grid_scale: float = 1e-4,
                    bias_scale: float = 0.0) -> np.ndarray:
    """He-uniform MLP weights, grid features U(-grid_scale, grid_scale), biases
    U(-bias_scale, bias_scale); float32 flat array in the layout above."""
    rng = np.random.default_rng(seed)
    flat = np.zeros(layout.n_floats, dtype=np.float32)
    off, _ = layout.offsets()
    for name, shape in layout.tensors():
        o, _ = off[name]
        n = int(np.prod(shape))
        if name.startswith("grid"):
            vals = rng.uniform(-grid_scale, grid_scale, n)
        elif name[0] in "Ww":
            fan_in = shape[-1]
            a = math.sqrt(6.0 / fan_in)
            vals = rng.uniform(-a, a, n)
        else:
            vals = rng.uniform(-bias_scale, bias_scale, n) if bias_scale else np.zeros(n)
        flat[o:o + n] = vals.astype(np.float32)
    return flat
