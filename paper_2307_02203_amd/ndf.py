"""Python binding of libndf.so: argument marshalling only.

Every function named ``ndf_*`` here calls the C entry point of the same name
(include/ndf.h) with raw device pointers taken from torch tensors and torch's
current HIP stream; every step of the dependence path runs in the library's
kernels.  PyTorch only provides device memory and streams.  If the library is
not built the import fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np
import torch

_LIB_PATH = Path(__file__).resolve().parent / "libndf.so"

NDF_OK, NDF_E_ARG, NDF_E_WORKSPACE, NDF_E_HIP, NDF_E_UNSUPPORTED = 0, -1, -2, -3, -5
NDF_E_NONFINITE, NDF_E_SCRATCH = -4, -6
NDF_PREC_FP32, NDF_PREC_SPLIT_BF16, NDF_PREC_BF16, NDF_PREC_FP8_E4M3 = 0, 1, 2, 3
NDF_OP_PEARSON_FIELD, NDF_OP_KSG_FIELD, NDF_OP_TRAIN, NDF_OP_INFER, NDF_OP_KSG_PAIRS = 1, 2, 3, 4, 5
NDF_OP_KSG_POINTS, NDF_OP_PREPARE, NDF_OP_INFER_CACHED = 6, 7, 8
NDF_FLAG_NONFINITE, NDF_FLAG_CONSTANT = 1, 2

EXPORTED = [
    "ndf_status_string", "ndf_workspace_bytes", "ndf_prepare", "ndf_pearson_field",
    "ndf_ksg_mi_field", "ndf_pearson_pairs", "ndf_ksg_mi_pairs", "ndf_net_param_bytes",
    "ndf_net_optstate_bytes", "ndf_net_init", "ndf_net_grad", "ndf_net_forward",
    "ndf_train_step", "ndf_net_qparam_bytes", "ndf_net_quantize", "ndf_infer_field",
    "ndf_infer_latent_bytes", "ndf_infer_latents", "ndf_infer_field_cached",
    "ndf_net_swap_encoders", "ndf_infer_points", "ndf_infer_field_difference",
    "ndf_pearson_points", "ndf_net_forward_at", "ndf_net_grad_at", "ndf_train_step_at",
    "ndf_ksg_mi_points", "ndf_ksg_scratch_bytes", "ndf_ksg_mi_field_noalloc",
]


class NdfError(RuntimeError):
    pass


class ndf_ensemble(ctypes.Structure):
    _fields_ = [("n_members", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("n_vars", ctypes.c_int32), ("x", ctypes.c_void_p),
                ("mean", ctypes.c_void_p), ("inv_std", ctypes.c_void_p),
                ("code", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("order", ctypes.c_void_p), ("xt", ctypes.c_void_p)]


class ndf_net_config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("res", (ctypes.c_int32 * 3) * 4),
                ("feats", ctypes.c_int32), ("width", ctypes.c_int32), ("n_enc", ctypes.c_int32),
                ("log2_hashmap", ctypes.c_int32), ("grid_only", ctypes.c_int32),
                ("fourier", ctypes.c_int32)]


_lib = None
_VP, _I32, _I64, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            raise NdfError(f"{_LIB_PATH} is missing: run __graft_entry__.build() or "
                           "python -m paper_2307_02203_amd.build")
        L = ctypes.CDLL(str(_LIB_PATH))
        E, C = ctypes.POINTER(ndf_ensemble), ctypes.POINTER(ndf_net_config)
        sig = {
            "ndf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
            "ndf_workspace_bytes": (_SZ, [_I32, E, C, _I64, _I32]),
            "ndf_prepare": (ctypes.c_int, [E, _VP, _SZ, _VP]),
            "ndf_pearson_field": (ctypes.c_int, [E, _I32, _I32, _VP, _I32, _VP, _I32, _VP, _SZ,
                                                 _VP]),
            "ndf_ksg_mi_field": (ctypes.c_int, [E, _I32, _I32, _VP, _I32, _I32, _VP, _VP, _VP,
                                                _SZ, _VP]),
            "ndf_ksg_scratch_bytes": (_SZ, []),
            "ndf_ksg_mi_field_noalloc": (ctypes.c_int, [E, _I32, _I32, _VP, _I32, _I32, _VP, _VP,
                                                        _VP]),
            "ndf_pearson_pairs": (ctypes.c_int, [E, _I32, _I32, _VP, _I64, _VP, _VP]),
            "ndf_pearson_points": (ctypes.c_int, [E, _I32, _I32, _VP, _I64, _VP, _VP]),
            "ndf_ksg_mi_points": (ctypes.c_int, [E, _I32, _I32, _VP, _I64, _I32, _VP, _VP, _VP,
                                                 _SZ, _VP]),
            "ndf_ksg_mi_pairs": (ctypes.c_int, [E, _I32, _I32, _VP, _I64, _I32, _VP, _VP, _VP,
                                                _SZ, _VP]),
            "ndf_net_param_bytes": (_SZ, [C]),
            "ndf_net_optstate_bytes": (_SZ, [C]),
            "ndf_net_init": (ctypes.c_int, [C, _VP, _VP, ctypes.c_uint64, _VP]),
            "ndf_net_grad": (ctypes.c_int, [C, _VP, _VP, _VP, _I64, _VP, _VP, _VP, _SZ, _VP]),
            "ndf_net_forward": (ctypes.c_int, [C, _VP, _VP, _I64, _VP, _VP, _SZ, _VP]),
            "ndf_net_grad_at": (ctypes.c_int, [C, _VP, _VP, _VP, _I64, _VP, _VP, _VP, _SZ, _VP]),
            "ndf_net_forward_at": (ctypes.c_int, [C, _VP, _VP, _I64, _VP, _VP, _SZ, _VP]),
            "ndf_train_step_at": (ctypes.c_int, [C, _VP, _VP, _I64, _VP, _VP, _I64,
                                                 ctypes.c_float, _VP, _VP, _SZ, _VP]),
            "ndf_train_step": (ctypes.c_int, [C, _VP, _VP, _I64, _VP, _VP, _I64, ctypes.c_float,
                                              _VP, _VP, _SZ, _VP]),
            "ndf_net_qparam_bytes": (_SZ, [C, _I32]),
            "ndf_net_quantize": (ctypes.c_int, [C, _VP, _I32, _VP, _VP]),
            "ndf_infer_field": (ctypes.c_int, [C, _VP, _I32, _VP, _I32, _VP, _VP, _SZ, _VP]),
            "ndf_infer_latent_bytes": (_SZ, [C]),
            "ndf_infer_latents": (ctypes.c_int, [C, _VP, _VP, _VP]),
            "ndf_infer_field_cached": (ctypes.c_int, [C, _VP, _VP, _I32, _VP, _VP, _VP, _SZ,
                                                      _VP]),
            "ndf_net_swap_encoders": (ctypes.c_int, [C, _VP, _VP, _VP]),
            "ndf_infer_points": (ctypes.c_int, [C, _VP, _I32, _VP, _I32, _VP, _I64, _VP, _VP,
                                                _SZ, _VP]),
            "ndf_infer_field_difference": (ctypes.c_int, [C, _VP, _I64, _I64, _VP, _VP, _VP,
                                                          _SZ, _VP]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int, name: str):
    if status != NDF_OK:
        raise NdfError(f"{name}: {lib().ndf_status_string(status).decode()} ({status})")


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _host_i64(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int64).reshape(-1))
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _ws(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ------------------------------------------------------------------ ensemble --
class Ensemble:
    """Device ensemble x[n_vars][N][V] (float32, member-major) plus the per-vertex
    statistics, KSG codes, (with orders=True) per-vertex sorted member orders and
    (with transposed=True) the vertex-major copy of x that ndf_prepare fills in."""

    def __init__(self, x: torch.Tensor, nx: int, ny: int, nz: int, orders: bool = True,
                 transposed: bool = False):
        if x.dim() == 2:
            x = x.unsqueeze(0)
        assert x.dtype == torch.float32 and x.is_contiguous()
        n_vars, N, V = x.shape
        assert V == nx * ny * nz
        dev = x.device
        self.x = x
        self.nx, self.ny, self.nz = nx, ny, nz
        self.n_members, self.n_vertices, self.n_vars = N, V, n_vars
        self.mean = torch.empty((n_vars, V), dtype=torch.float64, device=dev)
        self.inv_std = torch.empty((n_vars, V), dtype=torch.float64, device=dev)
        self.code = torch.empty((n_vars, V, N), dtype=torch.int32, device=dev)
        self.flags = torch.empty((n_vars, V), dtype=torch.int32, device=dev)
        # uint16 member indices, held in an int16 tensor
        self.order = (torch.empty((n_vars, V, N), dtype=torch.int16, device=dev)
                      if orders else None)
        self.xt = (torch.empty((n_vars, V, N), dtype=torch.float32, device=dev)
                   if transposed else None)
        self.c = ndf_ensemble(N, nx, ny, nz, n_vars, x.data_ptr(), self.mean.data_ptr(),
                              self.inv_std.data_ptr(), self.code.data_ptr(),
                              self.flags.data_ptr(),
                              self.order.data_ptr() if orders else None,
                              self.xt.data_ptr() if transposed else None)

    @property
    def device(self):
        return self.x.device


def ndf_workspace_bytes(op, ens=None, net=None, n=1, prec=0) -> int:
    e = ctypes.byref(ens.c) if ens is not None else None
    c = ctypes.byref(net) if net is not None else None
    return int(lib().ndf_workspace_bytes(op, e, c, int(n), int(prec)))


def ndf_prepare(ens: Ensemble, ws=None, stream=None):
    """ws (optional uint8 device tensor): receives the device status word."""
    n = 0 if ws is None else ws.numel()
    _check(lib().ndf_prepare(ctypes.byref(ens.c), _p(ws), n, _stream(stream)), "ndf_prepare")


def status_word(ws) -> int:
    """The device status word at the start of a call's workspace (after a sync)."""
    return int(ws[:4].view(torch.int32).item())


def ndf_pearson_field(ens, var_ref, var_qry, ref_v, out, prec, ws, stream=None):
    refs, rp = _host_i64(ref_v)
    _check(lib().ndf_pearson_field(ctypes.byref(ens.c), var_ref, var_qry, rp, len(refs),
                                   _p(out), prec, _p(ws), ws.numel(), _stream(stream)),
           "ndf_pearson_field")


def ndf_ksg_mi_field(ens, var_ref, var_qry, ref_v, k, out, counts, ws, stream=None):
    refs, rp = _host_i64(ref_v)
    _check(lib().ndf_ksg_mi_field(ctypes.byref(ens.c), var_ref, var_qry, rp, len(refs), k,
                                  _p(out), _p(counts), _p(ws), ws.numel(), _stream(stream)),
           "ndf_ksg_mi_field")


def ndf_ksg_scratch_bytes() -> int:
    return int(lib().ndf_ksg_scratch_bytes())


def ndf_ksg_mi_field_noalloc(ens, var_ref, var_qry, ref_v, k, out, counts, stream=None):
    refs, rp = _host_i64(ref_v)
    _check(lib().ndf_ksg_mi_field_noalloc(ctypes.byref(ens.c), var_ref, var_qry, rp, len(refs),
                                          k, _p(out), _p(counts), _stream(stream)),
           "ndf_ksg_mi_field_noalloc")


def ndf_pearson_pairs(ens, var_a, var_b, pairs, out, stream=None):
    _check(lib().ndf_pearson_pairs(ctypes.byref(ens.c), var_a, var_b, _p(pairs), pairs.shape[0],
                                   _p(out), _stream(stream)), "ndf_pearson_pairs")


def ndf_ksg_mi_pairs(ens, var_a, var_b, pairs, k, out, counts, ws, stream=None):
    _check(lib().ndf_ksg_mi_pairs(ctypes.byref(ens.c), var_a, var_b, _p(pairs), pairs.shape[0],
                                  k, _p(out), _p(counts), _p(ws), ws.numel(), _stream(stream)),
           "ndf_ksg_mi_pairs")


# Allocating conveniences used by tests, smoke and the benchmark.
def pearson_field(ens, ref_v, prec=NDF_PREC_FP32, var_ref=0, var_qry=0, stream=None):
    refs = np.atleast_1d(np.asarray(ref_v, dtype=np.int64))
    out = torch.empty((len(refs), ens.n_vertices), dtype=torch.float32, device=ens.device)
    ws = _ws(ndf_workspace_bytes(NDF_OP_PEARSON_FIELD, ens, None, len(refs), prec), ens.device)
    ndf_pearson_field(ens, var_ref, var_qry, refs, out, prec, ws, stream)
    return out


def ksg_field(ens, ref_v, k=4, counts=False, var_ref=0, var_qry=0, stream=None):
    refs = np.atleast_1d(np.asarray(ref_v, dtype=np.int64))
    out = torch.empty((len(refs), ens.n_vertices), dtype=torch.float32, device=ens.device)
    cnt = None
    if counts:
        cnt = torch.empty((len(refs), ens.n_vertices, 2, ens.n_members), dtype=torch.int32,
                          device=ens.device)
    ws = _ws(ndf_workspace_bytes(NDF_OP_KSG_FIELD, ens, None, len(refs), 0), ens.device)
    ndf_ksg_mi_field(ens, var_ref, var_qry, refs, k, out, cnt, ws, stream)
    return (out, cnt) if counts else out


def pearson_pairs(ens, pairs, var_a=0, var_b=0, stream=None):
    pairs = torch.as_tensor(pairs, dtype=torch.int64, device=ens.device).contiguous()
    out = torch.empty(pairs.shape[0], dtype=torch.float32, device=ens.device)
    ndf_pearson_pairs(ens, var_a, var_b, pairs, out, stream)
    return out


def ndf_pearson_points(ens, var_a, var_b, pos, out, stream=None):
    _check_pos_pairs(pos, "ndf_pearson_points")
    if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() < pos.shape[0]:
        raise NdfError("ndf_pearson_points: out must be a contiguous float32 [B] tensor")
    _check(lib().ndf_pearson_points(ctypes.byref(ens.c), var_a, var_b, _p(pos), pos.shape[0],
                                    _p(out), _stream(stream)), "ndf_pearson_points")


def pearson_points(ens, pos, var_a=0, var_b=0, stream=None):
    """r between the interpolated samples at pos[b][0] and pos[b][1] ([-1, 1]^3)."""
    pos = torch.as_tensor(pos, dtype=torch.float32, device=ens.device).contiguous()
    out = torch.empty(pos.shape[0], dtype=torch.float32, device=ens.device)
    ndf_pearson_points(ens, var_a, var_b, pos, out, stream)
    return out


def ndf_ksg_mi_points(ens, var_a, var_b, pos, k, out, counts, ws, stream=None):
    _check_pos_pairs(pos, "ndf_ksg_mi_points")
    if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() < pos.shape[0]:
        raise NdfError("ndf_ksg_mi_points: out must be a contiguous float32 [B] tensor")
    _check(lib().ndf_ksg_mi_points(ctypes.byref(ens.c), var_a, var_b, _p(pos), pos.shape[0], k,
                                   _p(out), _p(counts), _p(ws), ws.numel(), _stream(stream)),
           "ndf_ksg_mi_points")


def ksg_points(ens, pos, k=4, counts=False, var_a=0, var_b=0, stream=None):
    """KSG MI between the interpolated samples at pos[b][0] and pos[b][1]."""
    pos = torch.as_tensor(pos, dtype=torch.float32, device=ens.device).contiguous()
    B = pos.shape[0]
    out = torch.empty(B, dtype=torch.float32, device=ens.device)
    cnt = (torch.empty((B, 2, ens.n_members), dtype=torch.int32, device=ens.device)
           if counts else None)
    ws = _ws(ndf_workspace_bytes(NDF_OP_KSG_POINTS, ens, None, max(B, 1), 0), ens.device)
    ndf_ksg_mi_points(ens, var_a, var_b, pos, k, out, cnt, ws, stream)
    return (out, cnt) if counts else out


def ksg_pairs(ens, pairs, k=4, counts=False, var_a=0, var_b=0, stream=None):
    pairs = torch.as_tensor(pairs, dtype=torch.int64, device=ens.device).contiguous()
    out = torch.empty(pairs.shape[0], dtype=torch.float32, device=ens.device)
    cnt = None
    if counts:
        cnt = torch.empty((pairs.shape[0], 2, ens.n_members), dtype=torch.int32,
                          device=ens.device)
    ws = _ws(ndf_workspace_bytes(NDF_OP_KSG_PAIRS, ens, None, 1, 0), ens.device)
    ndf_ksg_mi_pairs(ens, var_a, var_b, pairs, k, out, cnt, ws, stream)
    return (out, cnt) if counts else out


# ------------------------------------------------------------------- network --
def net_config(nx, ny, nz, res, n_enc=1, feats=8, width=128, log2_hashmap=0, grid_only=False,
               fourier=0):
    c = ndf_net_config()
    c.nx, c.ny, c.nz = nx, ny, nz
    c.n_levels = len(res)
    for l, r in enumerate(res):
        for a in range(3):
            c.res[l][a] = int(r[a])
    c.feats, c.width, c.n_enc = feats, width, n_enc
    c.log2_hashmap = log2_hashmap
    c.grid_only = 1 if grid_only else 0
    c.fourier = int(fourier)
    return c


def ndf_net_param_bytes(cfg) -> int:
    return int(lib().ndf_net_param_bytes(ctypes.byref(cfg)))


def ndf_net_optstate_bytes(cfg) -> int:
    return int(lib().ndf_net_optstate_bytes(ctypes.byref(cfg)))


def ndf_net_qparam_bytes(cfg, prec) -> int:
    return int(lib().ndf_net_qparam_bytes(ctypes.byref(cfg), prec))


def ndf_net_init(cfg, params, opt_state, seed, stream=None):
    _check(lib().ndf_net_init(ctypes.byref(cfg), _p(params), _p(opt_state), seed,
                              _stream(stream)), "ndf_net_init")


def ndf_net_grad(cfg, params, pairs, targets, grad_out, loss_out, ws, stream=None):
    _check(lib().ndf_net_grad(ctypes.byref(cfg), _p(params), _p(pairs), _p(targets),
                              pairs.shape[0], _p(grad_out), _p(loss_out), _p(ws), ws.numel(),
                              _stream(stream)), "ndf_net_grad")


def ndf_net_forward(cfg, params, pairs, y, ws, stream=None):
    _check(lib().ndf_net_forward(ctypes.byref(cfg), _p(params), _p(pairs), pairs.shape[0],
                                 _p(y), _p(ws), ws.numel(), _stream(stream)), "ndf_net_forward")


def ndf_train_step(cfg, params, opt_state, step, pairs, targets, lr, loss_out, ws, stream=None):
    _check(lib().ndf_train_step(ctypes.byref(cfg), _p(params), _p(opt_state), int(step),
                                _p(pairs), _p(targets), pairs.shape[0], float(lr), _p(loss_out),
                                _p(ws), ws.numel(), _stream(stream)), "ndf_train_step")


def _check_pos_pairs(pos, name):
    if pos.dim() != 3 or tuple(pos.shape[1:]) != (2, 3) or pos.dtype != torch.float32 \
            or not pos.is_contiguous():
        raise NdfError(f"{name}: pos must be a contiguous float32 [B][2][3] tensor")


def ndf_net_grad_at(cfg, params, pos, targets, grad_out, loss_out, ws, stream=None):
    _check_pos_pairs(pos, "ndf_net_grad_at")
    _check(lib().ndf_net_grad_at(ctypes.byref(cfg), _p(params), _p(pos), _p(targets),
                                 pos.shape[0], _p(grad_out), _p(loss_out), _p(ws), ws.numel(),
                                 _stream(stream)), "ndf_net_grad_at")


def ndf_net_forward_at(cfg, params, pos, y, ws, stream=None):
    _check_pos_pairs(pos, "ndf_net_forward_at")
    _check(lib().ndf_net_forward_at(ctypes.byref(cfg), _p(params), _p(pos), pos.shape[0],
                                    _p(y), _p(ws), ws.numel(), _stream(stream)),
           "ndf_net_forward_at")


def ndf_train_step_at(cfg, params, opt_state, step, pos, targets, lr, loss_out, ws, stream=None):
    _check_pos_pairs(pos, "ndf_train_step_at")
    _check(lib().ndf_train_step_at(ctypes.byref(cfg), _p(params), _p(opt_state), int(step),
                                   _p(pos), _p(targets), pos.shape[0], float(lr), _p(loss_out),
                                   _p(ws), ws.numel(), _stream(stream)), "ndf_train_step_at")


def ndf_net_swap_encoders(cfg, params, params_out, stream=None):
    _check(lib().ndf_net_swap_encoders(ctypes.byref(cfg), _p(params), _p(params_out),
                                       _stream(stream)), "ndf_net_swap_encoders")


def ndf_net_quantize(cfg, params, prec, qparams, stream=None):
    _check(lib().ndf_net_quantize(ctypes.byref(cfg), _p(params), prec, _p(qparams),
                                  _stream(stream)), "ndf_net_quantize")


def ndf_infer_field(cfg, qparams, prec, ref_v, out, ws, stream=None):
    refs, rp = _host_i64(ref_v)
    _check(lib().ndf_infer_field(ctypes.byref(cfg), _p(qparams), prec, rp, len(refs), _p(out),
                                 _p(ws), ws.numel(), _stream(stream)), "ndf_infer_field")


def train_ws_bytes(cfg, B):
    return ndf_workspace_bytes(NDF_OP_TRAIN, None, cfg, B, 0)


def ndf_infer_latent_bytes(cfg):
    return int(lib().ndf_infer_latent_bytes(ctypes.byref(cfg)))


def ndf_infer_latents(cfg, qparams, cache, stream=None):
    _check(lib().ndf_infer_latents(ctypes.byref(cfg), _p(qparams), _p(cache), _stream(stream)),
           "ndf_infer_latents")


def ndf_infer_field_cached(cfg, qparams, ref_v, cache, out, ws, stream=None):
    refs, rp = _host_i64(ref_v)
    _check(lib().ndf_infer_field_cached(ctypes.byref(cfg), _p(qparams), rp, len(refs), _p(cache),
                                        _p(out), _p(ws), ws.numel(), _stream(stream)),
           "ndf_infer_field_cached")


def ndf_infer_points(cfg, qparams, prec, ref_v, pos, out, ws, stream=None):
    """out[r][i] = Phi(p_ref[r], pos[i]) for pos float32 [n][3] in [-1, 1]^3."""
    refs, rp = _host_i64(ref_v)
    if pos.dim() != 2 or pos.shape[1] != 3 or pos.dtype != torch.float32 \
            or not pos.is_contiguous():
        raise NdfError("ndf_infer_points: pos must be a contiguous float32 [n][3] tensor")
    if out.dtype != torch.float32 or not out.is_contiguous() \
            or out.numel() < len(refs) * pos.shape[0]:
        raise NdfError("ndf_infer_points: out must be a contiguous float32 [n_ref][n] tensor")
    _check(lib().ndf_infer_points(ctypes.byref(cfg), _p(qparams), prec, rp, len(refs), _p(pos),
                                  pos.shape[0], _p(out), _p(ws), ws.numel(), _stream(stream)),
           "ndf_infer_points")


def ndf_infer_field_difference(cfg, qparams, ref_a, ref_b, cache, out, ws, stream=None):
    _check(lib().ndf_infer_field_difference(ctypes.byref(cfg), _p(qparams), int(ref_a),
                                            int(ref_b), _p(cache), _p(out), _p(ws), ws.numel(),
                                            _stream(stream)), "ndf_infer_field_difference")


def infer_ws_bytes(cfg, n_ref, prec):
    return ndf_workspace_bytes(NDF_OP_INFER, None, cfg, n_ref, prec)


def cached_ws_bytes(cfg, n_ref):
    """Workspace of ndf_infer_field_cached / ndf_infer_field_difference."""
    return ndf_workspace_bytes(NDF_OP_INFER_CACHED, None, cfg, n_ref, NDF_PREC_BF16)
