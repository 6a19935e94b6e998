"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid arguments on the host before enqueuing
anything (the pointers below are never dereferenced)."""
import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

from paper_2307_02203_amd import ndf

ROOT = Path(__file__).resolve().parents[1]
FAKE = 0x1000  # non-null, never dereferenced: every call below fails validation first


def _declared():
    txt = (ROOT / "include" / "ndf.h").read_text()
    return sorted(set(re.findall(r"\b(ndf_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    L = ndf.lib()
    declared = _declared()
    assert len(declared) >= 16
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(ndf.EXPORTED) == declared


def test_status_strings():
    L = ndf.lib()
    assert L.ndf_status_string(0) == b"ok"
    assert b"workspace" in L.ndf_status_string(-2)


def _ens(N=64, nx=16, ny=16, nz=8, n_vars=1, stats=True):
    p = FAKE if stats else 0
    return ndf.ndf_ensemble(N, nx, ny, nz, n_vars, FAKE, p, p, p, p)


def test_prepare_rejects_bad_shapes():
    L = ndf.lib()
    for e in (_ens(N=1), _ens(nx=1), _ens(n_vars=0), _ens(stats=False), _ens(N=5000)):
        assert L.ndf_prepare(ctypes.byref(e), None, 0, None) == ndf.NDF_E_ARG
    assert L.ndf_prepare(None, None, 0, None) == ndf.NDF_E_ARG
    # the status word needs its workspace bytes
    e = _ens()
    need = L.ndf_workspace_bytes(ndf.NDF_OP_PREPARE, ctypes.byref(e), None, 0, 0)
    assert need == 256
    assert L.ndf_prepare(ctypes.byref(e), FAKE, need - 1, None) == ndf.NDF_E_WORKSPACE
    assert b"non-finite" in L.ndf_status_string(ndf.NDF_E_NONFINITE)


def test_field_calls_validate_before_launch():
    L = ndf.lib()
    e = _ens()
    refs = np.array([1160], dtype=np.int64)
    rp = refs.ctypes.data_as(ctypes.c_void_p)
    bad = np.array([2048], dtype=np.int64)
    bp = bad.ctypes.data_as(ctypes.c_void_p)
    ws_need = L.ndf_workspace_bytes(ndf.NDF_OP_PEARSON_FIELD, ctypes.byref(e), None, 1, 0)
    assert ws_need > 0
    E = ctypes.byref(e)
    # reference out of range, bad variable, missing output, small workspace, bad precision
    assert L.ndf_pearson_field(E, 0, 0, bp, 1, FAKE, 0, FAKE, ws_need, None) == ndf.NDF_E_ARG
    assert L.ndf_pearson_field(E, 1, 0, rp, 1, FAKE, 0, FAKE, ws_need, None) == ndf.NDF_E_ARG
    assert L.ndf_pearson_field(E, 0, 0, rp, 1, None, 0, FAKE, ws_need, None) == ndf.NDF_E_ARG
    assert L.ndf_pearson_field(E, 0, 0, rp, 0, FAKE, 0, FAKE, ws_need, None) == ndf.NDF_E_ARG
    assert (L.ndf_pearson_field(E, 0, 0, rp, 1, FAKE, 0, FAKE, ws_need - 1, None)
            == ndf.NDF_E_WORKSPACE)
    assert (L.ndf_pearson_field(E, 0, 0, rp, 1, FAKE, 0, None, ws_need, None)
            == ndf.NDF_E_WORKSPACE)
    assert L.ndf_pearson_field(E, 0, 0, rp, 1, FAKE, 7, FAKE, ws_need, None) == ndf.NDF_E_UNSUPPORTED
    kws = L.ndf_workspace_bytes(ndf.NDF_OP_KSG_FIELD, E, None, 1, 0)
    assert L.ndf_ksg_mi_field(E, 0, 0, rp, 1, 0, FAKE, None, FAKE, kws, None) == ndf.NDF_E_ARG
    assert L.ndf_ksg_mi_field(E, 0, 0, rp, 1, 64, FAKE, None, FAKE, kws, None) == ndf.NDF_E_ARG
    assert L.ndf_ksg_mi_field(E, 0, 0, rp, 1, 9, FAKE, None, FAKE, kws, None) == ndf.NDF_E_UNSUPPORTED
    assert (L.ndf_ksg_mi_field(E, 0, 0, rp, 1, 4, FAKE, None, FAKE, kws - 8, None)
            == ndf.NDF_E_WORKSPACE)
    big = _ens(N=3000)
    kb = L.ndf_workspace_bytes(ndf.NDF_OP_KSG_FIELD, ctypes.byref(big), None, 1, 0)
    assert (L.ndf_ksg_mi_field(ctypes.byref(big), 0, 0, rp, 1, 4, FAKE, None, FAKE, kb, None)
            == ndf.NDF_E_UNSUPPORTED)
    pws = L.ndf_workspace_bytes(ndf.NDF_OP_KSG_PAIRS, E, None, 1, 0)
    assert L.ndf_ksg_mi_pairs(E, 0, 0, FAKE, 0, 4, FAKE, None, FAKE, pws, None) == ndf.NDF_E_ARG
    assert L.ndf_pearson_pairs(E, 0, 0, None, 5, FAKE, None) == ndf.NDF_E_ARG


def test_noalloc_field_validates_and_bounds_the_scratch():
    # argument errors and requests beyond the static scratch are refused on the host
    L = ndf.lib()
    cap = L.ndf_ksg_scratch_bytes()
    assert cap == 1 << 20
    e = _ens(N=1000, nx=250, ny=352, nz=20)
    E = ctypes.byref(e)
    n_max = max(n for n in range(1, 400)
                if L.ndf_workspace_bytes(ndf.NDF_OP_KSG_FIELD, E, None, n, 0) <= cap)
    assert n_max == 129
    refs = np.zeros(n_max + 1, dtype=np.int64)
    rp = refs.ctypes.data_as(ctypes.c_void_p)
    assert L.ndf_ksg_mi_field_noalloc(E, 0, 0, rp, n_max + 1, 4, FAKE, None, None) == ndf.NDF_E_SCRATCH
    assert b"scratch" in L.ndf_status_string(ndf.NDF_E_SCRATCH)
    assert L.ndf_ksg_mi_field_noalloc(E, 0, 0, rp, 1, 0, FAKE, None, None) == ndf.NDF_E_ARG
    assert L.ndf_ksg_mi_field_noalloc(E, 0, 0, rp, 1, 4, None, None, None) == ndf.NDF_E_ARG
    assert L.ndf_ksg_mi_field_noalloc(E, 0, 0, rp, 1, 9, FAKE, None, None) == ndf.NDF_E_UNSUPPORTED
    big = _ens(N=2048, nx=250, ny=352, nz=20)
    B = ctypes.byref(big)
    assert max(n for n in range(1, 400)
               if L.ndf_workspace_bytes(ndf.NDF_OP_KSG_FIELD, B, None, n, 0) <= cap) == 62


def test_workspace_sizes_grow_with_references():
    L = ndf.lib()
    e = ctypes.byref(_ens(N=1000, nx=250, ny=352, nz=20))
    a = L.ndf_workspace_bytes(ndf.NDF_OP_PEARSON_FIELD, e, None, 1, ndf.NDF_PREC_SPLIT_BF16)
    b = L.ndf_workspace_bytes(ndf.NDF_OP_PEARSON_FIELD, e, None, 64, ndf.NDF_PREC_SPLIT_BF16)
    assert 0 < a < b
    assert L.ndf_workspace_bytes(ndf.NDF_OP_PEARSON_FIELD, e, None, 1, 9) == 0
    assert L.ndf_workspace_bytes(99, e, None, 1, 0) == 0


def test_net_config_validation_and_param_bytes():
    import gen
    L = ndf.lib()
    lay = gen.NetLayout.for_grid(250, 352, 20)
    cfg = ndf.net_config(250, 352, 20, lay.res)
    assert ndf.ndf_net_param_bytes(cfg) == 4 * lay.n_floats
    assert ndf.ndf_net_optstate_bytes(cfg) == 8 * lay.n_floats
    lay2 = gen.NetLayout.for_grid(16, 16, 8, n_enc=2)
    cfg2 = ndf.net_config(16, 16, 8, lay2.res, n_enc=2)
    assert ndf.ndf_net_param_bytes(cfg2) == 4 * lay2.n_floats
    bad = ndf.net_config(250, 352, 20, lay.res, width=64)
    assert ndf.ndf_net_param_bytes(bad) == 0
    assert L.ndf_net_init(ctypes.byref(bad), FAKE, None, 1, None) == ndf.NDF_E_UNSUPPORTED
    bad3 = ndf.net_config(250, 352, 20, lay.res, n_enc=3)
    assert L.ndf_net_init(ctypes.byref(bad3), FAKE, None, 1, None) == ndf.NDF_E_ARG
    # limits of the lookup's exact integer arithmetic: V < 2^24, n <= 65535,
    # (n - 1)(R - 1) < 2^24
    big = ndf.net_config(512, 512, 64, lay.res)              # V = 2^24
    assert L.ndf_net_init(ctypes.byref(big), FAKE, None, 1, None) == ndf.NDF_E_UNSUPPORTED
    assert ndf.ndf_net_param_bytes(big) == 0
    wide = ndf.net_config(70000, 2, 2, lay.res)
    assert L.ndf_net_init(ctypes.byref(wide), FAKE, None, 1, None) == ndf.NDF_E_UNSUPPORTED
    res_fine = [[4097, 8, 2], [4097, 8, 2], [4097, 8, 2], [4097, 8, 2]]
    fine = ndf.net_config(4097, 4, 2, res_fine)             # (n - 1)(R - 1) = 2^24
    assert L.ndf_net_init(ctypes.byref(fine), FAKE, None, 1, None) == ndf.NDF_E_UNSUPPORTED
    ok_cfg = ndf.net_config(4096, 4, 2, [[4096, 4, 2]] * 4)  # (n - 1)(R - 1) < 2^24
    assert ndf.ndf_net_param_bytes(ok_cfg) > 0
    need = ndf.train_ws_bytes(cfg, 1024)
    assert need > 0
    C = ctypes.byref(cfg)
    assert (L.ndf_net_grad(C, FAKE, FAKE, FAKE, 1024, FAKE, FAKE, FAKE, need - 1, None)
            == ndf.NDF_E_WORKSPACE)
    assert L.ndf_net_grad(C, FAKE, FAKE, FAKE, 0, FAKE, FAKE, FAKE, need, None) == ndf.NDF_E_ARG
    assert (L.ndf_train_step(C, FAKE, FAKE, 0, FAKE, FAKE, 1024, ctypes.c_float(1e-3), FAKE, FAKE,
                             need * 2, None) == ndf.NDF_E_ARG)
    refs = np.array([1_760_000], dtype=np.int64)
    assert (L.ndf_infer_field(C, FAKE, ndf.NDF_PREC_BF16, refs.ctypes.data_as(ctypes.c_void_p), 1,
                              FAKE, FAKE, 1 << 30, None) == ndf.NDF_E_ARG)
    assert (L.ndf_infer_field(C, FAKE, ndf.NDF_PREC_SPLIT_BF16,
                              refs.ctypes.data_as(ctypes.c_void_p), 1, FAKE, FAKE, 1 << 30, None)
            == ndf.NDF_E_UNSUPPORTED)
    # encoder swap (Sec. 6.4): two encoders only, distinct buffers
    cfg2e = ndf.net_config(250, 352, 20, lay.res, n_enc=2)
    FAKE2 = ctypes.c_void_p(0x2000)
    assert L.ndf_net_swap_encoders(C, FAKE, FAKE2, None) == ndf.NDF_E_ARG
    assert L.ndf_net_swap_encoders(ctypes.byref(cfg2e), FAKE, FAKE, None) == ndf.NDF_E_ARG
    assert L.ndf_net_swap_encoders(ctypes.byref(cfg2e), None, FAKE2, None) == ndf.NDF_E_ARG
    # query-latent cache: 256 bytes per vertex, V rounded up to 64-vertex tiles
    assert ndf.ndf_infer_latent_bytes(cfg) == -(-250 * 352 * 20 // 64) * 64 * 256
    assert ndf.ndf_infer_latent_bytes(bad) == 0
    assert L.ndf_infer_latents(C, FAKE, None, None) == ndf.NDF_E_ARG
    assert (L.ndf_infer_field_cached(C, FAKE, refs.ctypes.data_as(ctypes.c_void_p), 1, FAKE,
                                     FAKE, FAKE, 1 << 30, None) == ndf.NDF_E_ARG)
    ok_ref = np.array([5], dtype=np.int64)
    assert (L.ndf_infer_field_cached(C, FAKE, ok_ref.ctypes.data_as(ctypes.c_void_p), 1, FAKE,
                                     FAKE, FAKE, 16, None) == ndf.NDF_E_WORKSPACE)
    # learned field at continuous positions (ray-march sampling) and field differences
    okp = ok_ref.ctypes.data_as(ctypes.c_void_p)
    badp = refs.ctypes.data_as(ctypes.c_void_p)
    BF = ndf.NDF_PREC_BF16
    assert L.ndf_infer_points(C, FAKE, BF, okp, 1, None, 10, FAKE, FAKE, 1 << 30, None) == ndf.NDF_E_ARG
    assert L.ndf_infer_points(C, FAKE, BF, okp, 1, FAKE, 10, None, FAKE, 1 << 30, None) == ndf.NDF_E_ARG
    assert L.ndf_infer_points(C, FAKE, BF, okp, 1, FAKE, -1, FAKE, FAKE, 1 << 30, None) == ndf.NDF_E_ARG
    assert L.ndf_infer_points(C, FAKE, BF, okp, 0, FAKE, 10, FAKE, FAKE, 1 << 30, None) == ndf.NDF_E_ARG
    assert L.ndf_infer_points(C, FAKE, BF, badp, 1, FAKE, 10, FAKE, FAKE, 1 << 30, None) == ndf.NDF_E_ARG
    assert (L.ndf_infer_points(C, FAKE, ndf.NDF_PREC_FP32, okp, 1, FAKE, 10, FAKE, FAKE, 1 << 30,
                               None) == ndf.NDF_E_UNSUPPORTED)
    assert L.ndf_infer_points(C, FAKE, BF, okp, 1, FAKE, 10, FAKE, FAKE, 16, None) == ndf.NDF_E_WORKSPACE
    # n = 0 is valid and enqueues nothing (no device needed)
    assert L.ndf_infer_points(C, FAKE, BF, okp, 1, None, 0, None, FAKE, 1 << 30, None) == ndf.NDF_OK
    V = 250 * 352 * 20
    assert L.ndf_infer_field_difference(C, FAKE, 0, V, FAKE, FAKE, FAKE, 1 << 30, None) == ndf.NDF_E_ARG
    assert L.ndf_infer_field_difference(C, FAKE, -1, 0, FAKE, FAKE, FAKE, 1 << 30, None) == ndf.NDF_E_ARG
    assert L.ndf_infer_field_difference(C, FAKE, 0, 1, None, FAKE, FAKE, 1 << 30, None) == ndf.NDF_E_ARG
    need2 = ndf.cached_ws_bytes(cfg, 2)
    # a BF16 field of several references also holds the query latents of every vertex
    assert ndf.infer_ws_bytes(cfg, 2, BF) >= need2 + L.ndf_infer_latent_bytes(C)
    assert ndf.infer_ws_bytes(cfg, 1, BF) == ndf.cached_ws_bytes(cfg, 1)
    assert (L.ndf_infer_field_difference(C, FAKE, 0, 1, FAKE, FAKE, FAKE, need2 - 1, None)
            == ndf.NDF_E_WORKSPACE)


def test_positions_entry_points_reject_bad_arguments():
    """The calls at continuous positions validate on the host (no device needed)."""
    import gen
    L = ndf.lib()
    lay = gen.NetLayout.for_grid(250, 352, 20)
    cfg = ndf.net_config(250, 352, 20, lay.res)
    C = ctypes.byref(cfg)
    FAKE = ctypes.c_void_p(0x1000)
    need = ndf.train_ws_bytes(cfg, 64)
    assert L.ndf_net_forward_at(C, FAKE, None, 64, FAKE, FAKE, need, None) == ndf.NDF_E_ARG
    assert L.ndf_net_forward_at(C, FAKE, FAKE, 0, FAKE, FAKE, need, None) == ndf.NDF_E_ARG
    assert (L.ndf_net_forward_at(C, FAKE, FAKE, 64, FAKE, FAKE, need - 1, None)
            == ndf.NDF_E_WORKSPACE)
    assert (L.ndf_net_grad_at(C, FAKE, None, FAKE, 64, FAKE, FAKE, FAKE, need, None)
            == ndf.NDF_E_ARG)
    assert (L.ndf_net_grad_at(C, FAKE, FAKE, FAKE, 64, FAKE, FAKE, FAKE, need - 1, None)
            == ndf.NDF_E_WORKSPACE)
    assert (L.ndf_train_step_at(C, FAKE, FAKE, 0, FAKE, FAKE, 64, ctypes.c_float(1e-3), FAKE,
                                FAKE, need * 2, None) == ndf.NDF_E_ARG)
    assert (L.ndf_train_step_at(C, FAKE, FAKE, 1, FAKE, FAKE, 64, ctypes.c_float(1e-3), FAKE,
                                FAKE, need, None) == ndf.NDF_E_WORKSPACE)
    # Pearson at positions needs the vertex-major copy
    e = ndf.ndf_ensemble(16, 8, 8, 4, 1, 0x1000, 0x2000, 0x3000, 0x4000, 0x5000, None, None)
    E = ctypes.byref(e)
    assert L.ndf_pearson_points(E, 0, 0, FAKE, 10, FAKE, None) == ndf.NDF_E_ARG
    e.xt = 0x6000
    assert L.ndf_pearson_points(E, 0, 1, FAKE, 10, FAKE, None) == ndf.NDF_E_ARG
    assert L.ndf_pearson_points(E, 0, 0, None, 10, FAKE, None) == ndf.NDF_E_ARG
    assert L.ndf_pearson_points(E, 0, 0, FAKE, -1, FAKE, None) == ndf.NDF_E_ARG
    assert L.ndf_pearson_points(E, 0, 0, None, 0, None, None) == ndf.NDF_OK


def test_hash_grid_config():
    """Hash tables (Sec. 4.2): T in [8, 24]; the parameter layout matches the
    generator's (2^T cells for the levels larger than that); a dense level of
    2^28 cells or more needs hashing."""
    import gen
    L = ndf.lib()
    FAKE = ctypes.c_void_p(0x1000)
    lay = gen.NetLayout.for_grid(250, 352, 20, log2_hashmap=19)
    cfg = ndf.net_config(250, 352, 20, lay.res, log2_hashmap=19)
    assert ndf.ndf_net_param_bytes(cfg) == 4 * lay.n_floats
    assert lay.cells(3) == 1 << 19 and lay.cells(2) == 157 * 222 * 13
    dense = gen.NetLayout.for_grid(250, 352, 20)
    assert lay.n_floats < dense.n_floats
    for T in (5, 25, -1):
        bad = ndf.net_config(250, 352, 20, lay.res, log2_hashmap=T)
        assert L.ndf_net_init(ctypes.byref(bad), FAKE, None, 1, None) == ndf.NDF_E_ARG
    huge = [[4096, 4096, 16]] * 4                    # 2^28 cells per level
    assert ndf.ndf_net_param_bytes(ndf.net_config(2048, 2048, 2, huge)) == 0
    assert ndf.ndf_net_param_bytes(ndf.net_config(2048, 2048, 2, huge, log2_hashmap=20)) > 0


def test_fourier_config():
    """Fourier features (12 frequencies) widen W1 to 112 inputs in the library's
    parameter layout as in the generator's; other frequency counts, two encoders
    or a grid-only network with them are refused."""
    import gen
    lay = gen.NetLayout.for_grid(16, 16, 8, fourier=12)
    cfg = ndf.net_config(16, 16, 8, lay.res, fourier=12)
    assert ndf.ndf_net_param_bytes(cfg) == 4 * lay.n_floats
    plain = gen.NetLayout.for_grid(16, 16, 8)
    assert lay.n_floats - plain.n_floats == 128 * (112 - 32)
    for kw in ({"fourier": 5}, {"fourier": 12, "n_enc": 2}, {"fourier": 12, "grid_only": True}):
        assert ndf.ndf_net_param_bytes(ndf.net_config(16, 16, 8, lay.res, **kw)) == 0, kw
    q = ndf.ndf_net_qparam_bytes(cfg, ndf.NDF_PREC_BF16)
    assert q > ndf.ndf_net_qparam_bytes(ndf.net_config(16, 16, 8, lay.res), ndf.NDF_PREC_BF16)


def test_ksg_points_workspace_and_limits():
    """Workspace of the KSG targets at positions: the 2B code columns (4 B per member)
    and their sorted orders (2 B per member) dominate; B is limited to 2^29 and the
    call refuses more than 2048 members like the other KSG calls."""
    L = ndf.lib()
    e = ndf.ndf_ensemble(1000, 250, 352, 20, 1, 0x1000, 0x2000, 0x3000, 0x4000, 0x5000, None,
                         0x6000)
    B = 1 << 18
    ws = ndf.ndf_workspace_bytes(ndf.NDF_OP_KSG_POINTS, type("E", (), {"c": e})(), None, B, 0)
    cols = 2 * B * 1000
    assert cols * 6 <= ws <= cols * 6 + 2 * B * 12 + (1 << 16)
    assert ndf.ndf_workspace_bytes(ndf.NDF_OP_KSG_POINTS, type("E", (), {"c": e})(), None,
                                   (1 << 29) + 1, 0) == 0
    E = ctypes.byref(e)
    FAKE = ctypes.c_void_p(0x7000)
    assert (L.ndf_ksg_mi_points(E, 0, 0, FAKE, (1 << 29) + 1, 4, FAKE, None, FAKE, 1 << 40, None)
            == ndf.NDF_E_ARG)
    assert L.ndf_ksg_mi_points(E, 0, 0, FAKE, 16, 9, FAKE, None, FAKE, 1 << 40, None) == \
        ndf.NDF_E_UNSUPPORTED
    assert L.ndf_ksg_mi_points(E, 0, 0, FAKE, 16, 4, FAKE, None, FAKE, 16, None) == \
        ndf.NDF_E_WORKSPACE
    e.n_members = 4096
    assert L.ndf_ksg_mi_points(E, 0, 0, FAKE, 16, 4, FAKE, None, FAKE, 1 << 40, None) == \
        ndf.NDF_E_UNSUPPORTED
