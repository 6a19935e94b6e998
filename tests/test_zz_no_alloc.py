"""The no-allocation KSG field call against the workspace call, through the C ABI.

ndf_ksg_mi_field_noalloc runs the kernels of ndf_ksg_mi_field with the workspace
in the library's static device scratch, so fields and neighbour counts must be
identical bit for bit.  Two calls in a row, the second on a smaller input (fewer
members and references), check that the scratch left by the first call does not
leak into the second; the neighbour counts are also checked against the FP64
oracle (bit-exact) on a few vertices.
"""
import sys

import numpy as np
import pytest
import torch

import gen
from oracle import direct
from paper_2307_02203_amd import ndf

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _ens(name):
    cfg = gen.CONFIGS[name]
    x = gen.make_ensemble(cfg, device="cuda")
    e = ndf.Ensemble(x, cfg.nx, cfg.ny, cfg.nz)
    ndf.ndf_prepare(e)
    torch.cuda.synchronize()
    return cfg, e


def _both(e, refs, k):
    n = len(refs)
    out_a = torch.full((n, e.n_vertices), float("nan"), device="cuda")
    out_b = torch.full((n, e.n_vertices), float("nan"), device="cuda")
    cnt_a = torch.full((n, e.n_vertices, 2, e.n_members), -1, dtype=torch.int32, device="cuda")
    cnt_b = torch.full_like(cnt_a, -1)
    ws = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_KSG_FIELD, e, None, n, 0),
                     dtype=torch.uint8, device="cuda")
    ndf.ndf_ksg_mi_field(e, 0, 0, refs, k, out_a, cnt_a, ws)
    ndf.ndf_ksg_mi_field_noalloc(e, 0, 0, refs, k, out_b, cnt_b)
    torch.cuda.synchronize()
    return out_a, out_b, cnt_a, cnt_b


def test_noalloc_ksg_field_equals_workspace_call_twice():
    assert ndf.ndf_ksg_scratch_bytes() == 1 << 20
    # first call: mid ensemble (200 members, 11803 vertices), three references
    cfg, e = _ens("mid")
    refs = np.array([cfg.ref_v, 17, e.n_vertices - 1], dtype=np.int64)
    _log("no-alloc KSG: mid, refs", refs.tolist(), "k=4")
    a, b, ca, cb = _both(e, refs, 4)
    assert torch.equal(ca, cb)
    assert torch.equal(a, b)
    x = e.x[0].cpu().numpy()
    vs = [0, 5000, e.n_vertices - 1]
    _, nx_o, ny_o = direct.ksg_field(x[:, refs[0]], x[:, vs], 4, counts=True)
    for i, v in enumerate(vs):
        c = cb[0, v].cpu().numpy()
        assert np.array_equal(c[0], nx_o[i]) and np.array_equal(c[1], ny_o[i]), v
    del e
    # second call, smaller input: tiny ensemble (64 members, 2048 vertices), one reference
    cfg, e = _ens("tiny")
    refs = np.array([cfg.ref_v], dtype=np.int64)
    _log("no-alloc KSG: tiny, refs", refs.tolist(), "k=3")
    a, b, ca, cb = _both(e, refs, 3)
    assert torch.equal(ca, cb)
    assert torch.equal(a, b)
    mi_o = direct.ksg_field(e.x[0].cpu().numpy()[:, cfg.ref_v], e.x[0].cpu().numpy(), 3)
    assert np.max(np.abs(b[0].cpu().numpy() - mi_o)) <= 1e-4


def test_noalloc_rejects_requests_beyond_the_scratch():
    cfg, e = _ens("tiny")
    n_max = 1
    while (ndf.ndf_workspace_bytes(ndf.NDF_OP_KSG_FIELD, e, None, n_max + 1, 0)
           <= ndf.ndf_ksg_scratch_bytes()):
        n_max += 1
    refs = np.full(n_max + 1, cfg.ref_v, dtype=np.int64)
    out = torch.empty((n_max + 1, e.n_vertices), device="cuda")
    with pytest.raises(ndf.NdfError, match="scratch"):
        ndf.ndf_ksg_mi_field_noalloc(e, 0, 0, refs, 4, out, None)
