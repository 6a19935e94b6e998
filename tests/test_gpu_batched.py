"""GPU parity at the batched, reduced-precision workload: 256 reference vertices
against all 1.76M vertices of a two-variable paper-shaped ensemble (1000 members,
250x352x20; the second variable is the first one's smoothed blobs through tanh
plus independent noise), through the C ABI.

* direct Pearson across variables (R_{mu nu}, Sec. 3) as the split-BF16 MFMA
  contraction for all 256 references: |dr| <= 1e-5 on sampled vertices of every
  field, and 1 on the diagonal of the second variable's own batch;
* KSG-MI across variables: |dI| <= 1e-4 on sampled vertices, neighbour counts of
  pairs bit-exact;
* the learned field for all 256 references with an E4M3 decoder (on the cached
  BF16 query latents) and in BF16, both against the FP64 network oracle on
  sampled (reference, query) pairs.
"""
import sys

import numpy as np
import pytest
import torch

import gen
from oracle import direct
from oracle import ndf_net as nn
from paper_2307_02203_amd import ndf

pytestmark = pytest.mark.gpu

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from floors import BF16_OPS, check_floor, fp8_decoder_ops  # noqa: E402

PEARSON_TOL = 1e-5
MI_TOL = 1e-4
N_REF = 256


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ens2():
    cfg = gen.CONFIGS["paper2v"]
    _log("generating two-variable paper-shaped ensemble (2 x 1000 x 1.76M)")
    x = gen.make_ensemble(cfg, device="cuda")
    e = ndf.Ensemble(x, cfg.nx, cfg.ny, cfg.nz)
    ndf.ndf_prepare(e)
    torch.cuda.synchronize()
    return e


def _refs(V):
    cfg = gen.CONFIGS["paper2v"]
    return np.concatenate([[cfg.ref_v], gen.random_vertices(V, N_REF - 1, seed=2311)])


def _cols(e, var, idx):
    idx = torch.as_tensor(np.asarray(idx), dtype=torch.int64, device=e.device)
    return e.x[var][:, idx].cpu().numpy()


def test_batch256_pearson_across_variables(ens2):
    V = ens2.n_vertices
    refs = _refs(V)
    sample = np.unique(np.concatenate([gen.random_vertices(V, 150, seed=93), [0, V - 1]]))
    s_t = torch.as_tensor(sample, device="cuda")
    xr = _cols(ens2, 0, refs)
    xs = _cols(ens2, 1, sample)
    _log("batch 256 split-BF16 Pearson, variable 0 -> 1")
    got = ndf.pearson_field(ens2, refs, prec=ndf.NDF_PREC_SPLIT_BF16, var_ref=0, var_qry=1)
    assert torch.isfinite(got).all()
    g = got[:, s_t].cpu().numpy()
    worst = 0.0
    for i in range(N_REF):
        want = direct.pearson_field(xr[:, i], xs)
        worst = max(worst, float(np.max(np.abs(g[i] - want))))
    _log(f"batch 256 across variables: sampled max|dr|={worst:.2e}")
    assert worst <= PEARSON_TOL
    # the FP32 stream on the first reference gives the same field
    r32 = ndf.pearson_field(ens2, refs[:1], prec=ndf.NDF_PREC_FP32, var_ref=0, var_qry=1)
    assert (r32[0] - got[0]).abs().max().item() <= 2 * PEARSON_TOL
    del got, r32
    # the tanh variable against itself: 1 at every reference
    _log("batch 256 split-BF16 Pearson, variable 1 -> 1")
    got = ndf.pearson_field(ens2, refs, prec=ndf.NDF_PREC_SPLIT_BF16, var_ref=1, var_qry=1)
    r_t = torch.as_tensor(refs, device="cuda")
    diag = got[torch.arange(N_REF, device="cuda"), r_t]
    assert torch.all((diag - 1.0).abs() <= PEARSON_TOL)
    xr1 = _cols(ens2, 1, refs[:32])
    g = got[:32][:, s_t].cpu().numpy()
    for i in range(32):
        assert np.max(np.abs(g[i] - direct.pearson_field(xr1[:, i], xs))) <= PEARSON_TOL, i


def test_ksg_across_variables(ens2):
    V = ens2.n_vertices
    refs = _refs(V)[:2]
    sample = gen.random_vertices(V, 150, seed=94)
    s_t = torch.as_tensor(sample, device="cuda")
    _log("KSG field, 2 references, variable 0 -> 1")
    mi = ndf.ksg_field(ens2, refs, k=4, var_ref=0, var_qry=1)
    assert torch.isfinite(mi).all()
    g = mi[:, s_t].cpu().numpy()
    xs = _cols(ens2, 1, sample)
    xr = _cols(ens2, 0, refs)
    for i in range(len(refs)):
        err = np.max(np.abs(g[i] - direct.ksg_field(xr[:, i], xs, 4)))
        _log(f"KSG across variables ref {refs[i]}: sampled max|dI|={err:.2e}")
        assert err <= MI_TOL
    # pairs across variables, counts bit-exact
    pairs = gen.random_pairs(V, 48, seed=2313)
    _log("KSG pairs across variables with counts")
    mi_p, cnt = ndf.ksg_pairs(ens2, pairs, k=4, counts=True, var_a=1, var_b=0)
    mi_p = mi_p.cpu().numpy()
    cnt = cnt.cpu().numpy()
    xa = _cols(ens2, 1, pairs[:, 0])
    xb = _cols(ens2, 0, pairs[:, 1])
    for b in range(len(pairs)):
        want, wnx, wny = direct.ksg_field(xa[:, b], xb[:, b:b + 1], 4, counts=True)
        assert np.array_equal(cnt[b, 0], wnx[0]) and np.array_equal(cnt[b, 1], wny[0])
        assert abs(mi_p[b] - want[0]) <= MI_TOL


def test_learned_field_256_refs_fp8_vs_bf16():
    cfg = gen.CONFIGS["paper2v"]
    V = cfg.n_vertices
    lay = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz, n_enc=1)
    flat = gen.make_net_params(lay, seed=2328, grid_scale=0.5, bias_scale=0.1)
    c = ndf.net_config(cfg.nx, cfg.ny, cfg.nz, lay.res, n_enc=1)
    P = torch.from_numpy(flat).cuda()
    net = nn.Net(flat, (cfg.nx, cfg.ny, cfg.nz), lay.res, 8, 128, 1)
    refs = _refs(V)
    out = {}
    for prec in (ndf.NDF_PREC_BF16, ndf.NDF_PREC_FP8_E4M3):
        _log(f"learned field, 256 references, prec={prec}")
        q = torch.empty(ndf.ndf_net_qparam_bytes(c, prec), dtype=torch.uint8, device="cuda")
        ndf.ndf_net_quantize(c, P, prec, q)
        o = torch.empty((N_REF, V), dtype=torch.float32, device="cuda")
        ws = torch.empty(ndf.infer_ws_bytes(c, N_REF, prec), dtype=torch.uint8, device="cuda")
        ndf.ndf_infer_field(c, q, prec, refs, o, ws)
        torch.cuda.synchronize()
        assert torch.isfinite(o).all()
        out[prec] = o
    # sampled (reference, query) pairs against the FP64 network
    rng = np.random.default_rng(2399)
    ri = rng.integers(0, N_REF, 4000)
    qv = gen.random_vertices(V, 4000, seed=95)
    want, _ = nn.forward(net, refs[ri], qv)
    ri_t = torch.as_tensor(ri, device="cuda")
    qv_t = torch.as_tensor(qv, device="cuda")
    for prec, ops in ((ndf.NDF_PREC_BF16, BF16_OPS),
                      (ndf.NDF_PREC_FP8_E4M3, fp8_decoder_ops(net))):
        g = out[prec][ri_t, qv_t].cpu().numpy().astype(np.float64)
        check_floor(g, want, nn.forward(net, refs[ri], qv, ops)[0], f"256 refs prec={prec}")
    # the reference latent of row i is that of refs[i]: every row equals the one-reference
    # call, bit for bit (at this size the last, partial round of tiles is split over the
    # references of each launch, so both halves of a split tile are covered)
    q = torch.empty(ndf.ndf_net_qparam_bytes(c, ndf.NDF_PREC_BF16), dtype=torch.uint8,
                    device="cuda")
    ndf.ndf_net_quantize(c, P, ndf.NDF_PREC_BF16, q)
    o1 = torch.empty((1, V), dtype=torch.float32, device="cuda")
    ws = torch.empty(ndf.infer_ws_bytes(c, 1, ndf.NDF_PREC_BF16), dtype=torch.uint8,
                     device="cuda")
    _log("256 one-reference BF16 calls against the rows of the batched call")
    for i in range(N_REF):
        ndf.ndf_infer_field(c, q, ndf.NDF_PREC_BF16, refs[i:i + 1], o1, ws)
        assert torch.equal(o1[0], out[ndf.NDF_PREC_BF16][i]), i
