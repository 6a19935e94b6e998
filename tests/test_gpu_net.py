"""GPU parity of the learned field (Sec. 4-5) against the FP64 oracle, through the
C ABI: initialisation, forward, adjoint (gradients), Adam, fused inference, and
training convergence.

Bars.  BF16 MFMA operands with FP32 accumulate (and, for a11, microscaled E4M3)
cannot match FP64 exactly; how far they may deviate is measured on the CPU by the
same FP64 oracle with its products' operands rounded as the kernels round them
(oracle.ndf_net.Operands: bf16 weights, activations and gradient operands in
training; bf16 latents before the merge in inference; E4M3 with power-of-two
block scales for FP8 layers 2-5; bf16 grid features in inference).  Each GPU
result must stay within 1.25 times that emulated floor (relative L2 per output
vector or per gradient tensor, plus 1e-3 for results whose floor is near zero),
and its largest element error within 2 times the emulated one (plus 1e-3 of the
RMS); tests/floors.py holds the bars.  A kernel that rounds where the arithmetic
says it does passes, one with a wrong or missing term does not.  The
hand-built network is held to its bf16 input rounding; Adam exactly where the
gradient sign is unambiguous.  Parameters and pairs come from the seeded
generators; the oracle never sees a value produced by the GPU path.
"""
import math
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
from test_oracle_net import hand_built_params, hand_built_value, DIMS as HB_DIMS, RES as HB_RES  # noqa: E402
from floors import (BF16_OPS, TRAIN_OPS, fp8_decoder_ops, fp8_ops, check_floor as _check_floor,  # noqa: E402
                    check_grad_floor)


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _setup(name, n_enc=1, seed=2320, grid_scale=0.5, bias_scale=0.1):
    cfg = gen.CONFIGS[name]
    lay = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz, n_enc=n_enc)
    flat = gen.make_net_params(lay, seed=seed, grid_scale=grid_scale, bias_scale=bias_scale)
    c = ndf.net_config(cfg.nx, cfg.ny, cfg.nz, lay.res, n_enc=n_enc)
    P = torch.from_numpy(flat).cuda()
    net = nn.Net(flat, (cfg.nx, cfg.ny, cfg.nz), lay.res, 8, 128, n_enc)
    return cfg, lay, c, P, net




def _forward_gpu(c, P, pairs):
    pairs_t = torch.as_tensor(pairs, dtype=torch.int64, device="cuda").contiguous()
    y = torch.empty(len(pairs), dtype=torch.float32, device="cuda")
    ws = torch.empty(ndf.train_ws_bytes(c, len(pairs)), dtype=torch.uint8, device="cuda")
    ndf.ndf_net_forward(c, P, pairs_t, y, ws)
    return y.cpu().numpy().astype(np.float64)


def _grad_gpu(c, P, pairs, targets):
    B = len(pairs)
    pairs_t = torch.as_tensor(pairs, dtype=torch.int64, device="cuda").contiguous()
    t = torch.as_tensor(targets, dtype=torch.float32, device="cuda")
    g = torch.empty_like(P)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    ws = torch.empty(ndf.train_ws_bytes(c, B), dtype=torch.uint8, device="cuda")
    ndf.ndf_net_grad(c, P, pairs_t, t, g, loss, ws)
    return g.cpu().numpy().astype(np.float64), loss.item()


def _qparams(c, P, prec=ndf.NDF_PREC_BF16):
    q = torch.empty(ndf.ndf_net_qparam_bytes(c, prec), dtype=torch.uint8, device="cuda")
    ndf.ndf_net_quantize(c, P, prec, q)
    return q


def _infer_gpu(c, q, refs, V, prec=ndf.NDF_PREC_BF16):
    out = torch.empty((len(refs), V), dtype=torch.float32, device="cuda")
    ws = torch.empty(ndf.infer_ws_bytes(c, len(refs), prec), dtype=torch.uint8, device="cuda")
    ndf.ndf_infer_field(c, q, prec, refs, out, ws)
    return out


def test_init_statistics():
    cfg, lay, c, P, _ = _setup("tiny")
    opt = torch.full((2 * P.numel(),), 7.0, device="cuda")
    ndf.ndf_net_init(c, P, opt, 12345)
    p = P.cpu().numpy()
    assert torch.all(opt == 0)
    for name, shape in lay.tensors():
        v = lay.view(p, name)
        if name.startswith("grid"):
            assert np.all(np.abs(v) <= 1e-4) and v.std() > 4e-5
        elif name[0] in "Ww":
            a = math.sqrt(6.0 / shape[-1])
            assert np.all(np.abs(v) <= a) and abs(v.std() - a / math.sqrt(3)) < 0.1 * a
            assert abs(v.mean()) < 0.1 * a
        else:
            assert np.all(v == 0)
    P2 = torch.empty_like(P)
    ndf.ndf_net_init(c, P2, None, 12345)
    assert torch.equal(P, P2)
    ndf.ndf_net_init(c, P2, None, 54321)
    assert not torch.equal(P, P2)


def test_hand_built_network_closed_form():
    dims, res = HB_DIMS, HB_RES
    flat = hand_built_params()
    c = ndf.net_config(dims[0], dims[1], dims[2], res)
    P = torch.from_numpy(flat).cuda()
    V = dims[0] * dims[1] * dims[2]
    v1, v2 = np.meshgrid(np.arange(V), np.arange(V))
    pairs = np.stack([v1.ravel(), v2.ravel()], axis=1)
    want = hand_built_value(pairs[:, 0], pairs[:, 1], dims)
    y = _forward_gpu(c, P, pairs)
    # inputs are bf16 (8 bits): u_x + 2 in [2, 3] is rounded to 2^-7
    assert np.max(np.abs(y - want) / np.abs(want)) < 2e-2
    q = _qparams(c, P)
    out = _infer_gpu(c, q, [0, 17, V - 1], V).cpu().numpy()
    for i, r in enumerate([0, 17, V - 1]):
        w = hand_built_value(np.full(V, r), np.arange(V), dims)
        assert np.max(np.abs(out[i] - w) / np.abs(w)) < 2e-2


@pytest.mark.parametrize("name,n_enc", [("tiny", 1), ("mid", 1), ("mid", 2)])
def test_forward_parity(name, n_enc):
    cfg, lay, c, P, net = _setup(name, n_enc)
    pairs = gen.random_pairs(cfg.n_vertices, 3000, seed=11)
    y = _forward_gpu(c, P, pairs)
    want, _ = nn.forward(net, pairs[:, 0], pairs[:, 1])
    emul, _ = nn.forward(net, pairs[:, 0], pairs[:, 1], TRAIN_OPS)
    _check_floor(y, want, emul, f"forward {name} n_enc={n_enc}")


@pytest.mark.parametrize("name,n_enc,B", [("tiny", 1, 2048), ("mid", 1, 2001), ("mid", 2, 2048)])
@pytest.mark.parametrize("signs", ["same", "random"])
def test_gradient_parity(name, n_enc, B, signs):
    """Adjoint kernels vs the FP64 adjoint, every parameter tensor held to 1.25 times
    the error of the FP64 adjoint with the kernels' bf16 operand rounding.  With
    one residual sign for every pair the per-pair gradients add up; with random
    signs the batch gradient is a sum with heavy cancellation and its floor is
    near 1e-1 in every tensor (rounding flips ReLU masks; the rounding of the
    gradient operand itself contributes only a few 1e-3).  One encoder runs the
    fused kernels (B = 2001: a ragged last tile of 17 pairs), two encoders the
    layer-by-layer ones."""
    cfg, lay, c, P, net = _setup(name, n_enc, seed=2321)
    pairs = gen.random_pairs(cfg.n_vertices, B, seed=12)
    y, _ = nn.forward(net, pairs[:, 0], pairs[:, 1])
    if signs == "same":
        s = -np.ones(len(pairs))
    else:
        s = np.where(np.random.default_rng(5).random(len(pairs)) < 0.5, -1.0, 1.0)
    t = y - s            # residual y - t = s: fixed sign, far from the L1 kink
    loss_o, g_o, _ = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], t)
    _, g_e, _ = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], t, TRAIN_OPS)
    g, loss = _grad_gpu(c, P, pairs, t.astype(np.float32))
    assert abs(loss - loss_o) <= 1e-2 * loss_o
    check_grad_floor(lay, g, g_o.flat, g_e.flat, f"grad[{signs}] {name} n_enc={n_enc}")


def test_train_step_adam_parity():
    cfg, lay, c, P, net = _setup("tiny", 1, seed=2322)
    B = 1024
    pairs = gen.random_pairs(cfg.n_vertices, B, seed=13)
    y, _ = nn.forward(net, pairs[:, 0], pairs[:, 1])
    t = (y + 1.0).astype(np.float32)
    _, g_o, _ = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], t)
    lr = 1e-3
    p1, _, _ = nn.adam_update(net.flat, g_o.flat, np.zeros_like(net.flat),
                              np.zeros_like(net.flat), 1, lr)
    opt = torch.zeros(2 * P.numel(), device="cuda")
    ws = torch.empty(ndf.train_ws_bytes(c, B) + P.numel() * 4 + 256, dtype=torch.uint8,
                     device="cuda")
    loss = torch.empty(1, device="cuda")
    pairs_t = torch.as_tensor(pairs, device="cuda")
    ndf.ndf_train_step(c, P, opt, 1, pairs_t, torch.as_tensor(t, device="cuda"), lr, loss, ws)
    got = P.cpu().numpy().astype(np.float64)
    gabs = np.abs(g_o.flat)
    strong = gabs > 1e-2 * gabs.max()
    assert strong.sum() > 1000
    np.testing.assert_allclose(got[strong], p1[strong], rtol=0, atol=1e-6)
    # parameters without gradient stay put (a few ReLU units that are dead in FP64
    # but alive after bf16 rounding may move by lr)
    untouched = gabs == 0
    moved = got[untouched] != net.flat[untouched].astype(np.float32)
    assert moved.mean() < 5e-3
    # first moment m = 0.1 g, second v = 0.001 g^2 where the sign is unambiguous
    m = opt[:P.numel()].cpu().numpy()
    np.testing.assert_allclose(m[strong], 0.1 * g_o.flat[strong], rtol=5e-2, atol=0)


def test_nonfinite_loss_sets_status_and_skips_the_step():
    """A NaN target makes the loss non-finite: the workspace's status word becomes
    NDF_E_NONFINITE and Adam leaves parameters and moments as they were; the next
    step with finite targets clears the word and updates them."""
    cfg, lay, c, P, net = _setup("tiny", 1, seed=2329)
    B = 512
    pairs = torch.as_tensor(gen.random_pairs(cfg.n_vertices, B, seed=14), device="cuda")
    t = torch.zeros(B, device="cuda")
    t[17] = float("nan")
    opt = torch.zeros(2 * P.numel(), device="cuda")
    ws = torch.empty(ndf.train_ws_bytes(c, B) + P.numel() * 4 + 256, dtype=torch.uint8,
                     device="cuda")
    loss = torch.empty(1, device="cuda")
    P0 = P.clone()
    ndf.ndf_train_step(c, P, opt, 1, pairs, t, 1e-3, loss, ws)
    torch.cuda.synchronize()
    assert ndf.status_word(ws) == ndf.NDF_E_NONFINITE
    assert math.isnan(loss.item())
    assert torch.equal(P, P0) and torch.all(opt == 0)
    t[17] = 0.0
    ndf.ndf_train_step(c, P, opt, 1, pairs, t, 1e-3, loss, ws)
    torch.cuda.synchronize()
    assert ndf.status_word(ws) == ndf.NDF_OK
    assert math.isfinite(loss.item()) and not torch.equal(P, P0)
    # the gradient call reports through its own workspace too
    t[3] = float("inf")
    g = torch.empty_like(P)
    wsg = torch.empty(ndf.train_ws_bytes(c, B), dtype=torch.uint8, device="cuda")
    ndf.ndf_net_grad(c, P, pairs, t, g, loss, wsg)
    torch.cuda.synchronize()
    assert ndf.status_word(wsg) == ndf.NDF_E_NONFINITE


@pytest.mark.parametrize("name,n_enc", [("tiny", 1), ("mid", 1), ("mid", 2)])
def test_infer_field_parity(name, n_enc):
    cfg, lay, c, P, net = _setup(name, n_enc, seed=2323)
    V = cfg.n_vertices
    refs = [cfg.ref_v, 0, V - 1]
    q = _qparams(c, P)
    out = _infer_gpu(c, q, refs, V).cpu().numpy()
    for i, r in enumerate(refs):
        want = nn.field(net, r)
        _check_floor(out[i], want, nn.field(net, r, rnd=BF16_OPS),
                     f"infer {name} n_enc={n_enc} ref={r}")


@pytest.mark.parametrize("name,n_enc", [("mid", 1), ("mid", 2)])
def test_infer_field_cached_latents_bitwise(name, n_enc):
    """Fields from the query-latent cache, 35 references (two launches of 16 and a
    ragged one of 3), equal the fused single-reference fields bit for bit; so do
    the fields of one multi-reference ndf_infer_field call, which decodes from a
    latent cache in its workspace."""
    cfg, lay, c, P, net = _setup(name, n_enc, seed=2328)
    V = cfg.n_vertices
    refs = np.concatenate([[cfg.ref_v, 0, V - 1], gen.random_vertices(V, 32, seed=15)])
    q = _qparams(c, P, ndf.NDF_PREC_BF16)
    want = torch.cat([_infer_gpu(c, q, [r], V, ndf.NDF_PREC_BF16) for r in refs])
    cache = torch.empty(ndf.ndf_infer_latent_bytes(c), dtype=torch.uint8, device="cuda")
    ndf.ndf_infer_latents(c, q, cache)
    out = torch.full((len(refs), V), float("nan"), device="cuda")
    ws = torch.empty(ndf.cached_ws_bytes(c, len(refs)), dtype=torch.uint8, device="cuda")
    ndf.ndf_infer_field_cached(c, q, refs, cache, out, ws)
    torch.cuda.synchronize()
    assert torch.equal(out, want)
    multi = _infer_gpu(c, q, refs, V, ndf.NDF_PREC_BF16)
    assert torch.equal(multi, want)


def test_infer_self_field_symmetric_bitwise():
    cfg, lay, c, P, net = _setup("mid", 1, seed=2324)
    V = cfg.n_vertices
    refs = gen.random_vertices(V, 24, seed=9)
    q = _qparams(c, P)
    out = _infer_gpu(c, q, refs, V).cpu().numpy()
    for a in range(len(refs)):
        for b in range(len(refs)):
            assert out[a, refs[b]] == out[b, refs[a]]


def test_infer_two_encoder_swap_bitwise():
    """Cross-variable field (two encoders, Sec. 6.4): Phi_{nu mu}(p1, p2) =
    Phi_{mu nu}(p2, p1).  With the encoders' parameters swapped, the fused kernels
    give the same bits at swapped positions."""
    cfg, lay, c, P, net = _setup("mid", 2, seed=2326)
    V = cfg.n_vertices
    flat = P.cpu().numpy()
    sw = flat.copy()
    off, _ = lay.offsets()
    for e in (0, 1):
        for l in range(lay.n_levels):
            (o0, sh), (o1, _) = off[f"grid{e}_{l}"], off[f"grid{1 - e}_{l}"]
            n = int(np.prod(sh))
            sw[o1:o1 + n] = flat[o0:o0 + n]
        for t in ("W1", "b1", "W2", "b2", "W3", "b3"):
            (o0, sh), (o1, _) = off[f"{t}_{e}"], off[f"{t}_{1 - e}"]
            n = int(np.prod(sh))
            sw[o1:o1 + n] = flat[o0:o0 + n]
    refs = gen.random_vertices(V, 24, seed=12)
    out = _infer_gpu(c, _qparams(c, P), refs, V).cpu().numpy()
    out_sw = _infer_gpu(c, _qparams(c, torch.from_numpy(sw).cuda()), refs, V).cpu().numpy()
    for a in range(len(refs)):
        for b in range(len(refs)):
            assert out[a, refs[b]] == out_sw[b, refs[a]]
    # the cross field itself is not symmetric
    assert np.max(np.abs(out[:, refs] - out[:, refs].T)) > 1e-4


def test_infer_paper_size_sampled():
    cfg, lay, c, P, net = _setup("paper", 1, seed=2325)
    V = cfg.n_vertices
    q = _qparams(c, P)
    out = _infer_gpu(c, q, [cfg.ref_v], V)
    assert torch.isfinite(out).all()
    sample = np.unique(np.concatenate([gen.random_vertices(V, 3000, seed=31), [0, V - 1]]))
    g = out[0, torch.as_tensor(sample, device="cuda")].cpu().numpy()
    want, _ = nn.forward(net, np.full(len(sample), cfg.ref_v), sample)
    emul, _ = nn.forward(net, np.full(len(sample), cfg.ref_v), sample, BF16_OPS)
    _check_floor(g, want, emul, "infer paper")


def test_training_learns_pearson_field():
    """The learned field beats its initialisation and the best constant on
    held-out pairs of the tiny ensemble (targets from the direct GPU estimator,
    errors against the FP64 oracle)."""
    cfg = gen.CONFIGS["tiny"]
    x = gen.make_ensemble(cfg, device="cuda")
    e = ndf.Ensemble(x, cfg.nx, cfg.ny, cfg.nz)
    ndf.ndf_prepare(e)
    lay = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz)
    c = ndf.net_config(cfg.nx, cfg.ny, cfg.nz, lay.res)
    P = torch.empty(lay.n_floats, device="cuda")
    opt = torch.empty(2 * lay.n_floats, device="cuda")
    ndf.ndf_net_init(c, P, opt, 7)
    B = 4096
    ws = torch.empty(ndf.train_ws_bytes(c, B) + P.numel() * 4 + 256, dtype=torch.uint8,
                     device="cuda")
    loss = torch.empty(1, device="cuda")
    held = gen.random_pairs(cfg.n_vertices, 4000, seed=2399)
    xh = x[0].cpu().numpy()
    truth = np.array([direct.pearson(xh[:, a], xh[:, b]) for a, b in held])

    def mae():
        return np.mean(np.abs(_forward_gpu(c, P, held) - truth))

    mae0 = mae()
    losses = []
    for step in range(1, 401):
        pairs = torch.as_tensor(gen.random_pairs(cfg.n_vertices, B, seed=2312 + step),
                                device="cuda")
        t = ndf.pearson_pairs(e, pairs)
        ndf.ndf_train_step(c, P, opt, step, pairs, t, 3e-3, loss, ws)
        if step % 50 == 0:
            losses.append(loss.item())
    mae1 = mae()
    # the trained field through the fused inference kernels, BF16 and FP8
    q = _qparams(c, P, ndf.NDF_PREC_FP8_E4M3)
    refs = np.unique(held[:50, 0])
    f16 = _infer_gpu(c, q, refs, cfg.n_vertices, ndf.NDF_PREC_BF16).cpu().numpy()
    f8 = _infer_gpu(c, q, refs, cfg.n_vertices, ndf.NDF_PREC_FP8_E4M3).cpu().numpy()
    tru = np.stack([direct.pearson_field(xh[:, r], xh) for r in refs])
    mae16 = np.mean(np.abs(f16 - tru))
    mae8 = np.mean(np.abs(f8 - tru))
    _log(f"trained fields vs oracle: MAE bf16 {mae16:.4f} fp8 {mae8:.4f}")
    assert mae8 <= 1.25 * mae16 + 5e-3
    const = np.mean(np.abs(truth - np.median(truth)))
    _log(f"training: losses {['%.4f' % l for l in losses]} MAE init {mae0:.4f} "
         f"trained {mae1:.4f} best-constant {const:.4f}")
    assert losses[-1] < 0.6 * losses[0]
    assert mae1 < 0.5 * mae0 and mae1 < 0.6 * const


@pytest.mark.parametrize("name,n_enc", [("tiny", 1), ("mid", 1), ("mid", 2)])
def test_infer_field_fp8_parity(name, n_enc):
    """FP8 layers 2..5 (E4M3, 3 mantissa bits: unit roundoff 2^-4) on random
    weights, whose output is a small difference of O(1) terms, held to the FP64
    oracle with the same E4M3 operand rounding; BF16 of the same packed parameters
    to its bf16 floor.  The trained-network error is checked in the training test."""
    cfg, lay, c, P, net = _setup(name, n_enc, seed=2326)
    V = cfg.n_vertices
    refs = [cfg.ref_v, 0, V - 1]
    q = _qparams(c, P, ndf.NDF_PREC_FP8_E4M3)
    # the calibrated maxima of layers 2..5 (the blob's last 256 bytes start with
    # them) against the oracle's, up to one bf16 step (FP32 summation order)
    m_gpu = q[-256:-240].cpu().numpy().view(np.float32).astype(np.float64)
    m_o = nn.fp8_activation_maxima(net)
    _log(f"calibrated maxima gpu {m_gpu} oracle {m_o}")
    assert np.all(np.abs(m_gpu - m_o) <= 2.0 ** -7 * m_o)
    ops8 = nn.fp8_inference_operands(net, m_gpu)
    opsd = nn.fp8_decoder_operands(net, m_gpu)
    # one reference per call: layers 2..5 in E4M3; several: E4M3 decoder on the
    # cached BF16 query latents
    one8 = [_infer_gpu(c, q, [r], V, ndf.NDF_PREC_FP8_E4M3).cpu().numpy()[0] for r in refs]
    out8 = _infer_gpu(c, q, refs, V, ndf.NDF_PREC_FP8_E4M3).cpu().numpy()
    out16 = _infer_gpu(c, q, refs, V, ndf.NDF_PREC_BF16).cpu().numpy()
    for i, r in enumerate(refs):
        want = nn.field(net, r)
        _check_floor(one8[i], want, nn.field(net, r, rnd=ops8),
                     f"fp8 {name} n_enc={n_enc} ref={r}")
        _check_floor(out8[i], want, nn.field(net, r, rnd=opsd),
                     f"fp8 decoder {name} n_enc={n_enc} ref={r}")
        _check_floor(out16[i], want, nn.field(net, r, rnd=BF16_OPS),
                     f"bf16 of fp8 blob {name} n_enc={n_enc} ref={r}")


def test_infer_fp8_paper_size_sampled():
    cfg, lay, c, P, net = _setup("paper", 1, seed=2327)
    V = cfg.n_vertices
    q = _qparams(c, P, ndf.NDF_PREC_FP8_E4M3)
    out = _infer_gpu(c, q, [cfg.ref_v], V, ndf.NDF_PREC_FP8_E4M3)
    assert torch.isfinite(out).all()
    sample = gen.random_vertices(V, 3000, seed=32)
    g = out[0, torch.as_tensor(sample, device="cuda")].cpu().numpy()
    want, _ = nn.forward(net, np.full(len(sample), cfg.ref_v), sample)
    emul, _ = nn.forward(net, np.full(len(sample), cfg.ref_v), sample, fp8_ops(net))
    _check_floor(g, want, emul, "fp8 paper")


def test_correlation_volume_matrix_two_variables():
    """Multi-variable fields (Sec. 6.4): for d = 2 variables, three trained
    networks (Phi_00, Phi_11 self fields and the two-encoder Phi_01) give all four
    fields of the correlation volume matrix at a reference vertex, Phi_10 through
    the encoder swap.  Each field beats the best constant against the FP64 oracle,
    and the library's swap equals exchanging the encoder blocks by hand."""
    import dataclasses
    cfg = dataclasses.replace(gen.CONFIGS["tiny"], n_vars=2)
    x = gen.make_ensemble(cfg, device="cuda")
    e = ndf.Ensemble(x, cfg.nx, cfg.ny, cfg.nz)
    ndf.ndf_prepare(e)
    xh = x.cpu().numpy()
    V = cfg.n_vertices
    B = 4096

    def train(n_enc, va, vb, seed):
        lay = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz, n_enc=n_enc)
        c = ndf.net_config(cfg.nx, cfg.ny, cfg.nz, lay.res, n_enc=n_enc)
        P = torch.empty(lay.n_floats, device="cuda")
        opt = torch.empty(2 * lay.n_floats, device="cuda")
        ndf.ndf_net_init(c, P, opt, seed)
        ws = torch.empty(ndf.train_ws_bytes(c, B) + P.numel() * 4 + 256, dtype=torch.uint8,
                         device="cuda")
        loss = torch.empty(1, device="cuda")
        for step in range(1, 401):
            pairs = torch.as_tensor(gen.random_pairs(V, B, seed=4000 + 7 * seed + step),
                                    device="cuda")
            t = ndf.pearson_pairs(e, pairs, var_a=va, var_b=vb)
            ndf.ndf_train_step(c, P, opt, step, pairs, t, 3e-3, loss, ws)
        return lay, c, P

    nets = {(0, 0): train(1, 0, 0, 1), (1, 1): train(1, 1, 1, 2), (0, 1): train(2, 0, 1, 3)}
    lay01, c01, P01 = nets[(0, 1)]
    P10 = torch.empty_like(P01)
    ndf.ndf_net_swap_encoders(c01, P01, P10)
    # the swap by hand: encoder blocks exchanged, decoder kept
    flat, sw = P01.cpu().numpy(), P01.cpu().numpy().copy()
    off, _ = lay01.offsets()
    for enc in (0, 1):
        names = [f"grid{enc}_{l}" for l in range(lay01.n_levels)] + \
                [f"{t}_{enc}" for t in ("W1", "b1", "W2", "b2", "W3", "b3")]
        for name in names:
            o0, sh = off[name]
            o1, _ = off[name.replace(f"{enc}", f"{1 - enc}", 1) if name.startswith("grid")
                        else name[:-1] + str(1 - enc)]
            n = int(np.prod(sh))
            sw[o1:o1 + n] = flat[o0:o0 + n]
    assert np.array_equal(P10.cpu().numpy(), sw)
    nets[(1, 0)] = (lay01, c01, P10)
    ref = cfg.ref_v
    for (mu, nu), (lay, c, P) in sorted(nets.items()):
        field = _infer_gpu(c, _qparams(c, P), [ref], V).cpu().numpy()[0]
        want = direct.pearson_field(xh[mu][:, ref], xh[nu])
        mae = np.mean(np.abs(field - want))
        const = np.mean(np.abs(want - np.median(want)))
        _log(f"correlation volume ({mu},{nu}): MAE {mae:.4f} best constant {const:.4f}")
        assert mae < 0.3 * const, (mu, nu)


def _points_gpu(c, q, refs, pos, prec):
    pos_t = torch.as_tensor(pos, dtype=torch.float32, device="cuda").contiguous()
    out = torch.empty((len(refs), len(pos)), dtype=torch.float32, device="cuda")
    ws = torch.empty(ndf.infer_ws_bytes(c, len(refs), prec), dtype=torch.uint8, device="cuda")
    ndf.ndf_infer_points(c, q, prec, refs, pos_t, out, ws)
    return out.cpu().numpy()


@pytest.mark.parametrize("name,n_enc", [("tiny", 1), ("mid", 1), ("mid", 2)])
def test_infer_points_parity(name, n_enc):
    """The learned field at continuous positions, as a ray marcher samples it
    (Sec. 5): uniform positions in the domain, positions outside it (clamped),
    equally spaced samples along rays and the positions of grid vertices, 4517 in
    all (a ragged last tile).  BF16 and FP8 against the FP64 oracle, each held to
    its emulated rounding floor; at vertex positions the BF16 values equal the vertex
    field up to the FP32 rounding of the position (within 2% of the field RMS)."""
    cfg, lay, c, P, net = _setup(name, n_enc, seed=2330)
    V = cfg.n_vertices
    dims = (cfg.nx, cfg.ny, cfg.nz)
    vs = gen.random_vertices(V, 37, seed=44)
    vpos = (2.0 * nn.vertex_positions(vs, dims) - 1.0).astype(np.float32)
    pos = np.concatenate([gen.random_positions(3000, seed=41),
                          gen.random_positions(200, seed=42, spread=1.5),
                          gen.ray_positions(20, 64, seed=43), vpos]).astype(np.float32)
    refs = [cfg.ref_v, 0]
    q = _qparams(c, P, ndf.NDF_PREC_FP8_E4M3)
    out16 = _points_gpu(c, q, refs, pos, ndf.NDF_PREC_BF16)
    out8 = _points_gpu(c, q, refs, pos, ndf.NDF_PREC_FP8_E4M3)
    ops8 = fp8_ops(net)
    for i, r in enumerate(refs):
        p64 = pos.astype(np.float64)
        want = nn.field_points(net, r, p64)
        _check_floor(out16[i], want, nn.field_points(net, r, p64, BF16_OPS),
                     f"points {name} n_enc={n_enc} ref={r}")
        _check_floor(out8[i], want, nn.field_points(net, r, p64, ops8),
                     f"points fp8 {name} n_enc={n_enc} ref={r}")
    field = _infer_gpu(c, q, refs, V).cpu().numpy()[:, vs]
    for i in range(len(refs)):
        rms = np.sqrt(np.mean(field[i] ** 2))
        d = np.max(np.abs(out16[i, -len(vs):] - field[i]))
        _log(f"points at vertices vs vertex field: max|d| {d:.3g} (rms {rms:.3g})")
        assert d <= 0.02 * rms


def test_infer_field_difference():
    """Difference of two learned fields (Sec. 6.4) from the query-latent cache:
    bit for bit the FP32 difference of the two cached fields, zero for equal
    references, and within the BF16 bar of the FP64 difference."""
    cfg, lay, c, P, net = _setup("mid", 2, seed=2331)
    V = cfg.n_vertices
    q = _qparams(c, P)
    cache = torch.empty(ndf.ndf_infer_latent_bytes(c), dtype=torch.uint8, device="cuda")
    ndf.ndf_infer_latents(c, q, cache)
    a, b = cfg.ref_v, 5
    fields = torch.empty((2, V), device="cuda")
    ws = torch.empty(ndf.cached_ws_bytes(c, 2), dtype=torch.uint8, device="cuda")
    ndf.ndf_infer_field_cached(c, q, [a, b], cache, fields, ws)
    out = torch.full((V,), float("nan"), device="cuda")
    ndf.ndf_infer_field_difference(c, q, a, b, cache, out, ws)
    torch.cuda.synchronize()
    assert torch.equal(out, fields[0] - fields[1])
    same = torch.full((V,), float("nan"), device="cuda")
    ndf.ndf_infer_field_difference(c, q, a, a, cache, same, ws)
    assert torch.equal(same, torch.zeros_like(same))
    want = nn.field(net, a) - nn.field(net, b)
    emul = nn.field(net, a, rnd=BF16_OPS) - nn.field(net, b, rnd=BF16_OPS)
    _check_floor(out.cpu().numpy(), want, emul, "difference field")


# --------------------------------------------------------------- hash grids ----
def _setup_hash(name, n_enc, T, seed):
    cfg = gen.CONFIGS[name]
    lay = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz, n_enc=n_enc, log2_hashmap=T)
    flat = gen.make_net_params(lay, seed=seed, grid_scale=0.5, bias_scale=0.1)
    c = ndf.net_config(cfg.nx, cfg.ny, cfg.nz, lay.res, n_enc=n_enc, log2_hashmap=T)
    P = torch.from_numpy(flat).cuda()
    net = nn.Net(flat, (cfg.nx, cfg.ny, cfg.nz), lay.res, 8, 128, n_enc, T)
    return cfg, lay, c, P, net


@pytest.mark.parametrize("n_enc", [1, 2])
def test_hash_grid_forward_and_gradient(n_enc):
    """Hash-table levels (Sec. 4.2; T = 10 hashes every level of the mid grid
    above 1024 cells): the training forward and adjoint against the FP64 network
    with the same hash, at vertex pairs and at continuous positions (the
    vertex-pair tests' bars)."""
    cfg, lay, c, P, net = _setup_hash("mid", n_enc, 10, 2342)
    assert any(lay.cells(l) == 1024 for l in range(4))
    pairs = gen.random_pairs(cfg.n_vertices, 3000, seed=71)
    _check_floor(_forward_gpu(c, P, pairs), nn.forward(net, pairs[:, 0], pairs[:, 1])[0],
                 nn.forward(net, pairs[:, 0], pairs[:, 1], TRAIN_OPS)[0],
                 f"hash forward n_enc={n_enc}")
    pos = gen.random_positions(2 * 2048, seed=72).reshape(2048, 2, 3)
    y = nn.forward_points(net, pos)
    t = y + 1.0
    loss_o, g_o, _ = nn.loss_and_grad_points(net, pos, t)
    _, g_e, _ = nn.loss_and_grad_points(net, pos, t, TRAIN_OPS)
    g = torch.empty_like(P)
    loss = torch.empty(1, device="cuda")
    ws = torch.empty(ndf.train_ws_bytes(c, len(pos)), dtype=torch.uint8, device="cuda")
    ndf.ndf_net_grad_at(c, P, torch.as_tensor(pos, device="cuda"),
                        torch.as_tensor(t.astype(np.float32), device="cuda"), g, loss, ws)
    g = g.cpu().numpy().astype(np.float64)
    assert abs(loss.item() - loss_o) <= 1e-2 * loss_o
    check_grad_floor(lay, g, g_o.flat, g_e.flat, f"hash grad n_enc={n_enc}")


@pytest.mark.parametrize("n_enc", [1, 2])
def test_hash_grid_inference(n_enc):
    """Fused inference with hash-table levels: BF16 and FP8 fields and the field
    at continuous positions against the FP64 network; the cached-latent field
    bit for bit equal to the fused one."""
    cfg, lay, c, P, net = _setup_hash("mid", n_enc, 10, 2343)
    V = cfg.n_vertices
    refs = [cfg.ref_v, 0]
    q = _qparams(c, P, ndf.NDF_PREC_FP8_E4M3)
    out16 = _infer_gpu(c, q, refs, V, ndf.NDF_PREC_BF16)
    out8 = _infer_gpu(c, q, refs, V, ndf.NDF_PREC_FP8_E4M3).cpu().numpy()
    ops8 = fp8_decoder_ops(net)
    for i, r in enumerate(refs):
        want = nn.field(net, r)
        _check_floor(out16[i].cpu().numpy(), want, nn.field(net, r, rnd=BF16_OPS),
                     f"hash infer n_enc={n_enc} ref={r}")
        _check_floor(out8[i], want, nn.field(net, r, rnd=ops8),
                     f"hash infer fp8 n_enc={n_enc} ref={r}")
    pos = gen.random_positions(2000, seed=73)
    pts = _points_gpu(c, q, refs[:1], pos, ndf.NDF_PREC_BF16)
    p64 = pos.astype(np.float64)
    _check_floor(pts[0], nn.field_points(net, refs[0], p64),
                 nn.field_points(net, refs[0], p64, BF16_OPS), f"hash points n_enc={n_enc}")
    cache = torch.empty(ndf.ndf_infer_latent_bytes(c), dtype=torch.uint8, device="cuda")
    ndf.ndf_infer_latents(c, q, cache)
    oc = torch.empty((len(refs), V), device="cuda")
    ws = torch.empty(ndf.cached_ws_bytes(c, len(refs)), dtype=torch.uint8, device="cuda")
    ndf.ndf_infer_field_cached(c, q, refs, cache, oc, ws)
    single = torch.cat([_infer_gpu(c, q, [r], V, ndf.NDF_PREC_BF16) for r in refs])
    torch.cuda.synchronize()
    assert torch.equal(oc, single) and torch.equal(out16, single)


def test_hash_grid_paper_size_sampled():
    """The paper's grid with a 2^19-cell table: the finest level (1.76M cells) is
    hashed, the others dense; sampled vertices against the FP64 network."""
    cfg, lay, c, P, net = _setup_hash("paper", 1, 19, 2344)
    assert lay.cells(3) == 1 << 19
    V = cfg.n_vertices
    q = _qparams(c, P)
    out = _infer_gpu(c, q, [cfg.ref_v], V)
    sample = gen.random_vertices(V, 3000, seed=74)
    g = out[0, torch.as_tensor(sample, device="cuda")].cpu().numpy()
    want, _ = nn.forward(net, np.full(len(sample), cfg.ref_v), sample)
    emul, _ = nn.forward(net, np.full(len(sample), cfg.ref_v), sample, BF16_OPS)
    _check_floor(g, want, emul, "hash infer paper")


def test_field_calls_capture_into_a_graph():
    """A field call enqueues only kernels (no host copies, no memsets), so it can be
    captured into a graph: the fused field and the cached-latent field, each replayed
    three times with eager library work and synchronisations in between, equal the
    eager results bit for bit on every replay."""
    cfg, lay, c, P, net = _setup("mid", 1, seed=2345)
    V = cfg.n_vertices
    q = _qparams(c, P)
    ref, other = cfg.ref_v, 17
    want = _infer_gpu(c, q, [ref], V)
    cache = torch.empty(ndf.ndf_infer_latent_bytes(c), dtype=torch.uint8, device="cuda")
    ndf.ndf_infer_latents(c, q, cache)
    ws = torch.empty(ndf.infer_ws_bytes(c, 1, ndf.NDF_PREC_BF16), dtype=torch.uint8,
                     device="cuda")
    want_c = torch.empty((1, V), device="cuda")
    ndf.ndf_infer_field_cached(c, q, [ref], cache, want_c, ws)
    out = torch.empty((1, V), device="cuda")
    out_c = torch.empty((1, V), device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside the capture
        ndf.ndf_infer_field(c, q, ndf.NDF_PREC_BF16, [ref], out, ws)
        ndf.ndf_infer_field_cached(c, q, [ref], cache, out_c, ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ndf.ndf_infer_field(c, q, ndf.NDF_PREC_BF16, [ref], out, ws)
        ndf.ndf_infer_field_cached(c, q, [ref], cache, out_c, ws)
    for i in range(3):
        out.fill_(float("nan"))
        out_c.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want), i
        assert torch.equal(out_c, want_c), i
        _infer_gpu(c, q, [other], V)  # eager work between replays
        torch.cuda.synchronize()


# ----------------------------------------------------------- grid-only network --
@pytest.mark.parametrize("name,n_enc", [("tiny", 1), ("mid", 2)])
def test_grid_only_network(name, n_enc):
    """The grid-only network (encoder MLP omitted; the ablation of Sec. 6.3): its
    parameter layout, initialisation, training forward and adjoint, and BF16
    field and position inference against the FP64 oracle of the same network, to
    the emulated rounding floors; FP8 and the query-latent calls are refused."""
    cfg = gen.CONFIGS[name]
    dims = (cfg.nx, cfg.ny, cfg.nz)
    lay = gen.NetLayout.for_grid(*dims, n_enc=n_enc, grid_only=True)
    flat = gen.make_net_params(lay, seed=2345, grid_scale=0.5, bias_scale=0.1)
    c = ndf.net_config(*dims, lay.res, n_enc=n_enc, grid_only=True)
    assert ndf.ndf_net_param_bytes(c) == 4 * lay.n_floats
    net = nn.Net(flat, dims, lay.res, 8, 128, n_enc, grid_only=True)
    P = torch.from_numpy(flat).cuda()
    # initialisation: W4 He-uniform over its 32 inputs, no encoder tensors
    P0 = torch.empty_like(P)
    ndf.ndf_net_init(c, P0, None, 11)
    w4 = lay.view(P0.cpu().numpy(), "W4")
    assert w4.shape == (128, 32) and np.all(np.abs(w4) <= math.sqrt(6.0 / 32))
    assert w4.std() > 0.5 * math.sqrt(6.0 / 32) / math.sqrt(3)
    pairs = gen.random_pairs(cfg.n_vertices, 2048, seed=77)
    y = _forward_gpu(c, P, pairs)
    want, _ = nn.forward(net, pairs[:, 0], pairs[:, 1])
    _check_floor(y, want, nn.forward(net, pairs[:, 0], pairs[:, 1], TRAIN_OPS)[0],
                 f"grid-only forward {name} n_enc={n_enc}")
    s = np.where(np.random.default_rng(6).random(len(pairs)) < 0.5, -1.0, 1.0)
    t = want - s
    loss_o, g_o, _ = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], t)
    _, g_e, _ = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], t, TRAIN_OPS)
    g, loss = _grad_gpu(c, P, pairs, t.astype(np.float32))
    assert abs(loss - loss_o) <= 1e-2 * loss_o
    check_grad_floor(lay, g, g_o.flat, g_e.flat, f"grid-only grad {name} n_enc={n_enc}")
    V = cfg.n_vertices
    refs = [cfg.ref_v, 0, V - 1]
    q = _qparams(c, P, ndf.NDF_PREC_BF16)
    out = _infer_gpu(c, q, refs, V).cpu().numpy()
    for i, r in enumerate(refs):
        _check_floor(out[i], nn.field(net, r), nn.field(net, r, rnd=BF16_OPS),
                     f"grid-only field {name} n_enc={n_enc} ref={r}")
    pos = gen.random_positions(1500, seed=78)
    pts = _points_gpu(c, q, refs[:1], pos, ndf.NDF_PREC_BF16)
    p64 = pos.astype(np.float64)
    _check_floor(pts[0], nn.field_points(net, refs[0], p64),
                 nn.field_points(net, refs[0], p64, BF16_OPS), f"grid-only points {name}")
    with pytest.raises(ndf.NdfError):
        _qparams(c, P, ndf.NDF_PREC_FP8_E4M3)
    with pytest.raises(ndf.NdfError):
        _infer_gpu(c, q, refs[:1], V, ndf.NDF_PREC_FP8_E4M3)
    cache = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(ndf.NdfError):
        ndf.ndf_infer_latents(c, q, cache)


@pytest.mark.parametrize("name,T", [("tiny", 0), ("mid", 0), ("mid", 10)])
def test_fourier_feature_network(name, T):
    """Fourier features of the position (Sec. 4.2, Eq. 4; L = 12, 112 encoder
    inputs): the training forward and adjoint at vertex pairs (B = 2001, a
    ragged last tile) and at continuous positions, BF16 and FP8 fields, the field
    at positions, all against the FP64 network to the emulated rounding floors;
    the query-latent path equals the fused field bit for bit; two encoders are
    refused."""
    cfg = gen.CONFIGS[name]
    dims = (cfg.nx, cfg.ny, cfg.nz)
    lay = gen.NetLayout.for_grid(*dims, log2_hashmap=T, fourier=12)
    assert lay.enc_in == 112
    flat = gen.make_net_params(lay, seed=2351, grid_scale=0.5, bias_scale=0.1)
    c = ndf.net_config(*dims, lay.res, log2_hashmap=T, fourier=12)
    assert ndf.ndf_net_param_bytes(c) == 4 * lay.n_floats
    net = nn.Net(flat, dims, lay.res, 8, 128, 1, T, fourier=12)
    P = torch.from_numpy(flat).cuda()
    P0 = torch.empty_like(P)
    ndf.ndf_net_init(c, P0, None, 12)
    w1 = lay.view(P0.cpu().numpy(), "W1_0")
    assert w1.shape == (128, 112) and np.all(np.abs(w1) <= math.sqrt(6.0 / 112))
    pairs = gen.random_pairs(cfg.n_vertices, 2001, seed=79)
    y = _forward_gpu(c, P, pairs)
    want, _ = nn.forward(net, pairs[:, 0], pairs[:, 1])
    _check_floor(y, want, nn.forward(net, pairs[:, 0], pairs[:, 1], TRAIN_OPS)[0],
                 f"fourier forward {name} T={T}")
    s = np.where(np.random.default_rng(8).random(len(pairs)) < 0.5, -1.0, 1.0)
    t = want - s
    loss_o, g_o, _ = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], t)
    _, g_e, _ = nn.loss_and_grad(net, pairs[:, 0], pairs[:, 1], t, TRAIN_OPS)
    g, loss = _grad_gpu(c, P, pairs, t.astype(np.float32))
    assert abs(loss - loss_o) <= 1e-2 * loss_o
    check_grad_floor(lay, g, g_o.flat, g_e.flat, f"fourier grad {name} T={T}")
    # continuous positions, some outside the domain
    pos = np.concatenate([gen.random_positions(2 * 1500, seed=80),
                          gen.random_positions(2 * 100, seed=81, spread=1.5)]).reshape(1600, 2, 3)
    y = nn.forward_points(net, pos)
    t = y + 1.0
    loss_o, g_o, _ = nn.loss_and_grad_points(net, pos, t)
    _, g_e, _ = nn.loss_and_grad_points(net, pos, t, TRAIN_OPS)
    gp = torch.empty_like(P)
    lossp = torch.empty(1, device="cuda")
    ws = torch.empty(ndf.train_ws_bytes(c, len(pos)), dtype=torch.uint8, device="cuda")
    ndf.ndf_net_grad_at(c, P, torch.as_tensor(pos, device="cuda"),
                        torch.as_tensor(t.astype(np.float32), device="cuda"), gp, lossp, ws)
    assert abs(lossp.item() - loss_o) <= 1e-2 * loss_o
    check_grad_floor(lay, gp.cpu().numpy().astype(np.float64), g_o.flat, g_e.flat,
                     f"fourier grad at positions {name} T={T}")
    # inference
    V = cfg.n_vertices
    refs = [cfg.ref_v, 0, V - 1]
    q = _qparams(c, P, ndf.NDF_PREC_FP8_E4M3)
    f16 = _infer_gpu(c, q, refs, V, ndf.NDF_PREC_BF16)
    f8 = _infer_gpu(c, q, refs, V, ndf.NDF_PREC_FP8_E4M3).cpu().numpy()
    ops8, opsd = fp8_ops(net), fp8_decoder_ops(net)
    for i, r in enumerate(refs):
        want = nn.field(net, r)
        _check_floor(f16[i].cpu().numpy(), want, nn.field(net, r, rnd=BF16_OPS),
                     f"fourier field {name} T={T} ref={r}")
        _check_floor(f8[i], want, nn.field(net, r, rnd=opsd),
                     f"fourier field fp8 decoder {name} T={T} ref={r}")
        one8 = _infer_gpu(c, q, [r], V, ndf.NDF_PREC_FP8_E4M3).cpu().numpy()[0]
        _check_floor(one8, want, nn.field(net, r, rnd=ops8),
                     f"fourier field fp8 {name} T={T} ref={r}")
        one = _infer_gpu(c, q, [r], V, ndf.NDF_PREC_BF16)
        assert torch.equal(one[0], f16[i]), r  # query-latent path = fused field
    pq = gen.random_positions(2500, seed=82)
    pts = _points_gpu(c, q, refs[:1], pq, ndf.NDF_PREC_BF16)
    p64 = pq.astype(np.float64)
    _check_floor(pts[0], nn.field_points(net, refs[0], p64),
                 nn.field_points(net, refs[0], p64, BF16_OPS), f"fourier points {name} T={T}")
    c2 = ndf.net_config(*dims, lay.res, n_enc=2, log2_hashmap=T, fourier=12)
    assert ndf.ndf_net_param_bytes(c2) == 0
