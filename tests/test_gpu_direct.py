"""GPU parity of the direct estimators against the FP64 oracle, through the C ABI.

Tolerances: Pearson |dr| <= 1e-5 (FP32 stream and split-BF16 MFMA), KSG neighbour
counts bit-exact and MI |dI| <= 1e-4 nats; codes bit-exact; moments to 1e-12.
Sizes: the tiny ensemble (64 members, 2048 vertices) in full, a mid ensemble
with ragged tails everywhere (200 members, 37x29x11 = 11803 vertices) in full,
and the paper-shaped ensemble (1000 members, 1.76M vertices) on sampled vertices
at the launch configuration the benchmark times.
"""
import math
import sys

import numpy as np
import pytest
import torch

import gen
from oracle import direct
from paper_2307_02203_amd import ndf

pytestmark = pytest.mark.gpu

PEARSON_TOL = 1e-5
MI_TOL = 1e-4


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _ens(cfg, device="cuda"):
    x = gen.make_ensemble(cfg, device=device)
    e = ndf.Ensemble(x, cfg.nx, cfg.ny, cfg.nz)
    ndf.ndf_prepare(e)
    torch.cuda.synchronize()
    return e


@pytest.fixture(scope="module")
def tiny():
    return _ens(gen.CONFIGS["tiny"])


@pytest.fixture(scope="module")
def mid():
    return _ens(gen.CONFIGS["mid"])


def _cols(e, var, idx):
    """Member-major host block x[var][:, idx] (float32) for the oracle."""
    idx = torch.as_tensor(np.asarray(idx), dtype=torch.int64, device=e.device)
    return e.x[var][:, idx].cpu().numpy()


@pytest.mark.parametrize("name", ["tiny", "mid"])
def test_prepare_stats_and_codes(name, request):
    e = request.getfixturevalue(name)
    x = e.x[0].cpu().numpy()
    mean = e.mean[0].cpu().numpy()
    istd = e.inv_std[0].cpu().numpy()
    code = e.code[0].cpu().numpy()
    flags = e.flags[0].cpu().numpy()
    V = e.n_vertices
    assert np.all(flags == 0)
    for v in range(V):
        m, s = direct.moments(x[:, v])
        assert abs(mean[v] - m) <= 1e-12 * max(1.0, abs(m))
        assert abs(istd[v] * s - 1.0) <= 1e-12
        c, flat = direct.ksg_codes(x[:, v])
        assert not flat
        assert np.array_equal(code[v], c), v


def test_prepare_flags_constant_and_nonfinite():
    cfg = gen.CONFIGS["tiny"]
    x = gen.make_ensemble(cfg, device="cuda")
    x[0, :, 7] = 2.5                     # constant column
    x[0, 3, 9] = float("nan")            # non-finite sample
    e = ndf.Ensemble(x, cfg.nx, cfg.ny, cfg.nz)
    ws = torch.full((ndf.ndf_workspace_bytes(ndf.NDF_OP_PREPARE, e),), 0x55, dtype=torch.uint8,
                    device="cuda")
    ndf.ndf_prepare(e, ws)
    torch.cuda.synchronize()
    assert ndf.status_word(ws) == ndf.NDF_E_NONFINITE     # the device status word
    f = e.flags[0].cpu().numpy()
    assert f[7] == ndf.NDF_FLAG_CONSTANT and f[9] & ndf.NDF_FLAG_NONFINITE
    assert np.sum(f != 0) == 2
    assert e.inv_std[0, 7].item() == 0.0
    assert torch.all(e.code[0, 7] == 0)
    r = ndf.pearson_field(e, [1160])[0].cpu().numpy()
    assert r[7] == 0.0
    r7 = ndf.pearson_field(e, [7])[0].cpu().numpy()
    assert np.all(np.delete(r7, 9) == 0.0)           # the NaN column stays NaN
    assert math.isnan(r[9]) and math.isnan(r7[9])
    mi = ndf.ksg_field(e, [1160])[0].cpu().numpy()
    assert mi[7] == 0.0 and math.isnan(mi[9])
    # a finite ensemble (a constant column is finite) leaves the word at NDF_OK
    x[0, 3, 9] = 1.0
    ndf.ndf_prepare(e, ws)
    torch.cuda.synchronize()
    assert ndf.status_word(ws) == ndf.NDF_OK


@pytest.mark.parametrize("n_ref", [100, 300])
def test_pearson_many_references_one_pass(mid, n_ref):
    """More than 64 references run as one read of the ensemble per 256 references
    (four waves share each staged block of members): every field of a ragged
    batch (100: two of the four waves partly idle; 300: a second pass of 44) on
    the mid ensemble (11803 vertices, no 16-byte row alignment) against the
    oracle, and bit for bit equal to the same references in calls of 64."""
    V = mid.n_vertices
    refs = gen.random_vertices(V, n_ref, seed=16 + n_ref)
    _log(f"split-BF16 Pearson, {n_ref} references, mid")
    got = ndf.pearson_field(mid, refs, prec=ndf.NDF_PREC_SPLIT_BF16)
    x = mid.x[0].cpu().numpy()
    g = got.cpu().numpy()
    worst = 0.0
    for i in range(0, n_ref, 7):
        worst = max(worst, float(np.max(np.abs(g[i] - direct.pearson_field(x[:, refs[i]], x)))))
    _log(f"{n_ref} refs: max|dr| {worst:.2e}")
    assert worst <= PEARSON_TOL
    for r0 in range(0, n_ref, 64):
        part = ndf.pearson_field(mid, refs[r0:r0 + 64], prec=ndf.NDF_PREC_SPLIT_BF16)
        assert torch.equal(part, got[r0:r0 + 64]), r0


@pytest.mark.parametrize("name", ["tiny", "mid"])
@pytest.mark.parametrize("prec", [ndf.NDF_PREC_FP32, ndf.NDF_PREC_SPLIT_BF16])
def test_pearson_field_full(name, prec, request):
    e = request.getfixturevalue(name)
    cfg = gen.CONFIGS[name]
    refs = [cfg.ref_v, 0, e.n_vertices - 1]
    got = ndf.pearson_field(e, refs, prec=prec).cpu().numpy()
    x = e.x[0].cpu().numpy()
    for i, r in enumerate(refs):
        want = direct.pearson_field(x[:, r], x)
        err = np.max(np.abs(got[i] - want))
        _log(f"pearson {name} prec={prec} ref={r} max|err|={err:.2e}")
        assert err <= PEARSON_TOL
    assert abs(got[0][cfg.ref_v] - 1.0) <= PEARSON_TOL


@pytest.mark.parametrize("n_ref", [1, 5, 32, 33, 64, 70])
def test_pearson_batch_split_bf16(mid, n_ref):
    refs = gen.random_vertices(mid.n_vertices, n_ref, seed=40 + n_ref)
    got = ndf.pearson_field(mid, refs, prec=ndf.NDF_PREC_SPLIT_BF16).cpu().numpy()
    x = mid.x[0].cpu().numpy()
    for i, r in enumerate(refs):
        want = direct.pearson_field(x[:, r], x)
        assert np.max(np.abs(got[i] - want)) <= PEARSON_TOL, (n_ref, i)


@pytest.mark.parametrize("name", ["tiny", "mid"])
@pytest.mark.parametrize("k", [1, 3, 4, 8])
def test_ksg_field_full_counts_exact(name, k, request):
    e = request.getfixturevalue(name)
    cfg = gen.CONFIGS[name]
    ref = cfg.ref_v
    mi, cnt = ndf.ksg_field(e, [ref], k=k, counts=True)
    mi = mi[0].cpu().numpy()
    cnt = cnt[0].cpu().numpy()
    x = e.x[0].cpu().numpy()
    want, wnx, wny = direct.ksg_field(x[:, ref], x, k, counts=True)
    assert np.array_equal(cnt[:, 0, :], wnx)
    assert np.array_equal(cnt[:, 1, :], wny)
    err = np.max(np.abs(mi - want))
    _log(f"ksg {name} k={k} max|dI|={err:.2e}")
    assert err <= MI_TOL


def test_ksg_pairs_match_oracle_and_field(mid):
    cfg = gen.CONFIGS["mid"]
    rng = np.random.default_rng(3)
    pairs = np.stack([rng.integers(0, mid.n_vertices, 300),
                      rng.integers(0, mid.n_vertices, 300)], axis=1)
    pairs[:20, 0] = cfg.ref_v
    mi, cnt = ndf.ksg_pairs(mid, pairs, k=4, counts=True)
    mi = mi.cpu().numpy()
    cnt = cnt.cpu().numpy()
    x = mid.x[0].cpu().numpy()
    for b, (a, q) in enumerate(pairs):
        want, wnx, wny = direct.ksg_field(x[:, a], x[:, q:q + 1], 4, counts=True)
        assert np.array_equal(cnt[b, 0], wnx[0]) and np.array_equal(cnt[b, 1], wny[0]), b
        assert abs(mi[b] - want[0]) <= MI_TOL
    # the same sample ordering and summation as the field kernel: bit-identical
    field = ndf.ksg_field(mid, [cfg.ref_v], k=4)[0].cpu().numpy()
    assert np.array_equal(mi[:20], field[pairs[:20, 1]])


def test_pearson_pairs_match_oracle(mid):
    rng = np.random.default_rng(4)
    pairs = np.stack([rng.integers(0, mid.n_vertices, 500),
                      rng.integers(0, mid.n_vertices, 500)], axis=1)
    got = ndf.pearson_pairs(mid, pairs).cpu().numpy()
    x = mid.x[0].cpu().numpy()
    want = np.array([direct.pearson(x[:, a], x[:, b]) for a, b in pairs])
    assert np.max(np.abs(got - want)) <= PEARSON_TOL


def test_odd_member_count_all_estimators():
    """N = 75 (not a multiple of 4): the scalar row paths of the Pearson pairs and
    the ragged last k-step of the split-BF16 contraction, with KSG counts exact."""
    cfg = gen.CONFIGS["tiny"].with_members(75)
    e = _ens(cfg)
    x = e.x[0].cpu().numpy()
    refs = [cfg.ref_v, 3]
    for prec in (ndf.NDF_PREC_FP32, ndf.NDF_PREC_SPLIT_BF16):
        got = ndf.pearson_field(e, refs, prec=prec).cpu().numpy()
        for i, r in enumerate(refs):
            assert np.max(np.abs(got[i] - direct.pearson_field(x[:, r], x))) <= PEARSON_TOL
    pairs = gen.random_pairs(cfg.n_vertices, 300, seed=75)
    r = ndf.pearson_pairs(e, pairs).cpu().numpy()
    want = np.array([direct.pearson(x[:, a], x[:, b]) for a, b in pairs])
    assert np.max(np.abs(r - want)) <= PEARSON_TOL
    mi, cnt = ndf.ksg_pairs(e, pairs[:60], k=4, counts=True)
    mi, cnt = mi.cpu().numpy(), cnt.cpu().numpy()
    for b, (a, q) in enumerate(pairs[:60]):
        w, wnx, wny = direct.ksg_field(x[:, a], x[:, q:q + 1], 4, counts=True)
        assert np.array_equal(cnt[b, 0], wnx[0]) and np.array_equal(cnt[b, 1], wny[0]), b
        assert abs(mi[b] - w[0]) <= MI_TOL


@pytest.mark.parametrize("n_members", [11, 75])
def test_pearson_split_bf16_short_and_ragged_members(n_members):
    """Split-BF16 Pearson with fewer members than one 16-member k-step (N = 11) and with a
    ragged last k-step (N = 75), through every contraction kernel: 5 references (one
    32-reference block), 33 (two blocks), 100 (the one-pass many-reference kernel, whose
    loads past the last member read member N - 1 against a zero reference operand).
    Against the oracle, and the 100-reference call bit for bit against calls of 64.

    The bar is the split's own arithmetic bound.  With z = hi + lo in bf16 (unit
    roundoff 2^-8) each side carries |hi + lo - z| <= 2^-16 |z|, and the dropped lo*lo term
    is <= 2^-16 |z_r z_v|, so every product is off by at most 3 * 2^-16 |z_r z_v| and
    |dr| <= 3 * 2^-16 * mean_m |z_r z_v| (<= 4.6e-5 by Cauchy-Schwarz), plus FP32 slack.
    Over many members the per-member errors cancel far below it (the 1e-5 gate of the
    configured ensembles); over 11 members they do not."""
    cfg = gen.CONFIGS["tiny"].with_members(n_members)
    e = _ens(cfg)
    x = e.x[0].cpu().numpy()
    V = cfg.n_vertices
    xd = x.astype(np.float64)
    z = (xd - xd.mean(axis=0)) / xd.std(axis=0)
    refs = np.concatenate([[cfg.ref_v], gen.random_vertices(V, 99, seed=500 + n_members)])
    for n_ref in (5, 33, 100):
        _log(f"split-BF16 Pearson, N={n_members}, {n_ref} references")
        got = ndf.pearson_field(e, refs[:n_ref], prec=ndf.NDF_PREC_SPLIT_BF16).cpu().numpy()
        worst = 0.0
        for i, r in enumerate(refs[:n_ref]):
            err = np.abs(got[i] - direct.pearson_field(x[:, r], x))
            bound = 3.0 * 2.0 ** -16 * np.mean(np.abs(z[:, r:r + 1] * z), axis=0) + 1e-6
            assert np.all(err <= bound), (n_members, n_ref, i, float(np.max(err - bound)))
            worst = max(worst, float(np.max(err)))
        _log(f"  max|dr| {worst:.2e}")
    whole = ndf.pearson_field(e, refs, prec=ndf.NDF_PREC_SPLIT_BF16)
    for r0 in range(0, 100, 64):
        part = ndf.pearson_field(e, refs[r0:r0 + 64], prec=ndf.NDF_PREC_SPLIT_BF16)
        assert torch.equal(part, whole[r0:r0 + 64]), r0


@pytest.mark.parametrize("n_members", [96, 100, 120, 140, 150, 170, 192])
def test_pearson_many_refs_every_kstep_count(n_members):
    """The many-reference kernel runs its k-steps six to a loop iteration (three LDS
    buffers, three x register sets, two fragment sets) with the remaining one to five
    after the loop: member counts whose 16-member k-step counts are 6 .. 12 take every
    remainder.  100 references through it, bit for bit against calls of 64 (the
    64-reference kernel, another code path), and three of them against the oracle
    within the split's arithmetic bound."""
    cfg = gen.CONFIGS["tiny"].with_members(n_members)
    e = _ens(cfg)
    x = e.x[0].cpu().numpy()
    V = cfg.n_vertices
    xd = x.astype(np.float64)
    z = (xd - xd.mean(axis=0)) / xd.std(axis=0)
    refs = np.concatenate([[cfg.ref_v], gen.random_vertices(V, 99, seed=700 + n_members)])
    _log(f"split-BF16 Pearson, N={n_members} ({(n_members + 15) // 16} k-steps), 100 references")
    whole = ndf.pearson_field(e, refs, prec=ndf.NDF_PREC_SPLIT_BF16)
    for r0 in range(0, 100, 64):
        part = ndf.pearson_field(e, refs[r0:r0 + 64], prec=ndf.NDF_PREC_SPLIT_BF16)
        assert torch.equal(part, whole[r0:r0 + 64]), r0
    got = whole.cpu().numpy()
    for i in (0, 37, 99):
        r = refs[i]
        err = np.abs(got[i] - direct.pearson_field(x[:, r], x))
        bound = 3.0 * 2.0 ** -16 * np.mean(np.abs(z[:, r:r + 1] * z), axis=0) + 1e-6
        assert np.all(err <= bound), (n_members, i, float(np.max(err - bound)))


def test_ksg_without_stored_orders_matches(mid):
    """An ensemble prepared without the per-vertex sorted orders (order = NULL):
    the KSG kernels sort every column themselves and give bit-identical fields,
    counts and pair estimates."""
    cfg = gen.CONFIGS["mid"]
    e = ndf.Ensemble(mid.x, cfg.nx, cfg.ny, cfg.nz, orders=False)
    ndf.ndf_prepare(e)
    refs = [cfg.ref_v, 7]
    a, ca = ndf.ksg_field(mid, refs, k=4, counts=True)
    b, cb = ndf.ksg_field(e, refs, k=4, counts=True)
    assert torch.equal(a, b) and torch.equal(ca, cb)
    pairs = gen.random_pairs(cfg.n_vertices, 200, seed=8)
    assert torch.equal(ndf.ksg_pairs(mid, pairs), ndf.ksg_pairs(e, pairs))
    # the stored orders themselves: ascending codes, ties by member index
    codes = mid.code[0].cpu().numpy().astype(np.int64)
    order = mid.order[0].cpu().numpy().astype(np.int64) & 0xFFFF
    keys = codes * 65536 + np.arange(cfg.n_members)[None, :]
    assert np.array_equal(np.take_along_axis(keys, order, axis=1), np.sort(keys, axis=1))


@pytest.mark.parametrize("n_members", [1000, 200, 100])
def test_stored_orders_with_near_ties(n_members):
    """Sorted member orders on columns built to defeat the 32-bit sort keys: codes
    that agree above their two lowest bits (few distinct values, many repeats) and
    columns of many near-equal codes next to well-spread ones.  The stored order
    must be ascending (code, member) exactly, and the KSG counts of such pairs must
    equal the oracle's."""
    rng = np.random.default_rng(31)
    V = 96
    x = rng.standard_normal((1, n_members, V)).astype(np.float32)
    lo, hi = -1.0, 1.0
    step = (hi - lo) / 2.0 ** 23
    for v in range(0, V, 3):
        # codes 0..7 (two groups of four sharing code >> 2), plus the two range ends
        x[0, :, v] = lo + step * rng.integers(0, 8, n_members)
        x[0, 0, v], x[0, 1, v] = lo, hi
    for v in range(1, V, 3):
        # a dense cluster of codes 0..40 among spread values
        x[0, : n_members // 2, v] = lo + step * rng.integers(0, 41, n_members // 2)
        x[0, n_members // 2:, v] = rng.uniform(lo, hi, n_members - n_members // 2)
        x[0, 0, v], x[0, 1, v] = lo, hi
    xt = torch.from_numpy(x).cuda()
    e = ndf.Ensemble(xt, 6, 4, 4)
    ndf.ndf_prepare(e)
    torch.cuda.synchronize()
    codes = e.code[0].cpu().numpy().astype(np.int64)
    want_codes = np.stack([direct.ksg_codes(x[0][:, v])[0] for v in range(V)])
    assert np.array_equal(codes, want_codes)
    order = e.order[0].cpu().numpy().astype(np.int64) & 0xFFFF
    keys = codes * 65536 + np.arange(n_members)[None, :]
    assert np.array_equal(np.take_along_axis(keys, order, axis=1), np.sort(keys, axis=1))
    pairs = np.array([[0, 1], [3, 4], [1, 2], [6, 7], [9, 10]], dtype=np.int64)
    mi, cnt = ndf.ksg_pairs(e, pairs, k=4, counts=True)
    cnt = cnt.cpu().numpy()
    for b, (a, q) in enumerate(pairs):
        w, wnx, wny = direct.ksg_field(x[0][:, a], x[0][:, q:q + 1], 4, counts=True)
        assert np.array_equal(cnt[b, 0], wnx[0]) and np.array_equal(cnt[b, 1], wny[0]), b


def test_pairs_out_of_range_give_nan(mid):
    pairs = np.array([[0, 1], [-1, 3], [5, mid.n_vertices]], dtype=np.int64)
    r = ndf.pearson_pairs(mid, pairs).cpu().numpy()
    mi = ndf.ksg_pairs(mid, pairs).cpu().numpy()
    assert np.isfinite(r[0]) and np.isnan(r[1]) and np.isnan(r[2])
    assert np.isfinite(mi[0]) and np.isnan(mi[1]) and np.isnan(mi[2])


def test_ksg_field_is_deterministic(mid):
    a = ndf.ksg_field(mid, [gen.CONFIGS["mid"].ref_v, 17], k=4)
    b = ndf.ksg_field(mid, [gen.CONFIGS["mid"].ref_v, 17], k=4)
    assert torch.equal(a, b)


# ------------------------------------------------------ paper-shaped sizes --
@pytest.fixture(scope="module")
def paper():
    cfg = gen.CONFIGS["paper"]
    _log("generating paper-shaped ensemble (1000 x 1.76M)")
    e = _ens(cfg)
    return e


def test_paper_pearson_and_ksg_sampled(paper):
    cfg = gen.CONFIGS["paper"]
    ref = cfg.ref_v
    V = paper.n_vertices
    sample = np.unique(np.concatenate([
        gen.random_vertices(V, 400, seed=77), [0, 1, V - 1, V - 2, ref, ref + 1]]))
    xr = _cols(paper, 0, [ref])[:, 0]
    xs = _cols(paper, 0, sample)
    # stats and codes at the sampled vertices
    mean = paper.mean[0][torch.as_tensor(sample, device="cuda")].cpu().numpy()
    code = paper.code[0][torch.as_tensor(sample, device="cuda")].cpu().numpy()
    for i in range(len(sample)):
        m, _ = direct.moments(xs[:, i])
        assert abs(mean[i] - m) <= 1e-12 * max(1.0, abs(m))
        c, _ = direct.ksg_codes(xs[:, i])
        assert np.array_equal(code[i], c)
    want_r = direct.pearson_field(xr, xs)
    for prec in (ndf.NDF_PREC_FP32, ndf.NDF_PREC_SPLIT_BF16):
        got = ndf.pearson_field(paper, [ref], prec=prec)[0]
        g = got[torch.as_tensor(sample, device="cuda")].cpu().numpy()
        err = np.max(np.abs(g - want_r))
        _log(f"paper pearson prec={prec} sampled max|err|={err:.2e}")
        assert err <= PEARSON_TOL
        # properties at every vertex: finite, within [-1, 1] (+ rounding), 1 at ref
        assert torch.isfinite(got).all()
        assert got.abs().max().item() <= 1.0 + 1e-5
        assert abs(got[ref].item() - 1.0) <= PEARSON_TOL
    want_mi = direct.ksg_field(xr, xs, 4)
    mi = ndf.ksg_field(paper, [ref], k=4)[0]
    g = mi[torch.as_tensor(sample, device="cuda")].cpu().numpy()
    err = np.max(np.abs(g - want_mi))
    _log(f"paper ksg sampled max|dI|={err:.2e}")
    assert err <= MI_TOL
    assert torch.isfinite(mi).all()
    # the reference itself: y == x, so I = H_{N-1} - H_{k-1} when no codes tie
    assert abs(mi[ref].item() - 5.651137527217) <= MI_TOL


def test_paper_pearson_batch64_sampled(paper):
    cfg = gen.CONFIGS["paper"]
    V = paper.n_vertices
    refs = np.concatenate([[cfg.ref_v], gen.random_vertices(V, 63, seed=2311)])
    got = ndf.pearson_field(paper, refs, prec=ndf.NDF_PREC_SPLIT_BF16)
    sample = gen.random_vertices(V, 200, seed=91)
    xs = _cols(paper, 0, sample)
    xr = _cols(paper, 0, refs)
    g = got[:, torch.as_tensor(sample, device="cuda")].cpu().numpy()
    for i in range(len(refs)):
        want = direct.pearson_field(xr[:, i], xs)
        assert np.max(np.abs(g[i] - want)) <= PEARSON_TOL, i
    diag = got[torch.arange(64, device="cuda"), torch.as_tensor(refs, device="cuda")]
    assert torch.all((diag - 1.0).abs() <= PEARSON_TOL)


def test_paper_ksg_pairs_counts_exact(paper):
    V = paper.n_vertices
    pairs = gen.random_pairs(V, 64, seed=2312)
    mi, cnt = ndf.ksg_pairs(paper, pairs, k=4, counts=True)
    mi = mi.cpu().numpy()
    cnt = cnt.cpu().numpy()
    xa = _cols(paper, 0, pairs[:, 0])
    xb = _cols(paper, 0, pairs[:, 1])
    for b in range(len(pairs)):
        want, wnx, wny = direct.ksg_field(xa[:, b], xb[:, b:b + 1], 4, counts=True)
        assert np.array_equal(cnt[b, 0], wnx[0]) and np.array_equal(cnt[b, 1], wny[0])
        assert abs(mi[b] - want[0]) <= MI_TOL


def test_cross_variable_fields():
    """R_{mu nu}(p_ref, .) with mu != nu (Sec. 3): reference in variable 0, queries
    in variable 1 of a two-variable ensemble, and the reverse."""
    import dataclasses
    cfg = dataclasses.replace(gen.CONFIGS["mid"], n_vars=2)
    x = gen.make_ensemble(cfg, device="cuda")
    e = ndf.Ensemble(x, cfg.nx, cfg.ny, cfg.nz)
    ndf.ndf_prepare(e)
    xh = x.cpu().numpy()
    ref = cfg.ref_v
    for vr, vq in ((0, 1), (1, 0)):
        want = direct.pearson_field(xh[vr][:, ref], xh[vq])
        for prec in (ndf.NDF_PREC_FP32, ndf.NDF_PREC_SPLIT_BF16):
            got = ndf.pearson_field(e, [ref], prec=prec, var_ref=vr, var_qry=vq)[0].cpu().numpy()
            assert np.max(np.abs(got - want)) <= PEARSON_TOL
        mi, cnt = ndf.ksg_field(e, [ref], k=4, counts=True, var_ref=vr, var_qry=vq)
        w, wnx, wny = direct.ksg_field(xh[vr][:, ref], xh[vq], 4, counts=True)
        c = cnt[0].cpu().numpy()
        assert np.array_equal(c[:, 0], wnx) and np.array_equal(c[:, 1], wny)
        assert np.max(np.abs(mi[0].cpu().numpy() - w)) <= MI_TOL
    # pairs across variables
    pairs = gen.random_pairs(cfg.n_vertices, 200, seed=21)
    r = ndf.pearson_pairs(e, pairs, var_a=0, var_b=1).cpu().numpy()
    want = np.array([direct.pearson(xh[0][:, a], xh[1][:, b]) for a, b in pairs])
    assert np.max(np.abs(r - want)) <= PEARSON_TOL
    mi = ndf.ksg_pairs(e, pairs, k=4, var_a=1, var_b=0).cpu().numpy()
    want = np.array([direct.ksg_field(xh[1][:, a], xh[0][:, b:b + 1], 4)[0] for a, b in pairs])
    assert np.max(np.abs(mi - want)) <= MI_TOL


def test_maximum_member_counts():
    """The largest ensembles the calls accept: KSG at N = 2048 (its limit; the stored
    orders come from the block sort, counts exact on sampled queries) and Pearson at
    N = 4096 (its limit); a KSG call beyond 2048 members is refused on the host."""
    cfg = gen.CONFIGS["tiny"].with_members(2048)
    e = _ens(cfg)
    V = cfg.n_vertices
    x = e.x[0].cpu().numpy()
    ref = cfg.ref_v
    sample = np.unique(np.concatenate([gen.random_vertices(V, 40, seed=91), [ref]]))
    mi, cnt = ndf.ksg_field(e, [ref], k=4, counts=True)
    s_t = torch.as_tensor(sample, device="cuda")
    mi = mi[0, s_t].cpu().numpy()
    cnt = cnt[0, s_t].cpu().numpy()
    want, wnx, wny = direct.ksg_field(x[:, ref], x[:, sample], 4, counts=True)
    assert np.array_equal(cnt[:, 0], wnx) and np.array_equal(cnt[:, 1], wny)
    err = np.max(np.abs(mi - want))
    _log(f"KSG N=2048 sampled: max|dI| {err:.2e}")
    assert err <= MI_TOL
    cfg4 = gen.CONFIGS["tiny"].with_members(4096)
    x4 = gen.make_ensemble(cfg4, device="cuda")
    e4 = ndf.Ensemble(x4, cfg4.nx, cfg4.ny, cfg4.nz, orders=False)
    ndf.ndf_prepare(e4)
    xh4 = x4[0].cpu().numpy()
    for prec in (ndf.NDF_PREC_FP32, ndf.NDF_PREC_SPLIT_BF16):
        got = ndf.pearson_field(e4, [ref, 0], prec=prec).cpu().numpy()
        for i, r in enumerate([ref, 0]):
            e_ = np.max(np.abs(got[i] - direct.pearson_field(xh4[:, r], xh4)))
            _log(f"Pearson N=4096 prec={prec} ref={r}: max|dr| {e_:.2e}")
            assert e_ <= PEARSON_TOL
    with pytest.raises(ndf.NdfError):
        ndf.ksg_field(e4, [ref], k=4)
