"""GPU parity at continuous positions (Sec. 4.3: training pairs are positions in
the domain [-1,1]^3, the ensemble is sampled there by trilinear interpolation),
through the C ABI:

* ndf_pearson_points against the FP64 oracle (|dr| <= 1e-5), within and across
  variables, with positions outside the domain and NaN coordinates (clamped),
  and the edge cases: a non-finite corner (NaN unless its weight is 0), a
  constant column (r = 0);
* ndf_net_forward_at / ndf_net_grad_at against the FP64 network at the same
  positions, held to the emulated bf16 rounding floor (tests/floors.py);
* ndf_train_step_at on targets from ndf_pearson_points learns the field.
"""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import gen
from oracle import ndf_net as nn
from oracle import points as pt
from paper_2307_02203_amd import ndf

pytestmark = pytest.mark.gpu

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from floors import TRAIN_OPS, check_floor, check_grad_floor  # noqa: E402

PEARSON_TOL = 1e-5


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _pos_pairs(n, seed, spread=1.0):
    return gen.random_positions(2 * n, seed=seed, spread=spread).reshape(n, 2, 3)


def _ens(cfg, x=None):
    if x is None:
        x = gen.make_ensemble(cfg, device="cuda")
    e = ndf.Ensemble(x, cfg.nx, cfg.ny, cfg.nz, transposed=True)
    ndf.ndf_prepare(e)
    return e


@pytest.mark.parametrize("name", ["tiny", "mid"])
def test_pearson_points_parity(name):
    cfg = dataclasses.replace(gen.CONFIGS[name], n_vars=2)
    e = _ens(cfg)
    x = e.x.cpu().numpy()
    dims = (cfg.nx, cfg.ny, cfg.nz)
    pos = np.concatenate([_pos_pairs(1500, seed=51), _pos_pairs(100, seed=52, spread=1.4)])
    pos[-3:, 1, 0] = np.nan
    assert torch.equal(e.xt[0].T.contiguous(), e.x[0])
    for va, vb in ((0, 0), (0, 1), (1, 0)):
        got = ndf.pearson_points(e, pos, var_a=va, var_b=vb).cpu().numpy()
        want = pt.pearson_points(x[va], x[vb], dims, pos)
        err = np.max(np.abs(got - want))
        _log(f"pearson points {name} vars ({va},{vb}): max|dr| {err:.2e}")
        assert err <= PEARSON_TOL
    # pairs of vertex positions give the vertex-pair targets
    pairs = gen.random_pairs(cfg.n_vertices, 300, seed=53)
    ijk = np.stack([pairs % cfg.nx, (pairs // cfg.nx) % cfg.ny, pairs // (cfg.nx * cfg.ny)], -1)
    vpos = (2.0 * ijk / (np.array(dims) - 1) - 1.0).astype(np.float32)
    got = ndf.pearson_points(e, vpos).cpu().numpy()
    want = pt.pearson_points(x[0], x[0], dims, vpos)
    assert np.max(np.abs(got - want)) <= PEARSON_TOL
    r_pairs = ndf.pearson_pairs(e, pairs).cpu().numpy()
    assert np.max(np.abs(got - r_pairs)) <= 2 * PEARSON_TOL


def test_pearson_points_edge_cases():
    """A NaN member at vertex 0 and a constant column at the last vertex: pairs
    touching vertex 0 with nonzero weight give NaN, with zero weight a finite r;
    the constant column gives r = 0, half a cell away a finite r; B = 0 is a
    no-op."""
    cfg = gen.CONFIGS["tiny"]
    x = gen.make_ensemble(cfg, device="cuda")
    V = cfg.n_vertices
    x[0, 3, 0] = float("nan")
    x[0, :, V - 1] = 2.5
    e = _ens(cfg, x)
    xh = x[0].cpu().numpy()
    dims = (cfg.nx, cfg.ny, cfg.nz)
    q = gen.random_positions(5, seed=54)
    corner0 = np.array([-1.0, -1.0, -1.0], dtype=np.float32)
    cornerz = np.array([-1.0, -1.0, 1.0], dtype=np.float32)   # vertex (0, 0, nz-1)
    last = np.array([1.0, 1.0, 1.0], dtype=np.float32)
    half = np.array([1.0, 1.0, 1.0 - 1.0 / (cfg.nz - 1)], dtype=np.float32)
    near0 = np.array([-0.99, -1.0, -1.0], dtype=np.float32)
    pos = np.stack([np.stack([corner0, q[0]]), np.stack([q[1], near0]),
                    np.stack([cornerz, q[2]]), np.stack([last, q[3]]),
                    np.stack([half, q[4]])]).astype(np.float32)
    got = ndf.pearson_points(e, pos).cpu().numpy()
    want = pt.pearson_points(xh, xh, dims, pos)
    _log(f"edge cases: got {got} want {want}")
    assert np.isnan(got[0]) and np.isnan(got[1])
    assert np.isnan(want[0]) and np.isnan(want[1])
    assert np.isfinite(got[2]) and abs(got[2] - want[2]) <= PEARSON_TOL
    assert got[3] == 0.0 and want[3] == 0.0
    assert np.isfinite(got[4]) and abs(got[4] - want[4]) <= PEARSON_TOL
    empty = torch.empty((0, 2, 3), dtype=torch.float32, device="cuda")
    out = torch.empty(0, device="cuda")
    ndf.ndf_pearson_points(e, 0, 0, empty, out)


def _setup(name, n_enc, seed):
    cfg = gen.CONFIGS[name]
    lay = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz, n_enc=n_enc)
    flat = gen.make_net_params(lay, seed=seed, grid_scale=0.5, bias_scale=0.1)
    c = ndf.net_config(cfg.nx, cfg.ny, cfg.nz, lay.res, n_enc=n_enc)
    P = torch.from_numpy(flat).cuda()
    net = nn.Net(flat, (cfg.nx, cfg.ny, cfg.nz), lay.res, 8, 128, n_enc)
    return cfg, lay, c, P, net


@pytest.mark.parametrize("name,n_enc", [("tiny", 1), ("mid", 2)])
def test_forward_at_parity(name, n_enc):
    cfg, lay, c, P, net = _setup(name, n_enc, seed=2340)
    pos = np.concatenate([_pos_pairs(2900, seed=55), _pos_pairs(100, seed=56, spread=1.3)])
    pos_t = torch.as_tensor(pos, device="cuda")
    y = torch.empty(len(pos), device="cuda")
    ws = torch.empty(ndf.train_ws_bytes(c, len(pos)), dtype=torch.uint8, device="cuda")
    ndf.ndf_net_forward_at(c, P, pos_t, y, ws)
    got = y.cpu().numpy().astype(np.float64)
    check_floor(got, nn.forward_points(net, pos), nn.forward_points(net, pos, TRAIN_OPS),
                f"forward_at {name} n_enc={n_enc}")


@pytest.mark.parametrize("name,n_enc", [("tiny", 1), ("mid", 2)])
def test_gradient_at_parity(name, n_enc):
    """The adjoint at continuous positions, one residual sign for every pair, held
    to the emulated bf16 floor per tensor like the vertex-pair adjoint."""
    cfg, lay, c, P, net = _setup(name, n_enc, seed=2341)
    pos = _pos_pairs(2048, seed=57)
    y = nn.forward_points(net, pos)
    t = y + 1.0
    loss_o, g_o, _ = nn.loss_and_grad_points(net, pos, t)
    _, g_e, _ = nn.loss_and_grad_points(net, pos, t, TRAIN_OPS)
    pos_t = torch.as_tensor(pos, device="cuda")
    t_t = torch.as_tensor(t.astype(np.float32), device="cuda")
    g = torch.empty_like(P)
    loss = torch.empty(1, device="cuda")
    ws = torch.empty(ndf.train_ws_bytes(c, len(pos)), dtype=torch.uint8, device="cuda")
    ndf.ndf_net_grad_at(c, P, pos_t, t_t, g, loss, ws)
    g = g.cpu().numpy().astype(np.float64)
    assert abs(loss.item() - loss_o) <= 1e-2 * loss_o
    check_grad_floor(lay, g, g_o.flat, g_e.flat, f"grad_at {name} n_enc={n_enc}")


def test_training_at_positions_learns():
    """Training on continuous position pairs with targets from ndf_pearson_points
    (Sec. 4.3): the network beats its initialisation and the best constant on
    held-out position pairs, errors against the FP64 oracle's targets."""
    cfg = gen.CONFIGS["tiny"]
    e = _ens(cfg)
    x = e.x[0].cpu().numpy()
    dims = (cfg.nx, cfg.ny, cfg.nz)
    lay = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz)
    c = ndf.net_config(cfg.nx, cfg.ny, cfg.nz, lay.res)
    P = torch.empty(lay.n_floats, device="cuda")
    opt = torch.empty(2 * lay.n_floats, device="cuda")
    ndf.ndf_net_init(c, P, opt, 8)
    B = 4096
    ws = torch.empty(ndf.train_ws_bytes(c, B) + P.numel() * 4 + 256, dtype=torch.uint8,
                     device="cuda")
    loss = torch.empty(1, device="cuda")
    held = _pos_pairs(3000, seed=2400)
    truth = pt.pearson_points(x, x, dims, held)
    held_t = torch.as_tensor(held, device="cuda")
    yws = torch.empty(ndf.train_ws_bytes(c, len(held)), dtype=torch.uint8, device="cuda")

    def mae():
        y = torch.empty(len(held), device="cuda")
        ndf.ndf_net_forward_at(c, P, held_t, y, yws)
        return float(np.mean(np.abs(y.cpu().numpy() - truth)))

    mae0 = mae()
    for step in range(1, 401):
        pos = torch.as_tensor(_pos_pairs(B, seed=6000 + step), device="cuda")
        t = ndf.pearson_points(e, pos)
        ndf.ndf_train_step_at(c, P, opt, step, pos, t, 3e-3, loss, ws)
    mae1 = mae()
    const = float(np.mean(np.abs(truth - np.median(truth))))
    _log(f"training at positions: MAE init {mae0:.4f} trained {mae1:.4f} best-constant {const:.4f}")
    assert mae1 < 0.5 * mae0 and mae1 < 0.6 * const


@pytest.mark.parametrize("name", ["tiny", "mid"])
def test_ksg_points_parity(name):
    """KSG targets at continuous positions: the interpolated columns' codes and
    neighbour counts bit-exact against the FP64 oracle, |dI| <= 1e-4, within and
    across variables, including positions outside the domain and NaN
    coordinates; at vertex positions the estimate is the vertex pair's."""
    cfg = dataclasses.replace(gen.CONFIGS[name], n_vars=2)
    e = _ens(cfg)
    x = e.x.cpu().numpy()
    dims = (cfg.nx, cfg.ny, cfg.nz)
    pos = np.concatenate([_pos_pairs(150, seed=61), _pos_pairs(20, seed=62, spread=1.3)])
    pos[-2:, 0, 1] = np.nan
    for va, vb in ((0, 0), (1, 0)):
        mi, cnt = ndf.ksg_points(e, pos, k=4, counts=True, var_a=va, var_b=vb)
        mi, cnt = mi.cpu().numpy(), cnt.cpu().numpy()
        want, wcnt = pt.ksg_points(x[va], x[vb], dims, pos, 4, counts=True)
        err = np.max(np.abs(mi - want))
        _log(f"ksg points {name} vars ({va},{vb}): max|dI| {err:.2e}, "
             f"counts equal {np.array_equal(cnt, wcnt)}")
        assert np.array_equal(cnt, wcnt)
        assert err <= 1e-4
    # the domain's corners are exactly the grid's corner vertices (in FP32 too)
    signs = np.array([[sx, sy, sz] for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)],
                     dtype=np.float32)
    vert = np.array([(0 if sx < 0 else cfg.nx - 1) + cfg.nx * ((0 if sy < 0 else cfg.ny - 1)
                     + cfg.ny * (0 if sz < 0 else cfg.nz - 1)) for sx, sy, sz in signs])
    ia, ib = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
    cpos = np.stack([signs[ia.ravel()], signs[ib.ravel()]], axis=1)
    pairs = np.stack([vert[ia.ravel()], vert[ib.ravel()]], axis=1)
    got = ndf.ksg_points(e, cpos, k=4).cpu().numpy()
    want = ndf.ksg_pairs(e, pairs, k=4).cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-6


def test_points_ragged_members():
    """N = 37 members (not a multiple of 4: the scalar-load paths) and a 3-member
    edge case: Pearson and KSG at positions against the oracle."""
    for n_members, k in ((37, 4), (3, 1)):
        cfg = dataclasses.replace(gen.CONFIGS["tiny"], n_members=n_members)
        e = _ens(cfg)
        x = e.x[0].cpu().numpy()
        dims = (cfg.nx, cfg.ny, cfg.nz)
        pos = _pos_pairs(203, seed=81)
        r = ndf.pearson_points(e, pos).cpu().numpy()
        assert np.max(np.abs(r - pt.pearson_points(x, x, dims, pos))) <= PEARSON_TOL
        mi, cnt = ndf.ksg_points(e, pos, k=k, counts=True)
        want, wcnt = pt.ksg_points(x, x, dims, pos, k, counts=True)
        assert np.array_equal(cnt.cpu().numpy(), wcnt)
        assert np.max(np.abs(mi.cpu().numpy() - want)) <= 1e-4
        _log(f"ragged N={n_members}: pearson and KSG at positions match")
