"""Benchmark: ms per 1.76M-vertex dependence field, learned field (NDF) vs direct
Pearson / KSG-MI, on one MI355X.

Workload: synthetic paper-shaped ensemble (1000 members on 250x352x20 =
1,760,000 vertices, FP32, Gaussian-blob generator of gen/), reference vertex
(125,176,10).  One timed step is one pass of the whole hot path:

  prepare        per-vertex FP64 moments + KSG integer codes (1 variable)
  pearson_fp32   direct Pearson field, 1 reference, FP32 stream
  pearson_b64    direct Pearson fields, 64 references, split-BF16 MFMA
  ksg_field      direct KSG-MI field, 1 reference, k = 4
  targets        direct Pearson and KSG-MI targets for 2^18 random vertex pairs
  train_step     one learned-field training step on 2^18 pairs (BF16 MFMA, Adam)
  ndf_field      learned field for 1 reference at all vertices (fused BF16 kernel)
  ndf_field_fp8  the same field with MXFP8 (E4M3) layers 2..5
  ndf_field_cached  the same field from cached query latents (merge + decoder
                 only; the cache is built once per trained network, untimed)

After the timed steps the calls beyond that path are timed on their own
(`next_rows`, not part of a step): the same field at 1.76M sample positions along
rays, the difference of two fields from the latent cache, the field of a network
whose finest level is a 2^19-cell hash table, Pearson and KSG-MI targets for 2^18
pairs of continuous positions (trilinear interpolation of the ensemble) and a
training step on them.

`value` is the learned-field ms per field (the paper's headline quantity);
`fields` gives every row.  All launches go on torch's current stream and are
timed with HIP events on it.  Inputs are resident in HBM before timing starts.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

B_PAIRS = 1 << 18
N_BATCH = 64
K_NN = 4
LR = 1e-3
PREP_TRAIN_STEPS = 300
HASH_T = 19          # hash-table size 2^T of the hashed-grid row

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP8_TFLOPS = 5000.0
PEAK_ALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # 32-bit VALU lane operations (non-packed)


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--train-steps", type=int, default=PREP_TRAIN_STEPS,
                    help="learned-field training steps before timing")
    ap.add_argument("--mi-train-steps", type=int, default=PREP_TRAIN_STEPS,
                    help="training steps of the second learned field (KSG-MI targets)")
    ap.add_argument("--only", default=None,
                    help="profile one row (prepare, pearson_fp32, pearson_b64, ksg_field, "
                         "targets, train_step, ndf_field, ndf_field_fp8, ndf_field_cached, "
                         "or one of the next rows: ndf_points_rays, ndf_field_difference, "
                         "pearson_points, ksg_points, train_step_at, ndf_field_hash) W+K "
                         "times and exit")
    ap.add_argument("--no-next-rows", action="store_true",
                    help="skip timing the calls beyond the hot path")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 1 GiB device copy (counter calibration) and exit")
    return ap.parse_args()


def _copy_probe(a):
    import torch
    n = 1 << 28                      # 2^28 floats = 1 GiB
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.warmup + a.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                      "launches": a.warmup + a.steps}))


def main():
    a = _parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                          "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)
    if a.copy_probe:
        _copy_probe(a)
        return
    import torch
    import gen
    from paper_2307_02203_amd import ndf

    dev = "cuda"
    cfg = gen.CONFIGS["paper"]
    V, N = cfg.n_vertices, cfg.n_members
    ref = cfg.ref_v
    log = lambda *m: print(*m, file=sys.stderr, flush=True)  # noqa: E731

    log("bench: generating ensemble")
    x = gen.make_ensemble(cfg, device=dev)
    ens = ndf.Ensemble(x, cfg.nx, cfg.ny, cfg.nz)
    ndf.ndf_prepare(ens)

    refs64 = np.concatenate([[ref], gen.random_vertices(V, N_BATCH - 1, seed=2311)])
    lay = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz)
    net = ndf.net_config(cfg.nx, cfg.ny, cfg.nz, lay.res)
    P = torch.empty(lay.n_floats, device=dev)
    opt = torch.empty(2 * lay.n_floats, device=dev)
    ndf.ndf_net_init(net, P, opt, 2320)

    # buffers (allocated once, outside the timed region)
    out_p = torch.empty((1, V), device=dev)
    out_b = torch.empty((N_BATCH, V), device=dev)
    out_k = torch.empty((1, V), device=dev)
    out_n = torch.empty((1, V), device=dev)
    out_n8 = torch.empty((1, V), device=dev)
    ws_p = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_PEARSON_FIELD, ens, None, 1, 0),
                       dtype=torch.uint8, device=dev)
    ws_b = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_PEARSON_FIELD, ens, None, N_BATCH,
                                               ndf.NDF_PREC_SPLIT_BF16),
                       dtype=torch.uint8, device=dev)
    ws_k = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_KSG_FIELD, ens, None, 1, 0),
                       dtype=torch.uint8, device=dev)
    ws_kp = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_KSG_PAIRS, ens, None, 1, 0),
                        dtype=torch.uint8, device=dev)
    ws_t = torch.empty(ndf.train_ws_bytes(net, B_PAIRS) + lay.n_floats * 4 + 256,
                       dtype=torch.uint8, device=dev)
    qp = torch.empty(ndf.ndf_net_qparam_bytes(net, ndf.NDF_PREC_BF16), dtype=torch.uint8,
                     device=dev)
    ws_i = torch.empty(ndf.infer_ws_bytes(net, 1, ndf.NDF_PREC_BF16), dtype=torch.uint8,
                       device=dev)
    t_pear = torch.empty(B_PAIRS, device=dev)
    t_ksg = torch.empty(B_PAIRS, device=dev)
    loss = torch.empty(1, device=dev)
    pair_sets = [torch.as_tensor(gen.random_pairs(V, B_PAIRS, seed=2312 + s), device=dev)
                 for s in range(4)]

    # short training of the Pearson field so the timed inference runs a trained net
    n_train = 0 if a.only else a.train_steps
    log(f"bench: training the learned field ({n_train} steps of {B_PAIRS} pairs)")
    t0 = time.time()
    for s in range(1, n_train + 1):
        pr = torch.as_tensor(gen.random_pairs(V, B_PAIRS, seed=5000 + s), device=dev)
        ndf.ndf_pearson_pairs(ens, 0, 0, pr, t_pear)
        ndf.ndf_train_step(net, P, opt, s, pr, t_pear, LR, loss, ws_t)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    final_loss = loss.item()
    ndf.ndf_net_quantize(net, P, ndf.NDF_PREC_BF16, qp)
    step_no = [n_train]
    # query-latent cache of the trained network (for the cached-field row)
    cache = torch.empty(ndf.ndf_infer_latent_bytes(net), dtype=torch.uint8, device=dev)
    ev_c0, ev_c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev_c0.record()
    ndf.ndf_infer_latents(net, qp, cache)
    ev_c1.record()
    torch.cuda.synchronize()
    cache_ms = ev_c0.elapsed_time(ev_c1)
    out_nc = torch.empty((1, V), device=dev)

    # one network per measure: a second field trained on KSG-MI targets (same
    # architecture, so its inference cost is the timed ndf_field row)
    n_mi = 0 if (a.only or a.no_accuracy) else a.mi_train_steps
    out_mi = None
    mi_train = None
    if n_mi > 0:
        log(f"bench: training the KSG-MI learned field ({n_mi} steps)")
        P_mi = torch.empty(lay.n_floats, device=dev)
        opt_mi = torch.empty(2 * lay.n_floats, device=dev)
        ndf.ndf_net_init(net, P_mi, opt_mi, 2321)
        t0 = time.time()
        for s in range(1, n_mi + 1):
            pr = torch.as_tensor(gen.random_pairs(V, B_PAIRS, seed=6000 + s), device=dev)
            ndf.ndf_ksg_mi_pairs(ens, 0, 0, pr, K_NN, t_ksg, None, ws_kp)
            ndf.ndf_train_step(net, P_mi, opt_mi, s, pr, t_ksg, LR, loss, ws_t)
        torch.cuda.synchronize()
        mi_train = {"steps": n_mi, "seconds": time.time() - t0, "final_l1_loss": loss.item()}
        qp_mi = torch.empty_like(qp)
        ndf.ndf_net_quantize(net, P_mi, ndf.NDF_PREC_BF16, qp_mi)
        out_mi = torch.empty((1, V), device=dev)
        ndf.ndf_infer_field(net, qp_mi, ndf.NDF_PREC_BF16, [ref], out_mi, ws_i)
        del P_mi, opt_mi

    stream = torch.cuda.current_stream()
    rows = ["prepare", "pearson_fp32", "pearson_b64", "ksg_field", "targets", "train_step",
            "ndf_field", "ndf_field_fp8", "ndf_field_cached"]

    def row_prepare(it):
        ndf.ndf_prepare(ens)

    def row_pearson_fp32(it):
        ndf.ndf_pearson_field(ens, 0, 0, [ref], out_p, ndf.NDF_PREC_FP32, ws_p)

    def row_pearson_b64(it):
        ndf.ndf_pearson_field(ens, 0, 0, refs64, out_b, ndf.NDF_PREC_SPLIT_BF16, ws_b)

    def row_ksg_field(it):
        ndf.ndf_ksg_mi_field(ens, 0, 0, [ref], K_NN, out_k, None, ws_k)

    def row_targets(it):
        pr = pair_sets[it % 4]
        ndf.ndf_pearson_pairs(ens, 0, 0, pr, t_pear)
        ndf.ndf_ksg_mi_pairs(ens, 0, 0, pr, K_NN, t_ksg, None, ws_kp)

    def row_train_step(it):
        step_no[0] += 1
        ndf.ndf_train_step(net, P, opt, step_no[0], pair_sets[it % 4], t_pear, LR, loss, ws_t)

    def row_ndf_field(it):
        ndf.ndf_infer_field(net, qp, ndf.NDF_PREC_BF16, [ref], out_n, ws_i)

    def row_ndf_field_fp8(it):
        ndf.ndf_infer_field(net, qp, ndf.NDF_PREC_FP8_E4M3, [ref], out_n8, ws_i)

    def row_ndf_field_cached(it):
        ndf.ndf_infer_field_cached(net, qp, [ref], cache, out_nc, ws_i)

    row_fn = {"ndf_field_fp8": row_ndf_field_fp8, "ndf_field_cached": row_ndf_field_cached,
              "prepare": row_prepare,
              "pearson_fp32": row_pearson_fp32,
              "pearson_b64": row_pearson_b64, "ksg_field": row_ksg_field,
              "targets": row_targets, "train_step": row_train_step, "ndf_field": row_ndf_field}

    def next_rows():
        """The calls beyond the hot path, with their own buffers."""
        ens_t = ndf.Ensemble(x, cfg.nx, cfg.ny, cfg.nz, orders=False, transposed=True)
        ndf.ndf_prepare(ens_t)
        n_rays, n_steps = V // 256, 256
        ray_pos = torch.as_tensor(gen.ray_positions(n_rays, n_steps, seed=2350), device=dev)
        out_rp = torch.empty((1, ray_pos.shape[0]), device=dev)
        out_d = torch.empty(V, device=dev)
        ws_i2 = torch.empty(ndf.infer_ws_bytes(net, 2, ndf.NDF_PREC_BF16), dtype=torch.uint8,
                            device=dev)
        ref2 = int(gen.random_vertices(V, 1, seed=2351)[0])
        pos_sets = [torch.as_tensor(gen.random_positions(2 * B_PAIRS, seed=2360 + s)
                                    .reshape(B_PAIRS, 2, 3), device=dev) for s in range(4)]
        t_pp = torch.empty(B_PAIRS, device=dev)
        t_kp = torch.empty(B_PAIRS, device=dev)
        ws_kq = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_KSG_POINTS, ens_t, None, B_PAIRS,
                                                    0), dtype=torch.uint8, device=dev)
        P_at, opt_at = P.clone(), opt.clone()
        step_at = [step_no[0]]
        # the same network shape with the finest level as a 2^19-cell hash table
        lay_h = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz, log2_hashmap=HASH_T)
        net_h = ndf.net_config(cfg.nx, cfg.ny, cfg.nz, lay_h.res, log2_hashmap=HASH_T)
        P_h = torch.empty(lay_h.n_floats, device=dev)
        ndf.ndf_net_init(net_h, P_h, None, 2352)
        qp_h = torch.empty(ndf.ndf_net_qparam_bytes(net_h, ndf.NDF_PREC_BF16), dtype=torch.uint8,
                           device=dev)
        ndf.ndf_net_quantize(net_h, P_h, ndf.NDF_PREC_BF16, qp_h)
        out_h = torch.empty((1, V), device=dev)

        def rays(it):
            ndf.ndf_infer_points(net, qp, ndf.NDF_PREC_BF16, [ref], ray_pos, out_rp, ws_i)

        def diff(it):
            ndf.ndf_infer_field_difference(net, qp, ref, ref2, cache, out_d, ws_i2)

        def ppoints(it):
            ndf.ndf_pearson_points(ens_t, 0, 0, pos_sets[it % 4], t_pp)

        def hashed(it):
            ndf.ndf_infer_field(net_h, qp_h, ndf.NDF_PREC_BF16, [ref], out_h, ws_i)

        def kpoints(it):
            ndf.ndf_ksg_mi_points(ens_t, 0, 0, pos_sets[it % 4], K_NN, t_kp, None, ws_kq)

        def train_at(it):
            step_at[0] += 1
            ndf.ndf_train_step_at(net, P_at, opt_at, step_at[0], pos_sets[it % 4], t_pp, LR,
                                  loss, ws_t)

        ppoints(0)
        return {"ndf_points_rays": rays, "ndf_field_difference": diff,
                "pearson_points": ppoints, "ksg_points": kpoints, "ndf_field_hash": hashed,
                "train_step_at": train_at}, ray_pos.shape[0]

    def time_rows(fns, warmup, steps):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        out = {}
        for name, fn in fns.items():
            ms = []
            for it in range(warmup + steps):
                ev0.record(stream)
                fn(it)
                ev1.record(stream)
                torch.cuda.synchronize()
                if it >= warmup:
                    ms.append(ev0.elapsed_time(ev1))
            out[name] = ms
        return out

    if a.only and a.only not in row_fn:
        fns, _ = next_rows()
        ms = time_rows({a.only: fns[a.only]}, a.warmup, a.steps)[a.only]
        print(json.dumps({"row": a.only, "ms": ms, "median_ms": float(np.median(ms))}))
        return

    if a.only:
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ms = []
        for it in range(a.warmup + a.steps):
            ev0.record(stream)
            row_fn[a.only](it)
            ev1.record(stream)
            torch.cuda.synchronize()
            if it >= a.warmup:
                ms.append(ev0.elapsed_time(ev1))
        print(json.dumps({"row": a.only, "ms": ms, "median_ms": float(np.median(ms))}))
        return

    def run_step(it, ev):
        for i, r in enumerate(rows):
            ev[i].record(stream)
            row_fn[r](it)
        ev[len(rows)].record(stream)

    log(f"bench: {a.warmup} warmup + {a.steps} timed steps")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(rows) + 1)]
           for _ in range(a.warmup + a.steps)]
    for it in range(a.warmup):
        run_step(it, evs[it])
    torch.cuda.synchronize()
    t_start = time.time()
    for it in range(a.warmup, a.warmup + a.steps):
        run_step(it, evs[it])
    torch.cuda.synchronize()
    wall = time.time() - t_start
    per_row = {r: [] for r in rows}
    step_ms = []
    for it in range(a.warmup, a.warmup + a.steps):
        e = evs[it]
        for i, r in enumerate(rows):
            per_row[r].append(e[i].elapsed_time(e[i + 1]))
        step_ms.append(e[0].elapsed_time(e[len(rows)]))
    med = {r: float(np.median(v)) for r, v in per_row.items()}
    ms_step = float(np.median(step_ms))
    fields = {
        "ndf_field_bf16": med["ndf_field"],
        "ndf_field_fp8": med["ndf_field_fp8"],
        "ndf_field_bf16_cached_query_latents": med["ndf_field_cached"],
        "ndf_query_latent_cache_build_once": cache_ms,
        "pearson_field_fp32": med["pearson_fp32"],
        "pearson_batch64_split_bf16_per_field": med["pearson_b64"] / N_BATCH,
        "pearson_batch64_split_bf16_total": med["pearson_b64"],
        "ksg_mi_field_k4": med["ksg_field"],
        "prepare": med["prepare"],
        "targets_pearson_and_ksg_2^18_pairs": med["targets"],
        "train_step_2^18_pairs": med["train_step"],
    }

    # rooflines of the timed kernels (algorithmic bytes / flops per launch)
    roof = {
        "pearson_fp32": {"bound": "hbm", "achieved": 4.0 * N * V / (med["pearson_fp32"] * 1e-3)
                         / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"},
        "pearson_b64": {"bound": "hbm", "achieved": 4.0 * N * V / (med["pearson_b64"] * 1e-3)
                        / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"},
        "ndf_field": {"bound": "mfma", "achieved": 2.0 * 69760 * V / (med["ndf_field"] * 1e-3)
                      / 1e12, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s"},
        "ndf_field_fp8": {"bound": "mfma", "achieved": 2.0 * 69760 * V
                          / (med["ndf_field_fp8"] * 1e-3) / 1e12, "peak": PEAK_FP8_TFLOPS,
                          "unit": "TFLOP/s"},
        # merge + decoder: 32,896 MAC per vertex, plus 256 B of cached latent read
        "ndf_field_cached": {"bound": "mfma", "achieved": 2.0 * 32896 * V
                             / (med["ndf_field_cached"] * 1e-3) / 1e12,
                             "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                             "hbm_gbs": 256.0 * V / (med["ndf_field_cached"] * 1e-3) / 1e9},
    }
    for r in roof.values():
        r["frac"] = r["achieved"] / r["peak"]
    timed = {k: med[k] for k in rows}
    dominant = max(timed, key=timed.get)

    result = {
        "metric": "ms per 1.76M-vertex dependence field: NDF vs direct Pearson/KSG-MI",
        "value": med["ndf_field"],
        "unit": "ms",
        "higher_is_better": False,
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "wall_s_timed": wall,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": "paper-shaped ensemble, 1000 members x 250x352x20 (1.76M vertices) "
                        "FP32, 1 reference (125,176,10); learned field 4-level dense grid "
                        "(62x88x5..250x352x20, 8 feat) + 5x128 MLP in BF16 vs direct Pearson "
                        "(FP32) and KSG-MI (k=4)",
            "n_members": N, "grid": [cfg.nx, cfg.ny, cfg.nz], "n_vertices": V,
            "batch_refs": N_BATCH, "train_pairs": B_PAIRS, "k": K_NN,
        },
        "fields": fields,
        "speedup_ndf_vs_pearson_fp32": med["pearson_fp32"] / med["ndf_field"],
        "speedup_ndf_vs_ksg": med["ksg_field"] / med["ndf_field"],
        "speedup_ndf_vs_pearson_batch64_per_field": med["pearson_b64"] / N_BATCH / med["ndf_field"],
        "dominant_kernel": dominant,
        "rooflines": roof,
        "training": {"steps_before_timing": n_train, "seconds": train_s,
                     "final_l1_loss": final_loss, "lr": LR, "batch": B_PAIRS,
                     "ksg_mi_field": mi_train},
    }
    result["roofline"] = _roofline_of(dominant, roof, med, N, V)

    if not a.no_next_rows:
        log("bench: next rows (continuous positions, difference fields)")
        fns, n_ray = next_rows()
        nm = {k: float(np.median(v)) for k, v in time_rows(fns, 1, a.steps).items()}
        nroof = {
            "ndf_points_rays": {"bound": "mfma", "achieved": 2.0 * 69760 * n_ray
                                / (nm["ndf_points_rays"] * 1e-3) / 1e12,
                                "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s"},
            "ndf_field_difference": {"bound": "mfma", "achieved": 2.0 * 2 * 32896 * V
                                     / (nm["ndf_field_difference"] * 1e-3) / 1e12,
                                     "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s"},
            # 2 x 8 corner rows of N FP32 members per pair
            "pearson_points": {"bound": "hbm", "achieved": 16.0 * 4 * N * B_PAIRS
                               / (nm["pearson_points"] * 1e-3) / 1e9,
                               "peak": PEAK_HBM_GBS, "unit": "GB/s"},
        }
        for r in nroof.values():
            r["frac"] = r["achieved"] / r["peak"]
        result["next_rows"] = {
            "ms": {"ndf_points_rays_1.76M_samples": nm["ndf_points_rays"],
                   "ndf_field_difference_from_cache": nm["ndf_field_difference"],
                   "pearson_points_targets_2^18_pairs": nm["pearson_points"],
                   "ksg_points_targets_2^18_pairs": nm["ksg_points"],
                   "ndf_field_bf16_hash_table_2^19": nm["ndf_field_hash"],
                   "train_step_at_positions_2^18_pairs": nm["train_step_at"]},
            "rooflines": nroof,
            "workload": f"{n_ray} samples on {n_ray // 256} rays x 256 steps; two references "
                        "for the difference; 2^18 uniform position pairs in [-1,1]^3",
        }

    if not a.no_accuracy:
        acc, sample, r_o, mi_o = _accuracy(ens, out_p, out_b, out_k, out_n, out_n8, out_mi,
                                           refs64, cfg, out_nc)
        result["accuracy"] = acc
        log("bench: gain of the trained field over the method without it")
        result["gain"] = _gain(ens, cfg, net, lay, sample, r_o, mi_o, out_n, out_mi, med, log)
    if not a.no_cpu_baseline:
        result["cpu_baseline"] = _cpu_baseline(ens, cfg, lay, log)
    print(json.dumps(result))


# Brute-force KSG needs, per ordered sample pair, |dx| and |dy| (one v_sad_u32
# each), a max and a compare against the running k-th distance (4 lane ops) for
# the neighbour pass, and two compares and two conditional adds for the marginal
# counts: 8 32-bit VALU lane operations per pair.
KSG_OPS_PER_PAIR = 8


def _roofline_of(dominant, roof, med, N, V):
    if dominant in roof:
        r = dict(roof[dominant])
    elif dominant == "ksg_field":
        # algorithmic unit: brute-force-equivalent pair evaluations V N (N - 1)
        pairs = float(V) * N * (N - 1)
        r = {"bound": "alu", "achieved": pairs / (med[dominant] * 1e-3) / 1e12,
             "peak": PEAK_ALU_TOPS / KSG_OPS_PER_PAIR, "unit": "Tpair-evals/s"}
        r["frac"] = r["achieved"] / r["peak"]
        r["note"] = ("peak = brute-force pair evaluations/s at the 32-bit VALU peak "
                     f"({PEAK_ALU_TOPS:.1f} T lane-ops/s / {KSG_OPS_PER_PAIR} ops); the kernel "
                     "prunes the neighbour search, so frac > 1 is the pruning gain; its own "
                     "VALU issue rate and lane occupancy (rocprofv3 SQ counters, profiles/) "
                     "are valu_issue_frac and valu_lanes_active_frac")
    else:
        r = {"bound": "mixed", "achieved": None, "peak": None, "unit": None, "frac": None}
    r["kernel"] = dominant
    r["traffic"] = _measured_traffic(dominant)
    issue = _measured_issue(dominant)
    if issue is not None:
        # the kernel's own VALU issue and lane occupancy (rocprofv3 SQ counters)
        r["valu_issue_frac"], r["valu_lanes_active_frac"] = issue
    return r


# HBM bytes per launch measured with rocprofv3 PMC counters (FETCH_SIZE, WRITE_SIZE,
# scaled by a 1 GiB copy), recorded under profiles/ together with a hash of the
# kernel source; reported only while the source still matches.
_PMC_TRAFFIC = {
    "ksg_field": ("profiles/pmc_ksg_field_paper_1760000v_1000m.txt",
                  "paper_2307_02203_amd/csrc/ksg.hip"),
}


def _profile_text(row):
    """The counter profile of `row` while its kernel source still matches the hash
    recorded there (at measurement, or after a comment-only edit), else None."""
    import hashlib
    import re
    if row not in _PMC_TRAFFIC:
        return None
    prof, src = (os.path.join(ROOT, f) for f in _PMC_TRAFFIC[row])
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    shas = re.findall(r"sha256 prefix (?:at measurement|after a comment-only edit): "
                      r"([0-9a-f]+)", text)
    if not shas or not any(sha.startswith(h) for h in shas):
        return None
    return text


def _measured_traffic(row):
    import re
    text = _profile_text(row)
    m_val = re.search(r"traffic_bytes_per_launch: ([0-9.eE+]+)", text) if text else None
    return float(m_val.group(1)) if m_val else None


def _measured_issue(row):
    import re
    text = _profile_text(row)
    if not text:
        return None
    m_i = re.search(r"VALU issue: .*= (\d+)% of the kernel's cycles", text)
    m_l = re.search(r"VALU lanes active: .*= (\d+)%", text)
    if not (m_i and m_l):
        return None
    return int(m_i.group(1)) / 100.0, int(m_l.group(1)) / 100.0


N_MI_SAMPLE = 400   # vertices of the oracle KSG-MI comparison (brute force on the host)


def _accuracy(ens, out_p, out_b, out_k, out_n, out_n8, out_mi, refs64, cfg, out_nc):
    """Errors of the timed outputs against the FP64 oracle on sampled vertices."""
    import torch
    import gen
    from oracle import direct
    V = cfg.n_vertices
    sample = gen.random_vertices(V, 2000, seed=4242)
    idx = torch.as_tensor(sample, device="cuda")
    xs = ens.x[0][:, idx].cpu().numpy()
    xr = ens.x[0][:, cfg.ref_v].cpu().numpy()
    r_o = direct.pearson_field(xr, xs)
    mi_o = direct.ksg_field(xr, xs[:, :N_MI_SAMPLE], K_NN)
    p = out_p[0, idx].cpu().numpy()
    b0 = out_b[0, idx].cpu().numpy()
    k = out_k[0, idx[:N_MI_SAMPLE]].cpu().numpy()
    n = out_n[0, idx].cpu().numpy()
    n8 = out_n8[0, idx].cpu().numpy()
    extra = {}
    if out_mi is not None:
        m = out_mi[0, idx[:N_MI_SAMPLE]].cpu().numpy()
        extra = {"ndf_mi_vs_oracle_mae_400": float(np.mean(np.abs(m - mi_o))),
                 "ndf_mi_vs_oracle_max_abs_err_400": float(np.max(np.abs(m - mi_o)))}
    return {
        **extra,
        "sample_vertices": int(len(sample)),
        "pearson_fp32_max_abs_err": float(np.max(np.abs(p - r_o))),
        "pearson_split_bf16_max_abs_err": float(np.max(np.abs(b0 - r_o))),
        "ksg_mi_max_abs_err_400": float(np.max(np.abs(k - mi_o))),
        "ndf_vs_oracle_pearson_mae": float(np.mean(np.abs(n - r_o))),
        "ndf_vs_oracle_pearson_max_abs_err": float(np.max(np.abs(n - r_o))),
        "ndf_fp8_vs_oracle_pearson_mae": float(np.mean(np.abs(n8 - r_o))),
        "ndf_fp8_vs_ndf_bf16_max_abs_diff": float(np.max(np.abs(n8 - n))),
        "ndf_cached_equals_fused_bitwise": bool(torch.equal(out_nc, out_n)),
        "population_rho_mae_of_oracle": float(np.mean(np.abs(
            r_o - gen.population_rho(cfg, np.full(len(sample), cfg.ref_v), sample)))),
    }, sample, r_o, mi_o


def _gain(ens, cfg, net, lay, sample, r_o, mi_o, out_n, out_mi, med, log):
    """What the trained field gains over the method without it, on the sampled
    vertices against the FP64 oracle: the untrained (initialised) field, the best
    constant predictor, and the direct Pearson estimator with its members cut
    until one field costs what the learned field costs (equal time)."""
    import torch
    from paper_2307_02203_amd import ndf
    V, N = cfg.n_vertices, cfg.n_members
    idx = torch.as_tensor(sample, device="cuda")
    mae = lambda y: float(np.mean(np.abs(y - r_o)))  # noqa: E731
    out = {"ndf_trained_mae": mae(out_n[0, idx].cpu().numpy()),
           "best_constant_mae": mae(np.full_like(r_o, np.median(r_o)))}

    P0 = torch.empty(lay.n_floats, device="cuda")
    opt0 = torch.empty(2 * lay.n_floats, device="cuda")
    ndf.ndf_net_init(net, P0, opt0, 2320)
    qp0 = torch.empty(ndf.ndf_net_qparam_bytes(net, ndf.NDF_PREC_BF16), dtype=torch.uint8,
                      device="cuda")
    ndf.ndf_net_quantize(net, P0, ndf.NDF_PREC_BF16, qp0)
    ws_i = torch.empty(ndf.infer_ws_bytes(net, 1, ndf.NDF_PREC_BF16), dtype=torch.uint8,
                       device="cuda")
    y0 = torch.empty((1, V), device="cuda")
    ndf.ndf_infer_field(net, qp0, ndf.NDF_PREC_BF16, [cfg.ref_v], y0, ws_i)
    out["ndf_untrained_mae"] = mae(y0[0, idx].cpu().numpy())
    y0_mi = y0[0, idx[:N_MI_SAMPLE]].cpu().numpy()
    del P0, opt0, qp0, ws_i, y0

    # members of the equal-time direct estimator: its cost is linear in N
    m_eq = int(max(8, min(N, round(N * med["ndf_field"] / med["pearson_fp32"]))))
    sub = ndf.Ensemble(ens.x[:, :m_eq], cfg.nx, cfg.ny, cfg.nz)
    ndf.ndf_prepare(sub)
    ws = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_PEARSON_FIELD, sub, None, 1, 0),
                     dtype=torch.uint8, device="cuda")
    y = torch.empty((1, V), device="cuda")
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ms = []
    for it in range(7):
        ev0.record(stream)
        ndf.ndf_pearson_field(sub, 0, 0, [cfg.ref_v], y, ndf.NDF_PREC_FP32, ws)
        ev1.record(stream)
        torch.cuda.synchronize()
        if it >= 2:
            ms.append(ev0.elapsed_time(ev1))
    out["equal_time_direct_pearson"] = {
        "members": m_eq, "ms_per_field": float(np.median(ms)),
        "mae": mae(y[0, idx].cpu().numpy())}
    del sub, ws, y

    if out_mi is not None:
        # KSG-MI: its direct cost does not fall to the learned field's even at a
        # handful of members; report the smallest sensible member count instead
        mae_mi = lambda z: float(np.mean(np.abs(z - mi_o)))  # noqa: E731
        m_few = 16
        sub = ndf.Ensemble(ens.x[:, :m_few], cfg.nx, cfg.ny, cfg.nz)
        ndf.ndf_prepare(sub)
        ws = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_KSG_FIELD, sub, None, 1, 0),
                         dtype=torch.uint8, device="cuda")
        y = torch.empty((1, V), device="cuda")
        ms = []
        for it in range(4):
            ev0.record(stream)
            ndf.ndf_ksg_mi_field(sub, 0, 0, [cfg.ref_v], K_NN, y, None, ws)
            ev1.record(stream)
            torch.cuda.synchronize()
            if it >= 1:
                ms.append(ev0.elapsed_time(ev1))
        out["ksg_mi"] = {
            "ndf_trained_mae": mae_mi(out_mi[0, idx[:N_MI_SAMPLE]].cpu().numpy()),
            "ndf_untrained_mae": mae_mi(y0_mi),
            "best_constant_mae": mae_mi(np.full_like(mi_o, np.median(mi_o))),
            "direct_few_members": {"members": m_few, "ms_per_field": float(np.median(ms)),
                                   "mae": mae_mi(y[0, idx[:N_MI_SAMPLE]].cpu().numpy())},
            "sample_vertices": N_MI_SAMPLE}
        del sub, ws, y
    log(f"bench: gain {out}")
    return out


def _cpu_baseline(ens, cfg, lay, log):
    """The oracle as it stands, timed on bounded samples and scaled to ms per field."""
    import torch
    import gen
    from oracle import direct
    from oracle import ndf_net as onn
    V, N = cfg.n_vertices, cfg.n_members
    cores = len(os.sched_getaffinity(0))
    out = {}
    sample = gen.random_vertices(V, 400_000, seed=99)
    idx = torch.as_tensor(sample, device="cuda")
    xs = ens.x[0][:, idx].cpu().numpy()
    xr = ens.x[0][:, cfg.ref_v].cpu().numpy()
    log("cpu baseline: oracle Pearson")
    t0 = time.time()
    direct.pearson_field(xr, xs)
    tp = time.time() - t0
    out["pearson_ms_per_field"] = tp * 1e3 * V / len(sample)
    log("cpu baseline: oracle KSG")
    nk = 60_000
    t0 = time.time()
    direct.ksg_field(xr, xs[:, :nk], K_NN)
    tk = time.time() - t0
    out["ksg_ms_per_field"] = tk * 1e3 * V / nk
    log("cpu baseline: oracle learned field")
    flat = gen.make_net_params(lay)
    net = onn.Net(flat, (cfg.nx, cfg.ny, cfg.nz), lay.res, 8, 128, 1)
    nn_s = 400_000
    q = gen.random_vertices(V, nn_s, seed=98)
    t0 = time.time()
    onn.forward(net, np.full(nn_s, cfg.ref_v), q)
    tn = time.time() - t0
    value = tn * 1e3 * V / nn_s
    return {"value": value, "unit": "ms", "cores": cores, "kind": "oracle",
            "sample": f"learned field (FP64 numpy) on {nn_s} random vertices, Pearson (C, "
                      f"OpenMP) on {len(sample)}, KSG-MI (C brute force, OpenMP) on {nk}; "
                      "each scaled to the 1.76M-vertex field",
            "seconds": tp + tk + tn, **out}


if __name__ == "__main__":
    main()
