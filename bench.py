"""Benchmark: ms per 1.76M-vertex dependence field, learned field (NDF) vs direct
Pearson / KSG-MI, on one MI355X.

Workload: synthetic paper-shaped ensemble (1000 members on 250x352x20 =
1,760,000 vertices, FP32, Gaussian-blob generator of gen/), reference vertex
(125,176,10).  One timed step is one pass of the whole hot path:

  prepare        per-vertex FP64 moments + KSG integer codes + sorted orders
  pearson_fp32   direct Pearson field, 1 reference, FP32 stream
  pearson_b64    direct Pearson fields, 64 references, split-BF16 MFMA
  ksg_field      direct KSG-MI field, 1 reference, k = 4
  targets        direct Pearson and KSG-MI targets for 2^18 random vertex pairs
  train_step     one learned-field training step on 2^18 pairs (BF16 MFMA, Adam)
  ndf_field      learned field for 1 reference at all vertices (fused BF16 kernel)
  ndf_field_fp8  the same field with E4M3 layers 2..5
  ndf_field_cached  the same field from cached query latents (merge + decoder
                 only; the cache is built once per trained network, untimed)

Every row is reported as the median, p10 and p90 over the timed steps.  After the
steps, measured on their own (not part of a step):

  config3   the training runs before timing: loss curves of the Pearson and the
            KSG-MI field, and their error against the FP64 oracle on held-out
            pairs (10^6 Pearson pairs; a stated subset for KSG-MI)
  config5   256 references on a two-variable ensemble: split-BF16 Pearson GEMM,
            learned cross-variable field in BF16 and FP8, KSG-MI on a subset
  gain      what the trained field gains over the method without it
  next_rows the calls beyond the hot path (continuous positions, difference
            fields, hash-table grid)

`value` is the learned-field ms per field (the paper's headline quantity) and
`roofline` describes the kernel that produces it.  All launches go on torch's
current stream and are timed with HIP events on it.  Inputs are resident in HBM
before timing starts.
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
N_REF5 = 256         # references of the batched two-variable workload
K_NN = 4
LR = 3e-3            # peak learning rate (cosine schedule over each training run)
LR_GRID_ONLY = 1e-2  # the grid-only ablation trains best at a higher rate
PREP_TRAIN_STEPS = 1000
MI_TRAIN_STEPS = 1500
GRID_ONLY_STEPS = 1000
CROSS_TRAIN_STEPS = 300
LOSS_EVERY = 25
N_HELD = 1_000_000   # held-out Pearson pairs (oracle)
N_HELD_MI = 2000     # held-out KSG-MI pairs (brute-force oracle on the host)
N_SAMPLE = 2000      # sampled vertices of the one-reference fields (oracle)
HASH_T = 19          # hash-table size 2^T of the hashed-grid row

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP8_TFLOPS = 5000.0
PEAK_ALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # 32-bit VALU lane operations (non-packed)

# algorithmic work per unit
NDF_MAC = 69760      # per vertex: encoder 36,864 + merge/decoder 32,896
DEC_MAC = 32896      # merge + decoder per (reference, vertex)


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--field-runs", type=int, default=50,
                    help="after the timed steps, time each field row alone this many times "
                         "(after 5 warm-up calls) for its median and p10/p90; 0 skips")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the oracle comparisons (accuracy, config3 errors, gain)")
    ap.add_argument("--no-config5", action="store_true")
    ap.add_argument("--train-steps", type=int, default=PREP_TRAIN_STEPS,
                    help="learned-field training steps before timing")
    ap.add_argument("--mi-train-steps", type=int, default=MI_TRAIN_STEPS,
                    help="training steps of the second learned field (KSG-MI targets)")
    ap.add_argument("--only", default=None,
                    help="profile one row (prepare, pearson_fp32, pearson_b64, ksg_field, "
                         "targets, train_step, ndf_field, ndf_field_fp8, ndf_field_cached, "
                         "or one of the next rows: ndf_points_rays, ndf_field_difference, "
                         "pearson_points, ksg_points, train_step_at, ndf_field_hash, "
                         "pearson_b256) W+K "
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


def _stats(ms):
    ms = np.asarray(ms, dtype=np.float64)
    return {"median": float(np.median(ms)), "p10": float(np.percentile(ms, 10)),
            "p90": float(np.percentile(ms, 90)), "n": int(ms.size)}


def _timed(fn, reps, warmup=1):
    """HIP-event times (ms) of `reps` calls of fn on torch's current stream."""
    import torch
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ms = []
    for it in range(warmup + reps):
        ev0.record(stream)
        fn(it)
        ev1.record(stream)
        torch.cuda.synchronize()
        if it >= warmup:
            ms.append(ev0.elapsed_time(ev1))
    return ms


def _train(ndf, net, P, opt, steps, make_targets, pairs_seed, ws_t, loss, dev, log, what,
           lr0=LR):
    """`steps` Adam steps on fresh 2^18-pair batches with a cosine learning-rate
    schedule from lr0; the loss every LOSS_EVERY steps."""
    import torch
    import gen
    V = net.nx * net.ny * net.nz
    hist = torch.zeros(max(steps, 1), device=dev)
    log(f"bench: training the {what} field ({steps} steps of {B_PAIRS} pairs)")
    t0 = time.time()
    for s in range(1, steps + 1):
        pr = torch.as_tensor(gen.random_pairs(V, B_PAIRS, seed=pairs_seed + s), device=dev)
        t = make_targets(pr)
        lr = lr0 * 0.5 * (1.0 + math.cos(math.pi * (s - 1) / steps))
        ndf.ndf_train_step(net, P, opt, s, pr, t, lr, loss, ws_t)
        hist[s - 1] = loss[0]
    torch.cuda.synchronize()
    sec = time.time() - t0
    st = ndf.status_word(ws_t)
    h = hist.cpu().numpy()
    curve = [[s, float(h[s - 1])] for s in range(1, steps + 1) if s == 1 or s % LOSS_EVERY == 0]
    return {"steps": steps, "seconds": sec, "batch": B_PAIRS, "lr_peak": lr0,
            "lr_schedule": "cosine",
            "final_l1_loss": float(h[steps - 1]) if steps else None,
            "loss_curve": curve, "status_word": st}


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
    ws_prep = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_PREPARE, ens), dtype=torch.uint8,
                          device=dev)
    ndf.ndf_prepare(ens, ws_prep)
    torch.cuda.synchronize()
    if ndf.status_word(ws_prep) != ndf.NDF_OK:
        raise RuntimeError("ndf_prepare reported a non-finite ensemble value")

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

    def pearson_targets(pr):
        ndf.ndf_pearson_pairs(ens, 0, 0, pr, t_pear)
        return t_pear

    def ksg_targets(pr):
        ndf.ndf_ksg_mi_pairs(ens, 0, 0, pr, K_NN, t_ksg, None, ws_kp)
        return t_ksg

    # config 3: the Pearson field is trained so the timed inference runs a trained net
    n_train = 0 if a.only else a.train_steps
    train_p = _train(ndf, net, P, opt, n_train, pearson_targets, 5000, ws_t, loss, dev, log,
                     "Pearson")
    ndf.ndf_net_quantize(net, P, ndf.NDF_PREC_FP8_E4M3, qp)   # the blob holds both precisions
    step_no = [n_train]
    # query-latent cache of the trained network (for the cached-field row)
    cache = torch.empty(ndf.ndf_infer_latent_bytes(net), dtype=torch.uint8, device=dev)
    cache_ms = _timed(lambda it: ndf.ndf_infer_latents(net, qp, cache), 3)
    out_nc = torch.empty((1, V), device=dev)

    # one network per measure: a second field trained on KSG-MI targets (same
    # architecture, so its inference cost is the timed ndf_field row)
    n_mi = 0 if (a.only or a.no_accuracy) else a.mi_train_steps
    P_mi = qp_mi = out_mi = None
    train_mi = None
    if n_mi > 0:
        P_mi = torch.empty(lay.n_floats, device=dev)
        opt_mi = torch.empty(2 * lay.n_floats, device=dev)
        ndf.ndf_net_init(net, P_mi, opt_mi, 2321)
        train_mi = _train(ndf, net, P_mi, opt_mi, n_mi, ksg_targets, 6000, ws_t, loss, dev, log,
                          "KSG-MI")
        qp_mi = torch.empty_like(qp)
        ndf.ndf_net_quantize(net, P_mi, ndf.NDF_PREC_BF16, qp_mi)
        out_mi = torch.empty((1, V), device=dev)
        ndf.ndf_infer_field(net, qp_mi, ndf.NDF_PREC_BF16, [ref], out_mi, ws_i)
        del opt_mi

    stream = torch.cuda.current_stream()
    rows = ["prepare", "pearson_fp32", "pearson_b64", "ksg_field", "targets", "train_step",
            "ndf_field", "ndf_field_fp8", "ndf_field_cached"]

    def row_prepare(it):
        ndf.ndf_prepare(ens, ws_prep)

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

    def next_rows(profile_row=None):
        """The calls beyond the hot path, with their own buffers (and, for profiling
        only, the many-reference GEMM)."""
        ens_t = ndf.Ensemble(x, cfg.nx, cfg.ny, cfg.nz, orders=False, transposed=True)
        ndf.ndf_prepare(ens_t)
        n_rays, n_steps = V // 256, 256
        ray_pos = torch.as_tensor(gen.ray_positions(n_rays, n_steps, seed=2350), device=dev)
        out_rp = torch.empty((1, ray_pos.shape[0]), device=dev)
        out_d = torch.empty(V, device=dev)
        ws_i2 = torch.empty(ndf.cached_ws_bytes(net, 2), dtype=torch.uint8, device=dev)
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
        extra = {}
        if profile_row == "pearson_b256":
            # 256 references in one read of the ensemble (the many-reference GEMM)
            refs256 = np.concatenate([[ref], gen.random_vertices(V, 255, seed=2311)])
            out_256 = torch.empty((256, V), device=dev)
            ws_256 = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_PEARSON_FIELD, ens, None,
                                                         256, ndf.NDF_PREC_SPLIT_BF16),
                                 dtype=torch.uint8, device=dev)
            extra["pearson_b256"] = lambda it: ndf.ndf_pearson_field(
                ens, 0, 0, refs256, out_256, ndf.NDF_PREC_SPLIT_BF16, ws_256)

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
                "train_step_at": train_at, **extra}, ray_pos.shape[0]

    if a.only:
        fns = row_fn if a.only in row_fn else next_rows(a.only)[0]
        ms = _timed(fns[a.only], a.steps, a.warmup)
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
    st = {r: _stats(v) for r, v in per_row.items()}
    med = {r: s["median"] for r, s in st.items()}
    ms_step = float(np.median(step_ms))
    # each field row alone, outside the timed steps: a.field_runs calls after 5 warm-ups,
    # HIP events around every call
    field_rows = ("ndf_field", "ndf_field_fp8", "ndf_field_cached", "pearson_fp32",
                  "pearson_b64", "ksg_field")
    field_runs = ({r: _stats(_timed(row_fn[r], a.field_runs, 5)) for r in field_rows}
                  if a.field_runs > 0 else {})
    names = {
        "ndf_field": "ndf_field_bf16", "ndf_field_fp8": "ndf_field_fp8",
        "ndf_field_cached": "ndf_field_bf16_cached_query_latents",
        "pearson_fp32": "pearson_field_fp32", "pearson_b64": "pearson_batch64_split_bf16_total",
        "ksg_field": "ksg_mi_field_k4", "prepare": "prepare",
        "targets": "targets_pearson_and_ksg_2^18_pairs", "train_step": "train_step_2^18_pairs",
    }
    fields = {names[r]: med[r] for r in rows}
    fields["pearson_batch64_split_bf16_per_field"] = med["pearson_b64"] / N_BATCH
    fields["ndf_query_latent_cache_build_once"] = float(np.median(cache_ms))
    spread = {names[r]: {"p10": st[r]["p10"], "p90": st[r]["p90"]} for r in rows}

    roof = _rooflines(med, N, V)
    result = {
        "metric": "ms per 1.76M-vertex dependence field: NDF vs direct Pearson/KSG-MI",
        "value": med["ndf_field"],
        "unit": "ms",
        "higher_is_better": False,
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_p10_p90": [float(np.percentile(step_ms, 10)),
                                float(np.percentile(step_ms, 90))],
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
        "fields_p10_p90": spread,
        "field_runs": {names[r]: v for r, v in field_runs.items()},
        "speedup_ndf_vs_pearson_fp32": med["pearson_fp32"] / med["ndf_field"],
        "speedup_ndf_vs_ksg": med["ksg_field"] / med["ndf_field"],
        "speedup_ndf_vs_pearson_batch64_per_field": med["pearson_b64"] / N_BATCH / med["ndf_field"],
        "dominant_kernel_of_step": max(med, key=med.get),
        "roofline": _value_roofline(med),
        "rooflines": roof,
    }

    if not a.no_next_rows:
        log("bench: next rows (continuous positions, difference fields)")
        fns, n_ray = next_rows()
        nst = {k: _stats(_timed(f, a.steps)) for k, f in fns.items()}
        nm = {k: s["median"] for k, s in nst.items()}
        nroof = {
            "ndf_points_rays": {"bound": "mfma", "achieved": 2.0 * NDF_MAC * n_ray
                                / (nm["ndf_points_rays"] * 1e-3) / 1e12,
                                "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s"},
            "ndf_field_difference": {"bound": "mfma", "achieved": 2.0 * 2 * DEC_MAC * V
                                     / (nm["ndf_field_difference"] * 1e-3) / 1e12,
                                     "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s"},
            # 2 x 8 corner rows of N FP32 members per pair
            "pearson_points": {"bound": "hbm", "achieved": 16.0 * 4 * N * B_PAIRS
                               / (nm["pearson_points"] * 1e-3) / 1e9,
                               "peak": PEAK_HBM_GBS, "unit": "GB/s"},
        }
        for r in nroof.values():
            r["frac"] = r["achieved"] / r["peak"]
        keys = {"ndf_points_rays": "ndf_points_rays_1.76M_samples",
                "ndf_field_difference": "ndf_field_difference_from_cache",
                "pearson_points": "pearson_points_targets_2^18_pairs",
                "ksg_points": "ksg_points_targets_2^18_pairs",
                "ndf_field_hash": "ndf_field_bf16_hash_table_2^19",
                "train_step_at": "train_step_at_positions_2^18_pairs"}
        result["next_rows"] = {
            "ms": {keys[k]: nm[k] for k in keys},
            "p10_p90": {keys[k]: [nst[k]["p10"], nst[k]["p90"]] for k in keys},
            "rooflines": nroof,
            "workload": f"{n_ray} samples on {n_ray // 256} rays x 256 steps; two references "
                        "for the difference; 2^18 uniform position pairs in [-1,1]^3",
        }

    result["config3"] = {"pearson_field": train_p, "ksg_mi_field": train_mi}
    if not a.no_accuracy:
        acc, sample, r_o, mi_o = _accuracy(ens, out_p, out_b, out_k, out_n, out_n8, out_mi,
                                           refs64, cfg, out_nc)
        result["accuracy"] = acc
        log("bench: held-out errors of the trained fields")
        result["config3"]["held_out"], held, r_held = _held_out(ens, cfg, net, P, P_mi, ws_t,
                                                                 log)
        log("bench: capacity sweep over the hash-table size")
        result["capacity_sweep"] = _capacity_sweep(cfg, held, r_held, pearson_targets, ws_i,
                                                   log)
        log("bench: gain of the trained field over the method without it")
        result["gain"] = _gain(ens, cfg, net, lay, sample, r_o, mi_o, out_n, out_mi, med, log,
                               pearson_targets)
    if not a.no_config5:
        del out_b, cache
        torch.cuda.empty_cache()
        result["config5"] = _config5(a, log)
    if not a.no_cpu_baseline:
        result["cpu_baseline"] = _cpu_baseline(ens, cfg, lay, log)
    print(json.dumps(result))


# ------------------------------------------------------------------ rooflines --
def _value_roofline(med):
    """The roofline of the kernel behind `value`: the fused learned-field kernel,
    0.2456 TFLOP per field (69,760 MAC per vertex), its duration taken live with
    HIP events around its single launch."""
    t = med["ndf_field"] * 1e-3
    r = {"bound": "mfma", "achieved": 2.0 * NDF_MAC * 1_760_000 / t / 1e12,
         "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
         "kernel": "infer_kernel<0> (fused grid gather + 5-layer BF16 MLP, one launch per field)",
         "algorithmic_tflop_per_launch": 2.0 * NDF_MAC * 1_760_000 / 1e12}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = _measured_traffic("ndf_field")
    return r


def _rooflines(med, N, V):
    roof = {
        "pearson_fp32": {"bound": "hbm", "achieved": 4.0 * N * V / (med["pearson_fp32"] * 1e-3)
                         / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"},
        "pearson_b64": {"bound": "hbm", "achieved": 4.0 * N * V / (med["pearson_b64"] * 1e-3)
                        / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"},
        # x read twice (moments, then codes) + int32 codes written: 12 B per sample
        "prepare_moments_codes": None,
        "ndf_field": {"bound": "mfma", "achieved": 2.0 * NDF_MAC * V / (med["ndf_field"] * 1e-3)
                      / 1e12, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s"},
        "ndf_field_fp8": {"bound": "mfma", "achieved": 2.0 * NDF_MAC * V
                          / (med["ndf_field_fp8"] * 1e-3) / 1e12, "peak": PEAK_FP8_TFLOPS,
                          "unit": "TFLOP/s"},
        # merge + decoder: 32,896 MAC per vertex, plus 256 B of cached latent read
        "ndf_field_cached": {"bound": "mfma", "achieved": 2.0 * DEC_MAC * V
                             / (med["ndf_field_cached"] * 1e-3) / 1e12,
                             "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                             "hbm_gbs": 256.0 * V / (med["ndf_field_cached"] * 1e-3) / 1e9},
        # forward + data adjoint + weight gradient of every layer: 3 x 2 x MACs
        "train_step": {"bound": "mfma", "achieved": 6.0 * (36864 * 2 * B_PAIRS + DEC_MAC * B_PAIRS)
                       / (med["train_step"] * 1e-3) / 1e12, "peak": PEAK_BF16_TFLOPS,
                       "unit": "TFLOP/s"},
    }
    del roof["prepare_moments_codes"]
    for r in roof.values():
        r["frac"] = r["achieved"] / r["peak"]
    roof["ndf_field"]["traffic"] = _measured_traffic("ndf_field")
    roof["pearson_b64"]["traffic"] = _measured_traffic("pearson_b64")
    roof["ndf_field_fp8"]["traffic"] = _measured_traffic("ndf_field_fp8")
    # the fused training step streams its slabs through HBM: the measured bytes per
    # step over the step's time, beside the MFMA fraction
    tr = _measured_traffic("train_step")
    roof["train_step"]["traffic"] = tr
    roof["train_step"]["hbm_gbs_measured"] = (tr / (med["train_step"] * 1e-3) / 1e9
                                              if tr else None)
    roof["ksg_field"] = _ksg_roofline(med["ksg_field"], N, V)
    return roof


def _ksg_roofline(ms, N, V):
    """The KSG field kernel is bound by 32-bit VALU issue (integer distances and
    counts).  Its roofline fraction is the lane operations it executes per second
    (SQ_THREAD_CYCLES_VALU of its counter profile over the live kernel time)
    against the non-packed 32-bit lane-op peak; the counter profile also gives its
    VALU issue rate, lane occupancy and LDS bank-conflict cycles.  The pruned
    search's rate in brute-force-equivalent pair evaluations V N (N - 1) is
    reported for context only."""
    import re
    r = {"bound": "alu", "unit": "T lane-ops/s", "peak": PEAK_ALU_TOPS,
         "kernel": "ksg_field_kernel<4>",
         "brute_force_equivalent_pair_evals_per_s": float(V) * N * (N - 1) / (ms * 1e-3)}
    text = _profile_text("ksg_field")
    m_t = re.search(r"SQ_THREAD_CYCLES_VALU\s+([0-9.eE+]+)", text) if text else None
    if m_t:
        r["achieved"] = float(m_t.group(1)) / (ms * 1e-3) / 1e12
        r["frac"] = r["achieved"] / r["peak"]
    else:
        r["achieved"] = r["frac"] = None
    issue = _measured_issue("ksg_field")
    if issue is not None:
        r["valu_issue_frac"], r["valu_lanes_active_frac"] = issue
    m_c = re.search(r"LDS bank-conflict cycles: .*= (\d+)% of the kernel", text) if text else None
    r["lds_bank_conflict_frac"] = int(m_c.group(1)) / 100.0 if m_c else None
    r["traffic"] = _measured_traffic("ksg_field")
    return r


# HBM bytes per launch measured with rocprofv3 PMC counters (FETCH_SIZE, WRITE_SIZE,
# scaled by a 1 GiB copy), recorded under profiles/ together with hashes of the
# kernel sources; reported only while every source still matches.
_PMC_TRAFFIC = {
    "ksg_field": ("profiles/pmc_ksg_field_paper_1760000v_1000m.txt",
                  ["paper_2307_02203_amd/csrc/ksg.hip"]),
    "ndf_field": ("profiles/pmc_infer_bf16_paper_1760000v.txt",
                  ["paper_2307_02203_amd/csrc/net_infer.hip",
                   "paper_2307_02203_amd/csrc/net.hpp"]),
    "ndf_field_fp8": ("profiles/pmc_infer_fp8_paper_1760000v.txt",
                      ["paper_2307_02203_amd/csrc/net_infer.hip",
                       "paper_2307_02203_amd/csrc/net.hpp"]),
    "pearson_b64": ("profiles/pmc_pearson_paper_1760000v_1000m.txt",
                    ["paper_2307_02203_amd/csrc/pearson.hip"]),
    "pearson_b256": ("profiles/pmc_pearson_paper_1760000v_1000m.txt",
                     ["paper_2307_02203_amd/csrc/pearson.hip"]),
    # the sum over the kernels of one step
    "train_step": ("profiles/train_step_kernels_paper_2p18pairs.txt",
                   ["paper_2307_02203_amd/csrc/net_train.hip",
                    "paper_2307_02203_amd/csrc/net.hpp"]),
}


def _profile_text(row):
    """The counter profile of `row` while each of its kernel sources still matches
    the hash recorded there (`<file> sha256 prefix at measurement: <hex>`, or after a
    comment- or whitespace-only edit of it), else None."""
    import hashlib
    import re
    if row not in _PMC_TRAFFIC:
        return None
    prof, srcs = _PMC_TRAFFIC[row]
    try:
        text = open(os.path.join(ROOT, prof)).read()
    except OSError:
        return None
    for src in srcs:
        try:
            sha = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
        except OSError:
            return None
        base = os.path.basename(src)
        shas = re.findall(re.escape(base) + r" sha256 prefix (?:at measurement|after a "
                          r"(?:comment|whitespace)-only edit): ([0-9a-f]+)", text)
        if not shas or not any(sha.startswith(h) for h in shas):
            return None
    return text


def _measured_traffic(row):
    """HBM bytes per launch from the row's counter profile: the line tagged with the row
    (`traffic_bytes_per_launch[row]: X`, in a profile of several kernels), else the
    profile's untagged line."""
    import re
    text = _profile_text(row)
    if not text:
        return None
    m_val = (re.search(r"traffic_bytes_per_launch\[" + re.escape(row) + r"\]: ([0-9.eE+]+)", text)
             or re.search(r"traffic_bytes_per_launch: ([0-9.eE+]+)", text))
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


# ------------------------------------------------------------------- accuracy --
def _accuracy(ens, out_p, out_b, out_k, out_n, out_n8, out_mi, refs64, cfg, out_nc):
    """Errors of the timed outputs against the FP64 oracle on sampled vertices."""
    import torch
    import gen
    from oracle import direct
    V = cfg.n_vertices
    sample = gen.random_vertices(V, N_SAMPLE, seed=4242)
    idx = torch.as_tensor(sample, device="cuda")
    xs = ens.x[0][:, idx].cpu().numpy()
    xr = ens.x[0][:, cfg.ref_v].cpu().numpy()
    r_o = direct.pearson_field(xr, xs)
    mi_o = direct.ksg_field(xr, xs, K_NN)
    p = out_p[0, idx].cpu().numpy()
    b0 = out_b[0, idx].cpu().numpy()
    k = out_k[0, idx].cpu().numpy()
    n = out_n[0, idx].cpu().numpy()
    n8 = out_n8[0, idx].cpu().numpy()
    extra = {}
    if out_mi is not None:
        m = out_mi[0, idx].cpu().numpy()
        extra = {"ndf_mi_vs_oracle_mae": float(np.mean(np.abs(m - mi_o))),
                 "ndf_mi_vs_oracle_max_abs_err": float(np.max(np.abs(m - mi_o)))}
    return {
        **extra,
        "sample_vertices": int(len(sample)),
        "pearson_fp32_max_abs_err": float(np.max(np.abs(p - r_o))),
        "pearson_split_bf16_max_abs_err": float(np.max(np.abs(b0 - r_o))),
        "ksg_mi_max_abs_err": float(np.max(np.abs(k - mi_o))),
        "ndf_vs_oracle_pearson_mae": float(np.mean(np.abs(n - r_o))),
        "ndf_vs_oracle_pearson_max_abs_err": float(np.max(np.abs(n - r_o))),
        "ndf_fp8_vs_oracle_pearson_mae": float(np.mean(np.abs(n8 - r_o))),
        "ndf_fp8_vs_oracle_pearson_max_abs_err": float(np.max(np.abs(n8 - r_o))),
        "ndf_cached_equals_fused_bitwise": bool(torch.equal(out_nc, out_n)),
        "population_rho_mae_of_oracle": float(np.mean(np.abs(
            r_o - gen.population_rho(cfg, np.full(len(sample), cfg.ref_v), sample)))),
    }, sample, r_o, mi_o


def _columns(x, idx, chunk):
    """Host copies of the member columns x[:, idx] (torch gathers on the device)."""
    import torch
    for c0 in range(0, len(idx), chunk):
        it = torch.as_tensor(idx[c0:c0 + chunk], device=x.device)
        yield c0, x.index_select(1, it).cpu().numpy()


def _held_out(ens, cfg, net, P, P_mi, ws_t, log):
    """Held-out error of the trained fields (config 3): the Pearson field on 10^6
    uniformly drawn vertex pairs, the KSG-MI field on a 2,000-pair subset (the
    brute-force oracle costs N^2 per pair), each against the FP64 oracle, with
    the direct GPU estimator's own error on the same pairs alongside."""
    import torch
    import gen
    from oracle import direct
    from paper_2307_02203_amd import ndf
    V = cfg.n_vertices
    x0 = ens.x[0]
    held = gen.random_pairs(V, N_HELD, seed=2399)
    y = torch.empty(N_HELD, device="cuda")
    d = torch.empty(N_HELD, device="cuda")
    for c0 in range(0, N_HELD, B_PAIRS):
        pr = torch.as_tensor(held[c0:c0 + B_PAIRS], device="cuda")
        ndf.ndf_net_forward(net, P, pr, y[c0:c0 + len(pr)], ws_t)
        ndf.ndf_pearson_pairs(ens, 0, 0, pr, d[c0:c0 + len(pr)])
    y = y.cpu().numpy().astype(np.float64)
    d = d.cpu().numpy().astype(np.float64)
    t0 = time.time()
    r_o = np.empty(N_HELD)
    chunk = 50_000
    for (c0, xa), (_, xb) in zip(_columns(x0, held[:, 0], chunk), _columns(x0, held[:, 1], chunk)):
        r_o[c0:c0 + xa.shape[1]] = direct.pearson_pairs(xa, xb)
    rho = np.concatenate([gen.population_rho(cfg, held[c0:c0 + 100_000, 0],
                                             held[c0:c0 + 100_000, 1])
                          for c0 in range(0, N_HELD, 100_000)])
    log(f"bench: held-out Pearson oracle on {N_HELD} pairs: {time.time() - t0:.1f} s")
    out = {"pearson": {
        "pairs": N_HELD, "seed": 2399,
        "ndf_mae_vs_oracle": float(np.mean(np.abs(y - r_o))),
        "ndf_max_abs_err_vs_oracle": float(np.max(np.abs(y - r_o))),
        "ndf_mae_vs_population_rho": float(np.mean(np.abs(y - rho))),
        "oracle_mae_vs_population_rho": float(np.mean(np.abs(r_o - rho))),
        "direct_gpu_targets_max_abs_err_vs_oracle": float(np.max(np.abs(d - r_o))),
        "best_constant_mae_vs_oracle": float(np.mean(np.abs(r_o - np.median(r_o))))}}
    if P_mi is not None:
        hm = held[:N_HELD_MI]
        ym = torch.empty(N_HELD_MI, device="cuda")
        dm = torch.empty(N_HELD_MI, device="cuda")
        pr = torch.as_tensor(hm, device="cuda")
        ndf.ndf_net_forward(net, P_mi, pr, ym, ws_t)
        ws_kp = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_KSG_PAIRS, ens, None, 1, 0),
                            dtype=torch.uint8, device="cuda")
        ndf.ndf_ksg_mi_pairs(ens, 0, 0, pr, K_NN, dm, None, ws_kp)
        ym = ym.cpu().numpy().astype(np.float64)
        dm = dm.cpu().numpy().astype(np.float64)
        xa = x0.index_select(1, pr[:, 0]).cpu().numpy()
        xb = x0.index_select(1, pr[:, 1]).cpu().numpy()
        mi_o = direct.ksg_pairs(xa, xb, K_NN)
        out["ksg_mi"] = {
            "pairs": N_HELD_MI, "seed": 2399, "subset": f"the first {N_HELD_MI} held-out pairs",
            "ndf_mae_vs_oracle": float(np.mean(np.abs(ym - mi_o))),
            "ndf_max_abs_err_vs_oracle": float(np.max(np.abs(ym - mi_o))),
            "direct_gpu_targets_max_abs_err_vs_oracle": float(np.max(np.abs(dm - mi_o))),
            "best_constant_mae_vs_oracle": float(np.mean(np.abs(mi_o - np.median(mi_o))))}
    return out, held, r_o


# (log2 table size, Fourier frequencies): the table-size sweep, and at the dense
# size the input embedding with and without Fourier features (Sec. 4.2, Eq. 4)
SWEEP_MODELS = ((14, 0), (16, 0), (18, 0), (20, 0), (22, 0), (22, 12))
SWEEP_STEPS = 600


def _capacity_sweep(cfg, held, r_o, pearson_targets, ws_i, log):
    """Model size against accuracy (Sec. 6.3, Fig. 5) on the synthetic ensemble:
    the network with hash tables of 2^T cells (levels larger than that hashed; at
    T = 22 every level of this grid is dense), each trained for SWEEP_STEPS steps
    on the same Pearson targets, and its error on the 10^6 held-out pairs against
    the FP64 oracle.  The MLP widths are fixed by the kernels (5 x 128), so only
    the table size varies; at the dense size one more model adds the Fourier
    features of the position (L = 12) to the input embedding."""
    import torch
    import gen
    from paper_2307_02203_amd import ndf
    V = cfg.n_vertices
    out = []
    loss = torch.empty(1, device="cuda")
    for T, L in SWEEP_MODELS:
        lay = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz, log2_hashmap=T, fourier=L)
        net = ndf.net_config(cfg.nx, cfg.ny, cfg.nz, lay.res, log2_hashmap=T, fourier=L)
        P = torch.empty(lay.n_floats, device="cuda")
        opt = torch.empty(2 * lay.n_floats, device="cuda")
        ndf.ndf_net_init(net, P, opt, 2320)
        ws = torch.empty(ndf.train_ws_bytes(net, B_PAIRS) + lay.n_floats * 4 + 256,
                         dtype=torch.uint8, device="cuda")
        tr = _train(ndf, net, P, opt, SWEEP_STEPS, pearson_targets, 5000, ws, loss, "cuda", log,
                    f"T={T} fourier={L}")
        y = torch.empty(len(held), device="cuda")
        for c0 in range(0, len(held), B_PAIRS):
            pr = torch.as_tensor(held[c0:c0 + B_PAIRS], device="cuda")
            ndf.ndf_net_forward(net, P, pr, y[c0:c0 + len(pr)], ws)
        y = y.cpu().numpy().astype(np.float64)
        q = torch.empty(ndf.ndf_net_qparam_bytes(net, ndf.NDF_PREC_BF16), dtype=torch.uint8,
                        device="cuda")
        ndf.ndf_net_quantize(net, P, ndf.NDF_PREC_BF16, q)
        f = torch.empty((1, V), device="cuda")
        ms = _timed(lambda it: ndf.ndf_infer_field(net, q, ndf.NDF_PREC_BF16, [cfg.ref_v], f,
                                                   ws_i), 5, 1)
        out.append({"log2_hashmap": T, "fourier": L,
                    "cells_per_level": [lay.cells(l) for l in range(4)],
                    "param_mb": 4.0 * lay.n_floats / 1e6,
                    "inference_param_mb": ndf.ndf_net_qparam_bytes(net, ndf.NDF_PREC_BF16) / 1e6,
                    "held_out_mae_vs_oracle": float(np.mean(np.abs(y - r_o))),
                    "final_l1_loss": tr["final_l1_loss"], "field_ms": float(np.median(ms))})
        del P, opt, ws, q, f
    dense = [m for m in out if m["log2_hashmap"] == 22]
    emb = {f"fourier_{m['fourier']}": m["held_out_mae_vs_oracle"] for m in dense}
    return {"steps_per_model": SWEEP_STEPS, "lr_peak": LR, "held_out_pairs": len(held),
            "models": out, "embedding_held_out_mae": emb}


# ------------------------------------------------------------------------ gain --
def _coarse_axis(n, s):
    a = np.arange(0, n, s)
    return a if a[-1] == n - 1 else np.append(a, n - 1)


def _upsample(coarse, axes, v, cfg):
    """Trilinear interpolation of a field given on the coarse grid axes (ix, iy,
    iz) at vertices v."""
    i, j, k = (np.asarray(t, dtype=np.float64) for t in
               (v % cfg.nx, (v // cfg.nx) % cfg.ny, v // (cfg.nx * cfg.ny)))
    f = coarse.reshape(len(axes[2]), len(axes[1]), len(axes[0]))
    lo, w = [], []
    for ax, c in zip(axes, (i, j, k)):
        b = np.clip(np.searchsorted(ax, c, side="right") - 1, 0, len(ax) - 2)
        lo.append(b)
        w.append((c - ax[b]) / (ax[b + 1] - ax[b]))
    out = np.zeros(len(v))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                wt = ((w[0] if dx else 1 - w[0]) * (w[1] if dy else 1 - w[1])
                      * (w[2] if dz else 1 - w[2]))
                out += wt * f[lo[2] + dz, lo[1] + dy, lo[0] + dx]
    return out


def _equal_time_coarse(ens, cfg, budget_ms, measure, log, what):
    """The direct estimator evaluated only on a coarse sub-grid of vertices and
    interpolated trilinearly: the finest stride whose call fits the learned
    field's time.  Returns (stride, ms, coarse field, axes)."""
    import torch
    from paper_2307_02203_amd import ndf
    for s in (3, 4, 5, 6, 8, 10, 12, 16, 24, 32):
        axes = [_coarse_axis(cfg.nx, s), _coarse_axis(cfg.ny, s), _coarse_axis(cfg.nz, s)]
        iz, iy, ix = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        cv = (ix + cfg.nx * (iy + cfg.ny * iz)).reshape(-1)
        pairs = torch.as_tensor(np.stack([np.full(len(cv), cfg.ref_v), cv], axis=1),
                                device="cuda")
        out = torch.empty(len(cv), device="cuda")
        ms = float(np.median(_timed(lambda it: measure(pairs, out), 5, 2)))
        if ms <= budget_ms:
            log(f"bench: equal-time {what}: stride {s}, {len(cv)} vertices, {ms:.3f} ms")
            return s, ms, out.cpu().numpy().astype(np.float64), axes
    return None


def _gain(ens, cfg, net, lay, sample, r_o, mi_o, out_n, out_mi, med, log, pearson_targets):
    """What the trained field gains over the method without it, on the sampled
    vertices of one reference's field against the FP64 oracle: the untrained
    (initialised) field, the best constant predictor, and the direct estimator at
    the learned field's cost (equal time) two ways: members cut until one field
    costs that much, and the full estimator on a coarse sub-grid of vertices,
    interpolated trilinearly.  For KSG-MI the vertices in the untransformed half
    of the domain (bivariate Gaussian, so MI = -1/2 ln(1 - rho^2) in closed form)
    are also compared with that population MI, by bands of |rho|."""
    import torch
    import gen
    from paper_2307_02203_amd import ndf
    V, N = cfg.n_vertices, cfg.n_members
    idx = torch.as_tensor(sample, device="cuda")
    mae = lambda y: float(np.mean(np.abs(y - r_o)))  # noqa: E731
    t_ndf = med["ndf_field"]
    rho = gen.population_rho(cfg, np.full(len(sample), cfg.ref_v), sample)
    n_tr = out_n[0, idx].cpu().numpy().astype(np.float64)
    out = {"ndf_trained_mae": mae(n_tr),
           "best_constant_mae": mae(np.full_like(r_o, np.median(r_o))),
           "ndf_trained_mae_vs_population_rho": float(np.mean(np.abs(n_tr - rho))),
           "oracle_mae_vs_population_rho": float(np.mean(np.abs(r_o - rho)))}

    P0 = torch.empty(lay.n_floats, device="cuda")
    ndf.ndf_net_init(net, P0, None, 2320)
    qp0 = torch.empty(ndf.ndf_net_qparam_bytes(net, ndf.NDF_PREC_BF16), dtype=torch.uint8,
                      device="cuda")
    ndf.ndf_net_quantize(net, P0, ndf.NDF_PREC_BF16, qp0)
    ws_i = torch.empty(ndf.infer_ws_bytes(net, 1, ndf.NDF_PREC_BF16), dtype=torch.uint8,
                       device="cuda")
    y0 = torch.empty((1, V), device="cuda")
    ndf.ndf_infer_field(net, qp0, ndf.NDF_PREC_BF16, [cfg.ref_v], y0, ws_i)
    y0 = y0[0, idx].cpu().numpy().astype(np.float64)
    out["ndf_untrained_mae"] = mae(y0)
    del P0, qp0

    # the grid-only network (encoder MLP omitted, Sec. 6.3, Fig. 6), same targets
    lay_g = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz, grid_only=True)
    net_g = ndf.net_config(cfg.nx, cfg.ny, cfg.nz, lay_g.res, grid_only=True)
    P_g = torch.empty(lay_g.n_floats, device="cuda")
    opt_g = torch.empty(2 * lay_g.n_floats, device="cuda")
    ndf.ndf_net_init(net_g, P_g, opt_g, 2320)
    ws_g = torch.empty(ndf.train_ws_bytes(net_g, B_PAIRS) + lay_g.n_floats * 4 + 256,
                       dtype=torch.uint8, device="cuda")
    loss = torch.empty(1, device="cuda")
    tr_g = _train(ndf, net_g, P_g, opt_g, GRID_ONLY_STEPS, pearson_targets, 5000, ws_g, loss,
                  "cuda", log, "grid-only Pearson", lr0=LR_GRID_ONLY)
    qp_g = torch.empty(ndf.ndf_net_qparam_bytes(net_g, ndf.NDF_PREC_BF16), dtype=torch.uint8,
                       device="cuda")
    ndf.ndf_net_quantize(net_g, P_g, ndf.NDF_PREC_BF16, qp_g)
    y_g = torch.empty((1, V), device="cuda")
    ms_g = _timed(lambda it: ndf.ndf_infer_field(net_g, qp_g, ndf.NDF_PREC_BF16, [cfg.ref_v], y_g,
                                                 ws_i), 5, 1)
    out["grid_only_network"] = {
        "mae": mae(y_g[0, idx].cpu().numpy()), "ms_per_field": float(np.median(ms_g)),
        "training": {k: tr_g[k] for k in ("steps", "lr_peak", "final_l1_loss", "seconds")},
        "note": "encoder MLP omitted: the latent is the 32 grid features (Sec. 6.3 ablation)"}
    del P_g, opt_g, ws_g, qp_g, y_g, ws_i

    # equal time, fewer members: the direct cost is linear in N
    m_eq = int(max(8, min(N, round(N * t_ndf / med["pearson_fp32"]))))
    sub = ndf.Ensemble(ens.x[:, :m_eq], cfg.nx, cfg.ny, cfg.nz, orders=False)
    ndf.ndf_prepare(sub)
    ws = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_PEARSON_FIELD, sub, None, 1, 0),
                     dtype=torch.uint8, device="cuda")
    y = torch.empty((1, V), device="cuda")
    ms = _timed(lambda it: ndf.ndf_pearson_field(sub, 0, 0, [cfg.ref_v], y, ndf.NDF_PREC_FP32,
                                                 ws), 5, 2)
    out["equal_time_direct_pearson_fewer_members"] = {
        "members": m_eq, "ms_per_field": float(np.median(ms)), "mae": mae(y[0, idx].cpu().numpy())}
    del sub, ws, y
    # equal time, coarse grid: direct Pearson of (ref, v) pairs on a sub-grid
    co = _equal_time_coarse(ens, cfg, t_ndf,
                            lambda pr, o: ndf.ndf_pearson_pairs(ens, 0, 0, pr, o), log, "Pearson")
    if co:
        s, ms, f, axes = co
        out["equal_time_direct_pearson_coarse_grid"] = {
            "stride": s, "ms_per_field": ms, "mae": mae(_upsample(f, axes, sample, cfg)),
            "note": "direct Pearson at every s-th vertex per axis, trilinear upsampling"}

    if out_mi is not None:
        mae_mi = lambda z: float(np.mean(np.abs(z - mi_o)))  # noqa: E731
        m_tr = out_mi[0, idx].cpu().numpy().astype(np.float64)
        g = {"ndf_trained_mae": mae_mi(m_tr), "ndf_untrained_mae": mae_mi(y0),
             "best_constant_mae": mae_mi(np.full_like(mi_o, np.median(mi_o))),
             "sample_vertices": int(len(sample))}
        ws_kp = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_KSG_PAIRS, ens, None, 1, 0),
                            dtype=torch.uint8, device="cuda")
        co = _equal_time_coarse(
            ens, cfg, t_ndf,
            lambda pr, o: ndf.ndf_ksg_mi_pairs(ens, 0, 0, pr, K_NN, o, None, ws_kp), log, "KSG")
        up = None
        if co:
            s, ms, f, axes = co
            up = _upsample(f, axes, sample, cfg)
            g["equal_time_direct_ksg_coarse_grid"] = {
                "stride": s, "ms_per_field": ms, "mae": mae_mi(up),
                "note": "direct KSG-MI at every s-th vertex per axis, trilinear upsampling"}
        # population MI where (X, Y) is bivariate Gaussian: both vertices in the
        # untransformed half i >= nx/2 (the reference is)
        lin = (sample % cfg.nx) >= cfg.nx / 2.0
        mi_pop = -0.5 * np.log1p(-np.minimum(rho * rho, 1.0 - 1e-12))
        bands = []
        for lo, hi in ((0.0, 0.2), (0.2, 0.5), (0.5, 0.8), (0.8, 1.01)):
            sel = lin & (np.abs(rho) >= lo) & (np.abs(rho) < hi)
            if sel.sum() < 5:
                continue
            b = {"abs_rho": [lo, min(hi, 1.0)], "vertices": int(sel.sum()),
                 "population_mi_mean": float(np.mean(mi_pop[sel])),
                 "ndf_mae_vs_population_mi": float(np.mean(np.abs(m_tr[sel] - mi_pop[sel]))),
                 "direct_ksg_1000_members_mae_vs_population_mi":
                     float(np.mean(np.abs(mi_o[sel] - mi_pop[sel])))}
            if up is not None:
                b["equal_time_coarse_mae_vs_population_mi"] = float(
                    np.mean(np.abs(up[sel] - mi_pop[sel])))
            bands.append(b)
        g["linear_half_vs_population_mi"] = bands
        out["ksg_mi"] = g
    log(f"bench: gain {json.dumps(out)}")
    return out


# --------------------------------------------------------------------- config 5 --
def _config5(a, log):
    """256 references against all 1.76M vertices of a two-variable ensemble (the
    second variable: smoothed blobs through tanh plus independent noise): direct
    split-BF16 Pearson across variables, the learned cross-variable field (two
    encoders, trained on cross-variable targets) in BF16 and FP8, and direct
    KSG-MI across variables on two of the references."""
    import torch
    import gen
    from oracle import direct
    from oracle import ndf_net as onn
    from paper_2307_02203_amd import ndf
    cfg = gen.CONFIGS["paper2v"]
    V = cfg.n_vertices
    log("bench: config 5, two-variable ensemble")
    x = gen.make_ensemble(cfg, device="cuda")
    e = ndf.Ensemble(x, cfg.nx, cfg.ny, cfg.nz)
    ndf.ndf_prepare(e)
    refs = np.concatenate([[cfg.ref_v], gen.random_vertices(V, N_REF5 - 1, seed=2311)])
    res = {"workload": f"{N_REF5} references x {V} vertices, variable 0 -> variable 1, "
                       "1000 members"}
    out = torch.empty((N_REF5, V), device="cuda")
    # direct split-BF16 Pearson GEMM across variables
    ws = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_PEARSON_FIELD, e, None, N_REF5,
                                             ndf.NDF_PREC_SPLIT_BF16), dtype=torch.uint8,
                     device="cuda")
    st = _stats(_timed(lambda it: ndf.ndf_pearson_field(e, 0, 1, refs, out,
                                                        ndf.NDF_PREC_SPLIT_BF16, ws), 5, 1))
    kpad = (1000 + 15) // 16 * 16  # members padded to whole 16-member k-steps
    res["pearson_split_bf16_gemm"] = {
        **st, "ms_per_field": st["median"] / N_REF5,
        "hbm_gbs_algorithmic": (4.0 * 1000 * V + 4.0 * N_REF5 * V) / (st["median"] * 1e-3) / 1e9,
        # the contraction itself: one product over the members
        "tflops_algorithmic": 2.0 * N_REF5 * 1000 * V / (st["median"] * 1e-3) / 1e12,
        # what the matrix cores execute: three bf16 products (hi*hi, hi*lo, lo*hi)
        "mfma_tflops_executed": 3 * 2.0 * N_REF5 * kpad * V / (st["median"] * 1e-3) / 1e12,
        "traffic": _measured_traffic("pearson_b256")}
    sample = gen.random_vertices(V, 200, seed=93)
    s_t = torch.as_tensor(sample, device="cuda")
    g = out[:, s_t].cpu().numpy()
    xs = x[1][:, s_t].cpu().numpy()
    xr = x[0][:, torch.as_tensor(refs, device="cuda")].cpu().numpy()
    worst = max(float(np.max(np.abs(g[i] - direct.pearson_field(xr[:, i], xs))))
                for i in range(0, N_REF5, 8))
    res["pearson_split_bf16_gemm"]["max_abs_err_vs_oracle_sampled"] = worst
    del ws
    # the learned cross-variable field
    lay = gen.NetLayout.for_grid(cfg.nx, cfg.ny, cfg.nz, n_enc=2)
    net = ndf.net_config(cfg.nx, cfg.ny, cfg.nz, lay.res, n_enc=2)
    P = torch.empty(lay.n_floats, device="cuda")
    opt = torch.empty(2 * lay.n_floats, device="cuda")
    ndf.ndf_net_init(net, P, opt, 2330)
    ws_t = torch.empty(ndf.train_ws_bytes(net, B_PAIRS) + lay.n_floats * 4 + 256,
                       dtype=torch.uint8, device="cuda")
    loss = torch.empty(1, device="cuda")
    tg = torch.empty(B_PAIRS, device="cuda")

    def cross_targets(pr):
        ndf.ndf_pearson_pairs(e, 0, 1, pr, tg)
        return tg

    res["training"] = _train(ndf, net, P, opt, CROSS_TRAIN_STEPS, cross_targets, 7000, ws_t,
                             loss, "cuda", log, "cross-variable Pearson")
    del opt, ws_t
    qp = torch.empty(ndf.ndf_net_qparam_bytes(net, ndf.NDF_PREC_FP8_E4M3), dtype=torch.uint8,
                     device="cuda")
    ndf.ndf_net_quantize(net, P, ndf.NDF_PREC_FP8_E4M3, qp)
    rng = np.random.default_rng(2398)
    ri = rng.integers(0, N_REF5, 4000)
    qv = gen.random_vertices(V, 4000, seed=95)
    truth = np.array([direct.pearson(x[0][:, int(refs[i])].cpu().numpy(),
                                     x[1][:, int(q)].cpu().numpy())
                      for i, q in zip(ri[:400], qv[:400])])
    for prec, name in ((ndf.NDF_PREC_BF16, "ndf_bf16"), (ndf.NDF_PREC_FP8_E4M3, "ndf_fp8")):
        wsi = torch.empty(ndf.infer_ws_bytes(net, N_REF5, prec), dtype=torch.uint8,
                          device="cuda")
        st = _stats(_timed(lambda it: ndf.ndf_infer_field(net, qp, prec, refs, out, wsi), 3, 1))
        # both precisions: the query encoder once, the decoder per reference
        flops = 2.0 * (DEC_MAC * N_REF5 * V + 36864 * V)
        ri_t = torch.as_tensor(ri, device="cuda")
        qv_t = torch.as_tensor(qv, device="cuda")
        got = out[ri_t, qv_t].cpu().numpy().astype(np.float64)
        res[name] = {**st, "ms_per_field": st["median"] / N_REF5,
                     "mae_vs_oracle_400_pairs": float(np.mean(np.abs(got[:400] - truth))),
                     "algorithmic_tflops": flops / (st["median"] * 1e-3) / 1e12}
        if name == "ndf_bf16":
            flat = P.cpu().numpy()
            onet = onn.Net(flat, (cfg.nx, cfg.ny, cfg.nz), lay.res, 8, 128, 2)
            want, _ = onn.forward(onet, refs[ri], qv)
        res[name]["network_rel_l2_vs_fp64_network"] = float(
            np.linalg.norm(got - want) / np.linalg.norm(want))
        del wsi
    res["ndf_bf16"]["note"] = ("query latents computed once into the workspace, then 16 "
                               "references decoded per read of them")
    res["ndf_fp8"]["note"] = ("query latents computed once (BF16) into the workspace, then 16 "
                              "references per read of them through an E4M3 decoder")
    # direct KSG-MI across variables on two references
    wsk = torch.empty(ndf.ndf_workspace_bytes(ndf.NDF_OP_KSG_FIELD, e, None, 2, 0),
                      dtype=torch.uint8, device="cuda")
    st = _stats(_timed(lambda it: ndf.ndf_ksg_mi_field(e, 0, 1, refs[:2], K_NN, out[:2], None,
                                                       wsk), 2, 1))
    res["ksg_mi_field"] = {**st, "references": 2, "ms_per_field": st["median"] / 2}
    del x, e, out
    torch.cuda.empty_cache()
    return res


# ----------------------------------------------------------------- cpu baseline --
def _cpu_baseline(ens, cfg, lay, log):
    """The oracle as it stands, timed on bounded samples and scaled to ms per field."""
    import torch
    import gen
    from oracle import direct
    from oracle import ndf_net as onn
    V, N = cfg.n_vertices, cfg.n_members
    cores = direct.max_threads()
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
    direct.set_threads(1)
    t0 = time.time()
    direct.pearson_field(xr, xs[:, :50_000])
    out["pearson_ms_per_field_1_thread"] = (time.time() - t0) * 1e3 * V / 50_000
    direct.set_threads(cores)
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
                      f"OpenMP, {cores} threads; and 1 thread on 50000) on {len(sample)}, "
                      f"KSG-MI (C brute force, OpenMP) on {nk}; each scaled to the "
                      "1.76M-vertex field",
            "seconds": tp + tk + tn, **out}


if __name__ == "__main__":
    main()
