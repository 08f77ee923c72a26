#!/usr/bin/env python3
"""Throughput of the StereoVAE hot path on one MI355X.

One step = one pass of the whole inference path over a batch of pairs:
reduction + census of both views, Hamming cost + WTA, and the refinement
network's forward pass, on seeded synthetic 1242x375 pairs (9x7 census at
1/4 resolution = 311x94, D = 48 there = 192 full-res, network widths
2-32-64-128, latent 128) with inputs resident in HBM.

Timed regions (each: W warm-up steps, then exactly K steps bracketed by
torch.cuda.synchronize()):
  * the headline: the step replayed from a hipGraph, FP32 network, batch 1;
  * a profiled eager pass of the same step: HIP events around every kernel,
    on the stream it runs on, give each kernel's average duration, from which
    the dominant kernel's roofline fraction is computed;
  * variants: BF16 network at batch 1, FP32 / BF16 at batch 64.
The CPU oracle is timed on a bounded sample of the same workload.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# workload (one pair): KITTI-sized synthetic scene
H, W, F, WIN_W, WIN_H, D = 375, 1242, 4, 9, 7, 48
C1, C2, C3, LAT = 32, 64, 128, 128
NBITS = WIN_W * WIN_H - 1
WEIGHT_SEED = 7002
PROF_REPEAT = 10      # launches per event pair in the profiled pass at the headline batch

PEAK = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "mfma_TFLOPs": {"f32": 157.3, "bf16": 2500.0, "f16": 2500.0},
    "alu_Tops": 256 * 64 * 2.4e9 / 1e12,   # 256 CUs x 64 lanes x 2.4 GHz, one int op per lane-cycle
}


def levels(B):
    h0, w0 = -(-H // F), -(-W // F)
    hs, ws = [h0], [w0]
    for _ in range(3):
        hs.append(-(-hs[-1] // 2))
        ws.append(-(-ws[-1] // 2))
    return hs, ws


def stage_work(stage, B, dtype):
    """Algorithmic work of one launch of `stage` on a batch of B pairs:
    (bound, amount, unit) with unit GB or TFLOP or Tops."""
    hs, ws = levels(B)
    px = [B * hs[k] * ws[k] for k in range(4)]
    es = 4 if dtype == "f32" else 2
    if stage == "E1":  # direct stencil: read the coarse maps, write E1
        return "hbm", (2.0 * px[0] + px[1] * C1 * es) / 1e9, "GB"
    conv = {  # (M, N, K) of the implicit GEMM
        "E2": (px[2], C2, C1 * 9), "E3": (px[3], C3, C2 * 9),
        "HEAD": (px[3], 2 * LAT, C3), "G3": (px[3], C3, LAT),
        "G2": (px[2], C2, (C3 + C2) * 9), "G1": (px[1], C1, (C2 + C1) * 9),
        "G0": (px[0], C1, (C1 + 2) * 9),
    }
    if stage == "HEAD+G3":  # the two 1x1 layers of an inference pass, one kernel
        return "mfma", sum(2.0 * M * N * K for M, N, K in (conv["HEAD"], conv["G3"])) / 1e12, "TFLOP"
    if stage in conv:
        M, N, K = conv[stage]
        return "mfma", 2.0 * M * N * K / 1e12, "TFLOP"
    if stage == "census":   # read both full-res views, write both census maps + reduced left
        return "hbm", (2.0 * B * H * W + 2 * 8.0 * px[0] + px[0]) / 1e9, "GB"
    if stage == "cost_wta":  # 6 integer ops per (pixel, d): 2 xor, 2 popcount, pack, min
        return "alu", 6.0 * D * px[0] / 1e12, "Tops"
    if stage == "final_gather":  # write the full-res map; read the nine FP32 projections and the coarse map
        return "hbm", (4.0 * B * H * W + (9 * 4 + 1.0) * px[0]) / 1e9, "GB"
    return None, 0.0, ""


def merge_latent(prof):
    """An inference pass that runs the head and G3 as one kernel records it
    as the head's stage and nothing as G3's: name that entry HEAD+G3."""
    prof = dict(prof)
    if prof.get("G3", (0.0, 0))[1] == 0 and prof.get("HEAD", (0.0, 0))[1] > 0:
        prof["HEAD+G3"] = prof.pop("HEAD")
        prof.pop("G3", None)
    return prof


_INPUTS = {}


def make_inputs(B, device):
    """B seeded 1242x375 pairs (seeds 2000..2000+B-1), cached per batch size."""
    if (B, str(device)) in _INPUTS:
        return _INPUTS[(B, str(device))]
    import torch
    from synth import gen_preset
    pairs = [gen_preset("pair1242x375", i) for i in range(B)]
    left = torch.from_numpy(np.stack([p.left for p in pairs])).to(device)
    right = torch.from_numpy(np.stack([p.right for p in pairs])).to(device)
    gt = np.stack([p.gt for p in pairs])
    _INPUTS[(B, str(device))] = (left, right, gt)
    return left, right, gt


def make_params():
    from synth import he_init_params
    shapes = [(C1, 2, 3), (C2, C1, 3), (C3, C2, 3), (2 * LAT, C3, 1), (C3, LAT, 1),
              (C2, C3 + C2, 3), (C1, C2 + C1, 3), (C1, C1 + 2, 3), (1, C1 + 2, 3)]
    params = he_init_params(shapes, seed=WEIGHT_SEED)
    flat = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)
    return params, flat


class Path:
    """Preallocated buffers and the step of the whole path for one batch size and dtype."""

    def __init__(self, B, dtype, flat, left, right):
        import torch
        import paper_2305_11566_amd as sv
        self.sv, self.torch = sv, torch
        self.B, self.dtype = B, dtype
        self.left, self.right = left, right
        hs, ws = levels(B)
        dev = left.device
        self.cl = torch.empty((B, hs[0], ws[0]), dtype=torch.int64, device=dev)
        self.cr = torch.empty_like(self.cl)
        self.low = torch.empty((B, hs[0], ws[0]), dtype=torch.uint8, device=dev)
        self.disp = torch.empty_like(self.low)
        self.out = torch.empty((B, H, W), dtype=torch.float32, device=dev)
        self.ml = torch.empty((B, hs[3], ws[3], 2 * LAT), dtype=torch.float32, device=dev)
        self.ref = sv.Refiner(C1, C2, C3, LAT, F, dtype)
        self.ref.pack(torch.from_numpy(flat).to(dev))
        self.ref.workspace(B, H, W)
        self.graph = None

    def step(self):
        sv = self.sv
        sv.sv_census_pair(self.left, self.right, F, WIN_W, WIN_H, out=(self.cl, self.cr, self.low))
        sv.sv_cost_wta(self.cl, self.cr, D, NBITS, out=self.disp)
        self.ref.forward(self.disp, self.low, H, W, out=self.out, mu_logvar=self.ml)

    def capture(self):
        torch = self.torch
        self.step()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g

    def timed(self, steps, warmup, graph=True):
        torch = self.torch
        run = self.graph.replay if (graph and self.graph is not None) else self.step
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps


def _oracle_frame(i):
    """One whole frame through the oracle (census + WTA + FP64 network); the
    input generation is outside the timed part."""
    import oracle
    from oracle import vae
    from synth import gen_preset
    params, _ = make_params()
    p = gen_preset("pair1242x375", i)
    t0 = time.perf_counter()
    lo, _, _, d = oracle.match(p.left, p.right, F, WIN_W, WIN_H, D)
    vae.forward(params, d, lo, F, H, W)
    return time.perf_counter() - t0


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(budget_s=12.0, max_workers=16):
    """The oracle, as it stands, on whole frames of the workload: single thread
    until the budget is spent, then independent frames in parallel processes
    (one thread each), one per host thread this job may use (at most 16: the
    host's share of a one-GPU job).  Also the oracle's FP64 outputs of the
    256x128 precision workload, returned beside the record."""
    import concurrent.futures
    n, t0 = 0, time.perf_counter()
    while True:
        _oracle_frame(n)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 8:
            break
    single = n / el
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    cores = max(1, min(affinity, max_workers))
    frames = 2 * cores
    env_threads = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        # forked before this process touches the GPU (main() runs this first)
        import multiprocessing
        with concurrent.futures.ProcessPoolExecutor(max_workers=cores,
                                                    mp_context=multiprocessing.get_context("fork")) as ex:
            list(ex.map(_oracle_frame, range(cores)))   # start-up and imports, untimed
            t1 = time.perf_counter()
            list(ex.map(_oracle_frame, range(frames)))
            el_all = time.perf_counter() - t1
    finally:
        if env_threads is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = env_threads
    ref3, t3 = oracle_precision_reference()
    rec = {"value": frames / el_all, "unit": "frames/s", "cores": cores, "kind": "oracle",
           "sample": (f"{frames} whole frames (1242x375, census+WTA+FP64 network) over {cores} processes "
                      f"of one thread, {el_all:.1f} s; single thread: {n} frames in {el:.1f} s"),
           "single_thread_value": single, "host_cpu_count": os.cpu_count(), "host_threads_allowed": affinity,
           "cpu_model": _cpu_model(),
           "oracle_precision_reference_s": round(t3, 2)}
    return rec, ref3


TRAFFIC_JSON = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "traffic_1242x375_b1_f32.json")
LAYER_INDEX = {"E1": 0, "E2": 1, "E3": 2, "HEAD": 3, "G3": 4, "G2": 5, "G1": 6, "G0": 7}


def traffic_lookup(stage, f32_cfgs):
    """HBM bytes per launch of `stage` at the headline shape from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE counts (scaled by a plain copy), if they
    were taken on these very kernel sources and this layer configuration."""
    from paper_2305_11566_amd.profile_traffic import source_hash
    if not os.path.exists(TRAFFIC_JSON):
        return {}
    with open(TRAFFIC_JSON) as f:
        doc = json.load(f)
    if doc.get("source_hash") != source_hash():
        return {"traffic_note": "counters taken on other kernel sources"}
    if stage in LAYER_INDEX:
        e = doc["layers"].get(f"f32|B1|{H}x{W}|{stage}|{f32_cfgs[LAYER_INDEX[stage]]}")
    elif stage == "HEAD+G3":
        e = doc["layers"].get(f"f32|B1|{H}x{W}|{stage}|fused")
    else:
        e = doc.get(stage)
    if not e:
        return {"traffic_note": "no counters for this layer configuration"}
    return {"traffic": e["fetch_bytes"] + e["write_bytes"], "traffic_unit": "B",
            "traffic_source": os.path.relpath(TRAFFIC_JSON, os.path.dirname(os.path.abspath(__file__)))}


def run_sgm(sv, torch, dev, flat, K, Wm):
    """Census + SGM (four axis paths) + single matching phase + median on the
    1242x375 pairs, graph replayed: frames/s of the matching stage at batch 1
    and 64 (also with the ZNCC cost in place of the census cost), of matching
    + FP32 network at batch 1, and the SGM call's HBM rate
    (algorithmic bytes: both census maps read once per path direction, the
    four uint8 path-cost volumes written and read back, the map written)."""
    P1, P2 = 10, 120
    out = {"penalties": [P1, P2], "paths": 4}
    for B in (1, 64):
        left, right, _ = make_inputs(B, dev)
        hs, ws = levels(B)
        h, w = hs[0], ws[0]
        cl = torch.empty((B, h, w), dtype=torch.int64, device=dev)
        cr, low = torch.empty_like(cl), torch.empty((B, h, w), dtype=torch.uint8, device=dev)
        raw, disp = torch.empty_like(low), torch.empty_like(low)
        wsg = torch.empty(sv.lib().sv_sgm_workspace_bytes(B, h, w, D), dtype=torch.uint8, device=dev)
        wsm = torch.empty(sv.lib().sv_smp_workspace_bytes(B, h, w), dtype=torch.uint8, device=dev)
        ref = None
        if B == 1:
            ref = sv.Refiner(C1, C2, C3, LAT, F, "f32")
            ref.pack(torch.from_numpy(flat).to(dev))
            ref.workspace(B, H, W)
            res = torch.empty((B, H, W), dtype=torch.float32, device=dev)

        low_r = torch.empty_like(low)

        def match():
            sv.sv_census_pair(left, right, F, WIN_W, WIN_H, out=(cl, cr, low))
            sv.sv_sgm(cl, cr, D, NBITS, P1, P2, out=raw, workspace=wsg)
            sv.sv_smp_median(raw, D, out=disp, workspace=wsm)

        def match_zncc():  # ZNCC + SGM (the paper's main matcher) on the reduced images
            sv.sv_census(left, F, WIN_W, WIN_H, out=(cl, low))
            sv.sv_census(right, F, WIN_W, WIN_H, out=(cr, low_r))
            sv.sv_zncc_sgm(low, low_r, D, WIN_W, WIN_H, P1, P2, out=raw, workspace=wsg)
            sv.sv_smp_median(raw, D, out=disp, workspace=wsm)

        def full():
            match()
            ref.forward(disp, low, H, W, out=res)

        def graph_ms(fn):
            fn()
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                fn()
            for _ in range(Wm):
                g.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(K):
                g.replay()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) * 1e3 / K

        ms_m = graph_ms(match)
        ms_z = graph_ms(match_zncc)
        rec = {"match_ms": round(ms_m, 4), "match_frames_per_s": round(B * 1e3 / ms_m, 1),
               "zncc_match_ms": round(ms_z, 4), "zncc_match_frames_per_s": round(B * 1e3 / ms_z, 1)}
        if ref is not None:
            ms_f = graph_ms(full)
            rec.update(with_network_f32_ms=round(ms_f, 4),
                       with_network_f32_frames_per_s=round(B * 1e3 / ms_f, 1))
        # the SGM call alone (path sweeps + aggregation / WTA), HIP events on its stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        sv.sv_sgm(cl, cr, D, NBITS, P1, P2, out=raw, workspace=wsg)
        e0.record()
        for _ in range(K):
            sv.sv_sgm(cl, cr, D, NBITS, P1, P2, out=raw, workspace=wsg)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / K
        npx = B * h * w
        nbytes = npx * (4 * 16 + 4 * D + 4 * D + 1)
        rec.update(sgm_us=round(us, 2), sgm_hbm_GBs=round(nbytes / (us * 1e-6) / 1e9, 1),
                   sgm_hbm_frac=round(nbytes / (us * 1e-6) / 1e9 / PEAK["hbm_GBs"], 4))
        out[f"batch_{B}"] = rec
    return out


TABLE1_SEED = 7013


def table1_flops(B):
    """Algorithmic FLOPs of one Table I forward pass on B 1242x375 frames
    (2 per multiply-add of the layer definitions; a deconvolution counts every
    input sample times k^2 taps)."""
    hs, ws = levels(B)
    p1, p2, p3 = hs[0] * ws[0], hs[1] * ws[1], hs[2] * ws[2]
    macs = (p1 * 64 * 25                      # FE_1 and FE_2 (one input channel each)
            + p2 * 16 * 64 * 25 + p2 * 8 * 16 * 25      # EN_1, EN_1_R
            + p3 * 32 * 24 * 25 + p3 * 16 * 32 * 25     # EN_2, EN_2_R
            + p3 * 2 * 48 + p3 * 32                     # mu & sigma, D_1
            + p3 * 16 * 80 * 25 + p3 * 96 * 16 * 25     # D_1_R, D_2 (over its input)
            + p2 * 8 * 40 * 25 + p2 * 48 * 16 * 25      # D_2_R, D (over its input)
            + p1 * 81 * 25)                             # Y (over its input)
    return 2.0 * B * macs


# (out, in, k) per layer of Table I in parameter order
TABLE1_SHAPES = [(32, 1, 5), (32, 1, 5), (16, 64, 5), (8, 16, 5), (32, 24, 5), (16, 32, 5), (2, 48, 1),
                 (32, 1, 1), (16, 80, 5), (16, 96, 5), (8, 40, 5), (16, 48, 5), (1, 81, 5)]


def run_table1(sv, torch, dev, K, Wm, tune=True):
    """Census + WTA + the Table I network on the 1242x375 pairs, graph
    replayed, FP32 and BF16 at batch 1 and 64 (He-init weights, seed 7013),
    and the network alone with its MFMA-peak fraction."""
    from synth import he_init_params
    params = he_init_params(TABLE1_SHAPES, seed=TABLE1_SEED)
    flat = torch.from_numpy(np.concatenate([np.concatenate([w.ravel(), b.ravel()])
                                            for w, b in params]).astype(np.float32)).to(dev)
    out = {"weights": "He-init, seed 7013", "params": int(flat.numel())}

    def graph_ms(fn, k):
        fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        for _ in range(Wm):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            g.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / k

    for B in (1, 64):
        left, right, _ = make_inputs(B, dev)
        hs, ws = levels(B)
        cl = torch.empty((B, hs[0], ws[0]), dtype=torch.int64, device=dev)
        cr = torch.empty_like(cl)
        low = torch.empty((B, hs[0], ws[0]), dtype=torch.uint8, device=dev)
        disp = torch.empty_like(low)
        res = torch.empty((B, H, W), dtype=torch.float32, device=dev)
        k = K if B == 1 else max(5, min(K, 20))
        for dt in ("f32", "bf16"):
            if tune:
                sv.sv_tvae_autotune(dt, F, B, H, W)
            net = sv.TableVAE(F, dt)
            net.pack(flat)
            net.workspace(B, H, W)
            ms_sig = torch.empty(net.latent_shape(B, H, W) + (2,), dtype=torch.float32, device=dev)

            def path():
                sv.sv_census_pair(left, right, F, WIN_W, WIN_H, out=(cl, cr, low))
                sv.sv_cost_wta(cl, cr, D, NBITS, out=disp)
                net.forward(disp, low, H, W, out=res, mu_sigma=ms_sig)

            def net_only():
                net.forward(disp, low, H, W, out=res, mu_sigma=ms_sig)

            ms_p = graph_ms(path, k)
            ms_n = graph_ms(net_only, k)
            tf = table1_flops(B) / (ms_n * 1e-3) / 1e12
            out[f"{dt}_batch_{B}"] = {
                "layer_cfgs": sv.sv_tvae_layer_cfgs(dt, F, B, H, W),
                "path_ms": round(ms_p, 4), "frames_per_s": round(B * 1e3 / ms_p, 1),
                "network_ms": round(ms_n, 4), "network_TFLOPs": round(tf, 3),
                "network_mfma_frac": round(tf / PEAK["mfma_TFLOPs"][dt], 4)}
            del net
    out["gflop_per_frame"] = round(table1_flops(1) / 1e9, 4)
    # training: 512x256 crops, batch 16, f = 2, 5x5 census, D = 16, BF16,
    # loss of Eqs. (9)-(11), Adam; steps/s and the loss at the start and end
    from paper_2305_11566_amd.train import TableTrainer, make_pool, batch_indices
    tr = TableTrainer(flat.cpu().numpy(), factor=2, dtype="bf16")
    pl, pr, pg, pn, po = make_pool(64, 256, 512, seed0=5000, masks=True)
    losses = []

    def one():
        idx = batch_indices(tr.step, 16, 64).to(dev)
        return tr.train_step(pl[idx], pr[idx], pg[idx], pn[idx], po[idx])
    for _ in range(5):
        losses.append(float(one()[0]))
    torch.cuda.synchronize()
    nsteps = 100
    t0 = time.perf_counter()
    for _ in range(nsteps):
        l = one()
    torch.cuda.synchronize()
    sps = nsteps / (time.perf_counter() - t0)
    out["train_512x256_b16_bf16"] = {"steps_per_s": round(sps, 2), "steps": 5 + nsteps,
                                     "loss_first": losses[0], "loss_last": float(l[0])}
    return out
def run_int8(sv, torch, dev, flat, K, Wm, tune=True):
    """Census + WTA + the INT8 network (per-channel weight scales, dynamic
    per-tensor activation scales) on the 1242x375 pairs, graph replayed at
    batch 1 and 64, and its end-point error against the FP32 network on the
    same frames (He-init weights: a stress figure, not a trained accuracy)."""
    out = {"weights": "He-init, seed 7002 (the headline network)"}
    for B in (1, 64):
        left, right, _ = make_inputs(B, dev)
        k = K if B == 1 else max(5, min(K, 20))
        res = {}
        for dt in ("i8", "f32"):
            if tune:
                sv.sv_autotune(C1, C2, C3, LAT, F, dt, B, H, W, D, WIN_W, WIN_H)
            p = Path(B, dt, flat, left, right)
            p.capture()
            ms = p.timed(k, Wm)
            res[dt] = (ms, p.out.clone())
            del p
        d = (res["i8"][1] - res["f32"][1]).abs()
        out[f"batch_{B}"] = {"ms_per_step": round(res["i8"][0], 4),
                             "frames_per_s": round(B * 1e3 / res["i8"][0], 1),
                             "f32_frames_per_s": round(B * 1e3 / res["f32"][0], 1),
                             "i8_vs_f32_mean_px": float(d.mean()), "i8_vs_f32_max_px": float(d.max())}
    return out


def run_extras(sv, torch, dev, flat, K, Wm):
    """Uneven batch (64 pairs, one graph) vs the per-pair loop."""
    from synth import gen_preset
    out = {}
    # -- 64 uneven pairs, BF16 network ---------------------------------------------------
    ps = [gen_preset("uneven64", i) for i in range(64)]
    pairs = [(torch.from_numpy(p.left).to(dev), torch.from_numpy(p.right).to(dev), p.D) for p in ps]
    maxH, maxW, maxD = max(p.left.shape[0] for p in ps), max(p.left.shape[1] for p in ps), max(p.D for p in ps)
    sv.sv_autotune(C1, C2, C3, LAT, F, "bf16", 8, maxH, maxW, maxD, WIN_W, WIN_H)
    ref = sv.Refiner(C1, C2, C3, LAT, F, "bf16")
    ref.pack(torch.from_numpy(flat).to(dev))
    plan = sv.BatchPlan(C1, C2, C3, LAT, F, "bf16", 64, maxH, maxW, maxD, WIN_W, WIN_H)
    outs = [torch.empty(l.shape, dtype=torch.float32, device=dev) for l, _, _ in pairs]
    for _ in range(3):
        plan.run(pairs, ref.packed, outs=outs)
    torch.cuda.synchronize()
    kb = max(5, min(K, 20))
    t0 = time.perf_counter()
    for _ in range(kb):
        plan.run(pairs, ref.packed, outs=outs)
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t0) * 1e3 / kb
    px = sum(p.left.size for p in ps)

    def one_by_one():
        for (l, r, Dp), o in zip(pairs, outs):
            cl, cr, low = sv.sv_census_pair(l[None], r[None], F, WIN_W, WIN_H)
            disp = sv.sv_cost_wta(cl, cr, Dp, NBITS)
            ref.forward(disp, low, l.shape[0], l.shape[1], out=o[None])
    one_by_one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        one_by_one()
    torch.cuda.synchronize()
    ms_loop = (time.perf_counter() - t0) * 1e3 / 3
    out["uneven_batch_64"] = {
        "dtype": "bf16", "pairs": 64, "megapixels_per_view": round(px / 1e6, 3),
        "graph_ms": round(ms_batch, 4), "graph_frames_per_s": round(64e3 / ms_batch, 1),
        "loop_ms": round(ms_loop, 4), "loop_frames_per_s": round(64e3 / ms_loop, 1),
        "speedup": round(ms_loop / ms_batch, 2),
        # compulsory HBM bytes: both views read, the refined map written
        "hbm_GBs_compulsory": round(6.0 * px / (ms_batch * 1e-3) / 1e9, 2),
    }
    plan.close()
    del plan, outs

    # -- the paper's system (ZNCC + SGM + SMP + median, Table I network, BF16)
    # on the same 64 uneven pairs: one graph of the per-pair launch sequence
    from synth import he_init_params
    tparams = he_init_params(TABLE1_SHAPES, seed=TABLE1_SEED)
    tflat = torch.from_numpy(np.concatenate([np.concatenate([w.ravel(), b.ravel()])
                                             for w, b in tparams]).astype(np.float32)).to(dev)
    net = sv.TableVAE(F, "bf16")
    net.pack(tflat)
    pb = sv.PaperBatch("zncc", F, WIN_W, WIN_H, 10, 120, "bf16", True, maxH, maxW, maxD)
    pouts = [torch.empty(l.shape, dtype=torch.float32, device=dev) for l, _, _ in pairs]
    pb.run(pairs, net.packed, outs=pouts)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pb.run(pairs, net.packed, outs=pouts)
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    ms_g = (time.perf_counter() - t0) * 1e3 / 3
    t0 = time.perf_counter()
    for _ in range(3):
        pb.run(pairs, net.packed, outs=pouts)
    torch.cuda.synchronize()
    ms_e = (time.perf_counter() - t0) * 1e3 / 3
    out["paper_system_uneven_64"] = {
        "pipeline": "reduce + ZNCC + SGM (P1 10, P2 120) + single matching phase + 3x3 median + Table I network "
                    "(BF16, He-init seed 7013)",
        "pairs": 64, "graph_ms": round(ms_g, 3), "graph_frames_per_s": round(64e3 / ms_g, 1),
        "eager_ms": round(ms_e, 3), "eager_frames_per_s": round(64e3 / ms_e, 1)}
    del g, pb, net

    return out


# ---- the 256x128 precision workload and the 512x256 training workload -------------------
P_C, P_L, P_F, P_WIN, P_D = (16, 32, 64), 64, 2, (5, 5), 16
PRECISION_SEED = 7003


def precision_params():
    """He-init weights of the 256x128 network (seed 7003) with the final
    layer's weights and bias scaled by 0.01: a refinement term of a few px, as
    trained weights give, where plain He-init's is of order 100 px."""
    from synth import he_init_params
    from paper_2305_11566_amd.train import layer_shapes
    params = he_init_params(layer_shapes(*P_C, P_L), seed=PRECISION_SEED, bias_scale=0.1)
    wF, bF = params[8]
    params[8] = ((wF * np.float32(0.01)).astype(np.float32), (bF * np.float32(0.01)).astype(np.float32))
    flat = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)
    return params, flat


def precision_pairs():
    from synth import gen_preset
    return [gen_preset("batch8_256x128", i) for i in range(8)]   # seeds 3000-3007


def oracle_precision_reference():
    """The oracle's FP64 refined maps of the 8-pair 256x128 workload with the
    precision weights (its own census + WTA feeding its own network): the
    reference the GPU precisions are measured against."""
    import oracle
    from oracle import vae
    params, _ = precision_params()
    ps = precision_pairs()
    t0 = time.perf_counter()
    m = [oracle.match(p.left, p.right, P_F, P_WIN[0], P_WIN[1], P_D) for p in ps]
    lo = np.concatenate([r[0] for r in m])
    d = np.concatenate([r[3] for r in m])
    outs = vae.forward(params, d, lo, P_F, 128, 256)["out"]
    return outs, time.perf_counter() - t0


def _epe(a, b):
    e = (a.double() - b.double()).abs()
    return {"mean_px": float(f"{float(e.mean()):.4g}"), "max_px": float(f"{float(e.max()):.4g}")}


def run_config5(sv, torch, dev, steps=2000):
    """Training on the GPU: 512x256 crops of 128 generated pairs (seeds
    5000-5127), batch 16, BF16 compute with FP32 master weights and Adam,
    smooth-L1 + 1e-3 KL; steps/s, then the end-point error on 16 disjoint
    validation pairs (seeds 5500-5515) before and after training."""
    from paper_2305_11566_amd.train import Trainer, layer_shapes, make_pool, batch_indices
    from synth import he_init_params
    p0 = he_init_params(layer_shapes(*P_C, P_L), seed=7005)
    f0 = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in p0])
    tr = Trainer(f0, C=P_C, latent=P_L, dtype="bf16")
    pl, pr, pg = make_pool(128, 256, 512, seed0=5000)
    vl, vr, vg = make_pool(16, 256, 512, seed0=5500)

    def val(w):
        disp, low = tr.coarse(vl, vr)
        res = {}
        for dt in ("f32", "bf16", "i8"):
            r = sv.Refiner(*P_C, P_L, P_F, dt)
            r.pack(w)
            o, _ = r.forward(disp, low, 256, 512)
            res[dt] = _epe(o, vg)
        lin = torch.nn.functional.interpolate(disp[:, None].float() * P_F, size=(256, 512), mode="bilinear",
                                              align_corners=False)[:, 0]
        res["linear_upscaling"] = _epe(lin, vg)
        return res
    before = val(tr.w)
    for _ in range(5):
        idx = batch_indices(tr.step, 16, 128).to(dev)
        tr.train_step(pl[idx], pr[idx], pg[idx])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n0 = tr.step
    while tr.step < steps:
        idx = batch_indices(tr.step, 16, 128).to(dev)
        loss = tr.train_step(pl[idx], pr[idx], pg[idx])
    torch.cuda.synchronize()
    sps = (tr.step - n0) / (time.perf_counter() - t0)
    rec = {"steps_per_s": round(sps, 2), "ms_per_step": round(1e3 / sps, 4), "steps": steps,
           "loss_last": [round(float(x), 5) for x in loss.cpu()],
           "validation": {"pairs": "16 x 512x256, seeds 5500-5515 (training pool: seeds 5000-5127)",
                          "vs_gt_before_training": before, "vs_gt_after_training": val(tr.w)}}
    return rec, tr.w


def run_config3(sv, torch, dev, K, Wm, trained_w, oracle_ref):
    """The 8-pair 256x128 workload (seeds 3000-3007): census + WTA + the
    (16, 32, 64), latent 64 network per compute dtype.  End-point error of
    each dtype against FP32, against the FP64 oracle (precision weights; the
    oracle runs in the CPU leg) and against ground truth, on the precision
    weights and on the trained weights; frames/s per dtype, graph replayed."""
    ps = precision_pairs()
    B, H3, W3 = 8, 128, 256
    left = torch.from_numpy(np.stack([p.left for p in ps])).to(dev)
    right = torch.from_numpy(np.stack([p.right for p in ps])).to(dev)
    gt = torch.from_numpy(np.stack([p.gt for p in ps])).to(dev)
    nb = P_WIN[0] * P_WIN[1] - 1
    cl, cr, low = sv.sv_census_pair(left, right, P_F, *P_WIN)
    disp = sv.sv_cost_wta(cl, cr, P_D, nb)
    _, pflat = precision_params()
    dts = ("f32", "bf16", "f16", "i8")
    out = {"shape": "8 x 256x128, f = 2, 5x5 census, D = 16, network (16, 32, 64), latent 64",
           "reference": "oracle FP64 (its own census + WTA and network), computed in the CPU leg"}
    for wname, w in (("precision_weights", torch.from_numpy(pflat).to(dev)), ("trained_weights", trained_w)):
        if w is None:
            continue
        res = {}
        for dt in dts:
            r = sv.Refiner(*P_C, P_L, P_F, dt)
            r.pack(w)
            res[dt], _ = r.forward(disp, low, H3, W3)
        rec = {}
        for dt in dts:
            e = {"vs_gt": _epe(res[dt], gt)}
            if dt != "f32":
                e["vs_f32"] = _epe(res[dt], res["f32"])
            if wname == "precision_weights" and oracle_ref is not None:
                e["vs_oracle_f64"] = _epe(res[dt], torch.from_numpy(oracle_ref).to(dev))
            rec[dt] = e
        out[wname] = rec
    out["precision_weights"]["weights"] = "He-init seed 7003, final layer x 0.01"
    if "trained_weights" in out:
        out["trained_weights"]["weights"] = "after the 2000 training steps (512x256, batch 16, BF16)"
    # frames/s per dtype: the whole step (census + WTA + network) replayed from a graph
    cl_, cr_, low_, disp_ = (torch.empty_like(cl), torch.empty_like(cr), torch.empty_like(low),
                             torch.empty_like(disp))
    o_ = torch.empty((B, H3, W3), dtype=torch.float32, device=dev)
    fps = {}
    for dt in dts:
        r = sv.Refiner(*P_C, P_L, P_F, dt)
        r.pack(torch.from_numpy(pflat).to(dev))
        r.workspace(B, H3, W3)
        ls = r.latent_shape(B, H3, W3)
        ml = torch.empty(ls[:3] + (2 * ls[3],), dtype=torch.float32, device=dev)

        def step():
            sv.sv_census_pair(left, right, P_F, *P_WIN, out=(cl_, cr_, low_))
            sv.sv_cost_wta(cl_, cr_, P_D, nb, out=disp_)
            r.forward(disp_, low_, H3, W3, out=o_, mu_logvar=ml)
        step()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        for _ in range(Wm):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            g.replay()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / K
        fps[dt] = {"ms_per_step": round(ms, 4), "frames_per_s": round(B * 1e3 / ms, 1)}
        del g, r
    out["throughput_batch8"] = fps
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--dtype", choices=("f32", "bf16", "f16"), default="f32",
                    help="network compute dtype of the headline step (the metric is quoted on f32)")
    ap.add_argument("--big-batch", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the uneven batch, precision and training measurements")
    ap.add_argument("--section", choices=("sgm", "table1", "int8"), default=None,
                    help="run only this extras section (for profiling) and print it as the JSON line")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} (WORLD_SIZE {world}) is not "
              "supported; the path runs on a single MI355X and has no multi-GPU mode.",
              file=sys.stderr)
        sys.exit(2)

    # the CPU oracle first, while this process has not touched the GPU (its
    # worker processes are forked from here)
    cpu, ref3 = (None, None) if (args.no_cpu_baseline or args.section) else cpu_baseline()

    import torch
    import paper_2305_11566_amd as sv
    dev = torch.device("cuda:0")
    K, Wm = args.steps, args.warmup
    _, flat = make_params()
    if args.section:
        fn = {"sgm": lambda: run_sgm(sv, torch, dev, flat, K, Wm),
              "table1": lambda: run_table1(sv, torch, dev, K, Wm, not args.no_autotune),
              "int8": lambda: run_int8(sv, torch, dev, flat, K, Wm, not args.no_autotune)}[args.section]
        print(json.dumps({"section": args.section, "steps": K, "warmup": Wm, "result": fn()}))
        return
    left, right, gt = make_inputs(args.batch, dev)

    # ---- tile shapes: the library's autotuner for this shape ---------------------------
    if not args.no_autotune:
        for dt in ("f32", "bf16"):
            sv.sv_autotune(C1, C2, C3, LAT, F, dt, args.batch, H, W, D, WIN_W, WIN_H)
    tiles = {"cost_wta": sv.sv_tile_config(1),
             "f32": sv.sv_layer_cfgs(C1, C2, C3, LAT, F, "f32", args.batch, H, W),
             "bf16": sv.sv_layer_cfgs(C1, C2, C3, LAT, F, "bf16", args.batch, H, W)}

    # ---- headline: FP32 network (or --dtype), graph replay --------------------------------
    hdt = args.dtype
    p32 = Path(args.batch, hdt, flat, left, right)
    for _ in range(Wm):
        p32.step()
    torch.cuda.synchronize()
    eager_ms = p32.timed(K, 0, graph=False)
    # profiled eager pass: HIP events on the launch stream around PROF_REPEAT
    # back-to-back launches of every kernel, K times; a kernel's average
    # duration is the summed event time over its launches
    sv.sv_profile_enable(K)
    sv.sv_profile_repeat(PROF_REPEAT)
    p32.timed(K, 0, graph=False)
    prof = merge_latent(sv.sv_profile_read())
    sv.sv_profile_repeat(1)
    sv.sv_profile_enable(0)
    p32.capture()
    ms = p32.timed(K, Wm, graph=True)
    fps = args.batch * 1e3 / ms

    kernels = {}
    for stage, (tot, cnt) in prof.items():
        if cnt == 0:
            continue
        avg_ms = tot / cnt
        bound, amount, unit = stage_work(stage, args.batch, hdt)
        rec = {"avg_us": round(avg_ms * 1e3, 3), "launches": cnt}
        if bound:
            rate = amount / (avg_ms * 1e-3)
            if bound == "hbm":
                peak, runit, ach = PEAK["hbm_GBs"], "GB/s", rate
            elif bound == "mfma":
                peak, runit, ach = PEAK["mfma_TFLOPs"][hdt], "TFLOP/s", rate
            else:
                peak, runit, ach = PEAK["alu_Tops"], "Tops/s", rate
            rec.update(bound=bound, achieved=round(ach, 3), unit=runit, frac=round(ach / peak, 5))
        kernels[stage] = rec
    dom = max(kernels, key=lambda s: kernels[s]["avg_us"])
    d = kernels[dom]
    peak = {"GB/s": PEAK["hbm_GBs"], "TFLOP/s": PEAK["mfma_TFLOPs"][hdt],
            "Tops/s": PEAK["alu_Tops"]}.get(d.get("unit"), None)
    roofline = {"kernel": dom, "bound": d.get("bound"), "achieved": d.get("achieved"), "peak": peak,
                "unit": d.get("unit"), "frac": d.get("frac"), "traffic": None,
                "avg_us": d["avg_us"],
                "timing": f"HIP events on the launch stream around {PROF_REPEAT} back-to-back launches, "
                          f"{K} times ({d['launches']} launches)"}
    if args.batch == 1 and hdt == "f32":
        roofline.update(traffic_lookup(dom, tiles["f32"]))

    # ---- variants and EPE ---------------------------------------------------------------
    variants = []
    epe = None
    if not args.no_variants:
        pbf = Path(args.batch, "bf16", flat, left, right)
        pbf.capture()
        ms_bf = pbf.timed(K, Wm)
        variants.append({"dtype": "bf16", "batch": args.batch, "ms_per_step": round(ms_bf, 4),
                         "frames_per_s": round(args.batch * 1e3 / ms_bf, 1)})
        o32 = p32.out.double().cpu().numpy()
        obf = pbf.out.double().cpu().numpy()
        # He-init weights refine nothing: this compares the two precisions on the
        # same untrained network at full size; end-point errors against ground
        # truth with trained weights are in extras.precision_8x256x128
        epe = {"weights": "He-init (untrained), 1242x375",
               "bf16_vs_f32_mean_px": float(np.mean(np.abs(obf - o32))),
               "bf16_vs_f32_max_px": float(np.max(np.abs(obf - o32))),
               "mean_abs_f32_output_px": float(np.mean(np.abs(o32)))}
        del pbf
        bb = args.big_batch
        if bb and bb > 1:
            lb, rb, _ = make_inputs(bb, dev)
            for dt in ("f32", "bf16"):
                if not args.no_autotune:
                    sv.sv_autotune(C1, C2, C3, LAT, F, dt, bb, H, W, D, WIN_W, WIN_H)
                pb = Path(bb, dt, flat, lb, rb)
                kb = max(5, min(K, 20))
                # per-layer times from a profiled eager pass (launch overhead is
                # small next to batch-64 kernels): MFMA utilisation of the layers
                # that are dense contractions (E2, E3, G2, G1, G0)
                pb.timed(2, 0, graph=False)
                sv.sv_profile_enable(kb)
                pb.timed(kb, 0, graph=False)
                profb = merge_latent(sv.sv_profile_read())
                sv.sv_profile_enable(0)
                pb.capture()
                msb = pb.timed(kb, 3)
                rec = {"dtype": dt, "batch": bb, "ms_per_step": round(msb, 4),
                       "frames_per_s": round(bb * 1e3 / msb, 1)}
                flop, sec = 0.0, 0.0
                layers = {}
                for st_ in ("census", "cost_wta", "E1", "E2", "E3", "HEAD", "G3", "HEAD+G3", "G2", "G1", "G0",
                            "final_gather", "split_sum"):
                    tot, cnt = profb.get(st_, (0.0, 0))
                    if cnt == 0:
                        continue
                    bound, amount, _ = stage_work(st_, bb, dt)
                    us = tot / cnt * 1e3
                    if bound is None:  # the split sums of several layers
                        layers[st_] = {"avg_us": round(us, 2), "launches": cnt}
                        continue
                    rate = amount / (us * 1e-6)
                    peak = {"mfma": PEAK["mfma_TFLOPs"][dt], "hbm": PEAK["hbm_GBs"],
                            "alu": PEAK["alu_Tops"]}[bound]
                    layers[st_] = {"avg_us": round(us, 2), "bound": bound, "frac": round(rate / peak, 4)}
                    if st_ in ("E2", "E3", "G2", "G1", "G0"):
                        flop += amount
                        sec += us * 1e-6
                rec["layers"] = layers
                rec["mfma_frac_dense_layers"] = round(flop / sec / PEAK["mfma_TFLOPs"][dt], 4) if sec else None
                variants.append(rec)
                del pb
            torch.cuda.synchronize()

    extras = {} if args.no_extras else run_extras(sv, torch, dev, flat, K, Wm)
    if not args.no_extras:
        extras["train_512x256_b16"], trained = run_config5(sv, torch, dev)
        extras["precision_8x256x128"] = run_config3(sv, torch, dev, K, Wm, trained, ref3)
        extras["census_sgm_1242x375"] = run_sgm(sv, torch, dev, flat, K, Wm)
        extras["table1_network_1242x375"] = run_table1(sv, torch, dev, K, Wm, not args.no_autotune)
        extras["int8_network_1242x375"] = run_int8(sv, torch, dev, flat, K, Wm, not args.no_autotune)


    rec = {
        "metric": "frames/s at 1242x375 D=192 (census+WTA+VAE), BF16 vs FP32 at EPE; % roofline",
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": hdt,
        "data": "synthetic (seeded planar-cell scenes, KITTI-sized; random He-init weights)",
        "config": {"workload": f"1242x375 pair, batch {args.batch}: 9x7 census at 1/4 res (311x94), D=48 "
                               f"(192 full-res), WTA, VAE 2-32-64-128 latent 128 {hdt.upper()}, hipGraph replay",
                   "batch": args.batch, "H": H, "W": W, "factor": F, "D_low": D},
        "eager_ms_per_step": round(eager_ms, 5),
        "roofline": roofline,
        "kernels": kernels,
        "variants": variants,
        "epe": epe,
        "tiles": tiles,
        "extras": extras,
        "cpu_baseline": cpu,
        "context": {"paper_ms_per_frame_jetson_agx": 29.88,
                    "note": "paper: ZNCC+SGM+StereoVAE on Jetson AGX Xavier (Table II), not this pipeline"},
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
