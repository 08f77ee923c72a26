"""HBM traffic of the headline path's kernels from rocprofv3 counters.

Two modes:

``python -m paper_2305_11566_amd.profile_traffic run``
    One 1242x375 pair (the benchmark's inputs and weights), matched once, then
    one FP32 forward pass of the network per layer configuration with every
    layer set to that configuration and each layer its own launch (a tile
    shape that does not fit a layer runs as the fallback and is recorded under
    the fallback's name), one pass as inference runs it (the head and G3 as one
    kernel, recorded as HEAD+G3), then a plain 64 MiB device copy.  Meant to run under
    ``rocprofv3 --pmc FETCH_SIZE`` and, separately, ``--pmc WRITE_SIZE``.

``python -m paper_2305_11566_amd.profile_traffic summarize FETCH_DIR WRITE_DIR NAMES_JSON OUT_JSON``
    Reads the two counter collections, scales each counter by what it reads
    for the copy (bytes moved / counter), and writes per-launch HBM bytes for
    every (layer, configuration) plus census, cost + WTA and the final layer,
    keyed by a hash of the HIP sources so that a reader can tell whether the
    kernels have changed since.

``python -m paper_2305_11566_amd.profile_traffic trace TRACE_DIR``
    Per-launch durations from a ``rocprofv3 --kernel-trace`` collection,
    grouped by kernel and launch shape (grid and workgroup), so that layers
    which share a kernel template are told apart: a markdown table of calls
    and average / min / max duration in order of first launch.

``python -m paper_2305_11566_amd.profile_traffic busy PMC_DIR N``
    MFMA busy fraction of the last N dispatches of a run profiled with
    ``rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES ... GRBM_GUI_ACTIVE``.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

H, W, F, WIN_W, WIN_H, D = 375, 1242, 4, 9, 7, 48
C1, C2, C3, LAT = 32, 64, 128, 128
LAYERS = ("E1", "E2", "E3", "HEAD", "G3", "G2", "G1", "G0")
COPY_BYTES = 64 << 20


def source_hash() -> str:
    """sha256 over the HIP sources and headers of libsv.so (and include/sv.h)."""
    here = os.path.dirname(os.path.abspath(__file__))
    files = sorted(glob.glob(os.path.join(here, "csrc", "*.hip")) +
                   glob.glob(os.path.join(here, "csrc", "*.h")) +
                   [os.path.join(here, "..", "include", "sv.h")])
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def run() -> None:
    import numpy as np
    import torch

    import paper_2305_11566_amd as sv
    from synth import gen_preset, he_init_params

    dev = torch.device("cuda:0")
    p = gen_preset("pair1242x375", 0)
    left = torch.from_numpy(p.left[None]).to(dev)
    right = torch.from_numpy(p.right[None]).to(dev)
    shapes = [(C1, 2, 3), (C2, C1, 3), (C3, C2, 3), (2 * LAT, C3, 1), (C3, LAT, 1),
              (C2, C3 + C2, 3), (C1, C2 + C1, 3), (C1, C1 + 2, 3), (1, C1 + 2, 3)]
    params = he_init_params(shapes, seed=7002)
    flat = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)
    cl, cr, low = sv.sv_census_pair(left, right, F, WIN_W, WIN_H)
    disp = sv.sv_cost_wta(cl, cr, D, WIN_W * WIN_H - 1)
    ref = sv.Refiner(C1, C2, C3, LAT, F, "f32")
    ref.pack(torch.from_numpy(flat).to(dev))
    ref.workspace(1, H, W)
    out = torch.empty((1, H, W), dtype=torch.float32, device=dev)
    names = []
    try:
        # every layer as its own launch, so that each configuration of the head
        # and of G3 is counted too
        sv.sv_set_latent_fusion(False)
        for c in range(sv.sv_num_layer_cfgs()):
            for layer in range(9):
                sv.sv_set_layer_cfg(layer, c)
            names.append(sv.sv_layer_cfgs(C1, C2, C3, LAT, F, "f32", 1, H, W))
            ref.forward(disp, low, H, W, out=out)
            torch.cuda.synchronize()
    finally:
        for layer in range(9):
            sv.sv_set_layer_cfg(layer, -1)
        sv.sv_set_latent_fusion(True)
    # then one pass as inference runs it: head and G3 in one kernel
    names.append(sv.sv_layer_cfgs(C1, C2, C3, LAT, F, "f32", 1, H, W))
    ref.forward(disp, low, H, W, out=out)
    torch.cuda.synchronize()
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    with open(os.environ.get("SV_TRAFFIC_NAMES", "traffic_names.json"), "w") as f:
        json.dump(names, f)
    print("done", flush=True)


def _dispatches(d: str):
    """[(kernel name, counter value)] in dispatch order from a rocprofv3 counter collection."""
    rows = []
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            rows += list(csv.DictReader(f))
    acc = {}
    for r in rows:
        k = int(r["Dispatch_Id"])
        name, v = r["Kernel_Name"], float(r["Counter_Value"])
        acc[k] = (name, acc.get(k, (name, 0.0))[1] + v)
    return [acc[k] for k in sorted(acc)]


def summarize(fetch_dir: str, write_dir: str, names_json: str, out_json: str) -> None:
    fe, wr = _dispatches(fetch_dir), _dispatches(write_dir)
    assert [n for n, _ in fe] == [n for n, _ in wr], "the two runs dispatched different kernels"
    with open(names_json) as f:
        cfg_names = json.load(f)
    copy = [i for i, (n, _) in enumerate(fe) if "copyBuffer" in n or "elementwise" in n]
    ci = copy[-1]
    # counters are in KiB; the copy reads and writes COPY_BYTES
    s_fetch = COPY_BYTES / (fe[ci][1] * 1024.0)
    s_write = COPY_BYTES / (wr[ci][1] * 1024.0)
    seq = [(n, fe[i][1] * 1024.0 * s_fetch, wr[i][1] * 1024.0 * s_write) for i, (n, _) in enumerate(fe)]
    entries = {}
    census = cost = None
    forwards, cur = [], []
    for n, fb, wb in seq:
        if "k_reduce_census" in n:
            census = {"fetch_bytes": fb, "write_bytes": wb}
        elif "k_cost_wta" in n:
            cost = {"fetch_bytes": fb, "write_bytes": wb}
        elif "k_conv_split_reduce" in n:
            cur[-1][1] += fb
            cur[-1][2] += wb
        elif "k_conv<" in n or "k_latent<" in n or "k_enc1<" in n:
            cur.append([n, fb, wb])
        elif "k_final" in n:
            forwards.append((cur, (fb, wb)))
            cur = []
    assert len(forwards) == len(cfg_names), (len(forwards), len(cfg_names))
    final = None
    for (convs, fin), cfgs in zip(forwards, cfg_names):
        if any("k_latent<" in c[0] for c in convs):  # head and G3 as one kernel
            layers = LAYERS[:3] + ("HEAD+G3",) + LAYERS[5:]
            cfgs = list(cfgs[:3]) + ["fused"] + list(cfgs[5:8])
        else:
            layers = LAYERS
        assert len(convs) == len(layers)
        for layer, (n, fb, wb), cfg in zip(layers, convs, cfgs):
            entries[f"f32|B1|{H}x{W}|{layer}|{cfg}"] = {"fetch_bytes": round(fb), "write_bytes": round(wb),
                                                        "kernel": n.split("(")[0]}
        final = {"fetch_bytes": round(fin[0]), "write_bytes": round(fin[1])}
    doc = {"source_hash": source_hash(), "counter_scale": {"FETCH_SIZE": s_fetch, "WRITE_SIZE": s_write},
           "census": census, "cost_wta": cost, "final_gather": final, "layers": entries}
    with open(out_json, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    print(f"wrote {out_json}: {len(entries)} layer entries, scales {s_fetch:.3f} / {s_write:.3f}")


def _short(name: str) -> str:
    return name.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]


def trace(trace_dir: str) -> None:
    rows = []
    for path in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
        with open(path) as f:
            rows += list(csv.DictReader(f))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    groups = {}
    for r in rows:
        if "Grid_Size_X" in r:
            grid = f"{r['Grid_Size_X']}x{r['Grid_Size_Y']}x{r['Grid_Size_Z']}"
            wg = f"{r['Workgroup_Size_X']}x{r['Workgroup_Size_Y']}x{r['Workgroup_Size_Z']}"
        else:
            grid, wg = r.get("Grid_Size", "?"), r.get("Workgroup_Size", "?")
        key = (_short(r["Kernel_Name"]), grid, wg)
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        groups.setdefault(key, []).append(us)
    print("| kernel | grid (threads) | workgroup | calls | avg us | min us | max us |")
    print("|---|---|---|---|---|---|---|")
    for (name, grid, wg), v in groups.items():
        print(f"| `{name}` | {grid} | {wg} | {len(v)} | {sum(v) / len(v):.2f} | {min(v):.2f} | {max(v):.2f} |")


def busy(pmc_dir: str, nkernels: int) -> None:
    """MFMA busy fraction per kernel of the last step of a profiled run.  Per
    dispatch, GRBM_GUI_ACTIVE comes summed over the eight XCDs (each counts the
    kernel's duration in cycles) and SQ_VALU_MFMA_BUSY_CYCLES over all 1024
    SIMDs, so the fraction is busy / (GRBM_GUI_ACTIVE / 8 x 1024).  Prints a
    markdown table of the last `nkernels` dispatches."""
    rows = []
    for path in glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            rows += list(csv.DictReader(f))
    acc, names = {}, {}
    for r in rows:
        d = int(r["Dispatch_Id"])
        acc.setdefault(d, {})
        acc[d][r["Counter_Name"]] = acc[d].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        names[d] = r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]
    ds = sorted(acc)[-nkernels:]
    print("| kernel | duration us (GRBM / 8 at 2.4 GHz) | MFMA busy cycles | MFMA busy fraction | MFMA instructions / wave | VALU instructions / wave |")
    print("|---|---|---|---|---|---|")
    for d in ds:
        c = acc[d]
        act = c.get("GRBM_GUI_ACTIVE", 0.0)
        mb = c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        w = max(c.get("SQ_WAVES", 1.0), 1.0)
        frac = mb / (act / 8.0 * 1024.0) if act else 0.0
        print(f"| `{names[d]}` | {act / 8.0 / 2400.0:.1f} | {mb:.0f} | {frac:.3f} | {c.get('SQ_INSTS_MFMA', 0) / w:.0f} | "
              f"{c.get('SQ_INSTS_VALU', 0) / w:.0f} |")


if __name__ == "__main__":
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if here not in sys.path:
        sys.path.insert(0, here)
    if sys.argv[1] == "run":
        run()
    elif sys.argv[1] == "summarize":
        summarize(*sys.argv[2:6])
    elif sys.argv[1] == "trace":
        trace(sys.argv[2])
    elif sys.argv[1] == "busy":
        busy(sys.argv[2], int(sys.argv[3]))
    else:
        raise SystemExit("usage: profile_traffic run | summarize FETCH_DIR WRITE_DIR NAMES_JSON OUT_JSON | "
                         "trace TRACE_DIR | busy PMC_DIR N")
