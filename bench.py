"""Benchmark: consistent message-passing fwd+bwd edges/s on one MI355X.

Default workload (C4): 32^3 spectral elements of order 7 (225^3 =
11,390,625 GLL nodes, 68,040,000 directed edges), split into 64 uneven
sub-graphs by a seeded recursive coordinate bisection (1x-3x element
counts), each with its halo rows (11,852,352 rows, 69,866,496 sub-graph
edges in one set of buffers, one launch per kernel for all sub-graphs);
an encode-process-decode model with 4 consistent NMP layers, hidden width
64, LayerNorm, and the consistent MSE (Eq. 6) against the field shifted by
one node.  Seeded synthetic Taylor-Green-like input, Xavier-uniform
weights.  `--workload C1` (16^3 elements P=5, 16 z-slabs), `C3` (24^3
elements, H=128, one graph) and `T2R8` (the periodic 16 x 16 x 128-element
p=5 box in the 8 slabs of Table II's R=8 row) measure the other fwd+bwd
workloads the same way.  `--model table1-small|table1-large` runs a
workload with one of the paper's own models (Table I: extra hidden layers
in every MLP) on the FP32 deep-MLP kernels instead.

One step = the whole model forward, loss and backward (every layer's edge
update, aggregation, halo sum, node update and their adjoints, plus the
encoders, decoder and loss).  value = global directed edges x layers / step
time, for the BF16-GEMM path; the FP32 path is measured beside it.  The
message-passing layers alone (forward and adjoint of the 4 layers, no
encoders, decoder or loss) are timed in a separate loop and reported as
`mp_layers`.  The edge-kernel schedule is autotuned first, and per-kernel
times come from a separate profiled pass; neither is inside a timed region.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--workload C4]

Prints one JSON line.
"""

import argparse
import json
import sys
import time

import numpy as np

WORKLOADS = {
    "C1": {"desc": "C1 mesh fwd+bwd: 16^3 elements P=5 (531441 nodes, 3149280 edges), "
                   "R=16 z-slabs with halos, 4 layers, H=64, LayerNorm, consistent MSE", "R": None},
    "C3": {"desc": "C3 mesh fwd+bwd: 24^3 elements P=5 (1771561 nodes, 10541520 edges), "
                   "one graph, 4 layers, H=128, LayerNorm, MSE", "R": 1},
    "C4": {"desc": "C4 mesh fwd+bwd: 32^3 elements P=7 (11390625 nodes, 68040000 edges), "
                   "64 uneven sub-graphs (seeded bisection) with halos, 4 layers, H=64, LayerNorm, "
                   "consistent MSE", "R": None},
    "T2R8": {"desc": "Table II R=8 partition fwd+bwd: 16x16x128 elements P=5, periodic in x, y, z "
                     "(4096000 nodes, 24576000 edges), 8 z-slabs of 518400 rows with halos, 4 layers, "
                     "H=64, LayerNorm, consistent MSE", "R": None},
}


# The paper's own models (Table I): four layers, LayerNorm, extra hidden
# layers in every MLP; they run on the FP32 deep-MLP kernels.
TABLE1 = {"table1-small": dict(H=8, n_layers=4, n_hidden=2, layernorm=True),
          "table1-large": dict(H=32, n_layers=4, n_hidden=5, layernorm=True)}


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def global_edges(mesh):
    """Directed edges of the unpartitioned lattice graph (links along each
    axis; a periodic axis closes every line into a ring)."""
    n = mesh.npts
    total = 0
    for a in range(3):
        links = n[a] if mesh.periodic[a] else n[a] - 1
        total += links * n[(a + 1) % 3] * n[(a + 2) % 3]
    return 2 * total


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", default="C4", choices=sorted(WORKLOADS))
    ap.add_argument("--model", default="workload", choices=["workload"] + sorted(TABLE1),
                    help="the workload's own model, or one of the paper's Table I models")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 comparison path")
    ap.add_argument("--no-bf16-state", action="store_true",
                    help="skip the separately reported path with BF16 edge-state storage")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-autotune", action="store_true", help="use the library's default schedule")
    ap.add_argument("--sample-nodes", type=int, default=24, help="nodes for the error vs FP64")
    ap.add_argument("--profile-steps", type=int, default=2,
                    help="steps of the separate pass that records per-kernel times")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def copy_bandwidth(gib=2, reps=10):
    """Achievable HBM bandwidth for context: a device-to-device copy of
    `gib` GiB, timed with HIP events over `reps` copies (read + write bytes
    / time).  Runs before the timed steps, outside them."""
    import torch
    n = gib * (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    gbps = 2 * n * 4 * reps / (t0.elapsed_time(t1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbps


def copy_calibration():
    """A plain copy of a known size: FETCH_SIZE / WRITE_SIZE of this dispatch
    calibrate the counters against 256 MiB read and 256 MiB written."""
    import torch
    n = 256 * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4}), flush=True)


# Measured HBM traffic of the dominant kernel: summaries of two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE), scaled by the same counters on a plain
# copy of known size, in profiles/*_hbm_traffic.md.  Each record holds the
# SHA-256 of the kernel's source files and is used only while they are
# unchanged (else traffic is null).
TRAFFIC_GLOB = "profiles/*_hbm_traffic.md"
KERNEL_SOURCES = {"edge_bwd": ("mp_bwd.hip", "mp_device.hpp", "mp_kernels.hpp"),
                  "edge_fwd": ("mp_fwd.hip", "mp_device.hpp", "mp_kernels.hpp")}


def sources_sha256(kernel):
    import hashlib
    import os
    h = hashlib.sha256()
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2410_01657_amd", "csrc")
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel, workload, gemm="bf16", estate="f32"):
    """HBM bytes per launch (read + write) of `kernel` from the traffic
    summaries, or None when absent, for another workload or path, or stale."""
    import glob
    import os
    if kernel not in KERNEL_SOURCES:
        return None
    root = os.path.dirname(os.path.abspath(__file__))
    rec = {}
    for path in sorted(glob.glob(os.path.join(root, TRAFFIC_GLOB))):
        with open(path) as f:
            for line in f:
                if line.startswith("traffic:"):
                    kv = dict(t.split("=", 1) for t in line.split()[1:])
                    if (kv.get("kernel") == kernel and kv.get("workload") == workload
                            and kv.get("gemm", "bf16") == gemm and kv.get("estate", "f32") == estate):
                        rec = kv
    if not rec or rec.get("sources_sha256") != sources_sha256(kernel):
        return None
    return float(rec["read_bytes"]) + float(rec["write_bytes"])


KERNELS = ("pack", "tiles", "proj", "edge_fwd", "halo", "halo_adj", "node_fwd", "node_bwd", "edge_bwd", "edge_dw", "node_dw",
           "gq", "gq_dw", "wreduce", "mlp_fwd", "mlp_bwd", "edge_inputs", "loss",
           "deep_edge_fwd", "deep_node_fwd", "deep_node_bwd", "deep_edge_bwd", "deep_gather", "deep_edge_dw",
           "deep_node_dw", "deep_mlp_fwd", "deep_mlp_bwd", "deep_mlp_dw")


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def run_path(gemm, spec, params, prob, steps, warmup, schedule, profile_steps, estate="f32"):
    """Time `steps` full fwd+bwd steps (no per-launch instrumentation), then
    the message-passing layers alone, then record per-kernel times in a
    separate pass.  Returns a dict with the timings, per-kernel stats, the
    outputs, the loss and the parameter gradients of the last step."""
    import ctypes as C

    import torch

    from paper_2410_01657_amd._lib import call
    from paper_2410_01657_amd.model import ConsistentGNN

    model = ConsistentGNN(spec, params, "cuda", gemm=gemm, schedule=schedule,
                          estate=estate).requires_grad_(True)

    def step():
        for t in model.params.values():
            t.grad = None
        Y = model.forward(prob.dg, prob.X, prob.E0)
        loss = model.loss(prob.dg, Y, prob.T)
        loss.backward()
        return Y, loss

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0, t1 = _events()
    t0.record(stream)
    for _ in range(steps):
        Y, loss = step()
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    out = {"ms": ms, "Y": Y.detach(), "loss": float(loss.detach().cpu()),
           "grads": {k: t.grad.detach().clone() for k, t in model.params.items() if t.grad is not None}}
    del Y, loss
    out["mp_ms"] = _time_layers_only(model, prob, steps, max(1, warmup // 2))
    # per-kernel times: HIP events around every launch, in a pass of its own
    call("mp_profile_enable", 1)
    for _ in range(profile_steps):
        step()
    torch.cuda.synchronize()
    kernels = {}
    for name in KERNELS:
        tot, n = C.c_double(), C.c_int64()
        call("mp_profile_read", name.encode(), C.byref(tot), C.byref(n))
        if n.value:
            kernels[name] = {"ms_total": tot.value / profile_steps, "launches_per_step": n.value / profile_steps,
                             "ms_avg": tot.value / n.value}
    call("mp_profile_enable", 0)
    out["kernels"] = kernels
    for t in model.params.values():
        t.grad = None
    del model
    return out


def _time_layers_only(model, prob, steps, warmup):
    """Forward and adjoint of the message-passing layers alone (Eq. 4a-e and
    their adjoint, parameter gradients included), on the encoders' outputs
    with a fixed upstream gradient: the same entry points and launch
    configuration as the model step, none of its encoders, decoder or loss."""
    import torch

    with torch.no_grad():
        x0, e0 = model.encode(prob.X, prob.E0)
    g_top = torch.full_like(x0, 1.0 / x0.numel())

    def layers():
        for t in model.params.values():
            t.grad = None
        x, _ = model.process(prob.dg, x0, e0)
        torch.autograd.backward([x], [g_top])

    for _ in range(warmup):
        layers()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0, t1 = _events()
    t0.record(stream)
    for _ in range(steps):
        layers()
    t1.record(stream)
    torch.cuda.synchronize()
    del x0, e0, g_top
    torch.cuda.empty_cache()
    return t0.elapsed_time(t1) / steps


def cpu_baseline(cfg, spec, inp, n_layers, sample_gids, outs, min_seconds=10.0):
    """The FP64 oracle as it stands, timed on a bounded sample: full model
    fwd+bwd on whole sub-graphs 0, 1, 2, ... one at a time until at least
    `min_seconds` have been spent (for an unpartitioned workload, on the
    elements of successive 1/16 or 1/8 z-slabs); plus the oracle's exact
    outputs at sampled nodes, which state the GPU paths' error vs FP64."""
    from threadpoolctl import threadpool_info

    from mpinputs import slab_partition
    from oracle.ball import ball_output
    from oracle.graph import partition_graph
    from oracle.nmp import consistent_loss, edge_inputs, model_bwd, model_fwd

    mesh = inp.mesh
    n_parts = int(inp.elem_part.max()) + 1
    if n_parts > 1 and mesh.n_gid / n_parts <= 200_000:
        part = inp.elem_part
    elif n_parts > 1:          # large sub-graphs: one-element-thick z-slabs
        part = slab_partition(cfg.nel, cfg.nel[2])
    else:
        part = slab_partition(cfg.nel, 16 if cfg.nel[2] % 16 == 0 else 8)
    rows = edges = 0
    dt = 0.0
    parts = 0
    for p in range(int(part.max()) + 1):
        keep = part == p
        (G,), _ = partition_graph(mesh.elem_gid[keep], mesh.P, np.zeros(int(keep.sum()), np.int32), 1)
        X = inp.field.astype(np.float64)[G.gid]
        T = inp.target.astype(np.float64)[G.gid]
        E0 = edge_inputs(G, mesh.pos, mesh.period)
        t = time.perf_counter()
        Y, cache = model_fwd(inp.params, spec, [G], {}, [X], [E0])
        L, gY, _ = consistent_loss(Y, [T], [G])
        model_bwd(inp.params, spec, [G], {}, cache, gY)
        dt += time.perf_counter() - t
        rows, edges, parts = rows + G.n, edges + G.e, parts + 1
        del Y, cache, gY
        if dt >= min_seconds:
            break
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    ref = np.stack([ball_output(inp.params, spec, mesh, inp.field, int(c)) for c in sample_gids])
    errs = {}
    for name, Ys in outs.items():
        d = np.abs(Ys - ref)
        errs[name] = {"max_rel": float(d.max() / np.abs(ref).max()),
                      "mean_rel": float(d.mean() / np.abs(ref).mean())}
    base = {"value": edges * n_layers / dt, "unit": "edges/s", "cores": int(threads), "kind": "oracle",
            "sample": f"full model fwd+bwd (FP64 NumPy) on {parts} whole sub-graph(s), one at a time: "
                      f"{rows} rows, {edges} edges, {n_layers} layers, {dt:.1f} s"}
    return base, errs


def main():
    a = _parse()
    if a.gpus != 1:
        print(json.dumps({"error": "one GPU only: all sub-graphs share one device and the halo sum runs on it; there is no multi-GPU halo exchange",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    if a.copy_calibration:
        copy_calibration()
        return
    import torch

    from mpinputs import CONFIGS, ModelSpec, make_inputs
    from paper_2410_01657_amd.autotune import tuned_schedule
    from paper_2410_01657_amd.model import Problem
    from paper_2410_01657_amd.roofline import (PEAK, PEAK_HBM, PEAK_VALU, bound_of, deep_kernels,
                                               layer_kernels, layer_roof_seconds)

    wl = dict(WORKLOADS[a.workload])
    cfg = CONFIGS[a.workload]
    spec = cfg.spec
    if a.model != "workload":
        spec = ModelSpec(**TABLE1[a.model])
        wl["desc"] += (f", with Table I's {a.model.split('-')[1]} model (H={spec.H}, "
                       f"{spec.n_hidden} hidden layers per MLP, FP32)")
    deep = spec.n_hidden > 0 or spec.H in (8, 16)
    R = wl["R"] or cfg.R
    inp = make_inputs(cfg, base_seed=a.seed, R=R, spec=spec)
    prob = Problem(inp.mesh, inp.field, inp.target, inp.elem_part, R, "cuda")
    hg = prob.dg.host
    _progress(f"graph built: {hg.n_rows} rows, {hg.n_edges} edges, {hg.R} sub-graphs")
    E_global = global_edges(inp.mesh)
    N, E, G, M = hg.n_rows, hg.n_edges, hg.n_groups, int(hg.member.shape[0])

    rng = np.random.default_rng(a.seed + 1)
    sample_gids = rng.choice(inp.mesh.n_gid, size=a.sample_nodes, replace=False)
    order = np.argsort(hg.row_gid, kind="stable")
    sample_rows = order[np.searchsorted(hg.row_gid[order], sample_gids)]

    copy_gbps = copy_bandwidth()
    # path name -> (GEMM operand type, edge-state storage type)
    PATHS = {"bf16": ("bf16", "f32"), "f32": ("f32", "f32"), "bf16_state": ("bf16", "bf16")}
    paths = (["f32"] if deep else ["bf16"] + ([] if a.no_fp32 else ["f32"])
             + ([] if a.no_bf16_state else ["bf16_state"]))
    res, outs, scheds, grads = {}, {}, {}, {}
    for name in paths:
        gemm, estate = PATHS[name]
        sched = None if (a.no_autotune or deep) else tuned_schedule(prob.dg, spec.H, spec.layernorm, gemm,
                                                                    estate=estate)
        scheds[name] = sched
        _progress(f"{name}: schedule {sched}")
        r = run_path(gemm, spec, inp.params, prob, a.steps, a.warmup, sched, a.profile_steps, estate)
        _progress(f"{name}: {r['ms']:.3f} ms/step, message-passing layers alone {r['mp_ms']:.3f} ms")
        outs[name] = r.pop("Y").cpu().numpy()[sample_rows].astype(np.float64)
        grads[name] = {k: v.cpu().numpy().astype(np.float64) for k, v in r.pop("grads").items()}
        if not np.all(np.isfinite(outs[name])) or not np.isfinite(r["loss"]):
            raise RuntimeError(f"{name} path produced a non-finite output or loss")
        res[name] = r
        torch.cuda.empty_cache()

    main_gemm = paths[0]
    main_path = res[main_gemm]
    value = E_global * spec.n_layers / (main_path["ms"] * 1e-3)

    def dominant_roofline(name):
        """Roofline of the path's longest-running kernel: algorithmic bytes
        (or flops) per launch / its average launch time, against the peak
        of whichever roof bounds that kernel."""
        gemm, estate = PATHS[name]
        work = (deep_kernels(N, E, G, M, spec.H, spec.n_hidden, spec.n_layers) if deep
                else layer_kernels(N, E, G, M, spec.H, gemm, spec.n_layers, estate))
        kern = res[name]["kernels"]
        dom = max((k for k in kern if k in work), key=lambda k: kern[k]["ms_total"])
        w = work[dom]
        avg_s = kern[dom]["ms_avg"] * 1e-3
        if deep and w.flops / PEAK_VALU > w.bytes / PEAK_HBM:
            r = {"bound": "alu", "achieved": w.flops / avg_s / 1e12, "peak": PEAK_VALU / 1e12, "unit": "TFLOP/s"}
        elif bound_of(w, gemm) == "hbm":
            r = {"bound": "hbm", "achieved": w.bytes / avg_s / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
        else:
            r = {"bound": "mfma", "achieved": w.flops / avg_s / 1e12, "peak": PEAK[gemm] / 1e12,
                 "unit": "TFLOP/s"}
        r["frac"] = r["achieved"] / r["peak"]
        r.update({"kernel": dom, "ms_avg": kern[dom]["ms_avg"], "algorithmic_GB": w.bytes / 1e9,
                  "algorithmic_GFLOP": w.flops / 1e9})
        tr = None if deep else recorded_traffic(dom, a.workload, gemm, estate)
        r["traffic"] = tr / 1e9 if tr is not None else None  # GB per launch, measured
        r["traffic_unit"] = "GB per launch (HBM read + write)"
        # context: the same kernel against the bandwidth a plain 2 GiB copy reaches
        if r["bound"] == "hbm":
            r["copy_GBps"] = copy_gbps
            r["frac_of_copy"] = r["achieved"] / copy_gbps
        return r

    def mp_layers(name):
        """The message-passing layers alone: edges/s and the fraction of
        their roofline time (every layer kernel at the higher of its HBM and
        matrix floors, published peaks; and against the measured copy rate)."""
        gemm, estate = PATHS[name]
        ms = res[name]["mp_ms"]
        out = {"value": E_global * spec.n_layers / (ms * 1e-3), "ms": ms}
        if not deep:
            t_roof = layer_roof_seconds(N, E, G, M, spec.H, gemm, spec.n_layers, estate=estate)
            t_copy = layer_roof_seconds(N, E, G, M, spec.H, gemm, spec.n_layers, hbm=copy_gbps * 1e9,
                                        estate=estate)
            out.update({"roof_ms": t_roof * 1e3, "frac_of_roof": t_roof * 1e3 / ms,
                        "roof_ms_at_copy_rate": t_copy * 1e3, "frac_of_roof_at_copy_rate": t_copy * 1e3 / ms})
        return out

    # dominant kernel of the main path and its roofline
    roof = dominant_roofline(main_gemm)

    def grad_dev(name):
        """Parameter gradients of a BF16 path against the FP32 path's (which
        match the FP64 oracle to ~1e-5 in the parity tests): max |d| /
        max |g_fp32| per parameter tensor, the worst tensor reported."""
        dev = {k: float(np.abs(grads[name][k] - v).max() / max(np.abs(v).max(), 1e-30))
               for k, v in grads["f32"].items()}
        worst = max(dev, key=dev.get)
        return {"max": dev[worst], "tensor": worst, "median": float(np.median(list(dev.values())))}

    line = {
        "metric": "MP-layer fwd+bwd edges/sec, BF16-MFMA vs FP32, at stated rel. error vs FP64",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": main_path["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if main_gemm == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "sub_graphs": hg.R, "sub_graph_rows": N, "sub_graph_edges": E,
                   "halo_groups": G, "halo_members": M, "global_edges": E_global, "layers": spec.n_layers,
                   "H": spec.H, "schedule": scheds},
        "roofline": roof,
        "mp_layers": mp_layers(main_gemm),
    }
    if "f32" in res and main_gemm != "f32":
        line["fp32"] = {"value": E_global * spec.n_layers / (res["f32"]["ms"] * 1e-3),
                        "ms_per_step": res["f32"]["ms"], "roofline": dominant_roofline("f32"),
                        "mp_layers": mp_layers("f32")}
        line["bf16_over_fp32"] = res["f32"]["ms"] / main_path["ms"]
        line["bf16_over_fp32_mp_layers"] = res["f32"]["mp_ms"] / main_path["mp_ms"]
        line["bf16_grad_rel_dev_vs_fp32"] = grad_dev("bf16")
    if "bf16_state" in res:
        # BF16 GEMMs with the edge states (and their gradients) stored in
        # BF16 between kernels: a separate option, reported beside the line
        bs = res["bf16_state"]
        line["bf16_state"] = {"value": E_global * spec.n_layers / (bs["ms"] * 1e-3), "ms_per_step": bs["ms"],
                              "over_bf16": main_path["ms"] / bs["ms"] if main_gemm == "bf16" else None,
                              "roofline": dominant_roofline("bf16_state"), "mp_layers": mp_layers("bf16_state")}
        if "f32" in res:
            line["bf16_state"]["grad_rel_dev_vs_fp32"] = grad_dev("bf16_state")
    line["kernels"] = {g: {k: round(v["ms_total"], 4) for k, v in res[g]["kernels"].items()} for g in res}
    if not a.no_cpu_baseline:
        _progress("timing the FP64 oracle on a bounded sample")
        base, errs = cpu_baseline(cfg, spec, inp, spec.n_layers, sample_gids, outs)
        line["cpu_baseline"] = base
        line["rel_error_vs_fp64"] = errs
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
