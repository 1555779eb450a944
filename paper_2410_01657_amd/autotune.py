"""Schedule autotuner for the edge kernels of one layer.

The edge kernels run persistent workgroups over row-aligned tiles.  A
schedule sets, in mp_layer_cfg: edges per tile (tile_edges), the workgroup
counts of the forward and adjoint edge kernels (edge_grid, edge_bwd_grid),
the waves per workgroup of the edge adjoint (edge_bwd_waves: 4, or 8 for
BF16 GEMMs at H <= 64, i.e. 64 or 128 edges staged per weight-gradient
round, and at H > 64, where 8 puts two waves of the split adjoint on each
SIMD and 4 gives one wave all the registers it wants) and the tile order
of the edge forward (edge_fwd_queue: fixed round robin, or per-XCD atomic
tile counters).  The tuner times the library's own
forward and backward on the actual graph and keeps the fastest, cached per
(arch, H, GEMM type, edge-state type, LayerNorm, rows, edges, sub-graphs)
in a JSON file
($MPLAYER_TUNE_CACHE, default ~/.cache/mplayer/tune.json).  Every schedule
computes the same function; they differ only in the grouping of
floating-point sums (and the forward's tile order not even in that).

Not searched: 32 x 32 matrix-core tiles (every kernel's row-block layout is
built on 16 x 16 products; the BF16 path is not bound by its products, and
the FP32 products already issue back to back); the unsplit first edge
Linear (twice the flops for the same bytes, never faster).  BF16 storage of
the edge states (estate="bf16") is not a schedule: it changes the stored
precision, not just the grouping of sums, so tuned_schedule takes it from
the caller and keeps a separate entry for it; tuned_edge_state searches it
too, for callers that accept BF16 edge states.
"""

import json
import os

import torch

from .ops import layer_backward, layer_cfg, layer_forward

TILE_EDGES = (64, 128, 256, 512)
EDGE_GRIDS = (512, 1024, 2048)
EDGE_BWD_GRIDS = (256, 512, 1024)
EDGE_FWD_QUEUES = (0, 1)
SCHEDULE_FIELDS = ("tile_edges", "edge_grid", "edge_bwd_grid", "edge_bwd_waves", "edge_fwd_queue")


def edge_bwd_waves_options(H, gemm):
    """Waves per workgroup of the edge adjoint the library accepts (the
    fused kernel: 8 only with BF16 GEMMs; the split one at H > 64: both)."""
    return (4, 8) if (gemm == "bf16" and H <= 64) or H > 64 else (4,)


def candidates(H=64, gemm="bf16"):
    """Every schedule the tuner can return for this width and GEMM type, as
    mp_layer_cfg field values."""
    return [{"tile_edges": te, "edge_grid": eg, "edge_bwd_grid": bg, "edge_bwd_waves": w, "edge_fwd_queue": q}
            for te in TILE_EDGES for eg in EDGE_GRIDS for bg in EDGE_BWD_GRIDS
            for w in edge_bwd_waves_options(H, gemm) for q in EDGE_FWD_QUEUES]


def apply_schedule(cfg, schedule):
    """Set the schedule fields of an mp_layer_cfg from a schedule dict (other
    keys, such as recorded timings, are ignored)."""
    for f in SCHEDULE_FIELDS:
        setattr(cfg, f, int(schedule.get(f, 0)))
    return cfg


def _cache_path():
    return os.environ.get("MPLAYER_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mplayer", "tune.json"))


def _key(dg, H, layernorm, gemm, estate="f32"):
    arch = torch.cuda.get_device_properties(dg.device).gcnArchName.split(":")[0]
    es = "" if estate == "f32" else f"|es{estate}"
    return f"{arch}|H{H}|{gemm}{es}|ln{int(layernorm)}|N{dg.n_rows}|E{dg.n_edges}|R{dg.host.R}|v2"


def _load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # an unwritable cache only costs a re-tune


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_layer(dg, H, layernorm=True, gemm="bf16", reps=3, seed=0, estate="f32"):
    """Time the candidate schedules; returns the best as a dict.  For each
    tile size: the best forward over (edge_grid, edge_fwd_queue), then the
    best adjoint over (edge_bwd_grid, edge_bwd_waves) with that forward."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    dev = dg.device

    def rnd(*shape, scale=1.0):
        return (torch.randn(*shape, generator=g) * scale).to(dev)

    s = (1.0 / H) ** 0.5
    p = {"We1": rnd(H, 3 * H, scale=s), "be1": rnd(H, scale=0.1), "We2": rnd(H, H, scale=s),
         "be2": rnd(H, scale=0.1), "Wn1": rnd(H, 2 * H, scale=s), "bn1": rnd(H, scale=0.1),
         "Wn2": rnd(H, H, scale=s), "bn2": rnd(H, scale=0.1)}
    if layernorm:
        p.update({"ge": 1 + rnd(H, scale=0.1), "bge": rnd(H, scale=0.1),
                  "gn": 1 + rnd(H, scale=0.1), "bgn": rnd(H, scale=0.1)})
    edt = torch.bfloat16 if estate == "bf16" else torch.float32
    x, e = rnd(dg.n_rows, H), rnd(dg.n_edges, H).to(edt)
    gx, ge = rnd(dg.n_rows, H), rnd(dg.n_edges, H).to(edt)

    def cfg_of(sched):
        return apply_schedule(layer_cfg(H, layernorm, True, gemm, estate=estate), sched)

    best = None
    for te in TILE_EDGES:
        fwd = {}
        for eg in EDGE_GRIDS:
            for q in EDGE_FWD_QUEUES:
                c = cfg_of({"tile_edges": te, "edge_grid": eg, "edge_fwd_queue": q})
                fwd[(eg, q)] = _time(lambda: layer_forward(c, p, dg, x, e), reps)
        eg, q = min(fwd, key=fwd.get)
        sched = {"tile_edges": te, "edge_grid": eg, "edge_fwd_queue": q}
        _, _, a_star = layer_forward(cfg_of(sched), p, dg, x, e)
        bwd = {}
        for bg in EDGE_BWD_GRIDS:
            for w in edge_bwd_waves_options(H, gemm):
                c = cfg_of(dict(sched, edge_bwd_grid=bg, edge_bwd_waves=w))
                bwd[(bg, w)] = _time(lambda: layer_backward(c, p, dg, x, e, a_star, gx, ge), reps)
        bg, w = min(bwd, key=bwd.get)
        ms = fwd[(eg, q)] + bwd[(bg, w)]
        if best is None or ms < best["ms"]:
            best = dict(sched, edge_bwd_grid=bg, edge_bwd_waves=w, ms=ms, fwd_ms=fwd[(eg, q)],
                        bwd_ms=bwd[(bg, w)])
    del x, e, gx, ge
    torch.cuda.empty_cache()
    return best


def tuned_schedule(dg, H, layernorm=True, gemm="bf16", retune=False, estate="f32"):
    """The cached best schedule for this graph and layer shape (tuned on a miss)."""
    cache = _load()
    key = _key(dg, H, layernorm, gemm, estate)
    if retune or key not in cache:
        cache[key] = tune_layer(dg, H, layernorm, gemm, estate=estate)
        _store(cache)
    return cache[key]


def tuned_edge_state(dg, H, layernorm=True, gemm="bf16", retune=False):
    """The edge-state storage type searched as well (an opt-in, BF16 GEMMs
    only): the faster of the tuned schedules with FP32 and with BF16 edge
    states, its storage type under "estate" (pass it to ConsistentGNN or
    layer_cfg with the schedule).  BF16 storage rounds the edge states
    between layers, so only callers that accept that precision use it."""
    if gemm != "bf16":
        return dict(tuned_schedule(dg, H, layernorm, gemm, retune), estate="f32")
    best = None
    for es in ("f32", "bf16"):
        sched = tuned_schedule(dg, H, layernorm, gemm, retune, estate=es)
        if best is None or sched["ms"] < best["ms"]:
            best = dict(sched, estate=es)
    return best
