"""Schedule autotuner for the edge kernels of one layer.

The edge kernels run persistent workgroups over row-aligned tiles
(mp_layer_cfg.tile_edges, .edge_grid, .edge_bwd_grid).  The tuner times the
library's own forward and backward on the actual graph for a small set of
schedules and keeps the fastest, cached per (arch, H, GEMM type, LayerNorm,
rows, edges, sub-graphs) in a JSON file ($MPLAYER_TUNE_CACHE, default
~/.cache/mplayer/tune.json).  Every schedule computes the same function;
they differ only in the grouping of floating-point sums.
"""

import json
import os

import torch

from .ops import layer_backward, layer_cfg, layer_forward

TILE_EDGES = (64, 128, 256, 512)
EDGE_GRIDS = (512, 1024, 2048)
EDGE_BWD_GRIDS = (256, 512, 1024)


def candidates():
    """Every schedule the tuner can return, as mp_layer_cfg field values."""
    return [{"tile_edges": te, "edge_grid": eg, "edge_bwd_grid": bg}
            for te in TILE_EDGES for eg in EDGE_GRIDS for bg in EDGE_BWD_GRIDS]


def _cache_path():
    return os.environ.get("MPLAYER_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mplayer", "tune.json"))


def _key(dg, H, layernorm, gemm):
    arch = torch.cuda.get_device_properties(dg.device).gcnArchName.split(":")[0]
    return f"{arch}|H{H}|{gemm}|ln{int(layernorm)}|N{dg.n_rows}|E{dg.n_edges}|R{dg.host.R}"


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


def tune_layer(dg, H, layernorm=True, gemm="bf16", reps=3, seed=0):
    """Time the candidate schedules; returns the best as a dict."""
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
    x, e = rnd(dg.n_rows, H), rnd(dg.n_edges, H)
    gx, ge = rnd(dg.n_rows, H), rnd(dg.n_edges, H)
    best = None
    for te in TILE_EDGES:
        fwd = {}
        for eg in EDGE_GRIDS:
            c = layer_cfg(H, layernorm, True, gemm)
            c.tile_edges, c.edge_grid = te, eg
            fwd[eg] = _time(lambda: layer_forward(c, p, dg, x, e), reps)
        eg = min(fwd, key=fwd.get)
        c = layer_cfg(H, layernorm, True, gemm)
        c.tile_edges, c.edge_grid = te, eg
        _, _, a_star = layer_forward(c, p, dg, x, e)
        bwd = {}
        for bg in EDGE_BWD_GRIDS:
            c.edge_bwd_grid = bg
            bwd[bg] = _time(lambda: layer_backward(c, p, dg, x, e, a_star, gx, ge), reps)
        bg = min(bwd, key=bwd.get)
        ms = fwd[eg] + bwd[bg]
        if best is None or ms < best["ms"]:
            best = {"tile_edges": te, "edge_grid": eg, "edge_bwd_grid": bg, "ms": ms,
                    "fwd_ms": fwd[eg], "bwd_ms": bwd[bg]}
    del x, e, gx, ge
    torch.cuda.empty_cache()
    return best


def tuned_schedule(dg, H, layernorm=True, gemm="bf16", retune=False):
    """The cached best schedule for this graph and layer shape (tuned on a miss)."""
    cache = _load()
    key = _key(dg, H, layernorm, gemm)
    if retune or key not in cache:
        cache[key] = tune_layer(dg, H, layernorm, gemm)
        _store(cache)
    return cache[key]
