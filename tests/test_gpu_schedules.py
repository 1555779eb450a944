"""GPU parity of the one-layer forward and adjoint at every edge-kernel
schedule the autotuner may pick (Eq. 4a-e and their adjoint, Eq. 3).

A schedule (edges per row-aligned tile, workgroups of the forward and of
the adjoint edge kernels, waves per workgroup of the adjoint, fixed or
queued tile order of the forward) regroups floating-point sums only: every
candidate is compared element by element with the FP64 oracle at the
tolerances of the default-schedule tests, on the C0 mesh cut into 2x2x2
blocks, on a seeded uneven bisection with T-junctions, and on a
tetrahedral mesh whose in-degrees reach several dozen.  Outputs of every
candidate are also bitwise reproducible run to run.
"""

import numpy as np
import pytest
import torch

from mpinputs import CONFIGS, box_mesh, make_inputs, rcb_partition
from mpinputs.tetmesh import centroid_partition, tet_mesh
from oracle.graph import halo_lists, partition_graph
from oracle.nmp import nmp_layer_bwd, nmp_layer_fwd

from _util import layer_params, normwise, split_rows

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _graph(name):
    from paper_2410_01657_amd import DeviceGraph, build_graph
    links = None
    if name == "c0_blocks":
        inp = make_inputs(CONFIGS["C0"])
        m, part, R, P = inp.mesh, inp.elem_part, 8, inp.mesh.P
    elif name == "rcb":
        nel = (6, 5, 4)
        m = box_mesh(nel, 3)
        part, _ = rcb_partition(nel, 8, seed=11, ratio=(1.0, 10.0))
        R, P = 8, 3
    else:
        m = tet_mesh(1500, 7)
        R, P, links = 8, None, m.links
        part = centroid_partition(m, R)
    hg = build_graph(m.elem_gid, P, part, R, links, order="gid")  # rows in the oracle's order
    og, copies = partition_graph(m.elem_gid, P, part, R, links)
    return DeviceGraph(hg, DEV), og, halo_lists(og, copies)


def _candidates(H, gemm):
    from paper_2410_01657_amd.autotune import candidates
    return candidates(H, gemm)


@pytest.mark.parametrize("graph,H,gemm", [("c0_blocks", 64, "bf16"), ("c0_blocks", 64, "f32"),
                                          ("rcb", 64, "bf16"), ("tet", 64, "f32"), ("c0_blocks", 128, "bf16")])
def test_every_candidate_schedule_matches_the_oracle(graph, H, gemm):
    from paper_2410_01657_amd.ops import layer_backward, layer_cfg, layer_forward
    dg, og, pairs = _graph(graph)
    spec, o, names = layer_params(H, True)
    rng = np.random.default_rng(H + 17)
    x = rng.standard_normal((dg.n_rows, H)).astype(np.float32)
    e = rng.standard_normal((dg.n_edges, H)).astype(np.float32)
    gx = rng.standard_normal((dg.n_rows, H)).astype(np.float32)
    ge = rng.standard_normal((dg.n_edges, H)).astype(np.float32)
    n_off = [0] + list(np.cumsum([G.n for G in og]))
    e_off = [0] + list(np.cumsum([G.e for G in og]))
    xs, es = split_rows(x.astype(np.float64), n_off), split_rows(e.astype(np.float64), e_off)
    xo, eo, cache = nmp_layer_fwd(o, 0, spec, og, pairs, xs, es, True)
    ogr = {}
    gxs, ges = nmp_layer_bwd(o, 0, spec, og, pairs, cache, split_rows(gx.astype(np.float64), n_off),
                             split_rows(ge.astype(np.float64), e_off), ogr)
    ref = {"x": np.concatenate(xo), "e": np.concatenate(eo), "a": np.concatenate(cache["a_star"]),
           "gx": np.concatenate(gxs), "ge": np.concatenate(ges)}
    p = {k: _t(o[v]) for k, v in names.items()}
    X, Ein, GX, GE = _t(x), _t(e), _t(gx), _t(ge)
    tol_f, tol_b = (1e-5, 1e-4) if gemm == "f32" else (3e-2, 5e-2)
    worst = {}
    from paper_2410_01657_amd.autotune import apply_schedule
    for sched in _candidates(H, gemm):
        cfg = apply_schedule(layer_cfg(H, True, gemm=gemm), sched)
        runs = []
        for _ in range(2):
            xg, eg, ag = layer_forward(cfg, p, dg, X, Ein)
            g_x, g_e, grads = layer_backward(cfg, p, dg, X, Ein, ag, GX, GE)
            runs.append([xg, eg, ag, g_x, g_e] + [grads[k] for k in sorted(names)])
        for a, b in zip(*runs):
            assert torch.equal(a, b), sched
        xg, eg, ag, g_x, g_e = runs[0][:5]
        errs = {"x": normwise(xg.cpu().numpy(), ref["x"]), "e": normwise(eg.cpu().numpy(), ref["e"]),
                "a": normwise(ag.cpu().numpy(), ref["a"]), "gx": normwise(g_x.cpu().numpy(), ref["gx"]),
                "ge": normwise(g_e.cpu().numpy(), ref["ge"])}
        grads = runs[0][5:]
        for k, gk in zip(sorted(names), grads):
            errs["d" + k] = normwise(gk.cpu().numpy(), ogr[names[k]])
        for k, err in errs.items():
            tol = tol_f if k in ("x", "e", "a") else tol_b
            assert err < tol, (sched, k, err)
            worst[k] = max(worst.get(k, 0.0), err)
    print(f"{graph} H={H} {gemm}: {len(_candidates(H, gemm))} schedules, worst errors "
          + ", ".join(f"{k} {v:.1e}" for k, v in sorted(worst.items())))


@pytest.mark.parametrize("graph,H", [("c0_blocks", 64), ("rcb", 64), ("c0_blocks", 128)])
def test_every_candidate_schedule_with_bf16_edge_states(graph, H):
    """The BF16 edge-state option at every schedule: the FP32-state layer's
    results on the same BF16-representable e and g_e', bitwise, with e' and
    g_e rounded to nearest even (the FP32-state results themselves are
    checked against the oracle above)."""
    from paper_2410_01657_amd.autotune import apply_schedule
    from paper_2410_01657_amd.ops import layer_backward, layer_cfg, layer_forward
    dg, og, pairs = _graph(graph)
    spec, o, names = layer_params(H, True)
    rng = np.random.default_rng(H + 23)
    X, GX = _t(rng.standard_normal((dg.n_rows, H))), _t(rng.standard_normal((dg.n_rows, H)))
    E16 = _t(rng.standard_normal((dg.n_edges, H))).to(torch.bfloat16)
    GE16 = _t(rng.standard_normal((dg.n_edges, H))).to(torch.bfloat16)
    p = {k: _t(o[v]) for k, v in names.items()}
    for sched in _candidates(H, "bf16"):
        c32 = apply_schedule(layer_cfg(H, True, gemm="bf16"), sched)
        c16 = apply_schedule(layer_cfg(H, True, gemm="bf16", estate="bf16"), sched)
        xo, eo, a = layer_forward(c32, p, dg, X, E16.float())
        xo2, eo2, a2 = layer_forward(c16, p, dg, X, E16)
        assert torch.equal(xo, xo2) and torch.equal(a, a2), sched
        assert torch.equal(eo.to(torch.bfloat16), eo2), sched
        g1 = layer_backward(c32, p, dg, X, E16.float(), a, GX, GE16.float())
        g2 = layer_backward(c16, p, dg, X, E16, a2, GX, GE16)
        assert torch.equal(g1[0], g2[0]) and torch.equal(g1[1].to(torch.bfloat16), g2[1]), sched
        for k in names:
            assert torch.equal(g1[2][k], g2[2][k]), (sched, k)


def test_edge_state_search_returns_a_usable_choice(tmp_path, monkeypatch):
    """The opt-in search over the edge-state storage type returns one of the
    two tuned schedules with its storage type, and a model built with both
    runs forward and backward to finite values."""
    from paper_2410_01657_amd.autotune import tuned_edge_state, tuned_schedule
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    from mpinputs import ModelSpec
    monkeypatch.setenv("MPLAYER_TUNE_CACHE", str(tmp_path / "tune.json"))
    inp = make_inputs(CONFIGS["C0"])
    spec = ModelSpec(H=64, n_layers=2, layernorm=True)
    prob = Problem(inp.mesh, inp.field, inp.target, inp.elem_part, 8, DEV)
    best = tuned_edge_state(prob.dg, spec.H, spec.layernorm, "bf16")
    assert best["estate"] in ("f32", "bf16")
    other = tuned_schedule(prob.dg, spec.H, spec.layernorm, "bf16",
                           estate="bf16" if best["estate"] == "f32" else "f32")
    assert best["ms"] <= other["ms"]
    assert tuned_edge_state(prob.dg, spec.H, spec.layernorm, "f32")["estate"] == "f32"
    from mpinputs import init_params
    model = ConsistentGNN(spec, init_params(spec, 0), DEV, gemm="bf16", schedule=best,
                          estate=best["estate"]).requires_grad_(True)
    loss = model.loss(prob.dg, model.forward(prob.dg, prob.X, prob.E0), prob.T)
    loss.backward()
    assert torch.isfinite(loss).item()
    assert all(torch.isfinite(t.grad).all().item() for t in model.params.values())
