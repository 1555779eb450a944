"""The allocation-free layer forward (mp_layer_forward_noalloc), called
through the C ABI, against the workspace forward (mp_layer_forward) on the
same inputs: the same kernels on the same schedule, so every output must be
bitwise equal.  Two calls in a row on one GPU, the second on a smaller
graph, so the shared scratch holds the first call's weights and tile bounds
when the second starts; one call is also checked against the FP64 oracle
(Eq. 4a-e) at the one-layer FP32 tolerance."""

import numpy as np
import pytest
import torch

from mpinputs import CONFIGS, box_mesh, make_inputs
from oracle.graph import halo_lists, partition_graph
from oracle.nmp import nmp_layer_fwd

from _util import layer_params, normwise, split_rows

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _case(mesh, part, R, H, ln, gemm, seed, estate="f32"):
    from paper_2410_01657_amd import DeviceGraph, build_graph
    from paper_2410_01657_amd.ops import layer_cfg, layer_forward, layer_forward_noalloc
    hg = build_graph(mesh.elem_gid, mesh.P, part, R, order="gid")
    dg = DeviceGraph(hg, DEV)
    spec, o, names = layer_params(H, ln, seed=seed)
    p = {k: _t(o[v]) for k, v in names.items()}
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((dg.n_rows, H)).astype(np.float32)
    e = rng.standard_normal((dg.n_edges, H)).astype(np.float32)
    cfg = layer_cfg(H, ln, gemm=gemm, estate=estate)
    et = _t(e).to(torch.bfloat16 if estate == "bf16" else torch.float32)
    ref = layer_forward(cfg, p, dg, _t(x), et, want_pq=True)
    got = layer_forward_noalloc(cfg, p, dg, _t(x), et)
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    return dg, spec, o, x, e, got


def test_noalloc_forward_equals_the_workspace_forward_on_two_calls():
    inp = make_inputs(CONFIGS["C0"])
    # first call: the C0 mesh in 8 blocks, H=64 with LayerNorm, FP32
    dg, spec, o, x, e, (xg, eg, ag, _) = _case(inp.mesh, inp.elem_part, 8, 64, True, "f32", 5)
    og, copies = partition_graph(inp.mesh.elem_gid, inp.mesh.P, inp.elem_part, 8)
    n_off = [0] + list(np.cumsum([G.n for G in og]))
    e_off = [0] + list(np.cumsum([G.e for G in og]))
    xo, eo, cache = nmp_layer_fwd(o, 0, spec, og, halo_lists(og, copies), split_rows(x.astype(np.float64), n_off),
                                  split_rows(e.astype(np.float64), e_off), True)
    assert normwise(xg.cpu().numpy(), np.concatenate(xo)) < 1e-5
    assert normwise(eg.cpu().numpy(), np.concatenate(eo)) < 1e-5
    assert normwise(ag.cpu().numpy(), np.concatenate(cache["a_star"])) < 1e-5
    # second call: a smaller graph, BF16, H=32, no LayerNorm
    m = box_mesh((2, 2, 1), 2)
    _case(m, np.array([0, 1, 0, 1], np.int32), 2, 32, False, "bf16", 6)
    # and the first shape again, BF16 this time, then with BF16 edge states
    _case(inp.mesh, inp.elem_part, 8, 64, True, "bf16", 7)
    _case(m, np.array([0, 1, 0, 1], np.int32), 2, 128, True, "bf16", 8, estate="bf16")
