"""GPU parity on the smallest graphs the method admits (Eq. 4a-e).

A single P = 1 hexahedral element gives 8 rows and 24 directed edges: fewer
edges than one edge tile and fewer rows than one wave, so every kernel runs
only its ragged tail.  Two such elements cut into two sub-graphs of one
element each make every row of the shared face a halo copy (Eq. 4c, 4d), with
four two-member groups.  A 4 x 2 x 1 box cut into one element and the other
seven puts a one-element sub-graph beside a larger one in the same launch.
Forward and adjoint are compared element by element
with the FP64 oracle, at the tolerances of the one-layer parity tests.
"""

import numpy as np
import pytest
import torch

from mpinputs import box_mesh
from oracle.graph import halo_lists, partition_graph
from oracle.nmp import nmp_layer_bwd, nmp_layer_fwd

from _util import layer_params, normwise, split_rows

pytestmark = pytest.mark.gpu

DEV = "cuda"

CASES = {"one_element": ((1, 1, 1), [0], 1), "two_elements_R2": ((2, 1, 1), [0, 1], 2),
         "one_and_seven_R2": ((4, 2, 1), [0] + [1] * 7, 2)}


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("H,ln,gemm", [(32, False, "f32"), (64, True, "f32"), (64, True, "bf16")])
def test_smallest_graphs_forward_and_adjoint(case, H, ln, gemm):
    from paper_2410_01657_amd import DeviceGraph, build_graph
    from paper_2410_01657_amd.ops import layer_backward, layer_cfg, layer_forward
    nel, part, R = CASES[case]
    m = box_mesh(nel, 1)
    part = np.array(part, np.int32)
    hg = build_graph(m.elem_gid, m.P, part, R, order="gid")
    og, copies = partition_graph(m.elem_gid, m.P, part, R)
    pairs = halo_lists(og, copies)
    dg = DeviceGraph(hg, DEV)
    assert (dg.n_rows, dg.n_edges) == (sum(G.n for G in og), sum(G.e for G in og))
    assert og[0].n == 8 and og[0].e == 24
    spec, o, names = layer_params(H, ln)
    rng = np.random.default_rng(5 + H + R)
    x = rng.standard_normal((dg.n_rows, H)).astype(np.float32)
    e = rng.standard_normal((dg.n_edges, H)).astype(np.float32)
    gx = rng.standard_normal((dg.n_rows, H)).astype(np.float32)
    ge = rng.standard_normal((dg.n_edges, H)).astype(np.float32)
    cfg = layer_cfg(H, ln, gemm=gemm)
    p = {k: _t(o[v]) for k, v in names.items()}
    xg, eg, a_star = layer_forward(cfg, p, dg, _t(x), _t(e))
    g_x, g_e, grads = layer_backward(cfg, p, dg, _t(x), _t(e), a_star, _t(gx), _t(ge))

    n_off = [0] + list(np.cumsum([G.n for G in og]))
    e_off = [0] + list(np.cumsum([G.e for G in og]))
    xo, eo, cache = nmp_layer_fwd(o, 0, spec, og, pairs, split_rows(x.astype(np.float64), n_off),
                                  split_rows(e.astype(np.float64), e_off), True)
    ogr = {}
    gxs, ges = nmp_layer_bwd(o, 0, spec, og, pairs, cache, split_rows(gx.astype(np.float64), n_off),
                             split_rows(ge.astype(np.float64), e_off), ogr)
    tf, tb = (1e-5, 1e-4) if gemm == "f32" else (3e-2, 5e-2)
    assert normwise(a_star.cpu().numpy(), np.concatenate(cache["a_star"])) < tf
    assert normwise(eg.cpu().numpy(), np.concatenate(eo)) < tf
    assert normwise(xg.cpu().numpy(), np.concatenate(xo)) < tf
    assert normwise(g_x.cpu().numpy(), np.concatenate(gxs)) < tb
    assert normwise(g_e.cpu().numpy(), np.concatenate(ges)) < tb
    for k, v in names.items():
        err = normwise(grads[k].cpu().numpy(), ogr[v])
        assert err < tb, (k, err)
