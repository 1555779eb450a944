"""Periodic boxes on the GPU: the meshes of the paper's scaling study
(Table II partitions a periodic box into z-slabs whose first and last slab
meet through the wrap).

* a small periodic box: edge inputs bit-exact against the oracle's (nearest
  periodic image), outputs, loss and gradients at R = 1 and R = 8 against
  the FP64 oracle at R = 1;
* the Table II R = 8 partition at full size (16 x 16 x 128 elements, P=5,
  8 slabs of 518,400 rows): sampled outputs and gradients against the
  oracle's exact receptive-field evaluation, nodes on the wrap included.
"""

import numpy as np
import pytest
import torch

from mpinputs import CONFIGS, ModelSpec, box_mesh, init_params, make_inputs, slab_partition
from mpinputs.fields import velocity_field
from oracle.ball import ball_grad
from oracle.nmp import consistent_loss, model_bwd, model_fwd
from oracle.problem import build_problem

from _util import normwise, oracle_edge_order

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL = {"f32": (1e-4, 1e-4), "bf16": (3e-2, 5e-2)}


@pytest.fixture(scope="module")
def small():
    m = box_mesh((4, 4, 8), 3, periodic=(True, True, True))
    field = velocity_field(m.pos, 41, noise_sigma=0.01)
    target = np.roll(field, 1, axis=1)
    spec = ModelSpec(H=64, n_layers=2, layernorm=True)
    params = init_params(spec, 42, perturb=True)
    p = build_problem(m, field, target, None, 1)
    Y, c = model_fwd(params, spec, p.graphs, p.pair_lists, p.X, p.E0)
    L, gY, _ = consistent_loss(Y, p.T, p.graphs)
    grads, _ = model_bwd(params, spec, p.graphs, p.pair_lists, c, gY)
    return m, field, target, spec, params, Y[0], L, grads


def test_periodic_edge_inputs_bit_exact(small):
    from paper_2410_01657_amd.model import Problem
    m, field, target = small[:3]
    part = slab_partition(m.nel, 8)
    prob = Problem(m, field, target, part, 8, DEV)
    o = build_problem(m, field, target, part, 8)
    ref = np.concatenate(o.E0).astype(np.float32)
    np.testing.assert_array_equal(prob.E0.cpu().numpy()[oracle_edge_order(prob.host)], ref)


@pytest.mark.parametrize("gemm", ["f32", "bf16"])
@pytest.mark.parametrize("R", [1, 8])
def test_periodic_model_vs_oracle(small, gemm, R):
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    m, field, target, spec, params, Yo, Lo, go = small
    part = slab_partition(m.nel, R) if R > 1 else np.zeros(m.n_elem, np.int32)
    prob = Problem(m, field, target, part, R, DEV)
    model = ConsistentGNN(spec, params, DEV, gemm=gemm).requires_grad_(True)
    Y = model.forward(prob.dg, prob.X, prob.E0)
    loss = model.loss(prob.dg, Y, prob.T)
    loss.backward()
    tol_y, tol_g = TOL["bf16" if gemm == "bf16" else "f32"]
    assert normwise(Y.detach().cpu().numpy(), Yo[prob.host.row_gid]) < tol_y
    assert abs(float(loss.detach()) - Lo) / Lo < tol_y
    errs = {k: normwise(t.grad.cpu().numpy(), go[k]) for k, t in model.params.items()}
    worst = max(errs, key=errs.get)
    print(f"periodic {gemm} R={R}: worst parameter gradient {errs[worst]:.2e} ({worst})")
    assert errs[worst] < tol_g, (worst, errs[worst])


# Table I's models (deep narrow MLPs) on the same full-size partition
TABLE1 = {"table1-small": ModelSpec(H=8, n_layers=4, n_hidden=2, layernorm=True),
          "table1-large": ModelSpec(H=32, n_layers=4, n_hidden=5, layernorm=True)}


@pytest.mark.slow
@pytest.mark.parametrize("gemm", ["bf16", "f32", "table1-small", "table1-large"])
def test_table2_r8_sampled_outputs_and_gradients(gemm):
    """Full Table II R = 8 size (4.1M rows, the launch shapes bench.py times):
    ten nodes' outputs, and the gradient of a random projection of them,
    against the FP64 oracle evaluated exactly on each node's 4-hop ball."""
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    cfg = CONFIGS["T2R8"]
    spec = TABLE1.get(gemm, cfg.spec)
    inp = make_inputs(cfg, perturb=True, spec=spec)
    m = inp.mesh
    prob = Problem(m, inp.field, inp.target, inp.elem_part, cfg.R, DEV)
    hg = prob.dg.host
    assert (hg.n_rows, int(hg.halo_rows[0]), int(hg.neighbours[0])) == (8 * 518400, 12800, 2)
    model = ConsistentGNN(spec, inp.params, DEV, gemm="bf16" if gemm == "bf16" else "f32").requires_grad_(True)
    Y = model.forward(prob.dg, prob.X, prob.E0)
    n = m.npts
    rng = np.random.default_rng(7)
    # corners of the wrap, a slab interface (z = 80), and random nodes
    fixed = [0, n[0] - 1, m.n_gid - 1, n[0] * n[1] * 80 + 3, n[0] * n[1] * 79 + n[0] * (n[1] - 1)]
    gids = fixed + [int(c) for c in rng.choice(m.n_gid, 5, replace=False)]
    order = np.argsort(hg.row_gid, kind="stable")
    rows = order[np.searchsorted(hg.row_gid[order], gids)]
    w = rng.standard_normal((len(gids), spec.out))
    gY = torch.zeros_like(Y)
    gY[torch.as_tensor(rows, device=DEV)] = torch.as_tensor(w, dtype=torch.float32, device=DEV)
    Y.backward(gY)
    Ys = Y.detach()[torch.as_tensor(rows, device=DEV)].cpu().numpy()
    ref_y, ref_g = [], {}
    for c, wc in zip(gids, w):
        y, g = ball_grad(inp.params, spec, m, inp.field, c, wc)
        ref_y.append(y)
        for k, v in g.items():
            ref_g[k] = ref_g.get(k, 0.0) + v
    tol_y, tol_g = TOL["bf16" if gemm == "bf16" else "f32"]
    assert normwise(Ys, np.stack(ref_y)) < tol_y
    errs = {k: normwise(t.grad.cpu().numpy(), ref_g[k]) for k, t in model.params.items()}
    worst = max(errs, key=errs.get)
    print(f"Table II R=8 {gemm}: worst parameter gradient {errs[worst]:.2e} ({worst})")
    assert errs[worst] < tol_g, (worst, errs[worst])
