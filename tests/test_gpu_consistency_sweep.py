"""The consistency demonstration of Sec. III-A (the two panels of Fig. 6) on
the GPU, on a 32^3-element p = 1 box (33^3 nodes):

* loss of a randomly initialised model, with the input as target, against
  the number of sub-graphs R = 1 ... 64: flat for consistent layers (halo sums
  of Eq. 4c-d), growing with R for layers without them ("None" mode);
* SGD training from the same start at R = 1 and R = 8: the consistent R = 8
  curve follows the R = 1 curve, the "None" curve drifts away.

Both run with the model Fig. 6 uses, Table I's "small" one (H = 8, two
hidden H -> H layers per MLP, on the deep-MLP kernels), and with an H = 32
two-Linear model on the matrix-core kernels.  The loss values themselves
are checked against the FP64 oracle at R = 1 and, in "None" mode, at R = 8.
"""

import numpy as np
import pytest
import torch

from mpinputs import ModelSpec, init_params
from mpinputs.fields import velocity_field
from mpinputs.mesh import box_mesh
from mpinputs.partition import block_partition
from oracle.nmp import consistent_loss, model_fwd
from oracle.problem import build_problem

pytestmark = pytest.mark.gpu
DEV = "cuda"

NEL = (32, 32, 32)
SPECS = {"table1_small": ModelSpec(H=8, n_layers=4, n_hidden=2, layernorm=True),
         "h32": ModelSpec(H=32, n_layers=4, layernorm=True)}
# element blocks per axis for each sub-graph count (cut planes: 1, 2, 3, 5, 7, 9)
BLOCKS = {1: (1, 1, 1), 2: (2, 1, 1), 4: (2, 2, 1), 8: (2, 2, 2),
          16: (4, 2, 2), 32: (4, 4, 2), 64: (4, 4, 4)}


@pytest.fixture(scope="module", params=sorted(SPECS))
def setup(request):
    spec = SPECS[request.param]
    mesh = box_mesh(NEL, 1)
    field = velocity_field(mesh.pos, seed=11, noise_sigma=0.01)
    params = init_params(spec, seed=12, perturb=True)
    return spec, mesh, field, params


def _problem(mesh, field, R):
    from paper_2410_01657_amd.model import Problem
    return Problem(mesh, field, field, block_partition(NEL, BLOCKS[R]), R, DEV)


def _run(model, prob):
    with torch.no_grad():
        Y = model.forward(prob.dg, prob.X, prob.E0)
        return float(model.loss(prob.dg, Y, prob.T)), Y.cpu().numpy().astype(np.float64)


def test_loss_vs_r_sweep(setup):
    """Left panel of Fig. 6: the consistent loss is flat in R; without halo
    sums the outputs drift further from R = 1 as the share of boundary nodes
    grows (RMS over every row copy), and the loss moves with them."""
    from paper_2410_01657_amd.model import ConsistentGNN
    SPEC, mesh, field, params = setup
    cons = ConsistentGNN(SPEC, params, DEV, halo=True)
    none = ConsistentGNN(SPEC, params, DEV, halo=False)
    Rs = sorted(BLOCKS)
    Lc, Ln, drift = {}, {}, {}
    for R in Rs:
        prob = _problem(mesh, field, R)
        Lc[R], Yc = _run(cons, prob)
        Ln[R], Yn = _run(none, prob)
        gid = prob.host.row_gid
        if R == 1:
            Y1 = np.zeros((mesh.n_gid, 3))
            Y1[gid] = Yc
            rms1 = np.sqrt(np.mean(Y1 ** 2))
        assert np.max(np.abs(Yc - Y1[gid])) / np.max(np.abs(Y1)) < 1e-5   # Eq. 2
        drift[R] = np.sqrt(np.mean((Yn - Y1[gid]) ** 2)) / rms1
        del prob
    dc = np.array([abs(Lc[R] - Lc[1]) / Lc[1] for R in Rs])
    dn = np.array([abs(Ln[R] - Lc[1]) / Lc[1] for R in Rs])
    dr = np.array([drift[R] for R in Rs])
    print("R", Rs)
    print("consistent loss, rel. deviation from R=1", dc.tolist())
    print("None loss, rel. deviation from R=1", dn.tolist())
    print("None outputs, RMS drift from R=1", dr.tolist())
    assert Ln[1] == Lc[1]                        # one sub-graph has no halo
    assert np.all(dc < 1e-5)                     # consistent loss flat in R
    assert dr[0] == 0 and np.all(np.diff(dr) > 0)   # drift grows with R
    assert dn[-1] > 1e-3 and dn[-1] > 100 * max(dc.max(), 1e-7)

    # the values themselves: FP64 oracle at R = 1, and "None" mode at R = 8
    o1 = build_problem(mesh, field, field, None, 1)
    Y, _ = model_fwd(params, SPEC, o1.graphs, o1.pair_lists, o1.X, o1.E0)
    Lo1 = consistent_loss(Y, o1.T, o1.graphs)[0]
    assert abs(Lc[1] - Lo1) / Lo1 < 1e-5
    o8 = build_problem(mesh, field, field, block_partition(NEL, BLOCKS[8]), 8)
    Y, _ = model_fwd(params, SPEC, o8.graphs, o8.pair_lists, o8.X, o8.E0, halo=False)
    Lo8n = consistent_loss(Y, o8.T, o8.graphs)[0]
    assert abs(Ln[8] - Lo8n) / Lo8n < 1e-5


def _curve(spec, mesh, field, params, R, halo, steps, lr):
    from paper_2410_01657_amd.model import ConsistentGNN
    prob = _problem(mesh, field, R)
    model = ConsistentGNN(spec, params, DEV, halo=halo).requires_grad_(True)
    losses = torch.empty(steps, dtype=torch.float64, device=DEV)
    for it in range(steps):
        for t in model.params.values():
            t.grad = None
        loss = model.loss(prob.dg, model.forward(prob.dg, prob.X, prob.E0), prob.T)
        loss.backward()
        with torch.no_grad():
            losses[it] = loss.detach()
            for t in model.params.values():
                t -= lr * t.grad
    return losses.cpu().numpy()


@pytest.mark.slow
def test_training_1500_iterations_r1_vs_r8(setup):
    """Right panel of Fig. 6: 1,500 SGD iterations (forward, consistent loss,
    backward, update) at R = 1, and at R = 8 with and without halo sums."""
    spec, mesh, field, params = setup
    steps, lr = 1500, 0.01
    l1 = _curve(spec, mesh, field, params, 1, True, steps, lr)
    l8 = _curve(spec, mesh, field, params, 8, True, steps, lr)
    l8n = _curve(spec, mesh, field, params, 8, False, steps, lr)
    dc = np.abs(l8 - l1) / l1
    dn = np.abs(l8n - l1) / l1
    print("loss R=1 at 0/500/1000/1499:", l1[[0, 500, 1000, 1499]].tolist())
    print("max rel. deviation from R=1: consistent %.3e, None %.3e" % (dc.max(), dn.max()))
    assert np.all(np.isfinite(l1)) and l1[-1] < 0.5 * l1[0]     # it trains
    assert dc.max() < 1e-3                                       # same curve
    assert dn.max() > 10 * dc.max() and dn.max() > 1e-3          # "None" is not
