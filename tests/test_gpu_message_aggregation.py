"""The message-aggregation variant (Eq. 4b summing the edge MLP's output
instead of the updated edge state) on every kernel family: the fused edge
kernels (H = 32, 64), the split adjoint (H = 128) and the deep-MLP kernels
(Table I small model).  Outputs, loss and all parameter gradients at R = 1
and R = 8 against the FP64 oracle's unpartitioned values."""

import numpy as np
import pytest

from mpinputs import CONFIGS, ModelSpec, make_inputs
from oracle.nmp import consistent_loss, model_bwd, model_fwd
from oracle.problem import build_problem

from _util import normwise

pytestmark = pytest.mark.gpu

CASES = {
    "h32-f32": (ModelSpec(H=32, n_layers=2, layernorm=True, aggregate="message"), "f32"),
    "h64-bf16": (ModelSpec(H=64, n_layers=2, layernorm=True, aggregate="message"), "bf16"),
    "h64-f32": (ModelSpec(H=64, n_layers=2, layernorm=False, aggregate="message"), "f32"),
    "h128-bf16": (ModelSpec(H=128, n_layers=2, layernorm=True, aggregate="message"), "bf16"),
    "h128-f32": (ModelSpec(H=128, n_layers=2, layernorm=True, aggregate="message"), "f32"),
    "table1-small": (ModelSpec(H=8, n_layers=4, n_hidden=2, layernorm=True, aggregate="message"), "f32"),
}
TOL = {"f32": (1e-4, 1e-4), "bf16": (3e-2, 1e-1)}


@pytest.fixture(scope="module")
def oracle_r1():
    cache = {}

    def get(name):
        spec, _ = CASES[name]
        if spec not in cache:
            inp = make_inputs(CONFIGS["C0"], perturb=True, spec=spec)
            p = build_problem(inp.mesh, inp.field, inp.target, None, 1)
            Y, c = model_fwd(inp.params, spec, p.graphs, p.pair_lists, p.X, p.E0)
            L, gY, _ = consistent_loss(Y, p.T, p.graphs)
            grads, _ = model_bwd(inp.params, spec, p.graphs, p.pair_lists, c, gY)
            cache[spec] = (inp, Y[0], L, grads)
        return cache[spec]
    return get


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("R", [1, 8])
def test_message_aggregation_vs_oracle(oracle_r1, name, R):
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    spec, gemm = CASES[name]
    inp, Yo, Lo, go = oracle_r1(name)
    part = inp.elem_part if R > 1 else np.zeros(inp.mesh.n_elem, np.int32)
    print(f"message aggregation {name} R={R}", flush=True)
    prob = Problem(inp.mesh, inp.field, inp.target, part, R, "cuda")
    model = ConsistentGNN(spec, inp.params, "cuda", gemm=gemm).requires_grad_(True)
    Y = model.forward(prob.dg, prob.X, prob.E0)
    loss = model.loss(prob.dg, Y, prob.T)
    loss.backward()
    tol_y, tol_g = TOL[gemm]
    assert normwise(Y.detach().cpu().numpy(), Yo[prob.host.row_gid]) < tol_y
    assert abs(float(loss.detach()) - Lo) / Lo < tol_y
    for k, t in model.params.items():
        assert normwise(t.grad.cpu().numpy(), go[k]) < tol_g, k


def test_message_and_state_aggregation_differ(oracle_r1):
    """The flag reaches the kernels: the same parameters give other outputs."""
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    spec, gemm = CASES["h64-f32"]
    inp, Yo, _, _ = oracle_r1("h64-f32")
    prob = Problem(inp.mesh, inp.field, inp.target, np.zeros(inp.mesh.n_elem, np.int32), 1, "cuda")
    state = ModelSpec(**{**spec.__dict__, "aggregate": "state"})
    Y = ConsistentGNN(state, inp.params, "cuda", gemm=gemm).forward(prob.dg, prob.X, prob.E0)
    assert normwise(Y.detach().cpu().numpy(), Yo[prob.host.row_gid]) > 1e-3
