"""The paper's own models (Table I) on the deep-MLP kernels.

small: H = 8, two hidden H -> H layers in every MLP (3,979 parameters);
large: H = 32, five hidden layers (91,459 parameters); four consistent NMP
layers, LayerNorm on encoders and processor MLPs, node input 3, edge input
4, output 3.  Outputs, consistent loss and every parameter gradient at R = 1
and R = 8 against the FP64 oracle's unpartitioned values; the flat
parameter layout of the C ABI against the Table I counts (CPU).
"""

import numpy as np
import pytest
import torch

from mpinputs import CONFIGS, ModelSpec, count_params, init_params, make_inputs
from oracle.nmp import consistent_loss, mlp_bwd, mlp_fwd, model_bwd, model_fwd
from oracle.problem import build_problem

from _util import normwise, oracle_edge_order

TABLE1 = {"small": (ModelSpec(H=8, n_layers=4, n_hidden=2, layernorm=True), 3979),
          "large": (ModelSpec(H=32, n_layers=4, n_hidden=5, layernorm=True), 91459)}


@pytest.mark.parametrize("name", sorted(TABLE1))
def test_flat_parameter_layout_counts(name):
    """The C ABI's flat arrays (one per MLP) add up to Table I's counts."""
    from paper_2410_01657_amd.ops import deep_theta_size
    spec, count = TABLE1[name]
    H, L, ln = spec.H, spec.n_hidden, spec.layernorm
    total = (deep_theta_size(spec.node_in, H, L, H, ln) + deep_theta_size(spec.edge_in, H, L, H, ln)
             + spec.n_layers * (deep_theta_size(3 * H, H, L, H, ln) + deep_theta_size(2 * H, H, L, H, ln))
             + deep_theta_size(H, H, L, spec.out, False))
    assert total == count == count_params(spec)


def _gpu(spec, params, inp, part, R, halo=True):
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    prob = Problem(inp.mesh, inp.field, inp.target, part, R, "cuda")
    model = ConsistentGNN(spec, params, "cuda", halo=halo).requires_grad_(True)
    Y = model.forward(prob.dg, prob.X, prob.E0)
    loss = model.loss(prob.dg, Y, prob.T)
    loss.backward()
    grads = {k: v.grad.cpu().numpy() for k, v in model.params.items()}
    return prob, Y.detach().cpu().numpy(), float(loss.detach()), grads


@pytest.fixture(scope="module")
def oracle_r1():
    cache = {}

    def get(name):
        if name not in cache:
            spec, _ = TABLE1[name]
            inp = make_inputs(CONFIGS["C0"], perturb=True, spec=spec)
            p = build_problem(inp.mesh, inp.field, inp.target, None, 1)
            Y, c = model_fwd(inp.params, spec, p.graphs, p.pair_lists, p.X, p.E0)
            L, gY, _ = consistent_loss(Y, p.T, p.graphs)
            grads, _ = model_bwd(inp.params, spec, p.graphs, p.pair_lists, c, gY)
            cache[name] = (spec, inp, Y[0], L, grads)
        return cache[name]
    return get


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(TABLE1))
@pytest.mark.parametrize("R", [1, 8])
def test_table1_model_vs_oracle(oracle_r1, name, R):
    spec, inp, Yo, Lo, go = oracle_r1(name)
    part = inp.elem_part if R > 1 else np.zeros(inp.mesh.n_elem, np.int32)
    print(f"Table I {name} model, R={R}", flush=True)
    prob, Y, L, g = _gpu(spec, inp.params, inp, part, R)
    assert normwise(Y, Yo[prob.host.row_gid]) < 1e-4      # every copy = R=1 (Eq. 2)
    assert abs(L - Lo) / Lo < 1e-5
    for k in go:                                          # Eq. 3
        assert normwise(g[k], go[k]) < 1e-4, k


@pytest.mark.gpu
def test_table1_none_mode_differs(oracle_r1):
    spec, inp, Yo, Lo, go = oracle_r1("small")
    prob, Y, L, g = _gpu(spec, inp.params, inp, inp.elem_part, 8, halo=False)
    assert normwise(Y, Yo[prob.host.row_gid]) > 1e-3


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(TABLE1))
def test_table1_deterministic(name):
    spec, _ = TABLE1[name]
    inp = make_inputs(CONFIGS["C0"], perturb=True, spec=spec)
    runs = [_gpu(spec, inp.params, inp, inp.elem_part, 8) for _ in range(2)]
    assert np.array_equal(runs[0][1], runs[1][1])
    for k in runs[0][3]:
        assert np.array_equal(runs[0][3][k], runs[1][3][k]), k


# Other narrow deep MLPs: every tile count the fused edge adjoint is built
# for (3 to 12 weight tiles at H = 8 and 16), with and without LayerNorm.
VARIANTS = {"h8-nh0": ModelSpec(H=8, n_layers=2, n_hidden=0, layernorm=False),
            "h8-nh5-ln": ModelSpec(H=8, n_layers=2, n_hidden=5, layernorm=True),
            "h16-nh1-ln": ModelSpec(H=16, n_layers=2, n_hidden=1, layernorm=True),
            "h16-nh3": ModelSpec(H=16, n_layers=2, n_hidden=3, layernorm=False)}


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_deep_layer_variants_vs_oracle(name):
    spec = VARIANTS[name]
    inp = make_inputs(CONFIGS["C0"], perturb=True, spec=spec)
    p = build_problem(inp.mesh, inp.field, inp.target, None, 1)
    Yo, c = model_fwd(inp.params, spec, p.graphs, p.pair_lists, p.X, p.E0)
    Lo, gY, _ = consistent_loss(Yo, p.T, p.graphs)
    go, _ = model_bwd(inp.params, spec, p.graphs, p.pair_lists, c, gY)
    print(f"deep layer variant {name}, R=8", flush=True)
    prob, Y, L, g = _gpu(spec, inp.params, inp, inp.elem_part, 8)
    assert normwise(Y, Yo[0][prob.host.row_gid]) < 1e-4
    assert abs(L - Lo) / Lo < 1e-5
    for k in go:
        assert normwise(g[k], go[k]) < 1e-4, k


@pytest.mark.gpu
@pytest.mark.parametrize("H,NH", [(8, 2), (16, 1), (32, 5)])
def test_deep_mlp_h_to_h_vs_oracle(H, NH):
    """The H -> H form of the deep MLP entry point (not used by the model)."""
    from paper_2410_01657_amd.ops import DeepMLPFn, deep_mlp_cfg
    spec = ModelSpec(H=H, n_layers=1, n_hidden=NH, layernorm=True)
    full = init_params(spec, 5, perturb=True)
    pre = "mp0.node"
    # an H -> H MLP made from the node MLP's hidden and output layers
    rng = np.random.default_rng(3)
    W0 = rng.uniform(-0.3, 0.3, (H, H)).astype(np.float32)
    params = {f"{pre}.lin0.W": W0, f"{pre}.lin0.b": full[f"{pre}.lin0.b"]}
    for k in range(1, NH + 2):
        params[f"{pre}.lin{k}.W"] = full[f"{pre}.lin{k}.W"]
        params[f"{pre}.lin{k}.b"] = full[f"{pre}.lin{k}.b"]
    params[f"{pre}.ln.g"], params[f"{pre}.ln.b"] = full[f"{pre}.ln.g"], full[f"{pre}.ln.b"]
    n = 1000
    x = rng.standard_normal((n, H)).astype(np.float32)
    gy = rng.standard_normal((n, H)).astype(np.float32)
    y_o, cache = mlp_fwd(params, pre, x.astype(np.float64), spec, True)
    go = {}
    gx_o = mlp_bwd(params, pre, cache, gy.astype(np.float64), spec, True, go)
    names = [f"{pre}.lin{k}.{t}" for k in range(NH + 2) for t in ("W", "b")] + [f"{pre}.ln.g", f"{pre}.ln.b"]
    theta = torch.tensor(np.concatenate([params[k].reshape(-1) for k in names]), device="cuda",
                         requires_grad=True)
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    y = DeepMLPFn.apply(deep_mlp_cfg(H, H, NH, H, True), xt, theta)
    y.backward(torch.tensor(gy, device="cuda"))
    assert normwise(y.detach().cpu().numpy(), y_o) < 1e-5
    assert normwise(xt.grad.cpu().numpy(), gx_o) < 1e-5
    g = theta.grad.cpu().numpy()
    off = 0
    for k in names:
        sz = params[k].size
        assert normwise(g[off:off + sz].reshape(params[k].shape), go[k]) < 1e-5, k
        off += sz


@pytest.mark.gpu
@pytest.mark.parametrize("R", [1, 8])
def test_table1_small_with_seven_edge_inputs(R):
    """The seven-channel edge input (u_j - u_i added, Sec. III) with the small
    model: edge inputs bit-exact against the oracle's rounded FP64 values,
    then outputs, loss and gradients against the FP64 oracle at R = 1."""
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    spec = ModelSpec(H=8, n_layers=4, n_hidden=2, layernorm=True, edge_in=7)
    inp = make_inputs(CONFIGS["C0"], perturb=True, spec=spec)
    part = inp.elem_part if R > 1 else np.zeros(inp.mesh.n_elem, np.int32)
    prob = Problem(inp.mesh, inp.field, inp.target, part, R, "cuda", edge_in=7)
    o_r = build_problem(inp.mesh, inp.field, inp.target, part if R > 1 else None, R,
                        unpartitioned_from_lattice=False, edge_in=7)
    np.testing.assert_array_equal(prob.E0.cpu().numpy()[oracle_edge_order(prob.host)],
                                  np.concatenate(o_r.E0).astype(np.float32))
    p = build_problem(inp.mesh, inp.field, inp.target, None, 1, edge_in=7)
    Y, c = model_fwd(inp.params, spec, p.graphs, p.pair_lists, p.X, p.E0)
    Lo, gY, _ = consistent_loss(Y, p.T, p.graphs)
    go, _ = model_bwd(inp.params, spec, p.graphs, p.pair_lists, c, gY)
    model = ConsistentGNN(spec, inp.params, "cuda").requires_grad_(True)
    Yg = model.forward(prob.dg, prob.X, prob.E0)
    loss = model.loss(prob.dg, Yg, prob.T)
    loss.backward()
    assert normwise(Yg.detach().cpu().numpy(), Y[0][prob.host.row_gid]) < 1e-4
    assert abs(float(loss.detach()) - Lo) / Lo < 1e-5
    for k, t in model.params.items():
        assert normwise(t.grad.cpu().numpy(), go[k]) < 1e-4, k
