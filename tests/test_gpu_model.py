"""GPU parity of the whole encode-process-decode model (forward, loss,
backward) against the FP64 oracle, R-consistency on the GPU, and
sampled-node parity at full workload size."""

import numpy as np
import pytest
import torch

from mpinputs import CONFIGS, ModelSpec, init_params, make_inputs
from oracle.ball import ball_output
from oracle.nmp import consistent_loss, model_bwd, model_fwd
from oracle.problem import build_problem

from _util import by_gid, normwise, oracle_row_order

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _gpu_run(spec, params, inp, part, R, gemm="f32", backward=True, estate="f32"):
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    prob = Problem(inp.mesh, inp.field, inp.target, part, R, DEV)
    model = ConsistentGNN(spec, params, DEV, gemm=gemm, estate=estate).requires_grad_(backward)
    Y = model.forward(prob.dg, prob.X, prob.E0)
    loss = model.loss(prob.dg, Y, prob.T)
    grads = None
    if backward:
        loss.backward()
        grads = {k: v.grad.cpu().numpy() for k, v in model.params.items()}
    return prob, Y.detach().cpu().numpy(), float(loss.detach().cpu()), grads


def _oracle_run(spec, params, inp, part, R):
    prob = build_problem(inp.mesh, inp.field, inp.target, part, R)
    Y, cache = model_fwd(params, spec, prob.graphs, prob.pair_lists, prob.X, prob.E0)
    L, gY, _ = consistent_loss(Y, prob.T, prob.graphs)
    grads, _ = model_bwd(params, spec, prob.graphs, prob.pair_lists, cache, gY)
    return np.concatenate(Y), L, grads


MODELS = {
    # the tiny workload's own model
    "C0": ModelSpec(H=32, n_layers=2, layernorm=False),
    # the fwd+bwd workload's model (H=128, LayerNorm) on the 4^3 mesh
    "C3-model": ModelSpec(H=128, n_layers=4, layernorm=True),
    "H64-LN": ModelSpec(H=64, n_layers=4, layernorm=True),
}


@pytest.mark.parametrize("model", ["C0", "C3-model", "H64-LN"])
@pytest.mark.parametrize("R", [1, 8])
def test_model_fwd_bwd_fp32(model, R):
    spec = MODELS[model]
    inp = make_inputs(CONFIGS["C0"], perturb=True, spec=spec)
    part = inp.elem_part if R > 1 else None
    prob, Yg, Lg, gg = _gpu_run(spec, inp.params, inp, part if R > 1 else np.zeros(inp.mesh.n_elem, np.int32), R)
    Yg = Yg[oracle_row_order(prob.dg.host)]
    Yo, Lo, go = _oracle_run(spec, inp.params, inp, part, R)
    tol_y = 1e-5 if model == "C0" else 1e-4
    assert normwise(Yg, Yo) < tol_y
    assert abs(Lg - Lo) / abs(Lo) < 1e-5
    for k in go:
        err = normwise(gg[k], go[k])
        assert err < 1e-4, (k, err)


def test_model_bf16_error_bounded():
    spec = MODELS["H64-LN"]
    inp = make_inputs(CONFIGS["C0"], perturb=True, spec=spec)
    prob, Yg, Lg, gg = _gpu_run(spec, inp.params, inp, inp.elem_part, 8, gemm="bf16")
    Yg = Yg[oracle_row_order(prob.dg.host)]
    Yo, Lo, go = _oracle_run(spec, inp.params, inp, inp.elem_part, 8)
    assert normwise(Yg, Yo) < 3e-2
    assert abs(Lg - Lo) / abs(Lo) < 3e-2
    errs = {k: normwise(gg[k], go[k]) for k in go}
    worst = max(errs, key=errs.get)
    print(f"C0 H64-LN BF16: output {normwise(Yg, Yo):.2e}, worst parameter gradient {errs[worst]:.2e} ({worst})")
    assert errs[worst] < 5e-2, (worst, errs[worst])


@pytest.mark.parametrize("model", ["H64-LN", "C3-model"])
def test_model_bf16_edge_state_error_bounded(model):
    """The model with BF16 GEMMs and BF16 edge states (encoder output,
    layer edge states and their gradients) against the FP64 oracle, at the
    BF16 tolerances."""
    spec = MODELS[model]
    inp = make_inputs(CONFIGS["C0"], perturb=True, spec=spec)
    prob, Yg, Lg, gg = _gpu_run(spec, inp.params, inp, inp.elem_part, 8, gemm="bf16", estate="bf16")
    Yg = Yg[oracle_row_order(prob.dg.host)]
    Yo, Lo, go = _oracle_run(spec, inp.params, inp, inp.elem_part, 8)
    assert normwise(Yg, Yo) < 3e-2
    assert abs(Lg - Lo) / abs(Lo) < 3e-2
    errs = {k: normwise(gg[k], go[k]) for k in go}
    worst = max(errs, key=errs.get)
    print(f"C0 {model} BF16 edge states: output {normwise(Yg, Yo):.2e}, worst parameter gradient "
          f"{errs[worst]:.2e} ({worst})")
    assert errs[worst] < 5e-2, (worst, errs[worst])


@pytest.mark.parametrize("H,ln", [(64, True), (128, False)])
def test_edge_encoder_bf16_output_is_the_rounded_fp32_output(H, ln):
    """The edge encoder (4 inputs -> H) with a BF16 output stores the FP32
    output rounded to nearest even, and its adjoint given a BF16 output
    gradient equals the adjoint given that gradient in FP32, bitwise."""
    from paper_2410_01657_amd.ops import mlp_backward, mlp_cfg, mlp_forward
    rng = np.random.default_rng(H)
    n = 1000
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)
    p = {"W0": t(rng.standard_normal((H, 4)) * 0.5), "b0": t(rng.standard_normal(H) * 0.1),
         "W1": t(rng.standard_normal((H, H)) / H ** 0.5), "b1": t(rng.standard_normal(H) * 0.1)}
    if ln:
        p.update({"ln_g": t(1 + 0.1 * rng.standard_normal(H)), "ln_b": t(0.1 * rng.standard_normal(H))})
    x = t(rng.standard_normal((n, 4)))
    c32, c16 = mlp_cfg(4, H, H, ln, "bf16"), mlp_cfg(4, H, H, ln, "bf16", out="bf16")
    y32, y16 = mlp_forward(c32, p, x), mlp_forward(c16, p, x)
    assert y16.dtype == torch.bfloat16 and torch.equal(y32.to(torch.bfloat16), y16)
    g16 = t(rng.standard_normal((n, H))).to(torch.bfloat16)
    _, gr32 = mlp_backward(c32, p, x, g16.float(), False)
    _, gr16 = mlp_backward(c16, p, x, g16, False)
    for k in p:
        assert torch.equal(gr32[k], gr16[k]), k


def test_r_consistency_gpu_c0():
    """Eq. 2 and 3 on the GPU: R=8 copies match R=1 at the same global id,
    and the parameter gradients match."""
    spec = MODELS["H64-LN"]
    inp = make_inputs(CONFIGS["C0"], perturb=True, spec=spec)
    p1, Y1, L1, g1 = _gpu_run(spec, inp.params, inp, np.zeros(inp.mesh.n_elem, np.int32), 1)
    p8, Y8, L8, g8 = _gpu_run(spec, inp.params, inp, inp.elem_part, 8)
    assert normwise(Y8, by_gid(p1.dg.host, Y1)[p8.dg.host.row_gid]) < 1e-5
    assert abs(L8 - L1) / abs(L1) < 1e-5
    for k in g1:
        assert normwise(g8[k], g1[k]) < 1e-4, k


def test_none_mode_is_inconsistent_gpu():
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    spec = MODELS["H64-LN"]
    inp = make_inputs(CONFIGS["C0"], perturb=True, spec=spec)
    p1 = Problem(inp.mesh, inp.field, inp.target, np.zeros(inp.mesh.n_elem, np.int32), 1, DEV)
    p8 = Problem(inp.mesh, inp.field, inp.target, inp.elem_part, 8, DEV)
    with torch.no_grad():
        Y1 = ConsistentGNN(spec, inp.params, DEV).forward(p1.dg, p1.X, p1.E0).cpu().numpy()
        Y8 = ConsistentGNN(spec, inp.params, DEV, halo=False).forward(p8.dg, p8.X, p8.E0).cpu().numpy()
    assert normwise(Y8, by_gid(p1.dg.host, Y1)[p8.dg.host.row_gid]) > 1e-2


@pytest.mark.slow
def test_c1_consistency_and_sampled_parity():
    """Full C1 size (531k nodes, 3.1M edges, 4 layers, H=64, LayerNorm):
    R=16 slabs match R=1 (1e-5), and 48 seeded nodes match the oracle
    evaluated exactly on their 4-hop balls (1e-4)."""
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    cfg = CONFIGS["C1"]
    inp = make_inputs(cfg, perturb=True)
    outs = {}
    for R, part in ((1, np.zeros(inp.mesh.n_elem, np.int32)), (16, inp.elem_part)):
        prob = Problem(inp.mesh, inp.field, inp.target, part, R, DEV)
        with torch.no_grad():
            Y = ConsistentGNN(cfg.spec, inp.params, DEV).forward(prob.dg, prob.X, prob.E0)
        outs[R] = (prob.dg.host.row_gid, Y.cpu().numpy())
        if R == 1:
            outs[R] = (None, by_gid(prob.dg.host, outs[R][1]))
        del prob
    gid16, Y16 = outs[16]
    _, Y1 = outs[1]
    assert normwise(Y16, Y1[gid16]) < 1e-5
    rng = np.random.default_rng(17)
    n = inp.mesh.npts[0]
    centers = list(rng.integers(0, inp.mesh.n_gid, 40)) + [0, n - 1, n * n * n - 1, n * n * (n // 2),
                                                           (n // 2) * (1 + n + n * n), 5, 5 * n, 5 * n * n]
    got = np.stack([Y1[c] for c in centers])
    ref = np.stack([ball_output(inp.params, cfg.spec, inp.mesh, inp.field, int(c)) for c in centers])
    assert normwise(got, ref) < 1e-4
