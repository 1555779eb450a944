"""Training consistency (Eq. 3 in use): plain SGD on the consistent loss
(Eq. 6) gives the same loss curve for the unpartitioned graph and for 8
sub-graphs with the halo exchange, and a different one without it (the
"None" mode), as the paper's training demonstration describes (Sec. III-A).
Target = input field, as in that demonstration.
"""

import numpy as np
import pytest
import torch

from mpinputs import CONFIGS, ModelSpec, make_inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _curve(inp, spec, part, R, halo, steps=20, lr=0.002):
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    prob = Problem(inp.mesh, inp.field, inp.field, part, R, DEV)
    model = ConsistentGNN(spec, inp.params, DEV, halo=halo).requires_grad_(True)
    losses = []
    for _ in range(steps):
        for t in model.params.values():
            t.grad = None
        loss = model.loss(prob.dg, model.forward(prob.dg, prob.X, prob.E0), prob.T)
        loss.backward()
        with torch.no_grad():
            for t in model.params.values():
                t -= lr * t.grad
        losses.append(float(loss.detach()))
    return np.array(losses)


def test_training_curves_r1_vs_r8():
    spec = ModelSpec(H=32, n_layers=4, layernorm=True)
    inp = make_inputs(CONFIGS["C0"], spec=spec)
    l1 = _curve(inp, spec, np.zeros(inp.mesh.n_elem, np.int32), 1, True)
    l8 = _curve(inp, spec, inp.elem_part, 8, True)
    l8n = _curve(inp, spec, inp.elem_part, 8, False)
    assert l1[-1] < 0.5 * l1[0]                         # it trains
    assert np.max(np.abs(l8 - l1) / l1) < 1e-4          # consistent
    assert np.max(np.abs(l8n - l1) / l1) > 1e-2         # "None" mode is not


def test_checkpoint_resume_is_bitwise(tmp_path):
    # 3 SGD steps, checkpoint, reload into a fresh model, 2 more steps ==
    # 5 steps straight (deterministic kernels, no atomics)
    from paper_2410_01657_amd.model import ConsistentGNN, Problem, load_checkpoint
    spec = ModelSpec(H=32, n_layers=2, layernorm=True)
    inp = make_inputs(CONFIGS["C0"], spec=spec)
    prob = Problem(inp.mesh, inp.field, inp.field, inp.elem_part, 8, DEV)

    def steps(model, n, lr=0.002):
        out = []
        for _ in range(n):
            for t in model.params.values():
                t.grad = None
            loss = model.loss(prob.dg, model.forward(prob.dg, prob.X, prob.E0), prob.T)
            loss.backward()
            with torch.no_grad():
                for t in model.params.values():
                    t -= lr * t.grad
            out.append(float(loss.detach()))
        return out

    straight = ConsistentGNN(spec, inp.params, DEV).requires_grad_(True)
    l_straight = steps(straight, 5)
    first = ConsistentGNN(spec, inp.params, DEV).requires_grad_(True)
    l_first = steps(first, 3)
    path = tmp_path / "ckpt.npz"
    first.save(path, step=3, lr=0.002)
    params, spec_fields, meta = load_checkpoint(path)
    assert meta["step"] == 3 and ModelSpec(**spec_fields) == spec
    resumed = ConsistentGNN(spec, params, DEV).requires_grad_(True)
    l_resumed = steps(resumed, 2)
    assert l_first + l_resumed == l_straight
    for k, t in straight.params.items():
        assert torch.equal(t.detach(), resumed.params[k].detach()), k
