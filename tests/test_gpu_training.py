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
