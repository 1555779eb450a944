"""Model parameter layout and seeded initialisation.

The encode-process-decode model of Sec. III (Table I):
  * node encoder MLP  (node_in -> H) with LayerNorm on its output,
  * edge encoder MLP  (edge_in -> H) with LayerNorm on its output,
  * M message-passing layers, each with an edge MLP (3H -> H) and a node MLP
    (2H -> H), both with LayerNorm on the output,
  * node decoder MLP (H -> out), no LayerNorm.
Every MLP is ``Linear(in, H)``, then ``n_hidden`` times ``Linear(H, H)``,
then ``Linear(H, out)``, with ELU after every Linear but the last.
Weights follow ``torch.nn.Linear``: ``W[out, in]``, ``b[out]``.

With (H, n_hidden) = (8, 2) and (32, 5), node_in = 3, edge_in = 4, out = 3
and M = 4 this layout has 3,979 and 91,459 parameters, the counts of the
paper's small and large models (Table I).
"""

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class ModelSpec:
    H: int = 32
    n_layers: int = 2
    n_hidden: int = 0        # extra Linear(H, H) layers inside each MLP
    layernorm: bool = False
    node_in: int = 3
    edge_in: int = 4
    out: int = 3
    ln_eps: float = 1e-5
    aggregate: str = "state"  # Eq. 4b sums the updated edge state e'; "message": the MLP output


def _mlp_shapes(prefix, fan_in, H, out, n_hidden, ln):
    dims = [fan_in] + [H] * (n_hidden + 1) + [out]
    shapes = []
    for k in range(len(dims) - 1):
        shapes.append((f"{prefix}.lin{k}.W", (dims[k + 1], dims[k])))
        shapes.append((f"{prefix}.lin{k}.b", (dims[k + 1],)))
    if ln:
        shapes.append((f"{prefix}.ln.g", (out,)))
        shapes.append((f"{prefix}.ln.b", (out,)))
    return shapes


def param_shapes(spec):
    """Ordered list of (name, shape); the order fixes the random stream."""
    H, L, ln = spec.H, spec.n_hidden, spec.layernorm
    s = []
    s += _mlp_shapes("nenc", spec.node_in, H, H, L, ln)
    s += _mlp_shapes("eenc", spec.edge_in, H, H, L, ln)
    for m in range(spec.n_layers):
        s += _mlp_shapes(f"mp{m}.edge", 3 * H, H, H, L, ln)
        s += _mlp_shapes(f"mp{m}.node", 2 * H, H, H, L, ln)
    s += _mlp_shapes("dec", H, H, spec.out, L, False)
    return s


def count_params(spec):
    return int(sum(int(np.prod(shape)) for _, shape in param_shapes(spec)))


def init_params(spec, seed, perturb=False):
    """Seeded parameters, generated in FP64 and rounded to FP32.

    Weights: Xavier-uniform with gain 1, U(-a, a), a = sqrt(6/(fan_in+fan_out)).
    Biases 0, LayerNorm gain 1 and shift 0.  With ``perturb`` the biases,
    gains and shifts are drawn too (U(-0.2, 0.2), U(0.5, 1.5), U(-0.2, 0.2))
    so that tests see every parameter act.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = {}
    for name, shape in param_shapes(spec):
        kind = name.rsplit(".", 1)[-1]
        if kind == "W":
            fo, fi = shape
            a = np.sqrt(6.0 / (fi + fo))
            v = rng.uniform(-a, a, size=shape)
        elif name.endswith(".ln.g"):
            v = rng.uniform(0.5, 1.5, size=shape) if perturb else np.ones(shape)
        else:  # biases and LayerNorm shifts
            v = rng.uniform(-0.2, 0.2, size=shape) if perturb else np.zeros(shape)
        out[name] = v.astype(np.float32)
    return out
