"""Encode-process-decode GNN of consistent NMP layers (Sec. III, Table I).

Node encoder MLP (3 -> H), edge encoder MLP (4 -> H), M consistent
message-passing layers (Eq. 4a-e), node decoder MLP (H -> 3), and the
consistent MSE (Eq. 6).  Every piece runs through libmplayer.so.
"""

import dataclasses
import json

import numpy as np
import torch

from .graph import DeviceGraph, build_graph
from .autotune import apply_schedule
from .ops import (ConsistentMSEFn, DeepLayerFn, DeepMLPFn, MLPFn, MPLayerFn, deep_layer_cfg, deep_mlp_cfg,
                  edge_inputs, layer_cfg, mlp_cfg)


def _layer_param_names(m, ln):
    pre = f"mp{m}"
    names = {"We1": f"{pre}.edge.lin0.W", "be1": f"{pre}.edge.lin0.b",
             "We2": f"{pre}.edge.lin1.W", "be2": f"{pre}.edge.lin1.b",
             "Wn1": f"{pre}.node.lin0.W", "bn1": f"{pre}.node.lin0.b",
             "Wn2": f"{pre}.node.lin1.W", "bn2": f"{pre}.node.lin1.b"}
    if ln:
        names.update({"ge": f"{pre}.edge.ln.g", "bge": f"{pre}.edge.ln.b",
                      "gn": f"{pre}.node.ln.g", "bgn": f"{pre}.node.ln.b"})
    return names


def _mlp_param_names(prefix, ln):
    names = {"W0": f"{prefix}.lin0.W", "b0": f"{prefix}.lin0.b",
             "W1": f"{prefix}.lin1.W", "b1": f"{prefix}.lin1.b"}
    if ln:
        names.update({"ln_g": f"{prefix}.ln.g", "ln_b": f"{prefix}.ln.b"})
    return names


def save_checkpoint(path, params, spec, **meta):
    """Write a model to an .npz file that loads without unpickling: every
    parameter (name -> FP32 array, bitwise as held), the model description
    (the fields of the spec dataclass) and free-form metadata such as seeds,
    step counts or the learning rate, both as JSON text."""
    arrays = {}
    for k, v in params.items():
        t = v.detach().cpu().numpy() if isinstance(v, torch.Tensor) else np.asarray(v)
        arrays["param/" + k] = np.ascontiguousarray(t, dtype=np.float32)
    spec_fields = dataclasses.asdict(spec) if dataclasses.is_dataclass(spec) else dict(spec)
    arrays["spec"] = np.frombuffer(json.dumps(spec_fields, sort_keys=True).encode(), dtype=np.uint8)
    arrays["meta"] = np.frombuffer(json.dumps(meta, sort_keys=True).encode(), dtype=np.uint8)
    np.savez(path, **arrays)


def load_checkpoint(path):
    """Read a file written by save_checkpoint: (params as name -> FP32
    array, spec fields as a dict, metadata as a dict)."""
    with np.load(path, allow_pickle=False) as z:
        params = {k[len("param/"):]: z[k].copy() for k in z.files if k.startswith("param/")}
        spec_fields = json.loads(z["spec"].tobytes().decode())
        meta = json.loads(z["meta"].tobytes().decode())
    return params, spec_fields, meta


class ConsistentGNN:
    """Parameters live in ``self.params`` (name -> device tensor, FP32)."""

    LAYER_ORDER = ["We1", "be1", "We2", "be2", "ge", "bge", "Wn1", "bn1", "Wn2", "bn2", "gn", "bgn"]
    MLP_ORDER = ["W0", "b0", "W1", "b1", "ln_g", "ln_b"]

    def __init__(self, spec, params, device="cuda", gemm="f32", halo=True, schedule=None, estate="f32"):
        # Table I's narrow models (extra hidden layers, H = 8/16/32) run on
        # the deep-MLP kernels; two-Linear MLPs at H = 32/64/128 on the
        # matrix-core kernels.  estate: storage type of the edge states
        # between layers and of their gradients ("bf16" with gemm="bf16").
        self.deep = spec.n_hidden > 0 or spec.H in (8, 16)
        if self.deep and (gemm != "f32" or spec.H not in (8, 16, 32)):
            raise ValueError("deep MLPs run in FP32 at H = 8, 16 or 32")
        if estate not in ("f32", "bf16") or (estate == "bf16" and gemm != "bf16"):
            raise ValueError("estate is 'f32', or 'bf16' with gemm='bf16'")
        self.spec, self.gemm, self.halo, self.estate = spec, gemm, halo, estate
        # edge-kernel schedule: None (library defaults) or a dict of
        # mp_layer_cfg schedule fields (see autotune.SCHEDULE_FIELDS)
        self.schedule = schedule
        self.device = torch.device(device)
        self.params = {k: torch.as_tensor(np.asarray(v), dtype=torch.float32).to(self.device).contiguous()
                       for k, v in params.items()}

    def save(self, path, **meta):
        """Checkpoint the parameters, the spec and `meta` (see
        save_checkpoint); ConsistentGNN(spec, load_checkpoint(path)[0], ...)
        resumes from it."""
        save_checkpoint(path, self.params, self.spec, gemm=self.gemm, estate=self.estate, **meta)

    def requires_grad_(self, flag=True):
        for t in self.params.values():
            t.requires_grad_(flag)
        return self

    def _theta(self, prefix, ln):
        """The MLP's parameters as one flat tensor (differentiable)."""
        names = [f"{prefix}.lin{k}.{t}" for k in range(self.spec.n_hidden + 2) for t in ("W", "b")]
        if ln:
            names += [f"{prefix}.ln.g", f"{prefix}.ln.b"]
        return torch.cat([self.params[n].reshape(-1) for n in names])

    def _mlp(self, prefix, x, n_in, n_out, ln, out="f32"):
        if self.deep:
            s = self.spec
            cfg = deep_mlp_cfg(n_in, s.H, s.n_hidden, n_out, ln, s.ln_eps)
            return DeepMLPFn.apply(cfg, x, self._theta(prefix, ln))
        names = _mlp_param_names(prefix, ln)
        cfg = mlp_cfg(n_in, self.spec.H, n_out, ln, self.gemm, self.spec.ln_eps, out)
        args = [self.params[names[f]] if f in names else None for f in self.MLP_ORDER]
        return MLPFn.apply(cfg, x, *args)

    def encode(self, X, E0):
        s = self.spec
        x = self._mlp("nenc", X, s.node_in, s.H, s.layernorm)
        e = self._mlp("eenc", E0, s.edge_in, s.H, s.layernorm, self.estate)  # an edge state
        return x, e

    def process(self, dg, x, e, want_e=False):
        """The message-passing layers.  The last layer's edge state is
        returned only when want_e (nothing in the model reads it, so by
        default it is not written)."""
        s = self.spec
        if self.deep:
            cfg = deep_layer_cfg(s.H, s.n_hidden, s.layernorm, self.halo, s.ln_eps, s.aggregate)
            for m in range(s.n_layers):
                x, e = DeepLayerFn.apply(cfg, dg, x, e, self._theta(f"mp{m}.edge", s.layernorm),
                                         self._theta(f"mp{m}.node", s.layernorm))
            return x, e
        cfg = layer_cfg(s.H, s.layernorm, self.halo, self.gemm, s.ln_eps, s.aggregate, self.estate)
        if self.schedule:
            apply_schedule(cfg, self.schedule)
        for m in range(s.n_layers):
            names = _layer_param_names(m, s.layernorm)
            args = [self.params[names[f]] if f in names else None for f in self.LAYER_ORDER]
            last = m == s.n_layers - 1
            x, e = MPLayerFn.apply(cfg, dg, want_e or not last, x, e, *args)
        return x, e

    def decode(self, x):
        return self._mlp("dec", x, self.spec.H, self.spec.out, False)

    def forward(self, dg, X, E0):
        x, e = self.encode(X, E0)
        x, _ = self.process(dg, x, e)
        return self.decode(x)

    def loss(self, dg, Y, T):
        return ConsistentMSEFn.apply(dg, Y, T)


class Problem:
    """Device graph, node inputs, edge inputs and target for one workload."""

    def __init__(self, mesh, field, target, elem_part, R, device="cuda", edge_in=4):
        self.host = build_graph(mesh.elem_gid, mesh.P, elem_part, R, getattr(mesh, "links", None))
        self.dg = DeviceGraph(self.host, device)
        self.X = self.dg.rows_of(field).float().contiguous()
        self.T = self.dg.rows_of(target).float().contiguous()
        self.pos = self.dg.rows_of(mesh.pos).double().contiguous()
        # 4 edge channels (p_j - p_i, |p_j - p_i|), or 7 with u_j - u_i
        self.E0 = edge_inputs(self.dg, self.pos, getattr(mesh, "period", None),
                              self.X if edge_in == 7 else None)
