"""Shared helpers for the GPU parity tests."""

import numpy as np

from mpinputs import ModelSpec, init_params


def normwise(a, b):
    """max|a - b| / max|b| over all entries (the tolerance norm used throughout)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def layer_params(H, ln, seed=3, perturb=True):
    """Parameters of one layer, as (oracle dict keyed by model names,
    library dict keyed by ABI field names)."""
    spec = ModelSpec(H=H, n_layers=1, layernorm=ln)
    full = init_params(spec, seed, perturb=perturb)
    o = {k: v for k, v in full.items() if k.startswith("mp0.")}
    names = {"We1": "mp0.edge.lin0.W", "be1": "mp0.edge.lin0.b", "We2": "mp0.edge.lin1.W",
             "be2": "mp0.edge.lin1.b", "Wn1": "mp0.node.lin0.W", "bn1": "mp0.node.lin0.b",
             "Wn2": "mp0.node.lin1.W", "bn2": "mp0.node.lin1.b"}
    if ln:
        names.update({"ge": "mp0.edge.ln.g", "bge": "mp0.edge.ln.b", "gn": "mp0.node.ln.g",
                      "bgn": "mp0.node.ln.b"})
    return spec, o, names


def split_rows(a, off):
    return [a[off[r]:off[r + 1]] for r in range(len(off) - 1)]


def oracle_row_order(host):
    """Permutation that puts a host graph's rows in the oracle's order
    (sub-graph by sub-graph, ascending global id): rows[perm] lines up with
    the oracle's concatenated rows whatever numbering the library chose."""
    off = host.row_off
    return np.concatenate([off[r] + np.argsort(host.row_gid[off[r]:off[r + 1]], kind="stable")
                           for r in range(len(off) - 1)])


def oracle_edge_order(host):
    """Permutation that puts a host graph's edges in the oracle's order
    (sub-graph by sub-graph, by receiver then sender global id)."""
    parts = []
    for r in range(len(host.edge_off) - 1):
        e0, e1 = host.edge_off[r], host.edge_off[r + 1]
        gi, gj = host.row_gid[host.recv[e0:e1]], host.row_gid[host.col[e0:e1]]
        parts.append(e0 + np.lexsort((gj, gi)))
    return np.concatenate(parts)


def by_gid(host, Y):
    """Rows of a one-sub-graph run, indexed by global id."""
    out = np.zeros((int(host.row_gid.max()) + 1,) + Y.shape[1:], Y.dtype)
    out[host.row_gid] = Y
    return out

