"""Oracle: consistent NMP layer, encode-process-decode model, losses, adjoints.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain NumPy float64.

Readings of the paper that this file fixes (all listed in the design notes):
* Eq. 4a is a residual update: the edge state becomes e + MLP([x_i, x_j, e])
  with i the receiver and j the sender, and Eq. 4b sums that updated state.
* Eq. 4e is a residual update: x becomes x + MLP([a*_i, x_i]).
* MLP = Linear, then ELU (alpha = 1) after every Linear but the last, then
  LayerNorm (biased variance, eps from the model spec) on the output of the
  encoder and processor MLPs when the model uses LayerNorm (Sec. III).
* Edge inputs: (p_j - p_i, |p_j - p_i|), four channels.
* The halo exchange adds, to every copy of a global id, the local aggregates
  of all other copies (Eq. 4c swap, then Eq. 4d sum over rows of equal id).
"""

import numpy as np

# --------------------------------------------------------------------------
# Elementary operations and their adjoints
# --------------------------------------------------------------------------


def elu(z):
    return np.where(z > 0, z, np.expm1(np.minimum(z, 0.0)))


def elu_deriv(z):
    return np.where(z > 0, 1.0, np.exp(np.minimum(z, 0.0)))


def layer_norm_fwd(z, g, b, eps):
    mu = z.mean(axis=-1, keepdims=True)
    var = ((z - mu) ** 2).mean(axis=-1, keepdims=True)
    inv = 1.0 / np.sqrt(var + eps)
    zh = (z - mu) * inv
    return g * zh + b, (zh, inv)


def layer_norm_bwd(gy, g, cache):
    """Vector-Jacobian product of y = g * (z - mean)/sqrt(var + eps) + b."""
    zh, inv = cache
    gzh = gy * g
    H = zh.shape[-1]
    gz = inv * (gzh - gzh.sum(-1, keepdims=True) / H
                - zh * (gzh * zh).sum(-1, keepdims=True) / H)
    return gz, (gy * zh).sum(0), gy.sum(0)


def _p(params, name):
    return np.asarray(params[name], dtype=np.float64)


def n_linears(spec):
    return spec.n_hidden + 2


def mlp_fwd(params, prefix, x, spec, ln):
    """MLP of Sec. III on rows of x; returns output and a cache for mlp_bwd."""
    cache = {"in": [], "pre": []}
    h = x
    nl = n_linears(spec)
    for k in range(nl):
        W, b = _p(params, f"{prefix}.lin{k}.W"), _p(params, f"{prefix}.lin{k}.b")
        cache["in"].append(h)
        z = h @ W.T + b
        if k < nl - 1:
            cache["pre"].append(z)
            h = elu(z)
        else:
            h = z
    if ln:
        h, cache["ln"] = layer_norm_fwd(h, _p(params, f"{prefix}.ln.g"),
                                        _p(params, f"{prefix}.ln.b"), spec.ln_eps)
    return h, cache


def mlp_bwd(params, prefix, cache, gy, spec, ln, grads):
    """Adjoint of mlp_fwd; accumulates parameter gradients into ``grads``."""
    nl = n_linears(spec)
    g = gy
    if ln:
        g, gg, gb = layer_norm_bwd(g, _p(params, f"{prefix}.ln.g"), cache["ln"])
        _acc(grads, f"{prefix}.ln.g", gg)
        _acc(grads, f"{prefix}.ln.b", gb)
    for k in reversed(range(nl)):
        if k < nl - 1:
            g = g * elu_deriv(cache["pre"][k])
        W = _p(params, f"{prefix}.lin{k}.W")
        _acc(grads, f"{prefix}.lin{k}.W", g.T @ cache["in"][k])
        _acc(grads, f"{prefix}.lin{k}.b", g.sum(0))
        g = g @ W
    return g


def _acc(grads, name, v):
    if name in grads:
        grads[name] = grads[name] + v
    else:
        grads[name] = np.array(v, dtype=np.float64)


# --------------------------------------------------------------------------
# Graph operations (Eq. 4b-d) and their adjoints
# --------------------------------------------------------------------------


def edge_inputs(graph, pos, period=None, field=None):
    """Four edge input channels (p_j - p_i, |p_j - p_i|) per directed edge,
    and with a node field u (per global id) three more, u_j - u_i: the
    relative velocity Sec. III lists among the edge features.

    On a periodic axis of length L > 0 the difference is that of the nearest
    periodic image of p_j (the element-local difference; a link never spans
    half a period)."""
    dp = pos[graph.gid[graph.send]] - pos[graph.gid[graph.recv]]
    for ax, L in enumerate(period or ()):
        if L > 0:
            dp[:, ax] -= L * np.round(dp[:, ax] / L)
    cols = [dp, np.linalg.norm(dp, axis=1, keepdims=True)]
    if field is not None:
        u = np.asarray(field, np.float64)
        cols.append(u[graph.gid[graph.send]] - u[graph.gid[graph.recv]])
    return np.concatenate(cols, axis=1)


def local_aggregate(e, graph):
    """Eq. 4b: a_i = sum over edges into i of e_ij / d_ij."""
    a = np.zeros((graph.n, e.shape[1]))
    np.add.at(a, graph.recv, e / graph.d_edge[:, None])
    return a


def local_aggregate_adj(ga, graph):
    """Adjoint of Eq. 4b: g_e_ij = g_a_i / d_ij."""
    return ga[graph.recv] / graph.d_edge[:, None]


def halo_sync(a_list, pair_lists):
    """Eq. 4c (swap) then Eq. 4d (sum over rows of equal global id).

    Sub-graph r appends one halo row per (neighbour s, shared id): the local
    aggregate of s's copy (the receive buffer, filled from s's send mask).
    Synchronisation then adds each halo row to r's own row of that id.
    """
    out = [a.copy() for a in a_list]
    for (r, s), (rows_r, rows_s) in pair_lists.items():
        halo_rows = a_list[s][rows_s]          # receive buffer on r from s
        np.add.at(out[r], rows_r, halo_rows)  # sync: sum rows of equal id
    return out


def halo_sync_adj(g_list, pair_lists):
    """Adjoint of halo_sync: each halo row's gradient returns to the sender
    row it came from (the reverse exchange).  The map is symmetric, so the
    adjoint has the same form as the forward."""
    out = [g.copy() for g in g_list]
    for (r, s), (rows_r, rows_s) in pair_lists.items():
        np.add.at(out[s], rows_s, g_list[r][rows_r])
    return out


# --------------------------------------------------------------------------
# One consistent NMP layer (Eq. 4a-e) over all sub-graphs
# --------------------------------------------------------------------------


def nmp_layer_fwd(params, m, spec, graphs, pair_lists, x_list, e_list, halo=True):
    ln = spec.layernorm
    pre = f"mp{m}"
    cache = {"edge": [], "node": [], "x": x_list, "e": e_list}
    e_new, a_list = [], []
    for r, G in enumerate(graphs):
        x, e = x_list[r], e_list[r]
        inp = np.concatenate([x[G.recv], x[G.send], e], axis=1)     # Eq. 4a
        msg, c = mlp_fwd(params, pre + ".edge", inp, spec, ln)
        cache["edge"].append(c)
        e2 = e + msg
        e_new.append(e2)
        # Eq. 4b sums the updated edge state; the "message" variant sums the
        # MLP output alone
        a_list.append(local_aggregate(msg if spec.aggregate == "message" else e2, G))
    a_star = halo_sync(a_list, pair_lists) if halo else a_list         # Eq. 4c-d
    x_new = []
    for r, G in enumerate(graphs):
        inp = np.concatenate([a_star[r], x_list[r]], axis=1)           # Eq. 4e
        upd, c = mlp_fwd(params, pre + ".node", inp, spec, ln)
        cache["node"].append(c)
        x_new.append(x_list[r] + upd)
    cache["a_star"] = a_star
    cache["halo"] = halo
    return x_new, e_new, cache


def nmp_layer_bwd(params, m, spec, graphs, pair_lists, cache, gx_list, ge_list, grads):
    ln = spec.layernorm
    pre = f"mp{m}"
    H = spec.H
    ga_star, gx_in = [], []
    for r, G in enumerate(graphs):
        gin = mlp_bwd(params, pre + ".node", cache["node"][r], gx_list[r], spec, ln, grads)
        ga_star.append(gin[:, :H])
        gx_in.append(gx_list[r] + gin[:, H:])
    ga = halo_sync_adj(ga_star, pair_lists) if cache["halo"] else ga_star
    ge_in = []
    for r, G in enumerate(graphs):
        # gradient at the MLP output: through e' = e + MLP and through Eq. 4b
        gmsg = ge_list[r] + local_aggregate_adj(ga[r], G)
        gin = mlp_bwd(params, pre + ".edge", cache["edge"][r], gmsg, spec, ln, grads)
        gx = gx_in[r]
        np.add.at(gx, G.recv, gin[:, :H])
        np.add.at(gx, G.send, gin[:, H:2 * H])
        # the residual path carries the gradient of e' (which includes Eq.
        # 4b's when e' is what is summed)
        g_res = ge_list[r] if spec.aggregate == "message" else gmsg
        ge_in.append(g_res + gin[:, 2 * H:])
    return gx_in, ge_in


# --------------------------------------------------------------------------
# Encode-process-decode model (Sec. III) and losses (Eq. 5, Eq. 6)
# --------------------------------------------------------------------------


def model_fwd(params, spec, graphs, pair_lists, X_list, E0_list, halo=True):
    ln = spec.layernorm
    cache = {"nenc": [], "eenc": [], "layers": [], "dec": []}
    x_list, e_list = [], []
    for r in range(len(graphs)):
        x, c = mlp_fwd(params, "nenc", np.asarray(X_list[r], np.float64), spec, ln)
        cache["nenc"].append(c)
        e, c = mlp_fwd(params, "eenc", np.asarray(E0_list[r], np.float64), spec, ln)
        cache["eenc"].append(c)
        x_list.append(x)
        e_list.append(e)
    for m in range(spec.n_layers):
        x_list, e_list, c = nmp_layer_fwd(params, m, spec, graphs, pair_lists,
                                          x_list, e_list, halo)
        cache["layers"].append(c)
    Y = []
    for r in range(len(graphs)):
        y, c = mlp_fwd(params, "dec", x_list[r], spec, False)
        cache["dec"].append(c)
        Y.append(y)
    return Y, cache


def model_bwd(params, spec, graphs, pair_lists, cache, gY_list):
    grads = {}
    gx = [mlp_bwd(params, "dec", cache["dec"][r], gY_list[r], spec, False, grads)
          for r in range(len(graphs))]
    ge = [np.zeros((G.e, spec.H)) for G in graphs]
    for m in reversed(range(spec.n_layers)):
        gx, ge = nmp_layer_bwd(params, m, spec, graphs, pair_lists,
                               cache["layers"][m], gx, ge, grads)
    gX = []
    for r in range(len(graphs)):
        gX.append(mlp_bwd(params, "nenc", cache["nenc"][r], gx[r], spec, spec.layernorm, grads))
        mlp_bwd(params, "eenc", cache["eenc"][r], ge[r], spec, spec.layernorm, grads)
    return grads, gX


def mse_loss(Y, T):
    """Eq. 5 on the unpartitioned graph; returns loss and dL/dY."""
    N, F = Y.shape
    d = Y - T
    return float((d * d).sum() / (N * F)), 2.0 * d / (N * F)


def consistent_loss(Y_list, T_list, graphs):
    """Eq. 6a-c: degree-weighted squared error summed over sub-graphs
    (the AllReduce of S_r) over F times N_eff (the AllReduce of N_r)."""
    F = Y_list[0].shape[1]
    S = [((1.0 / G.d_node)[:, None] * (Y - T) ** 2).sum()
         for Y, T, G in zip(Y_list, T_list, graphs)]
    Nr = [(1.0 / G.d_node).sum() for G in graphs]
    n_eff = float(np.sum(Nr))
    L = float(np.sum(S)) / (n_eff * F)
    gY = [2.0 * (1.0 / G.d_node)[:, None] * (Y - T) / (n_eff * F)
          for Y, T, G in zip(Y_list, T_list, graphs)]
    return L, gY, n_eff
