"""Exact single-node evaluation on the receptive field (oracle, sampled parity).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

After M message-passing layers, the output at node c depends only on the
inputs of nodes within M hops of c and the edges among them: x^l at a node
at distance k needs x^(l-1) of its neighbours (distance <= k+1), so every
quantity c's output uses is complete inside the ball of radius M.  On the
box lattice, hop distance is the Manhattan distance of lattice indices
(taken modulo the period on a periodic axis).
Evaluating the unpartitioned model on that ball therefore gives the exact
R=1 output at c (Eq. 2 states every partitioned run must reproduce it).
"""

import numpy as np

from .graph import SubGraph
from .nmp import model_fwd, model_bwd, edge_inputs


def ball_graph(npts, center, radius, periodic=(False, False, False)):
    """The lattice nodes within ``radius`` hops of ``center`` (indices wrap on
    periodic axes, which must hold at least 2*radius+1 points) and the links
    among them, as a one-sub-graph SubGraph; also the centre's row."""
    n = npts
    c0 = (center % n[0], (center // n[0]) % n[1], center // (n[0] * n[1]))
    r = radius
    off = np.arange(-r, r + 1)
    di, dj, dk = np.meshgrid(off, off, off, indexing="ij")
    near = np.abs(di) + np.abs(dj) + np.abs(dk) <= r
    idx = []
    ok = near.copy()
    for ax, d in enumerate((di, dj, dk)):
        v = c0[ax] + d
        if periodic[ax]:
            if n[ax] < 2 * r + 1:
                raise ValueError("periodic axis too short for the ball")
            v = v % n[ax]
        else:
            ok &= (v >= 0) & (v < n[ax])
        idx.append(v)
    ii, jj, kk = (v[ok] for v in idx)
    gid = np.sort(ii + n[0] * (jj + n[1] * kk.astype(np.int64)))
    index = {g: k for k, g in enumerate(gid.tolist())}
    recv, send = [], []
    for g in gid.tolist():
        p = [g % n[0], (g // n[0]) % n[1], g // (n[0] * n[1])]
        for ax in range(3):
            for step in (1, -1):
                q = list(p)
                q[ax] += step
                if periodic[ax]:
                    q[ax] %= n[ax]
                elif not 0 <= q[ax] < n[ax]:
                    continue
                h = q[0] + n[0] * (q[1] + n[1] * q[2])
                if h in index:
                    recv.append(index[g])
                    send.append(index[h])
    recv = np.array(recv, dtype=np.int64)
    send = np.array(send, dtype=np.int64)
    order = np.lexsort((send, recv))
    return SubGraph(gid, recv[order], send[order], np.ones(len(recv)), np.ones(len(gid))), index[center]


def _ball(params, spec, mesh, field, center):
    G, c = ball_graph(mesh.npts, center, spec.n_layers, mesh.periodic)
    X = np.asarray(field, np.float64)[G.gid]
    Y, cache = model_fwd(params, spec, [G], {}, [X], [edge_inputs(G, mesh.pos, mesh.period)])
    return G, c, Y, cache


def ball_output(params, spec, mesh, field, center):
    """Exact R=1 model output [out] at global id ``center``."""
    _, c, Y, _ = _ball(params, spec, mesh, field, center)
    return Y[0][c]


def ball_grad(params, spec, mesh, field, center, weight):
    """Exact gradient of <weight, Y_center> with respect to every parameter."""
    G, c, Y, cache = _ball(params, spec, mesh, field, center)
    gY = np.zeros_like(Y[0])
    gY[c] = weight
    grads, _ = model_bwd(params, spec, [G], {}, cache, [gY])
    return Y[0][c], grads
