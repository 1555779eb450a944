"""Exact single-node evaluation on the receptive field (oracle, sampled parity).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

After M message-passing layers, the output at node c depends only on the
inputs of nodes within M hops of c and the edges among them: x^l at a node
at distance k needs x^(l-1) of its neighbours (distance <= k+1), so every
quantity c's output uses is complete inside the ball of radius M.  On the
box lattice, hop distance is the Manhattan distance of lattice indices.
Evaluating the unpartitioned model on that ball therefore gives the exact
R=1 output at c (Eq. 2 states every partitioned run must reproduce it).
"""

import numpy as np

from .graph import SubGraph
from .nmp import model_fwd, model_bwd, edge_inputs


def ball_graph(npts, center, radius):
    nx, ny, nz = npts
    ci, cj, ck = center % nx, (center // nx) % ny, center // (nx * ny)
    r = radius
    ii, jj, kk = np.meshgrid(np.arange(ci - r, ci + r + 1), np.arange(cj - r, cj + r + 1),
                             np.arange(ck - r, ck + r + 1), indexing="ij")
    ok = ((np.abs(ii - ci) + np.abs(jj - cj) + np.abs(kk - ck) <= r)
          & (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny) & (kk >= 0) & (kk < nz))
    gid = np.sort((ii[ok] + nx * (jj[ok] + ny * kk[ok].astype(np.int64))))
    recv, send = [], []
    inball = set(gid.tolist())
    index = {g: k for k, g in enumerate(gid.tolist())}
    for g in gid.tolist():
        i, j, k = g % nx, (g // nx) % ny, g // (nx * ny)
        for (di, dj, dk) in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            a, b, c = i + di, j + dj, k + dk
            if 0 <= a < nx and 0 <= b < ny and 0 <= c < nz:
                h = a + nx * (b + ny * c)
                if h in inball:
                    recv.append(index[g])
                    send.append(index[h])
    recv = np.array(recv, dtype=np.int64)
    send = np.array(send, dtype=np.int64)
    order = np.lexsort((send, recv))
    return SubGraph(gid, recv[order], send[order], np.ones(len(recv)), np.ones(len(gid))), index[center]


def ball_output(params, spec, mesh, field, center):
    """Exact R=1 model output [out] at global id ``center``."""
    G, c = ball_graph(mesh.npts, center, spec.n_layers)
    X = np.asarray(field, np.float64)[G.gid]
    Y, _ = model_fwd(params, spec, [G], {}, [X], [edge_inputs(G, mesh.pos)])
    return Y[0][c]


def ball_grad(params, spec, mesh, field, center, weight):
    """Exact gradient of <weight, Y_center> with respect to every parameter."""
    G, c = ball_graph(mesh.npts, center, spec.n_layers)
    X = np.asarray(field, np.float64)[G.gid]
    Y, cache = model_fwd(params, spec, [G], {}, [X], [edge_inputs(G, mesh.pos)])
    gY = np.zeros_like(Y[0])
    gY[c] = weight
    grads, _ = model_bwd(params, spec, [G], {}, cache, [gY])
    return Y[0][c], grads
