"""Oracle graph generation from a spectral-element mesh (Sec. II-A).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Graph nodes are the GLL quadrature points; undirected edges join
  neighbouring quadrature points of an element, and each becomes two
  directed edges (Sec. II-A, Fig. 2).
* Local coincident nodes (same global id inside one sub-graph) are collapsed
  to one row: the "reduced" distributed graph of Fig. 3c.  Rows are the
  distinct global ids of a sub-graph's elements.
* Non-local coincident nodes (same global id on several sub-graphs, Fig. 3b)
  are the rows that take part in the halo exchange (Fig. 4).
* Edge degree d_ij: number of sub-graphs holding a copy of the edge; it is
  above 1 only on shared interfaces (Sec. II-B, under Eq. 4).
* Node degree d_i: number of sub-graphs holding a copy of the node
  (Sec. II-C, Eq. 6b-c).
"""

from dataclasses import dataclass

import numpy as np


@dataclass
class SubGraph:
    gid: np.ndarray      # [n] global id of each row, ascending
    recv: np.ndarray     # [e] receiver row i of each directed edge
    send: np.ndarray     # [e] sender row j
    d_edge: np.ndarray   # [e] edge degree d_ij (float64)
    d_node: np.ndarray   # [n] node degree d_i (float64)

    @property
    def n(self):
        return int(self.gid.shape[0])

    @property
    def e(self):
        return int(self.recv.shape[0])


def lattice_graph(npts):
    """The R=1 graph written out from its definition on the GLL lattice.

    Every lattice point is joined to its +-1 neighbours along each axis; with
    coincident nodes collapsed this is exactly the union of all element
    graphs of a non-periodic box.  Edges sorted by (receiver, sender).
    """
    nx, ny, nz = npts
    g = np.arange(nx * ny * nz, dtype=np.int64)
    I, J, K = g % nx, (g // nx) % ny, g // (nx * ny)
    recv, send = [], []
    for (di, dj, dk) in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                         (0, 0, 1), (0, 0, -1)):
        ok = ((I + di >= 0) & (I + di < nx) & (J + dj >= 0) & (J + dj < ny)
              & (K + dk >= 0) & (K + dk < nz))
        recv.append(g[ok])
        send.append(g[ok] + di + nx * (dj + ny * dk))
    recv = np.concatenate(recv)
    send = np.concatenate(send)
    order = np.lexsort((send, recv))
    recv, send = recv[order], send[order]
    n = g.shape[0]
    return SubGraph(g, recv, send, np.ones(recv.shape[0]), np.ones(n))


def element_links(P):
    """Element-local undirected links between neighbouring GLL points."""
    q = P + 1
    pairs = []
    for c in range(q):
        for b in range(q):
            for a in range(q):
                i = a + q * (b + q * c)
                if a + 1 < q:
                    pairs.append((i, i + 1))
                if b + 1 < q:
                    pairs.append((i, i + q))
                if c + 1 < q:
                    pairs.append((i, i + q * q))
    return np.array(pairs, dtype=np.int64)


def partition_graph(elem_gid, P, elem_part, R, links=None):
    """Reduced sub-graphs, degrees and halo copies for an element partition.

    ``links`` lists the element-local point pairs joined by a link; by
    default those of a hexahedral element of order P.

    Returns ``(graphs, copies)`` where ``graphs[r]`` is the SubGraph of
    sub-graph r and ``copies`` maps each global id held by two or more
    sub-graphs to its list of (r, row) copies, in ascending r.
    """
    links = element_links(P) if links is None else np.asarray(links, np.int64)
    n_gid = int(elem_gid.max()) + 1
    und = []      # per sub-graph: unique undirected keys lo*n_gid + hi
    rows = []
    for r in range(R):
        eg = elem_gid[elem_part == r]
        rows.append(np.unique(eg))
        u = eg[:, links[:, 0]].reshape(-1)
        v = eg[:, links[:, 1]].reshape(-1)
        lo, hi = np.minimum(u, v), np.maximum(u, v)
        if np.any(lo == hi):
            raise ValueError("self-loop: an element wraps onto itself")
        und.append(np.unique(lo * n_gid + hi))
    all_keys, counts = np.unique(np.concatenate(und), return_counts=True)
    node_ids, node_counts = np.unique(np.concatenate(rows), return_counts=True)
    graphs = []
    for r in range(R):
        gid = rows[r]
        k = und[r]
        d = counts[np.searchsorted(all_keys, k)].astype(np.float64)
        lo, hi = k // n_gid, k % n_gid
        li = np.searchsorted(gid, lo)
        hj = np.searchsorted(gid, hi)
        recv = np.concatenate([li, hj])
        send = np.concatenate([hj, li])
        dd = np.concatenate([d, d])
        order = np.lexsort((send, recv))
        dn = node_counts[np.searchsorted(node_ids, gid)].astype(np.float64)
        graphs.append(SubGraph(gid, recv[order], send[order], dd[order], dn))
    copies = {}
    shared = node_ids[node_counts > 1]
    for r in range(R):
        gid = graphs[r].gid
        mask = np.isin(gid, shared)
        for row in np.nonzero(mask)[0]:
            copies.setdefault(int(gid[row]), []).append((r, int(row)))
    return graphs, copies


def halo_lists(graphs, copies):
    """Per ordered pair (r, s) of neighbouring sub-graphs: the rows of r whose
    global id also lives on s (r's send mask towards s) and the matching
    rows of s, in ascending global id (Fig. 4)."""
    pairs = {}
    for g, cps in sorted(copies.items()):
        for (r, i) in cps:
            for (s, k) in cps:
                if r != s:
                    pairs.setdefault((r, s), ([], []))
                    pairs[(r, s)][0].append(i)
                    pairs[(r, s)][1].append(k)
    return {key: (np.array(a), np.array(b)) for key, (a, b) in pairs.items()}


def table2_stats(graphs, copies):
    """Per sub-graph: rows, halo rows (one per copy held elsewhere), and the
    number of neighbouring sub-graphs (columns of Table II)."""
    R = len(graphs)
    halo = np.zeros(R, dtype=np.int64)
    nbrs = [set() for _ in range(R)]
    for cps in copies.values():
        ranks = [r for r, _ in cps]
        for r in ranks:
            halo[r] += len(ranks) - 1
            nbrs[r].update(s for s in ranks if s != r)
    rows = np.array([g.n for g in graphs])
    return rows, halo, np.array([len(s) for s in nbrs])
