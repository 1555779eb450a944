"""Oracle set-up: the inputs of one workload as per-sub-graph arrays.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""

from dataclasses import dataclass

import numpy as np

from .graph import lattice_graph, partition_graph, halo_lists
from .nmp import edge_inputs


@dataclass
class Problem:
    graphs: list
    copies: dict
    pair_lists: dict
    X: list          # per sub-graph [n, 3] node inputs (float64 of the FP32 field)
    E0: list         # per sub-graph [e, 4] (or [e, 7]) edge inputs
    T: list          # per sub-graph [n, 3] targets


def build_problem(mesh, field, target, elem_part=None, R=1, unpartitioned_from_lattice=True, edge_in=4):
    """R=1 on a box mesh uses the lattice definition of the graph; otherwise
    the element route (with the mesh's own links where it has them)."""
    links = getattr(mesh, "links", None)
    period = getattr(mesh, "period", None)
    if R == 1 and unpartitioned_from_lattice and links is None and not any(period or ()):
        graphs, copies = [lattice_graph(mesh.npts)], {}
    else:
        part = np.zeros(mesh.n_elem, np.int32) if elem_part is None else elem_part
        graphs, copies = partition_graph(mesh.elem_gid, mesh.P, part, R, links)
    pairs = halo_lists(graphs, copies)
    f = np.asarray(field, np.float64)
    t = np.asarray(target, np.float64)
    X = [f[G.gid] for G in graphs]
    T = [t[G.gid] for G in graphs]
    E0 = [edge_inputs(G, mesh.pos, period, f if edge_in == 7 else None) for G in graphs]
    return Problem(graphs, copies, pairs, X, E0, T)
