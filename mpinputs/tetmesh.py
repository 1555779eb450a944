"""Unstructured element meshes: the general input of the graph construction.

The graph construction of Sec. II-A needs only an element -> global-id table
and the list of element-local point pairs joined by a link; the spectral-
element box is one instance of it.  This module draws a seeded Delaunay
tetrahedralisation of random points in the unit cube (its eight corners
included): elements of four points, all six pairs of an element's points
linked, so node degrees vary widely (from 4 to several dozen) and a link is
shared by a variable number of elements, and hence of sub-graphs.
"""

from dataclasses import dataclass

import numpy as np

TET_LINKS = np.array([(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)], dtype=np.int32)


@dataclass
class ElementMesh:
    elem_gid: np.ndarray   # [n_elem, npe] int64 global node ids
    links: np.ndarray      # [n_links, 2] int32 element-local linked pairs
    pos: np.ndarray        # [n_gid, 3] float64 positions
    P = None               # not a spectral-element mesh

    @property
    def n_elem(self):
        return int(self.elem_gid.shape[0])

    @property
    def npe(self):
        return int(self.elem_gid.shape[1])

    @property
    def n_gid(self):
        return int(self.pos.shape[0])


def tet_mesh(n_points, seed):
    """Delaunay tetrahedra of ``n_points`` seeded points in [0, 1]^3."""
    from scipy.spatial import Delaunay
    rng = np.random.Generator(np.random.PCG64(seed))
    corners = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], np.float64)
    pts = np.concatenate([corners, rng.uniform(0.0, 1.0, size=(n_points - 8, 3))])
    simp = np.asarray(Delaunay(pts).simplices, dtype=np.int64)
    used = np.unique(simp)
    if used.size != pts.shape[0]:           # drop points no tetrahedron uses
        remap = np.full(pts.shape[0], -1, np.int64)
        remap[used] = np.arange(used.size)
        simp, pts = remap[simp], pts[used]
    return ElementMesh(np.ascontiguousarray(simp), TET_LINKS.copy(), pts)


def centroid_partition(mesh, R):
    """R = 2^k parts of equal element count (within one) by recursive
    median bisection of element centroids along the widest axis."""
    levels = int(round(np.log2(R)))
    if 2 ** levels != R:
        raise ValueError("R must be a power of two")
    cen = mesh.pos[mesh.elem_gid].mean(axis=1)
    part = np.zeros(mesh.n_elem, np.int32)
    groups = [np.arange(mesh.n_elem)]
    for _ in range(levels):
        nxt = []
        for g in groups:
            c = cen[g]
            ax = int(np.argmax(c.max(axis=0) - c.min(axis=0)))
            order = g[np.argsort(c[:, ax], kind="stable")]
            h = order.shape[0] // 2
            nxt += [order[:h], order[h:]]
        groups = nxt
    for r, g in enumerate(groups):
        part[g] = r
    return part
