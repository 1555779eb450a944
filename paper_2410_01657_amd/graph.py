"""Distributed mesh graph (Sec. II-A) through the C ABI, and its device copy.

``build_graph`` runs the library's host graph builder (graph_partition and
halo_plan_build) on an element mesh and returns NumPy arrays;
``DeviceGraph`` holds them as device tensors plus the descriptor the layer
entry points take.  All R sub-graphs share one set of buffers; sub-graph r
owns rows ``row_off[r]:row_off[r+1]`` and edges ``edge_off[r]:edge_off[r+1]``.
"""

import ctypes as C
from dataclasses import dataclass

import numpy as np

from ._lib import MpDevGraph, call, lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


@dataclass
class HostGraph:
    R: int
    row_off: np.ndarray
    edge_off: np.ndarray
    row_gid: np.ndarray
    rowptr: np.ndarray
    recv: np.ndarray
    col: np.ndarray
    rev: np.ndarray
    edge_mult: np.ndarray
    node_mult: np.ndarray
    group_ptr: np.ndarray
    member: np.ndarray
    pair_r: np.ndarray
    pair_s: np.ndarray
    pair_ptr: np.ndarray
    pair_rows_r: np.ndarray
    pair_rows_s: np.ndarray
    halo_rows: np.ndarray
    neighbours: np.ndarray
    graph_checksum: int = 0        # mp_graph_checksum
    plan_checksum: int = 0         # mp_halo_plan_checksum: the plan's own
    plan_graph_checksum: int = 0   # ... and that of the graph it was built on

    @property
    def n_rows(self):
        return int(self.row_gid.shape[0])

    @property
    def n_edges(self):
        return int(self.col.shape[0])

    @property
    def n_groups(self):
        return int(self.group_ptr.shape[0] - 1)


def hex_links(P):
    n = C.c_int32()
    call("mp_hex_links", P, None, C.byref(n))
    links = np.empty((n.value, 2), np.int32)
    call("mp_hex_links", P, _ptr(links), C.byref(n))
    return links


def build_graph(elem_gid, P, elem_part, R, links=None, order="locality"):
    """Reduced sub-graphs, CSR arrays, degrees and halo plan of a partition.

    ``links`` ([n_links, 2] element-local point pairs) defaults to the links
    of a hexahedral element of order P; any element type may pass its own.
    ``order``: "locality" renumbers each sub-graph's rows in reverse
    Cuthill-McKee order (graph_order_rows); "gid" keeps them in ascending
    global id."""
    if order not in ("locality", "gid"):
        raise ValueError("order must be 'locality' or 'gid'")
    eg = np.ascontiguousarray(elem_gid, dtype=np.int64)
    part = np.ascontiguousarray(elem_part, dtype=np.int32)
    links = hex_links(P) if links is None else np.ascontiguousarray(links, dtype=np.int32)
    g = C.c_void_p()
    call("graph_partition", eg.shape[0], eg.shape[1], _ptr(eg), links.shape[0], _ptr(links),
         _ptr(part), R, C.byref(g))
    try:
        if order == "locality":
            call("graph_order_rows", g)
        n, e, r = C.c_int64(), C.c_int64(), C.c_int32()
        call("mp_graph_sizes", g, C.byref(n), C.byref(e), C.byref(r))
        N, E = n.value, e.value
        arr = dict(row_off=np.empty(R + 1, np.int64), edge_off=np.empty(R + 1, np.int64),
                   row_gid=np.empty(N, np.int64), rowptr=np.empty(N + 1, np.int32),
                   recv=np.empty(E, np.int32), col=np.empty(E, np.int32), rev=np.empty(E, np.int32),
                   edge_mult=np.empty(E, np.uint8), node_mult=np.empty(N, np.uint8))
        call("mp_graph_export", g, *[_ptr(arr[k]) for k in
                                     ("row_off", "edge_off", "row_gid", "rowptr", "recv", "col",
                                      "rev", "edge_mult", "node_mult")])
        gcs = C.c_uint64()
        call("mp_graph_checksum", g, C.byref(gcs))
        h = C.c_void_p()
        call("halo_plan_build", g, C.byref(h))
        try:
            ng, nm, npair, nprow = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
            call("mp_halo_plan_sizes", h, C.byref(ng), C.byref(nm), C.byref(npair), C.byref(nprow))
            harr = dict(group_ptr=np.empty(ng.value + 1, np.int32), member=np.empty(nm.value, np.int32),
                        pair_r=np.empty(npair.value, np.int32), pair_s=np.empty(npair.value, np.int32),
                        pair_ptr=np.empty(npair.value + 1, np.int64),
                        pair_rows_r=np.empty(nprow.value, np.int32),
                        pair_rows_s=np.empty(nprow.value, np.int32),
                        halo_rows=np.empty(R, np.int64), neighbours=np.empty(R, np.int32))
            call("mp_halo_plan_export", h, *[_ptr(harr[k]) for k in
                                             ("group_ptr", "member", "pair_r", "pair_s", "pair_ptr",
                                              "pair_rows_r", "pair_rows_s", "halo_rows", "neighbours")])
            pcs, pgcs = C.c_uint64(), C.c_uint64()
            call("mp_halo_plan_checksum", h, C.byref(pcs), C.byref(pgcs))
        finally:
            lib().mp_halo_plan_destroy(h)
    finally:
        lib().mp_graph_destroy(g)
    return HostGraph(R=R, **arr, **harr, graph_checksum=gcs.value, plan_checksum=pcs.value,
                     plan_graph_checksum=pgcs.value)


def check_host_graph(hg):
    """Host-side check that every index the kernels follow stays in range."""
    N, E = hg.n_rows, hg.n_edges
    rp = hg.rowptr.astype(np.int64)
    ok = (rp.shape[0] == N + 1 and rp[0] == 0 and rp[-1] == E and np.all(np.diff(rp) >= 0)
          and hg.recv.shape[0] == E and hg.rev.shape[0] == E and hg.edge_mult.shape[0] == E
          and np.all((hg.col >= 0) & (hg.col < N)) and np.all((hg.rev >= 0) & (hg.rev < E))
          and np.all(hg.edge_mult >= 1)
          and np.array_equal(np.repeat(np.arange(N, dtype=np.int64), np.diff(rp)), hg.recv.astype(np.int64))
          and np.all(hg.recv[hg.rev] == hg.col) and np.all(hg.col[hg.rev] == hg.recv))
    gp = hg.group_ptr.astype(np.int64)
    ok = ok and gp[0] == 0 and gp[-1] == hg.member.shape[0] and np.all(np.diff(gp) >= 1)
    ok = ok and np.all((hg.member >= 0) & (hg.member < N))
    if not ok:
        raise ValueError("graph arrays are inconsistent; refusing to upload them")


class DeviceGraph:
    """Device copy of a HostGraph and the mp_dev_graph descriptor."""

    def __init__(self, hg, device="cuda"):
        import torch
        check_host_graph(hg)
        self.host = hg
        self.device = torch.device(device)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.device)
        self.rowptr = t(hg.rowptr)
        self.recv = t(hg.recv)
        self.col = t(hg.col)
        self.rev = t(hg.rev)
        self.edge_mult = t(hg.edge_mult)
        self.node_mult = t(hg.node_mult)
        self.group_ptr = t(hg.group_ptr)
        self.member = t(hg.member) if hg.member.size else torch.zeros(1, dtype=torch.int32, device=self.device)
        d = MpDevGraph()
        d.n_rows, d.n_edges = hg.n_rows, hg.n_edges
        d.n_groups, d.n_members = hg.n_groups, int(hg.member.shape[0])
        d.rowptr, d.recv, d.col = self.rowptr.data_ptr(), self.recv.data_ptr(), self.col.data_ptr()
        d.rev, d.edge_mult = self.rev.data_ptr(), self.edge_mult.data_ptr()
        d.group_ptr, d.member = self.group_ptr.data_ptr(), self.member.data_ptr()
        d.graph_checksum, d.plan_checksum = hg.graph_checksum, hg.plan_checksum
        d.plan_graph_checksum = hg.plan_graph_checksum
        # reads the arrays back and checks them against the host checksums
        call("mp_dev_graph_seal", C.byref(d), 1)
        self.desc = d

    @property
    def n_rows(self):
        return self.host.n_rows

    @property
    def n_edges(self):
        return self.host.n_edges

    def rows_of(self, per_gid):
        """Gather a per-global-id array onto the rows (all copies get the value)."""
        import torch
        v = np.asarray(per_gid)[self.host.row_gid]
        return torch.from_numpy(np.ascontiguousarray(v)).to(self.device)
