"""C ABI on the CPU: exports, the host graph builder against the oracle's
own graphs, halo plans, and the validation paths of the device entry
points (which must reject bad input before touching a GPU)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from mpinputs import CONFIGS, block_partition, box_mesh, make_inputs, rcb_partition, slab_partition
from oracle.graph import partition_graph, table2_stats

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2410_01657_amd import _lib
    return _lib


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "mplayer.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if not n.startswith("MP")))


def test_exports_every_declared_symbol(L):
    lib = L.lib()
    declared = _declared_functions()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(L.EXPORTED)
    assert lib.mp_abi_version() == L.ABI_VERSION == 4


def test_hex_links_counts():
    from paper_2410_01657_amd import hex_links
    from oracle.graph import element_links
    for P in (1, 2, 3, 5, 7):
        links = hex_links(P)
        assert links.shape == (3 * P * (P + 1) ** 2, 2)
        ref = element_links(P)
        assert set(map(tuple, links.tolist())) == set(map(tuple, ref.tolist()))


def _compare_with_oracle(mesh, part, R):
    from paper_2410_01657_amd import build_graph
    hg = build_graph(mesh.elem_gid, mesh.P, part, R, order="gid")
    og, copies = partition_graph(mesh.elem_gid, mesh.P, part, R)
    assert hg.R == R
    for r, G in enumerate(og):
        r0, r1 = hg.row_off[r], hg.row_off[r + 1]
        e0, e1 = hg.edge_off[r], hg.edge_off[r + 1]
        np.testing.assert_array_equal(hg.row_gid[r0:r1], G.gid)
        np.testing.assert_array_equal(hg.recv[e0:e1] - r0, G.recv)
        np.testing.assert_array_equal(hg.col[e0:e1] - r0, G.send)
        np.testing.assert_array_equal(hg.edge_mult[e0:e1], G.d_edge.astype(np.uint8))
        np.testing.assert_array_equal(hg.node_mult[r0:r1], G.d_node.astype(np.uint8))
    # CSR and reverse-edge invariants
    assert hg.rowptr[0] == 0 and hg.rowptr[-1] == hg.n_edges
    np.testing.assert_array_equal(np.repeat(np.arange(hg.n_rows), np.diff(hg.rowptr)), hg.recv)
    np.testing.assert_array_equal(hg.rev[hg.rev], np.arange(hg.n_edges))
    np.testing.assert_array_equal(hg.recv[hg.rev], hg.col)
    # halo groups = the oracle's copies, as global rows
    groups = {}
    for gidx in range(hg.n_groups):
        mem = hg.member[hg.group_ptr[gidx]:hg.group_ptr[gidx + 1]]
        gids = set(hg.row_gid[mem].tolist())
        assert len(gids) == 1
        groups[gids.pop()] = mem.tolist()
    ref = {g: [int(hg.row_off[r]) + i for r, i in cps] for g, cps in copies.items()}
    assert groups == ref
    rows, halo, nbrs = table2_stats(og, copies)
    np.testing.assert_array_equal(hg.halo_rows, halo)
    np.testing.assert_array_equal(hg.neighbours, nbrs)
    # pair lists: every (r, s) pair's rows share ids, in ascending id
    for k in range(hg.pair_r.shape[0]):
        a, b = hg.pair_ptr[k], hg.pair_ptr[k + 1]
        rr, rs = hg.pair_rows_r[a:b], hg.pair_rows_s[a:b]
        np.testing.assert_array_equal(hg.row_gid[rr], hg.row_gid[rs])
        assert np.all(np.diff(hg.row_gid[rr]) > 0)
    return hg


def test_graph_c0_r1_r8():
    inp = make_inputs(CONFIGS["C0"])
    _compare_with_oracle(inp.mesh, np.zeros(inp.mesh.n_elem, np.int32), 1)
    hg = _compare_with_oracle(inp.mesh, inp.elem_part, 8)
    assert (hg.n_rows, hg.n_edges, hg.n_groups, hg.member.shape[0]) == (2744, 14112, 469, 1016)


def test_graph_rcb_t_junctions():
    nel = (6, 5, 4)
    m = box_mesh(nel, 2)
    part, _ = rcb_partition(nel, 8, seed=11, ratio=(1.0, 10.0))
    hg = _compare_with_oracle(m, part, 8)
    assert 3 in set(hg.edge_mult.tolist())


def _by_gid(hg):
    """Everything of a host graph that does not depend on its row numbering:
    per sub-graph the rows (gid, node degree) and the edges (receiver gid,
    sender gid, edge degree), and the halo groups as gid -> (sub-graph, gid)."""
    out = []
    for r in range(hg.R):
        r0, r1 = hg.row_off[r], hg.row_off[r + 1]
        e0, e1 = hg.edge_off[r], hg.edge_off[r + 1]
        rows = sorted(zip(hg.row_gid[r0:r1].tolist(), hg.node_mult[r0:r1].tolist()))
        edges = sorted(zip(hg.row_gid[hg.recv[e0:e1]].tolist(), hg.row_gid[hg.col[e0:e1]].tolist(),
                           hg.edge_mult[e0:e1].tolist()))
        out.append((rows, edges))
    part = np.searchsorted(hg.row_off, np.arange(hg.n_rows), side="right") - 1
    groups = {}
    for k in range(hg.n_groups):
        mem = hg.member[hg.group_ptr[k]:hg.group_ptr[k + 1]]
        groups[int(hg.row_gid[mem[0]])] = [int(part[m]) for m in mem]
    return out, groups


def _csr_invariants(hg):
    assert hg.rowptr[0] == 0 and hg.rowptr[-1] == hg.n_edges
    np.testing.assert_array_equal(np.repeat(np.arange(hg.n_rows), np.diff(hg.rowptr)), hg.recv)
    np.testing.assert_array_equal(hg.rev[hg.rev], np.arange(hg.n_edges))
    np.testing.assert_array_equal(hg.recv[hg.rev], hg.col)
    for r in range(hg.R):  # senders ascend inside each receiver's range, inside the sub-graph
        e0, e1 = hg.edge_off[r], hg.edge_off[r + 1]
        key = hg.recv[e0:e1].astype(np.int64) * hg.n_rows + hg.col[e0:e1]
        assert np.all(np.diff(key) > 0)
        assert hg.col[e0:e1].min() >= hg.row_off[r] and hg.col[e0:e1].max() < hg.row_off[r + 1]


@pytest.mark.parametrize("case", ["c0_r8", "rcb_r8", "slab_r4", "tet_r8"])
def test_graph_locality_order_is_a_renumbering(case):
    """graph_order_rows changes only the row numbering: the same rows,
    edges, degrees and halo groups by global id, the CSR invariants hold,
    and the bandwidth (largest |receiver - sender|) does not grow -- on a
    z-slab it shrinks from a plane of the lattice to about a level of the
    breadth-first sweep."""
    from paper_2410_01657_amd import build_graph
    if case == "c0_r8":
        inp = make_inputs(CONFIGS["C0"])
        m, part, R = inp.mesh, inp.elem_part, 8
    elif case == "rcb_r8":
        nel = (6, 5, 4)
        m = box_mesh(nel, 2)
        part, _ = rcb_partition(nel, 8, seed=11, ratio=(1.0, 10.0))
        R = 8
    elif case == "slab_r4":
        nel = (8, 8, 8)
        m = box_mesh(nel, 3, with_positions=False)
        part, R = slab_partition(nel, 4), 4
    else:  # tetrahedra: irregular degrees, no lattice to follow
        from mpinputs.tetmesh import centroid_partition, tet_mesh
        m = tet_mesh(800, 3)
        part, R = centroid_partition(m, 8), 8
    links = getattr(m, "links", None)
    g0 = build_graph(m.elem_gid, m.P, part, R, links, order="gid")
    g1 = build_graph(m.elem_gid, m.P, part, R, links)
    _csr_invariants(g1)
    assert _by_gid(g1) == _by_gid(g0)
    bw0, bw1 = np.abs(g0.recv - g0.col).max(), np.abs(g1.recv - g1.col).max()
    assert bw1 <= bw0
    if case == "slab_r4":
        assert bw0 == 25 * 25 and bw1 < bw0 / 2
    g2 = build_graph(m.elem_gid, m.P, part, R, links)  # the order is a function of the graph
    for f in ("row_gid", "rowptr", "col", "rev", "edge_mult", "node_mult", "member", "pair_rows_r"):
        np.testing.assert_array_equal(getattr(g1, f), getattr(g2, f))


def test_graph_locality_order_disconnected_sub_graph():
    """A sub-graph made of two meshes that share no node (two connected
    components, each swept from its own start): still a renumbering, and
    each component's rows stay together."""
    from paper_2410_01657_amd import build_graph
    a = box_mesh((3, 2, 2), 2, with_positions=False)
    b = box_mesh((2, 2, 2), 2, with_positions=False)
    eg = np.concatenate([a.elem_gid, b.elem_gid + a.n_gid])
    part = np.zeros(eg.shape[0], np.int32)
    part[a.n_elem:] = 1  # sub-graph 1: mesh b alone
    part[: a.n_elem // 2] = 1  # ...and half of mesh a
    g0 = build_graph(eg, 2, part, 2, order="gid")
    g1 = build_graph(eg, 2, part, 2)
    _csr_invariants(g1)
    assert _by_gid(g1) == _by_gid(g0)
    r0, r1 = g1.row_off[1], g1.row_off[2]
    in_b = g1.row_gid[r0:r1] >= a.n_gid
    # the order is component by component: mesh b's rows are one contiguous run
    idx = np.flatnonzero(in_b)
    assert idx.size > 0 and idx[-1] - idx[0] + 1 == idx.size


@pytest.mark.slow
def test_graph_c1_r16_sizes():
    from paper_2410_01657_amd import build_graph
    cfg = CONFIGS["C1"]
    m = box_mesh(cfg.nel, cfg.P, with_positions=False)
    hg = build_graph(m.elem_gid, 5, slab_partition(cfg.nel, 16), 16)
    assert (hg.n_rows, hg.n_edges, hg.n_groups, hg.member.shape[0]) == (629856, 3538080, 98415, 196830)


@pytest.mark.slow
def test_graph_table2_r8_row():
    from paper_2410_01657_amd import build_graph
    nel = (16, 16, 128)
    m = box_mesh(nel, 5, periodic=(True, True, True), with_positions=False)
    hg = build_graph(m.elem_gid, 5, slab_partition(nel, 8), 8)
    np.testing.assert_array_equal(np.diff(hg.row_off), 518400)
    np.testing.assert_array_equal(hg.halo_rows, 12800)
    np.testing.assert_array_equal(hg.neighbours, 2)


# ------------------------------------------------------------ error paths


def test_graph_partition_rejects_bad_input(L):
    from paper_2410_01657_amd import hex_links
    from paper_2410_01657_amd._lib import MPError, call
    m = box_mesh((2, 1, 1), 1)
    links = hex_links(1)
    eg = np.ascontiguousarray(m.elem_gid)
    g = C.c_void_p()
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    bad_part = np.array([0, 2], np.int32)
    with pytest.raises(MPError) as e:
        call("graph_partition", 2, 8, ptr(eg), links.shape[0], ptr(links), ptr(bad_part), 2, C.byref(g))
    assert e.value.code == L.MP_EINVAL and "part" in str(e.value)
    empty_part = np.array([0, 0], np.int32)
    with pytest.raises(MPError):
        call("graph_partition", 2, 8, ptr(eg), links.shape[0], ptr(links), ptr(empty_part), 2, C.byref(g))
    bad_links = links.copy()
    bad_links[0] = (3, 3)
    with pytest.raises(MPError):
        call("graph_partition", 2, 8, ptr(eg), links.shape[0], ptr(bad_links), ptr(empty_part), 1, C.byref(g))
    with pytest.raises(MPError):
        call("graph_partition", 2, 8, None, links.shape[0], ptr(links), ptr(empty_part), 1, C.byref(g))
    assert g.value is None
    with pytest.raises(MPError) as e:
        call("graph_order_rows", None)
    assert e.value.code == L.MP_EINVAL


def _fake_desc(L, n_rows=10, n_edges=20):
    from paper_2410_01657_amd._lib import call
    d = L.MpDevGraph()
    d.n_rows, d.n_edges, d.n_groups, d.n_members = n_rows, n_edges, 0, 0
    for f in ("rowptr", "recv", "col", "rev", "edge_mult", "group_ptr"):
        setattr(d, f, 4096)  # never dereferenced: validation fails first
    call("mp_dev_graph_seal", C.byref(d), 0)  # checksums taken on trust (0 = 0), no device read
    return d


def _desc_from(L, hg, plan=None):
    """A descriptor holding hg's sizes and checksums, paired with the halo
    plan of `plan` (another HostGraph; default hg's own), on fake pointers."""
    plan = plan or hg
    d = L.MpDevGraph()
    d.n_rows, d.n_edges = hg.n_rows, hg.n_edges
    d.n_groups, d.n_members = plan.n_groups, int(plan.member.shape[0])
    for f in ("rowptr", "recv", "col", "rev", "edge_mult", "group_ptr", "member"):
        setattr(d, f, 4096)
    d.graph_checksum = hg.graph_checksum
    d.plan_checksum, d.plan_graph_checksum = plan.plan_checksum, plan.plan_graph_checksum
    return d


def test_graph_and_plan_checksums_catch_a_plan_from_another_graph(L):
    """Sec. II-A / Eq. 4c-d: a halo plan is only meaningful beside the graph
    whose rows it names.  The ascending-id and the locality-ordered graph of
    one mesh have identical sizes; pairing one's CSR with the other's plan
    is refused (MP_EPLAN) by the seal and by every entry point, before any
    device access."""
    from paper_2410_01657_amd import build_graph
    from paper_2410_01657_amd._lib import MPError, call
    from paper_2410_01657_amd.ops import layer_cfg
    m = box_mesh((4, 4, 4), 3)
    part = block_partition((4, 4, 4), (2, 2, 2))
    g_id = build_graph(m.elem_gid, m.P, part, 8, order="gid")
    g_rcm = build_graph(m.elem_gid, m.P, part, 8, order="locality")
    assert (g_id.n_rows, g_id.n_edges, g_id.n_groups) == (g_rcm.n_rows, g_rcm.n_edges, g_rcm.n_groups)
    assert g_id.graph_checksum != g_rcm.graph_checksum
    assert g_id.plan_checksum != g_rcm.plan_checksum
    for g in (g_id, g_rcm):
        assert g.plan_graph_checksum == g.graph_checksum
    # the checksum is a function of the content: rebuilding gives the same value
    assert build_graph(m.elem_gid, m.P, part, 8, order="gid").graph_checksum == g_id.graph_checksum
    # another partition of the same mesh
    g_r1 = build_graph(m.elem_gid, m.P, np.zeros(64, np.int32), 1, order="gid")
    assert g_r1.graph_checksum not in (g_id.graph_checksum, g_rcm.graph_checksum)
    # matched pairs seal; crossed pairs do not
    for g in (g_id, g_rcm):
        call("mp_dev_graph_seal", C.byref(_desc_from(L, g)), 0)
    for g, p in ((g_rcm, g_id), (g_id, g_rcm)):
        d = _desc_from(L, g, p)
        with pytest.raises(MPError) as e:
            call("mp_dev_graph_seal", C.byref(d), 0)
        assert e.value.code == L.MP_EPLAN
        assert d.seal == 0
    # a sealed descriptor whose plan is swapped afterwards is refused by the entry points
    d = _desc_from(L, g_rcm)
    call("mp_dev_graph_seal", C.byref(d), 0)
    cfg = layer_cfg(32)
    nb = C.c_size_t()
    call("mp_layer_workspace_size", C.byref(cfg), C.byref(d), 1, C.byref(nb))
    d.plan_checksum, d.plan_graph_checksum = g_id.plan_checksum, g_id.plan_graph_checksum
    with pytest.raises(MPError) as e:
        call("mp_layer_workspace_size", C.byref(cfg), C.byref(d), 1, C.byref(nb))
    assert e.value.code == L.MP_EPLAN
    d.seal = 0  # an unsealed descriptor
    d.plan_checksum, d.plan_graph_checksum = g_rcm.plan_checksum, g_rcm.plan_graph_checksum
    with pytest.raises(MPError) as e:
        call("mp_layer_workspace_size", C.byref(cfg), C.byref(d), 1, C.byref(nb))
    assert e.value.code == L.MP_EPLAN


_ALLOC_CHILD = r"""
import ctypes as C, resource, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from mpinputs import box_mesh, slab_partition
from paper_2410_01657_amd._lib import lib
from paper_2410_01657_amd.graph import hex_links
m = box_mesh((12, 12, 12), 5)
part = slab_partition((12, 12, 12), 4)
eg = np.ascontiguousarray(m.elem_gid, np.int64)
links = hex_links(5)
L = lib()
def vm():
    for line in open("/proc/self/status"):
        if line.startswith("VmSize:"):
            return int(line.split()[1]) * 1024
extra = int(sys.argv[2]) << 20
resource.setrlimit(resource.RLIMIT_AS, (vm() + extra, resource.RLIM_INFINITY))
g = C.c_void_p()
rc = L.graph_partition(eg.shape[0], eg.shape[1], eg.ctypes.data_as(C.c_void_p), links.shape[0],
                       links.ctypes.data_as(C.c_void_p), part.ctypes.data_as(C.c_void_p), 4, C.byref(g))
if rc == 0:
    rc = L.graph_order_rows(g)
print("rc", rc, flush=True)
"""


def test_graph_builder_reports_exhausted_memory_instead_of_aborting(tmp_path):
    """The graph builder runs its per-sub-graph work on threads; a failed
    allocation inside one must come back as MP_ENOMEM, not terminate the
    process.  The address space is capped at a range of levels so the
    failure lands in different places (before, inside and after the
    threaded parts)."""
    import subprocess
    import sys
    script = tmp_path / "child.py"
    script.write_text(_ALLOC_CHILD)
    codes = set()
    for extra_mib in (8, 24, 48, 96, 160, 256, 4096):
        p = subprocess.run([sys.executable, str(script), ROOT, str(extra_mib)], capture_output=True, text=True,
                           timeout=300)
        assert p.returncode == 0, (extra_mib, p.returncode, p.stderr[-2000:])
        rc = int(p.stdout.split()[-1])
        assert rc in (0, 3), (extra_mib, rc)
        codes.add(rc)
    assert codes == {0, 3}


def test_device_entry_points_validate_before_launch(L):
    from paper_2410_01657_amd._lib import MPError, call
    from paper_2410_01657_amd.ops import layer_cfg
    d = _fake_desc(L)
    nb = C.c_size_t()
    bad = layer_cfg(48)
    with pytest.raises(MPError) as e:
        call("mp_layer_workspace_size", C.byref(bad), C.byref(d), 0, C.byref(nb))
    assert e.value.code == L.MP_EINVAL
    cfg = layer_cfg(32)
    call("mp_layer_workspace_size", C.byref(cfg), C.byref(d), 1, C.byref(nb))
    assert nb.value > 0
    d.n_edges = 21  # descriptor changed after sealing
    with pytest.raises(MPError) as e:
        call("mp_layer_workspace_size", C.byref(cfg), C.byref(d), 0, C.byref(nb))
    assert e.value.code == L.MP_EPLAN
    d = _fake_desc(L)
    params = L.MpLayerParams()
    with pytest.raises(MPError) as e:  # NULL parameters
        call("mp_layer_forward", C.byref(cfg), C.byref(params), C.byref(d), None, None, None, None, None,
             None, None, 0, None)
    assert e.value.code == L.MP_EINVAL
    for f in L.LAYER_FIELDS:
        setattr(params, f, 4096)
    with pytest.raises(MPError) as e:  # workspace too small
        call("mp_layer_forward", C.byref(cfg), C.byref(params), C.byref(d), 4096, 8192, 12288, 16384, None,
             None, 4096, 16, None)
    assert e.value.code == L.MP_ENOMEM
    with pytest.raises(MPError) as e:  # aliasing
        call("mp_layer_forward", C.byref(cfg), C.byref(params), C.byref(d), 4096, 8192, 4096, 16384, None,
             None, 4096, 1 << 30, None)
    assert e.value.code == L.MP_EINVAL
    with pytest.raises(MPError):  # unaligned
        call("mp_layer_forward", C.byref(cfg), C.byref(params), C.byref(d), 4100, 8192, 12288, 16384, None,
             None, 4096, 1 << 30, None)


def test_mlp_and_loss_validation(L):
    from paper_2410_01657_amd._lib import MPError, call
    from paper_2410_01657_amd.ops import mlp_cfg
    nb = C.c_size_t()
    with pytest.raises(MPError):
        call("mp_mlp_workspace_size", C.byref(mlp_cfg(5, 64, 64, True)), 10, 0, C.byref(nb))
    with pytest.raises(MPError):
        call("mp_mlp_workspace_size", C.byref(mlp_cfg(3, 64, 3, False)), 10, 0, C.byref(nb))
    with pytest.raises(MPError):  # LayerNorm on a small output
        call("mp_mlp_workspace_size", C.byref(mlp_cfg(64, 64, 3, True)), 10, 0, C.byref(nb))
    call("mp_mlp_workspace_size", C.byref(mlp_cfg(64, 64, 3, False)), 10, 1, C.byref(nb))
    with pytest.raises(MPError):
        call("mp_consistent_mse", 0, 3, None, None, None, None, None, None, 0, None)


def test_deep_entry_points_validate_before_launch(L):
    """The deep-MLP entry points reject bad widths, depths, NULL or unaligned
    buffers, aliasing and short workspaces before any launch."""
    from paper_2410_01657_amd._lib import MPError, call
    from paper_2410_01657_amd.ops import deep_layer_cfg, deep_mlp_cfg, deep_theta_size
    d = _fake_desc(L)
    nb = C.c_size_t()
    for bad in (deep_layer_cfg(12, 2), deep_layer_cfg(64, 2), deep_layer_cfg(8, 9), deep_layer_cfg(8, -1)):
        with pytest.raises(MPError) as e:
            call("mp_deep_layer_workspace_size", C.byref(bad), C.byref(d), 1, C.byref(nb))
        assert e.value.code == L.MP_EINVAL
    cfg = deep_layer_cfg(8, 2)
    call("mp_deep_layer_workspace_size", C.byref(cfg), C.byref(d), 0, C.byref(nb))
    assert nb.value == 0
    call("mp_deep_layer_workspace_size", C.byref(cfg), C.byref(d), 1, C.byref(nb))
    assert nb.value > 0
    with pytest.raises(MPError) as e:  # a NULL buffer
        call("mp_deep_layer_forward", C.byref(cfg), 4096, 4096, C.byref(d), 8192, 12288, 16384, 20480, None,
             None)
    assert e.value.code == L.MP_EINVAL
    with pytest.raises(MPError) as e:  # aliasing
        call("mp_deep_layer_forward", C.byref(cfg), 4096, 4096, C.byref(d), 8192, 12288, 8192, 20480, 24576,
             None)
    assert e.value.code == L.MP_EINVAL
    with pytest.raises(MPError) as e:  # unaligned
        call("mp_deep_layer_forward", C.byref(cfg), 4096, 4096, C.byref(d), 8196, 12288, 16384, 20480, 24576,
             None)
    assert e.value.code == L.MP_EINVAL
    with pytest.raises(MPError) as e:  # workspace too small
        call("mp_deep_layer_backward", C.byref(cfg), 4096, 4096, C.byref(d), 8192, 12288, 16384, 20480, None,
             24576, 28672, 32768, 36864, 40960, 16, None)
    assert e.value.code == L.MP_ENOMEM
    for c in (deep_mlp_cfg(9, 8, 2, 8, True), deep_mlp_cfg(8, 8, 2, 3, True), deep_mlp_cfg(3, 8, 2, 3, False),
              deep_mlp_cfg(16, 8, 2, 8, False)):
        with pytest.raises(MPError) as e:
            call("mp_deep_mlp_workspace_size", C.byref(c), 10, 1, C.byref(nb))
        assert e.value.code == L.MP_EINVAL
    call("mp_deep_mlp_workspace_size", C.byref(deep_mlp_cfg(4, 32, 5, 32, True)), 10, 1, C.byref(nb))
    assert nb.value > 0
    # flat parameter sizes follow the torch.nn.Linear layout
    assert deep_theta_size(3, 8, 2, 8, True) == 8 * 3 + 8 + 2 * (64 + 8) + 64 + 8 + 16
    assert deep_theta_size(8, 8, 0, 3, False) == 64 + 8 + 24 + 3


def test_noalloc_forward_validates_before_touching_a_gpu(L):
    """mp_layer_forward_noalloc refuses, before any device call, a missing
    a_star_out / pq_out and a graph whose tile bounds would exceed its fixed
    scratch (32 MiB)."""
    from paper_2410_01657_amd._lib import MPError, call, lib
    from paper_2410_01657_amd.ops import layer_cfg
    assert lib().mp_layer_forward_noalloc_max_scratch() == 32 << 20
    cfg = layer_cfg(64)
    params = L.MpLayerParams()
    for f in L.LAYER_FIELDS:
        setattr(params, f, 4096)
    d = _fake_desc(L)
    with pytest.raises(MPError) as e:  # a_star_out and pq_out are required
        call("mp_layer_forward_noalloc", C.byref(cfg), C.byref(params), C.byref(d), 4096, 8192, 12288, 16384,
             None, None, None)
    assert e.value.code == L.MP_EINVAL and "required" in str(e.value)
    # 2^30 edges in 16-edge tiles: 2^26 tiles of 8 bytes, beyond the scratch
    big = _fake_desc(L, n_rows=1 << 20, n_edges=1 << 30)
    cfg.tile_edges = 16
    with pytest.raises(MPError) as e:
        call("mp_layer_forward_noalloc", C.byref(cfg), C.byref(params), C.byref(big), 4096, 8192, 12288, 16384,
             20480, 24576, None)
    assert e.value.code == L.MP_EINVAL and "maximum" in str(e.value)


def test_schedule_fields_are_validated(L):
    """The schedule dimensions of mp_layer_cfg are checked before any
    launch: waves per workgroup of the edge adjoint (0, 4, or 8 with BF16
    GEMMs at H <= 64 or at H > 64) and the forward's tile order (0 or 1)."""
    from paper_2410_01657_amd._lib import MPError, call
    from paper_2410_01657_amd.autotune import candidates
    from paper_2410_01657_amd.ops import layer_cfg
    d = _fake_desc(L)
    nb = C.c_size_t()
    for H, gemm, waves, q, ok in ((64, "bf16", 8, 1, True), (64, "bf16", 4, 0, True), (32, "bf16", 8, 0, True),
                                  (128, "bf16", 8, 0, True), (128, "f32", 8, 1, True), (32, "f32", 8, 0, False),
                                  (64, "f32", 8, 0, False), (64, "f32", 4, 1, True),
                                  (64, "bf16", 6, 0, False), (64, "bf16", 0, 2, False)):
        cfg = layer_cfg(H, gemm=gemm)
        cfg.edge_bwd_waves, cfg.edge_fwd_queue = waves, q
        if ok:
            call("mp_layer_workspace_size", C.byref(cfg), C.byref(d), 1, C.byref(nb))
        else:
            with pytest.raises(MPError) as e:
                call("mp_layer_workspace_size", C.byref(cfg), C.byref(d), 1, C.byref(nb))
            assert e.value.code == L.MP_EINVAL
    # every candidate the tuner may return is accepted
    for H, gemm in ((32, "bf16"), (64, "bf16"), (64, "f32"), (128, "bf16"), (128, "f32")):
        cs = candidates(H, gemm)
        assert len(cs) == len({tuple(sorted(c.items())) for c in cs})
        for sched in cs[:: max(1, len(cs) // 12)]:
            cfg = layer_cfg(H, gemm=gemm)
            for k, v in sched.items():
                setattr(cfg, k, v)
            call("mp_layer_workspace_size", C.byref(cfg), C.byref(d), 1, C.byref(nb))


def test_edge_state_dtype_is_validated(L):
    """BF16 edge states (estate_dtype) need BF16 GEMMs; a BF16 MLP output
    exists for the edge encoder's form only (small input, n_out == H, BF16
    GEMMs); other values are refused before any launch."""
    from paper_2410_01657_amd._lib import MPError, call
    from paper_2410_01657_amd.ops import layer_cfg, mlp_cfg
    d = _fake_desc(L)
    nb = C.c_size_t()
    for H in (32, 64, 128):
        call("mp_layer_workspace_size", C.byref(layer_cfg(H, gemm="bf16", estate="bf16")), C.byref(d), 1,
             C.byref(nb))
        with pytest.raises(MPError) as e:
            call("mp_layer_workspace_size", C.byref(layer_cfg(H, gemm="f32", estate="bf16")), C.byref(d), 1,
                 C.byref(nb))
        assert e.value.code == L.MP_EINVAL
    cfg = layer_cfg(64, gemm="bf16")
    cfg.estate_dtype = 2
    with pytest.raises(MPError) as e:
        call("mp_layer_workspace_size", C.byref(cfg), C.byref(d), 0, C.byref(nb))
    assert e.value.code == L.MP_EINVAL
    call("mp_mlp_workspace_size", C.byref(mlp_cfg(4, 64, 64, True, gemm="bf16", out="bf16")), 10, 1, C.byref(nb))
    for bad in (mlp_cfg(4, 64, 64, True, gemm="f32", out="bf16"), mlp_cfg(64, 64, 64, True, gemm="bf16", out="bf16"),
                mlp_cfg(64, 64, 3, False, gemm="bf16", out="bf16")):
        with pytest.raises(MPError) as e:
            call("mp_mlp_workspace_size", C.byref(bad), 10, 0, C.byref(nb))
        assert e.value.code == L.MP_EINVAL
