"""The device graph descriptor is sealed against the content of its arrays
(Sec. II-A: the reduced graph; Eq. 4c-d: the halo plan that names its rows).

mp_dev_graph_seal with device verification reads every uploaded array back
and recomputes the graph and plan checksums, so arrays uploaded from another
graph or plan, or changed on the device after upload, are refused with
MP_EPLAN before any kernel could use them.
"""

import ctypes as C

import numpy as np
import pytest
import torch

from mpinputs import block_partition, box_mesh

pytestmark = pytest.mark.gpu


def _desc(dg, **override):
    from paper_2410_01657_amd._lib import MpDevGraph
    d = MpDevGraph()
    C.memmove(C.byref(d), C.byref(dg.desc), C.sizeof(MpDevGraph))
    d.seal = 0
    for k, v in override.items():
        setattr(d, k, v)
    return d


def test_seal_reads_back_the_device_arrays():
    from paper_2410_01657_amd import DeviceGraph, build_graph
    from paper_2410_01657_amd._lib import MP_EPLAN, MPError, call
    m = box_mesh((4, 4, 4), 3)
    part = block_partition((4, 4, 4), (2, 2, 2))
    g_id = build_graph(m.elem_gid, m.P, part, 8, order="gid")
    g_rcm = build_graph(m.elem_gid, m.P, part, 8, order="locality")
    dg = DeviceGraph(g_rcm, "cuda")  # seals with verification
    d = _desc(dg)
    call("mp_dev_graph_seal", C.byref(d), 1)
    assert d.seal == dg.desc.seal != 0
    # the locality-ordered arrays under the ascending-id graph's checksums:
    # sizes and the checksum pairing agree, the content does not
    d = _desc(dg, graph_checksum=g_id.graph_checksum, plan_checksum=g_id.plan_checksum,
              plan_graph_checksum=g_id.plan_graph_checksum)
    with pytest.raises(MPError) as e:
        call("mp_dev_graph_seal", C.byref(d), 1)
    assert e.value.code == MP_EPLAN and d.seal == 0
    call("mp_dev_graph_seal", C.byref(d), 0)  # without reading back, the claim is taken on trust
    # the ascending-id graph's halo plan uploaded beside the locality CSR
    member_id = torch.from_numpy(g_id.member).cuda()
    d = _desc(dg, member=member_id.data_ptr())
    with pytest.raises(MPError) as e:
        call("mp_dev_graph_seal", C.byref(d), 1)
    assert e.value.code == MP_EPLAN
    # one sender index changed on the device after upload
    col = dg.col.clone()
    col[5] = (int(col[5]) + 1) % g_rcm.n_rows
    d = _desc(dg, col=col.data_ptr())
    with pytest.raises(MPError) as e:
        call("mp_dev_graph_seal", C.byref(d), 1)
    assert e.value.code == MP_EPLAN
    # one degree changed
    em = dg.edge_mult.clone()
    em[-1] = int(em[-1]) + 1
    d = _desc(dg, edge_mult=em.data_ptr())
    with pytest.raises(MPError) as e:
        call("mp_dev_graph_seal", C.byref(d), 1)
    assert e.value.code == MP_EPLAN
    torch.cuda.synchronize()
