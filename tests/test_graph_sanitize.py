"""The host graph builder (csrc/mp_graph.cpp: graph_partition,
graph_order_rows, halo_plan_build) compiled with g++ under AddressSanitizer
and UndefinedBehaviorSanitizer, driven through tests/native/graph_driver.cpp
on hexahedral and tetrahedral partitions and on rejected inputs: no
sanitizer report, and the same arrays and checksums as the library build
(CPU only)."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from mpinputs.mesh import box_mesh
from mpinputs.tetmesh import centroid_partition, tet_mesh
from paper_2410_01657_amd.graph import build_graph, hex_links

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV = dict(os.environ,
           ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=97",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=98")
MP_EINVAL = 1


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("sanitize") / "graph_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-pthread",
           os.path.join(ROOT, "tests", "native", "graph_driver.cpp"),
           os.path.join(ROOT, "paper_2410_01657_amd", "csrc", "mp_graph.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    return exe


def _run(driver, tmp_path, elem_gid, links, part, R, order):
    eg = np.ascontiguousarray(elem_gid, np.int64)
    ln = np.ascontiguousarray(links, np.int32)
    pt = np.ascontiguousarray(part, np.int32)
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as f:
        f.write(np.array([eg.shape[0]], np.int64).tobytes())
        f.write(np.array([eg.shape[1], ln.shape[0], R, order], np.int32).tobytes())
        f.write(eg.tobytes() + ln.tobytes() + pt.tobytes())
    r = subprocess.run([driver, str(src), str(dst)], capture_output=True, text=True, env=ENV, timeout=600)
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    assert r.returncode not in (97, 98), r.stderr
    return r.returncode, (dst.read_bytes() if r.returncode == 0 else None)


def _parse(blob):
    types = [np.int64, np.int64, np.int64, np.int32, np.int32, np.int32, np.int32, np.uint8, np.uint8,
             np.int32, np.int32, np.int32, np.int32, np.int64, np.int32, np.int32, np.int64, np.int32, np.uint64]
    names = ["row_off", "edge_off", "row_gid", "rowptr", "recv", "col", "rev", "edge_mult", "node_mult",
             "group_ptr", "member", "pair_r", "pair_s", "pair_ptr", "pair_rows_r", "pair_rows_s", "halo_rows",
             "neighbours", "checksums"]
    out, o = {}, 0
    for n, t in zip(names, types):
        nb = int(np.frombuffer(blob, np.int64, 1, o)[0])
        out[n] = np.frombuffer(blob, t, nb // np.dtype(t).itemsize, o + 8)
        o += 8 + nb
    assert o == len(blob)
    return out


def _compare(got, hg):
    for k in got:
        if k != "checksums":
            assert np.array_equal(got[k], getattr(hg, k)), k
    assert list(got["checksums"]) == [hg.graph_checksum, hg.plan_checksum, hg.plan_graph_checksum]


@pytest.mark.parametrize("order", ["gid", "locality"])
def test_hex_partition_under_sanitizers(driver, tmp_path, order):
    m = box_mesh((4, 3, 5), 3, with_positions=False)
    # scattered parts: every sub-graph is split, most nodes are halo nodes
    part = np.random.Generator(np.random.PCG64(5)).integers(0, 7, m.n_elem).astype(np.int32)
    assert np.unique(part).size == 7
    rc, blob = _run(driver, tmp_path, m.elem_gid, hex_links(3), part, 7, int(order == "locality"))
    assert rc == 0
    _compare(_parse(blob), build_graph(m.elem_gid, 3, part, 7, order=order))


def test_periodic_hex_partition_under_sanitizers(driver, tmp_path):
    m = box_mesh((3, 4, 4), 2, periodic=(True, False, True), with_positions=False)
    part = (np.arange(m.n_elem) % 5).astype(np.int32)
    rc, blob = _run(driver, tmp_path, m.elem_gid, hex_links(2), part, 5, 1)
    assert rc == 0
    _compare(_parse(blob), build_graph(m.elem_gid, 2, part, 5, order="locality"))


def test_tet_partition_under_sanitizers(driver, tmp_path):
    m = tet_mesh(300, seed=4)
    part = centroid_partition(m, 8)
    rc, blob = _run(driver, tmp_path, m.elem_gid, m.links, part, 8, 1)
    assert rc == 0
    _compare(_parse(blob), build_graph(m.elem_gid, None, part, 8, m.links, order="locality"))


def test_rejected_inputs_under_sanitizers(driver, tmp_path):
    m = box_mesh((2, 2, 2), 2, with_positions=False)
    links, part = hex_links(2), np.zeros(m.n_elem, np.int32)
    bad_gid = m.elem_gid.copy()
    bad_gid[1, 3] = -4                                     # id out of range
    bad_part = part.copy()
    bad_part[2] = 3                                        # part out of range for R = 2
    self_link = np.concatenate([links, [[5, 5]]]).astype(np.int32)
    bad_link = np.concatenate([links, [[0, m.npe]]]).astype(np.int32)
    for gid, lk, pt, R in [(bad_gid, links, part, 1), (m.elem_gid, links, bad_part, 2),
                           (m.elem_gid, self_link, part, 1), (m.elem_gid, bad_link, part, 1),
                           (m.elem_gid, links, part, 2)]:  # the last: sub-graph 1 is empty
        rc, _ = _run(driver, tmp_path, gid, lk, pt, R, 1)
        assert rc == MP_EINVAL
