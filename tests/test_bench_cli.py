"""bench.py's command-line contract that holds without a GPU: more than one
GPU is refused with a JSON message and exit status 2; the byte model and
the recorded-traffic lookup behave as documented."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_edge_adjoint_byte_model():
    sys.path.insert(0, ROOT)
    from paper_2410_01657_amd.roofline import layer_kernels
    N, E, H = 629856, 3538080, 64
    w = layer_kernels(N, E, 98415, 196830, H, "bf16", 4)["edge_bwd"]
    # e (4H) + 3/4 of the layers' g_e' (4H) + g_e (4H) + BF16 g_h (2H) + 9 index bytes per edge,
    # P, Q, g_a read and g_P written per row
    assert w.bytes == E * (4 * H + 3 * H + 4 * H + 2 * H + 9) + N * 16 * H
    w32 = layer_kernels(N, E, 98415, 196830, H, "f32", 1)["edge_bwd"]
    assert w32.bytes == E * (16 * H + 9) + N * 16 * H
    assert w.flops == E * 12 * H * H


def test_recorded_traffic_requires_matching_sources(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    # a workload or kernel without a record gives None
    assert bench.recorded_traffic("edge_bwd", "no-such-workload") is None
    assert bench.recorded_traffic("gq", "C1") is None
    sha = bench.sources_sha256("edge_bwd")
    assert len(sha) == 64 and sha == bench.sources_sha256("edge_bwd")


def test_split_adjoints_are_counted_where_their_products_run():
    """At H > 64 the edge and node adjoints run in two passes: the products
    are charged to the pass that executes them, and the total over the
    passes equals the fused form's count (6 H x H products per edge, 9 per
    node-update row; the sender-side pass 4 per row)."""
    sys.path.insert(0, ROOT)
    from paper_2410_01657_amd.roofline import layer_kernels, layer_roof_seconds
    N, E, G, M = 1771561, 10541520, 0, 0
    for gemm in ("bf16", "f32"):
        w64 = layer_kernels(N, E, G, M, 64, gemm, 4)
        assert "edge_dw" not in w64 and "node_dw" not in w64 and "gq_dw" not in w64
        H = 128
        w = layer_kernels(N, E, G, M, H, gemm, 4)
        assert w["edge_bwd"].flops == E * 8 * H * H
        assert w["edge_dw"].flops == E * 4 * H * H
        assert w["edge_bwd"].flops + w["edge_dw"].flops == E * 12 * H * H
        assert w["node_bwd"].flops + w["node_dw"].flops == N * 18 * H * H
        gq = w["gq"].flops + w.get("gq_dw", w["gq"].__class__(0, 0)).flops
        assert gq == N * 8 * H * H
        assert ("gq_dw" in w) == (gemm == "f32")
    # the layer roofline is the sum over kernels of the higher floor, per layer
    t = layer_roof_seconds(N, E, G, M, 128, "f32", 4)
    assert 0.09 < t < 0.11  # C3, FP32: about 25 ms of matrix time per layer


def test_bf16_edge_states_change_only_the_edge_state_bytes():
    """BF16 edge-state storage halves the bytes of e, e', g_e' and g_e in
    the edge kernels (and of e in the split weight-gradient pass); node
    arrays, flops and every other kernel are unchanged."""
    sys.path.insert(0, ROOT)
    from paper_2410_01657_amd.roofline import layer_kernels
    N, E, G, M = 11852352, 69866496, 449577, 911304
    for H in (64, 128):
        a = layer_kernels(N, E, G, M, H, "bf16", 4)
        b = layer_kernels(N, E, G, M, H, "bf16", 4, "bf16")
        assert a.keys() == b.keys()
        ge = 3 / 4  # three of four layers receive g_e'
        assert a["edge_fwd"].bytes - b["edge_fwd"].bytes == E * 2 * H * 2
        assert abs((a["edge_bwd"].bytes - b["edge_bwd"].bytes) - E * (2 + ge) * H * 2) < 1
        if H > 64:
            assert a["edge_dw"].bytes - b["edge_dw"].bytes == E * H * 2
        for k in a:
            assert a[k].flops == b[k].flops
            if k not in ("edge_fwd", "edge_bwd", "edge_dw"):
                assert a[k].bytes == b[k].bytes, k
