"""GPU parity of the consistent NMP layer against the FP64 oracle.

Every comparison runs the library through its C ABI and the oracle on the
same seeded inputs.  Tolerances are normwise, max|gpu - oracle| / max|oracle|:
FP32 forward 1e-5 (one layer), FP32 gradients 1e-4, BF16 GEMMs 3e-2.
Integer-valued aggregation checks are bitwise.
"""

import numpy as np
import pytest
import torch

from mpinputs import CONFIGS, ModelSpec, block_partition, box_mesh, make_inputs, rcb_partition
from oracle.graph import lattice_graph, partition_graph, halo_lists
from oracle.nmp import nmp_layer_bwd, nmp_layer_fwd

from _util import layer_params, normwise, split_rows

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _graphs(mesh, part, R):
    from paper_2410_01657_amd import DeviceGraph, build_graph
    hg = build_graph(mesh.elem_gid, mesh.P, part, R, order="gid")  # rows as the oracle's
    og, copies = partition_graph(mesh.elem_gid, mesh.P, part, R)
    return DeviceGraph(hg, DEV), og, halo_lists(og, copies)


@pytest.fixture(scope="module")
def c0():
    inp = make_inputs(CONFIGS["C0"])
    out = {}
    for R in (1, 8):
        part = np.zeros(inp.mesh.n_elem, np.int32) if R == 1 else inp.elem_part
        out[R] = _graphs(inp.mesh, part, R)
    return inp, out


@pytest.fixture(scope="module")
def rcb():
    nel = (6, 5, 4)
    m = box_mesh(nel, 3)
    part, _ = rcb_partition(nel, 8, seed=11, ratio=(1.0, 10.0))
    return m, _graphs(m, part, 8)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _lib_params(o, names):
    return {k: _t(o[v]) for k, v in names.items()}


# ------------------------------------------------------------ exact sums


def test_halo_sum_exact_in_degree(c0):
    """Zero weights, b2 = 1, e = 0: every edge state becomes 1, so a* is
    the global in-degree exactly, at every copy (1/d is a power of two)."""
    from paper_2410_01657_amd.ops import layer_cfg, layer_forward
    inp, gs = c0
    dg, og, _ = gs[8]
    H = 32
    _, o, names = layer_params(H, False)
    p = {k: torch.zeros_like(_t(o[v])) for k, v in names.items()}
    p["be2"] += 1.0
    x = torch.randn(dg.n_rows, H, device=DEV)
    e = torch.zeros(dg.n_edges, H, device=DEV)
    _, _, a_star = layer_forward(layer_cfg(H, False), p, dg, x, e)
    n = inp.mesh.npts[0]
    gid = dg.host.row_gid
    I, J, K = gid % n, (gid // n) % n, gid // (n * n)
    deg = sum((c > 0).astype(np.int64) + (c < n - 1).astype(np.int64) for c in (I, J, K))
    a = a_star.cpu().numpy()
    assert np.array_equal(a, np.repeat(deg[:, None].astype(np.float32), H, axis=1))


@pytest.mark.parametrize("which", ["c0", "rcb"])
def test_halo_sum_integer_messages(c0, rcb, which):
    """Zero weights and biases: e' = e.  With integer messages the
    consistent aggregate equals the R=1 integer sum bitwise (C0 blocks) or
    to rounding of 1/3 (T-junctions)."""
    from paper_2410_01657_amd.ops import layer_cfg, layer_forward
    if which == "c0":
        mesh, (dg, og, _) = c0[0].mesh, c0[1][8]
    else:
        mesh, (dg, og, _) = rcb
    H = 32
    _, o, names = layer_params(H, False)
    p = {k: torch.zeros_like(_t(o[v])) for k, v in names.items()}
    gid = dg.host.row_gid
    msg = ((gid[dg.host.recv] + 3 * gid[dg.host.col]) % 17).astype(np.float32)
    e = _t(np.repeat(msg[:, None], H, axis=1))
    x = torch.zeros(dg.n_rows, H, device=DEV)
    _, e_out, a_star = layer_forward(layer_cfg(H, False), p, dg, x, e)
    assert torch.equal(e_out, e)
    L = lattice_graph(mesh.npts)
    ref = np.zeros(L.n)
    np.add.at(ref, L.recv, (L.gid[L.recv] + 3 * L.gid[L.send]) % 17)
    a = a_star.cpu().numpy()[:, 0]
    if which == "c0":
        assert np.array_equal(a, ref[gid].astype(np.float32))
    else:
        np.testing.assert_allclose(a, ref[gid], rtol=1e-6, atol=0)


# ----------------------------------------------------- one-layer parity


def _oracle_layer(o, spec, og, pairs, x, e, halo=True):
    xs = split_rows(x.astype(np.float64), [0] + list(np.cumsum([G.n for G in og])))
    es = split_rows(e.astype(np.float64), [0] + list(np.cumsum([G.e for G in og])))
    xo, eo, cache = nmp_layer_fwd(o, 0, spec, og, pairs, xs, es, halo)
    return np.concatenate(xo), np.concatenate(eo), np.concatenate(cache["a_star"]), cache, xs, es


@pytest.mark.parametrize("H,ln,R,halo", [(32, False, 8, True), (32, True, 1, True), (64, True, 8, True),
                                         (128, True, 8, True), (64, False, 8, False)])
def test_layer_forward_fp32(c0, H, ln, R, halo):
    from paper_2410_01657_amd.ops import layer_cfg, layer_forward
    inp, gs = c0
    dg, og, pairs = gs[R]
    spec, o, names = layer_params(H, ln)
    rng = np.random.default_rng(H + R)
    x = rng.standard_normal((dg.n_rows, H)).astype(np.float32)
    e = rng.standard_normal((dg.n_edges, H)).astype(np.float32)
    xg, eg, ag = layer_forward(layer_cfg(H, ln, halo), _lib_params(o, names), dg, _t(x), _t(e))
    xr, er, ar, *_ = _oracle_layer(o, spec, og, pairs, x, e, halo)
    tol = 1e-5
    assert normwise(ag.cpu().numpy(), ar) < tol
    assert normwise(eg.cpu().numpy(), er) < tol
    assert normwise(xg.cpu().numpy(), xr) < tol


@pytest.mark.parametrize("H,ln", [(32, False), (64, True), (128, True)])
def test_layer_forward_bf16(c0, H, ln):
    from paper_2410_01657_amd.ops import layer_cfg, layer_forward
    inp, gs = c0
    dg, og, pairs = gs[8]
    spec, o, names = layer_params(H, ln)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((dg.n_rows, H)).astype(np.float32)
    e = rng.standard_normal((dg.n_edges, H)).astype(np.float32)
    xg, eg, ag = layer_forward(layer_cfg(H, ln, gemm="bf16"), _lib_params(o, names), dg, _t(x), _t(e))
    xr, er, ar, *_ = _oracle_layer(o, spec, og, pairs, x, e)
    for got, ref in ((ag, ar), (eg, er), (xg, xr)):
        err = normwise(got.cpu().numpy(), ref)
        assert 1e-6 < err < 3e-2, err  # rounded (not silently FP32) and close


def test_layer_forward_rcb(rcb):
    from paper_2410_01657_amd.ops import layer_cfg, layer_forward
    m, (dg, og, pairs) = rcb
    H = 64
    spec, o, names = layer_params(H, True)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((dg.n_rows, H)).astype(np.float32)
    e = rng.standard_normal((dg.n_edges, H)).astype(np.float32)
    xg, eg, ag = layer_forward(layer_cfg(H, True), _lib_params(o, names), dg, _t(x), _t(e))
    xr, er, ar, *_ = _oracle_layer(o, spec, og, pairs, x, e)
    assert normwise(ag.cpu().numpy(), ar) < 1e-5
    assert normwise(xg.cpu().numpy(), xr) < 1e-5


# ---------------------------------------------------- one-layer adjoint


# H=128 runs the split adjoints (per-edge / per-row factors + separate
# weight-gradient sums; the node update's split form is BF16 only); the
# other widths the fused kernels.  no_ge: the last layer's case,
# no gradient at the edge output.
@pytest.mark.parametrize("H,ln,R,gemm,no_ge", [(32, False, 8, "f32", False), (64, True, 8, "f32", False),
                                               (64, True, 1, "f32", False), (128, True, 8, "f32", False),
                                               (64, True, 8, "bf16", False), (128, True, 8, "bf16", False),
                                               (128, False, 1, "f32", True), (64, True, 8, "bf16", True),
                                               (128, False, 8, "bf16", False)])
def test_layer_backward(c0, H, ln, R, gemm, no_ge):
    from paper_2410_01657_amd.ops import layer_backward, layer_cfg, layer_forward
    inp, gs = c0
    dg, og, pairs = gs[R]
    spec, o, names = layer_params(H, ln)
    rng = np.random.default_rng(11 + H)
    x = rng.standard_normal((dg.n_rows, H)).astype(np.float32)
    e = rng.standard_normal((dg.n_edges, H)).astype(np.float32)
    gx = rng.standard_normal((dg.n_rows, H)).astype(np.float32)
    ge = rng.standard_normal((dg.n_edges, H)).astype(np.float32)
    if no_ge:
        ge[:] = 0.0
    cfg = layer_cfg(H, ln, gemm=gemm)
    p = _lib_params(o, names)
    _, _, a_star = layer_forward(cfg, p, dg, _t(x), _t(e))
    g_x, g_e, grads = layer_backward(cfg, p, dg, _t(x), _t(e), a_star, _t(gx), None if no_ge else _t(ge))
    xr, er, ar, cache, xs, es = _oracle_layer(o, spec, og, pairs, x, e)
    n_off = [0] + list(np.cumsum([G.n for G in og]))
    e_off = [0] + list(np.cumsum([G.e for G in og]))
    ogr = {}
    gxs, ges = nmp_layer_bwd(o, 0, spec, og, pairs, cache, split_rows(gx.astype(np.float64), n_off),
                             split_rows(ge.astype(np.float64), e_off), ogr)
    tol = 1e-4 if gemm == "f32" else 5e-2
    assert normwise(g_x.cpu().numpy(), np.concatenate(gxs)) < tol
    assert normwise(g_e.cpu().numpy(), np.concatenate(ges)) < tol
    for k, v in names.items():
        err = normwise(grads[k].cpu().numpy(), ogr[v])
        assert err < tol, (k, err)


@pytest.mark.parametrize("H,gemm", [(64, "f32"), (128, "bf16")])
def test_layer_deterministic(c0, H, gemm):
    from paper_2410_01657_amd.ops import layer_backward, layer_cfg, layer_forward
    inp, gs = c0
    dg, og, pairs = gs[8]
    spec, o, names = layer_params(H, True)
    rng = np.random.default_rng(0)
    x, e = _t(rng.standard_normal((dg.n_rows, H))), _t(rng.standard_normal((dg.n_edges, H)))
    gx, ge = _t(rng.standard_normal((dg.n_rows, H))), _t(rng.standard_normal((dg.n_edges, H)))
    cfg = layer_cfg(H, True, gemm=gemm)
    p = _lib_params(o, names)
    runs = []
    for _ in range(2):
        xo, eo, a = layer_forward(cfg, p, dg, x, e)
        g = layer_backward(cfg, p, dg, x, e, a, gx, ge)
        runs.append([xo, eo, a, g[0], g[1]] + [g[2][k] for k in sorted(names)])
    for a, b in zip(*runs):
        assert torch.equal(a, b)


@pytest.mark.parametrize("H,gemm", [(64, "bf16"), (128, "f32")])
def test_layer_backward_with_forward_projections(c0, H, gemm):
    """The backward given the forward's node projections (pq) equals the
    backward that recomputes them, bit for bit (same kernel, same inputs)."""
    from paper_2410_01657_amd.ops import layer_backward, layer_cfg, layer_forward
    inp, gs = c0
    dg, og, pairs = gs[8]
    spec, o, names = layer_params(H, True)
    rng = np.random.default_rng(5)
    x, e = _t(rng.standard_normal((dg.n_rows, H))), _t(rng.standard_normal((dg.n_edges, H)))
    gx, ge = _t(rng.standard_normal((dg.n_rows, H))), _t(rng.standard_normal((dg.n_edges, H)))
    cfg = layer_cfg(H, True, gemm=gemm)
    p = _lib_params(o, names)
    xo, eo, a, pq = layer_forward(cfg, p, dg, x, e, want_pq=True)
    xo2, eo2, a2 = layer_forward(cfg, p, dg, x, e)
    assert torch.equal(xo, xo2) and torch.equal(eo, eo2) and torch.equal(a, a2)
    g1 = layer_backward(cfg, p, dg, x, e, a, gx, ge, pq)
    g2 = layer_backward(cfg, p, dg, x, e, a, gx, ge)
    assert torch.equal(g1[0], g2[0]) and torch.equal(g1[1], g2[1])
    for k in names:
        assert torch.equal(g1[2][k], g2[2][k]), k


@pytest.mark.parametrize("gemm", ["f32", "bf16"])
def test_layer_forward_without_edge_output(c0, gemm):
    """A last layer's e' is read by nothing: with e_out = NULL the kernels
    skip its store, and x', a* (whose Eq. 4b sum still uses e') are bitwise
    those of the full forward; the adjoint without g_e' is unchanged."""
    from paper_2410_01657_amd.ops import layer_backward, layer_cfg, layer_forward
    inp, gs = c0
    dg, og, pairs = gs[8]
    H = 64
    spec, o, names = layer_params(H, True)
    rng = np.random.default_rng(9)
    x, e = _t(rng.standard_normal((dg.n_rows, H))), _t(rng.standard_normal((dg.n_edges, H)))
    gx = _t(rng.standard_normal((dg.n_rows, H)))
    cfg = layer_cfg(H, True, gemm=gemm)
    p = _lib_params(o, names)
    xo, eo, a, pq = layer_forward(cfg, p, dg, x, e, want_pq=True)
    xo2, eo2, a2, pq2 = layer_forward(cfg, p, dg, x, e, want_pq=True, want_e=False)
    assert eo2 is None
    assert torch.equal(xo, xo2) and torch.equal(a, a2) and torch.equal(pq, pq2)
    g1 = layer_backward(cfg, p, dg, x, e, a, gx, None, pq)
    g2 = layer_backward(cfg, p, dg, x, e, a2, gx, None, pq2)
    assert torch.equal(g1[0], g2[0]) and torch.equal(g1[1], g2[1])


# ------------------------------------------- BF16 edge-state storage


def _bf16(a):
    """FP32 array -> BF16 tensor on the device (round to nearest even)."""
    return _t(a).to(torch.bfloat16)


@pytest.mark.parametrize("H,ln,agg,R", [(32, False, "state", 8), (64, True, "state", 8), (64, True, "message", 1),
                                        (128, True, "state", 8), (128, False, "message", 8)])
def test_edge_state_bf16_is_the_rounded_fp32_state(c0, H, ln, agg, R):
    """BF16 edge-state storage changes only what is stored: given the same
    BF16-representable e and g_e', the layer computes exactly what the
    FP32-state layer computes (x', a*, P/Q, g_x and every parameter
    gradient bitwise equal) and stores e' and g_e rounded to nearest even."""
    from paper_2410_01657_amd.ops import layer_backward, layer_cfg, layer_forward
    dg, og, pairs = c0[1][R]
    spec, o, names = layer_params(H, ln)
    rng = np.random.default_rng(40 + H)
    x = _t(rng.standard_normal((dg.n_rows, H)))
    e16 = _bf16(rng.standard_normal((dg.n_edges, H)))
    gx = _t(rng.standard_normal((dg.n_rows, H)))
    ge16 = _bf16(rng.standard_normal((dg.n_edges, H)))
    p = _lib_params(o, names)
    c32 = layer_cfg(H, ln, gemm="bf16", aggregate=agg)
    c16 = layer_cfg(H, ln, gemm="bf16", aggregate=agg, estate="bf16")
    xo, eo, a, pq = layer_forward(c32, p, dg, x, e16.float(), want_pq=True)
    xo2, eo2, a2, pq2 = layer_forward(c16, p, dg, x, e16, want_pq=True)
    assert eo2.dtype == torch.bfloat16
    assert torch.equal(xo, xo2) and torch.equal(a, a2) and torch.equal(pq, pq2)
    assert torch.equal(eo.to(torch.bfloat16), eo2)
    for g_e_out in (ge16, None):   # a middle layer, and a last layer (no g_e')
        g1 = layer_backward(c32, p, dg, x, e16.float(), a, gx, None if g_e_out is None else g_e_out.float(), pq)
        g2 = layer_backward(c16, p, dg, x, e16, a2, gx, g_e_out, pq2)
        assert g2[1].dtype == torch.bfloat16
        assert torch.equal(g1[0], g2[0])
        assert torch.equal(g1[1].to(torch.bfloat16), g2[1])
        for k in names:
            assert torch.equal(g1[2][k], g2[2][k]), k


@pytest.mark.parametrize("H,ln,R", [(32, False, 8), (64, True, 8), (128, True, 1)])
def test_edge_state_bf16_against_the_oracle(c0, H, ln, R):
    """Forward and adjoint with BF16 edge states against the FP64 oracle
    (Eq. 4a-e, Eq. 3) on the same BF16-representable e and g_e', at the
    BF16-GEMM tolerances."""
    from paper_2410_01657_amd.ops import layer_backward, layer_cfg, layer_forward
    dg, og, pairs = c0[1][R]
    spec, o, names = layer_params(H, ln)
    rng = np.random.default_rng(70 + H)
    x = rng.standard_normal((dg.n_rows, H)).astype(np.float32)
    e16 = _bf16(rng.standard_normal((dg.n_edges, H)))
    gx = rng.standard_normal((dg.n_rows, H)).astype(np.float32)
    ge16 = _bf16(rng.standard_normal((dg.n_edges, H)))
    e, ge = e16.float().cpu().numpy(), ge16.float().cpu().numpy()
    cfg = layer_cfg(H, ln, gemm="bf16", estate="bf16")
    p = _lib_params(o, names)
    xg, eg, ag = layer_forward(cfg, p, dg, _t(x), e16)
    g_x, g_e, grads = layer_backward(cfg, p, dg, _t(x), e16, ag, _t(gx), ge16)
    xr, er, ar, cache, xs, es = _oracle_layer(o, spec, og, pairs, x, e)
    for got, ref in ((ag, ar), (eg, er), (xg, xr)):
        err = normwise(got.float().cpu().numpy(), ref)
        assert 1e-6 < err < 3e-2, err
    n_off = [0] + list(np.cumsum([G.n for G in og]))
    e_off = [0] + list(np.cumsum([G.e for G in og]))
    ogr = {}
    gxs, ges = nmp_layer_bwd(o, 0, spec, og, pairs, cache, split_rows(gx.astype(np.float64), n_off),
                             split_rows(ge.astype(np.float64), e_off), ogr)
    assert normwise(g_x.cpu().numpy(), np.concatenate(gxs)) < 5e-2
    assert normwise(g_e.float().cpu().numpy(), np.concatenate(ges)) < 5e-2
    for k, v in names.items():
        err = normwise(grads[k].cpu().numpy(), ogr[v])
        assert err < 5e-2, (k, err)


def test_edge_state_dtype_mismatch_is_rejected(c0):
    from paper_2410_01657_amd.ops import layer_cfg, layer_forward
    dg, og, pairs = c0[1][8]
    spec, o, names = layer_params(32, False)
    x = torch.zeros(dg.n_rows, 32, device=DEV)
    e = torch.zeros(dg.n_edges, 32, device=DEV)
    with pytest.raises(ValueError):
        layer_forward(layer_cfg(32, False, gemm="bf16", estate="bf16"), _lib_params(o, names), dg, x, e)
    with pytest.raises(ValueError):
        layer_forward(layer_cfg(32, False, gemm="bf16"), _lib_params(o, names), dg, x, e.to(torch.bfloat16))


@pytest.mark.parametrize("gemm", ["bf16", "f32"])
def test_split_adjoint_waves_per_workgroup(c0, gemm):
    """The split edge adjoint (H = 128) with 4 and with 8 waves per
    workgroup: the per-edge work is the same, so g_x and g_e are bitwise
    equal; the weight gradients differ only in the grouping of their sums
    (Eq. 3) and agree to FP32 rounding."""
    from paper_2410_01657_amd.ops import layer_backward, layer_cfg, layer_forward
    dg, og, pairs = c0[1][8]
    H = 128
    spec, o, names = layer_params(H, True)
    rng = np.random.default_rng(17)
    x, e = _t(rng.standard_normal((dg.n_rows, H))), _t(rng.standard_normal((dg.n_edges, H)))
    gx, ge = _t(rng.standard_normal((dg.n_rows, H))), _t(rng.standard_normal((dg.n_edges, H)))
    p = _lib_params(o, names)
    out = []
    for waves in (4, 8):
        cfg = layer_cfg(H, True, gemm=gemm)
        cfg.edge_bwd_waves = waves
        _, _, a = layer_forward(cfg, p, dg, x, e)
        out.append(layer_backward(cfg, p, dg, x, e, a, gx, ge))
    (gx4, ge4, w4), (gx8, ge8, w8) = out
    assert torch.equal(gx4, gx8) and torch.equal(ge4, ge8)
    for k in names:
        assert normwise(w4[k].cpu().numpy(), w8[k].cpu().numpy()) < 1e-5, k
