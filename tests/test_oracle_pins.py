"""Pins for the FP64 oracle: facts fixed by the paper and by mathematics.

Each test checks the oracle (or the shared input generators) against
something other than itself: closed forms, numbers the paper prints,
exact integer arithmetic, brute-force loops, hand-computed values,
symmetries, and central finite differences.
"""

import json
import math
import os

import numpy as np
import pytest

from mpinputs import (CONFIGS, ModelSpec, box_mesh, block_partition, count_params,
                      gll_points, init_params, make_inputs, rcb_partition,
                      slab_partition, velocity_field)
from oracle.graph import lattice_graph, partition_graph, halo_lists, table2_stats
from oracle.nmp import (consistent_loss, edge_inputs, elu, elu_deriv, halo_sync,
                        halo_sync_adj, layer_norm_fwd, local_aggregate, local_aggregate_adj,
                        mlp_fwd, model_bwd, model_fwd, mse_loss, nmp_layer_fwd)
from oracle.problem import build_problem
from oracle.ball import ball_output, ball_grad

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as f:
        return json.load(f)


def normwise(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# ---------------------------------------------------------------- P1 mesh


def test_gll_closed_forms():
    s5 = math.sqrt(5.0)
    np.testing.assert_allclose(gll_points(1), [-1, 1], atol=0)
    np.testing.assert_allclose(gll_points(2), [-1, 0, 1], atol=1e-16)
    np.testing.assert_allclose(gll_points(3), [-1, -1 / s5, 1 / s5, 1], atol=1e-15)
    r7 = 2 * math.sqrt(7.0) / 21
    a, b = math.sqrt(1 / 3 - r7), math.sqrt(1 / 3 + r7)
    np.testing.assert_allclose(gll_points(5), [-1, -b, -a, a, b, 1], atol=1e-15)
    np.testing.assert_allclose(
        gll_points(7)[4:],
        [0.209299217902479, 0.591700181433142, 0.871740148509607, 1.0], atol=1e-14)


def test_gll_quadrature_exactness():
    """GLL weights 2/(P(P+1) P_P(x)^2) integrate degree <= 2P-1 exactly."""
    for P in (3, 5, 7):
        x = gll_points(P)
        leg = np.polynomial.legendre.legval(x, [0] * P + [1])
        w = 2.0 / (P * (P + 1) * leg ** 2)
        for deg in range(2 * P):
            exact = (1 - (-1) ** (deg + 1)) / (deg + 1)
            assert abs(np.sum(w * x ** deg) - exact) < 1e-13


@pytest.mark.parametrize("name,n", [("C0", 13), ("C1", 81)])
def test_lattice_counts(name, n):
    cfg = CONFIGS[name]
    m = box_mesh(cfg.nel, cfg.P, with_positions=False)
    assert m.npts == (n, n, n)
    G = lattice_graph(m.npts)
    assert G.n == n ** 3
    assert G.e == 6 * n * n * (n - 1)
    assert G.e == {"C0": 12168, "C1": 3149280}[name]


def test_closed_form_counts_large():
    for n, e in ((121, 10541520), (225, 68040000)):
        assert 6 * n * n * (n - 1) == e


def test_element_route_equals_lattice_definition():
    cfg = CONFIGS["C0"]
    m = box_mesh(cfg.nel, cfg.P)
    L = lattice_graph(m.npts)
    (G,), copies = partition_graph(m.elem_gid, m.P, np.zeros(m.n_elem, np.int32), 1)
    assert copies == {}
    np.testing.assert_array_equal(G.gid, L.gid)
    np.testing.assert_array_equal(G.recv, L.recv)
    np.testing.assert_array_equal(G.send, L.send)
    assert np.all(G.d_edge == 1) and np.all(G.d_node == 1)


def test_partition_sizes_c0_r8():
    inp = make_inputs(CONFIGS["C0"])
    graphs, copies = partition_graph(inp.mesh.elem_gid, 3, inp.elem_part, 8)
    assert sum(g.n for g in graphs) == 2744
    assert sum(g.e for g in graphs) == 14112
    assert len(copies) == 469
    assert sum(len(v) for v in copies.values()) == 1016
    # tensor-product cut: edge degrees are 1, 2 or 4 (face or line of blocks)
    assert set(np.unique(np.concatenate([g.d_edge for g in graphs]))) == {1.0, 2.0, 4.0}


@pytest.mark.slow
def test_partition_sizes_c1_r16():
    cfg = CONFIGS["C1"]
    m = box_mesh(cfg.nel, cfg.P, with_positions=False)
    graphs, copies = partition_graph(m.elem_gid, 5, slab_partition(cfg.nel, 16), 16)
    assert sum(g.n for g in graphs) == 629856
    assert sum(g.e for g in graphs) == 3538080
    assert len(copies) == 98415
    assert sum(len(v) for v in copies.values()) == 196830


# ------------------------------------------------------- P8, P9 paper numbers


def test_table1_param_counts():
    g = _golden()["table1_param_counts"]
    for key in ("small", "large"):
        row = g[key]
        spec = ModelSpec(H=row["H"], n_layers=row["message_passing_layers"],
                         n_hidden=row["mlp_hidden_layers"], layernorm=True,
                         node_in=3, edge_in=4, out=3)
        assert count_params(spec) == row["trainable_parameters"]


@pytest.mark.slow
def test_table2_r8_row():
    """16 x 16 x 128 periodic p=5 elements in 8 z-slabs reproduce Table II R=8."""
    g = _golden()
    row = g["table2_r8_row"]
    nel = (16, 16, 128)
    m = box_mesh(nel, 5, periodic=(True, True, True), with_positions=False)
    graphs, copies = partition_graph(m.elem_gid, 5, slab_partition(nel, 8), 8)
    rows, halo, nbrs = table2_stats(graphs, copies)
    assert np.all(rows == 518400)
    assert round(rows[0] / 1000) == row["graph_nodes_thousands"]
    assert np.all(halo == 12800)
    assert halo[0] / 1000 == row["halo_nodes_thousands"]
    assert np.all(nbrs == row["neighbors"])
    total = int(rows.sum())
    assert total == 4147200
    assert round(total / 1e4) * 1e4 == g["total_nodes_r8"]["value"]


# ------------------------------------------------- P2, P3 aggregation sums


def test_aggregate_brute_force_loop():
    """Eq. 4b on a 2^3-element P=2 mesh, R=4, against an explicit loop."""
    m = box_mesh((2, 2, 2), 2)
    part = block_partition((2, 2, 2), (2, 2, 1))
    graphs, _ = partition_graph(m.elem_gid, 2, part, 4)
    rng = np.random.default_rng(3)
    for G in graphs:
        e = rng.standard_normal((G.e, 3))
        a = local_aggregate(e, G)
        for i in range(G.n):
            s = [0.0, 0.0, 0.0]
            for k in range(G.e):
                if G.recv[k] == i:
                    for c in range(3):
                        s[c] += e[k, c] / G.d_edge[k]
            assert np.allclose(a[i], s, rtol=0, atol=1e-14)


def test_aggregate_vs_per_node_search_c0():
    inp = make_inputs(CONFIGS["C0"])
    G = lattice_graph(inp.mesh.npts)
    e = np.random.default_rng(0).standard_normal((G.e, 4))
    a = local_aggregate(e, G)
    for i in range(0, G.n, 7):
        np.testing.assert_allclose(a[i], e[G.recv == i].sum(0), rtol=0, atol=1e-13)


def _global_in_degree(npts, gid):
    nx, ny, nz = npts
    I, J, K = gid % nx, (gid // nx) % ny, gid // (nx * ny)
    deg = np.zeros(gid.shape, np.int64)
    for c, n in ((I, nx), (J, ny), (K, nz)):
        deg += (c > 0).astype(np.int64) + (c < n - 1).astype(np.int64)
    return deg


@pytest.mark.parametrize("kind", ["blocks", "rcb"])
def test_exact_integer_halo_sums(kind):
    """Integer messages: a* at every copy equals the unpartitioned sum exactly.

    With m = 1 the consistent aggregate is the global in-degree (6 inside,
    5 on faces, 4 on edges, 3 at corners of the box).  With integer messages
    (gid_i + 3 gid_j) mod 17 it equals the R=1 integer sum bit for bit.
    Seeded RCB cuts give T-junctions with edge degree 3.
    """
    if kind == "blocks":
        nel, P, R = (4, 4, 4), 3, 8
        part = block_partition(nel, (2, 2, 2))
    else:
        nel, P, R = (6, 5, 4), 2, 8
        part, _ = rcb_partition(nel, R, seed=11, ratio=(1.0, 10.0))
    m = box_mesh(nel, P)
    graphs, copies = partition_graph(m.elem_gid, P, part, R)
    pairs = halo_lists(graphs, copies)
    if kind == "rcb":
        assert 3.0 in set(np.concatenate([g.d_edge for g in graphs]))
    # m = 1 on every edge copy, each weighted by 1/d: the sum counts edges once
    # (1/3 is inexact in binary, so T-junction sums are exact only to rounding)
    check = (np.testing.assert_array_equal if kind == "blocks" else
             (lambda a, b: np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)))
    a = [local_aggregate(np.ones((G.e, 1)), G) for G in graphs]
    a_star = halo_sync(a, pairs)
    for G, s in zip(graphs, a_star):
        check(s[:, 0], _global_in_degree(m.npts, G.gid))
    L = lattice_graph(m.npts)
    ref = np.zeros(L.n)
    np.add.at(ref, L.recv, (L.gid[L.recv] + 3 * L.gid[L.send]) % 17)
    msgs = [((G.gid[G.recv] + 3 * G.gid[G.send]) % 17).astype(np.float64)[:, None]
            for G in graphs]
    a_star = halo_sync([local_aggregate(mm, G) for mm, G in zip(msgs, graphs)], pairs)
    for G, s in zip(graphs, a_star):
        check(s[:, 0], ref[G.gid])


# --------------------------------------------- P4, P7, P12 consistency (Eq. 2)


def _c0(perturb=True):
    return make_inputs(CONFIGS["C0"], perturb=perturb)


def _run(inp, R, part=None, halo=True):
    prob = build_problem(inp.mesh, inp.field, inp.target, part, R)
    Y, cache = model_fwd(inp.params, inp.cfg.spec, prob.graphs, prob.pair_lists,
                         prob.X, prob.E0, halo=halo)
    return prob, Y, cache


def _copy_error(prob, Y, Y1):
    num = max(np.abs(Y[r] - Y1[G.gid]).max() for r, G in enumerate(prob.graphs))
    return num / np.abs(Y1).max()


@pytest.fixture(scope="module")
def c0_ref():
    inp = _c0()
    prob, Y, _ = _run(inp, 1)
    return inp, Y[0]


@pytest.mark.parametrize("blocks", [(2, 1, 1), (2, 2, 2), (4, 2, 2), (4, 4, 4)])
def test_consistency_blocks(c0_ref, blocks):
    inp, Y1 = c0_ref
    R = int(np.prod(blocks))
    part = block_partition(inp.mesh.nel, blocks)
    prob, Y, _ = _run(inp, R, part)
    assert _copy_error(prob, Y, Y1) <= 1e-12


def test_consistency_rcb_t_junctions():
    cfg = CONFIGS["C0"]
    inp = make_inputs(cfg, perturb=True)
    part, _ = rcb_partition(cfg.nel, 8, seed=5, ratio=(1.0, 10.0))
    prob, Y, _ = _run(inp, 8, part)
    _, Y1, _ = _run(inp, 1)
    assert _copy_error(prob, Y, Y1[0]) <= 1e-12


def test_none_mode_inconsistent_and_grows_with_r(c0_ref):
    """Without the halo exchange the error is large and grows with R."""
    inp, Y1 = c0_ref
    errs = []
    for blocks in [(2, 1, 1), (2, 2, 2), (4, 4, 4)]:
        part = block_partition(inp.mesh.nel, blocks)
        prob, Y, _ = _run(inp, int(np.prod(blocks)), part, halo=False)
        # the error over all copies, in the sense of the loss (Eq. 6)
        L, _, _ = consistent_loss(Y, [Y1[G.gid] for G in prob.graphs], prob.graphs)
        errs.append(L)
    assert errs[0] > 1e-6
    assert errs[0] < errs[1] < errs[2]


def test_consistent_loss_equals_mse(c0_ref):
    inp, Y1 = c0_ref
    L1, _ = mse_loss(Y1, inp.target.astype(np.float64))
    part = block_partition(inp.mesh.nel, (2, 2, 2))
    prob, Y, _ = _run(inp, 8, part)
    L8, _, n_eff = consistent_loss(Y, prob.T, prob.graphs)
    assert abs(n_eff - inp.mesh.n_gid) < 1e-9
    assert abs(L8 - L1) <= 1e-12 * abs(L1)


# ------------------------------------------------ P5, P6 gradients (Eq. 3)


def _tiny(perturb=True, ln=True, H=4, layers=2, hidden=0, aggregate="state", edge_in=4):
    spec = ModelSpec(H=H, n_layers=layers, n_hidden=hidden, layernorm=ln, aggregate=aggregate, edge_in=edge_in)
    m = box_mesh((2, 2, 1), 2)
    field = velocity_field(m.pos, 1, noise_sigma=0.05)
    params = init_params(spec, 2, perturb=perturb)
    return spec, m, field, params


def _loss_and_grads(spec, m, field, params, part, R):
    from mpinputs import shifted_target
    target = shifted_target(field, m.npts)
    prob = build_problem(m, field, target, part, R, unpartitioned_from_lattice=(R == 1), edge_in=spec.edge_in)
    Y, cache = model_fwd(params, spec, prob.graphs, prob.pair_lists, prob.X, prob.E0)
    L, gY, _ = consistent_loss(Y, prob.T, prob.graphs)
    grads, _ = model_bwd(params, spec, prob.graphs, prob.pair_lists, cache, gY)
    return L, grads


@pytest.mark.parametrize("ln,hidden,agg,edge_in", [(True, 0, "state", 4), (False, 0, "state", 4),
                                                    (True, 1, "state", 4), (True, 0, "message", 4),
                                                    (True, 1, "state", 7)])
def test_gradients_vs_central_differences(ln, hidden, agg, edge_in):
    spec, m, field, params = _tiny(ln=ln, hidden=hidden, aggregate=agg, edge_in=edge_in)
    part = block_partition((2, 2, 1), (2, 1, 1))
    L, grads = _loss_and_grads(spec, m, field, params, part, 2)
    rng = np.random.default_rng(7)
    for name in sorted(params):
        p = params[name]
        for _ in range(2):
            idx = tuple(rng.integers(0, s) for s in p.shape)
            # h = 1e-6: truncation error (~h^2) and rounding (~eps/h) both
            # stay near 1e-10, and a step this small rarely straddles the
            # kink of ELU's second derivative at 0
            h = 1e-6 * max(1.0, abs(float(p[idx])))
            pp = {k: v.astype(np.float64) for k, v in params.items()}
            pp[name][idx] += h
            Lp, _ = _loss_and_grads(spec, m, field, pp, part, 2)
            pp[name][idx] -= 2 * h
            Lm, _ = _loss_and_grads(spec, m, field, pp, part, 2)
            fd = (Lp - Lm) / (2 * h)
            g = grads[name][idx]
            assert abs(fd - g) <= 2e-8 * max(1.0, abs(g)), (name, idx, fd, g)


@pytest.mark.parametrize("agg,edge_in", [("state", 4), ("message", 4), ("state", 7)])
def test_gradient_consistency_r1_vs_r4(agg, edge_in):
    spec, m, field, params = _tiny(aggregate=agg, edge_in=edge_in)
    L1, g1 = _loss_and_grads(spec, m, field, params, None, 1)
    part = block_partition((2, 2, 1), (2, 2, 1))
    L4, g4 = _loss_and_grads(spec, m, field, params, part, 4)
    assert abs(L1 - L4) <= 1e-12 * abs(L1)
    for k in g1:
        assert normwise(g4[k], g1[k]) <= 1e-11, k


def test_adjoint_dot_products():
    inp = make_inputs(CONFIGS["C0"])
    part = block_partition(inp.mesh.nel, (2, 2, 2))
    graphs, copies = partition_graph(inp.mesh.elem_gid, 3, part, 8)
    pairs = halo_lists(graphs, copies)
    rng = np.random.default_rng(1)
    a = [rng.standard_normal((G.n, 5)) for G in graphs]
    b = [rng.standard_normal((G.n, 5)) for G in graphs]
    Sa, STb = halo_sync(a, pairs), halo_sync_adj(b, pairs)
    lhs = sum(np.sum(x * y) for x, y in zip(Sa, b))
    rhs = sum(np.sum(x * y) for x, y in zip(a, STb))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    for G in graphs:
        e = rng.standard_normal((G.e, 5))
        g = rng.standard_normal((G.n, 5))
        lhs = np.sum(local_aggregate(e, G) * g)
        rhs = np.sum(e * local_aggregate_adj(g, G))
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


# ------------------------------------------- P10 hand-computed special case


def test_hand_computed_single_element():
    """R=1, d=1: the standard edge -> sum -> node layer on one P=1 element.

    H=1, edge MLP weights [1, 1, 1] then 1, node MLP weights [1, 0] then 1,
    zero biases, no LayerNorm.  With x_k = k+1 and e = 0.5 on every edge,
    all pre-activations are positive, so e'_ij = x_i + x_j + 2 e and
    x'_i = x_i + sum_j e'_ij = 4 x_i + sum_{j in N(i)} x_j + 3.
    Worked by hand on the unit cube: 17, 22, 27, ..., 52.
    """
    spec = ModelSpec(H=1, n_layers=1, layernorm=False)
    m = box_mesh((1, 1, 1), 1)
    G = lattice_graph(m.npts)
    params = {"mp0.edge.lin0.W": np.array([[1.0, 1.0, 1.0]]), "mp0.edge.lin0.b": np.zeros(1),
              "mp0.edge.lin1.W": np.array([[1.0]]), "mp0.edge.lin1.b": np.zeros(1),
              "mp0.node.lin0.W": np.array([[1.0, 0.0]]), "mp0.node.lin0.b": np.zeros(1),
              "mp0.node.lin1.W": np.array([[1.0]]), "mp0.node.lin1.b": np.zeros(1)}
    x = (np.arange(8, dtype=np.float64) + 1.0)[:, None]
    e = np.full((G.e, 1), 0.5)
    xn, en, _ = nmp_layer_fwd(params, 0, spec, [G], {}, [x], [e])
    np.testing.assert_array_equal(xn[0][:, 0], [17, 22, 27, 32, 37, 42, 47, 52])
    # and the edge states: e' = x_i + x_j + 1 for the edge 0 <- 1 (receiver 0)
    k = np.nonzero((G.recv == 0) & (G.send == 1))[0][0]
    assert en[0][k, 0] == 1 + 2 + 1


def test_hand_computed_single_element_negative_branch():
    """The same P=1 element with pre-activations of both signs, so ELU's
    negative branch (exp(z) - 1) enters the result.

    H=1, edge MLP [1, -1, 0] then 1, node MLP [1, 0] then 1, zero biases,
    e = 0: e'_ij = ELU(x_i - x_j) and x'_i = x_i + ELU(sum_j e'_ij).  With
    x_k = k+1, node 0 (neighbours 1, 2, 4) gets sum = e^-1 + e^-2 + e^-4 - 3
    = -2.4784696367032108..., so x'_0 = 1 + (e^sum - 1) = e^sum; node 3
    (neighbours 1, 2, 7) gets 2 + 1 + (e^-4 - 1); node 7 (neighbours 3, 5,
    6) gets 4 + 2 + 1.  Decimals worked out to 40 digits.
    """
    spec = ModelSpec(H=1, n_layers=1, layernorm=False)
    m = box_mesh((1, 1, 1), 1)
    G = lattice_graph(m.npts)
    params = {"mp0.edge.lin0.W": np.array([[1.0, -1.0, 0.0]]), "mp0.edge.lin0.b": np.zeros(1),
              "mp0.edge.lin1.W": np.array([[1.0]]), "mp0.edge.lin1.b": np.zeros(1),
              "mp0.node.lin0.W": np.array([[1.0, 0.0]]), "mp0.node.lin0.b": np.zeros(1),
              "mp0.node.lin1.W": np.array([[1.0]]), "mp0.node.lin1.b": np.zeros(1)}
    x = (np.arange(8, dtype=np.float64) + 1.0)[:, None]
    e = np.zeros((G.e, 1))
    xn, en, _ = nmp_layer_fwd(params, 0, spec, [G], {}, [x], [e])
    np.testing.assert_allclose(xn[0][0, 0], 0.08387148126485265363, rtol=1e-14)
    np.testing.assert_allclose(xn[0][3, 0], 6.018315638888734180, rtol=1e-15)
    np.testing.assert_allclose(xn[0][7, 0], 15.0, rtol=1e-15)
    k = np.nonzero((G.recv == 0) & (G.send == 4))[0][0]
    np.testing.assert_allclose(en[0][k, 0], -0.9816843611112658, rtol=1e-15)   # e^-4 - 1


# ---------------------------------------- elementary functions of Sec. III


def test_elu_values():
    """ELU with alpha = 1: z for z > 0, exp(z) - 1 otherwise; its derivative
    1, else exp(z).  Decimal values of e^-1 - 1, e^-0.5 - 1 and e^-1."""
    z = np.array([-1.0, -0.5, 0.0, 2.0, -40.0, 1e-300])
    np.testing.assert_allclose(elu(z), [-0.63212055882855767840, -0.39346934028736657640, 0.0, 2.0,
                                        -1.0, 1e-300], rtol=1e-15, atol=0)
    # small |z|: exp(z) - 1 without cancellation (~z)
    np.testing.assert_allclose(elu(np.array([-1e-10])), [-9.9999999995e-11], rtol=1e-15)
    np.testing.assert_allclose(elu_deriv(np.array([-1.0, 3.0])), [0.36787944117144232160, 1.0],
                               rtol=1e-15)


def test_layer_norm_closed_forms():
    """LayerNorm over a row's features: mean, biased variance (divide by H),
    eps added inside the square root, then the per-feature gain and shift."""
    z = np.array([[1.0, 2.0, 3.0, 4.0]])
    one, zero = np.ones(4), np.zeros(4)
    # mean 5/2, biased variance 5/4; with eps = 1 the scale is 1/sqrt(9/4) = 2/3
    y, _ = layer_norm_fwd(z, one, zero, 1.0)
    np.testing.assert_allclose(y[0], [-1.0, -1.0 / 3.0, 1.0 / 3.0, 1.0], rtol=0, atol=2e-16)
    # eps = 1e-5: scale 1/sqrt(1.25001), decimals worked out to 40 digits
    y, _ = layer_norm_fwd(z, one, zero, 1e-5)
    np.testing.assert_allclose(y[0], [-1.3416354199689269826, -0.44721180665630899419,
                                      0.44721180665630899419, 1.3416354199689269826], rtol=1e-15)
    # gain and shift act per feature after the normalisation
    y, _ = layer_norm_fwd(z, np.array([2.0, 3.0, -1.0, 0.5]), np.array([0.5, 0.0, 1.0, -2.0]), 1.0)
    np.testing.assert_allclose(y[0], [-1.5, -1.0, 2.0 / 3.0, -1.5], rtol=0, atol=4e-16)
    # a constant row normalises to zero, leaving the shift
    y, _ = layer_norm_fwd(np.full((1, 4), 7.0), one, np.array([0.25, -1.0, 0.0, 3.0]), 1e-5)
    np.testing.assert_array_equal(y[0], [0.25, -1.0, 0.0, 3.0])


def test_mlp_with_layer_norm_hand_computed():
    """One row through Linear(1 -> 4), ELU, Linear(4 -> 4), LayerNorm: with
    W0 = (1, 2, -3, 4)^T, W1 = identity and zero biases the last Linear
    outputs (1, 2, e^-3 - 1, 4); LayerNorm with eps = 1 then gives its
    centred values over sqrt(biased variance + 1)."""
    spec = ModelSpec(H=4, n_layers=1, layernorm=True, ln_eps=1.0)
    params = {"t.lin0.W": np.array([[1.0], [2.0], [-3.0], [4.0]]), "t.lin0.b": np.zeros(4),
              "t.lin1.W": np.eye(4), "t.lin1.b": np.zeros(4),
              "t.ln.g": np.ones(4), "t.ln.b": np.zeros(4)}
    y, _ = mlp_fwd(params, "t", np.array([[1.0]]), spec, True)
    # v = (1, 2, -0.95021293163213605702, 4): mean 1.5124467670919659857,
    # biased variance 3.1882309305732950135; decimals worked out to 40 digits
    np.testing.assert_allclose(y[0], [-0.25039949445572325360, 0.23823563905617466003,
                                      -1.2033420506804218937, 1.2155059060799704873], rtol=1e-14)


def test_edge_input_orientation():
    """Edge inputs on one P=1 element of size 0.5 x 1 x 1: for receiver i and
    sender j they are (p_j - p_i, |p_j - p_i|).  Lattice ids: i + 3j + 6k."""
    m = box_mesh((2, 1, 1), 1)
    G = lattice_graph(m.npts)
    E = edge_inputs(G, m.pos)

    def at(i, j):
        return E[np.nonzero((G.recv == i) & (G.send == j))[0][0]]

    np.testing.assert_array_equal(at(0, 1), [0.5, 0.0, 0.0, 0.5])     # sender at x = 0.5
    np.testing.assert_array_equal(at(1, 0), [-0.5, 0.0, 0.0, 0.5])
    np.testing.assert_array_equal(at(0, 3), [0.0, 1.0, 0.0, 1.0])     # sender at y = 1
    np.testing.assert_array_equal(at(6, 0), [0.0, 0.0, -1.0, 1.0])    # receiver at z = 1
    np.testing.assert_array_equal(at(2, 1), [-0.5, 0.0, 0.0, 0.5])


# ------------------------------------------------------------ P11 symmetry


def test_permutation_invariance(c0_ref):
    inp, Y1 = c0_ref
    prob = build_problem(inp.mesh, inp.field, inp.target)
    G = prob.graphs[0]
    rng = np.random.default_rng(9)
    perm = rng.permutation(G.n)          # new row k holds old row perm[k]
    inv = np.empty_like(perm)
    inv[perm] = np.arange(G.n)
    eperm = rng.permutation(G.e)
    from oracle.graph import SubGraph
    Gp = SubGraph(G.gid[perm], inv[G.recv[eperm]], inv[G.send[eperm]],
                  G.d_edge[eperm], G.d_node[perm])
    Y, _ = model_fwd(inp.params, inp.cfg.spec, [Gp], {}, [prob.X[0][perm]],
                     [prob.E0[0][eperm]])
    assert normwise(Y[0], Y1[perm]) <= 1e-13


def test_translation_invariance(c0_ref):
    inp, Y1 = c0_ref
    mesh = inp.mesh
    shifted = type(mesh)(mesh.nel, mesh.P, mesh.periodic, mesh.npts, mesh.elem_gid,
                         mesh.pos + np.array([0.25, -0.5, 0.125]))
    prob = build_problem(shifted, inp.field, inp.target)
    Y, _ = model_fwd(inp.params, inp.cfg.spec, prob.graphs, {}, prob.X, prob.E0)
    assert normwise(Y[0], Y1) <= 1e-12


# ------------------------------------------------------ receptive-field ball


def test_ball_matches_full_graph(c0_ref):
    inp, Y1 = c0_ref
    n = inp.mesh.npts[0]
    centers = [0, n // 2 + n * (n // 2) + n * n * (n // 2), n * n * n - 1, 5 + n * 3]
    for c in centers:
        y = ball_output(inp.params, inp.cfg.spec, inp.mesh, inp.field, c)
        np.testing.assert_allclose(y, Y1[c], rtol=0, atol=1e-13)


def test_ball_gradient_matches_full_graph():
    spec, m, field, params = _tiny(H=3)
    prob = build_problem(m, field, field, None, 1)
    Y, cache = model_fwd(params, spec, prob.graphs, {}, prob.X, prob.E0)
    c = 7
    w = np.array([0.3, -1.2, 0.7])
    gY = np.zeros_like(Y[0])
    gY[c] = w
    g_full, _ = model_bwd(params, spec, prob.graphs, {}, cache, [gY])
    _, g_ball = ball_grad(params, spec, m, field, c, w)
    for k in g_full:
        np.testing.assert_allclose(g_ball[k], g_full[k], rtol=0, atol=1e-13)


# ------------------------------------------- periodic boxes (Table II meshes)


@pytest.fixture(scope="module")
def periodic_ref():
    """A periodic 4 x 4 x 8-element P=3 box (12 x 12 x 24 points)."""
    spec = ModelSpec(H=6, n_layers=2, layernorm=True)
    m = box_mesh((4, 4, 8), 3, periodic=(True, True, True))
    field = velocity_field(m.pos, 5, noise_sigma=0.02)
    params = init_params(spec, 6, perturb=True)
    prob = build_problem(m, field, field, None, 1)
    Y, _ = model_fwd(params, spec, prob.graphs, {}, prob.X, prob.E0)
    return spec, m, field, params, prob, Y[0]


def test_periodic_edge_inputs_are_element_local(periodic_ref):
    """Every link's difference is that of two neighbouring GLL points of one
    element: at most the widest GLL gap, wrap links included."""
    _, m, _, _, prob, _ = periodic_ref
    E0 = prob.E0[0]
    G = prob.graphs[0]
    assert G.e == 6 * m.n_gid                          # every line closes into a ring
    gap = np.max(np.diff(gll_points(3))) / 2 / 4       # widest gap on a 1/4 element
    gap_z = np.max(np.diff(gll_points(3))) / 2 / 8
    assert np.all(E0[:, 3] <= gap + 1e-15)
    assert np.all(E0[:, 3] >= gap_z * 0.5 - 1e-15)
    np.testing.assert_allclose(np.linalg.norm(E0[:, :3], axis=1), E0[:, 3], rtol=1e-15)


def test_periodic_shift_invariance(periodic_ref):
    """Shifting the input by one element along each periodic axis shifts the
    output the same way (the wrap links see the same differences)."""
    spec, m, field, params, prob, Y1 = periodic_ref
    n = m.npts
    g = np.arange(m.n_gid)
    I, J, K = g % n[0], (g // n[0]) % n[1], g // (n[0] * n[1])
    for dI, dJ, dK in ((3, 0, 0), (0, 3, 0), (0, 0, 3)):
        src = (I + dI) % n[0] + n[0] * ((J + dJ) % n[1] + n[1] * ((K + dK) % n[2]))
        p2 = build_problem(m, field[src], field[src], None, 1)
        Y, _ = model_fwd(params, spec, p2.graphs, {}, p2.X, p2.E0)
        assert normwise(Y[0], Y1[src]) <= 1e-12


def test_periodic_consistency_slabs(periodic_ref):
    """Eq. 2 on 8 periodic z-slabs: the first and last slab share nodes
    through the wrap, so every slab has two neighbours."""
    spec, m, field, params, _, Y1 = periodic_ref
    part = slab_partition(m.nel, 8)
    prob = build_problem(m, field, field, part, 8)
    _, halo, nbrs = table2_stats(prob.graphs, prob.copies)
    assert list(nbrs) == [2] * 8 and list(halo) == [2 * 12 * 12] * 8
    Y, _ = model_fwd(params, spec, prob.graphs, prob.pair_lists, prob.X, prob.E0)
    err = max(np.abs(Y[r] - Y1[G.gid]).max() for r, G in enumerate(prob.graphs))
    assert err / np.abs(Y1).max() <= 1e-12


def test_periodic_ball_matches_full_graph(periodic_ref):
    spec, m, field, params, _, Y1 = periodic_ref
    n = m.npts
    for c in (0, n[0] - 1, m.n_gid - 1, n[0] * n[1] * (n[2] - 1) + 5):
        y = ball_output(params, spec, m, field, c)
        np.testing.assert_allclose(y, Y1[c], rtol=0, atol=1e-13)


# ------------------------------------------- message aggregation (variant)


def _first_layer_aggregate(spec, m, field, params, zero_message=False):
    prob = build_problem(m, field, field, None, 1)
    G = prob.graphs[0]
    rng = np.random.default_rng(4)
    x = rng.standard_normal((G.n, spec.H))
    e = rng.standard_normal((G.e, spec.H))
    p = {k: v.astype(np.float64) for k, v in params.items()}
    if zero_message:
        last = spec.n_hidden + 1
        p[f"mp0.edge.lin{last}.W"][:] = 0.0
        p[f"mp0.edge.lin{last}.b"][:] = 0.0
    _, e_new, cache = nmp_layer_fwd(p, 0, spec, [G], {}, [x], [e], halo=False)
    return G, e, e_new[0], cache["a_star"][0]


def test_message_aggregation_sums_the_mlp_output():
    """With message aggregation the aggregate is the state aggregate minus
    the aggregate of the incoming edge states (e' = e + m), row by row."""
    spec, m, field, params = _tiny(ln=False)
    spec_m = ModelSpec(**{**spec.__dict__, "aggregate": "message"})
    G, e, e_new, a_state = _first_layer_aggregate(spec, m, field, params)
    _, _, e_new_m, a_msg = _first_layer_aggregate(spec_m, m, field, params)
    np.testing.assert_array_equal(e_new, e_new_m)          # edge states do not change
    ref = np.zeros_like(a_state)
    for k in range(G.e):                                    # brute-force sum of e / d
        ref[G.recv[k]] += e[k] / G.d_edge[k]
    np.testing.assert_allclose(a_msg, a_state - ref, rtol=0, atol=1e-13)


def test_message_aggregation_of_a_zero_message_is_zero():
    """An edge MLP whose last Linear is zero (no LayerNorm) sends nothing:
    e' = e, the message aggregate is exactly 0, the state aggregate sum e/d."""
    spec, m, field, params = _tiny(ln=False, aggregate="message")
    G, e, e_new, a_msg = _first_layer_aggregate(spec, m, field, params, zero_message=True)
    np.testing.assert_array_equal(e_new, e)
    assert np.all(a_msg == 0.0)


# ------------------------------------- seven edge input channels (variant)


def test_seven_channel_edge_inputs_reverse_antisymmetrically():
    """For the reverse edge j -> i the differences change sign and the
    distance does not: E0[rev(k)] = (-dp, |dp|, -du); and channels 4..6 vanish
    for a uniform field."""
    m = box_mesh((2, 2, 2), 3)
    field = velocity_field(m.pos, 9, noise_sigma=0.05)
    prob = build_problem(m, field, field, None, 1, edge_in=7)
    G, E = prob.graphs[0], prob.E0[0]
    assert E.shape == (G.e, 7)
    key = {(int(a), int(b)): k for k, (a, b) in enumerate(zip(G.recv, G.send))}
    rev = np.array([key[(int(b), int(a))] for a, b in zip(G.recv, G.send)])
    flip = np.array([-1, -1, -1, 1, -1, -1, -1])
    np.testing.assert_array_equal(E[rev], E * flip)
    np.testing.assert_array_equal(E[:, :4], build_problem(m, field, field, None, 1).E0[0])
    uni = np.ones_like(field) * np.array([0.3, -1.2, 2.0], np.float32)
    assert np.all(build_problem(m, uni, uni, None, 1, edge_in=7).E0[0][:, 4:] == 0.0)
