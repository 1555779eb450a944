"""Full-size parity for the larger workloads, on sampled outputs.

An output after M layers depends only on its M-hop ball, so the oracle can
evaluate it exactly for a few seeded nodes (oracle/ball.py).  Gradients are
checked the same way: the GPU back-propagates S = sum_c <w_c, Y_c> over the
sampled nodes (one copy of each), whose exact parameter gradient is the sum
of the oracle's per-ball gradients.

C3: 24^3 elements, P=5 (1.77M nodes, 10.5M edges), H=128, 4 layers, LN,
    8 sub-graphs; FP32 and BF16 GEMMs.
C4: 32^3 elements, P=7 (11.4M nodes, 68M edges), H=64, 4 layers, LN,
    64 uneven sub-graphs (seeded bisection); BF16 GEMMs; also R-consistency
    against the unpartitioned graph on the GPU.
"""

import numpy as np
import pytest
import torch

from mpinputs import CONFIGS, make_inputs
from oracle.ball import ball_grad, ball_output

from _util import by_gid, normwise

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
DEV = "cuda"


def _sample(mesh, n, seed):
    rng = np.random.default_rng(seed)
    nx = mesh.npts[0]
    fixed = [0, nx - 1, nx * nx * nx - 1, (nx // 2) * (1 + nx + nx * nx), 3 * nx * nx + 2]
    return [int(c) for c in list(rng.choice(mesh.n_gid, n - len(fixed), replace=False)) + fixed]


def _first_rows(row_gid, gids):
    order = np.argsort(row_gid, kind="stable")
    pos = np.searchsorted(row_gid[order], gids)
    return order[pos]


def _sampled_run(cfg_name, gemm, n_sample, seed, tuned=False, estate="f32"):
    """tuned: run under the schedule the autotuner picks for this graph
    (the launch configuration bench.py times), else the library default.
    estate: storage type of the edge states."""
    from paper_2410_01657_amd.autotune import tuned_schedule
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    cfg = CONFIGS[cfg_name]
    inp = make_inputs(cfg, perturb=True)
    prob = Problem(inp.mesh, inp.field, inp.target, inp.elem_part, cfg.R, DEV)
    sched = tuned_schedule(prob.dg, cfg.spec.H, cfg.spec.layernorm, gemm, estate=estate) if tuned else None
    if tuned:
        print(f"{cfg_name} {gemm} (edge states {estate}): tuned schedule {sched}")
    model = ConsistentGNN(cfg.spec, inp.params, DEV, gemm=gemm, schedule=sched,
                          estate=estate).requires_grad_(True)
    Y = model.forward(prob.dg, prob.X, prob.E0)
    gids = _sample(inp.mesh, n_sample, seed)
    rows = _first_rows(prob.dg.host.row_gid, np.array(gids))
    w = np.random.default_rng(seed + 1).standard_normal((len(gids), cfg.spec.out))
    gY = torch.zeros_like(Y)
    gY[torch.as_tensor(rows, device=DEV)] = torch.as_tensor(w, dtype=torch.float32, device=DEV)
    Y.backward(gY)
    Ys = Y.detach()[torch.as_tensor(rows, device=DEV)].cpu().numpy()
    grads = {k: v.grad.cpu().numpy() for k, v in model.params.items()}
    ref_y, ref_g = [], {}
    for c, wc in zip(gids, w):
        y, g = ball_grad(inp.params, cfg.spec, inp.mesh, inp.field, c, wc)
        ref_y.append(y)
        for k, v in g.items():
            ref_g[k] = ref_g.get(k, 0.0) + v
    return Ys, np.stack(ref_y), grads, ref_g


def _report(tag, Ys, Yr, g, gr):
    ey = normwise(Ys, Yr)
    eg = {k: normwise(g[k], gr[k]) for k in gr}
    worst = max(eg, key=eg.get)
    print(f"{tag}: output error {ey:.2e}, worst parameter-gradient error {eg[worst]:.2e} ({worst}), "
          f"median {np.median(list(eg.values())):.2e}")
    return ey, eg[worst]


@pytest.mark.parametrize("gemm,tol_y,tol_g", [("f32", 1e-4, 1e-4), ("bf16", 3e-2, 5e-2)])
def test_c3_sampled_outputs_and_gradients(gemm, tol_y, tol_g):
    ey, eg = _report(f"C3 {gemm}", *_sampled_run("C3", gemm, 24, 31))
    assert ey < tol_y
    assert eg < tol_g, eg


def test_c4_sampled_outputs_and_gradients_bf16():
    ey, eg = _report("C4 bf16", *_sampled_run("C4", "bf16", 24, 41))
    assert ey < 3e-2
    assert eg < 5e-2, eg


@pytest.mark.parametrize("gemm,estate,tol_y,tol_g", [("bf16", "f32", 3e-2, 5e-2), ("f32", "f32", 1e-4, 1e-4),
                                                     ("bf16", "bf16", 3e-2, 5e-2)])
def test_c4_sampled_outputs_and_gradients_tuned_schedule(gemm, estate, tol_y, tol_g):
    """The timed launch configurations: C4 at full size under the schedule
    the autotuner picks (BF16, FP32, and BF16 with BF16 edge states),
    outputs and parameter gradients against the oracle's exact
    receptive-field values (Eq. 2-3)."""
    ey, eg = _report(f"C4 {gemm} edge states {estate} tuned",
                     *_sampled_run("C4", gemm, 24, 43, tuned=True, estate=estate))
    assert ey < tol_y
    assert eg < tol_g, eg


def test_c4_r64_matches_r1_fp32():
    """Eq. 2 at full C4 size on the GPU (FP32, forward)."""
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    cfg = CONFIGS["C4"]
    inp = make_inputs(cfg, perturb=True)
    gids = np.array(_sample(inp.mesh, 4096, 5))
    out = {}
    for R, part in ((64, inp.elem_part), (1, np.zeros(inp.mesh.n_elem, np.int32))):
        prob = Problem(inp.mesh, inp.field, inp.target, part, R, DEV)
        with torch.no_grad():
            Y = ConsistentGNN(cfg.spec, inp.params, DEV).forward(prob.dg, prob.X, prob.E0)
        hg = prob.dg.host
        if R == 64:
            # every copy of every sampled id (copies on several sub-graphs)
            m = np.isin(hg.row_gid, gids)
            out[R] = (hg.row_gid[m], Y.cpu().numpy()[m])
            assert (hg.edge_mult == 3).any()  # T-junctions of the uneven cut
        else:
            out[R] = by_gid(hg, Y.cpu().numpy())
        del prob, Y
        torch.cuda.empty_cache()
    g64, y64 = out[64]
    assert normwise(y64, out[1][g64]) < 1e-5
    yb = np.stack([ball_output(inp.params, cfg.spec, inp.mesh, inp.field, int(c)) for c in gids[:16]])
    assert normwise(out[1][gids[:16]], yb) < 1e-4


def test_c3_gradients_vs_fp64_central_differences():
    """Eq. 3 at the C3 mesh: the GPU's FP32 gradient of S = sum_c <w_c, Y_c>
    over 8 seeded nodes (the model at full size, 1.77M nodes, H=128) against
    FP64 central differences of S with respect to 64 seeded weights.  S
    depends only on the nodes' 4-hop balls, so each perturbed evaluation is
    the oracle's exact FP64 output on those balls; step h = 1e-5 max(1, |w|)."""
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    cfg = CONFIGS["C3"]
    inp = make_inputs(cfg, perturb=True)
    prob = Problem(inp.mesh, inp.field, inp.target, inp.elem_part, cfg.R, DEV)
    model = ConsistentGNN(cfg.spec, inp.params, DEV, gemm="f32").requires_grad_(True)
    Y = model.forward(prob.dg, prob.X, prob.E0)
    gids = _sample(inp.mesh, 8, 77)
    rows = _first_rows(prob.dg.host.row_gid, np.array(gids))
    w = np.random.default_rng(78).standard_normal((len(gids), cfg.spec.out))
    gY = torch.zeros_like(Y)
    gY[torch.as_tensor(rows, device=DEV)] = torch.as_tensor(w, dtype=torch.float32, device=DEV)
    Y.backward(gY)
    grads = {k: v.grad.cpu().numpy() for k, v in model.params.items()}
    del model, Y, gY, prob
    torch.cuda.empty_cache()

    rng = np.random.default_rng(79)
    names = sorted(inp.params)
    sizes = np.array([np.asarray(inp.params[k]).size for k in names], np.float64)
    picks = []
    for k in rng.choice(len(names), 64, p=sizes / sizes.sum()):
        picks.append((names[k], int(rng.integers(np.asarray(inp.params[names[k]]).size))))
    base = {k: np.asarray(v, np.float64) for k, v in inp.params.items()}

    def S(params):
        return sum(float(np.dot(wc, ball_output(params, cfg.spec, inp.mesh, inp.field, c)))
                   for c, wc in zip(gids, w))

    fd, gpu = [], []
    for name, idx in picks:
        theta = base[name].reshape(-1)[idx]
        h = 1e-5 * max(1.0, abs(theta))
        vals = []
        for sgn in (1.0, -1.0):
            p = dict(base)
            a = base[name].copy().reshape(-1)
            a[idx] = theta + sgn * h
            p[name] = a.reshape(base[name].shape)
            vals.append(S(p))
        fd.append((vals[0] - vals[1]) / (2 * h))
        gpu.append(grads[name].reshape(-1)[idx])
    fd, gpu = np.array(fd), np.array(gpu)
    err = normwise(gpu, fd)
    print(f"C3 FP32 gradient vs FP64 central differences, 64 weights: {err:.2e} "
          f"(max |g| {np.abs(fd).max():.3e})")
    assert err < 1e-4, err


def test_c1_bf16_r16_matches_r1():
    """Eq. 2 with BF16 GEMMs at the C1 mesh (16^3 elements, P=5, 16 z-slabs):
    every copy of every node at R=16 against R=1.  BF16 roundings of a* and x
    differ between the two groupings, so the bound is 1e-2 normwise (FP32
    meets 1e-5); the measured value is printed."""
    from paper_2410_01657_amd.model import ConsistentGNN, Problem
    cfg = CONFIGS["C1"]
    inp = make_inputs(cfg, perturb=True)
    out = {}
    for R, part in ((16, inp.elem_part), (1, np.zeros(inp.mesh.n_elem, np.int32))):
        prob = Problem(inp.mesh, inp.field, inp.target, part, R, DEV)
        with torch.no_grad():
            Y = ConsistentGNN(cfg.spec, inp.params, DEV, gemm="bf16").forward(prob.dg, prob.X, prob.E0)
        hg = prob.dg.host
        out[R] = (hg.row_gid.copy(), Y.cpu().numpy())
        del prob, Y
        torch.cuda.empty_cache()
    g16, y16 = out[16]
    g1, y1r = out[1]
    y1 = np.zeros((int(g1.max()) + 1, y1r.shape[1]), y1r.dtype)
    y1[g1] = y1r
    err = normwise(y16, y1[g16])
    print(f"C1 BF16 R=16 vs R=1: {err:.2e}")
    assert err < 1e-2, err
