"""Algorithmic work of each kernel of one layer: the bytes it must move
through HBM and the flops it must execute, independent of how it is built.

Units: N rows (node copies over all sub-graphs), E directed sub-graph edges,
G halo groups with M members, hidden width H, FP32 node states, FP32 or BF16
edge states.
Index arrays: int32 receiver and sender per edge plus a uint8 degree;
int32 reverse-edge and row-offset arrays where a kernel follows them.
Each row or edge is counted once per kernel even when it is gathered several
times (repeat gathers are cache traffic, not algorithmic traffic).

Flops count the MLP products (2 per multiply-add); elementwise work (ELU,
LayerNorm, the 1/d sums) is below 1% and left out.
"""

from dataclasses import dataclass

# MI355X published peaks
PEAK_HBM = 8.0e12          # bytes/s
PEAK = {"f32": 157.3e12, "bf16": 2.5e15}   # dense MFMA flop/s by operand type
# FP32 vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2 (packed
# FP32) x 2.4 GHz.  The library is built without packed FP32 operations, so
# its own ceiling is half of this (78.6 TFLOP/s).
PEAK_VALU = 157.3e12


@dataclass(frozen=True)
class Work:
    bytes: float
    flops: float


def edge_bwd_split(H):
    """The library's edge adjoint runs in two passes (per-edge factors, then
    the weight-gradient sums) at widths above 64."""
    return H > 64


def node_bwd_split(H):
    return H > 64


def gq_split(H, gemm):
    return H > 64 and gemm == "f32"


def layer_kernels(N, E, G, M, H, gemm="bf16", n_layers=1, estate="f32"):
    """Per launch, for one layer; keys match the library's profile names.

    gemm: "bf16" stores the edge-state adjoint g_h in BF16 (2 bytes per
    value), "f32" in FP32.  n_layers: the adjoint kernels are averaged over
    the layers of a model, whose last layer gets no gradient at its edge
    output (g_e' is absent there).  estate: storage type of the edge states
    e, e' and their gradients ("bf16": 2 bytes per value).

    At H > 64 the edge and node adjoints (and, in FP32, the sender-side
    pass) run split: the first pass recomputes the MLP and forms the input
    gradients, a second pass (edge_dw / node_dw / gq_dw) sums the weight
    gradients from per-row factors the first pass stored.  The products are
    then counted where they run; the stored factors are implementation
    traffic, and each second pass is charged only the bytes of the factors
    it must read (one launch of edge_dw / node_dw / gq_dw stands for all of
    that pass's launches in a layer)."""
    f = 4.0                              # bytes per FP32 value
    fe = 2.0 if estate == "bf16" else 4.0  # bytes per edge-state value
    fh = 2.0 if gemm == "bf16" else 4.0  # bytes per g_h value (and per stored factor)
    ge = (n_layers - 1) / n_layers if n_layers > 1 else 1.0  # launches that read g_e'
    w = {
        # x -> P = W1a x + b1, Q = W1b x
        "proj": Work(N * 3 * H * f, N * 2 * 2 * H * H),
        # e, P_i, Q_j -> e', a ; per edge 2 H x H products
        "edge_fwd": Work(E * (2 * H * fe + 9) + N * 3 * H * f, E * 2 * 2 * H * H),
        # every member row read and written once, plus the plan
        "halo": Work(M * 2 * H * f + 4 * (M + G + 1), 0.0),
        "halo_adj": Work(M * 2 * H * f + 4 * (M + G + 1), 0.0),
        # [a*, x] -> x' ; products 2H x H and H x H
        "node_fwd": Work(N * 3 * H * f, N * 2 * 3 * H * H),
        # a*, x, g_x' -> g_a*, g_x ; recompute (3H^2) + input grads (3H^2) + weight grads (3H^2)
        "node_bwd": Work(N * 5 * H * f, N * 2 * 9 * H * H),
        # e, [g_e'], P_i, Q_j, g_a_i -> g_e, g_h, g_P ; 6 H x H products per edge
        "edge_bwd": Work(E * ((2 + ge) * H * fe + H * fh + 9) + N * 4 * H * f, E * 2 * 6 * H * H),
        # g_P, g_h (through reverse edges), x, g_x -> g_x ; 2 (2H x H) products per node
        "gq": Work(E * (H * fh + 4) + N * (4 * H * f + 4), N * 2 * 4 * H * H),
    }
    if edge_bwd_split(H):
        # pass 1: recompute (W1c, W2) and the input-gradient products (W2^T, W1c^T)
        w["edge_bwd"] = Work(w["edge_bwd"].bytes, E * 2 * 4 * H * H)
        # pass 2: dW1c = sum g_h e^T, dW2 = sum gm u^T (+ LayerNorm sums)
        w["edge_dw"] = Work(E * (H * fh + H * fe + 2 * H * fh + 2 * H * fh), E * 2 * 2 * H * H)
    if node_bwd_split(H):
        w["node_bwd"] = Work(w["node_bwd"].bytes, N * 2 * 6 * H * H)
        # dW1 = sum g_y u^T, dW0 = sum g_z [a*, x]^T (+ LayerNorm sums)
        w["node_dw"] = Work(N * (2 * H * fh + H * fh + 2 * H * f + H * fh + H * f), N * 2 * 3 * H * H)
    if gq_split(H, gemm):
        w["gq"] = Work(w["gq"].bytes, N * 2 * 2 * H * H)
        # dW1a = sum g_P x^T, dW1b = sum g_Q x^T
        w["gq_dw"] = Work(N * 3 * H * f, N * 2 * 2 * H * H)
    return w


# kernels that belong to the message-passing layers (the rest of a model
# step: encoders, decoder, loss, edge inputs)
LAYER_KERNEL_NAMES = ("pack", "tiles", "proj", "edge_fwd", "halo", "halo_adj", "node_fwd", "node_bwd",
                      "edge_bwd", "edge_dw", "node_dw", "gq", "gq_dw", "wreduce")


def layer_roof_seconds(N, E, G, M, H, gemm, n_layers, hbm=None, peak=None, estate="f32"):
    """Lower bound on the time of the message-passing layers' forward and
    adjoint: every kernel of every layer at the higher of its HBM floor
    (algorithmic bytes / bandwidth) and its product floor (flops / matrix
    peak of the operand type).  hbm / peak default to the published MI355X
    figures."""
    hbm = PEAK_HBM if hbm is None else hbm
    peak = PEAK[gemm] if peak is None else peak
    w = layer_kernels(N, E, G, M, H, gemm, n_layers, estate)
    return n_layers * sum(max(k.bytes / hbm, k.flops / peak) for k in w.values())


def bound_of(work, gemm):
    """'hbm' or 'mfma': whichever roof takes longer for this work."""
    return "hbm" if work.bytes / PEAK_HBM >= work.flops / PEAK[gemm] else "mfma"


def mlp_flops(K, H, NH, O):
    """Flops of one row through Linear(K->H), NH x Linear(H->H), Linear(H->O)."""
    return 2.0 * (K * H + NH * H * H + O * H)


def deep_kernels(N, E, G, M, H, NH, n_layers=1):
    """Per launch, one layer of the narrow deep-MLP kernels (keys match the
    library's profile names).  Bytes: the layer's inputs and outputs only
    (each row once); the per-row adjoint records the kernels keep in HBM are
    an implementation choice and not counted.  Flops: the MLP products
    (recomputed forward plus transposed products in the adjoint kernels; one
    product per weight per row in the weight-gradient sums)."""
    f = 4.0
    ge = (n_layers - 1) / n_layers if n_layers > 1 else 1.0
    fe, fn = mlp_flops(3 * H, H, NH, H), mlp_flops(2 * H, H, NH, H)
    return {
        "deep_edge_fwd": Work(E * (2 * H * f + 5) + N * (3 * H * f + 4), E * fe),
        "halo": Work(M * 2 * H * f + 4 * (M + G + 1), 0.0),
        "deep_node_fwd": Work(N * 3 * H * f, N * fn),
        "deep_node_bwd": Work(N * 5 * H * f, N * 2 * fn),
        "deep_edge_bwd": Work(E * ((2 + ge) * H * f + 5) + N * (3 * H * f + 4), E * 2 * fe),
        "deep_gather": Work(E * (H * f + 4) + N * (3 * H * f + 4), 0.0),
        "deep_edge_dw": Work(0.0, E * fe),
        "deep_node_dw": Work(0.0, N * fn),
    }
