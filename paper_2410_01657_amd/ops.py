"""Python binding of the layer, MLP, edge-input and loss entry points.

Tensors supply device memory and the current HIP stream; every step runs
in libmplayer.so.  The autograd Functions call the hand-written adjoint
entry points, so training goes through the library's kernels too.
"""

import ctypes as C

import torch

from ._lib import (LAYER_FIELDS, MLP_FIELDS, MP_BF16, MP_F32, MpDeepLayerCfg, MpDeepMlpCfg, MpLayerCfg,
                   MpLayerGrads, MpLayerParams, MpMlpCfg, MpMlpGrads, MpMlpParams, call)

_GEMM = {"f32": MP_F32, "bf16": MP_BF16}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p()


def _check(*ts):
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("tensor is not on the GPU")
        if not t.is_contiguous():
            raise ValueError("tensor is not contiguous")


class _Workspace:
    """Grow-only scratch buffer per device (the library never allocates)."""

    def __init__(self):
        self.buf = {}

    def get(self, nbytes, device):
        key = (device.type, device.index)
        b = self.buf.get(key)
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
            self.buf[key] = b
        return b


WS = _Workspace()


# ------------------------------------------------------------------ layer

_AGG = {"state": 0, "message": 1}


def layer_cfg(H, layernorm=True, halo=True, gemm="f32", ln_eps=1e-5, aggregate="state", estate="f32"):
    """estate: storage type of the edge states and their gradients, "f32",
    or "bf16" (with gemm="bf16")."""
    c = MpLayerCfg()
    c.H, c.layernorm, c.halo, c.gemm_dtype, c.ln_eps = H, int(layernorm), int(halo), _GEMM[gemm], ln_eps
    c.aggregate = _AGG[aggregate]
    c.estate_dtype = _GEMM[estate]
    return c


def estate_dtype(cfg):
    """torch dtype of a layer's edge states under cfg."""
    return torch.bfloat16 if cfg.estate_dtype == _GEMM["bf16"] else torch.float32


def _check_dtype(t, dtype, what):
    if t is not None and t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype} (got {t.dtype})")


def _layer_params(p):
    s = MpLayerParams()
    for f in LAYER_FIELDS:
        setattr(s, f, p[f].data_ptr() if p.get(f) is not None else None)
    return s


def layer_forward(cfg, p, dg, x, e, want_pq=False, want_e=True):
    """One consistent NMP layer; returns (x_out, e_out, a_star), plus the node
    projections pq = [P; Q] ([2, N, H], for the backward) when want_pq.
    want_e=False: the updated edge state is not written (e_out is None), for
    a last layer whose e' nothing reads."""
    _check(x, e)
    _check_dtype(e, estate_dtype(cfg), "the edge state")
    x_out, a_star = torch.empty_like(x), torch.empty_like(x)
    e_out = torch.empty_like(e) if want_e else None
    pq = torch.empty((2,) + tuple(x.shape), dtype=x.dtype, device=x.device) if want_pq else None
    nb = C.c_size_t()
    call("mp_layer_workspace_size", C.byref(cfg), C.byref(dg.desc), 0, C.byref(nb))
    ws = WS.get(nb.value, x.device)
    call("mp_layer_forward", C.byref(cfg), C.byref(_layer_params(p)), C.byref(dg.desc), _p(x), _p(e),
         _p(x_out), _p(e_out), _p(a_star), _p(pq), _p(ws), ws.numel(), _stream())
    return (x_out, e_out, a_star, pq) if want_pq else (x_out, e_out, a_star)


def layer_forward_noalloc(cfg, p, dg, x, e):
    """layer_forward through the entry point that allocates nothing (its
    scratch is a library-held module array); returns (x_out, e_out, a_star,
    pq).  The outputs here are torch tensors the caller allocates."""
    _check(x, e)
    _check_dtype(e, estate_dtype(cfg), "the edge state")
    x_out, e_out, a_star = torch.empty_like(x), torch.empty_like(e), torch.empty_like(x)
    pq = torch.empty((2,) + tuple(x.shape), dtype=x.dtype, device=x.device)
    call("mp_layer_forward_noalloc", C.byref(cfg), C.byref(_layer_params(p)), C.byref(dg.desc), _p(x), _p(e),
         _p(x_out), _p(e_out), _p(a_star), _p(pq), _stream())
    return x_out, e_out, a_star, pq


def layer_backward(cfg, p, dg, x, e, a_star, g_x_out, g_e_out, pq=None):
    """Adjoint of layer_forward; pq (from layer_forward(want_pq=True)) skips
    recomputing the node projections."""
    _check(x, e, a_star, g_x_out, g_e_out, pq)
    _check_dtype(e, estate_dtype(cfg), "the edge state")
    _check_dtype(g_e_out, estate_dtype(cfg), "the edge-state gradient")
    g_x, g_e = torch.empty_like(x), torch.empty_like(e)
    grads = {f: (torch.empty_like(p[f]) if p.get(f) is not None else None) for f in LAYER_FIELDS}
    gs = MpLayerGrads()
    for f in LAYER_FIELDS:
        setattr(gs, f, grads[f].data_ptr() if grads[f] is not None else None)
    nb = C.c_size_t()
    call("mp_layer_workspace_size", C.byref(cfg), C.byref(dg.desc), 1, C.byref(nb))
    ws = WS.get(nb.value, x.device)
    call("mp_layer_backward", C.byref(cfg), C.byref(_layer_params(p)), C.byref(dg.desc), _p(x), _p(e),
         _p(a_star), _p(pq), _p(g_x_out), _p(g_e_out), _p(g_x), _p(g_e), C.byref(gs), _p(ws), ws.numel(),
         _stream())
    return g_x, g_e, grads


class MPLayerFn(torch.autograd.Function):
    """(x, e, *layer params) -> (x', e') with the library's adjoint as backward.
    want_e=False returns e' = None (a last layer: the edge state is not
    written, and its gradient is zero)."""

    @staticmethod
    def forward(ctx, cfg, dg, want_e, x, e, *params):
        p = dict(zip(LAYER_FIELDS, params))
        x_out, e_out, a_star, pq = layer_forward(cfg, p, dg, x, e, want_pq=True, want_e=want_e)
        ctx.cfg, ctx.dg = cfg, dg
        # an unused edge-state output (the last layer's) arrives as None in
        # the backward instead of a materialised zero tensor
        ctx.set_materialize_grads(False)
        ctx.save_for_backward(x, e, a_star, pq, *[t if t is not None else torch.empty(0) for t in params])
        ctx.has = [t is not None for t in params]
        return x_out, e_out

    @staticmethod
    def backward(ctx, g_x_out, g_e_out):
        x, e, a_star, pq, *ps = ctx.saved_tensors
        p = {f: (t if h else None) for f, t, h in zip(LAYER_FIELDS, ps, ctx.has)}
        g_x_out = g_x_out.contiguous() if g_x_out is not None else torch.zeros_like(x)
        g_e_out = g_e_out.contiguous() if g_e_out is not None else None
        g_x, g_e, grads = layer_backward(ctx.cfg, p, ctx.dg, x, e, a_star, g_x_out, g_e_out, pq)
        return (None, None, None, g_x, g_e) + tuple(grads[f] for f in LAYER_FIELDS)


# -------------------------------------------------------------------- MLPs

def mlp_cfg(n_in, H, n_out, layernorm, gemm="f32", ln_eps=1e-5, out="f32"):
    """out: storage type of the output and its gradient, "f32", or "bf16"
    (the edge encoder of a model with BF16 edge states)."""
    c = MpMlpCfg()
    c.n_in, c.H, c.n_out, c.layernorm, c.gemm_dtype, c.ln_eps = n_in, H, n_out, int(layernorm), _GEMM[gemm], ln_eps
    c.out_dtype = _GEMM[out]
    return c


def _mlp_out_dtype(cfg):
    return torch.bfloat16 if cfg.out_dtype == _GEMM["bf16"] else torch.float32


def _mlp_params(p):
    s = MpMlpParams()
    for f in MLP_FIELDS:
        setattr(s, f, p[f].data_ptr() if p.get(f) is not None else None)
    return s


def mlp_forward(cfg, p, x):
    _check(x)
    out = torch.empty((x.shape[0], cfg.n_out), dtype=_mlp_out_dtype(cfg), device=x.device)
    nb = C.c_size_t()
    call("mp_mlp_workspace_size", C.byref(cfg), x.shape[0], 0, C.byref(nb))
    ws = WS.get(nb.value, x.device)
    call("mp_mlp_forward", C.byref(cfg), C.byref(_mlp_params(p)), x.shape[0], _p(x), _p(out), _p(ws),
         ws.numel(), _stream())
    return out


def mlp_backward(cfg, p, x, g_out, want_g_in):
    _check(x, g_out)
    _check_dtype(g_out, _mlp_out_dtype(cfg), "the output gradient")
    g_in = torch.empty_like(x) if want_g_in else None
    grads = {f: (torch.empty_like(p[f]) if p.get(f) is not None else None) for f in MLP_FIELDS}
    gs = MpMlpGrads()
    for f in MLP_FIELDS:
        setattr(gs, f, grads[f].data_ptr() if grads[f] is not None else None)
    nb = C.c_size_t()
    call("mp_mlp_workspace_size", C.byref(cfg), x.shape[0], 1, C.byref(nb))
    ws = WS.get(nb.value, x.device)
    call("mp_mlp_backward", C.byref(cfg), C.byref(_mlp_params(p)), x.shape[0], _p(x), _p(g_out), _p(g_in),
         C.byref(gs), _p(ws), ws.numel(), _stream())
    return g_in, grads


class MLPFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cfg, x, *params):
        p = dict(zip(MLP_FIELDS, params))
        ctx.cfg = cfg
        ctx.has = [t is not None for t in params]
        ctx.save_for_backward(x, *[t if t is not None else torch.empty(0) for t in params])
        return mlp_forward(cfg, p, x)

    @staticmethod
    def backward(ctx, g_out):
        x, *ps = ctx.saved_tensors
        p = {f: (t if h else None) for f, t, h in zip(MLP_FIELDS, ps, ctx.has)}
        want = ctx.needs_input_grad[1] and ctx.cfg.n_in > 4
        g_in, grads = mlp_backward(ctx.cfg, p, x, g_out.contiguous(), want)
        return (None, g_in) + tuple(grads[f] for f in MLP_FIELDS)


# ------------------------------------------- narrow deep MLPs (Table I)
# Each MLP's parameters travel as one flat FP32 tensor in torch.nn.Linear
# order (W0, b0, hidden W/b pairs, Wo, bo, LayerNorm gain and shift).

def deep_layer_cfg(H, n_hidden, layernorm=True, halo=True, ln_eps=1e-5, aggregate="state"):
    c = MpDeepLayerCfg()
    c.H, c.n_hidden, c.layernorm, c.halo, c.ln_eps = H, n_hidden, int(layernorm), int(halo), ln_eps
    c.aggregate = _AGG[aggregate]
    return c


def deep_mlp_cfg(n_in, H, n_hidden, n_out, layernorm, ln_eps=1e-5):
    c = MpDeepMlpCfg()
    c.n_in, c.H, c.n_hidden, c.n_out, c.layernorm, c.ln_eps = n_in, H, n_hidden, n_out, int(layernorm), ln_eps
    return c


def deep_theta_size(n_in, H, n_hidden, n_out, layernorm):
    n = C.c_int64()
    call("mp_deep_theta_size", n_in, H, n_hidden, n_out, int(layernorm), C.byref(n))
    return n.value


class DeepMLPFn(torch.autograd.Function):
    """Encoder / decoder MLP with n_hidden extra layers: (x, theta) -> out."""

    @staticmethod
    def forward(ctx, cfg, x, theta):
        _check(x, theta)
        if theta.numel() != deep_theta_size(cfg.n_in, cfg.H, cfg.n_hidden, cfg.n_out, cfg.layernorm):
            raise ValueError("flat MLP parameter array has the wrong size")
        if x.shape[1] != cfg.n_in:
            raise ValueError("input width does not match the MLP")
        out = torch.empty((x.shape[0], cfg.n_out), dtype=torch.float32, device=x.device)
        call("mp_deep_mlp_forward", C.byref(cfg), _p(theta), x.shape[0], _p(x), _p(out), _stream())
        ctx.cfg = cfg
        ctx.save_for_backward(x, theta)
        return out

    @staticmethod
    def backward(ctx, g_out):
        x, theta = ctx.saved_tensors
        cfg = ctx.cfg
        g_out = g_out.contiguous()
        g_in = torch.empty_like(x) if ctx.needs_input_grad[1] else None
        g_theta = torch.empty_like(theta)
        nb = C.c_size_t()
        call("mp_deep_mlp_workspace_size", C.byref(cfg), x.shape[0], 1, C.byref(nb))
        ws = WS.get(nb.value, x.device)
        call("mp_deep_mlp_backward", C.byref(cfg), _p(theta), x.shape[0], _p(x), _p(g_out), _p(g_in),
             _p(g_theta), _p(ws), ws.numel(), _stream())
        return None, g_in, g_theta


class DeepLayerFn(torch.autograd.Function):
    """(x, e, theta_edge, theta_node) -> (x', e') for deep MLPs, with the
    library's adjoint as backward."""

    @staticmethod
    def forward(ctx, cfg, dg, x, e, theta_e, theta_n):
        _check(x, e, theta_e, theta_n)
        H = cfg.H
        if (theta_e.numel() != deep_theta_size(3 * H, H, cfg.n_hidden, H, cfg.layernorm)
                or theta_n.numel() != deep_theta_size(2 * H, H, cfg.n_hidden, H, cfg.layernorm)):
            raise ValueError("flat MLP parameter arrays have the wrong size")
        if tuple(x.shape) != (dg.n_rows, H) or tuple(e.shape) != (dg.n_edges, H):
            raise ValueError("state shapes do not match the graph and H")
        x_out, e_out, a_star = torch.empty_like(x), torch.empty_like(e), torch.empty_like(x)
        call("mp_deep_layer_forward", C.byref(cfg), _p(theta_e), _p(theta_n), C.byref(dg.desc), _p(x), _p(e),
             _p(x_out), _p(e_out), _p(a_star), _stream())
        ctx.cfg, ctx.dg = cfg, dg
        ctx.set_materialize_grads(False)
        ctx.save_for_backward(x, e, a_star, theta_e, theta_n)
        return x_out, e_out

    @staticmethod
    def backward(ctx, g_x_out, g_e_out):
        x, e, a_star, theta_e, theta_n = ctx.saved_tensors
        g_x_out = g_x_out.contiguous() if g_x_out is not None else torch.zeros_like(x)
        g_e_out = g_e_out.contiguous() if g_e_out is not None else None
        g_x, g_e = torch.empty_like(x), torch.empty_like(e)
        g_te, g_tn = torch.empty_like(theta_e), torch.empty_like(theta_n)
        nb = C.c_size_t()
        call("mp_deep_layer_workspace_size", C.byref(ctx.cfg), C.byref(ctx.dg.desc), 1, C.byref(nb))
        ws = WS.get(nb.value, x.device)
        call("mp_deep_layer_backward", C.byref(ctx.cfg), _p(theta_e), _p(theta_n), C.byref(ctx.dg.desc), _p(x),
             _p(e), _p(a_star), _p(g_x_out), _p(g_e_out), _p(g_x), _p(g_e), _p(g_te), _p(g_tn), _p(ws),
             ws.numel(), _stream())
        return None, None, g_x, g_e, g_te, g_tn


# ----------------------------------------------------------- inputs, loss

def edge_inputs(dg, row_pos, period=None, row_u=None):
    """(p_j - p_i, |p_j - p_i|) per edge from FP64 row positions [N, 3];
    ``period`` (3 floats, 0 = not periodic) takes differences to the nearest
    periodic image.  With an FP32 node field ``row_u`` [N, 3] three more
    channels u_j - u_i follow (7 in all)."""
    _check(row_pos, row_u)
    if row_pos.dtype != torch.float64:
        raise ValueError("row positions must be float64")
    if row_u is not None and (row_u.dtype != torch.float32 or tuple(row_u.shape) != (dg.n_rows, 3)):
        raise ValueError("row_u must be float32 [N, 3]")
    e0 = torch.empty((dg.n_edges, 4 if row_u is None else 7), dtype=torch.float32, device=row_pos.device)
    L = None
    if period is not None and any(period):
        L = (C.c_double * 3)(*[float(v) for v in period])
    call("mp_edge_inputs", C.byref(dg.desc), _p(row_pos), L, _p(row_u), _p(e0), _stream())
    return e0


def consistent_mse(dg, Y, T, want_grad=True):
    """Eq. 6 loss over all rows (Eq. 5 when every node degree is 1)."""
    _check(Y, T)
    loss = torch.empty(1, dtype=torch.float32, device=Y.device)
    gY = torch.empty_like(Y) if want_grad else None
    nb = C.c_size_t()
    call("mp_consistent_mse_workspace_size", Y.shape[0], C.byref(nb))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=Y.device)
    call("mp_consistent_mse", Y.shape[0], Y.shape[1], _p(Y), _p(T), _p(dg.node_mult), _p(loss), _p(gY),
         _p(ws), ws.numel(), _stream())
    return loss, gY


class ConsistentMSEFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, dg, Y, T):
        loss, gY = consistent_mse(dg, Y, T, True)
        ctx.save_for_backward(gY)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (gY,) = ctx.saved_tensors
        return None, gY * g, None
