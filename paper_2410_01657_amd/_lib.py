"""ctypes view of libmplayer.so (the C ABI declared in include/mplayer.h).

Argument marshalling only: every computation happens in the library.
Loading fails loudly when the library has not been built; there is no
fallback path.
"""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmplayer.so")

MP_OK, MP_EINVAL, MP_EPLAN, MP_ENOMEM, MP_EHIP = 0, 1, 2, 3, 4
ABI_VERSION = 4
MP_F32, MP_BF16 = 0, 1
MP_AGG_STATE, MP_AGG_MESSAGE = 0, 1

c_i32, c_i64, c_u64, c_f32 = C.c_int32, C.c_int64, C.c_uint64, C.c_float
vp = C.c_void_p


class MpDevGraph(C.Structure):
    _fields_ = [("n_rows", c_i64), ("n_edges", c_i64), ("n_groups", c_i64), ("n_members", c_i64),
                ("rowptr", vp), ("recv", vp), ("col", vp), ("rev", vp), ("edge_mult", vp),
                ("group_ptr", vp), ("member", vp), ("graph_checksum", c_u64), ("plan_checksum", c_u64),
                ("plan_graph_checksum", c_u64), ("seal", c_u64)]


class MpLayerCfg(C.Structure):
    _fields_ = [("H", c_i32), ("layernorm", c_i32), ("halo", c_i32), ("gemm_dtype", c_i32),
                ("ln_eps", c_f32), ("tile_edges", c_i32), ("edge_grid", c_i32), ("edge_bwd_grid", c_i32),
                ("aggregate", c_i32), ("edge_bwd_waves", c_i32), ("edge_fwd_queue", c_i32),
                ("estate_dtype", c_i32)]


LAYER_FIELDS = ["We1", "be1", "We2", "be2", "ge", "bge", "Wn1", "bn1", "Wn2", "bn2", "gn", "bgn"]


class MpLayerParams(C.Structure):
    _fields_ = [(n, vp) for n in LAYER_FIELDS]


class MpLayerGrads(C.Structure):
    _fields_ = [(n, vp) for n in LAYER_FIELDS]


class MpMlpCfg(C.Structure):
    _fields_ = [("n_in", c_i32), ("H", c_i32), ("n_out", c_i32), ("layernorm", c_i32),
                ("gemm_dtype", c_i32), ("ln_eps", c_f32), ("out_dtype", c_i32)]


MLP_FIELDS = ["W0", "b0", "W1", "b1", "ln_g", "ln_b"]


class MpMlpParams(C.Structure):
    _fields_ = [(n, vp) for n in MLP_FIELDS]


class MpMlpGrads(C.Structure):
    _fields_ = [(n, vp) for n in MLP_FIELDS]


class MpDeepLayerCfg(C.Structure):
    _fields_ = [("H", c_i32), ("n_hidden", c_i32), ("layernorm", c_i32), ("halo", c_i32), ("ln_eps", c_f32),
                ("aggregate", c_i32)]


class MpDeepMlpCfg(C.Structure):
    _fields_ = [("n_in", c_i32), ("H", c_i32), ("n_hidden", c_i32), ("n_out", c_i32), ("layernorm", c_i32),
                ("ln_eps", c_f32)]


P = C.POINTER
_SIGS = {
    "mp_abi_version": (c_i32, []),
    "mp_last_error": (C.c_char_p, []),
    "mp_hex_links": (c_i32, [c_i32, vp, P(c_i32)]),
    "graph_partition": (c_i32, [c_i64, c_i32, vp, c_i32, vp, vp, c_i32, P(vp)]),
    "graph_order_rows": (c_i32, [vp]),
    "mp_graph_sizes": (c_i32, [vp, P(c_i64), P(c_i64), P(c_i32)]),
    "mp_graph_export": (c_i32, [vp] + [vp] * 9),
    "mp_graph_checksum": (c_i32, [vp, P(c_u64)]),
    "mp_graph_destroy": (c_i32, [vp]),
    "halo_plan_build": (c_i32, [vp, P(vp)]),
    "mp_halo_plan_sizes": (c_i32, [vp, P(c_i64), P(c_i64), P(c_i64), P(c_i64)]),
    "mp_halo_plan_export": (c_i32, [vp] + [vp] * 9),
    "mp_halo_plan_checksum": (c_i32, [vp, P(c_u64), P(c_u64)]),
    "mp_halo_plan_destroy": (c_i32, [vp]),
    "mp_dev_graph_seal": (c_i32, [P(MpDevGraph), c_i32]),
    "mp_layer_workspace_size": (c_i32, [P(MpLayerCfg), P(MpDevGraph), c_i32, P(C.c_size_t)]),
    "mp_layer_forward": (c_i32, [P(MpLayerCfg), P(MpLayerParams), P(MpDevGraph), vp, vp, vp, vp, vp,
                                 vp, vp, C.c_size_t, vp]),
    "mp_layer_forward_noalloc": (c_i32, [P(MpLayerCfg), P(MpLayerParams), P(MpDevGraph), vp, vp, vp, vp, vp,
                                         vp, vp]),
    "mp_layer_forward_noalloc_max_scratch": (C.c_size_t, []),
    "mp_layer_backward": (c_i32, [P(MpLayerCfg), P(MpLayerParams), P(MpDevGraph), vp, vp, vp, vp, vp, vp,
                                  vp, vp, P(MpLayerGrads), vp, C.c_size_t, vp]),
    "mp_mlp_workspace_size": (c_i32, [P(MpMlpCfg), c_i64, c_i32, P(C.c_size_t)]),
    "mp_mlp_forward": (c_i32, [P(MpMlpCfg), P(MpMlpParams), c_i64, vp, vp, vp, C.c_size_t, vp]),
    "mp_mlp_backward": (c_i32, [P(MpMlpCfg), P(MpMlpParams), c_i64, vp, vp, vp, P(MpMlpGrads), vp,
                                C.c_size_t, vp]),
    "mp_deep_theta_size": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_i32, P(c_i64)]),
    "mp_deep_layer_workspace_size": (c_i32, [P(MpDeepLayerCfg), P(MpDevGraph), c_i32, P(C.c_size_t)]),
    "mp_deep_layer_forward": (c_i32, [P(MpDeepLayerCfg), vp, vp, P(MpDevGraph), vp, vp, vp, vp, vp, vp]),
    "mp_deep_layer_backward": (c_i32, [P(MpDeepLayerCfg), vp, vp, P(MpDevGraph), vp, vp, vp, vp, vp, vp, vp,
                                       vp, vp, vp, C.c_size_t, vp]),
    "mp_deep_mlp_workspace_size": (c_i32, [P(MpDeepMlpCfg), c_i64, c_i32, P(C.c_size_t)]),
    "mp_deep_mlp_forward": (c_i32, [P(MpDeepMlpCfg), vp, c_i64, vp, vp, vp]),
    "mp_deep_mlp_backward": (c_i32, [P(MpDeepMlpCfg), vp, c_i64, vp, vp, vp, vp, vp, C.c_size_t, vp]),
    "mp_edge_inputs": (c_i32, [P(MpDevGraph), vp, vp, vp, vp, vp]),
    "mp_consistent_mse_workspace_size": (c_i32, [c_i64, P(C.c_size_t)]),
    "mp_consistent_mse": (c_i32, [c_i64, c_i32, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]),
    "mp_profile_enable": (c_i32, [c_i32]),
    "mp_profile_read": (c_i32, [C.c_char_p, P(C.c_double), P(c_i64)]),
}
EXPORTED = sorted(_SIGS)

_lib = None


class MPError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed with code {code}: {msg}")
        self.code = code


def lib():
    """The loaded library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2410_01657_amd.build` (or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if L.mp_abi_version() != ABI_VERSION:
            raise RuntimeError("libmplayer.so ABI version mismatch")
        _lib = L
    return _lib


def check(fn, rc):
    if rc != MP_OK:
        raise MPError(fn, rc, lib().mp_last_error().decode(errors="replace"))
    return rc


def call(fn, *args):
    return check(fn, getattr(lib(), fn)(*args))
