"""The five workloads, as seeded synthetic inputs.

C0  tiny:    4^3 elements, P=3, H=32, 2 layers, no LayerNorm, field + N(0, 0.01^2)
             noise; R=1 and R=8 (2x2x2 element blocks).
C1  medium:  16^3 elements, P=5, H=64, 4 layers, LayerNorm; R=1 and R=16 z-slabs.
C2  C1 with the MLP GEMMs in BF16 (same mesh, model and partition).
C3  fwd+bwd: 24^3 elements, P=5, H=128, 4 layers, LayerNorm, MSE against the
             field shifted one node in x; R=1 (R=8 blocks for gradient checks).
C4  batched: 32^3 elements, P=7, H=64, 4 layers, LayerNorm; 64 uneven
             sub-graphs from a seeded recursive coordinate bisection.
T2R8 the partition of Table II's R = 8 row: 16 x 16 x 128 elements, P=5,
             periodic on all three axes, 8 z-slabs of 518,400 rows each;
             C1's model (H=64, 4 layers, LayerNorm), target shifted in x.
"""

from dataclasses import dataclass, field as dc_field

import numpy as np

from .mesh import box_mesh
from .partition import block_partition, slab_partition, rcb_partition
from .fields import velocity_field, shifted_target
from .params import ModelSpec, init_params


@dataclass(frozen=True)
class Config:
    name: str
    nel: tuple
    P: int
    spec: ModelSpec
    partition: str           # "none", "blocks", "slabs", "rcb"
    R: int
    blocks: tuple = (1, 1, 1)
    noise: float = 0.0
    gemm: str = "f32"        # "f32" or "bf16"
    backward: bool = False
    periodic: tuple = (False, False, False)


CONFIGS = {
    "C0": Config("C0", (4, 4, 4), 3, ModelSpec(H=32, n_layers=2, layernorm=False),
                 "blocks", 8, blocks=(2, 2, 2), noise=0.01),
    "C1": Config("C1", (16, 16, 16), 5, ModelSpec(H=64, n_layers=4, layernorm=True),
                 "slabs", 16),
    "C2": Config("C2", (16, 16, 16), 5, ModelSpec(H=64, n_layers=4, layernorm=True),
                 "slabs", 16, gemm="bf16"),
    "C3": Config("C3", (24, 24, 24), 5, ModelSpec(H=128, n_layers=4, layernorm=True),
                 "blocks", 8, blocks=(2, 2, 2), backward=True),
    "C4": Config("C4", (32, 32, 32), 7, ModelSpec(H=64, n_layers=4, layernorm=True),
                 "rcb", 64, gemm="bf16", backward=True),
    "T2R8": Config("T2R8", (16, 16, 128), 5, ModelSpec(H=64, n_layers=4, layernorm=True),
                   "slabs", 8, gemm="bf16", backward=True, periodic=(True, True, True)),
}


def seeds_for(base_seed=0):
    """Independent integer seeds for field, weights and partition."""
    ss = np.random.SeedSequence(base_seed)
    kids = ss.spawn(3)
    names = ("field", "weights", "partition")
    return {n: int(k.generate_state(1, dtype=np.uint64)[0]) for n, k in zip(names, kids)}


def element_partition(cfg, R=None, seed=0):
    """Element -> sub-graph map for a config (R=1 gives all zeros)."""
    R = cfg.R if R is None else R
    n_elem = int(np.prod(cfg.nel))
    if R == 1 or cfg.partition == "none":
        return np.zeros(n_elem, dtype=np.int32)
    if cfg.partition == "blocks":
        return block_partition(cfg.nel, cfg.blocks)
    if cfg.partition == "slabs":
        return slab_partition(cfg.nel, R, axis=2)
    if cfg.partition == "rcb":
        part, _ = rcb_partition(cfg.nel, R, seed)
        return part
    raise ValueError(cfg.partition)


@dataclass
class Inputs:
    cfg: Config
    mesh: object
    field: np.ndarray        # [n_gid, 3] float32 node input
    target: np.ndarray       # [n_gid, 3] float32 target
    params: dict             # name -> float32 array
    elem_part: np.ndarray    # [n_elem] int32
    seeds: dict = dc_field(default_factory=dict)


def make_inputs(cfg, base_seed=0, R=None, perturb=False, spec=None):
    seeds = seeds_for(base_seed)
    mesh = box_mesh(cfg.nel, cfg.P, cfg.periodic)
    field = velocity_field(mesh.pos, seeds["field"], noise_sigma=cfg.noise)
    target = shifted_target(field, mesh.npts)
    params = init_params(spec or cfg.spec, seeds["weights"], perturb=perturb)
    part = element_partition(cfg, R, seeds["partition"])
    return Inputs(cfg, mesh, field, target, params, part, seeds)
