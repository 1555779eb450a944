"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

Nothing in this package performs a step of the consistent message-passing
method.  It only produces what the paper's workflow receives from outside the
GNN (Sec. II-A, Fig. 1): a spectral-element box mesh with global node ids and
GLL point positions (what the CFD solver supplies), an element -> sub-graph
map (what the solver's domain partitioner supplies), a velocity-like node
field, a target field, and randomly initialised model parameters.

Everything is a pure function of an integer seed, so the oracle and the GPU
path see bit-identical inputs without either importing the other.
"""

from .mesh import BoxMesh, gll_points, box_mesh
from .partition import block_partition, slab_partition, rcb_partition
from .fields import velocity_field, shifted_target
from .params import ModelSpec, param_shapes, init_params, count_params
from .configs import CONFIGS, Config, make_inputs, seeds_for

__all__ = [
    "BoxMesh", "gll_points", "box_mesh",
    "block_partition", "slab_partition", "rcb_partition",
    "velocity_field", "shifted_target",
    "ModelSpec", "param_shapes", "init_params", "count_params",
    "CONFIGS", "Config", "make_inputs", "seeds_for",
]
