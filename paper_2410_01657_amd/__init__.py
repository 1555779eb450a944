"""Consistent neural message passing on one MI355X (gfx950).

The consistent NMP layer of "Scalable and Consistent Graph Neural Networks
for Distributed Mesh-based Data-driven Modeling" (Eq. 4a-e), its adjoint,
the encode-process-decode model around it and the consistent loss (Eq. 6),
all as hand-written HIP kernels behind the C ABI of include/mplayer.h.
This package is the thin Python binding: graph building and kernel calls
go through libmplayer.so, which must be built first (``build.build()``).
"""

from ._lib import MPError, lib  # noqa: F401
from .graph import DeviceGraph, HostGraph, build_graph, hex_links  # noqa: F401
