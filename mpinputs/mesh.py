"""Spectral-element box mesh: hexahedral elements with (P+1)^3 GLL points.

This is the geometry a spectral-element CFD solver hands to the graph builder
(Sec. II-A): per element, the global node id of each element-local quadrature
point, and per global id, its physical position.  Points on shared element
faces carry the same global id (the "local coincident nodes" of Sec. II-A,
Fig. 3a).  No graph is built here.

Conventions
-----------
* ``nel = (nx, ny, nz)`` elements on the unit box ``[0, 1]^3``.
* Element id ``ex + nx*(ey + ny*ez)``.
* Element-local point ``(a, b, c)`` in ``[0, P]^3`` has local index
  ``a + (P+1)*(b + (P+1)*c)``.
* Global lattice index along an axis: ``I = ex*P + a``; ``n = nx*P + 1``
  points per axis (``nx*P`` when that axis is periodic, the index wrapping).
* ``gid = I + n_x*(J + n_y*K)``.
"""

from dataclasses import dataclass

import numpy as np


def _legendre_and_derivs(n, x):
    """Legendre polynomial P_n, P_n' and P_n'' at x (three-term recurrence)."""
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x), np.zeros_like(x)
    p1 = x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    pn, pnm1 = p1, p0
    # P_n' from (1 - x^2) P_n' = n (P_{n-1} - x P_n); valid off the end points
    dp = n * (pnm1 - x * pn) / (1.0 - x * x)
    # Legendre ODE: (1 - x^2) P'' = 2 x P' - n (n + 1) P
    d2p = (2.0 * x * dp - n * (n + 1) * pn) / (1.0 - x * x)
    return pn, dp, d2p


def gll_points(P):
    """The P+1 Gauss-Legendre-Lobatto points on [-1, 1], ascending.

    End points are -1 and 1; the interior points are the roots of P_P', the
    derivative of the Legendre polynomial of degree P (the quadrature rule
    the spectral-element solver places its nodes at, Sec. II-A).  Newton
    iteration from the Chebyshev-Gauss-Lobatto points, then symmetrised.
    """
    if P < 1:
        raise ValueError("polynomial order must be >= 1")
    x = -np.cos(np.pi * np.arange(P + 1) / P)
    if P >= 2:
        xi = x[1:-1].copy()
        for _ in range(100):
            _, dp, d2p = _legendre_and_derivs(P, xi)
            step = dp / d2p
            xi -= step
            if np.max(np.abs(step)) < 1e-16:
                break
        x[1:-1] = xi
    x[0], x[-1] = -1.0, 1.0
    x = 0.5 * (x - x[::-1])  # exact antisymmetry x_k = -x_{P-k}
    return x


@dataclass
class BoxMesh:
    nel: tuple            # elements per axis
    P: int                # polynomial order
    periodic: tuple       # per-axis periodicity
    npts: tuple           # distinct lattice points per axis
    elem_gid: np.ndarray  # [n_elem, (P+1)^3] int64 global node ids
    pos: np.ndarray       # [n_gid, 3] float64 positions in [0, 1)^3 (None if not asked for)

    @property
    def n_elem(self):
        return int(self.elem_gid.shape[0])

    @property
    def npe(self):
        return int(self.elem_gid.shape[1])

    @property
    def n_gid(self):
        return int(np.prod(self.npts))

    @property
    def period(self):
        """Per-axis period of the positions (1.0 on periodic axes, else 0)."""
        return tuple(1.0 if p else 0.0 for p in self.periodic)


def axis_coords(nel, P):
    """Positions of the nel*P+1 lattice points along one axis of [0, 1]."""
    xi = gll_points(P)
    t = (xi + 1.0) / 2.0
    c = np.empty(nel * P + 1)
    for e in range(nel):
        c[e * P:(e + 1) * P + 1] = (e + t) / nel
    c[-1] = 1.0
    return c


def box_mesh(nel, P, periodic=(False, False, False), with_positions=True):
    """Build the element -> global-id table (and positions) of a box mesh."""
    nel = tuple(int(v) for v in nel)
    periodic = tuple(bool(v) for v in periodic)
    npts = tuple(nel[a] * P + (0 if periodic[a] else 1) for a in range(3))
    q = P + 1
    a = np.arange(q)
    # element-local point (a, b, c) -> offsets along each axis
    la = np.tile(a, q * q)
    lb = np.tile(np.repeat(a, q), q)
    lc = np.repeat(a, q * q)
    ex, ey, ez = np.meshgrid(np.arange(nel[0]), np.arange(nel[1]),
                             np.arange(nel[2]), indexing="ij")
    # element id order: ex fastest
    ex = ex.transpose(2, 1, 0).reshape(-1)
    ey = ey.transpose(2, 1, 0).reshape(-1)
    ez = ez.transpose(2, 1, 0).reshape(-1)
    I = ex[:, None] * P + la[None, :]
    J = ey[:, None] * P + lb[None, :]
    K = ez[:, None] * P + lc[None, :]
    if periodic[0]:
        I %= npts[0]
    if periodic[1]:
        J %= npts[1]
    if periodic[2]:
        K %= npts[2]
    gid = (I + npts[0] * (J + npts[1] * K.astype(np.int64))).astype(np.int64)
    pos = None
    if with_positions:
        # a periodic axis has nel*P distinct points: the last one is the first
        cx, cy, cz = (axis_coords(nel[i], P)[:npts[i]] for i in range(3))
        n = npts[0] * npts[1] * npts[2]
        g = np.arange(n, dtype=np.int64)
        pos = np.empty((n, 3))
        pos[:, 0] = cx[g % npts[0]]
        pos[:, 1] = cy[(g // npts[0]) % npts[1]]
        pos[:, 2] = cz[g // (npts[0] * npts[1])]
    return BoxMesh(nel, P, periodic, npts, gid, pos)
