"""Synthetic node fields standing in for a solver's velocity snapshot.

The paper feeds a Taylor-Green-vortex velocity snapshot and uses it as the
target (Sec. III-B).  That data is not available; this module draws a seeded
Taylor-Green-like field instead.  Values are a function of the global id
only, so every copy of a coincident node sees the same value, as the paper
requires of node attributes on coincident nodes (Sec. II-A).
"""

import numpy as np


def velocity_field(pos, seed, noise_sigma=0.0, amplitude=1.0):
    """[n_gid, 3] float32 field at the given positions.

    u =  A sin(2 pi x + p1) cos(2 pi y + p2) cos(2 pi z + p3)
    v = -A cos(2 pi x + p1) sin(2 pi y + p2) cos(2 pi z + p3)
    w =  0
    with phases p ~ U[0, 2 pi) drawn from ``seed``; optional N(0, sigma^2)
    noise (sigma is the standard deviation) is added per value.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ph = rng.uniform(0.0, 2.0 * np.pi, size=3)
    tx = 2.0 * np.pi * pos[:, 0] + ph[0]
    ty = 2.0 * np.pi * pos[:, 1] + ph[1]
    tz = 2.0 * np.pi * pos[:, 2] + ph[2]
    f = np.zeros((pos.shape[0], 3))
    f[:, 0] = amplitude * np.sin(tx) * np.cos(ty) * np.cos(tz)
    f[:, 1] = -amplitude * np.cos(tx) * np.sin(ty) * np.cos(tz)
    if noise_sigma > 0.0:
        f += rng.normal(0.0, noise_sigma, size=f.shape)
    return f.astype(np.float32)


def shifted_target(field, npts):
    """Target = the field shifted by one lattice node along x, with wrap.

    ``T(I, J, K) = X((I + 1) mod n_x, J, K)`` on the global lattice.
    """
    nx, ny, nz = npts
    f = field.reshape(nz, ny, nx, -1)
    return np.ascontiguousarray(np.roll(f, -1, axis=2).reshape(field.shape))
