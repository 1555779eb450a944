"""Element -> sub-graph maps: the domain decomposition a CFD solver supplies.

The paper takes the sub-graphs from the solver's own partitioner (Sec. II-A,
Fig. 3b).  These generators stand in for it on box meshes: element blocks,
slabs, and a seeded recursive coordinate bisection with uneven pieces.
Each returns ``elem_part[n_elem]`` (int32, values in ``[0, R)``) in the
element-id order of :mod:`mpinputs.mesh`.
"""

import numpy as np


def _elem_coords(nel):
    nx, ny, nz = nel
    e = np.arange(nx * ny * nz)
    return e % nx, (e // nx) % ny, e // (nx * ny)


def block_partition(nel, blocks):
    """Tensor-product cut into ``bx*by*bz`` equal element blocks."""
    ex, ey, ez = _elem_coords(nel)
    bx, by, bz = blocks
    for n, b in zip(nel, blocks):
        if n % b:
            raise ValueError("element count must divide evenly into blocks")
    px = ex // (nel[0] // bx)
    py = ey // (nel[1] // by)
    pz = ez // (nel[2] // bz)
    return (px + bx * (py + by * pz)).astype(np.int32)


def slab_partition(nel, R, axis=2):
    """R slabs of equal thickness along one axis."""
    c = _elem_coords(nel)[axis]
    if nel[axis] % R:
        raise ValueError("element count must divide evenly into slabs")
    return (c // (nel[axis] // R)).astype(np.int32)


def _rcb_once(nel, levels, rng, frac):
    boxes = [((0, 0, 0), tuple(nel))]
    for _ in range(levels):
        nxt = []
        for lo, hi in boxes:
            ext = [hi[a] - lo[a] for a in range(3)]
            ax = int(np.argmax(ext))  # longest axis (first on ties)
            f = rng.uniform(frac[0], frac[1])
            cut = lo[ax] + int(round(f * ext[ax]))
            cut = min(max(cut, lo[ax] + 1), hi[ax] - 1)
            hi1 = list(hi); hi1[ax] = cut
            lo2 = list(lo); lo2[ax] = cut
            nxt.append((lo, tuple(hi1)))
            nxt.append((tuple(lo2), hi))
        boxes = nxt
    return boxes


def rcb_partition(nel, R, seed, frac=(0.40, 0.60), ratio=(2.5, 3.0),
                  max_tries=100000):
    """Seeded recursive coordinate bisection into R = 2^levels uneven blocks.

    Each box is cut on its longest axis at a fraction drawn from
    U[frac[0], frac[1]].  Draws are repeated until the ratio of the largest
    to the smallest block (in elements) lies in ``ratio``.
    Returns ``(elem_part, info)`` with the accepted draw count and ratio.
    """
    levels = int(round(np.log2(R)))
    if 2 ** levels != R:
        raise ValueError("R must be a power of two")
    rng = np.random.Generator(np.random.PCG64(seed))
    for attempt in range(1, max_tries + 1):
        boxes = _rcb_once(nel, levels, rng, frac)
        sizes = np.array([np.prod([hi[a] - lo[a] for a in range(3)])
                          for lo, hi in boxes])
        if sizes.min() <= 0:
            continue
        r = sizes.max() / sizes.min()
        if ratio[0] <= r <= ratio[1]:
            break
    else:
        raise RuntimeError("no partition within the requested size ratio")
    ex, ey, ez = _elem_coords(nel)
    part = np.full(ex.shape, -1, dtype=np.int32)
    for p, (lo, hi) in enumerate(boxes):
        m = ((ex >= lo[0]) & (ex < hi[0]) & (ey >= lo[1]) & (ey < hi[1])
             & (ez >= lo[2]) & (ez < hi[2]))
        part[m] = p
    assert (part >= 0).all()
    return part, {"tries": attempt, "ratio": float(r),
                  "sizes": sizes.tolist(), "boxes": boxes}
