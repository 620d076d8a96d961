"""Grid hierarchy of the multilevel decomposition (oracle; test infrastructure).

The paper builds a level hierarchy from the input grid (Algorithm 1, first
step) and decomposes level by level; it does not say how a grid whose size is
not 2^k + 1 coarsens.  Reading used here:

* axis coordinates are the grid indices x_i = i (the scale cancels in every
  operator that is used);
* one coarsening step keeps the nodes at even positions of the current level
  and, when the current node count n is even, also the last node n - 1; the
  other nodes are the "new" nodes of that level;
* all axes with more than one node coarsen together; the number of levels L
  is the number of steps until the smallest such axis has 2 nodes; axes of
  length 1 are squeezed out and never coarsen.

Level L is the input grid and level 0 the coarsest grid.
"""
from __future__ import annotations

import numpy as np


def coarse_positions(n: int) -> np.ndarray:
    """Positions (0..n-1) of the nodes that survive one coarsening step."""
    pos = list(range(0, n, 2))
    if n % 2 == 0:
        pos.append(n - 1)
    return np.asarray(pos, dtype=np.int64)


def new_positions(n: int) -> np.ndarray:
    """Positions of the nodes that exist at this level but not the next."""
    keep = set(coarse_positions(n).tolist())
    return np.asarray([i for i in range(n) if i not in keep], dtype=np.int64)


class Hierarchy:
    """Level structure of one array.

    Attributes
    ----------
    shape    the user's shape (any number of axes of length 1 allowed)
    active   indices of the axes with more than one node
    D        number of active axes
    L        number of decomposition levels
    sizes    sizes[l] = tuple of active-axis node counts at level l
    coords   coords[l][d] = coordinates of the level-l nodes on active axis d
    """

    def __init__(self, shape):
        self.shape = tuple(int(s) for s in shape)
        if any(s < 0 for s in self.shape):
            raise ValueError("negative axis length")
        self.N = int(np.prod(self.shape, dtype=np.int64)) if self.shape else 1
        self.active = [d for d, n in enumerate(self.shape) if n > 1]
        self.D = len(self.active)
        fine = tuple(self.shape[d] for d in self.active)
        levels = [fine]
        coords = [[np.arange(n, dtype=np.float64) for n in fine]]
        if self.N > 0 and self.D > 0:
            while min(levels[-1]) > 2:
                cur = levels[-1]
                nxt = tuple(len(coarse_positions(n)) for n in cur)
                coords.append([coords[-1][d][coarse_positions(cur[d])]
                               for d in range(self.D)])
                levels.append(nxt)
        # stored coarsest first: index l runs 0 (coarsest) .. L (input grid)
        self.sizes = levels[::-1]
        self.coords = coords[::-1]
        self.L = len(self.sizes) - 1

    def level_count(self, l: int) -> int:
        """Number of stream entries contributed by level l.

        Level 0 contributes all of its nodes; level l >= 1 its new nodes.
        """
        tot = int(np.prod(self.sizes[l], dtype=np.int64))
        if l == 0:
            return tot
        return tot - int(np.prod(self.sizes[l - 1], dtype=np.int64))

    def max_spacing(self, l: int):
        """Largest node spacing on each active axis at level l."""
        out = []
        for d in range(self.D):
            x = self.coords[l][d]
            out.append(float(np.max(np.diff(x))) if len(x) > 1 else 1.0)
        return out
