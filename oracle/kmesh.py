"""Crystal-momentum meshes for the oracle (test infrastructure).

A Monkhorst-Pack mesh of n0 x n1 x n2 points in the first Brillouin zone,
k = (j0/n0, j1/n1, j2/n2) in reciprocal-lattice units.  Momentum is
conserved modulo a reciprocal-lattice vector (Eq. momentum), so k points add
component by component, each component modulo its own n_d: the group
Z_n0 x Z_n1 x Z_n2.  A 1D chain (the systems of the paper) is the mesh
(Nk, 1, 1); the 3D mesh is the extension the paper lists as planned work
(Sec. V).  Points are stored by flat index (j0 * n1 + j1) * n2 + j2, so a
1D chain keeps its plain index j.

Every function of the oracle that takes `nk` accepts an int (a 1D chain), a
tuple of up to three mesh extents, or a Mesh.
"""
from __future__ import annotations

import numpy as np


class Mesh:
    def __init__(self, dims):
        dims = tuple(int(d) for d in dims)
        if not 1 <= len(dims) <= 3 or min(dims) < 1:
            raise ValueError(f"bad k mesh {dims}")
        self.dims = dims + (1,) * (3 - len(dims))
        self.size = int(np.prod(self.dims))

    def __repr__(self):
        return f"Mesh{self.dims}"

    def vec(self, k):
        """Integer coordinates (j0, j1, j2) of flat point k."""
        n0, n1, n2 = self.dims
        return (k // (n1 * n2), (k // n2) % n1, k % n2)

    def flat(self, j):
        n0, n1, n2 = self.dims
        return ((j[0] % n0) * n1 + (j[1] % n1)) * n2 + (j[2] % n2)

    def signed(self, terms):
        """Flat index of sum_i s_i k_i for terms [(s_i, k_i), ...]."""
        acc = [0, 0, 0]
        for s, k in terms:
            j = self.vec(k)
            for d in range(3):
                acc[d] += s * j[d]
        return self.flat(acc)

    def add(self, a, b):
        return self.signed([(1, a), (1, b)])

    def sub(self, a, b):
        return self.signed([(1, a), (-1, b)])

    def comb(self, a, b, c):
        """a + b - c: the fourth momentum of a conserving quartet."""
        return self.signed([(1, a), (1, b), (-1, c)])


def mesh_of(nk) -> Mesh:
    if isinstance(nk, Mesh):
        return nk
    if isinstance(nk, (tuple, list)):
        return Mesh(nk)
    return Mesh((int(nk),))
