"""Staggered grid pair and explicit incidence matrices (oracle; test infrastructure only).

Paper: Sec. II, eqs. maxwell_grid1 and maxwell_grid2 -- the discrete curls
C (primal, acting on edge voltages e) and C~ (dual, acting on h), the
divergences on the primal and dual grid, and n_dof ~ 3n.

Readings taken where the text is terse or garbled:

* The two divergence names are swapped in the text relative to the fields
  they act on; here ``S`` is the PRIMAL divergence (acts on b, lives on
  primal facets -> primal cells) and ``S~`` the DUAL divergence (acts on d,
  dual facets = primal edges -> dual cells = primal nodes).  The identities
  checked are S C = 0 and S~ C~ = 0.
* The paper counts grid POINTS; the API counts CELLS (points = cells + 1).

Orientation: primal edges point along +axis; a primal facet normal to axis a
is oriented by +a with right-handed circulation through (b, c) = the cyclic
successors of a.  Dual edges cross primal facets in +a direction; dual facets
are crossed by primal edges in +a direction; dual cells surround primal
nodes.  Every matrix entry is an integer in {-1, 0, 1}.

Each operator below is assembled from its own geometric construction; none
is derived from another by transposition, so that C~ = C^T, S C = 0,
S~ C~ = 0 and C G = 0 are genuine checks.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = ["Topology"]


def _succ(a: int):
    return (a + 1) % 3, (a + 2) % 3


class Topology:
    """Entities of an nx x ny x nz cell grid and their explicit incidences.

    Entity numbering (oracle-internal): nodes, cells, and per-direction blocks
    of edges and facets, each block x-fastest over its own index box.
    """

    def __init__(self, nx: int, ny: int, nz: int):
        if min(nx, ny, nz) < 1:
            raise ValueError("need at least one cell per axis")
        self.n = np.array([nx, ny, nz], dtype=np.int64)
        eye = np.eye(3, dtype=np.int64)
        self.node_box = self.n + 1
        self.cell_box = self.n.copy()
        # a-edges: n_a positions along a, n_b + 1 along the other axes
        self.edge_box = [self.n + 1 - eye[a] for a in range(3)]
        # a-facets: n_a + 1 positions along a, n_b along the others
        self.facet_box = [self.n + eye[a] for a in range(3)]
        self.edge_off = np.concatenate([[0], np.cumsum([np.prod(b) for b in self.edge_box])])
        self.facet_off = np.concatenate([[0], np.cumsum([np.prod(b) for b in self.facet_box])])
        self.n_nodes = int(np.prod(self.node_box))
        self.n_cells = int(np.prod(self.cell_box))
        self.n_edges = int(self.edge_off[-1])
        self.n_facets = int(self.facet_off[-1])

    # ------------------------------------------------------------------ index helpers
    @staticmethod
    def _coords(box):
        """All (i, j, k) of an index box, x fastest; returns three flat arrays."""
        k, j, i = np.meshgrid(np.arange(box[2]), np.arange(box[1]), np.arange(box[0]),
                              indexing="ij")
        return i.ravel(), j.ravel(), k.ravel()

    @staticmethod
    def _flat(box, p):
        return p[0] + box[0] * (p[1] + box[1] * p[2])

    @staticmethod
    def _inside(box, p):
        return (p[0] >= 0) & (p[0] < box[0]) & (p[1] >= 0) & (p[1] < box[1]) & \
               (p[2] >= 0) & (p[2] < box[2])

    def node(self, p):
        return self._flat(self.node_box, p)

    def cell(self, p):
        return self._flat(self.cell_box, p)

    def edge(self, a, p):
        return self.edge_off[a] + self._flat(self.edge_box[a], p)

    def facet(self, a, p):
        return self.facet_off[a] + self._flat(self.facet_box[a], p)

    def edge_coords(self, a):
        return np.stack(self._coords(self.edge_box[a]))

    def facet_coords(self, a):
        return np.stack(self._coords(self.facet_box[a]))

    def node_coords(self):
        return np.stack(self._coords(self.node_box))

    def cell_coords(self):
        return np.stack(self._coords(self.cell_box))

    @staticmethod
    def _shift(p, a, d):
        q = p.copy()
        q[a] += d
        return q

    # ------------------------------------------------------------------ primal operators
    def gradient(self) -> sp.csr_matrix:
        """G: nodes -> primal edges; (G phi) on the a-edge from node p to p + e_a
        is phi(p + e_a) - phi(p)."""
        rows, cols, vals = [], [], []
        for a in range(3):
            p = self.edge_coords(a)
            r = self.edge(a, p)
            rows += [r, r]
            cols += [self.node(p), self.node(self._shift(p, a, 1))]
            vals += [-np.ones_like(r), np.ones_like(r)]
        return self._assemble(rows, cols, vals, self.n_edges, self.n_nodes)

    def curl(self) -> sp.csr_matrix:
        """C: primal edges -> primal facets (eq. maxwell_grid1, C e = -d_t b).

        The a-facet anchored at node p is bounded by the b-edge at p (+), the
        c-edge at p + e_b (+), the b-edge at p + e_c (-) and the c-edge at
        p (-): the right-handed circulation seen from +a.
        """
        rows, cols, vals = [], [], []
        for a in range(3):
            b, c = _succ(a)
            p = self.facet_coords(a)
            r = self.facet(a, p)
            for ax, q, s in ((b, p, 1), (c, self._shift(p, b, 1), 1),
                             (b, self._shift(p, c, 1), -1), (c, p, -1)):
                rows.append(r)
                cols.append(self.edge(ax, q))
                vals.append(np.full_like(r, s))
        return self._assemble(rows, cols, vals, self.n_facets, self.n_edges)

    def divergence(self) -> sp.csr_matrix:
        """S: primal facets -> primal cells; outward flux of each cell (S b = 0)."""
        rows, cols, vals = [], [], []
        p = self.cell_coords()
        r = self.cell(p)
        for a in range(3):
            rows += [r, r]
            cols += [self.facet(a, p), self.facet(a, self._shift(p, a, 1))]
            vals += [-np.ones_like(r), np.ones_like(r)]
        return self._assemble(rows, cols, vals, self.n_cells, self.n_facets)

    # ------------------------------------------------------------------ dual operators
    def dual_curl(self) -> sp.csr_matrix:
        """C~: dual edges (numbered as the primal facets they cross) -> dual
        facets (numbered as the primal edges crossing them); C~ h = d_t d + j.

        The dual facet crossed by the a-edge at node p sits at a-coordinate
        p_a + 1/2 and spans [p_b - 1/2, p_b + 1/2] x [p_c - 1/2, p_c + 1/2].
        Walking its boundary counter-clockwise seen from +a:
          c = p_c - 1/2, along +b : dual b-edge crossing the b-facet at p - e_c  (+)
          b = p_b + 1/2, along +c : dual c-edge crossing the c-facet at p        (+)
          c = p_c + 1/2, along -b : dual b-edge crossing the b-facet at p        (-)
          b = p_b - 1/2, along -c : dual c-edge crossing the c-facet at p - e_b  (-)
        Dual edges that would cross a facet outside the domain do not exist
        (the dual facet of a boundary edge is truncated by the boundary).
        """
        rows, cols, vals = [], [], []
        for a in range(3):
            b, c = _succ(a)
            p = self.edge_coords(a)
            r = self.edge(a, p)
            for ax, q, s in ((b, self._shift(p, c, -1), 1), (c, p, 1),
                             (b, p, -1), (c, self._shift(p, b, -1), -1)):
                ok = self._inside(self.facet_box[ax], q)
                rows.append(r[ok])
                cols.append(self.facet(ax, q[:, ok]))
                vals.append(np.full(int(ok.sum()), s, dtype=np.int64))
        return self._assemble(rows, cols, vals, self.n_edges, self.n_facets)

    def dual_divergence(self) -> sp.csr_matrix:
        """S~: dual facets (primal edges) -> dual cells (primal nodes); outward
        flux of the dual cell around each node (S~ d = q)."""
        rows, cols, vals = [], [], []
        p = self.node_coords()
        r = self.node(p)
        for a in range(3):
            for q, s in ((p, 1), (self._shift(p, a, -1), -1)):
                ok = self._inside(self.edge_box[a], q)
                rows.append(r[ok])
                cols.append(self.edge(a, q[:, ok]))
                vals.append(np.full(int(ok.sum()), s, dtype=np.int64))
        return self._assemble(rows, cols, vals, self.n_nodes, self.n_edges)

    # ------------------------------------------------------------------ PEC restriction
    def interior_edges(self) -> np.ndarray:
        """Boolean mask over edges: True for edges not lying in a boundary
        plane.  Tangential e vanishes on a PEC wall, so the others are held 0."""
        m = np.zeros(self.n_edges, dtype=bool)
        for a in range(3):
            b, c = _succ(a)
            p = self.edge_coords(a)
            ok = (p[b] > 0) & (p[b] < self.n[b]) & (p[c] > 0) & (p[c] < self.n[c])
            m[self.edge(a, p)] = ok
        return m

    def interior_facets(self) -> np.ndarray:
        """Boolean mask over facets: True for facets not lying in a boundary
        plane (the normal flux b vanishes on a PEC wall)."""
        m = np.zeros(self.n_facets, dtype=bool)
        for a in range(3):
            p = self.facet_coords(a)
            m[self.facet(a, p)] = (p[a] > 0) & (p[a] < self.n[a])
        return m

    def interior_nodes(self) -> np.ndarray:
        p = self.node_coords()
        return (p[0] > 0) & (p[0] < self.n[0]) & (p[1] > 0) & (p[1] < self.n[1]) & \
               (p[2] > 0) & (p[2] < self.n[2])

    def canonical_ndof(self) -> int:
        """Size of u = [h; e] with 3 slots per grid point for each field
        (n_dof ~ 3n per field, phantom slots included)."""
        return 2 * 3 * int(np.prod(self.node_box))

    # ------------------------------------------------------------------ helpers
    @staticmethod
    def _assemble(rows, cols, vals, nr, nc):
        r = np.concatenate(rows)
        c = np.concatenate(cols)
        v = np.concatenate(vals).astype(np.float64)
        return sp.csr_matrix((v, (r, c)), shape=(nr, nc))
