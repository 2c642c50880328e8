"""Conversion between the oracle's entity numbering and slot arrays
(oracle; test infrastructure only).

Data is exchanged between tests, inputs and the oracle as arrays of shape
(3, nz, ny, nx): slot [a, k, j, i] holds the quantity of the edge (or facet)
of direction a anchored at node (i, j, k).  Every kept (PEC-interior) edge
and facet has a slot; other slots are zero on output and ignored on input.
"""
from __future__ import annotations

import numpy as np

from .leapfrog import Operators

__all__ = ["edges_from_slots", "edges_to_slots", "facets_from_slots", "facets_to_slots",
           "cells_from_array", "cells_to_array"]


def _slot_index(ops: Operators, kind: str):
    top = ops.top
    ids = ops.ie if kind == "edge" else ops.if_
    offs = top.edge_off if kind == "edge" else top.facet_off
    boxes = top.edge_box if kind == "edge" else top.facet_box
    a = np.searchsorted(offs, ids, side="right") - 1
    local = ids - offs[a]
    bx = np.array([boxes[q][0] for q in range(3)])[a]
    by = np.array([boxes[q][1] for q in range(3)])[a]
    out = np.empty((4, ids.size), dtype=np.int64)
    out[0] = a
    out[3] = local % bx                 # i
    out[2] = (local // bx) % by         # j
    out[1] = local // (bx * by)         # k
    return out


def edges_from_slots(ops: Operators, arr) -> np.ndarray:
    s = _slot_index(ops, "edge")
    return np.asarray(arr, dtype=np.float64)[s[0], s[1], s[2], s[3]]


def facets_from_slots(ops: Operators, arr) -> np.ndarray:
    s = _slot_index(ops, "facet")
    return np.asarray(arr, dtype=np.float64)[s[0], s[1], s[2], s[3]]


def edges_to_slots(ops: Operators, v) -> np.ndarray:
    n = ops.top.n
    out = np.zeros((3, n[2], n[1], n[0]))
    s = _slot_index(ops, "edge")
    out[s[0], s[1], s[2], s[3]] = v
    return out


def facets_to_slots(ops: Operators, v) -> np.ndarray:
    n = ops.top.n
    out = np.zeros((3, n[2], n[1], n[0]))
    s = _slot_index(ops, "facet")
    out[s[0], s[1], s[2], s[3]] = v
    return out


def cells_from_array(arr) -> np.ndarray:
    """(nz, ny, nx) per-cell array -> oracle cell numbering (x fastest)."""
    return np.asarray(arr, dtype=np.float64).ravel()


def cells_to_array(v, nx, ny, nz) -> np.ndarray:
    return np.asarray(v, dtype=np.float64).reshape(nz, ny, nx)
