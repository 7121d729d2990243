"""Fragments of damaged particles -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
use this module; the library never imports it.

Sec. 7.3 counts the child particles a particle breaks into.  Here a child is
a connected component of the graph whose vertices are the nodes and whose
edges are the intact bonds (a node that lost every bond is a component of
its own).  Bonds never join two particles, so every component lies in one
particle.  Each component is named by its smallest node index.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components


def components(row: np.ndarray, col: np.ndarray, broken: np.ndarray, n: int) -> np.ndarray:
    """label[i] = smallest node index of node i's component, over the bonds
    in CSR form (row offsets, column indices, one entry per direction); a
    bond joins its nodes while either of its directed entries is not
    broken."""
    row = np.asarray(row, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    keep = np.asarray(broken, dtype=bool) == False  # noqa: E712
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row))
    g = coo_matrix((np.ones(int(keep.sum())), (src[keep], col[keep])), shape=(n, n)).tocsr()
    k, comp = connected_components(g, directed=False)
    smallest = np.full(k, n, dtype=np.int64)
    np.minimum.at(smallest, comp, np.arange(n, dtype=np.int64))
    return smallest[comp].astype(np.int32)


def child_counts(label: np.ndarray, particle_offset: np.ndarray, min_nodes: int) -> np.ndarray:
    """Per particle, the number of components with at least min_nodes nodes."""
    label = np.asarray(label)
    n = label.shape[0]
    size = np.bincount(label, minlength=n)
    roots = np.nonzero(label == np.arange(n))[0]
    part = np.searchsorted(np.asarray(particle_offset), roots, side="right") - 1
    P = len(particle_offset) - 1
    return np.bincount(part[size[roots] >= min_nodes], minlength=P).astype(np.int32)
