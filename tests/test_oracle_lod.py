"""Pins of the oracle's sheet-based LoD hierarchy (Section 5, Section 5.1) on
the CPU, against facts fixed independently of it: the dyadic closed form of
structured grids and single columns (pairs of parallel sheets merge first,
then pairs of pairs, ...), sheet counts and sizes of the polygon prism
derived by hand, hand-counted face sets of small cell constellations, and
the singular-edge exceptions."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import lod


def ctz(p: int) -> int:
    return (p & -p).bit_length() - 1


@pytest.mark.parametrize("N", [1, 2, 4, 8])
def test_cubic_grid_is_dyadic(N):
    """On an N^3 grid (N a power of two) the hierarchy is the dyadic one:
    interior plane p disappears at level ctz(p) + 1, the boundary planes
    never, and an edge disappears with the first of its two planes."""
    levels, info = lod.sheet_lod(synth.grid_cells(N))
    assert info["sheets"] == 3 * N
    assert info["levels"] == int(np.log2(N))
    assert np.array_equal(levels, synth.dyadic_lod_levels(N))
    assert info["merges"] == [3 * (N - 1), 0, 0]  # each axis: N slabs -> 1, adjacent merges only
    assert info["components_left"] == 3


@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_single_column(N):
    """A 1 x 1 x N column: two sheets hold every cell, the N one-cell layers
    merge dyadically.  Horizontal edges at height p have level ctz(p) inside
    and L at the ends (one incident cell); vertical edges have one incident
    cell and keep L."""
    m = synth.box_grid(1, 1, N)
    levels, info = lod.sheet_lod(m.hex)
    L = int(np.log2(N))
    assert info["levels"] == L and info["sheets"] == N + 2
    for c in range(N):
        for e in range(12):
            if e >= 8:
                want = L
            else:
                p = c if e < 4 else c + 1
                want = L if p in (0, N) else ctz(p)
            assert levels[c, e] == want, (c, e)


@pytest.mark.parametrize("k,n,m", [(3, 2, 2), (3, 3, 4), (5, 2, 3), (6, 3, 2)])
def test_prism_sheets(k, n, m):
    """Polygon prism: m layer sheets of k n^2 cells, and k n chord sheets of
    2 n m cells (a chord crosses one block interface and two blocks)."""
    mesh = synth.polygon_prism(k, n, m)
    topo = lod.Topology(mesh.hex)
    sizes = sorted(len(c) for _, c in lod.extract_sheets(topo))
    assert sizes == sorted([k * n * n] * m + [2 * n * m] * (k * n))


def test_sheet_edges_partition_and_parallel_closure():
    mesh = synth.polygon_prism(5, 2, 3)
    topo = lod.Topology(mesh.hex)
    sheets = lod.extract_sheets(topo)
    owner = {}
    for s, (edges, _) in enumerate(sheets):
        for e in edges:
            assert e not in owner
            owner[e] = s
    assert len(owner) == topo.E
    for c in range(topo.C):
        for d in range(3):
            group = {owner[topo.cell_edges[c][le]] for le in range(12) if lod.EDGE_DIR[le] == d}
            assert len(group) == 1  # the four parallel edges of a cell share a sheet


def grid_cells_2d(nx, ny):
    """Cell index of (i, j) in an nx x ny x 1 box grid."""
    return lambda i, j: i + nx * j


def test_relation_classes_hand_counted():
    m = synth.box_grid(3, 3, 1)
    topo = lod.Topology(m.hex)
    c = grid_cells_2d(3, 3)
    col0 = {c(0, 0), c(0, 1), c(0, 2)}
    col1 = {c(1, 0), c(1, 1), c(1, 2)}
    col2 = {c(2, 0), c(2, 1), c(2, 2)}
    row0 = {c(0, 0), c(1, 0), c(2, 0)}
    hook = {c(0, 0), c(1, 0), c(1, 1)}
    # two columns side by side: the 3 faces between them
    cls, merged, tangent, shared = lod.relation(topo, col0, col1)
    assert (cls, len(merged), len(tangent), shared) == (lod.ADJACENT, 3, 3, 0)
    # column and row crossing at (0,0): the two faces around the crossing cell
    cls, merged, tangent, shared = lod.relation(topo, col0, row0)
    assert (cls, len(merged), len(tangent), shared) == (lod.INTERSECTING, 2, 0, 1)
    # column and a hook sharing (0,0) and touching along (0,1)|(1,1)
    cls, merged, tangent, shared = lod.relation(topo, col0, hook)
    assert (cls, len(merged), len(tangent), shared) == (lod.HYBRID, 3, 1, 1)
    # columns with a gap: not neighbours
    cls, merged, tangent, shared = lod.relation(topo, col0, col2)
    assert cls is None and not merged
    # boundary sizes: a column of 3 cells has 3 * 6 - 2 * 2 = 14 boundary faces
    assert len(lod.boundary(topo, col0)) == 14


def test_slab_boundary_and_first_merge():
    """4^3 grid: a slab has 2 * 16 + 4 * 4 = 48 boundary faces; the first
    merge joins the first two x slabs (sheets 0 and 3: cell 0 opens the x, y
    and z sheets 0, 1, 2 and cell 1 the second x sheet) over their 16 shared
    faces."""
    topo = lod.Topology(synth.grid_cells(4))
    sheets = lod.extract_sheets(topo)
    assert [len(lod.boundary(topo, c)) for _, c in sheets] == [48] * 12
    trace = []
    lod.sheet_lod(synth.grid_cells(4), trace=trace)
    level, a, b, new, cls, n_merged, n_tangent, size = trace[0]
    assert (level, a, b, new, cls, n_merged, n_tangent, size) == (1, 0, 3, 12, lod.ADJACENT, 16, 16, 32)
    # pairs before pairs of pairs: the merged sizes never decrease
    sizes = [t[7] for t in trace]
    assert sizes == sorted(sizes)


def test_eq5_prefers_smaller_components():
    """Eq. 5 at equal face ratio favours the smaller pair (Section 5.1)."""
    assert lod.eq5_weight(10, 20, 20, 5, 5) > lod.eq5_weight(10, 20, 20, 6, 6)
    assert lod.eq5_weight(11, 20, 20, 5, 5) > lod.eq5_weight(10, 20, 20, 5, 5)


@pytest.mark.parametrize("k,n,m", [(3, 2, 2), (3, 3, 4), (5, 4, 4), (5, 2, 8)])
def test_prism_singular_edges(k, n, m):
    """Edges with one incident cell keep the coarsest level.  The singular
    centre edges (k incident cells) lie on the faces between the innermost
    chords of neighbouring blocks, which become interior when those chords
    merge, so they disappear, and only at the coarsest level: level L - 1
    (for k = 5, n = 2, m = 8 their faces become interior two levels before
    the last).  Every level lies in [0, L]."""
    mesh = synth.polygon_prism(k, n, m)
    topo = lod.Topology(mesh.hex)
    levels, info = lod.sheet_lod(mesh.hex)
    L = info["levels"]
    assert L >= 1 and levels.max() <= L
    per_edge = {}
    for c in range(topo.C):
        for le in range(12):
            per_edge.setdefault(topo.cell_edges[c][le], set()).add(int(levels[c, le]))
    assert all(len(v) == 1 for v in per_edge.values())
    lv = {e: v.pop() for e, v in per_edge.items()}
    centre = [e for e in range(topo.E) if topo.valence[e] == k and not topo.on_boundary[e]]
    assert len(centre) == m
    for e in centre:
        assert lv[e] == L - 1
    ones = [e for e in range(topo.E) if topo.valence[e] == 1]
    # polygon corners (k m vertical edges) and the top and bottom outlines (2 * 2 k n)
    assert len(ones) == k * m + 4 * k * n
    assert all(lv[e] == L for e in ones)
    assert info["singular_edges"] == m + len(ones)


def test_prism_has_hybrid_and_intersecting_merges():
    """The triangle prism's innermost chords cross in one block and touch
    across the opposite block interface: a hybrid pair; layers and chords
    intersect."""
    mesh = synth.polygon_prism(3, 2, 2)
    topo = lod.Topology(mesh.hex)
    sheets = [c for _, c in lod.extract_sheets(topo)]
    classes = set()
    for i in range(len(sheets)):
        for j in range(i + 1, len(sheets)):
            cls = lod.relation(topo, sheets[i], sheets[j])[0]
            classes.add(cls)
    assert {lod.ADJACENT, lod.HYBRID, lod.INTERSECTING} <= classes
    levels, info = lod.sheet_lod(mesh.hex)
    assert info["merges"][1] >= 1 and info["merges"][2] >= 1


def test_errors():
    bad = synth.grid_cells(1).copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(ValueError):
        lod.sheet_lod(bad)
    levels, info = lod.sheet_lod(np.zeros((0, 8), np.int32))
    assert levels.shape == (0, 12) and info["levels"] == 0
