"""Oracle of the sheet-based level-of-detail edge hierarchy (Section 5 and
Section 5.1 of the paper), written for clarity, not speed: plain Python sets
and dictionaries, every pair statistic recomputed from its definition at
every merge step.  Test infrastructure only (the tests and the benchmark's
CPU leg use it); the library's own builder shares nothing with it.

What it computes, for a hexahedral mesh given as cells of 8 vertex ids in
VTK order, is the level `e_level` of every edge: the coarsest LoD level at
which the edge is still drawn (Section 3, Section 5).

1. Sheets (Section 5, after Woodbury et al.): starting from the
   lowest-numbered edge not yet visited, collect every cell incident to a
   collected edge and, in each such cell, the three edges topologically
   parallel to it, until nothing new is found.  The cells found form the
   sheet's component; repeat until every edge is visited.  Edges are
   numbered in order of first appearance, scanning cells in order and each
   cell's 12 edges in the local order below.
2. Components are cell sets.  The boundary of a component is the set of
   faces with exactly one incident cell in it (faces of the mesh boundary
   included).
3. Two components are neighbours when merging them turns at least one face
   of either boundary into an interior face (Section 5.1).  The pair is
   adjacent when they share no cell, hybrid when they share cells and also
   touch tangentially (a face between a cell of only the one and a cell of
   only the other), intersecting when they share cells and do not.
4. Priority (Section 5.1): adjacent before hybrid before intersecting; within
   a class the larger weight of Eq. 5 first, with the numerator the number
   of boundary faces that the merge makes interior; exact ties go to the pair
   with the smaller (smaller id, larger id).  Sheets have ids 0..S-1 in
   extraction order, a merged component the next free id.
5. Merging the best pair replaces both by their union.  The edges of the
   faces on both boundaries that become interior (the tangent faces; none
   for an intersecting pair) become invisible at the current level.
6. Levels: the first merge opens level 1.  A later merge whose result has
   more than twice as many cells as the larger of the two components whose
   merge opened the current level opens the next level (and belongs to it).
   Merging stops when no neighbouring pair is left.  The coarsest level L is
   the level of the last merge (0 if there was none).
7. e_level = (level at which the edge first became invisible) - 1, or L if
   it never did.  Singular edges (Section 5.1: on the boundary with other
   than 2 incident cells, inside with other than 4) are exceptions: an edge
   with one incident cell keeps L; any other singular edge that was made
   invisible gets L - 1.  (An edge with one incident cell lies on mesh
   boundary faces only, which never become interior, so with the readings
   above the first exception never changes a level; it is kept as stated.)

Readings where the paper leaves a choice are listed with the design notes.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

# local edges of a VTK hexahedron and their direction class
EDGES = ((0, 1), (1, 2), (2, 3), (3, 0), (4, 5), (5, 6), (6, 7), (7, 4),
         (0, 4), (1, 5), (2, 6), (3, 7))
EDGE_DIR = (0, 1, 0, 1, 0, 1, 0, 1, 2, 2, 2, 2)
# local faces (corner lists)
FACES = ((0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7))

ADJACENT, HYBRID, INTERSECTING = 0, 1, 2
CLASS_NAMES = ("adjacent", "hybrid", "intersecting")


class Topology:
    """Edges, faces and incidences of a hexahedral mesh."""

    def __init__(self, hexes):
        hexes = [tuple(int(v) for v in c) for c in np.asarray(hexes)]
        self.hex = hexes
        self.C = len(hexes)
        self.edge_id = {}          # (lo, hi) -> id, first-appearance order
        self.edge_cells = []       # id -> [(cell, local edge)]
        self.cell_edges = []       # cell -> [12 edge ids]
        for c, h in enumerate(hexes):
            if len(set(h)) != 8:
                raise ValueError(f"cell {c} has a repeated corner")
            ids = []
            for le, (a, b) in enumerate(EDGES):
                key = (min(h[a], h[b]), max(h[a], h[b]))
                if key not in self.edge_id:
                    self.edge_id[key] = len(self.edge_cells)
                    self.edge_cells.append([])
                e = self.edge_id[key]
                self.edge_cells[e].append((c, le))
                ids.append(e)
            self.cell_edges.append(ids)
        self.E = len(self.edge_cells)
        self.face_id = {}          # sorted corner tuple -> id
        self.face_cells = []       # id -> [cells]
        self.face_edges = []       # id -> [4 edge ids]
        self.cell_faces = []       # cell -> [6 face ids]
        for c, h in enumerate(hexes):
            ids = []
            for lf in FACES:
                key = tuple(sorted(h[v] for v in lf))
                if key not in self.face_id:
                    self.face_id[key] = len(self.face_cells)
                    self.face_cells.append([])
                    corners = [h[v] for v in lf]
                    self.face_edges.append([self.edge_id[(min(corners[q], corners[(q + 1) % 4]),
                                                          max(corners[q], corners[(q + 1) % 4]))]
                                            for q in range(4)])
                f = self.face_id[key]
                self.face_cells[f].append(c)
                ids.append(f)
            self.cell_faces.append(ids)
        if any(len(cs) > 2 for cs in self.face_cells):
            raise ValueError("a face is shared by more than two cells")
        self.F = len(self.face_cells)
        # valence and boundary flags of the edges
        self.valence = [len(cs) for cs in self.edge_cells]
        self.on_boundary = [False] * self.E
        for f, cs in enumerate(self.face_cells):
            if len(cs) == 1:
                for e in self.face_edges[f]:
                    self.on_boundary[e] = True

    def parallel_edges(self, cell, local_edge):
        """The edges of `cell` in the direction class of its `local_edge`."""
        d = EDGE_DIR[local_edge]
        return [self.cell_edges[cell][le] for le in range(12) if EDGE_DIR[le] == d]

    def singular(self, e):
        return self.valence[e] != (2 if self.on_boundary[e] else 4)


def extract_sheets(topo: Topology):
    """Sheets as (edge set, cell set), in extraction order (Section 5)."""
    visited = [False] * topo.E
    sheets = []
    for start in range(topo.E):
        if visited[start]:
            continue
        edges, cells = {start}, set()
        visited[start] = True
        frontier = [start]
        while frontier:
            nxt = []
            for e in frontier:
                for c, le in topo.edge_cells[e]:
                    cells.add(c)
                    for p in topo.parallel_edges(c, le):
                        if not visited[p]:
                            visited[p] = True
                            edges.add(p)
                            nxt.append(p)
            frontier = nxt
        sheets.append((edges, cells))
    return sheets


def boundary(topo: Topology, cells):
    """Faces with exactly one incident cell in `cells`."""
    count = {}
    for c in cells:
        for f in topo.cell_faces[c]:
            count[f] = count.get(f, 0) + 1
    return {f for f, n in count.items() if n == 1}


def relation(topo: Topology, ci, cj, bi=None, bj=None):
    """Neighbourhood of two components (Section 5.1).

    Returns (class or None, merged faces, tangent faces, shared cell count):
    merged = faces of either boundary that are interior to the union,
    tangent = faces on both boundaries that are interior to the union.
    class is None when the components are not neighbours."""
    bi = boundary(topo, ci) if bi is None else bi
    bj = boundary(topo, cj) if bj is None else bj
    union = ci | cj

    def interior_to_union(f):
        cs = topo.face_cells[f]
        return len(cs) == 2 and cs[0] in union and cs[1] in union

    merged = {f for f in bi | bj if interior_to_union(f)}
    tangent = {f for f in bi & bj if interior_to_union(f)}
    shared = len(ci & cj)
    if not merged:
        return None, merged, tangent, shared
    if shared == 0:
        cls = ADJACENT
    elif tangent:
        cls = HYBRID
    else:
        cls = INTERSECTING
    return cls, merged, tangent, shared


def eq5_weight(n_merged, bnd_i, bnd_j, size_i, size_j) -> Fraction:
    """Eq. 5: merged boundary faces over the two boundary sizes, times the
    inverse of the two cell counts (exact)."""
    return Fraction(n_merged, bnd_i + bnd_j) * Fraction(1, size_i + size_j)


def sheet_lod(hexes, trace=None):
    """Per-cell edge levels (uint8 [C, 12]) and a summary dict.

    `trace`, if a list, receives one tuple per merge:
    (level, id_a, id_b, new_id, class, n_merged, n_tangent, new_size)."""
    topo = Topology(hexes)
    sheets = extract_sheets(topo)
    comps = {i: set(cells) for i, (_, cells) in enumerate(sheets)}
    bnd = {i: boundary(topo, c) for i, c in comps.items()}
    next_id = len(sheets)
    hidden_at = [None] * topo.E
    level, level_ref = 0, 0
    last_level = 0
    merges = [0, 0, 0]
    while True:
        best = None
        ids = sorted(comps)
        for x in range(len(ids)):
            for y in range(x + 1, len(ids)):
                i, j = ids[x], ids[y]
                cls, merged, tangent, _ = relation(topo, comps[i], comps[j], bnd[i], bnd[j])
                if cls is None:
                    continue
                w = eq5_weight(len(merged), len(bnd[i]), len(bnd[j]), len(comps[i]), len(comps[j]))
                key = (cls, -w, i, j)
                if best is None or key < best[0]:
                    best = (key, tangent, len(merged))
        if best is None:
            break
        (cls, _, i, j), tangent, n_merged = best
        union = comps[i] | comps[j]
        if level == 0 or len(union) > 2 * level_ref:
            level += 1
            level_ref = max(len(comps[i]), len(comps[j]))
        for f in tangent:
            for e in topo.face_edges[f]:
                if hidden_at[e] is None:
                    hidden_at[e] = level
        del comps[i], comps[j], bnd[i], bnd[j]
        comps[next_id] = union
        bnd[next_id] = boundary(topo, union)
        if trace is not None:
            trace.append((level, i, j, next_id, cls, n_merged, len(tangent), len(union)))
        next_id += 1
        last_level = level
        merges[cls] += 1
    L = last_level
    e_level = []
    for e in range(topo.E):
        h = hidden_at[e]
        if topo.valence[e] == 1:
            lv = L
        elif topo.singular(e):
            lv = L if h is None else L - 1
        else:
            lv = L if h is None else h - 1
        e_level.append(lv)
    out = np.array([[e_level[e] for e in topo.cell_edges[c]] for c in range(topo.C)], dtype=np.int64)
    info = {
        "sheets": len(sheets),
        "sheet_sizes": [len(c) for _, c in sheets],
        "levels": L,
        "merges": merges,
        "components_left": len(comps),
        "edges": topo.E,
        "faces": topo.F,
        "singular_edges": sum(1 for e in range(topo.E) if topo.singular(e)),
    }
    return out.astype(np.uint8).reshape(topo.C, 12), info
