"""Mesh multiplication of hexahedral meshes with interface elements, plain
CPU reference (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the test-suite is the
only caller.  Nothing here is used by the HIP library or its binding.

Section 2.4 of the paper (Eq. mmu, Algorithm 3): one division level splits
every edge at its midpoint and every face at its centre and adds a node at
the centre of every bulk element, so that a hexahedron becomes eight.  An
8-node interface element (zero thickness, bottom face 0-3, top face 4-7) is
divided only by planes parallel to its normal (the stacking direction): its
bottom and top faces and their edges are divided, its four edges across the
thickness and its four lateral faces are not, and it has no centre node, so
it becomes four.  Algorithm 3 repeats the division ``ndivi`` times.

Numbering of the new mesh (so that two implementations can be compared
entry by entry): the old nodes keep their numbers; then one node per
divided edge in ascending order of its (smaller, larger) end node; then one
per divided face in ascending order of (smallest node, node diagonally
opposite it); then one per bulk element centre in element order.  Children
of element e are 8e .. 8e+7 (bulk, octant i + 2j + 4k of the natural
coordinates) and 4e .. 4e+3 (interface, quadrant i + 2j).  Positions: the
average of the edge's two end nodes (smaller number first), of the face's
four nodes (ascending numbers, summed left to right), of the element's
eight nodes (element order, summed left to right), each sum scaled by 1/2,
1/4 or 1/8.
"""
from __future__ import annotations

import numpy as np

# local topology of a hex8 (bottom 0-3 counter-clockwise, top 4-7)
EDGES = [(0, 1), (1, 2), (2, 3), (3, 0), (4, 5), (5, 6), (6, 7), (7, 4), (0, 4), (1, 5), (2, 6), (3, 7)]
FACES = [(0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]
# lattice positions (a, b, c) in {0, 1, 2}^3 of corners, edge midpoints, face centres, centre
CORNER_AT = [(0, 0, 0), (2, 0, 0), (2, 2, 0), (0, 2, 0), (0, 0, 2), (2, 0, 2), (2, 2, 2), (0, 2, 2)]
EDGE_AT = [(1, 0, 0), (2, 1, 0), (1, 2, 0), (0, 1, 0), (1, 0, 2), (2, 1, 2), (1, 2, 2), (0, 1, 2),
           (0, 0, 1), (2, 0, 1), (2, 2, 1), (0, 2, 1)]
FACE_AT = [(1, 1, 0), (1, 1, 2), (1, 0, 1), (2, 1, 1), (1, 2, 1), (0, 1, 1)]
CHILD = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]


def edge_key(a, b):
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    return (lo.astype(np.int64) << 32) | hi.astype(np.int64)


def face_key(q):
    """q: (n, 4) quads in cyclic order -> (smallest node, the node opposite it)."""
    m = np.argmin(q, axis=1)
    r = np.arange(len(q))
    return (q[r, m].astype(np.int64) << 32) | q[r, (m + 2) % 4].astype(np.int64)


def _edges(hexes, cohs):
    """Divided edges: all 12 of a bulk element, the 8 on the faces of an interface."""
    ks = [edge_key(hexes[:, a], hexes[:, b]) for a, b in EDGES]
    ks += [edge_key(cohs[:, a], cohs[:, b]) for a, b in EDGES[:8]]
    return ks


def _faces(hexes, cohs, lateral=False):
    """Divided faces (all 6 of a bulk element, bottom and top of an interface);
    with lateral=True, also the interface's 4 lateral faces (not divided)."""
    ks = [face_key(hexes[:, list(f)]) for f in FACES]
    ks += [face_key(cohs[:, list(f)]) for f in FACES[:2]]
    if lateral:
        ks += [face_key(cohs[:, list(f)]) for f in FACES[2:]]
    return ks


def counts(coords, hexes, cohs) -> dict:
    """The quantities of Eq. (mmu) for one division of the mesh: divided and
    undivided edges and faces, boundary faces (used by one element; those of
    interface elements are lateral faces), and the new element, node and
    boundary counts by the equation."""
    hexes, cohs = np.asarray(hexes, np.int64).reshape(-1, 8), np.asarray(cohs, np.int64).reshape(-1, 8)
    ne_b, ne_i = len(hexes), len(cohs)
    all_edges = np.unique(np.concatenate(
        [edge_key(hexes[:, a], hexes[:, b]) for a, b in EDGES] +
        [edge_key(cohs[:, a], cohs[:, b]) for a, b in EDGES])) if ne_b + ne_i else np.zeros(0)
    thick = np.unique(np.concatenate([edge_key(cohs[:, a], cohs[:, b]) for a, b in EDGES[8:]])) \
        if ne_i else np.zeros(0)
    all_faces, mult = np.unique(np.concatenate(_faces(hexes, cohs, lateral=True)), return_counts=True)
    lat = np.unique(np.concatenate([face_key(cohs[:, list(f)]) for f in FACES[2:]])) if ne_i else np.zeros(0)
    bnd = all_faces[mult == 1]
    nb0 = len(bnd)
    nb_int = int(np.isin(bnd, lat).sum())
    n_e0 = ne_b + ne_i
    return {
        "n_nodes0": len(coords), "n_bulk0": ne_b, "n_interface0": ne_i,
        "n_edges": len(all_edges), "n_faces": len(all_faces),
        "n_edges_interface": len(thick), "n_faces_interface": len(lat),
        "n_boundary0": nb0, "n_boundary_interface0": nb_int,
        # Eq. (mmu), with n_e,BULK^0 read as all elements of the base mesh
        "n_elements": 8 * n_e0 - 4 * ne_i,
        "n_nodes": len(coords) + len(all_edges) + len(all_faces) + n_e0 - ne_i - len(thick) - len(lat),
        "n_boundary": 4 * nb0 - 2 * nb_int,
    }


def divide(coords, hexes, cohs, hex_tag=None, coh_tag=None):
    """One division level (DivideMesh of Algorithm 3).  Returns the new
    coordinates, bulk and interface connectivity and tags (children inherit
    their parent's)."""
    X = np.asarray(coords, np.float64).reshape(-1, 3)
    H = np.asarray(hexes, np.int64).reshape(-1, 8)
    C = np.asarray(cohs, np.int64).reshape(-1, 8)
    nn, nh, nc = len(X), len(H), len(C)
    # unique divided edges and faces, ascending keys
    ekeys = np.concatenate(_edges(H, C)) if nh + nc else np.zeros(0, np.int64)
    fkeys = np.concatenate(_faces(H, C)) if nh + nc else np.zeros(0, np.int64)
    ue = np.unique(ekeys)
    uf = np.unique(fkeys)
    ne, nf = len(ue), len(uf)
    # positions
    out = np.zeros((nn + ne + nf + nh, 3))
    out[:nn] = X
    a, b = ue >> 32, ue & 0xFFFFFFFF
    out[nn:nn + ne] = 0.5 * (X[a] + X[b])
    # a face's nodes from one element that has it, in ascending order
    fq = np.concatenate([H[:, list(f)] for f in FACES] + [C[:, list(f)] for f in FACES[:2]])
    first = np.unique(fkeys, return_index=True)[1]
    q = np.sort(fq[first], axis=1)
    out[nn + ne:nn + ne + nf] = 0.25 * (((X[q[:, 0]] + X[q[:, 1]]) + X[q[:, 2]]) + X[q[:, 3]])
    cen = X[H[:, 0]]
    for k in range(1, 8):
        cen = cen + X[H[:, k]]
    out[nn + ne + nf:] = 0.125 * cen
    eid = lambda k: nn + np.searchsorted(ue, k)
    fid = lambda k: nn + ne + np.searchsorted(uf, k)
    # bulk children from the 3 x 3 x 3 lattice of each element
    L = np.zeros((nh, 3, 3, 3), np.int64)
    for c, (i, j, k) in enumerate(CORNER_AT):
        L[:, i, j, k] = H[:, c]
    for e, ((p, r), (i, j, k)) in enumerate(zip(EDGES, EDGE_AT)):
        L[:, i, j, k] = eid(edge_key(H[:, p], H[:, r]))
    for f, (i, j, k) in zip(FACES, FACE_AT):
        L[:, i, j, k] = fid(face_key(H[:, list(f)]))
    L[:, 1, 1, 1] = nn + ne + nf + np.arange(nh)
    Hn = np.zeros((nh, 8, 8), np.int64)
    for ch, (i, j, k) in enumerate(CHILD):
        for v, (a_, b_, c_) in enumerate(CHILD):
            Hn[:, ch, v] = L[:, i + a_, j + b_, k + c_]
    # interface children: 3 x 3 lattices on the bottom and top faces
    B = np.zeros((nc, 3, 3, 2), np.int64)
    for c in range(4):
        i, j, _ = CORNER_AT[c]
        B[:, i, j, 0], B[:, i, j, 1] = C[:, c], C[:, c + 4]
    for e in range(4):
        i, j, _ = EDGE_AT[e]
        p, r = EDGES[e]
        B[:, i, j, 0] = eid(edge_key(C[:, p], C[:, r]))
        p, r = EDGES[e + 4]
        B[:, i, j, 1] = eid(edge_key(C[:, p], C[:, r]))
    B[:, 1, 1, 0] = fid(face_key(C[:, [0, 1, 2, 3]]))
    B[:, 1, 1, 1] = fid(face_key(C[:, [4, 5, 6, 7]]))
    Cn = np.zeros((nc, 4, 8), np.int64)
    for ch, (i, j, _) in enumerate(CHILD[:4]):
        for v, (a_, b_, _) in enumerate(CHILD[:4]):
            Cn[:, ch, v] = B[:, i + a_, j + b_, 0]
            Cn[:, ch, v + 4] = B[:, i + a_, j + b_, 1]
    ht = None if hex_tag is None else np.repeat(np.asarray(hex_tag), 8)
    ct = None if coh_tag is None else np.repeat(np.asarray(coh_tag), 4)
    return out, Hn.reshape(-1, 8), Cn.reshape(-1, 8), ht, ct


def multiply(coords, hexes, cohs, ndivi: int, hex_tag=None, coh_tag=None):
    """Algorithm 3: ndivi division levels."""
    X, H, C = coords, hexes, cohs
    for _ in range(ndivi):
        X, H, C, hex_tag, coh_tag = divide(X, H, C, hex_tag, coh_tag)
    return X, H, C, hex_tag, coh_tag
