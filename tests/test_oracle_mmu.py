"""Pins of the host mesh multiplication (oracle/mmu.py; Section 2.4, Eq. mmu,
Algorithm 3) against what the paper and geometry fix: Table 3's element and
node counts of the AS4/8552 coupon at both refinement levels, the three
counts of Eq. (mmu), the structured mesh of the next level, conservation of
volume and interface area on distorted, renumbered meshes, and inheritance
of the ply."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import mmu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _volumes(X, H):
    return np.array([oracle.hex8_geometry(X[h])[1] for h in H])


def _quad_area(P):
    """Area of planar quads (n, 4, 3): half the norm of the diagonals' cross product."""
    return 0.5 * np.linalg.norm(np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 1]), axis=1)


def test_table3_counts_from_one_division_of_the_coupon():
    """Dividing the level-0 AS4/8552 coupon mesh (Table 3: 335,622 elements,
    364,320 nodes) once gives Table 3's level-1 mesh: 2,109,624 elements and
    2,219,983 nodes; Eq. (mmu) predicts both from the base mesh."""
    g = json.load(open(os.path.join(GOLD, "table3_mesh_counts.json")))
    X, H, C, hp, cp = W.hex_mesh(W.coupon_as4(0)["mesh"])
    assert len(H) + len(C) == g["levels"][0]["n_elements"] and len(X) == g["levels"][0]["n_nodes"]
    c = mmu.counts(X, H, C)
    X1, H1, C1, _, _ = mmu.divide(X, H, C)
    lv1 = g["levels"][1]
    assert len(H1) + len(C1) == lv1["n_elements"] == c["n_elements"]
    assert len(X1) == lv1["n_nodes"] == c["n_nodes"]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_eq_mmu_counts_on_renumbered_distorted_meshes(seed):
    """On seeded renumbered, distorted meshes with interfaces, one division has
    exactly the element, node and boundary-face counts of Eq. (mmu) (the
    boundary counted on the divided mesh itself), and two divisions those of
    the equation applied twice."""
    cfg = W.tiny(3 + seed, 2 + seed, 3, 1, angles=[0, 45, 90], cohesive=1)
    X, H, C, _, _ = W.hex_mesh(cfg["mesh"])
    X, H, C = W.renumbered(X, H, C, seed, distort=0.2)
    c = mmu.counts(X, H, C)
    assert c["n_interface0"] > 0 and c["n_boundary_interface0"] > 0
    X1, H1, C1, _, _ = mmu.divide(X, H, C)
    assert len(H1) + len(C1) == c["n_elements"] and len(C1) == 4 * len(C)
    assert len(X1) == c["n_nodes"]
    c1 = mmu.counts(X1, H1, C1)
    assert c1["n_boundary0"] == c["n_boundary"]
    X2, H2, C2, _, _ = mmu.multiply(X, H, C, 2)
    assert len(H2) == 64 * len(H) and len(C2) == 16 * len(C)
    assert len(X2) == c1["n_nodes"]


def test_division_conserves_volume_and_interface_area():
    """The children of a trilinear hexahedron are the parent's map restricted
    to the octants of its natural coordinates, so their volumes add up to the
    parent's, distorted or not; each is positive.  The four children of an
    interface element cover its area, and keep zero thickness."""
    cfg = W.tiny(4, 3, 2, 2, angles=[0, 90], cohesive=1)
    X, H, C, _, _ = W.hex_mesh(cfg["mesh"])
    X, H, C = W.renumbered(X, H, C, 7, distort=0.25)
    X1, H1, C1, _, _ = mmu.divide(X, H, C)
    v0, v1 = _volumes(X, H), _volumes(X1, H1)
    assert (v1 > 0).all()
    assert np.abs(v1.reshape(-1, 8).sum(axis=1) - v0).max() <= 1e-13 * v0.max()
    a0 = _quad_area(X[C[:, :4]])
    a1 = _quad_area(X1[C1[:, :4]]).reshape(-1, 4).sum(axis=1)
    assert np.abs(a1 - a0).max() <= 1e-13 * a0.max()
    # zero thickness kept (to rounding: the coincident faces' nodes are summed
    # in the order of their own numbers)
    assert np.abs(X1[C1[:, :4]] - X1[C1[:, 4:]]).max() <= 1e-15 * np.abs(X).max()


def test_division_of_a_structured_plate_is_the_next_level():
    """Dividing a structured plate with interfaces once gives the plate of
    twice the in-plane resolution and two elements per ply: the same node
    positions and the same elements (as sets of corner positions)."""
    m0 = W.tiny(5, 3, 3, 1, angles=[0, 90, 0], cohesive=1, lx=5e-3, ly=3e-3, ply_thickness=0.4e-3)["mesh"]
    m1 = dict(m0, nx=10, ny=6, elems_per_ply=2)
    X, H, C, _, _ = W.hex_mesh(m0)
    Xd, Hd, Cd, _, _ = mmu.divide(X, H, C)
    Y, G, D, _, _ = W.hex_mesh(m1)
    q = lambda P: np.round(P / 1e-12).astype(np.int64)
    kx = sorted(map(tuple, q(Xd)))
    ky = sorted(map(tuple, q(Y)))
    assert kx == ky
    el = lambda P, E: sorted(tuple(sorted(map(tuple, q(P[e])))) for e in E)
    assert el(Xd, Hd) == el(Y, G)
    assert el(Xd, Cd) == el(Y, D)


def test_children_inherit_the_ply():
    cfg = W.tiny(2, 2, 3, 1, angles=[0, 45, 90], cohesive=1)
    X, H, C, hp, cp = W.hex_mesh(cfg["mesh"])
    _, H1, C1, hp1, cp1 = mmu.divide(X, H, C, hp, cp)
    assert np.array_equal(hp1, np.repeat(hp, 8)) and np.array_equal(cp1, np.repeat(cp, 4))
