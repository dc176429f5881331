"""Workload definitions and seeded input generators.

This module is shared by the oracle harness and the HIP path's binding, so it
holds inputs only: mesh sizes, ply layups, material constants, impactor data
and seeded random numbers.  It contains none of the method's arithmetic (no
kinematics, no constitutive law, no time integration); the oracle and the
library each derive everything else (impact velocity from energy, stable time
step, stiffness, ...) in their own code.

Sources of the numbers:
  * Table 1 (material properties, AS4/8552 column) of the paper for strengths,
    toughness, softening shape factors and interface properties;
  * the elastic constants the workloads state (E1 = 130 GPa, E2 = E3 = 8 GPa,
    G12 = 4.5 GPa, nu12 = 0.3), with nu23 = 0.45 and rho = 1590 kg/m^3 from the
    AS4/8552 column and G23 = E2 / (2 (1 + nu23)) as Table 1's own G23 entries
    follow (7630/2.9 = 2631, 8540/2.9 = 2945);
  * Section 3.2 (ASTM D7136 set-up): 150 x 100 mm coupon, 125 x 75 mm frame
    cut-out, clamps at the four corners, 0.01 mm initial gap, gravity 9.81.
All values are SI (m, kg, s, N, Pa, J/m^2).
"""
from __future__ import annotations

import copy
import math

import numpy as np

# ---------------------------------------------------------------------------
# seeded generators
# ---------------------------------------------------------------------------

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea, Flood 2014), the published 64-bit mixer."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def randint(self, lo: int, hi: int) -> int:
        """Integer uniform on [lo, hi] inclusive."""
        return lo + int(self.uniform() * (hi - lo + 1))


def rng(seed: int) -> np.random.Generator:
    """numpy generator for synthetic states (parity inputs)."""
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------
# materials
# ---------------------------------------------------------------------------

LAW_ELASTIC = 0
LAW_CDM = 1
LAW_CDM_SURROGATE = 2

BC_CLAMPED_EDGES = 0
BC_ASTM_WINDOW = 1
BC_FREE = 2

PREC_FP64 = 0
PREC_MIXED = 1


def material_isotropic(E: float, nu: float, rho: float) -> dict:
    """Isotropic elastic solid written in the transversely isotropic fields."""
    G = E / (2.0 * (1.0 + nu))
    return dict(E1=E, E2=E, E3=E, nu12=nu, nu13=nu, nu23=nu, G12=G, G13=G, G23=G,
                rho=rho, law=LAW_ELASTIC,
                XT=0.0, XC=0.0, YT=0.0, YC=0.0, SL=0.0, alpha0_deg=53.0,
                GXT=0.0, GXC=0.0, GYT=0.0, GYC=0.0, GSL=0.0,
                fXT=0.0, fGT=0.0, fXC=0.0, fGC=0.0,
                KI=0.0, tauI=0.0, tauII=0.0, GIc=0.0, GIIc=0.0, eta_bk=1.0, Sp=0.0, Kp=0.0)


# Table 1, Hexply AS4/8552, matrix plasticity: yield stress S_p (MPa) and the
# hardening K_p (printed in N/mm; read as the plastic modulus over G12)
AS4_SP = 62.0e6
AS4_KP = 0.1936


def material_cfrp(outer: bool, ply_thickness: float, law: int = LAW_CDM, plastic: bool = False) -> dict:
    """Carbon/epoxy ply: workload elastic constants + Table 1 AS4/8552 damage data.

    ``outer`` selects the outer-ply in-situ strengths (Y_T = 74.2, S_L = 94.4 MPa)
    instead of the embedded-ply ones (Y_T = 117.5, S_L = 120.8 MPa).  The
    interface penalty is K_I = 50 E2 / t_ply (Section 2.3.2's lower bound), since
    Table 1's AS4 value violates that bound.  ``plastic`` adds Table 1's
    longitudinal shear plasticity (S_p, K_p); off, the law is elastic-damage.
    """
    E2 = 8.0e9
    nu23 = 0.45
    m = dict(E1=130.0e9, E2=E2, E3=E2, nu12=0.3, nu13=0.3, nu23=nu23,
             G12=4.5e9, G13=4.5e9, G23=E2 / (2.0 * (1.0 + nu23)), rho=1590.0,
             law=law,
             XT=2300.0e6, XC=1531.0e6,
             YT=(74.2e6 if outer else 117.5e6), YC=199.8e6,
             SL=(94.4e6 if outer else 120.8e6), alpha0_deg=53.0,
             GXT=81.5e3, GXC=106.3e3, GYT=280.0, GYC=1313.0, GSL=790.0,
             fXT=0.1, fGT=0.6, fXC=0.1, fGC=0.9,
             KI=50.0 * E2 / ply_thickness, tauI=74.2e6, tauII=94.36e6,
             GIc=280.0, GIIc=790.0, eta_bk=1.45,
             Sp=(AS4_SP if plastic else 0.0), Kp=(AS4_KP if plastic else 0.0))
    return m


def ply_materials(n_plies: int, ply_thickness: float, law: int = LAW_CDM, plastic: bool = False) -> list:
    return [material_cfrp(p == 0 or p == n_plies - 1, ply_thickness, law, plastic)
            for p in range(n_plies)]


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def _mesh(nx, ny, n_plies, elems_per_ply, lx, ly, ply_thickness, angles, *,
          cohesive=0, bc=BC_CLAMPED_EDGES, window_lx=0.0, window_ly=0.0,
          clamp_radius=0.0, precision=PREC_FP64, phi=1.0, cfl_safety=0.9,
          gravity=9.81, hourglass_kappa=0.05, integration=1):
    return dict(nx=nx, ny=ny, n_plies=n_plies, elems_per_ply=elems_per_ply,
                lx=lx, ly=ly, ply_thickness=ply_thickness,
                ply_angle_deg=[float(a) for a in angles], cohesive=cohesive,
                bc=bc, window_lx=window_lx, window_ly=window_ly,
                clamp_radius=clamp_radius, precision=precision, phi=phi,
                cfl_safety=cfl_safety, gravity=gravity,
                hourglass_kappa=hourglass_kappa, integration=integration)


def impactor(R, mass, *, v0=0.0, energy=0.0, gap=1.0e-5, x0=None, y0=None):
    """Rigid hemispherical striker; x0/y0 None = plate centre."""
    return dict(radius=R, mass=mass, v0=v0, energy=energy, gap=gap,
                x0=(float('nan') if x0 is None else x0),
                y0=(float('nan') if y0 is None else y0))


LAYUP_QI8 = [0, 45, -45, 90, 90, -45, 45, 0]      # [0/45/-45/90]s


def plate_iso_20x20x4() -> dict:
    """Isotropic plate 20x20x4, 50x50x2 mm, clamped edges, 0.5 kg at 2 m/s."""
    return dict(
        name="plain-fp64-isotropic-20x20x4",
        mesh=_mesh(20, 20, 1, 4, 0.05, 0.05, 0.002, [0.0]),
        materials=[material_isotropic(70.0e9, 0.3, 2700.0)],
        impactor=impactor(8.0e-3, 0.5, v0=2.0),
        steps=2000)


def plate_qi8_300x200x8(precision=PREC_MIXED) -> dict:
    """[0/45/-45/90]s, 150x100 mm, 300x200x8, CDM, 5.5 kg at 15 J."""
    t = 0.5e-3
    return dict(
        name="cdm-qi8-300x200x8",
        mesh=_mesh(300, 200, 8, 1, 0.150, 0.100, t, LAYUP_QI8,
                   bc=BC_ASTM_WINDOW, window_lx=0.125, window_ly=0.075,
                   clamp_radius=5.0e-3, precision=precision),
        materials=ply_materials(8, t),
        impactor=impactor(8.0e-3, 5.5, energy=15.0),
        steps=61000)


def plate_qi8_1200x800x16(precision=PREC_MIXED) -> dict:
    """Same laminate at 1200x800x16 (2 elements/ply) with cohesive interfaces, 25 J."""
    t = 0.5e-3
    return dict(
        name="cdm-czm-qi8-1200x800x16",
        mesh=_mesh(1200, 800, 8, 2, 0.150, 0.100, t, LAYUP_QI8, cohesive=1,
                   bc=BC_ASTM_WINDOW, window_lx=0.125, window_ly=0.075,
                   clamp_radius=5.0e-3, precision=precision),
        materials=ply_materials(8, t),
        impactor=impactor(8.0e-3, 5.5, energy=25.0),
        steps=20000)


def plate_qi8_150x100x16_cut(precision=PREC_FP64) -> dict:
    """A 150 x 100-column cut of the 1200 x 800 x 16 plate at its element size
    (0.125 x 0.125 x 0.25 mm, 18.75 x 12.5 mm), with its 6 cohesive
    interfaces, its striker (R = 8 mm, 5.5 kg at 25 J) and its support type:
    the window and the corner clamp discs scaled with the plate (window
    125/150 x 75/100 of the cut, clamp radius 5 mm x 18.75/150)."""
    c = plate_qi8_1200x800x16(precision)
    c["name"] = "cdm-czm-qi8-150x100x16-cut"
    m = c["mesh"]
    f = 150.0 / 1200.0
    m.update(nx=150, ny=100, lx=0.150 * f, ly=0.100 * f, window_lx=0.125 * f, window_ly=0.075 * f,
             clamp_radius=5.0e-3 * f)
    c["steps"] = 2000
    return c


def plate_qi8_1200x800x16_surrogate(precision=PREC_MIXED) -> dict:
    c = plate_qi8_1200x800x16(precision)
    c["name"] = "surrogate-qi8-1200x800x16"
    for m in c["materials"]:
        m["law"] = LAW_CDM_SURROGATE
    return c


# The AS4/8552 drop-weight coupon of Section 3.2.2: [45_4/0_4/-45_4/90_4]_S of
# 0.181 mm plies, modelled as eight clusters of four plies (the two middle 90
# clusters form the eight-ply cluster), interface elements between clusters of
# different angle (six), 150 x 100 mm on the 125 x 75 mm window, 5 kg striker
# of radius 8 mm at 2.78 m/s (19.3 J), 5 ms.  The in-plane grid reproduces the
# element and node counts of Table 3 at both refinement levels.
AS4_PLY = 0.181e-3
AS4_CLUSTERS = [45, 0, -45, 90, 90, -45, 0, 45]


def material_as4_8552(outer: bool, t_lam: float, law: int = LAW_CDM, plastic: bool = False) -> dict:
    """Table 1, Hexply AS4/8552 column, in SI.  ``outer`` selects the outer
    cluster's in-situ strengths (Y_T = 74.2, S_L = 94.4 MPa) instead of the
    embedded ones (Y_T = 117.5, S_L = 120.8 MPa; the same for 4- and 8-ply
    clusters).  Interface: tau_I = Y_T, tau_II = S_L of the base material,
    penalty K_I = 50 E2 / t_lam (Section 2.3.2's bound; Table 1's value
    violates it)."""
    E2 = 7.63e9
    return dict(E1=128.0e9, E2=E2, E3=E2, nu12=0.35, nu13=0.35, nu23=0.45,
                G12=4.358e9, G13=4.358e9, G23=2.631e9, rho=1590.0, law=law,
                XT=2300.0e6, XC=1531.0e6,
                YT=(74.2e6 if outer else 117.5e6), YC=199.8e6,
                SL=(94.4e6 if outer else 120.8e6), alpha0_deg=53.0,
                GXT=81.5e3, GXC=106.3e3, GYT=280.0, GYC=1313.0, GSL=790.0,
                fXT=0.1, fGT=0.6, fXC=0.1, fGC=0.9,
                KI=50.0 * E2 / t_lam, tauI=74.2e6, tauII=94.36e6,
                GIc=280.0, GIIc=790.0, eta_bk=1.45,
                Sp=(AS4_SP if plastic else 0.0), Kp=(AS4_KP if plastic else 0.0))


def coupon_as4(level: int = 0, precision=PREC_MIXED, phi: float = 1.033) -> dict:
    """The AS4/8552 coupon at refinement level 0 (183 x 131, one element per
    cluster) or 1 (366 x 262, two), with the dissipative Tchamwa-Wielgosz
    member phi = 1.033 of Section 2.2.1 by default, and Table 1's matrix
    shear plasticity."""
    nx, ny, epc = ((183, 131, 1), (366, 262, 2))[level]
    t = 4 * AS4_PLY
    return dict(
        name=f"as4-8552-coupon-level{level}",
        mesh=_mesh(nx, ny, 8, epc, 0.150, 0.100, t, AS4_CLUSTERS, cohesive=1,
                   bc=BC_ASTM_WINDOW, window_lx=0.125, window_ly=0.075,
                   clamp_radius=5.0e-3, precision=precision, phi=phi),
        materials=[material_as4_8552(p in (0, 7), t, plastic=True) for p in range(8)],
        impactor=impactor(8.0e-3, 5.0, v0=2.78),
        t_end=5.0e-3)


def batch_cases_64(n_cases=64, base_seed=0x9D5EED00) -> list:
    """Uneven batch: per case s, SplitMix64(base_seed + s) draws, in this order,
    plies P ~ U{4..16}, P angles from {0, 45, -45, 90}, target elements
    N_e ~ U[20k, 400k], impact energy ~ U[5, 40] J and mass ~ U[1, 6] kg."""
    cases = []
    t = 0.25e-3
    for s in range(n_cases):
        g = SplitMix64(base_seed + s)
        P = g.randint(4, 16)
        angles = [(0, 45, -45, 90)[g.randint(0, 3)] for _ in range(P)]
        Ne = 20000 + g.uniform() * 380000.0
        energy = 5.0 + 35.0 * g.uniform()
        mass = 1.0 + 5.0 * g.uniform()
        nx = max(2, int(round(math.sqrt(1.5 * Ne / P))))
        ny = max(2, int(round(Ne / (P * nx))))
        cases.append(dict(
            name=f"batch-case-{s}",
            mesh=_mesh(nx, ny, P, 1, 0.150, 0.100, t, angles,
                       bc=BC_ASTM_WINDOW, window_lx=0.125, window_ly=0.075,
                       clamp_radius=5.0e-3, precision=PREC_MIXED),
            materials=ply_materials(P, t),
            impactor=impactor(8.0e-3, mass, energy=energy),
            steps=1000))
    return cases


def scaled(cfg: dict, nx: int, ny: int, lx: float = None, ly: float = None,
           precision: int = None, **mesh_over) -> dict:
    """Copy of a workload on a smaller in-plane grid (same physics per element
    when lx/ly shrink with nx/ny)."""
    c = copy.deepcopy(cfg)
    m = c["mesh"]
    m["nx"], m["ny"] = nx, ny
    if lx is not None:
        m["lx"] = lx
    if ly is not None:
        m["ly"] = ly
    if precision is not None:
        m["precision"] = precision
    m.update(mesh_over)
    return c


def tiny(nx=4, ny=4, n_plies=2, elems_per_ply=1, *, angles=None, cohesive=0,
         law=LAW_ELASTIC, precision=PREC_FP64, lx=8.0e-3, ly=8.0e-3,
         ply_thickness=1.0e-3, bc=BC_CLAMPED_EDGES, energy=0.0, v0=3.0,
         mass=0.05, R=4.0e-3, gravity=9.81, isotropic=False, plastic=False) -> dict:
    """Small mesh for brute-force and parity cases."""
    if angles is None:
        angles = [0.0 if p % 2 == 0 else 90.0 for p in range(n_plies)]
    if isotropic:
        mats = [material_isotropic(70.0e9, 0.3, 2700.0) for _ in range(n_plies)]
    else:
        mats = ply_materials(n_plies, ply_thickness, law, plastic)
    return dict(
        name=f"tiny-{nx}x{ny}x{n_plies * elems_per_ply}",
        mesh=_mesh(nx, ny, n_plies, elems_per_ply, lx, ly, ply_thickness, angles,
                   cohesive=cohesive, bc=bc, window_lx=0.75 * lx,
                   window_ly=0.75 * ly, clamp_radius=0.1 * min(lx, ly),
                   precision=precision, gravity=gravity),
        materials=mats,
        impactor=impactor(R, mass, v0=v0, energy=energy),
        steps=50)


# ---------------------------------------------------------------------------
# explicit (unstructured) hexahedral meshes, for the mesh multiplication
# ---------------------------------------------------------------------------

def hex_mesh(mesh: dict):
    """The plate of a workload mesh dict as an explicit mesh: node coordinates
    (n_nodes x 3), bulk hex8 and 8-node interface connectivity (node order:
    bottom face counter-clockwise from (-,-), then the top face; an interface
    element's bottom and top nodes are the coincident nodes of the duplicated
    plane) and the ply of each element.  Node n = i + (nx+1)(j + (ny+1)k) on
    node plane k; elements i fastest, then j, then layer."""
    nx, ny, P, epp = mesh["nx"], mesh["ny"], mesh["n_plies"], mesh["elems_per_ply"]
    ang = mesh["ply_angle_deg"]
    hz = mesh["ply_thickness"] / epp
    coh_layer, ply = [], []
    for p in range(P):
        for _ in range(epp):
            coh_layer.append(False)
            ply.append(p)
        if mesh.get("cohesive", 0) and p + 1 < P and ang[p] != ang[p + 1]:
            coh_layer.append(True)
            ply.append(p)
    K = len(coh_layer) + 1
    z = np.zeros(K)
    for l, c in enumerate(coh_layer):
        z[l + 1] = z[l] + (0.0 if c else hz)
    i, j, k = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(K), indexing="ij")
    nid = lambda a, b, c: a + (nx + 1) * (b + (ny + 1) * c)
    coords = np.zeros(((nx + 1) * (ny + 1) * K, 3))
    n = nid(i, j, k).reshape(-1)
    coords[n, 0] = mesh["lx"] * i.reshape(-1) / nx
    coords[n, 1] = mesh["ly"] * j.reshape(-1) / ny
    coords[n, 2] = z[k.reshape(-1)]
    ie, je = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ie, je = ie.reshape(-1), je.reshape(-1)
    hexes, cohs, hply, cply = [], [], [], []
    for l, c in enumerate(coh_layer):
        e = np.stack([nid(ie, je, l), nid(ie + 1, je, l), nid(ie + 1, je + 1, l), nid(ie, je + 1, l),
                      nid(ie, je, l + 1), nid(ie + 1, je, l + 1), nid(ie + 1, je + 1, l + 1),
                      nid(ie, je + 1, l + 1)], axis=1)
        (cohs if c else hexes).append(e)
        (cply if c else hply).append(np.full(len(e), ply[l]))
    cat = lambda a: np.concatenate(a).astype(np.int32) if a else np.zeros((0, 8), np.int32)
    return (coords, cat(hexes), cat(cohs),
            np.concatenate(hply).astype(np.int32) if hply else np.zeros(0, np.int32),
            np.concatenate(cply).astype(np.int32) if cply else np.zeros(0, np.int32))


def renumbered(coords, hexes, cohs, seed: int, distort: float = 0.0):
    """A seeded random renumbering of the nodes and a shuffle of the element
    order of an explicit mesh, with the in-plane node positions moved by up
    to `distort` times the smallest in-plane spacing (the same move for the
    coincident nodes of an interface, so it keeps zero thickness)."""
    g = rng(seed)
    perm = g.permutation(len(coords))              # old node -> new node
    out = np.zeros_like(coords)
    out[perm] = coords
    if distort > 0:
        xs = np.unique(np.round(coords[:, 0], 12))
        ys = np.unique(np.round(coords[:, 1], 12))
        h = min(np.diff(xs).min(), np.diff(ys).min())
        key = np.round(coords[:, :2] / (1e-9 * h)).astype(np.int64)
        _, col = np.unique(key, axis=0, return_inverse=True)
        mv = g.uniform(-distort * h, distort * h, size=(col.max() + 1, 2))
        out[perm, 0] += mv[col.reshape(-1), 0]
        out[perm, 1] += mv[col.reshape(-1), 1]
    he = perm[hexes][g.permutation(len(hexes))] if len(hexes) else hexes
    ce = perm[cohs][g.permutation(len(cohs))] if len(cohs) else cohs
    return out, he.astype(np.int32), ce.astype(np.int32)


# ---------------------------------------------------------------------------
# synthetic states (seeded) for one-step parity at any size
# ---------------------------------------------------------------------------

def synthetic_state(n_nodes: int, n_gp: int, n_coh_pairs: int, seed: int,
                    disp_amp: float, vel_amp: float, r_max: float = 1.0,
                    rd_max: float = 0.0) -> dict:
    """Random nodal displacement/velocity and damage thresholds.

    disp:  3*n_nodes, uniform in [-disp_amp, disp_amp]
    vel:   3*n_nodes, uniform in [-vel_amp, vel_amp]
    r:     4*n_gp thresholds (r1+, r1-, r2+, r2-), 1 + U[0, r_max - 1]
    rd:    n_coh_pairs cohesive thresholds, U[0, rd_max]
    """
    g = rng(seed)
    d = g.uniform(-disp_amp, disp_amp, 3 * n_nodes)
    v = g.uniform(-vel_amp, vel_amp, 3 * n_nodes)
    r = 1.0 + g.uniform(0.0, max(r_max - 1.0, 0.0), 4 * n_gp)
    rd = g.uniform(0.0, rd_max, n_coh_pairs)
    return dict(disp=d, vel=v, r=r, rd=rd)


# ---------------------------------------------------------------------------
# strain paths for the constitutive surrogate's training set
# ---------------------------------------------------------------------------

SUR_SEED = 0x5EED5EED
SUR_INCREMENTS = 32
SUR_MAX_ONSET = 3.0


def sur_path(p: int, n_inc: int = SUR_INCREMENTS, seed: int = SUR_SEED) -> np.ndarray:
    """Strain path p in onset-scaled strain space, shape (n_inc, 6).

    SplitMix64(seed + p) draws, in this order: a direction u (six uniforms on
    [-1, 1), normalised); then for even p (monotone) an amplitude A ~ U[0, 3)
    and the path is A (i / n_inc) u, i = 1..n_inc; for odd p (cyclic) a count
    of reversals nr = 2 + floor(3 U) (2..4) and nr + 1 turning amplitudes a_j =
    (-1)^(j+1) 3 U, j = 1..nr+1, visited from 0 in order along u with
    n_inc // (nr + 1) increments per leg (the remainder added to the last).
    Every operation is one correctly rounded double operation, so other
    implementations of the recipe reproduce it bit for bit."""
    g = SplitMix64(seed + p)
    u = [2.0 * g.uniform() - 1.0 for _ in range(6)]
    nrm = math.sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + u[3] * u[3] + u[4] * u[4] + u[5] * u[5])
    u = [1.0, 0.0, 0.0, 0.0, 0.0, 0.0] if nrm == 0.0 else [c / nrm for c in u]
    amp = []
    if p % 2 == 0:
        A = SUR_MAX_ONSET * g.uniform()
        for i in range(1, n_inc + 1):
            amp.append(A * (i / n_inc))
    else:
        nr = 2 + int(3.0 * g.uniform())
        legs = nr + 1
        a = [0.0] + [(1.0 if j % 2 == 1 else -1.0) * (SUR_MAX_ONSET * g.uniform()) for j in range(1, legs + 1)]
        per = n_inc // legs
        for j in range(1, legs + 1):
            nj = per + (n_inc - per * legs if j == legs else 0)
            for i in range(1, nj + 1):
                amp.append(a[j - 1] + (a[j] - a[j - 1]) * (i / nj))
    return np.array([[s * c for c in u] for s in amp], dtype=np.float64)


def sur_scales(mat: dict) -> tuple:
    """(E_k, X_k) of the surrogate's normalisation: strain eps_k * E_k / X_k,
    stress sigma_k / X_k, components 11, 22, 33, 23, 13, 12."""
    E = (mat["E1"], mat["E2"], mat["E2"], mat["G23"], mat["G12"], mat["G12"])
    X = (mat["XT"], mat["YT"], mat["YT"], mat["SL"], mat["SL"], mat["SL"])
    return E, X
