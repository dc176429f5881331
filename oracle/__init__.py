"""Plain FP64 CPU oracle of the explicit PDN impact step.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here is imported by the HIP
library or its binding, and nothing here reads their output.

``build()`` compiles ``pdn_oracle.c`` with gcc (``-ffp-contract=off``, OpenMP
for the element loop when timed on several cores) into ``liborc.so`` next to
this file.  ``Oracle`` wraps one simulation built from a workload dict of the
``workloads`` module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdn_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None

DISP, VEL, GP_R, COH_R_IP, COH_R_BY_BOTTOM_NODE, MASS, COORDS, FINT, ACTIVE, FIX, FCONTACT, GP_EP = range(12)
DMG_FIBRE, DMG_MATRIX, DMG_SHEAR, DMG_COHESIVE, DMG_PROJ_FIBRE, DMG_PROJ_MATRIX, \
    DMG_PROJ_COHESIVE = range(7)


def build(force: bool = True) -> str:
    """Compile the oracle; returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class MeshDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("n_plies", C.c_int32),
                ("elems_per_ply", C.c_int32), ("lx", C.c_double), ("ly", C.c_double),
                ("ply_thickness", C.c_double), ("ply_angle_deg", C.POINTER(C.c_double)),
                ("cohesive", C.c_int32), ("bc", C.c_int32), ("window_lx", C.c_double),
                ("window_ly", C.c_double), ("clamp_radius", C.c_double), ("phi", C.c_double),
                ("cfl_safety", C.c_double), ("gravity", C.c_double),
                ("hourglass_kappa", C.c_double), ("node_coords", C.POINTER(C.c_double)),
                ("integration", C.c_int32)]


_MAT_FIELDS = ["E1", "E2", "E3", "nu12", "nu13", "nu23", "G12", "G13", "G23", "rho", "law",
               "XT", "XC", "YT", "YC", "SL", "alpha0_deg", "GXT", "GXC", "GYT", "GYC", "GSL",
               "fXT", "fGT", "fXC", "fGC", "KI", "tauI", "tauII", "GIc", "GIIc", "eta_bk", "Sp", "Kp"]


class Material(C.Structure):
    _fields_ = [(f, C.c_int32 if f == "law" else C.c_double) for f in _MAT_FIELDS]


class Impactor(C.Structure):
    _fields_ = [(f, C.c_double) for f in ("radius", "mass", "v0", "energy", "gap", "x0", "y0")]


class Energy(C.Structure):
    _fields_ = [(f, C.c_double) for f in (
        "level", "ke_plate", "ke_striker", "w_int", "w_grav", "w_contact_plate", "w_striker",
        "d_pdn", "ke0", "u_el", "residual")]


RHS = C.CFUNCTYPE(None, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER
        dp = P(C.c_double)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [P(MeshDesc)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_error.restype = C.c_char_p
        L.orc_error.argtypes = [C.c_void_p]
        L.orc_mesh_counts.argtypes = [P(MeshDesc), P(C.c_int64)]
        L.orc_set_material.argtypes = [C.c_void_p, C.c_int32, P(Material)]
        L.orc_set_impactor.argtypes = [C.c_void_p, P(Impactor)]
        L.orc_set_threads.argtypes = [C.c_void_p, C.c_int32]
        L.orc_set_assembly_order.argtypes = [C.c_void_p, C.c_int32]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_dt.restype = C.c_double
        L.orc_dt.argtypes = [C.c_void_p]
        L.orc_get.argtypes = [C.c_void_p, C.c_int32, dp, C.c_int64]
        L.orc_set.argtypes = [C.c_void_p, C.c_int32, dp, C.c_int64]
        L.orc_history.restype = C.c_int64
        L.orc_history.argtypes = [C.c_void_p, dp, dp, dp, C.c_int64]
        L.orc_energies.argtypes = [C.c_void_p, P(Energy)]
        L.orc_damage_field.restype = C.c_int64
        L.orc_damage_field.argtypes = [C.c_void_p, C.c_int32, dp, C.c_int64]
        L.orc_stats.argtypes = [C.c_void_p, P(C.c_int64)]
        L.orc_impactor_state.argtypes = [C.c_void_p, dp]
        L.orc_hex8_geometry.argtypes = [dp, dp, dp, dp]
        L.orc_hex8_force_elastic.restype = C.c_double
        L.orc_hex8_force_elastic.argtypes = [dp, dp, P(Material), C.c_double, C.c_double, dp]
        L.orc_hex8_force_elastic_full.restype = C.c_double
        L.orc_hex8_force_elastic_full.argtypes = [dp, dp, P(Material), C.c_double, dp]
        L.orc_hex8_mass.argtypes = [dp, C.c_double, dp]
        L.orc_cdm.argtypes = [P(Material), C.c_double, dp, dp, dp, dp]
        L.orc_cdm_plastic.argtypes = [P(Material), C.c_double, dp, dp, dp, dp, dp]
        L.orc_czm.restype = C.c_double
        L.orc_czm.argtypes = [P(Material), dp, dp, dp]
        L.orc_rk4.argtypes = [RHS, C.c_void_p, C.c_double, dp, C.c_int, C.c_double]
        L.orc_stable_dt.restype = C.c_double
        L.orc_stable_dt.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def material(m: dict) -> Material:
    return Material(**{f: (int(m[f]) if f == "law" else float(m.get(f, 0.0) if f in ("Sp", "Kp") else m[f]))
                       for f in _MAT_FIELDS})


def mesh_desc(mesh: dict, node_coords: np.ndarray | None = None):
    ang = np.ascontiguousarray(mesh["ply_angle_deg"], dtype=np.float64)
    d = MeshDesc(nx=mesh["nx"], ny=mesh["ny"], n_plies=mesh["n_plies"],
                 elems_per_ply=mesh["elems_per_ply"], lx=mesh["lx"], ly=mesh["ly"],
                 ply_thickness=mesh["ply_thickness"], ply_angle_deg=_dp(ang),
                 cohesive=mesh["cohesive"], bc=mesh["bc"], window_lx=mesh["window_lx"],
                 window_ly=mesh["window_ly"], clamp_radius=mesh["clamp_radius"],
                 phi=mesh["phi"], cfl_safety=mesh["cfl_safety"], gravity=mesh["gravity"],
                 hourglass_kappa=mesh["hourglass_kappa"],
                 node_coords=(_dp(node_coords) if node_coords is not None else None),
                 integration=int(mesh.get("integration", 1)))
    return d, (ang, node_coords)


def mesh_counts(mesh: dict) -> dict:
    d, keep = mesh_desc(mesh)
    out = (C.c_int64 * 7)()
    if lib().orc_mesh_counts(C.byref(d), out) != 0:
        raise ValueError("bad mesh description")
    return dict(n_nodes=out[0], n_bulk=out[1], n_cohesive=out[2], n_planes=out[3],
                n_layers=out[4], n_top=out[5])


class OracleError(RuntimeError):
    pass


class Oracle:
    """One oracle simulation of a workload dict (see ``workloads``)."""

    def __init__(self, cfg: dict, node_coords: np.ndarray | None = None, threads: int = 1):
        L = lib()
        self.cfg = cfg
        nc = None if node_coords is None else np.ascontiguousarray(node_coords, dtype=np.float64)
        d, self._keep = mesh_desc(cfg["mesh"], nc)
        self.h = L.orc_create(C.byref(d))
        if not self.h:
            raise OracleError("orc_create failed")
        self.counts = mesh_counts(cfg["mesh"])
        self.nn = self.counts["n_nodes"]
        self.ne = self.counts["n_bulk"]
        self.nc = self.counts["n_cohesive"]
        L.orc_set_threads(self.h, threads)
        mats = cfg["materials"]
        if len(mats) == 1:
            self._chk(L.orc_set_material(self.h, -1, C.byref(material(mats[0]))))
        else:
            for p, m in enumerate(mats):
                self._chk(L.orc_set_material(self.h, p, C.byref(material(m))))
        if cfg.get("impactor") is not None:
            self.set_impactor(cfg["impactor"])

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def _chk(self, rc):
        if rc != 0:
            raise OracleError(lib().orc_error(self.h).decode())

    def set_assembly_order(self, reverse: bool):
        """Sum nodal forces in descending element order (sensitivity runs)."""
        self._chk(lib().orc_set_assembly_order(self.h, int(reverse)))

    def set_impactor(self, imp: dict):
        self._chk(lib().orc_set_impactor(self.h, C.byref(Impactor(**imp))))

    def step(self, n: int):
        self._chk(lib().orc_step(self.h, n))

    @property
    def dt(self) -> float:
        return lib().orc_dt(self.h)

    def get(self, kind: int) -> np.ndarray:
        ngp = 8 if self.cfg["mesh"].get("integration", 1) == 8 else 1
        size = {DISP: 3 * self.nn, VEL: 3 * self.nn, FINT: 3 * self.nn, GP_R: 4 * ngp * self.ne,
                COH_R_IP: 4 * self.nc, COH_R_BY_BOTTOM_NODE: self.nn, MASS: self.nn,
                COORDS: 3 * self.nn, ACTIVE: self.nn, FCONTACT: 3 * self.nn, GP_EP: 3 * ngp * self.ne}[kind]
        out = np.zeros(max(size, 1))
        self._chk(lib().orc_get(self.h, kind, _dp(out), out.size))
        return out[:size]

    def set(self, kind: int, arr: np.ndarray):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        self._chk(lib().orc_set(self.h, kind, _dp(a), a.size))

    def history(self):
        n = lib().orc_history(self.h, None, None, None, 0)
        t, f, x = np.zeros(max(n, 1)), np.zeros(max(n, 1)), np.zeros(max(n, 1))
        lib().orc_history(self.h, _dp(t), _dp(f), _dp(x), n)
        return t[:n], f[:n], x[:n]

    def energies(self) -> dict:
        e = Energy()
        lib().orc_energies(self.h, C.byref(e))
        return {f: getattr(e, f) for f, _ in Energy._fields_}

    def damage_field(self, kind: int) -> np.ndarray:
        n = -lib().orc_damage_field(self.h, kind, None, 0)
        out = np.zeros(max(n, 1))
        lib().orc_damage_field(self.h, kind, _dp(out), n)
        return out[:n]

    def stats(self) -> dict:
        o = (C.c_int64 * 5)()
        lib().orc_stats(self.h, o)
        return dict(steps=o[0], reset_passes=o[1], released=o[2], active=o[3], max_passes=o[4])

    def impactor_state(self) -> dict:
        o = np.zeros(9)
        lib().orc_impactor_state(self.h, _dp(o))
        return dict(centre=o[0:3].copy(), velocity=o[3:6].copy(), force=o[6:9].copy())


# ---- single-routine helpers (pins) ----------------------------------------

def hex8_geometry(X: np.ndarray):
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(24)
    b, V, g = np.zeros(24), np.zeros(1), np.zeros(32)
    lib().orc_hex8_geometry(_dp(X), _dp(b), _dp(V), _dp(g))
    return b.reshape(8, 3), V[0], g.reshape(4, 8)


def hex8_force_elastic_full(X, u, mat: dict, angle_deg=0.0):
    """Element force and strain energy with full 2x2x2 Gauss integration."""
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(24)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(24)
    f = np.zeros(24)
    m = material(mat)
    W = lib().orc_hex8_force_elastic_full(_dp(X), _dp(u), C.byref(m), angle_deg, _dp(f))
    return f.reshape(8, 3), W


def hex8_force_elastic(X, u, mat: dict, angle_deg=0.0, kappa=0.05):
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(24)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(24)
    f = np.zeros(24)
    m = material(mat)
    W = lib().orc_hex8_force_elastic(_dp(X), _dp(u), C.byref(m), angle_deg, kappa, _dp(f))
    return f.reshape(8, 3), W


def hex8_mass(X, rho):
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(24)
    m = np.zeros(8)
    lib().orc_hex8_mass(_dp(X), rho, _dp(m))
    return m


def cdm(mat: dict, lc: float, eps, r):
    """One call of the intralaminar law; returns (sigma, r_new, damage[5])."""
    e = np.ascontiguousarray(eps, dtype=np.float64)
    rr = np.ascontiguousarray(r, dtype=np.float64).copy()
    sig, dmg = np.zeros(6), np.zeros(5)
    lib().orc_cdm(C.byref(material(mat)), lc, _dp(e), _dp(rr), _dp(sig), _dp(dmg))
    return sig, rr, dmg


def cdm_plastic(mat: dict, lc: float, eps, r, ep):
    """The intralaminar law with the plastic state (Algorithm 4 from its first
    line); returns (sigma, r_new, ep_new, damage[5])."""
    e = np.ascontiguousarray(eps, dtype=np.float64)
    rr = np.ascontiguousarray(r, dtype=np.float64).copy()
    pp = np.ascontiguousarray(ep, dtype=np.float64).copy()
    sig, dmg = np.zeros(6), np.zeros(5)
    lib().orc_cdm_plastic(C.byref(material(mat)), lc, _dp(e), _dp(rr), _dp(pp), _dp(sig), _dp(dmg))
    return sig, rr, pp, dmg


def czm(mat: dict, delta, rd: float):
    """One call of the cohesive law; returns (tau[3], rd_new, D)."""
    dl = np.ascontiguousarray(delta, dtype=np.float64)
    r = np.array([rd], dtype=np.float64)
    tau = np.zeros(3)
    D = lib().orc_czm(C.byref(material(mat)), _dp(dl), _dp(r), _dp(tau))
    return tau, r[0], D


def rk4(f, t: float, y: np.ndarray, dt: float) -> np.ndarray:
    """One RK4 step of y' = f(t, y) (f: python callable on numpy arrays)."""
    n = len(y)

    def cb(tt, yp, dyp, ctx):
        yy = np.ctypeslib.as_array(yp, shape=(n,))
        dy = f(tt, yy.copy())
        for i in range(n):
            dyp[i] = float(dy[i])

    cfun = RHS(cb)
    yy = np.ascontiguousarray(y, dtype=np.float64).copy()
    lib().orc_rk4(cfun, None, t, _dp(yy), n, dt)
    return yy
