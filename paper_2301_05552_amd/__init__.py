"""MI355X explicit PDN impact step: thin ctypes binding of libpdn.so.

Each method marshals arguments for the C call of the same name in
include/pdn.h; every step of the method runs in the library's HIP kernels.
Loading fails loudly when the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdn.so")
_lib = None

PDN_OK, PDN_EINVAL, PDN_ENOMEM, PDN_EDEVICE, PDN_ESTATE, PDN_EUNSTABLE, PDN_ERANGE = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
BC_CLAMPED_EDGES, BC_ASTM_WINDOW, BC_FREE = 0, 1, 2
LAW_ELASTIC, LAW_CDM, LAW_CDM_SURROGATE = 0, 1, 2
DMG_FIBRE, DMG_MATRIX, DMG_SHEAR, DMG_COHESIVE, DMG_PROJ_FIBRE, DMG_PROJ_MATRIX, DMG_PROJ_COHESIVE = range(7)
ARR_DISP, ARR_VEL, ARR_GP_R, ARR_COH_R, ARR_MASS, ARR_GP_EP = range(6)

EXPORTS = ["pdn_mesh_create", "pdn_material_set", "pdn_impactor_set", "pdn_step", "pdn_contact_force",
           "pdn_damage_field", "pdn_energies", "pdn_info_get", "pdn_array_get", "pdn_array_set",
           "pdn_state_save", "pdn_state_load", "pdn_set_tile", "pdn_kernel_times", "pdn_set_timing",
           "pdn_last_error", "pdn_destroy"]


class PdnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pdn error {code}: {msg}")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("n_plies", C.c_int32), ("elems_per_ply", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("ply_thickness", C.c_double),
                ("ply_angle_deg", C.POINTER(C.c_double)), ("cohesive", C.c_int32), ("bc", C.c_int32),
                ("window_lx", C.c_double), ("window_ly", C.c_double), ("clamp_radius", C.c_double),
                ("precision", C.c_int32), ("phi", C.c_double), ("cfl_safety", C.c_double),
                ("gravity", C.c_double), ("hourglass_kappa", C.c_double),
                ("x_coords", C.POINTER(C.c_double)), ("y_coords", C.POINTER(C.c_double)),
                ("device", C.c_int32), ("stream", C.c_void_p), ("integration", C.c_int32)]


_MAT = ["E1", "E2", "E3", "nu12", "nu13", "nu23", "G12", "G13", "G23", "rho", "law",
        "XT", "XC", "YT", "YC", "SL", "alpha0_deg", "GXT", "GXC", "GYT", "GYC", "GSL",
        "fXT", "fGT", "fXC", "fGC", "KI", "tauI", "tauII", "GIc", "GIIc", "eta_bk", "Sp", "Kp"]


class Material(C.Structure):
    _fields_ = [(f, C.c_int32 if f == "law" else C.c_double) for f in _MAT]


class Impactor(C.Structure):
    _fields_ = [(f, C.c_double) for f in ("radius", "mass", "v0", "energy", "gap", "x0", "y0")]


class Energy(C.Structure):
    _fields_ = [(f, C.c_double) for f in ("level", "ke_plate", "ke_striker", "w_int", "w_grav",
                                          "w_contact_plate", "w_striker", "d_pdn", "ke0", "u_el", "residual")]


class MmuCounts(C.Structure):
    _fields_ = [(f, C.c_int64) for f in ("n_nodes", "n_bulk", "n_interface", "n_edges", "n_faces",
                                          "n_boundary0", "n_boundary_interface0")]


class Info(C.Structure):
    _fields_ = [("dt", C.c_double)] + [(f, C.c_int64) for f in (
        "n_nodes", "n_bulk", "n_cohesive", "n_pairs", "n_planes", "n_layers", "n_candidates",
        "steps", "reset_passes", "released", "active", "max_passes")] + [
        ("fallback_fraction", C.c_double), ("precision", C.c_int32), ("tile_x", C.c_int32),
        ("tile_y", C.c_int32), ("blocks", C.c_int32), ("sur_consulted", C.c_double),
        ("sur_network_steps", C.c_int64)]


def lib():
    """Load libpdn.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libpdn.so not built at {LIB_PATH}: run `python -m paper_2301_05552_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, vp, dp, i64 = C.POINTER, C.c_void_p, C.POINTER(C.c_double), C.c_int64
        sig = {
            "pdn_mesh_create": [P(MeshDesc), P(vp)],
            "pdn_material_set": [vp, C.c_int32, P(Material)],
            "pdn_impactor_set": [vp, P(Impactor)],
            "pdn_step": [vp, i64],
            "pdn_contact_force": [vp, dp, dp, dp, i64, P(i64)],
            "pdn_damage_field": [vp, C.c_int32, dp, i64, P(i64)],
            "pdn_energies": [vp, P(Energy)],
            "pdn_info_get": [vp, P(Info)],
            "pdn_array_get": [vp, C.c_int32, dp, i64, P(i64)],
            "pdn_array_set": [vp, C.c_int32, dp, i64],
            "pdn_state_save": [vp, vp, i64, P(i64)],
            "pdn_state_load": [vp, vp, i64],
            "pdn_set_tile": [vp, C.c_int32, C.c_int32],
            "pdn_kernel_times": [vp, dp, dp],
            "pdn_set_timing": [vp, C.c_int32],
            "pdn_last_error": [vp],
            "pdn_destroy": [vp],
            "pdn_autotune": [vp, P(C.c_int32), P(C.c_int32)],
            "pdn_batch_create": [P(vp), C.c_int32, P(vp)],
            "pdn_batch_step": [vp, i64],
            "pdn_batch_info": [vp, P(C.c_int32), P(C.c_int32), P(i64), P(C.c_int32)],
            "pdn_batch_last_error": [vp],
            "pdn_batch_destroy": [vp],
            "pdn_surrogate_train": [P(SurTrain), P(Material), C.c_double, P(C.c_float), P(SurReport)],
            "pdn_surrogate_set": [vp, C.c_int32, P(C.c_float), i64, C.c_double, C.c_double],
            "pdn_surrogate_eval": [C.c_int32, vp, P(C.c_float), P(C.c_float), i64, P(C.c_float)],
            "pdn_surrogate_grad": [C.c_int32, vp, P(C.c_float), P(C.c_float), P(C.c_float), i64, P(C.c_float),
                                   P(C.c_double)],
            "pdn_surrogate_data": [C.c_int32, vp, P(Material), C.c_double, C.c_uint64, i64, i64, C.c_int32,
                                   P(C.c_float)],
            "pdn_surrogate_grad_noalloc": [C.c_int32, vp, vp, vp, vp, i64, vp, vp],
            "pdn_surrogate_kernel": [vp, C.c_int32],
            "pdn_surrogate_grad_fp32": [C.c_int32, vp, P(C.c_float), P(C.c_float), P(C.c_float), i64,
                                        P(C.c_float), P(C.c_double)],
            "pdn_stream_copy": [C.c_int32, vp, vp, vp, i64],
            "pdn_mesh_multiply": [C.c_int32, vp, P(C.c_double), i64, P(C.c_int32), i64, P(C.c_int32), i64,
                                  P(C.c_int32), P(C.c_int32), C.c_int32, P(C.c_double), P(C.c_int32),
                                  P(C.c_int32), P(C.c_int32), P(C.c_int32), i64, i64, i64, P(MmuCounts)],
            "pdn_global_last_error": [],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.pdn_last_error.restype = C.c_char_p
        L.pdn_destroy.restype = None
        L.pdn_batch_last_error.restype = C.c_char_p
        L.pdn_batch_destroy.restype = None
        L.pdn_global_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


SUR_NPARAM = 9674
SUR_GRAD_NOALLOC_MAX = 16384      # points; pdn_surrogate_grad_noalloc's fixed scratch
SUR_SEED = 0x5EED5EED


class SurTrain(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("n_paths", C.c_int64), ("increments", C.c_int32),
                ("seed", C.c_uint64), ("val_fraction", C.c_double), ("steps", C.c_int64), ("batch", C.c_int32),
                ("lr", C.c_double), ("lr_final", C.c_double), ("init_seed", C.c_uint64)]


class SurReport(C.Structure):
    _fields_ = [("loss_val_initial", C.c_double), ("loss_val", C.c_double), ("loss_train", C.c_double),
                ("data_seconds", C.c_double), ("train_seconds", C.c_double), ("samples_train", C.c_int64),
                ("samples_val", C.c_int64)]


def _gchk(rc):
    if rc != 0:
        raise PdnError(rc, lib().pdn_global_last_error().decode())


def _material(m: dict) -> Material:
    return Material(**{f: (int(m[f]) if f == "law" else float(m.get(f, 0.0) if f in ("Sp", "Kp") else m[f]))
                       for f, _ in Material._fields_})


def surrogate_train(mat: dict, crack_band: float, *, n_paths=10_000_000, increments=32, seed=SUR_SEED,
                    val_fraction=0.1, steps=4000, batch=65536, lr=2e-3, lr_final=2e-5, init_seed=1,
                    device=0, stream=None):
    """Generate the data set from the exact law on the device and train the
    surrogate there (pdn_surrogate_train).  Returns (weights, report)."""
    o = SurTrain(device=device, stream=stream, n_paths=n_paths, increments=increments, seed=seed,
                 val_fraction=val_fraction, steps=steps, batch=batch, lr=lr, lr_final=lr_final,
                 init_seed=init_seed)
    w = np.zeros(SUR_NPARAM, dtype=np.float32)
    rep = SurReport()
    _gchk(lib().pdn_surrogate_train(C.byref(o), C.byref(_material(mat)), crack_band, _fp(w), C.byref(rep)))
    return w, {f: getattr(rep, f) for f, _ in SurReport._fields_}


def surrogate_eval(w, x, device=0, stream=None):
    w = np.ascontiguousarray(w, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 10)
    y = np.zeros_like(x)
    _gchk(lib().pdn_surrogate_eval(device, stream, _fp(w), _fp(x), x.shape[0], _fp(y)))
    return y


def surrogate_grad(w, x, t, device=0, stream=None):
    w = np.ascontiguousarray(w, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 10)
    t = np.ascontiguousarray(t, dtype=np.float32).reshape(-1, 10)
    g = np.zeros(SUR_NPARAM, dtype=np.float32)
    loss = C.c_double()
    _gchk(lib().pdn_surrogate_grad(device, stream, _fp(w), _fp(x), _fp(t), x.shape[0], _fp(g), C.byref(loss)))
    return g, loss.value


def surrogate_grad_fp32(w, x, t, device=0, stream=None):
    """pdn_surrogate_grad_fp32: FP32 loss and gradient (host arrays)."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 10)
    t = np.ascontiguousarray(t, dtype=np.float32).reshape(-1, 10)
    g = np.zeros(SUR_NPARAM, dtype=np.float32)
    loss = C.c_double()
    _gchk(lib().pdn_surrogate_grad_fp32(device, stream, _fp(w), _fp(x), _fp(t), x.shape[0], _fp(g),
                                        C.byref(loss)))
    return g, loss.value


def surrogate_grad_noalloc(w_ptr: int, x_ptr: int, t_ptr: int, n: int, grad_ptr: int, loss_ptr: int | None,
                           device=0, stream=None):
    """pdn_surrogate_grad_noalloc on device pointers (e.g. tensor.data_ptr());
    only enqueues the work on the stream."""
    _gchk(lib().pdn_surrogate_grad_noalloc(device, stream, w_ptr, x_ptr, t_ptr, n, grad_ptr, loss_ptr))


def stream_copy(src_ptr: int, dst_ptr: int, nbytes: int, device=0, stream=None):
    """pdn_stream_copy on device pointers (enqueued on the stream)."""
    rc = lib().pdn_stream_copy(device, stream, src_ptr, dst_ptr, nbytes)
    if rc != 0:
        raise PdnError(rc, "pdn_stream_copy: bad size, alignment or device")


def _ip(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int32))


def mesh_multiply(coords, hexes, cohs, ndivi: int, hex_tag=None, coh_tag=None, device=0, stream=None,
                  counts=None):
    """pdn_mesh_multiply: ndivi division levels on the device.  Returns
    (coords, hexes, cohs, hex_tag, coh_tag, counts).  `counts` (the dict a
    previous call on the same mesh and ndivi returned) sizes the outputs and
    saves the sizing call."""
    X = np.ascontiguousarray(coords, dtype=np.float64).reshape(-1, 3)
    H = np.ascontiguousarray(hexes, dtype=np.int32).reshape(-1, 8)
    Cc = np.ascontiguousarray(cohs, dtype=np.int32).reshape(-1, 8)
    ht = None if hex_tag is None else np.ascontiguousarray(hex_tag, dtype=np.int32)
    ct = None if coh_tag is None else np.ascontiguousarray(coh_tag, dtype=np.int32)
    cnt = MmuCounts()
    args = (device, stream, _dp(X), len(X), _ip(H), len(H), _ip(Cc), len(Cc), _ip(ht), _ip(ct), ndivi)
    if counts is None:
        rc = lib().pdn_mesh_multiply(*args, None, None, None, None, None, 0, 0, 0, C.byref(cnt))
        if rc != -6:
            _gchk(rc)
    else:
        for f, _ in MmuCounts._fields_:
            setattr(cnt, f, int(counts[f]))
    Xo = np.zeros((cnt.n_nodes, 3))
    Ho = np.zeros((cnt.n_bulk, 8), np.int32)
    Co = np.zeros((cnt.n_interface, 8), np.int32)
    hto = None if ht is None else np.zeros(cnt.n_bulk, np.int32)
    cto = None if ct is None else np.zeros(cnt.n_interface, np.int32)
    _gchk(lib().pdn_mesh_multiply(*args, _dp(Xo), _ip(Ho), _ip(Co), _ip(hto), _ip(cto), len(Xo), len(Ho), len(Co),
                                  C.byref(cnt)))
    return Xo, Ho, Co, hto, cto, {f: getattr(cnt, f) for f, _ in MmuCounts._fields_}


def surrogate_data(mat: dict, crack_band: float, p0: int, n_paths: int, increments=32, seed=SUR_SEED,
                   device=0, stream=None):
    out = np.zeros((n_paths * increments, 20), dtype=np.float32)
    _gchk(lib().pdn_surrogate_data(device, stream, C.byref(_material(mat)), crack_band, seed, p0, n_paths,
                                   increments, _fp(out)))
    return out


class Simulation:
    """One impact simulation on one device (see include/pdn.h)."""

    def __init__(self, cfg: dict, device: int = 0, stream=None, x_coords=None, y_coords=None,
                 precision: int | None = None, tile: tuple | None = None):
        L = lib()
        m = cfg["mesh"]
        self._ang = np.ascontiguousarray(m["ply_angle_deg"], dtype=np.float64)
        self._xc = None if x_coords is None else np.ascontiguousarray(x_coords, dtype=np.float64)
        self._yc = None if y_coords is None else np.ascontiguousarray(y_coords, dtype=np.float64)
        prec = m["precision"] if precision is None else precision
        d = MeshDesc(nx=m["nx"], ny=m["ny"], n_plies=m["n_plies"], elems_per_ply=m["elems_per_ply"],
                     lx=m["lx"], ly=m["ly"], ply_thickness=m["ply_thickness"], ply_angle_deg=_dp(self._ang),
                     cohesive=m["cohesive"], bc=m["bc"], window_lx=m["window_lx"], window_ly=m["window_ly"],
                     clamp_radius=m["clamp_radius"], precision=prec, phi=m["phi"],
                     cfl_safety=m["cfl_safety"], gravity=m["gravity"], hourglass_kappa=m["hourglass_kappa"],
                     x_coords=None if self._xc is None else _dp(self._xc),
                     y_coords=None if self._yc is None else _dp(self._yc),
                     device=device, stream=stream, integration=int(m.get("integration", 1)))
        h = C.c_void_p()
        rc = L.pdn_mesh_create(C.byref(d), C.byref(h))
        if rc != 0:
            raise PdnError(rc, "pdn_mesh_create failed")
        self.h = h
        self.cfg = cfg
        if tile is not None:
            self.set_tile(*tile)
        mats = cfg["materials"]
        if len(mats) == 1:
            self.material_set(-1, mats[0])
        else:
            for p, mt in enumerate(mats):
                self.material_set(p, mt)
        if cfg.get("impactor") is not None:
            self.impactor_set(cfg["impactor"])

    def _chk(self, rc):
        if rc != 0:
            raise PdnError(rc, lib().pdn_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().pdn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- the six boundary calls ------------------------------------------------
    def material_set(self, ply: int, mat: dict):
        m = Material(**{f: (int(mat[f]) if f == "law" else float(mat[f])) for f in _MAT})
        self._chk(lib().pdn_material_set(self.h, ply, C.byref(m)))

    def impactor_set(self, imp: dict):
        x0 = imp.get("x0", float("nan"))
        y0 = imp.get("y0", float("nan"))
        s = Impactor(radius=imp["radius"], mass=imp["mass"], v0=imp.get("v0", 0.0),
                     energy=imp.get("energy", 0.0), gap=imp.get("gap", 1e-5),
                     x0=float("nan") if x0 is None else x0, y0=float("nan") if y0 is None else y0)
        self._chk(lib().pdn_impactor_set(self.h, C.byref(s)))

    def step(self, n: int = 1):
        return self._chk(lib().pdn_step(self.h, int(n)))

    def contact_force(self):
        n = C.c_int64()
        lib().pdn_contact_force(self.h, None, None, None, 0, C.byref(n))
        k = max(n.value, 1)
        t, f, x = np.zeros(k), np.zeros(k), np.zeros(k)
        self._chk(lib().pdn_contact_force(self.h, _dp(t), _dp(f), _dp(x), k, C.byref(n)))
        return t[:n.value], f[:n.value], x[:n.value]

    def damage_field(self, kind: int):
        n = C.c_int64()
        lib().pdn_damage_field(self.h, kind, None, 0, C.byref(n))
        out = np.zeros(max(n.value, 1))
        self._chk(lib().pdn_damage_field(self.h, kind, _dp(out), out.size, C.byref(n)))
        return out[:n.value]

    # ---- extensions --------------------------------------------------------------
    def energies(self) -> dict:
        e = Energy()
        self._chk(lib().pdn_energies(self.h, C.byref(e)))
        return {f: getattr(e, f) for f, _ in Energy._fields_}

    def info(self) -> dict:
        i = Info()
        self._chk(lib().pdn_info_get(self.h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in Info._fields_}

    def array_get(self, kind: int) -> np.ndarray:
        n = C.c_int64()
        lib().pdn_array_get(self.h, kind, None, 0, C.byref(n))
        out = np.zeros(max(n.value, 1))
        self._chk(lib().pdn_array_get(self.h, kind, _dp(out), out.size, C.byref(n)))
        return out[:n.value]

    def array_set(self, kind: int, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        self._chk(lib().pdn_array_set(self.h, kind, _dp(a), a.size))

    def state_save(self) -> bytes:
        n = C.c_int64()
        lib().pdn_state_save(self.h, None, 0, C.byref(n))
        buf = C.create_string_buffer(max(n.value, 1))
        self._chk(lib().pdn_state_save(self.h, buf, n.value, C.byref(n)))
        return buf.raw[:n.value]

    def state_load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._chk(lib().pdn_state_load(self.h, buf, len(blob)))

    def set_tile(self, tx: int, ty: int):
        self._chk(lib().pdn_set_tile(self.h, tx, ty))

    def set_timing(self, on: bool):
        self._chk(lib().pdn_set_timing(self.h, 1 if on else 0))

    def kernel_times(self):
        a, b = C.c_double(), C.c_double()
        self._chk(lib().pdn_kernel_times(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def surrogate_set(self, ply: int, w, dmg_thresh: float = 0.05, res_thresh: float = 1e-3):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._chk(lib().pdn_surrogate_set(self.h, ply, _fp(w), w.size, dmg_thresh, res_thresh))

    def surrogate_kernel(self, mode: int):
        """pdn_surrogate_kernel.  0: choose per step call between the plain
        build and the network build at 1 wave/SIMD; 1: always the network
        build held to 2 waves/SIMD; 2: always the 1-wave network build."""
        self._chk(lib().pdn_surrogate_kernel(self.h, mode))

    def autotune(self):
        tx, ty = C.c_int32(), C.c_int32()
        self._chk(lib().pdn_autotune(self.h, C.byref(tx), C.byref(ty)))
        return tx.value, ty.value


class Batch:
    """Independent cases advanced together (pdn_batch_*): one launch of each
    kernel per step serves every case.  The Simulations stay owned by the
    caller and must outlive the batch."""

    def __init__(self, sims):
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*[s.h for s in self.sims])
        h = C.c_void_p()
        rc = lib().pdn_batch_create(arr, len(self.sims), C.byref(h))
        if rc != 0:
            raise PdnError(rc, lib().pdn_last_error(self.sims[0].h).decode())
        self.h = h

    def _chk(self, rc):
        if rc != 0:
            raise PdnError(rc, lib().pdn_batch_last_error(self.h).decode())

    def step(self, n: int = 1):
        self._chk(lib().pdn_batch_step(self.h, n))

    def info(self) -> dict:
        tx, ty, nb, bl = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int32()
        self._chk(lib().pdn_batch_info(self.h, C.byref(tx), C.byref(ty), C.byref(nb), C.byref(bl)))
        return {"tile": (tx.value, ty.value), "n_bulk": nb.value, "blocks": bl.value}

    def close(self):
        if getattr(self, "h", None):
            lib().pdn_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
