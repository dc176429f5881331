"""Helpers shared by the GPU parity tests: run the oracle and the HIP path on
the same workload and compare what both expose."""
import copy

import numpy as np

import oracle
import paper_2301_05552_amd as pdn
import workloads as W


def interface_bottom_planes(mesh):
    """Node plane below each cohesive interface (layer index = bottom plane)."""
    planes, layer = [], 0
    ang = mesh["ply_angle_deg"]
    for p in range(mesh["n_plies"]):
        layer += mesh["elems_per_ply"]
        if p + 1 < mesh["n_plies"] and mesh["cohesive"] and ang[p] != ang[p + 1]:
            planes.append(layer)
            layer += 1
    return planes


def coh_pairs_from_oracle(o, mesh):
    """Oracle per-IP cohesive thresholds laid out per node pair."""
    by_node = o.get(oracle.COH_R_BY_BOTTOM_NODE)
    plane = (mesh["nx"] + 1) * (mesh["ny"] + 1)
    return np.concatenate([by_node[k * plane:(k + 1) * plane] for k in interface_bottom_planes(mesh)]) \
        if interface_bottom_planes(mesh) else np.zeros(0)


def rel(a, b, floor=0.0):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    if a.size == 0:
        return 0.0
    den = max(np.abs(b).max(), floor, 1e-300)
    return float(np.abs(a - b).max() / den)


def run_both(cfg, steps, precision=W.PREC_FP64, tile=None, chunks=1, threads=None):
    cfg = copy.deepcopy(cfg)
    cfg["mesh"]["precision"] = precision
    o = oracle.Oracle(cfg) if threads is None else oracle.Oracle(cfg, threads=threads)
    g = pdn.Simulation(cfg, tile=tile)
    o.step(steps)
    left = steps
    for k in range(chunks):
        n = left // (chunks - k)
        g.step(n)
        left -= n
    return o, g


def compare(o, g, cfg):
    """Relative differences of everything both sides expose."""
    out = {}
    out["dt"] = abs(g.info()["dt"] - o.dt) / o.dt
    to, fo, xo = o.history()
    tg, fg, xg = g.contact_force()
    out["hist_len"] = (len(fo), len(fg))
    out["t"] = rel(tg, to)
    out["force"] = rel(fg, fo)
    out["imp_disp"] = rel(xg, xo)
    out["disp"] = rel(g.array_get(pdn.ARR_DISP), o.get(oracle.DISP))
    out["vel"] = rel(g.array_get(pdn.ARR_VEL), o.get(oracle.VEL))
    out["mass"] = rel(g.array_get(pdn.ARR_MASS), o.get(oracle.MASS))
    if o.ne:
        out["gp_r"] = rel(g.array_get(pdn.ARR_GP_R), o.get(oracle.GP_R))
    if o.nc:
        out["coh_r"] = rel(g.array_get(pdn.ARR_COH_R), coh_pairs_from_oracle(o, cfg["mesh"]), floor=1.0)
    eo, eg = o.energies(), g.energies()
    scale = max(eo["ke0"], 1e-300)
    out["energy"] = max(abs(eg[k] - eo[k]) / scale for k in
                        ("ke_plate", "ke_striker", "w_int", "w_grav", "w_contact_plate", "w_striker", "u_el"))
    out["energy_level"] = (eo["level"], eg["level"])
    return out
