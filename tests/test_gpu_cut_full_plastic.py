"""Multi-step parity of the paper's element and law at the element size of the
1200 x 800 x 16 benchmark plate: its 150 x 100-column cut (2 elements per
ply, 6 cohesive interfaces, scaled window supports, 5.5 kg striker at 25 J)
with 2x2x2 Gauss points per bulk element (Section 2) and Table 1's matrix
shear plasticity on every ply (Algorithm 4 from its first line), 1750 steps
through first contact (step 315) into yield and damage under the striker,
in the 15 x 15-tile launch, against the stored FP64 oracle run
(tests/golden/qi8_150x100x16_full_plastic_fp64_oracle.json, written by
tests/golden/make_qi8_150x100x16_golden.py --full-plastic --steps 1750 from
the oracle alone).  The stored run stops where the oracle's two summation
orders still agree to 1e-8 N in force: in the next 250 steps the crushed
elements under the striker (this element has no hourglass control) turn
rounding into velocity differences of metres per second at single nodes.

FP64 mode: the contact-force and striker histories, the energy books and the
displacement, velocity, every Gauss point's thresholds and plastic state of
the sampled elements and the interface thresholds within 1e-10 of each
quantity's scale, or within 30 times what the oracle differs from itself when
its nodal sums run in the opposite element order (stored with the run).

Mixed precision (FP32 element arithmetic and Gauss-point state): through the
first 1250 steps the force history agrees with the FP64 run to 1e-6 of the
peak.  After that the elements under the striker soften (thresholds up to
seven times onset) and this window amplifies rounding about 1e5-fold: the
oracle's own two summation orders part by 2e-9 N (8e-12 of the peak) by step
1750, and FP32's rounding (6e-8) grows the same way to about 1 % of the peak
force.  So the stated 0.5 % bar for mixed precision does not hold here once
the crushed region softens; the test holds the early window to 1e-5 of the
peak and the whole window to 2 %, and prints what it measures.  FP64 mode is
the reference for this element and law in such windows.
"""
import json
import os
import sys

import numpy as np
import pytest

import paper_2301_05552_amd as pdn
import workloads as W

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "qi8_150x100x16_full_plastic_fp64_oracle.json")
TOL64 = 1e-10


def _note(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as fh:
        g = json.load(fh)
    assert g["integration"] == 8 and g["plastic"]
    return g


def _cfg(prec):
    cfg = W.plate_qi8_150x100x16_cut(prec)
    cfg["mesh"]["integration"] = 8
    for m in cfg["materials"]:
        m["Sp"], m["Kp"] = W.AS4_SP, W.AS4_KP
    return cfg


def _run(prec, steps):
    g = pdn.Simulation(_cfg(prec), tile=(15, 15))
    for _ in range(steps // 250):
        g.step(250)
    g.step(steps % 250)
    return g


def test_cut_full_plastic_fp64(gold):
    _note("cut 150x100x16+6, 2x2x2 points and plasticity, fp64 1750 steps, tile 15x15")
    g = _run(W.PREC_FP64, gold["steps"])
    try:
        info = g.info()
        sens = gold["reversed_assembly_deviation"]
        err, bar = {}, {}
        t, f, x = g.contact_force()
        fo, xo = np.array(gold["history"]["force"]), np.array(gold["history"]["imp_disp"])
        assert len(f) == len(fo) == gold["steps"]
        assert fo.max() > 10.0                                # the striker is in contact
        fmax = np.abs(fo).max()
        nb = sens["force_block_steps"]
        for b, dev in enumerate(sens["force_abs_by_block"]):
            err[f"force_block{b}"] = float(np.abs(f[b * nb:(b + 1) * nb] - fo[b * nb:(b + 1) * nb]).max())
            bar[f"force_block{b}"] = max(TOL64 * fmax, 30 * dev)
        err["dt"], bar["dt"] = abs(info["dt"] - gold["dt"]), TOL64 * gold["dt"]
        err["imp_disp"] = float(np.abs(x - xo).max())
        bar["imp_disp"] = max(TOL64 * np.abs(xo).max(), 30 * sens["imp_disp_abs_max"])
        n = np.array(gold["nodes"])
        d = g.array_get(pdn.ARR_DISP).reshape(-1, 3)[n]
        v = g.array_get(pdn.ARR_VEL).reshape(-1, 3)[n]
        err["disp"] = float(np.abs(d - np.array(gold["disp"])).max())
        bar["disp"] = max(TOL64 * gold["disp_absmax"], 30 * sens["disp_abs_max"])
        err["vel"] = float(np.abs(v - np.array(gold["vel"])).max())
        bar["vel"] = max(10 * TOL64 * gold["vel_absmax"], 30 * sens["vel_abs_max"])
        e_idx = np.array(gold["gps"])                         # sampled elements, all eight points each
        r = g.array_get(pdn.ARR_GP_R).reshape(-1, 32)
        err["r"] = float(np.abs(r[e_idx] - np.array(gold["r"])).max())
        bar["r"] = max(TOL64 * gold["r_max"], 30 * sens["r_abs_max"])
        ep = g.array_get(pdn.ARR_GP_EP).reshape(-1, 24)
        err["ep"] = float(np.abs(ep[e_idx] - np.array(gold["ep"])).max())
        bar["ep"] = max(TOL64 * max(gold["ep_max"], 1e-12), 30 * sens["ep_abs_max"])
        rd = g.array_get(pdn.ARR_COH_R)
        err["rd"] = float(np.abs(rd[np.array(gold["pairs"])] - np.array(gold["rd"])).max())
        bar["rd"] = max(TOL64, 30 * sens["rd_abs_max"])
        e, eo = g.energies(), gold["energies"]
        for k in ("ke_plate", "ke_striker", "w_int", "w_grav", "w_contact_plate", "w_striker", "u_el"):
            err[f"energy_{k}"], bar[f"energy_{k}"] = abs(e[k] - eo[k]), TOL64 * eo["ke0"]
        print("[cut full+plastic fp64] error / bar: " + ", ".join(f"{k} {err[k]:.2e}/{bar[k]:.2e}" for k in err),
              flush=True)
        print(f"[cut full+plastic fp64] peak force {fo.max():.2f} N, largest plastic strain {gold['ep_max']:.3e}, "
              f"largest threshold {gold['r_max']:.4f}", flush=True)
        for k in err:
            assert err[k] <= bar[k], (k, err[k], bar[k])
        assert abs(e["residual"]) <= 1e-6 * e["ke0"]
        assert info["active"] == gold["stats"]["active"]
    finally:
        g.close()


EARLY = 1250                          # steps before the softening under the striker


def test_cut_full_plastic_mixed(gold):
    _note("cut 150x100x16+6, 2x2x2 points and plasticity, mixed 1750 steps, tile 15x15")
    g = _run(W.PREC_MIXED, gold["steps"])
    try:
        _, f, x = g.contact_force()
        fo, xo = np.array(gold["history"]["force"]), np.array(gold["history"]["imp_disp"])
        early = np.abs(f[:EARLY] - fo[:EARLY]).max() / fo.max()
        ep = float(np.abs(g.array_get(pdn.ARR_GP_EP)).max())
        r = float(g.array_get(pdn.ARR_GP_R).max())
        print(f"[cut full+plastic mixed] first {EARLY} steps: force {early:.2e} of the peak; whole window: peak "
              f"force {f.max():.3f} N (oracle {fo.max():.3f} N, {(f.max() - fo.max()) / fo.max():+.2%}), striker "
              f"{x[-1]:.6e} m (oracle {xo[-1]:.6e} m), largest plastic strain {ep:.3e} (oracle "
              f"{gold['ep_max']:.3e}), largest threshold {r:.3f} (oracle {gold['r_max']:.3f})", flush=True)
        assert early <= 1e-5
        assert abs(f.max() - fo.max()) <= 2e-2 * fo.max()
        assert abs(x[-1] - xo[-1]) <= 5e-3 * abs(xo[-1])
        assert ep > 0 and gold["ep_max"] > 0                  # points have yielded in both
        e = g.energies()
        assert abs(e["residual"]) <= 1e-6 * e["ke0"]
    finally:
        g.close()
