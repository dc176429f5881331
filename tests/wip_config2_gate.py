"""Accuracy gate of the reduced-precision path over a whole impact.

The 8-ply [0/45/-45/90]s plate (150 x 100 mm, 300 x 200 x 8 hex8,
intralaminar damage, window supports of the drop-weight coupon, 5.5 kg
striker of radius 8 mm at 15 J; Sec. 4, Table 1) is run to 3 ms on the GPU
and compared with the FP64 oracle's run of the same case, stored in
tests/golden/config2_fp64_oracle.json by tests/golden/make_config2_golden.py
(which calls only the oracle and the input generators).

Bars:
  - mixed precision (FP32 element arithmetic and Gauss-point state, FP64
    nodal state, contact and books): the peak contact force within 0.5 % and
    the projected fibre and matrix damage areas (d > 0, d >= 0.5, d >= 0.999)
    within 2 % of the oracle's;
  - FP64: the same quantities much tighter (the two differ only in the order
    of floating-point sums), and the sampled force history point by point.
"""
import json
import os
import sys

import numpy as np
import pytest

import paper_2301_05552_amd as pdn
import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config2_fp64_oracle.json")
THRESHOLDS = ("0", "0.5", "0.999")


def _note(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as fh:
        return json.load(fh)


def _run(prec, g):
    cfg = W.config2(prec)
    sim = pdn.Simulation(cfg)
    try:
        assert sim.info()["dt"] == pytest.approx(g["dt"], rel=1e-12)
        sim.step(g["steps"])
        t, f, x = sim.contact_force()
        m = cfg["mesh"]
        cell = (m["lx"] / m["nx"]) * (m["ly"] / m["ny"])
        areas = {}
        for name, kind in (("fibre", pdn.DMG_PROJ_FIBRE), ("matrix", pdn.DMG_PROJ_MATRIX)):
            d = sim.damage_field(kind)
            areas[name] = {thr: (int((d > 0).sum()) if thr == "0" else int((d >= float(thr)).sum())) * cell
                           for thr in THRESHOLDS}
        return t, f, x, areas
    finally:
        sim.close()


def _check(g, run, f_tol, a_tol):
    t, f, x, areas = run
    assert len(f) == g["steps"]
    i = int(np.argmax(f))
    rel = abs(f[i] - g["peak_force_N"]) / g["peak_force_N"]
    print(f"  peak {f[i]:.3f} N (oracle {g['peak_force_N']:.3f} N), rel err {rel:.3e}", flush=True)
    assert rel <= f_tol
    for name in ("fibre", "matrix"):
        for thr in THRESHOLDS:
            ref = g["projected_damage"][name][thr]["area_m2"]
            got = areas[name][thr]
            err = abs(got - ref) / ref if ref > 0 else abs(got)
            print(f"  {name} area d{'>' if thr == '0' else '>='}{thr}: {got:.4e} m2 (oracle {ref:.4e}), "
                  f"rel err {err:.3e}", flush=True)
            assert err <= a_tol, (name, thr, got, ref)
    return t, f


def test_mixed_precision_gate(gold):
    """Peak force within 0.5 % and damage areas within 2 % of the FP64 oracle."""
    _note("config2 mixed, to 3 ms")
    _check(gold, _run(W.PREC_MIXED, gold), 5e-3, 2e-2)


def test_fp64_tracks_the_oracle(gold):
    """FP64 on the GPU differs from the oracle only in summation order."""
    _note("config2 fp64, to 3 ms")
    t, f = _check(gold, _run(W.PREC_FP64, gold), 1e-6, 1e-3)
    e = gold["history_every"]
    fs = np.asarray(gold["history"]["force"])
    fg = f[e - 1::e][:len(fs)]
    scale = gold["peak_force_N"]
    err = np.max(np.abs(fg - fs)) / scale
    print(f"  sampled force history: max |dF| / F_max = {err:.3e}", flush=True)
    assert err <= 1e-5
