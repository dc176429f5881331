"""Accuracy gate of the reduced-precision path over a whole impact.

The 8-ply [0/45/-45/90]s plate (150 x 100 mm, 300 x 200 x 8 hex8,
intralaminar damage, window supports of the drop-weight coupon, 5.5 kg
striker of radius 8 mm at 15 J; Sec. 3.2, Table 1) is run through its whole
loading, past the force peak (3.97 ms) and the striker's largest
displacement (4.00 ms), to 4.5 ms on the GPU, and compared with the FP64
oracle's run of the same case stored in
tests/golden/qi8_300x200x8_fp64_oracle.json by
tests/golden/make_qi8_300x200x8_golden.py (which calls only the oracle and
the input generators).

The bars are the stated ones: mixed precision (FP32 element arithmetic and
Gauss-point state, FP64 nodal values) reproduces the peak contact force
within 0.5 % and the projected matrix-damage areas (d > 0, >= 0.5, >= 0.999)
within 2 % of the FP64 run.  The peak is that of the contact force averaged
over the trailing 250 steps (12 us; the stored run's `filter_steps`): the
kinematic contact makes the per-step force spiky, and the raw maximum is a
property of that noise.

The impact amplifies rounding: up to the first releases of contact nodes
(about step 5,900) FP64 runs agree to 1e-11, and after that an entry or
release decision of one node turns a rounding difference into a whole node
reaction.  FP64 runs whose impact energy differs by 1e-12 end up to 1.7 %
apart in the filtered peak force and 2.5 % in damaged area, and the oracle
run with its nodal sums in the opposite order (stored beside the first)
ends 0.27 % and up to 0.52 % apart.  That spread is measured and printed
here beside the errors; the bars are not widened by it.
"""
import json
import os
import sys

import numpy as np
import pytest

import paper_2301_05552_amd as pdn
import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "qi8_300x200x8_fp64_oracle.json")
GOLD_REV = GOLD.replace(".json", "_reversed.json")   # the same run, nodal sums in the opposite order
THRESHOLDS = ("0", "0.5", "0.999")
EARLY = 5800                    # steps of the deterministic window


def _note(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as fh:
        return json.load(fh)


def _trailing_mean(f, n):
    c = np.concatenate([[0.0], np.cumsum(f)])
    k = np.arange(1, len(f) + 1)
    lo = np.maximum(k - n, 0)
    return (c[k] - c[lo]) / (k - lo)


def _run(prec, g, energy_scale=1.0):
    cfg = W.plate_qi8_300x200x8(prec)
    cfg["impactor"]["energy"] *= energy_scale
    sim = pdn.Simulation(cfg)
    try:
        sim.step(0)                                      # set-up: the stable time step
        assert sim.info()["dt"] == pytest.approx(g["dt"], rel=1e-12)
        sim.step(g["steps"])
        t, f, x = sim.contact_force()
        assert len(f) == g["steps"]
        e = g["history_every"]
        m = cfg["mesh"]
        cell = (m["lx"] / m["nx"]) * (m["ly"] / m["ny"])
        d = sim.damage_field(pdn.DMG_PROJ_MATRIX)
        en = sim.energies()
        return {"f": f[e - 1::e], "x_max": float(x.max()),
                "f_peak": float(_trailing_mean(f, g["filter_steps"]).max()),
                "area": {thr: (int((d > 0).sum()) if thr == "0" else int((d >= float(thr)).sum())) * cell
                         for thr in THRESHOLDS},
                "fibre_cols": int((sim.damage_field(pdn.DMG_PROJ_FIBRE) > 0).sum()),
                "e_abs": en["ke0"] - en["ke_striker"]}
    finally:
        sim.close()


def _oracle(g):
    en = g["energies"]
    return {"f": np.asarray(g["history"]["force"]), "x_max": g["max_imp_disp_m"],
            "f_peak": g["peak_force_filtered_N"],
            "area": {thr: g["projected_damage"]["matrix"][thr]["area_m2"] for thr in THRESHOLDS},
            "fibre_cols": g["projected_damage"]["fibre"]["0"]["columns"],
            "e_abs": en["ke0"] - en["ke_striker"]}


def _errors(a, o):
    out = {"f_peak": abs(a["f_peak"] - o["f_peak"]) / o["f_peak"],
           "x_max": abs(a["x_max"] - o["x_max"]) / o["x_max"],
           "e_abs": abs(a["e_abs"] - o["e_abs"]) / o["e_abs"]}
    for thr in THRESHOLDS:
        out[f"area_{thr}"] = abs(a["area"][thr] - o["area"][thr]) / o["area"][thr]
    return out


@pytest.fixture(scope="module")
def runs(gold):
    _note("300x200x8 plate to 4.5 ms: fp64, mixed, three fp64 runs with the energy perturbed by 1e-12")
    assert gold["t_peak_filtered_s"] < gold["t_end"] - 2e-4          # the stored run passes the peak
    assert gold["t_max_imp_disp_s"] < gold["t_end"] - 2e-4
    out = {"oracle": _oracle(gold), "fp64": _run(W.PREC_FP64, gold), "mixed": _run(W.PREC_MIXED, gold)}
    out["ensemble"] = [_run(W.PREC_FP64, gold, 1.0 + 1e-12 * k) for k in (1, 2, 3)]
    with open(GOLD_REV) as fh:
        out["oracle_reversed"] = _oracle(json.load(fh))
    return out


def _early(r, g):
    return r["f"][:EARLY // g["history_every"]]


def test_fp64_deterministic_window(gold, runs):
    fo, fa = _early(runs["oracle"], gold), _early(runs["fp64"], gold)
    df = np.abs(fa - fo).max() / np.abs(fo).max()
    print(f"  fp64 first {EARLY} steps: force {df:.2e}", flush=True)
    assert df <= 1e-10


def test_mixed_peak_force_deterministic_window(gold, runs):
    fo, fm = _early(runs["oracle"], gold), _early(runs["mixed"], gold)
    rel = abs(fm.max() - fo.max()) / fo.max()
    print(f"  mixed peak over the first {EARLY} steps: {fm.max():.2f} N (oracle {fo.max():.2f} N), {rel:.2e}",
          flush=True)
    assert rel <= 5e-3


def test_mixed_meets_the_bars_over_the_whole_loading(gold, runs):
    """The stated bars on the whole loading: filtered peak force within
    0.5 %, projected matrix-damage areas within 2 %; also the largest
    striker displacement within 0.5 % and the energy taken from the striker
    within 2 %."""
    o, m = runs["oracle"], runs["mixed"]
    err = _errors(m, o)
    ens = [_errors(r, o) for r in runs["ensemble"]] + [_errors(runs["fp64"], o)]
    spread = {k: max(e[k] for e in ens) for k in err}
    rev = _errors(runs["oracle_reversed"], o)
    print(f"  mixed: filtered peak {m['f_peak']:.1f} N (oracle {o['f_peak']:.1f} N)", flush=True)
    for k, v in err.items():
        print(f"  {k}: mixed {v:.2e}; fp64 runs perturbed by 1e-12 (and the fp64 run) up to {spread[k]:.2e}; "
              f"the oracle with its sums reversed {rev[k]:.2e}", flush=True)
    assert err["f_peak"] <= 5e-3
    for thr in THRESHOLDS:
        assert err[f"area_{thr}"] <= 2e-2
    assert err["x_max"] <= 5e-3 and err["e_abs"] <= 2e-2
    assert m["fibre_cols"] == o["fibre_cols"] == 0              # no fibre damage in this impact


def test_fp64_whole_loading(gold, runs):
    """FP64 on the GPU differs from the oracle only in rounding order; over
    the whole loading it is held to the well-conditioned bars and the area
    bar, and its filtered peak force to the 2 % that FP64 runs perturbed by
    1e-12 reach."""
    err = _errors(runs["fp64"], runs["oracle"])
    print("  fp64: " + ", ".join(f"{k} {v:.2e}" for k, v in err.items()), flush=True)
    assert err["x_max"] <= 5e-3 and err["e_abs"] <= 2e-2
    for thr in THRESHOLDS:
        assert err[f"area_{thr}"] <= 2e-2
    assert err["f_peak"] <= 2e-2


def test_the_impact_amplifies_rounding(gold, runs):
    """The perturbed FP64 runs agree with the oracle to 1e-10 in the
    deterministic window and then part: a 1e-12 change of the impact energy
    reaches per-mille to per-cent differences in the filtered peak force or
    the damaged area by the end of the loading."""
    o = runs["oracle"]
    worst = 0.0
    for r in runs["ensemble"]:
        fo, fr = _early(o, gold), _early(r, gold)
        assert np.abs(fr - fo).max() / np.abs(fo).max() <= 1e-10
        e = _errors(r, o)
        worst = max(worst, e["f_peak"], *(e[f"area_{thr}"] for thr in THRESHOLDS))
    print(f"  largest whole-loading difference of a perturbed fp64 run: {worst:.2e}", flush=True)
    assert worst >= 1e-3
