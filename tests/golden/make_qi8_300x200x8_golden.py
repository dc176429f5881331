"""Write qi8_300x200x8_fp64_oracle.json: the FP64 oracle's run of the 8-ply
[0/45/-45/90]s plate (300 x 200 x 8 hex8, intralaminar damage, ASTM window
supports, 5.5 kg striker at 15 J) through the whole loading of the impact,
past the force peak and the striker's largest displacement (4.5 ms).

The stored values (contact-force history, its peak, projected damage areas,
energy books) are the expected values of the reduced-precision gate: FP32
element arithmetic must reproduce the peak contact force within 0.5 % and the
projected damage areas within 2 % of this FP64 run.  The peak is taken on
the force averaged over the last FILTER steps (a trailing moving average,
about 12 us): the kinematic contact makes the per-step force spiky, and the
maximum of the raw history is a property of its noise, not of the impact.

With --reverse-assembly the oracle sums the nodal forces in descending
element order: the same arithmetic in another order.  That run, stored
beside the first, measures how far this impact amplifies rounding by itself.

Only the oracle and the input generators are called.  Usage (about three
hours on 6 cores each):

    python tests/golden/make_qi8_300x200x8_golden.py [--threads 6] [--t-end 4.5e-3]
    python tests/golden/make_qi8_300x200x8_golden.py --reverse-assembly \
        --out tests/golden/qi8_300x200x8_fp64_oracle_reversed.json
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402

THRESHOLDS = (0.0, 0.5, 0.999)       # d > 0, and d >= 0.5 / 0.999 (damage-area readings)
EVERY = 50
FILTER = 250                         # steps of the trailing moving average of the force
SNAP_EVERY = 10000                   # steps between stored projected-damage snapshots


def filtered(f, n=FILTER):
    """Trailing moving average over n steps (shorter at the start)."""
    c = np.concatenate([[0.0], np.cumsum(f)])
    k = np.arange(1, len(f) + 1)
    lo = np.maximum(k - n, 0)
    return (c[k] - c[lo]) / (k - lo)


def projected_areas(o, cfg):
    m = cfg["mesh"]
    cell = (m["lx"] / m["nx"]) * (m["ly"] / m["ny"])
    out = {}
    for name, kind in (("fibre", oracle.DMG_PROJ_FIBRE), ("matrix", oracle.DMG_PROJ_MATRIX)):
        d = o.damage_field(kind)
        out[name] = {}
        for thr in THRESHOLDS:
            n = int((d > 0).sum()) if thr == 0 else int((d >= thr).sum())
            out[name][f"{thr:g}"] = {"columns": n, "area_m2": n * cell}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=6)
    ap.add_argument("--t-end", type=float, default=4.5e-3)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "qi8_300x200x8_fp64_oracle.json"))
    ap.add_argument("--reverse-assembly", action="store_true",
                    help="sum nodal forces in descending element order (a second realization of the "
                         "same arithmetic in another order, for the problem's own sensitivity)")
    args = ap.parse_args()
    oracle.build(force=False)
    cfg = W.plate_qi8_300x200x8(W.PREC_FP64)
    o = oracle.Oracle(cfg, threads=args.threads)
    o.set_assembly_order(args.reverse_assembly)
    steps = int(math.ceil(args.t_end / o.dt))
    t0 = time.time()
    done = 0
    snaps = []
    while done < steps:
        n = min(1000, steps - done)
        o.step(n)
        done += n
        t, f, _ = o.history()
        print(f"[golden] {done}/{steps} steps, F={f[-1]:.1f} N, {time.time() - t0:.0f} s", flush=True)
        if done % SNAP_EVERY == 0:
            snaps.append({"steps": done, "t": float(t[-1]), "projected_damage": projected_areas(o, cfg)})
    t, f, x = o.history()
    i = int(np.argmax(f))
    ff = filtered(f)
    j = int(np.argmax(ff))
    k = int(np.argmax(x))
    res = {
        "source": "FP64 oracle (oracle/pdn_oracle.c) on workloads.plate_qi8_300x200x8, written by make_qi8_300x200x8_golden.py",
        "basis": "laminate, supports and striker of the drop-weight coupon (Sec. 4), Table 1 material; "
                 "contact force and projected damage are the outputs of Tabs. 2 and 4 and Fig. 9",
        "assembly_order": "descending" if args.reverse_assembly else "ascending",
        "dt": o.dt, "steps": steps, "t_end": float(t[-1]),
        "peak_force_N": float(f[i]), "t_peak_s": float(t[i]),
        "filter_steps": FILTER,
        "peak_force_filtered_N": float(ff[j]), "t_peak_filtered_s": float(t[j]), "step_peak_filtered": j,
        "max_imp_disp_m": float(x[k]), "t_max_imp_disp_s": float(t[k]),
        "history_every": EVERY,
        "history": {"t": t[EVERY - 1::EVERY].tolist(), "force": f[EVERY - 1::EVERY].tolist(),
                    "force_filtered": ff[EVERY - 1::EVERY].tolist(),
                    "imp_disp": x[EVERY - 1::EVERY].tolist()},
        "projected_damage": projected_areas(o, cfg),
        "projected_damage_snapshots": snaps,
        "energies": o.energies(),
        "oracle_seconds": time.time() - t0,
    }
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(f"[golden] wrote {args.out}: peak {f[i]:.2f} N at {t[i] * 1e3:.3f} ms, filtered peak "
          f"{ff[j]:.2f} N at {t[j] * 1e3:.3f} ms, largest striker displacement at {t[k] * 1e3:.3f} ms",
          flush=True)


if __name__ == "__main__":
    main()
