"""Write qi8_150x100x16_fp64_oracle.json: the FP64 oracle's run of the
150 x 100-column cut of the 1200 x 800 x 16 plate (same laminate, element size
0.125 x 0.125 x 0.25 mm with 2 elements per ply, 6 cohesive interfaces,
scaled window supports, 5.5 kg striker at 25 J) for 2000 steps, through
first contact (about step 320) and the first 17 us of loading.

Stored for the multi-step parity test of the library at this element size:
the whole contact-force and striker histories, the energy books, and the
displacement, velocity and damage thresholds at seeded sample points plus
every node, Gauss point and interface pair under the striker.

A second oracle run sums the nodal forces in the opposite element order
(the same arithmetic in another order): its deviation from the first,
stored per 250-step block for the force history and at the end for the
sampled state, is how far this problem amplifies rounding by itself, the
scale against which the library's differences (its own summation order and
library rounding) are judged.

With --full-plastic the same cut is run with the paper's element and law:
2x2x2 Gauss points per bulk element and Table 1's matrix shear plasticity on
every ply (qi8_150x100x16_full_plastic_fp64_oracle.json); the sampled
Gauss-point state is then every point of the sampled elements, thresholds
and plastic state.  That run is stored at 1750 steps (--steps 1750): in the
next 250 steps the oracle's two summation orders part (the crushed elements
under the striker, with no hourglass control in this element, turn rounding
into velocity differences of metres per second at single nodes).

Only the oracle and the input generators are called.  Usage (ten minutes;
with --full-plastic ten minutes on 8 threads):

    python tests/golden/make_qi8_150x100x16_golden.py [--threads 4]
    python tests/golden/make_qi8_150x100x16_golden.py --threads 8 --full-plastic --steps 1750
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from pdn_testutil import coh_pairs_from_oracle  # noqa: E402

STEPS = 2000
SAMPLE_SEED = 0x150100


def sample_indices(o, cfg):
    """Seeded sample nodes, Gauss points and interface pairs, plus all those
    within 1 mm of the plate centre in-plane (the contact zone)."""
    m = cfg["mesh"]
    nx, ny = m["nx"], m["ny"]
    hx, hy = m["lx"] / nx, m["ly"] / ny
    g = W.rng(SAMPLE_SEED)
    plane = (nx + 1) * (ny + 1)
    K = o.nn // plane
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1))
    near = (np.hypot(ii * hx - m["lx"] / 2, jj * hy - m["ly"] / 2) <= 1.0e-3).reshape(-1)
    node_cols = np.flatnonzero(near)
    nodes = set(g.integers(0, o.nn, 2000).tolist())
    for k in range(K):
        nodes.update((k * plane + node_cols).tolist())
    ie, je = np.meshgrid(np.arange(nx), np.arange(ny))
    nearc = (np.hypot((ie + 0.5) * hx - m["lx"] / 2, (je + 0.5) * hy - m["ly"] / 2) <= 1.0e-3).reshape(-1)
    cols = np.flatnonzero(nearc)
    L = o.ne // (nx * ny)
    gps = set(g.integers(0, o.ne, 2000).tolist())
    for l in range(L):
        gps.update((l * nx * ny + cols).tolist())
    npairs = 6 * plane
    pairs = set(g.integers(0, npairs, 1000).tolist())
    for c in range(6):
        pairs.update((c * plane + node_cols).tolist())
    return sorted(nodes), sorted(gps), sorted(pairs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=4)
    ap.add_argument("--full-plastic", action="store_true",
                    help="2x2x2 Gauss points and shear plasticity on every ply")
    ap.add_argument("--out", default=None)
    ap.add_argument("--steps", type=int, default=STEPS, help="a multiple of 250")
    args = ap.parse_args()
    here = os.path.dirname(os.path.abspath(__file__))
    if args.out is None:
        args.out = os.path.join(here, "qi8_150x100x16_full_plastic_fp64_oracle.json" if args.full_plastic
                                else "qi8_150x100x16_fp64_oracle.json")
    oracle.build(force=False)
    cfg = W.plate_qi8_150x100x16_cut(W.PREC_FP64)
    if args.full_plastic:
        cfg["mesh"]["integration"] = 8
        for mat in cfg["materials"]:
            mat["Sp"], mat["Kp"] = W.AS4_SP, W.AS4_KP
    ngp = 8 if args.full_plastic else 1
    o = oracle.Oracle(cfg, threads=args.threads)
    q = oracle.Oracle(cfg, threads=args.threads)
    q.set_assembly_order(True)
    t0 = time.time()
    steps = args.steps
    for k in range(steps // 250):
        o.step(250)
        q.step(250)
        print(f"[golden] {250 * (k + 1)}/{steps} steps, active {o.stats()['active']}, "
              f"{time.time() - t0:.0f} s", flush=True)
    nodes, gps, pairs = sample_indices(o, cfg)
    d = o.get(oracle.DISP).reshape(-1, 3)
    v = o.get(oracle.VEL).reshape(-1, 3)
    # Gauss-point records per element (all its points): thresholds, and with
    # plasticity the plastic state
    r = o.get(oracle.GP_R).reshape(-1, 4 * ngp)
    rd = coh_pairs_from_oracle(o, cfg["mesh"])
    t, f, x = o.history()
    _, fq, xq = q.history()
    dq, vq = q.get(oracle.DISP).reshape(-1, 3), q.get(oracle.VEL).reshape(-1, 3)
    rq, rdq = q.get(oracle.GP_R).reshape(-1, 4 * ngp), coh_pairs_from_oracle(q, cfg["mesh"])
    ep = o.get(oracle.GP_EP).reshape(-1, 3 * ngp) if args.full_plastic else None
    epq = q.get(oracle.GP_EP).reshape(-1, 3 * ngp) if args.full_plastic else None
    sens = {
        "force_block_steps": 250,
        "force_abs_by_block": [float(np.abs(fq[i:i + 250] - f[i:i + 250]).max()) for i in range(0, steps, 250)],
        "imp_disp_abs_max": float(np.abs(xq - x).max()),
        "disp_abs_max": float(np.abs(dq[nodes] - d[nodes]).max()),
        "vel_abs_max": float(np.abs(vq[nodes] - v[nodes]).max()),
        "r_abs_max": float(np.abs(rq[gps] - r[gps]).max()),
        "rd_abs_max": float(np.abs(rdq[pairs] - rd[pairs]).max()),
    }
    if ep is not None:
        sens["ep_abs_max"] = float(np.abs(epq[gps] - ep[gps]).max())
    res = {
        "source": "FP64 oracle (oracle/pdn_oracle.c) on workloads.plate_qi8_150x100x16_cut"
                  + (" with 2x2x2 Gauss points and shear plasticity (S_p, K_p of AS4/8552)" if args.full_plastic
                     else "") + ", written by make_qi8_150x100x16_golden.py",
        "integration": ngp, "plastic": bool(args.full_plastic),
        "dt": o.dt, "steps": steps, "stats": o.stats(), "energies": o.energies(),
        "history": {"t": t.tolist(), "force": f.tolist(), "imp_disp": x.tolist()},
        "nodes": nodes, "disp": d[nodes].tolist(), "vel": v[nodes].tolist(),
        "gps": gps, "r": r[gps].tolist(), "r_max": float(r.max()),
        "pairs": pairs, "rd": rd[pairs].tolist(), "rd_max": float(rd.max()),
        "disp_absmax": float(np.abs(d).max()), "vel_absmax": float(np.abs(v).max()),
        **({"ep": ep[gps].tolist(), "ep_max": float(np.abs(ep).max())} if ep is not None else {}),
        "reversed_assembly_deviation": sens,
        "oracle_seconds": time.time() - t0,
    }
    with open(args.out, "w") as fh:
        json.dump(res, fh)
    print(f"[golden] wrote {args.out}: peak force {f.max():.2f} N, r max {r.max():.4f}, rd max {rd.max():.4f}; "
          f"reversed order: force {max(sens['force_abs_by_block']):.3e} N", flush=True)


if __name__ == "__main__":
    main()
