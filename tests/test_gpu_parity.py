"""GPU (HIP path through the C-ABI) against the FP64 oracle.

FP64 mode: every exposed quantity within 1e-10 relative (the stated FP64
bar; differences come only from summation order and library rounding).
"""
import copy
import sys

import numpy as np
import pytest

import oracle
import paper_2301_05552_amd as pdn
import workloads as W
from pdn_testutil import compare, rel, run_both

pytestmark = pytest.mark.gpu
TOL64 = 1e-10


def _note(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


def contact_case():
    cfg = W.tiny(6, 6, 2, 2, isotropic=True, v0=5.0, mass=0.2, R=3e-3)
    cfg["mesh"]["lx"] = cfg["mesh"]["ly"] = 12e-3
    return cfg


def cdm_case():
    return W.tiny(12, 12, 4, 1, angles=[0, 90, 0, 90], law=W.LAW_CDM, lx=12e-3, ly=12e-3,
                  ply_thickness=0.5e-3, v0=20.0, mass=0.02, R=4e-3)


def czm_case():
    return W.tiny(12, 12, 4, 1, angles=[0, 90, 0, 90], cohesive=1, law=W.LAW_CDM, lx=12e-3, ly=12e-3,
                  ply_thickness=0.25e-3, v0=20.0, mass=0.05, R=4e-3)


def _check64(d, what=""):
    """1e-10 on the results (force history, striker motion, displacements,
    damage state, energies).  The velocity is a one-step difference quotient of
    displacements, (d^{n+1} - d^n)/dt, so its relative error is the
    displacement's times |d|/|dt v| (~10 here): it gets 1e-9."""
    assert d["hist_len"][0] == d["hist_len"][1]
    assert d["energy_level"][0] == d["energy_level"][1]
    for k in ("dt", "t", "force", "imp_disp", "disp", "mass", "gp_r", "coh_r", "energy"):
        if k in d:
            assert d[k] <= TOL64, f"{what} {k}: {d[k]:.3e}"
    assert d["vel"] <= 10 * TOL64, f"{what} vel: {d['vel']:.3e}"


def test_contact_elastic_fp64():
    _note("contact_elastic_fp64 6x6x4 300 steps")
    cfg = contact_case()
    o, g = run_both(cfg, 300)
    d = compare(o, g, cfg)
    _check64(d, "contact")
    assert o.history()[1].max() > 0


def test_isotropic_plate_20x20x4_fp64():
    """The 20x20x4 isotropic plate (50 x 50 x 2 mm, clamped edges, 0.5 kg at 2 m/s), 2000 steps, history and energies."""
    _note("isotropic plate 20x20x4 fp64 2000 steps")
    cfg = W.plate_iso_20x20x4()
    o, g = run_both(cfg, 2000, chunks=3)
    d = compare(o, g, cfg)
    _check64(d, "isotropic plate")
    e = g.energies()
    assert abs(e["residual"]) <= 1e-6 * e["ke0"]


def test_cdm_fp64_with_damage():
    _note("cdm fp64 12x12x4 400 steps")
    cfg = cdm_case()
    o, g = run_both(cfg, 400)
    d = compare(o, g, cfg)
    _check64(d, "cdm")
    r = g.array_get(pdn.ARR_GP_R).reshape(-1, 4)
    assert (r.max(axis=1) > 1).sum() > 10                  # damage developed
    for kind in (pdn.DMG_FIBRE, pdn.DMG_MATRIX, pdn.DMG_SHEAR, pdn.DMG_PROJ_MATRIX):
        assert rel(g.damage_field(kind), o.damage_field(kind), floor=1.0) <= 1e-9


def _amplification(cfg, steps, eps=1e-14):
    """Relative force and displacement differences between two oracle runs
    whose striker speed differs by eps (relative), after each of `steps`."""
    a = oracle.Oracle(cfg)
    c2 = copy.deepcopy(cfg)
    c2["impactor"]["v0"] *= 1.0 + eps
    b = oracle.Oracle(c2)
    out, done = [], 0
    for n in steps:
        a.step(n - done)
        b.step(n - done)
        done = n
        out.append({"force": rel(b.history()[1], a.history()[1]),
                    "disp": rel(b.get(oracle.DISP), a.get(oracle.DISP))})
    return out


def test_tw_phi_1033_fp64():
    """The dissipative Tchamwa-Wielgosz member (phi = 1.033, Section 2.2.1)
    with damage and contact, 400 steps, at the same 1e-10 bar as phi = 1.
    Past 300 steps its softening points amplify round-off quickly; the
    oracle measures that on itself (a 1e-14 change of the striker's speed
    grows to ~1e-11 in the force by step 300 and ~4e-11 by step 400, 3.5
    times more in the last 100 steps; phi = 1 shows no growth), and the GPU,
    whose element arithmetic rounds differently, still meets the bar."""
    _note("cdm fp64 12x12x4 phi=1.033 400 steps")
    cfg = cdm_case()
    cfg["mesh"]["phi"] = 1.033
    a300, a400 = _amplification(cfg, (300, 400))
    o, g = run_both(cfg, 400)
    d = compare(o, g, cfg)
    print(f"  oracle amplification of 1e-14: force {a300['force']:.2e} at 300 steps, {a400['force']:.2e} "
          f"at 400; GPU vs oracle at 400: force {d['force']:.2e}, disp {d['disp']:.2e}, "
          f"gp_r {d['gp_r']:.2e}", flush=True)
    assert a400["force"] > 2 * a300["force"]
    _check64(d, "tw phi 1.033")
    assert o.history()[1].max() > 0


def test_as4_coupon_fp64():
    """The AS4/8552 coupon of Section 3.2.2 as meshed at refinement level 0
    (183 x 131 x 8 clusters, six interfaces, Table 3's counts), with the
    dissipative phi = 1.033, through first contact.  No node lies under the
    striker axis on this grid (the nearest is 0.56 mm off it, where the sphere
    is 20 um higher), so contact starts after about 30 um of travel, near step
    300.  The largest force difference is that of the first touch (1.7e-8 N
    on an 84 N reaction, a difference quotient of nearly equal positions) and
    does not grow; over 500 steps it is 8e-11 of the history's peak."""
    _note("as4 coupon level 0 fp64 phi=1.033 500 steps")
    cfg = W.coupon_as4(0, W.PREC_FP64)
    o, g = run_both(cfg, 500, threads=8)
    d = compare(o, g, cfg)
    _check64(d, "as4 coupon")
    assert o.history()[1].max() > 0


def test_czm_fp64_with_delamination():
    """Window ends ~100 steps after the first node pairs separate completely:
    beyond that the softening interface amplifies round-off (~10x per 100
    steps), which is sensitivity of the problem, not a discrepancy."""
    _note("czm fp64 12x12x4+3 1300 steps")
    cfg = czm_case()
    o, g = run_both(cfg, 1300, chunks=2)
    d = compare(o, g, cfg)
    _check64(d, "czm")
    assert g.array_get(pdn.ARR_COH_R).max() == 1.0        # some pairs fully separated
    for kind in (pdn.DMG_COHESIVE, pdn.DMG_PROJ_COHESIVE):
        assert rel(g.damage_field(kind), o.damage_field(kind), floor=1.0) <= 1e-9
    e = g.energies()
    assert abs(e["residual"]) <= 1e-6 * e["ke0"]


@pytest.mark.parametrize("nx,ny,plies", [(1, 1, 3), (1, 5, 2), (7, 1, 2), (2, 2, 1)])
def test_degenerate_meshes_fp64(nx, ny, plies):
    _note(f"degenerate {nx}x{ny}x{plies}")
    cfg = W.tiny(nx, ny, plies, 1, isotropic=True, lx=2e-3 * nx, ly=2e-3 * ny, v0=2.0, R=2e-3)
    cfg["mesh"]["bc"] = W.BC_FREE
    o, g = run_both(cfg, 60)
    _check64(compare(o, g, cfg), f"{nx}x{ny}")


def test_ragged_multi_tile_astm_fp64():
    """Mesh spanning several tiles in both directions with ragged tails, ASTM supports."""
    _note("ragged 47x23x3 astm fp64")
    cfg = W.tiny(47, 23, 3, 1, angles=[0, 45, 90], law=W.LAW_CDM, lx=47e-3, ly=23e-3,
                 ply_thickness=0.5e-3, v0=8.0, mass=0.1, R=4e-3, bc=W.BC_ASTM_WINDOW)
    o, g = run_both(cfg, 250)
    _check64(compare(o, g, cfg), "ragged")


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_tile_shape_invariance_bitwise(prec):
    """Owner-computes tiling: the result does not depend on the tile shape."""
    _note(f"tile invariance prec={prec}")
    cfg = copy.deepcopy(W.tiny(47, 23, 3, 1, angles=[0, 45, 90], cohesive=1, law=W.LAW_CDM, lx=47e-3,
                               ly=23e-3, ply_thickness=0.5e-3, v0=8.0, mass=0.1, R=4e-3, precision=prec))
    res = []
    for tile in ((15, 15), (16, 16), (32, 8), (8, 8), (31, 15)):
        try:
            g = pdn.Simulation(cfg, tile=tile)
        except pdn.PdnError as e:                 # workgroup does not fit this device's LDS
            assert e.code == pdn.PDN_EINVAL
            continue
        g.step(120)
        res.append((g.array_get(pdn.ARR_DISP), g.array_get(pdn.ARR_VEL), g.contact_force()[1],
                    g.energies()["w_int"]))
        g.close()
    assert len(res) >= 2
    for r in res[1:]:
        assert np.array_equal(r[0], res[0][0]) and np.array_equal(r[1], res[0][1])
        assert np.array_equal(r[2], res[0][2])
        # energy books are sums of per-workgroup partials: the block layout changes
        # their summation order only
        assert abs(r[3] - res[0][3]) <= 1e-12 * abs(res[0][3])


def test_checkpoint_resume_bitwise():
    _note("checkpoint")
    cfg = cdm_case()
    a = pdn.Simulation(cfg)
    a.step(300)
    b = pdn.Simulation(cfg)
    b.step(150)
    blob = b.state_save()
    c = pdn.Simulation(cfg)
    c.state_load(blob)
    c.step(150)
    for kind in (pdn.ARR_DISP, pdn.ARR_VEL, pdn.ARR_GP_R):
        assert np.array_equal(a.array_get(kind), c.array_get(kind))
    assert np.array_equal(a.contact_force()[1], c.contact_force()[1])
    ea, ec = a.energies(), c.energies()
    for k in ea:
        assert ea[k] == ec[k], k


def test_forced_adhesion_release_gpu():
    _note("forced adhesion")
    cfg = contact_case()
    o = oracle.Oracle(cfg)
    g = pdn.Simulation(cfg)
    for _ in range(200):
        o.step(1)
        g.step(1)
        if o.stats()["active"] >= 1 and g.info()["active"] >= 1:
            break
    o.step(5)
    g.step(5)
    imp = dict(cfg["impactor"])
    imp["v0"] = -cfg["impactor"]["v0"]
    o.set_impactor(imp)
    g.impactor_set(imp)
    before = g.info()
    o.step(1)
    g.step(1)
    after = g.info()
    assert after["released"] > before["released"]
    assert after["max_passes"] == 2
    assert after["released"] == o.stats()["released"]
    o.step(20)
    g.step(20)
    assert rel(g.array_get(pdn.ARR_DISP), o.get(oracle.DISP)) <= TOL64


def test_mixed_precision_close_to_fp64_oracle():
    """FP32 elements / FP64 nodes: contact force within 0.5% of the FP64 oracle."""
    _note("mixed vs oracle cdm")
    cfg = cdm_case()
    o, g = run_both(cfg, 400, precision=W.PREC_MIXED)
    fo, fg = o.history()[1], g.contact_force()[1]
    assert abs(fg.max() - fo.max()) <= 5e-3 * fo.max()
    assert rel(fg, fo) <= 5e-3
    ro = o.get(oracle.GP_R).reshape(-1, 4)
    rg = g.array_get(pdn.ARR_GP_R).reshape(-1, 4)
    assert abs((rg.max(axis=1) > 1).sum() - (ro.max(axis=1) > 1).sum()) <= 0.02 * (ro.max(axis=1) > 1).sum() + 1
