"""Matrix shear plasticity (Section 2.3.1, Algorithm 4's first two lines;
Table 1's S_p, K_p) on the GPU against the FP64 oracle.

FP64 mode: every exposed quantity, the plastic state included, within 1e-10
relative of the oracle over a run in which points yield, harden and then
damage.  Mixed precision: the peak contact force within 0.5 % of the FP64
oracle.  The plastic state is bitwise independent of the tile shape (rim
elements are evaluated by two workgroups; the update is idempotent), runs
repeat bit for bit, and a checkpoint carries it.  The same with full 2x2x2
integration, a plastic state per Gauss point (the paper's element and law).
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
EINVAL = -1


def _note(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


def plastic_case(nx=12, ny=12, precision=W.PREC_FP64):
    return W.tiny(nx, ny, 4, 1, angles=[0, 45, -45, 90], cohesive=1, law=W.LAW_CDM, lx=nx * 1e-3,
                  ly=ny * 1e-3, ply_thickness=0.25e-3, v0=20.0, mass=0.05, R=4e-3, plastic=True,
                  precision=precision)


def test_plastic_fp64_matches_the_oracle():
    _note("plasticity fp64 12x12x4+3 1000 steps")
    cfg = plastic_case()
    o, g = run_both(cfg, 1000, chunks=3)
    d = compare(o, g, cfg)
    for k in ("dt", "t", "force", "imp_disp", "disp", "gp_r", "coh_r", "energy"):
        assert d[k] <= TOL64, f"{k}: {d[k]:.3e}"
    assert d["vel"] <= 10 * TOL64
    epo, epg = o.get(oracle.GP_EP), g.array_get(pdn.ARR_GP_EP)
    assert epo.max() > 0.01                                  # points have yielded and hardened
    assert (o.get(oracle.GP_R) > 1).any()                    # and then damaged
    assert rel(epg, epo) <= TOL64
    e = g.energies()
    assert abs(e["residual"]) <= 1e-6 * e["ke0"]
    assert e["w_int"] - e["u_el"] > 0                        # plastic work dissipated


def test_plastic_mixed_peak_force():
    _note("plasticity mixed 12x12x4+3 1000 steps")
    cfg = plastic_case()
    o, g = run_both(cfg, 1000, precision=W.PREC_MIXED)
    fo, fg = o.history()[1], g.contact_force()[1]
    assert abs(fg.max() - fo.max()) <= 5e-3 * fo.max()
    epo, epg = o.get(oracle.GP_EP), g.array_get(pdn.ARR_GP_EP)
    assert abs(epg.max() - epo.max()) <= 2e-2 * epo.max()


def test_plastic_state_is_tile_invariant_and_repeatable():
    """A ragged multi-tile plate: 15x15, 16x16 and 8x8 tiles give bitwise equal
    plastic states, thresholds and displacements (rim elements read their
    plastic state before or after its owner updates it), and a second run
    repeats the first bit for bit."""
    _note("plasticity mixed 41x29x4+3 tiles 15x15 / 16x16, repeat")
    cfg = plastic_case(41, 29, W.PREC_MIXED)
    runs = []
    for tile in ((15, 15), (16, 16), (8, 8), (15, 15)):
        g = pdn.Simulation(cfg, tile=tile)
        g.step(900)
        runs.append([g.array_get(pdn.ARR_GP_EP), g.array_get(pdn.ARR_GP_R), g.array_get(pdn.ARR_DISP),
                     g.contact_force()[1]])
        g.close()
    assert runs[0][0].max() > 0
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            assert np.array_equal(a, b)


def test_plastic_checkpoint_round_trip():
    _note("plasticity checkpoint mixed 12x12x4+3")
    cfg = plastic_case(precision=W.PREC_MIXED)
    a = pdn.Simulation(cfg)
    a.step(700)
    blob = a.state_save()
    a.step(200)
    b = pdn.Simulation(cfg)
    b.step(1)
    b.state_load(blob)
    b.step(200)
    assert a.array_get(pdn.ARR_GP_EP).max() > 0
    for k in (pdn.ARR_GP_EP, pdn.ARR_GP_R, pdn.ARR_DISP, pdn.ARR_VEL):
        assert np.array_equal(a.array_get(k), b.array_get(k))
    # a checkpoint of a plate without plasticity does not load into this one
    plain = copy.deepcopy(cfg)
    for m in plain["materials"]:
        m["Sp"] = 0.0
    c = pdn.Simulation(plain)
    c.step(3)
    with pytest.raises(pdn.PdnError) as e:
        b.state_load(c.state_save())
    assert e.value.code == EINVAL
    for s in (a, b, c):
        s.close()


def full_plastic_case(nx=12, ny=12, precision=W.PREC_FP64):
    c = plastic_case(nx, ny, precision)
    c["mesh"]["integration"] = 8
    return c


def test_full_integration_plastic_fp64_matches_the_oracle():
    """The paper's element with the paper's law: 2x2x2 Gauss points, each
    with its own thresholds and plastic state, against the oracle's fully
    integrated element in FP64."""
    _note("plasticity + full integration fp64 12x12x4+3 800 steps")
    cfg = full_plastic_case()
    o, g = run_both(cfg, 800, chunks=2)
    d = compare(o, g, cfg)
    for k in ("dt", "t", "force", "imp_disp", "disp", "gp_r", "coh_r", "energy"):
        assert d[k] <= TOL64, f"{k}: {d[k]:.3e}"
    assert d["vel"] <= 10 * TOL64
    epo, epg = o.get(oracle.GP_EP), g.array_get(pdn.ARR_GP_EP)
    assert epo.size == 3 * 8 * g.info()["n_bulk"] and epo.max() > 0.01
    assert rel(epg, epo) <= TOL64
    e = g.energies()
    assert abs(e["residual"]) <= 1e-6 * e["ke0"]
    assert e["w_int"] - e["u_el"] > 0


def test_full_integration_plastic_mixed_tiles_repeat_and_checkpoint():
    """Mixed precision: peak force within 0.5 % of the FP64 oracle; 15x15 and
    16x16 tiles give bitwise equal states on a ragged plate; a checkpoint
    carries the eight plastic states of every element."""
    _note("plasticity + full integration mixed 12x12x4+3 vs oracle; 41x29 tiles; checkpoint")
    cfg = full_plastic_case()
    o, g = run_both(cfg, 800, precision=W.PREC_MIXED)
    fo, fg = o.history()[1], g.contact_force()[1]
    assert abs(fg.max() - fo.max()) <= 5e-3 * fo.max()
    g.close()
    big = full_plastic_case(41, 29, W.PREC_MIXED)
    runs = []
    for tile in ((15, 15), (16, 16)):
        s = pdn.Simulation(big, tile=tile)
        s.step(700)
        runs.append([s.array_get(pdn.ARR_GP_EP), s.array_get(pdn.ARR_GP_R), s.array_get(pdn.ARR_DISP)])
        if tile == (15, 15):
            blob = s.state_save()
            s.step(150)
            after = [s.array_get(pdn.ARR_GP_EP), s.array_get(pdn.ARR_DISP)]
        s.close()
    assert runs[0][0].max() > 0
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)
    t = pdn.Simulation(big)
    t.step(1)
    t.state_load(blob)
    t.step(150)
    assert np.array_equal(t.array_get(pdn.ARR_GP_EP), after[0])
    assert np.array_equal(t.array_get(pdn.ARR_DISP), after[1])
    t.close()


def test_plastic_combinations_not_built_are_rejected():
    _note("plasticity: rejected combinations")
    cfg = plastic_case(precision=W.PREC_MIXED)
    bad = copy.deepcopy(cfg)
    bad["materials"][0]["G13"] = 0.9 * bad["materials"][0]["G12"]
    with pytest.raises(pdn.PdnError) as e:
        pdn.Simulation(bad)
    assert e.value.code == EINVAL
    s = pdn.Simulation(cfg)
    with pytest.raises(pdn.PdnError) as e:
        s.surrogate_set(0, np.zeros(pdn.SUR_NPARAM, np.float32), 0.05, 1e-3)
    assert e.value.code == EINVAL
    t = pdn.Simulation(cfg, tile=(31, 15))
    with pytest.raises(pdn.PdnError) as e:
        t.step(1)
    assert e.value.code == EINVAL
    s2 = pdn.Simulation(cfg)
    with pytest.raises(pdn.PdnError) as e:
        pdn.Batch([s, s2])
    assert e.value.code == EINVAL
    full = pdn.Simulation(full_plastic_case(precision=W.PREC_MIXED))
    with pytest.raises(pdn.PdnError) as e:
        full.set_tile(32, 8)
    assert e.value.code == EINVAL
    for x in (s, t, s2, full):
        x.close()
