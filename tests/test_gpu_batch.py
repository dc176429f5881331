"""Batched stepping of uneven cases (one launch per kernel per step serves
every case) and the tile autotuner, through the C-ABI.

A batched case must follow exactly the arithmetic of the same case stepped
alone in the same tile layout, so batched and single runs are compared
bitwise; one batched case is also compared with the FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle
import paper_2301_05552_amd as pdn
import workloads as W
from pdn_testutil import compare

pytestmark = pytest.mark.gpu


def _note(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


def _cases(prec):
    cs = [
        W.tiny(10, 7, 3, 1, angles=[0, 45, 90], law=W.LAW_CDM, lx=10e-3, ly=7e-3, ply_thickness=0.5e-3,
               v0=12.0, mass=0.05, R=3e-3, bc=W.BC_ASTM_WINDOW, precision=prec),
        W.tiny(23, 17, 4, 1, angles=[0, 90, 0, 90], cohesive=1, law=W.LAW_CDM, lx=23e-3, ly=17e-3,
               ply_thickness=0.25e-3, v0=15.0, mass=0.05, R=4e-3, precision=prec),
        W.tiny(6, 6, 2, 2, isotropic=True, v0=5.0, mass=0.2, R=3e-3, lx=12e-3, ly=12e-3, precision=prec),
        W.tiny(31, 5, 2, 1, law=W.LAW_CDM, lx=31e-3, ly=5e-3, ply_thickness=0.5e-3, v0=8.0, R=2e-3,
               precision=prec),
    ]
    for c in cs:                       # striker starts on the plate so contact acts early
        c["impactor"]["gap"] = 1e-7
    return cs


def _state(s):
    t, f, x = s.contact_force()
    return [s.array_get(pdn.ARR_DISP), s.array_get(pdn.ARR_VEL), s.array_get(pdn.ARR_GP_R),
            s.array_get(pdn.ARR_COH_R), t, f, x]


def _same(a, b, what):
    for k, (u, v) in enumerate(zip(_state(a), _state(b))):
        assert np.array_equal(u, v), f"{what}: state item {k} differs"
    ea, eb = a.energies(), b.energies()
    for k in ea:
        assert ea[k] == eb[k], f"{what}: energy {k}"


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_MIXED])
def test_batch_matches_single_bitwise(prec):
    _note(f"batch vs single prec={prec}")
    cfgs = _cases(prec)
    sims = [pdn.Simulation(c) for c in cfgs]
    batch = pdn.Batch(sims)
    tile = batch.info()["tile"]
    assert batch.info()["n_bulk"] == sum(s.info()["n_bulk"] for s in sims)
    refs = [pdn.Simulation(c, tile=tile) for c in cfgs]
    # graph replays (8 steps each) and a remainder, an odd count so the
    # buffer parity flips, then one case stepped alone between batched calls
    batch.step(37)
    for r in refs:
        r.step(37)
    sims[1].step(3)
    refs[1].step(3)
    batch.step(21)
    for r in refs:
        r.step(21)
    for k, (s, r) in enumerate(zip(sims, refs)):
        _same(s, r, f"case {k}")
        assert s.info()["steps"] == (61 if k == 1 else 58)
    assert max(s.info()["active"] for s in sims) > 0
    batch.close()


def test_64_case_batch_matches_solo_runs_bitwise():
    """The benchmark's batch (64 seeded plates of 20k-400k elements, 4-16
    plies, mixed precision) stepped 403 times in one launch per kernel and
    step: every case equals the same case stepped alone on the batch's tile,
    bit for bit (states, histories, energy books)."""
    _note("64-case batch (13.6M GPs) vs 64 solo runs, 403 steps")
    cfgs = W.batch_cases_64()
    sims = [pdn.Simulation(c) for c in cfgs]
    batch = pdn.Batch(sims)
    tile = batch.info()["tile"]
    batch.step(403)
    assert sum(s.info()["active"] > 0 for s in sims) > 0
    for k, c in enumerate(cfgs):
        r = pdn.Simulation(c, tile=tile)
        r.step(403)
        _same(sims[k], r, f"case {k}")
        r.close()
    batch.close()
    for s in sims:
        s.close()


def test_batched_case_matches_oracle_fp64():
    _note("batched case vs oracle")
    cfgs = _cases(W.PREC_FP64)
    sims = [pdn.Simulation(c) for c in cfgs]
    batch = pdn.Batch(sims)
    batch.step(150)
    o = oracle.Oracle(cfgs[1])
    o.step(150)
    d = compare(o, sims[1], cfgs[1])
    for k in ("force", "disp", "gp_r", "coh_r", "energy"):
        if k in d:
            assert d[k] <= 1e-10, (k, d[k])
    batch.close()


def test_batch_rejects_mixed_precision_and_duplicates():
    _note("batch errors")
    a = pdn.Simulation(_cases(W.PREC_FP64)[2])
    b = pdn.Simulation(_cases(W.PREC_MIXED)[2])
    with pytest.raises(pdn.PdnError) as e:
        pdn.Batch([a, b])
    assert e.value.code == pdn.PDN_EINVAL
    with pytest.raises(pdn.PdnError) as e:
        pdn.Batch([a, a])
    assert e.value.code == pdn.PDN_EINVAL


def test_autotune_keeps_state():
    _note("autotune")
    cfg = _cases(W.PREC_MIXED)[1]
    a = pdn.Simulation(cfg)
    a.step(40)
    tile = a.autotune()
    assert tile in [(15, 15), (16, 16), (32, 8), (8, 8), (31, 15)]
    assert a.info()["tile_x"] == tile[0] and a.info()["tile_y"] == tile[1]
    a.step(40)
    b = pdn.Simulation(cfg, tile=tile)
    b.step(80)
    # the timed passes changed nothing; the layout changes no displacement bit
    assert np.array_equal(a.array_get(pdn.ARR_DISP), b.array_get(pdn.ARR_DISP))
    assert np.array_equal(a.array_get(pdn.ARR_GP_R), b.array_get(pdn.ARR_GP_R))
    assert np.array_equal(a.contact_force()[1], b.contact_force()[1])
    assert a.autotune() == tile                     # remembered for this plate shape


def test_batch_restores_its_tile_after_a_case_is_retiled():
    """A case moved to another tile layout between batched calls is put back in
    the batch's layout (block table and step graph rebuilt as needed); the
    states stay bit for bit those of the cases stepped alone."""
    _note("batch after a case changed tile")
    cfgs = _cases(W.PREC_MIXED)
    sims = [pdn.Simulation(c) for c in cfgs]
    batch = pdn.Batch(sims)
    tile = batch.info()["tile"]
    refs = [pdn.Simulation(c, tile=tile) for c in cfgs]
    batch.step(17)
    for r in refs:
        r.step(17)
    other = (8, 8) if tile != (8, 8) else (15, 15)
    sims[0].set_tile(*other)
    sims[0].step(2)
    refs[0].step(2)
    batch.step(19)
    for r in refs:
        r.step(19)
    assert batch.info()["tile"] == tile
    for k, (s, r) in enumerate(zip(sims, refs)):
        _same(s, r, f"case {k}")
    batch.close()
