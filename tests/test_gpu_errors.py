"""Error behaviour of the C-ABI on a live context (include/pdn.h): each call
rejects bad arguments with the documented code and a message, and a rejected
call leaves the simulation state as it was, so the context steps on bitwise
like one that never saw the error."""
import copy
import ctypes as C
import sys

import numpy as np
import pytest

import paper_2301_05552_amd as pdn
import workloads as W

pytestmark = pytest.mark.gpu
EINVAL, ESTATE, ERANGE = -1, -4, -6


def _note(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


def _cfg():
    return W.tiny(9, 7, 3, 1, angles=[0, 45, 90], cohesive=1, law=W.LAW_CDM, lx=9e-3, ly=7e-3,
                  ply_thickness=0.5e-3, v0=12.0, mass=0.05, R=3e-3, precision=W.PREC_MIXED)


def _code(fn, *a):
    with pytest.raises(pdn.PdnError) as e:
        fn(*a)
    assert str(e.value).split(":", 1)[1].strip(), "empty error message"
    return e.value.code


def _state(s):
    return [s.array_get(pdn.ARR_DISP), s.array_get(pdn.ARR_VEL), s.array_get(pdn.ARR_GP_R),
            s.contact_force()[1]]


def test_calls_out_of_order_are_rejected():
    _note("errors: ESTATE before materials / striker / first step")
    cfg = _cfg()
    cfg["impactor"] = None
    s = pdn.Simulation(cfg)
    assert _code(s.step, 1) == ESTATE
    assert _code(s.state_save) == ESTATE
    assert _code(s.autotune) == ESTATE
    assert _code(s.state_load, b"\0" * 64) == ESTATE
    s.impactor_set(_cfg()["impactor"])
    assert _code(s.state_save) == ESTATE          # needs one completed step
    s.step(3)
    assert len(s.state_save()) > 0
    s.close()


def test_rejected_arguments_leave_the_state_unchanged():
    _note("errors: EINVAL / ERANGE mid-run, then bitwise continuation")
    cfg = _cfg()
    ref = pdn.Simulation(cfg)
    s = pdn.Simulation(cfg)
    ref.step(40)
    s.step(40)
    L = pdn.lib()
    mat = dict(cfg["materials"][0])
    assert _code(s.material_set, 7, mat) == EINVAL                      # ply out of range
    bad = dict(mat, E1=-1.0)
    assert _code(s.material_set, 0, bad) == EINVAL                      # non-positive stiffness
    imp = dict(cfg["impactor"], radius=0.0)
    assert _code(s.impactor_set, imp) == EINVAL
    assert _code(s.step, -1) == EINVAL
    assert _code(s.damage_field, 9) == EINVAL
    assert _code(s.array_get, 99) == EINVAL
    assert _code(s.array_set, pdn.ARR_DISP, np.zeros(5)) == EINVAL     # wrong length
    assert _code(s.state_load, b"\0" * 8) == EINVAL                     # too short
    other = pdn.Simulation(W.tiny(5, 4, 2, 1, law=W.LAW_CDM, lx=5e-3, ly=4e-3, precision=W.PREC_MIXED))
    other.step(2)
    assert _code(s.state_load, other.state_save()) == EINVAL            # another plate's checkpoint
    other.close()
    blob = ref.state_save()
    assert _code(s.state_load, blob[:-1]) == EINVAL                     # one byte short
    assert _code(s.state_load, blob + b"\0") == EINVAL                  # one byte long
    hdr = bytearray(blob)
    hdr[5 * 8:6 * 8] = (-1).to_bytes(8, "little", signed=True)          # negative history length
    assert _code(s.state_load, bytes(hdr)) == EINVAL
    hdr[5 * 8:6 * 8] = (1 << 60).to_bytes(8, "little", signed=True)     # huge history length
    assert _code(s.state_load, bytes(hdr)) == EINVAL
    assert _code(s.set_tile, 7, 3) == EINVAL                            # no such tile
    # output buffers that are too small: ERANGE and the size needed
    n = C.c_int64()
    buf = np.zeros(3)
    assert L.pdn_contact_force(s.h, None, pdn._dp(buf), None, 3, C.byref(n)) == ERANGE
    assert n.value == 40
    assert L.pdn_damage_field(s.h, pdn.DMG_PROJ_MATRIX, pdn._dp(buf), 3, C.byref(n)) == ERANGE
    assert n.value == 9 * 7
    assert L.pdn_state_save(s.h, None, 0, C.byref(n)) == ERANGE
    assert n.value == len(ref.state_save())
    # none of it moved the simulation
    ref.step(60)
    s.step(60)
    for a, b in zip(_state(ref), _state(s)):
        assert np.array_equal(a, b)
    ref.close()
    s.close()


def test_batch_rejects_cases_of_other_precisions():
    _note("errors: batch of mixed precisions")
    a = _cfg()
    b = copy.deepcopy(a)
    b["mesh"]["precision"] = W.PREC_FP64
    sims = [pdn.Simulation(a), pdn.Simulation(b)]
    with pytest.raises(pdn.PdnError) as e:
        pdn.Batch(sims)
    assert e.value.code == EINVAL
    assert "case 1" in str(e.value)                                     # reported through the first case
    with pytest.raises(pdn.PdnError) as e:
        pdn.Batch([sims[0], sims[0]])
    assert e.value.code == EINVAL and "repeats" in str(e.value)
    for s in sims:
        s.close()


def test_forced_instability_and_snap_back_rejection():
    """Failure paths forced from the host: a time step three times the stable
    one makes the explicit scheme diverge, and pdn_step reports
    PDN_EUNSTABLE (non-finite state) and keeps reporting it; a fibre law
    whose bilinear softening is not ordered at the element size (a toughness
    far too small for the crack band) is rejected by pdn_material_set."""
    _note("errors: forced instability (cfl_safety 3), snap-back rejection")
    EUNSTABLE = -5
    cfg = _cfg()
    cfg["mesh"]["cfl_safety"] = 3.0
    s = pdn.Simulation(cfg)
    code, steps = None, 0
    while code is None and steps < 5000:
        try:
            s.step(100)
            steps += 100
        except pdn.PdnError as e:
            code = e.code
    assert code == EUNSTABLE, (code, steps)
    assert _code(s.step, 1) == EUNSTABLE
    s.close()
    t = pdn.Simulation(_cfg())
    bad = copy.deepcopy(_cfg()["materials"][0])
    bad["GXT"] = 1.0                       # J/m^2: the softening would start below the onset strain
    assert _code(t.material_set, 0, bad) == EINVAL
    t.step(5)                              # the context keeps its materials and steps on
    t.close()
