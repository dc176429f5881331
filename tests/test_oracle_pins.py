"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself:
values printed in the paper (golden fixtures with citations), closed forms,
invariants, or finite differences.  None of these tests needs a GPU.
"""
import copy
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _free(cfg):
    cfg = copy.deepcopy(cfg)
    cfg["mesh"]["bc"] = 2
    return cfg


def _grid_coords(cfg):
    """Reference coordinates of the structured generator (for perturbation)."""
    o = oracle.Oracle(cfg)
    return o.get(oracle.COORDS).reshape(-1, 3)


def _elastic(mat):
    m = dict(mat)
    m["law"] = W.LAW_ELASTIC
    return m


AS4_ELASTIC = dict(W.material_isotropic(1.0, 0.0, 1590.0),
                   E1=128.0e9, E2=7.63e9, E3=7.63e9, nu12=0.35, nu13=0.35, nu23=0.45,
                   G12=4.358e9, G13=4.358e9, G23=2.631e9)


# ---------------------------------------------------------------------------
# mesh generator: Table 3 counts (and Eq. mmu)
# ---------------------------------------------------------------------------

def _table3_mesh(level):
    g = json.load(open(os.path.join(GOLD, "table3_mesh_counts.json")))
    lv = g["levels"][level]
    t = g["cluster_thickness_mm"] * 1e-3
    mesh = W._mesh(lv["nx"], lv["ny"], 8, lv["elements_per_cluster"], 0.150, 0.100, t,
                   g["cluster_angles_deg"], cohesive=1)
    return g, lv, mesh


@pytest.mark.parametrize("level", [0, 1])
def test_table3_counts(level):
    g, lv, mesh = _table3_mesh(level)
    c = oracle.mesh_counts(mesh)
    assert c["n_bulk"] + c["n_cohesive"] == lv["n_elements"]
    assert c["n_nodes"] == lv["n_nodes"]


@pytest.mark.parametrize("level", [0, 1])
def test_as4_coupon_workload_matches_table3(level):
    """The coupon workload's mesh is the one whose counts Table 3 prints."""
    _, lv, _ = _table3_mesh(level)
    c = oracle.mesh_counts(W.coupon_as4(level)["mesh"])
    assert c["n_bulk"] + c["n_cohesive"] == lv["n_elements"]
    assert c["n_nodes"] == lv["n_nodes"]
    assert c["n_cohesive"] == 6 * lv["nx"] * lv["ny"]      # six interfaces between differing clusters


def test_eq_mmu_element_count():
    """Eq. (mmu): n_e = 8 n_e^0 - 4 n_e,ELINT^0 with n_e^0 all base elements."""
    _, _, m0 = _table3_mesh(0)
    _, lv1, _ = _table3_mesh(1)
    c0 = oracle.mesh_counts(m0)
    n0 = c0["n_bulk"] + c0["n_cohesive"]
    assert 8 * n0 - 4 * c0["n_cohesive"] == lv1["n_elements"]


@pytest.mark.parametrize("level", [0, 1])
def test_table3_stable_increment_sanity(level):
    """Loose check (+-15%) of the critical step against Table 3's printed value,
    AS4/8552 elastic constants of Table 1, undamaged stiffness, no safety factor."""
    g, lv, mesh = _table3_mesh(level)
    h = lv["element_size_mm"] * 1e-3
    small = W._mesh(6, 6, 8, lv["elements_per_cluster"], 6 * h, 6 * h,
                    g["cluster_thickness_mm"] * 1e-3, g["cluster_angles_deg"], cfl_safety=1.0)
    cfg = dict(mesh=small, materials=[AS4_ELASTIC], impactor=W.impactor(8e-3, 1.0, v0=1.0))
    dt = oracle.Oracle(cfg).dt
    assert 0.85 < lv["stable_dt_s"] / dt < 1.15


def test_workload_counts():
    assert oracle.mesh_counts(W.plate_iso_20x20x4()["mesh"])["n_nodes"] == 21 * 21 * 5
    c3 = oracle.mesh_counts(W.plate_qi8_1200x800x16()["mesh"])
    assert c3["n_planes"] == 23 and c3["n_bulk"] == 15360000 and c3["n_cohesive"] == 5760000
    assert c3["n_nodes"] == 22126023


# ---------------------------------------------------------------------------
# element: patch test, finite differences, rigid rotation, mass
# ---------------------------------------------------------------------------

def _distorted(cfg, amp, seed):
    X = _grid_coords(cfg)
    m = cfg["mesh"]
    nx, ny = m["nx"], m["ny"]
    K = oracle.mesh_counts(m)["n_planes"]
    g = np.random.default_rng(seed)
    h = min(m["lx"] / nx, m["ly"] / ny, m["ply_thickness"] / m["elems_per_ply"])
    Xd = X.copy()
    for k in range(1, K - 1):
        for j in range(1, ny):
            for i in range(1, nx):
                n = i + (nx + 1) * (j + (ny + 1) * k)
                Xd[n] += g.uniform(-amp, amp, 3) * h
    return Xd


def _homog_cfg(angle=30.0, n=3):
    mat = _elastic(W.material_cfrp(True, 1e-3))
    cfg = dict(mesh=W._mesh(n, n, n, 1, n * 1e-3, n * 1e-3, 1e-3, [angle] * n, bc=2, gravity=0.0),
               materials=[mat], impactor=W.impactor(4e-3, 1.0, v0=0.0, gap=1.0))
    return cfg


@pytest.mark.parametrize("integration", [1, 8])
def test_patch_test_distorted_large_deformation(integration):
    """A linear displacement field on a distorted mesh leaves interior nodes in
    equilibrium (uniform F, E and S; hourglass forces vanish), with one-point
    and with full integration."""
    cfg = _homog_cfg()
    cfg["mesh"]["integration"] = integration
    Xd = _distorted(cfg, 0.2, 1)
    o = oracle.Oracle(cfg, node_coords=Xd.reshape(-1))
    A = np.array([[0.04, 0.01, -0.02], [0.015, -0.03, 0.01], [0.02, 0.005, 0.05]])
    u = Xd @ A.T + np.array([1e-4, -2e-4, 3e-4])
    o.set(oracle.DISP, u.reshape(-1))
    o.step(0)
    f = o.get(oracle.FINT).reshape(-1, 3)
    m = cfg["mesh"]
    interior = [i + 4 * (j + 4 * k) for k in (1, 2) for j in (1, 2) for i in (1, 2)]
    scale = np.abs(f).max()
    assert scale > 0
    assert np.abs(f[interior]).max() <= 1e-12 * scale
    # equilibrium of the whole body (internal forces sum to zero)
    assert np.abs(f.sum(axis=0)).max() <= 1e-12 * scale


def _one_hex(seed, amp=0.15, h=1e-3):
    g = np.random.default_rng(seed)
    X = np.array([[W_XI, W_ETA, W_ZETA] for W_XI, W_ETA, W_ZETA in
                  zip([-1, 1, 1, -1, -1, 1, 1, -1], [-1, -1, 1, 1, -1, -1, 1, 1],
                      [-1, -1, -1, -1, 1, 1, 1, 1])], dtype=float) * 0.5 * h
    return X + g.uniform(-amp, amp, X.shape) * h


@pytest.mark.parametrize("angle", [0.0, 30.0, 90.0])
def test_element_force_is_energy_gradient(angle):
    """f = dW/du (W = SVK strain energy + hourglass energy), central differences."""
    X = _one_hex(3)
    mat = _elastic(W.material_cfrp(False, 1e-3))
    g = np.random.default_rng(5)
    u = g.uniform(-1, 1, (8, 3)) * 2e-5
    f, _ = oracle.hex8_force_elastic(X, u, mat, angle, 0.05)
    fd = np.zeros(24)
    du = 1e-9
    uf = u.reshape(-1)
    for k in range(24):
        up, um = uf.copy(), uf.copy()
        up[k] += du
        um[k] -= du
        fd[k] = (oracle.hex8_force_elastic(X, up, mat, angle, 0.05)[1]
                 - oracle.hex8_force_elastic(X, um, mat, angle, 0.05)[1]) / (2 * du)
    assert np.abs(fd - f.reshape(-1)).max() <= 1e-6 * np.abs(f).max()


def test_hourglass_energy_gradient_pure_mode():
    """With a pure hourglass mode the stress part is tiny; the force is still the
    gradient of the hourglass energy and is non-zero."""
    X = _one_hex(11, amp=0.0)
    mat = _elastic(W.material_isotropic(70e9, 0.3, 2700.0))
    xi = np.array([-1, 1, 1, -1, -1, 1, 1, -1.0])
    eta = np.array([-1, -1, 1, 1, -1, -1, 1, 1.0])
    zeta = np.array([-1, -1, -1, -1, 1, 1, 1, 1.0])
    u = np.zeros((8, 3))
    u[:, 0] = 1e-6 * xi * eta * zeta
    f0, W0 = oracle.hex8_force_elastic(X, u, mat, 0.0, 0.0)
    f1, W1 = oracle.hex8_force_elastic(X, u, mat, 0.0, 0.05)
    assert np.abs(f0).max() < 1e-6 * np.abs(f1).max()   # 1-point element: zero energy mode
    assert W1 > 0 and np.abs(f1).max() > 0


# ---------------------------------------------------------------------------
# full 2x2x2 Gauss integration (the paper's element)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("angle", [0.0, 30.0])
def test_full_integration_force_is_energy_gradient(angle):
    """f = dW/du with W the sum over the eight Gauss points of det J times the
    SVK energy density (central differences, large strain)."""
    X = _one_hex(7)
    mat = _elastic(W.material_cfrp(False, 1e-3))
    g = np.random.default_rng(9)
    u = g.uniform(-1, 1, (8, 3)) * 1e-4
    f, _ = oracle.hex8_force_elastic_full(X, u, mat, angle)
    fd = np.zeros(24)
    du = 1e-9
    uf = u.reshape(-1)
    for k in range(24):
        up, um = uf.copy(), uf.copy()
        up[k] += du
        um[k] -= du
        fd[k] = (oracle.hex8_force_elastic_full(X, up, mat, angle)[1]
                 - oracle.hex8_force_elastic_full(X, um, mat, angle)[1]) / (2 * du)
    assert np.abs(fd - f.reshape(-1)).max() <= 1e-6 * np.abs(f).max()


def test_full_integration_matches_one_point_on_homogeneous_deformation():
    """A linear displacement field has the same gradient at every Gauss point,
    so both element forms give the same force (the hourglass part vanishes),
    also on a distorted element."""
    X = _one_hex(11)
    mat = _elastic(W.material_cfrp(False, 1e-3))
    A = np.array([[0.03, 0.01, -0.02], [0.015, -0.02, 0.01], [0.02, 0.005, 0.04]])
    u = X @ A.T + np.array([1e-5, 0.0, -2e-5])
    f1, w1 = oracle.hex8_force_elastic(X, u, mat, 30.0, 0.05)
    f8, w8 = oracle.hex8_force_elastic_full(X, u, mat, 30.0)
    assert np.abs(f8 - f1).max() <= 1e-10 * np.abs(f1).max()
    assert abs(w8 - w1) <= 1e-10 * abs(w1)


def _stiffness(force, X, mat, h=1e-9):
    u0 = np.zeros(24)
    K = np.zeros((24, 24))
    for k in range(24):
        up, um = u0.copy(), u0.copy()
        up[k] += h
        um[k] -= h
        K[:, k] = (force(X, up, mat).reshape(-1) - force(X, um, mat).reshape(-1)) / (2 * h)
    return 0.5 * (K + K.T)


def test_full_integration_has_only_rigid_zero_modes():
    """Small-strain stiffness of one element: full integration has exactly the
    six rigid-body zero-energy modes; one point without hourglass control has
    twelve more (the hourglass modes)."""
    X = _one_hex(13, amp=0.1)
    mat = _elastic(W.material_isotropic(70e9, 0.3, 2700.0))
    K8 = _stiffness(lambda X, u, m: oracle.hex8_force_elastic_full(X, u, m, 0.0)[0], X, mat)
    K1 = _stiffness(lambda X, u, m: oracle.hex8_force_elastic(X, u, m, 0.0, 0.0)[0], X, mat)
    for K, zeros in ((K8, 6), (K1, 18)):
        ev = np.sort(np.abs(np.linalg.eigvalsh(K)))
        assert (ev[:zeros] <= 1e-6 * ev[-1]).all()
        assert ev[zeros] > 1e-4 * ev[-1]


def test_full_integration_plate_energy_identity():
    """The energy identity holds with full integration over an impact with
    contact (isotropic plate, clamped edges)."""
    cfg = W.plate_iso_20x20x4()
    cfg["mesh"]["integration"] = 8
    o = oracle.Oracle(cfg)
    o.step(600)
    e = o.energies()
    assert o.history()[1].max() > 0
    assert abs(e["residual"]) <= 1e-6 * e["ke0"]
    assert o.get(oracle.GP_R).size == 4 * 8 * o.ne


def test_rigid_rotation_gives_zero_force():
    X = _one_hex(7)
    mat = _elastic(W.material_cfrp(True, 1e-3))
    ax = np.array([1.0, 2.0, 3.0]) / math.sqrt(14.0)
    th = math.pi / 2
    Kx = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    R = np.eye(3) + math.sin(th) * Kx + (1 - math.cos(th)) * Kx @ Kx
    u = X @ (R - np.eye(3)).T
    f, Wr = oracle.hex8_force_elastic(X, u, mat, 30.0, 0.05)
    fs, _ = oracle.hex8_force_elastic(X, X * 0.01, mat, 30.0, 0.05)
    assert np.abs(f).max() <= 1e-11 * np.abs(fs).max()


def test_mean_gradient_reproduces_linear_fields():
    X = _one_hex(13)
    b, V, gam = oracle.hex8_geometry(X)
    assert np.allclose(X.T @ b, np.eye(3), atol=1e-12)
    assert np.abs(gam @ X).max() < 1e-15 and np.abs(gam.sum(axis=1)).max() < 1e-15


def test_lumped_mass_sums_to_rho_V():
    cfg = _homog_cfg(n=3)
    Xd = _distorted(cfg, 0.25, 2)
    o = oracle.Oracle(cfg, node_coords=Xd.reshape(-1))
    m = o.get(oracle.MASS)
    rho = cfg["materials"][0]["rho"]
    assert abs(m.sum() - rho * 3e-3 * 3e-3 * 3e-3) <= 1e-13 * m.sum()
    assert (m > 0).all()


# ---------------------------------------------------------------------------
# integrator: 1D-strain column dispersion, TW identity, RK4
# ---------------------------------------------------------------------------

def _column(N=40, L=0.02, phi=1.0):
    h = L / N
    mat = W.material_isotropic(70e9, 0.3, 2700.0)
    cfg = dict(mesh=W._mesh(1, 1, 1, N, h, h, L, [0.0], bc=2, gravity=0.0, phi=phi),
               materials=[mat], impactor=W.impactor(1e-3, 1.0, v0=0.0, gap=1.0))
    o = oracle.Oracle(cfg)
    nn = o.nn
    fix = np.zeros((nn, 3))
    fix[:, 0] = fix[:, 1] = 1
    for n in range(nn):
        k = n // 4
        if k == 0 or k == N:
            fix[n, 2] = 1
    o.set(oracle.FIX, fix.reshape(-1))
    return o, cfg, h, mat


def _mode_amp(d, N, L, k):
    z = np.arange(N + 1) * (L / N)
    uz = d.reshape(-1, 3)[:, 2].reshape(N + 1, 4).mean(axis=1)
    s = np.sin(k * math.pi * z / L)
    return (uz @ s) / (s @ s), uz


@pytest.mark.parametrize("k", [1, 7, 39])
def test_column_discrete_dispersion(k):
    """Lumped-mass 1-point hex column in 1D strain = discrete chain:
    omega_k = 2 (c_D/h) sin(k pi / 2N); CD gives u^{n+1} + u^{n-1} = (2 - omega^2 dt^2) u^n."""
    N, L = 40, 0.02
    o, cfg, h, mat = _column(N, L)
    E, nu, rho = 70e9, 0.3, 2700.0
    cD = math.sqrt(E * (1 - nu) / ((1 + nu) * (1 - 2 * nu)) / rho)
    dt = o.dt
    assert abs(dt - 0.9 * h / cD) <= 1e-12 * dt
    A = 1e-5 * L / (k * math.pi)        # peak strain 1e-5: round-off and O(eps^2) both ~1e-10
    z = (np.arange(o.nn) // 4) * (L / N)
    d0 = np.zeros((o.nn, 3))
    d0[:, 2] = A * np.sin(k * math.pi * z / L)
    o.set(oracle.DISP, d0.reshape(-1))
    amps = []
    for n in range(60):
        a, uz = _mode_amp(o.get(oracle.DISP), N, L, k)
        amps.append(a)
        o.step(1)
    amps = np.array(amps)
    om = 2 * cD / h * math.sin(k * math.pi / (2 * N))
    res = amps[2:] + amps[:-2] - (2 - (om * dt) ** 2) * amps[1:-1]
    assert np.abs(res).max() <= 1e-8 * np.abs(amps).max()
    # continuum limit for k = 1, N = 40, L = 20 mm, dt = 0.9 h / c_D
    if k == 1:
        Om = 2 / dt * math.asin(om * dt / 2)
        assert abs(Om - math.pi * cD / L) / (math.pi * cD / L) < 1e-4


def test_tw_phi1_is_central_difference():
    """With phi = 1, d^{n+1} - d^n = dt v^{n+1} (central-difference velocity)."""
    o, cfg, h, mat = _column(10, 0.005)
    d0 = np.zeros((o.nn, 3))
    z = (np.arange(o.nn) // 4) * 0.0005
    d0[:, 2] = 1e-9 * np.sin(3 * math.pi * z / 0.005)
    o.set(oracle.DISP, d0.reshape(-1))
    o.step(1)
    dt = o.dt
    for _ in range(20):
        d_prev = o.get(oracle.DISP)
        o.step(1)
        d, v = o.get(oracle.DISP), o.get(oracle.VEL)
        assert np.abs(d - d_prev - dt * v).max() <= 1e-14 * np.abs(d).max() + 1e-30


def test_tw_phi_above_one_damps_highest_mode():
    """phi = 1.033 (Section 2.2.1) damps the highest-frequency mode; phi = 1 does not."""
    amps = {}
    for phi in (1.0, 1.033):
        o, cfg, h, mat = _column(20, 0.01, phi)
        z = (np.arange(o.nn) // 4) * 0.0005
        d0 = np.zeros((o.nn, 3))
        d0[:, 2] = 1e-10 * np.sin(19 * math.pi * z / 0.01)
        o.set(oracle.DISP, d0.reshape(-1))
        o.step(400)
        e = o.energies()
        amps[phi] = e["ke_plate"] + e["u_el"]
    assert amps[1.033] < 0.5 * amps[1.0]


def test_rk4_constant_force_exact():
    a0 = -9.81 + 123.0
    y = np.array([0.01, -2.0])
    dt = 1e-3
    t = 0.0
    for _ in range(200):
        y = oracle.rk4(lambda tt, yy: np.array([yy[1], a0]), t, y, dt)
        t += dt
    x_ex = 0.01 - 2.0 * t + 0.5 * a0 * t * t
    v_ex = -2.0 + a0 * t
    assert abs(y[0] - x_ex) <= 1e-13 * 1.0 and abs(y[1] - v_ex) <= 1e-12


def test_rk4_fourth_order():
    """Harmonic oscillator: halving dt divides the error by ~16 (k3/3 weight; the
    printed k3/4 makes the weights sum to 11/12 and the method inconsistent)."""
    w = 3.0

    def run(dt):
        y = np.array([1.0, 0.0])
        t = 0.0
        for _ in range(int(round(1.0 / dt))):
            y = oracle.rk4(lambda tt, yy: np.array([yy[1], -w * w * yy[0]]), t, y, dt)
            t += dt
        return abs(y[0] - math.cos(w * 1.0))

    e1, e2 = run(0.005), run(0.0025)
    assert 3.85 < math.log2(e1 / e2) < 4.15


# ---------------------------------------------------------------------------
# intralaminar law (Algorithm 4 reading)
# ---------------------------------------------------------------------------

def _compliance(m):
    """Textbook compliance of a transversely isotropic solid (engineering constants)."""
    S = np.zeros((6, 6))
    S[0, 0], S[1, 1], S[2, 2] = 1 / m["E1"], 1 / m["E2"], 1 / m["E3"]
    S[0, 1] = S[1, 0] = -m["nu12"] / m["E1"]
    S[0, 2] = S[2, 0] = -m["nu13"] / m["E1"]
    S[1, 2] = S[2, 1] = -m["nu23"] / m["E2"]
    S[3, 3], S[4, 4], S[5, 5] = 1 / m["G23"], 1 / m["G13"], 1 / m["G12"]
    return S


def test_cdm_undamaged_is_inverse_compliance():
    m = W.material_cfrp(False, 0.5e-3)
    S = _compliance(m)
    Cm = np.zeros((6, 6))
    for j in range(6):
        e = np.zeros(6)
        e[j] = 1e-7
        sig, r, d = oracle.cdm(m, 1e-4, e, np.ones(4))
        Cm[:, j] = sig / 1e-7
        assert (r == 1).all() and (d == 0).all()
    assert np.abs(Cm @ S - np.eye(6)).max() < 1e-12


LC3 = (0.125e-3 * 0.125e-3 * 0.25e-3) ** (1 / 3)


@pytest.mark.parametrize("mode,sgn,strength", [(0, 1, "XT"), (0, -1, "XC"), (1, 1, "YT"),
                                               (1, -1, "YC"), (5, 1, "SL")])
def test_cdm_peak_stress_uniaxial(mode, sgn, strength):
    """Uniaxial-stress / pure-shear paths: the peak stress equals the strength
    (onset at d = 0, where effective and nominal stress coincide)."""
    m = W.material_cfrp(True, 0.5e-3)
    X = m[strength]
    S = _compliance(m)
    r = np.ones(4)
    peak = 0.0
    for s in np.concatenate([np.linspace(0, 1, 201)[1:], 1 + np.linspace(0, 0.3, 61)[1:]]):
        sv = np.zeros(6)
        sv[mode] = sgn * s * X
        sig, r, d = oracle.cdm(m, LC3, S @ sv, r)
        peak = max(peak, sgn * sig[mode])
    assert abs(peak - X) <= 1e-9 * X


def _nu0(m):
    m = dict(m)
    m["nu12"] = m["nu13"] = m["nu23"] = 0.0
    return m


@pytest.mark.parametrize("mode,sgn,G,n", [(0, 1, "GXT", 400000), (0, -1, "GXC", 400000),
                                          (1, 1, "GYT", 400000), (1, -1, "GYC", 400000),
                                          (5, 1, "GSL", 400000)])
def test_cdm_dissipated_energy_crack_band(mode, sgn, G, n):
    """Monotonic strain path to full failure dissipates G / l_c per unit volume
    (crack band; exact with zero Poisson coupling)."""
    m = _nu0(W.material_cfrp(True, 0.5e-3))
    lc = LC3
    E = {0: m["E1"], 1: m["E2"], 5: m["G12"]}[mode]
    Xs = {("GXT"): m["XT"], "GXC": m["XC"], "GYT": m["YT"], "GYC": m["YC"], "GSL": m["SL"]}[G]
    e0 = Xs / E
    emax = e0 * (60.0 if mode != 0 else 1.0)
    if mode == 0:
        g = m[G] / lc
        fX = m["fXT"] if sgn > 0 else m["fXC"]
        fG = m["fGT"] if sgn > 0 else m["fGC"]
        emax = 1.05 * 2 * (1 - fG) * g / (fX * Xs)
    else:
        A = 2 * lc * Xs * Xs / (2 * E * m[G] - lc * Xs * Xs)
        emax = e0 * (1 + 45.0 / A) * 1.2
    es = np.linspace(0, emax, n)
    r = np.ones(4)
    sig = np.zeros(n)
    idx = {(0, 1): 0, (0, -1): 1, (1, 1): 2, (1, -1): 3, (5, 1): 4}[(mode, sgn)]
    stop = n
    for k, e in enumerate(es):
        eps = np.zeros(6)
        eps[mode] = sgn * e
        s, r, d = oracle.cdm(m, lc, eps, r)
        sig[k] = sgn * s[mode]
        if d[idx] >= 1.0 - 1.0000001e-6:     # saturated: only the residual stiffness is left
            stop = k + 1
            break
    work = np.trapezoid(sig[:stop], es[:stop])
    assert abs(work - m[G] / lc) <= 2e-5 * m[G] / lc


def test_cdm_irreversible_secant_unloading():
    m = _nu0(W.material_cfrp(False, 0.5e-3))
    e0 = m["YT"] / m["E2"]
    path = np.concatenate([np.linspace(0, 2 * e0, 50), np.linspace(2 * e0, 0, 50),
                           np.linspace(0, 3 * e0, 50), np.linspace(3 * e0, 0.5 * e0, 50)])
    r = np.ones(4)
    rs, secant = [], []
    for e in path:
        eps = np.zeros(6)
        eps[1] = e
        s, r, d = oracle.cdm(m, LC3, eps, r)
        rs.append(r.copy())
        secant.append(s[1] / e if e > 0 else np.nan)
    rs = np.array(rs)
    assert (np.diff(rs, axis=0) >= 0).all()
    un = np.array(secant[51:99])
    assert np.nanmax(np.abs(un - un[0])) <= 1e-12 * abs(un[0])


def test_cdm_closed_strain_cycle_returns_no_energy():
    """Second law (the model is thermodynamically consistent, Section 2.3.1):
    after matrix damage in transverse tension, a closed cycle in
    (eps22, gamma23) that opens the crack, shears it, closes it and unshears
    it, with no new damage, returns no energy: the net work of the stress
    around the cycle is not negative (here it is zero, the cycle is elastic).
    A shear stiffness that followed the crack-closure switch would give
    -d2+ G23 gamma^2 / 2."""
    m = W.material_cfrp(False, 0.5e-3)
    e0 = m["YT"] / m["E2"]
    r = np.ones(4)
    for e in np.concatenate([np.linspace(0, 3 * e0, 300), np.linspace(3 * e0, 0, 300)]):
        eps = np.zeros(6)
        eps[1] = e
        _, r, d = oracle.cdm(m, LC3, eps, r)
    assert d[2] > 0.3 and d[3] == 0.0                   # tensile matrix damage only
    a, g = 0.5 * e0, 0.5 * m["SL"] / m["G23"]
    corners = [(0.0, 0.0), (a, 0.0), (a, g), (-a, g), (-a, 0.0), (0.0, 0.0)]
    t = np.linspace(0.0, 1.0, 2001)
    path = np.concatenate([np.stack([p + (u - p) * t, q + (v - q) * t], 1)
                           for (p, q), (u, v) in zip(corners[:-1], corners[1:])])
    sig = np.zeros_like(path)
    for k, (e22, g23) in enumerate(path):
        eps = np.zeros(6)
        eps[1], eps[3] = e22, g23
        s, r2, _ = oracle.cdm(m, LC3, eps, r)
        assert (r2 == r).all()                          # no new damage on the cycle
        sig[k] = s[1], s[3]
    work = float(np.sum(0.5 * (sig[1:] + sig[:-1]) * np.diff(path, axis=0)))
    scale = 0.5 * m["G23"] * g * g
    assert work >= -1e-9 * scale
    assert abs(work) <= 1e-6 * scale


# ---------------------------------------------------------------------------
# matrix compression with shear: the fracture-plane criteria (LaRC reading)
# ---------------------------------------------------------------------------

def _mohr_coulomb_plane(m):
    """Friction coefficient eta_T and transverse shear strength S_T of the
    fracture plane, found numerically from their definition: under uniaxial
    transverse compression Y_C the Mohr-Coulomb effective shear
    tau_T + eta_T sigma_n on a plane at angle a (sigma_n = -Y_C cos^2 a,
    tau_T = Y_C sin a cos a) is largest on the fracture plane a0 of Table 1,
    and its value there is S_T.  The longitudinal coefficient follows from
    the same friction per unit strength: eta_L / S_L = eta_T / S_T."""
    from scipy.optimize import brentq, minimize_scalar
    a0 = math.radians(m["alpha0_deg"])

    def argmax(eta):
        r = minimize_scalar(lambda a: -(math.sin(a) * math.cos(a) - eta * math.cos(a) ** 2),
                            bounds=(0.0, 0.5 * math.pi), method="bounded",
                            options=dict(xatol=1e-14))
        return r.x

    eta_t = brentq(lambda e: argmax(e) - a0, 1e-6, 10.0, xtol=1e-15)
    s_t = m["YC"] * (math.sin(a0) * math.cos(a0) - eta_t * math.cos(a0) ** 2)
    return eta_t, s_t, eta_t * m["SL"] / s_t


def _sigma_to_strain(m, s22, t12, t13=0.0):
    """Strain whose effective (undamaged) stress is sigma22 = s22, tau12 = t12,
    tau13 = t13, all other components zero."""
    sv = np.zeros(6)
    sv[1], sv[4], sv[5] = s22, t13, t12
    return _compliance(m) @ sv


def _onset_shear(m, s22, hi):
    """In-plane shear stress at which the matrix threshold r2+ first grows at
    a fixed transverse stress s22 (bisection on the law's own verdict)."""
    lo = 0.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        _, r, _ = oracle.cdm(m, LC3, _sigma_to_strain(m, s22, mid), np.ones(4))
        if r[2] > 1.0:
            hi = mid
        else:
            lo = mid
        if hi - lo <= 1e-15 * hi:
            break
    _, r, _ = oracle.cdm(m, LC3, _sigma_to_strain(m, s22, hi), np.ones(4))
    assert r[3] == 1.0            # the tensile/shear criterion, not the compressive one, set in
    return hi


@pytest.mark.parametrize("outer", [True, False])
def test_cdm_compression_shear_onset_line(outer):
    """Under transverse compression the matrix shear criterion is of the
    Mohr-Coulomb kind: damage sets in where tau_L = S_L - eta_L sigma22,
    with eta_L fixed by the fracture plane (Table 1's alpha0).  The onset
    shear stress is continuous at sigma22 = 0 (where both branches give S_L)
    and grows with compression."""
    m = W.material_cfrp(outer, 0.5e-3)
    _, _, eta_l = _mohr_coulomb_plane(m)
    assert eta_l > 0
    S_L = m["SL"]
    assert abs(_onset_shear(m, 1e-9 * S_L, 2 * S_L) - S_L) <= 1e-9 * S_L
    assert abs(_onset_shear(m, -1e-9 * S_L, 2 * S_L) - S_L) <= 1e-9 * S_L
    prev = S_L
    for f in (0.1, 0.25, 0.45):
        s22 = -f * m["YC"]
        tau = _onset_shear(m, s22, 3 * S_L)
        assert abs(tau - (S_L - eta_l * s22)) <= 1e-9 * S_L, (f, tau)
        assert tau > prev
        prev = tau
    # at a fixed shear stress the tensile-branch loading function falls as
    # compression grows (r2+ reached on the path is smaller)
    rs = []
    for f in (0.0, 0.1, 0.3):
        _, r, _ = oracle.cdm(m, LC3, _sigma_to_strain(m, -f * m["YC"], 1.3 * S_L), np.ones(4))
        rs.append(r[2])
    assert rs[0] > rs[1] > rs[2]


def _fracture_plane_phi(m, s22, t12):
    """Compressive matrix loading function from the tractions on the fracture
    plane, computed with the stress tensor: the plane through the fibre axis
    (material 1) whose normal is tilted by alpha0 from direction 2 towards 3
    carries the normal traction sigma_n and the shear traction, whose
    transverse and longitudinal components are tau_T and tau_L at the angle
    theta = atan2(tau_L, tau_T); Mohr-Coulomb friction reduces each component
    by eta sigma_n along it."""
    eta_t, s_t, eta_l = _mohr_coulomb_plane(m)
    a0 = math.radians(m["alpha0_deg"])
    sig = np.array([[0.0, t12, 0.0], [t12, s22, 0.0], [0.0, 0.0, 0.0]])
    n = np.array([0.0, math.cos(a0), math.sin(a0)])
    e_l = np.array([1.0, 0.0, 0.0])
    e_t = np.cross(n, e_l)
    e_t *= np.sign(e_t @ (sig @ n)) if abs(e_t @ (sig @ n)) > 0 else 1.0
    tr = sig @ n
    s_n = n @ tr
    tau_t, tau_l = e_t @ tr, abs(e_l @ tr)
    th = math.atan2(tau_l, tau_t)
    te = max(tau_t + eta_t * s_n * math.cos(th), 0.0)
    le = max(tau_l + eta_l * s_n * math.sin(th), 0.0)
    return math.hypot(te / s_t, le / m["SL"])


@pytest.mark.parametrize("outer", [True, False])
@pytest.mark.parametrize("f22,f12", [(1.1, 0.0), (1.2, 0.6), (1.1, 0.3), (0.9, 1.3), (0.8, 1.5)])
def test_cdm_compressive_matrix_criterion_off_axis(outer, f22, f12):
    """The compressive matrix threshold r2- after one update from the
    undamaged state equals the fracture-plane loading function computed from
    the stress tensor's tractions (points with both normal and longitudinal
    shear stress, beyond onset so that r2- = phi2-)."""
    m = W.material_cfrp(outer, 0.5e-3)
    s22, t12 = -f22 * m["YC"], f12 * m["SL"]
    want = _fracture_plane_phi(m, s22, t12)
    assert want > 1.02
    _, r, _ = oracle.cdm(m, LC3, _sigma_to_strain(m, s22, t12), np.ones(4))
    assert abs(r[3] - want) <= 1e-9 * want, (r, want)
    assert r[2] >= r[3]


def test_cdm_uniaxial_compression_fracture_plane_is_alpha0():
    """Under pure transverse compression the fracture-plane loading function
    reaches 1 exactly at Y_C (the plane's strength S_T reproduces Y_C), and
    the oracle's threshold agrees beyond it."""
    m = W.material_cfrp(True, 0.5e-3)
    assert abs(_fracture_plane_phi(m, -m["YC"], 0.0) - 1.0) <= 1e-12
    _, r, _ = oracle.cdm(m, LC3, _sigma_to_strain(m, -1.3 * m["YC"], 0.0), np.ones(4))
    assert abs(r[3] - _fracture_plane_phi(m, -1.3 * m["YC"], 0.0)) <= 1e-9


# ---------------------------------------------------------------------------
# longitudinal shear plasticity (Algorithm 4, first two lines; Table 1 S_p, K_p)
# ---------------------------------------------------------------------------

def _plastic_mat(outer=True):
    m = W.material_cfrp(outer, 0.5e-3, plastic=True)
    assert m["Sp"] == 62.0e6 and m["Kp"] == 0.1936 and m["G13"] == m["G12"]
    return m


def _shear_path(m, gammas, direction=(1.0, 0.0)):
    """Strain path of longitudinal shear gamma along (gamma12, gamma13) =
    gamma * direction; returns tau_L along the direction, the states."""
    r, ep = np.ones(4), np.zeros(3)
    taus, eps_p, rs = [], [], []
    c, s_ = direction
    for g in gammas:
        e = np.zeros(6)
        e[5], e[4] = c * g, s_ * g
        sig, r, ep, _ = oracle.cdm_plastic(m, LC3, e, r, ep)
        taus.append(c * sig[5] + s_ * sig[4])
        eps_p.append(ep.copy())
        rs.append(r.copy())
    return np.array(taus), np.array(eps_p), np.array(rs)


def test_plastic_shear_yields_at_Sp_and_hardens_linearly():
    """Monotone in-plane shear below damage onset: elastic slope G12 up to the
    yield stress S_p, then tau = S_p + H gamma_p with gamma_p growing as
    (G12 gamma - S_p) / (G12 + H), H = K_p G12 (linear isotropic hardening),
    i.e. the tangent G12 H / (G12 + H); the accumulated plastic shear equals
    gamma_p on a monotone path; no damage."""
    m = _plastic_mat()
    G, H, Sp = m["G12"], m["Kp"] * m["G12"], m["Sp"]
    g_top = (0.9 * m["SL"] - Sp) / H + 0.9 * m["SL"] / G         # tau reaches 0.9 S_L
    gam = np.linspace(0.0, g_top, 801)[1:]
    tau, ep, rs = _shear_path(m, gam)
    el = gam <= Sp / G
    assert el.sum() > 50 and (~el).sum() > 50
    assert np.allclose(tau[el], G * gam[el], rtol=1e-13, atol=0)
    assert (ep[el] == 0).all()
    want = Sp + (G * gam[~el] - Sp) * H / (G + H)
    assert np.abs(tau[~el] - want).max() <= 1e-11 * Sp
    gp = (G * gam[~el] - Sp) / (G + H)
    assert np.abs(ep[~el, 0] - gp).max() <= 1e-12 * gp.max()
    assert np.abs(ep[~el, 2] - ep[~el, 0]).max() <= 1e-15 * gp.max()
    assert (ep[:, 1] == 0).all() and (rs == 1).all()
    assert tau.max() < m["SL"]


def test_plastic_unloading_keeps_plastic_strain_and_reverse_yield_is_isotropic():
    """Load past yield, unload: the slope is G12, no further plastic strain,
    and the stress vanishes at gamma = gamma_p (the plastic strain is kept).
    Reverse loading yields at -(S_p + H abar) (isotropic hardening)."""
    m = _plastic_mat()
    G, H, Sp = m["G12"], m["Kp"] * m["G12"], m["Sp"]
    g1 = 0.02
    up = np.linspace(0.0, g1, 401)[1:]
    tau_up, ep_up, _ = _shear_path(m, up)
    gp1, t1 = ep_up[-1, 0], tau_up[-1]
    assert gp1 > 0 and abs(t1 - (Sp + H * gp1)) <= 1e-11 * Sp
    r, ep = np.ones(4), ep_up[-1].copy()
    # unload to zero stress (gamma = gamma_p) and on to just before reverse yield
    g_rev = gp1 - (Sp + H * gp1) / G
    down = np.linspace(g1, g_rev * 0.999 + gp1 * 0.001, 400)
    for g in down:
        e = np.zeros(6)
        e[5] = g
        sig, r, ep2, _ = oracle.cdm_plastic(m, LC3, e, r, ep)
        assert np.array_equal(ep2, ep)                           # elastic unloading
        assert abs(sig[5] - G * (g - gp1)) <= 1e-9 * Sp
    e = np.zeros(6)
    e[5] = gp1
    sig, _, _, _ = oracle.cdm_plastic(m, LC3, e, r, ep)
    assert abs(sig[5]) <= 1e-9 * Sp                              # zero stress at gamma = gamma_p
    # reverse: yields at -(S_p + H abar)
    e[5] = g_rev * 1.001 - gp1 * 0.001
    sig, _, ep3, _ = oracle.cdm_plastic(m, LC3, e, r, ep)
    assert ep3[0] < gp1 and ep3[2] > ep[2]
    assert abs(sig[5] + (Sp + H * ep3[2])) <= 1e-9 * Sp


def test_plastic_dissipation_of_a_load_unload_cycle():
    """Loading to gamma_1 and unloading to zero stress dissipates
    S_p gamma_p + H gamma_p^2 / 2 per unit volume (the work of the yield
    stress on the plastic strain); the elastic energy is recovered."""
    m = _plastic_mat()
    G, H, Sp = m["G12"], m["Kp"] * m["G12"], m["Sp"]
    g1 = 0.025
    up = np.linspace(0.0, g1, 20001)
    tau_up, ep_up, _ = _shear_path(m, up)
    gp = ep_up[-1, 0]
    down = np.linspace(g1, gp, 2001)
    r, ep = np.ones(4), ep_up[-1].copy()
    tau_dn = []
    for g in down:
        e = np.zeros(6)
        e[5] = g
        sig, r, ep, _ = oracle.cdm_plastic(m, LC3, e, r, ep)
        tau_dn.append(sig[5])
    work = np.trapezoid(tau_up, up) + np.trapezoid(np.array(tau_dn), down)
    want = Sp * gp + 0.5 * H * gp * gp
    assert abs(work - want) <= 1e-6 * want


def test_plastic_shear_plane_is_isotropic():
    """G13 = G12: longitudinal shear along any direction of the (12, 13)
    plane follows the same tau_L - gamma_L curve, and the plastic strain is
    along the loading direction."""
    m = _plastic_mat()
    gam = np.linspace(0.0, 0.03, 301)[1:]
    t0, ep0, _ = _shear_path(m, gam)
    for beta in (0.4, 1.1, 2.5):
        d = (math.cos(beta), math.sin(beta))
        t, ep, _ = _shear_path(m, gam, d)
        assert np.abs(t - t0).max() <= 1e-12 * m["Sp"]
        assert np.abs(ep[:, 0] - d[0] * ep0[:, 0]).max() <= 1e-14 and np.abs(ep[:, 1] - d[1] * ep0[:, 0]).max() <= 1e-14
        assert np.abs(ep[:, 2] - ep0[:, 2]).max() <= 1e-14


def test_plastic_strain_comes_before_the_damage_criteria():
    """Algorithm 4's order: plastic strains, elastic strains, effective stress,
    criteria.  Under pure shear the shear criterion sees the effective stress
    of the elastic strain, so damage sets in at the total strain
    S_L / G12 + (S_L - S_p) / H (the hardening has lifted the stress to S_L),
    not at S_L / G12."""
    m = _plastic_mat()
    G, H, Sp, SL = m["G12"], m["Kp"] * m["G12"], m["Sp"], m["SL"]
    want = SL / G + (SL - Sp) / H
    lo, hi = 0.5 * want, 1.5 * want
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        n = 64
        tau, ep, rs = _shear_path(m, np.linspace(0.0, mid, n + 1)[1:])
        if rs[-1, 2] > 1.0:
            hi = mid
        else:
            lo = mid
        if hi - lo <= 1e-13 * want:
            break
    assert abs(hi - want) <= 1e-9 * want


def test_plasticity_off_is_the_elastic_damage_law():
    """With S_p = 0 the law is the elastic-damage law exactly, and with
    plasticity on, strains below yield give the same answers bit for bit."""
    m0 = W.material_cfrp(True, 0.5e-3)
    mp = _plastic_mat()
    rs = np.random.default_rng(31)
    for _ in range(300):
        e = rs.standard_normal(6) * np.array([4e-3, 6e-3, 4e-3, 8e-3, 8e-3, 8e-3]) * rs.uniform(0.05, 2.0)
        r0 = 1.0 + rs.uniform(0.0, 0.5, 4) * (rs.uniform() < 0.5)
        a = oracle.cdm(m0, LC3, e, r0)
        b = oracle.cdm_plastic(m0, LC3, e, r0, np.zeros(3))
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and (b[2] == 0).all()
        tL = m0["G12"] * math.hypot(e[4], e[5])
        if tL < mp["Sp"]:
            c = oracle.cdm_plastic(mp, LC3, e, r0, np.zeros(3))
            assert np.array_equal(a[0], c[0]) and (c[2] == 0).all()


@pytest.mark.parametrize("integration", [1, 8])
def test_plastic_plate_energy_identity(integration):
    """A small laminate struck hard enough to yield in shear, with one-point
    or fully integrated elements: the energy identity closes to 1e-6 of the
    impact energy, the plastic strains are non-zero, and the dissipated work
    W_int - U_el (U_el: energy of the elastic strains) is non-negative and
    grows."""
    cfg = W.tiny(8, 8, 4, 1, angles=[0, 45, -45, 90], law=W.LAW_CDM, lx=8e-3, ly=8e-3,
                 ply_thickness=0.25e-3, v0=12.0, mass=0.05, R=3e-3, plastic=True)
    cfg["mesh"]["integration"] = integration
    o = oracle.Oracle(cfg)
    dis = []
    for _ in range(6):
        o.step(100)
        e = o.energies()
        assert abs(e["residual"]) <= 1e-6 * e["ke0"]
        dis.append(e["w_int"] - e["u_el"])
    ep = o.get(oracle.GP_EP).reshape(-1, 3)
    assert ep[:, 2].max() > 0
    assert min(dis) >= -1e-9 * o.energies()["ke0"]
    assert dis[-1] > dis[0]


def test_velocity_carries_several_times_the_relative_difference_of_displacement():
    """Why the FP64 parity tests hold the velocity to ten times the
    displacement's bar: the velocity is a one-step difference quotient of
    displacements, so the same perturbation shows up several times larger
    in it, relative to its size.  Two oracle runs of the damaged 12 x 12 x 4
    parity plate whose striker speeds differ by 1e-14 (relative), 300 and
    400 steps."""
    cfg = W.tiny(12, 12, 4, 1, angles=[0, 90, 0, 90], law=W.LAW_CDM, lx=12e-3, ly=12e-3,
                 ply_thickness=0.5e-3, v0=20.0, mass=0.02, R=4e-3)
    a = oracle.Oracle(cfg)
    c2 = W.tiny(12, 12, 4, 1, angles=[0, 90, 0, 90], law=W.LAW_CDM, lx=12e-3, ly=12e-3,
                ply_thickness=0.5e-3, v0=20.0 * (1 + 1e-14), mass=0.02, R=4e-3)
    b = oracle.Oracle(c2)
    ratios = []
    for n in (300, 100):
        a.step(n)
        b.step(n)
        da, db = a.get(oracle.DISP), b.get(oracle.DISP)
        va, vb = a.get(oracle.VEL), b.get(oracle.VEL)
        rd = np.abs(db - da).max() / np.abs(da).max()
        rv = np.abs(vb - va).max() / np.abs(va).max()
        assert rd > 0
        ratios.append(rv / rd)
    assert min(ratios) >= 3.0, ratios


@pytest.mark.parametrize("angle", [0.0, 30.0])
def test_plastic_state_of_every_gauss_point_under_homogeneous_shear(angle):
    """A free one-ply plate given the displacement of a uniform in-plane
    simple shear beyond yield, u_x = gamma y, and its forces evaluated once
    at that configuration (a zero-step call re-initialises the level): every
    element, with one point or with 2x2x2 Gauss points, sees the same Green
    strain E = (G + G^T + G^T G)/2, so the plastic state of every point is
    the return map of that strain in the ply frame (the law called alone,
    from zero).  Pins where the plate keeps the state of each point.  (A
    step after it would move the free edges, whose tractions are not
    balanced, and the edge elements would flow further.)"""
    gam = 0.03
    th = math.radians(angle)
    c, s_ = math.cos(th), math.sin(th)
    E00, E01, E11 = 0.0, 0.5 * gam, 0.5 * gam * gam
    e = np.zeros(6)
    e[0] = c * c * E00 + 2 * c * s_ * E01 + s_ * s_ * E11
    e[1] = s_ * s_ * E00 - 2 * c * s_ * E01 + c * c * E11
    e[5] = 2 * (-c * s_ * E00 + (c * c - s_ * s_) * E01 + c * s_ * E11)
    states = {}
    for ngp in (1, 8):
        cfg = W.tiny(3, 3, 1, 1, angles=[angle], law=W.LAW_CDM, ply_thickness=0.5e-3, bc=W.BC_FREE,
                     v0=0.0, gravity=0.0, plastic=True)
        cfg["impactor"]["gap"] = 1.0
        cfg["mesh"]["integration"] = ngp
        m = cfg["mesh"]
        o = oracle.Oracle(cfg)
        o.step(1)
        nn = o.nn
        k = np.arange(nn)
        j = (k // (m["nx"] + 1)) % (m["ny"] + 1)
        d = np.zeros((nn, 3))
        d[:, 0] = gam * m["ly"] * j / m["ny"]
        o.set(oracle.DISP, d.reshape(-1))
        o.step(0)
        states[ngp] = o.get(oracle.GP_EP).reshape(-1, 3)
        assert len(states[ngp]) == ngp * o.ne
    mat = W.tiny(1, 1, 1, 1, law=W.LAW_CDM, plastic=True)["materials"][0]
    _, _, ep, _ = oracle.cdm_plastic(mat, 1e-3, e, np.ones(4), np.zeros(3))
    assert ep[2] > 1e-3                                     # the strain is beyond yield
    for ngp, st in states.items():
        assert np.abs(st - ep).max() <= 1e-9 * ep[2], ngp


def test_plasticity_needs_an_isotropic_shear_plane():
    cfg = W.tiny(2, 2, 1, 1, law=W.LAW_CDM, plastic=True)
    cfg["materials"][0]["G13"] = 0.9 * cfg["materials"][0]["G12"]
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(cfg)


# ---------------------------------------------------------------------------
# cohesive law (Algorithm 5 reading)
# ---------------------------------------------------------------------------

def _path_work(m, direction, smax, n=200000):
    r = 0.0
    ss = np.linspace(0, smax, n)
    taus = np.zeros((n, 3))
    for k, s in enumerate(ss):
        tau, r, D = oracle.czm(m, s * np.asarray(direction), r)
        taus[k] = tau
    work = np.trapezoid(taus @ np.asarray(direction), ss)
    return work, taus, ss


def test_czm_mode_I_peak_and_toughness():
    m = W.material_cfrp(True, 0.5e-3)
    do = m["tauI"] / m["KI"]
    tau, r, D = oracle.czm(m, [0, 0, do], 0.0)
    assert abs(tau[2] - m["tauI"]) <= 1e-12 * m["tauI"] and D == 0
    dc = 2 * m["GIc"] / m["tauI"]
    work, taus, ss = _path_work(m, [0, 0, 1], 1.5 * dc)
    assert abs(work - m["GIc"]) <= 1e-4 * m["GIc"]
    assert abs(taus[-1, 2]) < 1e-6 * m["tauI"]      # no tensile traction after D = 1


def test_czm_mode_II_toughness_and_peak():
    m = W.material_cfrp(True, 0.5e-3)
    dc = 2 * m["GIIc"] / m["tauII"]
    work, taus, ss = _path_work(m, [1, 0, 0], 1.5 * dc)
    assert abs(work - m["GIIc"]) <= 1e-4 * m["GIIc"]
    assert abs(taus[:, 0].max() - m["tauII"]) <= 1e-3 * m["tauII"]


@pytest.mark.parametrize("a,b", [(1.0, 1.0), (0.3, 1.0), (1.0, 0.2)])
def test_czm_mixed_mode_bk_toughness(a, b):
    """Proportional mixed-mode opening dissipates the Benzeggagh-Kenane toughness."""
    m = W.material_cfrp(True, 0.5e-3)
    Ksh = m["KI"] * (m["GIc"] / m["GIIc"]) * (m["tauII"] / m["tauI"]) ** 2
    n = np.array([a, 0.0, b]) / math.hypot(a, b)
    B = Ksh * n[0] ** 2 / (Ksh * n[0] ** 2 + m["KI"] * n[2] ** 2)
    Gc = m["GIc"] + (m["GIIc"] - m["GIc"]) * B ** m["eta_bk"]
    smax = 3 * 2 * m["GIIc"] / m["tauI"]
    work, taus, ss = _path_work(m, n, smax)
    assert abs(work - Gc) <= 2e-4 * Gc


def _screen_constants(m, lc_min, lc_max):
    """The GPU screen's per-ply constants (strengths capped at the largest crack
    band, eta_L of largest magnitude over the range, a 1e-5 margin)."""
    def capped(X, E, G, lc):
        lim = 1.8 * E * G / lc
        return math.sqrt(lim) if X * X > lim else X
    a0 = math.radians(m["alpha0_deg"])
    kst = math.cos(a0) * (math.sin(a0) + math.cos(a0) / math.tan(2 * a0))
    etat = -1.0 / math.tan(2 * a0)
    kel = -math.cos(2 * a0) / math.cos(a0) ** 2
    mg, lhi, llo = 1 + 1e-5, lc_max * (1 + 1e-6), lc_min * (1 - 1e-6)
    cands = [llo, lhi, 1.8 * m["G12"] * m["GSL"] / m["SL"] ** 2, 1.8 * m["E2"] * m["GYC"] / m["YC"] ** 2]
    rmax = max(capped(m["SL"], m["G12"], m["GSL"], lc) / capped(m["YC"], m["E2"], m["GYC"], lc)
               for lc in cands if llo <= lc <= lhi)
    return dict(kXT=mg * m["E1"] / m["XT"], kXC=mg * m["E1"] / m["XC"],
                iYT=mg / capped(m["YT"], m["E2"], m["GYT"], lhi), iSL=mg / capped(m["SL"], m["G12"], m["GSL"], lhi),
                iST=mg / (kst * capped(m["YC"], m["E2"], m["GYC"], lhi)), etaL=mg * kel * rmax,
                kT=math.cos(a0) * (math.sin(a0) + abs(etat) * math.cos(a0)), ca0=math.cos(a0))


@pytest.mark.parametrize("outer", [True, False])
def test_elastic_screen_bounds_hold_over_the_crack_band_range(outer):
    """The GPU's elastic screen passes a point only when the law leaves it
    undamaged: with constants derived for the ply's largest crack band, every
    screened strain stays below onset in the oracle's law at every crack band
    of the range (where the caps lower the matrix strengths differently)."""
    m = W.material_cfrp(outer, 0.25e-3)
    S = np.array([[1 / m["E1"], -m["nu12"] / m["E1"], -m["nu13"] / m["E1"]],
                  [-m["nu12"] / m["E1"], 1 / m["E2"], -m["nu23"] / m["E2"]],
                  [-m["nu13"] / m["E1"], -m["nu23"] / m["E2"], 1 / m["E3"]]])
    C = np.linalg.inv(S)
    lc_min, lc_max = 0.3e-3, 1.6e-3                 # spans the onset of the caps (about 0.47 mm)
    k = _screen_constants(m, lc_min, lc_max)
    rs = np.random.default_rng(23)
    screened = 0
    for _ in range(3000):
        e = rs.standard_normal(6) * np.array([4e-3, 6e-3, 4e-3, 8e-3, 8e-3, 8e-3]) * rs.uniform(0.05, 1.0)
        s1 = C[1] @ e[:3]
        t2 = (m["G12"] * e[5]) ** 2 + (m["G13"] * e[4]) ** 2
        grow = max(e[0], 0) * k["kXT"] > 1 or max(-e[0], 0) * k["kXC"] > 1
        if s1 >= 0:
            grow |= (s1 * k["iYT"]) ** 2 + t2 * k["iSL"] ** 2 > 1
        else:
            el = k["etaL"] * s1
            qL = 2 * (t2 + el * el) if el > 0 else t2
            grow |= qL * k["iSL"] ** 2 > 1
            bT = -s1 * k["kT"] * k["iST"]
            qL2 = 2 * k["ca0"] ** 2 * (t2 + (el * k["ca0"]) ** 2)
            grow |= bT * bT + qL2 * k["iSL"] ** 2 > 1
        if grow:
            continue
        screened += 1
        for lc in (lc_min, 0.47e-3, 0.8e-3, lc_max, rs.uniform(lc_min, lc_max)):
            sig, r, dmg = oracle.cdm(m, lc, e, np.ones(4))
            assert np.all(r == 1.0) and np.all(dmg == 0.0), (e, lc, r)
    assert screened > 500


def test_czm_no_onset_below_the_smallest_onset_opening():
    """An undamaged pair with Ksh |d_sh|^2 + KI <d3>^2 <= 2 GIo min(GIc, GIIc) / GIc
    (GIo = tau_I^2 / 2 KI) is below onset at every mode mixity: the law leaves it
    undamaged with tractions K d (the bound the GPU's cohesive screen uses).
    Just above the bound, the mixity with the smallest toughness starts to
    damage, so the bound is the tightest of its form."""
    m = W.material_cfrp(True, 0.5e-3)
    KI = m["KI"]
    Ksh = KI * (m["GIc"] / m["GIIc"]) * (m["tauII"] / m["tauI"]) ** 2
    GIo = m["tauI"] ** 2 / (2 * KI)
    bound = 2 * GIo * min(m["GIc"], m["GIIc"]) / m["GIc"]
    rs = np.random.default_rng(17)
    for _ in range(400):
        n = rs.standard_normal(3)
        n /= np.linalg.norm(n)
        den1 = Ksh * (n[0] ** 2 + n[1] ** 2) + KI * max(n[2], 0.0) ** 2
        if den1 <= 0:
            continue
        d = n * math.sqrt(bound * (1 - 1e-6) / den1)
        tau, r, D = oracle.czm(m, d, 0.0)
        assert r == 0.0 and D == 0.0
        assert np.allclose(tau, [Ksh * d[0], Ksh * d[1], KI * d[2]], rtol=1e-14, atol=0)
    # the mixity of smallest toughness (pure mode I here: GIc < GIIc) damages just above it
    assert m["GIc"] < m["GIIc"]
    tau, r, D = oracle.czm(m, [0.0, 0.0, math.sqrt(bound * 1.001 / KI)], 0.0)
    assert r > 0.0


def test_czm_compression_is_penalty_contact():
    m = W.material_cfrp(True, 0.5e-3)
    tau, r, D = oracle.czm(m, [0, 0, 1.0], 0.0)            # fully broken in tension
    assert r == 1.0
    tau, r2, D = oracle.czm(m, [0, 0, -1e-7], r)
    assert abs(tau[2] - m["KI"] * -1e-7) <= 1e-12 * abs(tau[2])


def test_czm_t800_equal_penalties_table1():
    """Table 1 T800S/M21 interface strengths were set (footnote d) so that the
    shear and normal penalties coincide: K_sh/K_I = (G_Ic/G_IIc)(tau_II/tau_I)^2 = 1."""
    g = json.load(open(os.path.join(GOLD, "table1_t800_interface.json")))
    m = W.material_cfrp(True, 0.5e-3)
    m.update(tauI=g["tauI_MPa"] * 1e6, tauII=g["tauII_MPa"] * 1e6,
             GIc=g["GIc_N_per_mm"] * 1e3, GIIc=g["GIIc_N_per_mm"] * 1e3)
    tau1, _, _ = oracle.czm(m, [1e-9, 0, 0], 0.0)
    tau3, _, _ = oracle.czm(m, [0, 0, 1e-9], 0.0)
    assert abs(tau1[0] / tau3[2] - 1.0) < 2e-3


# ---------------------------------------------------------------------------
# stable step of an interface node pair, projected damage maps
# ---------------------------------------------------------------------------

def _interface_column(safety):
    """One element column of two plies (0 and 90 degrees, so an interface lies
    between them), free, no gravity, with a soft elastic bulk so that the
    interface penalty K_I of the paper's set sets the stable step."""
    t = 0.25e-3
    mats = []
    for _ in range(2):
        m = dict(W.material_isotropic(1.0e8, 0.3, 1590.0))
        c = W.material_cfrp(True, t)
        m.update({k: c[k] for k in ("KI", "tauI", "tauII", "GIc", "GIIc", "eta_bk")})
        mats.append(m)
    mesh = W._mesh(1, 1, 2, 1, 1e-3, 1e-3, t, [0.0, 90.0], cohesive=1, bc=W.BC_FREE,
                   gravity=0.0, cfl_safety=safety)
    return dict(mesh=mesh, materials=mats, impactor=W.impactor(4e-3, 1.0, v0=0.0, gap=1.0))


def _interface_mode_growth(safety, steps, rel_amp=1e-3):
    """Largest displacement over the second half of the run divided by that
    over the first half, after an opening of the interface pairs (plus a
    little noise in every degree of freedom) far below onset."""
    o = oracle.Oracle(_interface_column(safety))
    nplane = 4
    m = o.get(oracle.MASS)
    d = np.zeros((o.nn, 3))
    amp = rel_amp * o.cfg["materials"][0]["tauI"] / o.cfg["materials"][0]["KI"]
    d[: 2 * nplane, 2] = -amp * m[2 * nplane:].sum() / m.sum()             # opening mode with
    d[2 * nplane:, 2] = amp * m[: 2 * nplane].sum() / m.sum()              # no net momentum
    d += 1e-3 * amp * np.random.default_rng(5).standard_normal(d.shape)
    o.set(oracle.DISP, d.reshape(-1))
    peak = np.zeros(steps)
    for k in range(steps):
        o.step(1)
        peak[k] = np.abs(o.get(oracle.DISP)).max()
    return peak[steps // 2:].max() / peak[: steps // 2].max(), o.get(oracle.COH_R_IP), o


def test_cohesive_pair_stable_step():
    """The interface penalty between two lumped masses is a two-mass spring of
    circular frequency sqrt(K_I A_p / m_eff); central differences are stable
    below 2 / omega and grow geometrically above it (a factor of about 1.33
    per step at 1.01 times the limit).  With the oracle's step at 0.99 of its
    limit the oscillation keeps its amplitude over 400 steps; at 1.01 it grows.
    The opening stays far below onset in both runs, so the pair is linear."""
    g_lo, r_lo, o = _interface_mode_growth(0.99, 400)
    assert o.nc == 1
    assert g_lo < 1.02 and (r_lo == 0).all(), g_lo
    g_hi, r_hi, _ = _interface_mode_growth(1.01, 80, rel_amp=1e-12)
    assert g_hi > 1e4 and (r_hi == 0).all(), g_hi
    # the bulk stays far below its own limit: the pair mode alone decides
    c_bulk = 1.0e8 * 0.7 / (1.3 * 0.4)
    assert o.dt < 0.1 * 0.25e-3 * math.sqrt(1590.0 / c_bulk)


def test_projected_damage_maps_take_the_max_over_thickness():
    """Damage maps (Fig. 9): per element (i fastest, then j, then layer) and
    projected onto the plate (max over the thickness).  Thresholds are set by
    hand in chosen elements of chosen layers, so the projected map has a
    known value and place; interface pairs likewise for the cohesive map."""
    cfg = W.tiny(5, 3, 4, 1, angles=[0, 90, 0, 90], cohesive=1, law=W.LAW_CDM, lx=5e-3, ly=3e-3,
                 ply_thickness=0.25e-3, v0=0.0)
    cfg["impactor"]["gap"] = 1.0
    o = oracle.Oracle(cfg)
    nx, ny, L = 5, 3, 4
    r = np.ones((L, ny, nx, 4))
    hot = {(0, 0): (2, 3.0), (4, 2): (0, 9.0), (2, 1): (3, 1.7), (1, 2): (1, 5.0)}
    for (i, j), (layer, val) in hot.items():
        r[layer, j, i, 2] = val                      # r2+ (matrix tension, drives shear)
    r[3, 2, 4, 2] = 2.0                              # below the column's max (layer 0: 9.0)
    o.set(oracle.GP_R, r.reshape(-1))
    per = o.damage_field(oracle.DMG_MATRIX).reshape(L, ny, nx)
    proj = o.damage_field(oracle.DMG_PROJ_MATRIX).reshape(ny, nx)
    shear = o.damage_field(oracle.DMG_SHEAR).reshape(L, ny, nx)
    # each damaged element carries the law's own damage for its threshold
    for (i, j), (layer, val) in hot.items():
        rr = np.ones(4)
        rr[2] = val
        _, _, dmg = oracle.cdm(cfg["materials"][layer], (5e-3 / 5 * 3e-3 / 3 * 0.25e-3) ** (1 / 3),
                               np.zeros(6), rr)
        assert per[layer, j, i] == dmg[2] > 0
        assert shear[layer, j, i] == dmg[4] > 0
        assert proj[j, i] == per[layer, j, i]
    assert per[3, 2, 4] < per[0, 2, 4]
    mask = np.zeros((ny, nx), bool)
    for (i, j) in hot:
        mask[j, i] = True
    assert (proj[~mask] == 0).all() and (per.sum(axis=0)[~mask] == 0).all()
    assert (o.damage_field(oracle.DMG_PROJ_FIBRE) == 0).all()
    # cohesive: one interface pair damaged (threshold 0.6) in the second
    # interface; it is a corner of the <= 4 interface elements around it
    assert o.nc == 3 * nx * ny
    rd = np.zeros((3, ny, nx, 4))
    for a, (di, dj) in enumerate(((0, 0), (1, 0), (1, 1), (0, 1))):   # corner a of element (i, j)
        i, j = 2 - di, 1 - dj
        rd[1, j, i, a] = 0.6                                          # node (2, 1) of interface 1
    o.set(oracle.COH_R_IP, rd.reshape(-1))
    coh = o.damage_field(oracle.DMG_COHESIVE).reshape(3, ny, nx)
    pc = o.damage_field(oracle.DMG_PROJ_COHESIVE).reshape(ny, nx)
    _, _, D = oracle.czm(cfg["materials"][1], [0.0, 0.0, 0.0], 0.6)
    assert D > 0.6
    want = np.zeros((ny, nx))
    want[0:2, 1:3] = D
    assert np.array_equal(pc, want)
    assert np.array_equal(coh[1], want) and (coh[0] == 0).all() and (coh[2] == 0).all()


# ---------------------------------------------------------------------------
# integration: energy, contact conditions, momentum, release
# ---------------------------------------------------------------------------

def test_isotropic_plate_energy_identity():
    o = oracle.Oracle(W.plate_iso_20x20x4())
    o.step(2000)
    e = o.energies()
    assert e["level"] == 1999
    assert abs(e["residual"]) <= 1e-6 * e["ke0"]
    assert abs(e["residual"]) <= 1e-12 * e["ke0"]        # the oracle closes to round-off
    t, f, x = o.history()
    assert len(f) == 2000 and f.max() > 0
    # elastic: internal work equals the stored secant energy (no dissipation)
    assert abs(e["w_int"] - e["u_el"]) <= 1e-5 * e["ke0"]


def test_free_vibration_conserves_energy():
    cfg = W.tiny(4, 4, 2, 2, gravity=0.0, isotropic=True)
    cfg["mesh"]["bc"] = 2
    cfg["impactor"]["gap"] = 1.0
    o = oracle.Oracle(cfg)
    # smooth field: the trapezoidal work is exact for the quadratic part of the
    # energy; the cubic (geometric) part errs by O(strain * (omega dt)^2)
    X = o.get(oracle.COORDS).reshape(-1, 3)
    lx, ly = cfg["mesh"]["lx"], cfg["mesh"]["ly"]
    d0 = np.zeros_like(X)
    d0[:, 2] = 1e-8 * np.sin(np.pi * X[:, 0] / lx) * np.sin(np.pi * X[:, 1] / ly)
    d0[:, 0] = 2e-9 * np.cos(np.pi * X[:, 1] / ly)
    o.set(oracle.DISP, d0.reshape(-1))
    o.step(1)
    u0 = o.energies()["u_el"]
    o.step(300)
    e = o.energies()
    assert abs(e["ke_plate"] + e["u_el"] - u0) <= 1e-8 * u0


def _contact_cfg():
    cfg = W.tiny(6, 6, 2, 2, isotropic=True, v0=5.0, mass=0.2, R=3e-3)
    cfg["mesh"]["lx"] = cfg["mesh"]["ly"] = 12e-3
    return cfg


def test_non_penetration_and_eq2_every_step():
    cfg = _contact_cfg()
    o = oracle.Oracle(cfg)
    R = cfg["impactor"]["radius"]
    X = o.get(oracle.COORDS).reshape(-1, 3)
    top = np.arange(o.nn - 49, o.nn)
    seen = 0
    for _ in range(400):
        o.step(1)
        d = o.get(oracle.DISP).reshape(-1, 3)
        c = o.impactor_state()["centre"]
        x = X[top] + d[top]
        dist = np.linalg.norm(x - c, axis=1)
        act = o.get(oracle.ACTIVE)[top] > 0
        below = x[:, 2] <= c[2]
        assert (np.abs(dist[act] - R) <= 1e-12 * R).all()
        assert (dist[below & ~act] - R >= -1e-12 * R).all()
        fc = o.get(oracle.FCONTACT).reshape(-1, 3)[top]
        nvec = (x - c) / dist[:, None]
        fn = (fc * nvec).sum(axis=1)
        assert (fn[act] >= 0).all()                    # Eq. 2 on the contact set
        seen += act.sum()
    assert seen > 0


def _graded(h0, w0, ratio, total):
    """Grid lines from 0: spacing h0 up to w0, then growing by `ratio` up to `total`."""
    xs = list(np.arange(0.0, w0 + 1e-12, h0))
    h = h0
    while xs[-1] < total - 1e-12:
        h *= ratio
        xs.append(xs[-1] + h)
    return np.array(xs)


def test_quasi_static_hertz_indentation():
    """The PDN contact (Section 2.1, Eqs. 2-3) against Hertz's closed form.

    A rigid sphere of radius 8 mm indents an elastic block (E = 70 GPa,
    nu = 0.3) at 1 m/s: the striker mass is 1e9 kg, so its displacement is
    prescribed to round-off and the load rises slowly against the block's
    wave transit time.  The block is 27 x 27 x 13.5 mm with its bottom fixed,
    deep enough that the rigid base stiffens it by well under 1 % (a 16 x 16 x 8
    mm block reads 1-3 % high), meshed at 0.1 mm under the striker and
    graded outwards.  At indentations of 20 and 50 um (contact radii 0.40 and
    0.63 mm) the force equals (4/3) E/(1 - nu^2) sqrt(R) delta^(3/2) =
    820.5 N and 3243 N within 3 %."""
    side = _graded(0.1e-3, 0.6e-3, 1.45, 12e-3)
    xs = np.concatenate([-side[::-1], side[1:]]) + side[-1]
    depth = _graded(0.1e-3, 0.6e-3, 1.45, 12e-3)
    H = depth[-1]
    zs = H - depth[::-1]
    nx, nz, L = len(xs) - 1, len(zs) - 1, xs[-1]
    E, nu = 70e9, 0.3
    cfg = dict(mesh=W._mesh(nx, nx, 1, nz, L, L, H, [0.0], bc=W.BC_FREE, gravity=0.0),
               materials=[W.material_isotropic(E, nu, 2700.0)],
               impactor=W.impactor(8e-3, 1e9, v0=1.0, gap=1e-7))
    X = np.stack(np.meshgrid(xs, xs, zs, indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    o = oracle.Oracle(cfg, node_coords=X.reshape(-1), threads=min(8, os.cpu_count() or 1))
    fix = np.zeros_like(X)
    fix[:(nx + 1) * (nx + 1)] = 1.0                 # bottom plane
    o.set(oracle.FIX, fix.reshape(-1))
    o.step(int((52e-6 + 1e-7) / 1.0 / o.dt) + 1)
    t, f, x = o.history()
    delta = x - 1e-7                                 # the sphere touches the centre node at x = gap
    Es = E / (1 - nu * nu)
    for d, F_h in ((20e-6, 820.5), (50e-6, 3243.4)):
        assert abs(4.0 / 3.0 * Es * np.sqrt(8e-3) * d ** 1.5 - F_h) <= 1e-3 * F_h
        F = np.interp(d, delta, f)
        assert abs(F - F_h) <= 0.03 * F_h, (d, F, F_h)


def test_free_plate_momentum_closure():
    cfg = _contact_cfg()
    cfg["mesh"]["bc"] = 2
    cfg["mesh"]["gravity"] = 0.0
    o = oracle.Oracle(cfg)
    m = o.get(oracle.MASS)
    ms = cfg["impactor"]["mass"]
    P0 = -ms * cfg["impactor"]["v0"]
    for _ in range(300):
        o.step(1)
        v = o.get(oracle.VEL).reshape(-1, 3)
        st = o.impactor_state()
        Pp = (m * v[:, 2]).sum()
        Ps = ms * st["velocity"][2]
        pending = st["force"][2] * o.dt
        assert abs(Pp + Ps - pending - P0) <= 1e-12 * abs(P0)


def test_forced_adhesion_releases_nodes():
    cfg = _contact_cfg()
    o = oracle.Oracle(cfg)
    while o.stats()["active"] < 1:
        o.step(1)
        assert o.stats()["steps"] < 2000
    o.step(5)
    assert o.stats()["active"] >= 1
    imp = dict(cfg["impactor"])
    imp["v0"] = -cfg["impactor"]["v0"]          # striker now moves away
    o.set_impactor(imp)
    before = o.stats()
    o.step(1)
    after = o.stats()
    assert after["released"] > before["released"]
    assert after["max_passes"] == 2
    assert after["reset_passes"] - before["reset_passes"] == 2


def test_cohesive_interface_uniform_opening():
    """Uniform normal opening delta < onset of a two-ply plate: the interface
    carries K_I delta over the whole area, equal and opposite on the two plies,
    and stores 0.5 K_I delta^2 A."""
    mats = W.ply_materials(2, 1e-3)
    for m in mats:
        m["law"] = W.LAW_ELASTIC
    cfg = dict(mesh=W._mesh(3, 2, 2, 1, 3e-3, 2e-3, 1e-3, [0.0, 90.0], cohesive=1, bc=2,
                            gravity=0.0),
               materials=mats, impactor=W.impactor(4e-3, 1.0, v0=0.0, gap=1.0))
    o = oracle.Oracle(cfg)
    assert o.nc == 6
    delta = 0.5 * mats[0]["tauI"] / mats[0]["KI"]
    X = o.get(oracle.COORDS).reshape(-1, 3)
    nplane = 4 * 3
    d = np.zeros_like(X)
    d[2 * nplane:, 2] = delta                      # planes 2, 3 (upper ply) move up
    o.set(oracle.DISP, d.reshape(-1))
    o.step(0)
    f = o.get(oracle.FINT).reshape(-1, 3)
    A = 3e-3 * 2e-3
    top = f[2 * nplane:, 2].sum()
    bot = f[:2 * nplane, 2].sum()
    assert abs(top - mats[0]["KI"] * delta * A) <= 1e-12 * abs(top)
    assert abs(top + bot) <= 1e-12 * abs(top)
    o.step(1)
    assert abs(o.energies()["u_el"] - 0.5 * mats[0]["KI"] * delta ** 2 * A) <= 1e-10 * 0.5 * mats[0]["KI"] * delta ** 2 * A


# ---------------------------------------------------------------------------
# the stored whole-impact runs: the impact's own amplification of rounding
# ---------------------------------------------------------------------------

def test_whole_impact_amplifies_the_order_of_summation():
    """The two stored FP64 oracle runs of the 300 x 200 x 8 plate through its
    whole loading differ only in the order in which nodal forces are summed
    (ascending and descending element order; tests/golden/
    make_qi8_300x200x8_golden.py).  Up to the first releases of contact
    nodes (about step 5,900) their force histories agree to 1e-10; by the
    end of the loading the contact decisions of Eq. 2 have turned that
    rounding into a macroscopic difference of the peak force or the damaged
    area.  Both runs close the energy identity."""
    with open(os.path.join(GOLD, "qi8_300x200x8_fp64_oracle.json")) as fh:
        a = json.load(fh)
    with open(os.path.join(GOLD, "qi8_300x200x8_fp64_oracle_reversed.json")) as fh:
        b = json.load(fh)
    # (the first run predates the field; its script summed in ascending order)
    assert a.get("assembly_order", "ascending") == "ascending" and b["assembly_order"] == "descending"
    assert a["steps"] == b["steps"] and a["dt"] == b["dt"]
    ev = a["history_every"]
    fa = np.asarray(a["history"]["force"])[:5800 // ev]
    fb = np.asarray(b["history"]["force"])[:5800 // ev]
    assert np.abs(fa - fb).max() <= 1e-10 * np.abs(fa).max()
    diffs = [abs(a["peak_force_filtered_N"] - b["peak_force_filtered_N"]) / a["peak_force_filtered_N"]]
    for thr in ("0", "0.5", "0.999"):
        x, y = a["projected_damage"]["matrix"][thr]["area_m2"], b["projected_damage"]["matrix"][thr]["area_m2"]
        diffs.append(abs(x - y) / x)
    print(f"  reversed order: filtered peak {diffs[0]:.2e}, damaged areas {', '.join(f'{d:.2e}' for d in diffs[1:])}")
    assert max(diffs) >= 1e-4
    for g in (a, b):
        assert abs(g["energies"]["residual"]) <= 1e-9 * g["energies"]["ke0"]
