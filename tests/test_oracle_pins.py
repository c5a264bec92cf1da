"""Pins for the CPU oracle: closed forms, published known answers, special
cases that reduce to textbook results or library routines, invariants and
brute force on tiny inputs.  None of these call the GPU path."""
import math
import os

import numpy as np
import pytest

from paper_1412_3387_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BIG = [50.0, 50.0, 50.0]


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _pair(r, axis=0):
    pos = np.array([[10.0, 10.0, 10.0], [10.0, 10.0, 10.0]])
    pos[1, axis] += r
    return pos


# ---------------------------------------------------------------- Philox

def test_philox_known_answers(orc):
    rows = _golden("philox4x32_10_kat.txt")
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_dpd_theta_symmetric_and_unit_variance(orc):
    rng = np.random.default_rng(5)
    pairs = rng.integers(0, 2**31 - 1, size=(20000, 2))
    th = np.array([orc.dpd_theta(int(a), int(b), 33, 7) for a, b in pairs])
    th_sw = np.array([orc.dpd_theta(int(b), int(a), 33, 7) for a, b in pairs[:2000]])
    assert np.array_equal(th[:2000], th_sw)
    assert np.all(th >= -math.sqrt(3)) and np.all(th < math.sqrt(3))
    # uniform on [-sqrt3, sqrt3): mean 0, variance 1 (5 sigma bounds)
    assert abs(th.mean()) < 5 * 1.0 / math.sqrt(len(th))
    assert abs(th.var() - 1.0) < 5 * math.sqrt(0.8 / len(th))
    # a new timestep or seed gives an uncorrelated stream
    th2 = np.array([orc.dpd_theta(int(a), int(b), 33, 8) for a, b in pairs])
    th3 = np.array([orc.dpd_theta(int(a), int(b), 34, 7) for a, b in pairs])
    assert abs(np.corrcoef(th, th2)[0, 1]) < 0.04
    assert abs(np.corrcoef(th, th3)[0, 1]) < 0.04


# ---------------------------------------------------------------- geometry

def test_min_image_rounds_half_to_even(orc):
    L = [10.0, 10.0, 10.0]
    assert np.allclose(orc.min_image([6.0, -6.0, 4.0], L), [-4.0, 4.0, 4.0])
    # exactly half a box: rint(0.5) = 0, rint(-0.5) = -0, rint(1.5) = 2
    assert np.array_equal(orc.min_image([5.0, -5.0, 15.0], L), [5.0, -5.0, -5.0])
    # open axes are left alone
    assert np.array_equal(orc.min_image([6.0, 6.0, 6.0], L, periodic=(0, 1, 0)), [6.0, -4.0, 6.0])


def test_wrap_folds_into_box(orc):
    L = [10.0, 10.0, 10.0]
    x = orc.wrap([[10.0, -1e-17, 19.999], [-3.0, 9.999999, 0.0]], L)
    assert np.all(x >= 0.0) and np.all(x < 10.0)
    assert x[0, 0] == 0.0 and x[0, 1] == 0.0
    assert abs(x[0, 2] - 9.999) < 1e-12 and x[1, 0] == 7.0


# ---------------------------------------------------------------- LJ

def _lj_unshifted(orc, r, rc=3.0, eps=1.0, sig=1.0):
    F, u, w, nc = orc.pair_forces("lj", _pair(r), BIG, [eps, sig, rc])
    s6 = (sig / rc) ** 6
    return u.sum() + 4 * eps * (s6 * s6 - s6), -F[0, 0], F, w


def test_lj_closed_forms(orc):
    for name, r, val, tol, *_ in _golden("closed_forms.txt"):
        if not name.startswith("lj_"):
            continue
        r, val, tol = float(r), float(val), float(tol)
        V, F, _, _ = _lj_unshifted(orc, r)
        got = V if name == "lj_V" else F
        assert abs(got - val) <= tol * max(abs(val), 1.0) + 1e-13, (name, r, got, val)


def test_lj_force_is_minus_energy_gradient(orc):
    for r in (0.92, 1.0, 1.3, 1.9, 2.4):
        h = 1e-5
        Vp, *_ = _lj_unshifted(orc, r + h)
        Vm, *_ = _lj_unshifted(orc, r - h)
        _, F, _, _ = _lj_unshifted(orc, r)
        assert abs(-(Vp - Vm) / (2 * h) - F) < 1e-6 * max(1.0, abs(F))


def test_lj_scales_with_eps_and_sigma(orc):
    V1, F1, *_ = _lj_unshifted(orc, 1.1)
    V2, F2, *_ = _lj_unshifted(orc, 1.1, eps=2.5)
    assert abs(V2 - 2.5 * V1) < 1e-12 and abs(F2 - 2.5 * F1) < 1e-12
    V3, F3, *_ = _lj_unshifted(orc, 2.2, rc=6.0, sig=2.0)
    assert abs(V3 - V1) < 1e-12 and abs(F3 - F1 / 2.0) < 1e-12


def test_lj_truncation_shift_and_direction(orc):
    rc = 2.5
    F, u, w, nc = orc.pair_forces("lj", _pair(rc - 1e-9), BIG, [1, 1, rc])
    assert nc.tolist() == [1, 1] and abs(u.sum()) < 1e-9       # shifted energy is continuous
    F, u, w, nc = orc.pair_forces("lj", _pair(rc + 1e-9), BIG, [1, 1, rc])
    assert nc.tolist() == [0, 0] and np.all(F == 0) and np.all(u == 0)
    # repulsive at r = 0.95: particle 0 (smaller x) is pushed towards -x
    F, u, w, nc = orc.pair_forces("lj", _pair(0.95, axis=2), BIG, [1, 1, rc])
    assert F[0, 2] < 0 and F[1, 2] > 0 and F[0, 0] == 0 and F[0, 1] == 0
    # pair virial: w_0 + w_1 = r_01 . F_01
    assert abs(w.sum() - (-0.95) * F[0, 2]) < 1e-12


def test_lj_pair_across_periodic_boundary(orc):
    L = [8.0, 8.0, 8.0]
    inside = np.array([[3.0, 4.0, 4.0], [4.1, 4.0, 4.0]])
    across = np.array([[0.3, 4.0, 4.0], [7.2, 4.0, 4.0]])
    Fa, ua, *_ = orc.pair_forces("lj", inside, L, [1, 1, 2.5])
    Fb, ub, *_ = orc.pair_forces("lj", across, L, [1, 1, 2.5])
    assert abs(abs(Fa[0, 0]) - abs(Fb[0, 0])) < 1e-12 and abs(ua.sum() - ub.sum()) < 1e-12
    assert Fb[0, 0] > 0  # the partner sits at x = -0.8 (image), pushes towards +x


def test_lj_newton_third_law(orc):
    s = inputs.lj_fluid(500, 3, 4)
    F, u, w, nc = orc.pair_forces("lj", s.pos, s.L, [1, 1, 2.5])
    frms = math.sqrt(np.mean(np.sum(F * F, axis=1)))
    assert np.all(np.abs(F.sum(axis=0)) < 500 * 1e-15 * frms * 10)


def test_lj_subset_equals_full(orc):
    s = inputs.lj_fluid(500, 3, 4)
    F, u, w, nc = orc.pair_forces("lj", s.pos, s.L, [1, 1, 2.5])
    which = np.array([7, 499, 0, 123])
    Fs, us, ws, ncs = orc.pair_forces("lj", s.pos, s.L, [1, 1, 2.5], which=which)
    assert np.array_equal(Fs, F[which]) and np.array_equal(us, u[which])


# ---------------------------------------------------------------- FENE + WCA

def test_fene_wca_closed_forms(orc):
    for name, r, val, tol, *_ in _golden("closed_forms.txt"):
        if not name.startswith("fene_"):
            continue
        r, val, tol = float(r), float(val), float(tol)
        F, u, w, ns = orc.bond_forces(_pair(r), BIG, [[0, 1]])
        got = u.sum() if name == "fene_wca_U" else -F[0, 0]
        assert abs(got - val) <= tol * max(abs(val), 1.0), (name, r, got, val)


def test_fene_equilibrium_and_harmonic_limit(orc):
    # the net bond force changes sign just below 0.97 sigma
    f = [-orc.bond_forces(_pair(r), BIG, [[0, 1]])[0][0, 0] for r in (0.95, 0.97)]
    assert f[0] > 0 > f[1]
    # r << R0: FENE is a harmonic spring of stiffness K (no WCA beyond 2^(1/6))
    r = 0.01
    F, u, w, ns = orc.bond_forces(_pair(r), BIG, [[0, 1]], with_wca=False)
    assert abs(u.sum() - 0.5 * 30.0 * r * r) < 1e-4 * 0.5 * 30.0 * r * r
    assert abs(-F[0, 0] - (-30.0 * r)) < 1e-4 * 30.0 * r


def test_fene_force_gradient_and_break(orc):
    for r in (0.8, 0.97, 1.1, 1.4):
        h = 1e-6
        up = orc.bond_forces(_pair(r + h), BIG, [[0, 1]])[1].sum()
        um = orc.bond_forces(_pair(r - h), BIG, [[0, 1]])[1].sum()
        F = -orc.bond_forces(_pair(r), BIG, [[0, 1]])[0][0, 0]
        assert abs(-(up - um) / (2 * h) - F) < 1e-5 * max(1.0, abs(F))
    assert orc.bond_forces(_pair(1.5), BIG, [[0, 1]])[3] == 1
    assert orc.bond_forces(_pair(1.6), BIG, [[0, 1]])[3] == 1


def test_wca_on_bonds_equals_wca_on_all_pairs(orc):
    """FENE+WCA per bond with bonded pairs excluded from the pair sum equals
    WCA between all pairs plus FENE alone (the Kremer-Grest definition)."""
    s = inputs.polymer_melt(6, seed_vel=9)
    rng = np.random.default_rng(1)
    pos = inputs.wrap(s.pos + rng.uniform(-0.1, 0.1, s.pos.shape), s.L)
    Fa, ua, wa, _ = orc.pair_forces("wca", pos, s.L, [1, 1], bonds=s.bonds)
    Fb, ub, wb, ns = orc.bond_forces(pos, s.L, s.bonds, with_wca=True)
    Fc, uc, wc, _ = orc.pair_forces("wca", pos, s.L, [1, 1])
    Fd, ud, wd, ns2 = orc.bond_forces(pos, s.L, s.bonds, with_wca=False)
    assert ns == 0 and ns2 == 0
    assert np.allclose(Fa + Fb, Fc + Fd, rtol=0, atol=1e-10)
    assert abs((ua + ub).sum() - (uc + ud).sum()) < 1e-9
    assert abs((wa + wb).sum() - (wc + wd).sum()) < 1e-9


# ---------------------------------------------------------------- DPD

def test_dpd_conservative_limit(orc):
    # gamma = kT = 0 leaves the soft repulsion A (1 - r/rc) rhat
    for r in (0.25, 0.5, 0.75, 0.999):
        F, u, w, nc = orc.pair_forces("dpd", _pair(r, axis=1), BIG, [25, 0, 0, 1.0, 0.02, 1])
        assert abs(-F[0, 1] - 25.0 * (1.0 - r)) < 1e-12
        assert abs(u.sum() - 0.5 * 25.0 * (1 - r) ** 2) < 1e-12
    F, u, w, nc = orc.pair_forces("dpd", _pair(1.0 + 1e-12), BIG, [25, 0, 0, 1.0, 0.02, 1])
    assert np.all(F == 0)


def test_dpd_pure_drag(orc):
    # kT = 0, A = 0: F_i = -gamma w^2 (rhat . v_ij) rhat
    r, g = 0.6, 4.5
    pos = _pair(r)
    vel = np.array([[0.3, 0.7, -0.2], [-0.1, 0.2, 0.5]])
    F, *_ = orc.pair_forces("dpd", pos, BIG, [0, g, 0, 1.0, 0.02, 1], vel=vel)
    rhat_v = -(vel[0, 0] - vel[1, 0])  # rhat = (x0 - x1)/r = -e_x
    expect = -g * (1 - r) ** 2 * rhat_v * np.array([-1.0, 0, 0])
    assert np.allclose(F[0], expect, atol=1e-14) and np.array_equal(F[1], -F[0])
    # motion perpendicular to the line of centres feels no drag
    vel2 = np.array([[0.0, 0.7, -0.2], [0.0, 0.2, 0.5]])
    F2, *_ = orc.pair_forces("dpd", pos, BIG, [0, g, 0, 1.0, 0.02, 1], vel=vel2)
    assert np.all(F2 == 0)


def test_dpd_pairwise_antisymmetry_and_momentum(orc):
    s = inputs.dpd_fluid(3000, 31, 32)
    prm = [25, 4.5, 1.0, 1.0, 0.02, 33]
    F, *_ = orc.pair_forces("dpd", s.pos, s.L, prm, vel=s.vel, tag=s.tag, timestep=11)
    frms = math.sqrt(np.mean(np.sum(F * F, axis=1)))
    assert np.all(np.abs(F.sum(axis=0)) < 3000 * 1e-15 * frms * 10)
    # a single pair: F_ij = -F_ji bitwise
    rng = np.random.default_rng(2)
    for _ in range(50):
        pos = np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0]]) + rng.uniform(-0.4, 0.4, (2, 3))
        vel = rng.normal(size=(2, 3))
        F, *_ = orc.pair_forces("dpd", pos, BIG, prm, vel=vel, tag=np.array([17, 4]), timestep=3)
        assert np.array_equal(F[0], -F[1])


# ---------------------------------------------------------------- neighbour sets

@pytest.mark.parametrize("rl,expect", [(1.5, 18), (1.8, 26), (2.0, 26), (2.01, 32)])
def test_neighbors_simple_cubic_shells(orc, rl, expect):
    g = np.arange(8, dtype=np.float64) + 0.5
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    off, idx = orc.neighbors(pos, [8.0] * 3, rl - 0.4, 0.4)
    assert np.all(np.diff(off) == expect)


def test_neighbors_fcc_first_shell(orc):
    L = 6.0
    pos = inputs.fcc_sites(4, L, offset_frac=0.25)
    a = L / 4
    off, idx = orc.neighbors(pos, [L] * 3, a / math.sqrt(2) + 0.01, 0.0)
    assert np.all(np.diff(off) == 12)


def test_neighbors_exclusions_and_rows(orc):
    s = inputs.polymer_melt(4, seed_vel=3)
    off0, idx0 = orc.neighbors(s.pos, s.L, 2 ** (1 / 6), 0.4)
    off1, idx1 = orc.neighbors(s.pos, s.L, 2 ** (1 / 6), 0.4, bonds=s.bonds)
    deg = np.zeros(s.n, dtype=np.int64)
    np.add.at(deg, s.bonds.ravel(), 1)
    assert np.array_equal(np.diff(off0) - np.diff(off1), deg)
    for i in range(0, s.n, 17):
        row = idx1[off1[i]:off1[i + 1]]
        assert np.all(np.diff(row) > 0) and i not in row


def test_neighbor_count_fcc_shells(orc):
    """fcc shells sit at a sqrt(k/2) holding 12, 6, 24, 12, 24, 8 sites; at
    density 0.8442 the sixth shell (2.909) lies just beyond r = 2.9."""
    s = inputs.lj_fluid(4000, 1, 2, noise=0.0)
    off, idx = orc.neighbors(s.pos, s.L, 2.5, 0.4)
    assert np.all(np.diff(off) == 12 + 6 + 24 + 12 + 24)
    off, idx = orc.neighbors(s.pos, s.L, 2.52, 0.4)
    assert np.all(np.diff(off) == 12 + 6 + 24 + 12 + 24 + 8)


def test_neighbor_count_matches_density(orc):
    s = inputs.dpd_fluid(6000, 31, 32)
    off, idx = orc.neighbors(s.pos, s.L, 1.0, 0.4)
    nbar = np.diff(off).mean()
    expect = 4.0 / 3.0 * math.pi * 1.4 ** 3 * 3.0
    assert abs(nbar - expect) < 5 * math.sqrt(expect / 6000) * 3


# ---------------------------------------------------------------- integrator

def test_free_flight_is_exact(orc):
    rng = np.random.default_rng(3)
    L = np.array([20.0, 20.0, 20.0])
    pos = rng.uniform(0, 20, (50, 3))
    vel = rng.normal(size=(50, 3))
    x, v, F, th, st = orc.run_nve("lj", pos, vel, L, [0.0, 1.0, 2.5], 0.005, 40)
    assert st == 0 and np.array_equal(v, vel) and np.all(F == 0)
    x2 = pos.copy()
    for _ in range(40):
        x2 = orc.wrap(x2 + 0.005 * vel, L)
    assert np.array_equal(x, x2)


def test_velocity_verlet_time_reversal(orc):
    s = inputs.lj_fluid(500, 5, 6)
    x, v, F, th, st = orc.run_nve("lj", s.pos, s.vel, s.L, [1, 1, 2.5], 0.005, 50)
    x2, v2, F2, th2, st2 = orc.run_nve("lj", x, -v, s.L, [1, 1, 2.5], 0.005, 50, force=F)
    d = x2 - s.pos
    d -= s.L * np.rint(d / s.L)
    assert st == 0 and st2 == 0
    assert np.max(np.abs(d)) < 1e-10 and np.max(np.abs(v2 + s.vel)) < 1e-10


def _dimer_energy_error(orc, dt, T=3.0):
    pos = _pair(1.3)
    vel = np.array([[0.4, 0.0, 0.0], [-0.4, 0.0, 0.0]])
    n = int(round(T / dt))
    x, v, F, th, st = orc.run_nve("lj", pos, vel, BIG, [1, 1, 3.0], dt, n, with_thermo=True)
    E = th[:, 0] + th[:, 1]
    return np.max(np.abs(E - E[0]))


def test_velocity_verlet_is_second_order(orc):
    e1 = _dimer_energy_error(orc, 0.004)
    e2 = _dimer_energy_error(orc, 0.002)
    assert 3.3 < e1 / e2 < 4.7


def test_velocity_verlet_matches_ode_solver(orc):
    """LJ dimer: the separation after t = 2 agrees with a high-accuracy
    Runge-Kutta solution of r'' = 2 F(r) (reduced mass 1/2) to O(dt^2)."""
    from scipy.integrate import solve_ivp
    r0, v0 = 1.3, 0.8

    def rhs(t, y):
        r = y[0]
        f = 24 * (2 / r ** 13 - 1 / r ** 7)
        return [y[1], 2 * f]
    sol = solve_ivp(rhs, (0, 2.0), [r0, -v0], rtol=1e-12, atol=1e-12)
    r_ref = sol.y[0, -1]
    pos = _pair(r0)
    vel = np.array([[0.4, 0, 0], [-0.4, 0, 0]])
    x, v, F, th, st = orc.run_nve("lj", pos, vel, BIG, [1, 1, 5.0], 0.001, 2000)
    assert abs((x[1, 0] - x[0, 0]) - r_ref) < 2e-5


def test_nve_energy_conserved_on_lj_small(orc):
    s = inputs.lj_small()
    x, v, F, th, st = orc.run_nve("lj", s.pos, s.vel, s.L, [1, 1, 2.5], 0.005, 20, with_thermo=True)
    E = th[:, 0] + th[:, 1]
    assert st == 0 and np.max(np.abs(E - E[0])) / abs(E[0]) < 2e-3
    assert abs(th[0, 3] - 1.2) < 1e-12


# ---------------------------------------------------------------- NVT

def test_nvt_without_coupling_is_nve(orc):
    """xi = 0 and an infinite tau (h / tau^2 = 0): the Nose-Hoover step is
    the velocity-Verlet step, bit for bit, and xi stays zero."""
    s = inputs.lj_fluid(500, 5, 6)
    x, v, F, th, st = orc.run_nve("lj", s.pos, s.vel, s.L, [1, 1, 2.5], 0.005, 30, with_thermo=True)
    x2, v2, F2, th2, ext, st2 = orc.run_nvt("lj", s.pos, s.vel, s.L, [1, 1, 2.5], 0.005, 30,
                                           T0=1.0, tau=1e200)
    assert st == 0 and st2 == 0
    assert np.array_equal(x, x2) and np.array_equal(v, v2) and np.array_equal(th, th2)
    assert np.all(ext == 0)


def _free_gas_nvt(orc, dt, t_end, T0, tau):
    rng = np.random.default_rng(11)
    L = np.array([40.0, 40.0, 40.0])
    pos = rng.uniform(0, 40, (64, 3))
    vel = rng.normal(size=(64, 3))
    n = int(round(t_end / dt))
    x, v, F, th, ext, st = orc.run_nvt("lj", pos, vel, L, [0.0, 1.0, 2.5], dt, n, T0=T0, tau=tau)
    assert st == 0 and np.all(F == 0)
    return vel, v, th, ext


def test_nvt_free_gas_matches_ode_solver(orc):
    """No forces: v(t) = v(0) exp(-zeta(t)) with zeta' = xi and
    xi' = (T(0) exp(-2 zeta) / T0 - 1) / tau^2, solved by a high-accuracy
    Runge-Kutta method; eta is zeta.  The discrete run converges to it at
    second order in the step."""
    from scipy.integrate import solve_ivp
    T0, tau, t_end = 1.7, 0.4, 2.0
    errs = []
    for dt in (0.004, 0.002):
        v0, v, th, ext = _free_gas_nvt(orc, dt, t_end, T0, tau)
        Ti = th[0, 3]

        def rhs(t, y):
            return [y[1], (Ti * np.exp(-2.0 * y[0]) / T0 - 1.0) / tau ** 2]
        sol = solve_ivp(rhs, (0, t_end), [0.0, 0.0], rtol=1e-12, atol=1e-13)
        zeta, xi = sol.y[0, -1], sol.y[1, -1]
        e = max(abs(ext[-1, 0] - xi), abs(ext[-1, 1] - zeta),
                np.max(np.abs(v - v0 * np.exp(-zeta))) / np.max(np.abs(v0)))
        errs.append(e)
    assert errs[0] < 5e-4 and 3.0 < errs[0] / errs[1] < 5.0


@pytest.fixture(scope="module")
def melted(orc):
    """The 500-particle LJ lattice after 1,000 NVE steps: a liquid at T ~ 0.65."""
    s = inputs.lj_fluid(500, 5, 6)
    x, v, F, th, st = orc.run_nve("lj", s.pos, s.vel, s.L, [1, 1, 2.5], 0.005, 1000)
    assert st == 0
    return x, v, s.L, s.n


def test_nvt_extended_energy_is_conserved(orc, melted):
    """The liquid heated towards T0 = 1: KE + PE alone changes by far more
    than the extended energy, whose drift falls as the square of the step."""
    x0, v0, L, n = melted
    T0, tau = 1.0, 0.5
    drift = []
    for dt, steps in ((0.004, 500), (0.002, 1000)):
        x, v, F, th, ext, st = orc.run_nvt("lj", x0, v0, L, [1, 1, 2.5], dt, steps, T0=T0, tau=tau)
        assert st == 0
        H = orc.nvt_conserved(th, ext, n, T0, tau)
        E = th[:, 0] + th[:, 1]
        drift.append(np.max(np.abs(H - H[0])))
        assert np.max(np.abs(E - E[0])) > 1000 * drift[-1]
    assert drift[0] / abs(H[0]) < 1e-3 and 3.0 < drift[0] / drift[1] < 5.5


def test_nvt_holds_the_set_temperature(orc, melted):
    """From T ~ 0.65 the thermostat brings the liquid to T0 = 1: the mean
    temperature over steps 1,000-3,000 is within 2 % of T0."""
    x0, v0, L, n = melted
    x, v, F, th, ext, st = orc.run_nvt("lj", x0, v0, L, [1, 1, 2.5], 0.005, 3000, T0=1.0, tau=0.2)
    assert st == 0 and th[0, 3] < 0.7
    assert abs(np.mean(th[1000:, 3]) - 1.0) < 0.02


# ---------------------------------------------------------------- thermo

def test_thermo_sums(orc):
    n = 10
    vel = np.zeros((n, 3))
    vel[0::2, 0] = 1.0
    vel[1::2, 0] = -1.0
    out = orc.thermo(vel, np.full(n, 0.25), np.full(n, -0.5))
    assert out[0] == n / 2 and out[1] == n * 0.25 and out[2] == -n * 0.5
    assert abs(out[3] - n / (3 * n - 3)) < 1e-15


# ---------------------------------------------------------------- cell list / Morton

def test_cell_list_is_stable_counting_sort(orc):
    s = inputs.lj_fluid(4000, 1, 2)
    bins = orc.cell_bins(s.L, 2.9)
    assert bins.tolist() == [5, 5, 5] and np.all(s.L / bins >= 2.9)
    cell_of, start, idx = orc.cell_list(s.pos, s.L, bins)
    assert np.array_equal(idx, np.argsort(cell_of, kind="stable"))
    assert np.array_equal(np.diff(start), np.bincount(cell_of, minlength=125))
    w = s.L / bins
    c = np.stack([cell_of % 5, (cell_of // 5) % 5, cell_of // 25], 1)
    assert np.all(s.pos >= c * w - 1e-12) and np.all(s.pos < (c + 1) * w + 1e-12)


def test_cell_bins_never_narrower_than_list_radius(orc):
    for L in (8.4, 8.7, 16.796, 100.776, 133.31, 69.336, 5.8, 2.0):
        b = orc.cell_bins([L] * 3, 2.9)
        assert b[0] >= 1 and (b[0] == 1 or L / b[0] >= 2.9)


def test_morton_keys_and_order(orc):
    L = [1024.0] * 3
    pos = np.array([[1.5, 0.5, 0.5], [0.5, 1.5, 0.5], [0.5, 0.5, 1.5], [1023.9] * 3,
                    [3.2, 0.0, 0.0], [0.0, 5.0, 0.0]])
    k = orc.morton_keys(pos, L)
    assert k.tolist() == [1, 2, 4, 2 ** 30 - 1, 9, (1 << 1) | (1 << 7)]
    rng = np.random.default_rng(0)
    keys = rng.integers(0, 50, 1000).astype(np.uint32)
    assert np.array_equal(orc.stable_order(keys), np.argsort(keys, kind="stable"))


# ---------------------------------------------------------------- ghosts

def test_ghost_mask_rule(orc):
    lo, hi, w = [0.0] * 3, [10.0] * 3, 2.0
    pos = np.array([[5, 5, 5], [9, 5, 5], [1, 5, 5], [9, 9, 5], [9, 9, 9], [1, 1, 1], [8.0, 5, 5]])
    m = orc.ghost_masks(pos, lo, hi, w)

    def d(dx, dy, dz):
        k = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
        return 1 << (k if k < 13 else k - 1)
    assert m[0] == 0 and m[1] == d(1, 0, 0) and m[2] == d(-1, 0, 0)
    assert m[3] == d(1, 0, 0) | d(0, 1, 0) | d(1, 1, 0)
    assert bin(int(m[4])).count("1") == 7 and bin(int(m[5])).count("1") == 7
    assert m[6] == d(1, 0, 0)  # x = hi - w is inside the layer (>=)
    counts, offs, idx = orc.ghost_list(m)
    assert counts.sum() == 1 + 1 + 3 + 7 + 7 + 1 and offs[0] == 0
    assert np.all(offs[1:] == np.cumsum(counts)[:-1])


def _sublattice_count(a, offset, lo, hi):
    """Number of points offset + k a (k integer) inside [lo, hi)."""
    return int(math.ceil((hi - offset) / a - 1e-12) - math.ceil((lo - offset) / a - 1e-12))


def test_ghost_counts_on_fcc_lattice(orc):
    """Face/edge/corner send counts of a 20^3-cell fcc subdomain (no noise)
    equal the product of per-axis counts on each simple-cubic sublattice."""
    m, L = 20, 33.592
    a = L / m
    pos = fcc_no_noise = inputs.fcc_sites(m, L)
    w = 2.9
    mask = orc.ghost_masks(fcc_no_noise, [0.0] * 3, [L] * 3, w)
    counts, offs, idx = orc.ghost_list(mask)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]) + 0.25
    rng_of = {-1: (0.0, w), 0: (0.0, L), 1: (L - w, L)}
    k = 0
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == dy == dz == 0:
                    continue
                expect = 0
                for b in basis:
                    p = 1
                    for ax, dd in enumerate((dx, dy, dz)):
                        lo_, hi_ = rng_of[dd]
                        p *= _sublattice_count(a, b[ax] * a, lo_, hi_)
                    expect += p
                assert counts[k] == expect, (dx, dy, dz)
                k += 1
    assert pos.shape[0] == 32000


def test_ghost_receive_equals_union_of_neighbour_sends(orc):
    sd = inputs.lj_subdomain_box(grid=3, cells=12)   # 6,912 particles, 256 per subdomain
    full, w = sd.full, 2.9
    L = full.L
    lo0, hi0 = sd.lo(0), sd.hi(0)
    ridx, rimg = orc.ghost_receive(full.pos, sd.owner, 0, L, lo0, hi0, w)
    got = []
    for s in range(27):
        if s == 0:
            continue
        loc = sd.local(s)
        m = orc.ghost_masks(full.pos[loc], sd.lo(s), sd.hi(s), w)
        counts, offs, idx = orc.ghost_list(m)
        # direction from s towards subdomain 0 (grid offset, periodic)
        cs = np.array([s % 3, (s // 3) % 3, s // 9])
        dvec = (-cs + 1) % 3 - 1
        kk = (dvec[2] + 1) * 9 + (dvec[1] + 1) * 3 + (dvec[0] + 1)
        kk = kk if kk < 13 else kk - 1
        got.extend(loc[idx[offs[kk]:offs[kk] + counts[kk]]].tolist())
    assert sorted(got) == sorted(ridx.tolist())
    assert len(set(got)) == len(got)
    assert np.all((rimg >= lo0 - w) & (rimg < hi0 + w))


# ---------------------------------------------------------------- inputs

def test_generators_are_seeded_and_exact():
    a = inputs.lj_fluid(4000, 1, 2)
    b = inputs.lj_fluid(4000, 1, 2)
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.vel, b.vel)
    assert np.all(a.pos >= 0) and np.all(a.pos < a.L)
    assert np.all(np.abs(a.vel.sum(axis=0)) < 1e-10)
    ke2 = np.sum(a.vel ** 2)
    assert abs(ke2 / (3 * 4000 - 3) - 1.2) < 1e-12
    assert abs(4000 / a.L[0] ** 3 - 0.8442) < 1e-12
    p = inputs.polymer_melt(20, seed_vel=5)
    d = p.pos[p.bonds[:, 1]] - p.pos[p.bonds[:, 0]]
    d -= p.L * np.rint(d / p.L)
    r = np.sqrt((d * d).sum(1))
    assert np.all(r < 1.5) and np.allclose(r, r[0])
    sd = inputs.lj_subdomain_box(grid=3, cells=12)
    assert np.all(np.bincount(sd.owner, minlength=27) == 256)


def test_dpd_random_force_amplitude(orc):
    """With v = 0 and A = 0 only the random term remains; over many
    timesteps its variance is sigma^2 w^2 / dt with sigma^2 = 2 gamma kT."""
    r, g, kT, dt = 0.4, 4.5, 1.0, 0.02
    pos = _pair(r)
    f = np.array([orc.pair_forces("dpd", pos, BIG, [0, g, kT, 1.0, dt, 33], timestep=t)[0][0, 0]
                  for t in range(20000)])
    expect = 2 * g * kT * (1 - r) ** 2 / dt
    assert abs(f.var() / expect - 1.0) < 5 * math.sqrt(0.8 / len(f))
    assert abs(f.mean()) < 5 * math.sqrt(expect / len(f))


def test_dpd_thermostat_reaches_kT(orc):
    """The dissipative and random terms together hold the fluid at kT
    (fluctuation-dissipation), starting from a colder state."""
    s = inputs.dpd_fluid(1500, 31, 32, kT=0.5)
    prm = [25, 4.5, 1.0, 1.0, 0.02, 33]
    x, v, F, th, st = orc.run_nve("dpd", s.pos, s.vel, s.L, prm, 0.02, 300, tag=s.tag,
                                  with_thermo=True)
    assert st == 0
    T = th[150:, 3].mean()
    assert abs(T - 1.0) < 0.06
