"""GPU parity: velocity-Verlet trajectories, thermo, rebuild logic and the
Morton reordering against the oracle."""
import numpy as np
import pytest

from paper_1412_3387_amd import inputs
from tests.gpu_helpers import LJ, by_tag, min_image_diff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1412_3387_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def ref50(orc):
    s = inputs.lj_small()
    x, v, F, th, st = orc.run_nve("lj", s.pos, s.vel, s.L, LJ, 0.005, 50, with_thermo=True)
    assert st == 0
    return s, x, v, F, th


@pytest.mark.parametrize("w", [1, 4, 16])
def test_lj_small_50_steps_fp64(B, ref50, w):
    s, xo, vo, Fo, tho = ref50
    p = B.ModelParams(precision=B.FP64, tpp_force=w)
    ctx = B.Context([p], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    ctx.step(0, 50, log_every=10)
    ctx.check()
    x, v, f, tag = ctx.host_state()
    x, v, f = by_tag(tag, x, v, f)
    assert np.max(np.abs(min_image_diff(x, xo, s.L))) <= 1e-10
    assert np.max(np.abs(v - vo)) <= 1e-10
    assert np.max(np.abs(f[:, :3] - Fo)) <= 1e-10 * np.sqrt(np.mean(Fo ** 2))
    log = ctx.thermo_log()
    assert log.shape[0] == 6
    for row in log[:, 0, :]:
        t = int(row[0])
        ref = tho[t]
        assert np.allclose(row[1:], ref, rtol=1e-10, atol=1e-9), (t, row, ref)
    assert ctx.build_count() >= 2


def test_lj_small_50_steps_mixed(B, ref50):
    s, xo, vo, Fo, tho = ref50
    ctx = B.Context([B.ModelParams(precision=B.MIXED)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    ctx.step(0, 50)
    ctx.check()
    x, v, f, tag = ctx.host_state()
    x, v = by_tag(tag, x, v)
    vs = np.sqrt(np.mean(vo ** 2))
    assert np.max(np.abs(min_image_diff(x, xo, s.L))) <= 1e-5
    assert np.max(np.abs(v - vo)) <= 1e-5 * vs


def test_split_calls_equal_one_call(B):
    s = inputs.lj_fluid(3000, 11, 12)
    a = B.Context([B.ModelParams(precision=0)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    a.step(0, 40)
    b = B.Context([B.ModelParams(precision=0)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    for k in range(4):
        b.step(10 * k, 10)
    xa, va, fa, ta = a.host_state()
    xb, vb, fb, tb = b.host_state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(ta, tb)


def test_deterministic_bitwise(B):
    s = inputs.lj_fluid(5000, 13, 14)
    out = []
    for _ in range(2):
        c = B.Context([B.ModelParams(precision=1, sort_period=7)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
        c.step(0, 30)
        out.append(c.host_state())
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_time_reversal_fp64(B):
    s = inputs.lj_fluid(2000, 15, 16)
    c = B.Context([B.ModelParams(precision=0)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    c.step(0, 50)
    x, v, f, tag = c.host_state()
    c2 = B.Context([B.ModelParams(precision=0)], [dict(pos=x, vel=-v, L=s.L, tag=tag)])
    c2.step(0, 50)
    x2, v2, f2, tag2 = c2.host_state()
    x2, v2 = by_tag(tag2, x2, v2)
    assert np.max(np.abs(min_image_diff(x2, s.pos, s.L))) < 1e-10
    assert np.max(np.abs(v2 + s.vel)) < 1e-10


def test_morton_sort_order_is_stable_key_order(orc, B):
    """After a sort the rows are the stable order of the oracle's Morton keys
    of the positions being sorted (previous row order = tag order)."""
    s = inputs.lj_fluid(6000, 17, 18)
    c = B.Context([B.ModelParams(precision=0, sort_period=1)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    c.step(0, 1)
    x, v, f, tag = c.host_state()
    keys = orc.morton_keys(x, s.L)
    order = orc.stable_order(keys)
    # x is already sorted: the stable order of its keys is the identity, and
    # ties keep ascending tags (the order before the sort)
    assert np.array_equal(order, np.arange(len(order)))
    k = keys.astype(np.int64)
    tie = k[1:] == k[:-1]
    assert np.all(tag[1:][tie] > tag[:-1][tie])
    assert sorted(tag.tolist()) == list(range(6000))


def test_morton_sort_preserves_trajectory(B):
    s = inputs.lj_fluid(4000, 19, 20)
    a = B.Context([B.ModelParams(precision=0)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    a.step(0, 30)
    b = B.Context([B.ModelParams(precision=0, sort_period=10)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    b.step(0, 30)
    xa, va, fa, ta = a.host_state()
    xb, vb, fb, tb = b.host_state()
    xa, va = by_tag(ta, xa, va)
    xb, vb = by_tag(tb, xb, vb)
    assert np.max(np.abs(min_image_diff(xa, xb, s.L))) < 1e-11
    assert np.max(np.abs(va - vb)) < 1e-11


def test_dpd_short_run_fp64(orc, B):
    s = inputs.dpd_fluid(3000, 31, 32)
    prm = [25.0, 4.5, 1.0, 1.0, 0.02, 33]
    xo, vo, Fo, th, st = orc.run_nve("dpd", s.pos, s.vel, s.L, prm, 0.02, 5, tag=s.tag, t0=100)
    p = B.ModelParams(precision=0, pair=B.PAIR_DPD, r_cut=1.0, r_buff=0.4, dt=0.02, dpd_seed=33,
                      sort_period=1000)
    c = B.Context([p], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    c.step(100, 5)
    c.check()
    x, v, f, tag = c.host_state()
    x, v = by_tag(tag, x, v)
    assert np.max(np.abs(min_image_diff(x, xo, s.L))) <= 1e-10
    assert np.max(np.abs(v - vo)) <= 1e-10


def test_polymer_short_run(orc, B):
    m = inputs.polymer_melt(40, seed_vel=5)
    xo, vo, Fo, th, st = orc.run_nve("polymer", m.pos, m.vel, m.L, [1.0, 1.0], 0.005, 20,
                                     bonds=m.bonds, bond_prm=[30.0, 1.5])
    assert st == 0
    p = B.ModelParams(precision=0, pair=B.PAIR_WCA, bond_cap=2, sort_period=10)
    c = B.Context([p], [dict(pos=m.pos, vel=m.vel, L=m.L, bonds=m.bonds)])
    c.step(0, 20)
    c.check()
    x, v, f, tag = c.host_state()
    x, v = by_tag(tag, x, v)
    assert np.max(np.abs(min_image_diff(x, xo, m.L))) <= 1e-10
    assert np.max(np.abs(v - vo)) <= 1e-10


@pytest.mark.parametrize("pair", ["lj", "dpd"])
def test_graph_replay_equals_eager(B, pair):
    """Captured pairs of middle steps reproduce eager launches bit for bit,
    across sorts, logged steps and several step() calls."""
    if pair == "lj":
        s = inputs.lj_fluid(5000, 23, 24)
        kw = dict(precision=1, sort_period=7)
    else:
        s = inputs.dpd_fluid(4000, 31, 32)
        kw = dict(precision=1, pair=B.PAIR_DPD, r_cut=1.0, r_buff=0.4, dt=0.02, dpd_seed=5,
                  sort_period=9)
    out = []
    for g in (0, 1):
        c = B.Context([B.ModelParams(use_graph=g, **kw)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
        c.step(0, 23, log_every=10)
        c.step(23, 18)
        c.check()
        out.append(c.host_state() + (c.thermo_log(),))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_energy_drift_mixed_not_worse_than_fp64(B):
    """NVE drift over 10^4 steps of the 4,000-particle liquid: at most 1e-4
    in either precision, and the mixed path may not add drift beyond
    max(1e-4, 2x the FP64 drift)."""
    s = inputs.lj_small()
    drift = {}
    for prec in (0, 1):
        c = B.Context([B.ModelParams(precision=prec, sort_period=500)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
        c.step(0, 10000, log_every=1000)
        c.check()
        log = c.thermo_log()[:, 0, :]
        E = log[:, 1] + log[:, 2]
        drift[prec] = abs(E[-1] - E[0]) / abs(E[0])
    assert drift[0] <= 1e-4 and drift[1] <= 1e-4, drift
    assert drift[1] <= max(1e-4, 2 * drift[0]), drift
