"""GPU: the autotuner (times every candidate launch shape, keeps the
fastest, caches the choice per kind of context, re-scans after a set number
of steps) and neighbour-list / force parity with every build shape it may
choose."""
import numpy as np
import pytest

from paper_1412_3387_amd import inputs
from tests.gpu_helpers import LJ, by_tag, frel, min_image_diff, neighbor_sets_equal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1412_3387_amd import binding
    binding.lib()
    return binding


def test_autotune_picks_argmin_and_keeps_parity(orc, B):
    s = inputs.lj_fluid(20000, 91, 92)
    ctx = B.Context([B.ModelParams(precision=B.MIXED, sort_period=500)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    t = ctx.autotune(1)
    fm, bm = np.array(t.force_ms[:]), np.array(t.build_ms[:])
    assert t.scans == 1 and t.from_cache == 0
    assert np.all(fm > 0) and np.all(bm > 0)
    assert t.tpp_force == B.FORCE_LANES[int(np.argmin(fm))] and t.block_force == 64 * t.tpp_force
    assert (t.tpp_nlist, t.block_nlist) == B.BUILD_SHAPES[int(np.argmin(bm))]
    # the state after the scan: the list of the chosen shape, forces as before
    ctx.check()
    rng = np.random.default_rng(3)
    which = np.sort(rng.choice(s.n, 400, replace=False))
    assert neighbor_sets_equal(orc, ctx, s.pos, s.L, 2.5, 0.4, which=which) == []
    ctx.compute_forces(0, 0)
    ctx.check()
    x, v, f, tag = ctx.host_state()
    f = f[np.argsort(tag)]
    F, u, w, nc = orc.pair_forces("lj", s.pos, s.L, LJ, which=which)
    assert frel(f[which, :3], F) <= 1e-5


@pytest.mark.parametrize("shape", [(64, 512), (64, 256), (32, 512), (32, 256)])
def test_every_build_shape_is_exact(orc, B, shape):
    """Each candidate shape of the framed build gives the oracle's neighbour
    sets (a liquid, a shuffled liquid that also goes to the general build,
    and a bead-spring melt with bonded exclusions) and the oracle's forces."""
    w, b = shape
    s = inputs.lj_small()
    ctx = B.Context([B.ModelParams(precision=B.FP64, sort_period=100, tpp_nlist=w, block_nlist=b)],
                    [dict(pos=s.pos, vel=s.vel, L=s.L)])
    ctx.build_nlist(True)
    ctx.check()
    assert neighbor_sets_equal(orc, ctx, s.pos, s.L, 2.5, 0.4) == []
    ctx.compute_forces(0, 0)
    x, v, f, tag = ctx.host_state()
    F, u, wv, nc = orc.pair_forces("lj", s.pos, s.L, LJ)
    assert frel(f[np.argsort(tag)][:, :3], F) <= 1e-12
    m = inputs.polymer_melt(80, seed_vel=93)
    rng = np.random.default_rng(4)
    m.pos = inputs.wrap(m.pos + rng.uniform(-0.08, 0.08, m.pos.shape), m.L)
    ctx = B.Context([B.ModelParams(precision=B.FP64, pair=B.PAIR_WCA, bond_cap=2, sort_period=100,
                                   tpp_nlist=w, block_nlist=b)],
                    [dict(pos=m.pos, vel=m.vel, L=m.L, bonds=m.bonds)])
    ctx.build_nlist(True)
    ctx.check()
    assert neighbor_sets_equal(orc, ctx, m.pos, m.L, 2.0 ** (1.0 / 6.0), 0.4, bonds=m.bonds) == []


def test_autotune_cache(B):
    s = inputs.lj_fluid(12000, 94, 95)
    sys_ = [dict(pos=s.pos, vel=s.vel, L=s.L)]
    a = B.Context([B.ModelParams(precision=B.MIXED, sort_period=500)], sys_)
    ta = a.autotune(1)
    b = B.Context([B.ModelParams(precision=B.MIXED, sort_period=500)], sys_)
    tb = b.autotune(2)
    assert tb.from_cache == 1 and tb.scans == 0
    assert (tb.tpp_force, tb.tpp_nlist, tb.block_nlist) == (ta.tpp_force, ta.tpp_nlist, ta.block_nlist)
    assert list(tb.force_ms) == list(ta.force_ms)
    # another kind of context (FP64) has no cached entry: it scans
    c = B.Context([B.ModelParams(precision=B.FP64, sort_period=500)], sys_)
    tc = c.autotune(2)
    assert tc.from_cache == 0 and tc.scans == 1


def test_tune_period_rescans_and_keeps_the_trajectory(orc, B):
    """With tune_period = 20, step() scans at its first call and again once
    20 steps have passed; the FP64 trajectory still equals the oracle's."""
    s = inputs.lj_small()
    ctx = B.Context([B.ModelParams(precision=B.FP64, tune_period=20)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    ctx.step(0, 30)
    assert ctx.autotune(0).scans == 1
    ctx.step(30, 20)
    assert ctx.autotune(0).scans == 2
    ctx.check()
    xo, vo, Fo, th, st = orc.run_nve("lj", s.pos, s.vel, s.L, LJ, 0.005, 50)
    x, v, f, tag = ctx.host_state()
    x, v = by_tag(tag, x, v)
    assert np.max(np.abs(min_image_diff(x, xo, s.L))) <= 1e-10
    assert np.max(np.abs(v - vo)) <= 1e-10
