"""GPU parity of the batched ensemble: many independent LJ and bead-spring
systems of uneven size advanced by the same launches."""
import numpy as np
import pytest

from paper_1412_3387_amd import inputs
from tests.gpu_helpers import LJ, by_tag, frel, min_image_diff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1412_3387_amd import binding
    binding.lib()
    return binding


def _batch(n_lj=5, n_poly=5):
    return inputs.batch_ensemble(n_lj=n_lj, n_poly=n_poly, lj_range=(500, 3000), chain_range=(20, 60))


def _params(B, sy, prec):
    if sy.kind == "lj":
        return B.ModelParams(precision=prec, pair=B.PAIR_LJ, tpp_force=4, sort_period=50)
    return B.ModelParams(precision=prec, pair=B.PAIR_WCA, bond_cap=2, tpp_force=4, sort_period=50)


def _systems(batch):
    return [dict(pos=sy.pos, vel=sy.vel, L=sy.L, bonds=sy.bonds, tag=sy.tag) for sy in batch]


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_forces_match_oracle(orc, B, prec):
    batch = _batch()
    ctx = B.Context([_params(B, sy, prec) for sy in batch], _systems(batch))
    ctx.compute_forces(0, 1)
    ctx.check()
    th = ctx.thermo()
    for k, sy in enumerate(batch):
        x, v, f, tag = ctx.host_state(k)
        f = f[np.argsort(tag)]
        if sy.kind == "lj":
            F, u, w, _ = orc.pair_forces("lj", sy.pos, sy.L, LJ)
        else:
            Fp, up, wp, _ = orc.pair_forces("wca", sy.pos, sy.L, [1.0, 1.0])
            Fb, ub, wb, _ = orc.bond_forces(sy.pos, sy.L, sy.bonds, with_wca=False)
            F, u, w = Fp + Fb, up + ub, wp + wb
        assert frel(f[:, :3], F) <= (1e-12 if prec == 0 else 1e-5), (k, sy.kind, sy.n)
        ref = orc.thermo(sy.vel, u, w)
        assert abs(th[k, 1] - ref[1]) <= (1e-11 if prec == 0 else 1e-6) * abs(ref[1])


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_step_equals_single_systems(B, prec):
    """Each system of a batch evolves bit for bit as it does alone, in both
    precisions: every system has its own displacement flag, so it is rebuilt
    at the same steps as alone (and only then), and its rows, sums and
    integration are those of the single-system run."""
    batch = _batch(3, 3)
    ctx = B.Context([_params(B, sy, prec) for sy in batch], _systems(batch))
    ctx.step(0, 40)
    ctx.check()
    builds_alone = []
    for k, sy in enumerate(batch):
        one = B.Context([_params(B, sy, prec)], _systems([sy]))
        one.step(0, 40)
        builds_alone.append(one.build_count())
        xa, va, fa, ta = ctx.host_state(k)
        xb, vb, fb, tb = one.host_state(0)
        assert np.array_equal(ta, tb), (k, sy.kind)
        assert np.array_equal(xa, xb) and np.array_equal(va, vb), (k, sy.kind)
    # the systems were rebuilt at different steps: a shared flag would have
    # rebuilt all of them together
    assert len(set(builds_alone)) > 1


def test_batch_short_run_fp64(orc, B):
    batch = _batch(2, 2)
    ctx = B.Context([_params(B, sy, 0) for sy in batch], _systems(batch))
    ctx.step(0, 20)
    ctx.check()
    for k, sy in enumerate(batch):
        if sy.kind == "lj":
            xo, vo, *_ = orc.run_nve("lj", sy.pos, sy.vel, sy.L, LJ, 0.005, 20)
        else:
            xo, vo, *_ = orc.run_nve("polymer", sy.pos, sy.vel, sy.L, [1.0, 1.0], 0.005, 20,
                                     bonds=sy.bonds, bond_prm=[30.0, 1.5])
        x, v, f, tag = ctx.host_state(k)
        x, v = by_tag(tag, x, v)
        assert np.max(np.abs(min_image_diff(x, xo, sy.L))) <= 1e-10
        assert np.max(np.abs(v - vo)) <= 1e-10


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_with_empty_and_one_particle_systems(B, prec):
    """Degenerate systems beside a 900-particle liquid: one without rows, one
    with 100 rows and no particle, and a lone particle in a periodic box.  The
    liquid evolves bit for bit as it does alone, the lone particle feels no
    force and moves in a straight line across the periodic boundary, and the
    empty systems report zero energies and temperature."""
    lj = inputs.lj_fluid(900, 51, 52)
    L = np.array([10.0, 10.0, 10.0])
    x1 = np.array([[9.9, 0.05, 5.0]])
    v1 = np.array([[0.7, -0.45, 0.3]])
    empty = dict(pos=np.zeros((0, 3)), vel=np.zeros((0, 3)), L=L)
    systems = [dict(pos=lj.pos, vel=lj.vel, L=lj.L), dict(empty), dict(empty, n_cap=100),
               dict(pos=x1, vel=v1, L=L)]
    p = B.ModelParams(precision=prec, sort_period=20)
    batch = B.Context([p] * 4, systems)
    print(f"[case] empty and one-particle systems, precision {prec}", flush=True)
    batch.step(0, 60, log_every=10)
    batch.check()
    one = B.Context([p], systems[:1])
    one.step(0, 60, log_every=10)
    one.check()
    for u, w in zip(batch.host_state(0), one.host_state(0)):
        assert np.array_equal(u, w)
    assert all(a.shape[0] == 0 for a in batch.host_state(1)) and all(a.shape[0] == 0 for a in batch.host_state(2))
    x, v, f, tag = batch.host_state(3)
    assert np.array_equal(v, v1) and np.all(f == 0) and tag[0] == 0
    # 60 steps of 0.005 along v, folded into [0, L): x crosses the boundary at 0
    assert np.max(np.abs(min_image_diff(x, x1 + 0.3 * v1, L))) <= 1e-12
    assert np.all((x >= 0) & (x < L)) and x[0, 0] < 1.0
    log = batch.thermo_log()
    assert np.all(log[:, 1:3, 1:] == 0)
    assert np.allclose(log[:, 3, 1], 0.5 * np.sum(v1 ** 2), rtol=1e-14) and np.all(log[:, 3, 2:] == 0)
    assert np.array_equal(log[:, 0, :], one.thermo_log()[:, 0, :])
