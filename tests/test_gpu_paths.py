"""GPU parity on the paths that the full-size workloads take: DPD tiles in
the force pass's second launch (per-pair images, halos beyond its LDS
stage), the 1,000,000-particle DPD fluid after diffusion, batches holding the
largest systems of the ensemble (20,000-particle liquid, 400-chain melt) in
both precisions, a batch whose systems differ in bond capacity, the
displacement check period with its dangerous-build status, and the energy
drift of the 2,000,000-particle liquid over 10^4 steps."""
import numpy as np
import pytest

from paper_1412_3387_amd import inputs
from tests.gpu_helpers import LJ, by_tag, frel, min_image_diff

pytestmark = pytest.mark.gpu
TOL = {0: 1e-12, 1: 1e-5}
DPD_PRM = [25.0, 4.5, 1.0, 1.0, 0.02, 33]
DPD_RARE_STAGE = 40 * 1024 // 52  # halo entries the second launch stages in LDS for DPD


@pytest.fixture(scope="module")
def B():
    from paper_1412_3387_amd import binding
    binding.lib()
    return binding


def _dpd_params(B, prec, sort_period=0):
    return B.ModelParams(precision=prec, pair=B.PAIR_DPD, r_cut=1.0, r_buff=0.4, dt=0.02,
                         dpd_A=25.0, dpd_gamma=4.5, dpd_kT=1.0, dpd_seed=33, sort_period=sort_period)


def _shuffled(sys_, seed):
    perm = np.random.default_rng(seed).permutation(sys_.n)
    return inputs.System(pos=sys_.pos[perm], vel=sys_.vel[perm], L=sys_.L, tag=perm.astype(np.int32)), perm


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [1500, 12000])
def test_dpd_forces_second_launch(orc, B, prec, n):
    """Unsorted rows of a DPD fluid: every tile spans the box, so it needs
    per-pair images; at 12,000 particles the tile halos (about 2,100
    entries) also exceed the 787 entries the second launch stages in LDS,
    so their tails are read from global memory (velocities and tags too)."""
    ref = inputs.dpd_fluid(n, 51, 52)
    s, perm = _shuffled(ref, 7)
    ctx = B.Context([_dpd_params(B, prec)], [dict(pos=s.pos, vel=s.vel, L=s.L, tag=s.tag)])
    ctx.compute_forces(29, 1)
    ctx.check()
    hn = ctx.halo_n()
    assert ctx.rare_tiles() == len(hn)             # every tile in the second launch
    assert np.all(hn >> 31 == 1)                     # with per-pair images
    if n == 12000:
        assert (hn & 0xFFFF).max() > DPD_RARE_STAGE  # beyond its LDS stage
    x, v, f, tag = ctx.host_state()
    fo = np.empty_like(f)
    fo[tag] = f
    F, u, w, nc = orc.pair_forces("dpd", ref.pos, ref.L, DPD_PRM, vel=ref.vel, tag=ref.tag, timestep=29)
    assert frel(fo[:, :3], F) <= TOL[prec]
    th = ctx.thermo()[0]
    assert abs(th[1] - u.sum()) <= (1e-12 if prec == 0 else 1e-6) * abs(u.sum())


def test_dpd_1M_after_diffusion_sampled(orc, B):
    """The 1,000,000-particle DPD fluid in mixed precision with the Morton
    sort every 100 steps, 199 steps in (99 steps of diffusion since the last
    sort): forces of sampled particles at that state against brute force
    over the whole box.  Some tiles then need the general build or the
    second force launch."""
    s = inputs.dpd_bulk()
    ctx = B.Context([_dpd_params(B, 1, sort_period=100)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    ctx.build_nlist(True)
    ctx.step(0, 199)
    ctx.check()
    ctx.build_nlist(True)
    gen, rare = ctx.general_tiles(), ctx.rare_tiles()
    ctx.compute_forces(199, 0)
    ctx.check()
    x, v, f, tag = ctx.host_state()
    x, v, f = by_tag(tag, x, v, f)
    print(f"general-build tiles {gen}, second-launch tiles {rare}")
    assert gen + rare > 0
    rng = np.random.default_rng(8)
    which = np.sort(rng.choice(s.n, 256, replace=False))
    F, u, w, nc = orc.pair_forces("dpd", x, s.L, DPD_PRM, vel=v, tag=np.arange(s.n, dtype=np.int32),
                                  timestep=199, which=which)
    fr = np.sqrt(np.mean(np.sum(F * F, axis=1)))
    err = np.max(np.sqrt(np.sum((f[which, :3] - F) ** 2, axis=1))) / fr
    assert err <= TOL[1], err


def _big_batch():
    """The largest shapes of the ensemble beside small ones: LJ 20,000 and
    500, melts of 400 and 20 chains of 50."""
    out = [inputs.lj_fluid(20000, 61, 62, seed_vac=63), inputs.lj_fluid(500, 64, 65, seed_vac=66),
           inputs.polymer_melt(400, seed_vel=67), inputs.polymer_melt(20, seed_vel=68)]
    rng = np.random.default_rng(9)
    for sy in out[2:]:
        sy.pos = inputs.wrap(sy.pos + rng.uniform(-0.08, 0.08, sy.pos.shape), sy.L)
    return out


def _params(B, sy, prec, bond_cap=2):
    if sy.kind == "lj":
        return B.ModelParams(precision=prec, pair=B.PAIR_LJ, tpp_force=4, sort_period=50)
    return B.ModelParams(precision=prec, pair=B.PAIR_WCA, bond_cap=bond_cap, tpp_force=4, sort_period=50)


def _systems(batch):
    return [dict(pos=sy.pos, vel=sy.vel, L=sy.L, bonds=sy.bonds, tag=sy.tag) for sy in batch]


def _oracle_forces(orc, sy):
    if sy.kind == "lj":
        return orc.pair_forces("lj", sy.pos, sy.L, LJ)
    Fp, up, wp, _ = orc.pair_forces("wca", sy.pos, sy.L, [1.0, 1.0])
    Fb, ub, wb, ns = orc.bond_forces(sy.pos, sy.L, sy.bonds, with_wca=False)
    assert ns == 0
    return Fp + Fb, up + ub, wp + wb, None


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_largest_shapes_forces(orc, B, prec):
    batch = _big_batch()
    ctx = B.Context([_params(B, sy, prec) for sy in batch], _systems(batch))
    ctx.compute_forces(0, 1)
    ctx.check()
    th = ctx.thermo()
    for k, sy in enumerate(batch):
        x, v, f, tag = ctx.host_state(k)
        f = f[np.argsort(tag)]
        F, u, w, _ = _oracle_forces(orc, sy)
        assert frel(f[:, :3], F) <= TOL[prec], (k, sy.kind, sy.n)
        ref = orc.thermo(sy.vel, u, w)
        assert abs(th[k, 1] - ref[1]) <= (1e-11 if prec == 0 else 1e-6) * abs(ref[1]), k


@pytest.fixture(scope="module")
def big_ref(orc):
    """The batch and the oracle's 10-step FP64 run of each of its systems."""
    batch = _big_batch()
    ref = []
    for sy in batch:
        if sy.kind == "lj":
            xo, vo, *_ = orc.run_nve("lj", sy.pos, sy.vel, sy.L, LJ, 0.005, 10)
        else:
            xo, vo, *_ = orc.run_nve("polymer", sy.pos, sy.vel, sy.L, [1.0, 1.0], 0.005, 10,
                                     bonds=sy.bonds, bond_prm=[30.0, 1.5])
        ref.append((xo, vo))
    return batch, ref


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_largest_shapes_trajectory(B, big_ref, prec):
    """10 steps of the batch (graph-replayed, persistent launches over all
    systems) against the FP64 oracle run of each system: x and v within
    1e-10 (FP64) and 1e-5 of the RMS velocity (mixed, FP32 pair
    arithmetic)."""
    batch, ref = big_ref
    ctx = B.Context([_params(B, sy, prec) for sy in batch], _systems(batch))
    ctx.step(0, 10)
    ctx.check()
    for k, sy in enumerate(batch):
        xo, vo = ref[k]
        x, v, f, tag = ctx.host_state(k)
        x, v = by_tag(tag, x, v)
        vs = np.sqrt(np.mean(vo ** 2))
        tol_x = 1e-10 if prec == 0 else 1e-5
        tol_v = 1e-10 if prec == 0 else 1e-5 * vs
        assert np.max(np.abs(min_image_diff(x, xo, sy.L))) <= tol_x, (k, sy.kind)
        assert np.max(np.abs(v - vo)) <= tol_v, (k, sy.kind)


def test_batch_mixed_bond_capacities(orc, B):
    """Systems of one batch with bond capacities 2 and 4 (and an LJ system
    with none) share one partner table: bond forces and exclusions of each
    must match the oracle."""
    rng = np.random.default_rng(10)
    a, b = inputs.polymer_melt(30, seed_vel=71), inputs.polymer_melt(45, seed_vel=72)
    for sy in (a, b):
        sy.pos = inputs.wrap(sy.pos + rng.uniform(-0.08, 0.08, sy.pos.shape), sy.L)
    lj = inputs.lj_fluid(1500, 73, 74)
    batch = [a, lj, b]
    params = [_params(B, a, 0, bond_cap=2), _params(B, lj, 0), _params(B, b, 0, bond_cap=4)]
    ctx = B.Context(params, _systems(batch))
    ctx.compute_forces(0, 1)
    ctx.check()
    for k, sy in enumerate(batch):
        x, v, f, tag = ctx.host_state(k)
        f = f[np.argsort(tag)]
        F, u, w, _ = _oracle_forces(orc, sy)
        assert frel(f[:, :3], F) <= TOL[0], (k, sy.kind)


def test_check_period_trajectory(B):
    """Displacement checks every third step since the build: with no
    dangerous build the list stays valid and the FP64 trajectory equals the
    one checked every step, to rounding."""
    s = inputs.lj_fluid(4000, 81, 82)
    out = []
    for k in (1, 3):
        c = B.Context([B.ModelParams(precision=0, check_period=k)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
        c.step(0, 60)
        assert c.sync_status()[0] == 0
        out.append((c.host_state(), c.build_count()))
    (xa, va, fa, ta), na = out[0]
    (xb, vb, fb, tb), nb = out[1]
    xa, va = by_tag(ta, xa, va)
    xb, vb = by_tag(tb, xb, vb)
    assert np.max(np.abs(min_image_diff(xa, xb, s.L))) < 1e-11
    assert np.max(np.abs(va - vb)) < 1e-10
    assert na >= 3 and nb >= 3


@pytest.mark.parametrize("use_graph", [0, 1])
def test_dangerous_build_is_reported(B, use_graph):
    """Particles fast enough (T about 11) to pass r_buff/2 within a check
    period of 8:
    the rebuild comes at the first check after the build and is latched as
    dangerous (a status, the run itself goes on)."""
    s = inputs.lj_fluid(4000, 83, 84, T=1.2)
    c = B.Context([B.ModelParams(precision=1, check_period=8, use_graph=use_graph)],
                  [dict(pos=s.pos, vel=s.vel * 3.0, L=s.L)])
    c.step(0, 20)
    assert c.sync_status()[0] == 10
    # checked every step, the same start is never dangerous
    c = B.Context([B.ModelParams(precision=1, check_period=1, use_graph=use_graph)],
                  [dict(pos=s.pos, vel=s.vel * 3.0, L=s.L)])
    c.step(0, 20)
    assert c.sync_status()[0] == 0


@pytest.mark.parametrize("prec", [0, 1])
def test_lj_2M_energy_drift(B, prec):
    """NVE energy drift of the 2,000,000-particle liquid (Morton sort every
    500 steps) over 10^4 steps: |E(t1) - E(t0)| / |E(t0)| <= 1e-4 in either
    precision."""
    s = inputs.lj_bulk()
    c = B.Context([B.ModelParams(precision=prec, sort_period=500)], [dict(pos=s.pos, vel=s.vel, L=s.L)])
    c.build_nlist(True)
    c.step(0, 10000, log_every=1000)
    c.check()
    log = c.thermo_log()[:, 0, :]
    E = log[:, 1] + log[:, 2]
    drift = abs(E[-1] - E[0]) / abs(E[0])
    print(f"precision {prec}: drift {drift:.3e} over 10^4 steps, T_end {log[-1, 4]:.4f}")
    assert drift <= 1e-4
