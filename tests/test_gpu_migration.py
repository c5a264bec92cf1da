"""GPU parity of stepping subdomains: a periodic box cut 3 x 3 x 3, the 27
subdomains held as the systems of one context, the exchange between them as
device copies on this GPU (a stand-in for the transport).  Each step: first
half of velocity Verlet; if a rebuild is due, particle migration and a new
ghost selection, else a ghost update; second half.  Checked against the
oracle: every particle owned once, by the subdomain its position lies in,
after each migration; the ghost set of subdomain 0 against brute force; the
whole trajectory against the oracle's full-box run (FP64, LJ and DPD, the
DPD ghosts carrying velocities and tags).  Bonded chains whose bonds are
longer than the ghost layer step the same way with the bond owner table of
Sec. 4.3.4 kept by its messages (a start exchange, then one before every
migration)."""
import numpy as np
import pytest

from paper_1412_3387_amd import inputs
from tests.gpu_helpers import LJ, by_tag, min_image_diff

pytestmark = pytest.mark.gpu
DPD_PRM = [25.0, 4.5, 1.0, 1.0, 0.02, 33]


@pytest.fixture(scope="module")
def B():
    from paper_1412_3387_amd import binding
    binding.lib()
    return binding


def _dir_to(s_from, s_to, g=3):
    a = np.array([s_from % g, (s_from // g) % g, s_from // (g * g)])
    b = np.array([s_to % g, (s_to // g) % g, s_to // (g * g)])
    d = (b - a + 1) % g - 1
    k = (d[2] + 1) * 9 + (d[1] + 1) * 3 + (d[0] + 1)
    return int(k if k < 13 else k - 1)


class Loopback:
    """27 subdomains in one context; exchanges as device copies."""

    def __init__(self, B, sd, params, width, margin, ghost_fields, bonds=None):
        import torch
        self.B, self.sd, self.torch = B, sd, torch
        full = sd.full
        self.L = full.L
        self.W = width
        frame = sd.side + 2 * (width + margin)
        rho = full.n / float(np.prod(full.L))
        systems = []
        for s in range(27):
            loc = sd.local(s)
            d = dict(pos=full.pos[loc], vel=full.vel[loc], tag=loc.astype(np.int32),
                     L=np.full(3, frame), lo=sd.lo(s) - width - margin, periodic=(0, 0, 0),
                     n_cap=int(1.4 * rho * frame ** 3) + 64)
            if bonds is not None:
                # every bond with a member here (tags are the full box's)
                d["bonds"] = bonds[np.isin(bonds[:, 0], loc) | np.isin(bonds[:, 1], loc)]
            systems.append(d)
        self.ctx = B.Context([params] * 27, systems)
        self.bonded = bonds is not None
        self.cap = int(8 * rho * sd.side ** 3) + 256  # up to seven destinations per particle
        self.gfields = ghost_fields
        self.grec = 8 * (3 * bool(ghost_fields & 1) + 3 * bool(ghost_fields & 2) + bool(ghost_fields & 4))
        dev = self.ctx.device
        mk = lambda n, dt: torch.zeros(n, dtype=dt, device=dev)
        self.gsend = [mk(self.cap * self.grec, torch.uint8) for _ in range(27)]
        self.mrec = self.ctx.migrate_record_bytes()
        self.msend = [mk(self.cap * self.mrec, torch.uint8) for _ in range(27)]
        # owner-table messages: at the start every remote partner is announced
        # to all 26 neighbours
        self.bcap = 26 * 2 * self.cap
        self.bsend = [mk(self.bcap * B.BOND_RECORD_BYTES, torch.uint8) for _ in range(27)] if self.bonded else []
        self.bond_messages = 0
        self.cnt = [mk(26, torch.int32) for _ in range(27)]
        self.off = [mk(26, torch.int32) for _ in range(27)]
        self.n_recv = [0] * 27
        self.migrations = 0
        self.moved = 0

    def _gather(self, bufs, rec, to):
        hc = [c.cpu().numpy() for c in self.cnt]
        ho = [o.cpu().numpy() for o in self.off]
        pieces = []
        for k in range(27):
            if k == to:
                continue
            d = _dir_to(k, to)
            a, n = int(ho[k][d]), int(hc[k][d])
            pieces.append(bufs[k][a * rec:(a + n) * rec])
        return self.torch.cat(pieces)

    def select_ghosts(self):
        B, sd = self.B, self.sd
        for s in range(27):
            self.ctx.pack_ghosts(s, sd.lo(s), sd.hi(s), self.W, B.GHOST_SELECT, self.gfields, self.gsend[s],
                                 self.cap, self.cnt[s], self.off[s])
        self.ctx.check()
        for s in range(27):
            recv = self._gather(self.gsend, self.grec, s)
            self.n_recv[s] = recv.numel() // self.grec
            self.ctx.unpack_ghosts(s, recv, self.n_recv[s], self.gfields, B.GHOST_SELECT, self.L)
        self.ctx.check()

    def update_ghosts(self):
        B, sd = self.B, self.sd
        for s in range(27):
            self.ctx.pack_ghosts(s, sd.lo(s), sd.hi(s), self.W, B.GHOST_UPDATE, self.gfields, self.gsend[s],
                                 self.cap, self.cnt[s], self.off[s])
        for s in range(27):
            recv = self._gather(self.gsend, self.grec, s)
            self.ctx.unpack_ghosts(s, recv, self.n_recv[s], self.gfields, B.GHOST_UPDATE, self.L)

    def bond_ranks(self, mode):
        """Owner-table messages of every subdomain, moved, then applied."""
        sd, rec = self.sd, self.B.BOND_RECORD_BYTES
        for s in range(27):
            self.bond_messages += self.ctx.pack_bond_ranks(s, sd.lo(s), sd.hi(s), mode, self.bsend[s], self.bcap,
                                                           self.cnt[s], self.off[s])
        for s in range(27):
            recv = self._gather(self.bsend, rec, s)
            self.ctx.unpack_bond_ranks(s, recv, recv.numel() // rec, mode)
        self.ctx.check()

    def start(self):
        if self.bonded:
            self.bond_ranks(self.B.BOND_START)
        self.select_ghosts()

    def migrate(self):
        sd = self.sd
        if self.bonded:
            self.bond_ranks(self.B.BOND_MIGRATE)
        for s in range(27):
            self.moved += self.ctx.migrate_particles(s, sd.lo(s), sd.hi(s), self.msend[s], self.cap,
                                                     self.cnt[s], self.off[s])
        for s in range(27):
            recv = self._gather(self.msend, self.mrec, s)
            self.ctx.receive_particles(s, recv, recv.numel() // self.mrec, self.L)
        self.ctx.check()
        self.migrations += 1

    def step(self, t):
        self.ctx.integrate_half_step(0, t)
        if self.ctx.rebuild_due():
            self.migrate()
            self.check_ownership()
            self.select_ghosts()
        else:
            self.update_ghosts()
        self.ctx.integrate_half_step(1, t + 1)

    def state(self):
        """Positions (wrapped into the box), velocities by tag, and owners."""
        n = self.sd.full.n
        x = np.full((n, 3), np.nan)
        v = np.full((n, 3), np.nan)
        owner = np.full(n, -1)
        seen = np.zeros(n, dtype=np.int64)
        for s in range(27):
            xs, vs, fs, ts = self.ctx.host_state(s)
            x[ts] = inputs.wrap(xs, self.L)
            v[ts] = vs
            owner[ts] = s
            np.add.at(seen, ts, 1)
        assert np.all(seen == 1), "every particle owned exactly once"
        return x, v, owner

    def check_ownership(self):
        x, v, owner = self.state()
        sd = self.sd
        c = np.clip(np.floor(x / sd.side).astype(np.int64), 0, sd.grid - 1)
        want = c[:, 0] + sd.grid * (c[:, 1] + sd.grid * c[:, 2])
        assert np.array_equal(owner, want)


def _run(orc, B, sd, params, width, margin, fields, model, prm, dt, steps, t0=0):
    lb = Loopback(B, sd, params, width, margin, fields)
    lb.start()
    lb.ctx.compute_forces(t0, 0)
    for k in range(steps):
        lb.step(t0 + k)
    lb.ctx.check()
    assert lb.migrations >= 2 and lb.moved > 0
    x, v, owner = lb.state()
    full = sd.full
    kw = dict(tag=full.tag, t0=t0) if model == "dpd" else {}
    xo, vo, Fo, th, st = orc.run_nve(model, full.pos, full.vel, full.L, prm, dt, steps, **kw)
    assert st == 0
    return lb, x, v, xo, vo


def _shifted_lj_box(cells=12):
    """The 3 x 3 x 3 LJ box with the lattice moved by a/5 per axis, so that
    rows of particles sit close to the subdomain faces and cross them within
    a few steps."""
    sd = inputs.lj_subdomain_box(grid=3, cells=cells)
    a = float(sd.full.L[0]) / cells
    full = sd.full
    full.pos = inputs.wrap(full.pos + 0.2 * a, full.L)
    c = np.clip(np.floor(full.pos / sd.side).astype(np.int64), 0, 2)
    owner = (c[:, 0] + 3 * (c[:, 1] + 3 * c[:, 2])).astype(np.int32)
    return inputs.Subdomains(full=full, grid=3, side=sd.side, owner=owner)


@pytest.mark.parametrize("prec", [0, 1])
def test_lj_subdomains_step_with_migration(orc, B, prec):
    """LJ subdomains: 40 steps with migrations against the full-box oracle,
    to 1e-10 in FP64 and to 1e-5 (positions; velocities relative to their
    RMS) in mixed precision."""
    sd = _shifted_lj_box()
    p = B.ModelParams(precision=prec, nlist_cap=160)
    lb, x, v, xo, vo = _run(orc, B, sd, p, 2.9, 0.6, B.FIELD_POS | B.FIELD_TAG, "lj", LJ, 0.005, 40)
    tol_x, tol_v = (1e-10, 1e-10) if prec == 0 else (1e-5, 1e-5 * np.sqrt(np.mean(vo ** 2)))
    assert np.max(np.abs(min_image_diff(x, xo, sd.full.L))) <= tol_x
    assert np.max(np.abs(v - vo)) <= tol_v
    # the ghost layer of subdomain 0 selected at the last migration, moved
    # with the particles since: re-select now and compare with brute force
    lb.select_ghosts()
    own = np.clip(np.floor(x / sd.side).astype(np.int64), 0, 2)
    owner_now = own[:, 0] + 3 * (own[:, 1] + 3 * own[:, 2])
    # ghosts are chosen by owner (the last migration), not by position now
    xx, vv, owner = lb.state()
    ridx, rimg = orc.ghost_receive(xx, owner, 0, sd.full.L, sd.lo(0), sd.hi(0), 2.9)
    ctx = lb.ctx
    o, n0 = ctx.offsets[0], ctx.n_local[0]
    ng = lb.n_recv[0]
    gtag = ctx.tag[o + n0:o + n0 + ng].cpu().numpy()
    gpos = ctx.pos[o + n0:o + n0 + ng, :3].cpu().numpy()
    og, oref = np.argsort(gtag), np.argsort(ridx)
    assert np.array_equal(gtag[og], ridx[oref])
    assert np.max(np.abs(gpos[og] - rimg[oref])) <= 1e-12
    del owner_now


def test_dpd_subdomains_step_with_migration(orc, B):
    """DPD: ghosts carry positions, velocities (the half-kicked ones the
    pair force reads) and tags (the pair noise is keyed on them)."""
    d = inputs.dpd_fluid(3000, 35, 36)
    side = float(d.L[0]) / 3
    c = np.clip(np.floor(d.pos / side).astype(np.int64), 0, 2)
    owner = (c[:, 0] + 3 * (c[:, 1] + 3 * c[:, 2])).astype(np.int32)
    sd = inputs.Subdomains(full=d, grid=3, side=side, owner=owner)
    p = B.ModelParams(precision=B.FP64, pair=B.PAIR_DPD, r_cut=1.0, r_buff=0.4, dt=0.02, dpd_seed=33,
                      nlist_cap=96)
    lb, x, v, xo, vo = _run(orc, B, sd, p, 1.4, 0.6, B.FIELD_POS | B.FIELD_VEL | B.FIELD_TAG, "dpd", DPD_PRM,
                            0.02, 12, t0=40)
    assert np.max(np.abs(min_image_diff(x, xo, d.L))) <= 1e-10
    assert np.max(np.abs(v - vo)) <= 1e-10


def _chain_box():
    """The stretched chains (bonds of about 2.2) cut 3 x 3 x 3."""
    full = inputs.stretched_chains()
    side = float(full.L[0]) / 3
    c = np.clip(np.floor(full.pos / side).astype(np.int64), 0, 2)
    owner = (c[:, 0] + 3 * (c[:, 1] + 3 * c[:, 2])).astype(np.int32)
    return inputs.Subdomains(full=full, grid=3, side=side, owner=owner)


CHAIN = dict(pair=1, bond_cap=2, fene_K=5.0, fene_R0=3.0, r_buff=0.2, dt=0.002)


@pytest.mark.parametrize("prec", [0, 1])
def test_bonded_subdomains_step_with_migration(orc, B, prec):
    """Chains whose bonds (about 2.2) are longer than the ghost layer
    (WCA cut-off + buffer = 1.32): a bond's partner across a face reaches
    its subdomain only as a ghost sent by the owner table.  60 steps with
    migrations of bonded particles match the oracle's full-box run (WCA on
    all pairs + FENE) to 1e-10 in FP64 and to 1e-5 (positions; velocities
    relative to their RMS) in mixed precision; subdomain 0 holds, beside the
    layer's ghosts, ghosts that are there only as partners of its
    particles."""
    sd = _chain_box()
    full = sd.full
    p = B.ModelParams(precision=prec, **CHAIN)
    width = 2 ** (1 / 6) + 0.2
    lb = Loopback(B, sd, p, width, 1.5, B.FIELD_POS | B.FIELD_TAG, bonds=full.bonds)
    lb.start()
    start_messages = lb.bond_messages
    lb.ctx.compute_forces(0, 0)
    lb.ctx.check()
    for k in range(60):
        lb.step(k)
    lb.ctx.check()
    assert start_messages > 0 and lb.bond_messages > start_messages
    assert lb.migrations >= 2 and lb.moved > 0
    x, v, owner = lb.state()
    xo, vo, Fo, th, st = orc.run_nve("polymer", full.pos, full.vel, full.L, [1.0, 1.0], CHAIN["dt"], 60,
                                     bonds=full.bonds, bond_prm=(CHAIN["fene_K"], CHAIN["fene_R0"]))
    assert st == 0
    tol_x, tol_v = (1e-10, 1e-10) if prec == 0 else (1e-5, 1e-5 * np.sqrt(np.mean(vo ** 2)))
    assert np.max(np.abs(min_image_diff(x, xo, full.L))) <= tol_x
    assert np.max(np.abs(v - vo)) <= tol_v
    # bonds split between subdomains, and ghosts that only the bonds bring
    a, b = full.bonds[:, 0], full.bonds[:, 1]
    assert np.count_nonzero(owner[a] != owner[b]) > 100
    ctx = lb.ctx
    o, n0 = ctx.offsets[0], ctx.n_local[0]
    gtag = ctx.tag[o + n0:o + n0 + lb.n_recv[0]].cpu().numpy()
    ridx, rimg = orc.ghost_receive(x, owner, 0, full.L, sd.lo(0), sd.hi(0), width)
    extra = np.setdiff1d(gtag, ridx)
    assert np.all(np.isin(ridx, gtag)) and extra.size > 0
    mine = np.nonzero(owner == 0)[0]
    partners = np.union1d(b[np.isin(a, mine)], a[np.isin(b, mine)])
    assert np.all(np.isin(extra, partners))


def test_bonded_subdomains_without_the_owner_table_report_it(B):
    """Skipping the start exchange leaves partners across faces of unknown
    owner: they never arrive, and the force pass reports a missing partner
    (status 12) instead of reading a wrong row."""
    sd = _chain_box()
    p = B.ModelParams(precision=B.FP64, **CHAIN)
    lb = Loopback(B, sd, p, 2 ** (1 / 6) + 0.2, 1.5, B.FIELD_POS | B.FIELD_TAG, bonds=sd.full.bonds)
    lb.select_ghosts()
    lb.ctx.compute_forces(0, 0)
    assert lb.ctx.sync_status()[0] == 12
