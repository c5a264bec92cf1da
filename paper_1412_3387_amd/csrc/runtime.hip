// runtime.hip -- host side of the C ABI: validation, workspace carving, the
// per-system descriptors, and the scheduling of one velocity-Verlet step as
// a fixed sequence of launches with device-side rebuild decisions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/hoomd_mi355x.h"
#include "device.h"
#include "launch.h"
#include "sort.h"
#include "ghost.h"

using namespace md;

#define HIP_OK(call)                                  \
    do {                                              \
        if ((call) != hipSuccess) return HOOMD_E_DEVICE; \
    } while (0)

namespace {

constexpr int kLogRows = 4096;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct Layout {
    // byte offsets into the workspace
    size_t sysdev, tpl, tpa, cpre, status, flags, tile_ctr, sysflags, thermo, thermo_log, partials, khalf, thermostat;
    size_t pos_alt, vel_alt, xbuild, nlist, nn, cell_count, cell_size, cell_idx, cell_xf, halo, halo_n;
    size_t ptag, pdir, prow, btmp, hash, slow_list, rare_list, plan, sort_ws, ghost_ws, total;
    // sizes
    int64_t rows, tiles_local, tiles_all, n_cells, nlist_entries, hash_slots;
    int cell_cap, nlist_cap, bond_cap, halo_cap, halo_lds;
    std::vector<SysDev> sys;
    std::vector<int32_t> tpl_host, tpa_host;
    std::vector<int64_t> cpre_host;
};

double pair_cut(const hoomd_params &p)
{
    if (p.pair == HOOMD_PAIR_WCA) return std::pow(2.0, 1.0 / 6.0) * p.sigma;
    return p.r_cut;
}

int cell_bins(double L, double rl)
{
    int64_t b = (int64_t)std::floor(L / rl);
    while (b > 1 && L / (double)b < rl) --b;
    return (int)std::max<int64_t>(b, 1);
}

static_assert(kForceAuto == HOOMD_FORCE_AUTO && kForceSplit == HOOMD_FORCE_SPLIT && kForceOne == HOOMD_FORCE_ONE,
              "force launch modes");

bool valid(const hoomd_params *p, int32_t n_sys, const hoomd_box *boxes)
{
    if (!p || !boxes || n_sys < 1) return false;
    // systems may be empty (no rows, or rows that hold no particle yet), but
    // a context has at least one row
    int64_t rows = 0;
    for (int s = 0; s < n_sys; ++s) rows += boxes[s].n_cap > 0 ? boxes[s].n_cap : 0;
    if (rows == 0) return false;
    for (int s = 0; s < n_sys; ++s) {
        const hoomd_params &q = p[s];
        const hoomd_box &b = boxes[s];
        if (q.precision != p[0].precision) return false;
        if (q.precision != HOOMD_FP64 && q.precision != HOOMD_MIXED) return false;
        if (q.pair < HOOMD_PAIR_LJ || q.pair > HOOMD_PAIR_DPD) return false;
        if (!(q.r_buff >= 0) || !(q.dt > 0)) return false;
        if (q.pair != HOOMD_PAIR_WCA && !(q.r_cut > 0)) return false;
        if (q.pair != HOOMD_PAIR_DPD && !(q.sigma > 0)) return false;
        // the rows of a tile share one workgroup's LDS with at least 64 halo entries
        // the framed build assembles a tile's rows in LDS
        if (q.nlist_cap < 1 || q.nlist_cap > 512) return false;
        if (q.cell_cap < 0 || q.cell_cap > 128) return false;
        if (q.halo_cap < 0 || q.halo_cap > 65535) return false;
        if (q.tpp_force < 0 || q.tpp_force > 16 || (q.tpp_force & (q.tpp_force - 1))) return false;
        if (q.bond_cap < 0 || q.bond_cap > kMaxBondCap) return false;
        if (q.check_period < 0 || q.check_period != p[0].check_period) return false;
        if (q.tune_period < 0 || q.tune_period != p[0].tune_period) return false;
        if (q.tpp_force != p[0].tpp_force || q.block_force != p[0].block_force) return false;
        if (q.integrator != HOOMD_NVE && q.integrator != HOOMD_NVT) return false;
        if (q.force_launch < HOOMD_FORCE_AUTO || q.force_launch > HOOMD_FORCE_ONE ||
            q.force_launch != p[0].force_launch)
            return false;
        if (q.integrator == HOOMD_NVT) {
            if (!(q.nvt_T0 > 0) || !std::isfinite(q.nvt_T0) || !(q.nvt_tau > 0) || !std::isfinite(q.nvt_tau))
                return false;
            if (q.nvt_group < 0) return false;
            // one thermostat per group: its systems share the step and the coupling
            for (int u = 0; u < s; ++u)
                if (q.nvt_group > 0 && p[u].integrator == HOOMD_NVT && p[u].nvt_group == q.nvt_group &&
                    (p[u].dt != q.dt || p[u].nvt_T0 != q.nvt_T0 || p[u].nvt_tau != q.nvt_tau))
                    return false;
        }
        // launch shapes: the framed build takes 64 or 32 lanes per row and 512
        // or 256 threads per workgroup (one shape for all systems); the force
        // pass runs 64 rows x tpp_force lanes per workgroup
        if (q.tpp_nlist != 0 && !nlist_shape_ok(q.tpp_nlist, nlist_block())) return false;
        if (q.block_nlist != 0 && !nlist_shape_ok(nlist_lanes_per_row(), q.block_nlist)) return false;
        if (q.tpp_nlist != p[0].tpp_nlist || q.block_nlist != p[0].block_nlist) return false;
        if (q.block_force != 0 && (q.tpp_force == 0 || q.block_force != 64 * q.tpp_force)) return false;
        if (b.n_local < 0 || b.n_cap < b.n_local || b.n_cap > (int64_t)1 << 30) return false;
        if (b.n_bonds < 0 || (b.n_bonds > 0 && q.bond_cap == 0)) return false;
        const double rl = pair_cut(q) + q.r_buff;
        for (int a = 0; a < 3; ++a) {
            if (!(b.L[a] > 0) || !std::isfinite(b.L[a]) || !std::isfinite(b.lo[a])) return false;
            if (b.periodic[a] && !(2.0 * rl < b.L[a])) return false;  // unique minimum image
        }
    }
    return true;
}

Layout make_layout(const hoomd_params *p, int32_t n_sys, const hoomd_box *boxes)
{
    Layout Lo{};
    Lo.nlist_cap = 0;
    Lo.cell_cap = 0;
    Lo.bond_cap = 0;
    int64_t row = 0, tile = 0, tile_all = 0, cell = 0, nl = 0, hslot = 0;
    Lo.tpl_host.push_back(0);
    Lo.tpa_host.push_back(0);
    Lo.cpre_host.push_back(0);
    Lo.halo_cap = 64;
    Lo.halo_lds = 64;
    for (int s = 0; s < n_sys; ++s) {
        Lo.nlist_cap = std::max(Lo.nlist_cap, p[s].nlist_cap);
        Lo.bond_cap = std::max(Lo.bond_cap, p[s].bond_cap);
    }
    for (int s = 0; s < n_sys; ++s) {
        // Halo of a compact 64-row tile (Morton-ordered rows): about the
        // density times (tile side + 2 r_list)^3.  The per-tile halo list in
        // global memory gets a wide margin; the force pass stages at most
        // halo_lds entries in LDS (sized for four or more workgroups per CU)
        // and reads any further entries from global memory.
        const int entry = force_halo_entry_bytes(p[s].pair);
        const int lds_budget = std::max(32768 / entry / 64 * 64, 64);
        const double vol = boxes[s].L[0] * boxes[s].L[1] * boxes[s].L[2];
        const double rho = (double)std::max<int64_t>(boxes[s].n_cap, 1) / vol;
        const double side = std::cbrt(64.0 / rho);
        const double rl = pair_cut(p[s]) + p[s].r_buff;
        const double est = rho * std::pow(side + 2.0 * rl, 3.0);
        const int64_t rows_up = (boxes[s].n_cap + 63) / 64 * 64;
        int hc = p[s].halo_cap;
        if (hc <= 0) {
            hc = p[s].sort_period > 0 ? (int)std::ceil((2.5 * est + 64.0) / 64.0) * 64 : 8192;
            hc = (int)std::min<int64_t>(hc, rows_up);
        }
        hc = std::min(std::max(hc, 64), 65535);
        int hl = p[s].sort_period > 0 ? (int)std::ceil(1.25 * est / 64.0) * 64 : lds_budget;
        // where the mean halo fits, stay within the share of seven
        // 256-thread workgroups in a CU's 160 KB of LDS: seven resident tiles
        // per CU outrun six, though a few more tiles go to the rare launch
        const int share7 = std::max(163840 / 7 / entry / 64 * 64, 64);
        if (p[s].sort_period > 0 && est <= share7) hl = std::min(hl, share7);
        hl = std::min(std::max(hl, 64), std::min(lds_budget, hc));
        Lo.halo_cap = std::max(Lo.halo_cap, hc);
        Lo.halo_lds = std::max(Lo.halo_lds, hl);
    }
    for (int s = 0; s < n_sys; ++s) {
        const hoomd_params &q = p[s];
        const hoomd_box &b = boxes[s];
        SysDev S{};
        const double rc = pair_cut(q);
        const double rl = rc + q.r_buff;
        double vol = 1.0;
        for (int a = 0; a < 3; ++a) {
            S.lo[a] = b.lo[a];
            S.L[a] = b.L[a];
            S.per[a] = b.periodic[a] ? 1 : 0;
            S.invL[a] = b.periodic[a] ? 1.0 / b.L[a] : 0.0;
            S.bins[a] = cell_bins(b.L[a], rl);
            S.scale[a] = (double)S.bins[a] / b.L[a];
            if (!S.per[a] || S.bins[a] >= 3) {
                S.nst[a] = 3;
                S.st[a][0] = -1; S.st[a][1] = 0; S.st[a][2] = 1;
            } else if (S.bins[a] == 2) {
                S.nst[a] = 2;
                S.st[a][0] = 0; S.st[a][1] = 1;
            } else {
                S.nst[a] = 1;
                S.st[a][0] = 0;
            }
            vol *= b.L[a];
        }
        S.row0 = row;
        S.n_local = (int32_t)b.n_local;
        S.n_total = (int32_t)b.n_local;
        S.n_cap = (int32_t)b.n_cap;
        S.nl0 = nl;
        S.cell0 = cell;
        S.tile0 = (int32_t)tile;
        S.tile0_all = (int32_t)tile_all;
        S.pair = q.pair;
        S.bond_cap = q.bond_cap;
        S.bond_stride = Lo.bond_cap;  // the partner table's row stride, shared by all systems
        S.rc2 = rc * rc;
        S.rl2 = rl * rl;
        S.disp2 = 0.25 * q.r_buff * q.r_buff;
        S.eps = q.eps;
        S.sig2 = q.sigma * q.sigma;
        if (q.pair == HOOMD_PAIR_LJ) {
            const double sr2 = S.sig2 / S.rc2;
            const double s6 = sr2 * sr2 * sr2;
            S.shift = 4.0 * q.eps * (s6 * s6 - s6);
        } else if (q.pair == HOOMD_PAIR_WCA) {
            S.shift = -q.eps;
        }
        S.dpd_A = q.dpd_A;
        S.dpd_gamma = q.dpd_gamma;
        S.dpd_sigma = std::sqrt(2.0 * q.dpd_gamma * q.dpd_kT);
        S.dpd_rc = q.r_cut;
        S.dpd_inv_rc = q.r_cut > 0 ? 1.0 / q.r_cut : 0.0;
        S.dpd_inv_sqrt_dt = 1.0 / std::sqrt(q.dt);
        S.dpd_seed = q.dpd_seed;
        S.fene_K = q.fene_K;
        S.fene_R02 = q.fene_R0 * q.fene_R0;
        S.wca_rc2 = std::pow(2.0, 1.0 / 3.0) * S.sig2;
        S.dt = q.dt;
        S.hdt = 0.5 * q.dt;
        // Nose-Hoover: the group's first system holds the thermostat
        S.nvt_slot = -1;
        if (q.integrator == HOOMD_NVT) {
            S.nvt_slot = s;
            if (q.nvt_group > 0)
                for (int u = 0; u < s; ++u)
                    if (p[u].integrator == HOOMD_NVT && p[u].nvt_group == q.nvt_group) {
                        S.nvt_slot = u;
                        break;
                    }
            S.nvt_c = q.dt / (q.nvt_tau * q.nvt_tau);
            S.nvt_T0 = q.nvt_T0;
        }
        const int64_t ncell = (int64_t)S.bins[0] * S.bins[1] * S.bins[2];
        // capacity of a cell: twice the mean occupancy plus a margin
        if (q.cell_cap > 0) {
            Lo.cell_cap = std::max(Lo.cell_cap, q.cell_cap);
        } else {
            const double mean = (double)std::max<int64_t>(b.n_cap, 1) / (double)ncell;
            int cc = (int)std::ceil((2.0 * mean + 16.0) / 8.0) * 8;
            Lo.cell_cap = std::max(Lo.cell_cap, std::min(cc, 128));
        }
        // bonded systems: a tag -> row table with at least twice as many
        // slots as rows (locals and ghosts)
        S.hash0 = hslot;
        S.hash_mask = 0;
        if (q.bond_cap > 0) {
            int64_t h = 64;
            while (h < 2 * b.n_cap) h *= 2;
            S.hash_mask = (int32_t)(h - 1);
            hslot += h;
        }
        Lo.sys.push_back(S);
        row += b.n_cap;
        // local tiles cover the rows the system may own (its capacity), so
        // that migration can change the local count without a new layout;
        // tiles past the local rows are empty
        tile += ceil_div(b.n_cap, kTile);
        tile_all += ceil_div(b.n_cap, kTile);
        cell += ncell;
        nl += ceil_div(b.n_cap, kTile) * kTile * (int64_t)Lo.nlist_cap;
        Lo.tpl_host.push_back((int32_t)tile);
        Lo.tpa_host.push_back((int32_t)tile_all);
        Lo.cpre_host.push_back(cell);
        (void)vol;
    }
    Lo.rows = row;
    Lo.hash_slots = hslot;
    Lo.tiles_local = tile;
    Lo.tiles_all = tile_all;
    Lo.n_cells = cell;
    Lo.nlist_entries = nl;

    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(std::max<size_t>(bytes, 1));
        return o;
    };
    const size_t rows = (size_t)std::max<int64_t>(row, 1);
    Lo.sysdev = take(sizeof(SysDev) * n_sys);
    Lo.tpl = take(sizeof(int32_t) * (n_sys + 1));
    Lo.tpa = take(sizeof(int32_t) * (n_sys + 1));
    Lo.cpre = take(sizeof(int64_t) * (n_sys + 1));
    Lo.status = take(sizeof(Status));
    Lo.flags = take(sizeof(int32_t) * 8);
    Lo.tile_ctr = take(sizeof(int32_t) * kTileCtrStride * kDies);
    Lo.sysflags = take(sizeof(int32_t) * 4 * (size_t)n_sys);
    Lo.thermo = take(sizeof(double) * 4 * n_sys);
    Lo.thermo_log = take(sizeof(double) * 5 * (size_t)n_sys * kLogRows);
    Lo.partials = take(sizeof(double) * 3 * (size_t)std::max<int64_t>(tile, 1) * 64);
    Lo.khalf = take(sizeof(double) * (size_t)std::max<int64_t>(tile, 1) * 16);
    Lo.thermostat = take(sizeof(double) * 2 * (size_t)n_sys);
    Lo.pos_alt = take(sizeof(double4) * rows);
    Lo.vel_alt = take(sizeof(double4) * rows);
    Lo.xbuild = take(sizeof(double4) * rows);
    // padded: the force pass reads up to force_row_over_read() entries past
    // any row's end
    Lo.nlist = take(sizeof(uint16_t) * ((size_t)std::max<int64_t>(nl, 1) + (size_t)force_row_over_read() * kTile));
    Lo.halo = take(sizeof(int32_t) * (size_t)std::max<int64_t>(tile, 1) * Lo.halo_cap);
    Lo.halo_n = take(sizeof(int32_t) * (size_t)std::max<int64_t>(tile, 1));
    Lo.nn = take(sizeof(int32_t) * rows);
    Lo.cell_count = take(sizeof(int32_t) * (size_t)cell);
    Lo.cell_size = take(sizeof(int32_t) * (size_t)cell);
    Lo.cell_idx = take(sizeof(int32_t) * (size_t)cell * Lo.cell_cap);
    Lo.cell_xf = take(sizeof(float4) * (size_t)cell * Lo.cell_cap);
    const size_t brows = Lo.bond_cap > 0 ? rows * (size_t)Lo.bond_cap : 1;
    Lo.ptag = take(sizeof(int32_t) * brows);
    Lo.pdir = take(sizeof(int32_t) * brows);
    Lo.prow = take(sizeof(int32_t) * brows);
    Lo.btmp = take(sizeof(int32_t) * brows);
    Lo.hash = take(sizeof(int2) * (size_t)std::max<int64_t>(Lo.hash_slots, 1));
    Lo.slow_list = take(sizeof(int32_t) * (size_t)std::max<int64_t>(tile, 1));
    Lo.rare_list = take(sizeof(int32_t) * (size_t)std::max<int64_t>(tile, 1));
    Lo.plan = take(build_plan_bytes(tile));
    Lo.sort_ws = take(sort_workspace_bytes((int64_t)rows));
    Lo.ghost_ws = take(ghost_workspace_bytes((int64_t)rows, n_sys));
    Lo.total = off;
    return Lo;
}

}  // namespace

struct hoomd_ctx {
    hipStream_t stream;
    int n_sys;
    std::vector<hoomd_params> prm;
    std::vector<hoomd_box> box;
    hoomd_arrays arr;
    char *ws;
    Layout lay;
    LaunchCtx L;
    SortBuffers sortb;
    GhostBuffers ghostb;
    int mixed;
    int pair_uniform;  // common Pair of all systems, or -1
    bool built;        // a neighbour list exists for the current rows
    int64_t ghosts;    // ghost rows appended over all systems (no sorting then)
    std::vector<char> bond_ok;  // per system: tag -> row table and partner rows match the rows
    int tpp_nlist, block_nlist, tpp_force, block_force;
    // autotuner state: shapes fixed by the caller are not tuned
    bool fixed_force, fixed_nlist;
    int tune_period;
    uint64_t last_tune_step;
    bool retune;
    int scans, from_cache;
    float force_ms[5], build_ms[4];
    int check_period;  // displacement check every this many steps after a build
    int last_log_rows;
    uint64_t steps_done;
    // phase timing (hoomd_profile)
    bool profiling;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used;
    std::vector<std::pair<size_t, size_t>> ev_force, ev_rebuild;
    // captured runs of middle steps, per buffer parity: [p][0] two steps,
    // [p][1] 2 kLongPairs steps
    hipStream_t cap_stream;
    hipGraphExec_t graph_exec[2][2];
    int graph_sig[2][2];  // launch shapes the graph was captured with
    ~hoomd_ctx()
    {
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        for (int p = 0; p < 2; ++p)
            for (int k = 0; k < 2; ++k)
                if (graph_exec[p][k]) (void)hipGraphExecDestroy(graph_exec[p][k]);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

namespace {

template <typename T> T *ws_ptr(hoomd_ctx *c, size_t off) { return reinterpret_cast<T *>(c->ws + off); }

// Tiles that hold local rows, over all systems (the force pass's choice of
// one launch or two depends on it).
void count_busy_tiles(hoomd_ctx *c)
{
    int64_t t = 0;
    for (const SysDev &S : c->lay.sys) t += (S.n_local + kTile - 1) / kTile;
    c->L.busy_tiles = (int)t;
}

void default_tuning(hoomd_ctx *c)
{
    // neighbours per particle and particles per CU decide the lane count;
    // the autotuner refines these on the live state
    // the build always runs 4 lanes per row, one 64-row tile per 256-thread
    // workgroup; the force pass runs W lanes per row, one tile per 64 W
    // threads
    const double per_cu = (double)c->lay.tiles_local * 64.0 / 256.0;
    c->tpp_nlist = nlist_lanes_per_row();
    c->block_nlist = nlist_block();
    if (c->prm[0].tpp_nlist > 0) c->tpp_nlist = c->prm[0].tpp_nlist;
    if (c->prm[0].block_nlist > 0) c->block_nlist = c->prm[0].block_nlist;
    c->fixed_nlist = c->prm[0].tpp_nlist > 0 || c->prm[0].block_nlist > 0;
    c->fixed_force = c->prm[0].tpp_force > 0;
    c->tpp_force = per_cu > 2048 ? 4 : 8;
    if (c->prm[0].tpp_force > 0) c->tpp_force = c->prm[0].tpp_force;
    c->block_force = 64 * c->tpp_force;
}

bool pow2_le(int v, int hi) { return v >= 1 && v <= hi && (v & (v - 1)) == 0; }

// Record the next pooled event on the stream when profiling; returns its
// index (unused otherwise).
size_t mark(hoomd_ctx *c)
{
    if (!c->profiling) return 0;
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
            c->profiling = false;
            return 0;
        }
        c->ev_pool.push_back(e);
    }
    const size_t k = c->ev_used++;
    if (hipEventRecord(c->ev_pool[k], c->stream) != hipSuccess) c->profiling = false;
    return k;
}

// Device flags: 0 and 1 rebuild flags of the two buffer parities, 2 the flag
// of explicit builds, 3 unused, 4 build counter, 5 step counter of replayed steps, 6
// tiles passed from the framed build to the general one, 7 tiles the force
// pass handles in its second launch.
int32_t *flag_ptr(hoomd_ctx *c, int k) { return ws_ptr<int32_t>(c, c->lay.flags) + k; }

// Per-system words, n_sys each: k = 0, 1, 2 the rebuild flags of each system
// that go with device flags 0, 1, 2 (a batch rebuilds only the systems whose
// particles moved far enough); k = 3 each system's steps since its last build.
int32_t *sflag_ptr(hoomd_ctx *c, int k) { return ws_ptr<int32_t>(c, c->lay.sysflags) + (size_t)k * c->n_sys; }

// Queue the rebuild sequence: bin -> per-cell sort -> neighbour rows.  Every
// kernel returns at once when *flag is clear.  The binning launch also keeps
// the count of steps since the last build: reset by a build, else advanced by
// since_inc (1 after a step, 0 after an explicit build request).
// nvt_w > 0: the binning launch also does the Nose-Hoover update of the
// force launch before it (w lanes per particle).
void queue_rebuild(hoomd_ctx *c, const double4 *pos, const int32_t *tag, int slot, int since_inc, int nvt_w = 0)
{
    c->L.flag = flag_ptr(c, slot);
    c->L.sflag = sflag_ptr(c, slot);
    c->L.since_inc = since_inc;
    launch_bin(c->L, pos, nvt_w);
    launch_cell_sort(c->L, pos);
    launch_nlist(c->L, pos, tag, c->tpp_nlist, c->block_nlist);
}

ForceLaunch base_force(hoomd_ctx *c)
{
    ForceLaunch F{};
    F.tag = c->arr.tag;
    F.force = c->arr.force;
    F.mixed = c->mixed;
    F.pair = c->pair_uniform;
    F.since = sflag_ptr(c, 3);
    F.check_period = c->check_period;
    F.thermostat = c->L.nvt ? c->L.thermostat : nullptr;
    F.khalf = nullptr;
    return F;
}

uint32_t *step_counter_ptr(hoomd_ctx *c) { return reinterpret_cast<uint32_t *>(flag_ptr(c, 5)); }

// One middle step at buffer parity p: fused launch, then the rebuild queue.
// Every argument depends only on p, so the pair (p, p^1) can be captured once
// and replayed.
void queue_mid_step(hoomd_ctx *c, int p, double4 *const *P, double4 *const *V, bool dpd)
{
    ForceLaunch F = base_force(c);
    F.pos = P[p];
    F.pos_out = P[p ^ 1];
    F.vel = V[dpd ? p : 0];
    F.vel_out = V[dpd ? p ^ 1 : 0];
    F.timestep_ptr = step_counter_ptr(c);
    F.mode = MODE_MID;
    F.flag_set = flag_ptr(c, p);
    F.flag_clear = flag_ptr(c, p ^ 1);
    F.sflag_set = sflag_ptr(c, p);
    F.sflag_clear = sflag_ptr(c, p ^ 1);
    if (c->L.nvt) F.khalf = c->L.khalf;
    launch_force(c->L, F, c->tpp_force, c->block_force);
    queue_rebuild(c, P[p ^ 1], c->arr.tag, p, 1, c->L.nvt ? c->tpp_force : 0);
}

// Pairs of middle steps in the long captured run: one graph launch per 16
// steps instead of per 2 (each launch leaves a gap of some microseconds).
constexpr int kLongPairs = 8;

int ensure_step_graph(hoomd_ctx *c, int p, int kind, double4 *const *P, double4 *const *V, bool dpd)
{
    hipGraphExec_t &ge = c->graph_exec[p][kind];
    const int sig = c->tpp_force | (c->tpp_nlist << 8) | (c->block_nlist << 16);
    if (ge && c->graph_sig[p][kind] == sig) return HOOMD_OK;
    if (ge) {
        (void)hipGraphExecDestroy(ge);
        ge = nullptr;
    }
    // capture on a private stream (the caller's may be the null stream, which
    // cannot be captured); the graph is launched on the caller's stream
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return HOOMD_E_DEVICE;
    const hipStream_t keep = c->L.stream;
    c->L.stream = c->cap_stream;
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        const int pairs = kind ? kLongPairs : 1;
        for (int k = 0; k < pairs; ++k) {
            queue_mid_step(c, p, P, V, dpd);
            queue_mid_step(c, p ^ 1, P, V, dpd);
        }
        ok = hipStreamEndCapture(c->cap_stream, &g) == hipSuccess && g;
    }
    c->L.stream = keep;
    if (ok) ok = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
        ge = nullptr;
        return HOOMD_E_DEVICE;
    }
    c->graph_sig[p][kind] = sig;
    return HOOMD_OK;
}

// Scans every candidate launch shape (or takes a cached choice); defined
// with the autotuner below.
int tune_now(hoomd_ctx *c, bool use_cache);

}  // namespace

extern "C" {

size_t hoomd_workspace_bytes(const hoomd_params *params, int32_t n_sys, const hoomd_box *boxes)
{
    if (!valid(params, n_sys, boxes)) return 0;
    return make_layout(params, n_sys, boxes).total;
}

int hoomd_init(hoomd_ctx **out, const hoomd_params *params, int32_t n_sys, const hoomd_box *boxes,
               const hoomd_arrays *arrays, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!out || !arrays || !workspace) return HOOMD_E_ARG;
    *out = nullptr;
    if (!valid(params, n_sys, boxes)) return HOOMD_E_ARG;
    if (!arrays->pos || !arrays->vel || !arrays->force || !arrays->tag) return HOOMD_E_ARG;
    Layout lay = make_layout(params, n_sys, boxes);
    if (workspace_bytes < lay.total) return HOOMD_E_WORKSPACE;
    int64_t nb_total = 0;
    for (int s = 0; s < n_sys; ++s) nb_total += boxes[s].n_bonds;
    if (nb_total > 0 && !arrays->bonds) return HOOMD_E_ARG;

    hoomd_ctx *c = new hoomd_ctx();
    c->stream = (hipStream_t)stream;
    c->n_sys = n_sys;
    c->prm.assign(params, params + n_sys);
    c->box.assign(boxes, boxes + n_sys);
    c->arr = *arrays;
    c->ws = (char *)workspace;
    c->lay = lay;
    c->mixed = params[0].precision == HOOMD_MIXED;
    // LJ and WCA run the same kernel (WCA is LJ with its own cut-off and
    // shift, carried per system); DPD needs its own and cannot be mixed in
    c->pair_uniform = params[0].pair == HOOMD_PAIR_DPD ? PAIR_DPD : PAIR_LJ;
    for (int s = 1; s < n_sys; ++s)
        if ((params[s].pair == HOOMD_PAIR_DPD) != (c->pair_uniform == PAIR_DPD)) c->pair_uniform = -1;
    if (c->pair_uniform < 0) {
        delete c;
        return HOOMD_E_ARG;
    }
    c->built = false;
    c->check_period = params[0].check_period > 1 ? params[0].check_period : 1;
    c->tune_period = params[0].tune_period;
    c->last_log_rows = 0;
    c->steps_done = 0;

    LaunchCtx &L = c->L;
    L.stream = c->stream;
    L.n_sys = n_sys;
    L.sys = ws_ptr<SysDev>(c, lay.sysdev);
    L.tprefix_local = ws_ptr<int32_t>(c, lay.tpl);
    L.tprefix_all = ws_ptr<int32_t>(c, lay.tpa);
    L.cprefix = ws_ptr<int64_t>(c, lay.cpre);
    L.tiles_local = (int)lay.tiles_local;
    L.tiles_all = (int)lay.tiles_all;
    L.n_cells = lay.n_cells;
    L.cell_cap = lay.cell_cap;
    L.cell_count = ws_ptr<int32_t>(c, lay.cell_count);
    L.cell_size = ws_ptr<int32_t>(c, lay.cell_size);
    L.cell_idx = ws_ptr<int32_t>(c, lay.cell_idx);
    L.cell_xf = ws_ptr<float4>(c, lay.cell_xf);
    L.nlist = ws_ptr<uint16_t>(c, lay.nlist);
    L.halo = ws_ptr<int32_t>(c, lay.halo);
    L.halo_n = ws_ptr<int32_t>(c, lay.halo_n);
    L.halo_cap = lay.halo_cap;
    L.halo_lds = std::min(lay.halo_lds, lay.halo_cap);
    L.nn = ws_ptr<int32_t>(c, lay.nn);
    L.nlist_cap = lay.nlist_cap;
    L.xbuild = ws_ptr<double4>(c, lay.xbuild);
    L.ptag = ws_ptr<int32_t>(c, lay.ptag);
    L.pdir = ws_ptr<int32_t>(c, lay.pdir);
    L.prow = ws_ptr<int32_t>(c, lay.prow);
    L.btmp = ws_ptr<int32_t>(c, lay.btmp);
    L.hash = ws_ptr<int2>(c, lay.hash);
    L.bond_stride = lay.bond_cap;
    L.has_bonds = nb_total > 0;
    L.flag = flag_ptr(c, 0);
    L.build_count = flag_ptr(c, 4);
    L.sflag = nullptr;  // set with L.flag by queue_rebuild
    L.since = sflag_ptr(c, 3);
    L.since_inc = 0;
    L.slow_list = ws_ptr<int32_t>(c, lay.slow_list);
    L.slow_n = flag_ptr(c, 6);
    L.rare_list = ws_ptr<int32_t>(c, lay.rare_list);
    L.plan = ws_ptr<char>(c, lay.plan);
    L.rare_n = flag_ptr(c, 7);
    L.tile_ctr = ws_ptr<int32_t>(c, lay.tile_ctr);
    L.status = ws_ptr<Status>(c, lay.status);
    L.partials = ws_ptr<double>(c, lay.partials);
    L.thermo = ws_ptr<double>(c, lay.thermo);
    L.thermo_log = ws_ptr<double>(c, lay.thermo_log);
    L.khalf = ws_ptr<double>(c, lay.khalf);
    L.thermostat = ws_ptr<double>(c, lay.thermostat);
    L.nvt = false;
    for (int s = 0; s < n_sys; ++s) L.nvt = L.nvt || params[s].integrator == HOOMD_NVT;
    L.force_launch = params[0].force_launch;
    count_busy_tiles(c);
    c->sortb = make_sort_buffers(c->ws + lay.sort_ws, lay.rows);
    c->ghostb = make_ghost_buffers(c->ws + lay.ghost_ws, lay.rows, n_sys);
    default_tuning(c);
    if (!pow2_le(c->tpp_force, 16)) {
        delete c;
        return HOOMD_E_ARG;
    }

    // descriptors, prefixes, cleared counters (synchronous: init is not hot)
    hipError_t e = prepare_nlist(lay.nlist_cap);
    if (e == hipSuccess) e = prepare_force();
    if (e == hipSuccess) e = hipMemcpy(c->ws + lay.sysdev, lay.sys.data(), sizeof(SysDev) * n_sys, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->ws + lay.tpl, lay.tpl_host.data(), sizeof(int32_t) * (n_sys + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->ws + lay.tpa, lay.tpa_host.data(), sizeof(int32_t) * (n_sys + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->ws + lay.cpre, lay.cpre_host.data(), sizeof(int64_t) * (n_sys + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(c->ws + lay.status, 0, sizeof(Status));
    if (e == hipSuccess) e = hipMemset(c->ws + lay.flags, 0, sizeof(int32_t) * 8);
    if (e == hipSuccess) e = hipMemset(c->ws + lay.tile_ctr, 0, sizeof(int32_t) * kTileCtrStride * kDies);
    if (e == hipSuccess) e = hipMemset(c->ws + lay.sysflags, 0, sizeof(int32_t) * 4 * (size_t)n_sys);
    if (e == hipSuccess) e = hipMemset(c->ws + lay.cell_count, 0, sizeof(int32_t) * (size_t)std::max<int64_t>(lay.n_cells, 1));
    if (e == hipSuccess) e = hipMemset(c->ws + lay.thermo, 0, sizeof(double) * 4 * n_sys);
    if (e == hipSuccess) e = hipMemset(c->ws + lay.thermostat, 0, sizeof(double) * 2 * n_sys);
    // bond partner entries per row (built on the host from the caller's table)
    if (e == hipSuccess && lay.bond_cap > 0) {
        // per row: partner tags and the direction of each partner's owner
        // (13 here; -1 not known yet: a subdomain's partners beyond its
        // frame, found by the start messages of pack_bond_ranks)
        std::vector<int32_t> ptag((size_t)lay.rows * lay.bond_cap, -1), pdir((size_t)lay.rows * lay.bond_cap, -1);
        std::vector<int32_t> pairs;
        std::vector<int32_t> tags((size_t)lay.rows);
        e = hipMemcpy(tags.data(), arrays->tag, sizeof(int32_t) * lay.rows, hipMemcpyDeviceToHost);
        int64_t b0 = 0;
        for (int s = 0; s < n_sys && e == hipSuccess; ++s) {
            const int64_t nb = boxes[s].n_bonds;
            const bool closed = boxes[s].periodic[0] && boxes[s].periodic[1] && boxes[s].periodic[2];
            // tags of the system's rows: unique, non-negative
            std::unordered_map<int32_t, int64_t> row_of;
            for (int64_t r = 0; r < boxes[s].n_local && e == hipSuccess; ++r) {
                const int32_t t = tags[(size_t)(lay.sys[s].row0 + r)];
                if (t < 0 || !row_of.emplace(t, lay.sys[s].row0 + r).second) e = hipErrorInvalidValue;
            }
            if (nb > 0 && e == hipSuccess) {
                pairs.resize((size_t)nb * 2);
                e = hipMemcpy(pairs.data(), arrays->bonds + 2 * b0, sizeof(int32_t) * 2 * nb, hipMemcpyDeviceToHost);
                for (int64_t k = 0; k < nb && e == hipSuccess; ++k) {
                    const int32_t ta = pairs[2 * k], tb = pairs[2 * k + 1];
                    const auto ia = row_of.find(ta), ib = row_of.find(tb);
                    const bool la = ia != row_of.end(), lb = ib != row_of.end();
                    // a bond has a local member; in a closed box both are local
                    if (ta < 0 || tb < 0 || ta == tb || (!la && !lb) || (closed && !(la && lb))) {
                        e = hipErrorInvalidValue;
                        break;
                    }
                    for (int side = 0; side < 2 && e == hipSuccess; ++side) {
                        if (!(side ? lb : la)) continue;
                        const int64_t me = side ? ib->second : ia->second;
                        const bool other_here = side ? la : lb;
                        int32_t *slot = &ptag[(size_t)me * lay.bond_cap];
                        int q = 0;
                        while (q < params[s].bond_cap && slot[q] >= 0) ++q;
                        if (q == params[s].bond_cap) {
                            e = hipErrorInvalidValue;
                            break;
                        }
                        slot[q] = side ? ta : tb;
                        pdir[(size_t)me * lay.bond_cap + q] = other_here ? 13 : -1;
                    }
                }
            }
            b0 += nb;
        }
        if (e == hipSuccess)
            e = hipMemcpy(c->ws + lay.ptag, ptag.data(), sizeof(int32_t) * ptag.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(c->ws + lay.pdir, pdir.data(), sizeof(int32_t) * pdir.size(), hipMemcpyHostToDevice);
        if (e == hipErrorInvalidValue) {
            delete c;
            return HOOMD_E_ARG;
        }
    }
    if (e != hipSuccess) {
        delete c;
        return HOOMD_E_DEVICE;
    }
    launch_bond_refresh(c->L, c->arr.tag, -1);
    c->bond_ok.assign((size_t)n_sys, 1);
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        delete c;
        return HOOMD_E_DEVICE;
    }
    *out = c;
    return HOOMD_OK;
}

void hoomd_destroy(hoomd_ctx *ctx) { delete ctx; }

int build_nlist(hoomd_ctx *c, int32_t force_rebuild)
{
    if (!c) return HOOMD_E_ARG;
    int32_t *flag = flag_ptr(c, 2);
    int32_t *sflag = sflag_ptr(c, 2);
    double4 *pos = reinterpret_cast<double4 *>(c->arr.pos);
    if (force_rebuild || !c->built) {
        // with spatial sorting enabled, every full build starts from Morton
        // order so that the 64-row tiles are compact clusters
        if (c->prm[0].sort_period > 0 && c->ghosts == 0) {
            if (queue_morton_sort(c->L, c->sortb, pos, reinterpret_cast<double4 *>(c->arr.vel), c->arr.tag,
                                  ws_ptr<double4>(c, c->lay.pos_alt), ws_ptr<double4>(c, c->lay.vel_alt)))
                return HOOMD_E_DEVICE;
            launch_bond_refresh(c->L, c->arr.tag, -1);
        }
        launch_set_flags(c->L, flag, sflag, 1);
    } else {
        launch_set_flags(c->L, flag, sflag, 0);
        launch_disp_check(c->L, pos, flag, sflag);
    }
    queue_rebuild(c, pos, c->arr.tag, 2, 0);
    c->built = true;
    return hipGetLastError() == hipSuccess ? HOOMD_OK : HOOMD_E_DEVICE;
}

int compute_forces(hoomd_ctx *c, uint64_t timestep, uint32_t flags)
{
    if (!c) return HOOMD_E_ARG;
    int rc = build_nlist(c, 0);
    if (rc) return rc;
    ForceLaunch F = base_force(c);
    F.pos = reinterpret_cast<const double4 *>(c->arr.pos);
    F.vel = reinterpret_cast<const double4 *>(c->arr.vel);
    F.vel_out = reinterpret_cast<double4 *>(c->arr.vel);
    F.timestep = (uint32_t)timestep;
    F.mode = MODE_FORCE;
    F.log = flags != 0;
    F.energy = (flags & HOOMD_ENERGY) ? 1 : 0;
    launch_force(c->L, F, c->tpp_force, c->block_force);
    if (F.log) launch_thermo_reduce(c->L, c->tpp_force, -1, (double)timestep);
    return hipGetLastError() == hipSuccess ? HOOMD_OK : HOOMD_E_DEVICE;
}

int step(hoomd_ctx *c, uint64_t t0, int32_t n_steps, int32_t log_every)
{
    if (!c || n_steps < 0) return HOOMD_E_ARG;
    if (n_steps == 0) return HOOMD_OK;
    for (int s = 0; s < c->n_sys; ++s)
        if (c->lay.sys[s].n_total != c->lay.sys[s].n_local || !c->box[s].periodic[0] ||
            !c->box[s].periodic[1] || !c->box[s].periodic[2])
            return HOOMD_E_STATE;  // stepping a subdomain needs particle migration
    if (c->tune_period > 0 &&
        (c->retune || c->scans + c->from_cache == 0 || c->steps_done - c->last_tune_step >= (uint64_t)c->tune_period)) {
        const int trc = tune_now(c, false);
        if (trc) return trc;
    }
    int rc = build_nlist(c, 0);
    if (rc) return rc;

    const bool dpd = c->pair_uniform == PAIR_DPD;
    double4 *P[2] = {reinterpret_cast<double4 *>(c->arr.pos), ws_ptr<double4>(c, c->lay.pos_alt)};
    double4 *V[2] = {reinterpret_cast<double4 *>(c->arr.vel), ws_ptr<double4>(c, c->lay.vel_alt)};
    int32_t *tag = c->arr.tag;
    int log_row = 0;
    const int sort_period = c->prm[0].sort_period;
    const bool graphs = c->prm[0].use_graph && !c->profiling;
    // the DPD key of each launch comes from a device counter that the
    // binning launch after it advances, so graph replays see the right step
    uint32_t *counter = step_counter_ptr(c);
    launch_set_flag(c->L, reinterpret_cast<int32_t *>(counter), (int32_t)(uint32_t)t0);
    c->L.step_counter = counter;
    auto sorts_after = [&](int32_t s) {
        return sort_period > 0 && ((t0 + (uint64_t)s + 1) % (uint64_t)sort_period) == 0;
    };
    auto logs_at = [&](int32_t s) { return log_every > 0 && (s % log_every == 0 || s == n_steps); };
    int32_t s = 0;
    while (s <= n_steps) {
        const uint64_t t = t0 + (uint64_t)s;
        const int p = s & 1;  // parity of the position (and DPD velocity) buffers
        // middle steps with nothing eager in between replay as one graph:
        // 2 kLongPairs of them where they all qualify, else two
        if (graphs && s > 0) {
            int run = 0;
            while (run < 2 * kLongPairs && s + run < n_steps && !logs_at(s + run) && !sorts_after(s + run))
                ++run;
            if (run >= 2) {
                const int kind = run == 2 * kLongPairs ? 1 : 0;
                if (ensure_step_graph(c, p, kind, P, V, dpd) != HOOMD_OK) {
                    c->L.step_counter = nullptr;
                    return HOOMD_E_DEVICE;
                }
                if (hipGraphLaunch(c->graph_exec[p][kind], c->stream) != hipSuccess) {
                    c->L.step_counter = nullptr;
                    return HOOMD_E_DEVICE;
                }
                s += kind ? 2 * kLongPairs : 2;
                continue;
            }
        }
        ForceLaunch F = base_force(c);
        F.pos = P[p];
        F.pos_out = P[p ^ 1];
        F.vel = V[dpd ? p : 0];
        F.vel_out = V[dpd ? p ^ 1 : 0];
        F.tag = tag;
        F.timestep = (uint32_t)t;
        F.timestep_ptr = counter;
        F.mode = s == 0 ? MODE_FIRST : (s == n_steps ? MODE_LAST : MODE_MID);
        F.flag_set = F.mode == MODE_LAST ? nullptr : flag_ptr(c, p);
        F.flag_clear = F.mode == MODE_LAST ? nullptr : flag_ptr(c, p ^ 1);
        F.sflag_set = F.mode == MODE_LAST ? nullptr : sflag_ptr(c, p);
        F.sflag_clear = F.mode == MODE_LAST ? nullptr : sflag_ptr(c, p ^ 1);
        F.log = logs_at(s);
        F.energy = F.mode == MODE_LAST ? 1 : 0;
        if (F.mode == MODE_LAST) F.log = F.log || log_every > 0;
        if (c->L.nvt && F.mode != MODE_LAST) F.khalf = c->L.khalf;
        const size_t e0 = mark(c);
        launch_force(c->L, F, c->tpp_force, c->block_force);
        if (c->profiling) c->ev_force.emplace_back(e0, mark(c));
        // (a force launch with half-step partials is followed by a rebuild
        // queue, whose binning launch does the thermostat update)
        if (F.log) {
            launch_thermo_reduce(c->L, c->tpp_force, log_row < kLogRows ? log_row : -1, (double)t);
            ++log_row;
        }
        if (F.mode == MODE_LAST) break;
        if (sorts_after(s)) {
            rc = queue_morton_sort(c->L, c->sortb, P[p ^ 1], V[dpd ? p ^ 1 : 0], tag, P[p],
                                   V[dpd ? p : 1]);
            if (rc) {
                c->L.step_counter = nullptr;
                return HOOMD_E_DEVICE;
            }
            launch_bond_refresh(c->L, tag, -1);
            launch_set_flags(c->L, flag_ptr(c, p), sflag_ptr(c, p), 1);  // a sort moves every system's rows
        }
        const size_t r0 = mark(c);
        queue_rebuild(c, P[p ^ 1], tag, p, 1, F.khalf ? c->tpp_force : 0);
        if (c->profiling) c->ev_rebuild.emplace_back(r0, mark(c));
        ++s;
    }
    c->L.step_counter = nullptr;
    const int pc = n_steps & 1;
    const int vc = dpd ? (n_steps + 1) & 1 : 0;
    // leave the final state in the caller's arrays
    if (pc == 1)
        HIP_OK(hipMemcpyAsync(c->arr.pos, P[1], sizeof(double4) * c->lay.rows, hipMemcpyDeviceToDevice, c->stream));
    if (vc == 1)
        HIP_OK(hipMemcpyAsync(c->arr.vel, V[1], sizeof(double4) * c->lay.rows, hipMemcpyDeviceToDevice, c->stream));
    c->last_log_rows = std::min(log_row, kLogRows);
    c->steps_done += (uint64_t)n_steps;
    return hipGetLastError() == hipSuccess ? HOOMD_OK : HOOMD_E_DEVICE;
}

int pack_ghosts(hoomd_ctx *c, int32_t sys, const hoomd_subdomain *sd, int32_t mode, uint32_t fields,
                void *send, int64_t send_cap, int32_t *counts26, int32_t *offsets26)
{
    if (!c || !sd || sys < 0 || sys >= c->n_sys || !counts26 || !offsets26) return HOOMD_E_ARG;
    if (mode != HOOMD_GHOST_SELECT && mode != HOOMD_GHOST_UPDATE) return HOOMD_E_ARG;
    if ((fields & ~7u) || send_cap < 0 || (send_cap > 0 && !send)) return HOOMD_E_ARG;
    if (!(sd->width >= 0)) return HOOMD_E_ARG;
    GhostArgs g{};
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = sd->lo[a];
        g.hi[a] = sd->hi[a];
    }
    g.width = sd->width;
    g.row0 = c->lay.sys[sys].row0;
    g.n_local = c->lay.sys[sys].n_local;
    g.fields = fields;
    g.send = send;
    g.send_cap = send_cap;
    g.counts = counts26;
    g.offsets = offsets26;
    g.pos = reinterpret_cast<const double4 *>(c->arr.pos);
    g.vel = reinterpret_cast<const double4 *>(c->arr.vel);
    g.tag = c->arr.tag;
    g.status = c->L.status;
    g.mask = c->ghostb.mask + c->lay.sys[sys].row0;
    g.list = c->ghostb.list + (int64_t)kGhostPerRow * c->lay.sys[sys].row0;
    g.list_cap = (int64_t)kGhostPerRow * c->box[sys].n_cap;
    g.total = c->ghostb.totals + sys;
    if (c->lay.sys[sys].bond_cap > 0) {
        // a particle also goes wherever one of its partners is owned (Sec. 4.3.4)
        g.ptag = c->L.ptag;
        g.pdir = c->L.pdir;
        g.bond_stride = c->lay.bond_cap;
        g.bond_cap = c->lay.sys[sys].bond_cap;
    }
    int rc = mode == HOOMD_GHOST_SELECT ? queue_ghost_select(c->stream, c->ghostb, g)
                                        : queue_ghost_update(c->stream, c->ghostb, g);
    return rc ? HOOMD_E_DEVICE : HOOMD_OK;
}

int pack_ghosts_noalloc(const double *pos, const double *vel, const int32_t *tag, int64_t n_local,
                        const hoomd_subdomain *sd, uint32_t fields, void *send, int64_t send_cap,
                        int32_t *counts26, int32_t *offsets26, void *stream)
{
    if (!sd || !counts26 || !offsets26 || n_local < 0 || n_local > ghost_static_max_rows()) return HOOMD_E_ARG;
    if ((fields & ~7u) || send_cap < 0 || (send_cap > 0 && !send)) return HOOMD_E_ARG;
    if ((n_local > 0 && !pos) || ((fields & HOOMD_FIELD_VEL) && !vel) || ((fields & HOOMD_FIELD_TAG) && !tag))
        return HOOMD_E_ARG;
    if (!(sd->width >= 0)) return HOOMD_E_ARG;
    GhostArgs g{};
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = sd->lo[a];
        g.hi[a] = sd->hi[a];
    }
    g.width = sd->width;
    g.row0 = 0;
    g.n_local = (int32_t)n_local;
    g.fields = fields;
    g.send = send;
    g.send_cap = send_cap;
    g.counts = counts26;
    g.offsets = offsets26;
    g.pos = reinterpret_cast<const double4 *>(pos);
    g.vel = reinterpret_cast<const double4 *>(vel);
    g.tag = tag;
    return queue_ghost_select_static((hipStream_t)stream, g) ? HOOMD_E_DEVICE : HOOMD_OK;
}

int integrate_half_step(hoomd_ctx *c, int32_t which, uint64_t timestep)
{
    if (!c || (which != 0 && which != 1)) return HOOMD_E_ARG;
    int32_t *flag = flag_ptr(c, 2), *sflag = sflag_ptr(c, 2);
    if (which == 1) {
        const int rc = compute_forces(c, timestep, 0);
        if (rc) return rc;
    } else {
        launch_set_flags(c->L, flag, sflag, 0);  // set again by the displacement check below
    }
    launch_half_step(c->L, reinterpret_cast<double4 *>(c->arr.pos), reinterpret_cast<double4 *>(c->arr.vel),
                     c->arr.force, c->mixed != 0, which, flag, sflag);
    if (which == 0) launch_nvt_update(c->L, 1);  // one wave per tile in the half-step launch
    return hipGetLastError() == hipSuccess ? HOOMD_OK : HOOMD_E_DEVICE;
}

int pack_bond_ranks(hoomd_ctx *c, int32_t sys, const hoomd_subdomain *sd, int32_t mode, void *send,
                    int64_t send_cap, int32_t *counts26, int32_t *offsets26, int64_t *n_sent)
{
    if (!c || !sd || sys < 0 || sys >= c->n_sys || !counts26 || !offsets26 || !n_sent) return HOOMD_E_ARG;
    if (mode != HOOMD_BOND_START && mode != HOOMD_BOND_MIGRATE) return HOOMD_E_ARG;
    if (send_cap < 0 || (send_cap > 0 && !send)) return HOOMD_E_ARG;
    const SysDev &S = c->lay.sys[sys];
    if (S.bond_cap == 0) return HOOMD_E_STATE;
    if (!c->bond_ok[sys]) return HOOMD_E_STATE;  // rows changed since the partner rows were found
    BondRankArgs a{};
    for (int k = 0; k < 3; ++k) {
        a.lo[k] = sd->lo[k];
        a.hi[k] = sd->hi[k];
    }
    a.row0 = S.row0;
    a.n_local = S.n_local;
    a.mode = mode;
    a.stride = c->lay.bond_cap;
    a.bond_cap = S.bond_cap;
    a.pos = reinterpret_cast<const double4 *>(c->arr.pos);
    a.tag = c->arr.tag;
    a.ptag = c->L.ptag;
    a.pdir = c->L.pdir;
    a.prow = c->L.prow;
    a.send = send;
    a.send_cap = send_cap;
    a.counts = counts26;
    a.offsets = offsets26;
    a.cursor = c->ghostb.cursor;
    a.status = c->L.status;
    if (queue_bond_ranks(c->stream, a, c->ghostb.cursor + 26)) return HOOMD_E_DEVICE;
    int32_t total = 0;
    HIP_OK(hipMemcpyAsync(&total, c->ghostb.cursor + 26, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    *n_sent = total;
    if (total > send_cap) return HOOMD_E_GHOST_OVERFLOW;
    return hipGetLastError() == hipSuccess ? HOOMD_OK : HOOMD_E_DEVICE;
}

int unpack_bond_ranks(hoomd_ctx *c, int32_t sys, const void *recv, int64_t n_recv, int32_t mode)
{
    if (!c || sys < 0 || sys >= c->n_sys || n_recv < 0 || (n_recv > 0 && !recv)) return HOOMD_E_ARG;
    if (mode != HOOMD_BOND_START && mode != HOOMD_BOND_MIGRATE) return HOOMD_E_ARG;
    const SysDev &S = c->lay.sys[sys];
    if (S.bond_cap == 0) return HOOMD_E_STATE;
    if (!c->bond_ok[sys]) return HOOMD_E_STATE;  // the tag -> row table is out of date
    BondApplyArgs a{};
    a.recv = recv;
    a.n = n_recv;
    a.row0 = S.row0;
    a.n_local = S.n_local;
    a.mode = mode;
    a.stride = c->lay.bond_cap;
    a.bond_cap = S.bond_cap;
    a.hash = c->L.hash + S.hash0;
    a.hash_mask = S.hash_mask;
    a.ptag = c->L.ptag;
    a.pdir = c->L.pdir;
    a.status = c->L.status;
    return queue_bond_apply(c->stream, a) ? HOOMD_E_DEVICE : HOOMD_OK;
}

int hoomd_rebuild_due(hoomd_ctx *c, int32_t *due)
{
    if (!c || !due) return HOOMD_E_ARG;
    int32_t v = 0;
    HIP_OK(hipMemcpyAsync(&v, flag_ptr(c, 2), sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    *due = v != 0;
    return HOOMD_OK;
}

int migrate_particles(hoomd_ctx *c, int32_t sys, const hoomd_subdomain *sd, void *send, int64_t send_cap,
                      int32_t *counts26, int32_t *offsets26, int64_t *n_sent)
{
    if (!c || !sd || sys < 0 || sys >= c->n_sys || !counts26 || !offsets26 || !n_sent) return HOOMD_E_ARG;
    if (send_cap < 0 || (send_cap > 0 && !send)) return HOOMD_E_ARG;
    SysDev &S = c->lay.sys[sys];
    GhostArgs g{};
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = sd->lo[a];
        g.hi[a] = sd->hi[a];
    }
    g.width = 0.0;
    g.row0 = S.row0;
    g.n_local = S.n_local;
    g.fields = HOOMD_FIELD_POS | HOOMD_FIELD_VEL | HOOMD_FIELD_TAG;
    g.send = send;
    g.send_cap = send_cap;
    g.counts = counts26;
    g.offsets = offsets26;
    g.pos = reinterpret_cast<const double4 *>(c->arr.pos);
    g.vel = reinterpret_cast<const double4 *>(c->arr.vel);
    g.tag = c->arr.tag;
    g.status = c->L.status;
    g.mask = c->ghostb.mask + S.row0;
    g.list = nullptr;
    g.list_cap = 0;
    g.total = c->ghostb.totals + sys;
    const bool bonded = S.bond_cap > 0;
    if (bonded) {
        // Sec. 4.3.4: the bonds travel with their particles
        g.fields |= kFieldBonds;
        g.ptag = c->L.ptag;
        g.pdir = c->L.pdir;
        g.bond_stride = c->lay.bond_cap;
        g.bond_cap = S.bond_cap;
    }
    double4 *pt = ws_ptr<double4>(c, c->lay.pos_alt), *vt = ws_ptr<double4>(c, c->lay.vel_alt);
    int32_t *tt = c->sortb.tag_tmp;
    // the partner-row table is rebuilt at the next ghost selection: scratch here
    if (queue_migrate(c->stream, c->ghostb, g, reinterpret_cast<double4 *>(c->arr.pos),
                      reinterpret_cast<double4 *>(c->arr.vel), c->arr.tag, pt, vt, tt, bonded ? c->L.ptag : nullptr,
                      bonded ? c->L.pdir : nullptr, c->L.prow, c->L.btmp))
        return HOOMD_E_DEVICE;
    if (S.n_local > 0) {
        HIP_OK(hipMemcpyAsync(reinterpret_cast<double4 *>(c->arr.pos) + S.row0, pt + S.row0,
                              sizeof(double4) * S.n_local, hipMemcpyDeviceToDevice, c->stream));
        HIP_OK(hipMemcpyAsync(reinterpret_cast<double4 *>(c->arr.vel) + S.row0, vt + S.row0,
                              sizeof(double4) * S.n_local, hipMemcpyDeviceToDevice, c->stream));
        HIP_OK(hipMemcpyAsync(c->arr.tag + S.row0, tt + S.row0, sizeof(int32_t) * S.n_local,
                              hipMemcpyDeviceToDevice, c->stream));
        if (bonded) {
            const size_t st = (size_t)c->lay.bond_cap;
            HIP_OK(hipMemcpyAsync(c->L.ptag + S.row0 * st, c->L.prow + S.row0 * st,
                                  sizeof(int32_t) * st * S.n_local, hipMemcpyDeviceToDevice, c->stream));
            HIP_OK(hipMemcpyAsync(c->L.pdir + S.row0 * st, c->L.btmp + S.row0 * st,
                                  sizeof(int32_t) * st * S.n_local, hipMemcpyDeviceToDevice, c->stream));
        }
    }
    // the counts decide the new local count: read them (migration happens at
    // neighbour-list builds only)
    int32_t cnt[2] = {0, 0};
    HIP_OK(hipMemcpyAsync(cnt, c->ghostb.counts2, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (cnt[0] + cnt[1] != S.n_local) return HOOMD_E_DEVICE;
    c->ghosts -= (int64_t)S.n_total - S.n_local;  // the ghost layer is invalid after a migration
    c->bond_ok[sys] = 0;                          // and so are the partner rows
    S.n_local = cnt[1];
    S.n_total = cnt[1];
    c->box[sys].n_local = cnt[1];
    launch_set_counts(c->L, sys, S.n_local, S.n_total);
    count_busy_tiles(c);
    c->built = false;
    c->retune = c->tune_period > 0;
    *n_sent = cnt[0];
    if (cnt[0] > send_cap) return HOOMD_E_GHOST_OVERFLOW;
    return hipGetLastError() == hipSuccess ? HOOMD_OK : HOOMD_E_DEVICE;
}

int receive_particles(hoomd_ctx *c, int32_t sys, const void *recv, int64_t n_recv, const double *box_L)
{
    if (!c || sys < 0 || sys >= c->n_sys || n_recv < 0 || (n_recv > 0 && !recv) || !box_L) return HOOMD_E_ARG;
    SysDev &S = c->lay.sys[sys];
    if (S.n_total != S.n_local) return HOOMD_E_STATE;  // ghosts are selected after the arrivals
    if (S.n_local + n_recv > c->box[sys].n_cap) return HOOMD_E_GHOST_OVERFLOW;
    if (n_recv == 0) return HOOMD_OK;
    UnpackArgs u{};
    for (int a = 0; a < 3; ++a) {
        u.box_L[a] = box_L[a];
        u.center[a] = S.lo[a] + 0.5 * S.L[a];
    }
    u.first = S.row0 + S.n_local;
    u.n = n_recv;
    u.fields = HOOMD_FIELD_POS | HOOMD_FIELD_VEL | HOOMD_FIELD_TAG;
    u.recv = recv;
    u.pos = reinterpret_cast<double4 *>(c->arr.pos);
    u.vel = reinterpret_cast<double4 *>(c->arr.vel);
    u.tag = c->arr.tag;
    if (c->lay.bond_cap > 0) {
        // records of a bonded context carry the partner entries (a system
        // without bonds receives empty ones)
        u.fields |= kFieldBonds;
        u.ptag = c->L.ptag;
        u.pdir = c->L.pdir;
        u.bond_stride = c->lay.bond_cap;
    }
    if (queue_ghost_unpack(c->stream, u)) return HOOMD_E_DEVICE;
    c->bond_ok[sys] = 0;
    S.n_local += (int32_t)n_recv;
    S.n_total = S.n_local;
    c->box[sys].n_local = S.n_local;
    launch_set_counts(c->L, sys, S.n_local, S.n_total);
    count_busy_tiles(c);
    c->built = false;
    c->retune = c->tune_period > 0;
    return hipGetLastError() == hipSuccess ? HOOMD_OK : HOOMD_E_DEVICE;
}

int unpack_ghosts(hoomd_ctx *c, int32_t sys, const void *recv, int64_t n_recv, uint32_t fields,
                  int32_t mode, const double *box_L)
{
    if (!c || sys < 0 || sys >= c->n_sys || n_recv < 0 || (n_recv > 0 && !recv) || !box_L)
        return HOOMD_E_ARG;
    if (mode != HOOMD_GHOST_SELECT && mode != HOOMD_GHOST_UPDATE) return HOOMD_E_ARG;
    if ((fields & ~7u) || !(fields & HOOMD_FIELD_POS)) return HOOMD_E_ARG;
    SysDev &S = c->lay.sys[sys];
    if (mode == HOOMD_GHOST_UPDATE && n_recv != S.n_total - S.n_local) return HOOMD_E_STATE;
    if (S.n_local + n_recv > c->box[sys].n_cap) {
        return HOOMD_E_GHOST_OVERFLOW;
    }
    UnpackArgs u{};
    for (int a = 0; a < 3; ++a) {
        u.box_L[a] = box_L[a];
        u.center[a] = S.lo[a] + 0.5 * S.L[a];
    }
    u.first = S.row0 + S.n_local;
    u.n = n_recv;
    u.fields = fields;
    u.recv = recv;
    u.pos = reinterpret_cast<double4 *>(c->arr.pos);
    u.vel = reinterpret_cast<double4 *>(c->arr.vel);
    u.tag = c->arr.tag;
    if (queue_ghost_unpack(c->stream, u)) return HOOMD_E_DEVICE;
    if (mode == HOOMD_GHOST_SELECT) {
        if (S.n_total != S.n_local + n_recv) c->retune = c->tune_period > 0;  // the shape changed
        c->ghosts += (int64_t)(S.n_local + n_recv) - S.n_total;
        S.n_total = (int32_t)(S.n_local + n_recv);
        launch_set_counts(c->L, sys, S.n_local, S.n_total);  // queued, no host wait
        c->built = false;
        // partners found among the locals and the new ghosts
        if (S.bond_cap > 0) launch_bond_refresh(c->L, c->arr.tag, sys);
        c->bond_ok[sys] = 1;
    }
    return hipGetLastError() == hipSuccess ? HOOMD_OK : HOOMD_E_DEVICE;
}

int hoomd_thermo(hoomd_ctx *c, double *out)
{
    if (!c || !out) return HOOMD_E_ARG;
    HIP_OK(hipMemcpyAsync(out, c->ws + c->lay.thermo, sizeof(double) * 4 * c->n_sys, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return HOOMD_OK;
}

int hoomd_thermostat(hoomd_ctx *c, double *xi_eta)
{
    if (!c || !xi_eta) return HOOMD_E_ARG;
    std::vector<double> dev(2 * (size_t)c->n_sys);
    HIP_OK(hipMemcpyAsync(dev.data(), c->ws + c->lay.thermostat, sizeof(double) * dev.size(), hipMemcpyDeviceToHost,
                          c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    for (int s = 0; s < c->n_sys; ++s) {
        const int slot = c->lay.sys[s].nvt_slot;
        xi_eta[2 * s] = slot >= 0 ? dev[2 * (size_t)slot] : 0.0;
        xi_eta[2 * s + 1] = slot >= 0 ? dev[2 * (size_t)slot + 1] : 0.0;
    }
    return HOOMD_OK;
}

int hoomd_set_thermostat(hoomd_ctx *c, const double *xi_eta)
{
    if (!c || !xi_eta) return HOOMD_E_ARG;
    std::vector<double> dev(2 * (size_t)c->n_sys, 0.0);
    for (int s = 0; s < c->n_sys; ++s) {
        const int slot = c->lay.sys[s].nvt_slot;
        if (slot < 0) continue;
        dev[2 * (size_t)slot] = xi_eta[2 * s];
        dev[2 * (size_t)slot + 1] = xi_eta[2 * s + 1];
    }
    HIP_OK(hipMemcpyAsync(c->ws + c->lay.thermostat, dev.data(), sizeof(double) * dev.size(), hipMemcpyHostToDevice,
                          c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return HOOMD_OK;
}

int hoomd_thermo_log(hoomd_ctx *c, double *out, int32_t max_rows, int32_t *rows)
{
    if (!c || !out || !rows || max_rows < 0) return HOOMD_E_ARG;
    const int n = std::min(max_rows, c->last_log_rows);
    if (n > 0)
        HIP_OK(hipMemcpyAsync(out, c->ws + c->lay.thermo_log, sizeof(double) * 5 * c->n_sys * n,
                              hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    *rows = n;
    return HOOMD_OK;
}

int hoomd_sync_status(hoomd_ctx *c, int64_t *required)
{
    if (!c) return HOOMD_E_ARG;
    Status st{};
    HIP_OK(hipMemcpyAsync(&st, c->ws + c->lay.status, sizeof(Status), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    HIP_OK(hipMemsetAsync(c->ws + c->lay.status, 0, sizeof(Status), c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (required) *required = st.required;
    return st.code;
}

int hoomd_build_count(hoomd_ctx *c, int64_t *builds)
{
    if (!c || !builds) return HOOMD_E_ARG;
    int32_t v = 0;
    HIP_OK(hipMemcpyAsync(&v, flag_ptr(c, 4), sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    *builds = v;
    return HOOMD_OK;
}

int hoomd_get_layout(hoomd_ctx *c, int32_t sys, hoomd_layout *out)
{
    if (!c || !out || sys < 0 || sys >= c->n_sys) return HOOMD_E_ARG;
    const SysDev &S = c->lay.sys[sys];
    out->nlist = c->L.nlist + S.nl0;
    out->nn = c->L.nn + S.row0;
    out->halo = c->L.halo + (int64_t)S.tile0 * c->lay.halo_cap;
    out->halo_n = c->L.halo_n + S.tile0;
    out->cell_idx = c->L.cell_idx + S.cell0 * c->lay.cell_cap;
    out->cell_size = c->L.cell_size + S.cell0;
    out->nlist_cap = c->lay.nlist_cap;
    out->cell_cap = c->lay.cell_cap;
    out->halo_cap = c->lay.halo_cap;
    for (int a = 0; a < 3; ++a) out->bins[a] = S.bins[a];
    out->row_offset = S.row0;
    out->cell_offset = S.cell0;
    out->tile_offset = S.tile0;
    out->general_tiles = c->L.slow_n;
    out->rare_tiles = c->L.rare_n;
    out->halo_lds = c->L.halo_lds;
    out->bond_stride = c->lay.bond_cap;
    out->n_local = S.n_local;
    out->n_total = S.n_total;
    return HOOMD_OK;
}

}  // extern "C"

// Median of five timed launches of `launch` on the context's stream (ms); a
// failing timer call gives +inf so the candidate is never chosen.
template <typename Fn>
static float median5(hoomd_ctx *c, Fn launch, hipEvent_t e0, hipEvent_t e1)
{
    float t[5];
    launch();  // warm-up
    for (int k = 0; k < 5; ++k) {
        bool ok = hipEventRecord(e0, c->stream) == hipSuccess;
        launch();
        ok = ok && hipEventRecord(e1, c->stream) == hipSuccess;
        ok = ok && hipEventSynchronize(e1) == hipSuccess;
        ok = ok && hipEventElapsedTime(&t[k], e0, e1) == hipSuccess;
        if (!ok) t[k] = 1e30f;
    }
    std::sort(t, t + 5);
    return t[2];
}

// ---------------------------------------------------------------------------
// Autotuner (Sec. 5.2): time every candidate launch shape on the live state,
// keep the fastest, remember it per kind of context for the process.
// ---------------------------------------------------------------------------

namespace {

constexpr int kBuildShapes[4][2] = {{64, 512}, {64, 256}, {32, 512}, {32, 256}};

struct TuneEntry {
    int tpp_force, tpp_nlist, block_nlist;
    float force_ms[5], build_ms[4];
};
std::mutex g_tune_mu;
std::map<uint64_t, TuneEntry> g_tune_cache;

// Kind of context: pair potential, precision, bonds, particle count (power of
// two) and the mean neighbour count of system 0 (bins of 4) from its density
// and list radius.
uint64_t tune_key(const hoomd_ctx *c)
{
    int64_t n = 0;
    for (const auto &b : c->box) n += b.n_local;
    int nb = 0;
    while (nb < 62 && ((int64_t)1 << (nb + 1)) <= n) ++nb;
    const hoomd_params &q = c->prm[0];
    const hoomd_box &b = c->box[0];
    const double rho = (double)std::max<int64_t>(b.n_cap, 1) / (b.L[0] * b.L[1] * b.L[2]);
    const double rl = pair_cut(q) + q.r_buff;
    const int nbar = (int)std::min(4.0 / 3.0 * M_PI * rl * rl * rl * rho / 4.0, 4095.0);
    return (uint64_t)(c->pair_uniform + 1) | ((uint64_t)c->mixed << 4) | ((uint64_t)(c->lay.bond_cap > 0) << 5) |
           ((uint64_t)nb << 8) | ((uint64_t)nbar << 16);
}

int tune_now(hoomd_ctx *c, bool use_cache)
{
    const uint64_t key = tune_key(c);
    if (use_cache) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            const TuneEntry &E = it->second;
            if (!c->fixed_force) {
                c->tpp_force = E.tpp_force;
                c->block_force = 64 * E.tpp_force;
            }
            if (!c->fixed_nlist) {
                c->tpp_nlist = E.tpp_nlist;
                c->block_nlist = E.block_nlist;
            }
            std::copy(E.force_ms, E.force_ms + 5, c->force_ms);
            std::copy(E.build_ms, E.build_ms + 4, c->build_ms);
            c->from_cache = 1;
            c->last_tune_step = c->steps_done;
            c->retune = false;
            return HOOMD_OK;
        }
    }
    // a current neighbour list, cells and plans
    int rc = build_nlist(c, 0);
    if (rc) return rc;
    const double4 *pos = reinterpret_cast<const double4 *>(c->arr.pos);
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return HOOMD_E_DEVICE;
    }
    std::fill(c->force_ms, c->force_ms + 5, 0.f);
    std::fill(c->build_ms, c->build_ms + 4, 0.f);
    if (!c->fixed_force) {
        // the force pass over lanes per row (the workgroup is 64 rows x W lanes)
        ForceLaunch F = base_force(c);
        F.pos = pos;
        F.vel = reinterpret_cast<const double4 *>(c->arr.vel);
        F.vel_out = reinterpret_cast<double4 *>(c->arr.vel);
        F.mode = MODE_FORCE;
        float best = 1e30f;
        int bw = c->tpp_force;
        for (int k = 0; k < 5; ++k) {
            const int w = 1 << k;
            const float t = median5(c, [&] { launch_force(c->L, F, w, 64 * w); }, e0, e1);
            c->force_ms[k] = t;
            if (t < best) {
                best = t;
                bw = w;
            }
        }
        c->tpp_force = bw;
        c->block_force = 64 * bw;
    }
    if (!c->fixed_nlist && c->lay.tiles_local > 0) {
        // the list build over its shapes, on the cells and plans just made:
        // each timed launch redoes the framed and the general build (the list
        // of tiles for the force pass's second launch is emptied first)
        int32_t *flag = flag_ptr(c, 2), *sflag = sflag_ptr(c, 2);
        float best = 1e30f;
        int bk = 0;
        for (int k = 0; k < 4; ++k) {
            const int w = kBuildShapes[k][0], b = kBuildShapes[k][1];
            const float t = median5(c,
                                    [&] {
                                        launch_set_flag(c->L, flag_ptr(c, 7), 0);
                                        (void)hipMemsetAsync(c->L.tile_ctr, 0, sizeof(int32_t) * kTileCtrStride * kDies,
                                                             c->stream);
                                        launch_set_flags(c->L, flag, sflag, 1);
                                        c->L.flag = flag;
                                        c->L.sflag = sflag;
                                        launch_nlist(c->L, pos, c->arr.tag, w, b);
                                    },
                                    e0, e1);
            c->build_ms[k] = t;
            if (t < best) {
                best = t;
                bk = k;
            }
        }
        c->tpp_nlist = kBuildShapes[bk][0];
        c->block_nlist = kBuildShapes[bk][1];
        // a whole rebuild with the chosen shape leaves the state as it was
        launch_set_flags(c->L, flag, sflag, 1);
        queue_rebuild(c, pos, c->arr.tag, 2, 0);
    }
    const bool ok = hipStreamSynchronize(c->stream) == hipSuccess;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok) return HOOMD_E_DEVICE;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        TuneEntry E{};
        E.tpp_force = c->tpp_force;
        E.tpp_nlist = c->tpp_nlist;
        E.block_nlist = c->block_nlist;
        std::copy(c->force_ms, c->force_ms + 5, E.force_ms);
        std::copy(c->build_ms, c->build_ms + 4, E.build_ms);
        g_tune_cache[key] = E;
    }
    ++c->scans;
    c->from_cache = 0;
    c->last_tune_step = c->steps_done;
    c->retune = false;
    return HOOMD_OK;
}

}  // namespace

extern "C" {

int hoomd_autotune(hoomd_ctx *c, int32_t do_tune, hoomd_tuning *out)
{
    if (!c || do_tune < 0 || do_tune > 2) return HOOMD_E_ARG;
    if (do_tune) {
        const int rc = tune_now(c, do_tune == 2);
        if (rc) return rc;
    }
    if (out) {
        out->tpp_nlist = c->tpp_nlist;
        out->block_nlist = c->block_nlist;
        out->tpp_force = c->tpp_force;
        out->block_force = c->block_force;
        for (int k = 0; k < 5; ++k) out->force_ms[k] = c->force_ms[k];
        for (int k = 0; k < 4; ++k) out->build_ms[k] = c->build_ms[k];
        out->scans = c->scans;
        out->from_cache = c->from_cache;
    }
    return hipGetLastError() == hipSuccess ? HOOMD_OK : HOOMD_E_DEVICE;
}

int hoomd_profile(hoomd_ctx *c, int32_t mode, hoomd_profile_t *out)
{
    if (!c || mode < 0 || mode > 2) return HOOMD_E_ARG;
    if (mode == 1) {
        c->profiling = true;
        c->ev_used = 0;
        c->ev_force.clear();
        c->ev_rebuild.clear();
        return HOOMD_OK;
    }
    if (mode == 0) {
        c->profiling = false;
        return HOOMD_OK;
    }
    if (!out) return HOOMD_E_ARG;
    HIP_OK(hipStreamSynchronize(c->stream));
    auto total = [&](const std::vector<std::pair<size_t, size_t>> &v, double &ms) {
        ms = 0.0;
        for (const auto &pr : v) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, c->ev_pool[pr.first], c->ev_pool[pr.second]) != hipSuccess) return false;
            ms += t;
        }
        return true;
    };
    if (!total(c->ev_force, out->force_ms) || !total(c->ev_rebuild, out->rebuild_ms)) return HOOMD_E_DEVICE;
    out->force_launches = (int64_t)c->ev_force.size();
    out->rebuild_launches = (int64_t)c->ev_rebuild.size();
    return HOOMD_OK;
}

const char *hoomd_strerror(int code)
{
    switch (code) {
    case HOOMD_OK: return "ok";
    case HOOMD_E_ARG: return "invalid argument";
    case HOOMD_E_DEVICE: return "HIP runtime error";
    case HOOMD_E_WORKSPACE: return "workspace too small";
    case HOOMD_E_STATE: return "call not valid in the current state";
    case HOOMD_E_NLIST_OVERFLOW: return "neighbour row capacity exceeded";
    case HOOMD_E_CELL_OVERFLOW: return "cell capacity exceeded";
    case HOOMD_E_GHOST_OVERFLOW: return "ghost capacity exceeded";
    case HOOMD_E_BOND_STRETCH: return "bond stretched beyond R0";
    case HOOMD_E_NAN: return "non-finite force";
    case HOOMD_E_DANGEROUS_BUILD: return "dangerous neighbour-list build";
    case HOOMD_E_HALO_OVERFLOW: return "tile halo capacity exceeded";
    case HOOMD_E_BOND_GHOST: return "bond partner missing or beyond the neighbouring subdomains";
    default: return "unknown status";
    }
}

}  // extern "C"
