// nlist.hip -- cell list and tile-halo Verlet neighbour list (Sec. 5.1,
// Fig. 4, rebuilt for LDS-staged tiles on CDNA).
//
// Cell list: fixed-capacity bins.  A binning pass assigns every row to the
// cell floor((x - lo) * bins / L); lanes of a wave that hit the same cell
// claim their slots with one integer atomic per distinct cell.  A per-cell
// pass then sorts the members of each cell by x coordinate, ties by row
// index (rank sort inside one wave), so the list is deterministic although
// the slots were claimed in arbitrary order, and a line of x-adjacent cells
// is ordered by x.  It also resets the counters for the next build.
//
// Neighbour list: one workgroup per tile of 64 consecutive rows (Morton
// ordered rows make a tile one or a few compact clusters).  The workgroup
//   1. collects the stencil cells of all its rows and sorts out the
//      distinct ones (bitonic sort in LDS), so any tile shape works,
//   2. stages the members of those cells (positions and row numbers) in LDS,
//      a chunk at a time,
//   3. lets W = 8 lanes per particle stride over the members of the
//      particle's own 27 stencil cells and test |x_j - x_i|^2 < r_list^2 in
//      FP64 (minimum image written as the stencil's image shift, which for
//      every pair inside r_list is bitwise the shift the exact quotient
//      gives), compacting hits into the row with a 64-bit ballot,
//   4. marks every staged member that some row uses, numbers the marked
//      members in staging order -- the tile's halo -- and rewrites the rows
//      as 16-bit halo indices.
// The force pass then loads each halo position once per tile into LDS
// instead of once per neighbour from L2.
//
// Row layout (uint16): entry k of row r of a system lives at
// nl0 + (r / 64) * cap * 64 + k * 64 + r % 64.
// Tile header halo_n[tile]: bits 0-15 halo size, bits 16-30 the longest row
// of the tile, bit 31 set when the tile is too wide for one periodic image
// per halo entry.
#include "launch.h"

namespace md {

constexpr int kBuildThreads = 512;   // 64 rows x 8 lanes
constexpr int kBuildW = 8;
constexpr int kChunk = 2048;         // members staged at once
constexpr int kSlotMax = 16384;      // members of a tile's stencil cells
constexpr int kRebuildGrid = 2048;   // blocks of the grid-stride rebuild kernels
constexpr int kPlanGrid = 8192;      // one-wave workgroups of the plan kernel
constexpr int kKeys = 2048;          // 64 rows x 27 stencil cells, padded
constexpr int kKpt = kKeys / kBuildThreads;  // stencil keys per thread
static_assert(kKeys % kBuildThreads == 0 && kKeys <= 8 * kBuildThreads, "key split");
static_assert(kBuildThreads == kTile * kBuildW, "one row per lane group");
constexpr int kStencil = 27;

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bin(const SysDev *__restrict__ sys,
                                             const int32_t *__restrict__ tprefix, int n_sys, int tiles,
                                             const double4 *__restrict__ pos,
                                             int32_t *__restrict__ cell_count,
                                             int32_t *__restrict__ cell_idx, int cell_cap,
                                             const int32_t *__restrict__ flag,
                                             const int32_t *__restrict__ sflag, Status *st,
                                             uint32_t *step_counter, int32_t *slow_n, int32_t *rare_n,
                                             int32_t *tile_ctr, int32_t *since, int since_inc,
                                             const int32_t *__restrict__ tprefix_local, int nvt_w,
                                             const double *__restrict__ khalf, double *__restrict__ thermostat)
{
    // The Nose-Hoover update of the force launch just before (its half-step
    // partials are complete at that launch's end), folded into this launch,
    // which follows every step's force launch: a workgroup per thermostat
    // group.  The next force launch reads the new state.
    if (khalf) {
        __shared__ double red[kNvtSums];
        for (int q = blockIdx.x; q < n_sys; q += gridDim.x)
            if (sys[q].nvt_slot == q)
                nvt_group_update(sys, tprefix_local, n_sys, nvt_w, khalf, thermostat, q, red, blockDim.x, threadIdx.x);
    }
    // the binning launch follows every fused step launch: it also advances
    // the device step counter read by graph-replayed steps, and each system's
    // count of steps since its last build read by the displacement check
    if (blockIdx.x == 0) {
        if (step_counter && threadIdx.x == 0) *step_counter += 1u;
        if (since)
            for (int s = threadIdx.x; s < n_sys; s += blockDim.x) since[s] = sflag[s] ? 0 : since[s] + since_inc;
    }
    if (*flag == 0) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *slow_n = 0;
        *rare_n = 0;
    }
    // the framed build's per-die tile counters
    if (blockIdx.x == 0 && threadIdx.x < kDies) tile_ctr[threadIdx.x * kTileCtrStride] = 0;
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const int waves = (int)(gridDim.x * blockDim.x) >> 6;
    for (int g = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); g < tiles; g += waves) {
        const int s = find_sys(tprefix, n_sys, g);
        if (!sflag[s]) continue;  // this system keeps its list
        const SysDev &S = sys[s];
        const int r = (g - S.tile0_all) * kTile + lane;
        const bool valid = r < S.n_total;
        int64_t c = -1;
        int64_t i = 0;
        if (valid) {
            i = S.row0 + r;
            const double4 x = pos[i];
            const int cx = cell_coord(x.x, S.lo[0], S.scale[0], S.bins[0]);
            const int cy = cell_coord(x.y, S.lo[1], S.scale[1], S.bins[1]);
            const int cz = cell_coord(x.z, S.lo[2], S.scale[2], S.bins[2]);
            c = S.cell0 + ((int64_t)cz * S.bins[1] + cy) * S.bins[0] + cx;
        }
        // one atomic per distinct cell of the wave
        uint64_t todo = __ballot(valid);
        while (todo) {
            const int leader = __ffsll((unsigned long long)todo) - 1;
            const int64_t lc = __shfl(c, leader, kWave);
            const uint64_t same = __ballot(valid && c == lc);
            int base = 0;
            if (lane == leader) base = atomicAdd(&cell_count[lc], __popcll(same));
            base = __shfl(base, leader, kWave);
            if (valid && c == lc) {
                const int slot = base + __popcll(same & lt);
                if (slot < cell_cap) cell_idx[c * cell_cap + slot] = (int32_t)i;
                else latch(st, 6 /*CELL_OVERFLOW*/, slot + 1);
            }
            todo &= ~same;
        }
    }
}

// System owning a cell: largest s with cprefix[s] <= c (cprefix holds each
// system's first cell; a compact array, so the search stays in the scalar
// cache).
__device__ __forceinline__ int find_sys_cell(const int64_t *__restrict__ cprefix, int n_sys, int64_t c)
{
    int lo = 0, hi = n_sys;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cprefix[mid] <= c) lo = mid;
        else hi = mid;
    }
    return lo;
}

// One wave per cell (wave w of W takes cells w, w + W, ...): members ranked
// by their FP32 x coordinate relative to the cell's corner, ties by row index
// (a total order on (bits, row), so the ranks are a permutation whatever the
// values), sizes published.  Next to each member's row the list keeps its
// position relative to the cell's lower corner in FP32 (row bits in w), so
// that the framed build stages a cell with one coalesced read.  The counts
// are left for the plan of the framed build, which runs beside this, and
// cleared by the framed scan.  cell_cap <= 64 * CPL.
template <int CPL>
__device__ __forceinline__ void cell_sort_waves(int64_t wfirst, int64_t wstep, const SysDev *__restrict__ sys,
                                                const int64_t *__restrict__ cprefix, int n_sys, const double4 *__restrict__ pos, int64_t n_cells,
                                                const int32_t *__restrict__ cell_count,
                                                int32_t *__restrict__ cell_size, int32_t *__restrict__ cell_idx,
                                                float4 *__restrict__ cell_xf, int cell_cap,
                                                const int32_t *__restrict__ sflag)
{
    const int lane = lane_id();
    for (int64_t c = wfirst; c < n_cells; c += wstep) {
        const int s = find_sys_cell(cprefix, n_sys, c);
        if (!sflag[s]) continue;  // this system keeps its list
        int m = cell_count[c];
        m = m < cell_cap ? m : cell_cap;
        const SysDev &S = sys[s];
        const int64_t key = c - S.cell0;
        const int cx = (int)(key % S.bins[0]), cy = (int)((key / S.bins[0]) % S.bins[1]),
                  cz = (int)(key / ((int64_t)S.bins[0] * S.bins[1]));
        const double ox = S.lo[0] + (double)cx * (S.L[0] / S.bins[0]);
        const double oy = S.lo[1] + (double)cy * (S.L[1] / S.bins[1]);
        const double oz = S.lo[2] + (double)cz * (S.L[2] / S.bins[2]);
        int32_t v[CPL];
        float4 f[CPL];
        int64_t ord[CPL];  // (x bits made order-preserving as a signed integer, row)
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const int k = q * kWave + lane;
            v[q] = k < m ? cell_idx[c * cell_cap + k] : INT32_MAX;
            f[q] = make_float4(0.f, 0.f, 0.f, 0.f);
            ord[q] = INT64_MAX;
            if (k < m) {
                const double4 x = pos[v[q]];
                f[q] = make_float4((float)(x.x - ox), (float)(x.y - oy), (float)(x.z - oz), __int_as_float(v[q]));
                const int32_t b = __float_as_int(f[q].x);
                ord[q] = ((int64_t)(b ^ ((b >> 31) & 0x7FFFFFFF)) << 32) | (uint32_t)v[q];
            }
        }
        int rank[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q) rank[q] = 0;
#pragma unroll
        for (int q2 = 0; q2 < CPL; ++q2) {
            const int tmax = m - q2 * kWave < kWave ? m - q2 * kWave : kWave;
            for (int t = 0; t < tmax; ++t) {
                const int64_t other = __shfl(ord[q2], t, kWave);
#pragma unroll
                for (int q = 0; q < CPL; ++q) rank[q] += other < ord[q] ? 1 : 0;
            }
        }
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const int k = q * kWave + lane;
            if (k < m) {
                cell_idx[c * cell_cap + rank[q]] = v[q];
                cell_xf[c * cell_cap + rank[q]] = f[q];
            }
        }
        if (lane == 0) cell_size[c] = m;
    }
}

// ---------------------------------------------------------------------------
// tile-halo neighbour list
// ---------------------------------------------------------------------------

// Wrap a cell coordinate difference into [-bins/2, bins - bins/2).
__device__ __forceinline__ int wrap_rel(int d, int bins)
{
    const int h = bins / 2;
    d = ((d + h) % bins + bins) % bins - h;
    return d;
}

struct BuildShared {
    double cx[kChunk], cy[kChunk], cz[kChunk];
    int32_t cj[kChunk];
    int32_t keys[kKeys];              // stencil cells, then distinct cells
    int32_t ucount[kKeys];            // flags / members of each distinct cell
    int32_t ustart[kKeys + 1];        // first slot of each distinct cell
    uint32_t used[kSlotMax / 32];
    int32_t wpre[kSlotMax / 32 + 1];
    int16_t su[kTile][kStencil];      // distinct-cell index of each row's stencil cell (-1: none)
    int8_t sm[kTile][kStencil];       // image code (mx+1) + 3 (my+1) + 9 (mz+1)
    int32_t scan[kBuildThreads];
    int32_t ext[6];                   // min / max cell offset from the first row
    int32_t info[4];                  // distinct cells, per-pair image flag, longest row
};

// Exclusive scan of n <= 8 * NT values held in LDS `a` (in place) by a block
// of NT threads; returns the total.
template <int NT>
__device__ __forceinline__ int block_scan(int32_t *a, int n, int32_t *scan)
{
    const int tid = threadIdx.x;
    const int b = 8 * tid;
    int v[8];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = b + k < n ? a[b + k] : 0;
        sum += v[k];
    }
    scan[tid] = sum;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
        const int add = tid >= off ? scan[tid - off] : 0;
        __syncthreads();
        scan[tid] += add;
        __syncthreads();
    }
    int run = tid > 0 ? scan[tid - 1] : 0;
    const int total = scan[NT - 1];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (b + k < n) {
            a[b + k] = run;
            run += v[k];
        }
    __syncthreads();
    return total;
}

// The same with wave-level shuffles: two barriers instead of 2 log2(NT).
// The barriers order LDS accesses only (the caller's global accesses may stay
// in flight).
template <int NT>
__device__ __forceinline__ int block_scan_w(int32_t *a, int n, int32_t *wsum)
{
    constexpr int NW = NT / kWave;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid >> 6;
    const int b = 8 * tid;
    int v[8];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = b + k < n ? a[b + k] : 0;
        sum += v[k];
    }
    int inc = sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += y;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    lds_barrier();
    int before = 0, total = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        const int x = wsum[q];
        before += q < w ? x : 0;
        total += x;
    }
    int run = before + inc - sum;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (b + k < n) {
            a[b + k] = run;
            run += v[k];
        }
    lds_barrier();
    return total;
}

__device__ __forceinline__ int block_scan8(int32_t *a, int n, int32_t *scan)
{
    return block_scan<kBuildThreads>(a, n, scan);
}

// Index of the largest entry <= x in the ascending array a[0..n).
__device__ __forceinline__ int upper_idx(const int32_t *a, int n, int x)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <bool EXCL>
__global__ __launch_bounds__(kBuildThreads) void k_build_tile(
    const SysDev *__restrict__ sys, const int32_t *__restrict__ tprefix, int n_sys, int tiles,
    const double4 *__restrict__ pos, const int32_t *__restrict__ tag, const int32_t *__restrict__ ptag,
    const int32_t *__restrict__ cell_size, const int32_t *__restrict__ cell_idx, int cell_cap,
    uint16_t *__restrict__ nlist, int32_t *__restrict__ nn, int cap, int32_t *__restrict__ halo,
    int32_t *__restrict__ halo_n, int halo_cap, double4 *__restrict__ xbuild,
    const int32_t *__restrict__ list, const int32_t *__restrict__ list_n, int halo_lds,
    int32_t *__restrict__ rare_list, int32_t *__restrict__ rare_n,
    const int32_t *__restrict__ flag, int32_t *build_count, Status *st)
{
    if (*flag == 0) return;
    // with a list: only the tiles named there (those the framed build passed on)
    const int ntiles = list ? *list_n : tiles;
    if ((int)blockIdx.x >= ntiles && !(build_count && blockIdx.x == 0)) return;
    __shared__ BuildShared sh;
    constexpr int W = kBuildW;
    constexpr int P = kWave / W;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int w = tid >> 6;
    const int pl = lane % P;
    const int sl = lane / P;
    const int t = w * P + pl;  // particle slot in the tile
    const uint64_t seg = segment_bits(pl, P);
    const uint64_t below = lanemask_lt();
    if (build_count && blockIdx.x == 0 && tid == 0) atomicAdd(build_count, 1);

    int64_t tfirst = blockIdx.x, tend = ntiles;
    int tstep = gridDim.x;
    if (!list) die_range(blockIdx.x, gridDim.x, ntiles, tfirst, tend, tstep);
    for (int it = (int)tfirst; it < tend; it += tstep) {
        const int tile = list ? list[it] : it;
        const int s = find_sys(tprefix, n_sys, tile);
        const SysDev &S = sys[s];
        // per-system constants, held in registers for the whole tile
        const double Lx = S.L[0], Ly = S.L[1], Lz = S.L[2];
        const double iLx = S.invL[0], iLy = S.invL[1], iLz = S.invL[2];
        const int bx = S.bins[0], by = S.bins[1], bz = S.bins[2];
        const int px = S.per[0], py = S.per[1], pz = S.per[2];
        const int64_t row0 = S.row0, cell0 = S.cell0, nl0 = S.nl0;
        const int n_local = S.n_local;
        const double rl2 = S.rl2;
        const int r0 = (tile - S.tile0) * kTile;
        const int r = r0 + t;
        const bool active = r < n_local;
        const int64_t i = row0 + (active ? r : r0);
        const double4 xi = pos[i];
        int ci[3];
        ci[0] = cell_coord(xi.x, S.lo[0], S.scale[0], bx);
        ci[1] = cell_coord(xi.y, S.lo[1], S.scale[1], by);
        ci[2] = cell_coord(xi.z, S.lo[2], S.scale[2], bz);
        const double4 x0 = pos[row0 + r0];
        const int c0[3] = {cell_coord(x0.x, S.lo[0], S.scale[0], bx), cell_coord(x0.y, S.lo[1], S.scale[1], by),
                           cell_coord(x0.z, S.lo[2], S.scale[2], bz)};

        // ---- 1. distinct stencil cells of the tile ---------------------------
        // stencil k = (oz * 3 + oy) * 3 + ox over the de-duplicated offsets
        if (tid < 3) {
            sh.ext[tid] = INT32_MAX;
            sh.ext[3 + tid] = INT32_MIN;
        }
        if (tid == 0) sh.info[2] = 0;
        for (int k = sl; k < kStencil; k += W) {
            const int ox = k % 3, oy = (k / 3) % 3, oz = k / 9;
            int key = INT32_MAX;
            int code = 0;
            if (active && ox < S.nst[0] && oy < S.nst[1] && oz < S.nst[2]) {
                const int off[3] = {S.st[0][ox], S.st[1][oy], S.st[2][oz]};
                const int bins[3] = {bx, by, bz};
                const int per[3] = {px, py, pz};
                int cc[3];
                bool inside = true;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    cc[a] = ci[a] + off[a];
                    int m = 0;
                    if (per[a]) {
                        // image of the neighbour cell across a periodic face
                        if (cc[a] < 0) {
                            cc[a] += bins[a];
                            m = 1;
                        } else if (cc[a] >= bins[a]) {
                            cc[a] -= bins[a];
                            m = -1;
                        }
                    } else {
                        inside = inside && cc[a] >= 0 && cc[a] < bins[a];
                    }
                    code += (m + 1) * (a == 0 ? 1 : (a == 1 ? 3 : 9));
                }
                if (inside) key = (cc[2] * by + cc[1]) * bx + cc[0];
            }
            sh.keys[t * kStencil + k] = key;
            sh.sm[t][k] = (int8_t)code;
        }
        for (int k = kTile * kStencil + tid; k < kKeys; k += kBuildThreads) sh.keys[k] = INT32_MAX;
        __syncthreads();
        if (active && sl == 0) {
            const int bins[3] = {bx, by, bz};
            const int per[3] = {px, py, pz};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int d = ci[a] - c0[a];
                const int rel = per[a] ? wrap_rel(d, bins[a]) : d;
                atomicMin(&sh.ext[a], rel);
                atomicMax(&sh.ext[3 + a], rel);
            }
        }
        // the key of every row's stencil cell, kept for the lookup below
        int32_t mykeys[(kStencil + W - 1) / W];
#pragma unroll
        for (int q = 0; q < (kStencil + W - 1) / W; ++q) {
            const int k = sl + q * W;
            mykeys[q] = k < kStencil ? sh.keys[t * kStencil + k] : INT32_MAX;
        }
        __syncthreads();
        // bitonic sort of the keys
        for (int k = 2; k <= kKeys; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int e = tid; e < kKeys / 2; e += kBuildThreads) {
                    const int a = ((e & ~(j - 1)) << 1) | (e & (j - 1));
                    const int b = a | j;
                    const int32_t ka = sh.keys[a], kb = sh.keys[b];
                    if ((ka > kb) == ((a & k) == 0)) {
                        sh.keys[a] = kb;
                        sh.keys[b] = ka;
                    }
                }
                __syncthreads();
            }
        }
        // distinct keys: flag first occurrences, scan, compact (kKpt keys
        // per thread)
        int flg[kKpt];
        int32_t kv[kKpt];
#pragma unroll
        for (int k = 0; k < kKpt; ++k) {
            const int q = kKpt * tid + k;
            kv[k] = sh.keys[q];
            flg[k] = (kv[k] != INT32_MAX && (q == 0 || kv[k] != sh.keys[q - 1])) ? 1 : 0;
            sh.ucount[q] = flg[k];
        }
        __syncthreads();
        const int nu = block_scan8(sh.ucount, kKeys, sh.scan);
#pragma unroll
        for (int k = 0; k < kKpt; ++k)
            if (flg[k]) sh.keys[sh.ucount[kKpt * tid + k]] = kv[k];
        if (tid == 0) {
            int pp = 0;
            const double Ls[3] = {Lx, Ly, Lz};
            const int bins[3] = {bx, by, bz};
            const int per[3] = {px, py, pz};
            for (int a = 0; a < 3; ++a)
                if (per[a] && (double)(sh.ext[3 + a] - sh.ext[a] + 3) * (Ls[a] / bins[a]) >= 0.5 * Ls[a]) pp = 1;
            sh.info[1] = pp;
        }
        __syncthreads();
        // member counts of the distinct cells and their prefix
        for (int u = tid; u < nu; u += kBuildThreads) sh.ucount[u] = cell_size[cell0 + sh.keys[u]];
        __syncthreads();
        const int nslot = block_scan8(sh.ucount, nu, sh.scan);
        for (int u = tid; u < nu; u += kBuildThreads) sh.ustart[u] = sh.ucount[u];
        if (tid == 0) sh.ustart[nu] = nslot;
        // each row's stencil cells as distinct-cell indices
#pragma unroll
        for (int q = 0; q < (kStencil + W - 1) / W; ++q) {
            const int k = sl + q * W;
            if (k < kStencil) sh.su[t][k] = mykeys[q] == INT32_MAX ? (int16_t)-1 : (int16_t)upper_idx(sh.keys, nu, mykeys[q]);
        }
        if (nslot > kSlotMax) {
            if (tid == 0) latch(st, 11 /*HALO_OVERFLOW*/, nslot);
            if (active && sl == 0) nn[i] = 0;
            if (tid == 0) halo_n[tile] = 0;
            __syncthreads();
            continue;
        }
        for (int q = tid; q < (nslot + 31) / 32; q += kBuildThreads) sh.used[q] = 0u;

        // ---- 2./3. stage chunks, scan each row's stencil ------------------------
        int32_t part[kMaxBondCap];
        if constexpr (EXCL) {
#pragma unroll
            for (int b = 0; b < kMaxBondCap; ++b) part[b] = -1;
            if (active) {
                const int64_t prow = i * S.bond_stride;
                for (int b = 0; b < S.bond_cap && b < kMaxBondCap; ++b) part[b] = ptag[prow + b];
            }
        }
        const int64_t rowbase = nl0 + (int64_t)(r >> 6) * cap * kTile + (r & 63);
        const bool fx_ = px && bx < 3, fy_ = py && by < 3, fz_ = pz && bz < 3;
        const bool few = fx_ || fy_ || fz_;
        const bool few_axis[3] = {fx_, fy_, fz_};
        // offset of the particle inside its cell and the cell widths (FP32),
        // for the conservative per-cell distance test
        const float cellw[3] = {(float)(Lx / bx), (float)(Ly / by), (float)(Lz / bz)};
        const float frel[3] = {(float)(xi.x - S.lo[0]) - (float)ci[0] * cellw[0],
                               (float)(xi.y - S.lo[1]) - (float)ci[1] * cellw[1],
                               (float)(xi.z - S.lo[2]) - (float)ci[2] * cellw[2]};
        const float rl2f = (float)rl2 * 1.0001f + 1e-3f;
        int ntot = 0;
        for (int q0 = 0; q0 < nslot; q0 += kChunk) {
            const int q1 = q0 + kChunk < nslot ? q0 + kChunk : nslot;
            __syncthreads();
            for (int q = q0 + tid; q < q1; q += kBuildThreads) {
                const int u = upper_idx(sh.ustart, nu, q);
                const int32_t j = cell_idx[(cell0 + sh.keys[u]) * cell_cap + (q - sh.ustart[u])];
                const double4 xj = pos[j];
                sh.cx[q - q0] = xj.x;
                sh.cy[q - q0] = xj.y;
                sh.cz[q - q0] = xj.z;
                sh.cj[q - q0] = j;
            }
            __syncthreads();
            if (!active) continue;
            for (int k = 0; k < kStencil; ++k) {
                const int u = sh.su[t][k];
                if (u < 0) continue;
                // skip a neighbour cell whose nearest face lies beyond r_list
                // (FP32 with a relative margin: it never drops a cell that can
                // hold a neighbour)
                {
                    const int ox = k % 3, oy = (k / 3) % 3, oz = k / 9;
                    float g2 = 0.f;
                    const int offs[3] = {S.st[0][ox < S.nst[0] ? ox : 0], S.st[1][oy < S.nst[1] ? oy : 0],
                                         S.st[2][oz < S.nst[2] ? oz : 0]};
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        if (offs[a] == 0 || few_axis[a]) continue;
                        const float g = offs[a] < 0 ? frel[a] : cellw[a] - frel[a];
                        g2 += g > 0.f ? g * g : 0.f;
                    }
                    if (g2 > rl2f) continue;
                }
                const int code = sh.sm[t][k];
                const double sx = Lx * (double)(code % 3 - 1);
                const double sy = Ly * (double)((code / 3) % 3 - 1);
                const double sz = Lz * (double)(code / 9 - 1);
                const bool shifted = code != 13;
                int a0 = sh.ustart[u], a1 = sh.ustart[u + 1];
                a0 = a0 > q0 ? a0 : q0;
                a1 = a1 < q1 ? a1 : q1;
                for (int k0 = a0; k0 < a1; k0 += 2 * W) {
                    bool hit[2];
                    int qq[2];
                    int32_t jj[2];
                    double ddx[2], ddy[2], ddz[2];
#pragma unroll
                    for (int v = 0; v < 2; ++v) {
                        qq[v] = k0 + sl + v * W;
                        const int qs = (qq[v] < a1 ? qq[v] : a0) - q0;
                        jj[v] = sh.cj[qs];
                        ddx[v] = sh.cx[qs] - xi.x;
                        ddy[v] = sh.cy[qs] - xi.y;
                        ddz[v] = sh.cz[qs] - xi.z;
                    }
#pragma unroll
                    for (int v = 0; v < 2; ++v) {
                        if (few) {
                            // fewer than 3 cells: several images share a cell, take the nearest
                            ddx[v] = fx_ ? min_image(ddx[v], Lx, iLx) : ddx[v] - sx;
                            ddy[v] = fy_ ? min_image(ddy[v], Ly, iLy) : ddy[v] - sy;
                            ddz[v] = fz_ ? min_image(ddz[v], Lz, iLz) : ddz[v] - sz;
                        } else if (shifted) {
                            ddx[v] -= sx;
                            ddy[v] -= sy;
                            ddz[v] -= sz;
                        }
                        hit[v] = qq[v] < a1 && jj[v] != (int32_t)i && norm2_exact(ddx[v], ddy[v], ddz[v]) < rl2;
                        if constexpr (EXCL) {
                            if (hit[v]) {
                                const int32_t tj = tag[jj[v]];
#pragma unroll
                                for (int b = 0; b < kMaxBondCap; ++b) hit[v] = hit[v] && (part[b] != tj);
                            }
                        }
                    }
#pragma unroll
                    for (int v = 0; v < 2; ++v) {
                        const uint64_t mask = __ballot(hit[v]) & seg;
                        if (hit[v]) {
                            const int p = ntot + __popcll(mask & below);
                            if (p < cap) nlist[rowbase + (int64_t)p * kTile] = (uint16_t)qq[v];
                            atomicOr(&sh.used[qq[v] >> 5], 1u << (qq[v] & 31));
                        }
                        ntot += __popcll(mask);
                    }
                }
            }
        }
        if (active && sl == 0) atomicMax(&sh.info[2], ntot < cap ? ntot : cap);
        __syncthreads();
        // ---- 4. halo numbering and row rewrite ---------------------------------
        const int nwords = (nslot + 31) / 32;
        for (int q = tid; q < nwords; q += kBuildThreads) sh.wpre[q] = __popc(sh.used[q]);
        __syncthreads();
        const int nhalo = block_scan8(sh.wpre, nwords, sh.scan);
        if (nhalo > halo_cap) {
            if (tid == 0) latch(st, 11 /*HALO_OVERFLOW*/, nhalo);
            if (active && sl == 0) nn[i] = 0;
            if (tid == 0) halo_n[tile] = 0;
            __syncthreads();
            continue;
        }
        // halo list: row number of every used member, in staging order
        int32_t *hl = halo + (int64_t)tile * halo_cap;
        for (int q = tid; q < nslot; q += kBuildThreads) {
            const uint32_t word = sh.used[q >> 5];
            if (word & (1u << (q & 31))) {
                const int u = upper_idx(sh.ustart, nu, q);
                const int h = sh.wpre[q >> 5] + __popc(word & ((1u << (q & 31)) - 1u));
                hl[h] = cell_idx[(cell0 + sh.keys[u]) * cell_cap + (q - sh.ustart[u])];
            }
        }
        if (tid == 0) {
            halo_n[tile] = (int32_t)((uint32_t)nhalo | ((uint32_t)sh.info[2] << 16) | (sh.info[1] ? 0x80000000u : 0u));
            // per-pair images or a halo beyond the force pass's LDS staging
            if (sh.info[1] || nhalo > halo_lds) rare_list[atomicAdd(rare_n, 1)] = tile;
        }
        __threadfence_block();
        __syncthreads();
        if (active) {
            const int n = ntot < cap ? ntot : cap;
            for (int k = sl; k < n; k += 2 * W) {
                const int64_t a = rowbase + (int64_t)k * kTile;
                const int64_t b = a + (int64_t)W * kTile;
                const bool has_b = k + W < n;
                const int qa = nlist[a];
                const int qb = has_b ? nlist[b] : 0;
                const uint32_t wa = sh.used[qa >> 5], wb = sh.used[qb >> 5];
                nlist[a] = (uint16_t)(sh.wpre[qa >> 5] + __popc(wa & ((1u << (qa & 31)) - 1u)));
                if (has_b) nlist[b] = (uint16_t)(sh.wpre[qb >> 5] + __popc(wb & ((1u << (qb & 31)) - 1u)));
            }
            if (sl == 0) {
                nn[i] = n;
                xbuild[i] = xi;
                if (ntot > cap) latch(st, 5 /*NLIST_OVERFLOW*/, ntot);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// framed tile build
// ---------------------------------------------------------------------------
//
// The common case of the build above, reorganised so that the work per
// candidate is a handful of FP32 operations:
//   * The tile's cells are placed in one frame: cell coordinates relative to
//     the first row's cell, unwrapped across periodic faces.  The stencil
//     cells of all rows are marked in a bitmap over the frame's box (home
//     cells +-1), so the distinct cells come out in box order and the three
//     x-adjacent cells of a row's stencil line are three consecutive distinct
//     cells: a row's candidates are nine contiguous slot ranges ("runs").
//   * Members are staged as FP32 positions in the frame, relative to the
//     first row: the cell list keeps each member's position from its cell's
//     corner in FP32, and staging adds the corner's frame position (one
//     coalesced read per member).  One wave takes one row at a time; its 64
//     lanes split the
//     nine runs in proportion to their lengths (at least one lane each), so
//     a row takes about (members / 55) + 1 passes.  A candidate whose FP32
//     distance lies clearly inside or outside r_list is decided there; one
//     within a relative band of 2^-10 of r_list^2 is decided by the exact
//     FP64 test (difference of the stored positions, then the periodic
//     shift), so the list is exactly the FP64 one.  Three roundings of
//     magnitude at most F (the frame extent) per coordinate bound the FP32
//     error of r^2 by about 6 sqrt(3) F 2^-24 / r_list relative; tiles with
//     F > 512 r_list are passed on.
//   * Rows are assembled in LDS and written out coalesced after the halo
//     numbering, without a read-back.
// Tiles that do not fit (a frame wider than a periodic box, fewer than three
// cells on a periodic axis, too many distinct cells or members) are appended
// to a device list and built by k_build_tile.

constexpr int kFastThreads = 512;           // threads per workgroup by default (8 waves)
constexpr int kFastWavesMax = 8;            // waves per workgroup at most
constexpr int kFastChunk = 2560;     // members staged at once (float4 each)
constexpr int kBoxMax = 8192;        // cells of the frame box
constexpr int kBoxWords = kBoxMax / 32;
constexpr int kUMax = 256;           // distinct cells of a framed tile
constexpr int kFastSlotMax = 8192;   // members of a framed tile's stencil cells
constexpr int kRuns = 9;
static_assert(kUMax <= 256, "slot map holds distinct cells as bytes");

// DPP lane move within rows of 16 lanes (every lane of the wave active).
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}

// Minimum / maximum over the 64 lanes of a fully active wave: swaps within
// quads, half rows and rows, then the four row results.
__device__ __forceinline__ int wave_min_full(int v)
{
    v = min(v, dpp_mov<0xB1>(v));   // quad_perm [1,0,3,2]
    v = min(v, dpp_mov<0x4E>(v));   // quad_perm [2,3,0,1]
    v = min(v, dpp_mov<0x141>(v));  // row_half_mirror
    v = min(v, dpp_mov<0x140>(v));  // row_mirror
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Values that are the same in every lane (read from LDS or computed from
// such values), moved to scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ double uni(double v)
{
    const int64_t b = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __longlong_as_double((int64_t)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ int wave_max_full(int v)
{
    v = max(v, dpp_mov<0xB1>(v));
    v = max(v, dpp_mov<0x4E>(v));
    v = max(v, dpp_mov<0x141>(v));
    v = max(v, dpp_mov<0x140>(v));
    return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

struct FastShared {
    float4 cp[kFastChunk];               // member position in the frame (FP32), row in w
    int32_t ucell[kUMax];                // cell index of each distinct cell
    float4 uoff[kUMax];                  // frame position of each distinct cell's corner (FP32)
    int32_t ustart[kUMax + 1];           // first slot of each distinct cell
    uint32_t used[kFastSlotMax / 32];
    int32_t wpre[kFastSlotMax / 32 + 1];
    uint32_t run[kTile][kRuns];          // slot range of each row line: lo | hi << 16
    uint32_t runc[kTile][kRuns];         // the same cut to the chunk and to the line's x-window
    float hw[kTile][kRuns];              // half width in x of each row line
    float4 xrow[kTile];                  // row position in the frame (FP32)
    int32_t rown[kTile];                 // hits of each row so far
    uint64_t lmask[kTile];               // per row: bit of the last lane of each (non-empty) line but the last
    uint8_t lb[kTile][kRuns + 1];        // per row: first lane of each (non-empty) line, then the lanes used
    uint8_t ln[kTile][kRuns];            // 32 lanes per row: the non-empty lines in order
    uint8_t nk[kTile];                   // 32 lanes per row: non-empty lines in this chunk
    int32_t scan[kFastWavesMax];         // per-wave totals of the block scans
    uint8_t smap[kFastChunk];            // distinct cell of each slot of the chunk
    double xref[3];                      // first row's position: the frame reference
    int32_t info[5];                     // distinct cells, per-pair image flag, longest row, slots,
                                         // FP32 decision band (float bits)
    int32_t grab[2];                     // tile indices taken from the die's counter
};

// Per-tile plan of the framed build, written by k_cells_and_plan and read by
// k_build_fast: a header {distinct cells (-1: passed on), slots, per-pair
// image flag, 0}, then per distinct cell {cell, first slot} and its corner
// in the frame, per row its frame position, and per row line its slot range
// and the half width in x that its y-z distance leaves.
struct PlanPtrs {
    int4 *hdr;
    int2 *cell;
    float4 *off;
    float4 *xrow;
    uint32_t *run;
    float *hw;
};

__host__ __device__ inline PlanPtrs plan_ptrs(char *base, int64_t tiles)
{
    PlanPtrs P;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        char *p = base + off;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    P.hdr = reinterpret_cast<int4 *>(carve(sizeof(int4) * tiles));
    P.cell = reinterpret_cast<int2 *>(carve(sizeof(int2) * tiles * kUMax));
    P.off = reinterpret_cast<float4 *>(carve(sizeof(float4) * tiles * kUMax));
    P.xrow = reinterpret_cast<float4 *>(carve(sizeof(float4) * tiles * kTile));
    P.run = reinterpret_cast<uint32_t *>(carve(sizeof(uint32_t) * tiles * kTile * kRuns));
    P.hw = reinterpret_cast<float *>(carve(sizeof(float) * tiles * kTile * kRuns));
    return P;
}

// Exclusive scan in place of a[0..n), n <= 4 * 64, by one fully active
// wave; returns the total.
__device__ __forceinline__ int wave_scan_excl(int32_t *a, int n)
{
    const int lane = lane_id();
    int v[4];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = lane * 4 + k;
        v[k] = i < n ? a[i] : 0;
        sum += v[k];
    }
    int inc = sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += y;
    }
    const int total = __shfl(inc, kWave - 1, kWave);
    int run = inc - sum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = lane * 4 + k;
        if (i < n) a[i] = run;
        run += v[k];
    }
    return total;
}
static_assert(kBoxWords <= 4 * kWave && kUMax <= 4 * kWave, "one-wave scans of the plan");

// The plan of one tile per wave (workgroups of one wave: no block barriers
// wait on other waves, so many tiles are in flight per CU).  Lane t takes
// row t: its home cell in the frame (cell coordinates relative to the first
// row's cell, unwrapped across periodic faces with the cut opposite the first
// row or through it, whichever gives the shorter extent), its nine x-lines of
// three cells marked in a bitmap over the frame's box, the distinct cells in
// box order with their sizes and first slots, and every line cut to the cells
// within r_list.  The rows' build positions are written here.  Tiles that do
// not fit (a frame wider than a periodic box, fewer than three cells on a
// periodic axis, too many distinct cells or members) go to the general build.
struct PlanShared {
    uint32_t box[kBoxWords];
    int32_t bpre[kBoxWords + 1];
    int32_t ucell[kUMax];
    int32_t ustart[kUMax + 1];
};

__device__ __forceinline__ void plan_tiles(
    PlanShared &ps, int pb, int npb, const SysDev *__restrict__ sys, const int32_t *__restrict__ tprefix,
    int n_sys, int tiles, const double4 *__restrict__ pos, const int32_t *__restrict__ cell_count, int cell_cap,
    double4 *__restrict__ xbuild, int32_t *__restrict__ slow_list, int32_t *__restrict__ slow_n, PlanPtrs plan,
    const int32_t *__restrict__ sflag, int32_t *__restrict__ halo_n, int halo_lds,
    int32_t *__restrict__ rare_list, int32_t *__restrict__ rare_n)
{
    uint32_t *box = ps.box;
    int32_t *bpre = ps.bpre;
    int32_t *ucell = ps.ucell;
    int32_t *ustart = ps.ustart;
    const int lane = lane_id();
    int64_t tfirst, tend;
    int tstep;
    die_range(pb, npb, tiles, tfirst, tend, tstep);
    for (int tile = (int)tfirst; tile < tend; tile += tstep) {
        const int s = find_sys(tprefix, n_sys, tile);
        if (!sflag[s]) {
            // a system that keeps its list: its tile goes back on the list of
            // the force pass's second launch if its last build put it there
            // (the binning launch before this one emptied that list)
            if (lane == 0) {
                const int32_t hn = halo_n[tile];
                if (hn < 0 || (hn & 0xFFFF) > halo_lds) rare_list[atomicAdd(rare_n, 1)] = tile;
            }
            continue;
        }
        const SysDev &S = sys[s];
        const double Ls[3] = {S.L[0], S.L[1], S.L[2]};
        const int bins[3] = {S.bins[0], S.bins[1], S.bins[2]};
        const int per[3] = {S.per[0], S.per[1], S.per[2]};
        const int64_t row0 = S.row0, cell0 = S.cell0;
        const int n_local = S.n_local;
        const double rl2 = S.rl2;
        const int r0 = (tile - S.tile0) * kTile;
        if (r0 >= n_local) {
            // a tile past the local rows (room for particles that may
            // arrive): an empty list and halo, nothing to build
            if (lane == 0) {
                plan.hdr[tile] = make_int4(0, 0, 0, 0);
                halo_n[tile] = 0;
            }
            continue;
        }
        const float cw[3] = {(float)(Ls[0] / bins[0]), (float)(Ls[1] / bins[1]), (float)(Ls[2] / bins[2])};
        auto pass_on = [&]() {
            if (lane == 0) {
                slow_list[atomicAdd(slow_n, 1)] = tile;
                plan.hdr[tile] = make_int4(-1, 0, 0, 0);
            }
        };

        // ---- rows: home cell in the frame, frame position, build position ----
        const int r = r0 + lane;
        const bool act = r < n_local;
        const double4 xi = pos[row0 + (act ? r : r0)];
        if (act) xbuild[row0 + r] = make_double4(xi.x, xi.y, xi.z, 0.0);
        const double xr[3] = {uni(xi.x), uni(xi.y), uni(xi.z)};  // row 0 of the tile
        const double xa[3] = {xi.x, xi.y, xi.z};
        int c0[3], h[3], elo[3], ehi[3];
        float xf[3], frel[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            c0[a] = uni(cell_coord(xr[a], S.lo[a], S.scale[a], bins[a]));
            const int ci = cell_coord(xa[a], S.lo[a], S.scale[a], bins[a]);
            const int d = ci - c0[a];
            const int sft = bins[a] / 2;
            const int hc[2] = {per[a] ? wrap_rel(d, bins[a]) : d, per[a] ? sft + wrap_rel(d - sft, bins[a]) : d};
            int mn[2], mx[2];
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                mn[v] = wave_min_full(act ? hc[v] : INT32_MAX);
                mx[v] = wave_max_full(act ? hc[v] : INT32_MIN);
            }
            const int pick = mx[1] - mn[1] < mx[0] - mn[0] ? 1 : 0;
            h[a] = hc[pick];
            elo[a] = pick ? mn[1] : mn[0];
            ehi[a] = pick ? mx[1] : mx[0];
            // image of the row in the frame: the home cell at c0 + h
            const int kimg = per[a] ? (c0[a] + h[a] - ci) / bins[a] : 0;
            xf[a] = (float)((xa[a] + (double)kimg * Ls[a]) - xr[a]);
            frel[a] = (float)(xa[a] - S.lo[a]) - (float)ci * cw[a];
        }
        plan.xrow[(int64_t)tile * kTile + lane] = make_float4(xf[0], xf[1], xf[2], 0.f);
        // spread of the rows around row 0 per axis (xf is relative to it;
        // non-negative floats order as their bit patterns)
        float spread[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            spread[a] = __int_as_float(wave_max_full(act ? __float_as_int(fabsf(xf[a])) : 0));

        // ---- frame box and the stencil-cell bitmap ----------------------------
        int blo[3], X[3];
        bool pass = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int lo_ = elo[a] - 1, hi_ = ehi[a] + 1;
            if (!per[a]) {
                lo_ = lo_ > -c0[a] ? lo_ : -c0[a];
                hi_ = hi_ < bins[a] - 1 - c0[a] ? hi_ : bins[a] - 1 - c0[a];
            } else if (bins[a] < 3 || hi_ - lo_ + 1 > bins[a]) {
                pass = true;
            }
            blo[a] = lo_;
            X[a] = hi_ - lo_ + 1;
            if ((double)X[a] * (double)cw[a] > 512.0 * sqrt(rl2)) pass = true;
        }
        const int vol = X[0] * X[1] * X[2];
        if (pass || vol > kBoxMax) {
            pass_on();
            continue;
        }
        const int nbw = (vol + 31) >> 5;
        __syncthreads();  // LDS of the previous tile no longer read
        for (int q = lane; q < nbw; q += kWave) box[q] = 0u;
        __syncthreads();
        // a row's stencil as nine x-lines of (up to) three adjacent cells:
        // consecutive bits of one box row
        if (act) {
            for (int rr = 0; rr < kRuns; ++rr) {
                const int fy = h[1] + rr % 3 - 1, fz = h[2] + rr / 3 - 1;
                if (!per[1] && (c0[1] + fy < 0 || c0[1] + fy >= bins[1])) continue;
                if (!per[2] && (c0[2] + fz < 0 || c0[2] + fz >= bins[2])) continue;
                int xa_ = h[0] - 1, xb_ = h[0] + 1;
                if (!per[0]) {
                    xa_ = c0[0] + xa_ >= 0 ? xa_ : -c0[0];
                    xb_ = c0[0] + xb_ < bins[0] ? xb_ : bins[0] - 1 - c0[0];
                }
                const int b = ((fz - blo[2]) * X[1] + (fy - blo[1])) * X[0] + (xa_ - blo[0]);
                const uint64_t bits = ((1ull << (xb_ - xa_ + 1)) - 1ull) << (b & 31);
                atomicOr(&box[b >> 5], (uint32_t)bits);
                if (bits >> 32) atomicOr(&box[(b >> 5) + 1], (uint32_t)(bits >> 32));
            }
        }
        __syncthreads();

        // ---- distinct cells (box order), sizes, first slots ----------------------
        for (int q = lane; q < nbw; q += kWave) bpre[q] = __popc(box[q]);
        __syncthreads();
        const int nu = uni(wave_scan_excl(bpre, nbw));
        __syncthreads();
        if (nu > kUMax || nu < 1) {
            pass_on();
            continue;
        }
        for (int b = lane; b < vol; b += kWave) {
            const uint32_t word = box[b >> 5];
            if ((word >> (b & 31)) & 1u) ucell[bpre[b >> 5] + __popc(word & ((1u << (b & 31)) - 1u))] = b;
        }
        __syncthreads();
        // four distinct cells per lane; every lane reads a valid cell (the
        // last one again past the end) so that the reads are in flight together
        int cells[4];
        float4 offs[4];
        int sizes[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int u = lane + k * kWave;
            const int b = ucell[u < nu ? u : nu - 1];
            const int f[3] = {b % X[0] + blo[0], (b / X[0]) % X[1] + blo[1], b / (X[0] * X[1]) + blo[2]};
            int pc[3];
            float off[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                pc[a] = c0[a] + f[a];
                const int ki = pc[a] >= bins[a] ? 1 : (pc[a] < 0 ? -1 : 0);
                pc[a] -= ki * bins[a];
                // the cell's lower corner in the frame, relative to the reference
                off[a] = (float)((S.lo[a] + (double)pc[a] * (Ls[a] / bins[a]) + (double)ki * Ls[a]) - xr[a]);
            }
            cells[k] = (int32_t)(cell0 + ((int64_t)pc[2] * bins[1] + pc[1]) * bins[0] + pc[0]);
            offs[k] = make_float4(off[0], off[1], off[2], 0.f);
            sizes[k] = cell_count[cells[k]];
        }
        __syncthreads();  // ucell no longer read
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int u = lane + k * kWave;
            if (u < nu) ustart[u] = sizes[k] < cell_cap ? sizes[k] : cell_cap;
        }
        __syncthreads();
        const int nslot = uni(wave_scan_excl(ustart, nu));
        if (lane == 0) ustart[nu] = nslot;
        __syncthreads();
        if (nslot > kFastSlotMax) {
            pass_on();
            continue;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int u = lane + k * kWave;
            if (u < nu) {
                plan.cell[(int64_t)tile * kUMax + u] = make_int2(cells[k], ustart[u]);
                plan.off[(int64_t)tile * kUMax + u] = offs[k];
            }
        }

        // ---- every row line cut to the cells within r_list; x half widths -----
        const float rl2f = (float)rl2 * 1.0001f + 1e-3f;
        float fext = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) fext = fmaxf(fext, (float)X[a] * cw[a]);
        // bound on the FP32 error of a frame x difference, with room to spare
        const float xmargin = 1e-3f + fext * 0x1p-18f;
        const int64_t pr = ((int64_t)tile * kTile + lane) * kRuns;
        for (int rr = 0; rr < kRuns; ++rr) {
            uint32_t v = 0u;
            float hwv = 0.f;
            if (act) {
                const int dy = rr % 3 - 1, dz = rr / 3 - 1;
                const int hx = h[0], hy = h[1] + dy, hz = h[2] + dz;
                bool in = (per[1] || (c0[1] + hy >= 0 && c0[1] + hy < bins[1])) &&
                          (per[2] || (c0[2] + hz >= 0 && c0[2] + hz < bins[2]));
                // squared distance in y and z from the row to the line's cells
                // (a lower bound for every member of the line)
                float gyz = 0.f;
                if (dy != 0) {
                    const float gg = dy < 0 ? frel[1] : cw[1] - frel[1];
                    gyz += gg > 0.f ? gg * gg : 0.f;
                }
                if (dz != 0) {
                    const float gg = dz < 0 ? frel[2] : cw[2] - frel[2];
                    gyz += gg > 0.f ? gg * gg : 0.f;
                }
                in = in && gyz <= rl2f;
                if (in) {
                    const float fx = frel[0];
                    const float gl = fx > 0.f ? fx : 0.f, gr = cw[0] - fx > 0.f ? cw[0] - fx : 0.f;
                    const bool left = (per[0] || c0[0] + hx - 1 >= 0) && gl * gl + gyz <= rl2f;
                    const bool right = (per[0] || c0[0] + hx + 1 < bins[0]) && gr * gr + gyz <= rl2f;
                    const int xa_ = hx + (left ? -1 : 0), xb_ = hx + (right ? 1 : 0);
                    const int b = ((hz - blo[2]) * X[1] + (hy - blo[1])) * X[0] + (xa_ - blo[0]);
                    const int u0 = bpre[b >> 5] + __popc(box[b >> 5] & ((1u << (b & 31)) - 1u));
                    const int u1 = u0 + (xb_ - xa_);
                    v = (uint32_t)ustart[u0] | ((uint32_t)ustart[u1 + 1] << 16);
                    hwv = sqrtf(fmaxf(rl2f - gyz, 0.f)) + xmargin;
                }
            }
            plan.run[pr + rr] = v;
            plan.hw[pr + rr] = hwv;
        }
        // One image per halo entry (the one nearest row 0, taken by the force
        // pass at every step) is every row's minimum image while, per
        // periodic axis, spread + r_list + 2 r_buff < L/2: until the next
        // build each particle moves at most r_buff/2, so a row stays within
        // spread + r_buff of row 0 and a listed pair within r_list + r_buff,
        // and the partner image nearest the row is within L/2 of row 0 (the
        // rows' FP32 offsets get a margin of 1e-5 L).  Otherwise the force
        // pass takes the minimum image per pair.
        int pp = 0;
        {
            const double rlist = sqrt(rl2), rbuff = 2.0 * sqrt(S.disp2);
            for (int a = 0; a < 3; ++a)
                if (per[a] && (double)spread[a] + rlist + 2.0 * rbuff + 1e-5 * Ls[a] >= 0.5 * Ls[a]) pp = 1;
        }
        // relative band around r_list^2 inside which the FP32 distance of a
        // candidate cannot decide the test: a bound on the FP32 rounding of
        // frame coordinates up to E in magnitude (cell-relative position,
        // cell corner, their sum, the row's position: |error| <= 2^-24 (4E +
        // |dx|) per separation), propagated through r^2 and doubled
        const double Ef = (double)fext + (double)fmaxf(cw[0], fmaxf(cw[1], cw[2]));
        const double rl = sqrt(rl2);
        const double eta = 0x1p-24 * (4.0 * Ef + 1.01 * rl);
        const double dr2 = 2.0 * sqrt(3.0) * rl * eta + 3.0 * eta * eta + 3.0 * 0x1p-24 * rl2 * 1.01;
        const float band = (float)(2.0 * (dr2 / rl2 + 3.0 * 0x1p-24));
        if (lane == 0) plan.hdr[tile] = make_int4(nu, nslot, pp, __float_as_int(band));
    }
}

// The cell sort and the plans of the framed build in one launch of one-wave
// workgroups: both read only the binning results, so the first n_sort
// workgroups sort cells while the others plan tiles.
template <int CPL>
__global__ __launch_bounds__(kWave) void k_cells_and_plan(
    int n_sort, const SysDev *__restrict__ sys, const int64_t *__restrict__ cprefix, int n_sys,
    const int32_t *__restrict__ tprefix, int tiles,
    const double4 *__restrict__ pos, int64_t n_cells, const int32_t *__restrict__ cell_count,
    int32_t *__restrict__ cell_size, int32_t *__restrict__ cell_idx, float4 *__restrict__ cell_xf, int cell_cap,
    double4 *__restrict__ xbuild, int32_t *__restrict__ slow_list, int32_t *__restrict__ slow_n, PlanPtrs plan,
    const int32_t *__restrict__ flag, const int32_t *__restrict__ sflag, int32_t *__restrict__ halo_n,
    int halo_lds, int32_t *__restrict__ rare_list, int32_t *__restrict__ rare_n)
{
    if (*flag == 0) return;
    if ((int)blockIdx.x < n_sort) {
        cell_sort_waves<CPL>(blockIdx.x, n_sort, sys, cprefix, n_sys, pos, n_cells, cell_count, cell_size, cell_idx,
                             cell_xf, cell_cap, sflag);
    } else {
        __shared__ PlanShared ps;
        plan_tiles(ps, (int)blockIdx.x - n_sort, (int)gridDim.x - n_sort, sys, tprefix, n_sys, tiles, pos,
                   cell_count, cell_cap, xbuild, slow_list, slow_n, plan, sflag, halo_n, halo_lds, rare_list, rare_n);
    }
}

// Counts back to zero for the next binning (systems without local tiles,
// whose builds have no framed scan).
__global__ void k_zero_counts(int32_t *__restrict__ cell_count, int64_t n_cells, const int32_t *__restrict__ flag)
{
    if (*flag == 0) return;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells; c += (int64_t)gridDim.x * blockDim.x)
        cell_count[c] = 0;
}

// One tile index from a die's counter, by one lane.  The pointer gets a zero
// from a vector register that the compiler cannot see through: taken as
// divergent, the atomic is issued plainly and its result waited for where it
// is used (the pass that merges the atomics of a wave into one would wait
// for it at once).
__device__ __forceinline__ int take_tile(int32_t *ctr)
{
    int zero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    return atomicAdd(ctr + zero, 1);
}

// A plan header read through the vector memory path: the index gets a zero
// from a vector register that the compiler cannot see through, so the read is
// not made a scalar one (a pending scalar read would be waited for at the
// next LDS barrier).
__device__ __forceinline__ int4 next_header(const int4 *hdr, int tile)
{
    int zero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    return hdr[tile + zero];
}

// NT threads per workgroup (NT / 64 waves share a tile); LPR lanes scan one
// row: 64 (a wave per row) or 32 (two rows per wave).
template <bool EXCL, int NT, int LPR>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_build_fast(
    const SysDev *__restrict__ sys, const int32_t *__restrict__ tprefix, int n_sys, int tiles,
    const double4 *__restrict__ pos, const int32_t *__restrict__ tag, const int32_t *__restrict__ ptag,
    const int32_t *__restrict__ cell_size, const int32_t *__restrict__ cell_idx,
    const float4 *__restrict__ cell_xf, int cell_cap,
    uint16_t *__restrict__ nlist, int32_t *__restrict__ nn, int cap, int rstride,
    int32_t *__restrict__ halo, int32_t *__restrict__ halo_n, int halo_cap, PlanPtrs plan,
    int halo_lds, int32_t *__restrict__ rare_list, int32_t *__restrict__ rare_n, int32_t *__restrict__ tile_ctr,
    int32_t *__restrict__ cell_count, int64_t n_cells,
    const int32_t *__restrict__ flag, const int32_t *__restrict__ sflag, int32_t *build_count, Status *st)
{
    if (*flag == 0) return;
    // the binning counts, read by the cell sort and the plans, back to zero
    // for the next build
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells; c += (int64_t)gridDim.x * blockDim.x)
        cell_count[c] = 0;
    __shared__ FastShared sh;
    extern __shared__ uint16_t srows[];  // [kTile][rstride]: staged slot of each hit
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wv = tid >> 6;
    constexpr int kWaves = NT / kWave;
    static_assert(kWaves >= 2 && kWaves <= kFastWavesMax, "a loader wave and at least one more");
    static_assert(LPR == 32 || LPR == 64, "a row per wave or per half wave");
    if (blockIdx.x == 0 && tid == 0) atomicAdd(build_count, 1);

    // Each die's workgroups walk one contiguous run of tiles.  With one
    // system every tile of the run is built, and the tiles are handed out one
    // at a time from the die's counter (cleared by the binning launch): a
    // workgroup that meets costly tiles takes fewer, so the launch ends with
    // its run.  The loader wave (which makes no global writes, so its wait
    // for the count waits for no write) takes the tile after next as a tile
    // starts.  A batch rebuilds only some systems, and a count for every tile
    // it skips would cost more than it balances: there the workgroups of a
    // die take every step-th tile of the run, and skip without a barrier.
    const bool dyn = n_sys == 1;
    const int D = (int)gridDim.x < kDies ? (int)gridDim.x : kDies;
    const int die = (int)blockIdx.x % D;
    int64_t tfirst, tend;
    int tstep;
    die_range(blockIdx.x, gridDim.x, tiles, tfirst, tend, tstep);
    const int64_t dfirst = (int64_t)tiles * die / D;
    int32_t *ctr = tile_ctr + die * kTileCtrStride;
    int grabbed = 0;
    int64_t t_next = tfirst;
    if (dyn) {
        if (tid == kWave) {
            sh.grab[0] = take_tile(ctr);
            grabbed = take_tile(ctr);
        }
        lds_barrier();
        t_next = dfirst + sh.grab[0];
    }
    int par = 0;
    // each tile's plan header is read one tile ahead, by every thread, with
    // no branch, so that the read stays in flight until its use
    int4 hd_next = next_header(plan.hdr, t_next < tend ? (int)t_next : 0);
    bool built = false;  // a tile was built since the last barrier (its LDS may still be read)
    for (;;) {
        if (dyn) {
            // the next tile's index, taken during the last tile
            par ^= 1;
            if (tid == kWave) sh.grab[par] = grabbed;
        }
        if (dyn || built) lds_barrier();  // LDS of the previous tile no longer read; the index published
        built = false;
        const int64_t t_cur = t_next;
        t_next = dyn ? dfirst + sh.grab[par] : t_cur + tstep;
        if (t_cur >= tend) break;
        if (dyn && tid == kWave) grabbed = take_tile(ctr);  // the tile after next
        const int tile = (int)t_cur;
        const int4 hd_tile = hd_next;
        hd_next = next_header(plan.hdr, t_next < tend ? (int)t_next : tile);
        const int s = find_sys(tprefix, n_sys, tile);
        if (!sflag[s]) continue;  // a system that keeps its list
        built = true;
        const SysDev &S = sys[s];
        const double Ls[3] = {S.L[0], S.L[1], S.L[2]};
        const double iL[3] = {S.invL[0], S.invL[1], S.invL[2]};
        const int bins[3] = {S.bins[0], S.bins[1], S.bins[2]};
        const int per[3] = {S.per[0], S.per[1], S.per[2]};
        const int64_t row0 = S.row0, nl0 = S.nl0;
        const int n_local = S.n_local;
        const double rl2 = S.rl2;
        const int r0 = (tile - S.tile0) * kTile;

        // ---- 1. the tile's plan ------------------------------------------------
        // Wave 1 does this tile's global reads and no global writes: a wave's
        // wait for a read also waits for all of its earlier writes, and the
        // other waves still have the previous tile's rows in flight.
        const bool loader = wv == 1;
        const int tr = tid - kWave;  // lane of the loader wave
        if (loader) {
            const int4 hd = hd_tile;
            if (tr == 0) {
                sh.info[0] = hd.x;
                sh.info[1] = hd.z;
                sh.info[3] = hd.y;
                sh.info[4] = hd.w;
            }
            if (hd.x > 0) {
                const int nu_ = hd.x < kUMax ? hd.x : kUMax;
                const int64_t pu = (int64_t)tile * kUMax, pr = (int64_t)tile * kTile * kRuns;
                // every read issued before the first is used: cells past the
                // end read the last one again
                int2 cs[kUMax / kWave];
                float4 os[kUMax / kWave];
                uint32_t rv[kRuns];
                float hv[kRuns];
#pragma unroll
                for (int k = 0; k < kUMax / kWave; ++k) {
                    const int u = tr + k * kWave;
                    cs[k] = plan.cell[pu + (u < nu_ ? u : nu_ - 1)];
                    os[k] = plan.off[pu + (u < nu_ ? u : nu_ - 1)];
                }
#pragma unroll
                for (int k = 0; k < kRuns; ++k) {
                    rv[k] = plan.run[pr + tr + k * kWave];
                    hv[k] = plan.hw[pr + tr + k * kWave];
                }
                const float4 xw = plan.xrow[(int64_t)tile * kTile + tr];
                const double4 x0 = pos[row0 + r0];
#pragma unroll
                for (int k = 0; k < kUMax / kWave; ++k) {
                    const int u = tr + k * kWave;
                    if (u < nu_) {
                        sh.ucell[u] = cs[k].x;
                        sh.ustart[u] = cs[k].y;
                        sh.uoff[u] = os[k];
                    }
                }
#pragma unroll
                for (int k = 0; k < kRuns; ++k) {
                    const int e = tr + k * kWave;
                    sh.run[e / kRuns][e % kRuns] = rv[k];
                    sh.hw[e / kRuns][e % kRuns] = hv[k];
                }
                sh.xrow[tr] = xw;
                if (tr == 0) {
                    sh.ustart[nu_] = hd.y;
                    sh.xref[0] = x0.x;
                    sh.xref[1] = x0.y;
                    sh.xref[2] = x0.z;
                }
            }
        } else if (wv == 0) {
            sh.rown[tid] = r0 + tid < n_local ? 0 : -1;
        }
        lds_barrier();
        const int nu = uni(sh.info[0]);
        const int nslot = uni(sh.info[3]);
        if (nu <= 0 || nu > kUMax || nslot > kFastSlotMax) continue;  // built by the general kernel
        const double xr[3] = {uni(sh.xref[0]), uni(sh.xref[1]), uni(sh.xref[2])};
        for (int q = tid; q < (nslot + 31) / 32; q += NT) sh.used[q] = 0u;
        // ---- 5. stage members a chunk at a time, scan every row's lines -------------
        const bool one_chunk = nslot <= kFastChunk;
        // FP32 distances below lo_f are hits, above hi_f misses, in between
        // the exact FP64 test decides (the band comes with the tile's plan)
        const double band = (double)__int_as_float(uni(sh.info[4]));
        const float lo_f = (float)(rl2 * (1.0 - band)), hi_f = (float)(rl2 * (1.0 + band));
        for (int q0 = 0; q0 < nslot; q0 += kFastChunk) {
            const int q1 = q0 + kFastChunk < nslot ? q0 + kFastChunk : nslot;
            lds_barrier();
            // slot -> distinct cell of the chunk: each cell writes its index
            // over its own slots
            for (int u = tid; u < nu; u += NT) {
                int qa = sh.ustart[u], qb = sh.ustart[u + 1];
                qa = qa > q0 ? qa : q0;
                qb = qb < q1 ? qb : q1;
                for (int q = qa; q < qb; ++q) sh.smap[q - q0] = (uint8_t)u;
            }
            lds_barrier();
            // staging: one coalesced read per member (cell-relative FP32
            // position and row), moved into the frame by its cell's corner;
            // four reads of a thread in flight at once
            {
                constexpr int kB = 4;
                for (int qb = q0 + tid; qb < q1; qb += kB * NT) {
                    int us[kB], qs[kB];
                    float4 cs[kB];
#pragma unroll
                    for (int k = 0; k < kB; ++k) {
                        const int q = qb + k * NT;
                        qs[k] = q;
                        us[k] = q < q1 ? (int)sh.smap[q - q0] : 0;
                    }
#pragma unroll
                    for (int k = 0; k < kB; ++k)
                        if (qs[k] < q1) cs[k] = cell_xf[(int64_t)sh.ucell[us[k]] * cell_cap + (qs[k] - sh.ustart[us[k]])];
#pragma unroll
                    for (int k = 0; k < kB; ++k) {
                        const int q = qb + k * NT;
                        if (q < q1) {
                            const float4 o = sh.uoff[us[k]];
                            sh.cp[q - q0] = make_float4(cs[k].x + o.x, cs[k].y + o.y, cs[k].z + o.z, cs[k].w);
                        }
                    }
                }
            }
            lds_barrier();
            // members of a line are ordered by x (cells in x order, each sorted
            // by x): cut every line, within this chunk, to the slots within the
            // half width that its y-z distance leaves (|dx|^2 <= r_list^2 - gap^2,
            // widened by a margin for the FP32 frame coordinates)
            for (int e = tid; e < kTile * kRuns; e += NT) {
                const int t = e / kRuns, rr = e - kRuns * (e / kRuns);
                const uint32_t v = sh.run[t][rr];
                int a = (int)(v & 0xffffu), b = (int)(v >> 16);
                a = a > q0 ? a : q0;
                b = b < q1 ? b : q1;
                if (b <= a) {
                    sh.runc[t][rr] = 0u;
                    continue;
                }
                const float hw = sh.hw[t][rr];
                const float xc = sh.xrow[t].x;
                const float tlo = xc - hw, thi = xc + hw;
                // first slot with x >= tlo, first slot with x > thi
                int pa = a, pb = a;
                int step = 1;
                while (2 * step <= b - a) step *= 2;
                for (; step > 0; step >>= 1) {
                    if (pa + step <= b && sh.cp[pa + step - 1 - q0].x < tlo) pa += step;
                    if (pb + step <= b && sh.cp[pb + step - 1 - q0].x <= thi) pb += step;
                }
                sh.runc[t][rr] = (uint32_t)pa | ((uint32_t)(pb > pa ? pb : pa) << 16);
            }
            lds_barrier();
            if constexpr (LPR == 64) {
                // lanes to lines, one thread per row: line r takes lanes [B_r, B_r+1)
                // with B_r = r + about 55 P_r / T (P_r the members of the row's lines
                // before line r in this chunk, T all of them), so every line keeps at
                // least one lane and longer lines get more.  Kept as the first lanes
                // and a mask with the last lane of every line but the last.
                if (tid < kTile) {
                    int lens[kRuns];
                    int tot = 0;
    #pragma unroll
                    for (int r = 0; r < kRuns; ++r) {
                        const uint32_t rv = sh.runc[tid][r];
                        const int x0_ = (int)(rv & 0xffffu), x1_ = (int)(rv >> 16);
                        lens[r] = x1_ > x0_ ? x1_ - x0_ : 0;
                        tot += lens[r];
                    }
                    const uint32_t inv = tot > 0 ? 65536u / (uint32_t)tot : 0u;  // floor(2^16 / T)
                    uint64_t mask = 0;
                    int pre = 0, b0 = 0;
    #pragma unroll
                    for (int r = 0; r < kRuns; ++r) {
                        const int pn = pre + lens[r];
                        const int b1 = r == kRuns - 1 ? kWave : r + 1 + (int)((55u * (uint32_t)pn * inv) >> 16);
                        sh.lb[tid][r] = (uint8_t)b0;
                        if (r < kRuns - 1) mask |= 1ull << (b1 - 1);
                        b0 = b1;
                        pre = pn;
                    }
                    sh.lb[tid][kRuns] = (uint8_t)kWave;
                    sh.lmask[tid] = tot > 0 ? mask : 0ull;
                    if (tot == 0 && sh.rown[tid] >= 0) sh.lb[tid][0] = 0xFF;  // nothing to scan in this chunk
                }
                lds_barrier();
                for (int t = wv; t < kTile; t += kWaves) {
                    int ntot = uni(sh.rown[t]);
                    if (ntot < 0) continue;  // inactive row
                    if (uni((int)sh.lb[t][0]) == 0xFF) continue;  // no members in this chunk
                    // this lane's line: the lines that end before it; its lanes,
                    // members (cut to the chunk) and stride
                    const uint64_t lm = sh.lmask[t];
                    int myline = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(lm >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)lm, 0u));
                    myline = myline < kRuns - 1 ? myline : kRuns - 1;
                    const int blo_ = sh.lb[t][myline], bhi_ = sh.lb[t][myline + 1];
                    const uint32_t rv = sh.runc[t][myline];
                    const int x0_ = (int)(rv & 0xffffu), x1_ = (int)(rv >> 16);
                    const int gsz = bhi_ - blo_ > 1 ? bhi_ - blo_ : 1;
                    const int base = x0_ + (lane - blo_);
                    const int end = x1_;
                    const float4 xt0 = sh.xrow[t];
                    const float4 xt = make_float4(uni(xt0.x), uni(xt0.y), uni(xt0.z), 0.f);
                    const int32_t it = (int32_t)(row0 + r0 + t);
                    int32_t part[kMaxBondCap];
                    if constexpr (EXCL) {
                        const int64_t prow = (int64_t)it * S.bond_stride;
    #pragma unroll
                        for (int bnd = 0; bnd < kMaxBondCap; ++bnd)
                            part[bnd] = bnd < S.bond_cap ? ptag[prow + bnd] : -1;
                    }
                    uint16_t *myrow = srows + t * rstride;
                    // exact FP64 decision of a candidate whose FP32 distance is
                    // within the band around r_list
                    auto exact = [&](const float4 c) -> bool {
                        const int32_t j = __float_as_int(c.w);
                        const double4 xa = pos[it], xb = pos[j];
                        const double cj[3] = {(double)c.x, (double)c.y, (double)c.z};
                        const double xt3[3] = {(double)xt.x, (double)xt.y, (double)xt.z};
                        const double pa[3] = {xa.x, xa.y, xa.z}, pb[3] = {xb.x, xb.y, xb.z};
                        double d[3];
    #pragma unroll
                        for (int ax = 0; ax < 3; ++ax) {
                            // frame images of both: k = round((frame - stored) / L)
                            const double kj = rint((cj[ax] + xr[ax] - pb[ax]) * iL[ax]);
                            const double ki = rint((xt3[ax] + xr[ax] - pa[ax]) * iL[ax]);
                            d[ax] = pb[ax] - pa[ax];
                            if (kj != ki) d[ax] = d[ax] + (kj - ki) * Ls[ax];
                        }
                        return norm2_exact(d[0], d[1], d[2]) < rl2 && j != it;
                    };
                    auto excluded = [&](bool hit, const float4 c) -> bool {
                        if constexpr (EXCL) {
                            if (hit) {
                                const int32_t tj = tag[__float_as_int(c.w)];
    #pragma unroll
                                for (int bnd = 0; bnd < kMaxBondCap; ++bnd) hit = hit && part[bnd] != tj;
                            }
                        }
                        return hit;
                    };
                    // a hit goes to the row's next entry (entries past the
                    // capacity land on the row's spare slot) and marks its slot
                    auto append = [&](bool hit, uint64_t mask, int q) {
                        if (hit) {
                            const int p = ntot + (int)__builtin_amdgcn_mbcnt_hi(
                                                     (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                            myrow[p < cap ? p : cap] = (uint16_t)q;
                            atomicOr(&sh.used[q >> 5], 1u << (q & 31));
                        }
                        ntot += __popcll(mask);
                    };
                    // every lane reads a slot of the chunk, clamped: lanes past
                    // their line's end take no part
                    const float4 *cq = sh.cp - q0;
                    const int qlast = q1 - 1;
                    for (int qa = base;; qa += 2 * gsz) {
                        const int qb = qa + gsz;
                        const bool ona = qa < end, onb = qb < end;
                        if (__ballot(ona) == 0ull) break;
                        const float4 ca = cq[qa < qlast ? qa : qlast];
                        const float4 cb = cq[qb < qlast ? qb : qlast];
                        const float dxa = ca.x - xt.x, dya = ca.y - xt.y, dza = ca.z - xt.z;
                        const float dxb = cb.x - xt.x, dyb = cb.y - xt.y, dzb = cb.z - xt.z;
                        const float r2a = dxa * dxa + dya * dya + dza * dza;
                        const float r2b = dxb * dxb + dyb * dyb + dzb * dzb;
                        bool ha = ona && r2a < lo_f && __float_as_int(ca.w) != it;
                        bool hb = onb && r2b < lo_f && __float_as_int(cb.w) != it;
                        const bool ba = ona && r2a >= lo_f && r2a <= hi_f;
                        const bool bb = onb && r2b >= lo_f && r2b <= hi_f;
                        if (__builtin_expect(__ballot(ba || bb) != 0ull, 0)) {
                            if (ba) ha = exact(ca);
                            if (bb) hb = exact(cb);
                        }
                        ha = excluded(ha, ca);
                        hb = excluded(hb, cb);
                        const uint64_t ma = __ballot(ha), mb = __ballot(hb);
                        append(ha, ma, qa);
                        append(hb, mb, qb);
                    }
                    if (lane == 0) sh.rown[t] = ntot;
                }
            } else {
                // lanes to lines, one thread per row.  Two rows share a wave, 32
                // lanes each, two members per lane per pass: the fewest passes P
                // such that ceil(len / 2P) lanes for every non-empty line of the
                // row (in this chunk) take at most 32 lanes.  Kept per row: the
                // non-empty lines in order with their first lanes (then the lanes
                // used), and a mask with the last lane of each line but the last.
                if (tid < kTile) {
                    int lens[kRuns];
                    int tot = 0;
    #pragma unroll
                    for (int r = 0; r < kRuns; ++r) {
                        const uint32_t rv = sh.runc[tid][r];
                        const int x0_ = (int)(rv & 0xffffu), x1_ = (int)(rv >> 16);
                        lens[r] = x1_ > x0_ ? x1_ - x0_ : 0;
                        tot += lens[r];
                    }
                    // at 2P >= the longest line every non-empty line takes one
                    // lane (at most nine), so the search ends
                    int d = 2 * ((tot + 63) >> 6);
                    d = d > 2 ? d : 2;
                    for (;;) {
                        int lanes = 0;
    #pragma unroll
                        for (int r = 0; r < kRuns; ++r) lanes += (lens[r] + d - 1) / d;
                        if (lanes <= 32) break;
                        d += 2;
                    }
                    uint32_t mask = 0u;
                    int nk = 0, b0 = 0;
    #pragma unroll
                    for (int r = 0; r < kRuns; ++r) {
                        if (lens[r] == 0) continue;
                        if (nk > 0) mask |= 1u << (b0 - 1);
                        sh.ln[tid][nk] = (uint8_t)r;
                        sh.lb[tid][nk] = (uint8_t)b0;
                        b0 += (lens[r] + d - 1) / d;
                        ++nk;
                    }
                    sh.lb[tid][nk] = (uint8_t)b0;
                    sh.lmask[tid] = mask;
                    sh.nk[tid] = (uint8_t)nk;
                }
                lds_barrier();
                // rows t0 (lanes 0-31) and t0 + 1 (lanes 32-63) of each wave
                const int hh = lane >> 5, hl = lane & 31;
                const float4 *cq = sh.cp - q0;
                const int qlast = q1 - 1;
                for (int t0 = 2 * wv; t0 < kTile; t0 += 2 * kWaves) {
                    const int t = t0 + hh;
                    const int nk = sh.nk[t];
                    int ntot = sh.rown[t];
                    const bool row_on = ntot >= 0 && nk > 0;  // an active row with members in this chunk
                    if (__ballot(row_on) == 0ull) continue;
                    // this lane's line: the lines that end before it; its lanes,
                    // members (cut to the chunk) and stride.  Lanes without a line
                    // start at the chunk's first slot with nothing to scan.
                    int base = q0, end = q0, gsz = 1;
                    if (row_on) {
                        const int used_lanes = sh.lb[t][nk];
                        if (hl < used_lanes) {
                            int k = __popc(sh.lmask[t] & ((1u << hl) - 1u));
                            k = k < nk - 1 ? k : nk - 1;
                            const int r = sh.ln[t][k];
                            const int blo_ = sh.lb[t][k], bhi_ = sh.lb[t][k + 1];
                            const uint32_t rv = sh.runc[t][r];
                            gsz = bhi_ - blo_;
                            base = (int)(rv & 0xffffu) + (hl - blo_);
                            end = (int)(rv >> 16);
                        }
                    }
                    const float4 xt = sh.xrow[t];
                    const int32_t it = (int32_t)(row0 + r0 + t);
                    int32_t part[kMaxBondCap];
                    if constexpr (EXCL) {
    #pragma unroll
                        for (int bnd = 0; bnd < kMaxBondCap; ++bnd) part[bnd] = -1;
                        if (row_on) {
                            const int64_t prow = (int64_t)it * S.bond_stride;
    #pragma unroll
                            for (int bnd = 0; bnd < kMaxBondCap; ++bnd)
                                part[bnd] = bnd < S.bond_cap ? ptag[prow + bnd] : -1;
                        }
                    }
                    uint16_t *myrow = srows + t * rstride;
                    // exact FP64 decision of a candidate whose FP32 distance is
                    // within the band around r_list
                    auto exact = [&](const float4 c) -> bool {
                        const int32_t j = __float_as_int(c.w);
                        const double4 xa = pos[it], xb = pos[j];
                        const double cj[3] = {(double)c.x, (double)c.y, (double)c.z};
                        const double xt3[3] = {(double)xt.x, (double)xt.y, (double)xt.z};
                        const double pa[3] = {xa.x, xa.y, xa.z}, pb[3] = {xb.x, xb.y, xb.z};
                        double d[3];
    #pragma unroll
                        for (int ax = 0; ax < 3; ++ax) {
                            // frame images of both: k = round((frame - stored) / L)
                            const double kj = rint((cj[ax] + xr[ax] - pb[ax]) * iL[ax]);
                            const double ki = rint((xt3[ax] + xr[ax] - pa[ax]) * iL[ax]);
                            d[ax] = pb[ax] - pa[ax];
                            if (kj != ki) d[ax] = d[ax] + (kj - ki) * Ls[ax];
                        }
                        return norm2_exact(d[0], d[1], d[2]) < rl2 && j != it;
                    };
                    auto excluded = [&](bool hit, const float4 c) -> bool {
                        if constexpr (EXCL) {
                            if (hit) {
                                const int32_t tj = tag[__float_as_int(c.w)];
    #pragma unroll
                                for (int bnd = 0; bnd < kMaxBondCap; ++bnd) hit = hit && part[bnd] != tj;
                            }
                        }
                        return hit;
                    };
                    // a hit goes to its row's next entry (entries past the
                    // capacity land on the row's spare slot); the count of each
                    // half of the wave is its own row's
                    auto append = [&](bool hit, int q) {
                        const uint64_t m = __ballot(hit);
                        const uint32_t mlo = (uint32_t)m, mhi = (uint32_t)(m >> 32);
                        if (hit) {
                            const int below = hh ? (int)__builtin_amdgcn_mbcnt_hi(mhi, 0u)
                                                 : (int)__builtin_amdgcn_mbcnt_lo(mlo, 0u);
                            const int p = ntot + below;
                            myrow[p < cap ? p : cap] = (uint16_t)q;
                        }
                        ntot += hh ? __popc(mhi) : __popc(mlo);
                    };
                    // every lane reads a slot of the chunk, clamped: lanes past
                    // their line's end take no part
                    for (int qa = base;; qa += 2 * gsz) {
                        const int qb = qa + gsz;
                        const bool ona = qa < end, onb = qb < end;
                        if (__ballot(ona) == 0ull) break;
                        const float4 ca = cq[qa < qlast ? qa : qlast];
                        const float4 cb = cq[qb < qlast ? qb : qlast];
                        const float dxa = ca.x - xt.x, dya = ca.y - xt.y, dza = ca.z - xt.z;
                        const float dxb = cb.x - xt.x, dyb = cb.y - xt.y, dzb = cb.z - xt.z;
                        const float r2a = dxa * dxa + dya * dya + dza * dza;
                        const float r2b = dxb * dxb + dyb * dyb + dzb * dzb;
                        const bool la = r2a < lo_f, lb2 = r2b < lo_f;
                        bool ha = ona && la && __float_as_int(ca.w) != it;
                        bool hb = onb && lb2 && __float_as_int(cb.w) != it;
                        const bool ba = ona && !la && r2a <= hi_f;
                        const bool bb = onb && !lb2 && r2b <= hi_f;
                        if (__builtin_expect(__ballot(ba || bb) != 0ull, 0)) {
                            if (ba) ha = exact(ca);
                            if (bb) hb = exact(cb);
                        }
                        ha = excluded(ha, ca);
                        hb = excluded(hb, cb);
                        append(ha, qa);
                        append(hb, qb);
                    }
                    if (hl == 0 && row_on) sh.rown[t] = ntot;
                }
            }
        }
        lds_barrier();
        // ---- 6. halo numbering, rows out ------------------------------------------
        // writers: every wave but the loader
        const int wid = wv == 0 ? tid : tid - kWave;
        constexpr int kWriters = NT - kWave;
        const bool act0 = tid < kTile && r0 + tid < n_local;
        const int64_t i0 = row0 + r0 + tid;
        if (wv == 0) {
            // longest row of the tile: a wave reduction
            int n = act0 ? sh.rown[tid] : 0;
            n = wave_max_full(n < cap ? n : cap);
            if (tid == 0) sh.info[2] = n;
        }
        if constexpr (LPR == 32) {
            // the staged slots that some row lists (the 64-lane scan marks
            // them as it finds them)
            lds_barrier();
            const int kmax_ = uni(sh.info[2]);
            for (int e = tid; e < kmax_ * kTile; e += NT) {
                const int t = e & (kTile - 1), k = e >> 6;
                int n = sh.rown[t];
                n = n < cap ? n : cap;
                if (k < n) {
                    const int q = srows[t * rstride + k];
                    atomicOr(&sh.used[q >> 5], 1u << (q & 31));
                }
            }
            lds_barrier();  // every mark made before the words are counted
        }
        const int nwords = (nslot + 31) / 32;
        for (int q = tid; q < nwords; q += NT) sh.wpre[q] = __popc(sh.used[q]);
        lds_barrier();
        const int nhalo = uni(block_scan_w<NT>(sh.wpre, nwords, sh.scan));
        if (nhalo > halo_cap) {
            if (tid == 0) latch(st, 11 /*HALO_OVERFLOW*/, nhalo);
            if (act0) nn[i0] = 0;
            if (tid == 0) halo_n[tile] = 0;
            continue;
        }
        int32_t *hl = halo + (int64_t)tile * halo_cap;
        for (int q = loader ? nslot : wid; q < nslot; q += kWriters) {
            const uint32_t word = sh.used[q >> 5];
            if (word & (1u << (q & 31))) {
                const int h = sh.wpre[q >> 5] + __popc(word & ((1u << (q & 31)) - 1u));
                int32_t j;
                if (one_chunk) {
                    j = __float_as_int(sh.cp[q].w);
                } else {
                    const int u = upper_idx(sh.ustart, nu, q);
                    j = cell_idx[(int64_t)sh.ucell[u] * cell_cap + (q - sh.ustart[u])];
                }
                hl[h] = j;
            }
        }
        const int kmax = uni(sh.info[2]);
        if (tid == 0) {
            halo_n[tile] = (int32_t)((uint32_t)nhalo | ((uint32_t)kmax << 16) | (sh.info[1] ? 0x80000000u : 0u));
            // per-pair images or a halo beyond the force pass's LDS staging
            if (sh.info[1] || nhalo > halo_lds) rare_list[atomicAdd(rare_n, 1)] = tile;
        }
        uint16_t *out = nlist + nl0 + (int64_t)(r0 >> 6) * cap * kTile;
        // four entries of a thread at a time, their LDS reads issued together
        constexpr int kOut = 4;
        for (int e0 = loader ? kmax * kTile : wid; e0 < kmax * kTile; e0 += kOut * kWriters) {
            int q[kOut];
#pragma unroll
            for (int b = 0; b < kOut; ++b) {
                const int e = e0 + b * kWriters;
                const int k = e >> 6, t = e & 63;
                const int n = sh.rown[t];
                q[b] = e < kmax * kTile && k < n && k < cap ? (int)srows[t * rstride + k] : -1;
            }
#pragma unroll
            for (int b = 0; b < kOut; ++b) {
                const int e = e0 + b * kWriters;
                if (e < kmax * kTile) {
                    uint16_t v = 0;
                    if (q[b] >= 0) {
                        const uint32_t word = sh.used[q[b] >> 5];
                        v = (uint16_t)(sh.wpre[q[b] >> 5] + __popc(word & ((1u << (q[b] & 31)) - 1u)));
                    }
                    out[e] = v;
                }
            }
        }
        if (act0) {
            const int n = sh.rown[tid];
            nn[i0] = n < cap ? n : cap;
            if (n > cap) latch(st, 5 /*NLIST_OVERFLOW*/, n);
        }
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

static int capped(int64_t blocks) { return (int)(blocks < kRebuildGrid ? (blocks > 0 ? blocks : 1) : kRebuildGrid); }

void launch_bin(const LaunchCtx &L, const double4 *pos, int nvt_w)
{
    if (L.tiles_all == 0) return;
    const int blocks = capped(((int64_t)L.tiles_all * kWave + 255) / 256);
    hipLaunchKernelGGL(k_bin, dim3(blocks), dim3(256), 0, L.stream, L.sys, L.tprefix_all, L.n_sys,
                       L.tiles_all, pos, L.cell_count, L.cell_idx, L.cell_cap, L.flag, L.sflag, L.status,
                       L.step_counter, L.slow_n, L.rare_n, L.tile_ctr, L.since, L.since_inc, L.tprefix_local, nvt_w,
                       nvt_w > 0 && L.nvt ? L.khalf : nullptr, L.thermostat);
}

void launch_cell_sort(const LaunchCtx &L, const double4 *pos)
{
    if (L.n_cells == 0) return;
    // one-wave workgroups: the cell sort (a multiple of the die count, so
    // that the plan workgroups keep their die mapping), then the plans
    int64_t n_sort = L.n_cells < 8192 ? L.n_cells : 8192;
    n_sort = (n_sort + kDies - 1) / kDies * kDies;
    const int n_plan = L.tiles_local < kPlanGrid ? L.tiles_local : kPlanGrid;
    const PlanPtrs plan = plan_ptrs(L.plan, L.tiles_local);
    const dim3 grid((unsigned)(n_sort + n_plan));
    if (L.cell_cap <= 64)
        hipLaunchKernelGGL(k_cells_and_plan<1>, grid, dim3(kWave), 0, L.stream, (int)n_sort, L.sys, L.cprefix, L.n_sys,
                           L.tprefix_local, L.tiles_local, pos, L.n_cells, L.cell_count, L.cell_size, L.cell_idx,
                           L.cell_xf, L.cell_cap, L.xbuild, L.slow_list, L.slow_n, plan, L.flag, L.sflag,
                           L.halo_n, L.halo_lds, L.rare_list, L.rare_n);
    else
        hipLaunchKernelGGL(k_cells_and_plan<2>, grid, dim3(kWave), 0, L.stream, (int)n_sort, L.sys, L.cprefix, L.n_sys,
                           L.tprefix_local, L.tiles_local, pos, L.n_cells, L.cell_count, L.cell_size, L.cell_idx,
                           L.cell_xf, L.cell_cap, L.xbuild, L.slow_list, L.slow_n, plan, L.flag, L.sflag,
                           L.halo_n, L.halo_lds, L.rare_list, L.rare_n);
}

int nlist_row_stride(int cap)
{
    // uint16 entries per staged row; an odd number of words keeps the
    // transposed read-out free of bank conflicts
    // one spare entry past the capacity takes the writes of an overflowing row
    int r = cap + 1 + ((cap + 1) & 1);
    if (((r / 2) & 1) == 0) r += 2;
    return r;
}

int nlist_lanes_per_row() { return kWave; }
int nlist_block() { return kFastThreads; }
bool nlist_shape_ok(int lanes_per_row, int block)
{
    return (lanes_per_row == 32 || lanes_per_row == 64) && (block == 256 || block == 512);
}

size_t fast_build_lds_bytes(int cap) { return sizeof(FastShared) + (size_t)kTile * nlist_row_stride(cap) * 2; }

size_t build_plan_bytes(int64_t tiles)
{
    // the carving of plan_ptrs, with every part rounded to 256 bytes
    auto r = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t t = (size_t)(tiles > 0 ? tiles : 1);
    return r(sizeof(int4) * t) + r(sizeof(int2) * t * kUMax) + r(sizeof(float4) * t * kUMax) +
           r(sizeof(float4) * t * kTile) + r(sizeof(uint32_t) * t * kTile * kRuns) +
           r(sizeof(float) * t * kTile * kRuns);
}

template <bool EXCL, int NT, int LPR>
static hipError_t fast_attr(int dyn)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_build_fast<EXCL, NT, LPR>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
}

hipError_t prepare_nlist(int cap)
{
    const int dyn = kTile * nlist_row_stride(cap) * 2;
    const hipError_t es[8] = {fast_attr<false, 512, 64>(dyn), fast_attr<false, 256, 64>(dyn),
                              fast_attr<false, 512, 32>(dyn), fast_attr<false, 256, 32>(dyn),
                              fast_attr<true, 512, 64>(dyn),  fast_attr<true, 256, 64>(dyn),
                              fast_attr<true, 512, 32>(dyn),  fast_attr<true, 256, 32>(dyn)};
    for (hipError_t e : es)
        if (e != hipSuccess) return e;
    return hipSuccess;
}

template <bool EXCL, int NT, int LPR>
static void fast_inst(const LaunchCtx &L, const double4 *pos, const int32_t *tag, int blocks, int rs, size_t dyn,
                      const PlanPtrs &plan)
{
    hipLaunchKernelGGL((k_build_fast<EXCL, NT, LPR>), dim3(blocks), dim3(NT), dyn, L.stream, L.sys, L.tprefix_local,
                       L.n_sys, L.tiles_local, pos, tag, L.ptag, L.cell_size, L.cell_idx, L.cell_xf, L.cell_cap,
                       L.nlist, L.nn, L.nlist_cap, rs, L.halo, L.halo_n, L.halo_cap, plan, L.halo_lds, L.rare_list,
                       L.rare_n, L.tile_ctr, L.cell_count, L.n_cells, L.flag, L.sflag, L.build_count, L.status);
}

template <bool EXCL>
static void fast_shape(const LaunchCtx &L, const double4 *pos, const int32_t *tag, int blocks, int rs, size_t dyn,
                       const PlanPtrs &plan, int w, int block)
{
    if (w == 32) {
        if (block == 256) fast_inst<EXCL, 256, 32>(L, pos, tag, blocks, rs, dyn, plan);
        else fast_inst<EXCL, 512, 32>(L, pos, tag, blocks, rs, dyn, plan);
    } else {
        if (block == 256) fast_inst<EXCL, 256, 64>(L, pos, tag, blocks, rs, dyn, plan);
        else fast_inst<EXCL, 512, 64>(L, pos, tag, blocks, rs, dyn, plan);
    }
}

// w: lanes per row of the framed build (64 or 32); block: its threads per
// workgroup (512 or 256).  The general build's shape is fixed.
void launch_nlist(const LaunchCtx &L, const double4 *pos, const int32_t *tag, int w, int block)
{
    if (L.tiles_local == 0) {
        // no framed scan to clear the cell counts
        if (L.n_cells > 0)
            hipLaunchKernelGGL(k_zero_counts, dim3(256), dim3(256), 0, L.stream, L.cell_count, L.n_cells, L.flag);
        return;
    }
    const int blocks = capped(L.tiles_local);
    const int rs = nlist_row_stride(L.nlist_cap);
    const size_t dyn = (size_t)kTile * rs * 2;
    const PlanPtrs plan = plan_ptrs(L.plan, L.tiles_local);
    if (L.has_bonds) {
        fast_shape<true>(L, pos, tag, blocks, rs, dyn, plan, w, block);
        hipLaunchKernelGGL(k_build_tile<true>, dim3(blocks), dim3(kBuildThreads), 0, L.stream, L.sys,
                           L.tprefix_local, L.n_sys, L.tiles_local, pos, tag, L.ptag, L.cell_size,
                           L.cell_idx, L.cell_cap, L.nlist, L.nn, L.nlist_cap, L.halo, L.halo_n,
                           L.halo_cap, L.xbuild, L.slow_list, L.slow_n, L.halo_lds, L.rare_list, L.rare_n, L.flag,
                           nullptr, L.status);
    } else {
        fast_shape<false>(L, pos, tag, blocks, rs, dyn, plan, w, block);
        hipLaunchKernelGGL(k_build_tile<false>, dim3(blocks), dim3(kBuildThreads), 0, L.stream, L.sys,
                           L.tprefix_local, L.n_sys, L.tiles_local, pos, tag, L.ptag, L.cell_size,
                           L.cell_idx, L.cell_cap, L.nlist, L.nn, L.nlist_cap, L.halo, L.halo_n,
                           L.halo_cap, L.xbuild, L.slow_list, L.slow_n, L.halo_lds, L.rare_list, L.rare_n, L.flag,
                           nullptr, L.status);
    }
}

}  // namespace md
