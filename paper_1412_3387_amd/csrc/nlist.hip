// nlist.hip -- cell list and tile-halo Verlet neighbour list (Sec. 5.1,
// Fig. 4, rebuilt for LDS-staged tiles on CDNA).
//
// Cell list: fixed-capacity bins.  A binning pass assigns every row to the
// cell floor((x - lo) * bins / L); lanes of a wave that hit the same cell
// claim their slots with one integer atomic per distinct cell.  A per-cell
// pass then sorts the members of each cell by row index (rank sort inside
// one wave), so the list is deterministic although the slots were claimed
// in arbitrary order.  It also resets the counters for the next build.
//
// Neighbour list: one workgroup per tile of 64 consecutive rows (Morton
// ordered rows make a tile one or a few compact clusters).  The workgroup
//   1. collects the stencil cells of all its rows and sorts out the
//      distinct ones (bitonic sort in LDS), so any tile shape works,
//   2. stages the members of those cells (positions and row numbers) in LDS,
//      a chunk at a time,
//   3. lets W = 4 lanes per particle stride over the members of the
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

constexpr int kBuildThreads = 256;   // 64 rows x 4 lanes
constexpr int kBuildW = 4;
constexpr int kChunk = 512;          // members staged at once
constexpr int kSlotMax = 16384;      // members of a tile's stencil cells
constexpr int kRebuildGrid = 2048;   // blocks of the grid-stride rebuild kernels
constexpr int kKeys = 2048;          // 64 rows x 27 stencil cells, padded
constexpr int kStencil = 27;

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bin(const SysDev *__restrict__ sys,
                                             const int32_t *__restrict__ tprefix, int n_sys, int tiles,
                                             const double4 *__restrict__ pos,
                                             int32_t *__restrict__ cell_count,
                                             int32_t *__restrict__ cell_idx, int cell_cap,
                                             const int32_t *__restrict__ flag, Status *st,
                                             uint32_t *step_counter)
{
    // the binning launch follows every fused step launch: it also advances
    // the device step counter read by graph-replayed steps
    if (step_counter && blockIdx.x == 0 && threadIdx.x == 0) *step_counter += 1u;
    if (*flag == 0) return;
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const int waves = (int)(gridDim.x * blockDim.x) >> 6;
    for (int g = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); g < tiles; g += waves) {
        const int s = find_sys(tprefix, n_sys, g);
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

// One wave per cell: members ranked by row index, sizes published, counters
// cleared.  cell_cap <= 64 * CPL.
template <int CPL>
__global__ __launch_bounds__(256) void k_cell_sort(int64_t n_cells, int32_t *__restrict__ cell_count,
                                                   int32_t *__restrict__ cell_size,
                                                   int32_t *__restrict__ cell_idx, int cell_cap,
                                                   const int32_t *__restrict__ flag)
{
    if (*flag == 0) return;
    const int lane = lane_id();
    const int64_t waves = (int64_t)(gridDim.x * blockDim.x) >> 6;
    for (int64_t c = (int64_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); c < n_cells; c += waves) {
        int m = cell_count[c];
        m = m < cell_cap ? m : cell_cap;
        int32_t v[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const int k = q * kWave + lane;
            v[q] = k < m ? cell_idx[c * cell_cap + k] : INT32_MAX;
        }
        int rank[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q) rank[q] = 0;
#pragma unroll
        for (int q2 = 0; q2 < CPL; ++q2) {
            const int tmax = m - q2 * kWave < kWave ? m - q2 * kWave : kWave;
            for (int t = 0; t < tmax; ++t) {
                const int32_t other = __shfl(v[q2], t, kWave);
#pragma unroll
                for (int q = 0; q < CPL; ++q) rank[q] += other < v[q] ? 1 : 0;
            }
        }
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const int k = q * kWave + lane;
            if (k < m) cell_idx[c * cell_cap + rank[q]] = v[q];
        }
        if (lane == 0) {
            cell_size[c] = m;
            cell_count[c] = 0;
        }
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

// Exclusive block scan of n <= 8 * kBuildThreads values held in LDS `a`
// (in place); returns the total.
__device__ __forceinline__ int block_scan8(int32_t *a, int n, int32_t *scan)
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
    for (int off = 1; off < kBuildThreads; off <<= 1) {
        const int add = tid >= off ? scan[tid - off] : 0;
        __syncthreads();
        scan[tid] += add;
        __syncthreads();
    }
    int run = tid > 0 ? scan[tid - 1] : 0;
    const int total = scan[kBuildThreads - 1];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (b + k < n) {
            a[b + k] = run;
            run += v[k];
        }
    __syncthreads();
    return total;
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
    const double4 *__restrict__ pos, const int32_t *__restrict__ tag, const int32_t *__restrict__ partners,
    const int32_t *__restrict__ cell_size, const int32_t *__restrict__ cell_idx, int cell_cap,
    uint16_t *__restrict__ nlist, int32_t *__restrict__ nn, int cap, int32_t *__restrict__ halo,
    int32_t *__restrict__ halo_n, int halo_cap, double4 *__restrict__ xbuild,
    const int32_t *__restrict__ flag, int32_t *build_count, Status *st)
{
    if (*flag == 0) return;
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
    if (blockIdx.x == 0 && tid == 0) atomicAdd(build_count, 1);

    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
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
        // distinct keys: flag first occurrences, scan, compact
        int flags8[8];
        int32_t kv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = 8 * tid + k;
            kv[k] = sh.keys[q];
            flags8[k] = (kv[k] != INT32_MAX && (q == 0 || kv[k] != sh.keys[q - 1])) ? 1 : 0;
            sh.ucount[q] = flags8[k];
        }
        __syncthreads();
        const int nu = block_scan8(sh.ucount, kKeys, sh.scan);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (flags8[k]) sh.keys[sh.ucount[8 * tid + k]] = kv[k];
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
                const int64_t prow = (row0 + tag[i]) * S.bond_cap;
                for (int b = 0; b < S.bond_cap && b < kMaxBondCap; ++b) part[b] = partners[prow + b];
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
        if (tid == 0)
            halo_n[tile] = (int32_t)((uint32_t)nhalo | ((uint32_t)sh.info[2] << 16) | (sh.info[1] ? 0x80000000u : 0u));
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
// host-side launchers
// ---------------------------------------------------------------------------

static int capped(int64_t blocks) { return (int)(blocks < kRebuildGrid ? (blocks > 0 ? blocks : 1) : kRebuildGrid); }

void launch_bin(const LaunchCtx &L, const double4 *pos)
{
    if (L.tiles_all == 0) return;
    const int blocks = capped(((int64_t)L.tiles_all * kWave + 255) / 256);
    hipLaunchKernelGGL(k_bin, dim3(blocks), dim3(256), 0, L.stream, L.sys, L.tprefix_all, L.n_sys,
                       L.tiles_all, pos, L.cell_count, L.cell_idx, L.cell_cap, L.flag, L.status,
                       L.step_counter);
}

void launch_cell_sort(const LaunchCtx &L)
{
    if (L.n_cells == 0) return;
    const int blocks = capped((L.n_cells * kWave + 255) / 256);
    if (L.cell_cap <= 64)
        hipLaunchKernelGGL(k_cell_sort<1>, dim3(blocks), dim3(256), 0, L.stream, L.n_cells, L.cell_count,
                           L.cell_size, L.cell_idx, L.cell_cap, L.flag);
    else
        hipLaunchKernelGGL(k_cell_sort<2>, dim3(blocks), dim3(256), 0, L.stream, L.n_cells, L.cell_count,
                           L.cell_size, L.cell_idx, L.cell_cap, L.flag);
}

void launch_nlist(const LaunchCtx &L, const double4 *pos, const int32_t *tag, int w, int block)
{
    (void)w;
    (void)block;
    if (L.tiles_local == 0) return;
    const int blocks = capped(L.tiles_local);
    if (L.has_bonds)
        hipLaunchKernelGGL(k_build_tile<true>, dim3(blocks), dim3(kBuildThreads), 0, L.stream, L.sys,
                           L.tprefix_local, L.n_sys, L.tiles_local, pos, tag, L.partners, L.cell_size,
                           L.cell_idx, L.cell_cap, L.nlist, L.nn, L.nlist_cap, L.halo, L.halo_n,
                           L.halo_cap, L.xbuild, L.flag, L.build_count, L.status);
    else
        hipLaunchKernelGGL(k_build_tile<false>, dim3(blocks), dim3(kBuildThreads), 0, L.stream, L.sys,
                           L.tprefix_local, L.n_sys, L.tiles_local, pos, tag, L.partners, L.cell_size,
                           L.cell_idx, L.cell_cap, L.nlist, L.nn, L.nlist_cap, L.halo, L.halo_n,
                           L.halo_cap, L.xbuild, L.flag, L.build_count, L.status);
}

}  // namespace md
