// nlist.hip -- cell list and Verlet neighbour list (Sec. 5.1, Fig. 4).
//
// Cell list: fixed-capacity bins.  A binning pass assigns every row to the
// cell floor((x - lo) * bins / L) with an integer atomic slot; a per-cell
// pass then sorts the members of each cell by row index (rank sort inside
// one wave), so the list is deterministic although the slots were claimed
// in arbitrary order.  The per-cell pass also resets the atomic counters for
// the next build, so no memset is needed between builds.
//
// Neighbour list: W lanes cooperate on one particle (lane = s * P + pl, P =
// 64 / W particles per wave).  The W lanes stride over the members of each
// stencil cell, test |x_j - x_i|^2 < r_list^2 in FP64, and compact the hits
// into the particle's row with one 64-bit ballot: the write position is the
// running count plus the number of hits of the same particle on lower lanes.
// Rows are stored tile-major: entry k of row r of a system lives at
// nl0 + (r / 64) * cap * 64 + k * 64 + r % 64, so a wave that reads entry k
// of 64/W consecutive particles touches consecutive words.
#include "device.h"
#include "launch.h"

namespace md {

// All kernels below return at once unless the rebuild flag is set, so the
// whole rebuild sequence can be queued every step without a host round trip.

__global__ void k_bin(const SysDev *__restrict__ sys, const int32_t *__restrict__ tprefix,
                      int n_sys, int tiles, const double4 *__restrict__ pos,
                      int32_t *__restrict__ cell_count, int32_t *__restrict__ cell_idx,
                      int cell_cap, const int32_t *__restrict__ flag, Status *st)
{
    if (*flag == 0) return;
    const int g = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (g >= tiles) return;
    const int s = find_sys(tprefix, n_sys, g);
    const SysDev &S = sys[s];
    const int r = (g - S.tile0_all) * kTile + lane_id();
    if (r >= S.n_total) return;
    const int64_t i = S.row0 + r;
    const double4 x = pos[i];
    const int cx = cell_coord(x.x, S.lo[0], S.scale[0], S.bins[0]);
    const int cy = cell_coord(x.y, S.lo[1], S.scale[1], S.bins[1]);
    const int cz = cell_coord(x.z, S.lo[2], S.scale[2], S.bins[2]);
    const int64_t c = S.cell0 + ((int64_t)cz * S.bins[1] + cy) * S.bins[0] + cx;
    const int slot = atomicAdd(&cell_count[c], 1);
    if (slot < cell_cap) cell_idx[c * cell_cap + slot] = (int32_t)i;
    else latch(st, 6 /*CELL_OVERFLOW*/, slot + 1);
}

// One wave per cell: members ranked by row index, sizes published, counters
// cleared.  cell_cap <= 64 * CPL.
template <int CPL>
__global__ void k_cell_sort(int64_t n_cells, int32_t *__restrict__ cell_count,
                            int32_t *__restrict__ cell_size, int32_t *__restrict__ cell_idx,
                            int cell_cap, const int32_t *__restrict__ flag)
{
    if (*flag == 0) return;
    const int64_t c = (int64_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (c >= n_cells) return;
    const int lane = lane_id();
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
    for (int t = 0; t < m; ++t) {
        const int32_t other = __shfl(v[t / kWave], t % kWave, kWave);
#pragma unroll
        for (int q = 0; q < CPL; ++q) rank[q] += other < v[q] ? 1 : 0;
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

template <int W, bool EXCL>
__global__ void k_nlist(const SysDev *__restrict__ sys, const int32_t *__restrict__ tprefix,
                        int n_sys, int tiles, const double4 *__restrict__ pos,
                        const int32_t *__restrict__ tag, const int32_t *__restrict__ partners,
                        const int32_t *__restrict__ cell_size, const int32_t *__restrict__ cell_idx,
                        int cell_cap, int32_t *__restrict__ nlist, int32_t *__restrict__ nn,
                        int cap, double4 *__restrict__ xbuild, const int32_t *__restrict__ flag,
                        int32_t *build_count, Status *st)
{
    if (*flag == 0) return;
    constexpr int P = kWave / W;
    const int lane = lane_id();
    const int pl = lane % P;
    const int sl = lane / P;
    const int gw = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int tile = gw / W;
    if (tile >= tiles) return;
    if (gw == 0 && lane == 0) atomicAdd(build_count, 1);
    const int s = find_sys(tprefix, n_sys, tile);
    const SysDev &S = sys[s];
    const int r = (tile - S.tile0) * kTile + (gw % W) * P + pl;
    const bool active = r < S.n_local;
    const int64_t i = S.row0 + (active ? r : 0);
    const double4 xi = pos[i];
    const int cx = cell_coord(xi.x, S.lo[0], S.scale[0], S.bins[0]);
    const int cy = cell_coord(xi.y, S.lo[1], S.scale[1], S.bins[1]);
    const int cz = cell_coord(xi.z, S.lo[2], S.scale[2], S.bins[2]);

    int32_t part[kMaxBondCap];
    if constexpr (EXCL) {
#pragma unroll
        for (int b = 0; b < kMaxBondCap; ++b) part[b] = -1;
        if (active) {
            const int64_t prow = (S.row0 + tag[i]) * S.bond_cap;
            for (int b = 0; b < S.bond_cap && b < kMaxBondCap; ++b) part[b] = partners[prow + b];
        }
    }

    const uint64_t seg = segment_bits(pl, P);
    const uint64_t below = lanemask_lt();
    const int64_t rowbase = S.nl0 + (int64_t)(r >> 6) * cap * kTile + (r & 63);
    const double rl2 = S.rl2;
    int ntot = 0;
    if (active) {
        for (int a = 0; a < S.nst[2]; ++a) {
            int z = cz + S.st[2][a];
            if (S.per[2]) z = z < 0 ? z + S.bins[2] : (z >= S.bins[2] ? z - S.bins[2] : z);
            else if (z < 0 || z >= S.bins[2]) continue;
            for (int b = 0; b < S.nst[1]; ++b) {
                int y = cy + S.st[1][b];
                if (S.per[1]) y = y < 0 ? y + S.bins[1] : (y >= S.bins[1] ? y - S.bins[1] : y);
                else if (y < 0 || y >= S.bins[1]) continue;
                for (int e = 0; e < S.nst[0]; ++e) {
                    int x = cx + S.st[0][e];
                    if (S.per[0]) x = x < 0 ? x + S.bins[0] : (x >= S.bins[0] ? x - S.bins[0] : x);
                    else if (x < 0 || x >= S.bins[0]) continue;
                    const int64_t c = S.cell0 + ((int64_t)z * S.bins[1] + y) * S.bins[0] + x;
                    const int m = cell_size[c];
                    const int32_t *members = cell_idx + c * cell_cap;
                    for (int k0 = 0; k0 < m; k0 += W) {
                        const int k = k0 + sl;
                        bool hit = false;
                        int32_t j = 0;
                        if (k < m) {
                            j = members[k];
                            if (j != (int32_t)i) {
                                const double4 xj = pos[j];
                                const double dx = min_image(xj.x - xi.x, S.L[0], S.invL[0]);
                                const double dy = min_image(xj.y - xi.y, S.L[1], S.invL[1]);
                                const double dz = min_image(xj.z - xi.z, S.L[2], S.invL[2]);
                                hit = norm2_exact(dx, dy, dz) < rl2;
                                if constexpr (EXCL) {
                                    if (hit) {
                                        const int32_t tj = tag[j];
#pragma unroll
                                        for (int q = 0; q < kMaxBondCap; ++q) hit = hit && (part[q] != tj);
                                    }
                                }
                            }
                        }
                        const uint64_t mask = __ballot(hit) & seg;
                        if (hit) {
                            const int p = ntot + __popcll(mask & below);
                            if (p < cap) nlist[rowbase + (int64_t)p * kTile] = j;
                        }
                        ntot += __popcll(mask);
                    }
                }
            }
        }
        if (sl == 0) {
            nn[i] = ntot < cap ? ntot : cap;
            xbuild[i] = xi;
            if (ntot > cap) latch(st, 5 /*NLIST_OVERFLOW*/, ntot);
        }
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

void launch_bin(const LaunchCtx &L, const double4 *pos)
{
    const int threads = 256;
    const int blocks = (L.tiles_all * kWave + threads - 1) / threads;
    if (blocks == 0) return;
    hipLaunchKernelGGL(k_bin, dim3(blocks), dim3(threads), 0, L.stream, L.sys, L.tprefix_all,
                       L.n_sys, L.tiles_all, pos, L.cell_count, L.cell_idx, L.cell_cap, L.flag,
                       L.status);
}

void launch_cell_sort(const LaunchCtx &L)
{
    const int threads = 256;
    const int64_t blocks = (L.n_cells * kWave + threads - 1) / threads;
    if (blocks == 0) return;
    if (L.cell_cap <= 64)
        hipLaunchKernelGGL(k_cell_sort<1>, dim3((unsigned)blocks), dim3(threads), 0, L.stream,
                           L.n_cells, L.cell_count, L.cell_size, L.cell_idx, L.cell_cap, L.flag);
    else
        hipLaunchKernelGGL(k_cell_sort<2>, dim3((unsigned)blocks), dim3(threads), 0, L.stream,
                           L.n_cells, L.cell_count, L.cell_size, L.cell_idx, L.cell_cap, L.flag);
}

template <int W, bool EXCL>
static void nlist_w(const LaunchCtx &L, const double4 *pos, const int32_t *tag, int block)
{
    const int64_t threads_total = (int64_t)L.tiles_local * W * kWave;
    const int blocks = (int)((threads_total + block - 1) / block);
    if (blocks == 0) return;
    hipLaunchKernelGGL((k_nlist<W, EXCL>), dim3(blocks), dim3(block), 0, L.stream, L.sys,
                       L.tprefix_local, L.n_sys, L.tiles_local, pos, tag, L.partners,
                       L.cell_size, L.cell_idx, L.cell_cap, L.nlist, L.nn, L.nlist_cap,
                       L.xbuild, L.flag, L.build_count, L.status);
}

template <bool EXCL>
static void nlist_excl(const LaunchCtx &L, const double4 *pos, const int32_t *tag, int w, int block)
{
    switch (w) {
    case 1: nlist_w<1, EXCL>(L, pos, tag, block); break;
    case 2: nlist_w<2, EXCL>(L, pos, tag, block); break;
    case 4: nlist_w<4, EXCL>(L, pos, tag, block); break;
    case 8: nlist_w<8, EXCL>(L, pos, tag, block); break;
    case 16: nlist_w<16, EXCL>(L, pos, tag, block); break;
    case 32: nlist_w<32, EXCL>(L, pos, tag, block); break;
    default: nlist_w<64, EXCL>(L, pos, tag, block); break;
    }
}

void launch_nlist(const LaunchCtx &L, const double4 *pos, const int32_t *tag, int w, int block)
{
    if (L.has_bonds) nlist_excl<true>(L, pos, tag, w, block);
    else nlist_excl<false>(L, pos, tag, w, block);
}

}  // namespace md
