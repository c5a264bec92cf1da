// bonds.hip -- bonded groups across subdomains (Sec. 4.3.4, Fig. 3).
//
// A bond is kept with each of its member particles: every row carries the
// tags of its partners (bond_stride slots), so a bond that a migration
// splits is held by both subdomains and leaves a subdomain with its last
// local member.  Beside each partner tag the row keeps the direction of the
// subdomain that owns the partner (13: this one), the rank table of Fig. 3:
//   * at the start every subdomain sends, for each partner it does not own,
//     "your particle b has its partner a at my place" to all 26 neighbours;
//     the neighbour that owns b records the direction it came from;
//   * at a migration, before the particles move, every leaving particle tells
//     the owner of each remote partner where it goes (a local partner finds
//     out from the leaver's position itself), and the partner directions a
//     migrating row carries are made relative to its new owner;
//   * ghost selection sends each particle, besides the layer rule, to every
//     neighbour that owns one of its partners, so a bond of any length up to
//     the neighbour distance finds its partner as a local particle or ghost.
// The force pass reads partners through a per-row table of partner rows,
// filled from a per-system tag -> row hash table whenever rows change.
#include "device.h"
#include "ghost.h"
#include "launch.h"

namespace md {

namespace {

__device__ __forceinline__ uint32_t hash_start(int32_t key, int32_t mask)
{
    return ((uint32_t)key * 2654435761u) & (uint32_t)mask;
}

// Row of tag `key` in the system's table, or -1.
__device__ __forceinline__ int32_t hash_find(const int2 *__restrict__ h, int32_t mask, int32_t key)
{
    for (uint32_t p = hash_start(key, mask);; p = (p + 1) & (uint32_t)mask) {
        const int2 e = h[p];
        if (e.x == key) return e.y;
        if (e.x == -1) return -1;
    }
}

// Direction code of the subdomain a position lies in, seen from [lo, hi).
__device__ __forceinline__ int place_code(const double4 x, const double *lo, const double *hi)
{
    const double xs[3] = {x.x, x.y, x.z};
    int d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = xs[a] >= hi[a] ? 1 : (xs[a] < lo[a] ? -1 : 0);
    return dir_code(d[0], d[1], d[2]);
}

}  // namespace

// ---------------------------------------------------------------------------
// tag -> row tables and partner rows
// ---------------------------------------------------------------------------

__global__ void k_hash_clear(const SysDev *__restrict__ sys, int n_sys, int only, int2 *__restrict__ hash)
{
    const int s0 = only >= 0 ? only : 0, s1 = only >= 0 ? only + 1 : n_sys;
    for (int s = s0; s < s1; ++s) {
        const SysDev &S = sys[s];
        if (S.bond_cap == 0) continue;
        const int64_t n = (int64_t)S.hash_mask + 1;
        for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
            hash[S.hash0 + k] = make_int2(-1, -1);
    }
}

__global__ void k_hash_insert(const SysDev *__restrict__ sys, const int32_t *__restrict__ tprefix, int n_sys,
                              int tiles, int only, const int32_t *__restrict__ tag, int2 *__restrict__ hash)
{
    const int g = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (g >= tiles) return;
    const int s = find_sys(tprefix, n_sys, g);
    if (only >= 0 && s != only) return;
    const SysDev &S = sys[s];
    if (S.bond_cap == 0) return;
    const int r = (g - S.tile0_all) * kTile + lane_id();
    if (r >= S.n_total) return;
    const int64_t i = S.row0 + r;
    const int32_t key = tag[i];
    int2 *h = hash + S.hash0;
    // linear probing; the table has at least twice as many slots as rows
    for (uint32_t p = hash_start(key, S.hash_mask);; p = (p + 1) & (uint32_t)S.hash_mask) {
        const int old = atomicCAS(&h[p].x, -1, key);
        if (old == -1) {
            h[p].y = (int32_t)i;
            break;
        }
        if (old == key) break;  // a tag seen twice keeps its first row
    }
}

__global__ void k_partner_rows(const SysDev *__restrict__ sys, const int32_t *__restrict__ tprefix, int n_sys,
                               int tiles, int only, const int32_t *__restrict__ ptag, const int2 *__restrict__ hash,
                               int32_t *__restrict__ prow)
{
    const int g = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (g >= tiles) return;
    const int s = find_sys(tprefix, n_sys, g);
    if (only >= 0 && s != only) return;
    const SysDev &S = sys[s];
    if (S.bond_cap == 0) return;
    const int r = (g - S.tile0_all) * kTile + lane_id();
    if (r >= S.n_local) return;
    const int64_t i = S.row0 + r;
    for (int b = 0; b < S.bond_stride; ++b) {
        const int32_t t = b < S.bond_cap ? ptag[i * S.bond_stride + b] : -1;
        int32_t j = -1;
        if (t >= 0) {
            j = hash_find(hash + S.hash0, S.hash_mask, t);
            if (j < 0) j = -2;  // not here (yet): the force pass reports it
        }
        prow[i * S.bond_stride + b] = j;
    }
}

void launch_bond_refresh(const LaunchCtx &L, const int32_t *tag, int sys)
{
    if (L.bond_stride == 0 || L.tiles_all == 0) return;
    hipLaunchKernelGGL(k_hash_clear, dim3(256), dim3(256), 0, L.stream, L.sys, L.n_sys, sys, L.hash);
    const int blocks = (L.tiles_all * kWave + 255) / 256;
    hipLaunchKernelGGL(k_hash_insert, dim3(blocks), dim3(256), 0, L.stream, L.sys, L.tprefix_all, L.n_sys,
                       L.tiles_all, sys, tag, L.hash);
    hipLaunchKernelGGL(k_partner_rows, dim3(blocks), dim3(256), 0, L.stream, L.sys, L.tprefix_all, L.n_sys,
                       L.tiles_all, sys, L.ptag, L.hash, L.prow);
}

// ---------------------------------------------------------------------------
// rank-table messages
// ---------------------------------------------------------------------------

// One pass over the local rows of a system: PASS 0 counts the messages per
// direction, PASS 1 writes them (16 bytes each: {tag of the particle whose
// partner entry the receiver updates, tag of that partner, the partner's
// owner direction seen from the receiver, 0}) and, when migrating, updates
// the entries of partners that leave this subdomain.
template <int PASS>
__global__ void k_bond_ranks(BondRankArgs a)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_local) return;
    const int64_t i = a.row0 + r;
    const int32_t me = a.tag[i];
    const int here = a.mode == 1 ? place_code(a.pos[i], a.lo, a.hi) : 13;
    for (int s = 0; s < a.bond_cap; ++s) {
        const int64_t e = i * a.stride + s;
        const int32_t t = a.ptag[e];
        if (t < 0) continue;
        const int d = a.pdir[e];
        if (a.mode == 0) {
            // start: partners of unknown owner are announced to every neighbour
            if (d != -1) continue;
            for (int k = 0; k < 26; ++k) {
                if (PASS == 0) {
                    atomicAdd(&a.cursor[k], 1);
                } else {
                    const int code = dir_of_index(k);
                    const int back = dir_sub(13, code);  // this subdomain, seen from the receiver
                    const int64_t p = atomicAdd(&a.cursor[k], 1);
                    if (p < a.send_cap) reinterpret_cast<int4 *>(a.send)[p] = make_int4(t, me, back, 0);
                }
            }
            continue;
        }
        if (d == -1) {
            if (PASS == 0 && a.status) latch(a.status, 12 /*BOND_GHOST*/, 0);  // rank table never set up
            continue;
        }
        if (d == 13) {
            // a local partner: if it leaves, its entry here follows it
            if (PASS == 1) {
                const int32_t j = a.prow[e];
                if (j >= 0) {
                    const int pj = place_code(a.pos[j], a.lo, a.hi);
                    if (pj != 13) a.pdir[e] = pj;
                }
            }
            continue;
        }
        if (here == 13) continue;  // this particle stays: its remote partners' tables hold
        // this particle leaves: the owner of the partner (direction d) learns
        // where it goes, seen from there
        const int code = dir_sub(here, d);
        if (code < 0) {
            if (PASS == 0 && a.status) latch(a.status, 12 /*BOND_GHOST*/, 0);  // beyond the neighbours
            continue;
        }
        const int k = dir_index(d);
        if (PASS == 0) {
            atomicAdd(&a.cursor[k], 1);
        } else {
            const int64_t p = atomicAdd(&a.cursor[k], 1);
            if (p < a.send_cap) reinterpret_cast<int4 *>(a.send)[p] = make_int4(t, me, code, 0);
        }
    }
}

// Counts -> offsets (exclusive, in direction order); the cursors restart at
// the offsets for the writing pass; the total goes to *total.
__global__ void k_bond_offsets(BondRankArgs a, int32_t *total)
{
    if (threadIdx.x != 0) return;
    int32_t run = 0;
    for (int k = 0; k < 26; ++k) {
        const int32_t c = a.cursor[k];
        a.counts[k] = c;
        a.offsets[k] = run;
        a.cursor[k] = run;
        run += c;
    }
    *total = run;
    if (a.status && (int64_t)run > a.send_cap) latch(a.status, 7 /*GHOST_OVERFLOW*/, run);
}

__global__ void k_bond_cursor_clear(int32_t *cursor)
{
    if (threadIdx.x < 26) cursor[threadIdx.x] = 0;
}

// Received messages: the local particle with the record's first tag sets the
// owner direction of its partner with the second tag.
__global__ void k_bond_apply(BondApplyArgs a)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const int4 m = reinterpret_cast<const int4 *>(a.recv)[k];
    const int32_t i = hash_find(a.hash, a.hash_mask, m.x);
    const bool local = i >= 0 && i - a.row0 < a.n_local;
    bool done = false;
    if (local)
        for (int s = 0; s < a.bond_cap; ++s)
            if (a.ptag[(int64_t)i * a.stride + s] == m.y) {
                a.pdir[(int64_t)i * a.stride + s] = m.z;
                done = true;
            }
    // at the start every neighbour hears the announcement; only the owner acts
    if (!done && a.mode == 1 && a.status) latch(a.status, 12 /*BOND_GHOST*/, 0);
}

int queue_bond_ranks(hipStream_t stream, const BondRankArgs &a, int32_t *total)
{
    const int blocks = a.n_local > 0 ? (a.n_local + 255) / 256 : 1;
    hipLaunchKernelGGL(k_bond_cursor_clear, dim3(1), dim3(64), 0, stream, a.cursor);
    hipLaunchKernelGGL(k_bond_ranks<0>, dim3(blocks), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_bond_offsets, dim3(1), dim3(64), 0, stream, a, total);
    hipLaunchKernelGGL(k_bond_ranks<1>, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

int queue_bond_apply(hipStream_t stream, const BondApplyArgs &a)
{
    if (a.n <= 0) return 0;
    const int blocks = (int)((a.n + 255) / 256);
    hipLaunchKernelGGL(k_bond_apply, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // namespace md
