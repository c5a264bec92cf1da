// ghost.h -- ghost-layer selection, packing and unpacking for one subdomain.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace md {

constexpr int kGhostBlock = 256;     // rows per selection block
constexpr int kGhostPerRow = 8;      // stored list entries per local row (7 needed)
constexpr uint32_t kFieldBonds = 8u; // record field (migration only): partner tags and owner directions

// Directions between neighbouring subdomains: an offset (dx, dy, dz) with
// components in {-1, 0, 1} has the code (dz+1) 9 + (dy+1) 3 + (dx+1), 13 for
// the subdomain itself; the 26 others are sent in the order of their codes
// (send index = code, less one above 13).
__host__ __device__ inline int dir_code(int dx, int dy, int dz) { return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1); }
__host__ __device__ inline int dir_index(int code) { return code < 13 ? code : code - 1; }
__host__ __device__ inline int dir_of_index(int k) { return k < 13 ? k : k + 1; }
// Code of offset(a) - offset(b), or -1 when a component leaves {-1, 0, 1}
// (or either code is -1).
__host__ __device__ inline int dir_sub(int a, int b)
{
    if (a < 0 || b < 0) return -1;
    const int dx = (a % 3) - (b % 3), dy = (a / 3) % 3 - (b / 3) % 3, dz = a / 9 - b / 9;
    if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) return -1;
    return dir_code(dx, dy, dz);
}

struct GhostBuffers {
    uint32_t *mask;       // direction bits per row
    int32_t *blk_counts;  // [26][blocks] entries per direction per block, scanned in place
    int32_t *blk_sums;    // block sums of that scan
    int32_t *list;        // kGhostPerRow slots per row: system s owns [8 row0_s, 8 (row0_s + n_cap_s))
    int32_t *totals;      // entries of the stored list of each system
    int32_t *stay;        // migration: 1 per local row that stays, scanned in place
    int32_t *stay_sums;   // block sums of that scan
    int32_t *counts2;     // migration: {rows leaving, rows staying}
    int32_t *cursor;      // bond rank messages: 26 direction cursors, then the total
    int64_t rows;
};

// Rank-table messages of one system (Sec. 4.3.4, Fig. 3): mode 0 announces
// the partners of unknown owner to all neighbours, mode 1 tells the owners
// of remote partners where leaving particles go.
struct BondRankArgs {
    double lo[3], hi[3];
    int64_t row0;
    int32_t n_local;
    int32_t mode;
    int32_t stride;
    int32_t bond_cap;
    const double4 *pos;
    const int32_t *tag;
    const int32_t *ptag;
    int32_t *pdir;
    const int32_t *prow;
    void *send;
    int64_t send_cap;
    int32_t *counts;
    int32_t *offsets;
    int32_t *cursor;
    Status *status;
};

struct BondApplyArgs {
    const void *recv;
    int64_t n;
    int64_t row0;
    int32_t n_local;
    int32_t mode;
    int32_t stride;
    int32_t bond_cap;
    const int2 *hash;     // this system's tag -> row table
    int32_t hash_mask;
    const int32_t *ptag;
    int32_t *pdir;
    Status *status;
};

int queue_bond_ranks(hipStream_t stream, const BondRankArgs &a, int32_t *total);
int queue_bond_apply(hipStream_t stream, const BondApplyArgs &a);

struct GhostArgs {
    double lo[3], hi[3], width;
    int64_t row0;
    int32_t n_local;
    uint32_t fields;
    void *send;
    int64_t send_cap;
    int32_t *counts;
    int32_t *offsets;
    const double4 *pos;
    const double4 *vel;
    const int32_t *tag;
    Status *status;
    uint32_t *mask;       // this system's rows of the mask
    int32_t *list;        // this system's stored send list
    int64_t list_cap;
    int32_t *total;       // this system's list length
    // bonded systems: the owner direction of each partner, per row
    // (bond_stride entries; selection adds the directions of the partners
    // that live elsewhere, Sec. 4.3.4) and, for migration records
    // (kFieldBonds), the partner tags
    const int32_t *ptag;
    const int32_t *pdir;
    int32_t bond_stride;
    int32_t bond_cap;
};

struct UnpackArgs {
    double box_L[3];
    double center[3];
    int64_t first;
    int64_t n;
    uint32_t fields;
    const void *recv;
    double4 *pos;
    double4 *vel;
    int32_t *tag;
    int32_t *ptag;        // kFieldBonds: partner tags and owner directions, per row
    int32_t *pdir;
    int32_t bond_stride;
};

size_t ghost_workspace_bytes(int64_t rows, int n_sys);
GhostBuffers make_ghost_buffers(char *base, int64_t rows, int n_sys);
int queue_ghost_select(hipStream_t stream, const GhostBuffers &B, const GhostArgs &g);
int queue_ghost_update(hipStream_t stream, const GhostBuffers &B, const GhostArgs &g);
int queue_ghost_unpack(hipStream_t stream, const UnpackArgs &u);

// Migration of the local rows that left the subdomain [g.lo, g.hi) (Sec.
// 4.3.1): each leaving row goes to the one neighbour its position lies in
// (direction index as for ghosts), packed into g.send ordered by direction
// then row (counts / offsets per direction as for ghosts); the rows that stay
// are compacted in order to the front of the system's rows with the scratch
// arrays pos_tmp / vel_tmp / tag_tmp.  B.counts2 receives {left, stayed}.
int queue_migrate(hipStream_t stream, const GhostBuffers &B, const GhostArgs &g, double4 *pos, double4 *vel,
                  int32_t *tag, double4 *pos_tmp, double4 *vel_tmp, int32_t *tag_tmp, int32_t *ptag,
                  int32_t *pdir, int32_t *ptag_tmp, int32_t *pdir_tmp);

// Selection + packing with the library's fixed device scratch instead of a
// workspace (no stored list, no status word): rows [0, n_local) of g.pos.
int queue_ghost_select_static(hipStream_t stream, GhostArgs g);
int64_t ghost_static_max_rows();
size_t ghost_static_bytes();

// Bytes of one packed record for a field set (kFieldBonds adds the partner
// tags, then the partners' owner directions, bond_stride int32 each).
__host__ __device__ inline int ghost_record_bytes(uint32_t fields, int bond_stride = 0)
{
    return 8 * (((fields & 1u) ? 3 : 0) + ((fields & 2u) ? 3 : 0) + ((fields & 4u) ? 1 : 0)) +
           ((fields & kFieldBonds) ? 8 * bond_stride : 0);
}

}  // namespace md
