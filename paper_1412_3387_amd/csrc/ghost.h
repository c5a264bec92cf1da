// ghost.h -- ghost-layer selection, packing and unpacking for one subdomain.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace md {

constexpr int kGhostBlock = 256;     // rows per selection block
constexpr int kGhostPerRow = 8;      // stored list entries per local row (7 needed)

struct GhostBuffers {
    uint32_t *mask;       // direction bits per row
    int32_t *blk_counts;  // [26][blocks] entries per direction per block, scanned in place
    int32_t *blk_sums;    // block sums of that scan
    int32_t *list;        // kGhostPerRow slots per row: system s owns [8 row0_s, 8 (row0_s + n_cap_s))
    int32_t *totals;      // entries of the stored list of each system
    int32_t *stay;        // migration: 1 per local row that stays, scanned in place
    int32_t *stay_sums;   // block sums of that scan
    int32_t *counts2;     // migration: {rows leaving, rows staying}
    int64_t rows;
};

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
                  int32_t *tag, double4 *pos_tmp, double4 *vel_tmp, int32_t *tag_tmp);

// Selection + packing with the library's fixed device scratch instead of a
// workspace (no stored list, no status word): rows [0, n_local) of g.pos.
int queue_ghost_select_static(hipStream_t stream, GhostArgs g);
int64_t ghost_static_max_rows();
size_t ghost_static_bytes();

// Bytes of one packed record for a field set.
__host__ __device__ inline int ghost_record_bytes(uint32_t fields)
{
    return 8 * (((fields & 1u) ? 3 : 0) + ((fields & 2u) ? 3 : 0) + ((fields & 4u) ? 1 : 0));
}

}  // namespace md
