// sort.h -- spatial (Morton) reordering of the particle rows and the
// device-wide exclusive scan shared with the ghost kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.h"

namespace md {

struct SortBuffers {
    uint64_t *keys[2];
    int32_t *vals[2];
    int32_t *hist;      // 256 digit counts per tile
    int32_t *hist_sums; // block sums of the histogram scan
    int32_t *tag_tmp;
    int64_t rows;
    int64_t tiles;      // radix tiles of kRadixTile rows
};

constexpr int kRadixTile = 1024;

size_t sort_workspace_bytes(int64_t rows);
SortBuffers make_sort_buffers(char *base, int64_t rows);

// Permute pos, vel and tag of every system by the stable order of the keys
// (system index << 30 | 30-bit Morton key of the position); rows beyond
// n_local keep their places at the end of their system.  pos_tmp / vel_tmp
// are scratch of the same size.  Queued on L.stream.
int queue_morton_sort(const LaunchCtx &L, const SortBuffers &B, double4 *pos, double4 *vel,
                      int32_t *tag, double4 *pos_tmp, double4 *vel_tmp);

// Keys only (for inspection): keys[row] = (system << 30) | morton.
void launch_morton_keys(const LaunchCtx &L, const double4 *pos, uint64_t *keys, int32_t *vals);

// Exclusive scan of n int32 values; out may alias in.  If total != nullptr
// the sum is written there.  Two levels: the sums of blocks of kScanTile
// values (in sums, scan_sums_len(n) entries), their scan in one workgroup,
// then every block's scan offset by its prefix.
constexpr int kScanTile = 4096;
inline int64_t scan_sums_len(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }
void launch_scan(hipStream_t stream, const int32_t *in, int32_t *out, int64_t n, int32_t *total,
                 int32_t *sums);

}  // namespace md
