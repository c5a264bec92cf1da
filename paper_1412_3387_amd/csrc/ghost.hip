// ghost.hip -- ghost-layer exchange of one subdomain (Sec. 4.3.2, Fig. 2).
//
// The paper marks a per-particle bitfield of destinations, expands (index,
// destination) pairs with a load-balancing search, merge-sorts them by
// destination and finds segment bounds by binary search.  With at most 26
// destinations the same ordered list falls out of a counting sort: one pass
// builds the 26-bit mask of every local particle and counts, per block and
// direction, how many go each way (one ballot per direction and wave); a scan
// of the direction-major count table gives every (direction, block) its
// first slot; a second pass places each entry at that slot plus its rank
// among the same-direction entries of lower rows (ballot prefix counts) and
// gathers the requested fields into the send record at once.  The result is
// ordered by direction, then by ascending row, with no atomics.
#include "ghost.h"
#include "sort.h"

#include <mutex>

namespace md {

static size_t a256(size_t x) { return (x + 255) / 256 * 256; }

size_t ghost_workspace_bytes(int64_t rows, int n_sys)
{
    const int64_t blocks = (rows + kGhostBlock - 1) / kGhostBlock;
    return a256(sizeof(uint32_t) * rows) + a256(sizeof(int32_t) * 26 * (size_t)blocks) +
           a256(sizeof(int32_t) * scan_sums_len(26 * blocks)) +
           a256(sizeof(int32_t) * kGhostPerRow * (size_t)rows) + a256(sizeof(int32_t) * n_sys) +
           a256(sizeof(int32_t) * rows) + a256(sizeof(int32_t) * scan_sums_len(rows)) + a256(sizeof(int32_t) * 2) +
           a256(sizeof(int32_t) * 32) + 256;
}

GhostBuffers make_ghost_buffers(char *base, int64_t rows, int n_sys)
{
    GhostBuffers B{};
    const int64_t blocks = (rows + kGhostBlock - 1) / kGhostBlock;
    size_t off = 0;
    B.mask = reinterpret_cast<uint32_t *>(base + off); off += a256(sizeof(uint32_t) * rows);
    B.blk_counts = reinterpret_cast<int32_t *>(base + off); off += a256(sizeof(int32_t) * 26 * (size_t)blocks);
    B.blk_sums = reinterpret_cast<int32_t *>(base + off); off += a256(sizeof(int32_t) * scan_sums_len(26 * blocks));
    B.list = reinterpret_cast<int32_t *>(base + off); off += a256(sizeof(int32_t) * kGhostPerRow * (size_t)rows);
    B.totals = reinterpret_cast<int32_t *>(base + off); off += a256(sizeof(int32_t) * n_sys);
    B.stay = reinterpret_cast<int32_t *>(base + off); off += a256(sizeof(int32_t) * rows);
    B.stay_sums = reinterpret_cast<int32_t *>(base + off); off += a256(sizeof(int32_t) * scan_sums_len(rows));
    B.counts2 = reinterpret_cast<int32_t *>(base + off); off += a256(sizeof(int32_t) * 2);
    B.cursor = reinterpret_cast<int32_t *>(base + off);
    B.rows = rows;
    return B;
}

__device__ __forceinline__ uint32_t ghost_mask(const double4 x, const GhostArgs &g)
{
    const double xs[3] = {x.x, x.y, x.z};
    uint32_t up = 0, dn = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        up |= (xs[a] >= g.hi[a] - g.width ? 1u : 0u) << a;
        dn |= (xs[a] < g.lo[a] + g.width ? 1u : 0u) << a;
    }
    uint32_t m = 0;
    int bit = 0;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                const int d[3] = {dx, dy, dz};
                bool ok = true;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (d[a] == 1) ok = ok && ((up >> a) & 1u);
                    if (d[a] == -1) ok = ok && ((dn >> a) & 1u);
                }
                m |= (ok ? 1u : 0u) << bit;
                ++bit;
            }
    return m;
}

// Record k of the send buffer from row `row`, sent in direction `code`.
__device__ __forceinline__ void pack_record(const GhostArgs &g, int64_t k, int64_t row, int code)
{
    double *rec = reinterpret_cast<double *>(static_cast<char *>(g.send) +
                                             k * ghost_record_bytes(g.fields, g.bond_stride));
    int q = 0;
    if (g.fields & 1u) {
        const double4 x = g.pos[row];
        rec[q++] = x.x;
        rec[q++] = x.y;
        rec[q++] = x.z;
    }
    if (g.fields & 2u) {
        const double4 v = g.vel[row];
        rec[q++] = v.x;
        rec[q++] = v.y;
        rec[q++] = v.z;
    }
    if (g.fields & 4u) {
        int32_t *t = reinterpret_cast<int32_t *>(rec + q);
        t[0] = g.tag[row];
        t[1] = 0;
        ++q;
    }
    if (g.fields & kFieldBonds) {
        // a migrating row takes its partners along; their owners' directions
        // become relative to the receiver (one step `code` away)
        int32_t *b = reinterpret_cast<int32_t *>(rec + q);
        for (int s = 0; s < g.bond_stride; ++s) {
            const int32_t t = g.ptag[row * g.bond_stride + s];
            int32_t d = -1;
            if (t >= 0) {
                d = dir_sub(g.pdir[row * g.bond_stride + s], code);
                if (d < 0 && g.status) latch(g.status, 12 /*BOND_GHOST*/, 0);
            }
            b[s] = t;
            b[g.bond_stride + s] = d;
        }
    }
}

// Directions of the partners of row `row` that live in other subdomains, as
// send bits (Sec. 4.3.4: a particle goes as a ghost wherever a bond partner
// is owned).
__device__ __forceinline__ uint32_t bond_dir_mask(const GhostArgs &g, int64_t row)
{
    uint32_t m = 0;
    for (int s = 0; s < g.bond_cap; ++s) {
        const int32_t d = g.pdir[row * g.bond_stride + s];
        if (d >= 0 && d != 13 && g.ptag[row * g.bond_stride + s] >= 0) m |= 1u << dir_index(d);
    }
    return m;
}

// Per-wave, per-direction counts into LDS: wc[wave][d].
__device__ __forceinline__ void wave_dir_counts(uint32_t m, int32_t (*wc)[26])
{
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    for (int d = 0; d < 26; ++d) {
        const uint64_t b = __ballot((m >> d) & 1u);
        if (lane == d) wc[w][d] = __popcll(b);
    }
}

__global__ __launch_bounds__(kGhostBlock) void k_ghost_mask(GhostArgs g, int32_t *__restrict__ blk_counts,
                                                           int nblocks)
{
    __shared__ int32_t wc[kGhostBlock / 64][26];
    const int r = blockIdx.x * kGhostBlock + threadIdx.x;
    uint32_t m = 0;
    if (r < g.n_local) {
        m = ghost_mask(g.pos[g.row0 + r], g);
        if (g.pdir) m |= bond_dir_mask(g, g.row0 + r);
        g.mask[r] = m;
    }
    wave_dir_counts(m, wc);
    __syncthreads();
    if (threadIdx.x < 26) {
        int32_t t = 0;
        for (int w = 0; w < kGhostBlock / 64; ++w) t += wc[w][threadIdx.x];
        blk_counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = t;
    }
}

__global__ void k_ghost_totals(const int32_t *__restrict__ scanned, const int32_t *__restrict__ total,
                               int nblocks, int32_t *__restrict__ counts, int32_t *__restrict__ offsets,
                               int64_t send_cap, int64_t list_cap, Status *st)
{
    const int d = threadIdx.x;
    if (d < 26) {
        const int32_t a = scanned[(int64_t)d * nblocks];
        const int32_t b = d < 25 ? scanned[(int64_t)(d + 1) * nblocks] : *total;
        offsets[d] = a;
        counts[d] = b - a;
    }
    if (st && d == 0 && ((int64_t)*total > send_cap || (int64_t)*total > list_cap))
        latch(st, 7 /*GHOST_OVERFLOW*/, *total);
}

__global__ __launch_bounds__(kGhostBlock) void k_ghost_scatter(GhostArgs g, const int32_t *__restrict__ scanned,
                                                              int nblocks)
{
    __shared__ int32_t wc[kGhostBlock / 64][26];
    const int r = blockIdx.x * kGhostBlock + threadIdx.x;
    const uint32_t m = r < g.n_local ? g.mask[r] : 0u;
    wave_dir_counts(m, wc);
    __syncthreads();
    const int w = threadIdx.x >> 6;
    const uint64_t lt = lanemask_lt();
    for (int d = 0; d < 26; ++d) {
        const bool sel = (m >> d) & 1u;
        const uint64_t b = __ballot(sel);
        if (!sel) continue;
        int64_t p = scanned[(int64_t)d * nblocks + blockIdx.x] + __popcll(b & lt);
        for (int v = 0; v < w; ++v) p += wc[v][d];
        if (g.list && p < g.list_cap) g.list[p] = r;
        if (p < g.send_cap) pack_record(g, p, g.row0 + r, dir_of_index(d));
    }
}

__global__ void k_ghost_regather(GhostArgs g)
{
    int64_t n = *g.total;
    n = n < g.list_cap ? n : g.list_cap;
    n = n < g.send_cap ? n : g.send_cap;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        pack_record(g, k, g.row0 + g.list[k], 13);
}

__global__ void k_ghost_unpack(UnpackArgs u)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= u.n) return;
    const double *rec = reinterpret_cast<const double *>(static_cast<const char *>(u.recv) +
                                                         k * ghost_record_bytes(u.fields, u.bond_stride));
    const int64_t row = u.first + k;
    int q = 0;
    if (u.fields & 1u) {
        double x[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double v = rec[q++];
            x[a] = v - u.box_L[a] * rint((v - u.center[a]) / u.box_L[a]);
        }
        u.pos[row] = make_double4(x[0], x[1], x[2], 0.0);
    }
    if (u.fields & 2u) {
        u.vel[row] = make_double4(rec[q], rec[q + 1], rec[q + 2], 0.0);
        q += 3;
    }
    if (u.fields & 4u) {
        u.tag[row] = reinterpret_cast<const int32_t *>(rec + q)[0];
        ++q;
    }
    if (u.fields & kFieldBonds) {
        const int32_t *b = reinterpret_cast<const int32_t *>(rec + q);
        for (int s = 0; s < u.bond_stride; ++s) {
            u.ptag[row * u.bond_stride + s] = b[s];
            u.pdir[row * u.bond_stride + s] = b[u.bond_stride + s];
        }
    }
}

// Destination of a local row after a drift: per axis +1 at or beyond hi, -1
// below lo, else 0; the direction's bit (index as for ghosts), or 0 when the
// row stays.
__device__ __forceinline__ uint32_t leave_mask(const double4 x, const GhostArgs &g)
{
    const double xs[3] = {x.x, x.y, x.z};
    int d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = xs[a] >= g.hi[a] ? 1 : (xs[a] < g.lo[a] ? -1 : 0);
    if (d[0] == 0 && d[1] == 0 && d[2] == 0) return 0u;
    int k = (d[2] + 1) * 9 + (d[1] + 1) * 3 + (d[0] + 1);
    k = k < 13 ? k : k - 1;
    return 1u << k;
}

__global__ __launch_bounds__(kGhostBlock) void k_migrate_mask(GhostArgs g, int32_t *__restrict__ blk_counts,
                                                             int nblocks, int32_t *__restrict__ stay)
{
    __shared__ int32_t wc[kGhostBlock / 64][26];
    const int r = blockIdx.x * kGhostBlock + threadIdx.x;
    uint32_t m = 0;
    if (r < g.n_local) {
        m = leave_mask(g.pos[g.row0 + r], g);
        g.mask[r] = m;
        stay[r] = m == 0u ? 1 : 0;
    }
    wave_dir_counts(m, wc);
    __syncthreads();
    if (threadIdx.x < 26) {
        int32_t t = 0;
        for (int w = 0; w < kGhostBlock / 64; ++w) t += wc[w][threadIdx.x];
        blk_counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = t;
    }
}

// Rows that stay, in order, to the front (through the scratch arrays).
__global__ void k_migrate_compact(int64_t row0, int n_local, const int32_t *__restrict__ mask,
                                  const int32_t *__restrict__ dst, const double4 *__restrict__ pos,
                                  const double4 *__restrict__ vel, const int32_t *__restrict__ tag,
                                  double4 *__restrict__ pos_tmp, double4 *__restrict__ vel_tmp,
                                  int32_t *__restrict__ tag_tmp, const int32_t *__restrict__ ptag,
                                  const int32_t *__restrict__ pdir, int32_t *__restrict__ ptag_tmp,
                                  int32_t *__restrict__ pdir_tmp, int stride)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_local || mask[r] != 0) return;
    const int64_t d = row0 + dst[r];
    pos_tmp[d] = pos[row0 + r];
    vel_tmp[d] = vel[row0 + r];
    tag_tmp[d] = tag[row0 + r];
    for (int s = 0; s < stride; ++s) {
        ptag_tmp[d * stride + s] = ptag[(row0 + r) * stride + s];
        pdir_tmp[d * stride + s] = pdir[(row0 + r) * stride + s];
    }
}

__global__ void k_migrate_counts(const int32_t *__restrict__ left, int32_t *__restrict__ counts2, int any_local)
{
    counts2[0] = *left;
    if (!any_local) counts2[1] = 0;
}

int queue_ghost_select(hipStream_t stream, const GhostBuffers &B, const GhostArgs &g)
{
    const int nblocks = (g.n_local + kGhostBlock - 1) / kGhostBlock;
    const int nb = nblocks > 0 ? nblocks : 1;
    hipLaunchKernelGGL(k_ghost_mask, dim3(nb), dim3(kGhostBlock), 0, stream, g, B.blk_counts, nb);
    launch_scan(stream, B.blk_counts, B.blk_counts, 26 * (int64_t)nb, g.total, B.blk_sums);
    // without a stored list (list == nullptr) only the send buffer bounds the total
    const int64_t list_cap = g.list ? g.list_cap : INT64_MAX;
    hipLaunchKernelGGL(k_ghost_totals, dim3(1), dim3(64), 0, stream, B.blk_counts, g.total, nb, g.counts,
                       g.offsets, g.send_cap, list_cap, g.status);
    hipLaunchKernelGGL(k_ghost_scatter, dim3(nb), dim3(kGhostBlock), 0, stream, g, B.blk_counts, nb);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

int queue_migrate(hipStream_t stream, const GhostBuffers &B, const GhostArgs &g, double4 *pos, double4 *vel,
                  int32_t *tag, double4 *pos_tmp, double4 *vel_tmp, int32_t *tag_tmp, int32_t *ptag,
                  int32_t *pdir, int32_t *ptag_tmp, int32_t *pdir_tmp)
{
    const int nblocks = (g.n_local + kGhostBlock - 1) / kGhostBlock;
    const int nb = nblocks > 0 ? nblocks : 1;
    // leaving rows: direction masks and counts, the ordered send records
    hipLaunchKernelGGL(k_migrate_mask, dim3(nb), dim3(kGhostBlock), 0, stream, g, B.blk_counts, nb, B.stay);
    launch_scan(stream, B.blk_counts, B.blk_counts, 26 * (int64_t)nb, g.total, B.blk_sums);
    const int64_t list_cap = g.list ? g.list_cap : INT64_MAX;
    hipLaunchKernelGGL(k_ghost_totals, dim3(1), dim3(64), 0, stream, B.blk_counts, g.total, nb, g.counts,
                       g.offsets, g.send_cap, list_cap, g.status);
    hipLaunchKernelGGL(k_ghost_scatter, dim3(nb), dim3(kGhostBlock), 0, stream, g, B.blk_counts, nb);
    // staying rows: their new places (the scan's total is the count that
    // stays), then the compacted copy into the scratch arrays
    if (g.n_local > 0) {
        launch_scan(stream, B.stay, B.stay, g.n_local, B.counts2 + 1, B.stay_sums);
        const int blocks = (g.n_local + 255) / 256;
        hipLaunchKernelGGL(k_migrate_compact, dim3(blocks), dim3(256), 0, stream, g.row0, g.n_local,
                           reinterpret_cast<const int32_t *>(g.mask), B.stay, pos, vel, tag, pos_tmp, vel_tmp,
                           tag_tmp, ptag, pdir, ptag_tmp, pdir_tmp, ptag ? g.bond_stride : 0);
    }
    hipLaunchKernelGGL(k_migrate_counts, dim3(1), dim3(1), 0, stream, g.total, B.counts2, g.n_local > 0 ? 1 : 0);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

int queue_ghost_update(hipStream_t stream, const GhostBuffers &B, const GhostArgs &g)
{
    (void)B;
    hipLaunchKernelGGL(k_ghost_regather, dim3(256), dim3(256), 0, stream, g);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

int queue_ghost_unpack(hipStream_t stream, const UnpackArgs &u)
{
    if (u.n <= 0) return 0;
    const int blocks = (int)((u.n + 255) / 256);
    hipLaunchKernelGGL(k_ghost_unpack, dim3(blocks), dim3(256), 0, stream, u);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // namespace md

// ---------------------------------------------------------------------------
// Ghost selection and packing without a caller workspace (for callers that
// cannot allocate device memory).  The per-row direction masks, the
// direction-by-block count table, the scan's block sums and the list total
// live in one file-scope device array of fixed size.  Host code never uses
// the array's name as an address: at the first call on a device (that device
// current) its device address is looked up once with hipGetSymbolAddress and
// kept per device, and only that address is handed to the kernels.
// ---------------------------------------------------------------------------

namespace md {
namespace {

constexpr int64_t kStaticRows = (int64_t)1 << 21;  // locals per call at most
constexpr int64_t kStaticBlocks = kStaticRows / kGhostBlock;
constexpr size_t up256(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t kStaticTotalOff = 0;                  // int32 list total
constexpr size_t kStaticMaskOff = 256;                 // uint32 per row
constexpr size_t kStaticCountsOff = kStaticMaskOff + up256(sizeof(uint32_t) * kStaticRows);
constexpr size_t kStaticSumsOff = kStaticCountsOff + up256(sizeof(int32_t) * 26 * kStaticBlocks);
constexpr size_t kStaticBytes =
    kStaticSumsOff + up256(sizeof(int32_t) * (size_t)((26 * kStaticBlocks + kScanTile - 1) / kScanTile + 1));
static_assert(kStaticRows % kGhostBlock == 0, "whole selection blocks");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_dev[kMaxDevices];  // device address of `scratch` per device (nullptr: not looked up)

}  // namespace

}  // namespace md

static __device__ __align__(256) char scratch[md::kStaticBytes];

namespace md {

// Device address of the array on the current device (looked up once).
static hipError_t static_scratch(char **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

int64_t ghost_static_max_rows() { return kStaticRows; }
size_t ghost_static_bytes() { return kStaticBytes; }

// Queue selection + packing of rows [0, n_local) on `stream` with the
// static scratch.  Returns 0, 1 on a launch error, 2 when the scratch
// address cannot be found.
int queue_ghost_select_static(hipStream_t stream, GhostArgs g)
{
    char *base = nullptr;
    if (static_scratch(&base) != hipSuccess) return 2;
    GhostBuffers B{};
    B.mask = reinterpret_cast<uint32_t *>(base + kStaticMaskOff);
    B.blk_counts = reinterpret_cast<int32_t *>(base + kStaticCountsOff);
    B.blk_sums = reinterpret_cast<int32_t *>(base + kStaticSumsOff);
    B.list = nullptr;
    B.totals = reinterpret_cast<int32_t *>(base + kStaticTotalOff);
    B.rows = kStaticRows;
    g.mask = B.mask;
    g.list = nullptr;
    g.list_cap = 0;
    g.total = B.totals;
    g.status = nullptr;
    return queue_ghost_select(stream, B, g);
}

}  // namespace md
