// sort.hip -- Morton order of the particle rows (keeps spatial neighbours
// close in memory so neighbour gathers hit the caches).  Keys are 30-bit
// Morton codes (10 bits per axis) prefixed by the system index; a stable
// least-significant-digit radix sort with 8-bit digits orders them.  Inside
// a tile each wave ranks its 64 keys per digit with eight ballots (lanes
// whose digits agree on every bit), so the sort is stable and deterministic
// without any atomics on the output positions.
#include "sort.h"

namespace md {

static size_t a256(size_t x) { return (x + 255) / 256 * 256; }

size_t sort_workspace_bytes(int64_t rows)
{
    const int64_t tiles = (rows + kRadixTile - 1) / kRadixTile;
    return 2 * a256(sizeof(uint64_t) * rows) + 2 * a256(sizeof(int32_t) * rows) +
           a256(sizeof(int32_t) * 256 * (size_t)tiles) + a256(sizeof(int32_t) * scan_sums_len(256 * tiles)) +
           a256(sizeof(int32_t) * rows) + 256;
}

SortBuffers make_sort_buffers(char *base, int64_t rows)
{
    SortBuffers B{};
    B.rows = rows;
    B.tiles = (rows + kRadixTile - 1) / kRadixTile;
    size_t off = 0;
    B.keys[0] = reinterpret_cast<uint64_t *>(base + off); off += a256(sizeof(uint64_t) * rows);
    B.keys[1] = reinterpret_cast<uint64_t *>(base + off); off += a256(sizeof(uint64_t) * rows);
    B.vals[0] = reinterpret_cast<int32_t *>(base + off); off += a256(sizeof(int32_t) * rows);
    B.vals[1] = reinterpret_cast<int32_t *>(base + off); off += a256(sizeof(int32_t) * rows);
    B.hist = reinterpret_cast<int32_t *>(base + off); off += a256(sizeof(int32_t) * 256 * (size_t)B.tiles);
    B.hist_sums = reinterpret_cast<int32_t *>(base + off);
    off += a256(sizeof(int32_t) * scan_sums_len(256 * B.tiles));
    B.tag_tmp = reinterpret_cast<int32_t *>(base + off);
    return B;
}

// Spread the low 10 bits of v so that bit b lands on bit 3b.
__device__ __forceinline__ uint32_t spread3(uint32_t v)
{
    v &= 0x3FFu;
    v = (v ^ (v << 16)) & 0xFF0000FFu;
    v = (v ^ (v << 8)) & 0x0300F00Fu;
    v = (v ^ (v << 4)) & 0x030C30C3u;
    v = (v ^ (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t quant10(double x, double L)
{
    int q = (int)floor(x * (1024.0 / L));
    q = q < 0 ? 0 : (q > 1023 ? 1023 : q);
    return (uint32_t)q;
}

__global__ void k_morton_keys(const SysDev *__restrict__ sys, const int32_t *__restrict__ tprefix,
                              int n_sys, int tiles, const double4 *__restrict__ pos,
                              uint64_t *__restrict__ keys, int32_t *__restrict__ vals)
{
    const int g = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (g >= tiles) return;
    const int s = find_sys(tprefix, n_sys, g);
    const SysDev &S = sys[s];
    const int r = (g - S.tile0_all) * kTile + lane_id();
    if (r >= S.n_cap) return;
    const int64_t i = S.row0 + r;
    uint32_t code = 0x3FFFFFFFu;
    if (r < S.n_local) {
        const double4 x = pos[i];
        code = spread3(quant10(x.x - S.lo[0], S.L[0])) | (spread3(quant10(x.y - S.lo[1], S.L[1])) << 1) |
               (spread3(quant10(x.z - S.lo[2], S.L[2])) << 2);
    }
    keys[i] = ((uint64_t)s << 30) | code;
    vals[i] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t rows,
                                                    int shift, int64_t tiles, int32_t *__restrict__ hist)
{
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int q = threadIdx.x; q < kRadixTile; q += 256) {
        const int64_t k = base + q;
        if (k < rows) atomicAdd(&h[(keys[k] >> shift) & 0xFF], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter.  Wave w of the block owns rows [w*256, w*256+256) of the
// tile, visited in 4 chunks of 64 in order.
__global__ __launch_bounds__(256) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                       const int32_t *__restrict__ vin,
                                                       uint64_t *__restrict__ kout,
                                                       int32_t *__restrict__ vout, int64_t rows,
                                                       int shift, int64_t tiles,
                                                       const int32_t *__restrict__ offs)
{
    __shared__ int32_t wc[4][256];
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    for (int d = lane; d < 256; d += 64) wc[w][d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile + w * 256;
    const uint64_t lt = lanemask_lt();
    uint64_t key[4];
    int32_t val[4];
    int local[4];
    int dig[4];
    bool ok[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int64_t k = base + c * 64 + lane;
        ok[c] = k < rows;
        key[c] = ok[c] ? kin[k] : 0;
        val[c] = ok[c] ? vin[k] : 0;
        const uint32_t d = (uint32_t)(key[c] >> shift) & 0xFFu;
        dig[c] = (int)d;
        uint64_t m = __ballot(ok[c]);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const int before = wc[w][d];
        local[c] = before + __popcll(m & lt);
        // the lowest lane of each digit group advances the wave counter
        if (ok[c] && (m & lt) == 0) wc[w][d] = before + __popcll(m);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (!ok[c]) continue;
        int p = offs[(int64_t)dig[c] * tiles + blockIdx.x] + local[c];
        for (int v = 0; v < w; ++v) p += wc[v][dig[c]];
        kout[p] = key[c];
        vout[p] = val[c];
    }
}

__global__ void k_gather_rows(int64_t rows, const int32_t *__restrict__ perm, const double4 *__restrict__ pos,
                              const double4 *__restrict__ vel, const int32_t *__restrict__ tag,
                              double4 *__restrict__ pos_o, double4 *__restrict__ vel_o,
                              int32_t *__restrict__ tag_o)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= rows) return;
    const int32_t o = perm[k];
    pos_o[k] = pos[o];
    vel_o[k] = vel[o];
    tag_o[k] = tag[o];
}

// The partner entries (tags and owner directions) move with their rows.
__global__ void k_gather_bonds(int64_t rows, int stride, const int32_t *__restrict__ perm,
                               const int32_t *__restrict__ ptag, const int32_t *__restrict__ pdir,
                               int32_t *__restrict__ ptag_o, int32_t *__restrict__ pdir_o)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= rows) return;
    const int64_t o = perm[k];
    for (int s = 0; s < stride; ++s) {
        ptag_o[k * stride + s] = ptag[o * stride + s];
        pdir_o[k * stride + s] = pdir[o * stride + s];
    }
}

// One workgroup of 1024 threads: each thread sums a contiguous chunk, the
// chunk sums are scanned in LDS, then each thread writes its chunk.
__global__ __launch_bounds__(1024) void k_scan_single(const int32_t *in, int32_t *out, int64_t n,
                                                      int32_t *total)
{
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t b = (int64_t)t * chunk;
    const int64_t e = b + chunk < n ? b + chunk : n;
    int32_t s = 0;
    for (int64_t k = b; k < e; ++k) s += in[k];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = t > 0 ? part[t - 1] : 0;
    if (t == 1023 && total) *total = part[1023];
    for (int64_t k = b; k < e; ++k) {
        const int32_t v = in[k];
        out[k] = run;
        run += v;
    }
}

// Sum of each block of kScanTile values (coalesced reads, fixed-order
// integer reduction).
__global__ __launch_bounds__(256) void k_scan_block_sums(const int32_t *__restrict__ in, int64_t n,
                                                         int32_t *__restrict__ sums)
{
    __shared__ int32_t ws[4];
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile;
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanTile / 256; ++k) {
        const int64_t i = b0 + k * 256 + threadIdx.x;
        s += i < n ? in[i] : 0;
    }
    s = wave_sum(s);
    if (lane_id() == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) sums[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Exclusive scan of each block, offset by the block's scanned sum: every
// thread reads its 16 consecutive values before writing them (in-place safe).
__global__ __launch_bounds__(256) void k_scan_block_apply(const int32_t *in, int32_t *out, int64_t n,
                                                          const int32_t *__restrict__ sums)
{
    constexpr int kPer = kScanTile / 256;
    __shared__ int32_t ws[4];
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile + (int64_t)kPer * threadIdx.x;
    int32_t v[kPer];
    int32_t tot = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        v[k] = b0 + k < n ? in[b0 + k] : 0;
        tot += v[k];
    }
    const int lane = lane_id();
    int32_t inc = tot;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int32_t y = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += y;
    }
    if (lane == kWave - 1) ws[threadIdx.x >> 6] = inc;
    __syncthreads();
    int32_t run = sums[blockIdx.x] + inc - tot;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) run += ws[w];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (b0 + k < n) out[b0 + k] = run;
        run += v[k];
    }
}

void launch_scan(hipStream_t stream, const int32_t *in, int32_t *out, int64_t n, int32_t *total,
                 int32_t *sums)
{
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb > 0) hipLaunchKernelGGL(k_scan_block_sums, dim3((unsigned)nb), dim3(256), 0, stream, in, n, sums);
    // the block sums, scanned in place by one workgroup (also writes the total)
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, stream, sums, sums, nb, total);
    if (nb > 0) hipLaunchKernelGGL(k_scan_block_apply, dim3((unsigned)nb), dim3(256), 0, stream, in, out, n, sums);
}

void launch_morton_keys(const LaunchCtx &L, const double4 *pos, uint64_t *keys, int32_t *vals)
{
    const int threads = 256;
    const int blocks = (L.tiles_all * kWave + threads - 1) / threads;
    if (blocks == 0) return;
    hipLaunchKernelGGL(k_morton_keys, dim3(blocks), dim3(threads), 0, L.stream, L.sys, L.tprefix_all,
                       L.n_sys, L.tiles_all, pos, keys, vals);
}

int queue_morton_sort(const LaunchCtx &L, const SortBuffers &B, double4 *pos, double4 *vel,
                      int32_t *tag, double4 *pos_tmp, double4 *vel_tmp)
{
    if (B.rows <= 0) return 0;
    launch_morton_keys(L, pos, B.keys[0], B.vals[0]);
    int bits = 30;
    while ((1 << (bits - 30)) < L.n_sys) ++bits;
    const int passes = (bits + 7) / 8;
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)B.tiles), dim3(256), 0, L.stream, B.keys[cur],
                           B.rows, shift, B.tiles, B.hist);
        launch_scan(L.stream, B.hist, B.hist, 256 * B.tiles, nullptr, B.hist_sums);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)B.tiles), dim3(256), 0, L.stream, B.keys[cur],
                           B.vals[cur], B.keys[cur ^ 1], B.vals[cur ^ 1], B.rows, shift, B.tiles, B.hist);
        cur ^= 1;
    }
    const int blocks = (int)((B.rows + 255) / 256);
    hipLaunchKernelGGL(k_gather_rows, dim3(blocks), dim3(256), 0, L.stream, B.rows, B.vals[cur], pos, vel,
                       tag, pos_tmp, vel_tmp, B.tag_tmp);
    if (hipMemcpyAsync(pos, pos_tmp, sizeof(double4) * B.rows, hipMemcpyDeviceToDevice, L.stream) != hipSuccess) return 1;
    if (hipMemcpyAsync(vel, vel_tmp, sizeof(double4) * B.rows, hipMemcpyDeviceToDevice, L.stream) != hipSuccess) return 1;
    if (hipMemcpyAsync(tag, B.tag_tmp, sizeof(int32_t) * B.rows, hipMemcpyDeviceToDevice, L.stream) != hipSuccess) return 1;
    if (L.bond_stride > 0) {
        // the partner-row table is rebuilt after the sort: it serves as scratch
        const size_t nb = sizeof(int32_t) * (size_t)B.rows * (size_t)L.bond_stride;
        hipLaunchKernelGGL(k_gather_bonds, dim3(blocks), dim3(256), 0, L.stream, B.rows, L.bond_stride, B.vals[cur],
                           L.ptag, L.pdir, L.prow, L.btmp);
        if (hipMemcpyAsync(L.ptag, L.prow, nb, hipMemcpyDeviceToDevice, L.stream) != hipSuccess) return 1;
        if (hipMemcpyAsync(L.pdir, L.btmp, nb, hipMemcpyDeviceToDevice, L.stream) != hipSuccess) return 1;
    }
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // namespace md
