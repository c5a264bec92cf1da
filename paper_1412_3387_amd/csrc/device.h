// device.h -- shared device definitions of the MI355X MD hot path: the
// per-system descriptor, the tile -> system mapping used by every
// per-particle kernel, minimum image and folding, wave64 primitives, and the
// counter-based generator of the DPD pair noise.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace md {

constexpr int kWave = 64;       // CDNA wavefront width
constexpr int kTile = 64;       // rows per neighbour-list tile (one wave)
constexpr int kMaxBondCap = 4;  // partners per particle held in registers

enum Pair : int32_t { PAIR_LJ = 0, PAIR_WCA = 1, PAIR_DPD = 2 };

// Status word (device): first latched code and the capacity that would
// have avoided an overflow.
struct Status {
    int32_t code;       // first non-zero code latched
    int32_t flags;      // OR of (1 << code) of every condition seen
    int64_t required;   // max capacity seen missing
};

// One system, as the kernels see it.  Lives in device memory; every field is
// read with the system index uniform across a wave.
struct SysDev {
    double lo[3];
    double L[3];
    double invL[3];         // 1/L on periodic axes, 0 on open axes
    double scale[3];        // bins / L  (cell coordinate of x: floor((x-lo)*scale))
    int32_t per[3];
    int32_t bins[3];
    int32_t nst[3];         // stencil offsets per axis (after de-duplication)
    int32_t st[3][3];       // the offsets themselves
    int64_t row0;           // first row of this system in the particle arrays
    int32_t n_local;        // rows integrated
    int32_t n_total;        // locals + ghosts (rows binned / neighbours)
    int32_t n_cap;          // rows reserved for this system
    int32_t bond_stride;    // entries per particle of the partner table (same for all systems)
    int64_t nl0;            // first neighbour-list entry of this system
    int64_t cell0;          // first cell of this system
    int64_t hash0;          // first slot of this system's tag -> row table (bonded systems)
    int32_t hash_mask;      // its slots - 1 (a power of two minus one)
    int32_t hash_pad;
    int32_t tile0;          // first local tile (64 rows) of this system
    int32_t tile0_all;      // first tile over all rows (locals + ghosts)
    int32_t pair;           // Pair
    int32_t bond_cap;       // partner slots used by this system (0 = none), <= bond_stride
    double rc2;             // cut-off^2 (FP64 test, both precisions)
    double rl2;             // (r_cut + r_buff)^2
    double disp2;           // (r_buff / 2)^2
    // LJ / WCA
    double eps, sig2, shift;   // shift = V(r_cut) subtracted from the energy
    // DPD
    double dpd_A, dpd_gamma, dpd_sigma, dpd_inv_rc, dpd_inv_sqrt_dt, dpd_rc;
    uint32_t dpd_seed;
    int32_t nvt_slot;       // Nose-Hoover: first system of the thermostat group; -1 = NVE
    // FENE + WCA bonds
    double fene_K, fene_R02, wca_rc2;
    double dt, hdt;
    double nvt_c, nvt_T0;   // Nose-Hoover: dt / tau^2 and the set temperature
};

// Workgroup b of a launch runs on accelerator die b % kDies, and each die has
// its own L2.  Neighbouring tiles share most of their halo, so the tiles are
// handed out so that the workgroups of one die walk one contiguous run of
// them (Morton-ordered rows make that run one compact region of space).
constexpr int kDies = 8;

// Tile of workgroup b in a launch of nb workgroups, one tile each.
__device__ __forceinline__ int die_tile(int b, int nb)
{
    const int x = b % kDies, l = b / kDies;
    const int per = nb / kDies, rem = nb % kDies;
    return x * per + (x < rem ? x : rem) + l;
}

// Items [first, end) with stride step of workgroup b when nb workgroups loop
// over n items: the dies that have workgroups split the items into
// contiguous runs.
__device__ __forceinline__ void die_range(int b, int nb, int64_t n, int64_t &first, int64_t &end, int &step)
{
    const int D = nb < kDies ? nb : kDies;
    const int x = b % D, l = b / D;
    step = nb / D + (x < nb % D ? 1 : 0);
    first = n * x / D + l;
    end = n * (x + 1) / D;
}

// System owning a tile: largest s with prefix[s] <= tile (prefix has n_sys+1
// entries, prefix[0] = 0).  Called with a wave-uniform tile.
__device__ __forceinline__ int find_sys(const int32_t *__restrict__ prefix, int n_sys, int tile)
{
    int lo = 0, hi = n_sys;  // invariant prefix[lo] <= tile < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= tile) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Minimum image along periodic axes: d - L * rint(d / L), written with the
// reciprocal.  For |d| < L/2 - ulp the image index equals the one the exact
// quotient gives, so every separation shorter than half a box is bitwise the
// same as with a true division.  Open axes have invL = 0 and pass through.
__device__ __forceinline__ double min_image(double d, double L, double invL)
{
    return __fma_rn(-L, rint(d * invL), d);
}

// Squared length with the summation order fixed and no fused multiply-add,
// so that neighbour decisions reproduce any IEEE evaluation of the same
// expression bit for bit.
__device__ __forceinline__ double norm2_exact(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    const double xx = dx * dx;
    const double yy = dy * dy;
    const double zz = dz * dz;
    return (xx + yy) + zz;
}

// Fold a coordinate of a periodic axis once into [lo, lo + L).
__device__ __forceinline__ double fold(double x, double lo, double L)
{
    const double hi = lo + L;
    if (x >= hi) x -= L;
    else if (x < lo) x += L;
    if (x >= hi) x -= L;
    return x;
}

// Cell coordinate along one axis, clamped to the grid.
__device__ __forceinline__ int cell_coord(double x, double lo, double scale, int bins)
{
    int c = (int)floor((x - lo) * scale);
    c = c < 0 ? 0 : c;
    c = c > bins - 1 ? bins - 1 : c;
    return c;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Workgroup barrier for kernels whose waves share data only through LDS:
// waits until this wave's LDS (and scalar) accesses are done, but not for its
// global loads and stores, which stay in flight across the barrier (a full
// __syncthreads() also waits for those).  The memory clobber keeps the
// compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Bits {pl, pl + P, pl + 2P, ...} of a 64-bit mask: the lanes that share one
// particle when lane = s * P + pl.
__device__ __forceinline__ uint64_t segment_bits(int pl, int P)
{
    uint64_t m = 0;
    for (int b = pl; b < kWave; b += P) m |= 1ull << b;
    return m;
}

template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int m)
{
    return __shfl_xor(v, m, kWave);
}

// Sum over the W lanes of a particle (lanes pl + P*s, s < W), all lanes
// receive the total.  Fixed butterfly order: deterministic.
template <int W, typename T>
__device__ __forceinline__ T segment_sum(T v)
{
    constexpr int P = kWave / W;
#pragma unroll
    for (int m = P; m < kWave; m <<= 1) v += shfl_xor(v, m);
    return v;
}

// Wave-wide sum in a fixed butterfly order.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) v += shfl_xor(v, m);
    return v;
}

__device__ __forceinline__ void latch(Status *st, int code, int64_t required)
{
    atomicCAS(&st->code, 0, code);
    atomicOr(&st->flags, 1 << code);
    if (required > 0) atomicMax((unsigned long long *)&st->required, (unsigned long long)required);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32 -> 64-bit products of counter words 0 and 2 with fixed multipliers,
// the high halves xored with the other counter words and the round key, the
// key advanced by a Weyl sequence between rounds.  Only the first output word
// is used by the DPD noise.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t philox_first_word(uint32_t c0, uint32_t c1, uint32_t c2,
                                                      uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c0;
}

// Unit-variance uniform pair variate, symmetric in the two tags.
__device__ __forceinline__ uint32_t dpd_bits(uint32_t ta, uint32_t tb, uint32_t seed, uint32_t step)
{
    const uint32_t a = ta < tb ? ta : tb;
    const uint32_t b = ta < tb ? tb : ta;
    return philox_first_word(a, b, 0u, 0u, seed, step) >> 8;
}

// Nose-Hoover update of the thermostat group whose first system is s, by a
// workgroup of nt threads (this one tid; every thread calls it): the group's
// half-step kinetic-energy partials (w per tile, tiles in order) summed as
// kNvtSums strided partial sums and a tree over them, the same order for
// any workgroup size, then
//   xi' = xi + dt/tau^2 (T/T0 - 1),  eta' = eta + dt/2 (xi + xi'),
// with T = 2 KE / (3 N - 3) over the group's N local particles.  red holds
// kNvtSums doubles in LDS.
constexpr int kNvtSums = 256;
__device__ inline void nvt_group_update(const SysDev *__restrict__ sys, const int32_t *__restrict__ tprefix,
                                        int n_sys, int w, const double *__restrict__ khalf,
                                        double *__restrict__ thermostat, int s, double *red, int nt, int tid)
{
    for (int v = tid; v < kNvtSums; v += nt) {
        double k = 0.0;
        for (int q = s; q < n_sys; ++q) {
            if (sys[q].nvt_slot != s) continue;
            const int64_t w0 = (int64_t)tprefix[q] * w, w1 = (int64_t)tprefix[q + 1] * w;
            int64_t p = w0 + v;
            // eight loads in flight, added in the same order as one at a time
            for (; p + 7 * kNvtSums < w1; p += 8 * kNvtSums) {
                double a[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] = khalf[p + u * kNvtSums];
#pragma unroll
                for (int u = 0; u < 8; ++u) k += a[u];
            }
            for (; p < w1; p += kNvtSums) k += khalf[p];
        }
        red[v] = k;
    }
    __syncthreads();
    for (int m = kNvtSums / 2; m > 0; m >>= 1) {
        for (int v = tid; v < m; v += nt) red[v] += red[v + m];
        __syncthreads();
    }
    if (tid == 0) {
        int64_t n = 0;
        for (int q = s; q < n_sys; ++q)
            if (sys[q].nvt_slot == s) n += sys[q].n_local;
        const SysDev &S = sys[s];
        const double g = 3.0 * (double)n - 3.0;
        const double T = g > 0 ? 2.0 * red[0] / g : S.nvt_T0;
        const double xi = thermostat[2 * s];
        const double xn = xi + S.nvt_c * (T / S.nvt_T0 - 1.0);
        thermostat[2 * s + 1] = thermostat[2 * s + 1] + S.hdt * (xi + xn);
        thermostat[2 * s] = xn;
    }
    __syncthreads();  // red free again
}

}  // namespace md
