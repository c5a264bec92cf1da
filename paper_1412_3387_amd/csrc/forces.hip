// forces.hip -- pair + bond forces fused with the velocity-Verlet update.
//
// Sec. 5.1: W lanes cooperate on one particle, striding over its neighbour
// row, and a lane reduction totals the force.  One workgroup handles one tile
// of 64 rows: it first copies the tile's halo (the union of the rows'
// neighbours) from HBM/L2 into LDS, each halo position moved to its periodic
// image nearest the tile, so every neighbour read afterwards is an LDS read
// and needs no minimum-image arithmetic.  The same launch then does the whole
// step of each particle: the closing half kick of the previous step, the
// thermo sums, the opening half kick, the drift, the fold into the box, and
// the displacement check that decides the next neighbour-list rebuild
// (Sec. 4.2: rebuild once a particle has moved more than r_buff / 2).  New
// positions go to the other half of a position double buffer, so every halo
// read in the launch sees the old ones; DPD double-buffers the velocities
// too, because the pair force reads neighbour velocities.
//
// Precision: every separation, the cut-off test, the force sums and the
// integrator are FP64.  With MIXED the pair and bond arithmetic after the
// cut-off test is FP32 (each pair's F/r is widened before it is summed);
// energies and virials are summed in FP64.
#include <type_traits>

#include "device.h"
#include "launch.h"

namespace md {

template <typename T> __device__ __forceinline__ T recip(T x);
template <> __device__ __forceinline__ float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double recip<double>(double x) { return 1.0 / x; }

template <typename T> __device__ __forceinline__ T tsqrt(T x);
template <> __device__ __forceinline__ float tsqrt<float>(float x) { return __builtin_sqrtf(x); }
template <> __device__ __forceinline__ double tsqrt<double>(double x) { return __builtin_sqrt(x); }

template <typename T> __device__ __forceinline__ T tlog(T x);
template <> __device__ __forceinline__ float tlog<float>(float x) { return __logf(x); }
template <> __device__ __forceinline__ double tlog<double>(double x) { return log(x); }

// LJ-family pair term for one neighbour inside the cut-off.  Returns the
// force divided by r (F_i = ff * (x_i - x_j)), 24 eps s6 (2 s6 - 1) / r^2 with
// s6 = (sigma^2 / r^2)^3 written as s6 (48 eps s6 - 24 eps) / r^2; adds energy
// and virial.  Zero where in is false, whatever r2 holds (masked lanes pass
// the separations of stale entries).
template <typename T, bool LOG>
__device__ __forceinline__ T lj_pair(double r2, T eps, T sig2, double shift, double &e, double &vir,
                                    bool in = true)
{
    // a pair outside (in == false) gets 1/r^2 = 0, hence a zero force
    const T r2inv = in ? recip<T>((T)r2) : (T)0;
    const T s2 = sig2 * r2inv;
    const T s6 = s2 * s2 * s2;
    const T ff = s6 * ((T)48 * eps * s6 - (T)24 * eps) * r2inv;
    if constexpr (LOG) {
        if (in) {
            e += (double)((T)4 * eps * s6 * (s6 - (T)1)) - shift;
            vir += (double)(ff * (T)r2);
        }
    }
    return ff;
}

// Bytes of LDS per halo entry.
__host__ __device__ constexpr int halo_entry_bytes(int pot) { return pot == PAIR_DPD ? 52 : 24; }

// Rows may be read this many entries past their end (two passes of the
// widest split): the neighbour list is padded by as many tile columns.
constexpr int kRowOverRead = 2 * 4 * 16;
constexpr int kRareGrid = 1024;  // workgroups of the launch over the rare tiles
constexpr size_t kRareLds = 40 * 1024;  // LDS of a workgroup of that launch, at most (four per CU)

// One tile of the fused step.  RARE selects the code for tiles with a
// per-pair image or a halo larger than the LDS staging area; the main
// launch leaves those to a second, small launch, so that its own code needs
// fewer registers (more waves per CU).
template <int W, bool MIXED, int POT, bool LOG, bool RARE>
__device__ __forceinline__ void force_tile(int tile, double *lds, const SysDev *__restrict__ sys,
                                           const int32_t *__restrict__ tprefix, int n_sys,
                                           const uint16_t *__restrict__ nlist,
                                           const int32_t *__restrict__ nn, int cap,
                                           const int32_t *__restrict__ halo,
                                           const int32_t *__restrict__ halo_n, int halo_cap, int halo_lds,
                                           const int32_t *__restrict__ prow,
                                           const double4 *__restrict__ xbuild,
                                           double *__restrict__ partials, Status *st, const ForceLaunch &a)
{
    using T = typename std::conditional<MIXED, float, double>::type;
    // LDS holds the halo only: positions interleaved per entry (one address
    // for x, y, z), then for DPD the velocities and tags.  Rows stream from
    // global memory one pass ahead of their use.
    double *hxyz = lds;
    double *hv = hxyz + 3 * halo_lds;
    int32_t *htag = reinterpret_cast<int32_t *>(hv + 3 * halo_lds);

    constexpr int P = kWave / W;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wv = tid >> 6;
    const int pl = lane % P;
    const int sl = lane / P;
    const int gw = tile * W + wv;
    const int t = wv * P + pl;  // row slot in the tile
    const int s = find_sys(tprefix, n_sys, tile);
    const SysDev &S = sys[s];
    // per-system constants, held in registers for the whole launch
    const double Lx = S.L[0], Ly = S.L[1], Lz = S.L[2];
    const double iLx = S.invL[0], iLy = S.invL[1], iLz = S.invL[2];
    const int64_t row0 = S.row0;
    const int n_local = S.n_local;
    const int64_t nl0 = S.nl0;
    const double rc2 = S.rc2;
    const T eps = (T)S.eps, sig2 = (T)S.sig2;
    const double shift = S.shift;
    // Nose-Hoover friction of this system for the whole launch (NVE: none)
    const bool nvt = a.thermostat != nullptr && S.nvt_slot >= 0;
    const double xi_nh = nvt ? a.thermostat[2 * S.nvt_slot] : 0.0;
    const int r0 = (tile - S.tile0) * kTile;
    const int r = r0 + t;
    const bool active = r < n_local;
    const int64_t i = row0 + (active ? r : r0);

    // ---- the row's first pass, then the halo ------------------------------
    constexpr int U = 4;
    const int32_t hn = halo_n[tile];
    const int nh = hn & 0xFFFF;
    const bool per_pair = hn < 0;  // tile too wide for one image per halo entry
    int n = active ? nn[i] : 0;
    n = n < cap ? n : cap;
    // entry k of this row at rowp[k * 64]; the list is padded so that reads up
    // to two passes past any row's end stay inside it (their values are masked)
    const uint16_t *rowp = nlist + nl0 + (int64_t)(r0 >> 6) * cap * kTile + t;
    int hnext[U];
#pragma unroll
    for (int u = 0; u < U; ++u) hnext[u] = rowp[(int64_t)(sl + u * W) * kTile];
    const double4 xref = a.pos[row0 + r0];
    const int32_t *hl = halo + (int64_t)tile * halo_cap;
    // halo entry h: its position moved to the image nearest the tile's first
    // row (unless the tile needs per-pair images)
    auto halo_pos = [&](int h, double &px, double &py, double &pz) {
        const double4 x = a.pos[hl[h]];
        px = x.x;
        py = x.y;
        pz = x.z;
        if (!per_pair) {
            px = __fma_rn(-Lx, rint((px - xref.x) * iLx), px);
            py = __fma_rn(-Ly, rint((py - xref.y) * iLy), py);
            pz = __fma_rn(-Lz, rint((pz - xref.z) * iLz), pz);
        }
    };
    // the first halo_lds entries are staged in LDS; a tile with more reads
    // the rest from global memory (rare: halo_lds is sized for occupancy)
    const int ns = nh < halo_lds ? nh : halo_lds;
    // a tile without neighbours still has a finite halo entry 0 (read by
    // masked lanes)
    if (nh == 0 && tid == 0) {
        hxyz[0] = xref.x;
        hxyz[1] = xref.y;
        hxyz[2] = xref.z;
    }
    // the row's own position, read before the staging so that its latency
    // overlaps it
    const double4 xi = a.pos[i];
    // SB entries per thread per batch: every index load of a batch issues
    // before any gather, and every gather before any use, so a tile waits for
    // two memory round trips per batch instead of two per entry (indices past
    // the halo's end are clamped to its last entry and not stored)
    constexpr int SB = 4;
    constexpr int NT = W * kWave;
    for (int h0 = tid; h0 < ns; h0 += SB * NT) {
        int32_t jb[SB];
#pragma unroll
        for (int b = 0; b < SB; ++b) {
            const int h = h0 + b * NT;
            jb[b] = hl[h < ns ? h : ns - 1];
        }
        double4 xb[SB];
#pragma unroll
        for (int b = 0; b < SB; ++b) xb[b] = a.pos[jb[b]];
        double4 vb[SB];
        int32_t tb[SB];
        if constexpr (POT == PAIR_DPD) {
#pragma unroll
            for (int b = 0; b < SB; ++b) {
                vb[b] = a.vel[jb[b]];
                tb[b] = a.tag[jb[b]];
            }
        }
#pragma unroll
        for (int b = 0; b < SB; ++b) {
            const int h = h0 + b * NT;
            if (h >= ns) break;
            double px = xb[b].x, py = xb[b].y, pz = xb[b].z;
            if (!per_pair) {
                px = __fma_rn(-Lx, rint((px - xref.x) * iLx), px);
                py = __fma_rn(-Ly, rint((py - xref.y) * iLy), py);
                pz = __fma_rn(-Lz, rint((pz - xref.z) * iLz), pz);
            }
            hxyz[3 * h] = px;
            hxyz[3 * h + 1] = py;
            hxyz[3 * h + 2] = pz;
            if constexpr (POT == PAIR_DPD) {
                hv[3 * h] = vb[b].x;
                hv[3 * h + 1] = vb[b].y;
                hv[3 * h + 2] = vb[b].z;
                htag[h] = tb[b];
            }
        }
    }
    __syncthreads();

    // the row's own position, moved to the same frame as the halo images
    double xs = xi.x, ys = xi.y, zs = xi.z;
    if (!per_pair) {
        xs = __fma_rn(-Lx, rint((xs - xref.x) * iLx), xs);
        ys = __fma_rn(-Ly, rint((ys - xref.y) * iLy), ys);
        zs = __fma_rn(-Lz, rint((zs - xref.z) * iLz), zs);
    }
    double4 vi;
    if constexpr (POT == PAIR_DPD) vi = a.vel[i];
    int32_t ti = 0;
    if constexpr (POT == PAIR_DPD) ti = a.tag[i];
    uint32_t step_key = a.timestep;
    if constexpr (POT == PAIR_DPD)
        if (a.timestep_ptr) step_key = *a.timestep_ptr;
    double fx = 0, fy = 0, fz = 0;
    double e = 0.0, vir = 0.0;

    // four neighbours per pass: all LDS reads of a pass issue before any use.
    // The per-pair image branch is taken once per tile, outside the loop.
    auto pair_loop = [&](auto per_pair_tag, auto spill_tag) {
        constexpr bool PP = decltype(per_pair_tag)::value;
        constexpr bool OVF = decltype(spill_tag)::value;
        for (int k0 = sl; k0 < n; k0 += U * W) {
            int hh[U];
            bool ok[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int kk = k0 + u * W;
                ok[u] = kk < n;
                // past the row's end: stale or foreign values, masked
                hh[u] = ok[u] ? hnext[u] : 0;
                hnext[u] = rowp[(int64_t)(kk + U * W) * kTile];
            }
            double dx[U], dy[U], dz[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                double px, py, pz;
                if (!OVF || hh[u] < halo_lds) {
                    const double *hp = reinterpret_cast<const double *>(
                        reinterpret_cast<const char *>(hxyz) + (uint32_t)hh[u] * 24u);
                    px = hp[0];
                    py = hp[1];
                    pz = hp[2];
                } else {
                    halo_pos(hh[u], px, py, pz);
                }
                dx[u] = xs - px;
                dy[u] = ys - py;
                dz[u] = zs - pz;
            }
            if constexpr (PP) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    dx[u] = min_image(dx[u], Lx, iLx);
                    dy[u] = min_image(dy[u], Ly, iLy);
                    dz[u] = min_image(dz[u], Lz, iLz);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // FP64 in both precisions; the FP64 path keeps the unfused,
                // fixed-order sum of the reference, the mixed path fuses it
                const double r2 = MIXED ? __fma_rn(dx[u], dx[u], __fma_rn(dy[u], dy[u], dz[u] * dz[u]))
                                        : norm2_exact(dx[u], dy[u], dz[u]);
                if constexpr (POT == PAIR_LJ || POT == PAIR_WCA) {
                    // branch-free: lanes outside the cut-off add zero
                    const bool in = ok[u] && r2 < rc2;
                    const T ff = lj_pair<T, LOG>(r2, eps, sig2, shift, e, vir, in);
                    fx = __fma_rn((double)ff, dx[u], fx);
                    fy = __fma_rn((double)ff, dy[u], fy);
                    fz = __fma_rn((double)ff, dz[u], fz);
                    continue;
                }
                if (ok[u] && r2 < rc2) {
                    T ff;
                    {
                        if (r2 == 0.0) continue;
                        const int h = hh[u];
                        const T tr2 = (T)r2;
                        const T rr = tsqrt<T>(tr2);
                        const T rinv = recip<T>(rr);
                        const T w = (T)1 - rr * (T)S.dpd_inv_rc;
                        double vx, vy, vz;
                        int32_t tj;
                        if (!OVF || h < halo_lds) {
                            vx = hv[3 * h];
                            vy = hv[3 * h + 1];
                            vz = hv[3 * h + 2];
                            tj = htag[h];
                        } else {
                            const int32_t j = hl[h];
                            const double4 vj = a.vel[j];
                            vx = vj.x;
                            vy = vj.y;
                            vz = vj.z;
                            tj = a.tag[j];
                        }
                        const T dvx = (T)(vi.x - vx), dvy = (T)(vi.y - vy), dvz = (T)(vi.z - vz);
                        const T rv = ((T)dx[u] * dvx + (T)dy[u] * dvy + (T)dz[u] * dvz) * rinv;
                        const uint32_t bits = dpd_bits((uint32_t)ti, (uint32_t)tj, S.dpd_seed, step_key);
                        const T uu = (T)bits * (T)(1.0 / 16777216.0);
                        const T theta = (T)1.7320508075688772 * ((T)2 * uu - (T)1);
                        const T mag = (T)S.dpd_A * w - (T)S.dpd_gamma * w * w * rv +
                                      (T)S.dpd_sigma * w * theta * (T)S.dpd_inv_sqrt_dt;
                        ff = mag * rinv;
                        if constexpr (LOG) {
                            e += 0.5 * S.dpd_A * S.dpd_rc * (double)(w * w);
                            vir += (double)(ff * tr2);
                        }
                    }
                    fx = __fma_rn((double)ff, dx[u], fx);
                    fy = __fma_rn((double)ff, dy[u], fy);
                    fz = __fma_rn((double)ff, dz[u], fz);
                }
            }
        }
    };
    if constexpr (RARE) {
        if (nh > halo_lds) {
            if (per_pair) pair_loop(std::true_type{}, std::true_type{});
            else pair_loop(std::false_type{}, std::true_type{});
        } else {
            if (per_pair) pair_loop(std::true_type{}, std::false_type{});
            else pair_loop(std::false_type{}, std::false_type{});
        }
    } else {
        pair_loop(std::false_type{}, std::false_type{});
    }

    fx = segment_sum<W>(fx);
    fy = segment_sum<W>(fy);
    fz = segment_sum<W>(fz);
    if constexpr (LOG) {
        e = segment_sum<W>(e);
        vir = segment_sum<W>(vir);
    }

    double ke = 0.0, kh = 0.0;
    const bool owner = active && sl == 0;
    if (owner) {
        double Fx = (double)fx, Fy = (double)fy, Fz = (double)fz;
        double ue = 0.5 * e, uw = 0.5 * vir;
        // bonds: FENE + WCA with the partner rows found at the last change
        // of rows (a local row or a ghost)
        if (S.bond_cap > 0) {
            const int64_t pr = i * S.bond_stride;
            for (int b = 0; b < S.bond_cap; ++b) {
                const int32_t j = prow[pr + b];
                if (j < 0) {
                    if (j == -2) latch(st, 12 /*BOND_GHOST*/, 0);  // a partner that is not here
                    continue;
                }
                const double4 xj = a.pos[j];
                const double ddx = min_image(xi.x - xj.x, Lx, iLx);
                const double ddy = min_image(xi.y - xj.y, Ly, iLy);
                const double ddz = min_image(xi.z - xj.z, Lz, iLz);
                const double r2 = norm2_exact(ddx, ddy, ddz);
                if (!(r2 < S.fene_R02)) {
                    latch(st, 8 /*BOND_STRETCH*/, 0);
                    continue;
                }
                const T g = (T)1 - (T)r2 * (T)(1.0 / S.fene_R02);
                T ff = -(T)S.fene_K * recip<T>(g);
                double eb = 0.0, vb = 0.0;
                if constexpr (LOG) eb = -0.5 * S.fene_K * S.fene_R02 * (double)tlog<T>(g);
                if (r2 < S.wca_rc2) {
                    double e2 = 0.0, v2 = 0.0;
                    ff += lj_pair<T, LOG>(r2, eps, sig2, -S.eps, e2, v2);
                    eb += e2;
                }
                if constexpr (LOG) vb = (double)(ff * (T)r2);
                Fx += (double)(ff * (T)ddx);
                Fy += (double)(ff * (T)ddy);
                Fz += (double)(ff * (T)ddz);
                ue += 0.5 * eb;
                uw += 0.5 * vb;
            }
        }
        if (!__builtin_isfinite(Fx + Fy + Fz)) latch(st, 9 /*NAN*/, 0);

        double4 v = (POT == PAIR_DPD) ? vi : a.vel[i];
        const double hdt = S.hdt;
        if (a.mode == MODE_MID || a.mode == MODE_LAST) {
            v.x += hdt * Fx;
            v.y += hdt * Fy;
            v.z += hdt * Fz;
            if (nvt) {
                // the closing half of the Nose-Hoover step, implicit in v
                const double d = 1.0 + hdt * xi_nh;
                v.x = v.x / d;
                v.y = v.y / d;
                v.z = v.z / d;
            }
        }
        if constexpr (LOG) ke = 0.5 * ((v.x * v.x + v.y * v.y) + v.z * v.z);
        if (a.mode == MODE_FIRST || a.mode == MODE_MID) {
            if (nvt) {
                v.x += hdt * (Fx - xi_nh * v.x);
                v.y += hdt * (Fy - xi_nh * v.y);
                v.z += hdt * (Fz - xi_nh * v.z);
                kh = 0.5 * ((v.x * v.x + v.y * v.y) + v.z * v.z);
            } else {
                v.x += hdt * Fx;
                v.y += hdt * Fy;
                v.z += hdt * Fz;
            }
            double4 x = xi;
            const double dt = S.dt;
            x.x += dt * v.x;
            x.y += dt * v.y;
            x.z += dt * v.z;
            if (S.per[0]) x.x = fold(x.x, S.lo[0], Lx);
            if (S.per[1]) x.y = fold(x.y, S.lo[1], Ly);
            if (S.per[2]) x.z = fold(x.z, S.lo[2], Lz);
            a.pos_out[i] = x;
            a.vel_out[i] = v;
            // displacement check (Sec. 4.2) on the steps of the check period,
            // counted from the last build; a rebuild at the first check after a
            // build may have come late when the period is above one (Sec. 6.1:
            // a dangerous build)
            const int since1 = a.since ? a.since[s] + 1 : 1;
            if (a.check_period <= 1 || since1 % a.check_period == 0) {
                const double4 xb = xbuild[i];
                const double bx = min_image(x.x - xb.x, Lx, iLx);
                const double by = min_image(x.y - xb.y, Ly, iLy);
                const double bz = min_image(x.z - xb.z, Lz, iLz);
                if ((bx * bx + by * by) + bz * bz > S.disp2) {
                    // this system's list is rebuilt after the step
                    *a.flag_set = 1;
                    a.sflag_set[s] = 1;
                    if (a.check_period > 1 && since1 == a.check_period) latch(st, 10 /*DANGEROUS_BUILD*/, 0);
                }
            }
        } else {
            if (a.mode == MODE_LAST) a.vel_out[i] = v;
            if (MIXED) {
                float4 f = make_float4((float)Fx, (float)Fy, (float)Fz, a.energy ? (float)ue : 0.0f);
                reinterpret_cast<float4 *>(a.force)[i] = f;
            } else {
                double4 f = make_double4(Fx, Fy, Fz, a.energy ? ue : 0.0);
                reinterpret_cast<double4 *>(a.force)[i] = f;
            }
        }
        e = ue;
        vir = uw;
    }
    if (a.khalf) {
        // per-wave kinetic energy of the half-step velocities, summed per
        // thermostat group after the launch
        double k = owner ? kh : 0.0;
        k = wave_sum(k);
        if (lane == 0) a.khalf[gw] = k;
    }
    if constexpr (LOG) {
        double k3 = owner ? ke : 0.0;
        double e3 = owner ? e : 0.0;
        double w3 = owner ? vir : 0.0;
        k3 = wave_sum(k3);
        e3 = wave_sum(e3);
        w3 = wave_sum(w3);
        if (lane == 0) {
            partials[3 * (int64_t)gw + 0] = k3;
            partials[3 * (int64_t)gw + 1] = e3;
            partials[3 * (int64_t)gw + 2] = w3;
        }
    }
}

#define FORCE_ARGS                                                                                       \
    const SysDev *__restrict__ sys, const int32_t *__restrict__ tprefix, int n_sys,                      \
        const uint16_t *__restrict__ nlist, const int32_t *__restrict__ nn, int cap,                     \
        const int32_t *__restrict__ halo, const int32_t *__restrict__ halo_n, int halo_cap, int halo_lds, \
        const int32_t *__restrict__ prow,                                                               \
        const double4 *__restrict__ xbuild, double *__restrict__ partials, Status *st,                   \
        const int32_t *__restrict__ rare_list, const int32_t *__restrict__ rare_n, ForceLaunch a
#define FORCE_PASS sys, tprefix, n_sys, nlist, nn, cap, halo, halo_n, halo_cap, halo_lds, prow, \
                   xbuild, partials, st, a

// Main launch: one workgroup per tile; rare tiles return at once.
template <int W, bool MIXED, int POT, bool LOG>
__global__ __launch_bounds__(1024) void k_force(FORCE_ARGS)
{
    extern __shared__ double lds[];
    if (a.flag_clear && blockIdx.x == 0) {
        if (threadIdx.x == 0) *a.flag_clear = 0;
        for (int q = threadIdx.x; q < n_sys; q += blockDim.x) a.sflag_clear[q] = 0;
    }
    const int tile = die_tile(blockIdx.x, gridDim.x);
    const int32_t hn = halo_n[tile];
    if (hn < 0 || (hn & 0xFFFF) > halo_lds) return;
    force_tile<W, MIXED, POT, LOG, false>(tile, lds, FORCE_PASS);
}

// The tiles the last build listed as rare (per-pair images or a halo larger
// than the staging area), or, without a list, every local tile (the whole
// pass in one launch).
template <int W, bool MIXED, int POT, bool LOG>
__global__ __launch_bounds__(1024) void k_force_rare(FORCE_ARGS)
{
    extern __shared__ double lds[];
    if (!rare_list && a.flag_clear && blockIdx.x == 0) {
        if (threadIdx.x == 0) *a.flag_clear = 0;
        for (int q = threadIdx.x; q < n_sys; q += blockDim.x) a.sflag_clear[q] = 0;
    }
    const int cnt = rare_list ? *rare_n : tprefix[n_sys];
    for (int k = blockIdx.x; k < cnt; k += gridDim.x) {
        force_tile<W, MIXED, POT, LOG, true>(rare_list ? rare_list[k] : k, lds, FORCE_PASS);
        __syncthreads();
    }
}

// Per-system totals of the wave partials, in a fixed order.
__global__ __launch_bounds__(1024) void k_thermo_reduce(const SysDev *__restrict__ sys,
                                                        const int32_t *__restrict__ tprefix, int W,
                                                        const double *__restrict__ partials,
                                                        double *__restrict__ thermo,
                                                        double *__restrict__ log_rows, int n_sys,
                                                        int log_row, double timestep)
{
    __shared__ double red[3][1024];
    const int s = blockIdx.x;
    const SysDev &S = sys[s];
    const int64_t w0 = (int64_t)tprefix[s] * W;
    const int64_t w1 = (int64_t)tprefix[s + 1] * W;
    double k = 0, e = 0, v = 0;
    const int64_t st = blockDim.x;
    int64_t q = w0 + threadIdx.x;
    // four partials in flight, added in the same order as one at a time
    for (; q + 3 * st < w1; q += 4 * st) {
        double a[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 3; ++c) a[u][c] = partials[3 * (q + u * st) + c];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            k += a[u][0];
            e += a[u][1];
            v += a[u][2];
        }
    }
    for (; q < w1; q += st) {
        k += partials[3 * q + 0];
        e += partials[3 * q + 1];
        v += partials[3 * q + 2];
    }
    red[0][threadIdx.x] = k;
    red[1][threadIdx.x] = e;
    red[2][threadIdx.x] = v;
    __syncthreads();
    for (int m = blockDim.x / 2; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m) {
            red[0][threadIdx.x] += red[0][threadIdx.x + m];
            red[1][threadIdx.x] += red[1][threadIdx.x + m];
            red[2][threadIdx.x] += red[2][threadIdx.x + m];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double KE = red[0][0], PE = red[1][0], VW = red[2][0];
        const double dof = 3.0 * S.n_local - 3.0;
        const double T = dof > 0 ? 2.0 * KE / dof : 0.0;
        thermo[4 * s + 0] = KE;
        thermo[4 * s + 1] = PE;
        thermo[4 * s + 2] = VW;
        thermo[4 * s + 3] = T;
        if (log_row >= 0) {
            double *o = log_rows + ((int64_t)log_row * n_sys + s) * 5;
            o[0] = timestep;
            o[1] = KE;
            o[2] = PE;
            o[3] = VW;
            o[4] = T;
        }
    }
}

__global__ void k_set_flag(int32_t *flag, int32_t v) { *flag = v; }

// The local and total row counts of one system's device descriptor (values
// passed as arguments: no host memory is read when the launch runs).
__global__ void k_set_counts(SysDev *sys, int s, int32_t n_local, int32_t n_total)
{
    sys[s].n_local = n_local;
    sys[s].n_total = n_total;
}

__global__ void k_set_flags(int32_t *flag, int32_t *sflag, int n_sys, int32_t v)
{
    if (threadIdx.x == 0) *flag = v;
    for (int s = threadIdx.x; s < n_sys; s += blockDim.x) sflag[s] = v;
}

// Sets *flag and the flag of the particle's system when some local particle
// moved more than r_buff / 2 (minimum image) since the positions recorded at
// the last build.
__global__ void k_disp_check(const SysDev *__restrict__ sys, const int32_t *__restrict__ tprefix,
                             int n_sys, int tiles, const double4 *__restrict__ pos,
                             const double4 *__restrict__ xbuild, int32_t *flag, int32_t *sflag)
{
    const int g = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (g >= tiles) return;
    const int s = find_sys(tprefix, n_sys, g);
    const SysDev &S = sys[s];
    const int r = (g - S.tile0) * kTile + lane_id();
    if (r >= S.n_local) return;
    const int64_t i = S.row0 + r;
    const double4 x = pos[i], xb = xbuild[i];
    const double bx = min_image(x.x - xb.x, S.L[0], S.invL[0]);
    const double by = min_image(x.y - xb.y, S.L[1], S.invL[1]);
    const double bz = min_image(x.z - xb.z, S.L[2], S.invL[2]);
    if ((bx * bx + by * by) + bz * bz > S.disp2) {
        *flag = 1;
        sflag[s] = 1;
    }
}

// x += dt v (folded on periodic axes), then the displacement check since the
// last build (Sec. 4.2) sets the rebuild flags.
__device__ __forceinline__ void drift_and_check(const SysDev &S, int s, int64_t i, const double4 &v,
                                                double4 *__restrict__ pos, const double4 *__restrict__ xbuild,
                                                int32_t *flag, int32_t *sflag)
{
    double4 x = pos[i];
    x.x += S.dt * v.x;
    x.y += S.dt * v.y;
    x.z += S.dt * v.z;
    if (S.per[0]) x.x = fold(x.x, S.lo[0], S.L[0]);
    if (S.per[1]) x.y = fold(x.y, S.lo[1], S.L[1]);
    if (S.per[2]) x.z = fold(x.z, S.lo[2], S.L[2]);
    pos[i] = x;
    const double4 xb = xbuild[i];
    const double bx = min_image(x.x - xb.x, S.L[0], S.invL[0]);
    const double by = min_image(x.y - xb.y, S.L[1], S.invL[1]);
    const double bz = min_image(x.z - xb.z, S.L[2], S.invL[2]);
    if ((bx * bx + by * by) + bz * bz > S.disp2) {
        *flag = 1;
        sflag[s] = 1;
    }
}

// One half of a velocity-Verlet step over the local rows, from the force
// array of the last force evaluation (unit mass).  which = 0: v += dt/2 F,
// x += dt v (folded on periodic axes), and the displacement check since the
// last build (Sec. 4.2) sets the rebuild flags; which = 1: v += dt/2 F.
template <bool MIXED>
__global__ void k_half_step(const SysDev *__restrict__ sys, const int32_t *__restrict__ tprefix, int n_sys,
                            int tiles, double4 *__restrict__ pos, double4 *__restrict__ vel,
                            const void *__restrict__ force, int which, const double4 *__restrict__ xbuild,
                            int32_t *flag, int32_t *sflag, const double *__restrict__ thermostat,
                            double *__restrict__ khalf)
{
    const int g = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (g >= tiles) return;  // whole waves
    const int s = find_sys(tprefix, n_sys, g);
    const SysDev &S = sys[s];
    const int r = (g - S.tile0) * kTile + lane_id();
    const bool nvt = thermostat != nullptr && S.nvt_slot >= 0;
    if (nvt) {
        // Nose-Hoover halves; the first also leaves the tile's half-step
        // kinetic energy for the thermostat update
        const double xi_nh = thermostat[2 * S.nvt_slot];
        double kh = 0.0;
        if (r < S.n_local) {
            const int64_t i = S.row0 + r;
            double fx, fy, fz;
            if (MIXED) {
                const float4 f = reinterpret_cast<const float4 *>(force)[i];
                fx = f.x;
                fy = f.y;
                fz = f.z;
            } else {
                const double4 f = reinterpret_cast<const double4 *>(force)[i];
                fx = f.x;
                fy = f.y;
                fz = f.z;
            }
            double4 v = vel[i];
            if (which != 0) {
                const double d = 1.0 + S.hdt * xi_nh;
                v.x = (v.x + S.hdt * fx) / d;
                v.y = (v.y + S.hdt * fy) / d;
                v.z = (v.z + S.hdt * fz) / d;
                vel[i] = v;
            } else {
                v.x += S.hdt * (fx - xi_nh * v.x);
                v.y += S.hdt * (fy - xi_nh * v.y);
                v.z += S.hdt * (fz - xi_nh * v.z);
                vel[i] = v;
                kh = 0.5 * ((v.x * v.x + v.y * v.y) + v.z * v.z);
                drift_and_check(S, s, i, v, pos, xbuild, flag, sflag);
            }
        }
        if (which == 0 && khalf) {
            kh = wave_sum(kh);
            if (lane_id() == 0) khalf[g] = kh;
        }
        return;
    }
    if (r >= S.n_local) return;
    const int64_t i = S.row0 + r;
    double fx, fy, fz;
    if (MIXED) {
        const float4 f = reinterpret_cast<const float4 *>(force)[i];
        fx = f.x;
        fy = f.y;
        fz = f.z;
    } else {
        const double4 f = reinterpret_cast<const double4 *>(force)[i];
        fx = f.x;
        fy = f.y;
        fz = f.z;
    }
    double4 v = vel[i];
    v.x += S.hdt * fx;
    v.y += S.hdt * fy;
    v.z += S.hdt * fz;
    vel[i] = v;
    if (which != 0) return;
    drift_and_check(S, s, i, v, pos, xbuild, flag, sflag);
}

// Nose-Hoover update, one workgroup per system (the first system of each
// group does its group).
__global__ __launch_bounds__(kNvtSums) void k_nvt_update(const SysDev *__restrict__ sys,
                                                         const int32_t *__restrict__ tprefix, int n_sys, int w,
                                                         const double *__restrict__ khalf,
                                                         double *__restrict__ thermostat)
{
    __shared__ double red[kNvtSums];
    const int s = blockIdx.x;
    if (sys[s].nvt_slot != s) return;
    nvt_group_update(sys, tprefix, n_sys, w, khalf, thermostat, s, red, blockDim.x, threadIdx.x);
}

// ---------------------------------------------------------------------------

int force_row_over_read() { return kRowOverRead; }

int force_halo_entry_bytes(int pair) { return halo_entry_bytes(pair); }

size_t force_lds_bytes(int pair, int halo_cap, int nlist_cap)
{
    (void)nlist_cap;
    return (size_t)halo_entry_bytes(pair) * (size_t)(halo_cap > 1 ? halo_cap : 1);
}

template <int W, bool MIXED, int POT, bool LOG>
static void force_inst(const LaunchCtx &L, const ForceLaunch &F)
{
    if (L.tiles_local == 0) return;
    // the launch over rare tiles runs few workgroups: it stages up to the
    // whole halo list (at most kRareLds bytes), so that oversized halos are
    // read from LDS too
    const int rb = L.tiles_local < kRareGrid ? L.tiles_local : kRareGrid;
    int rare_lds_entries = (int)(kRareLds / (size_t)halo_entry_bytes(POT));
    rare_lds_entries = rare_lds_entries < L.halo_cap ? rare_lds_entries : L.halo_cap;
    rare_lds_entries = rare_lds_entries > L.halo_lds ? rare_lds_entries : L.halo_lds;
    const size_t rare_lds = force_lds_bytes(POT, rare_lds_entries, L.nlist_cap);
    // One launch of the second kind over every tile when the workgroups of
    // all tiles that hold local rows are resident at once: at most 16 waves
    // per CU (it takes up to 128 VGPRs) and as many workgroups as the CU's
    // 160 KB of LDS holds
    bool one = L.force_launch == kForceOne;
    if (L.force_launch == kForceAuto) {
        const int by_waves = 16 / W > 0 ? 16 / W : 1;
        const int by_lds = (int)((size_t)163840 / (rare_lds > 0 ? rare_lds : 1));
        const int per_cu = by_waves < by_lds ? by_waves : by_lds;
        one = L.busy_tiles <= 256 * per_cu;
    }
    if (one) {
        hipLaunchKernelGGL((k_force_rare<W, MIXED, POT, LOG>), dim3(rb), dim3(W * kWave), rare_lds, L.stream,
                           L.sys, L.tprefix_local, L.n_sys, L.nlist, L.nn, L.nlist_cap, L.halo, L.halo_n,
                           L.halo_cap, rare_lds_entries, L.prow, L.xbuild, L.partials, L.status,
                           (const int32_t *)nullptr, (const int32_t *)nullptr, F);
        return;
    }
    const size_t lds = force_lds_bytes(POT, L.halo_lds, L.nlist_cap);
    hipLaunchKernelGGL((k_force<W, MIXED, POT, LOG>), dim3(L.tiles_local), dim3(W * kWave), lds, L.stream,
                       L.sys, L.tprefix_local, L.n_sys, L.nlist, L.nn, L.nlist_cap, L.halo, L.halo_n,
                       L.halo_cap, L.halo_lds, L.prow, L.xbuild, L.partials, L.status,
                       L.rare_list, L.rare_n, F);
    hipLaunchKernelGGL((k_force_rare<W, MIXED, POT, LOG>), dim3(rb), dim3(W * kWave), rare_lds, L.stream, L.sys,
                       L.tprefix_local, L.n_sys, L.nlist, L.nn, L.nlist_cap, L.halo, L.halo_n, L.halo_cap,
                       rare_lds_entries, L.prow, L.xbuild, L.partials, L.status, L.rare_list,
                       L.rare_n, F);
}

// Lets every instantiation of the rare-tile kernel take kRareLds bytes of
// dynamic LDS (above the default limit).
template <int W, bool MIXED, int POT, bool LOG>
static hipError_t rare_attr()
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_force_rare<W, MIXED, POT, LOG>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRareLds);
}

template <int W>
static hipError_t rare_attr_w()
{
    const hipError_t es[8] = {rare_attr<W, true, PAIR_LJ, true>(),   rare_attr<W, true, PAIR_LJ, false>(),
                              rare_attr<W, true, PAIR_DPD, true>(),  rare_attr<W, true, PAIR_DPD, false>(),
                              rare_attr<W, false, PAIR_LJ, true>(),  rare_attr<W, false, PAIR_LJ, false>(),
                              rare_attr<W, false, PAIR_DPD, true>(), rare_attr<W, false, PAIR_DPD, false>()};
    for (hipError_t e : es)
        if (e != hipSuccess) return e;
    return hipSuccess;
}

hipError_t prepare_force()
{
    const hipError_t es[5] = {rare_attr_w<1>(), rare_attr_w<2>(), rare_attr_w<4>(), rare_attr_w<8>(),
                              rare_attr_w<16>()};
    for (hipError_t e : es)
        if (e != hipSuccess) return e;
    return hipSuccess;
}

template <int W, bool MIXED, int POT>
static void force_log(const LaunchCtx &L, const ForceLaunch &F)
{
    if (F.log) force_inst<W, MIXED, POT, true>(L, F);
    else force_inst<W, MIXED, POT, false>(L, F);
}

template <int W, bool MIXED>
static void force_pot(const LaunchCtx &L, const ForceLaunch &F)
{
    switch (F.pair) {
    case PAIR_LJ: force_log<W, MIXED, PAIR_LJ>(L, F); break;
    default: force_log<W, MIXED, PAIR_DPD>(L, F); break;
    }
}

template <int W>
static void force_prec(const LaunchCtx &L, const ForceLaunch &F)
{
    if (F.mixed) force_pot<W, true>(L, F);
    else force_pot<W, false>(L, F);
}

void launch_force(const LaunchCtx &L, const ForceLaunch &F, int w, int block)
{
    (void)block;
    switch (w) {
    case 1: force_prec<1>(L, F); break;
    case 2: force_prec<2>(L, F); break;
    case 4: force_prec<4>(L, F); break;
    case 8: force_prec<8>(L, F); break;
    default: force_prec<16>(L, F); break;
    }
}

void launch_thermo_reduce(const LaunchCtx &L, int w, int log_row, double timestep)
{
    hipLaunchKernelGGL(k_thermo_reduce, dim3(L.n_sys), dim3(1024), 0, L.stream, L.sys, L.tprefix_local, w,
                       L.partials, L.thermo, L.thermo_log, L.n_sys, log_row, timestep);
}

void launch_set_flag(const LaunchCtx &L, int32_t *flag, int32_t value)
{
    hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(1), 0, L.stream, flag, value);
}

void launch_set_counts(const LaunchCtx &L, int s, int32_t n_local, int32_t n_total)
{
    hipLaunchKernelGGL(k_set_counts, dim3(1), dim3(1), 0, L.stream, const_cast<SysDev *>(L.sys), s, n_local, n_total);
}

void launch_set_flags(const LaunchCtx &L, int32_t *flag, int32_t *sflag, int32_t value)
{
    hipLaunchKernelGGL(k_set_flags, dim3(1), dim3(256), 0, L.stream, flag, sflag, L.n_sys, value);
}

void launch_disp_check(const LaunchCtx &L, const double4 *pos, int32_t *flag, int32_t *sflag)
{
    const int threads = 256;
    const int blocks = (L.tiles_local * kWave + threads - 1) / threads;
    if (blocks == 0) return;
    hipLaunchKernelGGL(k_disp_check, dim3(blocks), dim3(threads), 0, L.stream, L.sys,
                       L.tprefix_local, L.n_sys, L.tiles_local, pos, L.xbuild, flag, sflag);
}

void launch_half_step(const LaunchCtx &L, double4 *pos, double4 *vel, const void *force, bool mixed, int which,
                      int32_t *flag, int32_t *sflag)
{
    const int threads = 256;
    const int blocks = (L.tiles_local * kWave + threads - 1) / threads;
    if (blocks == 0) return;
    const double *th = L.nvt ? L.thermostat : nullptr;
    double *kh = L.nvt ? L.khalf : nullptr;
    if (mixed)
        hipLaunchKernelGGL(k_half_step<true>, dim3(blocks), dim3(threads), 0, L.stream, L.sys, L.tprefix_local,
                           L.n_sys, L.tiles_local, pos, vel, force, which, L.xbuild, flag, sflag, th, kh);
    else
        hipLaunchKernelGGL(k_half_step<false>, dim3(blocks), dim3(threads), 0, L.stream, L.sys, L.tprefix_local,
                           L.n_sys, L.tiles_local, pos, vel, force, which, L.xbuild, flag, sflag, th, kh);
}

void launch_nvt_update(const LaunchCtx &L, int w)
{
    if (!L.nvt) return;
    hipLaunchKernelGGL(k_nvt_update, dim3(L.n_sys), dim3(kNvtSums), 0, L.stream, L.sys, L.tprefix_local, L.n_sys,
                       w, L.khalf, L.thermostat);
}


}  // namespace md
