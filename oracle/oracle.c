/*
 * oracle.c -- plain, slow, FP64 CPU reference for the single-GPU hot path of
 * domain-decomposed molecular dynamics (Glaser et al., "Strong scaling of
 * general-purpose molecular dynamics simulations on GPUs").
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the timed
 * CPU baseline of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU path; both sides are fed the same
 * seeded inputs and nothing else.
 *
 * Every quantity is computed from its plain definition, by brute force over
 * all particle pairs (O(N^2)), in IEEE double precision, compiled with FMA
 * contraction off.  Where the paper only names a model (LJ, DPD, FENE,
 * velocity Verlet) the textbook form is written out; the readings taken where
 * the paper is silent are listed next to each function.
 *
 * Conventions
 *   positions  (n,3) row-major doubles; a periodic box is [0, L) per axis.
 *   minimum image along a periodic axis: d -= L * rint(d / L)  (ties to even)
 *   "within r" means r^2 < r*r  (strict), with r^2 = (dx*dx + dy*dy) + dz*dz.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */

/* Minimum-image separation along periodic axes (Sec. 4.1: the usual minimum
 * image convention is used along every dimension that is not split). */
static void min_image(double d[3], const double *L, const int32_t *per)
{
    for (int a = 0; a < 3; ++a)
        if (per[a]) d[a] -= L[a] * rint(d[a] / L[a]);
}

static double norm2(const double d[3])
{
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* d = x_j - x_i, folded by the minimum image. */
static void separation(const double *pos, int64_t i, int64_t j, const double *L,
                       const int32_t *per, double d[3])
{
    for (int a = 0; a < 3; ++a) d[a] = pos[3 * j + a] - pos[3 * i + a];
    min_image(d, L, per);
}

ORC_API void orc_min_image(double *d, const double *L, const int32_t *per)
{
    min_image(d, L, per);
}

/* Fold positions into [0, L): one period is added or removed, then a value
 * that rounded up to L is folded once more.  Valid while a particle moves
 * less than one box length per step. */
static double wrap1(double x, double L)
{
    if (x >= L) x -= L;
    else if (x < 0.0) x += L;
    if (x >= L) x -= L;
    return x;
}

ORC_API void orc_wrap(int64_t n, double *pos, const double *L)
{
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) pos[3 * i + a] = wrap1(pos[3 * i + a], L[a]);
}

static int is_excluded(int64_t i, int64_t j, const int64_t *excl_off, const int32_t *excl_idx)
{
    if (!excl_off) return 0;
    for (int64_t k = excl_off[i]; k < excl_off[i + 1]; ++k)
        if (excl_idx[k] == j) return 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Verlet neighbour sets (Sec. 4.2 and Sec. 5.1, Fig. 4)                      */
/*   N_i = { j != i : |x_j - x_i|^2 < (r_cut + r_buff)^2 }, minus excluded    */
/*   (bonded) partners.  The neighbour radius is cut-off plus buffer; the     */
/*   comparison in Fig. 4 against the cut-off alone is read as that radius.   */
/* ------------------------------------------------------------------------ */

ORC_API int64_t orc_neighbor_counts(int64_t n, const double *pos, const double *L,
                                    const int32_t *per, double r_cut, double r_buff,
                                    const int64_t *which, int64_t m,
                                    const int64_t *excl_off, const int32_t *excl_idx,
                                    int64_t *counts)
{
    const double rl = r_cut + r_buff;
    const double rl2 = rl * rl;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int64_t q = 0; q < m; ++q) {
        const int64_t i = which ? which[q] : q;
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            separation(pos, i, j, L, per, d);
            if (norm2(d) < rl2 && !is_excluded(i, j, excl_off, excl_idx)) ++c;
        }
        counts[q] = c;
        total += c;
    }
    return total;
}

/* Neighbour indices of each requested particle, ascending, packed at
 * offsets[q] (offsets from the counts above). */
ORC_API void orc_neighbor_lists(int64_t n, const double *pos, const double *L,
                                const int32_t *per, double r_cut, double r_buff,
                                const int64_t *which, int64_t m,
                                const int64_t *excl_off, const int32_t *excl_idx,
                                const int64_t *offsets, int32_t *idx)
{
    const double rl = r_cut + r_buff;
    const double rl2 = rl * rl;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < m; ++q) {
        const int64_t i = which ? which[q] : q;
        int64_t k = offsets[q];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            separation(pos, i, j, L, per, d);
            if (norm2(d) < rl2 && !is_excluded(i, j, excl_off, excl_idx)) idx[k++] = (int32_t)j;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers for DPD (Sec. 9: the pair random force is    */
/* seeded with global particle IDs).  Philox4x32-10 as published by Salmon,  */
/* Moraes, Dror and Shaw (SC'11): ten rounds of two 32x32->64 multiplies     */
/* with a Weyl-sequence key schedule.                                       */
/* ------------------------------------------------------------------------ */

static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

ORC_API void orc_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof(c));
}

/* Pair random variate theta_ij: uniform on [-sqrt3, sqrt3) (unit variance),
 * symmetric in (i, j).  Counter = (min tag, max tag, 0, 0), key = (seed,
 * low 32 bits of the timestep); u = (first word >> 8) * 2^-24. */
ORC_API double orc_dpd_theta(uint32_t tag_i, uint32_t tag_j, uint32_t seed, uint64_t timestep)
{
    const uint32_t a = tag_i < tag_j ? tag_i : tag_j;
    const uint32_t b = tag_i < tag_j ? tag_j : tag_i;
    const uint32_t ctr[4] = {a, b, 0u, 0u};
    const uint32_t key[2] = {seed, (uint32_t)timestep};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    const double u = (double)(out[0] >> 8) * (1.0 / 16777216.0);
    return sqrt(3.0) * (2.0 * u - 1.0);
}

/* ------------------------------------------------------------------------ */
/* Pair forces, brute force over all j (Sec. 3 lists the LJ and DPD pair     */
/* potentials; the paper gives no formulas, so the textbook forms are used). */
/*                                                                           */
/* kind 0  LJ   prm = {eps, sigma, r_cut}                                    */
/*         V(r) = 4 eps [(s/r)^12 - (s/r)^6]; force truncated at r_cut;      */
/*         energy reported shifted, V(r) - V(r_cut).                         */
/* kind 1  WCA  prm = {eps, sigma}: LJ cut at 2^(1/6) sigma, shifted up by   */
/*         eps (the purely repulsive bead-bead interaction).                 */
/* kind 2  DPD  prm = {A, gamma, kT, r_cut, dt, seed} (Groot-Warren form):   */
/*         F_ij = [A w - gamma w^2 (rhat.v_ij) + sigma w theta_ij/sqrt(dt)]  */
/*                rhat,  w = 1 - r/r_cut, sigma^2 = 2 gamma kT,             */
/*         pair energy (A r_cut / 2) w^2.                                    */
/* Outputs per requested particle: F (force on i), u (half of its pair       */
/* energies), w (half of sum r_ij . F_ij), nc (pairs inside the cut-off).    */
/* ------------------------------------------------------------------------ */

ORC_API int orc_pair_forces(int kind, int64_t n, const double *pos, const double *vel,
                            const int32_t *tag, const double *L, const int32_t *per,
                            const double *prm, uint64_t timestep,
                            const int64_t *which, int64_t m,
                            const int64_t *excl_off, const int32_t *excl_idx,
                            double *F, double *u, double *w, int64_t *nc)
{
    double eps = 0, sig = 1, rc = 0, shift = 0;
    double A = 0, gam = 0, kT = 0, dt = 1;
    uint32_t seed = 0;
    if (kind == 0) {
        eps = prm[0]; sig = prm[1]; rc = prm[2];
        const double s6 = pow(sig / rc, 6.0);
        shift = 4.0 * eps * (s6 * s6 - s6);
    } else if (kind == 1) {
        eps = prm[0]; sig = prm[1]; rc = pow(2.0, 1.0 / 6.0) * sig;
        shift = -eps; /* V - V(rc) with V(rc) = -eps gives V + eps */
    } else if (kind == 2) {
        A = prm[0]; gam = prm[1]; kT = prm[2]; rc = prm[3]; dt = prm[4];
        seed = (uint32_t)prm[5];
    } else {
        return -1;
    }
    const double rc2 = rc * rc;
    const double sigma_r = sqrt(2.0 * gam * kT);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t q = 0; q < m; ++q) {
        const int64_t i = which ? which[q] : q;
        double fx = 0, fy = 0, fz = 0, ui = 0, wi = 0;
        int64_t cnt = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            /* r_ij = x_i - x_j */
            for (int a = 0; a < 3; ++a) d[a] = pos[3 * i + a] - pos[3 * j + a];
            min_image(d, L, per);
            const double r2 = norm2(d);
            if (!(r2 < rc2)) continue;
            if (is_excluded(i, j, excl_off, excl_idx)) continue;
            ++cnt;
            double fr2; /* force magnitude divided by r: F_ij = fr2 * r_ij */
            double e;
            if (kind == 0 || kind == 1) {
                const double sr2 = sig * sig / r2;
                const double s6 = sr2 * sr2 * sr2;
                fr2 = 24.0 * eps * (2.0 * s6 * s6 - s6) / r2;
                e = 4.0 * eps * (s6 * s6 - s6) - shift;
            } else {
                if (r2 == 0.0) continue;
                const double r = sqrt(r2);
                const double wr = 1.0 - r / rc;
                double rv = 0;
                for (int a = 0; a < 3; ++a) rv += d[a] * (vel[3 * i + a] - vel[3 * j + a]);
                const double rhat_v = rv / r;
                const double th = orc_dpd_theta((uint32_t)tag[i], (uint32_t)tag[j], seed, timestep);
                const double mag = A * wr - gam * wr * wr * rhat_v + sigma_r * wr * th / sqrt(dt);
                fr2 = mag / r;
                e = 0.5 * A * rc * wr * wr;
            }
            if (!isfinite(fr2)) bad = 1;
            fx += fr2 * d[0];
            fy += fr2 * d[1];
            fz += fr2 * d[2];
            ui += 0.5 * e;
            wi += 0.5 * fr2 * r2;
        }
        F[3 * q + 0] = fx;
        F[3 * q + 1] = fy;
        F[3 * q + 2] = fz;
        if (u) u[q] = ui;
        if (w) w[q] = wi;
        if (nc) nc[q] = cnt;
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Bond forces (Sec. 3 lists FENE bonds; Sec. 4.3.4: a bond is an unordered  */
/* pair of particle IDs with a type).  prm = {K, R0, eps, sigma, with_wca}.  */
/*   U_FENE(r) = -1/2 K R0^2 ln(1 - (r/R0)^2),                               */
/*   plus, when with_wca != 0, the WCA term of kind 1 above.                 */
/* Forces and energies are accumulated (+=) into F, u, w over all n; each    */
/* particle of a bond receives half of its energy and virial.  Returns the   */
/* number of bonds stretched to r >= R0 (their terms are skipped).           */
/* ------------------------------------------------------------------------ */

ORC_API int64_t orc_bond_forces(int64_t n, const double *pos, const double *L, const int32_t *per,
                                int64_t nb, const int32_t *bonds, const double *prm,
                                double *F, double *u, double *w)
{
    (void)n;
    const double K = prm[0], R0 = prm[1], eps = prm[2], sig = prm[3];
    const int with_wca = prm[4] != 0.0;
    const double R02 = R0 * R0;
    const double rwca2 = pow(2.0, 1.0 / 3.0) * sig * sig;
    int64_t stretched = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t i = bonds[2 * b], j = bonds[2 * b + 1];
        double d[3];
        for (int a = 0; a < 3; ++a) d[a] = pos[3 * i + a] - pos[3 * j + a];
        min_image(d, L, per);
        const double r2 = norm2(d);
        if (!(r2 < R02)) {
            ++stretched;
            continue;
        }
        const double g = 1.0 - r2 / R02;
        double fr2 = -K / g;
        double e = -0.5 * K * R02 * log(g);
        if (with_wca && r2 < rwca2) {
            const double sr2 = sig * sig / r2;
            const double s6 = sr2 * sr2 * sr2;
            fr2 += 24.0 * eps * (2.0 * s6 * s6 - s6) / r2;
            e += 4.0 * eps * (s6 * s6 - s6) + eps;
        }
        for (int a = 0; a < 3; ++a) {
            F[3 * i + a] += fr2 * d[a];
            F[3 * j + a] -= fr2 * d[a];
        }
        if (u) {
            u[i] += 0.5 * e;
            u[j] += 0.5 * e;
        }
        if (w) {
            w[i] += 0.5 * fr2 * r2;
            w[j] += 0.5 * fr2 * r2;
        }
    }
    return stretched;
}

/* ------------------------------------------------------------------------ */
/* Thermodynamic sums (Sec. 4.3.3 names kinetic energy and virial as the     */
/* global reductions).  out = {KE, PE, W, T}: KE = 1/2 sum v^2 (unit mass),  */
/* PE = sum u_i, W = sum w_i, T = 2 KE / (3n - 3).  Neumaier-compensated.    */
/* ------------------------------------------------------------------------ */

typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double x)
{
    const double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}

ORC_API void orc_thermo(int64_t n, const double *vel, const double *u, const double *w, double *out)
{
    ksum ke = {0, 0}, pe = {0, 0}, vir = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) kadd(&ke, 0.5 * vel[3 * i + a] * vel[3 * i + a]);
        if (u) kadd(&pe, u[i]);
        if (w) kadd(&vir, w[i]);
    }
    out[0] = ke.s + ke.c;
    out[1] = pe.s + pe.c;
    out[2] = vir.s + vir.c;
    out[3] = n > 1 ? 2.0 * out[0] / (double)(3 * n - 3) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Velocity-Verlet NVE (Sec. 3: NVE uses the velocity-Verlet update).        */
/*   v += dt/2 F;  x += dt v;  fold x into the box;  F <- F(x, v, t+1);      */
/*   v += dt/2 F.   Unit mass.  For DPD the new force sees the half-kicked   */
/*   velocity.  Polymer systems use WCA between all pairs plus FENE bonds.   */
/* model: 0 LJ (pair prm {eps, sigma, r_cut}), 1 polymer (pair prm {eps,     */
/* sigma}, bond prm {K, R0}), 2 DPD (pair prm as kind 2).                    */
/* F holds F(x(t0), v(t0), t0) on entry if have_force != 0, and the final    */
/* force on return.  thermo (nsteps+1 rows of {KE, PE, W, T}) may be NULL.   */
/* Returns 0, or 1 if a force became non-finite, or 2 if a bond broke.       */
/* ------------------------------------------------------------------------ */

static int total_forces(int model, int64_t n, const double *pos, const double *vel,
                        const int32_t *tag, const double *L, const double *pprm,
                        int64_t nb, const int32_t *bonds, const double *bprm, uint64_t t,
                        double *F, double *u, double *w)
{
    static const int32_t per[3] = {1, 1, 1};
    const int kind = model == 0 ? 0 : (model == 1 ? 1 : 2);
    int rc = orc_pair_forces(kind, n, pos, vel, tag, L, per, pprm, t, NULL, n, NULL, NULL,
                             F, u, w, NULL);
    if (rc) return 1;
    if (model == 1 && nb > 0) {
        const double fene[5] = {bprm[0], bprm[1], 0.0, 1.0, 0.0};
        if (orc_bond_forces(n, pos, L, per, nb, bonds, fene, F, u, w) != 0) return 2;
    }
    return 0;
}

ORC_API int orc_run_nve(int model, int64_t n, double *pos, double *vel, const int32_t *tag,
                        const double *L, const double *pprm, int64_t nb, const int32_t *bonds,
                        const double *bprm, double dt, uint64_t t0, int64_t nsteps,
                        double *F, int have_force, double *thermo)
{
    double *u = (double *)calloc((size_t)n, sizeof(double));
    double *w = (double *)calloc((size_t)n, sizeof(double));
    int status = 0;
    const double hdt = 0.5 * dt;
    if (!have_force) status = total_forces(model, n, pos, vel, tag, L, pprm, nb, bonds, bprm, t0, F, u, w);
    else if (thermo) status = total_forces(model, n, pos, vel, tag, L, pprm, nb, bonds, bprm, t0, F, u, w);
    if (thermo) orc_thermo(n, vel, u, w, thermo);
    for (int64_t s = 0; s < nsteps && status == 0; ++s) {
        for (int64_t k = 0; k < 3 * n; ++k) vel[k] = vel[k] + hdt * F[k];
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a)
                pos[3 * i + a] = wrap1(pos[3 * i + a] + dt * vel[3 * i + a], L[a]);
        status = total_forces(model, n, pos, vel, tag, L, pprm, nb, bonds, bprm,
                              t0 + (uint64_t)s + 1u, F, u, w);
        for (int64_t k = 0; k < 3 * n; ++k) vel[k] = vel[k] + hdt * F[k];
        if (thermo) orc_thermo(n, vel, u, w, thermo + 4 * (s + 1));
    }
    free(u);
    free(w);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Nose-Hoover NVT (Sec. 6.1: the weak-scaling LJ runs use a Nose-Hoover     */
/* thermostat that is not fully symplectic and needs one global kinetic-     */
/* energy sum per step).  The paper gives no equations; the reading taken:   */
/* the flow  dx/dt = v,  dv/dt = F - xi v,  dxi/dt = (T/T0 - 1) / tau^2,      */
/* T = 2 KE / g with g = 3n - 3, advanced per step of length h as            */
/*   v(t+h/2) = v(t) + h/2 (F(t) - xi(t) v(t))                               */
/*   x(t+h)   = x(t) + h v(t+h/2), folded into the box                       */
/*   xi(t+h)  = xi(t) + h/tau^2 (T(t+h/2)/T0 - 1)   (the one KE sum)         */
/*   F(t+h)   = F(x(t+h), ...)                                               */
/*   v(t+h)   = (v(t+h/2) + h/2 F(t+h)) / (1 + h/2 xi(t+h))                  */
/* and eta(t+h) = eta(t) + h/2 (xi(t) + xi(t+h)) (trapezoid), deta/dt = xi.   */
/* The flow conserves KE + PE + g T0 (tau^2 xi^2 / 2 + eta).                  */
/* nvt = {T0, tau}; xi_eta = {xi, eta} in and out; thermo as orc_run_nve;     */
/* ext (nsteps+1 rows of {xi, eta}) may be NULL.  Forces are computed at the  */
/* start.  Returns as orc_run_nve.                                           */
/* ------------------------------------------------------------------------ */

ORC_API int orc_run_nvt(int model, int64_t n, double *pos, double *vel, const int32_t *tag,
                        const double *L, const double *pprm, int64_t nb, const int32_t *bonds,
                        const double *bprm, double dt, uint64_t t0, int64_t nsteps,
                        const double *nvt, double *xi_eta, double *F, double *thermo, double *ext)
{
    double *u = (double *)calloc((size_t)n, sizeof(double));
    double *w = (double *)calloc((size_t)n, sizeof(double));
    const double hdt = 0.5 * dt, T0 = nvt[0], tau = nvt[1];
    const double g = (double)(3 * n - 3);
    double xi = xi_eta[0], eta = xi_eta[1];
    int status = total_forces(model, n, pos, vel, tag, L, pprm, nb, bonds, bprm, t0, F, u, w);
    if (thermo) orc_thermo(n, vel, u, w, thermo);
    if (ext) {
        ext[0] = xi;
        ext[1] = eta;
    }
    for (int64_t s = 0; s < nsteps && status == 0; ++s) {
        for (int64_t k = 0; k < 3 * n; ++k) vel[k] = vel[k] + hdt * (F[k] - xi * vel[k]);
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a)
                pos[3 * i + a] = wrap1(pos[3 * i + a] + dt * vel[3 * i + a], L[a]);
        double half[4];
        orc_thermo(n, vel, NULL, NULL, half);
        const double T_half = 2.0 * half[0] / g;
        const double xi_new = xi + dt / (tau * tau) * (T_half / T0 - 1.0);
        eta = eta + hdt * (xi + xi_new);
        xi = xi_new;
        status = total_forces(model, n, pos, vel, tag, L, pprm, nb, bonds, bprm,
                              t0 + (uint64_t)s + 1u, F, u, w);
        const double d = 1.0 + hdt * xi;
        for (int64_t k = 0; k < 3 * n; ++k) vel[k] = (vel[k] + hdt * F[k]) / d;
        if (thermo) orc_thermo(n, vel, u, w, thermo + 4 * (s + 1));
        if (ext) {
            ext[2 * (s + 1)] = xi;
            ext[2 * (s + 1) + 1] = eta;
        }
    }
    xi_eta[0] = xi;
    xi_eta[1] = eta;
    free(u);
    free(w);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Cell list (Sec. 4.3.3 mentions the cell list; Fig. 4 step 1 looks up the  */
/* cell neighbours).  bins_a = floor(L_a / r_list), reduced while a cell     */
/* would be narrower than r_list; cell of x = floor((x - lo) * (bins / L)),  */
/* clamped to [0, bins-1]; id = (cz * by + cy) * bx + cx.  The list is the    */
/* stable counting sort of particle indices by cell id.                      */
/* ------------------------------------------------------------------------ */

ORC_API void orc_cell_bins(const double *L, double r_list, int32_t *bins)
{
    for (int a = 0; a < 3; ++a) {
        int64_t b = (int64_t)floor(L[a] / r_list);
        while (b > 1 && L[a] / (double)b < r_list) --b;
        if (b < 1) b = 1;
        bins[a] = (int32_t)b;
    }
}

ORC_API void orc_cell_list(int64_t n, const double *pos, const double *lo, const double *L,
                           const int32_t *bins, int32_t *cell_of, int32_t *cell_start,
                           int32_t *cell_idx)
{
    const int64_t ncell = (int64_t)bins[0] * bins[1] * bins[2];
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            const double s = (double)bins[a] / L[a];
            int64_t v = (int64_t)floor((pos[3 * i + a] - lo[a]) * s);
            if (v < 0) v = 0;
            if (v > bins[a] - 1) v = bins[a] - 1;
            c[a] = v;
        }
        cell_of[i] = (int32_t)((c[2] * bins[1] + c[1]) * bins[0] + c[0]);
    }
    for (int64_t c = 0; c <= ncell; ++c) cell_start[c] = 0;
    for (int64_t i = 0; i < n; ++i) cell_start[cell_of[i] + 1]++;
    for (int64_t c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncell > 0 ? ncell : 1));
    for (int64_t c = 0; c < ncell; ++c) fill[c] = cell_start[c];
    for (int64_t i = 0; i < n; ++i) cell_idx[fill[cell_of[i]]++] = (int32_t)i;
    free(fill);
}

/* ------------------------------------------------------------------------ */
/* Spatial (Morton) order.  Not described by the paper; used to keep         */
/* neighbouring particles close in memory.  q_a = floor(x_a * 1024 / L_a)    */
/* clamped to [0, 1023]; key bit 3b+a holds bit b of q_a (a = x, y, z).      */
/* The order is the stable sort of the keys.                                 */
/* ------------------------------------------------------------------------ */

ORC_API void orc_morton_keys(int64_t n, const double *pos, const double *L, uint32_t *keys)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t q[3];
        for (int a = 0; a < 3; ++a) {
            const double s = 1024.0 / L[a];
            int64_t v = (int64_t)floor(pos[3 * i + a] * s);
            if (v < 0) v = 0;
            if (v > 1023) v = 1023;
            q[a] = (uint32_t)v;
        }
        uint32_t k = 0;
        for (int b = 0; b < 10; ++b)
            for (int a = 0; a < 3; ++a) k |= ((q[a] >> b) & 1u) << (3 * b + a);
        keys[i] = k;
    }
}

typedef struct { uint32_t key; int32_t idx; } kv;
static int kv_cmp(const void *pa, const void *pb)
{
    const kv *a = (const kv *)pa, *b = (const kv *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

ORC_API void orc_stable_order(int64_t n, const uint32_t *keys, int32_t *order)
{
    kv *t = (kv *)malloc(sizeof(kv) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        t[i].key = keys[i];
        t[i].idx = (int32_t)i;
    }
    qsort(t, (size_t)n, sizeof(kv), kv_cmp);
    for (int64_t i = 0; i < n; ++i) order[i] = t[i].idx;
    free(t);
}

/* ------------------------------------------------------------------------ */
/* Ghost layer (Sec. 4.2, Fig. 1: width r_cut + r_buff; Sec. 4.3.2, Fig. 2:  */
/* one flag per neighbouring direction, entries ordered by destination).    */
/* A local particle goes to direction d in {-1,0,1}^3 \ {0} when, on every   */
/* axis where d_a != 0, it lies within `width` of that face:                 */
/*   d_a = +1 : x_a >= hi_a - width        d_a = -1 : x_a < lo_a + width.    */
/* Direction index: (dz+1)*9 + (dy+1)*3 + (dx+1), with the centre (13)       */
/* removed, giving 0..25.  The send list is ordered by direction, then by    */
/* ascending particle index.                                                 */
/* ------------------------------------------------------------------------ */

static int dir_index(int dx, int dy, int dz)
{
    const int k = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
    return k < 13 ? k : k - 1;
}

ORC_API void orc_ghost_masks(int64_t n, const double *pos, const double *lo, const double *hi,
                             double width, uint32_t *mask)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t m = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dx == 0 && dy == 0 && dz == 0) continue;
                    const int d[3] = {dx, dy, dz};
                    int ok = 1;
                    for (int a = 0; a < 3; ++a) {
                        const double x = pos[3 * i + a];
                        if (d[a] == 1 && !(x >= hi[a] - width)) ok = 0;
                        if (d[a] == -1 && !(x < lo[a] + width)) ok = 0;
                    }
                    if (ok) m |= 1u << dir_index(dx, dy, dz);
                }
        mask[i] = m;
    }
}

ORC_API int64_t orc_ghost_list(int64_t n, const uint32_t *mask, int32_t *counts, int32_t *offsets,
                               int32_t *idx)
{
    int64_t k = 0;
    for (int d = 0; d < 26; ++d) {
        offsets[d] = (int32_t)k;
        for (int64_t i = 0; i < n; ++i)
            if (mask[i] & (1u << d)) idx[k++] = (int32_t)i;
        counts[d] = (int32_t)(k - offsets[d]);
    }
    return k;
}

/* Brute-force receive set of one subdomain [lo, hi) of a periodic box: every
 * particle not owned by `self` that has an image inside [lo - width, hi +
 * width).  Writes its index and that image, in ascending index order.  With
 * at least three subdomains per axis the image is unique. */
ORC_API int64_t orc_ghost_receive(int64_t n, const double *pos, const int32_t *owner, int32_t self,
                                  const double *L, const double *lo, const double *hi,
                                  double width, int32_t *idx, double *img, int64_t cap)
{
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (owner[i] == self) continue;
        for (int nz = -1; nz <= 1; ++nz)
            for (int ny = -1; ny <= 1; ++ny)
                for (int nx = -1; nx <= 1; ++nx) {
                    const int s[3] = {nx, ny, nz};
                    double x[3];
                    int in = 1;
                    for (int a = 0; a < 3; ++a) {
                        x[a] = pos[3 * i + a] + (double)s[a] * L[a];
                        if (!(x[a] >= lo[a] - width && x[a] < hi[a] + width)) in = 0;
                    }
                    if (!in) continue;
                    if (k < cap) {
                        idx[k] = (int32_t)i;
                        for (int a = 0; a < 3; ++a) img[3 * k + a] = x[a];
                    }
                    ++k;
                }
    }
    return k;
}
