/*
 * hoomd_mi355x.h -- C ABI of the single-GPU molecular-dynamics hot path for
 * AMD MI355X (gfx950): cell list, Verlet neighbour list, LJ / WCA / DPD pair
 * forces, FENE+WCA bonds, velocity-Verlet NVE, and ghost-layer selection with
 * pack / unpack for one subdomain.
 *
 * The operations follow the statement of the problem in Glaser et al.,
 * "Strong scaling of general-purpose molecular dynamics simulations on GPUs"
 * (HOOMD-blue 1.0 with domain decomposition):
 *   - short-range pair forces with a cut-off r_cut and a Verlet buffer
 *     r_buff whose sum is the neighbour radius and the ghost width
 *     (Sec. 4.2, Fig. 1);
 *   - the neighbour list is rebuilt when a particle has moved more than
 *     r_buff / 2 since the last build (Sec. 4.2);
 *   - neighbour list and forces with w cooperating lanes per particle and a
 *     compacting prefix sum (Sec. 5.1, Fig. 4), tuned at run time (Sec. 5.2);
 *   - a bond is an unordered pair of particle IDs (Sec. 4.3.4);
 *   - ghosts are selected by a per-direction bitfield, ordered by
 *     destination, gathered into a send buffer, and appended after the local
 *     particles (Sec. 4.3.2, Fig. 2); DPD ghosts carry velocities and IDs
 *     (Sec. 9);
 *   - the integrator is NVE velocity Verlet (Sec. 3).
 *
 * Memory ownership.  The caller allocates and owns every device buffer: the
 * particle arrays and one workspace block sized by hoomd_workspace_bytes().
 * The library borrows the pointers for the life of the context, never
 * allocates or frees device memory, and never aborts.  All work is queued
 * asynchronously on the stream given to hoomd_init(); only the calls marked
 * "synchronises" wait for the device.  A context is not thread-safe; use one
 * context per stream.
 *
 * Particle layout (all device pointers, n_cap rows, 64-bit aligned):
 *   pos    double[n_cap][4]  x, y, z, w.  w is carried along and ignored.
 *   vel    double[n_cap][4]  vx, vy, vz, w.  Unit mass.
 *   force  float[n_cap][4] (HOOMD_MIXED) or double[n_cap][4] (HOOMD_FP64):
 *          fx, fy, fz, and the particle's pair + bond energy.
 *   tag    int32[n_cap]      identity of each particle (0..n-1 per system).
 * Rows [0, n_local) are the particles the library integrates; rows
 * [n_local, n_local + n_ghost) hold ghosts appended by unpack_ghosts().
 * A spatial sort permutes rows of pos, vel, force and tag together; tags
 * keep track of identity.
 *
 * Positions of a periodic axis lie in [lo, lo + L); after each drift a
 * coordinate is folded once: x >= hi -> x - L, else x < lo -> x + L, and a
 * value that rounded up to hi is folded again.
 */
#ifndef HOOMD_MI355X_H
#define HOOMD_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hoomd_ctx hoomd_ctx;

/* Return codes.  Codes >= HOOMD_E_NLIST_OVERFLOW are detected on the device,
 * latched in a status word and reported by hoomd_sync_status(). */
typedef enum {
    HOOMD_OK = 0,
    HOOMD_E_ARG = 1,             /* invalid argument; nothing was queued    */
    HOOMD_E_DEVICE = 2,          /* a HIP runtime call failed               */
    HOOMD_E_WORKSPACE = 3,       /* workspace smaller than required         */
    HOOMD_E_STATE = 4,           /* call not valid in the context's state   */
    HOOMD_E_NLIST_OVERFLOW = 5,  /* a neighbour row exceeded nlist_cap      */
    HOOMD_E_CELL_OVERFLOW = 6,   /* a cell held more than cell_cap members  */
    HOOMD_E_GHOST_OVERFLOW = 7,  /* send list or buffer capacity exceeded   */
    HOOMD_E_BOND_STRETCH = 8,    /* a FENE bond reached r >= R0             */
    HOOMD_E_NAN = 9,             /* a non-finite force or position          */
    HOOMD_E_DANGEROUS_BUILD = 10,/* rebuild found a particle beyond r_buff/2
                                    when the check period is > 1            */
    HOOMD_E_HALO_OVERFLOW = 11,  /* a 64-row tile needs more halo entries
                                    than halo_cap (or its cell box is too
                                    large); Morton-sorted rows avoid it      */
    HOOMD_E_BOND_GHOST = 12      /* a bond partner is neither a local particle
                                    nor a ghost, a bond would span more than
                                    neighbouring subdomains, or the bond rank
                                    table was not set up (Sec. 4.3.4)       */
} hoomd_status;

/* Arithmetic of the pair and bond terms.  Positions, velocities, the
 * integrator and every energy / virial reduction are FP64 in both modes. */
enum { HOOMD_FP64 = 0, HOOMD_MIXED = 1 };

/* Pair potential of a system (the paper's Sec. 3 names LJ and DPD; WCA is the
 * bead-bead repulsion of bead-spring polymers).
 *   LJ : V = 4 eps [(s/r)^12 - (s/r)^6] for r < r_cut, force truncated,
 *        energy shifted by -V(r_cut).
 *   WCA: LJ cut at 2^(1/6) sigma and shifted up by eps (r_cut is ignored).
 *   DPD: F = [A w - gamma w^2 (rhat.v_ij) + sqrt(2 gamma kT) w theta/sqrt(dt)]
 *        rhat with w = 1 - r/r_cut; theta from Philox4x32-10 with counter
 *        (min tag, max tag, 0, 0) and key (seed, timestep), mapped to a
 *        uniform variate of unit variance; pair energy (A r_cut / 2) w^2. */
enum { HOOMD_PAIR_LJ = 0, HOOMD_PAIR_WCA = 1, HOOMD_PAIR_DPD = 2 };

typedef struct {
    int32_t precision;     /* HOOMD_FP64 or HOOMD_MIXED                      */
    int32_t pair;          /* HOOMD_PAIR_*                                  */
    double r_cut;          /* pair cut-off (LJ, DPD)                        */
    double r_buff;         /* Verlet buffer; list radius r_cut + r_buff      */
    double dt;             /* time step                                      */
    double eps, sigma;     /* LJ / WCA parameters                            */
    double dpd_A, dpd_gamma, dpd_kT;
    uint32_t dpd_seed;
    int32_t bond_cap;      /* max bonds per particle (0 = no bonds)          */
    double fene_K, fene_R0;/* FENE + WCA(eps, sigma) bond term              */
    int32_t nlist_cap;     /* neighbour row capacity (entries per particle)  */
    int32_t cell_cap;      /* cell capacity (0 = derived from the density)   */
    int32_t halo_cap;      /* halo list entries per 64-row tile, <= 65535
                              (0 = derived: from the density when
                              sort_period > 0, else 8192).  The force pass
                              stages up to about 1.25x the expected halo in
                              LDS and reads any further entries from global
                              memory, so this bounds memory, not speed      */
    int32_t sort_period;   /* Morton sort every this many steps (0 = never)  */
    int32_t check_period;  /* step() checks displacements on every k-th step
                              counted from the last build (0 or 1 = every
                              step; equal in all systems).  With k > 1 a
                              rebuild found at the first check after a build
                              latches HOOMD_E_DANGEROUS_BUILD: a particle may
                              have passed r_buff/2 before it was seen
                              (Sec. 4.2, Sec. 6.1)                          */
    int32_t tpp_nlist;     /* lanes per particle of the neighbour-list build:
                              0 or the fixed value hoomd_autotune() reports
                              (anything else is HOOMD_E_ARG)               */
    int32_t tpp_force;     /* lanes per particle, forces: 1, 2, 4, 8 or 16
                              (0 = chosen from the system size; hoomd_autotune
                              times the candidates) (Sec. 5.1, 5.2)         */
    int32_t block_nlist;   /* threads per workgroup of the build: 0 or the
                              value hoomd_autotune() reports                */
    int32_t block_force;   /* threads per workgroup of the force pass: 0 or
                              64 * tpp_force (one 64-row tile each)         */
    int32_t use_graph;     /* 1: step() replays captured pairs of middle steps
                              (HIP graph, captured once per context)          */
    int32_t tune_period;   /* > 0: step() re-runs the autotuner at its first
                              call once this many steps have passed since the
                              last scan, or after the ghost count changed
                              (Sec. 5.2); 0: tune only on request.  Equal in
                              all systems                                    */
    int32_t integrator;    /* HOOMD_NVE or HOOMD_NVT (Sec. 6.1)              */
    int32_t nvt_group;     /* NVT: 0 = a thermostat of its own; k > 0 = one
                              thermostat shared by every system with group
                              k, over their summed kinetic energy (the
                              subdomains of one box; equal dt, nvt_T0 and
                              nvt_tau required)                              */
    double nvt_T0;         /* NVT: set temperature (> 0)                     */
    double nvt_tau;        /* NVT: coupling time (> 0)                       */
    int32_t force_launch;  /* force pass (equal in all systems):
                              HOOMD_FORCE_AUTO, _SPLIT or _ONE               */
    int32_t pad_;
} hoomd_params;

/* Launches of the force pass.  SPLIT: a launch over the tiles whose halo fits
 * the LDS stage of a workgroup sized for full occupancy, then a small launch
 * over the rest (tiles that need per-pair images, or larger halos).  ONE: a
 * single launch of the second kind over every tile: no occupancy budget, but
 * one launch latency per pass instead of two.  AUTO: ONE when every
 * workgroup of that launch is resident at once (a context of few tiles: a
 * small system, a subdomain), else SPLIT.  The results are the same bit for
 * bit. */
enum { HOOMD_FORCE_AUTO = 0, HOOMD_FORCE_SPLIT = 1, HOOMD_FORCE_ONE = 2 };

/* Integrators (Sec. 3: NVE by velocity Verlet; Sec. 6.1: the weak-scaling LJ
 * runs use a Nose-Hoover thermostat that is not fully symplectic and takes
 * one global kinetic-energy sum per step).  HOOMD_NVT follows the flow
 *   dx/dt = v,  dv/dt = F - xi v,  dxi/dt = (T/T0 - 1) / tau^2,
 * T = 2 KE / g with g = 3N - 3 (N the group's local particles), per step h:
 *   v(t+h/2) = v(t) + h/2 (F(t) - xi(t) v(t));  x(t+h) = x(t) + h v(t+h/2);
 *   xi(t+h) = xi(t) + h/tau^2 (T(t+h/2)/T0 - 1)   (the one KE sum);
 *   v(t+h) = (v(t+h/2) + h/2 F(t+h)) / (1 + h/2 xi(t+h)),
 * with eta(t+h) = eta(t) + h/2 (xi(t) + xi(t+h)).  The flow conserves
 * KE + PE + g T0 (tau^2 xi^2 / 2 + eta). */
enum { HOOMD_NVE = 0, HOOMD_NVT = 1 };

/* Geometry of one system.  For a periodic box lo = 0 and L is the box.  For
 * a subdomain frame with ghosts the open axes have periodic = 0 and [lo, lo
 * + L) must contain every local and ghost position. */
typedef struct {
    double lo[3];
    double L[3];
    int32_t periodic[3];
    int32_t pad_;
    int64_t n_local;       /* particles integrated and given forces (>= 0)   */
    int64_t n_cap;         /* rows available (locals + room for ghosts)      */
    int64_t n_bonds;       /* entries in the bond table                      */
} hoomd_box;
/* A system may be empty (n_local = 0, with or without rows): it takes no
 * part in any launch and reports zero energies.  A context needs at least one
 * row over all its systems (HOOMD_E_ARG otherwise). */

/* Device arrays of one context (see the layout above).  bonds: int32[n_bonds]
 * [2] pairs of tags (unordered), or NULL.  When n_sys > 1 the arrays of all
 * systems are concatenated, system s starting at row sum_{t<s} n_cap_t and at
 * bond sum_{t<s} n_bonds_t. */
typedef struct {
    double *pos;
    double *vel;
    void *force;
    int32_t *tag;
    const int32_t *bonds;
} hoomd_arrays;

/* Bytes of device workspace needed for these systems and parameters.  Returns
 * 0 on invalid arguments. */
size_t hoomd_workspace_bytes(const hoomd_params *params, int32_t n_sys, const hoomd_box *boxes);

/* Create a context over caller-owned device arrays.  params and boxes hold
 * n_sys entries each (one per independent system).  All systems share the
 * precision; LJ and WCA systems (with or without bonds) may be mixed in one
 * context, DPD systems only with other DPD systems.  Every kernel covers all
 * systems in one launch.  `stream` is a hipStream_t (NULL = the null
 * stream).  Copies the descriptors and the bond table (as per-particle
 * partner rows) to the device synchronously; validates tags of bonded
 * systems.  Errors: HOOMD_E_ARG, HOOMD_E_WORKSPACE, HOOMD_E_DEVICE. */
int hoomd_init(hoomd_ctx **out, const hoomd_params *params, int32_t n_sys,
               const hoomd_box *boxes, const hoomd_arrays *arrays, void *workspace,
               size_t workspace_bytes, void *stream);

void hoomd_destroy(hoomd_ctx *ctx);

/* Build the cell list and the Verlet neighbour list of every system from the
 * current positions (Sec. 5.1, Fig. 4): particle j != i is listed in row i
 * when |x_j - x_i|^2 < (r_cut + r_buff)^2 in FP64, minimum image along
 * periodic axes, excluding bonded partners.  force_rebuild = 0 builds only
 * if some particle moved more than r_buff/2 since the last build (Sec. 4.2).
 * A row holds 16-bit indices into the halo of its 64-row tile (the tile's
 * distinct neighbours, see hoomd_get_layout); the order of the entries in a
 * row is unspecified (it follows the build's staging order), the set is
 * exact.  With sort_period > 0 the rows are first put in Morton order.
 * Overflow of a row, a cell or a halo latches a status. */
int build_nlist(hoomd_ctx *ctx, int32_t force_rebuild);

/* Flags of compute_forces() and step(). */
enum { HOOMD_ENERGY = 1u, HOOMD_VIRIAL = 2u };

/* Forces on the local particles at the current state (Sec. 3: LJ, DPD;
 * Sec. 4.3.4: FENE + WCA bonds; Sec. 5.1: w lanes per particle), keyed (for
 * DPD) on `timestep`.  Builds the neighbour list first if needed.  Writes `force`
 * (energy in the w component when HOOMD_ENERGY is set) and, with flags, the
 * per-system thermo sums read by hoomd_thermo(). */
int compute_forces(hoomd_ctx *ctx, uint64_t timestep, uint32_t flags);

/* Advance every system n_steps velocity-Verlet (NVE, Sec. 3) or Nose-Hoover
 * (NVT, Sec. 6.1, as stated at HOOMD_NVT) steps with rebuilds decided on the
 * device (Sec. 4.2), the state before the call being that of timestep
 * first_timestep: per NVE step v += dt/2 F; x += dt v (folded); rebuild when
 * needed; F <- F(x, v, t+1); v += dt/2 F.  With
 * log_every > 0 the thermo sums are recorded every log_every steps (and at
 * the last step) in a device ring read by hoomd_thermo_log().  Morton sorts
 * happen every sort_period steps.  On return pos, vel, force and tag hold
 * the final state. */
int step(hoomd_ctx *ctx, uint64_t first_timestep, int32_t n_steps, int32_t log_every);

/* Ghost selection and packing for system `sys` (Sec. 4.3.2, Fig. 2).
 * subdomain = {lo[3], hi[3], width}: a local particle is sent in direction
 * d in {-1,0,1}^3 \ {0} (index (dz+1)*9 + (dy+1)*3 + (dx+1), centre removed,
 * 0..25) when on every axis with d_a = +1 it has x_a >= hi_a - width and on
 * every axis with d_a = -1 it has x_a < lo_a + width.
 * mode HOOMD_GHOST_SELECT recomputes the send list (ordered by direction,
 * then ascending local index) and stores it in the context;
 * mode HOOMD_GHOST_UPDATE re-gathers the fields of the stored list.
 * fields (HOOMD_FIELD_*) choose what is packed; the send buffer holds, for
 * the whole list and in this order, double[k][3] positions, double[k][3]
 * velocities, int32[k] tags (only the chosen ones), k = total entries.
 * counts26 / offsets26: device int32[26] outputs (entries per direction and
 * exclusive offsets).  send_cap is the capacity in entries; a longer list
 * latches HOOMD_E_GHOST_OVERFLOW and packs nothing past the capacity. */
typedef struct { double lo[3]; double hi[3]; double width; } hoomd_subdomain;
enum { HOOMD_GHOST_SELECT = 0, HOOMD_GHOST_UPDATE = 1 };
enum { HOOMD_FIELD_POS = 1u, HOOMD_FIELD_VEL = 2u, HOOMD_FIELD_TAG = 4u };
int pack_ghosts(hoomd_ctx *ctx, int32_t sys, const hoomd_subdomain *subdomain, int32_t mode,
                uint32_t fields, void *send, int64_t send_cap, int32_t *counts26,
                int32_t *offsets26);

/* pack_ghosts() in HOOMD_GHOST_SELECT mode without a context or workspace,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc).  Selects and
 * packs rows [0, n_local) of pos (double[n_local][4]; vel and tag as in the
 * particle layout, needed only when HOOMD_FIELD_VEL / HOOMD_FIELD_TAG are
 * asked for) with the same send rule, order and record layout as
 * pack_ghosts(); counts26 / offsets26 are device int32[26] outputs.  The
 * per-row masks and scan partials live in a fixed device array of the
 * library (about 9 MB per GPU, held until the process ends): n_local above
 * HOOMD_NOALLOC_MAX_ROWS returns HOOMD_E_ARG and queues nothing.  No device
 * memory is allocated.  No send list is stored (there is no UPDATE mode),
 * and overflow is not latched: a total (offsets26[25] + counts26[25]) above
 * send_cap means the records past send_cap were not written.  Every call on
 * one GPU uses that GPU's one array, so calls that overlap in time on the
 * same GPU (different streams or threads) race; calls queued on one stream
 * are safe.  Queued on `stream` (a hipStream_t, NULL = null stream). */
#define HOOMD_NOALLOC_MAX_ROWS 2097152
int pack_ghosts_noalloc(const double *pos, const double *vel, const int32_t *tag, int64_t n_local,
                        const hoomd_subdomain *subdomain, uint32_t fields, void *send, int64_t send_cap,
                        int32_t *counts26, int32_t *offsets26, void *stream);

/* Velocity-Verlet in two halves around a ghost exchange or a migration
 * (Sec. 3, Sec. 4.2), for subdomains whose neighbours live elsewhere:
 *   which = 0: v += dt/2 F (F from the last compute_forces() or second half),
 *              x += dt v (folded on periodic axes), and the displacement
 *              check (r_buff/2 since the last build) that hoomd_rebuild_due()
 *              reports;
 *   which = 1: forces at `timestep` (building the list first if needed, e.g.
 *              after ghosts were selected anew), then v += dt/2 F.
 * NVT systems take the Nose-Hoover halves instead (HOOMD_NVT): the first
 * half ends with the thermostat update over the kinetic energy of each
 * group (Sec. 6.1: the one global sum of the step).
 * The caller updates the ghosts between the halves (pack / unpack UPDATE),
 * or, when a rebuild is due, migrates particles and selects ghosts anew.
 * Both halves cover the local rows of every system and only queue work. */
int integrate_half_step(hoomd_ctx *ctx, int32_t which, uint64_t timestep);

/* 1 in *due when the last first half step found a particle of some system
 * farther than r_buff/2 from its position at the last build.  Synchronises. */
int hoomd_rebuild_due(hoomd_ctx *ctx, int32_t *due);

/* Particle migration (Sec. 4.3.1) for system `sys`: every local particle
 * outside the subdomain [lo, hi) (per axis: x >= hi goes up, x < lo goes
 * down; it moves at most one subdomain per rebuild) leaves for the neighbour
 * its position lies in, direction index as for ghosts.  Its position,
 * velocity and tag are packed into `send` (record layout of pack_ghosts with
 * all three fields, ordered by direction then row; counts26 / offsets26 as
 * there), and the particles that stay are compacted in their order to the
 * front of the system's rows.  The ghosts of the system are dropped (select
 * them again after the arrivals).  *n_sent receives the number that left;
 * more than send_cap returns HOOMD_E_GHOST_OVERFLOW (records past send_cap
 * are not written).  Synchronises (the counts set the new local count).
 * In a context with bonds (bond_stride = the largest bond_cap, > 0) every
 * record is followed by the particle's bond_stride partner tags (-1 none)
 * and the directions of their owners seen from the receiver, int32 each
 * (Sec. 4.3.4: bonds migrate with their particles): 56 + 8 bond_stride
 * bytes per record.  With bonds, call pack_bond_ranks(HOOMD_BOND_MIGRATE)
 * and unpack_bond_ranks() in every subdomain first. */
int migrate_particles(hoomd_ctx *ctx, int32_t sys, const hoomd_subdomain *subdomain, void *send,
                      int64_t send_cap, int32_t *counts26, int32_t *offsets26, int64_t *n_sent);

/* Append n_recv migrated particles (records as migrate_particles() writes
 * them: position, velocity, tag, partner entries) after the locals of system `sys`; each
 * position is moved to its periodic image nearest the centre of the
 * system's frame (box_L = the full periodic box).  Requires the system to
 * hold no ghosts; exceeding n_cap returns HOOMD_E_GHOST_OVERFLOW. */
int receive_particles(hoomd_ctx *ctx, int32_t sys, const void *recv, int64_t n_recv, const double *box_L);

/* Ghost unpacking (Sec. 4.3.2: ghosts are appended after the local
 * particles; Sec. 9: DPD ghosts carry velocities and IDs).  Append
 * (HOOMD_GHOST_SELECT) or overwrite in place (HOOMD_GHOST_UPDATE)
 * the n_recv ghosts of a receive buffer laid out as pack_ghosts() writes it,
 * after the locals of system `sys`.  Each received position is moved to its
 * periodic image nearest the centre of the frame [lo, lo + L) of the
 * system (box_L = the full periodic box).  Exceeding n_cap latches
 * HOOMD_E_GHOST_OVERFLOW. */
int unpack_ghosts(hoomd_ctx *ctx, int32_t sys, const void *recv, int64_t n_recv,
                  uint32_t fields, int32_t mode, const double *box_L);

/* Bonded groups across subdomains (Sec. 4.3.4, Fig. 3).  A bond is kept
 * with each member: every row carries its partners' tags and, for each, the
 * direction of the subdomain that owns the partner (direction codes
 * (dz+1) 9 + (dy+1) 3 + (dx+1), 13 = this subdomain; the 26 others are sent
 * in code order, the ghost direction index).  hoomd_init() takes, per
 * system, every bond with a local member (tags as in `tag`; a closed
 * periodic box must hold both members) and marks partners it does not hold
 * as of unknown owner.  pack_ghosts(SELECT) sends each particle, beside the
 * layer rule, to every neighbour that owns one of its partners, and
 * unpack_ghosts(SELECT) finds every partner among the locals and ghosts (a
 * missing one latches HOOMD_E_BOND_GHOST at the next force evaluation), so
 * bonds need no wider ghost layer than the pair cut-off.  The owner table
 * is kept by 16-byte messages {int32 tag of the receiver's particle, int32
 * tag of its partner, int32 owner direction of that partner seen from the
 * receiver, 0}, laid out per direction like pack_ghosts() (counts26 /
 * offsets26, *n_sent; more than send_cap returns HOOMD_E_GHOST_OVERFLOW):
 *   HOOMD_BOND_START: before the first ghost selection, every particle
 *     with a partner of unknown owner announces itself to all 26
 *     neighbours; the neighbour that owns the partner records where it is;
 *   HOOMD_BOND_MIGRATE: at a rebuild, before migrate_particles(), every
 *     particle outside [lo, hi) tells the owner of each remote partner where
 *     it goes (entries of local partners are updated in place).
 * Call pack_bond_ranks() in every subdomain, move the messages, then
 * unpack_bond_ranks() in every subdomain, before any particle moves.
 * pack_bond_ranks() synchronises; both return HOOMD_E_STATE for a system
 * without bonds or after its rows changed without a ghost selection.  As
 * for ghosts, the 26 neighbours of a subdomain must be distinct (three or
 * more subdomains along every split axis), so that a particle has one copy
 * per subdomain. */
enum { HOOMD_BOND_START = 0, HOOMD_BOND_MIGRATE = 1 };
int pack_bond_ranks(hoomd_ctx *ctx, int32_t sys, const hoomd_subdomain *subdomain, int32_t mode, void *send,
                    int64_t send_cap, int32_t *counts26, int32_t *offsets26, int64_t *n_sent);
int unpack_bond_ranks(hoomd_ctx *ctx, int32_t sys, const void *recv, int64_t n_recv, int32_t mode);

/* Per-system thermo {KE, PE, W, T} (Sec. 4.3.3: energies and virial summed
 * once per evaluation) of the last evaluation that asked for energies (compute_forces with flags, or a logged step), FP64, summed in a
 * fixed order.  out holds 4 * n_sys doubles.  Synchronises. */
int hoomd_thermo(hoomd_ctx *ctx, double *out);

/* Nose-Hoover state {xi, eta} of each system's thermostat (the shared one
 * for a group; zeros for NVE systems), 2 * n_sys doubles in host memory
 * (Sec. 6.1).  hoomd_set_thermostat() sets them (for a group, the values of
 * its last system win).  Both synchronise.  hoomd_init() starts every
 * thermostat at {0, 0}. */
int hoomd_thermostat(hoomd_ctx *ctx, double *xi_eta);
int hoomd_set_thermostat(hoomd_ctx *ctx, const double *xi_eta);

/* Copy up to max_rows logged rows {timestep, KE, PE, W, T} per system
 * (row-major [row][sys][5]) of the last step() call.  Synchronises.  Returns
 * the number of rows via *rows. */
int hoomd_thermo_log(hoomd_ctx *ctx, double *out, int32_t max_rows, int32_t *rows);

/* Read and clear the device status word (overflow of a row, cell, halo or
 * ghost list; bond stretch; NaN; dangerous build, Sec. 4.2 and Sec. 6.1).  Returns the first latched
 * condition (HOOMD_OK if none); *required (may be NULL) receives the
 * capacity that would have avoided an overflow (row entries, cell members or
 * ghost entries).  Synchronises. */
int hoomd_sync_status(hoomd_ctx *ctx, int64_t *required);

/* Number of neighbour-list builds since hoomd_init.  Synchronises. */
int hoomd_build_count(hoomd_ctx *ctx, int64_t *builds);

/* Device pointers into the workspace for inspection, for system `sys`:
 *   nlist  uint16, row of local particle i at entries (i/64)*64*cap +
 *          k*64 + i%64, k < nn[i]; an entry is an index into the halo of
 *          the row's 64-row tile;
 *   nn     int32[n] row lengths;
 *   halo   int32, halo_cap array rows (global row numbers) per tile, the
 *          first (halo_n[tile] & 0xffff) valid; bits 16-30 of halo_n hold
 *          the tile's longest row, bit 31 marks a tile wider than half a
 *          periodic box (per-pair minimum image in the force pass);
 *   cell_idx / cell_size: cell c holds cell_idx[c * cell_cap + k], k <
 *          cell_size[c] (global row numbers, ascending);
 *   bins per axis.  Row i of system s is row row_offset + i of the arrays,
 *   tile t of the system is tile tile_offset + t of halo and halo_n.
 *   The local rows of a system are tiled over its capacity n_cap, so the
 *   tiles past n_local are empty (rows arriving by migration fill them).
 *   general_tiles: int32 count, over all systems, of the tiles that the
 *   last build handed from the framed build to the general one;
 *   rare_tiles: int32 count, over all systems, of the tiles that the force
 *   pass handles in its second launch (per-pair images, or a halo above
 *   halo_lds, the entries the first launch stages in LDS). */
typedef struct {
    const uint16_t *nlist;
    const int32_t *nn;
    const int32_t *halo;
    const int32_t *halo_n;
    const int32_t *cell_idx;
    const int32_t *cell_size;
    int32_t nlist_cap;
    int32_t cell_cap;
    int32_t halo_cap;
    int32_t bins[3];
    int64_t row_offset;
    int64_t cell_offset;
    int64_t tile_offset;
    const int32_t *general_tiles;
    const int32_t *rare_tiles;
    int32_t halo_lds;
    int32_t bond_stride; /* partner entries per row (largest bond_cap; 0: no bonds) */
    int64_t n_local;   /* current local rows of the system (migration changes it) */
    int64_t n_total;   /* locals + ghosts */
} hoomd_layout;
int hoomd_get_layout(hoomd_ctx *ctx, int32_t sys, hoomd_layout *out);

/* Autotuner (Sec. 5.2): launch shapes in use, and the timings of the last
 * scan.  do_tune = 0 reports; 1 times every candidate on the current state
 * (median of 5 launches each, after one untimed launch) and keeps the
 * fastest; 2 takes the shapes a scan found for the same kind of context
 * (pair potential, precision, particle count to within a factor of 2, mean
 * neighbour count to within 4) from a process-wide cache, and scans only
 * when there is none.  Candidates: the force pass with W = 1, 2, 4, 8, 16
 * lanes per particle (64 W threads per workgroup); the framed list build
 * with (lanes per row, threads per workgroup) = (64, 512), (64, 256),
 * (32, 512), (32, 256).  A scan rebuilds the neighbour list afterwards, so
 * the state is what it was.  Synchronises when tuning.  Fields given
 * explicitly in hoomd_params are kept (not tuned). */
typedef struct {
    int32_t tpp_nlist, block_nlist, tpp_force, block_force;
    float force_ms[5];   /* median launch time of each force candidate in the last scan (0: not timed) */
    float build_ms[4];   /* the same for the build candidates, in the order above */
    int32_t scans;       /* scans run by this context */
    int32_t from_cache;  /* 1 when the shapes in use came from the cache */
} hoomd_tuning;
int hoomd_autotune(hoomd_ctx *ctx, int32_t do_tune, hoomd_tuning *out);

/* Device time per phase of step(), measured with HIP events recorded on the
 * context's stream around every fused force launch and every queued rebuild
 * sequence (cell list + neighbour list, including launches that find no
 * rebuild needed).  mode 1 = start (clears the totals), 0 = stop, 2 = read
 * (synchronises; fills *out with the totals since the last start). */
typedef struct {
    double force_ms;
    int64_t force_launches;
    double rebuild_ms;
    int64_t rebuild_launches;
} hoomd_profile_t;
int hoomd_profile(hoomd_ctx *ctx, int32_t mode, hoomd_profile_t *out);

const char *hoomd_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* HOOMD_MI355X_H */
