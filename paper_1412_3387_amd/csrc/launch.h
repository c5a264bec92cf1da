// launch.h -- what the host runtime hands to the kernel launchers: device
// pointers carved from the workspace plus the launch geometry.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace md {

enum StepMode : int32_t {
    MODE_FORCE = 0,  // F(t) only
    MODE_FIRST = 1,  // F(t) from v(t); v(t+1/2); x(t+1)
    MODE_MID = 2,    // F(t) from v(t-1/2); v(t); v(t+1/2); x(t+1)
    MODE_LAST = 3    // F(t) from v(t-1/2); v(t); writes F
};

// The framed build's per-die tile counters sit this many words apart: one
// cache line each, so that the dies' atomics do not queue on one line.
constexpr int kTileCtrStride = 64;

// Launches of the force pass (the values of the public HOOMD_FORCE_*).
constexpr int kForceAuto = 0, kForceSplit = 1, kForceOne = 2;

struct LaunchCtx {
    hipStream_t stream;
    int n_sys;
    const SysDev *sys;
    const int32_t *tprefix_local;  // n_sys+1 prefix of local tiles
    const int32_t *tprefix_all;    // n_sys+1 prefix of tiles over all rows
    const int64_t *cprefix;        // n_sys+1 prefix of cells
    int tiles_local;
    int tiles_all;
    int64_t n_cells;
    int cell_cap;
    int32_t *cell_count;
    int32_t *cell_size;
    int32_t *cell_idx;
    float4 *cell_xf;               // member position from the cell corner (FP32), row bits in w
    uint16_t *nlist;               // halo indices, tile-major rows
    int32_t *nn;
    int nlist_cap;
    int32_t *halo;                 // halo_cap row numbers per tile
    int32_t *halo_n;               // halo size per tile (top bit: per-pair images)
    int halo_cap;
    int halo_lds;                  // halo entries the force pass stages in LDS
    double4 *xbuild;
    int32_t *ptag;                 // per row: bond_stride partner tags (-1 = none), moved with the row
    int32_t *pdir;                 // per row and partner: direction code of the partner's owner
                                   // (13 = this system, -1 = not known yet)
    int32_t *prow;                 // per row and partner: the partner's row (-1 none, -2 not present)
    int32_t *btmp;                 // rows x bond_stride scratch (reordering ptag / pdir)
    int2 *hash;                    // tag -> row tables of the bonded systems
    int bond_stride;
    bool has_bonds;
    int32_t *slow_list;            // tiles the framed build passes on to the general one
    char *plan;                    // per-tile plans of the framed build (build_plan_bytes)
    int32_t *slow_n;               // their number (cleared by the binning launch)
    int32_t *rare_list;            // tiles the force pass handles in its second launch
    int32_t *rare_n;               // their number (cleared by the binning launch)
    int32_t *tile_ctr;             // kDies counters of tiles taken by the framed build's workgroups,
                                   // kTileCtrStride words apart (cleared by the binning launch)
    int force_launch;              // kForceAuto / kForceSplit / kForceOne
    int busy_tiles;                // tiles holding local rows (the others have nothing to do)
    int32_t *flag;                 // rebuild flag read by the rebuild kernels (some system needs one)
    int32_t *sflag;                // per-system rebuild flags of the same slot (n_sys entries)
    int32_t *build_count;
    uint32_t *step_counter;        // advanced by the binning launch when set (graph steps)
    int32_t *since;                // per system, steps since its last build: the binning launch resets
                                   // it on a build and otherwise adds since_inc (1 in step(), 0 elsewhere)
    int32_t since_inc;
    Status *status;
    double *partials;              // 3 doubles per wave
    double *thermo;                // 4 doubles per system
    double *khalf;                 // Nose-Hoover: kinetic energy of the half-step velocities, one per wave
    double *thermostat;            // Nose-Hoover: {xi, eta} per system (used at each group's first system)
    bool nvt;                      // some system integrates NVT
    double *thermo_log;            // rows of 5 doubles per system
};

struct ForceLaunch {
    const double4 *pos;
    double4 *pos_out;
    const double4 *vel;
    double4 *vel_out;
    const int32_t *tag;
    void *force;
    int32_t *flag_set;
    int32_t *flag_clear;
    int32_t *sflag_set;     // per-system flags of flag_set / flag_clear (n_sys entries each)
    int32_t *sflag_clear;
    uint32_t timestep;
    const uint32_t *timestep_ptr;  // when set, the timestep is read from the device
    int32_t mode;
    int32_t log;      // accumulate energy / virial, write thermo partials
    int32_t energy;   // write the energy into force.w
    int32_t mixed;
    int32_t pair;     // one Pair for every system of the launch, or -1 = mixed batch
    const int32_t *since;   // per system, steps since its last build before this step, or nullptr
    int32_t check_period;   // displacement check every this many steps since the build (>= 1)
    const double *thermostat;  // Nose-Hoover state per system (nullptr: every system NVE)
    double *khalf;             // where the launch writes the half-step kinetic-energy partials
};

// nvt_w > 0: the launch also does the Nose-Hoover update of the force launch
// just before it (launch_nvt_update(L, nvt_w) folded in).
void launch_bin(const LaunchCtx &L, const double4 *pos, int nvt_w = 0);
void launch_cell_sort(const LaunchCtx &L, const double4 *pos);
void launch_nlist(const LaunchCtx &L, const double4 *pos, const int32_t *tag, int w, int block);
void launch_force(const LaunchCtx &L, const ForceLaunch &F, int w, int block);
void launch_thermo_reduce(const LaunchCtx &L, int w, int log_row, double timestep);
void launch_set_flag(const LaunchCtx &L, int32_t *flag, int32_t value);
// Sets the local and total row counts in system s's device descriptor.
void launch_set_counts(const LaunchCtx &L, int s, int32_t n_local, int32_t n_total);
// Sets a rebuild flag and all per-system flags of its slot.
void launch_set_flags(const LaunchCtx &L, int32_t *flag, int32_t *sflag, int32_t value);
// Tag -> row tables and the partner rows of the bonded systems (all of them
// when sys < 0), from the current rows (locals and ghosts).
void launch_bond_refresh(const LaunchCtx &L, const int32_t *tag, int sys);
// Half a velocity-Verlet step over the local rows (which = 0: kick, drift,
// displacement check into flag / sflag; 1: kick) from the force array.
void launch_half_step(const LaunchCtx &L, double4 *pos, double4 *vel, const void *force, bool mixed, int which,
                      int32_t *flag, int32_t *sflag);
// Nose-Hoover: per thermostat group, sum the half-step kinetic-energy
// partials (w per tile) of its systems, then advance xi and eta.
void launch_nvt_update(const LaunchCtx &L, int w);
void launch_disp_check(const LaunchCtx &L, const double4 *pos, int32_t *flag, int32_t *sflag);
size_t force_lds_bytes(int pair, int halo_cap, int nlist_cap);
int force_row_over_read();
int force_halo_entry_bytes(int pair);
size_t fast_build_lds_bytes(int nlist_cap);
int nlist_lanes_per_row();  // lanes that scan one row in the framed build (default)
int nlist_block();          // threads per workgroup of the framed build (default)
bool nlist_shape_ok(int lanes_per_row, int block);  // a shape launch_nlist runs
size_t build_plan_bytes(int64_t tiles);
hipError_t prepare_nlist(int nlist_cap);
// Raises the dynamic-LDS limit of the rare-tile force kernels (init time).
hipError_t prepare_force();

}  // namespace md
