// Host-side internals of the TSLB library: the context and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/tslb.h"
#include "tslb_device.h"

namespace tslb {

// A view of one state buffer.
struct StateView {
    void *mom;      // ten planes of the storage type
    int32_t *phi;   // phase-field plane (fixed point, 30 fractional bits)
};

// One lattice of a multi-domain fused step launch (device-resident table).
struct FusedDomain {
    Geo g;
    Phys ph;
    Scales sc;
    StateView in, out;
    unsigned long long step_next;  // step index of the state written
    int lz, tiles_x, tiles_y;      // z chunk and tile grid
    int work_begin, work_count;    // work items [work_begin, work_begin + work_count)
};

// Scratch planes (binary32) used off the per-step path: host staging of
// physical fields and the interface geometry of set/readout.
struct Scratch {
    float *stage = nullptr;  // 11 planes: rho - 1, u(3), P(6), phi
    float *geo = nullptr;    // 9 planes: G(3), n(3), F(3)
    double *partial = nullptr;      // per block: sum rho', finite probe
    long long *partial_i = nullptr; // per block: sum of fixed-point phi
    double *result = nullptr;       // sum rho', finite probe
    long long *result_i = nullptr;  // sum of fixed-point phi
    size_t partial_blocks = 0;
};

// Time averages of the physical fields (jet statistics), accumulated every
// `every` steps of tslb_step: binary64 sums of phi, u_x, u_y, u_z and u_z^2.
struct Stats {
    double *sum = nullptr;  // 5 planes of ld doubles
    int every = 0;          // 0: not accumulating
    long long samples = 0;
};

struct StepTimer {
    bool enabled = false;
    std::vector<hipEvent_t> ev;  // pairs (start, stop) per timed launch
    size_t used = 0;             // pairs recorded in the last tslb_step
};

}  // namespace tslb

struct tslb_ctx {
    tslb_params p;
    tslb::Geo geo;
    tslb::Phys phys;
    tslb::Scales scales;
    int storage;
    bool has_boundary;
    bool phase = true;    // two components (a phase-field plane); false: single component
    bool vd = false;      // variable density and viscosity (velocity-based scheme)
    size_t plane_bytes;   // bytes of one moment plane (storage type)
    size_t buffer_bytes;  // bytes of one state buffer
    void *base = nullptr; // both buffers
    bool owns_base = false;
    tslb::StateView buf[2];
    int cur = 0;
    int64_t step = 0;
    bool state_set = false;
    bool mass_ref_set = false;  // mass_ref taken since the last state was set
    double mass_ref = 0.0;      // mass when stepping started (max_mass_drift)
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    tslb::Scratch scratch;
    tslb::StepTimer timer;
    tslb::Stats stats;
    int kernel = TSLB_KERNEL_FUSED;  // step kernel selected by tslb_set_kernel
    int chunk_z = 0;                 // z planes per workgroup of the fused kernel (0: automatic)
    int tile_rows = 0;               // rows of a fused-step tile, 16 or 20 (0: automatic)
    int plan_rows = 16, plan_lz = 1; // the fused step's tile height and z chunk (fused_plan, kept current)
    int cu_count = 256;              // compute units of the device
    tslb_group *group = nullptr;     // serving group that currently advances this ctx
    std::string err;
};

namespace tslb {

// Error text of a failed call that had no context (read by tslb_last_error(NULL)).
void set_thread_error(const std::string &msg);
// Remove a member from its group (waits for the group's queued work).
void group_detach(tslb_group *g, tslb_ctx *c);

// Parameter checks of tslb_create (false with the reason in why).
bool validate_params(const tslb_params *p, std::string &why);
// Lattice geometry and storage scales of a validated parameter set.
void derive_layout(const tslb_params *p, Geo &g, Scales &sc);

size_t plane_elems(long long N);
// Device memory a context holds now: its two state buffers (caller-owned or
// not), the diagnostics partials and any scratch planes currently allocated.
size_t ctx_device_bytes(const tslb_ctx *c);
size_t state_buffer_bytes(long long N, int storage, bool phase);

// Launchers (all asynchronous on `s`); each returns the hipError_t of the launch.
hipError_t launch_geometry(const tslb_ctx *c, const int32_t *phi, float *geo_planes, hipStream_t s);
hipError_t launch_set_state(const tslb_ctx *c, const float *stage, float *geo_planes, StateView out, hipStream_t s);
hipError_t launch_readout(const tslb_ctx *c, StateView in, const float *geo_planes, float *stage, hipStream_t s);
hipError_t launch_boundary(const tslb_ctx *c, StateView st, int64_t step, hipStream_t s);
hipError_t launch_step(const tslb_ctx *c, StateView in, StateView out, int64_t step_next, hipStream_t s);
hipError_t launch_step_fused(const tslb_ctx *c, StateView in, StateView out, int lz, int64_t step_next,
                             hipStream_t s);
// Tile height (16 or 20 rows) and z chunk of the fused step of ctx c.
struct FusedPlan {
    int rows = 16;
    int lz = 1;
};
FusedPlan fused_plan(const tslb_ctx *c);
int fused_chunk(const tslb_ctx *c);
int fused_rows(const tslb_ctx *c);
// Whether the 20-row tile serves ctx c (two components, equal densities).
bool fused_wide_allowed(const tslb_ctx *c);
// Describe one step of ctx c (in -> out) as a domain of a multi-domain launch
// whose work items start at work_begin; lz > 0 fixes the z chunk (else the
// lattice's own choice).
FusedDomain fused_domain(const tslb_ctx *c, StateView in, StateView out, int64_t step_next, int work_begin,
                         int lz = 0);
// Work items of one fused step of ctx c with z chunk lz.
int fused_work_items(const tslb_ctx *c, int lz);
// One fused step of every domain of a device table (all of one storage type,
// component count, density model and tile height).
hipError_t launch_step_fused_multi(const FusedDomain *doms, int ndom, int total_work, int storage, bool phase,
                                   bool vd, int rows, hipStream_t s);
hipError_t launch_copy_probe(const void *src, void *dst, size_t bytes, hipStream_t s);
hipError_t launch_diagnostics(const tslb_ctx *c, StateView st, const Scratch &sc, hipStream_t s);
size_t diagnostics_blocks(const tslb_ctx *c);
// The same two diagnostics kernels for any state buffer of geometry g: per-block
// partials (sum rho', finite probe; sum of fixed-point phi) of `blocks` blocks,
// then their fixed-order total in result[0..1] and *result_i.
hipError_t launch_diagnostics_raw(const Geo &g, const Scales &sc, int storage, StateView st, double *partial,
                                  long long *partial_i, int blocks, double *result, long long *result_i,
                                  hipStream_t s);
int diagnostics_blocks_for(long long N);
// Add phi, u (= ubar + F/(2 rho), F from geo) and u_z^2 of every node of st to the sums.
hipError_t launch_stats_accum(const tslb_ctx *c, StateView st, const float *geo, double *sum, hipStream_t s);

}  // namespace tslb
