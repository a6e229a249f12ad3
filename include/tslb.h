/*
 * tslb.h -- C-ABI of the MI355X (gfx950) multicomponent thread-safe lattice
 * Boltzmann (TSLB) time step.
 *
 * The method is that of Montessori, Hegele Jr. and Lauricella, "A
 * high-performance lattice Boltzmann model for multicomponent turbulent jet
 * simulations" (arXiv:2403.15773):
 *   - hydrodynamics on D3Q27, stored as moments (density, velocity and the
 *     non-equilibrium momentum flux) instead of populations (Methodology, the
 *     paragraph after Eq. 7); each step rebuilds the post-collision populations
 *     from the neighbours' moments and sums them into the node (Eqs. 5, 6, 8 and
 *     the thread-safe sketch), with the third-order Hermite equilibrium (Eq. 16)
 *     and third-order regularised non-equilibrium part (Eqs. 18, 19);
 *   - surface tension by the continuum-surface force F = -sigma kappa grad(phi)
 *     (Eqs. 20, 21), entered with Guo's forcing;
 *   - the phase field on D3Q7 with a first-order equilibrium, unit relaxation and
 *     the anti-diffusion source (Eqs. 22-24);
 *   - boundaries by imposing density and/or velocity on one-node boundary layers
 *     and copying the non-equilibrium part from the nearest interior node
 *     (Eqs. 9, 10).
 *
 * Conventions shared by every call:
 *   - Every function returns an int status (TSLB_OK or a negative TSLB_E_*);
 *     nothing throws across this interface.  tslb_last_error() gives the text.
 *   - A context is used by one host thread at a time.  Work is queued on the
 *     context's HIP stream; calls that hand results to the host synchronise it.
 *   - Host arrays are owned by the caller and hold exactly N = nx*ny*nz values
 *     per component, structure of arrays, x fastest: value (x, y, z) of
 *     component c at [c*N + x + nx*(y + ny*z)].  Symmetric tensors use the
 *     component order xx, yy, zz, xy, xz, yz.
 *   - Device memory is owned by the context unless the caller passes
 *     device_buffer, which must then stay allocated until tslb_destroy().
 *   - A call that issues device work first makes the context's (or group's)
 *     device current on the calling thread and leaves it current.
 */
#ifndef TSLB_H
#define TSLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSLB_ABI_VERSION 4

enum {
    TSLB_OK = 0,
    TSLB_E_INVAL = -1,    /* bad argument or parameter set */
    TSLB_E_NOMEM = -2,    /* device or host allocation failed, or budget exceeded */
    TSLB_E_DEVICE = -3,   /* a HIP call failed */
    TSLB_E_UNSTABLE = -4, /* a non-finite value appeared, or the mass left the bound of
                             max_mass_drift; state kept at the failing step */
    TSLB_E_STATE = -5     /* call out of order (e.g. step before any state was set) */
};

/* Face rules (faces in the order -x, +x, -y, +y, -z, +z). */
enum {
    TSLB_BC_PERIODIC = 0, /* both faces of the axis must be periodic */
    TSLB_BC_FREESLIP = 1, /* normal velocity and normal-tangential stress zero; rest copied */
    TSLB_BC_INLET = 2,    /* -z face only: round nozzle, u_z = U s(r)(1 + a xi), phi = s(r) */
    TSLB_BC_OUTFLOW = 3,  /* density 1; velocity, stress and phase copied */
    TSLB_BC_NOSLIP = 4    /* velocity zero; rest copied */
};

/* Storage type of the ten moment planes (the phase field is always one 32-bit
 * plane, fixed point with 30 fractional bits).  Bytes per node and buffer:
 * FP32 44, FP16 and BF16 24, FP16Q 32.  Arithmetic is binary32 in every case. */
enum {
    TSLB_STORE_FP32 = 0,
    TSLB_STORE_FP16 = 1,  /* scaled deviations rho'/U^2, ubar/U, Q/U^2, round to nearest even */
    TSLB_STORE_BF16 = 2,  /* the same in bfloat16 */
    TSLB_STORE_FP16Q = 3  /* rho' and ubar in binary32, only the stress Q/U^2 in binary16: rounding
                             of rho' leaks into the small stress through neighbour differences,
                             so keeping it (and ubar) exact meets a 1e-3 moment error where FP16 does not */
};

/* Step kernels (tslb_set_kernel). */
enum {
    TSLB_KERNEL_FUSED = 0,  /* one fused kernel per step (default) */
    TSLB_KERNEL_GATHER = 1  /* simple reference: materialised geometry, then one
                               thread per node gathering its 27 sources */
};

typedef struct tslb_ctx tslb_ctx;

typedef struct tslb_params {
    int32_t abi_version;     /* must equal TSLB_ABI_VERSION */
    int32_t nx, ny, nz;      /* lattice size; each >= 4 on a non-periodic axis, >= 1 otherwise;
                                nx*ny < 2^30 and nx*ny*nz < 2^33 */
    int32_t bc[6];           /* TSLB_BC_* for faces -x,+x,-y,+y,-z,+z */
    double nu;               /* kinematic viscosity > 0; omega = 1/(3 nu + 1/2) < 2 (Eqs. 3-4) */
    double sigma;            /* surface tension >= 0 (Eq. 20) */
    double width;            /* interface width W > 0 */
    double gamma;            /* anti-diffusion constant of Eq. 24; <= 0 selects 2/W */
    double eps;              /* n = G/(|G| + eps) (Eq. 21); >= 1e-30, or < 0 for the default 1e-4 */
    double inlet_u;          /* nozzle velocity U (TSLB_BC_INLET) */
    double inlet_d;          /* nozzle diameter D; axis at ((nx-1)/2, (ny-1)/2) */
    double inlet_noise;      /* relative amplitude a of the inlet perturbation */
    uint64_t seed;           /* key of the counter-based inlet noise */
    int32_t storage;         /* TSLB_STORE_* */
    double u_scale;          /* U of the scaled-deviation storage; <= 0 selects 0.05 */
    int32_t check_interval;  /* steps between finite/mass checks inside tslb_step; 0 = never */
    int32_t device;          /* HIP device ordinal */
    void *device_buffer;     /* optional caller-owned device allocation for the state */
    size_t device_buffer_bytes;
    void *stream;            /* optional hipStream_t; NULL = the context creates its own */
    int32_t components;      /* 2 (default): two components, the phase field of Eqs. 20-24 coupled
                                through surface tension; 1: a single component, the high-order
                                regularised hydrodynamics alone (no phase plane in the state,
                                F = 0; sigma, width, gamma and eps are ignored, tslb_phase returns
                                zeros and the phase sum is 0) */
    double max_mass_drift;   /* > 0: at every check (check_interval) the mass sum(rho) must stay
                                within this relative distance of its value when stepping started
                                from the last state set; else TSLB_E_UNSTABLE.  The method conserves
                                mass on a closed lattice (periodic, no-slip or free-slip faces), to
                                binary32 rounding; inlet and outflow faces exchange mass.  0 = off */
    /* Components of different density and viscosity (the paper's model has equal
     * ones and names this extension as future work; the Results and Conclusions
     * sections).  variable_density = 1 selects the velocity-based phase-field form
     * of the step for immiscible fluids of different density, in the
     * regularised Hermite form of the rest of the step:
     *   rho(phi) = density_b + phi (density_a - density_b), nu(phi) = nu_b + phi
     *   (nu_a - nu_b) (phi clamped to [0, 1]; component A is phi = 1), omega per
     *   node from nu(phi);
     *   the first stored moment is the normalised pressure p* (pressure
     *   p = rho(phi) p* c_s^2) instead of rho - 1, the velocity terms of the
     *   population rebuild take unit density, and the force is the acceleration
     *   a = (F_s + F_p + F_mu)/rho(phi) + gravity with the surface tension
     *   F_s = -sigma kappa grad(phi) (Eq. 20), the pressure force
     *   F_p = -p* c_s^2 grad(rho) and the viscous force
     *   F_mu = -(1 - omega/2) Q . grad(rho) (Q the stored non-equilibrium stress);
     *   a = 0 on boundary layers.
     * Then rho_dev of tslb_set_state/tslb_moments is p*, u is the velocity,
     * pi_neq is P = Q + a a/4, and the mass of tslb_diagnostics is
     * density_b N + (density_a - density_b) sum(phi).  Requires two components,
     * binary32 storage and the fused kernel; nu is ignored.  0 = the paper's
     * equal-density model (gravity must then be zero). */
    int32_t variable_density;
    double density_a, density_b;  /* > 0 */
    double nu_a, nu_b;            /* > 0, each with omega < 2 */
    double gravity[3];            /* body acceleration g (finite) */
} tslb_params;

/* Fill *p with defaults: periodic 32^3, nu = 0.1, sigma = 0, W = 3, FP32, two components. */
void tslb_params_init(tslb_params *p);

/* sizeof(tslb_params) as compiled into the library (binding layout check). */
size_t tslb_params_size(void);

/* Bytes of device memory the state needs (two buffers); the size device_buffer
 * must have.  0 if the parameters are invalid. */
size_t tslb_required_bytes(const tslb_params *p);

/* Validate p, derive omega = 1/(3 nu + 1/2) (Eqs. 3-4) and gamma (Eq. 24),
 * allocate (or adopt) device memory, zero it and bind the stream.  On success
 * *out owns the context.  TSLB_E_INVAL (reason in tslb_last_error(NULL)),
 * TSLB_E_NOMEM, TSLB_E_DEVICE. */
int tslb_create(const tslb_params *p, tslb_ctx **out);

/* Set the state at step `step` from physical host fields: rho_dev = rho - 1
 * (N; the deviation, because binary32 cannot resolve small density changes
 * around 1), u (3N), pi_neq (6N: the Guo-corrected non-equilibrium momentum
 * flux P), phi (N; NULL for one component).  These are the moments the method
 * stores in place of populations (Methodology, after Eq. 7: density, velocity
 * and the non-equilibrium momentum flux).  The stored raw state is rho - 1,
 * ubar = u - F/(2 rho), Q = P - F F/(4 rho) and phi rounded to the fixed-point
 * grid 2^-30 (clamped to [-0.45, 1.45]), with F the surface-tension force of
 * Eqs. 20-21 computed from that phi (Guo's half-force shift).  Allocates and
 * releases 80 B per node of staging planes on the device.  Synchronises.
 * TSLB_E_INVAL for a NULL field, TSLB_E_NOMEM, TSLB_E_DEVICE. */
int tslb_set_state(tslb_ctx *ctx, const float *rho_dev, const float *u, const float *pi_neq, const float *phi,
                   int64_t step);

/* Set the state of a fluid at rest at step `step`: rho = 1, u = 0, P = 0 and
 * phi = 0 everywhere (in the stored deviation form every word is zero), the
 * quiescent ambient into which the paper's jets are injected (Results, jet
 * set-up).  No host transfer; the boundary layers are filled by the first
 * tslb_step.  Synchronises. */
int tslb_set_state_rest(tslb_ctx *ctx, int64_t step);

/* Queue nsteps time steps of the method (Eqs. 5, 6, 8: every node's moments
 * rebuilt from its neighbours' post-collision populations, with the phase
 * field of Eqs. 22-24 and the boundary layers of Eqs. 9-10).  Asynchronous
 * unless check_interval triggers a check, which synchronises and returns
 * TSLB_E_UNSTABLE on a non-finite value or a mass outside max_mass_drift (the
 * state is then the one of the failing step).  TSLB_E_STATE before any state
 * was set. */
int tslb_step(tslb_ctx *ctx, int64_t nsteps);

/* Wait for queued work. */
int tslb_sync(tslb_ctx *ctx);

/* Physical moments at the current step, the inverse of tslb_set_state's
 * mapping: rho_dev = rho - 1 (N), u = ubar + F/(2 rho) (3N), pi_neq =
 * Q + F F/(4 rho) (6N), F from the current phi (Eqs. 20-21); any pointer may
 * be NULL.  Boundary layers are filled first (Eqs. 9-10).  Allocates and
 * releases 80 B per node of staging planes.  Synchronises.  TSLB_E_STATE before
 * any state was set. */
int tslb_moments(tslb_ctx *ctx, float *rho_dev, float *u, float *pi_neq);

/* Phase field phi (N) at the current step (the order parameter of Eqs. 22-24,
 * 1 in component A), converted from the stored fixed point.  Synchronises.
 * TSLB_E_STATE before any state was set. */
int tslb_phase(tslb_ctx *ctx, float *phi);

/* Device memory the context holds now, in bytes: its two state buffers, the
 * diagnostics partials (a few kilobytes) and any scratch planes allocated at
 * the time (those of running statistics, 76 B per node, or of the gather
 * kernel, 36 B per node; set-state and readout release theirs before they
 * return).  What a serving group charges against its budget.  0 for NULL. */
size_t tslb_device_bytes(const tslb_ctx *ctx);

/* Raw state as stored (bitwise checkpoint): bytes must equal tslb_state_bytes(). */
size_t tslb_state_bytes(const tslb_ctx *ctx);
int tslb_get_state_raw(tslb_ctx *ctx, void *host, size_t bytes);
int tslb_set_state_raw(tslb_ctx *ctx, const void *host, size_t bytes, int64_t step);

/* Conservation diagnostics of the current state: mass = sum rho (binary32
 * compensated sums per thread, binary64 across threads), phase = sum phi (exact
 * integer sum of the fixed-point field, returned as binary64), the current step
 * index and whether every stored moment is finite.  The collision conserves
 * mass (the zeroth moments of every correction of Eqs. 7, 16-19 and of the
 * forcing vanish) and the phase step conserves phi (Eqs. 23-24), so on a
 * closed lattice both stay put to rounding; the phase sum is kept exactly by
 * the integer streaming.  With variable density the mass is
 * density_b N + (density_a - density_b) sum(phi).  Boundary layers are filled
 * first.  Synchronises.  TSLB_E_STATE before any state was set. */
int tslb_diagnostics(tslb_ctx *ctx, double *mass, double *phase_sum, int64_t *step, int32_t *finite);

/* For callers that cannot allocate device memory (work under HIP stream
 * capture, serving loops and harnesses that forbid hipMalloc): the
 * diagnostics of tslb_diagnostics for one state buffer the caller holds in
 * device memory, computed with no allocation of any kind.
 *   p      parameters of the lattice the buffer belongs to (validated as by
 *          tslb_create; device_buffer and stream are ignored, p->device is
 *          made current);
 *   state  device pointer, read only, 4-byte aligned: one state buffer in the
 *          layout tslb_get_state_raw() returns (tslb_state_bytes() bytes);
 *          every node is summed as stored (tslb_diagnostics fills the
 *          boundary layers first; a buffer written by a step or read back by
 *          tslb_get_state_raw already has them);
 *   stream hipStream_t the two kernels are queued on (NULL: the null stream);
 *   out    device pointer, 8-byte aligned, receives 3 doubles: the mass, the
 *          phase sum and 1.0 if every stored moment is finite (else 0.0),
 *          bit for bit what tslb_diagnostics returns for the same buffer.
 * Asynchronous: out is valid once the stream has reached it.  The partial sums
 * live in a static device array (24.6 KB per device, held until the process
 * ends) with room for 1024 blocks; the kernels stride over the nodes, so every
 * lattice tslb_create accepts fits, and parameters it rejects are rejected
 * here (TSLB_E_INVAL).  Calls on one device share that array: calls that
 * overlap in time (other streams or host threads) race and must be
 * serialised by the caller.  TSLB_E_DEVICE for a failed launch; the message
 * is in tslb_last_error(NULL). */
int tslb_diagnostics_noalloc(const tslb_params *p, const void *state, void *stream, double *out);

/* Current step index (no synchronisation). */
int64_t tslb_step_index(const tslb_ctx *ctx);

/* Enable (1) or disable (0) per-launch HIP-event timing of the fused step
 * kernel on the context's stream.  Off by default. */
int tslb_set_timing(tslb_ctx *ctx, int enable);

/* Average duration in milliseconds of one fused step-kernel launch over the
 * last tslb_step() call made with timing enabled; synchronises.  Returns 0 if
 * no timed launch exists. */
double tslb_last_step_kernel_ms(tslb_ctx *ctx);

/* Per-launch durations (ms) of the fused step kernel over the last tslb_step()
 * call made with timing enabled: up to cap values are written to ms (host
 * array, may be NULL when cap is 0) and *count receives the number of timed
 * launches (at most 8192 per call).  Synchronises. */
int tslb_step_kernel_times(tslb_ctx *ctx, float *ms, int64_t cap, int64_t *count);

/* Select the step kernel (TSLB_KERNEL_*) and, for the fused kernel, the number
 * of z planes a workgroup marches through: chunk_z >= 1 fixes it, 0 (the
 * default) lets the library choose per lattice (at most 128 planes on 16-row
 * tiles and 256 on 20-row tiles, the length
 * that minimises the rounds of workgroups per compute unit times the planes
 * each round walks, its chunk plus a pipeline of 6).  Both kernels compute the
 * same step up to rounding, and the fused result does not depend on chunk_z. */
int tslb_set_kernel(tslb_ctx *ctx, int kernel, int chunk_z);

/* Height of the fused step's tiles (workgroups of 32 x rows destination
 * columns): rows = 16 or 20 fixes it, 0 (the default) lets the library choose
 * per lattice together with the z chunk, by the same cost model (a 20-row
 * workgroup walks a plane in 1.18 times the time of a 16-row one and updates
 * 1.25 times the columns; the height that gives each compute unit the least
 * time wins).  20 rows serve the two-component step with equal densities only
 * (TSLB_E_INVAL otherwise); the result is bitwise the same at either height.
 * Not while the ctx is in a serving group (TSLB_E_STATE). */
int tslb_set_tile(tslb_ctx *ctx, int rows);

/* The tile height the fused step of ctx uses (16 or 20); TSLB_E_INVAL for a
 * NULL ctx. */
int tslb_tile_rows(const tslb_ctx *ctx);

/* Free and total device memory of HIP device `device` in bytes (hipMemGetInfo):
 * what a serving loop admits requests against. */
int tslb_device_memory(int32_t device, size_t *free_bytes, size_t *total_bytes);

/* Measurement utility: copy `bytes` (a multiple of 16) between two device
 * buffers it allocates on `device`, `iters` times with a plain streaming copy
 * kernel, and report the median rate as read + written bytes per second in GB/s
 * (*gbps) and the median kernel time in ms (*ms).  Used as the measured HBM
 * ceiling and as the reference for scaling hardware byte counters. */
int tslb_copy_bandwidth(int device, size_t bytes, int iters, double *gbps, double *ms);

/* Measurement utility: the moment-to-population projection of the step (the 27
 * brackets f_i/w_i - 1 - rho' of a node from its 16 scaled Hermite coefficients,
 * Eqs. 15-19) evaluated `reps` times per node over `nodes` nodes, each time with
 * every coefficient raised by 1e-3, and accumulated.  kind 0 = the tensor product
 * on the vector ALU that the step uses; kind 1 = the same 27 x 16 map as FP32
 * matrix-core tiles (v_mfma_f32_32x32x2_f32).  coef_host: 16 x nodes floats
 * (coefficient-major, order K1x K1y K1z K2xx K2yy K2zz K2xy K2xz K2yz K3xxy K3xxz
 * K3yyx K3yyz K3zzx K3zzy K3xyz), host memory, read only.  nodes: a multiple of 64,
 * at most 2^28.  out_host: NULL, or 27 x nodes floats (velocity-major, index
 * 9 (c_z + 1) + (c_x + 1) + 3 (c_y + 1)) receiving the accumulated brackets.  *ms:
 * mean kernel time over `iters` launches after one warm-up.  Allocates and frees
 * its own device buffers on `device`.  TSLB_E_INVAL for bad arguments,
 * TSLB_E_DEVICE for a HIP failure (message in tslb_last_error(NULL)). */
int tslb_probe_projection(int32_t kind, const float *coef_host, int64_t nodes, int32_t reps, int32_t iters,
                          int32_t device, float *out_host, double *ms);

/* ---- Time averages (jet statistics) ---------------------------------------
 *
 * The statistics the paper's jet analysis rests on (Results: mean phase field
 * and mean axial velocity along the centreline and across the jet): once
 * started, tslb_step adds, after every step whose index is a multiple of
 * `every`, the phase field phi, the physical velocity u (half-force shifted)
 * and u_z^2 of every node to binary64 sums on the device.  tslb_stats_start
 * (every >= 1) clears the sums (allocating 40 bytes per node on first use;
 * TSLB_E_INVAL for every < 1, TSLB_E_NOMEM if the allocation fails);
 * tslb_stats_stop ends accumulation and keeps them.  A sample costs about as
 * much as one step (the interface force is recomputed for the velocity).  Not
 * accumulated while the context is in a serving group. */
int tslb_stats_start(tslb_ctx *ctx, int32_t every);
int tslb_stats_stop(tslb_ctx *ctx);

/* Means over the samples taken so far: mean_phi (N), mean_u (3N), rms_uz (N,
 * the root-mean-square fluctuation of u_z); each pointer may be NULL.
 * *samples (may be NULL) receives the sample count.  Synchronises.
 * TSLB_E_STATE if a field is requested before any sample was taken. */
int tslb_stats_get(tslb_ctx *ctx, float *mean_phi, float *mean_u, float *rms_uz, int64_t *samples);

/* Release the context and everything it allocated.  A member of a serving
 * group is first removed from it (after the group's queued work). */
void tslb_destroy(tslb_ctx *ctx);

/* Text of the last error of ctx, or of the calling thread when ctx is NULL. */
const char *tslb_last_error(const tslb_ctx *ctx);

/* ---- Serving: continuous batching of many lattices ------------------------
 *
 * A group advances several contexts (lattices of different sizes and
 * parameters, the mixed request stream of a solver service) together: every
 * tslb_group_poll() launches ONE fused step kernel that updates every member
 * with steps left (one launch per storage type and component count present),
 * so requests that arrive while others run share the device from their first
 * step on.  A
 * member's update reads and writes only its own lattice (the step of the
 * method has no cross-node reduction), so its result is bitwise the one it
 * gets when run alone.  Admission is by HBM budget and slot count; members
 * join and leave between steps.
 *
 * While a context is a member, the group owns it: every tslb_* call on it
 * except tslb_destroy returns TSLB_E_STATE until a poll has retired it.
 * Groups use the fused kernel only; diagnostics (tslb_diagnostics) are the
 * caller's, after retirement. */
typedef struct tslb_group tslb_group;

/* Create a group on the current HIP device.  hbm_budget_bytes caps the summed
 * device bytes the members hold (two state buffers each, the diagnostics
 * partials, and any scratch planes still allocated, e.g. those of running
 * statistics); a caller admitting by free HBM derives it from
 * tslb_device_memory().  max_domains (1..4096)
 * caps their count; stream is a hipStream_t for the group's launches, or NULL
 * for one the group creates.  Errors: TSLB_E_INVAL, TSLB_E_NOMEM,
 * TSLB_E_DEVICE (text from tslb_last_error(NULL)). */
int tslb_group_create(size_t hbm_budget_bytes, int32_t max_domains, void *stream, tslb_group **out);

/* Admit ctx (state set, fused kernel, same device) to run nsteps more steps.
 * The group's launches start after the work already queued on ctx's stream.
 * Returns TSLB_E_NOMEM when the budget or the slots would be exceeded: the
 * caller defers the request and retries after a poll has retired members.
 * nsteps may be 0 (the member is retired by the next poll). */
int tslb_group_admit(tslb_group *g, tslb_ctx *ctx, int64_t nsteps);

/* Retire finished members and launch the next step of the others.  A member is
 * retired once the device has finished its last step; up to cap retired
 * contexts are written to done[] (admission order) and counted in *ndone.
 * Retired contexts are the caller's again, at step index start + nsteps.  At
 * most 4 steps are in flight: a poll may wait for the oldest. */
int tslb_group_poll(tslb_group *g, tslb_ctx **done, int32_t cap, int32_t *ndone);

/* Bytes charged to the budget, number of members and launches so far (each
 * pointer may be NULL). */
int tslb_group_status(const tslb_group *g, size_t *bytes_in_use, int32_t *members, int64_t *launches);

/* Device-busy time of the group: *busy_ms receives the summed durations of its
 * completed launches (each from the start of its table upload to the end of
 * its last kernel, HIP events on the group's stream) and *completed (may be
 * NULL) their number.  Does not wait. */
int tslb_group_busy(tslb_group *g, double *busy_ms, int64_t *completed);

/* Wait for the group's work and release it; members become free contexts at
 * the step their last launched update reached. */
void tslb_group_destroy(tslb_group *g);

/* Text of the last error of g, or of the calling thread when g is NULL. */
const char *tslb_group_last_error(const tslb_group *g);

#ifdef __cplusplus
}
#endif

#endif /* TSLB_H */
