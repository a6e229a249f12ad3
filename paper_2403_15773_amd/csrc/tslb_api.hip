// C-ABI of the TSLB library: context lifetime, state transfer, the step loop
// and diagnostics.  Declarations and contracts are in include/tslb.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tslb_internal.h"

using namespace tslb;

namespace {

thread_local std::string g_thread_error;

int fail(tslb_ctx *c, int code, const std::string &msg) {
    if (c)
        c->err = msg;
    else
        g_thread_error = msg;
    return code;
}

#define HIP_TRY(c, expr)                                                                                  \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess)                                                                             \
            return fail((c), TSLB_E_DEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_));    \
    } while (0)

bool axis_ok(int lo, int hi, int n, int axis, std::string &why) {
    if ((lo == TSLB_BC_PERIODIC) != (hi == TSLB_BC_PERIODIC)) {
        why = "periodic faces must come in pairs (axis " + std::to_string(axis) + ")";
        return false;
    }
    for (int side = 0; side < 2; ++side) {
        int b = side ? hi : lo;
        if (b < TSLB_BC_PERIODIC || b > TSLB_BC_NOSLIP) {
            why = "unknown boundary rule " + std::to_string(b);
            return false;
        }
        if (b == TSLB_BC_INLET && !(axis == 2 && side == 0)) {
            why = "the inlet rule is only defined on the -z face";
            return false;
        }
    }
    if (lo != TSLB_BC_PERIODIC && n < 4) {
        why = "a non-periodic axis needs at least 4 nodes";
        return false;
    }
    return true;
}

bool validate(const tslb_params *p, std::string &why) {
    if (!p) { why = "params is NULL"; return false; }
    if (p->abi_version != TSLB_ABI_VERSION) { why = "abi_version mismatch"; return false; }
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) { why = "lattice sizes must be positive"; return false; }
    long long N = (long long)p->nx * p->ny * p->nz;
    if (N >= (1ll << 31) * 4) { why = "lattice too large"; return false; }
    if ((long long)p->nx * p->ny >= (1ll << 30)) { why = "inlet plane exceeds the noise counter range"; return false; }
    const int n[3] = {p->nx, p->ny, p->nz};
    for (int a = 0; a < 3; ++a)
        if (!axis_ok(p->bc[2 * a], p->bc[2 * a + 1], n[a], a, why)) return false;
    if (!(p->nu > 0.0) || !std::isfinite(p->nu)) { why = "nu must be positive"; return false; }
    if (!(1.0 / (3.0 * p->nu + 0.5) < 2.0)) { why = "omega must stay below 2"; return false; }
    if (!(p->sigma >= 0.0) || !std::isfinite(p->sigma)) { why = "sigma must be >= 0"; return false; }
    if (!(p->width > 0.0) || !std::isfinite(p->width)) { why = "width must be positive"; return false; }
    // eps regularises n = G/(|G| + eps) where G vanishes (Eq. 21): zero, non-finite
    // or below the binary32 normal range would turn flat regions into NaN
    if (!std::isfinite(p->eps) || (p->eps >= 0.0 && !(p->eps >= 1e-30))) {
        why = "eps must be >= 1e-30 (or < 0 for the default)";
        return false;
    }
    if (p->storage < TSLB_STORE_FP32 || p->storage > TSLB_STORE_FP16Q) { why = "unknown storage"; return false; }
    if (p->components != 1 && p->components != 2) { why = "components must be 1 or 2"; return false; }
    if (p->check_interval < 0) { why = "check_interval must be >= 0"; return false; }
    if (!(p->max_mass_drift >= 0.0) || !std::isfinite(p->max_mass_drift)) {
        why = "max_mass_drift must be finite and >= 0";
        return false;
    }
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->gravity[a])) { why = "gravity must be finite"; return false; }
    if (p->variable_density != 0 && p->variable_density != 1) { why = "variable_density must be 0 or 1"; return false; }
    if (p->variable_density) {
        if (p->components != 2) { why = "variable density needs two components"; return false; }
        if (p->storage != TSLB_STORE_FP32) { why = "variable density supports binary32 storage only"; return false; }
        if (!(p->density_a > 0.0) || !(p->density_b > 0.0) || !std::isfinite(p->density_a) ||
            !std::isfinite(p->density_b)) {
            why = "density_a and density_b must be positive";
            return false;
        }
        const double nus[2] = {p->nu_a, p->nu_b};
        for (double v : nus)
            if (!(v > 0.0) || !std::isfinite(v) || !(1.0 / (3.0 * v + 0.5) < 2.0)) {
                why = "nu_a and nu_b must be positive";
                return false;
            }
    } else if (p->gravity[0] != 0.0 || p->gravity[1] != 0.0 || p->gravity[2] != 0.0) {
        why = "gravity needs variable_density = 1";
        return false;
    }
    if (p->bc[4] == TSLB_BC_INLET && !(p->inlet_d > 0.0)) { why = "inlet_d must be positive"; return false; }
    return true;
}

// Scratch planes (binary32, 80 B per node together) used by set-state and
// readout (staging and geometry), by the statistics samples (geometry) and by
// the materialised-geometry step (geometry).  Allocated on demand; an
// allocation failure is TSLB_E_NOMEM.
int ensure_planes(tslb_ctx *c, bool stage, bool geo) {
    const size_t ld = (size_t)c->geo.ld;
    if (stage && !c->scratch.stage) {
        hipError_t e = hipMalloc((void **)&c->scratch.stage, 11 * ld * sizeof(float));
        if (e != hipSuccess) {
            c->scratch.stage = nullptr;
            return fail(c, TSLB_E_NOMEM, std::string("hipMalloc(staging planes): ") + hipGetErrorString(e));
        }
    }
    if (geo && !c->scratch.geo) {
        hipError_t e = hipMalloc((void **)&c->scratch.geo, 9 * ld * sizeof(float));
        if (e != hipSuccess) {
            c->scratch.geo = nullptr;
            return fail(c, TSLB_E_NOMEM, std::string("hipMalloc(geometry planes): ") + hipGetErrorString(e));
        }
    }
    return TSLB_OK;
}

// Give back the scratch planes once a set-state or readout call is done with
// them, so that between calls a context holds its two state buffers (what a
// serving group charges) plus the few kilobytes of diagnostics partials.  The
// geometry planes stay while statistics are sampled or the materialised-geometry
// step is selected.  Synchronises the stream first.
int release_planes(tslb_ctx *c) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->scratch.stage) {
        HIP_TRY(c, hipFree(c->scratch.stage));
        c->scratch.stage = nullptr;
    }
    if (c->scratch.geo && c->stats.every == 0 && c->kernel != TSLB_KERNEL_GATHER) {
        HIP_TRY(c, hipFree(c->scratch.geo));
        c->scratch.geo = nullptr;
    }
    return TSLB_OK;
}

int fill_boundary_now(tslb_ctx *c) {
    HIP_TRY(c, launch_boundary(c, c->buf[c->cur], c->step, c->stream));
    return TSLB_OK;
}

// Mass of a state from its diagnostics sums: N + sum rho' (equal densities), or
// with variable density rho_b N + (rho_a - rho_b) sum(phi), the sum of
// rho(phi) (exactly conserved with the phase field).
double mass_of(const tslb_ctx *c, const double d[2], long long phi_fixed) {
#pragma clang fp contract(off)  // products and sum rounded separately (as the no-alloc path forms them)
    if (c->vd)
        return c->p.density_b * (double)c->geo.N +
               (c->p.density_a - c->p.density_b) * std::ldexp((double)phi_fixed, -kPhiFrac);
    return (double)c->geo.N + d[0];
}

// out[0] = sum rho', out[1] = finite probe (NaN iff a stored moment is not finite),
// *phi_fixed = exact sum of the fixed-point phase field.
int run_diagnostics(tslb_ctx *c, double out[2], long long *phi_fixed) {
    HIP_TRY(c, launch_diagnostics(c, c->buf[c->cur], c->scratch, c->stream));
    HIP_TRY(c, hipMemcpyAsync(out, c->scratch.result, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(phi_fixed, c->scratch.result_i, sizeof(long long), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TSLB_OK;
}

}  // namespace

namespace tslb {
void set_thread_error(const std::string &msg) { g_thread_error = msg; }

bool validate_params(const tslb_params *p, std::string &why) { return validate(p, why); }

void derive_layout(const tslb_params *p, Geo &g, Scales &sc) {
    g.nx = p->nx; g.ny = p->ny; g.nz = p->nz;
    for (int a = 0; a < 3; ++a) g.per[a] = p->bc[2 * a] == TSLB_BC_PERIODIC;
    g.N = (long long)p->nx * p->ny * p->nz;
    g.ld = (long long)plane_elems(g.N);
    double U = p->u_scale > 0.0 ? p->u_scale : 0.05;
    if (p->storage == TSLB_STORE_FP32) U = 1.0;
    sc.s1 = (float)U;
    sc.s2 = (float)(U * U);
    sc.inv_s1 = (float)(1.0 / U);
    sc.inv_s2 = (float)(1.0 / (U * U));
}

size_t ctx_device_bytes(const tslb_ctx *c) {
    const size_t ld = (size_t)c->geo.ld;
    size_t b = 2 * c->buffer_bytes;
    b += c->scratch.partial_blocks * (2 * sizeof(double) + sizeof(long long)) + 2 * sizeof(double) + sizeof(long long);
    if (c->scratch.stage) b += 11 * ld * sizeof(float);
    if (c->scratch.geo) b += 9 * ld * sizeof(float);
    if (c->stats.sum) b += 5 * ld * sizeof(double);
    return b;
}
}  // namespace tslb

// A context that is a member of a serving group is advanced by the group; every
// call that reads or writes its state waits until the group has retired it.
#define NOT_IN_GROUP(c)                                                                                  \
    do {                                                                                                 \
        if ((c)->group) return fail((c), TSLB_E_STATE, "ctx is a member of a serving group");           \
    } while (0)

// Every call that issues device work first makes the context's device current,
// so a caller may switch devices between calls.
#define ON_DEVICE(c) HIP_TRY((c), hipSetDevice((c)->p.device))

extern "C" {

void tslb_params_init(tslb_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->abi_version = TSLB_ABI_VERSION;
    p->nx = p->ny = p->nz = 32;
    p->nu = 0.1;
    p->sigma = 0.0;
    p->width = 3.0;
    p->gamma = 0.0;
    p->eps = -1.0;
    p->storage = TSLB_STORE_FP32;
    p->components = 2;
    p->u_scale = 0.0;
}

size_t tslb_params_size(void) { return sizeof(tslb_params); }

size_t tslb_required_bytes(const tslb_params *p) {
    std::string why;
    if (!validate(p, why)) return 0;
    long long N = (long long)p->nx * p->ny * p->nz;
    return 2 * state_buffer_bytes(N, p->storage, p->components == 2);
}

int tslb_create(const tslb_params *p, tslb_ctx **out) {
    if (!out) return fail(nullptr, TSLB_E_INVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    if (!validate(p, why)) return fail(nullptr, TSLB_E_INVAL, why);
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return fail(nullptr, TSLB_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    tslb_ctx *c = new (std::nothrow) tslb_ctx();
    if (!c) return fail(nullptr, TSLB_E_NOMEM, "host allocation failed");
    c->p = *p;
    c->storage = p->storage;
    c->phase = p->components == 2;
    c->vd = p->variable_density == 1;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus > 0)
            c->cu_count = cus;
    }
    derive_layout(p, c->geo, c->scales);
    {
        const FusedPlan pl = fused_plan(c);
        c->plan_rows = pl.rows;
        c->plan_lz = pl.lz;
    }
    const Geo &g = c->geo;
    c->has_boundary = !(g.per[0] && g.per[1] && g.per[2]);
    Phys &ph = c->phys;
    ph.omega = (float)(1.0 / (3.0 * p->nu + 0.5));
    ph.sigma = c->phase ? (float)p->sigma : 0.0f;
    ph.gamma = (float)(p->gamma > 0.0 ? p->gamma : 2.0 / p->width);
    ph.eps = (float)(p->eps >= 0.0 ? p->eps : 1e-4);
    ph.width = (float)p->width;
    ph.inlet_u = (float)p->inlet_u;
    ph.inlet_d = (float)p->inlet_d;
    ph.inlet_noise = (float)p->inlet_noise;
    ph.noise_key = splitmix_finalise(p->seed + 0x9e3779b97f4a7c15ULL);
    for (int s = 0; s < 6; ++s) ph.bc[s] = p->bc[s];
    ph.rho_b = c->vd ? (float)p->density_b : 1.0f;
    ph.drho = c->vd ? (float)(p->density_a - p->density_b) : 0.0f;
    ph.nu_b = c->vd ? (float)p->nu_b : (float)p->nu;
    ph.dnu = c->vd ? (float)(p->nu_a - p->nu_b) : 0.0f;
    for (int a = 0; a < 3; ++a) ph.grav[a] = (float)p->gravity[a];
    c->buffer_bytes = state_buffer_bytes(g.N, c->storage, c->phase);
    size_t need = 2 * c->buffer_bytes;
    if (p->device_buffer) {
        if (p->device_buffer_bytes < need) {
            delete c;
            return fail(nullptr, TSLB_E_INVAL, "device_buffer is smaller than tslb_required_bytes()");
        }
        if (((uintptr_t)p->device_buffer & 255u) != 0) {
            delete c;
            return fail(nullptr, TSLB_E_INVAL, "device_buffer must be 256-byte aligned");
        }
        c->base = p->device_buffer;
        c->owns_base = false;
    } else {
        e = hipMalloc(&c->base, need);
        if (e != hipSuccess) {
            delete c;
            return fail(nullptr, TSLB_E_NOMEM, std::string("hipMalloc(state): ") + hipGetErrorString(e));
        }
        c->owns_base = true;
    }
    const size_t mom_bytes = moment_bytes(c->storage, g.ld);
    for (int b = 0; b < 2; ++b) {
        char *base = (char *)c->base + b * c->buffer_bytes;
        c->buf[b].mom = base;
        c->buf[b].phi = c->phase ? (int32_t *)(base + mom_bytes) : nullptr;
    }
    if (p->stream) {
        c->stream = (hipStream_t)p->stream;
        c->owns_stream = false;
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            tslb_destroy(c);
            return fail(nullptr, TSLB_E_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
        c->owns_stream = true;
    }
    c->scratch.partial_blocks = diagnostics_blocks(c);
    e = hipMalloc((void **)&c->scratch.partial, c->scratch.partial_blocks * 2 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&c->scratch.partial_i, c->scratch.partial_blocks * sizeof(long long));
    if (e == hipSuccess) e = hipMalloc((void **)&c->scratch.result, 2 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&c->scratch.result_i, sizeof(long long));
    if (e == hipSuccess) e = hipMemsetAsync(c->base, 0, need, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        tslb_destroy(c);
        return fail(nullptr, TSLB_E_DEVICE, std::string("context set-up: ") + hipGetErrorString(e));
    }
    *out = c;
    return TSLB_OK;
}

int tslb_set_state(tslb_ctx *c, const float *rho_dev, const float *u, const float *pi_neq, const float *phi,
                   int64_t step) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    ON_DEVICE(c);
    if (!rho_dev || !u || !pi_neq || (!phi && c->phase)) return fail(c, TSLB_E_INVAL, "every field is required");
    if (step < 0) return fail(c, TSLB_E_INVAL, "step must be >= 0");
    int rc = ensure_planes(c, true, true);
    if (rc) return rc;
    const size_t N = (size_t)c->geo.N, ld = (size_t)c->geo.ld;
    float *st = c->scratch.stage;
    hipError_t e = hipMemcpyAsync(st, rho_dev, N * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpy2DAsync(st + ld, ld * 4, u, N * 4, N * 4, 3, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(st + 4 * ld, ld * 4, pi_neq, N * 4, N * 4, 6, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && c->phase) e = hipMemcpyAsync(st + 10 * ld, phi, N * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_set_state(c, st, c->scratch.geo, c->buf[c->cur], c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    rc = release_planes(c);
    if (e != hipSuccess) return fail(c, TSLB_E_DEVICE, std::string("set state: ") + hipGetErrorString(e));
    if (rc) return rc;
    c->step = step;
    c->state_set = true;
    c->mass_ref_set = false;
    return TSLB_OK;
}

int tslb_set_state_rest(tslb_ctx *c, int64_t step) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    ON_DEVICE(c);
    if (step < 0) return fail(c, TSLB_E_INVAL, "step must be >= 0");
    // rho' = 0, ubar = 0, Q = 0 and phi = 0 are all-zero words in every storage type
    HIP_TRY(c, hipMemsetAsync(c->buf[c->cur].mom, 0, c->buffer_bytes, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->step = step;
    c->state_set = true;
    c->mass_ref_set = false;
    return TSLB_OK;
}

int tslb_step(tslb_ctx *c, int64_t nsteps) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    ON_DEVICE(c);
    if (nsteps < 0) return fail(c, TSLB_E_INVAL, "nsteps must be >= 0");
    if (!c->state_set) return fail(c, TSLB_E_STATE, "no state: call tslb_set_state first");
    int rc = ensure_planes(c, false, c->kernel == TSLB_KERNEL_GATHER || c->stats.every > 0);
    if (rc) return rc;
    StepTimer &tm = c->timer;
    const size_t max_timed = 8192;
    size_t timed = 0;
    if (tm.enabled) {
        size_t want = (size_t)(nsteps < (int64_t)max_timed ? nsteps : (int64_t)max_timed);
        try {
            tm.ev.reserve(2 * want);
        } catch (const std::bad_alloc &) {
            return fail(c, TSLB_E_NOMEM, "host allocation failed (timing events)");
        }
        while (tm.ev.size() < 2 * want) {
            hipEvent_t ev;
            HIP_TRY(c, hipEventCreate(&ev));
            tm.ev.push_back(ev);  // capacity reserved: does not throw
        }
        tm.used = 0;
    }
    // The fused kernel writes the boundary layers of the state it produces; the
    // current state's layers are filled once here (the fill is idempotent).
    const bool fused = c->kernel == TSLB_KERNEL_FUSED;
    if (fused && nsteps > 0) HIP_TRY(c, launch_boundary(c, c->buf[c->cur], c->step, c->stream));
    // the mass bound is relative to the mass of the state stepping started from
    const bool mass_check = c->p.check_interval > 0 && c->p.max_mass_drift > 0.0;
    if (mass_check && nsteps > 0 && !c->mass_ref_set) {
        double d[2];
        long long phi_sum;
        if (!fused) {
            rc = fill_boundary_now(c);
            if (rc) return rc;
        }
        rc = run_diagnostics(c, d, &phi_sum);
        if (rc) return rc;
        c->mass_ref = mass_of(c, d, phi_sum);
        c->mass_ref_set = true;
    }
    for (int64_t s = 0; s < nsteps; ++s) {
        if (!fused) HIP_TRY(c, launch_boundary(c, c->buf[c->cur], c->step, c->stream));
        bool timing = tm.enabled && timed < max_timed;
        if (timing) HIP_TRY(c, hipEventRecord(tm.ev[2 * timed], c->stream));
        HIP_TRY(c, launch_step(c, c->buf[c->cur], c->buf[c->cur ^ 1], c->step + 1, c->stream));
        if (timing) {
            HIP_TRY(c, hipEventRecord(tm.ev[2 * timed + 1], c->stream));
            ++timed;
        }
        c->cur ^= 1;
        c->step += 1;
        if (c->stats.every > 0 && c->step % c->stats.every == 0) {
            HIP_TRY(c, launch_geometry(c, c->buf[c->cur].phi, c->scratch.geo, c->stream));
            HIP_TRY(c, launch_stats_accum(c, c->buf[c->cur], c->scratch.geo, c->stats.sum, c->stream));
            c->stats.samples += 1;
        }
        if (c->p.check_interval > 0 && c->step % c->p.check_interval == 0) {
            double d[2];
            long long phi_sum;
            rc = fill_boundary_now(c);
            if (rc) return rc;
            rc = run_diagnostics(c, d, &phi_sum);
            if (rc) return rc;
            if (!std::isfinite(d[1])) {
                tm.used = timed;
                char msg[160];
                std::snprintf(msg, sizeof msg, "non-finite state at step %lld", (long long)c->step);
                return fail(c, TSLB_E_UNSTABLE, msg);
            }
            if (mass_check) {
                const double mass = mass_of(c, d, phi_sum);
                const double drift = std::fabs(mass - c->mass_ref) / std::fabs(c->mass_ref);
                if (!(drift <= c->p.max_mass_drift)) {
                    tm.used = timed;
                    char msg[200];
                    std::snprintf(msg, sizeof msg, "mass drifted by %.3e (relative, bound %.3e) at step %lld", drift,
                                  c->p.max_mass_drift, (long long)c->step);
                    return fail(c, TSLB_E_UNSTABLE, msg);
                }
            }
        }
    }
    if (tm.enabled) tm.used = timed;
    return TSLB_OK;
}

int tslb_sync(tslb_ctx *c) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    ON_DEVICE(c);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TSLB_OK;
}

int tslb_moments(tslb_ctx *c, float *rho_dev, float *u, float *pi_neq) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    ON_DEVICE(c);
    if (!c->state_set) return fail(c, TSLB_E_STATE, "no state");
    int rc = fill_boundary_now(c);
    if (rc) return rc;
    rc = ensure_planes(c, true, true);
    if (rc) return rc;
    const size_t N = (size_t)c->geo.N, ld = (size_t)c->geo.ld;
    float *st = c->scratch.stage;
    hipError_t e = launch_geometry(c, c->buf[c->cur].phi, c->scratch.geo, c->stream);
    if (e == hipSuccess) e = launch_readout(c, c->buf[c->cur], c->scratch.geo, st, c->stream);
    if (e == hipSuccess && rho_dev) e = hipMemcpyAsync(rho_dev, st, N * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && u) e = hipMemcpy2DAsync(u, N * 4, st + ld, ld * 4, N * 4, 3, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && pi_neq)
        e = hipMemcpy2DAsync(pi_neq, N * 4, st + 4 * ld, ld * 4, N * 4, 6, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    rc = release_planes(c);
    if (e != hipSuccess) return fail(c, TSLB_E_DEVICE, std::string("readout: ") + hipGetErrorString(e));
    return rc;
}

int tslb_phase(tslb_ctx *c, float *phi) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    ON_DEVICE(c);
    if (!phi) return fail(c, TSLB_E_INVAL, "phi is NULL");
    if (!c->state_set) return fail(c, TSLB_E_STATE, "no state");
    int rc = fill_boundary_now(c);
    if (rc) return rc;
    const size_t N = (size_t)c->geo.N;
    if (!c->phase) {  // a single component has no phase field
        std::fill(phi, phi + N, 0.0f);
        return TSLB_OK;
    }
    // the fixed-point words land in the caller's array and are converted in place
    HIP_TRY(c, hipMemcpyAsync(phi, c->buf[c->cur].phi, N * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < N; ++i) {
        int32_t v;
        std::memcpy(&v, phi + i, 4);
        phi[i] = phi_to_float(v);
    }
    return TSLB_OK;
}

size_t tslb_state_bytes(const tslb_ctx *c) { return c ? c->buffer_bytes : 0; }

size_t tslb_device_bytes(const tslb_ctx *c) { return c ? ctx_device_bytes(c) : 0; }

int tslb_get_state_raw(tslb_ctx *c, void *host, size_t bytes) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    ON_DEVICE(c);
    if (!host || bytes != c->buffer_bytes) return fail(c, TSLB_E_INVAL, "bytes must equal tslb_state_bytes()");
    if (!c->state_set) return fail(c, TSLB_E_STATE, "no state");
    int rc = fill_boundary_now(c);
    if (rc) return rc;
    HIP_TRY(c, hipMemcpyAsync(host, c->buf[c->cur].mom, bytes, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return TSLB_OK;
}

int tslb_set_state_raw(tslb_ctx *c, const void *host, size_t bytes, int64_t step) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    ON_DEVICE(c);
    if (!host || bytes != c->buffer_bytes) return fail(c, TSLB_E_INVAL, "bytes must equal tslb_state_bytes()");
    if (step < 0) return fail(c, TSLB_E_INVAL, "step must be >= 0");
    HIP_TRY(c, hipMemcpyAsync(c->buf[c->cur].mom, host, bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->step = step;
    c->state_set = true;
    c->mass_ref_set = false;
    return TSLB_OK;
}

int tslb_diagnostics(tslb_ctx *c, double *mass, double *phase_sum, int64_t *step, int32_t *finite) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    ON_DEVICE(c);
    if (!c->state_set) return fail(c, TSLB_E_STATE, "no state");
    int rc = fill_boundary_now(c);
    if (rc) return rc;
    double d[2];
    long long phi_fixed = 0;
    rc = run_diagnostics(c, d, &phi_fixed);
    if (rc) return rc;
    if (mass) *mass = mass_of(c, d, phi_fixed);
    if (phase_sum) *phase_sum = std::ldexp((double)phi_fixed, -kPhiFrac);
    if (step) *step = c->step;
    if (finite) *finite = std::isfinite(d[1]) ? 1 : 0;
    return TSLB_OK;
}

int64_t tslb_step_index(const tslb_ctx *c) { return c ? c->step : -1; }

int tslb_set_kernel(tslb_ctx *c, int kernel, int chunk_z) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    if (kernel != TSLB_KERNEL_FUSED && kernel != TSLB_KERNEL_GATHER) return fail(c, TSLB_E_INVAL, "unknown kernel");
    if (kernel == TSLB_KERNEL_GATHER && c->vd)
        return fail(c, TSLB_E_INVAL, "variable density runs on the fused kernel only");
    if (chunk_z < 0) return fail(c, TSLB_E_INVAL, "chunk_z must be >= 0");
    c->kernel = kernel;
    c->chunk_z = chunk_z;
    const FusedPlan pl = fused_plan(c);
    c->plan_rows = pl.rows;
    c->plan_lz = pl.lz;
    return TSLB_OK;
}

int tslb_set_tile(tslb_ctx *c, int rows) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    if (rows != 0 && rows != 16 && rows != 20) return fail(c, TSLB_E_INVAL, "rows must be 0, 16 or 20");
    if (rows == 20 && !fused_wide_allowed(c))
        return fail(c, TSLB_E_INVAL, "20-row tiles serve the two-component step with equal densities only");
    c->tile_rows = rows;
    const FusedPlan pl = fused_plan(c);
    c->plan_rows = pl.rows;
    c->plan_lz = pl.lz;
    return TSLB_OK;
}

int tslb_tile_rows(const tslb_ctx *c) { return c ? c->plan_rows : TSLB_E_INVAL; }

int tslb_set_timing(tslb_ctx *c, int enable) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    c->timer.enabled = enable != 0;
    c->timer.used = 0;
    return TSLB_OK;
}

double tslb_last_step_kernel_ms(tslb_ctx *c) {
    if (!c || c->timer.used == 0) return 0.0;
    if (hipSetDevice(c->p.device) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) return 0.0;
    double total = 0.0;
    for (size_t k = 0; k < c->timer.used; ++k) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->timer.ev[2 * k], c->timer.ev[2 * k + 1]) != hipSuccess) return 0.0;
        total += ms;
    }
    return total / (double)c->timer.used;
}

int tslb_step_kernel_times(tslb_ctx *c, float *ms, int64_t cap, int64_t *count) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    if (cap < 0 || (cap > 0 && !ms) || !count) return fail(c, TSLB_E_INVAL, "bad output arguments");
    ON_DEVICE(c);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int64_t n = (int64_t)c->timer.used;
    for (int64_t k = 0; k < n && k < cap; ++k)
        HIP_TRY(c, hipEventElapsedTime(&ms[k], c->timer.ev[2 * k], c->timer.ev[2 * k + 1]));
    *count = n;
    return TSLB_OK;
}

int tslb_device_memory(int32_t device, size_t *free_bytes, size_t *total_bytes) {
    if (!free_bytes || !total_bytes) return fail(nullptr, TSLB_E_INVAL, "output pointers are required");
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMemGetInfo(free_bytes, total_bytes);
    if (e != hipSuccess) return fail(nullptr, TSLB_E_DEVICE, std::string("hipMemGetInfo: ") + hipGetErrorString(e));
    return TSLB_OK;
}

int tslb_copy_bandwidth(int device, size_t bytes, int iters, double *gbps, double *ms) {
    if (bytes == 0 || bytes % 16 != 0 || iters < 1 || !gbps || !ms)
        return fail(nullptr, TSLB_E_INVAL, "bytes must be a positive multiple of 16 and iters >= 1");
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, TSLB_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    void *a = nullptr, *b = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<float> times;
    try {
        times.reserve((size_t)iters);
    } catch (const std::bad_alloc &) {
        return fail(nullptr, TSLB_E_NOMEM, "host allocation failed");
    }
    int rc = TSLB_OK;
    e = hipMalloc(&a, bytes);
    if (e == hipSuccess) e = hipMalloc(&b, bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMemsetAsync(a, 0, bytes, s);
    for (int k = 0; e == hipSuccess && k < iters + 1; ++k) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = launch_copy_probe(a, b, bytes, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e == hipSuccess && k > 0) times.push_back(t);  // the first launch is a warm-up
    }
    if (e != hipSuccess) {
        rc = fail(nullptr, TSLB_E_DEVICE, std::string("copy probe: ") + hipGetErrorString(e));
    } else {
        std::sort(times.begin(), times.end());
        const double med = times[times.size() / 2];
        *ms = med;
        *gbps = 2.0 * (double)bytes / (med * 1e-3) / 1e9;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    return rc;
}

int tslb_stats_start(tslb_ctx *c, int32_t every) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    ON_DEVICE(c);
    if (every < 1) return fail(c, TSLB_E_INVAL, "every must be >= 1");
    if (c->vd) return fail(c, TSLB_E_INVAL, "time averages are not available with variable density");
    int rc = ensure_planes(c, false, true);
    if (rc) return rc;
    const size_t bytes = 5 * (size_t)c->geo.ld * sizeof(double);
    if (!c->stats.sum) {
        hipError_t e = hipMalloc((void **)&c->stats.sum, bytes);
        if (e != hipSuccess) return fail(c, TSLB_E_NOMEM, std::string("hipMalloc(stats): ") + hipGetErrorString(e));
    }
    HIP_TRY(c, hipMemsetAsync(c->stats.sum, 0, bytes, c->stream));
    c->stats.every = every;
    c->stats.samples = 0;
    return TSLB_OK;
}

int tslb_stats_stop(tslb_ctx *c) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    ON_DEVICE(c);
    c->stats.every = 0;
    return release_planes(c);
}

int tslb_stats_get(tslb_ctx *c, float *mean_phi, float *mean_u, float *rms_uz, int64_t *samples) {
    if (!c) return fail(nullptr, TSLB_E_INVAL, "ctx is NULL");
    NOT_IN_GROUP(c);
    ON_DEVICE(c);
    if (samples) *samples = c->stats.samples;
    if (!mean_phi && !mean_u && !rms_uz) return TSLB_OK;
    if (!c->stats.sum || c->stats.samples == 0) return fail(c, TSLB_E_STATE, "no samples: call tslb_stats_start and step");
    const size_t N = (size_t)c->geo.N, ld = (size_t)c->geo.ld;
    // the five sum planes come over in blocks of nodes through a bounded host buffer
    const size_t blk = std::min(N, (size_t)1 << 22);
    std::vector<double> h;
    try {
        h.resize(5 * blk);
    } catch (const std::bad_alloc &) {
        return fail(c, TSLB_E_NOMEM, "host allocation failed (statistics block)");
    }
    const double inv = 1.0 / (double)c->stats.samples;
    for (size_t b0 = 0; b0 < N; b0 += blk) {
        const size_t nb = std::min(blk, N - b0);
        HIP_TRY(c, hipMemcpy2DAsync(h.data(), blk * sizeof(double), c->stats.sum + b0, ld * sizeof(double),
                                    nb * sizeof(double), 5, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (size_t k = 0; k < nb; ++k) {
            const size_t i = b0 + k;
            if (mean_phi) mean_phi[i] = (float)(h[k] * inv);
            if (mean_u)
                for (int a = 0; a < 3; ++a) mean_u[a * N + i] = (float)(h[(1 + a) * blk + k] * inv);
            if (rms_uz) {
                const double m = h[3 * blk + k] * inv, var = h[4 * blk + k] * inv - m * m;
                rms_uz[i] = (float)std::sqrt(var > 0.0 ? var : 0.0);
            }
        }
    }
    return TSLB_OK;
}

void tslb_destroy(tslb_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->p.device);
    if (c->group) group_detach(c->group, c);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t ev : c->timer.ev) (void)hipEventDestroy(ev);
    if (c->scratch.stage) (void)hipFree(c->scratch.stage);
    if (c->scratch.geo) (void)hipFree(c->scratch.geo);
    if (c->scratch.partial) (void)hipFree(c->scratch.partial);
    if (c->scratch.partial_i) (void)hipFree(c->scratch.partial_i);
    if (c->scratch.result) (void)hipFree(c->scratch.result);
    if (c->scratch.result_i) (void)hipFree(c->scratch.result_i);
    if (c->stats.sum) (void)hipFree(c->stats.sum);
    if (c->owns_base && c->base) (void)hipFree(c->base);
    if (c->owns_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *tslb_last_error(const tslb_ctx *c) { return c ? c->err.c_str() : g_thread_error.c_str(); }

}  // extern "C"
