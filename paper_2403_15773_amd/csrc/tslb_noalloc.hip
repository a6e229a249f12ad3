// Conservation diagnostics of a caller-held state buffer without any device
// allocation (tslb_diagnostics_noalloc in include/tslb.h).
//
// tslb_diagnostics sums into per-context partials that tslb_create allocates.
// This variant runs the same two kernels (per-block partials, then their total
// in a fixed order) with its partials in `scratch`, a static device array of
// fixed size that every call on a device shares, so it calls no hipMalloc,
// hipFree or allocating library routine and can run where allocation is not
// allowed (under stream capture, in serving loops that forbid it).
//
// Host code never uses the array's name as a device address: the address of
// each device's copy is looked up once per device with hipGetSymbolAddress
// (with that device current) and kept in g_scratch_addr.
#include <cstring>
#include <mutex>
#include <string>

#include "tslb_internal.h"

using namespace tslb;

namespace {

constexpr int kMaxBlocks = 1024;  // partials of at most this many blocks (diagnostics_blocks_for's cap)
constexpr size_t kPartialBytes = (size_t)kMaxBlocks * 2 * sizeof(double);
constexpr size_t kPartialIBytes = (size_t)kMaxBlocks * sizeof(long long);
constexpr size_t kResultOffset = kPartialBytes + kPartialIBytes;
constexpr size_t kScratchBytes = kResultOffset + 2 * sizeof(double) + sizeof(long long);

// The scratch of every call on a device: block partials (2 doubles each), block
// phase sums (int64 each), then the totals (2 doubles, one int64).  24.6 KB.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (the device is current).
hipError_t scratch_address(int device, void **addr) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = p;
    }
    *addr = g_scratch_addr[device];
    return hipSuccess;
}

// out[0] = mass (N + sum rho', or with variable density rho_b N + drho sum phi),
// out[1] = phase sum (the exact fixed-point sum scaled by 2^-30), out[2] = 1 if
// every stored moment is finite, else 0: the values tslb_diagnostics returns,
// formed with the same binary64 operations.
__global__ void k_diag_export(const double *result, const long long *result_i, long long N, int vd, double rho_b,
                              double drho, double *out) {
#pragma clang fp contract(off)  // the host forms the same products and sum unfused
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double phase = (double)result_i[0] * (1.0 / (double)(1ll << kPhiFrac));
    out[0] = vd ? rho_b * (double)N + drho * phase : (double)N + result[0];
    out[1] = phase;
    out[2] = isfinite(result[1]) ? 1.0 : 0.0;
}

}  // namespace

extern "C" int tslb_diagnostics_noalloc(const tslb_params *p, const void *state, void *stream, double *out) {
    std::string why;
    if (!validate_params(p, why)) {
        set_thread_error(why);
        return TSLB_E_INVAL;
    }
    if (!state || !out) {
        set_thread_error("state and out must be device pointers");
        return TSLB_E_INVAL;
    }
    if (((uintptr_t)state & 3u) != 0 || ((uintptr_t)out & 7u) != 0) {
        set_thread_error("state must be 4-byte and out 8-byte aligned");
        return TSLB_E_INVAL;
    }
    if (p->device < 0 || p->device >= kMaxDevices) {
        set_thread_error("device ordinal out of range");
        return TSLB_E_INVAL;
    }
    Geo g;
    Scales sc;
    derive_layout(p, g, sc);
    const int blocks = diagnostics_blocks_for(g.N);
    if (blocks < 1 || blocks > kMaxBlocks) {  // diagnostics_blocks_for caps at kMaxBlocks
        set_thread_error("lattice needs more diagnostics partials than the static scratch holds");
        return TSLB_E_INVAL;
    }
    hipError_t e = hipSetDevice(p->device);
    void *base = nullptr;
    if (e == hipSuccess) e = scratch_address(p->device, &base);
    if (e != hipSuccess) {
        set_thread_error(std::string("scratch lookup: ") + hipGetErrorString(e));
        return TSLB_E_DEVICE;
    }
    char *b = (char *)base;
    double *partial = (double *)b;
    long long *partial_i = (long long *)(b + kPartialBytes);
    double *result = (double *)(b + kResultOffset);
    long long *result_i = (long long *)(b + kResultOffset + 2 * sizeof(double));
    StateView st;
    st.mom = const_cast<void *>(state);  // read only
    st.phi = p->components == 2 ? (int32_t *)((char *)st.mom + moment_bytes(p->storage, g.ld)) : nullptr;
    hipStream_t s = (hipStream_t)stream;
    e = launch_diagnostics_raw(g, sc, p->storage, st, partial, partial_i, blocks, result, result_i, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_diag_export, dim3(1), dim3(64), 0, s, result, result_i, g.N, p->variable_density,
                           p->density_b, p->density_a - p->density_b, out);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        set_thread_error(std::string("diagnostics launch: ") + hipGetErrorString(e));
        return TSLB_E_DEVICE;
    }
    return TSLB_OK;
}
