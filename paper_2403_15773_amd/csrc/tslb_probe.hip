// Measurement probe of the moment-to-population projection: 27 brackets tau_i of
// one node from its 16 scaled Hermite coefficients (a 27 x 16 linear map, see
// tslb_hermite.h), evaluated two ways on the same inputs:
//   kind 0: the tensor product of 1-D quadratics on the vector ALU (the step's code);
//   kind 1: the same map as FP32 matrix-core tiles, v_mfma_f32_32x32x2_f32.
// Each thread repeats the projection `reps` times with its coefficients moved by
// a constant step each time and accumulates the results, so the timed work is
// the projection itself (the inputs and outputs cross HBM once).
//
// Matrix-core mapping (one wave = 64 nodes = two 32-node column blocks): for the
// coefficient pair (k, k+1), block 0 needs coefficient k of nodes 0-31 in lanes
// 0-31 and coefficient k+1 of the same nodes in lanes 32-63, block 1 the same for
// nodes 32-63.  One v_permlane32_swap of (coef k, coef k+1) produces both
// operands.  The A operand holds the matrix entries A[m = lane % 32][k + lane / 32]
// (rows 27-31 zero); each block accumulates its 32 x 32 result in 16 registers.
#include <algorithm>
#include <new>
#include <vector>

#include "tslb_hermite.h"
#include "tslb_internal.h"

namespace tslb {
namespace probe {

constexpr int kThreads = 256;
constexpr float kStep = 1.0e-3f;  // coefficient step between repetitions

typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float h1(float c) { return c * c - 1.0f / 3.0f; }

// Entry of the projection matrix: basis function k of the coefficient list
// (K1x K1y K1z K2xx K2yy K2zz K2xy K2xz K2yz K3xxy K3xxz K3yyx K3yyz K3zzx K3zzy K3xyz)
// at velocity m = 9 (c_z + 1) + (c_x + 1) + 3 (c_y + 1); 0 for the padding rows m >= 27.
__device__ __forceinline__ float basis(int m, int k) {
    if (m >= 27) return 0.f;
    const float cz = (float)(m / 9 - 1), cx = (float)(m % 3 - 1), cy = (float)((m % 9) / 3 - 1);
    switch (k) {
    case 0: return cx;
    case 1: return cy;
    case 2: return cz;
    case 3: return h1(cx);
    case 4: return h1(cy);
    case 5: return h1(cz);
    case 6: return cx * cy;
    case 7: return cx * cz;
    case 8: return cy * cz;
    case 9: return h1(cx) * cy;
    case 10: return h1(cx) * cz;
    case 11: return h1(cy) * cx;
    case 12: return h1(cy) * cz;
    case 13: return h1(cz) * cx;
    case 14: return h1(cz) * cy;
    default: return cx * cy * cz;
    }
}

__device__ __forceinline__ void load_coef(const float *__restrict__ coef, long long n, long long id, float K[16]) {
#pragma unroll
    for (int k = 0; k < 16; ++k) K[k] = coef[k * n + id];
}

__global__ __launch_bounds__(kThreads) void k_project_valu(const float *__restrict__ coef, float *__restrict__ out,
                                                          long long n, int reps) {
    const long long id = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (id >= n) return;
    float K[16];
    load_coef(coef, n, id, K);
    float acc[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) acc[i] = 0.f;
    for (int r = 0; r < reps; ++r) {
        HermiteK h{K[0], K[1], K[2], K[3], K[4], K[5], K[6], K[7], K[8], K[9], K[10], K[11], K[12], K[13], K[14], K[15]};
        float tm[9], t0[9], tp[9];
        populations_from_hermite(h, tm, t0, tp);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            acc[i] += tm[i];
            acc[9 + i] += t0[i];
            acc[18 + i] += tp[i];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) K[k] += kStep;
    }
#pragma unroll
    for (int i = 0; i < 27; ++i) out[i * n + id] = acc[i];
}

// n is a multiple of 64 (whole waves): every lane of a wave takes part in the MFMA.
__global__ __launch_bounds__(kThreads) void k_project_mfma(const float *__restrict__ coef, float *__restrict__ out,
                                                          long long n, int reps) {
    const long long id = (long long)blockIdx.x * kThreads + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const long long wave_base = id - lane;
    if (wave_base >= n) return;  // a whole wave past the end (n is a multiple of 64)
    float K[16];
    load_coef(coef, n, id, K);
    float A[8];
#pragma unroll
    for (int kp = 0; kp < 8; ++kp) A[kp] = basis(lane & 31, 2 * kp + (lane >> 5));
    floatx16 acc0 = {}, acc1 = {};
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int kp = 0; kp < 8; ++kp) {
            const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(K[2 * kp]), __float_as_uint(K[2 * kp + 1]),
                                                             false, false);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(A[kp], __uint_as_float(sw[0]), acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(A[kp], __uint_as_float(sw[1]), acc1, 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) K[k] += kStep;
    }
    // result register q of a lane holds row 8 (q / 4) + 4 (lane / 32) + q % 4 of column lane % 32
    const long long col0 = wave_base + (lane & 31), col1 = col0 + 32;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int row = 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        if (row < 27) {
            out[row * n + col0] = acc0[q];
            out[row * n + col1] = acc1[q];
        }
    }
}

}  // namespace probe
}  // namespace tslb

using namespace tslb;

static int probe_fail(int code, const std::string &msg) {
    set_thread_error(msg);
    return code;
}

int tslb_probe_projection(int32_t kind, const float *coef_host, int64_t nodes, int32_t reps, int32_t iters,
                          int32_t device, float *out_host, double *ms) {
    if ((kind != 0 && kind != 1) || !coef_host || nodes <= 0 || nodes % 64 != 0 || reps < 1 || iters < 1 || !ms)
        return probe_fail(TSLB_E_INVAL, "kind 0/1, coef, nodes > 0 and a multiple of 64, reps >= 1, iters >= 1, ms");
    if (nodes > (1ll << 28)) return probe_fail(TSLB_E_INVAL, "nodes must be <= 2^28");
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return probe_fail(TSLB_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    const size_t in_bytes = 16 * (size_t)nodes * sizeof(float), out_bytes = 27 * (size_t)nodes * sizeof(float);
    float *d_in = nullptr, *d_out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<float> times;
    try {
        times.reserve((size_t)iters);
    } catch (const std::bad_alloc &) {
        return probe_fail(TSLB_E_NOMEM, "host allocation failed");
    }
    e = hipMalloc((void **)&d_in, in_bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&d_out, out_bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMemcpyAsync(d_in, coef_host, in_bytes, hipMemcpyHostToDevice, s);
    const unsigned blocks = (unsigned)((nodes + probe::kThreads - 1) / probe::kThreads);
    for (int k = 0; e == hipSuccess && k < iters + 1; ++k) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) {
            if (kind == 0)
                hipLaunchKernelGGL(probe::k_project_valu, dim3(blocks), dim3(probe::kThreads), 0, s, d_in, d_out,
                                   (long long)nodes, (int)reps);
            else
                hipLaunchKernelGGL(probe::k_project_mfma, dim3(blocks), dim3(probe::kThreads), 0, s, d_in, d_out,
                                   (long long)nodes, (int)reps);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e == hipSuccess && k > 0) times.push_back(t);  // the first launch is a warm-up
    }
    if (e == hipSuccess && out_host) e = hipMemcpyAsync(out_host, d_out, out_bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int rc = TSLB_OK;
    if (e != hipSuccess) {
        rc = probe_fail(TSLB_E_DEVICE, std::string("projection probe: ") + hipGetErrorString(e));
    } else {
        double sum = 0.0;
        for (float t : times) sum += t;
        *ms = sum / (double)times.size();
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (d_in) (void)hipFree(d_in);
    if (d_out) (void)hipFree(d_out);
    return rc;
}
