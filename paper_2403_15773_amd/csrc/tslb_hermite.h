// Moment-to-population projection of the step: the regularised post-collision
// populations of one node, written as brackets tau_i = f_i/w_i - 1 - rho', from
// the scaled Hermite coefficients of that node (Eqs. 15-19):
//   tau(c) = K1 . c + K2_aa h(c_a) + K2_ab c_a c_b + K3_aab h(c_a) c_b + K3_xyz c_x c_y c_z,
// with h(c) = c^2 - 1/3, K1 = 3 J, K2_aa = 4.5 a2_aa, K2_ab = 9 a2_ab (a != b),
// K3_aab = 13.5 a3_aab, K3_xyz = 27 a3_xyz.  The fused step (stage S4) evaluates
// the same tensor product inline, with the scale factors of the coefficients
// folded into the constants of the multiply-adds that take them (eleven fewer
// multiplies); the projection probe keeps the scaled coefficients as its inputs
// and times this form of the same product.  (Routing the step itself through
// this function changes its instruction schedule and costs ~3 %.)
#pragma once

#include <hip/hip_runtime.h>

namespace tslb {

struct HermiteK {
    float K1x, K1y, K1z;
    float K2xx, K2yy, K2zz, K2xy, K2xz, K2yz;
    float K3xxy, K3xxz, K3yyx, K3yyz, K3zzx, K3zzy, K3xyz;
};

// Quadratic A + B c + C (c^2 - 1/3) at c = -1, 0, +1.
__device__ __forceinline__ void quad3(float A, float B, float C, float &vm, float &v0, float &vp) {
    const float m = fmaf(C, 2.0f / 3.0f, A);
    v0 = fmaf(C, -1.0f / 3.0f, A);
    vm = m - B;
    vp = m + B;
}

// tau on the 27 velocities as a tensor product of 1-D quadratics in c_x, c_y, c_z:
// tau = T0 + c_z T1 + h(c_z) T2 with T0 = U0 + c_y U1 + h(c_y) U2 (per c_x), etc.
// Groups tm, t0, tp hold c_z = -1, 0, +1, index (c_x + 1) + 3 (c_y + 1).
__device__ __forceinline__ void populations_from_hermite(const HermiteK &k, float tm[9], float t0[9], float tp[9]) {
    float U0[3], U1[3], V0[3], W0[3];
    quad3(0.0f, k.K1x, k.K2xx, U0[0], U0[1], U0[2]);
    quad3(k.K1y, k.K2xy, k.K3xxy, U1[0], U1[1], U1[2]);
    quad3(k.K1z, k.K2xz, k.K3xxz, V0[0], V0[1], V0[2]);
    W0[0] = k.K2zz - k.K3zzx;
    W0[1] = k.K2zz;
    W0[2] = k.K2zz + k.K3zzx;
#pragma unroll
    for (int ix = 0; ix < 3; ++ix) {
        const float cx = (float)(ix - 1);
        const float U2 = fmaf(k.K3yyx, cx, k.K2yy);  // linear in c_x
        const float V1 = fmaf(k.K3xyz, cx, k.K2yz);
        float T0[3], T1[3], T2[3];
        quad3(U0[ix], U1[ix], U2, T0[0], T0[1], T0[2]);
        quad3(V0[ix], V1, k.K3yyz, T1[0], T1[1], T1[2]);
        T2[0] = W0[ix] - k.K3zzy;
        T2[1] = W0[ix];
        T2[2] = W0[ix] + k.K3zzy;
#pragma unroll
        for (int iy = 0; iy < 3; ++iy) {
            const int i = ix + 3 * iy;
            const float mid = fmaf(T2[iy], 2.0f / 3.0f, T0[iy]);
            t0[i] = fmaf(T2[iy], -1.0f / 3.0f, T0[iy]);
            tm[i] = mid - T1[iy];
            tp[i] = mid + T1[iy];
        }
    }
}

}  // namespace tslb
