// Device-side definitions shared by the HIP kernels of the TSLB library (gfx950).
//
// State layout in HBM (one buffer; the library keeps two, A and B):
//   ten moment planes, each `ld` elements of the storage type T, in the order
//     0 rho' = rho - 1, 1..3 ubar = j/rho, 4..9 Q = Pi - rho c_s^2 I - j j/rho
//     (xx, yy, zz, xy, xz, yz),
//   then one plane of the phase field phi as signed fixed point: int32 with 30
//   fractional bits (resolution 2^-30 = 9.3e-10, values clamped to
//   [-0.45, 1.45] so that any difference of two values fits in int32), so that
//   phi near 1 keeps 64x finer resolution than binary32 and the phase streaming
//   runs in exact integer arithmetic (the phase sum is conserved bit for bit).
// Node (x, y, z) sits at element x + nx*(y + ny*z) of every plane.  `ld` is N
// rounded up to a multiple of 64, so every plane starts 256-byte aligned.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tslb {

constexpr int kPlanes = 10;  // stored moment planes (phi is separate)

// Lattice geometry as the kernels see it.
struct Geo {
    int nx, ny, nz;
    int per[3];      // 1 = periodic axis
    long long N;     // nx*ny*nz
    long long ld;    // plane stride in elements
};

// Physical parameters in binary32.
struct Phys {
    float omega;       // 1/(3 nu + 1/2)
    float sigma;       // surface tension
    float gamma;       // anti-diffusion constant
    float eps;         // regulariser of |grad phi|
    float width;       // interface width W
    float inlet_u, inlet_d, inlet_noise;
    unsigned long long noise_key;  // SplitMix64(seed)
    int bc[6];
    // variable density and viscosity (the fused kernel's VD instantiation):
    // rho(phi) = rho_b + drho phi, nu(phi) = nu_b + dnu phi (phi clamped to
    // [0, 1]), body acceleration grav
    float rho_b, drho, nu_b, dnu;
    float grav[3];
};

// Scaled-deviation storage: value = stored * scale.  FP32 storage uses scale 1.
struct Scales {
    float s2, s1;          // U^2 for rho' and Q, U for ubar
    float inv_s2, inv_s1;
};

// ---- storage traits -------------------------------------------------------

// FP32: ten binary32 planes.  FP16 / BF16: ten 16-bit planes holding the scaled
// deviations rho'/U^2, ubar/U, Q/U^2.  FP16Q: rho' and ubar in binary32, only
// the stress Q in binary16 (Q/U^2).
enum { ST_FP32 = 0, ST_FP16 = 1, ST_BF16 = 2, ST_FP16Q = 3 };

// Memory views.  A kernel that takes its state pointers from a table in memory
// (the multi-lattice step) can access them as global_t pointers (G = true): the
// compiler cannot tell otherwise that they address global memory and uses flat
// instructions, which also hold up every LDS wait.  The typed view keeps more
// plane addresses in scalar registers, so it pays only where those do not spill
// (binary32 storage of the multi-lattice step).  Where the pointers are kernel
// arguments the plain view (G = false) compiles better (the compiler infers
// global itself).
template <class T>
using global_t = __attribute__((address_space(1))) T;
template <bool G, class T> struct MemView { using P = T *; };
template <class T> struct MemView<true, T> { using P = global_t<T> *; };
template <bool G, class T>
__device__ __forceinline__ typename MemView<G, T>::P mem(T *p) {
    if constexpr (G)
        return (typename MemView<G, T>::P)p;
    else
        return p;
}

// binary32 -> bfloat16 bits, rounded to nearest even (a NaN stays a quiet NaN):
// one hardware conversion on gfx950 (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint16_t bf16_bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }

// binary32 -> binary16, rounded to nearest even, as a binary32 multiply (by the
// caller) and a separate conversion.  The empty asm keeps the compiler from
// folding the two into the mixed-precision multiply-add whose 16-bit result
// keeps the upper half of its destination register (and so waits for that
// register's previous value): the folded form made the FP16 step 2.5 % slower.
__device__ __forceinline__ _Float16 f16_of(float v) {
    __asm__("" : "+v"(v));
    return (_Float16)v;
}

template <int ST> struct Store;

template <> struct Store<ST_FP32> {
    using T = float;
    static __device__ __forceinline__ float load(const T *p, long long i, float) { return p[i]; }
    static __device__ __forceinline__ void store(T *p, long long i, float v, float) { p[i] = v; }
};

template <> struct Store<ST_FP16> {
    using T = _Float16;
    static __device__ __forceinline__ float load(const T *p, long long i, float s) { return (float)p[i] * s; }
    // the float -> half conversion rounds to nearest even
    static __device__ __forceinline__ void store(T *p, long long i, float v, float inv_s) { p[i] = f16_of(v * inv_s); }
};

template <> struct Store<ST_BF16> {
    using T = uint16_t;
    static __device__ __forceinline__ float load(const T *p, long long i, float s) {
        return __uint_as_float((uint32_t)p[i] << 16) * s;
    }
    static __device__ __forceinline__ void store(T *p, long long i, float v, float inv_s) { p[i] = bf16_bits(v * inv_s); }
};

// Bytes of the ten moment planes of one state buffer (planes of ld elements),
// rounded up to 256 so that the phase plane that follows is aligned.
__host__ __device__ inline size_t moment_bytes(int storage, long long ld) {
    const size_t per_node = storage == ST_FP32 ? 40 : (storage == ST_FP16Q ? 28 : 20);
    return ((size_t)ld * per_node + 255) / 256 * 256;
}

// Moment p of node id (0: rho', 1-3: ubar, 4-9: Q) from the planes at mom, as
// the binary32 physical value.  p is a compile-time constant at every call, so
// the plane's type and scale are resolved statically.
template <int ST>
__device__ __forceinline__ float load_moment(const void *mom, long long ld, int p, long long id, const Scales &sc) {
    if constexpr (ST == ST_FP32) {
        return ((const float *)mom)[p * ld + id];
    } else if constexpr (ST == ST_FP16Q) {
        if (p < 4) return ((const float *)mom)[p * ld + id];
        return Store<ST_FP16>::load((const _Float16 *)((const float *)mom + 4 * ld) + (p - 4) * ld, id, sc.s2);
    } else {
        using S = Store<ST>;
        return S::load((const typename S::T *)mom + p * ld, id, (p >= 1 && p < 4) ? sc.s1 : sc.s2);
    }
}

// The same moment in two halves, so that a prefetch can be issued long before
// its value is used: load_moment_bits returns the stored word (a 16-bit word
// zero-extended), decode_moment turns it into what load_moment returns.
template <int ST, bool G = false>
__device__ __forceinline__ uint32_t load_moment_bits(const void *mom, long long ld, int p, long long id) {
    if constexpr (ST == ST_FP32) {
        return mem<G>((const uint32_t *)mom)[p * ld + id];
    } else if constexpr (ST == ST_FP16Q) {
        if (p < 4) return mem<G>((const uint32_t *)mom)[p * ld + id];
        return mem<G>((const uint16_t *)((const float *)mom + 4 * ld))[(p - 4) * ld + id];
    } else {
        return mem<G>((const uint16_t *)mom)[p * ld + id];
    }
}

template <int ST>
__device__ __forceinline__ float decode_moment(uint32_t b, int p, const Scales &sc) {
    if constexpr (ST == ST_FP32) {
        return __uint_as_float(b);
    } else if constexpr (ST == ST_FP16Q) {
        if (p < 4) return __uint_as_float(b);
        return (float)__builtin_bit_cast(_Float16, (uint16_t)b) * sc.s2;
    } else if constexpr (ST == ST_FP16) {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)b) * ((p >= 1 && p < 4) ? sc.s1 : sc.s2);
    } else {
        return __uint_as_float(b << 16) * ((p >= 1 && p < 4) ? sc.s1 : sc.s2);
    }
}

// Stores of a new state carry the non-temporal hint: the fused step never reads
// back what it writes, and lines written without the hint take L2 capacity from
// the halo lines that its neighbouring workgroups read again.
template <class T, class P>
__device__ __forceinline__ void store_nt(P ptr, T v) {
    __builtin_nontemporal_store(v, ptr);
}

template <int ST, bool G = false>
__device__ __forceinline__ void store_moment(void *mom, long long ld, int p, long long id, float v, const Scales &sc) {
    if constexpr (ST == ST_FP32) {
        store_nt(&mem<G>((float *)mom)[p * ld + id], v);
    } else if constexpr (ST == ST_FP16Q) {
        if (p < 4)
            store_nt(&mem<G>((float *)mom)[p * ld + id], v);
        else
            store_nt(&mem<G>((_Float16 *)((float *)mom + 4 * ld) + (p - 4) * ld)[id], f16_of(v * sc.inv_s2));
    } else if constexpr (ST == ST_FP16) {
        store_nt(&mem<G>((_Float16 *)mom + p * ld)[id], f16_of(v * ((p >= 1 && p < 4) ? sc.inv_s1 : sc.inv_s2)));
    } else {
        store_nt(&mem<G>((uint16_t *)mom + p * ld)[id], bf16_bits(v * ((p >= 1 && p < 4) ? sc.inv_s1 : sc.inv_s2)));
    }
}

// ---- fixed-point phase field ----------------------------------------------

constexpr int kPhiFrac = 30;
constexpr int32_t kPhiOne = 1 << kPhiFrac;
constexpr float kPhiUlp = 1.0f / (float)(1 << kPhiFrac);   // 2^-30
constexpr float kPhiInvUlp = (float)(1 << kPhiFrac);       // 2^30
constexpr float kPhiMin = -0.45f, kPhiMax = 1.45f;

// The clamp bounds on the fixed-point grid.  Every stored phase value lies in
// [kPhiLo, kPhiHi], so a difference of two of them, (1.45 + 0.45) 2^30 at most,
// never overflows int32; a diverging run saturates there instead.
constexpr int32_t kPhiLo = (int32_t)(-0.45 * (double)(1 << kPhiFrac));
constexpr int32_t kPhiHi = (int32_t)(1.45 * (double)(1 << kPhiFrac));

__host__ __device__ inline float phi_to_float(int32_t v) { return (float)v * kPhiUlp; }

__device__ __forceinline__ int32_t phi_clamp(int32_t v) { return min(max(v, kPhiLo), kPhiHi); }

// Round to the nearest representable value, clamped to [kPhiMin, kPhiMax].
__device__ __forceinline__ int32_t phi_from_float(float v) {
    float s = fminf(fmaxf(v, kPhiMin), kPhiMax) * kPhiInvUlp;
    return __float2int_rn(s);
}

// ---- lattice ---------------------------------------------------------------

// D3Q27 weight of velocity (cx, cy, cz): 8/27, 2/27, 1/54, 1/216 by |c|^2.
__host__ __device__ constexpr float w27(int cx, int cy, int cz) {
    return (cx * cx + cy * cy + cz * cz) == 0   ? 8.0f / 27.0f
           : (cx * cx + cy * cy + cz * cz) == 1 ? 2.0f / 27.0f
           : (cx * cx + cy * cy + cz * cz) == 2 ? 1.0f / 54.0f
                                                : 1.0f / 216.0f;
}

// Neighbour coordinate v = c + d with |d| <= 1 (or a clamped halo further out):
// wrapped on a periodic axis, clamped to [0, n-1] otherwise.
__device__ __forceinline__ int nb_coord(int v, int n, int periodic) {
    if (periodic) return v < 0 ? v + n : (v >= n ? v - n : v);
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

__device__ __forceinline__ bool is_boundary_node(const Geo &g, int x, int y, int z) {
    return (!g.per[0] && (x == 0 || x == g.nx - 1)) || (!g.per[1] && (y == 0 || y == g.ny - 1)) ||
           (!g.per[2] && (z == 0 || z == g.nz - 1));
}

__device__ __forceinline__ long long node_id(const Geo &g, int x, int y, int z) {
    return (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);
}

// ---- counter-based noise: SplitMix64 finaliser (Steele, Lea, Flood 2014) ----

__host__ __device__ inline unsigned long long splitmix_finalise(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// xi in [-1, 1) from 24 random bits; counter = stream*2^62 + step*2^32 + node*4 + comp.
__device__ __forceinline__ float noise_xi(unsigned long long key, unsigned long long stream,
                                          unsigned long long step, unsigned long long node,
                                          unsigned long long comp) {
    unsigned long long ctr = (stream << 62) + (step << 32) + (node << 2) + comp;
    unsigned long long h = splitmix_finalise(key ^ ctr);
    return (float)(unsigned int)(h >> 40) * (1.0f / 8388608.0f) - 1.0f;
}

// ---- boundary-layer rules (Eqs. 9, 10) ------------------------------------

// Face a boundary node belongs to (0..5 = -x,+x,-y,+y,-z,+z): the face of the
// highest non-periodic axis on which it lies (z, then y, then x); -1 if interior.
__device__ __forceinline__ int boundary_face(const Geo &g, int x, int y, int z) {
    if (!g.per[2] && (z == 0 || z == g.nz - 1)) return z == 0 ? 4 : 5;
    if (!g.per[1] && (y == 0 || y == g.ny - 1)) return y == 0 ? 2 : 3;
    if (!g.per[0] && (x == 0 || x == g.nx - 1)) return x == 0 ? 0 : 1;
    return -1;
}

// Raw moments m[10] (rho', ubar, Q) and phase of boundary node (x, y) on `face`
// at step `step`, given those of its nearest interior node on input: the rule
// imposes density and/or velocity and keeps the copied non-equilibrium part.
__device__ __forceinline__ void apply_boundary_rule(const Phys &ph, const Geo &g, int face, int x, int y,
                                                    unsigned long long step, float m[10], int32_t &phi) {
    const int axis = face >> 1;
    // constant indices keep the rule table in scalar registers
    const int rule = face == 0 ? ph.bc[0] : face == 1 ? ph.bc[1] : face == 2 ? ph.bc[2]
                   : face == 3 ? ph.bc[3] : face == 4 ? ph.bc[4] : ph.bc[5];
    switch (rule) {
    case 1:  // free slip: no normal velocity, no normal-tangential stress
        m[1 + axis] = 0.f;
        if (axis == 0) { m[7] = 0.f; m[8] = 0.f; }
        if (axis == 1) { m[7] = 0.f; m[9] = 0.f; }
        if (axis == 2) { m[8] = 0.f; m[9] = 0.f; }
        break;
    case 4:  // no slip
        m[1] = m[2] = m[3] = 0.f;
        break;
    case 3:  // outflow: unit density
        m[0] = 0.f;
        break;
    case 2: {  // inlet disc on -z: u = U s(r)(1 + a xi) e_z, phi = s(r)
        const float dx = x - 0.5f * (g.nx - 1), dy = y - 0.5f * (g.ny - 1);
        const float r = sqrtf(dx * dx + dy * dy);
        const float s = 0.5f * (1.0f - tanhf(2.0f * (r - 0.5f * ph.inlet_d) / ph.width));
        const float xi = noise_xi(ph.noise_key, 1ull, step, (unsigned long long)(x + (long long)g.nx * y), 2ull);
        m[1] = 0.f;
        m[2] = 0.f;
        m[3] = ph.inlet_u * s * (1.0f + ph.inlet_noise * xi);
        phi = phi_from_float(s);
        break;
    }
    default:
        break;
    }
}

}  // namespace tslb
