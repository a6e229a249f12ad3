// Fused thread-safe LB step for gfx950: one kernel reads the raw moments and
// phase field of step t once from HBM and writes those of step t+1 once.
//
// Work decomposition.  A workgroup owns a 32 x 16 tile of (x, y) destination
// columns and marches through a chunk of z planes.  Its 640 threads are
//   t <  512 : destination column (t % 32, t / 32), also the source of that column,
//   t <  612 : one of the 100 columns of the one-node halo ring (sources only),
//   t >= 612 : idle in the source stages.
// For every z plane the workgroup
//   S1  stages the fixed-point phase field of plane p (3-node halo) in LDS,
//   S2  computes G = grad(phi) and n = G/(|G| + eps) of plane p-1 (2-node halo),
//   S3  computes kappa = div n and F = -sigma kappa G of plane p-2 (1-node halo),
//   S4  rebuilds at every source of plane p-2 the 27 post-collision populations
//       (as brackets t_i = f_i/w_i - 1) and the 7 phase populations,
//   S5  moves them: x and y through LDS, z through registers (the populations of
//       velocity c_z = -1, 0, +1 belong to destination planes p-3, p-2, p-1),
//   S6  finishes destination plane p-3 and stores it.
// Each destination node is written by exactly one thread and every read is of
// step t, so the update is race-free (the thread-safe property of the method).
//
// Arithmetic (Eqs. 5-8, 15-19 with Guo forcing; Eqs. 20-24):
//   source:  u = ubar + F/(2 rho), P = Q + F F/(4 rho), J = rho u + F/2,
//            a2 = rho u u + (1-omega) P + (u F + F u)/2,
//            a3_aab = rho u_a^2 u_b + (1-omega)(2 u_a P_ab + u_b P_aa),
//            a3_xyz = rho u_x u_y u_z + (1-omega)(u_x P_yz + u_y P_xz + u_z P_xy),
//            t(c) = rho' + 3 c.J + 4.5 H2(c):a2 + 4.5 H3(c):a3, evaluated on the
//            27 velocities as a tensor product of 1-D quadratics in c_x, c_y, c_z;
//   destination: moments sum_i w_i H(c_i) t_i(x - c_i) as a tensor product of
//            1-D three-point transforms written relative to the middle value, so
//            the large isotropic part cancels before rounding.
// Variable density and viscosity (VD): the velocity-based form of the phase-field
// scheme for components of different density.  The stored rho' is then the
// normalised pressure p*, the velocity terms of the rebuild take unit density,
// omega follows nu(phi) per source, and F is replaced by the acceleration
//   a = (-sigma kappa G - p* c_s^2 drho G - (1 - omega/2) drho Q.G) / rho(phi) + g
// (surface tension, pressure and viscous forces over rho(phi) = rho_b + drho phi,
// plus gravity; zero on boundary layers), so that at the destination
// ubar = j and Q = Pi - rho c_s^2 I - j j.
// Precision: the source builds tau = t - rho' (no density part) and publishes its
// rho' once; the destination forms t_i - rho'(own column, same plane) as
// tau_i + (rho'(source) - rho'(own column)), exact differences of neighbours, and
// puts rho'(own column) back into the zeroth moment only.  No sum is rounded at
// the magnitude of rho' except the final density itself.
#include <algorithm>

#include "tslb_internal.h"

namespace tslb {
namespace fused {

// Tile shapes.  A workgroup owns TX x TY destination columns; its sources, the
// geometry and the staged phase field cover the tile plus a halo of 1, 2 and 3
// columns.  Two heights: 16 rows with 640 threads (10 waves) and 20 rows with
// 768 threads (12 waves, three on every SIMD, less halo per column), chosen per
// lattice by the host (fused_plan); the one-component and variable-density
// steps take 16 rows.
template <int ROWS> struct Tile {
    static constexpr int TX = 32, TY = ROWS;
    static constexpr int SX = TX + 2, SY = TY + 2, NSRC = SX * SY;   // sources: 34 x 18 or 34 x 22
    static constexpr int GX = TX + 4, GY = TY + 4, NGEO = GX * GY;   // geometry: 36 x 20 or 36 x 24
    static constexpr int PX = TX + 6, PY = TY + 6, NPHI = PX * PY;   // phase field: 38 x 22 or 38 x 26
    static constexpr int NDST = TX * TY;                              // 512 or 640
    static constexpr int NT = ROWS == 16 ? 640 : 768;                 // threads per workgroup
    static_assert(ROWS == 16 || ROWS == 20, "tile heights: 16 or 20 rows");
    static_assert(NSRC <= NT && NDST <= NSRC, "tile does not fit the workgroup");
    static_assert(NPHI <= 2 * NT && NGEO <= 2 * NT, "staging loops assume two items per thread");
};
constexpr int NXCH = 35;   // exchange slots per source (two components)
constexpr int NXCH1 = 28;  // exchange slots per source (one component)

// LDS of a workgroup: PH = two components (with the phase field), else one.
// The gradient ring holds G itself for the variable-density step (its forces
// take G directly), else only |G| + eps: the force is rebuilt as n (|G| + eps)
// from the stored normal, which keeps the 20-row tile within 160 KB of LDS.
template <bool PH, bool VD, int ROWS> struct Smem {
    using T = Tile<ROWS>;
    int32_t phi[4][T::NPHI];           // fixed-point phase field, ring of 4 planes
    float n[3][3][T::NGEO];            // unit normal, ring of 3 planes
    float G[3][VD ? 3 : 1][T::NSRC];   // gradient (VD) or |G| + eps on the source region, ring of 3 planes
    float xch[NXCH][T::NSRC];          // populations crossing columns
};
template <bool VD, int ROWS> struct Smem<false, VD, ROWS> {
    float xch[NXCH1][Tile<ROWS>::NSRC];  // populations crossing columns
};
static_assert(sizeof(Smem<true, false, 20>) <= 160 * 1024 && sizeof(Smem<true, true, 16>) <= 160 * 1024,
              "LDS of one workgroup");

// 1-D three-point transform of (a_-, a_0, a_+) with weights (1/6, 2/3, 1/6):
// m0 = sum w a, m1 = sum w c a, m2 = sum w (c^2 - 1/3) a, written relative to a_0.
struct Tr3 {
    float m0, m1, m2;
};
__device__ __forceinline__ Tr3 tr3(float am, float a0, float ap) {
    const float dm = am - a0, dp = ap - a0;
    const float s = dm + dp;
    Tr3 r;
    r.m0 = fmaf(s, 1.0f / 6.0f, a0);
    r.m1 = (dp - dm) * (1.0f / 6.0f);
    r.m2 = s * (1.0f / 9.0f);
    return r;
}
__device__ __forceinline__ float tr3_m0(float am, float a0, float ap) {
    return fmaf((am - a0) + (ap - a0), 1.0f / 6.0f, a0);
}

// 1/x for a normal x (a density near 1, or |G| + eps): the hardware reciprocal
// refined by one Newton-Raphson step, e = 1 - x r, r' = r + r e, within an ulp.
__device__ __forceinline__ float recip(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Weighted three-point sum with the one-dimensional D3Q27 weights:
// (1/6) m + (2/3) z + (1/6) p.
__device__ __forceinline__ float w1sum(float m, float z, float p) { return fmaf(z, 2.0f / 3.0f, (m + p) * (1.0f / 6.0f)); }

// Quadratic A + B c + C (c^2 - 1/3) at c = -1, 0, +1.
__device__ __forceinline__ void quad3(float A, float B, float C, float &vm, float &v0, float &vp) {
    const float m = fmaf(C, 2.0f / 3.0f, A);
    v0 = fmaf(C, -1.0f / 3.0f, A);
    vm = m - B;
    vp = m + B;
}

// Slot of direction (cx, cy) != (0, 0) in the exchange buffer of one z group.
__device__ __forceinline__ constexpr int xy_slot(int cx, int cy) {
    return ((cx + 1) + 3 * (cy + 1)) < 4 ? ((cx + 1) + 3 * (cy + 1)) : ((cx + 1) + 3 * (cy + 1)) - 1;
}

__device__ __forceinline__ int wrap_or_clamp(int v, int n, int periodic) {
    if (periodic) {
        v %= n;
        return v < 0 ? v + n : v;
    }
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

// The six 2-D moments X_pq = sum_{cx,cy} w(cx) w(cy) h_p(cx) h_q(cy) t(cx, cy) of
// one z group, p, q in {00, 10, 01, 20, 02, 11} (order of the output array).
__device__ __forceinline__ void xy_moments(const float t[9], float X[6]) {
    // y stage, per c_x: t[(cx+1) + 3(cy+1)]
    Tr3 y0 = tr3(t[0], t[3], t[6]);   // c_x = -1
    Tr3 y1 = tr3(t[1], t[4], t[7]);   // c_x = 0
    Tr3 y2 = tr3(t[2], t[5], t[8]);   // c_x = +1
    Tr3 a = tr3(y0.m0, y1.m0, y2.m0);
    X[0] = a.m0;                       // 00
    X[1] = a.m1;                       // 10
    X[3] = a.m2;                       // 20
    Tr3 b = tr3(y0.m1, y1.m1, y2.m1);
    X[2] = b.m0;                       // 01
    X[5] = b.m1;                       // 11
    X[4] = tr3_m0(y0.m2, y1.m2, y2.m2);  // 02
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Work item w is assigned so that every XCD receives a contiguous range of w:
// the tiles of one z chunk then run side by side on one XCD and their
// overlapping halos are served by that XCD's L2 instead of HBM.
__device__ __forceinline__ int xcd_work_item(int b, int nb) {
    const int q8 = nb >> 3, rem8 = nb & 7;
    const int xcd = b & 7, slot = b >> 3;
    return (xcd < rem8 ? xcd * (q8 + 1) : rem8 * (q8 + 1) + (xcd - rem8) * q8) + slot;
}

// One work item (a tile and a z chunk) of one lattice.  G: access the state
// through global-address-space pointers (for state pointers read from memory).
// MULTI marks the multi-lattice kernel's instantiation: it keeps that kernel's
// copy of the step apart from the single-lattice kernel's, whose code is
// otherwise changed (and slowed) by the second user of the same instantiation.
template <int ST, bool PH, bool G, bool MULTI, bool VD, int ROWS>
__device__ __forceinline__ void step_fused(Smem<PH, VD, ROWS> &sm, const Geo &g, const Phys &ph, const Scales &sc,
                                           const StateView &in, const StateView &out, int lz, int tiles_x,
                                           int tiles_y, unsigned long long step_next, int w) {
    using T = Tile<ROWS>;
    constexpr int TX = T::TX, TY = T::TY, SX = T::SX, SY = T::SY, NSRC = T::NSRC, GX = T::GX, GY = T::GY,
                  NGEO = T::NGEO, PX = T::PX, NPHI = T::NPHI, NDST = T::NDST, NT = T::NT;
    // exchange slots: 0-23 the x/y-crossing populations of the three z groups,
    // then (two components) 24-27 phase +-x, +-y; rho'; phase rest, +z, -z;
    // and the three populations of velocity (0, 0, c_z)
    constexpr int kRho = PH ? 28 : 24, kCen = PH ? 32 : 25;
    const int tile = w % (tiles_x * tiles_y);
    const int chunk = w / (tiles_x * tiles_y);
    // The tile owns columns [xo, xo + TX) x [yo, yo + TY); its origin (x0, y0) is
    // pulled inward at the high edge so that all TX x TY columns lie in the
    // lattice (a wall column's nearest interior node is then always in the tile).
    const int xo = (tile % tiles_x) * TX, yo = (tile / tiles_x) * TY;
    const int x0 = g.nx > TX ? min(xo, g.nx - TX) : 0;
    const int y0 = g.ny > TY ? min(yo, g.ny - TY) : 0;
    const int z0 = chunk * lz;
    const int z1 = min(z0 + lz, g.nz);  // destination planes [z0, z1)
    const int t = threadIdx.x;
    const long long plane = (long long)g.nx * g.ny;

    // ---- this thread's source column (local sx, sy in the 34 x 18 region) ----
    int sx = 0, sy = 0;
    const bool is_dst = t < NDST;
    const bool is_src = t < NSRC;
    if (is_dst) {
        sx = t % TX + 1;
        sy = t / TX + 1;
    } else if (is_src) {
        const int r = t - NDST;
        if (r < SX) { sx = r; sy = 0; }
        else if (r < 2 * SX) { sx = r - SX; sy = SY - 1; }
        else if (r < 2 * SX + TY) { sx = 0; sy = r - 2 * SX + 1; }
        else { sx = SX - 1; sy = r - 2 * SX - TY + 1; }
    }
    const int sidx = sy * SX + sx;
    const int gxs = x0 + sx - 1, gys = y0 + sy - 1;          // unwrapped global source column
    const int cxs = wrap_or_clamp(gxs, g.nx, g.per[0]);
    const int cys = wrap_or_clamp(gys, g.ny, g.per[1]);
    const long long col_src = (long long)cxs + (long long)g.nx * cys;
    const bool src_bnd_xy = (!g.per[0] && (gxs <= 0 || gxs >= g.nx - 1)) ||
                            (!g.per[1] && (gys <= 0 || gys >= g.ny - 1));
    // Destination columns: every owned column, walls included.  A wall column
    // finishes the moments of its nearest interior node x_F (one node in from the
    // wall) and stores them through its face rule (Eqs. 9, 10), so each
    // destination thread reads the exchange buffer around fidx = x_F.
    const bool owned = is_dst && gxs >= xo && gxs < xo + TX && gxs < g.nx && gys >= yo && gys < yo + TY &&
                       gys < g.ny;
    const int dxf = (!g.per[0] && gxs == 0) ? 1 : ((!g.per[0] && gxs == g.nx - 1) ? -1 : 0);
    const int dyf = (!g.per[1] && gys == 0) ? 1 : ((!g.per[1] && gys == g.ny - 1) ? -1 : 0);
    const int fidx = (sy + dyf) * SX + (sx + dxf);

    // ---- staging columns of the phase field (<= 2 per thread) ----
    long long col_phi[2];
    int phi_item[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int i = t + k * NT;
        phi_item[k] = i < NPHI ? i : -1;
        const int px = i % PX, py = i / PX;
        const int gx = wrap_or_clamp(x0 - 3 + px, g.nx, g.per[0]);
        const int gy = wrap_or_clamp(y0 - 3 + py, g.ny, g.per[1]);
        col_phi[k] = (long long)gx + (long long)g.nx * gy;
    }
    // Geometry items (S2 of plane p): centre (gx, gy) in the GX x GY region.
    // Waves are placed on the four SIMDs round-robin (wave w on SIMD w % 4), and
    // each phase ends at a barrier.  The normal and gradient of plane p are first
    // read in the next iteration, so an item may run in either phase.
    // 16 rows: SIMDs 0 and 1 run three source waves (0, 4, 8 and 1, 5, 9), SIMDs
    // 2 and 3 two, so in phase A waves 0-7 take items 0-511 and waves 2 and 3 the
    // next 80; the last 128 run in phase B on waves 8 and 9, which have no
    // destination.
    // 20 rows: phase A holds three source waves on every SIMD, phase B three
    // destination waves on SIMDs 0 and 1 but two on SIMDs 2 and 3, so threads
    // 0-479 (two waves per SIMD) take one item in phase A, and in phase B waves 10
    // and 11 (no destination) and waves 2, 3, 6 and 7 (before their destination)
    // one item each.
    // The variable-density step (16 rows; its items store all of G) keeps every
    // item in phase A, where that measured faster: waves 0-7 take items 0-511 and
    // waves 2, 3, 6 and 7 the other 208.
    static_assert(GX >= 32 && GX < 64, "geometry rows are split into 32 + (GX - 32) columns");
    constexpr int NGEO_B = VD ? 0 : (TY == 16 ? NT - NDST : 384);  // phase-B items
    constexpr int NGEO_A = NGEO - NGEO_B;                          // phase-A items
    static_assert(VD || NT - NDST == 128, "two waves without a destination");
    int geo_a[2] = {-1, -1};
    {
        const int wv = t >> 6, lane = t & 63;
        if constexpr (TY == 16 && VD) {
            static_assert(NDST == 512 && NGEO - NDST <= 256, "16-row geometry map: 512 + 4 waves of items");
            const int rank = wv == 2 ? 0 : wv == 3 ? 1 : wv == 6 ? 2 : wv == 7 ? 3 : -1;
            const int i = NDST + rank * 64 + lane;
            geo_a[0] = t < NDST ? t : -1;
            if (rank >= 0 && i < NGEO) geo_a[1] = i;
        } else if constexpr (TY == 16) {
            static_assert(NDST == 512 && NGEO_A == NDST + 80, "16-row geometry map: 512 + 80 items in phase A");
            geo_a[0] = t < NDST ? t : -1;
            if ((wv == 2 || wv == 3) && lane < 40) geo_a[1] = NDST + (wv - 2) * 40 + lane;
        } else {
            static_assert(!VD && NGEO_A == 480, "20-row geometry map: waves 0-7 in phase A");
            geo_a[0] = t < NGEO_A ? t : -1;
        }
    }
    int geo_b = (NGEO_B > 0 && t >= NDST) ? NGEO_A + (t - NDST) : -1;  // waves without a destination
    if constexpr (TY == 20) {  // and waves 2, 3, 6, 7, before their destination work
        const int wv = t >> 6, lane = t & 63;
        const int r4 = wv == 2 ? 0 : wv == 3 ? 1 : wv == 6 ? 2 : wv == 7 ? 3 : -1;
        if (r4 >= 0) geo_b = NGEO_A + 128 + r4 * 64 + lane;
    }

    const float omega1 = 1.0f - ph.omega;
    const float sigma = ph.sigma, gamma = ph.gamma, eps = ph.eps;

    // carried destination state (see the S5 comment)
    float XA[6], XB[6], XC[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) XA[k] = XB[k] = XC[k] = 0.f;
    int32_t PA = 0, PC = 0;  // phase partial sums of planes r - 1 and r (column x_F)
    float cA = 0.f, cB = 0.f, cC = 0.f, eA = 0.f, eB = 0.f, eC = 0.f;  // curvature partial sums (S3a)

    // prefetched raw moments of the next source plane (own column)
    // (stored words: a 16-bit moment is converted only when the next iteration
    // takes it over, so its load is not waited for in the iteration that issues it)
    uint32_t mom[10] = {};  // defined before the first prefetch (decoded but unused until then)
    int32_t phi_next[2] = {0, 0};

    // z is uniform and at most a few planes outside [0, nz): wrap by whole periods
    // (no integer division in the loop)
    auto plane_of = [&](int z) {
        if (g.per[2]) {
            while (z < 0) z += g.nz;
            while (z >= g.nz) z -= g.nz;
            return z;
        }
        return z < 0 ? 0 : (z >= g.nz ? g.nz - 1 : z);
    };
    auto load_moments = [&](int z, uint32_t m[10]) {
        const long long id = col_src + plane * plane_of(z);
#pragma unroll
        for (int p = 0; p < 10; ++p) m[p] = load_moment_bits<ST, G>(in.mom, g.ld, p, id);
    };
    auto load_phi = [&](int z, int32_t v[2]) {
        const long long zoff = plane * plane_of(z);
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (phi_item[k] >= 0) v[k] = mem<G>(in.phi)[col_phi[k] + zoff];
    };

    // ---- S2: G and n of plane p from phi planes p-1, p, p+1 (slots it-1, it, it+1),
    // one geometry item i ----
    auto geometry_item = [&](int i, int it) {
        if constexpr (PH) {
            const int32_t *pm = sm.phi[(it + 3) & 3], *p0 = sm.phi[it & 3], *pp = sm.phi[(it + 1) & 3];
            // items 0 .. 32 GY - 1 cover columns 0-31 of each row, one row per
            // half-wave (contiguous LDS addresses, no bank conflicts); the
            // rest cover columns 32 .. GX - 1
            const int gxl = i < 32 * GY ? (i & 31) : 32 + (i - 32 * GY) % (GX - 32);
            const int gyl = i < 32 * GY ? (i >> 5) : (i - 32 * GY) / (GX - 32);
            const int gi = gyl * GX + gxl;  // position in the geometry region
            const int c = (gyl + 1) * PX + (gxl + 1);  // centre in the phi region
            float G0 = 0.f, G1 = 0.f, G2 = 0.f;
#pragma unroll
            for (int cz = -1; cz <= 1; ++cz)
#pragma unroll
                for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
                    for (int cx = -1; cx <= 1; ++cx) {
                        const bool lead = cx > 0 || (cx == 0 && (cy > 0 || (cy == 0 && cz > 0)));
                        if (!lead) continue;
                        const int32_t *pa = cz > 0 ? pp : (cz < 0 ? pm : p0);
                        const int32_t *pb = cz > 0 ? pm : (cz < 0 ? pp : p0);
                        const int32_t a = pa[c + cy * PX + cx];
                        const int32_t bb = pb[c - cy * PX - cx];
                        const float d = (float)(a - bb);
                        const float w = 3.0f * w27(cx, cy, cz) * kPhiUlp;
                        if (cx) G0 = fmaf(w * cx, d, G0);
                        if (cy) G1 = fmaf(w * cy, d, G1);
                        if (cz) G2 = fmaf(w * cz, d, G2);
                    }
            // hardware square root (1 ulp) and a refined reciprocal: |G| + eps >= eps
            const float den = __builtin_amdgcn_sqrtf(fmaf(G0, G0, fmaf(G1, G1, G2 * G2))) + eps;
            const float inv = recip(den);
            float *n = &sm.n[it % 3][0][0];
            n[gi] = G0 * inv;
            n[NGEO + gi] = G1 * inv;
            n[2 * NGEO + gi] = G2 * inv;
            const int ssx = gxl - 1, ssy = gyl - 1;
            if (ssx >= 0 && ssx < SX && ssy >= 0 && ssy < SY) {
                float *Gs = &sm.G[it % 3][0][0];
                const int si = ssy * SX + ssx;
                if constexpr (VD) {
                    Gs[si] = G0;
                    Gs[NSRC + si] = G1;
                    Gs[2 * NSRC + si] = G2;
                } else {
                    Gs[si] = den;
                }
            }
        }
    };

    const int nit = (z1 - z0) + 6;
    // prologue: phase planes z0 - 3 and z0 - 2 staged (slots 0, 1)
    if constexpr (PH) {
        int32_t v[2] = {0, 0};
        load_phi(z0 - 3, v);
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (phi_item[k] >= 0) sm.phi[0][phi_item[k]] = v[k];
        load_phi(z0 - 2, v);
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (phi_item[k] >= 0) sm.phi[1][phi_item[k]] = v[k];
    }
    __syncthreads();

    // Iteration it works on three planes: p = z0 - 3 + it (geometry), q = p - 1
    // (normal of the curvature sums) and r = p - 2 (sources), and finishes
    // destination plane r - 1.  Rings: phi plane p at slot it mod 4, n and G of
    // plane p at slot it mod 3.  Phase A (sources and geometry) and phase B
    // (destinations and phase staging) are separated by barriers.
    for (int it = 0; it < nit; ++it) {
        const int p = z0 - 3 + it;
        const int r = p - 2;

        // moments of source plane r + 1 for the next iteration
        float mom_cur[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) mom_cur[k] = decode_moment<ST>(mom[k], k, sc);
        if (is_src && it >= 3) load_moments(r + 1, mom);
        // phase plane p + 2, staged at the start of phase B.  Issued here, next to
        // the moment prefetch, so that both have all of phase A to arrive (both are
        // waited for at the start of phase B).
        if constexpr (PH) {
            if (it + 3 <= nit) load_phi(p + 2, phi_next);
        }

        // ================= phase A =================
        // ---- S3a: per-column partial sums of the curvature stencil (plane q) ----
        // With w_i = w1(c_x) w1(c_y) w1(c_z), w1(0) = 2/3, w1(+-1) = 1/6, the stencil
        // kappa = 3 sum_i w_i c_i . n(x + c_i) factorises into sums over one plane:
        //   kappa(r) = (1/2) [ sum_cz w1(cz) C(r + cz) + E(r + 1) - E(r - 1) ],
        //   C = sum_cy w1(cy) (n_x(x+1, y+cy) - n_x(x-1, y+cy))
        //     + sum_cx w1(cx) (n_y(x+cx, y+1) - n_y(x+cx, y-1)),
        //   E = sum_{cx,cy} w1(cx) w1(cy) n_z(x+cx, y+cy),
        // so each source keeps C and E of three planes in registers.
        if constexpr (PH) {
            if (it >= 2 && is_src) {
                const float *nq = &sm.n[(it + 2) % 3][0][0];  // plane q, written one iteration ago
                const float *nyq = nq + NGEO, *nzq = nq + 2 * NGEO;
                const int c = (sy + 1) * GX + (sx + 1);  // centre in the geometry region
                const float Cx = w1sum(nq[c - GX + 1] - nq[c - GX - 1], nq[c + 1] - nq[c - 1], nq[c + GX + 1] - nq[c + GX - 1]);
                const float Cy = w1sum(nyq[c + GX - 1] - nyq[c - GX - 1], nyq[c + GX] - nyq[c - GX],
                                       nyq[c + GX + 1] - nyq[c - GX + 1]);
                const float E = w1sum(w1sum(nzq[c - GX - 1], nzq[c - GX], nzq[c - GX + 1]),
                                      w1sum(nzq[c - 1], nzq[c], nzq[c + 1]),
                                      w1sum(nzq[c + GX - 1], nzq[c + GX], nzq[c + GX + 1]));
                cA = cB;
                cB = cC;
                cC = Cx + Cy;
                eA = eB;
                eB = eC;
                eC = E;
            }
        }

        if (it >= 4) {
            // ---- S3: kappa and F at the source (plane r = q - 1) ----
            float F0 = 0.f, F1 = 0.f, F2 = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f;
            float Gx = 0.f, Gy = 0.f, Gz = 0.f;  // grad(phi) at the source (VD)
            bool sbnd = false;                   // the source is a boundary-layer node (VD)
            int32_t phis = 0;
            if constexpr (PH) {
                if (is_src) {
                    const float kap = 0.5f * (w1sum(cA, cB, cC) + (eC - eA));
                    const int zr = r;
                    const bool bnd = src_bnd_xy || (!g.per[2] && (zr <= 0 || zr >= g.nz - 1));
                    const float a = bnd ? 0.f : -sigma * kap;
                    const float *nr = &sm.n[(it + 1) % 3][0][0];  // plane r
                    const int c = (sy + 1) * GX + (sx + 1);
                    n0 = nr[c];
                    n1 = nr[NGEO + c];
                    n2 = nr[2 * NGEO + c];
                    const float *Gs = &sm.G[(it + 1) % 3][0][0];  // plane r
                    if constexpr (VD) {
                        Gx = Gs[sidx];
                        Gy = Gs[NSRC + sidx];
                        Gz = Gs[2 * NSRC + sidx];
                        sbnd = bnd;
                        F0 = a * Gx;
                        F1 = a * Gy;
                        F2 = a * Gz;
                    } else {
                        const float ag = a * Gs[sidx];  // G = n (|G| + eps)
                        F0 = ag * n0;
                        F1 = ag * n1;
                        F2 = ag * n2;
                    }
                    phis = sm.phi[(it - 2) & 3][(sy + 2) * PX + (sx + 2)];
                }
            }

            // ---- S4: post-collision populations of the source ----
            float tm[9], t0[9], tp[9];  // groups c_z = -1, 0, +1, index (cx+1) + 3(cy+1)
            int32_t base = 0, ax = 0, ay = 0, az = 0;
            if (is_src) {
                const float rp = mom_cur[0];
                float om1 = omega1;
                if constexpr (VD) {
                    // rho(phi), omega(phi) and the acceleration that replaces F
                    const float pc = fminf(fmaxf(phi_to_float(phis), 0.0f), 1.0f);
                    const float om = recip(fmaf(3.0f, fmaf(ph.dnu, pc, ph.nu_b), 0.5f));
                    om1 = 1.0f - om;
                    if (sbnd) {
                        F0 = F1 = F2 = 0.f;
                    } else {
                        const float ir = recip(fmaf(ph.drho, pc, ph.rho_b));
                        const float cp = (-1.0f / 3.0f) * ph.drho * rp;     // pressure force / G
                        const float cm = (0.5f * om - 1.0f) * ph.drho;      // viscous force / (Q.G)
                        const float QG0 = fmaf(mom_cur[4], Gx, fmaf(mom_cur[7], Gy, mom_cur[8] * Gz));
                        const float QG1 = fmaf(mom_cur[7], Gx, fmaf(mom_cur[5], Gy, mom_cur[9] * Gz));
                        const float QG2 = fmaf(mom_cur[8], Gx, fmaf(mom_cur[9], Gy, mom_cur[6] * Gz));
                        F0 = fmaf(fmaf(cm, QG0, fmaf(cp, Gx, F0)), ir, ph.grav[0]);
                        F1 = fmaf(fmaf(cm, QG1, fmaf(cp, Gy, F1)), ir, ph.grav[1]);
                        F2 = fmaf(fmaf(cm, QG2, fmaf(cp, Gz, F2)), ir, ph.grav[2]);
                    }
                }
                const float rho = VD ? 1.0f : 1.0f + rp;  // density of the velocity terms
                const float inv = VD ? 1.0f : recip(rho);
                const float hF = 0.5f * inv, qF = 0.25f * inv;
                const float u0 = fmaf(hF, F0, mom_cur[1]), u1 = fmaf(hF, F1, mom_cur[2]), u2 = fmaf(hF, F2, mom_cur[3]);
                const float Pxx = fmaf(qF * F0, F0, mom_cur[4]), Pyy = fmaf(qF * F1, F1, mom_cur[5]);
                const float Pzz = fmaf(qF * F2, F2, mom_cur[6]), Pxy = fmaf(qF * F0, F1, mom_cur[7]);
                const float Pxz = fmaf(qF * F0, F2, mom_cur[8]), Pyz = fmaf(qF * F1, F2, mom_cur[9]);
                // Hermite coefficients, pre-scaled: t(c) = K0 + sum K1 c + ... (see header)
                const float Jx = fmaf(rho, u0, 0.5f * F0), Jy = fmaf(rho, u1, 0.5f * F1), Jz = fmaf(rho, u2, 0.5f * F2);
                const float mxx = om1 * Pxx, myy = om1 * Pyy, mzz = om1 * Pzz;
                const float mxy = om1 * Pxy, mxz = om1 * Pxz, myz = om1 * Pyz;
                const float ru0 = rho * u0, ru1 = rho * u1, ru2 = rho * u2;
                const float a2xx = fmaf(ru0, u0, mxx) + u0 * F0;
                const float a2yy = fmaf(ru1, u1, myy) + u1 * F1;
                const float a2zz = fmaf(ru2, u2, mzz) + u2 * F2;
                const float a2xy = fmaf(ru0, u1, mxy) + 0.5f * (u0 * F1 + F0 * u1);
                const float a2xz = fmaf(ru0, u2, mxz) + 0.5f * (u0 * F2 + F0 * u2);
                const float a2yz = fmaf(ru1, u2, myz) + 0.5f * (u1 * F2 + F1 * u2);
                // a3_aab = u_a (rho u_a u_b + 2 m_ab) + u_b m_aa
                const float a3xxy = fmaf(u0, fmaf(ru0, u1, 2.0f * mxy), u1 * mxx);
                const float a3xxz = fmaf(u0, fmaf(ru0, u2, 2.0f * mxz), u2 * mxx);
                const float a3yyx = fmaf(u1, fmaf(ru1, u0, 2.0f * mxy), u0 * myy);
                const float a3yyz = fmaf(u1, fmaf(ru1, u2, 2.0f * myz), u2 * myy);
                const float a3zzx = fmaf(u2, fmaf(ru2, u0, 2.0f * mxz), u0 * mzz);
                const float a3zzy = fmaf(u2, fmaf(ru2, u1, 2.0f * myz), u1 * mzz);
                const float a3xyz = fmaf(ru0 * u1, u2, fmaf(u0, myz, fmaf(u1, mxz, u2 * mxy)));
                // The scale factors of the coefficients (3 J, 4.5 a2_aa, 9 a2_ab, 13.5 a3_aab,
                // 27 a3_xyz) are folded into the constants of the multiply-adds that take
                // a coefficient as a slope or curvature term; only the five that enter as
                // an addend are scaled explicitly.
                const float K1y = 3.0f * Jy, K1z = 3.0f * Jz;
                const float K2yy = 4.5f * a2yy, K2zz = 4.5f * a2zz, K2yz = 9.0f * a2yz;
                // t = T0 + cz T1 + h(cz) T2; T0 = U0 + cy U1 + h(cy) U2 (per cx), etc.
                float U0[3], U1[3], V0[3], W0[3];
                {   // U0 = quad3(0, 3 Jx, 4.5 a2xx): tau = t - rho'
                    const float m = 3.0f * a2xx;
                    U0[1] = -1.5f * a2xx;
                    U0[0] = fmaf(-3.0f, Jx, m);
                    U0[2] = fmaf(3.0f, Jx, m);
                }
                {   // U1 = quad3(3 Jy, 9 a2xy, 13.5 a3xxy)
                    const float m = fmaf(9.0f, a3xxy, K1y);
                    U1[1] = fmaf(-4.5f, a3xxy, K1y);
                    U1[0] = fmaf(-9.0f, a2xy, m);
                    U1[2] = fmaf(9.0f, a2xy, m);
                }
                {   // V0 = quad3(3 Jz, 9 a2xz, 13.5 a3xxz)
                    const float m = fmaf(9.0f, a3xxz, K1z);
                    V0[1] = fmaf(-4.5f, a3xxz, K1z);
                    V0[0] = fmaf(-9.0f, a2xz, m);
                    V0[2] = fmaf(9.0f, a2xz, m);
                }
                W0[0] = fmaf(-13.5f, a3zzx, K2zz);
                W0[1] = K2zz;
                W0[2] = fmaf(13.5f, a3zzx, K2zz);
#pragma unroll
                for (int ix = 0; ix < 3; ++ix) {
                    const float cx = (float)(ix - 1);
                    const float U2 = ix == 1 ? K2yy : fmaf(13.5f * cx, a3yyx, K2yy);  // linear in cx
                    const float V1 = ix == 1 ? K2yz : fmaf(27.0f * cx, a3xyz, K2yz);
                    float T0[3], T1[3], T2[3];
                    quad3(U0[ix], U1[ix], U2, T0[0], T0[1], T0[2]);
                    {   // T1 = quad3(V0, V1, 13.5 a3yyz)
                        const float m = fmaf(9.0f, a3yyz, V0[ix]);
                        T1[1] = fmaf(-4.5f, a3yyz, V0[ix]);
                        T1[0] = m - V1;
                        T1[2] = m + V1;
                    }
                    T2[0] = fmaf(-13.5f, a3zzy, W0[ix]);
                    T2[1] = W0[ix];
                    T2[2] = fmaf(13.5f, a3zzy, W0[ix]);
#pragma unroll
                    for (int iy = 0; iy < 3; ++iy) {
                        const int k = ix + 3 * iy;
                        const float mid = fmaf(T2[iy], 2.0f / 3.0f, T0[iy]);
                        t0[k] = fmaf(T2[iy], -1.0f / 3.0f, T0[iy]);
                        tm[k] = mid - T1[iy];
                        tp[k] = mid + T1[iy];
                    }
                }
                if constexpr (PH) {
                    // phase: base to every axis neighbour, +-a_e along +-e, phi - 6 base stays
                    const float phif = phi_to_float(phis);
                    const float omphi = (float)(kPhiOne - phis) * kPhiUlp;
                    const float gph = gamma * omphi;
                    const float h8 = 0.125f * phif * kPhiInvUlp;
                    base = (phis + 4) >> 3;
                    ax = __float2int_rn(h8 * fmaf(4.0f, u0, gph * n0));
                    ay = __float2int_rn(h8 * fmaf(4.0f, u1, gph * n1));
                    az = __float2int_rn(h8 * fmaf(4.0f, u2, gph * n2));
                }

                // ---- S5a: publish what crosses columns ----
#pragma unroll
                for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
                    for (int cx = -1; cx <= 1; ++cx) {
                        if (!cx && !cy) continue;
                        const int k = (cx + 1) + 3 * (cy + 1);
                        const int s = xy_slot(cx, cy);
                        sm.xch[s][sidx] = tm[k];
                        sm.xch[8 + s][sidx] = t0[k];
                        sm.xch[16 + s][sidx] = tp[k];
                    }
                if constexpr (PH) {
                    sm.xch[24][sidx] = __int_as_float(base + ax);        // +x
                    sm.xch[25][sidx] = __int_as_float(base - ax);        // -x
                    sm.xch[26][sidx] = __int_as_float(base + ay);        // +y
                    sm.xch[27][sidx] = __int_as_float(base - ay);        // -y
                    sm.xch[29][sidx] = __int_as_float(phis - 6 * base);  // rest
                    sm.xch[30][sidx] = __int_as_float(base + az);        // +z
                    sm.xch[31][sidx] = __int_as_float(base - az);        // -z
                }
                sm.xch[kRho][sidx] = rp;
                sm.xch[kCen][sidx] = tm[4];
                sm.xch[kCen + 1][sidx] = t0[4];
                sm.xch[kCen + 2][sidx] = tp[4];
            }
        }

        // ---- S2, phase-A items ----
        if constexpr (PH) if (it >= 1 && it + 2 <= nit) {
            for (int k = 0; k < 2; ++k)
                if (geo_a[k] >= 0) geometry_item(geo_a[k], it);
        }
        __syncthreads();

        // ================= phase B =================
        // Wait here, before any store of the iteration, for the loads issued at its
        // top (vmcnt 0; expcnt and lgkmcnt fields at their maxima, i.e. not waited
        // for).  Loads and stores share one in-order counter, and the stores below
        // are conditional, so a wait for the prefetched words placed after them (at
        // the phase staging or at the loop latch, where the prefetched moments are
        // copied) can only be vmcnt(0) and also waits until every store of the
        // iteration has been acknowledged.  Waited for here, on every path, the
        // loads are known complete at the latch and the stores drain during the
        // next iteration.
        __builtin_amdgcn_s_waitcnt(0x0F70);
        // ---- S1: stage phi(p + 2) for the geometry of the next iteration (slot of
        // plane p - 2, whose last reader, the sources of phase A, is done) ----
        if constexpr (PH) {
            if (it + 3 <= nit) {
#pragma unroll
                for (int k = 0; k < 2; ++k)
                    if (phi_item[k] >= 0) sm.phi[(it + 2) & 3][phi_item[k]] = phi_next[k];
            }
        }
        // ---- S2, phase-B items, before any destination work (the slots read are not the
        // one staged above) ----
        if constexpr (PH) if (geo_b >= 0 && it >= 1 && it + 2 <= nit) geometry_item(geo_b, it);
        if (it >= 4) {
            // ---- S5b/S6: gather at the destination and finish plane r - 1 ----
            if (is_dst) {
                float gm[9], g0[9], gp[9];
                const float rp_ref = sm.xch[kRho][fidx];
                gm[4] = sm.xch[kCen][fidx];
                g0[4] = sm.xch[kCen + 1][fidx];
                gp[4] = sm.xch[kCen + 2][fidx];
#pragma unroll
                for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
                    for (int cx = -1; cx <= 1; ++cx) {
                        if (!cx && !cy) continue;
                        const int k = (cx + 1) + 3 * (cy + 1);
                        const int s = xy_slot(cx, cy);
                        const int src = fidx - cy * SX - cx;
                        const float drp = sm.xch[kRho][src] - rp_ref;
                        gm[k] = sm.xch[s][src] + drp;
                        g0[k] = sm.xch[8 + s][src] + drp;
                        gp[k] = sm.xch[16 + s][src] + drp;
                    }
                float Xm[6], X0[6], Xp[6];
                xy_moments(gm, Xm);
                xy_moments(g0, X0);
                xy_moments(gp, Xp);
                Xm[0] += rp_ref;
                X0[0] += rp_ref;
                Xp[0] += rp_ref;
                int32_t pin = 0, prest = 0, pup = 0, pdown = 0;
                if constexpr (PH) {
                    pin = __float_as_int(sm.xch[24][fidx - 1]) + __float_as_int(sm.xch[25][fidx + 1]) +
                          __float_as_int(sm.xch[26][fidx - SX]) + __float_as_int(sm.xch[27][fidx + SX]);
                    prest = __float_as_int(sm.xch[29][fidx]);
                    pup = __float_as_int(sm.xch[30][fidx]);
                    pdown = __float_as_int(sm.xch[31][fidx]);
                }
                // destination plane r - 1: X(-1) from source plane r, X(0) = XB, X(+1) = XA
                const int zd = r - 1;
                if (owned && zd >= z0 && zd < z1 && (g.per[2] || (zd > 0 && zd < g.nz - 1))) {
                    const Tr3 m00 = tr3(Xm[0], XB[0], XA[0]);  // rho', j_z, H_zz
                    const Tr3 m10 = tr3(Xm[1], XB[1], XA[1]);  // j_x, H_xz
                    const Tr3 m01 = tr3(Xm[2], XB[2], XA[2]);  // j_y, H_yz
                    const float Hxx = tr3_m0(Xm[3], XB[3], XA[3]);
                    const float Hyy = tr3_m0(Xm[4], XB[4], XA[4]);
                    const float Hxy = tr3_m0(Xm[5], XB[5], XA[5]);
                    const float drho = m00.m0;
                    const float jx = m10.m0, jy = m01.m0, jz = m00.m1;
                    const float inv = VD ? 1.0f : recip(1.0f + drho);
                    float m[10];
                    m[0] = drho;
                    m[1] = jx * inv;
                    m[2] = jy * inv;
                    m[3] = jz * inv;
                    m[4] = fmaf(-jx * inv, jx, Hxx);
                    m[5] = fmaf(-jy * inv, jy, Hyy);
                    m[6] = fmaf(-jz * inv, jz, m00.m2);
                    m[7] = fmaf(-jx * inv, jy, Hxy);
                    m[8] = fmaf(-jx * inv, jz, m10.m1);
                    m[9] = fmaf(-jy * inv, jz, m01.m1);
                    // streamed phase, held to the clamp range (a stable run never reaches it)
                    const int32_t phin = phi_clamp(PA + pdown);
                    // the z walls of this column take the values of planes 1 and nz-2
                    // (x_F of an edge node is interior in every coordinate, so the
                    // image is made from the moments before any x/y rule)
                    if (!g.per[2] && (zd == 1 || zd == g.nz - 2)) {
                        const int zb = zd == 1 ? 0 : g.nz - 1;
                        float mb[10];
#pragma unroll
                        for (int k = 0; k < 10; ++k) mb[k] = m[k];
                        int32_t pb = phin;
                        apply_boundary_rule(ph, g, zd == 1 ? 4 : 5, gxs, gys, step_next, mb, pb);
                        const long long ib = (long long)gxs + (long long)g.nx * gys + plane * zb;
#pragma unroll
                        for (int k = 0; k < 10; ++k) store_moment<ST, G>(out.mom, g.ld, k, ib, mb[k], sc);
                        if constexpr (PH) store_nt(&mem<G>(out.phi)[ib], pb);
                    }
                    // the node itself: interior, or on an x/y wall (face rule of step t+1)
                    int32_t po = phin;
                    if (dxf | dyf) {
                        const int face = boundary_face(g, gxs, gys, zd);
                        apply_boundary_rule(ph, g, face, gxs, gys, step_next, m, po);
                    }
                    const long long id = (long long)gxs + (long long)g.nx * gys + plane * zd;
#pragma unroll
                    for (int k = 0; k < 10; ++k) store_moment<ST, G>(out.mom, g.ld, k, id, m[k], sc);
                    if constexpr (PH) store_nt(&mem<G>(out.phi)[id], po);
                }
                // carry: plane r gets X(+1) = XC, X(0) = X0; plane r+1 gets X(+1) = Xp
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    XA[k] = XC[k];
                    XB[k] = X0[k];
                    XC[k] = Xp[k];
                }
                PA = PC + prest + pin;
                PC = pup;
            }
        }
        __syncthreads();
    }
}


template <int ST, bool PH, bool VD, int ROWS>
__global__ __launch_bounds__(Tile<ROWS>::NT) void k_step_fused(Geo g, Phys ph, Scales sc, StateView in, StateView out,
                                                               int lz, int tiles_x, int tiles_y,
                                                               unsigned long long step_next) {
    __shared__ Smem<PH, VD, ROWS> sm;
    step_fused<ST, PH, false, false, VD, ROWS>(sm, g, ph, sc, in, out, lz, tiles_x, tiles_y, step_next,
                                               xcd_work_item(blockIdx.x, gridDim.x));
}

// Several lattices in one launch: the work items of domain k are
// [work_begin, work_begin + tiles * chunks); domains are sorted by work_begin.
template <int ST, bool PH, bool VD, int ROWS>
__global__ __launch_bounds__(Tile<ROWS>::NT) void k_step_fused_multi(const FusedDomain *__restrict__ doms, int ndom) {
    __shared__ Smem<PH, VD, ROWS> sm;
    const int w = xcd_work_item(blockIdx.x, gridDim.x);
    int lo = 0, hi = ndom - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (doms[mid].work_begin <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    const FusedDomain &d = doms[lo];
    // Every field is read once, here, into fresh local objects.  Used through the
    // reference instead, the record's fields are loaded where the step needs them,
    // inside the plane loop (the loads sit in conditional code, so the compiler
    // does not hoist them), together with the 64-bit products derived from them;
    // copied as a whole, the record stays in scratch memory.  Field by field, the
    // step compiles to the same loop as the single-lattice kernel.  The state is
    // accessed through global-address-space pointers for binary32 storage only:
    // for 16-bit storage that view spills scalar registers, and the flat
    // instructions cost less.
    Geo g;
    g.nx = d.g.nx; g.ny = d.g.ny; g.nz = d.g.nz;
    g.per[0] = d.g.per[0]; g.per[1] = d.g.per[1]; g.per[2] = d.g.per[2];
    g.N = d.g.N; g.ld = d.g.ld;
    Phys ph;
    ph.omega = d.ph.omega; ph.sigma = d.ph.sigma; ph.gamma = d.ph.gamma; ph.eps = d.ph.eps; ph.width = d.ph.width;
    ph.inlet_u = d.ph.inlet_u; ph.inlet_d = d.ph.inlet_d; ph.inlet_noise = d.ph.inlet_noise;
    ph.noise_key = d.ph.noise_key;
    ph.bc[0] = d.ph.bc[0]; ph.bc[1] = d.ph.bc[1]; ph.bc[2] = d.ph.bc[2];
    ph.bc[3] = d.ph.bc[3]; ph.bc[4] = d.ph.bc[4]; ph.bc[5] = d.ph.bc[5];
    if constexpr (VD) {
        ph.rho_b = d.ph.rho_b; ph.drho = d.ph.drho; ph.nu_b = d.ph.nu_b; ph.dnu = d.ph.dnu;
        ph.grav[0] = d.ph.grav[0]; ph.grav[1] = d.ph.grav[1]; ph.grav[2] = d.ph.grav[2];
    }
    Scales sc;
    sc.s2 = d.sc.s2; sc.s1 = d.sc.s1; sc.inv_s2 = d.sc.inv_s2; sc.inv_s1 = d.sc.inv_s1;
    StateView in, out;
    in.mom = d.in.mom; in.phi = d.in.phi; out.mom = d.out.mom; out.phi = d.out.phi;
    const int lz = d.lz, tx = d.tiles_x, ty = d.tiles_y, wb = d.work_begin;
    const unsigned long long sn = d.step_next;
    step_fused<ST, PH, (ST == ST_FP32), true, VD, ROWS>(sm, g, ph, sc, in, out, lz, tx, ty, sn, w - wb);
}

}  // namespace fused

// Tile height and z planes per workgroup.  A workgroup on a chunk of lz planes
// walks lz + 6 planes (the pipeline refills its rings), and the W work items of
// a launch give each CU ceil(W / CUs) of them, so the cost of a plan is
// ceil(W / CUs) (lz + 6) c, with c the time of one pipeline plane of a
// workgroup: 1 for 16 rows and kWideCost for 20 rows (measured on the
// 512 x 512 x 2048 jet: a 32 x 20 workgroup walks a plane in 1.18 times the
// time of a 32 x 16 one and updates 1.25 times the columns).  Long chunks
// recompute less halo, short ones keep every unit busy; ties go to the shorter
// chunk, then to 16 rows.  Chunks are capped (kMaxChunk16, kMaxChunk20 planes):
// workgroups that share halo columns run side by side, but over a long chunk
// they drift apart in z and their shared halo planes leave L2 before the
// neighbour reads them (HBM reads 1.48x the state at 2048 planes on a
// 512 x 512 x 2048 lattice, against 1.06x at 64 on 128 x 128 x 512).  The caps
// are measured on that lattice: 16-row tiles gained nothing beyond 128 planes,
// 20-row tiles ran 1.6 % faster at 256 than at 128 and slower at 342 or 683.
// 20 rows serve the two-component
// step with equal densities; the one-component step (whose 16-row workgroups
// fit twice in a CU's LDS) and the variable-density step take 16.  A height or
// chunk length fixed with tslb_set_tile / tslb_set_kernel is taken as given.
constexpr int kMaxChunk16 = 128, kMaxChunk20 = 256;
constexpr double kWideCost = 1.18;

bool fused_wide_allowed(const tslb_ctx *c) { return c->phase && !c->vd; }

namespace {

int tiles_of(const tslb_ctx *c, int rows) {
    return ((c->geo.nx + fused::Tile<16>::TX - 1) / fused::Tile<16>::TX) * ((c->geo.ny + rows - 1) / rows);
}

// Cheapest chunk length for `rows` and its cost (in 16-row plane times).
double best_chunk(const tslb_ctx *c, int rows, int *lz_out) {
    const long long tiles = tiles_of(c, rows);
    const long long cus = std::max(1, c->cu_count);
    const int nz = c->geo.nz;
    const double f = rows == 16 ? 1.0 : kWideCost;
    auto cost_of = [&](int lz) {
        const long long w = tiles * ((nz + lz - 1) / lz);
        return (double)((w + cus - 1) / cus) * (double)(lz + 6) * f;
    };
    if (c->chunk_z > 0) {
        *lz_out = c->chunk_z;
        return cost_of(c->chunk_z);
    }
    int best_lz = std::min(nz, 4);
    double best = -1.0;
    for (int k = 1; k <= nz; ++k) {  // k chunks of ceil(nz / k) planes
        const int lz = (nz + k - 1) / k;
        if (lz < 4 && k > 1) break;
        if (k > 1 && lz == (nz + k - 2) / (k - 1)) continue;  // same length as k - 1 chunks
        if (lz > (rows == 16 ? kMaxChunk16 : kMaxChunk20)) continue;
        const double cost = cost_of(lz);
        if (best < 0 || cost <= best) {
            best = cost;
            best_lz = lz;
        }
    }
    *lz_out = best_lz;
    return best < 0 ? cost_of(best_lz) : best;
}

}  // namespace

FusedPlan fused_plan(const tslb_ctx *c) {
    FusedPlan pl;
    int lz16 = 0, lz20 = 0;
    const double c16 = best_chunk(c, 16, &lz16);
    pl.rows = 16;
    pl.lz = lz16;
    if (!fused_wide_allowed(c) || c->tile_rows == 16) return pl;
    const double c20 = best_chunk(c, 20, &lz20);
    if (c->tile_rows == 20 || c20 < c16) {
        pl.rows = 20;
        pl.lz = lz20;
    }
    return pl;
}

int fused_chunk(const tslb_ctx *c) { return c->plan_lz; }

int fused_rows(const tslb_ctx *c) { return c->plan_rows; }

int fused_work_items(const tslb_ctx *c, int lz) {
    return tiles_of(c, fused_rows(c)) * ((c->geo.nz + lz - 1) / lz);
}

FusedDomain fused_domain(const tslb_ctx *c, StateView in, StateView out, int64_t step_next, int work_begin,
                         int lz) {
    FusedDomain d;
    d.g = c->geo;
    d.ph = c->phys;
    d.sc = c->scales;
    d.in = in;
    d.out = out;
    d.step_next = (unsigned long long)step_next;
    d.lz = lz > 0 ? lz : c->plan_lz;
    d.tiles_x = (c->geo.nx + fused::Tile<16>::TX - 1) / fused::Tile<16>::TX;
    d.tiles_y = (c->geo.ny + c->plan_rows - 1) / c->plan_rows;
    d.work_begin = work_begin;
    d.work_count = d.tiles_x * d.tiles_y * ((c->geo.nz + d.lz - 1) / d.lz);
    return d;
}

// Launch the fused step over the whole lattice.
namespace {

template <int ST, bool PH, bool VD, int ROWS>
void launch_one(unsigned blocks, hipStream_t s, const tslb_ctx *c, StateView in, StateView out, int lz, int tiles_x,
                int tiles_y, unsigned long long sn) {
    using namespace fused;
    hipLaunchKernelGGL((k_step_fused<ST, PH, VD, ROWS>), dim3(blocks), dim3(Tile<ROWS>::NT), 0, s, c->geo, c->phys,
                       c->scales, in, out, lz, tiles_x, tiles_y, sn);
}

template <int ST, bool PH, bool VD, int ROWS>
void launch_multi(unsigned blocks, hipStream_t s, const FusedDomain *doms, int ndom) {
    using namespace fused;
    hipLaunchKernelGGL((k_step_fused_multi<ST, PH, VD, ROWS>), dim3(blocks), dim3(Tile<ROWS>::NT), 0, s, doms, ndom);
}

}  // namespace

hipError_t launch_step_fused(const tslb_ctx *c, StateView in, StateView out, int lz, int64_t step_next,
                             hipStream_t s) {
    const int rows = fused_rows(c);
    const int tiles_x = (c->geo.nx + fused::Tile<16>::TX - 1) / fused::Tile<16>::TX;
    const int tiles_y = (c->geo.ny + rows - 1) / rows;
    const int chunks = (c->geo.nz + lz - 1) / lz;
    const unsigned blocks = (unsigned)tiles_x * tiles_y * chunks;
    const unsigned long long sn = (unsigned long long)step_next;
    if (c->vd) {  // variable density: binary32 storage, two components, 16 rows (validated at creation)
        if (c->storage != ST_FP32 || !c->phase || rows != 16) return hipErrorInvalidValue;
        launch_one<ST_FP32, true, true, 16>(blocks, s, c, in, out, lz, tiles_x, tiles_y, sn);
        return hipGetLastError();
    }
#define TSLB_FUSED_CASE(ST)                                                                            \
    case ST:                                                                                           \
        if (!c->phase)                                                                                 \
            launch_one<ST, false, false, 16>(blocks, s, c, in, out, lz, tiles_x, tiles_y, sn);         \
        else if (rows == 20)                                                                           \
            launch_one<ST, true, false, 20>(blocks, s, c, in, out, lz, tiles_x, tiles_y, sn);          \
        else                                                                                           \
            launch_one<ST, true, false, 16>(blocks, s, c, in, out, lz, tiles_x, tiles_y, sn);          \
        break;
    switch (c->storage) {
        TSLB_FUSED_CASE(ST_FP32)
        TSLB_FUSED_CASE(ST_FP16)
        TSLB_FUSED_CASE(ST_BF16)
        TSLB_FUSED_CASE(ST_FP16Q)
    default:
        return hipErrorInvalidValue;
    }
#undef TSLB_FUSED_CASE
    return hipGetLastError();
}

hipError_t launch_step_fused_multi(const FusedDomain *doms, int ndom, int total_work, int storage, bool phase,
                                   bool vd, int rows, hipStream_t s) {
    if (ndom <= 0 || total_work <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)total_work;
    if (vd) {
        if (storage != ST_FP32 || !phase || rows != 16) return hipErrorInvalidValue;
        launch_multi<ST_FP32, true, true, 16>(blocks, s, doms, ndom);
        return hipGetLastError();
    }
    if (rows != 16 && (rows != 20 || !phase)) return hipErrorInvalidValue;
#define TSLB_MULTI_CASE(ST)                                                                            \
    case ST:                                                                                           \
        if (!phase)                                                                                    \
            launch_multi<ST, false, false, 16>(blocks, s, doms, ndom);                                 \
        else if (rows == 20)                                                                           \
            launch_multi<ST, true, false, 20>(blocks, s, doms, ndom);                                  \
        else                                                                                           \
            launch_multi<ST, true, false, 16>(blocks, s, doms, ndom);                                  \
        break;
    switch (storage) {
        TSLB_MULTI_CASE(ST_FP32)
        TSLB_MULTI_CASE(ST_FP16)
        TSLB_MULTI_CASE(ST_BF16)
        TSLB_MULTI_CASE(ST_FP16Q)
    default:
        return hipErrorInvalidValue;
    }
#undef TSLB_MULTI_CASE
    return hipGetLastError();
}

}  // namespace tslb
