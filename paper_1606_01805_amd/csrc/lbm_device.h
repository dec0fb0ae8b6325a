// Device helpers shared by the forward and adjoint kernels of the coupled
// LBM / MLS-IBM step: lattice constants, population addressing and pulls,
// Zou-He closures, moments, force-patch lookups, the MLS operator and the
// per-tile particle lists.
#pragma once

#include <hip/hip_fp16.h>

#include "lbm_internal.h"

namespace lbmk {

// D2Q9 velocities in the order of Eq. (3) and their weights.
__device__ __forceinline__ constexpr int ex(int i) {
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__device__ __forceinline__ constexpr int ey(int i) {
    return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__device__ __forceinline__ constexpr double wd(int i) {
    return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}
__device__ __forceinline__ constexpr float wf(int i) {
    return i == 0 ? 4.0f / 9.0f : (i < 5 ? 1.0f / 9.0f : 1.0f / 36.0f);
}
__device__ __forceinline__ constexpr int wclass(int i) { return i == 0 ? 0 : (i < 5 ? 1 : 2); }

template <int ST> struct Sto;
template <> struct Sto<ST_F64> { using T = double; };
template <> struct Sto<ST_F32> { using T = float; };
template <> struct Sto<ST_F16S> { using T = __half; };

__device__ __forceinline__ long long pidx(const ChanDev& c, int i, int y, int x) {
    return c.off + (long long)i * c.plane + (long long)y * c.pitch + x;
}

// Byte offset of population i at node (x, y) from the start of the channel's
// block.  The library admits only channels whose block is below 4 GiB, so the
// offset is exact in 32 bits; it is zero-extended at the access, which lets
// the access use a scalar base with a 32-bit vector offset.
template <typename T>
__device__ __forceinline__ unsigned boff(const ChanDev& c, int i, int y, int x) {
    return ((unsigned)i * (unsigned)c.plane + (unsigned)y * (unsigned)c.pitch + (unsigned)x) *
           (unsigned)sizeof(T);
}
template <typename T>
__device__ __forceinline__ const T& at(const char* base, unsigned off) {
    return *(const T*)(base + off);
}
template <typename T>
__device__ __forceinline__ T& at(char* base, unsigned off) {
    return *(T*)(base + off);
}

// Source node of population i for a pull at (x, y).  Periodic axes wrap.  A
// source beyond a wall-bounded edge is replaced by the node itself (always a
// valid address): that population enters through the wall and is
// overwritten by the wall closure, which reads only the known populations.
__device__ __forceinline__ int pull_coord(int v, int self, int n, bool periodic) {
    const int lo = v < 0, hi = v >= n;
    return periodic ? v + (lo - hi) * n : ((lo | hi) ? self : v);
}

__device__ __forceinline__ void pull_src(const ChanDev& c, int i, int x, int y, int& xs, int& ys) {
    xs = pull_coord(x - ex(i), x, c.nx, c.bcx == 0);
    ys = pull_coord(y - ey(i), y, c.ny, c.bcy == 0);
}

// Wave-uniform copies (scalar registers) of values every lane holds alike.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ long long uni(long long v) {
    const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double uni(double v) { return __longlong_as_double(uni(__double_as_longlong(v))); }

// The channel descriptor a whole workgroup works on, in scalar registers:
// branches on the boundary kinds stay uniform.
__device__ __forceinline__ ChanDev load_chan(const ChanDev* p) {
    ChanDev c;
    c.nx = uni(p->nx);
    c.ny = uni(p->ny);
    c.pitch = uni(p->pitch);
    c.bcx = uni(p->bcx);
    c.bcy = uni(p->bcy);
    c.p_begin = uni(p->p_begin);
    c.p_end = uni(p->p_end);
    c.kernel = uni(p->kernel);
    c.spread_unit = uni(p->spread_unit);
    c.pad0 = 0;
    c.off = uni(p->off);
    c.plane = uni(p->plane);
    c.tau = uni(p->tau);
    c.nu = uni(p->nu);
    for (int s = 0; s < 4; ++s)
        for (int k = 0; k < 2; ++k) {
            c.uw[s][k] = uni(p->uw[s][k]);
            c.f_uw[s][k] = uni(p->f_uw[s][k]);
        }
    for (int k = 0; k < 2; ++k) {
        c.g[k] = uni(p->g[k]);
        c.grav[k] = uni(p->grav[k]);
        c.f_g[k] = uni(p->f_g[k]);
    }
    c.rw = uni(p->rw);
    c.alpha = uni(p->alpha);
    c.dn = uni(p->dn);
    c.f_omega = uni(p->f_omega);
    c.f_pref = uni(p->f_pref);
    for (int k = 0; k < 3; ++k) {
        c.sc[k] = uni(p->sc[k]);
        c.isc[k] = uni(p->isc[k]);
    }
    c.tile0 = uni(p->tile0);
    c.tiles_x = uni(p->tiles_x);
    return c;
}

// ---------------------------------------------------------------------------
// FP64 form: populations f_i, expressions in reference order.
// ---------------------------------------------------------------------------
// Zou-He known-velocity wall (Sec. 1.1): mass and normal momentum fix rho,
// bounce-back of the non-equilibrium normal population, tangential momentum
// for the two diagonals; target momentum m = rho u_w - g/2.
// Zou-He closures of the four walls (node on the wall, known wall velocity
// u_w, body force g): the unknown populations follow from the density and
// the target momentum m = rho u_w - g/2, with the bounce-back of the
// non-equilibrium normal part.  Each axis is one pass that evaluates both
// of its walls' closures from the incoming populations and selects per
// lane, so the arrays are only ever indexed by constants (a store behind a
// per-lane branch can be merged by the compiler into one store at a computed
// index, which sends the whole array to private memory).  The pass runs only
// if a lane of the wave lies on one of its walls.  The wall velocities are
// read from w: the register copy c itself, or the descriptor in memory, so a
// kernel with tight scalar registers loads them only in the wall rows.
__device__ __forceinline__ void walls_f64(const ChanDev& c, const ChanDev& w, int x, int y, double f[9]) {
    const double gx = c.g[0], gy = c.g[1];
    const bool s2 = c.bcy == 1 && y == 0;
    const bool s3 = c.bcy == 1 && !s2 && y == c.ny - 1;
    if (__any(s2 || s3)) {
        // y = 0 (side 2): unknowns 2, 5, 6
        double rho = (f[0] + f[1] + f[3] + 2.0 * (f[4] + f[7] + f[8]) - 0.5 * gy) / (1.0 - w.uw[2][1]);
        double mx = rho * w.uw[2][0] - 0.5 * gx;
        double my = rho * w.uw[2][1] - 0.5 * gy;
        const double a2 = f[4] + 2.0 * my / 3.0;
        const double a5 = f[7] - 0.5 * (f[1] - f[3]) + 0.5 * mx + my / 6.0;
        const double a6 = f[8] + 0.5 * (f[1] - f[3]) - 0.5 * mx + my / 6.0;
        // y = ny - 1 (side 3): unknowns 4, 7, 8
        rho = (f[0] + f[1] + f[3] + 2.0 * (f[2] + f[5] + f[6]) + 0.5 * gy) / (1.0 + w.uw[3][1]);
        mx = rho * w.uw[3][0] - 0.5 * gx;
        my = rho * w.uw[3][1] - 0.5 * gy;
        const double b4 = f[2] - 2.0 * my / 3.0;
        const double b7 = f[5] + 0.5 * (f[1] - f[3]) - 0.5 * mx - my / 6.0;
        const double b8 = f[6] - 0.5 * (f[1] - f[3]) + 0.5 * mx - my / 6.0;
        f[2] = s2 ? a2 : f[2];
        f[5] = s2 ? a5 : f[5];
        f[6] = s2 ? a6 : f[6];
        f[4] = s3 ? b4 : f[4];
        f[7] = s3 ? b7 : f[7];
        f[8] = s3 ? b8 : f[8];
    }
    const bool s0 = c.bcx == 1 && x == 0;
    const bool s1 = c.bcx == 1 && !s0 && x == c.nx - 1;
    if (__any(s0 || s1)) {
        // x = 0 (side 0): unknowns 1, 5, 8
        double rho = (f[0] + f[2] + f[4] + 2.0 * (f[3] + f[6] + f[7]) - 0.5 * gx) / (1.0 - w.uw[0][0]);
        double mx = rho * w.uw[0][0] - 0.5 * gx;
        double my = rho * w.uw[0][1] - 0.5 * gy;
        const double a1 = f[3] + 2.0 * mx / 3.0;
        const double a5 = f[7] - 0.5 * (f[2] - f[4]) + mx / 6.0 + 0.5 * my;
        const double a8 = f[6] + 0.5 * (f[2] - f[4]) + mx / 6.0 - 0.5 * my;
        // x = nx - 1 (side 1): unknowns 3, 7, 6
        rho = (f[0] + f[2] + f[4] + 2.0 * (f[1] + f[5] + f[8]) + 0.5 * gx) / (1.0 + w.uw[1][0]);
        mx = rho * w.uw[1][0] - 0.5 * gx;
        my = rho * w.uw[1][1] - 0.5 * gy;
        const double b3 = f[1] - 2.0 * mx / 3.0;
        const double b7 = f[5] + 0.5 * (f[2] - f[4]) - mx / 6.0 - 0.5 * my;
        const double b6 = f[8] - 0.5 * (f[2] - f[4]) - mx / 6.0 + 0.5 * my;
        f[1] = s0 ? a1 : f[1];
        f[5] = s0 ? a5 : f[5];
        f[8] = s0 ? a8 : f[8];
        f[3] = s1 ? b3 : f[3];
        f[7] = s1 ? b7 : f[7];
        f[6] = s1 ? b6 : f[6];
    }
}

// ---------------------------------------------------------------------------
// Reduced forms: deviations d_i = f_i - w_i in FP32.
// ---------------------------------------------------------------------------
// A stored F16S value h times the inverse scale 2^-(K + k_i).  The product is
// exact in FP32, so one mixed-precision FMA (which reads the half directly)
// gives the value of convert-then-multiply; the +0 addend (a -0 one would be
// folded back into the multiply) only turns a -0 product into +0.
__device__ __forceinline__ float unscale_h(__half h, float isc) {
    return __builtin_fmaf(__half2float(h), isc, 0.0f);
}

template <int ST>
__device__ __forceinline__ float load_dev(const typename Sto<ST>::T* p, long long k, int i,
                                          const ChanDev& c) {
    if constexpr (ST == ST_F32) {
        return p[k];
    } else {
        return unscale_h(p[k], c.isc[wclass(i)]);
    }
}

template <int ST>
__device__ __forceinline__ void store_dev(typename Sto<ST>::T* p, long long k, int i, float d,
                                          const ChanDev& c) {
    if constexpr (ST == ST_F32) {
        p[k] = d;
    } else {
        p[k] = __float2half_rn(d * c.sc[wclass(i)]);
    }
}

// The Zou-He closures of walls_f64 written for deviations: the weights of
// the known populations entering rho sum to 1, and w_i cancels in every
// difference.  Same pass structure and the same source w of the wall
// velocities.
__device__ __forceinline__ void walls_dev(const ChanDev& c, const ChanDev& w, int x, int y, float d[9]) {
    const float gx = c.f_g[0], gy = c.f_g[1];
    const bool s2 = c.bcy == 1 && y == 0;
    const bool s3 = c.bcy == 1 && !s2 && y == c.ny - 1;
    if (__any(s2 || s3)) {
        float uwx = w.f_uw[2][0], uwy = w.f_uw[2][1];
        float sm = d[0] + d[1] + d[3] + 2.0f * (d[4] + d[7] + d[8]);
        float rho = 1.0f + (sm - 0.5f * gy + uwy) / (1.0f - uwy);
        float mx = rho * uwx - 0.5f * gx;
        float my = rho * uwy - 0.5f * gy;
        const float a2 = d[4] + (2.0f / 3.0f) * my;
        const float a5 = d[7] - 0.5f * (d[1] - d[3]) + 0.5f * mx + my * (1.0f / 6.0f);
        const float a6 = d[8] + 0.5f * (d[1] - d[3]) - 0.5f * mx + my * (1.0f / 6.0f);
        uwx = w.f_uw[3][0];
        uwy = w.f_uw[3][1];
        sm = d[0] + d[1] + d[3] + 2.0f * (d[2] + d[5] + d[6]);
        rho = 1.0f + (sm + 0.5f * gy - uwy) / (1.0f + uwy);
        mx = rho * uwx - 0.5f * gx;
        my = rho * uwy - 0.5f * gy;
        const float b4 = d[2] - (2.0f / 3.0f) * my;
        const float b7 = d[5] + 0.5f * (d[1] - d[3]) - 0.5f * mx - my * (1.0f / 6.0f);
        const float b8 = d[6] - 0.5f * (d[1] - d[3]) + 0.5f * mx - my * (1.0f / 6.0f);
        d[2] = s2 ? a2 : d[2];
        d[5] = s2 ? a5 : d[5];
        d[6] = s2 ? a6 : d[6];
        d[4] = s3 ? b4 : d[4];
        d[7] = s3 ? b7 : d[7];
        d[8] = s3 ? b8 : d[8];
    }
    const bool s0 = c.bcx == 1 && x == 0;
    const bool s1 = c.bcx == 1 && !s0 && x == c.nx - 1;
    if (__any(s0 || s1)) {
        float uwx = w.f_uw[0][0], uwy = w.f_uw[0][1];
        float sm = d[0] + d[2] + d[4] + 2.0f * (d[3] + d[6] + d[7]);
        float rho = 1.0f + (sm - 0.5f * gx + uwx) / (1.0f - uwx);
        float mx = rho * uwx - 0.5f * gx;
        float my = rho * uwy - 0.5f * gy;
        const float a1 = d[3] + (2.0f / 3.0f) * mx;
        const float a5 = d[7] - 0.5f * (d[2] - d[4]) + mx * (1.0f / 6.0f) + 0.5f * my;
        const float a8 = d[6] + 0.5f * (d[2] - d[4]) + mx * (1.0f / 6.0f) - 0.5f * my;
        uwx = w.f_uw[1][0];
        uwy = w.f_uw[1][1];
        sm = d[0] + d[2] + d[4] + 2.0f * (d[1] + d[5] + d[8]);
        rho = 1.0f + (sm + 0.5f * gx - uwx) / (1.0f + uwx);
        mx = rho * uwx - 0.5f * gx;
        my = rho * uwy - 0.5f * gy;
        const float b3 = d[1] - (2.0f / 3.0f) * mx;
        const float b7 = d[5] + 0.5f * (d[2] - d[4]) - mx * (1.0f / 6.0f) - 0.5f * my;
        const float b6 = d[8] - 0.5f * (d[2] - d[4]) - mx * (1.0f / 6.0f) + 0.5f * my;
        d[1] = s0 ? a1 : d[1];
        d[5] = s0 ? a5 : d[5];
        d[8] = s0 ? a8 : d[8];
        d[3] = s1 ? b3 : d[3];
        d[7] = s1 ? b7 : d[7];
        d[6] = s1 ? b6 : d[6];
    }
}

// Closed boxes (Zou-He walls on both axes, walls at rest, no fluid body
// force): a corner node has five unknown populations.  The axis and
// diagonal ones that point into the fluid bounce back their opposites; the
// two buried diagonals (along neither wall normal) share what the density
// rho_c of the diagonal interior neighbour leaves after the other seven.
// The neighbour is interior, so its pulled populations need no closure.
// (sx, sy): the direction of that neighbour.  The arrays are indexed only by
// constants: the four corners are selected per lane.
__device__ __forceinline__ bool corner_dir(const ChanDev& c, int x, int y, int& sx, int& sy) {
    const bool x0 = x == 0, x1 = x == c.nx - 1, y0 = y == 0, y1 = y == c.ny - 1;
    sx = x0 ? 1 : -1;
    sy = y0 ? 1 : -1;
    return (x0 || x1) && (y0 || y1);
}

template <typename V>
__device__ __forceinline__ void corner_closure(V f[9], V rho_c, int sx, int sy, V half) {
    const bool bl = sx > 0 && sy > 0, br = sx < 0 && sy > 0, tl = sx > 0 && sy < 0,
               tr = sx < 0 && sy < 0;
    const V f1 = sx > 0 ? f[3] : f[1], f3 = sx < 0 ? f[1] : f[3];
    const V f2 = sy > 0 ? f[4] : f[2], f4 = sy < 0 ? f[2] : f[4];
    const V f5 = bl ? f[7] : f[5], f6 = br ? f[8] : f[6];
    const V f7 = tr ? f[5] : f[7], f8 = tl ? f[6] : f[8];
    const bool pair68 = sx == sy;  // buried pair (6, 8), else (5, 7)
    const V rest = pair68 ? f[0] + f1 + f2 + f3 + f4 + f5 + f7 : f[0] + f1 + f2 + f3 + f4 + f6 + f8;
    const V b = half * (rho_c - rest);
    f[1] = f1;
    f[2] = f2;
    f[3] = f3;
    f[4] = f4;
    f[5] = pair68 ? f5 : b;
    f[7] = pair68 ? f7 : b;
    f[6] = pair68 ? b : f6;
    f[8] = pair68 ? b : f8;
}

// FP64 populations f at node (x, y) after the side closures: the corner
// closure, with rho_c summed over the neighbour's pulled populations in
// ascending order.  base: the channel's block of the input buffer.
__device__ __forceinline__ void corners_f64(const char* base, const ChanDev& c, int x, int y, double f[9]) {
    if (!(c.bcx == 1 && c.bcy == 1)) return;
    int sx, sy;
    const bool corner = corner_dir(c, x, y, sx, sy);
    if (!__any(corner)) return;
    if (corner) {
        double rc = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int xs, ys;
            pull_src(c, i, x + sx, y + sy, xs, ys);
            rc += at<double>(base, boff<double>(c, i, ys, xs));
        }
        corner_closure<double>(f, rc, sx, sy, 0.5);
    }
}

// The same for FP32 deviations d_i = f_i - w_i: the weights of the seven
// populations outside the buried pair sum to 17/18, which leaves
// d_b = (drho_c - sum of the seven d) / 2 for the buried pair.
template <int ST>
__device__ __forceinline__ void corners_dev(const char* base, const ChanDev& c, int x, int y, float d[9]) {
    using T = typename Sto<ST>::T;
    if (!(c.bcx == 1 && c.bcy == 1)) return;
    int sx, sy;
    const bool corner = corner_dir(c, x, y, sx, sy);
    if (!__any(corner)) return;
    if (corner) {
        float g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int xs, ys;
            pull_src(c, i, x + sx, y + sy, xs, ys);
            const T v = at<T>(base, boff<T>(c, i, ys, xs));
            if constexpr (ST == ST_F32) g[i] = v;
            else g[i] = unscale_h(v, c.isc[wclass(i)]);
        }
        const float drc = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
        corner_closure<float>(d, drc, sx, sy, 0.5f);
    }
}

// The nine stored values that the pull of node (x, y) reads, loaded with no
// arithmetic on them, so that their latency can overlap other work.
template <int ST>
__device__ __forceinline__ void pull_load(const void* fin, const ChanDev& c, int x, int y,
                                          typename Sto<ST>::T raw[9]) {
    using T = typename Sto<ST>::T;
    const char* base = (const char*)fin + c.off * (long long)sizeof(T);  // the channel's block
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int xs, ys;
        pull_src(c, i, x, y, xs, ys);
        raw[i] = at<T>(base, boff<T>(c, i, ys, xs));
    }
}

// Streamed populations f^n at node (x, y) from its loaded values, as FP64 f_i
// (all forms): deviations restored, walls applied.
template <int ST>
__device__ __forceinline__ void pull_finish_f64(const void* fin, const ChanDev& c, int x, int y,
                                                const typename Sto<ST>::T raw[9], double f[9]) {
    using T = typename Sto<ST>::T;
    const char* base = (const char*)fin + c.off * (long long)sizeof(T);  // the channel's block
    if constexpr (ST == ST_F64) {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = raw[i];
        walls_f64(c, c, x, y, f);
        corners_f64(base, c, x, y, f);
    } else {
        float d[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            if constexpr (ST == ST_F32) d[i] = raw[i];
            else d[i] = unscale_h(raw[i], c.isc[wclass(i)]);
        }
        walls_dev(c, c, x, y, d);
        corners_dev<ST>(base, c, x, y, d);
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = wd(i) + (double)d[i];
    }
}

// Streamed populations f^n at one node, as FP64 f_i (all forms).
template <int ST>
__device__ __forceinline__ void pull_node_f64(const void* fin, const ChanDev& c, int x, int y,
                                              double f[9]) {
    typename Sto<ST>::T raw[9];
    pull_load<ST>(fin, c, x, y, raw);
    pull_finish_f64<ST>(fin, c, x, y, raw, f);
}

// Moments of Eqs. (6), (7) before the IB force is known: rho and
// j* = sum f e + g/2, summed over i in ascending order.
__device__ __forceinline__ void moments_f64(const double f[9], const ChanDev& c, double& rho,
                                            double& jx, double& jy) {
    rho = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) rho += f[i];
    // the sums of f_i e_i in ascending i over the directions with e != 0
    // (the others add signed zeros, which change no nonzero sum)
    jx = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
    jy = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
    jx += 0.5 * c.g[0];
    jy += 0.5 * c.g[1];
}

// IB force of particle P's patch at patch cell `cell`.  For a particle of
// several rounds of kRound markers, with a.sum_partials set, it is the sum of
// the per-round partial patches in ascending round order (the first round
// starts the sum), exactly what the partial-sum kernel writes into the patch.
__device__ __forceinline__ double2 patch_value(const StepArgs& a, const PartDev& P, long long cell) {
    const int nr = (P.nm + kRound - 1) / kRound;
    if (nr == 1 || !a.sum_partials) return a.patch[P.patch_off + cell];
    const double2* part = a.partial + P.part_off + cell;
    double2 acc = part[0];
    for (int r = 1; r < nr; ++r) {
        const double2 v = part[(long long)r * P.patch_cap];
        acc.x += v.x;
        acc.y += v.y;
    }
    return acc;
}

// Force patches of a channel's particles covering node (x, y), summed in
// ascending particle order.  Boxes hold wrapped origins on periodic axes.
__device__ __forceinline__ void patch_force(const StepArgs& a, const ChanDev& c, int x, int y,
                                            double& fx, double& fy) {
    fx = 0.0;
    fy = 0.0;
    for (int q = c.p_begin; q < c.p_end; ++q) {
        const PartDev& P = a.parts[q];
        int dx = x - P.bx0, dy = y - P.by0;
        if (c.bcx == 0 && dx < 0) dx += c.nx;
        if (c.bcy == 0 && dy < 0) dy += c.ny;
        if (dx >= 0 && dx < P.bw && dy >= 0 && dy < P.bh) {
            const double2 v = patch_value(a, P, (long long)dy * P.bw + dx);
            fx += v.x;
            fy += v.y;
        }
    }
}

// The same sum over a short list of candidate particles (ascending).
__device__ __forceinline__ void patch_force_list(const StepArgs& a, const ChanDev& c,
                                                 const int* list, int n, int x, int y,
                                                 double& fx, double& fy) {
    fx = 0.0;
    fy = 0.0;
    for (int j = 0; j < n; ++j) {
        const PartDev& P = a.parts[list[j]];
        int dx = x - P.bx0, dy = y - P.by0;
        if (c.bcx == 0 && dx < 0) dx += c.nx;
        if (c.bcy == 0 && dy < 0) dy += c.ny;
        if (dx >= 0 && dx < P.bw && dy >= 0 && dy < P.bh) {
            const double2 v = patch_value(a, P, (long long)dy * P.bw + dx);
            fx += v.x;
            fy += v.y;
        }
    }
}

// A listed particle's force patch as the lattice pass reads it: its box, the
// first of its values (the patch, or the first round's partial patch when the
// partials are summed by their readers), and the rounds and their stride.
struct PatchRef {
    const double2* base;
    int bx0, by0, bw, bh;
    int nr;                  // values added per cell (rounds of kRound markers)
    int cap;                 // stride between the rounds' partial patches
};

__device__ __forceinline__ PatchRef patch_ref(const StepArgs& a, const PartDev& P) {
    PatchRef R;
    const int nr = (P.nm + kRound - 1) / kRound;
    const bool parts = nr > 1 && a.sum_partials;
    R.base = parts ? a.partial + P.part_off : a.patch + P.patch_off;
    R.bx0 = P.bx0;
    R.by0 = P.by0;
    R.bw = P.bw;
    R.bh = P.bh;
    R.nr = parts ? nr : 1;
    R.cap = P.patch_cap;
    return R;
}

// The sum of patch_value over the particles of a tile, from their PatchRef
// table (ascending particle index): the same terms in the same order as the
// sum over the particle records.
__device__ __forceinline__ void patch_force_tab(const ChanDev& c, const PatchRef* tab, int n, int x, int y,
                                                double& fx, double& fy) {
    fx = 0.0;
    fy = 0.0;
    for (int j = 0; j < n; ++j) {
        const PatchRef R = tab[j];
        int dx = x - R.bx0, dy = y - R.by0;
        if (c.bcx == 0 && dx < 0) dx += c.nx;
        if (c.bcy == 0 && dy < 0) dy += c.ny;
        if (dx >= 0 && dx < R.bw && dy >= 0 && dy < R.bh) {
            const double2* p = R.base + ((long long)dy * R.bw + dx);
            double2 v = p[0];
            for (int r = 1; r < R.nr; ++r) {
                const double2 u = p[(long long)r * R.cap];
                v.x += u.x;
                v.y += u.y;
            }
            fx += v.x;
            fy += v.y;
        }
    }
}

// patch_force_tab for the NV consecutive nodes [xb, xb + NV) of row y at
// once (nodes at or past the channel's last column excluded): per node the
// same terms in the same order, with each round's values for all NV nodes
// requested together rather than node by node.
template <int NV>
__device__ __forceinline__ void patch_force_row(const ChanDev& c, const PatchRef* tab, int n, int xb, int y,
                                               double (&fx)[NV], double (&fy)[NV]) {
#pragma unroll
    for (int j = 0; j < NV; ++j) fx[j] = fy[j] = 0.0;
    for (int e = 0; e < n; ++e) {
        const PatchRef R = tab[e];
        int dy = y - R.by0;
        if (c.bcy == 0 && dy < 0) dy += c.ny;
        if (dy < 0 || dy >= R.bh) continue;
        const double2* row = R.base + (long long)dy * R.bw;
        bool in[NV];
        int cx[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            int dx = xb + j - R.bx0;
            if (c.bcx == 0 && dx < 0) dx += c.nx;
            in[j] = xb + j < c.nx && dx >= 0 && dx < R.bw;
            cx[j] = in[j] ? dx : 0;
        }
        double2 v[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = in[j] ? row[cx[j]] : make_double2(0.0, 0.0);
        for (int r = 1; r < R.nr; ++r) {
            const double2* pr = row + (long long)r * R.cap;
            double2 u[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) u[j] = in[j] ? pr[cx[j]] : make_double2(0.0, 0.0);
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                v[j].x += u[j].x;
                v[j].y += u[j].y;
            }
        }
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (in[j]) {
                fx[j] += v[j].x;
                fy[j] += v[j].y;
            }
    }
}

// Inserts v into the ascending register list L[0, n) unless present.
template <int N>
__device__ __forceinline__ void list_insert(int (&L)[N], int& n, int v) {
    bool dup = false;
    int pos = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const bool in = m < n;
        dup |= in && L[m] == v;
        pos += (in && L[m] < v) ? 1 : 0;
    }
    if (dup || n >= N) return;
#pragma unroll
    for (int m = N - 1; m >= 1; --m) L[m] = m < pos ? L[m] : (m == pos ? v : L[m - 1]);
    L[0] = pos == 0 ? v : L[0];
    ++n;
}

// Do the boxes [x0, x0 + w) x [y0, y0 + h) and [u0, u0 + p) x [v0, v0 + q)
// intersect?  Origins may be unwrapped; periodic axes compare modulo n.
// acc + v[0] + v[stride] + ... + v[(n - 1) * stride], added in that order,
// with the (LDS) reads issued eight at a time instead of one per add.
__device__ __forceinline__ double ordered_sum(double acc, const double* v, int n, int stride) {
    int m = 0;
    for (; m + 8 <= n; m += 8) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = v[(m + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += t[u];
    }
    for (; m < n; ++m) acc += v[m * stride];
    return acc;
}

__device__ __forceinline__ bool span_overlap(int x0, int w, int u0, int p, int n, bool per) {
    if (!per) return x0 < u0 + p && u0 < x0 + w;
    if (w >= n || p >= n) return true;
    int d1 = (u0 - x0) % n, d2 = (x0 - u0) % n;
    if (d1 < 0) d1 += n;
    if (d2 < 0) d2 += n;
    return d1 < w || d2 < p;
}

__device__ __forceinline__ bool boxes_overlap(const ChanDev& c, int x0, int y0, int w, int h,
                                              int u0, int v0, int p, int q) {
    return span_overlap(x0, w, u0, p, c.nx, c.bcx == 0) && span_overlap(y0, h, v0, q, c.ny, c.bcy == 0);
}

// ---------------------------------------------------------------------------
// MLS transfer operator (Sec. 1.2, Eqs. (8)-(10)) at one point, FP64.
// 3x3 nodes around the nearest node (round half up); shifted linear basis
// (1, x_k - x, y_k - y); nodes beyond a wall-bounded edge are dropped; the 3x3
// moment matrix is inverted through its adjugate.  Outputs the anchor, the
// validity mask and the value / x-derivative / y-derivative weights.
// ---------------------------------------------------------------------------
// Kernels of Sec. 2.2: exponential (Eq. (10)), cubic, quartic, cosine
// (Eqs. (17)-(19)) and polynomial (Eq. (20)), the last with its two branches
// evaluated at q = 2 r (break points q = 1 and 2: the four-point delta
// function of immersed-boundary methods).
__device__ __forceinline__ double kernel_weight(int kind, double r, double alpha) {
    if (r > 1.0) return 0.0;
    if (kind == 0) {
        double q = r / alpha;
        return exp(-(q * q));
    } else if (kind == 1) {
        return 2.0 / 3.0 - 4.0 * r * r + 4.0 * r * r * r;
    } else if (kind == 2) {
        return 1.0 - 6.0 * r * r + 8.0 * r * r * r - 3.0 * r * r * r * r;
    } else if (kind == 3) {
        return 0.25 * (1.0 + cos(3.14159265358979323846 / 2.0 * r));
    }
    const double q = 2.0 * r;
    if (q <= 1.0) return (3.0 - 2.0 * q + sqrt(1.0 + 4.0 * q - 4.0 * q * q)) / 8.0;
    return (5.0 - 2.0 * q - sqrt(-7.0 + 12.0 * q - 4.0 * q * q)) / 8.0;
}

__device__ __forceinline__ int wrapc(int v, int n, int periodic) {
    if (!periodic) return v;
    // one period either side by a conditional add; the remainder (an
    // integer division) only where some lane of the wave lies further out
    if (__any(v < -n || v >= 2 * n)) {
        v %= n;
        return v < 0 ? v + n : v;
    }
    v += v < 0 ? n : 0;
    return v >= n ? v - n : v;
}

// Box [x0, x0 + w) x [y0, y0 + h), in unwrapped lattice coordinates, that
// holds every 3x3 stencil node of any point within `reach` of (X0, X1):
// anchors round half up, plus one node on each side.
__device__ __forceinline__ void stencil_box(double X0, double X1, double reach, int& x0, int& y0,
                                            int& w, int& h) {
    const double r = reach + 1e-6;
    x0 = (int)floor(X0 - r + 0.5) - 1;
    y0 = (int)floor(X1 - r + 0.5) - 1;
    w = (int)floor(X0 + r + 0.5) + 2 - x0;
    h = (int)floor(X1 + r + 0.5) + 2 - y0;
}

// Marker kinematics of Sec. 1.2: body-frame offset rotated by theta.
struct Marker {
    double rx, ry, xl, yl;
    int i0, j0;
};

__device__ __forceinline__ Marker marker_from(double2 x, double X0, double X1, double cs, double sn) {
    Marker m;
    m.rx = cs * x.x - sn * x.y;
    m.ry = sn * x.x + cs * x.y;
    m.xl = X0 + m.rx;
    m.yl = X1 + m.ry;
    m.i0 = (int)floor(m.xl + 0.5);
    m.j0 = (int)floor(m.yl + 0.5);
    return m;
}

__device__ __forceinline__ Marker marker_at(const StepArgs& a, int idx, double X0, double X1,
                                            double cs, double sn) {
    return marker_from(a.xi[idx], X0, X1, cs, sn);
}

// Stencil node k of the 3x3 support around anchor (i0, j0): distance
// components d = x_k - x, wrapped node, validity (beyond a wall-bounded edge
// the node is dropped).
__device__ __forceinline__ bool stencil_node(const ChanDev& c, int i0, int j0, int k, double x,
                                             double y, double& dx, double& dy, int& ni, int& nj) {
    const int ii = i0 + k % 3 - 1, jj = j0 + k / 3 - 1;
    dx = (double)ii - x;
    dy = (double)jj - y;
    ni = wrapc(ii, c.nx, c.bcx == 0);
    nj = wrapc(jj, c.ny, c.bcy == 0);
    return (c.bcx == 0 || (ii >= 0 && ii < c.nx)) && (c.bcy == 0 || (jj >= 0 && jj < c.ny));
}

__device__ __forceinline__ bool node_valid(const ChanDev& c, int ii, int jj) {
    return (c.bcx == 0 || (ii >= 0 && ii < c.nx)) && (c.bcy == 0 || (jj >= 0 && jj < c.ny));
}

__device__ __forceinline__ double stencil_weight(const ChanDev& c, double dx, double dy) {
    const double r = sqrt(dx * dx + dy * dy) / c.rw;
    return kernel_weight(c.kernel, r, c.alpha);
}

// Inverse (through the adjugate) of the moment matrix of Eq. (9), accumulated
// over the valid nodes in ascending k from the weights in w[0..8].
struct MlsInv {
    double i00, i01, i02, i11, i12, i22;
};

// w[q] must be exactly zero at stencil nodes dropped beyond a wall: their
// terms are then signed zeros, which leave every sum (started at +0) bitwise
// unchanged, so the loop needs no branch.
__device__ __forceinline__ MlsInv mls_inverse(const double* w, int i0, int j0, double x, double y,
                                              bool all) {
    double A00 = 0.0, A01 = 0.0, A02 = 0.0, A11 = 0.0, A12 = 0.0, A22 = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int ii = i0 + q % 3 - 1, jj = j0 + q / 3 - 1;
        const double dx = (double)ii - x, dy = (double)jj - y, wk = w[q];
        A00 += wk;
        A01 += wk * dx;
        A02 += wk * dy;
        A11 += wk * dx * dx;
        A12 += wk * dx * dy;
        A22 += wk * dy * dy;
    }
    const double c00 = A11 * A22 - A12 * A12;
    const double c01 = A02 * A12 - A01 * A22;
    const double c02 = A01 * A12 - A02 * A11;
    const double det = A00 * c00 + A01 * c01 + A02 * c02;
    MlsInv r;
    r.i00 = c00 / det;
    r.i01 = c01 / det;
    r.i02 = c02 / det;
    r.i11 = r.i12 = r.i22 = 0.0;
    if (all) {
        const double c11 = A00 * A22 - A02 * A02;
        const double c12 = A01 * A02 - A00 * A12;
        const double c22 = A00 * A11 - A01 * A01;
        r.i11 = c11 / det;
        r.i12 = c12 / det;
        r.i22 = c22 / det;
    }
    return r;
}

// Append particle pid to the lists of the lattice tiles that its patch box
// [x0, x0 + w) x [y0, y0 + h) (unwrapped coordinates) overlaps, so the
// lattice pass looks up particle forces only there and only for listed
// particles.  Periodic ranges split into at most two pieces.
__device__ __forceinline__ void mark_tiles(const StepArgs& a, const ChanDev& c, int pid, int x0,
                                           int y0, int w, int h, int tid, int nthr) {
    int xr[2][2], yr[2][2], nxr = 0, nyr = 0;
    auto split = [](int lo, int len, int n, bool per, int r[2][2]) {
        int cnt = 0;
        if (per) {
            int s0 = wrapc(lo, n, 1);
            int e0 = s0 + len - 1;
            if (e0 < n) {
                r[0][0] = s0; r[0][1] = e0; cnt = 1;
            } else {
                r[0][0] = s0; r[0][1] = n - 1; r[1][0] = 0; r[1][1] = e0 - n; cnt = 2;
            }
        } else {
            int s0 = max(lo, 0), e0 = min(lo + len - 1, n - 1);
            if (s0 <= e0) { r[0][0] = s0; r[0][1] = e0; cnt = 1; }
        }
        return cnt;
    };
    nxr = split(x0, w, c.nx, c.bcx == 0, xr);
    nyr = split(y0, h, c.ny, c.bcy == 0, yr);
    int* tl = a.tlist + (long long)a.parity * a.ntiles * kTileList;
    for (int p = 0; p < nxr; ++p)
        for (int q = 0; q < nyr; ++q) {
            const int tx0 = xr[p][0] / a.tile_w, tx1 = xr[p][1] / a.tile_w;
            const int ty0 = yr[q][0] / a.tile_h, ty1 = yr[q][1] / a.tile_h;
            const int ntx = tx1 - tx0 + 1, cnt = ntx * (ty1 - ty0 + 1);
            for (int t = tid; t < cnt; t += nthr) {
                int* e = tl + (long long)(c.tile0 + (ty0 + t / ntx) * c.tiles_x + tx0 + t % ntx) * kTileList;
                const int slot = atomicAdd(e, 1);
                if (slot < kTileList - 1) e[1 + slot] = pid;
            }
        }
}

}  // namespace lbmk
