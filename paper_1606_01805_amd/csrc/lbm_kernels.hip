// gfx950 kernels of the coupled LBM / MLS-IBM time step.
//
// Per step, in stream order:
//   ibm_force  one workgroup per round of 64 markers of a particle: marker
//              kinematics, MLS shape functions at the markers (Sec. 1.2,
//              Eqs. (8)-(10)), velocity interpolation from the pulled
//              populations, Lagrangian force (Eq. (11)) and an atomic-free,
//              deterministic spreading of c_l phi F_l into the particle's
//              force patch, or into the round's partial patch for particles of
//              several rounds (Eq. (12)).
//   lattice    one workgroup per tile (or a persistent grid striding over the
//              tile table of all channels): pull streaming, Zou-He walls,
//              moments, forced BGK collision (Eqs. (2)-(7)), SoA store.
//   traction   one workgroup per round of 64 markers: probe MLS, surface
//              stress; the particle's last workgroup sums force and moment
//              (Eqs. (13), (14)), advances BDF2 (Eqs. (15), (16)) and records.
// lattice_traction runs the last two as one launch (particle workgroups
// first), and patch_sum adds partial patches for the adjoint's tape.
//
// Populations are SoA: [channel block][9][ny][pitch], x fastest.  The buffer
// read by a step holds the post-collision populations of the previous step;
// pulling f_i(x) = f^c_i(x - e_i) gives the streamed populations on the fly.
//
// The FP64 form evaluates every expression in the order of the plain
// reference formulation (compiled without FMA contraction), so that for the
// same inputs its lattice arithmetic is the same IEEE operation sequence.
// The FP32 and FP16S forms keep the deviation d_i = f_i - w_i and compute in
// FP32, with fused multiply-adds.  The immersed-boundary and rigid-body stages are FP64 in every form.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "lbm_device.h"

namespace lbmk {

// ---------------------------------------------------------------------------
// Cross-workgroup completion of a particle whose markers span several
// workgroups (one per round of 64 markers).  Every workgroup publishes its
// per-marker results to global scratch, then counts itself done; the one that
// counts last finishes the particle from the published results.
//
// Each XCD has its own L2, so data that crosses workgroups inside a launch
// is stored and loaded with relaxed device-scope atomics, which the compiler
// emits as accesses coherent across the L2s.  Ordering against the counter
// comes from waiting for the stores to complete before counting, and from
// loading only after the counter has been read (workgroup-scope fences keep
// the compiler from moving accesses across).  The counter is reset by the
// finisher, so it reads zero at every launch boundary.  No workgroup ever
// waits for another, and the finishing arithmetic runs in a fixed order, so
// the result does not depend on which workgroup finishes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pub_store(double* p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                       (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double pub_load(const double* p) {
    return __longlong_as_double((long long)__hip_atomic_load(
        reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
// s_waitcnt with vmcnt = 0 (expcnt, lgkmcnt left at their maxima): every
// vector memory access of the thread has completed.
constexpr int kWaitVmem = 0 | (0x7 << 4) | (0xf << 8);

__device__ __forceinline__ bool finish_last(int* counter, int n) {
    __shared__ int s_last;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(kWaitVmem);
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(counter, 1) == n - 1;
    __syncthreads();
    const bool last = s_last != 0;
    if (last && threadIdx.x == 0) *counter = 0;
    __builtin_amdgcn_s_waitcnt(kWaitVmem);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return last;
}

// ---------------------------------------------------------------------------
// Kernel 1: immersed-boundary force and spreading (each workgroup takes a
// range of rounds of 64 markers of one particle).
//
// Each round runs 576 threads, one per (marker, stencil node) pair: each pair
// thread evaluates one MLS weight and pulls the moments of one stencil node;
// the k = 0 thread of each marker then assembles the 3x3 moment matrix and
// interpolant in ascending node order, exactly as the reference formulation
// does, and leaves the marker's contributions c_l phi_k F_l in LDS, and the
// round spreads them.  A particle of one round spreads into its force patch
// directly.  A particle of several rounds spreads each round into a partial
// patch of its own, and the next kernel adds the partial patches cell by
// cell in ascending round order.  Every node thus sums its terms in a fixed
// order: ascending markers within a round, then ascending rounds.
// ---------------------------------------------------------------------------

// Spreading f_lb(x_k) = sum_l c_l phi^l_k F_l.  The contributions of the
// round's markers are in s_con and their stencil anchors in s_anc.  The
// markers are spread in consecutive groups [g0, g1): a group's anchor masks
// (one bit per marker of the round) live on the bounding box of its anchors,
// [gx0, gx0 + gw) x [gy0, gy0 + gh) in unwrapped lattice coordinates, which
// must fit kMaskCells.  The lowest marker of the group covering a node owns
// it and adds the group's terms in ascending marker order onto the value the
// earlier groups left (the first group starts from zero), so each node sums
// the round's terms in ascending marker order, with no float atomics.
constexpr int kMaskCells = 3072;

__device__ __forceinline__ void spread_group(const ChanDev& c, const unsigned long long* gmask,
                                            const double2* s_con, const int2* s_anc, double2* target,
                                            int bx0u, int by0u, int bw, int gx0, int gy0, int gw,
                                            int gh, int lo, int k, bool mine, bool first) {
    if (!mine) return;
    const int2 an = s_anc[lo];
    const int ni = an.x + k % 3 - 1, nj = an.y + k / 3 - 1;
    if (!node_valid(c, ni, nj)) return;
    unsigned long long msk = 0ull;
    for (int db = -1; db <= 1; ++db) {
        const int cy = nj + db - gy0;
        if (cy < 0 || cy >= gh) continue;
        for (int da = -1; da <= 1; ++da) {
            const int cx = ni + da - gx0;
            if (cx < 0 || cx >= gw) continue;
            msk |= gmask[cy * gw + cx];
        }
    }
    if (msk & ((1ull << lo) - 1ull)) return;
    const int cell = (nj - by0u) * bw + (ni - bx0u);
    double2 acc = make_double2(0.0, 0.0);
    if (!first) acc = target[cell];
    while (msk) {
        const int b = __ffsll((long long)msk) - 1;
        msk &= msk - 1ull;
        const int2 a2 = s_anc[b];
        const int k2 = 3 * (nj - a2.y + 1) + (ni - a2.x + 1);
        const double2 v = s_con[b * 9 + k2];
        acc.x += v.x;
        acc.y += v.y;
    }
    target[cell] = acc;
}

__device__ __forceinline__ int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// Work entry of particle-kernel workgroup b.  The first comes with the
// kernel arguments, so that its particle loads need no dependent read.
__device__ __forceinline__ int4 work_of(const StepArgs& a, int b) {
    int4 w;
    if (b == 0) {
        w = a.work0;
    } else {
        w = a.work[b];
    }
    return w;
}

// Two of the particle kernels' 9-wave workgroups share a CU only at six or
// more waves per SIMD (a workgroup places three of its waves on one SIMD;
// measured: at five waves per SIMD one workgroup runs per CU), and only
// while each takes less than 60 KB of LDS (no third one fits beside them
// once a workgroup takes a few KB), hence the register cap here and the
// mask size above.
template <int ST>
__global__ __launch_bounds__(kIbmThreads) __attribute__((amdgpu_waves_per_eu(6)))
void ibm_force_kernel(StepArgs a) {
    __shared__ unsigned long long gmask[kMaskCells];  // anchor masks of the group being spread
    __shared__ double s_w[kIbmThreads], s_ux[kIbmThreads], s_uy[kIbmThreads];
    __shared__ double2 s_con[kIbmThreads];            // c_l phi_k F_l of the round
    __shared__ int2 s_anc[kRound];
    __shared__ double s_mk[kRound][3];                 // marker: x_l, y_l, c_l
    __shared__ double s_ml[kRound][5];                 // MLS row (i00, i01, i02), F_l
    __shared__ int s_grp[5];                           // g1, gx0, gy0, gw, gh
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) atomicAdd((unsigned long long*)a.dstep, 1ull);
    if ((int)blockIdx.x >= a.nwork) return;
    const int4 wk = work_of(a, (int)blockIdx.x);
    const int pid = wk.x, rnd = work_round(wk), nact = work_count(wk);
    PartDev* P = a.parts + pid;
    const ChanDev c = load_chan(a.chan + wk.z);  // issued beside the particle's loads
    // the pair's marker offset too: the work entry locates it
    const int lo = tid / 9, k = tid % 9;
    const bool act = lo < nact;
    const double2 xoff = act ? a.xi[wk.w + lo] : make_double2(0.0, 0.0);
    const int nm = P->nm;
    const int nr = (nm + kRound - 1) / kRound;
    const bool lead = rnd == 0;  // the round-0 workgroup owns the particle's bookkeeping
    const double X0 = P->X[0], X1 = P->X[1], th = P->th;
    const double V0 = P->V[0], V1 = P->V[1], Om = P->Om;
    const double cs = P->cth, sn = P->sth;  // the rotation R(theta)
    // A particle whose state is no longer finite, or far outside any
    // lattice, is flagged and skipped: its stencil anchors would be
    // meaningless and must never index memory.
    const double lim = 1e8;
    if (!(fabs(X0) < lim) || !(fabs(X1) < lim) || !(fabs(th) < lim)) {
        if (lead && tid == 0) {
            P->bw = 0;
            P->bh = 0;
            a.flags[0] = 1;
            atomicMin(&a.flags[1], (int)(*a.dstep - 1));
            if (a.snap) a.snap[pid] = *P;
        }
        return;
    }
    // Force patch: a box that holds every possible stencil node of markers
    // within rb of the centroid (anchors round half up, plus one node).
    int bx0u, by0u, bw, bh;
    stencil_box(X0, X1, P->rb, bx0u, by0u, bw, bh);
    if (bw > c.nx || bh > c.ny || (long long)bw * bh > P->patch_cap) {
        if (lead && tid == 0) {
            atomicOr(&a.flags[2], 1);
            P->bw = 0;
            P->bh = 0;
            if (a.snap) a.snap[pid] = *P;
        }
        return;
    }
    const int ncell = bw * bh;
    double2* patch = a.patch + P->patch_off;
    // nr partial patches of patch_cap cells (nr > 1)
    double2* target = nr == 1 ? patch : a.partial + P->part_off + (long long)rnd * P->patch_cap;
    for (int q = tid; q < kMaskCells; q += blockDim.x) gmask[q] = 0ull;
    if (lead && tid == 0) {
        P->bx0 = wrapc(bx0u, c.nx, c.bcx == 0);
        P->by0 = wrapc(by0u, c.ny, c.bcy == 0);
        P->bw = bw;
        P->bh = bh;
        if (a.snap) a.snap[pid] = *P;
    }
    // (1) one weight and the force-free velocity u* = j*/rho of one node
    if (act) {
        const Marker m = marker_from(xoff, X0, X1, cs, sn);
        double dx, dy;
        int ni, nj;
        double w = 0.0, ux = 0.0, uy = 0.0;
        if (stencil_node(c, m.i0, m.j0, k, m.xl, m.yl, dx, dy, ni, nj)) {
            w = stencil_weight(c, dx, dy);
            double f[9], rho, jx, jy;
            pull_node_f64<ST>(a.fin, c, ni, nj, f);
            moments_f64(f, c, rho, jx, jy);
            ux = jx / rho;
            uy = jy / rho;
        }
        s_w[tid] = w;
        s_ux[tid] = ux;
        s_uy[tid] = uy;
        if (k == 0) {
            s_anc[lo] = make_int2(m.i0, m.j0);
            s_mk[lo][0] = m.xl;
            s_mk[lo][1] = m.yl;
            s_mk[lo][2] = c.spread_unit ? 1.0 : a.ds[wk.w + lo];
            // the rigid-body velocity at the marker
            s_ml[lo][3] = V0 - Om * m.ry;
            s_ml[lo][4] = V1 + Om * m.rx;
        }
    }
    __syncthreads();
    if (tid < kRound) {
        // (2) per marker, all in the first wave (thread lo leads marker
        // lo of the round): the MLS row, U = sum phi u* (k ascending) and
        // F = U_b - U (dt = 1)
        if (tid < nact) {
            const int lo = tid;
            const int2 an = s_anc[lo];
            const double xl = s_mk[lo][0], yl = s_mk[lo][1];
            const double* w = s_w + lo * 9;
            // w, u* and v* are zero at dropped nodes (phase 1), so their terms
            // are signed zeros and need no branch
            const MlsInv iv = mls_inverse(w, an.x, an.y, xl, yl, false);
            double Ux = 0.0, Uy = 0.0;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int ii = an.x + q % 3 - 1, jj = an.y + q / 3 - 1;
                const double dx = (double)ii - xl, dy = (double)jj - yl;
                const double phi = w[q] * (iv.i00 + iv.i01 * dx + iv.i02 * dy);
                Ux += phi * s_ux[lo * 9 + q];
                Uy += phi * s_uy[lo * 9 + q];
            }
            const double Fx = s_ml[lo][3] - Ux, Fy = s_ml[lo][4] - Uy;
            s_ml[lo][0] = iv.i00;
            s_ml[lo][1] = iv.i01;
            s_ml[lo][2] = iv.i02;
            s_ml[lo][3] = Fx;  // the body velocity stored here has been read
            s_ml[lo][4] = Fy;
        }
    } else if (tid < 2 * kRound) {
        // meanwhile the second wave forms the anchor box of the whole round
        // (lane j: marker j of the round); when it fits the masks, they are set here
        // and the round spreads as one group
        const int j = tid - kRound;
        const bool in = j < nact;
        const int2 an = s_anc[in ? j : 0];
        const int x0 = wave_min(in ? an.x : INT_MAX), y0 = wave_min(in ? an.y : INT_MAX);
        const int x1 = wave_max(in ? an.x : INT_MIN), y1 = wave_max(in ? an.y : INT_MIN);
        const bool fits = (long long)(x1 - x0 + 1) * (y1 - y0 + 1) <= kMaskCells;
        if (fits && in) atomicOr(&gmask[(an.y - y0) * (x1 - x0 + 1) + (an.x - x0)], 1ull << j);
        if (j == 0) {
            s_grp[0] = fits ? nact : 0;
            s_grp[1] = x0;
            s_grp[2] = y0;
            s_grp[3] = x1 - x0 + 1;
            s_grp[4] = y1 - y0 + 1;
        }
    } else {
        // and the other waves clear the round's target (the patch, or the
        // round's partial patch), and the lead lists the tiles the patch
        // covers for the lattice pass
        constexpr int kFirst = 2 * kRound;
        for (int q = tid - kFirst; q < ncell; q += blockDim.x - kFirst) target[q] = make_double2(0.0, 0.0);
        if (lead) mark_tiles(a, c, pid, bx0u, by0u, bw, bh, tid - kFirst, blockDim.x - kFirst);
    }
    __syncthreads();
    // (2b) the contribution c_l phi_k F_l of each (marker, node) pair, by the
    // pair's own thread
    if (act) {
        const int2 an = s_anc[lo];
        const int ii = an.x + k % 3 - 1, jj = an.y + k / 3 - 1;
        double2 v = make_double2(0.0, 0.0);
        if (node_valid(c, ii, jj)) {
            const double dx = (double)ii - s_mk[lo][0], dy = (double)jj - s_mk[lo][1];
            const double phi = s_w[tid] * (s_ml[lo][0] + s_ml[lo][1] * dx + s_ml[lo][2] * dy);
            const double cl = s_mk[lo][2];
            v = make_double2(cl * phi * s_ml[lo][3], cl * phi * s_ml[lo][4]);
        }
        s_con[tid] = v;
    }
    __syncthreads();
    // (3) spreading: the whole round as one group, or else in groups of
    // markers whose anchor box fits the masks
    if (s_grp[0] == nact) {
        spread_group(c, gmask, s_con, s_anc, target, bx0u, by0u, bw, s_grp[1], s_grp[2], s_grp[3],
                     s_grp[4], lo, k, act, true);
        return;
    }
    __syncthreads();  // every thread has read s_grp before the groups rewrite it
    for (int g0 = 0; g0 < nact;) {
        if (tid < 64) {
            // the first wave picks the largest group [g0, g0 + n), n halving
            // from all remaining markers, whose anchor box fits
            int n = nact - g0, x0, y0, x1, y1;
            for (;;) {
                const bool in = tid >= g0 && tid < g0 + n;
                const int2 an = s_anc[tid < nact ? tid : 0];
                x0 = wave_min(in ? an.x : INT_MAX);
                y0 = wave_min(in ? an.y : INT_MAX);
                x1 = wave_max(in ? an.x : INT_MIN);
                y1 = wave_max(in ? an.y : INT_MIN);
                if (n == 1 || (long long)(x1 - x0 + 1) * (y1 - y0 + 1) <= kMaskCells) break;
                n = (n + 1) / 2;
            }
            if (tid == 0) {
                s_grp[0] = g0 + n;
                s_grp[1] = x0;
                s_grp[2] = y0;
                s_grp[3] = x1 - x0 + 1;
                s_grp[4] = y1 - y0 + 1;
            }
        }
        __syncthreads();
        const int g1 = s_grp[0], gx0 = s_grp[1], gy0 = s_grp[2], gw = s_grp[3], gh = s_grp[4];
        if (tid >= g0 && tid < g1)
            atomicOr(&gmask[(s_anc[tid].y - gy0) * gw + (s_anc[tid].x - gx0)], 1ull << tid);
        __syncthreads();
        spread_group(c, gmask, s_con, s_anc, target, bx0u, by0u, bw, gx0, gy0, gw, gh, lo, k,
                     act && lo >= g0 && lo < g1, g0 == 0);
        if (g1 == nact) break;
        // another group follows: it may read the cells just written, and the
        // masks are cleared for it
        __syncthreads();
        if (tid >= g0 && tid < g1) gmask[(s_anc[tid].y - gy0) * gw + (s_anc[tid].x - gx0)] = 0ull;
        __syncthreads();
        g0 = g1;
    }
}

// Force patches of particles of several rounds: the sum of the partial
// patches in ascending round order (the first round starts the sum), one
// thread per patch cell; workgroups take (particle, 256-cell chunk) pairs.
__global__ __launch_bounds__(256) void patch_sum_kernel(StepArgs a) {
    if ((int)blockIdx.x >= a.npsum) return;
    const int2 e = a.psum[blockIdx.x];
    const PartDev& P = a.parts[e.x];
    const int q = e.y + (int)threadIdx.x;
    if (q >= P.bw * P.bh) return;  // bw = 0 for a particle the force stage skipped
    const int nr = (P.nm + kRound - 1) / kRound;
    const double2* part = a.partial + P.part_off + q;
    const long long cap = P.patch_cap;
    double2 acc = part[0];
    for (int r = 1; r < nr; ++r) {
        const double2 v = part[r * cap];
        acc.x += v.x;
        acc.y += v.y;
    }
    a.patch[P.patch_off + q] = acc;
}

// ---------------------------------------------------------------------------
// Kernel 2: the lattice pass.
// ---------------------------------------------------------------------------
// FP64 form, reference expression order.  f holds the pulled populations;
// out receives the post-collision populations of node (x, y).
// (flbx, flby): the IB force at the node.
__device__ __forceinline__ void collide_f64_force(const StepArgs& a, const ChanDev& c,
                                                  const ChanDev* cm, int x, int y, double f[9],
                                                  double flbx, double flby,
                                                  const char* __restrict__ fin, double out[9]) {
    walls_f64(c, *cm, x, y, f);
    corners_f64(fin, c, x, y, f);
    double rho, jx, jy;
    moments_f64(f, c, rho, jx, jy);
    const double gx = c.g[0], gy = c.g[1];
    const double ux = (jx + 0.5 * flbx) / rho;
    const double uy = (jy + 0.5 * flby) / rho;
    const double Gx = gx + flbx;
    const double Gy = gy + flby;
    const double usq = ux * ux + uy * uy;
    const double tau = c.tau;
    const double pref = 1.0 - 1.0 / (2.0 * tau);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double exi = (double)ex(i), eyi = (double)ey(i);
        const double eu = exi * ux + eyi * uy;
        const double feq = wd(i) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
        const double Fi = pref * wd(i) * ((3.0 * (exi - ux) + 9.0 * eu * exi) * Gx +
                                          (3.0 * (eyi - uy) + 9.0 * eu * eyi) * Gy);
        out[i] = f[i] - (f[i] - feq) / tau + Fi;
    }
    if (!(rho > 0.0) || !isfinite(rho)) {
        a.flags[0] = 1;
        atomicMin(&a.flags[1], (int)(*a.dstep - 1));
    }
}

// The same with the IB force read from the tile's patch table.
__device__ __forceinline__ void collide_f64(const StepArgs& a, const ChanDev& c,
                                            const ChanDev* cm, int x,
                                            int y, double f[9], const PatchRef* tab, int nlist,
                                            const char* __restrict__ fin, double out[9]) {
    double flbx = 0.0, flby = 0.0;
    if (nlist >= kTileList) patch_force(a, c, x, y, flbx, flby);
    else if (nlist > 0) patch_force_tab(c, tab, nlist, x, y, flbx, flby);
    collide_f64_force(a, c, cm, x, y, f, flbx, flby, fin, out);
}

__device__ __forceinline__ void collide_store_f64(const StepArgs& a, const ChanDev& c,
                                                  const ChanDev* cm, int x,
                                                  int y, double f[9], const PatchRef* tab, int nlist,
                                                  const char* __restrict__ fin, char* __restrict__ fout) {
    double out[9];
    collide_f64(a, c, cm, x, y, f, tab, nlist, fin, out);
#pragma unroll
    for (int i = 0; i < 9; ++i) at<double>(fout, boff<double>(c, i, y, x)) = out[i];
}

// Reduced forms: deviations in FP32.  d holds the pulled deviations; out
// receives the post-collision deviations of node (x, y); (flbx, flby): the
// IB force at the node, rounded to FP32.
template <int ST>
__device__ __forceinline__ void collide_dev_force(const StepArgs& a, const ChanDev& c,
                                                  const ChanDev* cm, int x, int y, float d[9],
                                                  float flbx, float flby,
                                                  const char* __restrict__ fin, float out[9]) {
    walls_dev(c, *cm, x, y, d);
    corners_dev<ST>(fin, c, x, y, d);
    const float drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    const float rho = 1.0f + drho;
    const float gx = c.f_g[0], gy = c.f_g[1];
    const float Gx = gx + flbx, Gy = gy + flby;
    // Written with fused multiply-adds: the FP32 arithmetic is what bounds
    // the F16S pass besides its bytes.  1/rho is the hardware reciprocal
    // (within 1 ulp) refined by one Newton-Raphson step, r + r (1 - rho r);
    // the unrefined reciprocal alone biases u enough to double the phase
    // error of a tumbling particle over 50 000 steps.
    const float jx = fmaf(0.5f, Gx, ((d[1] - d[3]) + (d[5] - d[6])) + (d[8] - d[7]));
    const float jy = fmaf(0.5f, Gy, ((d[2] - d[4]) + (d[5] + d[6])) - (d[7] + d[8]));
    const float r0 = __builtin_amdgcn_rcpf(rho);
    const float irho = fmaf(r0, fmaf(-rho, r0, 1.0f), r0);
    const float ux = jx * irho, uy = jy * irho;
    const float usq = fmaf(ux, ux, uy * uy);
    const float om = c.f_omega, pref = c.f_pref;
    // Equilibrium deviation and Guo term by pairs of opposite directions
    // (e_j = -e_i): e.u and e.G change sign, their product and squares do
    // not, so with
    //   C = drho + rho (4.5 (e.u)^2 - 1.5 u.u),  D = 3 rho e.u,
    //   A = 9 (e.u)(e.G) - 3 u.G,                B = 3 e.G,
    // deq_i = w (C + D), deq_j = w (C - D), F_i = pref w (A + B) and
    // F_j = pref w (A - B), where deq = w (drho + rho (3 e.u + 4.5 (e.u)^2
    // - 1.5 u.u)) and F = pref w ((3 (e - u) + 9 (e.u) e) . G) (Eqs. (4), (5)).
    // Each population leaves as d + (deq - d) om + F.
    const float uG = fmaf(ux, Gx, uy * Gy);
    const float c0 = 1.5f * usq;
    const float r3 = 3.0f * rho, m3uG = -3.0f * uG;
    out[0] = fmaf(pref * wf(0), m3uG, fmaf(fmaf(wf(0), fmaf(-rho, c0, drho), -d[0]), om, d[0]));
    auto pair = [&](int i, int j, float eu, float eG) {
        const float C = fmaf(rho, fmaf(4.5f * eu, eu, -c0), drho);
        const float D = r3 * eu;
        const float A = fmaf(9.0f * eu, eG, m3uG);
        const float B = 3.0f * eG;
        const float w = wf(i), pw = pref * wf(i);
        out[i] = fmaf(pw, A + B, fmaf(fmaf(w, C + D, -d[i]), om, d[i]));
        out[j] = fmaf(pw, A - B, fmaf(fmaf(w, C - D, -d[j]), om, d[j]));
    };
    pair(1, 3, ux, Gx);
    pair(2, 4, uy, Gy);
    pair(5, 7, ux + uy, Gx + Gy);
    pair(6, 8, uy - ux, Gy - Gx);
    if (!(rho > 0.0f) || !isfinite(rho)) {
        a.flags[0] = 1;
        atomicMin(&a.flags[1], (int)(*a.dstep - 1));
    }
}

// The same with the IB force read from the tile's patch table.
template <int ST>
__device__ __forceinline__ void collide_dev(const StepArgs& a, const ChanDev& c,
                                            const ChanDev* cm, int x,
                                            int y, float d[9], const PatchRef* tab, int nlist,
                                            const char* __restrict__ fin, float out[9]) {
    float flbx = 0.0f, flby = 0.0f;
    if (nlist > 0) {
        double fx, fy;
        if (nlist >= kTileList) patch_force(a, c, x, y, fx, fy);
        else patch_force_tab(c, tab, nlist, x, y, fx, fy);
        flbx = (float)fx;
        flby = (float)fy;
    }
    collide_dev_force<ST>(a, c, cm, x, y, d, flbx, flby, fin, out);
}

template <int ST>
__device__ __forceinline__ void collide_store_dev(const StepArgs& a, const ChanDev& c,
                                                  const ChanDev* cm, int x,
                                                  int y, float d[9], const PatchRef* tab, int nlist,
                                                  const char* __restrict__ fin, char* __restrict__ fout) {
    using T = typename Sto<ST>::T;
    float out[9];
    collide_dev<ST>(a, c, cm, x, y, d, tab, nlist, fin, out);
#pragma unroll
    for (int i = 0; i < 9; ++i) store_dev<ST>(&at<T>(fout, boff<T>(c, i, y, x)), 0, i, out[i], c);
}

// One tile of the lattice pass: lane (lx, ly) of a TW-wide workgroup handles
// NPT consecutive rows of column x0 + lx.
template <int ST, int TW, int NPT>
__device__ __forceinline__ void lattice_tile(const StepArgs& a, int t, int lx, int ly) {
    using T = typename Sto<ST>::T;
    const int* tl_cur = a.tlist + (long long)a.parity * a.ntiles * kTileList;
    int* tl_next = a.tlist + (long long)(1 - a.parity) * a.ntiles * kTileList;
    const TileDev* tp = a.tiles + t;
    const int tx0 = uni(tp->x0), ty0 = uni(tp->y0);
    // the descriptor in scalar registers, and in memory for the wall
    // velocities (needed only in wall rows)
    const ChanDev* cm = a.chan + uni(tp->chan);
    const ChanDev c = load_chan(cm);
    // the channel's blocks in the two buffers; accesses below add 32-bit
    // byte offsets
    const char* __restrict__ fin = (const char*)a.fin + c.off * (long long)sizeof(T);
    char* __restrict__ fout = (char*)a.fout + c.off * (long long)sizeof(T);
    const int x = tx0 + lx;
    const int xl = x < c.nx ? x : c.nx - 1;  // loads of lanes past the edge stay in bounds
    // Particles whose force patches overlap this tile, appended by the
    // particle kernel of this step; sorted ascending and deduplicated so
    // overlapping patches add in a fixed order.  The other half of the
    // list store is reset for the next step.
    const int* e = tl_cur + (long long)t * kTileList;
    const int cnt = uni(e[0]);
    if (threadIdx.x == 0) tl_next[(long long)t * kTileList] = 0;
    int list[kTileList - 1] = {};
    int nlist = 0;
    if (cnt > kTileList - 1) {
        nlist = kTileList;  // more patches than slots: scan the channel's particles
    } else {
        for (int j = 0; j < cnt; ++j) list_insert(list, nlist, uni(e[1 + j]));
    }
    // The listed particles' patch references, formed once per tile in LDS
    // (nlist is the same for the whole workgroup, so are the barriers).
    __shared__ PatchRef s_tab[kTileList - 1];
    if (nlist > 0 && nlist < kTileList) {
        __syncthreads();  // a persistent workgroup's previous tile is done with the table
#pragma unroll
        for (int j = 0; j < kTileList - 1; ++j)
            if (j < nlist && (int)threadIdx.x == j) s_tab[j] = patch_ref(a, a.parts[list[j]]);
        __syncthreads();
    }
    // all pulls of the thread's rows first, then collide and store
    if constexpr (ST == ST_F64) {
        double f[NPT][9];
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            const int y = ty0 + ly * NPT + r;
            const int yl = y < c.ny ? y : c.ny - 1;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                int xs, ys;
                pull_src(c, i, xl, yl, xs, ys);
                f[r][i] = at<double>(fin, boff<double>(c, i, ys, xs));
            }
        }
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            const int y = ty0 + ly * NPT + r;
            if (x < c.nx && y < c.ny) collide_store_f64(a, c, cm, x, y, f[r], s_tab, nlist, fin, fout);
        }
    } else {
        float d[NPT][9];
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            const int y = ty0 + ly * NPT + r;
            const int yl = y < c.ny ? y : c.ny - 1;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                int xs, ys;
                pull_src(c, i, xl, yl, xs, ys);
                d[r][i] = load_dev<ST>(&at<T>(fin, boff<T>(c, i, ys, xs)), 0, i, c);
            }
        }
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            const int y = ty0 + ly * NPT + r;
            if (x < c.nx && y < c.ny) collide_store_dev<ST>(a, c, cm, x, y, d[r], s_tab, nlist, fin, fout);
        }
    }
}

// ---------------------------------------------------------------------------
// Vector form of the lattice pass: lane l of a wave takes NV consecutive
// nodes of a row, [x0 + l NV, x0 + (l + 1) NV), so each population plane of
// a row arrives in one aligned load of NV elements (at most 16 bytes) and
// leaves in one store, instead of one access per node.  The pull shift
// along x is taken from the same chunk: a population streaming in from the
// left (e_x = +1) needs the element before the chunk, one streaming in from
// the right (e_x = -1) the element after the node's last one, each loaded on
// its own with the periodic wrap or wall clamp of the per-node pull.  A tile
// is 64 NV nodes wide and 4 NPT rows high (one wave per NPT rows).  Per
// node the arithmetic is that of the per-node form, so the results are bit
// for bit the same.
// ---------------------------------------------------------------------------
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
template <int B> struct VecOf;
template <> struct VecOf<2> { using type = unsigned short; };
template <> struct VecOf<4> { using type = unsigned; };
template <> struct VecOf<8> { using type = u32x2; };
template <> struct VecOf<16> { using type = u32x4; };

template <typename T, int NV>
__device__ __forceinline__ void vload(const char* base, unsigned off, T (&out)[NV]) {
    using V = typename VecOf<NV * (int)sizeof(T)>::type;
    const V v = *(const V*)(base + off);
    __builtin_memcpy(out, &v, sizeof(V));
}

// NT: a nontemporal store, which does not keep the line in the caches.  It
// pays where the two population buffers exceed the 256 MB Infinity Cache
// (the next step's reads miss it anyway) and costs where they fit.
template <typename T, int NV, bool NT>
__device__ __forceinline__ void vstore(char* base, unsigned off, const T (&in)[NV]) {
    using V = typename VecOf<NV * (int)sizeof(T)>::type;
    V v;
    __builtin_memcpy(&v, in, sizeof(V));
    if constexpr (NT) __builtin_nontemporal_store(v, (V*)(base + off));
    else *(V*)(base + off) = v;
}

// The NV streamed values of population i for the nodes [xb, xb + NV) of row
// y (xb < nx, a multiple of NV): source row y - e_y (wrapped or clamped),
// columns x - e_x.  k: position of the channel's last node nx - 1 in the
// chunk, or NV - 1 when the chunk ends before it.
template <typename T, int NV>
__device__ __forceinline__ void pull_chunk(const char* fin, const ChanDev& c, int i, int xb, int y, int k,
                                           T (&v)[NV]) {
    const int ys = pull_coord(y - ey(i), y, c.ny, c.bcy == 0);
    T A[NV];
    vload<T, NV>(fin, boff<T>(c, i, ys, xb), A);
    if (ex(i) == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = A[j];
    } else if (ex(i) > 0) {
        // node xb + j takes column xb + j - 1: the element before the chunk first
        const T B = at<T>(fin, boff<T>(c, i, ys, pull_coord(xb - 1, xb, c.nx, c.bcx == 0)));
        v[0] = B;
#pragma unroll
        for (int j = 1; j < NV; ++j) v[j] = A[j - 1];
    } else {
        // node xb + j takes column xb + j + 1; past the chunk, or past the
        // channel's last node, one element of its own
        const int xk = xb + k;
        const T B = at<T>(fin, boff<T>(c, i, ys, pull_coord(xk + 1, xk, c.nx, c.bcx == 0)));
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = j < k ? A[j + 1 < NV ? j + 1 : NV - 1] : B;
    }
}

template <int ST, int NV, int NPT, bool NT>
__device__ __forceinline__ void lattice_vtile(const StepArgs& a, int t, int lane, int wv) {
    using T = typename Sto<ST>::T;
    const int* tl_cur = a.tlist + (long long)a.parity * a.ntiles * kTileList;
    int* tl_next = a.tlist + (long long)(1 - a.parity) * a.ntiles * kTileList;
    const TileDev* tp = a.tiles + t;
    const int tx0 = uni(tp->x0), ty0 = uni(tp->y0);
    const ChanDev* cm = a.chan + uni(tp->chan);
    const ChanDev c = load_chan(cm);
    const char* __restrict__ fin = (const char*)a.fin + c.off * (long long)sizeof(T);
    char* __restrict__ fout = (char*)a.fout + c.off * (long long)sizeof(T);
    const int xb = tx0 + lane * NV;
    const bool xin = xb < c.nx;
    const int xbl = xin ? xb : 0;  // lanes past the channel's edge load column 0 and store nothing
    const int k = min(c.nx - 1 - xbl, NV - 1);
    // the tile's particle list, as in the per-node form
    const int* e = tl_cur + (long long)t * kTileList;
    const int cnt = uni(e[0]);
    if (threadIdx.x == 0) tl_next[(long long)t * kTileList] = 0;
    int list[kTileList - 1] = {};
    int nlist = 0;
    if (cnt > kTileList - 1) {
        nlist = kTileList;
    } else {
        for (int j = 0; j < cnt; ++j) list_insert(list, nlist, uni(e[1 + j]));
    }
    __shared__ PatchRef s_tab[kTileList - 1];
    if (nlist > 0 && nlist < kTileList) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kTileList - 1; ++j)
            if (j < nlist && (int)threadIdx.x == j) s_tab[j] = patch_ref(a, a.parts[list[j]]);
        __syncthreads();
    }
    // With up to four nodes per lane, the IB force of the lane's nodes is
    // loaded first, every patch value requested at once (node by node, each
    // node's patch loads would wait for the pulls and then for each other);
    // with eight, that costs more registers than it saves.
    constexpr bool kEarly = NV <= 4;
    using FT = typename std::conditional<ST == ST_F64, double, float>::type;
    FT gfx[NPT][NV], gfy[NPT][NV];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        const int y = ty0 + wv * NPT + r;
        double fx[NV], fy[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) fx[j] = fy[j] = 0.0;
        if (kEarly && nlist > 0 && xin && y < c.ny) {
            if (nlist >= kTileList) {
#pragma unroll
                for (int j = 0; j < NV; ++j)
                    if (xbl + j < c.nx) patch_force(a, c, xbl + j, y, fx[j], fy[j]);
            } else {
                patch_force_row<NV>(c, s_tab, nlist, xbl, y, fx, fy);
            }
        }
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            gfx[r][j] = (FT)fx[j];
            gfy[r][j] = (FT)fy[j];
        }
    }
    T raw[NPT][9][NV];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        const int y = ty0 + wv * NPT + r;
        const int yl = y < c.ny ? y : c.ny - 1;
#pragma unroll
        for (int i = 0; i < 9; ++i) pull_chunk<T, NV>(fin, c, i, xbl, yl, k, raw[r][i]);
    }
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        const int y = ty0 + wv * NPT + r;
        if (!xin || y >= c.ny) continue;
        T res[9][NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int x = xbl + j;
            if constexpr (ST == ST_F64) {
                double f[9], o[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = raw[r][i][j];
                if (x < c.nx) {
                    if constexpr (kEarly) collide_f64_force(a, c, cm, x, y, f, gfx[r][j], gfy[r][j], fin, o);
                    else collide_f64(a, c, cm, x, y, f, s_tab, nlist, fin, o);
                }
                else
#pragma unroll
                    for (int i = 0; i < 9; ++i) o[i] = 0.0;
#pragma unroll
                for (int i = 0; i < 9; ++i) res[i][j] = o[i];
            } else {
                float d[9], o[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) d[i] = load_dev<ST>(&raw[r][i][j], 0, i, c);
                if (x < c.nx) {
                    if constexpr (kEarly) collide_dev_force<ST>(a, c, cm, x, y, d, gfx[r][j], gfy[r][j], fin, o);
                    else collide_dev<ST>(a, c, cm, x, y, d, s_tab, nlist, fin, o);
                }
                else
#pragma unroll
                    for (int i = 0; i < 9; ++i) o[i] = 0.0f;
#pragma unroll
                for (int i = 0; i < 9; ++i) store_dev<ST>(&res[i][j], 0, i, o[i], c);
            }
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) vstore<T, NV, NT>(fout, boff<T>(c, i, y, xbl), res[i]);
    }
}

// Waves per SIMD the one-row FP32 vector pass is held to (its occupancy
// before the IB force of its nodes was loaded ahead of the pulls); the
// other shapes are left to the compiler.
template <int ST, int NPT>
constexpr int kVecWaves = NPT == 1 && ST == ST_F32 ? 5 : 1;

template <int ST, int NV, int NPT, bool NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kVecWaves<ST, NPT>)))
void lattice_vkernel(StepArgs a) {
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
    const int stride = a.persistent ? (int)gridDim.x : a.ntiles;
    int t0 = blockIdx.x;
    if (a.xcd_remap && !a.persistent) {
        const int per = (int)gridDim.x / 8;
        t0 = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    }
    for (int t = t0; t < a.ntiles; t += stride) lattice_vtile<ST, NV, NPT, NT>(a, t, lane, wv);
}

template <int ST, int TW, int NPT>
__global__ __launch_bounds__(256) void lattice_kernel(StepArgs a) {
    const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
    const int stride = a.persistent ? (int)gridDim.x : a.ntiles;
    // Workgroups are dispatched round-robin over the 8 XCDs.  With the remap
    // (one workgroup per tile, grid rounded up to a multiple of 8) XCD x
    // takes the contiguous tile block [x * per, (x + 1) * per).
    int t0 = blockIdx.x;
    if (a.xcd_remap && !a.persistent) {
        const int per = (int)gridDim.x / 8;
        t0 = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    }
    for (int t = t0; t < a.ntiles; t += stride) lattice_tile<ST, TW, NPT>(a, t, lx, ly);
}

// ---------------------------------------------------------------------------
// Kernel 3: surface stress, force, moment and BDF2 (one workgroup per round
// of 64 markers of a particle).  Pair threads (marker, probe-stencil node)
// evaluate one weight and the corrected fields of one node; the k = 0 thread
// of each marker builds the probe's MLS value and gradient weights and the
// marker's traction.
// ---------------------------------------------------------------------------
// Probe geometry of one (marker, probe-stencil node) pair: the marker's
// offset and normal rotated by theta, its probe point x_l + dn n_l, the
// probe stencil anchor and the pair's node (false: dropped beyond a wall).
struct ProbePair {
    double rx, ry, nxl, nyl, xp, yp, dx, dy;
    int i0, j0, ni, nj;
    bool node;
};

__device__ __forceinline__ ProbePair probe_pair(const ChanDev& c, double2 x, double2 nb, int k, double X0,
                                                double X1, double cs, double sn, double dn) {
    ProbePair g;
    g.rx = cs * x.x - sn * x.y;
    g.ry = sn * x.x + cs * x.y;
    g.nxl = cs * nb.x - sn * nb.y;
    g.nyl = sn * nb.x + cs * nb.y;
    g.xp = X0 + g.rx + dn * g.nxl;
    g.yp = X1 + g.ry + dn * g.nyl;
    g.i0 = (int)floor(g.xp + 0.5);
    g.j0 = (int)floor(g.yp + 0.5);
    g.node = stencil_node(c, g.i0, g.j0, k, g.xp, g.yp, g.dx, g.dy, g.ni, g.nj);
    return g;
}

// The pair's weight and force-corrected fields at its node (rho = 1, u = 0
// and weight 0 at a dropped node), into the round's LDS rows; the k = 0
// pair of a marker also stores the marker's geometry.
template <int ST>
__device__ __forceinline__ void probe_fields(const StepArgs& a, const ChanDev& c, const ProbePair& g,
                                             const typename Sto<ST>::T (&raw)[9], const int* s_nb,
                                             int nnb, int p, int lo, int k, double ds, double* s_w,
                                             double* s_r, double* s_ux, double* s_uy,
                                             double (*s_pg)[7], int2* s_pa) {
    double w = 0.0, rho = 1.0, ux = 0.0, uy = 0.0;
    if (g.node) {
        w = stencil_weight(c, g.dx, g.dy);
        double f[9], jx, jy, fx, fy;
        pull_finish_f64<ST>(a.fin, c, g.ni, g.nj, raw, f);
        moments_f64(f, c, rho, jx, jy);
        if (nnb <= kMaxNeighbours) patch_force_list(a, c, s_nb, nnb, g.ni, g.nj, fx, fy);
        else patch_force(a, c, g.ni, g.nj, fx, fy);
        ux = (jx + 0.5 * fx) / rho;
        uy = (jy + 0.5 * fy) / rho;
    }
    s_w[p] = w;
    s_r[p] = rho;
    s_ux[p] = ux;
    s_uy[p] = uy;
    if (k == 0) {
        s_pg[lo][0] = g.rx;
        s_pg[lo][1] = g.ry;
        s_pg[lo][2] = g.nxl;
        s_pg[lo][3] = g.nyl;
        s_pg[lo][4] = g.xp;
        s_pg[lo][5] = g.yp;
        s_pg[lo][6] = ds;
        s_pa[lo] = make_int2(g.i0, g.j0);
    }
}

// TPB threads per round: 576 (one pair per thread, whose loads leave before
// the neighbour list is built), or 256 (the combined launch with the
// vector lattice pass: each thread takes pairs tid, tid + 256, tid + 512 in
// turn).  The arithmetic of each pair and marker, and every sum, is the
// same in both.
template <int ST, int TPB = kIbmThreads>
__device__ __forceinline__ void traction_body(const StepArgs& a, const int4 wk) {
    __shared__ double s_w[kIbmThreads], s_r[kIbmThreads], s_ux[kIbmThreads], s_uy[kIbmThreads];
    __shared__ double s_t[3][kRound];
    __shared__ double s_pg[kRound][7];  // marker: r_x, r_y, n_x, n_y, probe x, probe y, S
    __shared__ int2 s_pa[kRound];       // probe stencil anchor
    __shared__ double sums[3];
    constexpr bool kOnePair = TPB == kIbmThreads;
    const int tid = threadIdx.x;
    const int b = wk.x, rnd = work_round(wk), nact = work_count(wk);
    PartDev* P = a.parts + b;
    const ChanDev c = load_chan(a.chan + wk.z);  // issued beside the particle's loads
    // and the pair's marker offset and normal, located by the work entry
    const int lo = tid / 9, k = tid % 9;
    const bool mk = kOnePair && lo < nact;
    double2 xoff = make_double2(0.0, 0.0), noff = xoff;
    if (mk) {
        xoff = a.xi[wk.w + lo];
        noff = a.nrm[wk.w + lo];
    }
    const int nm = P->nm, mb = P->mbeg;
    const double X0 = P->X[0], X1 = P->X[1], th = P->th, Om = P->Om;
    const double acc0 = P->acc[0], acc1 = P->acc[1], alp = P->alp;
    const double nu = c.nu, dn = c.dn;
    const bool skip = P->bw <= 0;  // flagged by the force stage
    // One workgroup per round of 64 markers; a particle of several rounds
    // publishes the per-marker terms and its last workgroup sums them.  A
    // skipped particle is finished by its round-0 workgroup alone.
    if (skip && rnd > 0) return;
    const int nr = (nm + kRound - 1) / kRound;
    const bool multi = nr > 1 && !skip;
    const double cs = skip ? 1.0 : P->cth, sn = skip ? 0.0 : P->sth;
    const bool act = !skip && mk;
    // (0) with one pair per thread, the probe stencil node of the pair and
    // its stored populations, loaded before the neighbour list is known
    // (only the patch forces need it), so the two latencies overlap
    ProbePair g0 = {};
    typename Sto<ST>::T raw[9];
    if (act) {
        g0 = probe_pair(c, xoff, noff, k, X0, X1, cs, sn, dn);
        if (g0.node) pull_load<ST>(a.fin, c, g0.ni, g0.nj, raw);
    }
    // Particles of the channel whose force patches can reach this particle's
    // probe stencils (its own box grown by the probe reach), ascending.
    __shared__ int s_nb[kMaxNeighbours];
    __shared__ int s_nnb;
    int nnb;
    if (c.p_end - c.p_begin == 1) {
        // the channel's only particle: the list is the particle itself
        // unless the force stage skipped it (its grown box always overlaps
        // its own box), so no list is built and no barrier is needed; every
        // thread writes the same entry and reads its own write
        nnb = skip ? 0 : 1;
        s_nb[0] = b;
    } else {
        if (tid < 64) {
            // lane j tests particle p_begin + j of each 64-particle chunk; the
            // ballot keeps the list in ascending order
            int n = 0;
            const int grow = (int)ceil(dn) + 2;
            for (int q0 = c.p_begin; q0 < c.p_end; q0 += 64) {
                const int q = q0 + tid;
                bool hit = false;
                if (q < c.p_end) {
                    const PartDev& Q = a.parts[q];
                    hit = Q.bw > 0 && boxes_overlap(c, P->bx0 - grow, P->by0 - grow, P->bw + 2 * grow,
                                                    P->bh + 2 * grow, Q.bx0, Q.by0, Q.bw, Q.bh);
                }
                const unsigned long long bal = __ballot(hit);
                if (hit) {
                    const int pos = n + __popcll(bal & ((1ull << tid) - 1ull));
                    if (pos < kMaxNeighbours) s_nb[pos] = q;
                }
                n += __popcll(bal);
            }
            if (tid == 0) s_nnb = n;
        }
        __syncthreads();
        nnb = s_nnb;
    }

    if (!skip) {
        if constexpr (kOnePair) {
            if (act)
                probe_fields<ST>(a, c, g0, raw, s_nb, nnb, tid, lo, k, k == 0 ? a.ds[wk.w + lo] : 0.0, s_w,
                                 s_r, s_ux, s_uy, s_pg, s_pa);
        } else {
            for (int p = tid; p < kIbmThreads; p += TPB) {
                const int lp = p / 9, kp = p % 9;
                if (lp >= nact) continue;
                const ProbePair g = probe_pair(c, a.xi[wk.w + lp], a.nrm[wk.w + lp], kp, X0, X1, cs, sn, dn);
                typename Sto<ST>::T rp[9];
                if (g.node) pull_load<ST>(a.fin, c, g.ni, g.nj, rp);
                probe_fields<ST>(a, c, g, rp, s_nb, nnb, p, lp, kp, kp == 0 ? a.ds[wk.w + lp] : 0.0, s_w,
                                 s_r, s_ux, s_uy, s_pg, s_pa);
            }
        }
        __syncthreads();
        if (tid < nact) {
            // marker lm of the round, led from the first wave
            const int lm = tid, lo = lm;
            const double rx = s_pg[lo][0], ry = s_pg[lo][1];
            const double nxl = s_pg[lo][2], nyl = s_pg[lo][3];
            const double xp = s_pg[lo][4], yp = s_pg[lo][5];
            const int i0 = s_pa[lo].x, j0 = s_pa[lo].y;
            const double* w = s_w + lo * 9;
            // w is zero at dropped nodes (phase 1, with rho = 1 and u = 0
            // there), so their terms are signed zeros and need no branch
            const MlsInv iv = mls_inverse(w, i0, j0, xp, yp, true);
            double rP = 0.0, dudx = 0.0, dudy = 0.0, dvdx = 0.0, dvdy = 0.0;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int ii = i0 + q % 3 - 1, jj = j0 + q / 3 - 1;
                const double dx = (double)ii - xp, dy = (double)jj - yp;
                const double phi = w[q] * (iv.i00 + iv.i01 * dx + iv.i02 * dy);
                const double dpx = w[q] * (iv.i01 + iv.i11 * dx + iv.i12 * dy);
                const double dpy = w[q] * (iv.i02 + iv.i12 * dx + iv.i22 * dy);
                const double rq = s_r[lo * 9 + q], uq = s_ux[lo * 9 + q], vq = s_uy[lo * 9 + q];
                rP += phi * rq;
                dudx += dpx * uq;
                dudy += dpy * uq;
                dvdx += dpx * vq;
                dvdy += dpy * vq;
            }
            const double pP = (rP - 1.0) / 3.0;
            const double txx = nu * (2.0 * dudx);
            const double txy = nu * (dudy + dvdx);
            const double tyy = nu * (2.0 * dvdy);
            const double alx = acc0 - alp * ry - Om * Om * rx;
            const double aly = acc1 + alp * rx - Om * Om * ry;
            const double pl = pP + dn * (alx * nxl + aly * nyl);
            const double tx = txx * nxl + txy * nyl - pl * nxl;
            const double ty = txy * nxl + tyy * nyl - pl * nyl;
            const double S = s_pg[lo][6];
            const double t0 = tx * S, t1 = ty * S, t2 = (rx * ty - ry * tx) * S;
            if (multi) {
                double* o = a.mscr + (long long)(wk.w + lm) * 4;
                pub_store(o, t0);
                pub_store(o + 1, t1);
                pub_store(o + 2, t2);
            } else {
                s_t[0][lm] = t0;
                s_t[1][lm] = t1;
                s_t[2][lm] = t2;
            }
        }
        __syncthreads();
    }
    if (multi && !finish_last(a.pcount + b, nr)) return;
    // Force and moment: sums over the markers in ascending order (thread
    // tid < 3 sums component tid).  Published terms are staged through LDS
    // 192 markers at a time, every thread loading one term.
    double fsum = 0.0;
    if (multi) {
        constexpr int kStage = TPB / 3;
        for (int base = 0; base < nm; base += kStage) {
            const int l = base + tid / 3;
            s_w[tid] = l < nm ? pub_load(a.mscr + (long long)(mb + l) * 4 + tid % 3) : 0.0;
            __syncthreads();
            if (tid < 3) {
                const int n = nm - base < kStage ? nm - base : kStage;
                fsum = ordered_sum(fsum, s_w + tid, n, 3);
            }
            __syncthreads();
        }
    } else if (!skip && tid < 3) {
        fsum = ordered_sum(fsum, s_t[tid], nm, 1);
    }
    if (tid < 3) sums[tid] = fsum;
    __syncthreads();
    if (tid != 0) return;
    const double Fx = sums[0], Fy = sums[1], Mz = sums[2];
    const double buoy = 1.0 - 1.0 / P->ratio;
    const double ax = Fx / P->m + buoy * c.grav[0];
    const double ay = Fy / P->m + buoy * c.grav[1];
    const double al = Mz / P->I;
    const double vx = 2.0 / 3.0 * (2.0 * P->V[0] - 0.5 * P->Vm[0] + ax);
    const double vy = 2.0 / 3.0 * (2.0 * P->V[1] - 0.5 * P->Vm[1] + ay);
    const double om = 2.0 / 3.0 * (2.0 * P->Om - 0.5 * P->Omm + al);
    const double nX0 = 2.0 / 3.0 * (2.0 * X0 - 0.5 * P->Xm[0] + vx);
    const double nX1 = 2.0 / 3.0 * (2.0 * X1 - 0.5 * P->Xm[1] + vy);
    const double nth = 2.0 / 3.0 * (2.0 * th - 0.5 * P->thm + om);
    P->Vm[0] = P->V[0];
    P->Vm[1] = P->V[1];
    P->Omm = P->Om;
    P->Xm[0] = X0;
    P->Xm[1] = X1;
    P->thm = th;
    P->V[0] = vx;
    P->V[1] = vy;
    P->Om = om;
    P->X[0] = nX0;
    P->X[1] = nX1;
    P->th = nth;
    P->acc[0] = ax;
    P->acc[1] = ay;
    P->alp = al;
    P->F[0] = Fx;
    P->F[1] = Fy;
    P->M = Mz;
    const long long step = *a.dstep - 1;
    double* r = a.rec + ((step % kRecSlots) * a.nparts + b) * 10;
    r[0] = nX0;
    r[1] = nX1;
    r[2] = nth;
    r[3] = vx;
    r[4] = vy;
    r[5] = om;
    r[6] = Fx;
    r[7] = Fy;
    r[8] = Mz;
    r[9] = (double)P->chan;
    // cos and sin of the new angle for the next step's kinematics, last so
    // that the stores above are already on their way
    double snt, cst;
    sincos(nth, &snt, &cst);
    P->cth = cst;
    P->sth = snt;
    const bool fin = isfinite(vx) && isfinite(vy) && isfinite(om) && isfinite(nX0) &&
                     isfinite(nX1) && isfinite(nth);
    if (!fin || skip) {
        a.flags[0] = 1;
        atomicMin(&a.flags[1], (int)step);
    }
}

// PAIR: the register cap that lets two workgroups share a CU, for launches
// of more rounds than CUs; it spills a few registers, which costs a single
// round about a microsecond, so smaller launches take the plain kernel.
template <int ST, bool PAIR>
__global__ __launch_bounds__(kIbmThreads) __attribute__((amdgpu_waves_per_eu(PAIR ? 6 : 1)))
void traction_kernel(StepArgs a) {
    if ((int)blockIdx.x < a.nwork) {
        const int4 wk = work_of(a, (int)blockIdx.x);
        traction_body<ST>(a, wk);
    }
}

// The surface stress of step n reads the populations entering the step and
// the force patches of the step, the lattice pass reads the same and writes
// only the populations leaving it, so the two share one launch: workgroups
// [0, tb) take the particles' marker rounds (tb = the number of rounds
// rounded up to a multiple of 8, so that lattice workgroup j lands on XCD
// j mod 8 as in the lattice kernel) and the rest take lattice tiles of
// 64 x 9*NPT nodes.  The particle workgroups are dispatched first and run
// alongside the lattice tiles.
template <int ST, int NPT>
__global__ __launch_bounds__(kIbmThreads) void lattice_traction_kernel(StepArgs a, int tb) {
    const int j = (int)blockIdx.x - tb;
    if (j < 0) {
        if ((int)blockIdx.x < a.nwork) {
            const int4 wk = work_of(a, (int)blockIdx.x);
            traction_body<ST>(a, wk);
        }
        return;
    }
    int t = j;
    if (a.xcd_remap) {
        const int per = ((int)gridDim.x - tb) / 8;
        t = (j % 8) * per + j / 8;
    }
    if (t < a.ntiles) lattice_tile<ST, 64, NPT>(a, t, (int)threadIdx.x % 64, (int)threadIdx.x / 64);
}

// The same launch with the vector form of the lattice pass, in 256-thread
// workgroups: the lattice tiles are those of lattice_vkernel (64 NV x 4
// nodes), and a particle round runs its 576 (marker, node) pairs on 256
// threads.  The reduced forms are held to 128 VGPRs (four workgroups per
// CU beside the surface stress's 24 KB of LDS): at 96 VGPRs, the occupancy
// of lattice_vkernel in FP32, the surface stress spills 172 bytes per lane,
// and that scratch traffic costs the lattice pass more than the fifth
// workgroup gains (ensemble step 387 -> 374 us at 128).
template <int ST, int NV, bool NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ST == ST_F64 ? 1 : 4)))
void lattice_traction_vkernel(StepArgs a, int tb) {
    const int j = (int)blockIdx.x - tb;
    if (j < 0) {
        if ((int)blockIdx.x < a.nwork) {
            const int4 wk = work_of(a, (int)blockIdx.x);
            traction_body<ST, 256>(a, wk);
        }
        return;
    }
    int t = j;
    if (a.xcd_remap) {
        const int per = ((int)gridDim.x - tb) / 8;
        t = (j % 8) * per + j / 8;
    }
    if (t < a.ntiles) lattice_vtile<ST, NV, 1, NT>(a, t, (int)threadIdx.x % 64, (int)threadIdx.x / 64);
}

// ---------------------------------------------------------------------------
// Initial state, field extraction, population upload.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void initial_velocity(const ChanDev& c, int init, int y, double& ux,
                                                 double& uy) {
    ux = 0.0;
    uy = 0.0;
    if (init == 1) {
        double lo = c.uw[2][0], hi = c.uw[3][0];
        ux = lo + (hi - lo) * (double)y / (double)(c.ny - 1);
    }
}

// Writes the post-collision pre-image whose pull gives f^eq(1, u0(x)) at every
// node: population i at node x holds f^eq_i(1, u0(x + e_i)).
template <int ST>
__global__ void init_kernel(StepArgs a, int chan, int init) {
    const ChanDev c = a.chan[chan];
    const long long n = (long long)c.nx * c.ny;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(t % c.nx), y = (int)(t / c.nx);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int ys = y + ey(i);
            if (c.bcy == 0) ys = ys < 0 ? ys + c.ny : (ys >= c.ny ? ys - c.ny : ys);
            else if (ys < 0 || ys >= c.ny) ys = y;
            double ux, uy;
            initial_velocity(c, init, ys, ux, uy);
            const double exi = (double)ex(i), eyi = (double)ey(i);
            const double usq = ux * ux + uy * uy;
            const double eu = exi * ux + eyi * uy;
            const long long k = pidx(c, i, y, x);
            if constexpr (ST == ST_F64) {
                const double rho = 1.0;
                ((double*)a.fout)[k] = wd(i) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
            } else {
                const double dev = wd(i) * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
                store_dev<ST>((typename Sto<ST>::T*)a.fout, k, i, (float)dev, c);
            }
        }
    }
}

template <int ST>
__global__ void fields_kernel(StepArgs a, int chan, double* fo, double* rho_o, double* ux_o,
                              double* uy_o) {
    const ChanDev c = a.chan[chan];
    const long long n = (long long)c.nx * c.ny;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(t % c.nx), y = (int)(t / c.nx);
        double f[9], rho, jx, jy;
        pull_node_f64<ST>(a.fin, c, x, y, f);
        moments_f64(f, c, rho, jx, jy);
        if (fo)
            for (int i = 0; i < 9; ++i) fo[i * n + t] = f[i];
        if (rho_o) rho_o[t] = rho;
        if (ux_o) ux_o[t] = jx / rho;
        if (uy_o) uy_o[t] = jy / rho;
    }
}

// Inverse of the pull: population i at node x takes f_i(x + e_i).
template <int ST>
__global__ void set_pop_kernel(StepArgs a, int chan, const double* fi) {
    const ChanDev c = a.chan[chan];
    const long long n = (long long)c.nx * c.ny;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(t % c.nx), y = (int)(t / c.nx);
        for (int i = 0; i < 9; ++i) {
            int xd = x + ex(i), yd = y + ey(i);
            if (c.bcx == 0) xd = xd < 0 ? xd + c.nx : (xd >= c.nx ? xd - c.nx : xd);
            else if (xd < 0 || xd >= c.nx) xd = x;
            if (c.bcy == 0) yd = yd < 0 ? yd + c.ny : (yd >= c.ny ? yd - c.ny : yd);
            else if (yd < 0 || yd >= c.ny) yd = y;
            const double v = fi[i * n + (long long)yd * c.nx + xd];
            const long long k = pidx(c, i, y, x);
            if constexpr (ST == ST_F64) {
                ((double*)a.fout)[k] = v;
            } else {
                store_dev<ST>((typename Sto<ST>::T*)a.fout, k, i, (float)(v - wd(i)), c);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Plain device copy: each workgroup copies a contiguous block of 4 x 256
// 16-byte elements, four nontemporal loads in flight per lane before the
// four nontemporal stores (the fastest of the shapes measured on this part:
// grid-stride loops, deeper unrolling and cached accesses were slower).  The
// ceiling that HBM-bound passes are measured against.
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kCopyUnroll = 4;

__global__ __launch_bounds__(256) void copy_kernel(v4f* __restrict__ dst, const v4f* __restrict__ src,
                                                   long long n) {
    const long long base = (long long)blockIdx.x * 256 * kCopyUnroll + threadIdx.x;
    v4f v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const long long i = base + (long long)u * 256;
        if (i < n) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const long long i = base + (long long)u * 256;
        if (i < n) __builtin_nontemporal_store(v[u], dst + i);
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_copy(void* dst, const void* src, long long n16, hipStream_t s) {
    const long long per = 256LL * kCopyUnroll;
    const long long grid = (n16 + per - 1) / per;
    if (grid > INT_MAX) return hipErrorInvalidValue;
    copy_kernel<<<(int)grid, 256, 0, s>>>((v4f*)dst, (const v4f*)src, n16);
    return hipGetLastError();
}

#define LBM_DISPATCH(store, F)                     \
    switch (store) {                               \
        case ST_F64: F(ST_F64); break;             \
        case ST_F32: F(ST_F32); break;             \
        default: F(ST_F16S); break;                \
    }

static int grid_for(long long n, int block) {
    long long g = (n + block - 1) / block;
    return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

hipError_t launch_init(int store, const StepArgs& a, int chan, int init, int nx, int ny,
                       hipStream_t s) {
    const int grid = grid_for((long long)nx * ny, 256);
#define L_(ST) init_kernel<ST><<<grid, 256, 0, s>>>(a, chan, init)
    LBM_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

// Static LDS of the force kernel, as compiled (the mask store takes the rest).
hipError_t launch_ibm_force(int store, const StepArgs& a, hipStream_t s) {
    const int grid = a.nwork > 0 ? a.nwork : 1;  // workgroup 0 also counts the step
#define L_(ST) ibm_force_kernel<ST><<<grid, kIbmThreads, 0, s>>>(a)
    LBM_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

template <int ST>
static hipError_t lattice_dispatch(const StepArgs& a, int tile_w, int npt, int grid,
                                   hipStream_t s) {
#define LK(TW, NPT) lattice_kernel<ST, TW, NPT><<<grid, 256, 0, s>>>(a)
    if (tile_w == 64) {
        if (npt == 1) LK(64, 1);
        else if (npt == 2) LK(64, 2);
        else LK(64, 4);
    } else if (tile_w == 128) {
        if (npt == 1) LK(128, 1);
        else if (npt == 2) LK(128, 2);
        else LK(128, 4);
    } else {
        if (npt == 1) LK(256, 1);
        else if (npt == 2) LK(256, 2);
        else LK(256, 4);
    }
#undef LK
    return hipGetLastError();
}

template <int ST, int NV>
static hipError_t vdispatch_npt(const StepArgs& a, int npt, int grid, hipStream_t s) {
    if (a.nt_store) {
        if (npt == 1) lattice_vkernel<ST, NV, 1, true><<<grid, 256, 0, s>>>(a);
        else lattice_vkernel<ST, NV, 2, true><<<grid, 256, 0, s>>>(a);
    } else {
        if (npt == 1) lattice_vkernel<ST, NV, 1, false><<<grid, 256, 0, s>>>(a);
        else lattice_vkernel<ST, NV, 2, false><<<grid, 256, 0, s>>>(a);
    }
    return hipGetLastError();
}

// NV = tile_w / 64 nodes per lane; chunks of at most 16 bytes.
template <int ST>
static hipError_t lattice_vdispatch(const StepArgs& a, int tile_w, int npt, int grid, hipStream_t s) {
    constexpr int kMaxNv = 16 / (int)sizeof(typename Sto<ST>::T);
    const int nv = tile_w / 64;
    if (nv > kMaxNv || npt > 2) return hipErrorInvalidValue;
    switch (nv) {
        case 1: return vdispatch_npt<ST, 1>(a, npt, grid, s);
        case 2: return vdispatch_npt<ST, 2>(a, npt, grid, s);
        case 4:
            if constexpr (kMaxNv >= 4) return vdispatch_npt<ST, 4>(a, npt, grid, s);
            return hipErrorInvalidValue;
        case 8:
            if constexpr (kMaxNv >= 8) return vdispatch_npt<ST, 8>(a, npt, grid, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lattice(int store, const StepArgs& a, int tile_w, int npt, int vec, hipStream_t s) {
    int grid = a.persistent > 0 ? (a.persistent < a.ntiles ? a.persistent : a.ntiles) : a.ntiles;
    if (a.xcd_remap && a.persistent <= 0) grid = (a.ntiles + 7) / 8 * 8;
    if (grid <= 0) return hipSuccess;
    if (vec) {
        switch (store) {
            case ST_F64: return lattice_vdispatch<ST_F64>(a, tile_w, npt, grid, s);
            case ST_F32: return lattice_vdispatch<ST_F32>(a, tile_w, npt, grid, s);
            default: return lattice_vdispatch<ST_F16S>(a, tile_w, npt, grid, s);
        }
    }
    switch (store) {
        case ST_F64: return lattice_dispatch<ST_F64>(a, tile_w, npt, grid, s);
        case ST_F32: return lattice_dispatch<ST_F32>(a, tile_w, npt, grid, s);
        default: return lattice_dispatch<ST_F16S>(a, tile_w, npt, grid, s);
    }
}

hipError_t launch_patch_sum(const StepArgs& a, hipStream_t s) {
    if (a.npsum <= 0) return hipSuccess;
    patch_sum_kernel<<<a.npsum, 256, 0, s>>>(a);
    return hipGetLastError();
}

// Compute units of the current device (queried once per device).
static int cu_count() {
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] <= 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

hipError_t launch_traction(int store, const StepArgs& a, hipStream_t s) {
    if (a.nwork <= 0) return hipSuccess;
    const bool pair = a.nwork > cu_count();
#define L_(ST)                                                                          \
    if (pair) traction_kernel<ST, true><<<a.nwork, kIbmThreads, 0, s>>>(a);            \
    else traction_kernel<ST, false><<<a.nwork, kIbmThreads, 0, s>>>(a)
    LBM_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

template <int ST>
static hipError_t lattice_traction_dispatch(const StepArgs& a, int npt, int tb, int grid,
                                            hipStream_t s) {
    if (npt == 1) lattice_traction_kernel<ST, 1><<<grid, kIbmThreads, 0, s>>>(a, tb);
    else if (npt == 2) lattice_traction_kernel<ST, 2><<<grid, kIbmThreads, 0, s>>>(a, tb);
    else lattice_traction_kernel<ST, 4><<<grid, kIbmThreads, 0, s>>>(a, tb);
    return hipGetLastError();
}

template <int ST, int NV>
static hipError_t lattice_traction_vdispatch_nv(const StepArgs& a, int tb, int grid, hipStream_t s) {
    if (a.nt_store) lattice_traction_vkernel<ST, NV, true><<<grid, 256, 0, s>>>(a, tb);
    else lattice_traction_vkernel<ST, NV, false><<<grid, 256, 0, s>>>(a, tb);
    return hipGetLastError();
}

// The vector combined launch is built for the chunk widths that fill 16 or 8
// bytes: nv 1, 2 (FP64), 2, 4 (FP32), 4, 8 (F16S).
template <int ST>
static hipError_t lattice_traction_vdispatch(const StepArgs& a, int tb, int grid, hipStream_t s) {
    constexpr int kMaxNv = 16 / (int)sizeof(typename Sto<ST>::T);
    switch (a.tile_w / 64) {
        case 1: return lattice_traction_vdispatch_nv<ST, 1>(a, tb, grid, s);
        case 2: return lattice_traction_vdispatch_nv<ST, 2>(a, tb, grid, s);
        case 4:
            if constexpr (kMaxNv >= 4) return lattice_traction_vdispatch_nv<ST, 4>(a, tb, grid, s);
            return hipErrorInvalidValue;
        case 8:
            if constexpr (kMaxNv >= 8) return lattice_traction_vdispatch_nv<ST, 8>(a, tb, grid, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lattice_traction(int store, const StepArgs& a, int npt, int vec, hipStream_t s) {
    if (a.persistent > 0 || (vec ? npt != 1 || a.tile_h != 4 : a.tile_w != 64 || a.tile_h != 9 * npt))
        return hipErrorInvalidValue;
    const long long tb = a.nwork > 0 ? ((long long)a.nwork + 7) / 8 * 8 : 0;
    const long long tl = a.xcd_remap ? ((long long)a.ntiles + 7) / 8 * 8 : a.ntiles;
    const long long grid = tb + tl;
    if (grid <= 0) return hipSuccess;
    if (grid > INT_MAX) return hipErrorInvalidValue;
    if (vec) {
        switch (store) {
            case ST_F64: return lattice_traction_vdispatch<ST_F64>(a, (int)tb, (int)grid, s);
            case ST_F32: return lattice_traction_vdispatch<ST_F32>(a, (int)tb, (int)grid, s);
            default: return lattice_traction_vdispatch<ST_F16S>(a, (int)tb, (int)grid, s);
        }
    }
    switch (store) {
        case ST_F64: return lattice_traction_dispatch<ST_F64>(a, npt, (int)tb, (int)grid, s);
        case ST_F32: return lattice_traction_dispatch<ST_F32>(a, npt, (int)tb, (int)grid, s);
        default: return lattice_traction_dispatch<ST_F16S>(a, npt, (int)tb, (int)grid, s);
    }
}

hipError_t launch_fields(int store, const StepArgs& a, int chan, int nx, int ny, double* f_out,
                         double* rho, double* ux, double* uy, hipStream_t s) {
    const int grid = grid_for((long long)nx * ny, 256);
#define L_(ST) fields_kernel<ST><<<grid, 256, 0, s>>>(a, chan, f_out, rho, ux, uy)
    LBM_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

hipError_t launch_set_pop(int store, const StepArgs& a, int chan, int nx, int ny,
                          const double* f_in, hipStream_t s) {
    const int grid = grid_for((long long)nx * ny, 256);
#define L_(ST) set_pop_kernel<ST><<<grid, 256, 0, s>>>(a, chan, f_in)
    LBM_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

}  // namespace lbmk
