// gfx950 kernels of the discrete adjoint of the coupled LBM / MLS-IBM step.
//
// The forward step n maps (f^n, particle state P^n) to (f^{n+1}, P^{n+1})
// through the moments (Eqs. (6), (7)), the immersed-boundary force and its
// spreading (Eqs. (8)-(12)), the forced collision (Eqs. (4), (5)), the surface
// stress with force and moment (Eqs. (13), (14)), BDF2 (Eqs. (15), (16)),
// streaming and the Zou-He closure (App. A).  Its transpose has three
// stages per step, in this order (as three kernels, or, when no channel holds
// more than one particle, as adj_particle_kernel + adj_lattice_kernel or as
// the single adj_step_kernel):
//
//   adj_traction  one workgroup per particle: transpose of BDF2 and of the
//                 probe traction; the field terms (d/d rho and d/d u at the
//                 probe stencil nodes) go into the particle's adjoint patch.
//   adj_ibm       one workgroup per particle: adjoint of the IB force at the
//                 marker stencil nodes (it needs the collision transpose there),
//                 transpose of interpolation and spreading including the
//                 motion of the MLS weights with the markers; the d/d u* terms
//                 go into the adjoint patch.
//   adj_lattice   one wave per 64-node chunk of a tile: adjoint streaming (a pull from
//                 x + e_i), transpose of the collision and of the moments with
//                 the patch terms added, transpose of the Zou-He closure on
//                 wall nodes, whose wall-speed derivatives accumulate per node.
//
// MLS stencil anchors are piecewise constant in the particle state and are
// held fixed, so this is the derivative of the smooth branch of the step.
// Field arithmetic is FP64; the adjoint populations are stored in FP64 for the
// FP64 form and in FP32 otherwise.  Every sum has a fixed order (no float
// atomics), so the adjoint is bitwise reproducible.
#include <climits>

#include "lbm_adjoint.h"
#include "lbm_device.h"

namespace lbmk {

// The particle kernels of the adjoint hold more live FP64 state per thread
// than the forward ones: they run 56 markers x 9 stencil nodes per round in
// 512-thread workgroups (two waves per SIMD, 256 VGPRs each, no spills).
constexpr int kAdjRound = 56;
constexpr int kAdjThreads = 512;
// Patch cells of an adjoint box that the deposit can index by anchor masks
// (64-bit, one bit per marker of a round); larger boxes scan the markers.
constexpr int kAdjMaskCells = 4096;

template <int ST> struct LamT { using T = float; };
template <> struct LamT<ST_F64> { using T = double; };

// Adjoint of the population i pulled at (x, y) by the next step: the pull
// read the node x - e_i, so its adjoint is read at x + e_i.  Beyond a
// wall-bounded edge nothing was pulled: zero.  Branch-free (the address is
// clamped to a valid node and the value masked), so the nine reads of a node
// are issued together.
template <int ST>
__device__ __forceinline__ double lam_push(const void* lam, const ChanDev& c, int i, int x, int y) {
    const int xd = x + ex(i), yd = y + ey(i);
    const int xs = pull_coord(xd, x, c.nx, c.bcx == 0), ys = pull_coord(yd, y, c.ny, c.bcy == 0);
    const bool ok = (c.bcx == 0 || (xd >= 0 && xd < c.nx)) && (c.bcy == 0 || (yd >= 0 && yd < c.ny));
    using LT = typename LamT<ST>::T;
    const char* base = (const char*)lam + c.off * (long long)sizeof(LT);  // the channel's block
    const double v = (double)at<LT>(base, boff<LT>(c, i, ys, xs));
    return ok ? v : 0.0;
}

// Streamed populations at (x, y) before any wall closure, FP64.
template <int ST>
__device__ __forceinline__ void pull_raw_f64(const void* fin, const ChanDev& c, int x, int y, double f[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int xs, ys;
        pull_src(c, i, x, y, xs, ys);
        if constexpr (ST == ST_F64) {
            f[i] = ((const double*)fin)[pidx(c, i, ys, xs)];
        } else {
            f[i] = wd(i) + (double)load_dev<ST>((const typename Sto<ST>::T*)fin, pidx(c, i, ys, xs), i, c);
        }
    }
}

// W'(r)/r of the interpolation kernels of kernel_weight.
__device__ __forceinline__ double kernel_dw(int kind, double r, double alpha) {
    if (r > 1.0) return 0.0;
    if (kind == 0) {
        const double q = r / alpha;
        return -2.0 / (alpha * alpha) * exp(-(q * q));
    } else if (kind == 1) {
        return -8.0 + 12.0 * r;
    } else if (kind == 2) {
        return -12.0 + 24.0 * r - 12.0 * r * r;
    } else if (kind == 3) {
        const double h = 3.14159265358979323846 / 2.0;
        if (r < 1e-8) return -h * h / 4.0;
        return -0.25 * h * sin(h * r) / r;
    }
    // polynomial kernel W(r) = phi(2 r): W'(r) / r = 2 phi'(2 r) / r, which
    // tends to -4 as r -> 0 (phi(q) = 1/2 - q^2/2 + O(q^3))
    if (r < 1e-8) return -4.0;
    const double q = 2.0 * r;
    const double dphi = q <= 1.0 ? (-2.0 + (2.0 - 4.0 * q) / sqrt(1.0 + 4.0 * q - 4.0 * q * q)) / 8.0
                                 : (-2.0 - (6.0 - 4.0 * q) / sqrt(-7.0 + 12.0 * q - 4.0 * q * q)) / 8.0;
    return 2.0 * dphi / r;
}

// Transpose of the forced collision of one node (Eqs. (4), (5)) at (rho, u, G)
// applied to the adjoint lfc of its outputs: the feq part of d/d rho, d/d u
// and d/d G.  Every term is linear in the weighted moments of lfc,
// A0 = sum w_i a_i, A_a = sum w_i a_i e_ia, A_ab = sum w_i a_i e_ia e_ib,
// because feq and the Guo term are polynomials in e_i of degree two:
//   d/d rho = (A0 (1 - 1.5 u.u) + 3 u.A1 + 4.5 u.A2.u) / tau
//   d/d u   = rho/tau (3 A1 + 9 A2 u - 3 u A0) + pref (9 A2 G - 3 G A0)
//   d/d G   = pref (3 A1 - 3 u A0 + 9 A2 u)
struct CollAdj {
    double lrho, lux, luy, lGx, lGy;
};

__device__ __forceinline__ CollAdj collide_adj(const double lfc[9], double rho, double ux, double uy,
                                               double Gx, double Gy, double tau) {
    const double pref = 1.0 - 1.0 / (2.0 * tau);
    const double itau = 1.0 / tau;
    // e: 0 (0,0) 1 (1,0) 2 (0,1) 3 (-1,0) 4 (0,-1) 5 (1,1) 6 (-1,1) 7 (-1,-1) 8 (1,-1)
    const double w0 = 4.0 / 9.0, w1 = 1.0 / 9.0, w2 = 1.0 / 36.0;
    const double ax = lfc[1] + lfc[3], ay = lfc[2] + lfc[4];
    const double dg = lfc[5] + lfc[6] + lfc[7] + lfc[8];
    const double A0 = w0 * lfc[0] + w1 * (ax + ay) + w2 * dg;
    const double Ax = w1 * (lfc[1] - lfc[3]) + w2 * ((lfc[5] - lfc[6]) + (lfc[8] - lfc[7]));
    const double Ay = w1 * (lfc[2] - lfc[4]) + w2 * ((lfc[5] + lfc[6]) - (lfc[7] + lfc[8]));
    const double Axx = w1 * ax + w2 * dg;
    const double Ayy = w1 * ay + w2 * dg;
    const double Axy = w2 * ((lfc[5] + lfc[7]) - (lfc[6] + lfc[8]));
    const double usq = ux * ux + uy * uy;
    const double A2u_x = Axx * ux + Axy * uy, A2u_y = Axy * ux + Ayy * uy;
    const double A2G_x = Axx * Gx + Axy * Gy, A2G_y = Axy * Gx + Ayy * Gy;
    CollAdj r;
    r.lrho = (A0 * (1.0 - 1.5 * usq) + 3.0 * (ux * Ax + uy * Ay) + 4.5 * (ux * A2u_x + uy * A2u_y)) * itau;
    r.lux = rho * itau * (3.0 * Ax + 9.0 * A2u_x - 3.0 * ux * A0) + pref * (9.0 * A2G_x - 3.0 * Gx * A0);
    r.luy = rho * itau * (3.0 * Ay + 9.0 * A2u_y - 3.0 * uy * A0) + pref * (9.0 * A2G_y - 3.0 * Gy * A0);
    r.lGx = pref * (3.0 * Ax - 3.0 * ux * A0 + 9.0 * A2u_x);
    r.lGy = pref * (3.0 * Ay - 3.0 * uy * A0 + 9.0 * A2u_y);
    return r;
}

// Transpose of the Zou-He closure of walls_f64 at one wall node.  fr holds
// the streamed (known) populations; L the adjoint of the closed populations,
// replaced by the adjoint of the streamed ones (zero for the three unknowns,
// which the closure overwrites).  Adds the wall-velocity derivatives.
__device__ __forceinline__ void zouhe_adj(int side, const double fr[9], double L[9], double uwx,
                                          double uwy, double gx, double gy, double& gux, double& guy) {
    double D, rho, lmx, lmy;
    if (side == 2) {
        D = 1.0 - uwy;
        rho = (fr[0] + fr[1] + fr[3] + 2.0 * (fr[4] + fr[7] + fr[8]) - 0.5 * gy) / D;
        lmy = 2.0 / 3.0 * L[2] + L[5] / 6.0 + L[6] / 6.0;
        lmx = 0.5 * L[5] - 0.5 * L[6];
        const double lr = (lmx * uwx + lmy * uwy) / D;
        gux += lmx * rho;
        guy += lmy * rho + lr * rho;
        L[0] += lr;
        L[1] += -0.5 * L[5] + 0.5 * L[6] + lr;
        L[3] += 0.5 * L[5] - 0.5 * L[6] + lr;
        L[4] += L[2] + 2.0 * lr;
        L[7] += L[5] + 2.0 * lr;
        L[8] += L[6] + 2.0 * lr;
        L[2] = L[5] = L[6] = 0.0;
    } else if (side == 3) {
        D = 1.0 + uwy;
        rho = (fr[0] + fr[1] + fr[3] + 2.0 * (fr[2] + fr[5] + fr[6]) + 0.5 * gy) / D;
        lmy = -2.0 / 3.0 * L[4] - L[7] / 6.0 - L[8] / 6.0;
        lmx = -0.5 * L[7] + 0.5 * L[8];
        const double lr = (lmx * uwx + lmy * uwy) / D;
        gux += lmx * rho;
        guy += lmy * rho - lr * rho;
        L[0] += lr;
        L[1] += 0.5 * L[7] - 0.5 * L[8] + lr;
        L[3] += -0.5 * L[7] + 0.5 * L[8] + lr;
        L[2] += L[4] + 2.0 * lr;
        L[5] += L[7] + 2.0 * lr;
        L[6] += L[8] + 2.0 * lr;
        L[4] = L[7] = L[8] = 0.0;
    } else if (side == 0) {
        D = 1.0 - uwx;
        rho = (fr[0] + fr[2] + fr[4] + 2.0 * (fr[3] + fr[6] + fr[7]) - 0.5 * gx) / D;
        lmx = 2.0 / 3.0 * L[1] + L[5] / 6.0 + L[8] / 6.0;
        lmy = 0.5 * L[5] - 0.5 * L[8];
        const double lr = (lmx * uwx + lmy * uwy) / D;
        gux += lmx * rho + lr * rho;
        guy += lmy * rho;
        L[0] += lr;
        L[2] += -0.5 * L[5] + 0.5 * L[8] + lr;
        L[4] += 0.5 * L[5] - 0.5 * L[8] + lr;
        L[3] += L[1] + 2.0 * lr;
        L[7] += L[5] + 2.0 * lr;
        L[6] += L[8] + 2.0 * lr;
        L[1] = L[5] = L[8] = 0.0;
    } else {
        D = 1.0 + uwx;
        rho = (fr[0] + fr[2] + fr[4] + 2.0 * (fr[1] + fr[5] + fr[8]) + 0.5 * gx) / D;
        lmx = -2.0 / 3.0 * L[3] - L[7] / 6.0 - L[6] / 6.0;
        lmy = -0.5 * L[7] + 0.5 * L[6];
        const double lr = (lmx * uwx + lmy * uwy) / D;
        gux += lmx * rho - lr * rho;
        guy += lmy * rho;
        L[0] += lr;
        L[2] += 0.5 * L[7] - 0.5 * L[6] + lr;
        L[4] += -0.5 * L[7] + 0.5 * L[6] + lr;
        L[1] += L[3] + 2.0 * lr;
        L[5] += L[7] + 2.0 * lr;
        L[8] += L[6] + 2.0 * lr;
        L[3] = L[7] = L[6] = 0.0;
    }
}

// Inverse of the MLS moment matrix (as mls_inverse) with one reciprocal of
// the determinant: the adjoint linearises the step at the taped state, where
// the last bits of B do not matter.  As in mls_inverse, w is zero at dropped
// nodes, whose terms are then signed zeros, so the loop has no branch.
__device__ __forceinline__ MlsInv mls_inverse_adj(const double* w, int i0, int j0, double x, double y) {
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
    const double c00 = A11 * A22 - A12 * A12, c01 = A02 * A12 - A01 * A22, c02 = A01 * A12 - A02 * A11;
    const double idet = 1.0 / (A00 * c00 + A01 * c01 + A02 * c02);
    MlsInv r;
    r.i00 = c00 * idet;
    r.i01 = c01 * idet;
    r.i02 = c02 * idet;
    r.i11 = (A00 * A22 - A02 * A02) * idet;
    r.i12 = (A01 * A02 - A00 * A12) * idet;
    r.i22 = (A00 * A11 - A01 * A01) * idet;
    return r;
}

// Cell of the box (wrapped origin x0, y0, extent w x h) holding node (x, y),
// or -1.
__device__ __forceinline__ int box_cell(const ChanDev& c, int x0, int y0, int w, int h, int x, int y) {
    int dx = x - x0, dy = y - y0;
    if (c.bcx == 0 && dx < 0) dx += c.nx;
    if (c.bcy == 0 && dy < 0) dy += c.ny;
    return (dx >= 0 && dx < w && dy >= 0 && dy < h) ? dy * w + dx : -1;
}

// Force f_lb and the first NF adjoint-patch terms at node (x, y) from the
// particles of a list (n <= kMaxNeighbours) or, when the list overflowed, of
// the channel.  Ascending particle order.
template <int NF>
__device__ __forceinline__ void patch_terms(const AdjArgs& a, const ChanDev& c, const int* list, int n,
                                            int x, int y, double& fx, double& fy, double t[kAdjCell]) {
    fx = 0.0;
    fy = 0.0;
#pragma unroll
    for (int k = 0; k < kAdjCell; ++k) t[k] = 0.0;
    const bool all = n > kMaxNeighbours;
    const int cnt = all ? c.p_end - c.p_begin : n;
    for (int j = 0; j < cnt; ++j) {
        const int q = all ? c.p_begin + j : list[j];
        const PartDev& P = a.s.parts[q];
        if (P.bw > 0) {
            const int cf = box_cell(c, P.bx0, P.by0, P.bw, P.bh, x, y);
            if (cf >= 0) {
                const double2 v = a.s.patch[P.patch_off + cf];
                fx += v.x;
                fy += v.y;
            }
        }
        const AdjPart& Q = a.ap[q];
        const int ca = box_cell(c, Q.ax0, Q.ay0, Q.aw, Q.ah, x, y);
        if (ca >= 0) {
            const double* v = a.apatch + (Q.aoff + ca) * kAdjCell;
#pragma unroll
            for (int k = 0; k < NF; ++k) t[k] += v[k];
        }
    }
}

// Boxes of the neighbour particles' force and adjoint patches, staged in LDS
// so that a node's patch addresses are known as soon as the node is, and the
// patch reads go out together with the population reads.
struct NbBox {
    int fx0, fy0, fw, fh;    // force patch (fw = 0: none)
    int ax0, ay0, aw, ah;    // adjoint patch (aw = 0: none)
    long long foff, aoff;
};

template <int NF>
__device__ __forceinline__ void patch_terms_lds(const AdjArgs& a, const ChanDev& c, const NbBox* nb, int n, int x,
                                                int y, double& fx, double& fy, double t[kAdjCell]) {
    fx = 0.0;
    fy = 0.0;
#pragma unroll
    for (int k = 0; k < kAdjCell; ++k) t[k] = 0.0;
    // reads from clamped (always allocated) cells, masked: no load waits on
    // a branch
    for (int j = 0; j < n; ++j) {
        const NbBox& B = nb[j];
        const int cf = box_cell(c, B.fx0, B.fy0, B.fw, B.fh, x, y);
        const double2 v = a.s.patch[B.foff + (cf >= 0 ? cf : 0)];
        fx += cf >= 0 ? v.x : 0.0;
        fy += cf >= 0 ? v.y : 0.0;
        if (NF > 0) {
            const int ca = box_cell(c, B.ax0, B.ay0, B.aw, B.ah, x, y);
            const double* va = a.apatch + (B.aoff + (ca >= 0 ? ca : 0)) * kAdjCell;
#pragma unroll
            for (int k = 0; k < NF; ++k) t[k] += ca >= 0 ? va[k] : 0.0;
        }
    }
}

// Force f_lb alone at (x, y) from a list of forward patches (ascending).
__device__ __forceinline__ void fwd_force(const AdjArgs& a, const ChanDev& c, const int* list, int n,
                                          int x, int y, double& fx, double& fy) {
    fx = 0.0;
    fy = 0.0;
    const bool all = n > kMaxNeighbours;
    const int cnt = all ? c.p_end - c.p_begin : n;
    for (int j = 0; j < cnt; ++j) {
        const int q = all ? c.p_begin + j : list[j];
        const PartDev& P = a.s.parts[q];
        if (P.bw <= 0) continue;
        const int cf = box_cell(c, P.bx0, P.by0, P.bw, P.bh, x, y);
        if (cf >= 0) {
            const double2 v = a.s.patch[P.patch_off + cf];
            fx += v.x;
            fy += v.y;
        }
    }
}

// ---------------------------------------------------------------------------
// Motion of the MLS weights with the evaluation point x, anchors held fixed.
// Psi_k = (phi_k, Dx_k, Dy_k) = W_k B p_k are the value and derivative
// weights of Eq. (8) (B = A^{-1}, p_k = (1, x_k - x)).  With z_k = B p_k,
// y_k = B lam_k and S = sum_k W_k z_k y_k^T,
//   d/dx_b sum_k lam_k . Psi_k = sum_k dW_k/dx_b (lam_k . z_k - p_k^T S p_k)
//                              + sum_k W_k ((S^T p_k)_b + (S p_k)_b - (y_k)_b)
// (b the x or y slot of p; dp_k/dx_b = -e_b).  Split over the nine stencil
// threads of a marker: each leaves its share of S, the shares are summed,
// then each forms its term.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mls_share(const double* B6, const double p[3], const double lam[3], double w,
                                          double z[3], double y[3], double* S9) {
    const double B[3][3] = {{B6[0], B6[1], B6[2]}, {B6[1], B6[3], B6[4]}, {B6[2], B6[4], B6[5]}};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        z[r] = B[r][0] * p[0] + B[r][1] * p[1] + B[r][2] * p[2];
        y[r] = B[r][0] * lam[0] + B[r][1] * lam[1] + B[r][2] * lam[2];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) S9[3 * r + q] = w * z[r] * y[q];
}

__device__ __forceinline__ void mls_term(const ChanDev& c, const double* S9, const double p[3], const double z[3],
                                         const double y[3], const double lam[3], double w, double& ox, double& oy) {
    double Sp[3], STp[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        Sp[r] = S9[3 * r] * p[0] + S9[3 * r + 1] * p[1] + S9[3 * r + 2] * p[2];
        STp[r] = S9[r] * p[0] + S9[3 + r] * p[1] + S9[6 + r] * p[2];
    }
    const double lz = lam[0] * z[0] + lam[1] * z[1] + lam[2] * z[2];
    const double pSp = p[0] * Sp[0] + p[1] * Sp[1] + p[2] * Sp[2];
    const double dx = p[1], dy = p[2];
    const double r = sqrt(dx * dx + dy * dy) / c.rw;
    const double dw = kernel_dw(c.kernel, r, c.alpha) / (c.rw * c.rw);
    ox = -dw * dx * (lz - pSp) + w * (STp[1] + Sp[1]) - w * y[1];
    oy = -dw * dy * (lz - pSp) + w * (STp[2] + Sp[2]) - w * y[2];
}

// Deposit the round's per-(marker, node) terms d[m * 9 + k][0..NF) into the
// particle's adjoint patch (fields F0..F0+NF): each cell sums the markers
// whose stencils cover it in ascending order (found from the anchor masks of
// its 3x3 neighbourhood, or by a scan when the box is larger than the mask
// store); a cell is handled by the same thread in every round.  The first
// round writes the cell (and zeroes fields NZ.. when NZ < kAdjCell), later
// rounds add to it.
template <int NF, int F0, int W, int NZ>
__device__ __forceinline__ void deposit_round(double* apatch, int ax0u, int ay0u, int aw, int ah, int ncell,
                                              const int2* anc, const unsigned long long* mask,
                                              const double (*d)[W], int nr, bool first) {
    const bool masked = ncell <= kAdjMaskCells;
    for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
        const int qx = q % aw, qy = q / aw;
        const int cx = ax0u + qx, cy = ay0u + qy;
        double t[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) t[f] = 0.0;
        if (masked) {
            unsigned long long msk = 0ull;
            for (int dy = -1; dy <= 1; ++dy) {
                const int yy = qy + dy;
                if (yy < 0 || yy >= ah) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int xx = qx + dx;
                    if (xx < 0 || xx >= aw) continue;
                    msk |= mask[yy * aw + xx];
                }
            }
            while (msk) {
                const int m = __ffsll((long long)msk) - 1;
                msk &= msk - 1ull;
                const int2 an = anc[m];
                const int kk = 3 * (cy - an.y + 1) + (cx - an.x + 1);
#pragma unroll
                for (int f = 0; f < NF; ++f) t[f] += d[m * 9 + kk][f];
            }
        } else {
            for (int m = 0; m < nr; ++m) {
                const int2 an = anc[m];
                const int ddx = cx - an.x, ddy = cy - an.y;
                if (ddx < -1 || ddx > 1 || ddy < -1 || ddy > 1) continue;
                const int kk = 3 * (ddy + 1) + (ddx + 1);
#pragma unroll
                for (int f = 0; f < NF; ++f) t[f] += d[m * 9 + kk][f];
            }
        }
        double* v = apatch + (long long)q * kAdjCell;
        if (first) {
#pragma unroll
            for (int f = 0; f < NF; ++f) v[F0 + f] = t[f];
#pragma unroll
            for (int f = NZ; f < kAdjCell; ++f) v[f] = 0.0;
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) v[F0 + f] += t[f];
        }
    }
}

// ---------------------------------------------------------------------------
// Kernel A: transpose of BDF2 and of the surface-stress force (one workgroup
// per particle, markers in rounds of 64, one thread per (marker, probe
// stencil node)).
// ---------------------------------------------------------------------------
// LDS of the traction part of a reversed step.
struct AdjTracLds {
    double w[kAdjThreads], r[kAdjThreads], ux[kAdjThreads], uy[kAdjThreads];
    double dep[kAdjThreads][3];
    double S[kAdjThreads][9];  // per node: share of S, then its term
    double Sm[kAdjRound][9];
    double B[kAdjRound][6];
    double sc[kAdjRound][5];   // d/d rho_P, d/d (du/dx, du/dy, dv/dx, dv/dy)
    double xp[kAdjRound][2];
    double geo[kAdjRound][4];  // r and n of the marker
    double g[kAdjRound][5];    // its accumulated shape gradients
    double pt[kAdjRound][8];   // its particle terms
    int2 anc[kAdjRound];
    double part[AL_N], lF[3], run[8];
    int nb[kMaxNeighbours], nnb;
    NbBox box[kMaxNeighbours];
    unsigned long long mask[kAdjMaskCells];
};

template <int ST>
__device__ __forceinline__ void adj_traction_body(const AdjArgs& a, AdjTracLds& sh) {
    auto& s_w = sh.w;
    auto& s_r = sh.r;
    auto& s_ux = sh.ux;
    auto& s_uy = sh.uy;
    auto& s_dep = sh.dep;
    auto& s_S = sh.S;
    auto& s_Sm = sh.Sm;
    auto& s_B = sh.B;
    auto& s_sc = sh.sc;
    auto& s_xp = sh.xp;
    auto& s_geo = sh.geo;
    auto& s_g = sh.g;
    auto& s_pt = sh.pt;
    auto& s_anc = sh.anc;
    auto& s_part = sh.part;
    auto& s_lF = sh.lF;
    auto& s_run = sh.run;
    auto& s_nb = sh.nb;
    auto& s_nnb = sh.nnb;
    auto& s_box = sh.box;
    auto& s_mask = sh.mask;
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    if (b >= a.s.nparts) return;
    const PartDev* P = a.s.parts + b;
    AdjPart* A = a.ap + b;
    const ChanDev c = load_chan(a.s.chan + P->chan);  // in registers: not re-read after each barrier
    const int nm = P->nm, mb = P->mbeg;
    // marker geometry of the first round, requested before anything else
    double2 pre_x = make_double2(0.0, 0.0), pre_n = make_double2(0.0, 0.0);
    if (tid / 9 < kAdjRound && tid / 9 < nm) {
        pre_x = a.s.xi[mb + tid / 9];
        pre_n = a.s.nrm[mb + tid / 9];
    }
    const double X0 = P->X[0], X1 = P->X[1], Om = P->Om;
    const double acc0 = P->acc[0], acc1 = P->acc[1], alp = P->alp;
    if (tid < 8) s_run[tid] = 0.0;
    const double nu = c.nu, dn = c.dn;
    const double cs = P->cth, sn = P->sth;

    // adjoint patch box (covers probe and marker stencils)
    int ax0u, ay0u, aw, ah;
    stencil_box(X0, X1, P->rb + dn, ax0u, ay0u, aw, ah);
    const bool fits = (long long)aw * ah <= A->acap && aw <= c.nx && ah <= c.ny;
    if (tid == 64) {
        // BDF2 transpose (Eqs. (15), (16) with the position update): the
        // adjoint of the new velocity collects that of the new position.
        // (First lane of the second wave: overlaps the neighbour scan.)
        const double* Ln = A->l;
        const double lV1x = Ln[AL_V] + 2.0 / 3.0 * Ln[AL_X];
        const double lV1y = Ln[AL_V + 1] + 2.0 / 3.0 * Ln[AL_X + 1];
        const double lO1 = Ln[AL_OM] + 2.0 / 3.0 * Ln[AL_TH];
        const double lax = 2.0 / 3.0 * lV1x + Ln[AL_ACC];
        const double lay = 2.0 / 3.0 * lV1y + Ln[AL_ACC + 1];
        const double lal = 2.0 / 3.0 * lO1 + Ln[AL_ALP];
        s_part[AL_X] = 4.0 / 3.0 * Ln[AL_X] + Ln[AL_XM];
        s_part[AL_X + 1] = 4.0 / 3.0 * Ln[AL_X + 1] + Ln[AL_XM + 1];
        s_part[AL_XM] = -1.0 / 3.0 * Ln[AL_X];
        s_part[AL_XM + 1] = -1.0 / 3.0 * Ln[AL_X + 1];
        s_part[AL_TH] = 4.0 / 3.0 * Ln[AL_TH] + Ln[AL_THM];
        s_part[AL_THM] = -1.0 / 3.0 * Ln[AL_TH];
        s_part[AL_V] = 4.0 / 3.0 * lV1x + Ln[AL_VM];
        s_part[AL_V + 1] = 4.0 / 3.0 * lV1y + Ln[AL_VM + 1];
        s_part[AL_VM] = -1.0 / 3.0 * lV1x;
        s_part[AL_VM + 1] = -1.0 / 3.0 * lV1y;
        s_part[AL_OM] = 4.0 / 3.0 * lO1 + Ln[AL_OMM];
        s_part[AL_OMM] = -1.0 / 3.0 * lO1;
        s_part[AL_ACC] = 0.0;
        s_part[AL_ACC + 1] = 0.0;
        s_part[AL_ALP] = 0.0;
        // a = F/m + (1 - 1/ratio) g, alpha = M/I
        const PartDev* Pn = a.pnext + b;
        const double m = P->m, I = P->I;
        A->gm += -(lax * Pn->F[0] + lay * Pn->F[1]) / (m * m);
        A->gI += -lal * Pn->M / (I * I);
        s_lF[0] = lax / m + (a.first ? A->seed[0] : 0.0);
        s_lF[1] = lay / m + (a.first ? A->seed[1] : 0.0);
        s_lF[2] = lal / I + (a.first ? A->seed[2] : 0.0);
        if (a.first) A->seed[0] = A->seed[1] = A->seed[2] = 0.0;
        A->ax0 = wrapc(ax0u, c.nx, c.bcx == 0);
        A->ay0 = wrapc(ay0u, c.ny, c.bcy == 0);
        A->aw = fits ? aw : 0;
        A->ah = fits ? ah : 0;
        if (!fits) atomicOr(&a.s.flags[2], 2);
    }
    if (!fits) return;
    // neighbours: particles of the channel whose adjoint boxes overlap ours
    // (their force patches lie inside their adjoint boxes)
    if (tid < 64 && c.p_end - c.p_begin == 1) {
        // alone in its channel: the list is the particle itself (its box
        // overlaps itself), with no scan
        if (tid == 0) {
            s_nb[0] = b;
            NbBox& B = s_box[0];
            B.fx0 = P->bx0;
            B.fy0 = P->by0;
            B.fw = P->bw > 0 ? P->bw : 0;
            B.fh = P->bh;
            B.foff = P->patch_off;
            B.ax0 = B.ay0 = B.aw = B.ah = 0;
            B.aoff = 0;
            s_nnb = 1;
            A->nnb = 1;
            A->nb[0] = b;
        }
    } else if (tid < 64) {
        int n = 0;
        for (int q0 = c.p_begin; q0 < c.p_end; q0 += 64) {
            const int q = q0 + tid;
            bool hit = false;
            if (q < c.p_end) {
                const PartDev& Q = a.s.parts[q];
                int qx0, qy0, qw, qh;
                stencil_box(Q.X[0], Q.X[1], Q.rb + dn, qx0, qy0, qw, qh);
                hit = boxes_overlap(c, ax0u, ay0u, aw, ah, qx0, qy0, qw, qh);
            }
            const unsigned long long bal = __ballot(hit);
            if (hit) {
                const int pos = n + __popcll(bal & ((1ull << tid) - 1ull));
                if (pos < kMaxNeighbours) {
                    const PartDev& Q = a.s.parts[q];
                    s_nb[pos] = q;
                    NbBox& B = s_box[pos];
                    B.fx0 = Q.bx0;
                    B.fy0 = Q.by0;
                    B.fw = Q.bw > 0 ? Q.bw : 0;
                    B.fh = Q.bh;
                    B.foff = Q.patch_off;
                    B.ax0 = B.ay0 = B.aw = B.ah = 0;
                    B.aoff = 0;
                }
            }
            n += __popcll(bal);
        }
        if (tid == 0) {
            s_nnb = n;
            A->nnb = n;
            for (int j = 0; j < n && j < kMaxNeighbours; ++j) A->nb[j] = s_nb[j];
        }
    }
    const int ncell = aw * ah;
    double* apatch = a.apatch + A->aoff * kAdjCell;
    for (int q = tid; q < min(ncell, kAdjMaskCells); q += blockDim.x) s_mask[q] = 0ull;
    __syncthreads();
    const int nnb = s_nnb;
    const double lFx = s_lF[0], lFy = s_lF[1], lM = s_lF[2];

    const int lo = tid / 9, k = tid % 9;
    for (int r0 = 0; r0 < nm; r0 += kAdjRound) {
        const int l = r0 + lo;
        const bool act = lo < kAdjRound && l < nm;
        const bool lead = tid < kAdjRound && r0 + tid < nm;
        // (1) one probe-stencil node per thread: weight and level-n fields
        if (act) {
            const double2 x = r0 == 0 ? pre_x : a.s.xi[mb + l], nb = r0 == 0 ? pre_n : a.s.nrm[mb + l];
            const double rx = cs * x.x - sn * x.y, ry = sn * x.x + cs * x.y;
            const double nxl = cs * nb.x - sn * nb.y, nyl = sn * nb.x + cs * nb.y;
            const double xp = X0 + rx + dn * nxl, yp = X1 + ry + dn * nyl;
            const int i0 = (int)floor(xp + 0.5), j0 = (int)floor(yp + 0.5);
            double dx, dy;
            int ni, nj;
            double w = 0.0, rho = 1.0, ux = 0.0, uy = 0.0;
            if (stencil_node(c, i0, j0, k, xp, yp, dx, dy, ni, nj)) {
                w = stencil_weight(c, dx, dy);
                // every load of the pair first (in-order completion makes
                // them one latency), the arithmetic after
                typename Sto<ST>::T raw[9];
                pull_load<ST>(a.s.fin, c, ni, nj, raw);
                double f[9], jx, jy, fx, fy;
                if (nnb <= kMaxNeighbours) {
                    double t[kAdjCell];
                    patch_terms_lds<0>(a, c, s_box, nnb, ni, nj, fx, fy, t);
                } else {
                    fwd_force(a, c, s_nb, nnb, ni, nj, fx, fy);
                }
                pull_finish_f64<ST>(a.s.fin, c, ni, nj, raw, f);
                moments_f64(f, c, rho, jx, jy);
                ux = (jx + 0.5 * fx) / rho;
                uy = (jy + 0.5 * fy) / rho;
            }
            s_w[tid] = w;
            s_r[tid] = rho;
            s_ux[tid] = ux;
            s_uy[tid] = uy;
            if (k == 0) {
                s_anc[lo] = make_int2(i0, j0);
                if (ncell <= kAdjMaskCells) atomicOr(&s_mask[(j0 - ay0u) * aw + (i0 - ax0u)], 1ull << lo);
                s_xp[lo][0] = xp;
                s_xp[lo][1] = yp;
                s_geo[lo][0] = rx;
                s_geo[lo][1] = ry;
                s_geo[lo][2] = nxl;
                s_geo[lo][3] = nyl;
            } else if (k == 1) {
                const double* gk = a.gmk + (long long)(mb + l) * 5;
                for (int e = 0; e < 5; ++e) s_g[lo][e] = gk[e];
            }
        }
        __syncthreads();
        // (2) per marker: MLS inverse, the forward traction, and the
        // transpose of t -> F, M down to the probe field derivatives
        double rx = 0.0, ry = 0.0, nxl = 0.0, nyl = 0.0, lrx = 0.0, lry = 0.0, lnx = 0.0, lny = 0.0;
        double c_alp = 0.0, c_om = 0.0, lalx = 0.0, laly = 0.0;
        if (lead) {
            const int lm = tid, lg = r0 + lm;
            rx = s_geo[lm][0];
            ry = s_geo[lm][1];
            nxl = s_geo[lm][2];
            nyl = s_geo[lm][3];
            const double xp = s_xp[lm][0], yp = s_xp[lm][1];
            const int i0 = s_anc[lm].x, j0 = s_anc[lm].y;
            const double* w = s_w + lm * 9;
            const MlsInv iv = mls_inverse_adj(w, i0, j0, xp, yp);
            s_B[lm][0] = iv.i00;
            s_B[lm][1] = iv.i01;
            s_B[lm][2] = iv.i02;
            s_B[lm][3] = iv.i11;
            s_B[lm][4] = iv.i12;
            s_B[lm][5] = iv.i22;
            // w is zero at dropped nodes (rho = 1, u = 0 there): no branch
            double rP = 0.0, dudx = 0.0, dudy = 0.0, dvdx = 0.0, dvdy = 0.0;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int ii = i0 + q % 3 - 1, jj = j0 + q / 3 - 1;
                const double ddx = (double)ii - xp, ddy = (double)jj - yp;
                const double phi = w[q] * (iv.i00 + iv.i01 * ddx + iv.i02 * ddy);
                const double dpx = w[q] * (iv.i01 + iv.i11 * ddx + iv.i12 * ddy);
                const double dpy = w[q] * (iv.i02 + iv.i12 * ddx + iv.i22 * ddy);
                const double rq = s_r[lm * 9 + q], uq = s_ux[lm * 9 + q], vq = s_uy[lm * 9 + q];
                rP += phi * rq;
                dudx += dpx * uq;
                dudy += dpy * uq;
                dvdx += dpx * vq;
                dvdy += dpy * vq;
            }
            const double pP = (rP - 1.0) / 3.0;
            const double txx = nu * (2.0 * dudx), txy = nu * (dudy + dvdx), tyy = nu * (2.0 * dvdy);
            const double alx = acc0 - alp * ry - Om * Om * rx;
            const double aly = acc1 + alp * rx - Om * Om * ry;
            const double pl = pP + dn * (alx * nxl + aly * nyl);
            const double tx = txx * nxl + txy * nyl - pl * nxl;
            const double ty = txy * nxl + tyy * nyl - pl * nyl;
            const double S = a.s.ds[mb + lg];
            // F = sum t S, M = sum (r x t) S
            const double ltx = S * (lFx - lM * ry), lty = S * (lFy + lM * rx);
            s_g[lm][4] += lFx * tx + lFy * ty + lM * (rx * ty - ry * tx);
            lrx = S * lM * ty;
            lry = -S * lM * tx;
            // t = tau n - p_l n
            const double ltxx = ltx * nxl, ltxy = ltx * nyl + lty * nxl, ltyy = lty * nyl;
            const double lpl = -(ltx * nxl + lty * nyl);
            lnx = ltx * (txx - pl) + lty * txy;
            lny = ltx * txy + lty * (tyy - pl);
            // p_l = p_P + dn (a_l . n), a_l = acc + alp z x r - Om^2 r
            lalx = dn * lpl * nxl;
            laly = dn * lpl * nyl;
            lnx += dn * lpl * alx;
            lny += dn * lpl * aly;
            c_alp = -ry * lalx + rx * laly;
            c_om = -2.0 * Om * (lalx * rx + laly * ry);
            lrx += -Om * Om * lalx + alp * laly;
            lry += -alp * lalx - Om * Om * laly;
            // p_P = (rho_P - 1)/3, tau = nu (grad u + grad u^T)
            s_sc[lm][0] = lpl / 3.0;
            s_sc[lm][1] = 2.0 * nu * ltxx;
            s_sc[lm][2] = nu * ltxy;
            s_sc[lm][3] = nu * ltxy;
            s_sc[lm][4] = 2.0 * nu * ltyy;
        }
        __syncthreads();
        // (3) per node: field terms for the patch and the share of S
        double p[3] = {1.0, 0.0, 0.0}, z[3] = {0.0, 0.0, 0.0}, y[3] = {0.0, 0.0, 0.0};
        double lp[3] = {0.0, 0.0, 0.0}, wk = 0.0;
        if (act) {
            const int2 an = s_anc[lo];
            const int ii = an.x + k % 3 - 1, jj = an.y + k / 3 - 1;
            double S9[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            s_dep[tid][0] = s_dep[tid][1] = s_dep[tid][2] = 0.0;
            if (node_valid(c, ii, jj)) {
                const double* B6 = s_B[lo];
                wk = s_w[tid];
                p[1] = (double)ii - s_xp[lo][0];
                p[2] = (double)jj - s_xp[lo][1];
                const double phi = wk * (B6[0] + B6[1] * p[1] + B6[2] * p[2]);
                const double dpx = wk * (B6[1] + B6[3] * p[1] + B6[4] * p[2]);
                const double dpy = wk * (B6[2] + B6[4] * p[1] + B6[5] * p[2]);
                const double lrP = s_sc[lo][0], ldudx = s_sc[lo][1], ldudy = s_sc[lo][2];
                const double ldvdx = s_sc[lo][3], ldvdy = s_sc[lo][4];
                s_dep[tid][0] = phi * lrP;
                s_dep[tid][1] = dpx * ldudx + dpy * ldudy;
                s_dep[tid][2] = dpx * ldvdx + dpy * ldvdy;
                const double rq = s_r[tid], uq = s_ux[tid], vq = s_uy[tid];
                lp[0] = lrP * rq;
                lp[1] = ldudx * uq + ldvdx * vq;
                lp[2] = ldudy * uq + ldvdy * vq;
                mls_share(B6, p, lp, wk, z, y, S9);
            }
#pragma unroll
            for (int e = 0; e < 9; ++e) s_S[tid][e] = S9[e];
        }
        __syncthreads();
        // (4) S of each marker (thread (marker, entry)); deposit the field terms
        if (act) {
            double Se = 0.0;
            for (int q = 0; q < 9; ++q) Se += s_S[lo * 9 + q][k];
            s_Sm[lo][k] = Se;
        }
        deposit_round<3, 0, 3, 3>(apatch, ax0u, ay0u, aw, ah, ncell, s_anc, s_mask, s_dep, min(kAdjRound, nm - r0), r0 == 0);
        __syncthreads();
        // (5) per node: its term of the derivative with respect to the probe
        if (act) {
            double ox = 0.0, oy = 0.0;
            if (wk != 0.0) mls_term(c, s_Sm[lo], p, z, y, lp, wk, ox, oy);
            s_S[tid][0] = ox;
            s_S[tid][1] = oy;
        }
        __syncthreads();
        // (6) per marker: probe position = X + r + dn n, r = R(th) xi, n = R(th) nu
        if (lead) {
            const int lm = tid, lg = r0 + lm;
            double lxp = 0.0, lyp = 0.0;
            for (int q = 0; q < 9; ++q) {
                lxp += s_S[lm * 9 + q][0];
                lyp += s_S[lm * 9 + q][1];
            }
            lrx += lxp;
            lry += lyp;
            lnx += dn * lxp;
            lny += dn * lyp;
            double* gk = a.gmk + (long long)(mb + lg) * 5;
            gk[0] = s_g[lm][0] + (cs * lrx + sn * lry);
            gk[1] = s_g[lm][1] + (-sn * lrx + cs * lry);
            gk[2] = s_g[lm][2] + (cs * lnx + sn * lny);
            gk[3] = s_g[lm][3] + (-sn * lnx + cs * lny);
            gk[4] = s_g[lm][4];
            s_pt[lm][0] = lxp;
            s_pt[lm][1] = lyp;
            s_pt[lm][2] = -nyl * lnx + nxl * lny - ry * lrx + rx * lry;
            s_pt[lm][3] = c_om;
            s_pt[lm][4] = lalx;
            s_pt[lm][5] = laly;
            s_pt[lm][6] = c_alp;
        }
        __syncthreads();
        // clear the round's anchor bits; running per-particle sums over the
        // markers, ascending
        if (act && k == 0 && ncell <= kAdjMaskCells) s_mask[(s_anc[lo].y - ay0u) * aw + (s_anc[lo].x - ax0u)] = 0ull;
        if (tid < 7) s_run[tid] = ordered_sum(s_run[tid], &s_pt[0][tid], min(kAdjRound, nm - r0), 8);
        __syncthreads();
    }
    if (tid == 0) {
        double* L = A->l;
        for (int j = 0; j < AL_N; ++j) L[j] = s_part[j];
        L[AL_X] += s_run[0];
        L[AL_X + 1] += s_run[1];
        L[AL_TH] += s_run[2];
        L[AL_OM] += s_run[3];
        L[AL_ACC] += s_run[4];
        L[AL_ACC + 1] += s_run[5];
        L[AL_ALP] += s_run[6];
    }
    // list the tiles the adjoint patch touches for the lattice pass (its
    // latency overlaps the end of the kernel)
    StepArgs sa = a.s;
    sa.tlist = a.atlist;
    mark_tiles(sa, c, (int)blockIdx.x, ax0u, ay0u, aw, ah, tid, blockDim.x);
}

template <int ST>
__global__ __launch_bounds__(kAdjThreads) void adj_traction_kernel(AdjArgs a) {
    __shared__ AdjTracLds sh;
    adj_traction_body<ST>(a, sh);
}

// ---------------------------------------------------------------------------
// Kernel B: adjoint of the immersed-boundary force and spreading.
// ---------------------------------------------------------------------------
// LDS of the immersed-boundary part of a reversed step.
struct AdjIbmLds {
    double w[kAdjThreads], usx[kAdjThreads], usy[kAdjThreads];
    double lfx[kAdjThreads], lfy[kAdjThreads];
    double dep[kAdjThreads][2];
    double S[kAdjThreads][9];
    double Sm[kAdjRound][9];
    double B[kAdjRound][6];
    double sc[kAdjRound][5];   // F (2), d/d U (2), c_l
    double xp[kAdjRound][2];
    double geo[kAdjRound][2];  // r of the marker
    double g[kAdjRound][5];    // its accumulated shape gradients
    double pt[kAdjRound][8];   // its particle terms
    int2 anc[kAdjRound];
    double run[8];
    int nb[kMaxNeighbours];
    NbBox box[kMaxNeighbours];
    unsigned long long mask[kAdjMaskCells];
};

template <int ST>
__device__ __forceinline__ void adj_ibm_body(const AdjArgs& a, AdjIbmLds& sh) {
    auto& s_w = sh.w;
    auto& s_usx = sh.usx;
    auto& s_usy = sh.usy;
    auto& s_lfx = sh.lfx;
    auto& s_lfy = sh.lfy;
    auto& s_dep = sh.dep;
    auto& s_S = sh.S;
    auto& s_Sm = sh.Sm;
    auto& s_B = sh.B;
    auto& s_sc = sh.sc;
    auto& s_xp = sh.xp;
    auto& s_geo = sh.geo;
    auto& s_g = sh.g;
    auto& s_pt = sh.pt;
    auto& s_anc = sh.anc;
    auto& s_run = sh.run;
    auto& s_nb = sh.nb;
    auto& s_box = sh.box;
    auto& s_mask = sh.mask;
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    if (b >= a.s.nparts) return;
    const PartDev* P = a.s.parts + b;
    AdjPart* A = a.ap + b;
    const ChanDev c = load_chan(a.s.chan + P->chan);  // in registers: not re-read after each barrier
    if (A->aw <= 0) return;
    const int nm = P->nm, mb = P->mbeg;
    const double X0 = P->X[0], X1 = P->X[1];
    const double Om = P->Om, V0 = P->V[0], V1 = P->V[1];
    const double cs = P->cth, sn = P->sth;
    // alone in its channel, the surface-stress part listed only the
    // particle itself: no dependent read of that list
    const bool alone = c.p_end - c.p_begin == 1;
    const int nnb = alone ? 1 : A->nnb;
    // marker geometry of the first round, requested early
    double2 pre_x = make_double2(0.0, 0.0);
    if (tid / 9 < kAdjRound && tid / 9 < nm) pre_x = a.s.xi[mb + tid / 9];
    if (tid < kMaxNeighbours) {
        const int q = alone ? b : A->nb[tid];
        s_nb[tid] = q;
        if (tid < nnb) {
            const PartDev& Q = a.s.parts[q];
            const AdjPart& QA = a.ap[q];
            NbBox& B = s_box[tid];
            B.fx0 = Q.bx0;
            B.fy0 = Q.by0;
            B.fw = Q.bw > 0 ? Q.bw : 0;
            B.fh = Q.bh;
            B.foff = Q.patch_off;
            B.ax0 = QA.ax0;
            B.ay0 = QA.ay0;
            B.aw = QA.aw;
            B.ah = QA.ah;
            B.aoff = QA.aoff;
        }
    }
    if (tid < 8) s_run[tid] = 0.0;
    int ax0u, ay0u, aw, ah;
    stencil_box(X0, X1, P->rb + c.dn, ax0u, ay0u, aw, ah);
    const int ncell = aw * ah;
    double* apatch = a.apatch + A->aoff * kAdjCell;
    for (int q = tid; q < min(ncell, kAdjMaskCells); q += blockDim.x) s_mask[q] = 0ull;
    __syncthreads();

    const int lo = tid / 9, k = tid % 9;
    for (int r0 = 0; r0 < nm; r0 += kAdjRound) {
        const int l = r0 + lo;
        const bool act = lo < kAdjRound && l < nm;
        const bool lead = tid < kAdjRound && r0 + tid < nm;
        // (1) one marker-stencil node per thread: u*, and d/d f_lb from the
        // transpose of the collision there (probe terms included)
        if (act) {
            Marker m;
            if (r0 == 0) {
                m.rx = cs * pre_x.x - sn * pre_x.y;
                m.ry = sn * pre_x.x + cs * pre_x.y;
                m.xl = X0 + m.rx;
                m.yl = X1 + m.ry;
                m.i0 = (int)floor(m.xl + 0.5);
                m.j0 = (int)floor(m.yl + 0.5);
            } else {
                m = marker_at(a.s, mb + l, X0, X1, cs, sn);
            }
            double dx, dy;
            int ni, nj;
            double w = 0.0, usx = 0.0, usy = 0.0, lfx = 0.0, lfy = 0.0;
            if (stencil_node(c, m.i0, m.j0, k, m.xl, m.yl, dx, dy, ni, nj)) {
                w = stencil_weight(c, dx, dy);
                // every load of the pair first (in-order completion makes
                // them one latency), the arithmetic after
                typename Sto<ST>::T raw[9];
                pull_load<ST>(a.s.fin, c, ni, nj, raw);
                double f[9], rho, jx, jy, fx, fy, t[kAdjCell], lfc[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) lfc[i] = lam_push<ST>(a.lam_in, c, i, ni, nj);
                // probe terms only: the marker terms are being written
                if (nnb <= kMaxNeighbours) patch_terms_lds<3>(a, c, s_box, nnb, ni, nj, fx, fy, t);
                else patch_terms<3>(a, c, s_nb, nnb, ni, nj, fx, fy, t);
                pull_finish_f64<ST>(a.s.fin, c, ni, nj, raw, f);
                moments_f64(f, c, rho, jx, jy);
                usx = jx / rho;
                usy = jy / rho;
                const double ux = (jx + 0.5 * fx) / rho, uy = (jy + 0.5 * fy) / rho;
                const CollAdj ca = collide_adj(lfc, rho, ux, uy, c.g[0] + fx, c.g[1] + fy, c.tau);
                const double lux = ca.lux + t[1], luy = ca.luy + t[2];
                lfx = lux / (2.0 * rho) + ca.lGx;
                lfy = luy / (2.0 * rho) + ca.lGy;
            }
            s_w[tid] = w;
            s_usx[tid] = usx;
            s_usy[tid] = usy;
            s_lfx[tid] = lfx;
            s_lfy[tid] = lfy;
            if (k == 0) {
                s_anc[lo] = make_int2(m.i0, m.j0);
                if (ncell <= kAdjMaskCells) atomicOr(&s_mask[(m.j0 - ay0u) * aw + (m.i0 - ax0u)], 1ull << lo);
                s_xp[lo][0] = m.xl;
                s_xp[lo][1] = m.yl;
                s_geo[lo][0] = m.rx;
                s_geo[lo][1] = m.ry;
            } else if (k == 1) {
                const double* gk = a.gmk + (long long)(mb + l) * 5;
                for (int e = 0; e < 5; ++e) s_g[lo][e] = gk[e];
            }
        }
        __syncthreads();
        // (2) per marker: MLS inverse
        if (lead) {
            const int lm = tid;
            const MlsInv iv = mls_inverse_adj(s_w + lm * 9, s_anc[lm].x, s_anc[lm].y, s_xp[lm][0], s_xp[lm][1]);
            s_B[lm][0] = iv.i00;
            s_B[lm][1] = iv.i01;
            s_B[lm][2] = iv.i02;
            s_B[lm][3] = iv.i11;
            s_B[lm][4] = iv.i12;
            s_B[lm][5] = iv.i22;
        }
        __syncthreads();
        // (3) per node: phi and its products
        double p[3] = {1.0, 0.0, 0.0}, phi = 0.0, wk = 0.0;
        if (act) {
            const int2 an = s_anc[lo];
            const int ii = an.x + k % 3 - 1, jj = an.y + k / 3 - 1;
            if (node_valid(c, ii, jj)) {
                const double* B6 = s_B[lo];
                wk = s_w[tid];
                p[1] = (double)ii - s_xp[lo][0];
                p[2] = (double)jj - s_xp[lo][1];
                phi = wk * (B6[0] + B6[1] * p[1] + B6[2] * p[2]);
            }
            s_S[tid][0] = phi * s_usx[tid];
            s_S[tid][1] = phi * s_usy[tid];
            s_S[tid][2] = phi * s_lfx[tid];
            s_S[tid][3] = phi * s_lfy[tid];
        }
        __syncthreads();
        // (4) per marker: U = sum phi u*, F = U_b - U, the adjoint of F_l
        // from f_lb = sum c_l phi F_l, and of U
        double lFx = 0.0, lFy = 0.0, mrx = 0.0, mry = 0.0;
        if (lead) {
            const int lm = tid, lg = r0 + lm;
            mrx = s_geo[lm][0];
            mry = s_geo[lm][1];
            double Ux = 0.0, Uy = 0.0, slx = 0.0, sly = 0.0;
            for (int q = 0; q < 9; ++q) {
                Ux += s_S[lm * 9 + q][0];
                Uy += s_S[lm * 9 + q][1];
                slx += s_S[lm * 9 + q][2];
                sly += s_S[lm * 9 + q][3];
            }
            const double cl = c.spread_unit ? 1.0 : a.s.ds[mb + lg];
            const double Fx = (V0 - Om * mry) - Ux, Fy = (V1 + Om * mrx) - Uy;
            lFx = cl * slx;
            lFy = cl * sly;
            if (!c.spread_unit) s_g[lm][4] += Fx * slx + Fy * sly;
            s_sc[lm][0] = Fx;
            s_sc[lm][1] = Fy;
            s_sc[lm][2] = -lFx;
            s_sc[lm][3] = -lFy;
            s_sc[lm][4] = cl;
        }
        __syncthreads();
        // (5) per node: d/d phi_k, the u* terms for the patch, share of S
        double z[3] = {0.0, 0.0, 0.0}, y[3] = {0.0, 0.0, 0.0}, lp[3] = {0.0, 0.0, 0.0};
        if (act) {
            double S9[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            const double Fx = s_sc[lo][0], Fy = s_sc[lo][1], lUx = s_sc[lo][2], lUy = s_sc[lo][3];
            s_dep[tid][0] = phi * lUx;
            s_dep[tid][1] = phi * lUy;
            if (wk != 0.0) {
                lp[0] = s_sc[lo][4] * (Fx * s_lfx[tid] + Fy * s_lfy[tid]) + lUx * s_usx[tid] + lUy * s_usy[tid];
                mls_share(s_B[lo], p, lp, wk, z, y, S9);
            }
#pragma unroll
            for (int e = 0; e < 9; ++e) s_S[tid][e] = S9[e];
        }
        __syncthreads();
        if (act) {
            double Se = 0.0;
            for (int q = 0; q < 9; ++q) Se += s_S[lo * 9 + q][k];
            s_Sm[lo][k] = Se;
        }
        deposit_round<2, 3, 2, kAdjCell>(apatch, ax0u, ay0u, aw, ah, ncell, s_anc, s_mask, s_dep, min(kAdjRound, nm - r0), r0 == 0);
        __syncthreads();
        if (act) {
            double ox = 0.0, oy = 0.0;
            if (wk != 0.0) mls_term(c, s_Sm[lo], p, z, y, lp, wk, ox, oy);
            s_S[tid][0] = ox;
            s_S[tid][1] = oy;
        }
        __syncthreads();
        // (6) per marker: x_l = X + r, U_b = V + Om z x r, r = R(th) xi
        if (lead) {
            const int lm = tid, lg = r0 + lm;
            double lx = 0.0, ly = 0.0;
            for (int q = 0; q < 9; ++q) {
                lx += s_S[lm * 9 + q][0];
                ly += s_S[lm * 9 + q][1];
            }
            const double lrx = Om * lFy + lx, lry = -Om * lFx + ly;
            double* gk = a.gmk + (long long)(mb + lg) * 5;
            gk[0] = s_g[lm][0] + (cs * lrx + sn * lry);
            gk[1] = s_g[lm][1] + (-sn * lrx + cs * lry);
            gk[2] = s_g[lm][2];
            gk[3] = s_g[lm][3];
            gk[4] = s_g[lm][4];
            s_pt[lm][0] = lx;
            s_pt[lm][1] = ly;
            s_pt[lm][2] = -mry * lrx + mrx * lry;
            s_pt[lm][3] = lFx;
            s_pt[lm][4] = lFy;
            s_pt[lm][5] = -mry * lFx + mrx * lFy;
        }
        __syncthreads();
        if (act && k == 0 && ncell <= kAdjMaskCells) s_mask[(s_anc[lo].y - ay0u) * aw + (s_anc[lo].x - ax0u)] = 0ull;
        if (tid < 6) s_run[tid] = ordered_sum(s_run[tid], &s_pt[0][tid], min(kAdjRound, nm - r0), 8);
        __syncthreads();
    }
    if (tid == 0) {
        double* L = A->l;
        L[AL_X] += s_run[0];
        L[AL_X + 1] += s_run[1];
        L[AL_TH] += s_run[2];
        L[AL_V] += s_run[3];
        L[AL_V + 1] += s_run[4];
        L[AL_OM] += s_run[5];
    }
}

template <int ST>
__global__ __launch_bounds__(kAdjThreads) void adj_ibm_kernel(AdjArgs a) {
    __shared__ AdjIbmLds sh;
    adj_ibm_body<ST>(a, sh);
}

// Kernels A and B as one launch, for handles whose channels hold at most one
// particle each.  A particle alone in its channel has no neighbour, so
// everything its IB part reads from the traction part (the probe terms of its
// adjoint patch, its adjoint box and neighbour list, the marker gradients and
// the particle adjoint) was written by its own workgroup before the barrier.
// The arithmetic and its order are those of the two launches; the LDS is
// shared between the parts.
template <int ST>
__global__ __launch_bounds__(kAdjThreads) void adj_particle_kernel(AdjArgs a) {
    __shared__ union {
        AdjTracLds t;
        AdjIbmLds i;
    } sh;
    adj_traction_body<ST>(a, sh.t);
    __syncthreads();
    adj_ibm_body<ST>(a, sh.i);
}

// ---------------------------------------------------------------------------
// Kernel C: the adjoint lattice pass.
// ---------------------------------------------------------------------------
// First accumulator of the wall node at (x, y) of a channel, or -1.
__device__ __forceinline__ long long wall_slot(const AdjArgs& a, int chan, const ChanDev& c, int x, int y,
                                               int& side) {
    const long long o = a.gw_off[chan];
    if (c.bcy == 1) {
        if (y == 0) { side = 2; return o + 2LL * x; }
        if (y == c.ny - 1) { side = 3; return o + 2LL * (c.nx + x); }
    }
    if (c.bcx == 1) {
        if (x == 0) { side = 0; return o + 2LL * y; }
        if (x == c.nx - 1) { side = 1; return o + 2LL * (c.ny + y); }
    }
    return -1;
}

// Density and velocities of a node: rho, u = (j + f/2)/rho and u* = j/rho.
struct NodeVel {
    double rho, ux, uy, usx, usy;
};

// Moments of node (x, y) from its raw pulled populations fr, with the walls
// applied on load.
__device__ __forceinline__ void adj_node_moments(const ChanDev& c, int x, int y, const double fr[9], double& rho,
                                                 double& jx, double& jy) {
    double f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = fr[i];
    walls_f64(c, c, x, y, f);
    moments_f64(f, c, rho, jx, jy);
}

__device__ __forceinline__ NodeVel node_vel(double rho, double jx, double jy, double fx, double fy) {
    NodeVel v;
    v.rho = rho;
    v.ux = (jx + 0.5 * fx) / rho;
    v.uy = (jy + 0.5 * fy) / rho;
    v.usx = jx / rho;
    v.usy = jy / rho;
    return v;
}

// The rest of the adjoint lattice update of node (x, y) of channel ch, from
// its raw pulled populations fr, its density and velocities, the adjoint
// populations L pushed to it (overwritten), the force (fx, fy) and the
// adjoint patch terms tt: the transposes of the collision and of the
// moments, and on wall nodes of the Zou-He closure; stores the node's
// adjoint populations.
template <int ST>
__device__ __forceinline__ void adj_node_finish(const AdjArgs& a, const ChanDev& c, int ch, int x, int y,
                                                const double fr[9], const NodeVel& v, double L[9], double fx,
                                                double fy, const double tt[kAdjCell]) {
    using LT = typename LamT<ST>::T;
    LT* __restrict__ lout = (LT*)a.lam_out;
    const double rho = v.rho, ux = v.ux, uy = v.uy, usx = v.usx, usy = v.usy;
    const CollAdj ca = collide_adj(L, rho, ux, uy, c.g[0] + fx, c.g[1] + fy, c.tau);
    // u = (j + f_lb/2)/rho, u* = j/rho, rho = sum f, j = sum f e + g/2
    const double lux = ca.lux + tt[1], luy = ca.luy + tt[2];
    const double ljx = (lux + tt[3]) / rho, ljy = (luy + tt[4]) / rho;
    const double lrho = ca.lrho + tt[0] - (lux * ux + luy * uy) / rho - (tt[3] * usx + tt[4] * usy) / rho;
    const double keep = 1.0 - 1.0 / c.tau;
#pragma unroll
    for (int i = 0; i < 9; ++i) L[i] = keep * L[i] + lrho + ljx * (double)ex(i) + ljy * (double)ey(i);
    int side = -1;
    const long long ws = wall_slot(a, ch, c, x, y, side);
    if (ws >= 0) {
        double gux = 0.0, guy = 0.0;
        // wall velocity by branches: a runtime index into the channel
        // descriptor would move it to scratch memory
        const double uwx = side == 0 ? c.uw[0][0] : (side == 1 ? c.uw[1][0] : (side == 2 ? c.uw[2][0] : c.uw[3][0]));
        const double uwy = side == 0 ? c.uw[0][1] : (side == 1 ? c.uw[1][1] : (side == 2 ? c.uw[2][1] : c.uw[3][1]));
        zouhe_adj(side, fr, L, uwx, uwy, c.g[0], c.g[1], gux, guy);
        a.gwall[ws] += gux;
        a.gwall[ws + 1] += guy;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) lout[pidx(c, i, y, x)] = (LT)L[i];
}

// The adjoint lattice update of node (x, y) of channel ch: adjoint
// streaming (the pushes of the next step's adjoint populations) and the
// force and adjoint patch terms of the listed particles (ascending), then
// adj_node_finish.
template <int ST>
__device__ __forceinline__ void adj_node(const AdjArgs& a, const ChanDev& c, int ch, const int* list, int nlist,
                                         int x, int y) {
    double fr[9];
    pull_raw_f64<ST>(a.s.fin, c, x, y, fr);
    double rho, jx, jy;
    adj_node_moments(c, x, y, fr, rho, jx, jy);
    double fx = 0.0, fy = 0.0, tt[kAdjCell] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (nlist > 0) patch_terms<kAdjCell>(a, c, list, nlist, x, y, fx, fy, tt);
    const NodeVel v = node_vel(rho, jx, jy, fx, fy);
    double L[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) L[i] = lam_push<ST>(a.lam_in, c, i, x, y);
    adj_node_finish<ST>(a, c, ch, x, y, fr, v, L, fx, fy, tt);
}

// The loads of one node of a particle's own adjoint box (cell q of the box),
// issued together: its pulled populations, the adjoint populations pushed
// to it, and its cells of the particle's force and adjoint patches, whose
// boxes are known.  The values and their sums are those of adj_node with
// the particle as the only listed one (patch_terms starts from zero and adds
// only inside a box).
struct BoxNode {
    int x, y;
    bool ok;
    double fr[9], L[9], fx, fy, tt[kAdjCell];
};

template <int ST>
__device__ __forceinline__ void box_node_load(const AdjArgs& a, const ChanDev& c, const PartDev& P,
                                              const AdjPart& A, int q, BoxNode& n) {
    int x = A.ax0 + q % A.aw, y = A.ay0 + q / A.aw;
    if (c.bcx == 0 && x >= c.nx) x -= c.nx;
    if (c.bcy == 0 && y >= c.ny) y -= c.ny;
    n.ok = x >= 0 && x < c.nx && y >= 0 && y < c.ny;
    // a node outside the channel reads node 0 and is not stored
    n.x = n.ok ? x : 0;
    n.y = n.ok ? y : 0;
    pull_raw_f64<ST>(a.s.fin, c, n.x, n.y, n.fr);
#pragma unroll
    for (int i = 0; i < 9; ++i) n.L[i] = lam_push<ST>(a.lam_in, c, i, n.x, n.y);
    const int cf = P.bw > 0 ? box_cell(c, P.bx0, P.by0, P.bw, P.bh, n.x, n.y) : -1;
    const double2 v = a.s.patch[P.patch_off + (cf >= 0 ? cf : 0)];
    n.fx = 0.0;
    n.fy = 0.0;
    if (cf >= 0) {
        n.fx += v.x;
        n.fy += v.y;
    }
    const double* va = a.apatch + (A.aoff + q) * kAdjCell;
#pragma unroll
    for (int k = 0; k < kAdjCell; ++k) {
        n.tt[k] = 0.0;
        n.tt[k] += va[k];
    }
}

// One wave per 64-node chunk of a tile (chunks = tile nodes / 64): the
// forward tile table and its particle lists are reused, and small lattices
// still spread over many compute units.
template <int ST>
__global__ __launch_bounds__(64) void adj_lattice_kernel(AdjArgs a, int tw, int chunks) {
    const int t = blockIdx.x / chunks, part = blockIdx.x % chunks;
    if (t >= a.s.ntiles) return;
    const int* tl_cur = a.atlist + (long long)a.s.parity * a.s.ntiles * kTileList;
    int* tl_next = a.atlist + (long long)(1 - a.s.parity) * a.s.ntiles * kTileList;
    const TileDev* tp = a.s.tiles + t;
    const int tx0 = uni(tp->x0), ty0 = uni(tp->y0), ch = uni(tp->chan);
    const ChanDev c = load_chan(a.s.chan + ch);
    const int* e = tl_cur + (long long)t * kTileList;
    const int cnt = uni(e[0]);
    int list[kMaxNeighbours];
    int nlist = 0;
    if (cnt > kTileList - 1) {
        nlist = kMaxNeighbours + 1;  // overflow: scan the channel's particles
    } else {
        for (int j = 0; j < cnt; ++j) {
            const int v = uni(e[1 + j]);
            bool dup = false;
            for (int m = 0; m < nlist; ++m) dup |= list[m] == v;
            if (dup) continue;
            int k = nlist;
            while (k > 0 && list[k - 1] > v) {
                list[k] = list[k - 1];
                --k;
            }
            list[k] = v;
            ++nlist;
        }
    }
    const int node = part * 64 + (int)threadIdx.x;
    const int x = tx0 + node % tw, y = ty0 + node / tw;
    if (x < c.nx && y < c.ny) adj_node<ST>(a, c, ch, list, nlist, x, y);
    // reset the other parity's list (read by no kernel of this step) for the
    // next reverse step
    if (part == 0 && threadIdx.x == 0) tl_next[(long long)t * kTileList] = 0;
}

// A whole reversed step as one launch, for handles whose channels hold at
// most one particle each and whose lattice is small enough that the launch
// is latency-bound.  The first nparts workgroups run the two particle
// kernels (as adj_particle_kernel) and then the adjoint lattice update of
// the nodes of their own adjoint box, whose patch terms they have just
// written.  The other workgroups take the 64-node chunks of the tiles, one
// wave each, from the start and skip the nodes of that box.  They find the
// box from the particle's taped state with the surface-stress part's own
// test, not from the adjoint state being written beside them.  The force
// patch lies inside the adjoint box (same centre, shorter reach), so a node
// outside it has neither force nor adjoint patch terms: the update of every
// node is bitwise that of adj_lattice_kernel.
template <int ST>
__global__ __launch_bounds__(kAdjThreads) void adj_step_kernel(AdjArgs a, int tw, int chunks) {
    __shared__ union {
        AdjTracLds t;
        AdjIbmLds i;
    } sh;
    const int b = blockIdx.x;
    if (b < a.s.nparts) {
        adj_traction_body<ST>(a, sh.t);
        __syncthreads();
        adj_ibm_body<ST>(a, sh.i);
        __syncthreads();
        // the nodes of the particle's adjoint box (aw = 0: none), two per
        // thread with all their loads issued before either's arithmetic
        const PartDev& P = a.s.parts[b];
        const AdjPart& A = a.ap[b];
        const int ch = P.chan;
        const ChanDev c = load_chan(a.s.chan + ch);
        const int ncell = A.aw * A.ah;
        for (int q = threadIdx.x; q < ncell; q += 2 * kAdjThreads) {
            const bool two = q + kAdjThreads < ncell;
            BoxNode n0, n1;
            box_node_load<ST>(a, c, P, A, q, n0);
            if (two) box_node_load<ST>(a, c, P, A, q + kAdjThreads, n1);
            if (n0.ok) {
                double rho, jx, jy;
                adj_node_moments(c, n0.x, n0.y, n0.fr, rho, jx, jy);
                const NodeVel v = node_vel(rho, jx, jy, n0.fx, n0.fy);
                adj_node_finish<ST>(a, c, ch, n0.x, n0.y, n0.fr, v, n0.L, n0.fx, n0.fy, n0.tt);
            }
            if (two && n1.ok) {
                double rho, jx, jy;
                adj_node_moments(c, n1.x, n1.y, n1.fr, rho, jx, jy);
                const NodeVel v = node_vel(rho, jx, jy, n1.fx, n1.fy);
                adj_node_finish<ST>(a, c, ch, n1.x, n1.y, n1.fr, v, n1.L, n1.fx, n1.fy, n1.tt);
            }
        }
        return;
    }
    const int gc = (b - a.s.nparts) * (kAdjThreads / 64) + (int)threadIdx.x / 64;
    const int t = gc / chunks, part = gc % chunks;
    if (t >= a.s.ntiles) return;
    int* tl_next = a.atlist + (long long)(1 - a.s.parity) * a.s.ntiles * kTileList;
    const TileDev* tp = a.s.tiles + t;
    const int tx0 = uni(tp->x0), ty0 = uni(tp->y0), ch = uni(tp->chan);
    const ChanDev c = load_chan(a.s.chan + ch);
    int bx0 = 0, by0 = 0, bw = 0, bh = 0;
    if (c.p_end > c.p_begin) {
        const int q = c.p_begin;
        const PartDev* P = a.s.parts + q;
        int ax0u, ay0u, aw, ah;
        stencil_box(P->X[0], P->X[1], P->rb + c.dn, ax0u, ay0u, aw, ah);
        if ((long long)aw * ah <= a.ap[q].acap && aw <= c.nx && ah <= c.ny) {
            bx0 = wrapc(ax0u, c.nx, c.bcx == 0);
            by0 = wrapc(ay0u, c.ny, c.bcy == 0);
            bw = aw;
            bh = ah;
        }
    }
    const int node = part * 64 + (int)threadIdx.x % 64;
    const int x = tx0 + node % tw, y = ty0 + node / tw;
    if (x < c.nx && y < c.ny && box_cell(c, bx0, by0, bw, bh, x, y) < 0)
        adj_node<ST>(a, c, ch, nullptr, 0, x, y);
    // reset the other parity's list for the next reverse step, as
    // adj_lattice_kernel does (the surface-stress part still fills this
    // step's list, so the two launch forms can follow each other)
    if (part == 0 && threadIdx.x % 64 == 0) tl_next[(long long)t * kTileList] = 0;
}

// ---------------------------------------------------------------------------
// Wall-speed gradients of one channel: the Couette start (Sec. 3.1)
// f^eq(1, u0(y)) with u0 linear between the y- and y+ wall speeds, then the
// per-node wall accumulators, all in ascending order.  out8 = [4][2].
// ---------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(256) void adj_finish_kernel(AdjArgs a, int chan, int with_init, double* out8) {
    using LT = typename LamT<ST>::T;
    const LT* lam = (const LT*)a.lam_in;
    const ChanDev c = a.s.chan[chan];
    const long long o = a.gw_off[chan];
    const long long nwall = c.bcy == 1 ? 2LL * c.nx : (c.bcx == 1 ? 2LL * c.ny : 0);
    double* rows = a.gwall + o + 2 * nwall;
    if (with_init) {
        const double lo = c.uw[2][0], hi = c.uw[3][0];
        for (int y = threadIdx.x; y < c.ny; y += blockDim.x) {
            const double u0 = lo + (hi - lo) * (double)y / (double)(c.ny - 1);
            double s = 0.0;
            for (int x = 0; x < c.nx; ++x)
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const double exi = (double)ex(i);
                    const double dfdu = wd(i) * (3.0 * exi + 9.0 * exi * u0 * exi - 3.0 * u0);
                    s += (double)lam[pidx(c, i, y, x)] * dfdu;
                }
            rows[y] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double g[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    if (c.bcy == 1) {
        for (int s = 0; s < 2; ++s)
            for (int x = 0; x < c.nx; ++x) {
                g[2 + s][0] += a.gwall[o + 2LL * (s * c.nx + x)];
                g[2 + s][1] += a.gwall[o + 2LL * (s * c.nx + x) + 1];
            }
    } else if (c.bcx == 1) {
        for (int s = 0; s < 2; ++s)
            for (int y = 0; y < c.ny; ++y) {
                g[s][0] += a.gwall[o + 2LL * (s * c.ny + y)];
                g[s][1] += a.gwall[o + 2LL * (s * c.ny + y) + 1];
            }
    }
    if (with_init) {
        for (int y = 0; y < c.ny; ++y) {
            const double t = (double)y / (double)(c.ny - 1);
            g[2][0] += rows[y] * (1.0 - t);
            g[3][0] += rows[y] * t;
        }
    }
    for (int s = 0; s < 4; ++s) {
        out8[2 * s] = g[s][0];
        out8[2 * s + 1] = g[s][1];
    }
}

// Adjoint populations of one channel as FP64 [9][ny][nx].
template <int ST>
__global__ void adj_field_kernel(AdjArgs a, int chan, double* out) {
    using LT = typename LamT<ST>::T;
    const LT* lam = (const LT*)a.lam_in;
    const ChanDev c = a.s.chan[chan];
    const long long n = (long long)c.nx * c.ny;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(t % c.nx), y = (int)(t / c.nx);
#pragma unroll
        for (int i = 0; i < 9; ++i) out[i * n + t] = (double)lam[pidx(c, i, y, x)];
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
#define ADJ_DISPATCH(store, F)                     \
    switch (store) {                               \
        case ST_F64: F(ST_F64); break;             \
        case ST_F32: F(ST_F32); break;             \
        default: F(ST_F16S); break;                \
    }

hipError_t launch_adj_traction(int store, const AdjArgs& a, hipStream_t s) {
    if (a.s.nparts <= 0) return hipSuccess;
#define L_(ST) adj_traction_kernel<ST><<<a.s.nparts, kAdjThreads, 0, s>>>(a)
    ADJ_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

hipError_t launch_adj_ibm(int store, const AdjArgs& a, hipStream_t s) {
    if (a.s.nparts <= 0) return hipSuccess;
#define L_(ST) adj_ibm_kernel<ST><<<a.s.nparts, kAdjThreads, 0, s>>>(a)
    ADJ_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

hipError_t launch_adj_particle(int store, const AdjArgs& a, hipStream_t s) {
    if (a.s.nparts <= 0) return hipSuccess;
#define L_(ST) adj_particle_kernel<ST><<<a.s.nparts, kAdjThreads, 0, s>>>(a)
    ADJ_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

hipError_t launch_adj_lattice(int store, const AdjArgs& a, hipStream_t s) {
    // one 64-node chunk per workgroup; tile widths are multiples of 64
    if (a.s.tile_w % 64 != 0 || a.s.tile_h < 1) return hipErrorInvalidValue;
    const int chunks = a.s.tile_w / 64 * a.s.tile_h;
    const long long grid = (long long)a.s.ntiles * chunks;
    if (grid <= 0) return hipSuccess;
    if (grid > INT_MAX) return hipErrorInvalidValue;
#define L_(ST) adj_lattice_kernel<ST><<<(int)grid, 64, 0, s>>>(a, a.s.tile_w, chunks)
    ADJ_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

int adj_step_workgroups(const AdjArgs& a) {
    if (a.s.tile_w % 64 != 0 || a.s.tile_h < 1) return -1;
    const long long chunks = (long long)a.s.ntiles * (a.s.tile_w / 64 * a.s.tile_h);
    const long long g = a.s.nparts + (chunks + kAdjThreads / 64 - 1) / (kAdjThreads / 64);
    return g > INT_MAX ? -1 : (int)g;
}

hipError_t launch_adj_step(int store, const AdjArgs& a, hipStream_t s) {
    const int grid = adj_step_workgroups(a);
    if (grid < 0) return hipErrorInvalidValue;
    if (grid == 0) return hipSuccess;
    const int chunks = a.s.tile_w / 64 * a.s.tile_h;
#define L_(ST) adj_step_kernel<ST><<<grid, kAdjThreads, 0, s>>>(a, a.s.tile_w, chunks)
    ADJ_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

hipError_t launch_adj_finish(int store, const AdjArgs& a, int chan, int with_init, double* out8,
                             hipStream_t s) {
#define L_(ST) adj_finish_kernel<ST><<<1, 256, 0, s>>>(a, chan, with_init, out8)
    ADJ_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

hipError_t launch_adj_field(int store, const AdjArgs& a, int chan, double* out, hipStream_t s) {
    const ChanDev* unused = nullptr;
    (void)unused;
    const int grid = 256;
#define L_(ST) adj_field_kernel<ST><<<grid, 256, 0, s>>>(a, chan, out)
    ADJ_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

}  // namespace lbmk
