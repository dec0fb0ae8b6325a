// gfx950 kernels of the discrete adjoint of the coupled LBM / MLS-IBM step.
//
// The forward step n maps (f^n, particle state P^n) to (f^{n+1}, P^{n+1})
// through the moments (Eqs. (6), (7)), the immersed-boundary force and its
// spreading (Eqs. (8)-(12)), the forced collision (Eqs. (4), (5)), the surface
// stress with force and moment (Eqs. (13), (14)), BDF2 (Eqs. (15), (16)),
// streaming and the Zou-He closure (App. A).  Its transpose runs as three
// kernels per step, in stream order:
//
//   adj_traction  one workgroup per particle: transpose of BDF2 and of the
//                 probe traction; the field terms (d/d rho and d/d u at the
//                 probe stencil nodes) go into the particle's adjoint patch.
//   adj_ibm       one workgroup per particle: adjoint of the IB force at the
//                 marker stencil nodes (it needs the collision transpose there),
//                 transpose of interpolation and spreading including the
//                 motion of the MLS weights with the markers; the d/d u* terms
//                 go into the adjoint patch.
//   adj_lattice   one workgroup per tile: adjoint streaming (a pull from
//                 x + e_i), transpose of the collision and of the moments with
//                 the patch terms added, transpose of the Zou-He closure on
//                 wall nodes, whose wall-speed derivatives accumulate per node.
//
// MLS stencil anchors are piecewise constant in the particle state and are
// held fixed, so this is the derivative of the smooth branch of the step.
// Field arithmetic is FP64; the adjoint populations are stored in FP64 for the
// FP64 form and in FP32 otherwise.  Every sum has a fixed order (no float
// atomics), so the adjoint is bitwise reproducible.
#include "lbm_device.h"

namespace lbmk {

template <int ST> struct LamT { using T = float; };
template <> struct LamT<ST_F64> { using T = double; };

// Adjoint of the population i pulled at (x, y) by the next step: the pull
// read the node x - e_i, so its adjoint is read at x + e_i.  Beyond a
// wall-bounded edge nothing was pulled: zero.
template <int ST>
__device__ __forceinline__ double lam_push(const void* lam, const ChanDev& c, int i, int x, int y) {
    int xd = x + ex(i), yd = y + ey(i);
    if (c.bcx == 0) xd = xd < 0 ? xd + c.nx : (xd >= c.nx ? xd - c.nx : xd);
    else if (xd < 0 || xd >= c.nx) return 0.0;
    if (c.bcy == 0) yd = yd < 0 ? yd + c.ny : (yd >= c.ny ? yd - c.ny : yd);
    else if (yd < 0 || yd >= c.ny) return 0.0;
    return (double)((const typename LamT<ST>::T*)lam)[pidx(c, i, yd, xd)];
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
    }
    const double h = 3.14159265358979323846 / 2.0;
    if (r < 1e-8) return -h * h / 4.0;
    return -0.25 * h * sin(h * r) / r;
}

// d/d(x, y) of sum_k lam_k . (phi_k, Dx_k, Dy_k), the MLS value and
// derivative weights of Eq. (8) at the point (x, y), anchors held fixed.
// With B = A^{-1}, z_k = B p_k, y_k = B lam_k and S = sum_k W_k z_k y_k^T:
//   d/dx_b = sum_k dW_k/dx_b (lam_k . z_k - p_k^T S p_k)
//          + sum_k W_k ((S^T p_k)_b + (S p_k)_b) - sum_k W_k (y_k)_b,
// b the x or y slot of p (dp_k/dx_b = -e_b).
__device__ __forceinline__ void mls_point_adj(const ChanDev& c, const double* w, const MlsInv& iv, int i0, int j0,
                              double x, double y, const double (*lam)[3], double& ox, double& oy) {
    const double B[3][3] = {{iv.i00, iv.i01, iv.i02}, {iv.i01, iv.i11, iv.i12}, {iv.i02, iv.i12, iv.i22}};
    double S[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int ii = i0 + q % 3 - 1, jj = j0 + q / 3 - 1;
        if (!node_valid(c, ii, jj)) continue;
        const double p[3] = {1.0, (double)ii - x, (double)jj - y};
        double z[3], yv[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            z[r] = B[r][0] * p[0] + B[r][1] * p[1] + B[r][2] * p[2];
            yv[r] = B[r][0] * lam[q][0] + B[r][1] * lam[q][1] + B[r][2] * lam[q][2];
        }
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int s = 0; s < 3; ++s) S[r][s] += w[q] * z[r] * yv[s];
    }
    const double irw2 = 1.0 / (c.rw * c.rw);
    ox = 0.0;
    oy = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int ii = i0 + q % 3 - 1, jj = j0 + q / 3 - 1;
        if (!node_valid(c, ii, jj)) continue;
        const double dx = (double)ii - x, dy = (double)jj - y;
        const double p[3] = {1.0, dx, dy};
        double z[3], yv[3], Sp[3], STp[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            z[r] = B[r][0] * p[0] + B[r][1] * p[1] + B[r][2] * p[2];
            yv[r] = B[r][0] * lam[q][0] + B[r][1] * lam[q][1] + B[r][2] * lam[q][2];
            Sp[r] = S[r][0] * p[0] + S[r][1] * p[1] + S[r][2] * p[2];
            STp[r] = S[0][r] * p[0] + S[1][r] * p[1] + S[2][r] * p[2];
        }
        const double lz = lam[q][0] * z[0] + lam[q][1] * z[1] + lam[q][2] * z[2];
        const double pSp = p[0] * Sp[0] + p[1] * Sp[1] + p[2] * Sp[2];
        const double r = sqrt(dx * dx + dy * dy) / c.rw;
        const double dw = kernel_dw(c.kernel, r, c.alpha);
        ox += -dw * dx * irw2 * (lz - pSp) + w[q] * (STp[1] + Sp[1]) - w[q] * yv[1];
        oy += -dw * dy * irw2 * (lz - pSp) + w[q] * (STp[2] + Sp[2]) - w[q] * yv[2];
    }
}

// Transpose of the forced collision of one node (Eqs. (4), (5)) at (rho, u, G)
// applied to the adjoint lfc of its outputs: the feq part of d/d rho, d/d u
// and d/d G.
struct CollAdj {
    double lrho, lux, luy, lGx, lGy;
};

__device__ __forceinline__ CollAdj collide_adj(const double lfc[9], double rho, double ux, double uy,
                                               double Gx, double Gy, double tau) {
    const double pref = 1.0 - 1.0 / (2.0 * tau);
    const double itau = 1.0 / tau;
    const double usq = ux * ux + uy * uy;
    CollAdj r{0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double exi = (double)ex(i), eyi = (double)ey(i), w = wd(i), a = lfc[i];
        const double eu = exi * ux + eyi * uy, eg = exi * Gx + eyi * Gy;
        r.lrho += a * w * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq) * itau;
        r.lux += a * (w * rho * (3.0 * exi + 9.0 * eu * exi - 3.0 * ux) * itau + pref * w * (-3.0 * Gx + 9.0 * exi * eg));
        r.luy += a * (w * rho * (3.0 * eyi + 9.0 * eu * eyi - 3.0 * uy) * itau + pref * w * (-3.0 * Gy + 9.0 * eyi * eg));
        r.lGx += a * pref * w * (3.0 * (exi - ux) + 9.0 * eu * exi);
        r.lGy += a * pref * w * (3.0 * (eyi - uy) + 9.0 * eu * eyi);
    }
    return r;
}

// Transpose of the Zou-He closure of zouhe_f64 at one wall node.  fr holds
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
// Kernel A: transpose of BDF2 and of the surface-stress force (one workgroup
// per particle, markers in rounds of 64, one thread per (marker, probe
// stencil node)).
// ---------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(kIbmThreads) void adj_traction_kernel(AdjArgs a) {
    __shared__ double s_w[kIbmThreads], s_r[kIbmThreads], s_ux[kIbmThreads], s_uy[kIbmThreads];
    __shared__ double s_dep[kIbmThreads][3];
    __shared__ int2 s_anc[kRound];
    __shared__ double s_part[AL_N], s_lF[3], s_sum[8];
    __shared__ int s_nb[kMaxNeighbours], s_nnb;
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    if (b >= a.s.nparts) return;
    const PartDev* P = a.s.parts + b;
    AdjPart* A = a.ap + b;
    const ChanDev& c = a.s.chan[P->chan];
    const int nm = P->nm, mb = P->mbeg;
    const double X0 = P->X[0], X1 = P->X[1], th = P->th, Om = P->Om;
    const double acc0 = P->acc[0], acc1 = P->acc[1], alp = P->alp;
    const double nu = c.nu, dn = c.dn;
    const double cs = cos(th), sn = sin(th);

    // adjoint patch box (covers probe and marker stencils)
    int ax0u, ay0u, aw, ah;
    stencil_box(X0, X1, P->rb + dn, ax0u, ay0u, aw, ah);
    const bool fits = (long long)aw * ah <= A->acap && aw <= c.nx && ah <= c.ny;
    if (tid == 0) {
        // BDF2 transpose (Eqs. (15), (16) with the position update): the
        // adjoint of the new velocity collects that of the new position.
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
    if (tid < 64) {
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
                if (pos < kMaxNeighbours) s_nb[pos] = q;
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
    for (int q = tid; q < ncell * kAdjCell; q += blockDim.x) apatch[q] = 0.0;
    {
        StepArgs sa = a.s;
        sa.tlist = a.atlist;
        mark_tiles(sa, c, ax0u, ay0u, aw, ah, tid, blockDim.x);
    }
    __syncthreads();
    const int nnb = s_nnb;
    const double lFx = s_lF[0], lFy = s_lF[1], lM = s_lF[2];

    const int lo = tid / 9, k = tid % 9;
    for (int r0 = 0; r0 < nm; r0 += kRound) {
        const int l = r0 + lo;
        if (l < nm) {
            const double2 x = a.s.xi[mb + l], nb = a.s.nrm[mb + l];
            const double rx = cs * x.x - sn * x.y, ry = sn * x.x + cs * x.y;
            const double nxl = cs * nb.x - sn * nb.y, nyl = sn * nb.x + cs * nb.y;
            const double xp = X0 + rx + dn * nxl, yp = X1 + ry + dn * nyl;
            const int i0 = (int)floor(xp + 0.5), j0 = (int)floor(yp + 0.5);
            double dx, dy;
            int ni, nj;
            double w = 0.0, rho = 1.0, ux = 0.0, uy = 0.0;
            if (stencil_node(c, i0, j0, k, xp, yp, dx, dy, ni, nj)) {
                w = stencil_weight(c, dx, dy);
                double f[9], jx, jy, fx, fy;
                pull_node_f64<ST>(a.s.fin, c, ni, nj, f);
                moments_f64(f, c, rho, jx, jy);
                fwd_force(a, c, s_nb, nnb, ni, nj, fx, fy);
                ux = (jx + 0.5 * fx) / rho;
                uy = (jy + 0.5 * fy) / rho;
            }
            s_w[tid] = w;
            s_r[tid] = rho;
            s_ux[tid] = ux;
            s_uy[tid] = uy;
            if (k == 0) s_anc[lo] = make_int2(i0, j0);
        }
        __syncthreads();
        if (tid < kRound && r0 + tid < nm) {
            const int lm = tid, l = r0 + lm;
            const double2 x = a.s.xi[mb + l], nb = a.s.nrm[mb + l];
            const double rx = cs * x.x - sn * x.y, ry = sn * x.x + cs * x.y;
            const double nxl = cs * nb.x - sn * nb.y, nyl = sn * nb.x + cs * nb.y;
            const double xp = X0 + rx + dn * nxl, yp = X1 + ry + dn * nyl;
            const int i0 = s_anc[lm].x, j0 = s_anc[lm].y;
            const double* w = s_w + lm * 9;
            const MlsInv iv = mls_inverse(c, w, i0, j0, xp, yp, true);
            double phi[9], dpx[9], dpy[9];
            double rP = 0.0, dudx = 0.0, dudy = 0.0, dvdx = 0.0, dvdy = 0.0;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int ii = i0 + q % 3 - 1, jj = j0 + q / 3 - 1;
                phi[q] = dpx[q] = dpy[q] = 0.0;
                if (!node_valid(c, ii, jj)) continue;
                const double ddx = (double)ii - xp, ddy = (double)jj - yp;
                phi[q] = w[q] * (iv.i00 + iv.i01 * ddx + iv.i02 * ddy);
                dpx[q] = w[q] * (iv.i01 + iv.i11 * ddx + iv.i12 * ddy);
                dpy[q] = w[q] * (iv.i02 + iv.i12 * ddx + iv.i22 * ddy);
                const double rq = s_r[lm * 9 + q], uq = s_ux[lm * 9 + q], vq = s_uy[lm * 9 + q];
                rP += phi[q] * rq;
                dudx += dpx[q] * uq;
                dudy += dpy[q] * uq;
                dvdx += dpx[q] * vq;
                dvdy += dpy[q] * vq;
            }
            const double pP = (rP - 1.0) / 3.0;
            const double txx = nu * (2.0 * dudx), txy = nu * (dudy + dvdx), tyy = nu * (2.0 * dvdy);
            const double alx = acc0 - alp * ry - Om * Om * rx;
            const double aly = acc1 + alp * rx - Om * Om * ry;
            const double pl = pP + dn * (alx * nxl + aly * nyl);
            const double tx = txx * nxl + txy * nyl - pl * nxl;
            const double ty = txy * nxl + tyy * nyl - pl * nyl;
            const double S = a.s.ds[mb + l];
            // transpose of F = sum t S, M = sum (r x t) S
            const double ltx = S * (lFx - lM * ry), lty = S * (lFy + lM * rx);
            double* gk = a.gmk + (long long)(mb + l) * 5;
            gk[4] += lFx * tx + lFy * ty + lM * (rx * ty - ry * tx);
            double lrx = S * lM * ty, lry = -S * lM * tx;
            // t = tau n - p_l n
            const double ltxx = ltx * nxl, ltxy = ltx * nyl + lty * nxl, ltyy = lty * nyl;
            const double lpl = -(ltx * nxl + lty * nyl);
            double lnx = ltx * (txx - pl) + lty * txy, lny = ltx * txy + lty * (tyy - pl);
            // p_l = p_P + dn (a_l . n), a_l = acc + alp z x r - Om^2 r
            const double lalx = dn * lpl * nxl, laly = dn * lpl * nyl;
            lnx += dn * lpl * alx;
            lny += dn * lpl * aly;
            const double c_alp = -ry * lalx + rx * laly;
            const double c_om = -2.0 * Om * (lalx * rx + laly * ry);
            lrx += -Om * Om * lalx + alp * laly;
            lry += -alp * lalx - Om * Om * laly;
            // p_P = (rho_P - 1)/3, tau = nu (grad u + grad u^T)
            const double lrP = lpl / 3.0;
            const double ldudx = 2.0 * nu * ltxx, ldudy = nu * ltxy, ldvdx = nu * ltxy, ldvdy = 2.0 * nu * ltyy;
            double lpsi[9][3];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const double rq = s_r[lm * 9 + q], uq = s_ux[lm * 9 + q], vq = s_uy[lm * 9 + q];
                s_dep[lm * 9 + q][0] = phi[q] * lrP;
                s_dep[lm * 9 + q][1] = dpx[q] * ldudx + dpy[q] * ldudy;
                s_dep[lm * 9 + q][2] = dpx[q] * ldvdx + dpy[q] * ldvdy;
                lpsi[q][0] = lrP * rq;
                lpsi[q][1] = ldudx * uq + ldvdx * vq;
                lpsi[q][2] = ldudy * uq + ldvdy * vq;
            }
            double lxp, lyp;
            mls_point_adj(c, w, iv, i0, j0, xp, yp, lpsi, lxp, lyp);
            lrx += lxp;
            lry += lyp;
            lnx += dn * lxp;
            lny += dn * lyp;
            // n = R(th) nu, r = R(th) xi
            gk[2] += cs * lnx + sn * lny;
            gk[3] += -sn * lnx + cs * lny;
            gk[0] += cs * lrx + sn * lry;
            gk[1] += -sn * lrx + cs * lry;
            const double c_th = -nyl * lnx + nxl * lny - ry * lrx + rx * lry;
            double* ps = a.pscr + (long long)(mb + l) * 8;
            ps[0] = lxp;
            ps[1] = lyp;
            ps[2] = c_th;
            ps[3] = c_om;
            ps[4] = lalx;
            ps[5] = laly;
            ps[6] = c_alp;
        }
        __syncthreads();
        // deposit the round's field terms, each cell summing its markers in
        // ascending order (the cell's thread is the same in every round)
        const int nr = min(kRound, nm - r0);
        for (int q = tid; q < ncell; q += blockDim.x) {
            const int cx = ax0u + q % aw, cy = ay0u + q / aw;
            double t0 = 0.0, t1 = 0.0, t2 = 0.0;
            for (int m = 0; m < nr; ++m) {
                const int2 an = s_anc[m];
                const int ddx = cx - an.x, ddy = cy - an.y;
                if (ddx < -1 || ddx > 1 || ddy < -1 || ddy > 1) continue;
                const int kk = 3 * (ddy + 1) + (ddx + 1);
                t0 += s_dep[m * 9 + kk][0];
                t1 += s_dep[m * 9 + kk][1];
                t2 += s_dep[m * 9 + kk][2];
            }
            double* v = apatch + (long long)q * kAdjCell;
            v[0] += t0;
            v[1] += t1;
            v[2] += t2;
        }
        __syncthreads();
    }
    // per-particle sums over the markers, ascending
    if (tid < 7) {
        double s = 0.0;
        for (int l = 0; l < nm; ++l) s += a.pscr[(long long)(mb + l) * 8 + tid];
        s_sum[tid] = s;
    }
    __syncthreads();
    if (tid == 0) {
        double* L = A->l;
        for (int j = 0; j < AL_N; ++j) L[j] = s_part[j];
        L[AL_X] += s_sum[0];
        L[AL_X + 1] += s_sum[1];
        L[AL_TH] += s_sum[2];
        L[AL_OM] += s_sum[3];
        L[AL_ACC] += s_sum[4];
        L[AL_ACC + 1] += s_sum[5];
        L[AL_ALP] += s_sum[6];
    }
}

// ---------------------------------------------------------------------------
// Kernel B: adjoint of the immersed-boundary force and spreading.
// ---------------------------------------------------------------------------
template <int ST>
__global__ __launch_bounds__(kIbmThreads) void adj_ibm_kernel(AdjArgs a) {
    __shared__ double s_w[kIbmThreads], s_usx[kIbmThreads], s_usy[kIbmThreads];
    __shared__ double s_lfx[kIbmThreads], s_lfy[kIbmThreads];
    __shared__ double s_dep[kIbmThreads][2];
    __shared__ int2 s_anc[kRound];
    __shared__ double s_sum[8];
    __shared__ int s_nb[kMaxNeighbours];
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    if (b >= a.s.nparts) return;
    const PartDev* P = a.s.parts + b;
    AdjPart* A = a.ap + b;
    const ChanDev& c = a.s.chan[P->chan];
    if (A->aw <= 0) return;
    const int nm = P->nm, mb = P->mbeg;
    const double X0 = P->X[0], X1 = P->X[1], th = P->th;
    const double Om = P->Om;
    const double cs = cos(th), sn = sin(th);
    const int nnb = A->nnb;
    if (tid < kMaxNeighbours) s_nb[tid] = A->nb[tid];
    int ax0u, ay0u, aw, ah;
    stencil_box(X0, X1, P->rb + c.dn, ax0u, ay0u, aw, ah);
    const int ncell = aw * ah;
    double* apatch = a.apatch + A->aoff * kAdjCell;
    __syncthreads();

    const int lo = tid / 9, k = tid % 9;
    for (int r0 = 0; r0 < nm; r0 += kRound) {
        const int l = r0 + lo;
        if (l < nm) {
            const Marker m = marker_at(a.s, mb + l, X0, X1, cs, sn);
            double dx, dy;
            int ni, nj;
            double w = 0.0, usx = 0.0, usy = 0.0, lfx = 0.0, lfy = 0.0;
            if (stencil_node(c, m.i0, m.j0, k, m.xl, m.yl, dx, dy, ni, nj)) {
                w = stencil_weight(c, dx, dy);
                double f[9], rho, jx, jy, fx, fy, t[kAdjCell], lfc[9];
                pull_node_f64<ST>(a.s.fin, c, ni, nj, f);
                moments_f64(f, c, rho, jx, jy);
                usx = jx / rho;
                usy = jy / rho;
                // probe terms only: the marker terms are being written
                patch_terms<3>(a, c, s_nb, nnb, ni, nj, fx, fy, t);
                const double ux = (jx + 0.5 * fx) / rho, uy = (jy + 0.5 * fy) / rho;
#pragma unroll
                for (int i = 0; i < 9; ++i) lfc[i] = lam_push<ST>(a.lam_in, c, i, ni, nj);
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
            if (k == 0) s_anc[lo] = make_int2(m.i0, m.j0);
        }
        __syncthreads();
        if (tid < kRound && r0 + tid < nm) {
            const int lm = tid, l = r0 + lm;
            const Marker m = marker_at(a.s, mb + l, X0, X1, cs, sn);
            const double cl = c.spread_unit ? 1.0 : a.s.ds[mb + l];
            const double* w = s_w + lm * 9;
            const MlsInv iv = mls_inverse(c, w, m.i0, m.j0, m.xl, m.yl, true);
            double phi[9];
            double Ux = 0.0, Uy = 0.0, slx = 0.0, sly = 0.0;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int ii = m.i0 + q % 3 - 1, jj = m.j0 + q / 3 - 1;
                phi[q] = 0.0;
                if (!node_valid(c, ii, jj)) continue;
                const double ddx = (double)ii - m.xl, ddy = (double)jj - m.yl;
                phi[q] = w[q] * (iv.i00 + iv.i01 * ddx + iv.i02 * ddy);
                Ux += phi[q] * s_usx[lm * 9 + q];
                Uy += phi[q] * s_usy[lm * 9 + q];
                slx += phi[q] * s_lfx[lm * 9 + q];
                sly += phi[q] * s_lfy[lm * 9 + q];
            }
            const double ubx = P->V[0] - Om * m.ry, uby = P->V[1] + Om * m.rx;
            const double Fx = ubx - Ux, Fy = uby - Uy;
            // f_lb = sum_l c_l phi_l F_l, F_l = U_b - sum phi u*
            const double lFx = cl * slx, lFy = cl * sly;
            double* gk = a.gmk + (long long)(mb + l) * 5;
            if (!c.spread_unit) gk[4] += Fx * slx + Fy * sly;
            const double lUx = -lFx, lUy = -lFy;
            double lpsi[9][3];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                lpsi[q][0] = cl * (Fx * s_lfx[lm * 9 + q] + Fy * s_lfy[lm * 9 + q]) +
                             lUx * s_usx[lm * 9 + q] + lUy * s_usy[lm * 9 + q];
                lpsi[q][1] = lpsi[q][2] = 0.0;
                s_dep[lm * 9 + q][0] = phi[q] * lUx;
                s_dep[lm * 9 + q][1] = phi[q] * lUy;
            }
            double lx, ly;
            mls_point_adj(c, w, iv, m.i0, m.j0, m.xl, m.yl, lpsi, lx, ly);
            // U_b = V + Om z x r, x_l = X + r, r = R(th) xi
            const double lrx = Om * lFy + lx, lry = -Om * lFx + ly;
            gk[0] += cs * lrx + sn * lry;
            gk[1] += -sn * lrx + cs * lry;
            double* ps = a.pscr + (long long)(mb + l) * 8;
            ps[0] = lx;
            ps[1] = ly;
            ps[2] = -m.ry * lrx + m.rx * lry;
            ps[3] = lFx;
            ps[4] = lFy;
            ps[5] = -m.ry * lFx + m.rx * lFy;
        }
        __syncthreads();
        const int nr = min(kRound, nm - r0);
        for (int q = tid; q < ncell; q += blockDim.x) {
            const int cx = ax0u + q % aw, cy = ay0u + q / aw;
            double t0 = 0.0, t1 = 0.0;
            for (int mm = 0; mm < nr; ++mm) {
                const int2 an = s_anc[mm];
                const int ddx = cx - an.x, ddy = cy - an.y;
                if (ddx < -1 || ddx > 1 || ddy < -1 || ddy > 1) continue;
                const int kk = 3 * (ddy + 1) + (ddx + 1);
                t0 += s_dep[mm * 9 + kk][0];
                t1 += s_dep[mm * 9 + kk][1];
            }
            double* v = apatch + (long long)q * kAdjCell;
            v[3] += t0;
            v[4] += t1;
        }
        __syncthreads();
    }
    if (tid < 6) {
        double s = 0.0;
        for (int l = 0; l < nm; ++l) s += a.pscr[(long long)(mb + l) * 8 + tid];
        s_sum[tid] = s;
    }
    __syncthreads();
    if (tid == 0) {
        double* L = A->l;
        L[AL_X] += s_sum[0];
        L[AL_X + 1] += s_sum[1];
        L[AL_TH] += s_sum[2];
        L[AL_V] += s_sum[3];
        L[AL_V + 1] += s_sum[4];
        L[AL_OM] += s_sum[5];
    }
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

template <int ST>
__global__ __launch_bounds__(256) void adj_lattice_kernel(AdjArgs a, int tw, int npt) {
    using LT = typename LamT<ST>::T;
    LT* __restrict__ lout = (LT*)a.lam_out;
    const int lx = threadIdx.x % tw, ly = threadIdx.x / tw;
    const int* tl_cur = a.atlist + (long long)a.s.parity * a.s.ntiles * kTileList;
    int* tl_next = a.atlist + (long long)(1 - a.s.parity) * a.s.ntiles * kTileList;
    for (int t = blockIdx.x; t < a.s.ntiles; t += gridDim.x) {
        const TileDev* tp = a.s.tiles + t;
        const int tx0 = uni(tp->x0), ty0 = uni(tp->y0), ch = uni(tp->chan);
        const ChanDev c = load_chan(a.s.chan + ch);
        const int* e = tl_cur + (long long)t * kTileList;
        const int cnt = uni(e[0]);
        if (threadIdx.x == 0) tl_next[(long long)t * kTileList] = 0;
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
        const int x = tx0 + lx;
        for (int r = 0; r < npt; ++r) {
            const int y = ty0 + ly * npt + r;
            if (x >= c.nx || y >= c.ny) continue;
            double fr[9], f[9];
            pull_raw_f64<ST>(a.s.fin, c, x, y, fr);
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = fr[i];
            walls_f64(c, x, y, f);
            double rho, jx, jy;
            moments_f64(f, c, rho, jx, jy);
            double fx = 0.0, fy = 0.0, tt[kAdjCell] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (nlist > 0) patch_terms<kAdjCell>(a, c, list, nlist, x, y, fx, fy, tt);
            const double ux = (jx + 0.5 * fx) / rho, uy = (jy + 0.5 * fy) / rho;
            const double usx = jx / rho, usy = jy / rho;
            double L[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) L[i] = lam_push<ST>(a.lam_in, c, i, x, y);
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
    }
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
#define L_(ST) adj_traction_kernel<ST><<<a.s.nparts, kIbmThreads, 0, s>>>(a)
    ADJ_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

hipError_t launch_adj_ibm(int store, const AdjArgs& a, hipStream_t s) {
    if (a.s.nparts <= 0) return hipSuccess;
#define L_(ST) adj_ibm_kernel<ST><<<a.s.nparts, kIbmThreads, 0, s>>>(a)
    ADJ_DISPATCH(store, L_)
#undef L_
    return hipGetLastError();
}

hipError_t launch_adj_lattice(int store, const AdjArgs& a, int tile_w, int npt, hipStream_t s) {
    const int grid = a.s.ntiles;
    if (grid <= 0) return hipSuccess;
#define L_(ST) adj_lattice_kernel<ST><<<grid, 256, 0, s>>>(a, tile_w, npt)
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
