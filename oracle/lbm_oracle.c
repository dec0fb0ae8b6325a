/*
 * Plain FP64 CPU oracle of the coupled LBM / MLS-IBM method (Coclite et al.).
 * TEST INFRASTRUCTURE ONLY: see lbm_oracle.h.
 *
 * One time step follows the paper's order (Sec. 1.2, last paragraph; Sec. 1.3):
 *   moments of f^n (Eqs. (6), (7))
 *   -> MLS interpolation of the velocity to the markers (Eqs. (8)-(10))
 *   -> Lagrangian force (Eq. (11)) and its spreading to the lattice (Eq. (12))
 *   -> forced BGK collision (Eqs. (2), (4), (5))
 *   -> surface-stress force and moment from normal probes (Eqs. (13), (14))
 *   -> BDF2 rigid-body update (Eqs. (15), (16))
 *   -> streaming (left-hand side of Eq. (4)) and Zou-He walls (Sec. 1.1).
 * Everything is serial and in the most literal loop order.  No blocking, no
 * fusion, no reordering beyond the summation order that reading R20 fixes.
 * Readings of silent or garbled passages (numbered as in the design notes):
 *   R1 viscosity nu = c_s^2 (tau - 1/2)  (the printed relation is garbled)
 *   R2 rho u = sum f e + G/2 with G the total body-force vector (Eq. (7))
 *   R3 the force-corrected u enters f^eq and the forcing term
 *   R4 Zou-He walls sit on the first/last node row or column; wall nodes
 *      collide like fluid nodes; the momentum target of the unknown
 *      populations is rho u_w - g/2 (g = uniform fluid body force)
 *   R5 MLS support: the 3x3 nodes around the nearest node (round half up),
 *      shifted linear basis (1, x_k - x, y_k - y); nodes beyond a wall-bounded
 *      edge are dropped
 *   R6 desired velocity U_b = rigid-body velocity at the marker; no density
 *      factor in F_l
 *   R7 c_l = S_l, from force conservation with dV_k = 1 and dV_l = S_l dx
 *   R8 markers sit on segment centres; S_l = segment length (2-D)
 *   R9 MLS derivatives are the linear coefficients of the fit at the probe
 *   R10 p_l = p_P + dn (a_l . n_l), from dp/dn = -rho0 a.n; a_l is the rigid
 *       acceleration of the marker lagged by one step
 *   R11 viscous stress tau = rho0 nu (grad u + grad u^T); r_l runs from the
 *       centroid to the marker
 *   R12 positions and angles use the same BDF2 with the new velocity; the
 *       history at the first step is the initial state; m = ratio * area,
 *       I = ratio * polar moment; gravity acts on the particle only, as
 *       (1 - rho_f/rho_s) g
 *   R13 F^n and M^n, computed from level-n fields, advance the particle from
 *       n to n+1 (weak coupling, Sec. 1.3)
 *   R14 the polynomial kernel of Eq. (20) is Peskin's four-point function
 *       evaluated at 2 r_k (its printed break points 0.5 and 1 are those of
 *       2 r_k = 1 and 2)
 *   R18 force and moment sums run over the markers in ascending order
 *   R20 the spread sum at a node is formed per particle in rounds of 64
 *       consecutive markers (see one_step)
 *   R23 closed boxes: a node on two walls takes the corner closure of
 *       apply_corners (walls at rest, no fluid body force)
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define Q 9
/* markers per round of the spreading order (reading R20) */
#define ORC_ROUND 64

/* ---------------------------------------------------------------------- */
/* D2Q9 lattice, Sec. 1.1, Eq. (3) and the weights that follow it.          */
/* The velocity set is evaluated from the printed cos/sin formula so the    */
/* numbering is the paper's, then rounded to the exact integers.            */
/* ---------------------------------------------------------------------- */
void orc_lattice(double e[9][2], double w[9]) {
    const double pi = 3.14159265358979323846;
    e[0][0] = 0.0;
    e[0][1] = 0.0;
    w[0] = 4.0 / 9.0;
    for (int i = 1; i <= 4; ++i) {
        e[i][0] = nearbyint(cos((i - 1) * pi / 2.0)) + 0.0; /* + 0.0 turns -0 into +0 */
        e[i][1] = nearbyint(sin((i - 1) * pi / 2.0)) + 0.0;
        w[i] = 1.0 / 9.0;
    }
    for (int i = 5; i <= 8; ++i) {
        e[i][0] = nearbyint(sqrt(2.0) * cos((2 * i - 9) * pi / 4.0)) + 0.0;
        e[i][1] = nearbyint(sqrt(2.0) * sin((2 * i - 9) * pi / 4.0)) + 0.0;
        w[i] = 1.0 / 36.0;
    }
}

static double E[9][2];
static double W[9];
static int lattice_ready = 0;
static void ensure_lattice(void) {
    if (!lattice_ready) {
        orc_lattice(E, W);
        lattice_ready = 1;
    }
}

/* Equilibrium, Eq. (2), with 1/c_s^2 = 3, 1/(2 c_s^4) = 4.5, 1/(2 c_s^2) = 1.5. */
void orc_equilibrium(double rho, double ux, double uy, double feq[9]) {
    ensure_lattice();
    double usq = ux * ux + uy * uy;
    for (int i = 0; i < Q; ++i) {
        double eu = E[i][0] * ux + E[i][1] * uy;
        feq[i] = W[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
    }
}

/* Forced BGK collision of one node: Eq. (4) with the Guo term of Eq. (5),
 * moments from Eqs. (6), (7) (readings R2, R3).  gx, gy: uniform fluid body
 * force; flbx, flby: IB force f_lb at the node. */
void orc_collide_node(const double f[9], double gx, double gy, double flbx, double flby,
                      double tau, double fc[9], double* rho_out, double* ux_out,
                      double* uy_out) {
    ensure_lattice();
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < Q; ++i) rho += f[i];
    for (int i = 0; i < Q; ++i) jx += f[i] * E[i][0];
    for (int i = 0; i < Q; ++i) jy += f[i] * E[i][1];
    jx += 0.5 * gx;
    jy += 0.5 * gy;
    double ux = (jx + 0.5 * flbx) / rho;
    double uy = (jy + 0.5 * flby) / rho;
    double Gx = gx + flbx;
    double Gy = gy + flby;
    double usq = ux * ux + uy * uy;
    double pref = 1.0 - 1.0 / (2.0 * tau);
    for (int i = 0; i < Q; ++i) {
        double ex = E[i][0], ey = E[i][1];
        double eu = ex * ux + ey * uy;
        double feq = W[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
        /* (e_i - u)/c_s^2 + (e_i . u) e_i / c_s^4, dotted with G */
        double Fi = pref * W[i] * ((3.0 * (ex - ux) + 9.0 * eu * ex) * Gx +
                                   (3.0 * (ey - uy) + 9.0 * eu * ey) * Gy);
        fc[i] = f[i] - (f[i] - feq) / tau + Fi;
    }
    if (rho_out) *rho_out = rho;
    if (ux_out) *ux_out = ux;
    if (uy_out) *uy_out = uy;
}

/* Zou-He known-velocity wall (Sec. 1.1, reading R4).  The unknown populations
 * are those streaming into the domain.  Density comes from the mass and
 * normal-momentum constraints; the unknown normal population is fixed by
 * bounce-back of its non-equilibrium part; the two unknown diagonals by the
 * tangential momentum constraint.  Target momentum m = rho u_w - g/2. */
void orc_zouhe(int side, double f[9], double uwx, double uwy, double gx, double gy) {
    double rho, mx, my;
    switch (side) {
        case ORC_SIDE_YLO: /* unknown 2, 5, 6 */
            rho = (f[0] + f[1] + f[3] + 2.0 * (f[4] + f[7] + f[8]) - 0.5 * gy) / (1.0 - uwy);
            mx = rho * uwx - 0.5 * gx;
            my = rho * uwy - 0.5 * gy;
            f[2] = f[4] + 2.0 * my / 3.0;
            f[5] = f[7] - 0.5 * (f[1] - f[3]) + 0.5 * mx + my / 6.0;
            f[6] = f[8] + 0.5 * (f[1] - f[3]) - 0.5 * mx + my / 6.0;
            break;
        case ORC_SIDE_YHI: /* unknown 4, 7, 8 */
            rho = (f[0] + f[1] + f[3] + 2.0 * (f[2] + f[5] + f[6]) + 0.5 * gy) / (1.0 + uwy);
            mx = rho * uwx - 0.5 * gx;
            my = rho * uwy - 0.5 * gy;
            f[4] = f[2] - 2.0 * my / 3.0;
            f[7] = f[5] + 0.5 * (f[1] - f[3]) - 0.5 * mx - my / 6.0;
            f[8] = f[6] - 0.5 * (f[1] - f[3]) + 0.5 * mx - my / 6.0;
            break;
        case ORC_SIDE_XLO: /* unknown 1, 5, 8 */
            rho = (f[0] + f[2] + f[4] + 2.0 * (f[3] + f[6] + f[7]) - 0.5 * gx) / (1.0 - uwx);
            mx = rho * uwx - 0.5 * gx;
            my = rho * uwy - 0.5 * gy;
            f[1] = f[3] + 2.0 * mx / 3.0;
            f[5] = f[7] - 0.5 * (f[2] - f[4]) + mx / 6.0 + 0.5 * my;
            f[8] = f[6] + 0.5 * (f[2] - f[4]) + mx / 6.0 - 0.5 * my;
            break;
        default: /* ORC_SIDE_XHI: unknown 3, 6, 7 */
            rho = (f[0] + f[2] + f[4] + 2.0 * (f[1] + f[5] + f[8]) + 0.5 * gx) / (1.0 + uwx);
            mx = rho * uwx - 0.5 * gx;
            my = rho * uwy - 0.5 * gy;
            f[3] = f[1] - 2.0 * mx / 3.0;
            f[7] = f[5] + 0.5 * (f[2] - f[4]) - mx / 6.0 - 0.5 * my;
            f[6] = f[8] - 0.5 * (f[2] - f[4]) - mx / 6.0 + 0.5 * my;
            break;
    }
}

/* Interpolation kernels: exponential, Eq. (10); cubic, quartic and cosine,
 * Eqs. (17)-(19); polynomial, Eq. (20) under reading R14: its two branches
 * are evaluated at q = 2 r, the first for q <= 1, the second for 1 < q <= 2.
 * r is the distance normalised by r_w. */
double orc_kernel_weight(int kind, double r, double alpha) {
    if (r > 1.0) return 0.0;
    switch (kind) {
        case ORC_W_POLY: {
            double q = 2.0 * r;
            if (q <= 1.0) return (3.0 - 2.0 * q + sqrt(1.0 + 4.0 * q - 4.0 * q * q)) / 8.0;
            return (5.0 - 2.0 * q - sqrt(-7.0 + 12.0 * q - 4.0 * q * q)) / 8.0;
        }
        case ORC_W_EXP: {
            double q = r / alpha;
            return exp(-(q * q));
        }
        case ORC_W_CUBIC:
            return 2.0 / 3.0 - 4.0 * r * r + 4.0 * r * r * r;
        case ORC_W_QUARTIC:
            return 1.0 - 6.0 * r * r + 8.0 * r * r * r - 3.0 * r * r * r * r;
        case ORC_W_COSINE:
            return 0.25 * (1.0 + cos(3.14159265358979323846 / 2.0 * r));
        default:
            return NAN;
    }
}

/* MLS transfer operator at point (x, y): Sec. 1.2, Eqs. (8)-(10), readings R5,
 * R9.  Minimising Eq. (9) with p = (1, x_k - x, y_k - y) gives the normal
 * equations A a = sum_k W_k p_k u_k with A = sum_k W_k p_k p_k^T, so
 * phi_k = W_k [A^{-1} p_k]_0, and the linear coefficients of the fit give the
 * derivative weights W_k [A^{-1} p_k]_{1,2}.  A is inverted through its
 * adjugate (A is symmetric positive definite for >= 3 non-collinear nodes). */
int orc_mls(const orc_config* cfg, double x, double y, int32_t node_i[9], int32_t node_j[9],
            int32_t valid[9], double phi[9], double dphx[9], double dphy[9]) {
    int i0 = (int)floor(x + 0.5);
    int j0 = (int)floor(y + 0.5);
    double dx[9], dy[9], wk[9];
    double A00 = 0.0, A01 = 0.0, A02 = 0.0, A11 = 0.0, A12 = 0.0, A22 = 0.0;
    int nvalid = 0;
    int k = 0;
    for (int b = -1; b <= 1; ++b) {
        for (int a = -1; a <= 1; ++a, ++k) {
            int ii = i0 + a, jj = j0 + b;
            dx[k] = (double)ii - x;
            dy[k] = (double)jj - y;
            int ok = 1;
            if (cfg->bc_x == ORC_PERIODIC) {
                ii %= cfg->nx;
                if (ii < 0) ii += cfg->nx;
            } else if (ii < 0 || ii >= cfg->nx) {
                ok = 0;
            }
            if (cfg->bc_y == ORC_PERIODIC) {
                jj %= cfg->ny;
                if (jj < 0) jj += cfg->ny;
            } else if (jj < 0 || jj >= cfg->ny) {
                ok = 0;
            }
            node_i[k] = ii;
            node_j[k] = jj;
            valid[k] = ok;
            wk[k] = 0.0;
            if (!ok) continue;
            double r = sqrt(dx[k] * dx[k] + dy[k] * dy[k]) / cfg->mls_rw;
            wk[k] = orc_kernel_weight(cfg->mls_kernel, r, cfg->mls_alpha);
            A00 += wk[k];
            A01 += wk[k] * dx[k];
            A02 += wk[k] * dy[k];
            A11 += wk[k] * dx[k] * dx[k];
            A12 += wk[k] * dx[k] * dy[k];
            A22 += wk[k] * dy[k] * dy[k];
            ++nvalid;
        }
    }
    double c00 = A11 * A22 - A12 * A12;
    double c01 = A02 * A12 - A01 * A22;
    double c02 = A01 * A12 - A02 * A11;
    double c11 = A00 * A22 - A02 * A02;
    double c12 = A01 * A02 - A00 * A12;
    double c22 = A00 * A11 - A01 * A01;
    double det = A00 * c00 + A01 * c01 + A02 * c02;
    double i00 = c00 / det, i01 = c01 / det, i02 = c02 / det;
    double i11 = c11 / det, i12 = c12 / det, i22 = c22 / det;
    for (k = 0; k < 9; ++k) {
        if (!valid[k]) {
            phi[k] = 0.0;
            dphx[k] = 0.0;
            dphy[k] = 0.0;
            continue;
        }
        phi[k] = wk[k] * (i00 + i01 * dx[k] + i02 * dy[k]);
        dphx[k] = wk[k] * (i01 + i11 * dx[k] + i12 * dy[k]);
        dphy[k] = wk[k] * (i02 + i12 * dx[k] + i22 * dy[k]);
    }
    return nvalid;
}

/* BDF2 ("explicit second-order Euler"), Eqs. (15), (16), dt = 1, and the
 * same scheme for the position with the new velocity (reading R13). */
void orc_bdf2(double v, double vm, double acc, double x, double xm, double* v_new,
              double* x_new) {
    double vn = 2.0 / 3.0 * (2.0 * v - 0.5 * vm + acc);
    *v_new = vn;
    *x_new = 2.0 / 3.0 * (2.0 * x - 0.5 * xm + vn);
}

/* ---------------------------------------------------------------------- */
/* Simulation state                                                        */
/* ---------------------------------------------------------------------- */
typedef struct {
    double X[2], Xm[2], th, thm;
    double V[2], Vm[2], Om, Omm;
    double acc[2], alp; /* accelerations of the previous step (R10) */
    double F[2], M;
    double m, I, ratio;
    int nm;
    double *xi, *nu, *ds;
    double* rec; /* [nm][8] marker record of the last step */
} particle;

struct orc_sim {
    orc_config cfg;
    int nx, ny;
    size_t n;
    double *f, *fc, *rho, *jx, *jy, *ux, *uy, *flbx, *flby;
    /* spreading order (reading R20): one round's sums, one particle's sums,
     * the nodes each has touched and their markers */
    double *rfx, *rfy, *pfx, *pfy;
    int32_t *rlist, *plist;
    unsigned char *rmark, *pmark;
    int np, cap;
    particle* p;
    uint64_t anchor_hash;
    int steps_done;
    int threads; /* threads of the node loops (1 unless orc_set_threads) */
};

static size_t idx(const orc_sim* s, int i, int y, int x) {
    return ((size_t)i * s->ny + (size_t)y) * s->nx + (size_t)x;
}

static int wall_side_count(const orc_config* c) {
    return (c->bc_x == ORC_ZOUHE) + (c->bc_y == ORC_ZOUHE);
}

/* Closed-box corners (reading R23, walls at rest, no fluid body force).  A
 * corner node lies on two walls, so five of its populations stream in from
 * outside.  The three that point into the fluid along a wall normal or the
 * corner diagonal take the bounce-back of their opposites; the two buried
 * diagonal ones (parallel to neither wall normal) share what the density
 * rho_c of the diagonal interior neighbour leaves after the other seven.
 * (x, y): the corner; (x + sx, y + sy): its diagonal interior neighbour;
 * in1..in3 / out1..out3: the unknown populations and their opposites;
 * b1, b2: the buried pair. */
static void corner_closure(orc_sim* s, int x, int y, int sx, int sy) {
    double f[9], rc = 0.0;
    for (int i = 0; i < Q; ++i) f[i] = s->f[idx(s, i, y, x)];
    for (int i = 0; i < Q; ++i) rc += s->f[idx(s, i, y + sy, x + sx)];
    /* unknown: the axis population pointing into the fluid along x and
     * along y, and the diagonal pointing into the fluid */
    int ix = sx > 0 ? 1 : 3, iy = sy > 0 ? 2 : 4;
    int id = sx > 0 ? (sy > 0 ? 5 : 8) : (sy > 0 ? 6 : 7);
    int b1 = sx == sy ? 6 : 5, b2 = sx == sy ? 8 : 7; /* the buried pair */
    static const int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    f[ix] = f[opp[ix]];
    f[iy] = f[opp[iy]];
    f[id] = f[opp[id]];
    double rest = 0.0;
    for (int i = 0; i < Q; ++i)
        if (i != b1 && i != b2) rest += f[i];
    double b = 0.5 * (rc - rest);
    f[b1] = b;
    f[b2] = b;
    for (int i = 0; i < Q; ++i) s->f[idx(s, i, y, x)] = f[i];
}

static void apply_walls(orc_sim* s) {
    const orc_config* c = &s->cfg;
    double fl[9];
    double gx = c->body_force[0], gy = c->body_force[1];
    /* with walls on both axes the four corner nodes take the corner closure */
    const int box = c->bc_x == ORC_ZOUHE && c->bc_y == ORC_ZOUHE;
    if (c->bc_y == ORC_ZOUHE) {
        for (int side = ORC_SIDE_YLO; side <= ORC_SIDE_YHI; ++side) {
            int y = side == ORC_SIDE_YLO ? 0 : s->ny - 1;
            for (int x = box; x < s->nx - box; ++x) {
                for (int i = 0; i < Q; ++i) fl[i] = s->f[idx(s, i, y, x)];
                orc_zouhe(side, fl, c->u_wall[side][0], c->u_wall[side][1], gx, gy);
                for (int i = 0; i < Q; ++i) s->f[idx(s, i, y, x)] = fl[i];
            }
        }
    }
    if (c->bc_x == ORC_ZOUHE) {
        for (int side = ORC_SIDE_XLO; side <= ORC_SIDE_XHI; ++side) {
            int x = side == ORC_SIDE_XLO ? 0 : s->nx - 1;
            for (int y = box; y < s->ny - box; ++y) {
                for (int i = 0; i < Q; ++i) fl[i] = s->f[idx(s, i, y, x)];
                orc_zouhe(side, fl, c->u_wall[side][0], c->u_wall[side][1], gx, gy);
                for (int i = 0; i < Q; ++i) s->f[idx(s, i, y, x)] = fl[i];
            }
        }
    }
    if (box) {
        corner_closure(s, 0, 0, 1, 1);
        corner_closure(s, s->nx - 1, 0, -1, 1);
        corner_closure(s, 0, s->ny - 1, 1, -1);
        corner_closure(s, s->nx - 1, s->ny - 1, -1, -1);
    }
}

orc_sim* orc_create(const orc_config* cfg) {
    ensure_lattice();
    if (!cfg) return NULL;
    if (cfg->nx < 3 || cfg->ny < 3) return NULL;
    if (!(cfg->tau > 0.5) || !isfinite(cfg->tau)) return NULL;
    if ((cfg->bc_x != ORC_PERIODIC && cfg->bc_x != ORC_ZOUHE) ||
        (cfg->bc_y != ORC_PERIODIC && cfg->bc_y != ORC_ZOUHE))
        return NULL;
    if (wall_side_count(cfg) > 1) { /* closed box: walls at rest, no fluid force (R23) */
        for (int k = 0; k < 4; ++k)
            if (cfg->u_wall[k][0] != 0.0 || cfg->u_wall[k][1] != 0.0) return NULL;
        if (cfg->body_force[0] != 0.0 || cfg->body_force[1] != 0.0) return NULL;
    }
    if (cfg->init == ORC_INIT_COUETTE && cfg->bc_y != ORC_ZOUHE) return NULL;
    if (cfg->mls_kernel < ORC_W_EXP || cfg->mls_kernel > ORC_W_POLY) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->cfg = *cfg;
    s->nx = cfg->nx;
    s->ny = cfg->ny;
    s->n = (size_t)cfg->nx * cfg->ny;
    s->f = (double*)calloc(Q * s->n, sizeof(double));
    s->fc = (double*)calloc(Q * s->n, sizeof(double));
    s->rho = (double*)calloc(s->n, sizeof(double));
    s->jx = (double*)calloc(s->n, sizeof(double));
    s->jy = (double*)calloc(s->n, sizeof(double));
    s->ux = (double*)calloc(s->n, sizeof(double));
    s->uy = (double*)calloc(s->n, sizeof(double));
    s->flbx = (double*)calloc(s->n, sizeof(double));
    s->flby = (double*)calloc(s->n, sizeof(double));
    s->rfx = (double*)calloc(s->n, sizeof(double));
    s->rfy = (double*)calloc(s->n, sizeof(double));
    s->pfx = (double*)calloc(s->n, sizeof(double));
    s->pfy = (double*)calloc(s->n, sizeof(double));
    s->rlist = (int32_t*)calloc(s->n, sizeof(int32_t));
    s->plist = (int32_t*)calloc(s->n, sizeof(int32_t));
    s->rmark = (unsigned char*)calloc(s->n, 1);
    s->pmark = (unsigned char*)calloc(s->n, 1);
    s->anchor_hash = 1469598103934665603ULL;
    s->threads = 1;
    /* Initial populations: f^eq(1, u0) (Sec. 3.1: planar Couette start), then
     * the wall reconstruction so f^0 satisfies the boundary conditions. */
    double feq[9];
    for (int y = 0; y < s->ny; ++y) {
        for (int x = 0; x < s->nx; ++x) {
            double u0x = 0.0, u0y = 0.0;
            if (cfg->init == ORC_INIT_COUETTE) {
                double lo = cfg->u_wall[ORC_SIDE_YLO][0], hi = cfg->u_wall[ORC_SIDE_YHI][0];
                u0x = lo + (hi - lo) * (double)y / (double)(s->ny - 1);
            }
            orc_equilibrium(1.0, u0x, u0y, feq);
            for (int i = 0; i < Q; ++i) s->f[idx(s, i, y, x)] = feq[i];
        }
    }
    apply_walls(s);
    return s;
}

void orc_destroy(orc_sim* s) {
    if (!s) return;
    for (int p = 0; p < s->np; ++p) {
        free(s->p[p].xi);
        free(s->p[p].nu);
        free(s->p[p].ds);
        free(s->p[p].rec);
    }
    free(s->p);
    free(s->f);
    free(s->fc);
    free(s->rho);
    free(s->jx);
    free(s->jy);
    free(s->ux);
    free(s->uy);
    free(s->flbx);
    free(s->flby);
    free(s->rfx);
    free(s->rfy);
    free(s->pfx);
    free(s->pfy);
    free(s->rlist);
    free(s->plist);
    free(s->rmark);
    free(s->pmark);
    free(s);
}

int orc_add_particle(orc_sim* s, const orc_particle_desc* d) {
    if (!s || !d || d->n_markers < 3 || !(d->density_ratio > 0.0) || !(d->area > 0.0) ||
        !(d->polar_moment > 0.0))
        return -1;
    if (s->np == s->cap) {
        s->cap = s->cap ? 2 * s->cap : 4;
        s->p = (particle*)realloc(s->p, (size_t)s->cap * sizeof(particle));
    }
    particle* p = &s->p[s->np];
    memset(p, 0, sizeof(*p));
    p->X[0] = p->Xm[0] = d->x;
    p->X[1] = p->Xm[1] = d->y;
    p->th = p->thm = d->theta;
    p->V[0] = p->Vm[0] = d->u;
    p->V[1] = p->Vm[1] = d->v;
    p->Om = p->Omm = d->omega;
    p->ratio = d->density_ratio;
    p->m = d->density_ratio * d->area;
    p->I = d->density_ratio * d->polar_moment;
    p->nm = d->n_markers;
    p->xi = (double*)malloc(sizeof(double) * 2 * p->nm);
    p->nu = (double*)malloc(sizeof(double) * 2 * p->nm);
    p->ds = (double*)malloc(sizeof(double) * p->nm);
    p->rec = (double*)calloc((size_t)8 * p->nm, sizeof(double));
    memcpy(p->xi, d->xi, sizeof(double) * 2 * p->nm);
    memcpy(p->nu, d->nrm, sizeof(double) * 2 * p->nm);
    memcpy(p->ds, d->ds, sizeof(double) * p->nm);
    return s->np++;
}

int orc_n_particles(const orc_sim* s) { return s->np; }

static void particle_record(const particle* p, double* out) {
    out[0] = p->X[0];
    out[1] = p->X[1];
    out[2] = p->th;
    out[3] = p->V[0];
    out[4] = p->V[1];
    out[5] = p->Om;
    out[6] = p->F[0];
    out[7] = p->F[1];
    out[8] = p->M;
    out[9] = 0.0;
}

void orc_get_particles(const orc_sim* s, double* out) {
    for (int p = 0; p < s->np; ++p) particle_record(&s->p[p], out + (size_t)p * ORC_PSTATE);
}

void orc_get_populations(const orc_sim* s, double* f) {
    memcpy(f, s->f, sizeof(double) * Q * s->n);
}
void orc_set_populations(orc_sim* s, const double* f) {
    memcpy(s->f, f, sizeof(double) * Q * s->n);
}

void orc_get_fields(const orc_sim* s, double* rho, double* ux, double* uy) {
    double gx = s->cfg.body_force[0], gy = s->cfg.body_force[1];
    for (int y = 0; y < s->ny; ++y) {
        for (int x = 0; x < s->nx; ++x) {
            double r = 0.0, jx = 0.0, jy = 0.0;
            for (int i = 0; i < Q; ++i) r += s->f[idx(s, i, y, x)];
            for (int i = 0; i < Q; ++i) jx += s->f[idx(s, i, y, x)] * E[i][0];
            for (int i = 0; i < Q; ++i) jy += s->f[idx(s, i, y, x)] * E[i][1];
            jx += 0.5 * gx;
            jy += 0.5 * gy;
            size_t n = (size_t)y * s->nx + x;
            rho[n] = r;
            ux[n] = jx / r;
            uy[n] = jy / r;
        }
    }
}

void orc_get_last_force(const orc_sim* s, double* fx, double* fy) {
    memcpy(fx, s->flbx, sizeof(double) * s->n);
    memcpy(fy, s->flby, sizeof(double) * s->n);
}
void orc_get_last_velocity(const orc_sim* s, double* ux, double* uy) {
    memcpy(ux, s->ux, sizeof(double) * s->n);
    memcpy(uy, s->uy, sizeof(double) * s->n);
}

int orc_get_marker_record(const orc_sim* s, int32_t p, double* out, int32_t cap) {
    if (p < 0 || p >= s->np) return -1;
    int nm = s->p[p].nm;
    if (cap < nm) return nm;
    memcpy(out, s->p[p].rec, sizeof(double) * 8 * nm);
    return nm;
}

uint64_t orc_anchor_hash(const orc_sim* s) { return s->anchor_hash; }

void orc_set_threads(orc_sim* s, int32_t n) { s->threads = n < 1 ? 1 : n; }

/* Running hash of every MLS stencil anchor used (markers and probes).  The
 * anchors are piecewise constant in the particle state, so two runs with equal
 * hashes differ only through the smooth part of the step map. */
static void hash_anchor(uint64_t* hp, double x, double y) {
    int64_t a = (int64_t)floor(x + 0.5), b = (int64_t)floor(y + 0.5);
    uint64_t h = *hp;
    h ^= (uint64_t)a * 0x9E3779B97F4A7C15ULL;
    h *= 1099511628211ULL;
    h ^= (uint64_t)b * 0xC2B2AE3D27D4EB4FULL;
    h *= 1099511628211ULL;
    *hp = h;
}

static int all_finite(const double* v, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Surface-stress force and moment on one body, Eqs. (13), (14), readings
 * R9-R12: each marker gets a probe at dn along its normal; MLS at the probe
 * gives the density and the velocity gradient of the (force-corrected)
 * fields; p_P = c_s^2 (rho_P - rho0); the marker pressure adds the rigid
 * acceleration correction; the traction is tau.n - p n; sums run over the
 * markers in ascending order.  rho, ux, uy are [ny][nx] level-n fields. */
static void surface_force(const orc_config* c, const double* rho, const double* ux,
                          const double* uy, double X, double Y, double th, double Om,
                          const double acc[3], int nm, const double* xi, const double* nu_b,
                          const double* ds, double out[3], uint64_t* hash) {
    const int nx = c->nx;
    const double nu = (c->tau - 0.5) / 3.0;
    double cs = cos(th), sn = sin(th);
    double Fx = 0.0, Fy = 0.0, Mz = 0.0;
    for (int l = 0; l < nm; ++l) {
        double rx = cs * xi[2 * l] - sn * xi[2 * l + 1];
        double ry = sn * xi[2 * l] + cs * xi[2 * l + 1];
        double nxl = cs * nu_b[2 * l] - sn * nu_b[2 * l + 1];
        double nyl = sn * nu_b[2 * l] + cs * nu_b[2 * l + 1];
        double xp = X + rx + c->probe_dn * nxl;
        double yp = Y + ry + c->probe_dn * nyl;
        int32_t ni[9], nj[9], ok[9];
        double phi[9], dpx[9], dpy[9];
        orc_mls(c, xp, yp, ni, nj, ok, phi, dpx, dpy);
        if (hash) hash_anchor(hash, xp, yp);
        double rP = 0.0, dudx = 0.0, dudy = 0.0, dvdx = 0.0, dvdy = 0.0;
        for (int k = 0; k < 9; ++k) {
            if (!ok[k]) continue;
            size_t n = (size_t)nj[k] * nx + ni[k];
            rP += phi[k] * rho[n];
            dudx += dpx[k] * ux[n];
            dudy += dpy[k] * ux[n];
            dvdx += dpx[k] * uy[n];
            dvdy += dpy[k] * uy[n];
        }
        double pP = (rP - 1.0) / 3.0;
        double txx = nu * (2.0 * dudx);
        double txy = nu * (dudy + dvdx);
        double tyy = nu * (2.0 * dvdy);
        double alx = acc[0] - acc[2] * ry - Om * Om * rx;
        double aly = acc[1] + acc[2] * rx - Om * Om * ry;
        double pl = pP + c->probe_dn * (alx * nxl + aly * nyl);
        double tx = txx * nxl + txy * nyl - pl * nxl;
        double ty = txy * nxl + tyy * nyl - pl * nyl;
        Fx += tx * ds[l];
        Fy += ty * ds[l];
        Mz += (rx * ty - ry * tx) * ds[l];
    }
    out[0] = Fx;
    out[1] = Fy;
    out[2] = Mz;
}

void orc_surface_force(const orc_config* cfg, const double* rho, const double* ux,
                       const double* uy, const orc_particle_desc* d, const double acc[3],
                       double out[3]) {
    surface_force(cfg, rho, ux, uy, d->x, d->y, d->theta, d->omega, acc, d->n_markers, d->xi,
                  d->nrm, d->ds, out, NULL);
}

/* One time step; returns 1 if the state became invalid. */
static int one_step(orc_sim* s, double* rec_out) {
    const orc_config* c = &s->cfg;
    const int nx = s->nx, ny = s->ny;
    const double gx = c->body_force[0], gy = c->body_force[1];
    int bad = 0;

    /* Moments of f^n, Eqs. (6), (7): rho and j* = sum f e + g/2 (the IB
     * force is not known yet, reading R2).  The node loops of this function
     * may run their rows on several threads (orc_set_threads): every node is
     * computed on its own, so the results do not depend on the thread count. */
#pragma omp parallel for reduction(| : bad) num_threads(s->threads)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            double r = 0.0, jx = 0.0, jy = 0.0;
            for (int i = 0; i < Q; ++i) r += s->f[idx(s, i, y, x)];
            for (int i = 0; i < Q; ++i) jx += s->f[idx(s, i, y, x)] * E[i][0];
            for (int i = 0; i < Q; ++i) jy += s->f[idx(s, i, y, x)] * E[i][1];
            jx += 0.5 * gx;
            jy += 0.5 * gy;
            size_t n = (size_t)y * nx + x;
            s->rho[n] = r;
            s->jx[n] = jx;
            s->jy[n] = jy;
            if (!(r > 0.0) || !isfinite(r)) bad = 1;
        }
    }

    /* Immersed boundary, Sec. 1.2: interpolate u* = j* / rho to every marker
     * (Eq. (8)), Lagrangian force F_l = U_b - U (Eq. (11), dt = 1), and the
     * spread f_lb(x_k) = sum_l c_l phi^l_k F_l (Eq. (12)).  Loop order:
     * particles, markers, stencil nodes, all ascending.  Eq. (12) fixes no
     * order for the sum at a node; reading R20: a particle's markers are
     * summed in rounds of ORC_ROUND consecutive markers, each round in
     * ascending marker order starting from zero, the round sums are added in
     * ascending round order, and the particles' sums are added to the node's
     * force (zero before the first) in ascending particle order. */
    memset(s->flbx, 0, sizeof(double) * s->n);
    memset(s->flby, 0, sizeof(double) * s->n);
    for (int pi = 0; pi < s->np; ++pi) {
        particle* p = &s->p[pi];
        double cs = cos(p->th), sn = sin(p->th);
        int np_touched = 0, nr_touched = 0;
        for (int l = 0; l < p->nm; ++l) {
            double rx = cs * p->xi[2 * l] - sn * p->xi[2 * l + 1];
            double ry = sn * p->xi[2 * l] + cs * p->xi[2 * l + 1];
            double xl = p->X[0] + rx, yl = p->X[1] + ry;
            double ubx = p->V[0] - p->Om * ry;
            double uby = p->V[1] + p->Om * rx;
            int32_t ni[9], nj[9], ok[9];
            double phi[9], dpx[9], dpy[9];
            orc_mls(c, xl, yl, ni, nj, ok, phi, dpx, dpy);
            hash_anchor(&s->anchor_hash, xl, yl);
            double Ux = 0.0, Uy = 0.0;
            for (int k = 0; k < 9; ++k) {
                if (!ok[k]) continue;
                size_t n = (size_t)nj[k] * nx + ni[k];
                Ux += phi[k] * (s->jx[n] / s->rho[n]);
                Uy += phi[k] * (s->jy[n] / s->rho[n]);
            }
            double Fx = ubx - Ux, Fy = uby - Uy;
            double cl = c->spread_scale == ORC_SPREAD_UNIT ? 1.0 : p->ds[l];
            for (int k = 0; k < 9; ++k) {
                if (!ok[k]) continue;
                size_t n = (size_t)nj[k] * nx + ni[k];
                if (!s->rmark[n]) { /* first term of this round at the node */
                    s->rmark[n] = 1;
                    s->rlist[nr_touched++] = (int32_t)n;
                    s->rfx[n] = 0.0;
                    s->rfy[n] = 0.0;
                }
                s->rfx[n] += cl * phi[k] * Fx;
                s->rfy[n] += cl * phi[k] * Fy;
            }
            if ((l + 1) % ORC_ROUND == 0 || l + 1 == p->nm) {
                /* end of a round: its sums join the particle's, in round order */
                for (int q = 0; q < nr_touched; ++q) {
                    size_t n = (size_t)s->rlist[q];
                    if (!s->pmark[n]) {
                        s->pmark[n] = 1;
                        s->plist[np_touched++] = (int32_t)n;
                        s->pfx[n] = s->rfx[n];
                        s->pfy[n] = s->rfy[n];
                    } else {
                        s->pfx[n] += s->rfx[n];
                        s->pfy[n] += s->rfy[n];
                    }
                    s->rmark[n] = 0;
                }
                nr_touched = 0;
            }
            double* rr = p->rec + 8 * l;
            rr[0] = xl;
            rr[1] = yl;
            rr[2] = ubx;
            rr[3] = uby;
            rr[4] = Ux;
            rr[5] = Uy;
            rr[6] = Fx;
            rr[7] = Fy;
        }
        /* the particle's sums join the node's force, in particle order */
        for (int q = 0; q < np_touched; ++q) {
            size_t n = (size_t)s->plist[q];
            s->flbx[n] += s->pfx[n];
            s->flby[n] += s->pfy[n];
            s->pmark[n] = 0;
        }
    }

    /* Forced collision of every node, Eqs. (4), (5) (readings R2, R3). */
#pragma omp parallel for num_threads(s->threads)
    for (int y = 0; y < ny; ++y) {
        double fl[9], fo[9];
        for (int x = 0; x < nx; ++x) {
            size_t n = (size_t)y * nx + x;
            for (int i = 0; i < Q; ++i) fl[i] = s->f[idx(s, i, y, x)];
            double r, ux, uy;
            orc_collide_node(fl, gx, gy, s->flbx[n], s->flby[n], c->tau, fo, &r, &ux, &uy);
            for (int i = 0; i < Q; ++i) s->fc[idx(s, i, y, x)] = fo[i];
            s->ux[n] = ux;
            s->uy[n] = uy;
        }
    }

    /* Force and moment on each body, Eqs. (13), (14), from level-n fields,
     * then the BDF2 update, Eqs. (15), (16) (readings R9-R15). */
    for (int pi = 0; pi < s->np; ++pi) {
        particle* p = &s->p[pi];
        double out[3];
        double acc[3] = {p->acc[0], p->acc[1], p->alp};
        surface_force(c, s->rho, s->ux, s->uy, p->X[0], p->X[1], p->th, p->Om, acc, p->nm,
                      p->xi, p->nu, p->ds, out, &s->anchor_hash);
        double Fx = out[0], Fy = out[1], Mz = out[2];
        p->F[0] = Fx;
        p->F[1] = Fy;
        p->M = Mz;
        double buoy = 1.0 - 1.0 / p->ratio;
        double ax = Fx / p->m + buoy * c->gravity[0];
        double ay = Fy / p->m + buoy * c->gravity[1];
        double al = Mz / p->I;
        double vx, vy, om, X0, X1, th;
        orc_bdf2(p->V[0], p->Vm[0], ax, p->X[0], p->Xm[0], &vx, &X0);
        orc_bdf2(p->V[1], p->Vm[1], ay, p->X[1], p->Xm[1], &vy, &X1);
        orc_bdf2(p->Om, p->Omm, al, p->th, p->thm, &om, &th);
        p->Vm[0] = p->V[0];
        p->Vm[1] = p->V[1];
        p->Omm = p->Om;
        p->Xm[0] = p->X[0];
        p->Xm[1] = p->X[1];
        p->thm = p->th;
        p->V[0] = vx;
        p->V[1] = vy;
        p->Om = om;
        p->X[0] = X0;
        p->X[1] = X1;
        p->th = th;
        p->acc[0] = ax;
        p->acc[1] = ay;
        p->alp = al;
        double st[6] = {vx, vy, om, X0, X1, th};
        if (!all_finite(st, 6)) bad = 1;
    }

    /* Streaming, left-hand side of Eq. (4): f_i(x, n+1) = f^c_i(x - e_i, n).
     * Periodic axes wrap; populations entering through a wall are left to
     * the Zou-He reconstruction. */
    for (int i = 0; i < Q; ++i) {
        int ex = (int)E[i][0], ey = (int)E[i][1];
#pragma omp parallel for num_threads(s->threads)
        for (int y = 0; y < ny; ++y) {
            int ys = y - ey;
            if (c->bc_y == ORC_PERIODIC) {
                ys = (ys + ny) % ny;
            } else if (ys < 0 || ys >= ny) {
                continue;
            }
            for (int x = 0; x < nx; ++x) {
                int xs = x - ex;
                if (c->bc_x == ORC_PERIODIC) {
                    xs = (xs + nx) % nx;
                } else if (xs < 0 || xs >= nx) {
                    continue;
                }
                s->f[idx(s, i, y, x)] = s->fc[idx(s, i, ys, xs)];
            }
        }
    }
    apply_walls(s);

    if (rec_out) {
        for (int pi = 0; pi < s->np; ++pi)
            particle_record(&s->p[pi], rec_out + (size_t)pi * ORC_PSTATE);
    }
    return bad;
}

int orc_step(orc_sim* s, int32_t n, double* traj) {
    ensure_lattice();
    for (int t = 0; t < n; ++t) {
        double* rec = traj ? traj + (size_t)t * s->np * ORC_PSTATE : NULL;
        int bad = one_step(s, rec);
        s->steps_done++;
        if (bad) return t + 1;
    }
    return 0;
}
