/*
 * Plain FP64 CPU oracle of the coupled lattice-Boltzmann / moving-least-squares
 * immersed-boundary method of Coclite, de Tullio, Pascazio and Decuzzi,
 * "A combined Lattice Boltzmann and Immersed Boundary approach for predicting
 * the vascular transport of differently shaped particles" (Computers and Fluids).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the checker the GPU path is
 * compared against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no source, header, table or
 * helper with the GPU library; the two are written independently from the
 * paper's equations.
 *
 * Every routine is a direct, slow, serial transcription of one passage of the
 * paper (cited in lbm_oracle.c).  Readings of passages that are silent,
 * ambiguous or garbled are stated where they are used.
 *
 * Units: lattice units, dx = dt = 1 (Sec. 1.3), reference density rho0 = 1.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PERIODIC = 0, ORC_ZOUHE = 1 };
enum { ORC_INIT_REST = 0, ORC_INIT_COUETTE = 1 };
enum { ORC_SIDE_XLO = 0, ORC_SIDE_XHI = 1, ORC_SIDE_YLO = 2, ORC_SIDE_YHI = 3 };
enum { ORC_SPREAD_SEGMENT = 0, ORC_SPREAD_UNIT = 1 };
/* Interpolation kernels of Sec. 2.2, Eqs. (10) and (17)-(20). */
enum { ORC_W_EXP = 0, ORC_W_CUBIC = 1, ORC_W_QUARTIC = 2, ORC_W_COSINE = 3, ORC_W_POLY = 4 };

#define ORC_PSTATE 10 /* x, y, theta, u, v, omega, Fx, Fy, M, channel */

typedef struct orc_config {
    int32_t nx, ny;
    double tau;
    int32_t bc_x, bc_y;        /* ORC_PERIODIC or ORC_ZOUHE */
    double u_wall[4][2];       /* wall velocity of sides x-, x+, y-, y+ */
    int32_t init;              /* ORC_INIT_REST or ORC_INIT_COUETTE */
    double body_force[2];      /* uniform body force on the fluid (tests) */
    double gravity[2];         /* gravity acting on the particles */
    double mls_rw;             /* support size r_w (2.6) */
    double mls_alpha;          /* exponential-kernel width alpha (0.3) */
    double probe_dn;           /* probe length along the normal (1.2) */
    int32_t mls_kernel;        /* ORC_W_* */
    int32_t spread_scale;      /* ORC_SPREAD_SEGMENT: c_l = S_l; ORC_SPREAD_UNIT: c_l = 1 */
} orc_config;

typedef struct orc_particle_desc {
    double x, y, theta, u, v, omega;
    double density_ratio;      /* rho_s / rho_f */
    double area;               /* area of the body */
    double polar_moment;       /* integral of r^2 over the body (unit density) */
    int32_t n_markers;
    const double* xi;          /* [n][2] body-frame marker positions */
    const double* nrm;         /* [n][2] body-frame outward unit normals */
    const double* ds;          /* [n] segment lengths S_l */
} orc_particle_desc;

typedef struct orc_sim orc_sim;

/* Returns NULL on invalid configuration. */
orc_sim* orc_create(const orc_config* cfg);
void orc_destroy(orc_sim* s);
/* Returns particle index >= 0, or -1 on invalid input. */
int orc_add_particle(orc_sim* s, const orc_particle_desc* d);
/* Advances n steps.  traj (may be NULL): [n][n_particles][ORC_PSTATE].
 * Returns 0, or the 1-based index of the first step that produced a
 * non-finite population / non-positive density / non-finite particle state. */
int orc_step(orc_sim* s, int32_t n, double* traj);
int orc_n_particles(const orc_sim* s);
void orc_get_particles(const orc_sim* s, double* out /* [np][ORC_PSTATE] */);
/* Populations f^n after streaming and wall reconstruction, [9][ny][nx]. */
void orc_get_populations(const orc_sim* s, double* f);
void orc_set_populations(orc_sim* s, const double* f);
/* Density and force-free velocity (sum f e + g/2)/rho of f^n, each [ny][nx]. */
void orc_get_fields(const orc_sim* s, double* rho, double* ux, double* uy);
/* Eulerian IB force f_lb and corrected velocity of the last completed step. */
void orc_get_last_force(const orc_sim* s, double* fx, double* fy);
void orc_get_last_velocity(const orc_sim* s, double* ux, double* uy);
/* Marker-level record of the last completed step, [np_markers][8]:
 * x, y, Ub_x, Ub_y, U_x, U_y, F_x, F_y (interpolated and Lagrangian force). */
int orc_get_marker_record(const orc_sim* s, int32_t p, double* out, int32_t cap);
/* Hash of all stencil anchors used so far (for finite-difference validity). */
uint64_t orc_anchor_hash(const orc_sim* s);
/* Threads that the node loops (moments, collision, streaming) may use; the
 * immersed-boundary and particle stages stay serial.  Results do not depend
 * on it (every node is computed on its own).  Default 1. */
void orc_set_threads(orc_sim* s, int32_t n);

/* ---- stage functions, exposed for the closed-form tests ---- */
void orc_lattice(double e[9][2], double w[9]);
void orc_equilibrium(double rho, double ux, double uy, double feq[9]);
/* Forced BGK collision of one node; G = total force (body force + IB force). */
void orc_collide_node(const double f[9], double gx, double gy, double flbx, double flby,
                      double tau, double fc[9], double* rho, double* ux, double* uy);
/* Zou-He reconstruction of the unknown populations of a wall node, in place. */
void orc_zouhe(int side, double f[9], double uwx, double uwy, double gx, double gy);
/* MLS shape functions at point (x, y).  Returns number of valid nodes.
 * node_i/node_j: wrapped lattice indices; valid[k] = 0 for dropped nodes. */
int orc_mls(const orc_config* cfg, double x, double y, int32_t node_i[9], int32_t node_j[9],
            int32_t valid[9], double phi[9], double dphx[9], double dphy[9]);
double orc_kernel_weight(int kind, double r, double alpha);
/* Surface-stress force and moment (Eqs. (13), (14)) of a body with pose and
 * angular velocity taken from d, on level-n fields rho, ux, uy ([ny][nx], ux/uy
 * the force-corrected velocity); acc = (a_x, a_y, alpha) of the previous step.
 * out = (F_x, F_y, M). */
void orc_surface_force(const orc_config* cfg, const double* rho, const double* ux,
                       const double* uy, const orc_particle_desc* d, const double acc[3],
                       double out[3]);
/* One BDF2 update of a scalar velocity/position pair (Eqs. (15), (16)). */
void orc_bdf2(double v, double vm, double acc, double x, double xm, double* v_new, double* x_new);

#ifdef __cplusplus
}
#endif
#endif
