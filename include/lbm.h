/*
 * lbm.h -- C ABI of the MI355X (gfx950) implementation of the coupled
 * lattice-Boltzmann / moving-least-squares immersed-boundary method of
 * Coclite, de Tullio, Pascazio and Decuzzi ("A combined Lattice Boltzmann and
 * Immersed Boundary approach for predicting the vascular transport of
 * differently shaped particles", Computers and Fluids).
 *
 * One call to lbm_step advances every channel of a handle by whole time steps
 * of the method (Sec. 1.2, last paragraph, and Sec. 1.3):
 *   - D2Q9 BGK collision on the Hermite equilibrium with the Guo body-force
 *     term (Sec. 1.1, Eqs. (2)-(7)), pull streaming (left-hand side of Eq. (4))
 *     and Zou-He known-velocity walls (Sec. 1.1);
 *   - MLS interpolation of the fluid velocity to the Lagrangian markers,
 *     Lagrangian force and its spreading back to the lattice (Sec. 1.2,
 *     Eqs. (8)-(12));
 *   - surface-stress force and moment from normal probes (Sec. 1.3,
 *     Eqs. (13), (14)) and the BDF2 rigid-body update (Eqs. (15), (16)).
 * Lattice units throughout: dx = dt = 1, reference density 1, c_s^2 = 1/3,
 * kinematic viscosity nu = (tau - 1/2)/3.
 *
 * Conventions
 *   - All pointers passed to the library are HOST pointers unless stated.
 *     `workspace` is a DEVICE pointer; `hip_stream` is a hipStream_t.
 *   - Every entry point returns an lbm_status; none throws.  After a failure,
 *     lbm_last_error(h) describes it (a handle-less failure of lbm_init is
 *     described by lbm_last_error(NULL)).
 *   - A handle is used from one host thread at a time.  All GPU work is
 *     enqueued on the handle's stream.
 *   - Lattice arrays exchanged with the host are row-major [ny][nx] in FP64;
 *     population arrays are [9][ny][nx] in the velocity order of Eq. (3):
 *     e0 = (0,0), e1 = (1,0), e2 = (0,1), e3 = (-1,0), e4 = (0,-1),
 *     e5 = (1,1), e6 = (-1,1), e7 = (-1,-1), e8 = (1,-1).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lbm_status {
    LBM_OK = 0,
    LBM_EINVAL = 1,    /* invalid argument or configuration */
    LBM_ENOMEM = 2,    /* allocation failed or workspace too small */
    LBM_EDEVICE = 3,   /* HIP runtime error */
    LBM_ESTATE = 4,    /* call not allowed in the handle's current state */
    LBM_ECAPACITY = 5, /* caller buffer or internal capacity too small */
    LBM_EUNSTABLE = 6  /* non-finite or non-positive density detected */
} lbm_status;

enum { LBM_BC_PERIODIC = 0, LBM_BC_ZOUHE = 1 };
enum { LBM_INIT_REST = 0, LBM_INIT_COUETTE = 1 };
/* Population storage.  F64: FP64 populations, FP64 arithmetic.  F32: FP32
 * storage of the deviation f_i - w_i, FP32 arithmetic.  F16S: FP16 storage of
 * s_i (f_i - w_i) with s_i = 2^(fp16_exp + k_i), k_i = 1, 3, 5 for the rest,
 * axis and diagonal directions, FP32 arithmetic.  In every form the
 * immersed-boundary and rigid-body stages run in FP64. */
enum { LBM_STORE_F64 = 0, LBM_STORE_F32 = 1, LBM_STORE_F16S = 2 };
enum { LBM_SIDE_XLO = 0, LBM_SIDE_XHI = 1, LBM_SIDE_YLO = 2, LBM_SIDE_YHI = 3 };
/* Interpolation kernels of Sec. 2.2: exponential (Eq. (10)), cubic, quartic
 * and cosine (Eqs. (17)-(19)), and polynomial (Eq. (20)).  The printed
 * polynomial kernel has break points 0.5 and 1 in r_k but takes the square
 * root of a negative number between 0.5 and about 0.79; its two branches are
 * read as functions of q = 2 r_k (break points q = 1 and 2), which makes it
 * the four-point delta function: W(0) = 1/2, W(1/2) = 1/4, W(1) = 0. */
enum { LBM_W_EXP = 0, LBM_W_CUBIC = 1, LBM_W_QUARTIC = 2, LBM_W_COSINE = 3, LBM_W_POLY = 4 };
/* c_l of Eq. (12): segment length (force conservation) or 1. */
enum { LBM_SPREAD_SEGMENT = 0, LBM_SPREAD_UNIT = 1 };

#define LBM_PSTATE 10 /* per particle: x, y, theta, u, v, omega, Fx, Fy, M, channel */
/* per particle, lbm_adjoint_gradients:
 *   [0, 15)  dJ/d of the state at the adjoint position: X(2), X_prev(2),
 *            theta, theta_prev, V(2), V_prev(2), omega, omega_prev, acc(2),
 *            alpha (the lagged accelerations of Sec. 1.3);
 *   15, 16   dJ/dm and dJ/dI accumulated over the reversed steps;
 *   [17, 23) dJ/d of a start from the state at the adjoint position with the
 *            BDF2 history equal to it (at position 0: the initial x, y,
 *            theta, u, v, omega), i.e. the sums of the current and previous
 *            slots;
 *   23, 24   dJ/d area and dJ/d polar_moment (m = density_ratio * area,
 *            I = density_ratio * polar_moment, Eqs. (15), (16)). */
#define LBM_AGRAD 25

/* One channel (an independent lattice).  Channels of one handle must share
 * `storage`.  Zou-He walls on both axes make a closed box: its walls must be
 * at rest and its body force zero, and each corner node takes the corner
 * closure (the populations pointing into the fluid bounce back, the two
 * buried diagonals share the density of the diagonal interior neighbour that
 * the other seven leave); the adjoint does not support closed boxes. */
typedef struct lbm_channel_config {
    int32_t nx, ny;          /* lattice nodes, >= 3 each */
    double tau;              /* BGK relaxation time, > 1/2 */
    int32_t bc_x, bc_y;      /* LBM_BC_PERIODIC or LBM_BC_ZOUHE */
    double u_wall[4][2];     /* wall velocities of sides x-, x+, y-, y+ */
    int32_t init;            /* LBM_INIT_REST, or LBM_INIT_COUETTE (needs bc_y =
                                ZOUHE): u_x linear in y between the y- and y+
                                wall speeds (Sec. 3.1) */
    double body_force[2];    /* uniform body force on the fluid */
    double gravity[2];       /* gravity on the particles, applied as
                                (1 - rho_f/rho_s) g */
    int32_t storage;         /* LBM_STORE_* */
    int32_t fp16_exp;        /* scale exponent K of the F16S form (0..24):
                                the largest scaled deviation s_i (f_i - w_i)
                                must stay below the FP16 maximum 65504, so K
                                goes down as the flow's Mach number goes up
                                (14 suits |u| up to about 0.05) */
    double mls_rw;           /* MLS support size r_w (Sec. 1.2: 2.6) */
    double mls_alpha;        /* exponential-kernel width (Eq. (10): 0.3) */
    double probe_dn;         /* probe length along the normal (Sec. 1.3: 1.2) */
    int32_t mls_kernel;      /* LBM_W_* */
    int32_t spread_scale;    /* LBM_SPREAD_* */
} lbm_channel_config;

/* One rigid particle as a closed set of Lagrangian markers (Sec. 1.2): the
 * markers sit on segment centres in the body frame (centroid at the origin);
 * nrm are outward unit normals; ds the segment lengths S_l of Eqs. (12)-(14).
 * Mass m = density_ratio * area and moment of inertia
 * I = density_ratio * polar_moment (Eqs. (15), (16)). */
typedef struct lbm_particle_desc {
    double x, y, theta;      /* initial centroid and angle (theta rotates the
                                body frame counter-clockwise) */
    double u, v, omega;      /* initial linear and angular velocity */
    double density_ratio;    /* rho_s / rho_f, > 0 */
    double area;             /* body area, > 0 */
    double polar_moment;     /* integral of |r|^2 over the body, > 0 */
    int32_t n_markers;       /* >= 3 */
    const double* xi;        /* [n_markers][2] */
    const double* nrm;       /* [n_markers][2] */
    const double* ds;        /* [n_markers] */
} lbm_particle_desc;

/* Launch and schedule choices of the lattice pass (see lbm_set_tuning). */
typedef struct lbm_tuning {
    int32_t tile_w;          /* nodes per tile along x: 64, 128 or 256 */
    int32_t rows_per_thread; /* consecutive rows handled by one thread: 1, 2, 4 */
    int32_t persistent_wgs;  /* 0: one workgroup per tile; > 0: that many
                                workgroups striding over the tile table */
    int32_t use_graph;       /* 1: replay lbm_step's steps from a HIP graph */
    int32_t xcd_remap;       /* 1: hand each of the 8 XCDs (one L2 each) a
                                contiguous block of tiles, so tiles that share
                                halo cache lines run under the same L2 */
    int32_t overlap;         /* 1: run the lattice pass and the surface-stress /
                                rigid-body stage as one launch (both read only
                                the step's input populations and force
                                patches): the first workgroups take the
                                particles' rounds of 64 markers, the rest
                                take lattice tiles: 64 x 9*rows_per_thread
                                nodes in 576-thread workgroups (vec = 0), or
                                the vec = 1 tiles in 256-thread workgroups.
                                Needs persistent_wgs = 0, and tile_w = 64
                                unless vec = 1 (else LBM_EINVAL); results are
                                bitwise those of 0 */
    int32_t vec;             /* 1: vector form of the lattice pass: each lane
                                takes nv = tile_w / 64 consecutive nodes of a
                                row and moves each population plane of them
                                with one load and one store of nv elements
                                (at most 16 bytes: nv <= 2 in FP64, 4 in
                                FP32, 8 in F16S; tile_w 512 is allowed for
                                F16S); tiles of tile_w x 4 * rows_per_thread
                                nodes, rows_per_thread 1 or 2 (1 with
                                overlap = 1).  Results are bitwise those of
                                vec = 0 */
    int32_t nt_store;        /* 1 (needs vec = 1): the lattice pass stores
                                nontemporally, bypassing the caches; faster
                                when the two population buffers exceed the
                                256 MB Infinity Cache, slower when they fit */
    int32_t adj_fused;       /* launches of a reversed adjoint step when no
                                channel holds more than one particle.  0: three
                                (surface stress, immersed boundary, lattice);
                                1: the two particle kernels as one launch;
                                2 (default): the whole step as one launch
                                when its workgroups (the particles, then one
                                512-thread workgroup per 8 x 64 lattice nodes)
                                fit the device's compute units at once, else
                                as 1.  With several particles in a channel
                                the three launches are used.  Results are
                                bitwise the same in every form */
} lbm_tuning;

typedef struct lbm_handle lbm_handle;

/* Device bytes needed for the population buffers (two ping-pong buffers) of
 * n_channels channels.  0 on invalid input. */
size_t lbm_workspace_bytes(const lbm_channel_config* cfg, int32_t n_channels);

/* Create a handle for n_channels (>= 1) independent channels; n_channels > 1
 * advances all of them by single launches per kernel phase (batched form).
 * cfg: host array of n_channels configs, copied.  hip_stream: the stream all
 * work is enqueued on (NULL = the null stream).  workspace: device memory of
 * at least lbm_workspace_bytes(cfg, n) bytes, owned by the caller and kept
 * alive until lbm_destroy; NULL makes the library allocate it.  The
 * populations are initialised to the equilibrium of density 1 and the initial
 * velocity (rest or Couette) and the walls are applied.
 * Errors: LBM_EINVAL (bad field, tau <= 1/2, nx or ny < 3, a closed box with
 * a moving wall or a body force, mixed storage, a channel whose 9 x ny x pitch populations reach 4 GiB, with
 * pitch = nx rounded up to 64), LBM_ENOMEM (workspace_bytes too small),
 * LBM_EDEVICE. */
int lbm_init(const lbm_channel_config* cfg, int32_t n_channels, void* hip_stream,
             void* workspace, size_t workspace_bytes, lbm_handle** out);

/* Add a particle to `channel` before the first lbm_step (or after lbm_reset).
 * The marker arrays are copied.  The history of the
 * BDF2 scheme starts equal to the initial state.
 * Errors: LBM_EINVAL (n_markers < 3 or > 2048, non-unit normal, non-finite or
 * non-positive value, body closer than 3 nodes to a wall, body wider than
 * the channel), LBM_ESTATE (after the first step), LBM_ECAPACITY (body too
 * large for the per-particle force patch). */
int lbm_add_particle(lbm_handle* h, int32_t channel, const lbm_particle_desc* d, int32_t* out_id);

/* Return the handle to the state lbm_init left it in, so that another run
 * (with other particles) can use the same handle: the populations are set
 * to each channel's initial state again (rest, or the Couette start of
 * Sec. 3.1, as its config asks), every particle is removed, the step counter is zero, and the
 * checkpoints, captured graphs and adjoint state are released.  The channel
 * configs, stream, workspace and tuning are kept.  Waits for the handle's
 * stream.  Errors: LBM_EINVAL (NULL handle), LBM_EDEVICE. */
int lbm_reset(lbm_handle* h);

/* Advance every channel by n_steps (>= 0) time steps.  If traj is not NULL
 * (host pointer) it receives [n_steps][n_particles][LBM_PSTATE]: the
 * particle state at level n+1 and the force and moment of level n, for each
 * step n, particles in the order they were added.  Returns after the work is
 * complete.  Errors: LBM_EUNSTABLE (a density became non-positive or
 * non-finite, or a particle state non-finite; the step is in lbm_last_error),
 * LBM_ECAPACITY (a particle outgrew its force patch), LBM_EDEVICE. */
int lbm_step(lbm_handle* h, int32_t n_steps, double* traj);

/* Current state of all particles: out[n][LBM_PSTATE] (host), the last step's
 * force and moment included.  *n_out receives the particle count even when
 * cap is too small (then LBM_ECAPACITY). */
int lbm_get_particles(const lbm_handle* h, double* out, int32_t cap, int32_t* n_out);

/* Density and velocity (sum f e + g/2)/rho of the current populations of a
 * channel, each [ny][nx] (host); any pointer may be NULL. */
int lbm_get_fields(lbm_handle* h, int32_t channel, double* rho, double* ux, double* uy);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or diagnostic loops, harnesses that forbid
 * hipMalloc): lbm_get_fields without any allocation.  The fields are staged
 * in a fixed device array of the library (3 x 2^18 doubles, 6 MiB, on each
 * GPU the library runs on, held until the process ends), so the channel may
 * have at most 262 144 nodes (nx * ny), else LBM_ECAPACITY and nothing is
 * written.  Results are those of lbm_get_fields, bit for bit.  Calls on one
 * GPU share that array: calls that overlap in time on one GPU (from several
 * host threads, or handles on different streams) race; calls from one host
 * thread are safe, as each returns after its copies complete.  Errors:
 * LBM_EINVAL (NULL handle, bad channel), LBM_ECAPACITY, LBM_EDEVICE. */
int lbm_get_fields_noalloc(lbm_handle* h, int32_t channel, double* rho, double* ux, double* uy);

/* Current populations f^n (after streaming and walls) of a channel, converted
 * to FP64, [9][ny][nx] (host). */
int lbm_get_populations(lbm_handle* h, int32_t channel, double* f);

/* Replace the current populations of a channel by f [9][ny][nx] (host, FP64),
 * rounded to the channel's storage form.  The values must already satisfy the
 * wall conditions they are meant to (walls are applied from the next step). */
int lbm_set_populations(lbm_handle* h, int32_t channel, const double* f);

/* Save / restore the complete state (populations, particles, step counter) in
 * slot 0..63; slots are allocated on first use.  Restoring a slot saved with a
 * different particle set is LBM_ESTATE. */
int lbm_checkpoint_save(lbm_handle* h, int32_t slot);
int lbm_checkpoint_restore(lbm_handle* h, int32_t slot);

/* Lattice-pass launch choices; takes effect at the next lbm_step. */
int lbm_set_tuning(lbm_handle* h, const lbm_tuning* t);
int lbm_get_tuning(const lbm_handle* h, lbm_tuning* t);

/* Average device time per launch, in microseconds, of the three kernels of a
 * step (out_us[0] = immersed-boundary force and spreading, with the sum of
 * the per-round partial patches of particles of more than 64 markers,
 * [1] = lattice pass,
 * [2] = surface stress and rigid-body update), measured with HIP events on the
 * handle's stream over `reps` back-to-back launches of each kernel alone.  The
 * first force launch runs before the lattice launches, so that the lattice
 * pass works on the tile lists of a step and adds the IB force where a step
 * does.  The launches run real steps, so the state advances by reps steps
 * per kernel phase; use a checkpoint around the call to keep it.  With overlap = 1,
 * out_us[1] times the combined launch without its particle workgroups. */
int lbm_time_kernels(lbm_handle* h, int32_t reps, double out_us[3]);

/* ---- Discrete adjoint of the step (reverse-mode gradients) ----------------
 * J is a linear function of the particle records after the last step taken:
 * J = sum_p seed[p] . record[p] (LBM_PSTATE entries; the channel entry is
 * ignored).  Its gradient is computed by reversing the steps segment by
 * segment: each segment restarts from a checkpoint (lbm_checkpoint_save),
 * recomputes its steps into a tape and reverses them with the transposes of
 * the moments and Guo collision (Eqs. (4)-(7)), the IB interpolation, force
 * and spreading (Eqs. (8)-(12)) including the motion of the MLS weights with
 * the markers, the surface stress, force and moment (Eqs. (13), (14)), BDF2
 * (Eqs. (15), (16)), streaming and the Zou-He closure (App. A).  MLS stencil
 * anchors are held fixed (the step map is piecewise smooth in the particle
 * state).  Sums have a fixed order: results are bitwise reproducible.
 *
 * lbm_adjoint_begin: start at the current step with the seed
 * [n_particles][LBM_PSTATE] (host, particles in the order they were added)
 * and allocate a tape of max_segment steps: max_segment population buffers
 * plus force patches and particle snapshots.  Errors: LBM_EINVAL (NULL or
 * non-finite seed, probe reach wider than the channel, a channel whose
 * 9 x ny x pitch adjoint populations reach 4 GiB: 8 bytes each in the FP64
 * form, 4 in the others), LBM_ENOMEM. */
int lbm_adjoint_begin(lbm_handle* h, const double* seed, int32_t max_segment);

/* Reverse n_steps (1..max_segment) steps that end at the current adjoint
 * position and start at the checkpoint in `slot`: restores it, recomputes the
 * steps, reverses them, and restores the checkpoint again (the forward state
 * is left at the checkpoint).  The adjoint position moves back by n_steps.
 * Segments must be taken from the last one backwards.  Errors: LBM_ESTATE (no
 * adjoint begun, empty slot, or checkpoint step + n_steps != position),
 * LBM_EINVAL, LBM_EUNSTABLE / LBM_ECAPACITY from the recomputation (the
 * adjoint is then abandoned). */
int lbm_adjoint_segment(lbm_handle* h, int32_t slot, int32_t n_steps);

/* Reverse n_segments segments of n_steps each, from the last one backwards:
 * slots[j] (host array of n_segments) holds the checkpoint n_steps before
 * that of slots[j - 1], and slots[0] the one n_steps before the adjoint
 * position.  Gives bitwise the results of lbm_adjoint_segment called on each
 * slot in turn, and leaves the forward state at the checkpoint of the last
 * slot.  The recomputation of segment j + 1 runs on a second stream of the
 * library beside the reversal of segment j (the checkpointing schedule is
 * unchanged: each segment is recomputed once), which takes a second tape of
 * max_segment steps, allocated at the first call and freed with the first
 * tape; where it does not fit, the segments run one after the other.
 * Errors: those of lbm_adjoint_segment; LBM_EUNSTABLE / LBM_ECAPACITY of any
 * segment are reported after the last one (the adjoint is then
 * abandoned). */
int lbm_adjoint_sweep(lbm_handle* h, const int32_t* slots, int32_t n_segments, int32_t n_steps);

/* Gradients at the current adjoint position (host outputs, each may be NULL):
 *   part_out   [n_particles][LBM_AGRAD] (layout above), particles in the
 *              order added; at position 0 entries [17, 25) are the
 *              derivatives with respect to the initial pose and velocities,
 *              the area and the polar moment (the BDF2 history starts equal
 *              to the initial state);
 *   marker_out [sum of n_markers][5]: dJ/d xi (2), d nrm (2), d ds per
 *              marker, particles in the order added;
 *   wall_out   [n_channels][4][2]: dJ/d u_wall.  At position 0 this includes
 *              the Couette start (Sec. 3.1) unless the populations were
 *              replaced with lbm_set_populations. */
int lbm_adjoint_gradients(lbm_handle* h, double* part_out, double* marker_out, double* wall_out);

/* dJ/d populations at the adjoint position, [9][ny][nx] FP64 (host).  On wall
 * nodes the entries are with respect to the streamed populations before the
 * Zou-He closure (zero for the three it reconstructs). */
int lbm_adjoint_field(lbm_handle* h, int32_t channel, double* out);

/* Bandwidth of a plain device-to-device copy of `bytes` (a positive multiple
 * of 16) from src to dst (DEVICE pointers, not overlapping, owned by the
 * caller) with the library's own copy kernel (16-byte nontemporal loads and
 * stores, 4 per lane, one contiguous 16 KiB block per workgroup of 256
 * threads): *gbps receives
 * the read plus written bytes per second, in GB/s, averaged over `reps`
 * back-to-back launches on hip_stream after one untimed launch (HIP
 * events).  This is the practical ceiling of the HBM-bound lattice pass.
 * Errors: LBM_EINVAL (NULL pointer, reps < 1, bad size), LBM_EDEVICE; the
 * text is in lbm_last_error(NULL). */
int lbm_measure_copy(void* dst, const void* src, size_t bytes, int32_t reps, void* hip_stream, double* gbps);

/* Step index the adjoint currently refers to (-1: none in progress). */
int64_t lbm_adjoint_position(const lbm_handle* h);

/* Total steps taken by the handle. */
int64_t lbm_steps_done(const lbm_handle* h);

/* Text of the last failure on h (or of the last handle-less failure when h is
 * NULL).  Owned by the library; valid until the next call on h. */
const char* lbm_last_error(const lbm_handle* h);

/* Free the handle and everything the library allocated (not a caller
 * workspace).  NULL is accepted. */
int lbm_destroy(lbm_handle* h);

#ifdef __cplusplus
}
#endif
#endif
