// Internal structures shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmk {

constexpr int kMaxCells = 32768;         // force-patch cells of one particle
constexpr int kMaxMarkers = 2048;        // markers of one particle
constexpr int kRecSlots = 1024;          // trajectory ring-buffer depth (steps)
constexpr int kMaxNeighbours = 8;        // short candidate lists of force patches
constexpr int kTileList = 8;             // per-tile list: count + 7 particle indices
constexpr int kRound = 64;               // markers per round of the particle kernels
constexpr int kIbmThreads = 9 * kRound;  // one thread per (marker, stencil node)

// One channel: lattice geometry, walls and physical constants.  Read by the
// kernels through scalar loads (one channel per tile / particle).
struct ChanDev {
    int nx, ny, pitch, bcx, bcy;
    int p_begin, p_end;      // particle index range of this channel
    int kernel, spread_unit;
    int pad0;
    long long off;           // element offset of the channel in a buffer
    long long plane;         // ny * pitch: elements per population plane
    double tau, nu;
    double uw[4][2];
    double g[2];             // uniform body force on the fluid
    double grav[2];          // gravity on the particles
    double rw, alpha, dn;
    // FP32 copies for the reduced-precision lattice pass
    float f_omega, f_pref;
    float f_g[2];
    float f_uw[4][2];
    float sc[3], isc[3];     // F16S scales (rest, axis, diagonal) and inverses
    int tile0, tiles_x;      // first tile of the channel, tiles per tile row
};

struct TileDev {
    int chan, x0, y0, pad;
};

// Rigid particle state (FP64) plus its force patch.
struct PartDev {
    double X[2], Xm[2], th, thm;
    double cth, sth;         // cos(th), sin(th), evaluated once wherever th is set
    double V[2], Vm[2], Om, Omm;
    double acc[2], alp;      // accelerations of the previous step
    double F[2], M;          // force and moment of the last step
    double m, I, ratio;
    double rb;               // largest marker distance from the centroid
    int chan, mbeg, nm, patch_cap;
    int bx0, by0, bw, bh;    // patch box in unwrapped lattice coordinates
    long long patch_off;     // first cell of the patch in the patch pool
    long long part_off;      // first cell of the per-round partial patches (several rounds)
};

// A particle-kernel work entry carries what the first loads of a round
// need (its markers' place in the marker arrays and their count), so that
// the marker loads leave with the particle record's, not after it.
__host__ __device__ inline int4 work_entry(int particle, int round, int count, int chan, int first) {
    return make_int4(particle, round | (count << 16), chan, first);
}
__host__ __device__ inline int work_round(int4 w) { return w.y & 0xffff; }
__host__ __device__ inline int work_count(int4 w) { return w.y >> 16; }

struct StepArgs {
    const void* fin;         // post-collision populations of step n-1
    void* fout;              // post-collision populations of step n
    const ChanDev* chan;
    int nchan;
    const TileDev* tiles;
    int ntiles;
    PartDev* parts;
    int nparts;
    int persistent;          // lattice pass: 0 = one WG per tile
    int xcd_remap;           // lattice pass: contiguous tile blocks per XCD
    int nt_store;            // vector lattice pass: nontemporal stores
    const double2* xi;       // marker pool (body frame)
    const double2* nrm;
    const double* ds;
    double2* patch;          // force patches
    double* mscr;            // [markers][4] traction terms (particles of several rounds)
    int* flags;              // [0] unstable, [1] first bad step, [2] capacity
    long long* dstep;        // steps started so far
    double* rec;             // [kRecSlots][nparts][10]
    int* tlist;              // [2][ntiles][kTileList] particles whose patches touch a tile
    int parity;              // which half of tlist this step fills / reads
    int tile_w, tile_h;      // tile extent in nodes
    PartDev* snap;           // optional: copy of each particle after the force stage
    const int4* work;        // [nwork] particle-kernel workgroups, particle-major:
                             // (particle, round of kRound markers | markers of the
                             // round << 16, channel, first marker of the round in the
                             // marker arrays); see work_entry
    int nwork;
    int4 work0;              // work[0], carried in the arguments: the first workgroup's
                             // particle loads need no dependent read of the table
    int* pcount;             // [nparts] finished surface-stress workgroups; 0 between launches
    double2* partial;        // per-round partial force patches of particles of several rounds
    int sum_partials;        // 1: readers of the patch of a particle of several rounds add
                             // its partial patches themselves (no partial-sum launch)
    const int2* psum;        // [npsum] (particle, first cell) chunks of 256 patch cells of
                             // particles of several rounds
    int npsum;
};

enum { ST_F64 = 0, ST_F32 = 1, ST_F16S = 2 };

// Launchers (lbm_kernels.hip).
hipError_t launch_init(int store, const StepArgs& a, int chan, int init, int nx, int ny,
                       hipStream_t s);
hipError_t launch_ibm_force(int store, const StepArgs& a, hipStream_t s);
// vec = 1: the vector form (tile_w / 64 nodes per lane, tile_h = 4 * npt).
hipError_t launch_lattice(int store, const StepArgs& a, int tile_w, int npt, int vec, hipStream_t s);
hipError_t launch_traction(int store, const StepArgs& a, hipStream_t s);
// Force patches of particles of several rounds from their partial patches
// (after launch_ibm_force).
hipError_t launch_patch_sum(const StepArgs& a, hipStream_t s);
// Lattice pass and surface stress in one launch (tile_h 9 * npt, no
// persistent workgroups; tile_w 64, or with vec = 1 the vector form with
// tile_w = 64 * nv and npt = 1).
hipError_t launch_lattice_traction(int store, const StepArgs& a, int npt, int vec, hipStream_t s);
// Plain copy of n16 16-byte elements (lbm_measure_copy).
hipError_t launch_copy(void* dst, const void* src, long long n16, hipStream_t s);
hipError_t launch_fields(int store, const StepArgs& a, int chan, int nx, int ny, double* f_out,
                         double* rho, double* ux, double* uy, hipStream_t s);
hipError_t launch_set_pop(int store, const StepArgs& a, int chan, int nx, int ny,
                          const double* f_in, hipStream_t s);

}  // namespace lbmk
