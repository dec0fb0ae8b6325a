// Device-side state and launchers of the discrete adjoint (lbm_adjoint.hip).
#pragma once

#include "lbm_internal.h"

namespace lbmk {

// Adjoint state of one particle (adjoint of its step-n state, accumulated
// shape and mass gradients) and its adjoint patch, which covers the stencils
// of its markers and of its probes.
enum { AL_X = 0, AL_XM = 2, AL_TH = 4, AL_THM = 5, AL_V = 6, AL_VM = 8, AL_OM = 10, AL_OMM = 11,
       AL_ACC = 12, AL_ALP = 14, AL_N = 15 };
constexpr int kAdjCell = 5;  // lam_rho, lam_ux, lam_uy (probe terms), lam_u*x, lam_u*y (marker terms)

struct AdjPart {
    double l[AL_N];          // adjoint of X, Xm, th, thm, V, Vm, Om, Omm, acc, alp
    double seed[3];          // adjoint of the last step's F, M (consumed by its reverse)
    double gm, gI;           // dJ/dm, dJ/dI
    int ax0, ay0, aw, ah;    // adjoint patch box, wrapped origin
    int acap, nnb;
    long long aoff;          // first cell of the adjoint patch
    int nb[kMaxNeighbours];  // particles whose adjoint boxes overlap this one, ascending
};

struct AdjArgs {
    StepArgs s;              // the forward step being reversed: fin is its input buffer,
                             // parts the particle snapshot taken after its force stage,
                             // patch its force patches
    const PartDev* pnext;    // particle snapshot after the step (its F and M)
    const void* lam_in;      // adjoint of the populations after the step
    void* lam_out;           // adjoint of the populations before the step
    AdjPart* ap;
    double* apatch;          // [cells][kAdjCell]
    double* gmk;             // [markers][5]: d xi (2), d nrm (2), d ds
    double* gwall;           // per wall node (2 doubles), then per row (1 double)
    const long long* gw_off; // per channel: first wall accumulator
    int* atlist;             // [2][ntiles][kTileList] particles whose adjoint patches touch a tile
    int first;               // 1 when this is the last step of the run: consume the seeds
};

hipError_t launch_adj_traction(int store, const AdjArgs& a, hipStream_t s);
hipError_t launch_adj_ibm(int store, const AdjArgs& a, hipStream_t s);
// launch_adj_traction then launch_adj_ibm as one launch; only for handles
// whose channels hold at most one particle each
hipError_t launch_adj_particle(int store, const AdjArgs& a, hipStream_t s);
hipError_t launch_adj_lattice(int store, const AdjArgs& a, hipStream_t s);
// The whole reversed step (both particle kernels and the adjoint lattice
// pass) as one launch of adj_step_workgroups(a) workgroups of 512 threads
// (-1: a shape it cannot take); only for handles whose channels hold at most
// one particle each.
int adj_step_workgroups(const AdjArgs& a);
hipError_t launch_adj_step(int store, const AdjArgs& a, hipStream_t s);
hipError_t launch_adj_finish(int store, const AdjArgs& a, int chan, int with_init, double* out8,
                             hipStream_t s);
hipError_t launch_adj_field(int store, const AdjArgs& a, int chan, double* out, hipStream_t s);

}  // namespace lbmk
