// Host side of the C ABI declared in include/lbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_adjoint.h"
#include "lbm_internal.h"

using namespace lbmk;

// Staging of lbm_get_fields_noalloc: the density and two velocity fields of
// a channel of at most kScratchNodes nodes, in a fixed device array (6 MiB
// on every GPU the library runs on, held until the process ends).  Host code
// never passes `scratch` itself to a kernel or copy (in host code the name is
// a host-side stand-in, not the device address): it uses the address
// hipGetSymbolAddress gives for the current device, looked up once per
// device by lbm_init.
constexpr int kScratchNodes = 1 << 18;
static __device__ __align__(256) double scratch[3 * kScratchNodes];

namespace {

thread_local std::string g_err;

struct PartHost {
    lbm_particle_desc d;
    std::vector<double> xi, nrm, ds;
    int chan;
    double rb;
    int cap;
};

constexpr int kCheckpoints = 64;

struct Checkpoint {
    void* f = nullptr;
    PartDev* p = nullptr;
    long long* step = nullptr;
    long long steps = 0;
    int cur = 0;
    int nparts = -1;
};

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// The device addresses of `scratch`, one per GPU, looked up by lbm_init.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up on the
// first call for that device), or NULL with *err set.
double* scratch_for_current_device(hipError_t* err) {
    int dev = -1;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = (double*)p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

struct lbm_handle {
    std::vector<lbm_channel_config> cfg;
    int store = 0;
    size_t elem = 8;
    hipStream_t stream = nullptr;
    void* buf[2] = {nullptr, nullptr};
    void* ws_alloc = nullptr;
    size_t buf_bytes = 0;
    std::vector<ChanDev> hchan;
    ChanDev* dchan = nullptr;
    std::vector<TileDev> htiles;
    TileDev* dtiles = nullptr;
    lbm_tuning tune{256, 1, 0, 1, 1, 0, 0, 0, 2};
    int cus = 256;                 // compute units of the device
    bool tiles_dirty = true;
    std::vector<PartHost> parts;
    std::vector<int> dev_of_user;  // user particle id -> device index
    std::vector<int> user_of_dev;
    PartDev* dparts = nullptr;
    double2* dxi = nullptr;
    double2* dnrm = nullptr;
    double* dds = nullptr;
    double2* dpatch = nullptr;
    int4* dwork = nullptr;         // particle-kernel workgroups (particle, round, channel, 0)
    int4 hwork0 = {0, 0, 0, 0};    // its first entry
    int nwork = 0;
    int2* dpsum = nullptr;         // partial-patch sum chunks (particle, first cell)
    int npsum = 0;
    int* dpcount = nullptr;        // [nparts] completion counters
    double2* dpartial = nullptr;   // per-round partial patches of particles of several rounds
    double* dmscr = nullptr;
    int* dflags = nullptr;
    int* dtlist = nullptr;
    long long* dstep = nullptr;
    double* drec = nullptr;
    int nparts = 0;
    bool alone = true;             // no channel holds more than one particle
    int tape_np = -1;              // particles and patch cells the tapes were sized for
    long long tape_cells = -1;
    int max_cells = kMaxCells;
    int cur = 0;
    long long steps = 0;
    bool finalized = false;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    Checkpoint ck[kCheckpoints];
    long long cells = 0;           // force-patch pool size
    bool pop_modified = false;     // populations replaced since lbm_init
    // adjoint (lbm_adjoint_*)
    int adj_seg = 0;               // tape capacity in steps
    std::vector<void*> tape_f;     // post-collision populations of each taped step
    PartDev* tape_p = nullptr;     // [adj_seg + 1][nparts] particle snapshots
    double2* tape_patch = nullptr; // [adj_seg][cells] force patches
    // lbm_adjoint_sweep: a second tape, filled on a second stream while the
    // first is reversed; events: [0], [1] tape k recomputed, [2], [3] tape k
    // reversed
    std::vector<void*> tape2_f;
    PartDev* tape2_p = nullptr;
    double2* tape2_patch = nullptr;
    hipStream_t stream2 = nullptr;
    hipEvent_t tape_ev[4] = {nullptr, nullptr, nullptr, nullptr};
    void* lam[2] = {nullptr, nullptr};
    size_t lam_bytes = 0;
    int lcur = 0;
    int apar = 0;
    AdjPart* dap = nullptr;
    double* dapatch = nullptr;
    double* dgmk = nullptr;
    double* dgwall = nullptr;
    long long* dgwoff = nullptr;
    int* datlist = nullptr;
    double* dgout = nullptr;
    size_t gwall_n = 0;
    long long adj_pos = -1;        // step of the state the adjoint currently refers to
    bool adj_first = false;
    double* scratch = nullptr;     // this device's address of `scratch` (lbm_get_fields_noalloc)
    std::string err;
};

#define FAIL(h, code, ...)                                                       \
    do {                                                                         \
        char _b[512];                                                            \
        snprintf(_b, sizeof(_b), __VA_ARGS__);                                   \
        if (h) (h)->err = _b; else g_err = _b;                                   \
        return code;                                                             \
    } while (0)

#define HIPCHK(h, expr)                                                          \
    do {                                                                         \
        hipError_t _e = (expr);                                                  \
        if (_e != hipSuccess)                                                    \
            FAIL(h, LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

static bool finite_all(const double* v, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

static size_t elem_size(int store) { return store == LBM_STORE_F64 ? 8 : (store == LBM_STORE_F32 ? 4 : 2); }

static int validate_cfg(const lbm_channel_config& c, int idx) {
    auto bad = [&](const char* what) {
        char b[256];
        snprintf(b, sizeof(b), "channel %d: %s", idx, what);
        g_err = b;
        return LBM_EINVAL;
    };
    if (c.nx < 3 || c.ny < 3) return bad("nx and ny must be >= 3");
    if ((long long)c.nx * c.ny > (1LL << 31) / 16) return bad("lattice too large");
    // the lattice pass addresses a channel's populations with 32-bit byte
    // offsets: 9 planes of ny x pitch elements must stay below 4 GiB
    if (9LL * c.ny * (((long long)c.nx + 63) / 64 * 64) * elem_size(c.storage) >= (1LL << 32))
        return bad("channel too large for 32-bit population offsets (9 * ny * pitch * element size >= 4 GiB)");
    if (!std::isfinite(c.tau) || !(c.tau > 0.5)) return bad("tau must be finite and > 1/2");
    if ((c.bc_x != LBM_BC_PERIODIC && c.bc_x != LBM_BC_ZOUHE) ||
        (c.bc_y != LBM_BC_PERIODIC && c.bc_y != LBM_BC_ZOUHE))
        return bad("bad boundary kind");
    if (c.bc_x == LBM_BC_ZOUHE && c.bc_y == LBM_BC_ZOUHE) {
        // a closed box: its corner closure is defined for walls at rest and
        // no fluid body force
        for (int s = 0; s < 4; ++s)
            if (c.u_wall[s][0] != 0.0 || c.u_wall[s][1] != 0.0)
                return bad("a closed box (walls on both axes) needs every wall at rest");
        if (c.body_force[0] != 0.0 || c.body_force[1] != 0.0)
            return bad("a closed box (walls on both axes) takes no fluid body force");
    }
    if (c.init != LBM_INIT_REST && c.init != LBM_INIT_COUETTE) return bad("bad init");
    if (c.init == LBM_INIT_COUETTE && c.bc_y != LBM_BC_ZOUHE) return bad("Couette start needs walls on y");
    if (c.storage < LBM_STORE_F64 || c.storage > LBM_STORE_F16S) return bad("bad storage");
    if (c.fp16_exp < 0 || c.fp16_exp > 24) return bad("fp16_exp must be in 0..24");
    if (!finite_all(&c.u_wall[0][0], 8) || !finite_all(c.body_force, 2) || !finite_all(c.gravity, 2))
        return bad("non-finite wall speed, body force or gravity");
    for (int s = 0; s < 4; ++s)
        if (std::fabs(c.u_wall[s][0]) >= 1.0 || std::fabs(c.u_wall[s][1]) >= 1.0)
            return bad("wall speed must be below 1 lattice unit");
    if (!std::isfinite(c.mls_rw) || !(c.mls_rw > 2.13)) return bad("mls_rw must exceed the 3x3 stencil radius 1.5*sqrt(2)");
    if (!std::isfinite(c.mls_alpha) || !(c.mls_alpha > 0)) return bad("mls_alpha must be > 0");
    if (!std::isfinite(c.probe_dn) || c.probe_dn < 0) return bad("probe_dn must be >= 0");
    if (c.mls_kernel < LBM_W_EXP || c.mls_kernel > LBM_W_POLY) return bad("bad mls_kernel");
    if (c.spread_scale != LBM_SPREAD_SEGMENT && c.spread_scale != LBM_SPREAD_UNIT) return bad("bad spread_scale");
    return LBM_OK;
}

static size_t pitch_of(int nx) { return round_up((size_t)nx, 64); }

static size_t plane_of(const lbm_channel_config& c) { return (size_t)c.ny * pitch_of(c.nx); }

static size_t buffer_bytes(const lbm_channel_config* cfg, int n, size_t elem) {
    size_t e = 0;
    for (int i = 0; i < n; ++i) e += 9 * plane_of(cfg[i]);
    return round_up(e * elem, 4096);
}


extern "C" size_t lbm_workspace_bytes(const lbm_channel_config* cfg, int32_t n) {
    if (!cfg || n < 1) return 0;
    for (int i = 0; i < n; ++i)
        if (validate_cfg(cfg[i], i) != LBM_OK || cfg[i].storage != cfg[0].storage) return 0;
    return 2 * buffer_bytes(cfg, n, elem_size(cfg[0].storage));
}

// Tile height of the lattice pass: 256-thread workgroups cover
// (256 / tile_w) * rows rows; the combined lattice / surface-stress launch
// of the per-node form runs 64-wide tiles in workgroups of the particle
// kernel's size (9 waves).
static int tile_height(const lbm_tuning& t) {
    // the vector form, alone or combined: one wave per rows_per_thread rows
    // of a 256-thread workgroup
    if (t.vec) return 4 * t.rows_per_thread;
    return t.overlap ? kIbmThreads / 64 * t.rows_per_thread : (256 / t.tile_w) * t.rows_per_thread;
}

static StepArgs make_args(lbm_handle* h, int cur, int parity = -1) {
    StepArgs a{};
    a.parity = parity < 0 ? cur : parity;
    a.tlist = h->dtlist;
    a.tile_w = h->tune.tile_w;
    a.tile_h = tile_height(h->tune);
    a.fin = h->buf[cur];
    a.fout = h->buf[1 - cur];
    a.chan = h->dchan;
    a.nchan = (int)h->cfg.size();
    a.tiles = h->dtiles;
    a.ntiles = (int)h->htiles.size();
    a.parts = h->dparts;
    a.nparts = h->nparts;
    a.persistent = h->tune.persistent_wgs;
    a.xcd_remap = h->tune.xcd_remap;
    a.nt_store = h->tune.nt_store;
    a.xi = h->dxi;
    a.nrm = h->dnrm;
    a.ds = h->dds;
    a.patch = h->dpatch;
    a.work = h->dwork;
    a.nwork = h->nwork;
    a.work0 = h->hwork0;
    a.psum = h->dpsum;
    a.npsum = h->npsum;
    a.sum_partials = 1;
    a.pcount = h->dpcount;
    a.partial = h->dpartial;
    a.mscr = h->dmscr;
    a.flags = h->dflags;
    a.dstep = h->dstep;
    a.rec = h->drec;
    return a;
}

static void drop_graphs(lbm_handle* h) {
    for (int i = 0; i < 2; ++i)
        if (h->gexec[i]) {
            (void)hipGraphExecDestroy(h->gexec[i]);
            h->gexec[i] = nullptr;
        }
}

static int build_tiles(lbm_handle* h) {
    const int tw = h->tune.tile_w, th = tile_height(h->tune);
    h->htiles.clear();
    for (int c = 0; c < (int)h->cfg.size(); ++c) {
        h->hchan[c].tile0 = (int)h->htiles.size();
        h->hchan[c].tiles_x = (h->cfg[c].nx + tw - 1) / tw;
        for (int y0 = 0; y0 < h->cfg[c].ny; y0 += th)
            for (int x0 = 0; x0 < h->cfg[c].nx; x0 += tw) h->htiles.push_back(TileDev{c, x0, y0, 0});
    }
    if (h->dtiles) (void)hipFree(h->dtiles);
    if (h->dtlist) (void)hipFree(h->dtlist);
    h->dtiles = nullptr;
    h->dtlist = nullptr;
    const size_t nt = h->htiles.size();
    HIPCHK(h, hipMalloc(&h->dtiles, sizeof(TileDev) * nt));
    HIPCHK(h, hipMemcpy(h->dtiles, h->htiles.data(), sizeof(TileDev) * nt, hipMemcpyHostToDevice));
    HIPCHK(h, hipMalloc(&h->dtlist, sizeof(int) * 2 * nt * kTileList));
    HIPCHK(h, hipMemset(h->dtlist, 0, sizeof(int) * 2 * nt * kTileList));
    HIPCHK(h, hipMemcpy(h->dchan, h->hchan.data(), sizeof(ChanDev) * h->hchan.size(), hipMemcpyHostToDevice));
    h->tiles_dirty = false;
    drop_graphs(h);
    return LBM_OK;
}

static void fill_chan(ChanDev& d, const lbm_channel_config& c, long long off) {
    memset(&d, 0, sizeof(d));
    d.nx = c.nx;
    d.ny = c.ny;
    d.pitch = (int)pitch_of(c.nx);
    d.bcx = c.bc_x;
    d.bcy = c.bc_y;
    d.kernel = c.mls_kernel;
    d.spread_unit = c.spread_scale == LBM_SPREAD_UNIT;
    d.off = off;
    d.plane = (long long)plane_of(c);
    d.tau = c.tau;
    d.nu = (c.tau - 0.5) / 3.0;
    for (int s = 0; s < 4; ++s)
        for (int k = 0; k < 2; ++k) {
            d.uw[s][k] = c.u_wall[s][k];
            d.f_uw[s][k] = (float)c.u_wall[s][k];
        }
    for (int k = 0; k < 2; ++k) {
        d.g[k] = c.body_force[k];
        d.grav[k] = c.gravity[k];
        d.f_g[k] = (float)c.body_force[k];
    }
    d.rw = c.mls_rw;
    d.alpha = c.mls_alpha;
    d.dn = c.probe_dn;
    d.f_omega = (float)(1.0 / c.tau);
    d.f_pref = (float)(1.0 - 1.0 / (2.0 * c.tau));
    const int kk[3] = {1, 3, 5};
    for (int k = 0; k < 3; ++k) {
        d.sc[k] = std::ldexp(1.0f, c.fp16_exp + kk[k]);
        d.isc[k] = std::ldexp(1.0f, -(c.fp16_exp + kk[k]));
    }
}

extern "C" int lbm_init(const lbm_channel_config* cfg, int32_t n, void* stream, void* workspace,
                        size_t workspace_bytes, lbm_handle** out) {
    if (!out) FAIL((lbm_handle*)nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg || n < 1) FAIL((lbm_handle*)nullptr, LBM_EINVAL, "need at least one channel config");
    for (int i = 0; i < n; ++i) {
        int r = validate_cfg(cfg[i], i);
        if (r) return r;
        if (cfg[i].storage != cfg[0].storage)
            FAIL((lbm_handle*)nullptr, LBM_EINVAL, "all channels of a handle must share the storage form");
    }
    lbm_handle* h = new (std::nothrow) lbm_handle();
    if (!h) FAIL((lbm_handle*)nullptr, LBM_ENOMEM, "out of host memory");
    {
        hipError_t e = hipSuccess;
        h->scratch = scratch_for_current_device(&e);
        if (!h->scratch) {
            delete h;
            FAIL((lbm_handle*)nullptr, LBM_EDEVICE, "address of the staging array: %s", hipGetErrorString(e));
        }
    }
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            h->cus = ncu;
    }
    h->cfg.assign(cfg, cfg + n);
    h->store = cfg[0].storage;
    h->elem = elem_size(h->store);
    h->stream = (hipStream_t)stream;
    h->buf_bytes = buffer_bytes(cfg, n, h->elem);
    const size_t need = 2 * h->buf_bytes;
    auto fail_init = [&](int code) {
        g_err = h->err;
        lbm_destroy(h);
        return code;
    };
    if (workspace) {
        if (workspace_bytes < need) {
            char b[200];
            snprintf(b, sizeof(b), "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, need);
            h->err = b;
            return fail_init(LBM_ENOMEM);
        }
        h->buf[0] = workspace;
    } else {
        if (hipMalloc(&h->ws_alloc, need) != hipSuccess) {
            h->err = "hipMalloc of the population buffers failed";
            return fail_init(LBM_ENOMEM);
        }
        h->buf[0] = h->ws_alloc;
    }
    h->buf[1] = (char*)h->buf[0] + h->buf_bytes;
    long long off = 0;
    h->hchan.resize(n);
    for (int i = 0; i < n; ++i) {
        fill_chan(h->hchan[i], cfg[i], off);
        off += 9LL * (long long)plane_of(cfg[i]);
    }
    int r;
    if (hipMalloc(&h->dchan, sizeof(ChanDev) * n) != hipSuccess ||
        hipMalloc(&h->dflags, sizeof(int) * 4) != hipSuccess ||
        hipMalloc(&h->dstep, sizeof(long long)) != hipSuccess) {
        h->err = "hipMalloc of handle state failed";
        return fail_init(LBM_ENOMEM);
    }
    if (hipMemcpy(h->dchan, h->hchan.data(), sizeof(ChanDev) * n, hipMemcpyHostToDevice) != hipSuccess) {
        h->err = "upload of channel table failed";
        return fail_init(LBM_EDEVICE);
    }
    int fl[4] = {0, INT_MAX, 0, 0};
    long long z = 0;
    if (hipMemcpy(h->dflags, fl, sizeof(fl), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->dstep, &z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess) {
        h->err = "upload of flags failed";
        return fail_init(LBM_EDEVICE);
    }
    if ((r = build_tiles(h)) != LBM_OK) return fail_init(r);
    StepArgs a = make_args(h, 1);  // fout = buf[0]
    for (int c = 0; c < n; ++c) {
        hipError_t e = launch_init(h->store, a, c, cfg[c].init, cfg[c].nx, cfg[c].ny, h->stream);
        if (e != hipSuccess) {
            h->err = std::string("init kernel: ") + hipGetErrorString(e);
            return fail_init(LBM_EDEVICE);
        }
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess) {
        h->err = "init synchronisation failed";
        return fail_init(LBM_EDEVICE);
    }
    h->cur = 0;
    *out = h;
    return LBM_OK;
}

extern "C" int lbm_add_particle(lbm_handle* h, int32_t channel, const lbm_particle_desc* d, int32_t* out_id) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    if (h->finalized) FAIL(h, LBM_ESTATE, "particles can only be added before the first step (or after lbm_reset)");
    if (!d || channel < 0 || channel >= (int)h->cfg.size()) FAIL(h, LBM_EINVAL, "bad channel or descriptor");
    const int n = d->n_markers;
    if (n < 3 || n > kMaxMarkers) FAIL(h, LBM_EINVAL, "n_markers must be in 3..%d", kMaxMarkers);
    if (!d->xi || !d->nrm || !d->ds) FAIL(h, LBM_EINVAL, "marker arrays must not be NULL");
    double sc[9] = {d->x, d->y, d->theta, d->u, d->v, d->omega, d->density_ratio, d->area, d->polar_moment};
    if (!finite_all(sc, 9) || !finite_all(d->xi, 2 * (size_t)n) || !finite_all(d->nrm, 2 * (size_t)n) ||
        !finite_all(d->ds, n))
        FAIL(h, LBM_EINVAL, "non-finite particle value");
    if (!(d->density_ratio > 0) || !(d->area > 0) || !(d->polar_moment > 0))
        FAIL(h, LBM_EINVAL, "density_ratio, area and polar_moment must be > 0");
    double rb = 0;
    for (int l = 0; l < n; ++l) {
        double nn = d->nrm[2 * l] * d->nrm[2 * l] + d->nrm[2 * l + 1] * d->nrm[2 * l + 1];
        if (std::fabs(nn - 1.0) > 1e-6) FAIL(h, LBM_EINVAL, "marker %d: normal is not a unit vector", l);
        if (!(d->ds[l] > 0)) FAIL(h, LBM_EINVAL, "marker %d: ds must be > 0", l);
        rb = std::max(rb, std::sqrt(d->xi[2 * l] * d->xi[2 * l] + d->xi[2 * l + 1] * d->xi[2 * l + 1]));
    }
    const lbm_channel_config& c = h->cfg[channel];
    const double reach = rb + 3.0;
    if (c.bc_y == LBM_BC_ZOUHE && (d->y - reach < 0 || d->y + reach > c.ny - 1))
        FAIL(h, LBM_EINVAL, "particle closer than 3 nodes to a wall");
    if (c.bc_x == LBM_BC_ZOUHE && (d->x - reach < 0 || d->x + reach > c.nx - 1))
        FAIL(h, LBM_EINVAL, "particle closer than 3 nodes to a wall");
    if (c.bc_y == LBM_BC_PERIODIC && (d->y < -1e6 || d->y > 1e6)) FAIL(h, LBM_EINVAL, "position out of range");
    if (c.bc_x == LBM_BC_PERIODIC && (d->x < -1e6 || d->x > 1e6)) FAIL(h, LBM_EINVAL, "position out of range");
    // the force patch spans the anchors of [X - rb, X + rb] plus one node of
    // stencil on each side: at most ceil(2 rb) + 4 nodes per axis
    const int side = (int)std::ceil(2.0 * rb) + 6;
    if (side > c.nx || side > c.ny) FAIL(h, LBM_EINVAL, "particle wider than the channel");
    if ((long long)side * side > h->max_cells)
        FAIL(h, LBM_ECAPACITY, "particle too large for the force patch (%d cells > %d)", side * side, h->max_cells);
    PartHost p;
    p.d = *d;
    p.xi.assign(d->xi, d->xi + 2 * n);
    p.nrm.assign(d->nrm, d->nrm + 2 * n);
    p.ds.assign(d->ds, d->ds + n);
    p.chan = channel;
    p.rb = rb;
    p.cap = side * side;
    h->parts.push_back(std::move(p));
    if (out_id) *out_id = (int)h->parts.size() - 1;
    return LBM_OK;
}

// The device buffers finalize allocates for the particle set.
static void free_particle_buffers(lbm_handle* h) {
    void** bufs[] = {(void**)&h->dparts, (void**)&h->dxi, (void**)&h->dnrm, (void**)&h->dds,
                     (void**)&h->dpatch, (void**)&h->dmscr, (void**)&h->drec, (void**)&h->dwork,
                     (void**)&h->dpsum, (void**)&h->dpcount, (void**)&h->dpartial};
    for (void** p : bufs) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
}

static int finalize(lbm_handle* h) {
    if (h->finalized) return LBM_OK;
    // a finalize that failed part-way left some buffers: start from none
    free_particle_buffers(h);
    const int np = (int)h->parts.size();
    std::vector<int> order(np);
    for (int i = 0; i < np; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return h->parts[a].chan < h->parts[b].chan; });
    h->dev_of_user.assign(np, 0);
    h->user_of_dev = order;
    std::vector<PartDev> pd(np);
    std::vector<double2> xi, nrm;
    std::vector<double> ds;
    long long cells = 0;
    for (auto& ch : h->hchan) ch.p_begin = ch.p_end = 0;
    for (int k = 0; k < np; ++k) {
        const PartHost& P = h->parts[order[k]];
        h->dev_of_user[order[k]] = k;
        PartDev& q = pd[k];
        memset(&q, 0, sizeof(q));
        q.X[0] = q.Xm[0] = P.d.x;
        q.X[1] = q.Xm[1] = P.d.y;
        q.th = q.thm = P.d.theta;
        q.cth = std::cos(q.th);
        q.sth = std::sin(q.th);
        q.V[0] = q.Vm[0] = P.d.u;
        q.V[1] = q.Vm[1] = P.d.v;
        q.Om = q.Omm = P.d.omega;
        q.ratio = P.d.density_ratio;
        q.rb = P.rb;
        q.m = P.d.density_ratio * P.d.area;
        q.I = P.d.density_ratio * P.d.polar_moment;
        q.chan = P.chan;
        q.mbeg = (int)ds.size();
        q.nm = P.d.n_markers;
        q.patch_cap = P.cap;
        q.patch_off = cells;
        cells += P.cap;
        for (int l = 0; l < q.nm; ++l) {
            xi.push_back(make_double2(P.xi[2 * l], P.xi[2 * l + 1]));
            nrm.push_back(make_double2(P.nrm[2 * l], P.nrm[2 * l + 1]));
            ds.push_back(P.ds[l]);
        }
        ChanDev& ch = h->hchan[P.chan];
        if (ch.p_end == ch.p_begin) ch.p_begin = k;
        ch.p_end = k + 1;
    }
    h->nparts = np;
    h->cells = cells;
    h->alone = true;
    for (const auto& ch : h->hchan) h->alone = h->alone && ch.p_end - ch.p_begin <= 1;
    const size_t nmk = std::max<size_t>(ds.size(), 1);
    HIPCHK(h, hipMalloc(&h->dparts, sizeof(PartDev) * std::max(np, 1)));
    HIPCHK(h, hipMalloc(&h->dxi, sizeof(double2) * nmk));
    HIPCHK(h, hipMalloc(&h->dnrm, sizeof(double2) * nmk));
    HIPCHK(h, hipMalloc(&h->dds, sizeof(double) * nmk));
    HIPCHK(h, hipMalloc(&h->dpatch, sizeof(double2) * std::max<long long>(cells, 1)));
    HIPCHK(h, hipMalloc(&h->dmscr, sizeof(double) * 4 * nmk));
    // Particle-kernel work: one workgroup per round of kRound markers in both
    // particle kernels.  A particle of several rounds gets one partial force
    // patch per round, summed by chunks of 256 cells.
    std::vector<int4> work;
    std::vector<int2> psum;
    long long pcells = 0;
    for (int k = 0; k < np; ++k) {
        const int nr = (pd[k].nm + kRound - 1) / kRound;
        for (int r = 0; r < nr; ++r)
            work.push_back(work_entry(k, r, std::min(kRound, pd[k].nm - r * kRound), pd[k].chan,
                                      pd[k].mbeg + r * kRound));
        pd[k].part_off = pcells;
        if (nr > 1) {
            pcells += (long long)nr * pd[k].patch_cap;
            for (int q = 0; q < pd[k].patch_cap; q += 256) psum.push_back(make_int2(k, q));
        }
    }
    h->nwork = (int)work.size();
    h->hwork0 = work.empty() ? make_int4(0, 0, 0, 0) : work[0];
    h->npsum = (int)psum.size();
    HIPCHK(h, hipMalloc(&h->dpartial, sizeof(double2) * std::max<long long>(pcells, 1)));
    HIPCHK(h, hipMalloc(&h->dwork, sizeof(int4) * std::max<size_t>(work.size(), 1)));
    HIPCHK(h, hipMalloc(&h->dpsum, sizeof(int2) * std::max<size_t>(psum.size(), 1)));
    HIPCHK(h, hipMalloc(&h->dpcount, sizeof(int) * std::max(np, 1)));
    HIPCHK(h, hipMemset(h->dpcount, 0, sizeof(int) * std::max(np, 1)));
    if (!work.empty())
        HIPCHK(h, hipMemcpy(h->dwork, work.data(), sizeof(int4) * work.size(), hipMemcpyHostToDevice));
    if (!psum.empty())
        HIPCHK(h, hipMemcpy(h->dpsum, psum.data(), sizeof(int2) * psum.size(), hipMemcpyHostToDevice));
    HIPCHK(h, hipMalloc(&h->drec, sizeof(double) * 10 * kRecSlots * std::max(np, 1)));
    if (np) {
        HIPCHK(h, hipMemcpy(h->dparts, pd.data(), sizeof(PartDev) * np, hipMemcpyHostToDevice));
        HIPCHK(h, hipMemcpy(h->dxi, xi.data(), sizeof(double2) * xi.size(), hipMemcpyHostToDevice));
        HIPCHK(h, hipMemcpy(h->dnrm, nrm.data(), sizeof(double2) * nrm.size(), hipMemcpyHostToDevice));
        HIPCHK(h, hipMemcpy(h->dds, ds.data(), sizeof(double) * ds.size(), hipMemcpyHostToDevice));
    }
    HIPCHK(h, hipMemset(h->dpatch, 0, sizeof(double2) * std::max<long long>(cells, 1)));
    HIPCHK(h, hipMemcpy(h->dchan, h->hchan.data(), sizeof(ChanDev) * h->hchan.size(), hipMemcpyHostToDevice));
    h->finalized = true;
    return LBM_OK;
}

// Lattice pass and surface stress of one step, after its force stage: two
// launches, or one combined launch in the overlap mode.
static int enqueue_rest(lbm_handle* h, const StepArgs& a, hipStream_t s) {
    if (h->tune.overlap) {
        HIPCHK(h, launch_lattice_traction(h->store, a, h->tune.rows_per_thread, h->tune.vec, s));
    } else {
        HIPCHK(h, launch_lattice(h->store, a, h->tune.tile_w, h->tune.rows_per_thread, h->tune.vec, s));
        HIPCHK(h, launch_traction(h->store, a, s));
    }
    return LBM_OK;
}

static int enqueue_step(lbm_handle* h, int cur) {
    StepArgs a = make_args(h, cur);
    HIPCHK(h, launch_ibm_force(h->store, a, h->stream));
    return enqueue_rest(h, a, h->stream);
}

static int run_steps(lbm_handle* h, long long n) {
    const bool graph = h->tune.use_graph && h->stream != nullptr;
    while (n > 0) {
        if (graph && n >= 2) {
            const int par = h->cur;
            // both parities' two-step graphs are built together, so that a
            // later call starting at the other parity (after an odd number of
            // steps) replays without capturing
            for (int q = 0; q < 2; ++q) {
                const int p = (par + q) & 1;
                if (h->gexec[p]) continue;
                hipGraph_t g = nullptr;
                HIPCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
                int r1 = enqueue_step(h, p);
                int r2 = r1 == LBM_OK ? enqueue_step(h, 1 - p) : r1;
                hipError_t e = hipStreamEndCapture(h->stream, &g);
                if (r2 != LBM_OK) return r2;
                HIPCHK(h, e);
                hipError_t ei = hipGraphInstantiate(&h->gexec[p], g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                HIPCHK(h, ei);
            }
            const long long reps = n / 2;
            for (long long r = 0; r < reps; ++r) HIPCHK(h, hipGraphLaunch(h->gexec[par], h->stream));
            h->steps += 2 * reps;
            n -= 2 * reps;
        } else {
            int r = enqueue_step(h, h->cur);
            if (r) return r;
            h->cur = 1 - h->cur;
            h->steps += 1;
            n -= 1;
        }
    }
    return LBM_OK;
}

static int check_flags(lbm_handle* h) {
    int fl[4];
    HIPCHK(h, hipMemcpyAsync(fl, h->dflags, sizeof(fl), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (fl[2] & 2) FAIL(h, LBM_ECAPACITY, "a particle's probe reach outgrew its adjoint patch");
    if (fl[2]) FAIL(h, LBM_ECAPACITY, "a particle outgrew its force patch");
    if (fl[0])
        FAIL(h, LBM_EUNSTABLE, "non-finite or non-positive density or particle state in step %d (counting from 1)",
             fl[1] + 1);
    return LBM_OK;
}

extern "C" int lbm_step(lbm_handle* h, int32_t n, double* traj) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    if (n < 0) FAIL(h, LBM_EINVAL, "n_steps must be >= 0");
    int r;
    if ((r = finalize(h)) != LBM_OK) return r;
    if (h->tiles_dirty && (r = build_tiles(h)) != LBM_OK) return r;
    if (!traj || h->nparts == 0) {
        if ((r = run_steps(h, n)) != LBM_OK) return r;
        return check_flags(h);
    }
    std::vector<double> rec((size_t)kRecSlots * h->nparts * 10);
    long long done = 0;
    while (done < n) {
        const long long chunk = std::min<long long>(kRecSlots, n - done);
        const long long s0 = h->steps;
        if ((r = run_steps(h, chunk)) != LBM_OK) return r;
        HIPCHK(h, hipMemcpyAsync(rec.data(), h->drec, sizeof(double) * rec.size(), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        for (long long j = 0; j < chunk; ++j) {
            const long long slot = (s0 + j) % kRecSlots;
            for (int u = 0; u < h->nparts; ++u) {
                const int k = h->dev_of_user[u];
                memcpy(traj + ((done + j) * h->nparts + u) * 10, &rec[(slot * h->nparts + k) * 10], 10 * sizeof(double));
            }
        }
        done += chunk;
    }
    return check_flags(h);
}

extern "C" int lbm_get_particles(const lbm_handle* hc, double* out, int32_t cap, int32_t* n_out) {
    lbm_handle* h = const_cast<lbm_handle*>(hc);
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    const int np = (int)h->parts.size();
    if (n_out) *n_out = np;
    if (cap < np) FAIL(h, LBM_ECAPACITY, "output holds %d particles, %d needed", cap, np);
    if (np == 0) return LBM_OK;
    if (!out) FAIL(h, LBM_EINVAL, "out is NULL");
    if (!h->finalized) {
        for (int u = 0; u < np; ++u) {
            const lbm_particle_desc& d = h->parts[u].d;
            double v[10] = {d.x, d.y, d.theta, d.u, d.v, d.omega, 0, 0, 0, (double)h->parts[u].chan};
            memcpy(out + 10 * u, v, sizeof(v));
        }
        return LBM_OK;
    }
    std::vector<PartDev> pd(np);
    HIPCHK(h, hipMemcpyAsync(pd.data(), h->dparts, sizeof(PartDev) * np, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int u = 0; u < np; ++u) {
        const PartDev& q = pd[h->dev_of_user[u]];
        double v[10] = {q.X[0], q.X[1], q.th, q.V[0], q.V[1], q.Om, q.F[0], q.F[1], q.M, (double)q.chan};
        memcpy(out + 10 * u, v, sizeof(v));
    }
    return LBM_OK;
}

extern "C" int lbm_get_populations(lbm_handle* h, int32_t ch, double* f) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    if (ch < 0 || ch >= (int)h->cfg.size() || !f) FAIL(h, LBM_EINVAL, "bad channel or NULL output");
    int r;
    if ((r = finalize(h)) != LBM_OK) return r;
    const size_t n = (size_t)h->cfg[ch].nx * h->cfg[ch].ny;
    double* d = nullptr;
    HIPCHK(h, hipMalloc(&d, sizeof(double) * 9 * n));
    StepArgs a = make_args(h, h->cur);
    hipError_t e = launch_fields(h->store, a, ch, h->cfg[ch].nx, h->cfg[ch].ny, d, nullptr, nullptr, nullptr, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, d, sizeof(double) * 9 * n, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(d);
    HIPCHK(h, e);
    return LBM_OK;
}

extern "C" int lbm_get_fields(lbm_handle* h, int32_t ch, double* rho, double* ux, double* uy) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    if (ch < 0 || ch >= (int)h->cfg.size()) FAIL(h, LBM_EINVAL, "bad channel");
    int r;
    if ((r = finalize(h)) != LBM_OK) return r;
    const size_t n = (size_t)h->cfg[ch].nx * h->cfg[ch].ny;
    double* d = nullptr;
    HIPCHK(h, hipMalloc(&d, sizeof(double) * 3 * n));
    StepArgs a = make_args(h, h->cur);
    hipError_t e = launch_fields(h->store, a, ch, h->cfg[ch].nx, h->cfg[ch].ny, nullptr, d, d + n, d + 2 * n, h->stream);
    double* outs[3] = {rho, ux, uy};
    for (int k = 0; k < 3 && e == hipSuccess; ++k)
        if (outs[k]) e = hipMemcpyAsync(outs[k], d + k * n, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(d);
    HIPCHK(h, e);
    return LBM_OK;
}

extern "C" int lbm_get_fields_noalloc(lbm_handle* h, int32_t ch, double* rho, double* ux, double* uy) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    if (ch < 0 || ch >= (int)h->cfg.size()) FAIL(h, LBM_EINVAL, "bad channel");
    const long long n = (long long)h->cfg[ch].nx * h->cfg[ch].ny;
    if (n > kScratchNodes)
        FAIL(h, LBM_ECAPACITY, "channel %d has %lld nodes; lbm_get_fields_noalloc stages at most %d (use lbm_get_fields)",
             ch, n, kScratchNodes);
    double* d = h->scratch;  // this device's staging array, no allocation
    StepArgs a = make_args(h, h->cur);
    HIPCHK(h, launch_fields(h->store, a, ch, h->cfg[ch].nx, h->cfg[ch].ny, nullptr, d, d + n, d + 2 * n, h->stream));
    double* outs[3] = {rho, ux, uy};
    for (int k = 0; k < 3; ++k)
        if (outs[k]) HIPCHK(h, hipMemcpyAsync(outs[k], d + k * n, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

extern "C" int lbm_set_populations(lbm_handle* h, int32_t ch, const double* f) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    if (ch < 0 || ch >= (int)h->cfg.size() || !f) FAIL(h, LBM_EINVAL, "bad channel or NULL input");
    const size_t n = (size_t)h->cfg[ch].nx * h->cfg[ch].ny;
    if (!finite_all(f, 9 * n)) FAIL(h, LBM_EINVAL, "non-finite population");
    h->pop_modified = true;
    double* d = nullptr;
    HIPCHK(h, hipMalloc(&d, sizeof(double) * 9 * n));
    hipError_t e = hipMemcpyAsync(d, f, sizeof(double) * 9 * n, hipMemcpyHostToDevice, h->stream);
    StepArgs a = make_args(h, 1 - h->cur);  // fout = buf[cur]
    if (e == hipSuccess) e = launch_set_pop(h->store, a, ch, h->cfg[ch].nx, h->cfg[ch].ny, d, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(d);
    HIPCHK(h, e);
    return LBM_OK;
}

extern "C" int lbm_checkpoint_save(lbm_handle* h, int32_t slot) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    if (slot < 0 || slot >= kCheckpoints) FAIL(h, LBM_EINVAL, "slot must be in 0..%d", kCheckpoints - 1);
    int r;
    if ((r = finalize(h)) != LBM_OK) return r;
    Checkpoint& c = h->ck[slot];
    if (!c.f) HIPCHK(h, hipMalloc(&c.f, h->buf_bytes));
    if (!c.p) HIPCHK(h, hipMalloc(&c.p, sizeof(PartDev) * std::max(h->nparts, 1)));
    if (!c.step) HIPCHK(h, hipMalloc(&c.step, sizeof(long long)));
    HIPCHK(h, hipMemcpyAsync(c.f, h->buf[h->cur], h->buf_bytes, hipMemcpyDeviceToDevice, h->stream));
    if (h->nparts) HIPCHK(h, hipMemcpyAsync(c.p, h->dparts, sizeof(PartDev) * h->nparts, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(c.step, h->dstep, sizeof(long long), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    c.steps = h->steps;
    c.cur = h->cur;
    c.nparts = h->nparts;
    return LBM_OK;
}

extern "C" int lbm_checkpoint_restore(lbm_handle* h, int32_t slot) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    if (slot < 0 || slot >= kCheckpoints) FAIL(h, LBM_EINVAL, "slot must be in 0..%d", kCheckpoints - 1);
    Checkpoint& c = h->ck[slot];
    if (!c.f || c.nparts != h->nparts || !h->finalized) FAIL(h, LBM_ESTATE, "slot %d holds no compatible checkpoint", slot);
    HIPCHK(h, hipMemcpyAsync(h->buf[c.cur], c.f, h->buf_bytes, hipMemcpyDeviceToDevice, h->stream));
    if (h->nparts) HIPCHK(h, hipMemcpyAsync(h->dparts, c.p, sizeof(PartDev) * h->nparts, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->dstep, c.step, sizeof(long long), hipMemcpyDeviceToDevice, h->stream));
    int fl[4] = {0, INT_MAX, 0, 0};
    HIPCHK(h, hipMemcpyAsync(h->dflags, fl, sizeof(fl), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->cur = c.cur;
    h->steps = c.steps;
    return LBM_OK;
}

static void free_adjoint(lbm_handle* h);

// Back to the state lbm_init leaves: the initial populations, no particles,
// step 0.  The channel configs, the stream, the workspace and the tuning are
// kept; the particle buffers, checkpoints, graphs and adjoint state go.
extern "C" int lbm_reset(lbm_handle* h) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    HIPCHK(h, hipStreamSynchronize(h->stream));  // nothing of the old run in flight
    drop_graphs(h);
    free_adjoint(h);
    free_particle_buffers(h);
    for (auto& c : h->ck) {
        if (c.f) (void)hipFree(c.f);
        if (c.p) (void)hipFree(c.p);
        if (c.step) (void)hipFree(c.step);
        c = Checkpoint{};
    }
    h->parts.clear();
    h->dev_of_user.clear();
    h->user_of_dev.clear();
    h->nparts = h->nwork = h->npsum = 0;
    h->cells = 0;
    h->finalized = false;
    h->pop_modified = false;
    h->steps = 0;
    for (auto& ch : h->hchan) ch.p_begin = ch.p_end = 0;
    int r;
    if ((r = build_tiles(h)) != LBM_OK) return r;  // cleared tile lists, channel table uploaded
    int fl[4] = {0, INT_MAX, 0, 0};
    long long z = 0;
    HIPCHK(h, hipMemcpy(h->dflags, fl, sizeof(fl), hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(h->dstep, &z, sizeof(z), hipMemcpyHostToDevice));
    StepArgs a = make_args(h, 1);  // fout = buf[0]
    for (int c = 0; c < (int)h->cfg.size(); ++c)
        HIPCHK(h, launch_init(h->store, a, c, h->cfg[c].init, h->cfg[c].nx, h->cfg[c].ny, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->cur = 0;
    return LBM_OK;
}

extern "C" int lbm_set_tuning(lbm_handle* h, const lbm_tuning* t) {
    if (!h || !t) FAIL(h, LBM_EINVAL, "NULL argument");
    if (t->vec != 0 && t->vec != 1) FAIL(h, LBM_EINVAL, "vec must be 0 or 1");
    if (t->nt_store != 0 && t->nt_store != 1) FAIL(h, LBM_EINVAL, "nt_store must be 0 or 1");
    if (t->nt_store && !t->vec) FAIL(h, LBM_EINVAL, "nt_store = 1 needs vec = 1");
    if (!t->vec && t->tile_w != 64 && t->tile_w != 128 && t->tile_w != 256)
        FAIL(h, LBM_EINVAL, "tile_w must be 64, 128 or 256");
    if (t->vec) {
        // tile_w / 64 nodes per lane, one chunk of at most 16 bytes per plane
        const int nv = t->tile_w / 64;
        if (t->tile_w % 64 != 0 || (nv != 1 && nv != 2 && nv != 4 && nv != 8) || nv * (int)h->elem > 16)
            FAIL(h, LBM_EINVAL, "vec = 1 needs tile_w = 64 * nv with nv in {1, 2, 4, 8} and nv * element size <= 16 bytes");
        if (t->rows_per_thread > 2) FAIL(h, LBM_EINVAL, "vec = 1 needs rows_per_thread 1 or 2");
        if (t->overlap && (t->rows_per_thread != 1 || t->persistent_wgs != 0))
            FAIL(h, LBM_EINVAL, "vec = 1 with overlap = 1 needs rows_per_thread 1 and persistent_wgs 0");
    }
    if (t->rows_per_thread != 1 && t->rows_per_thread != 2 && t->rows_per_thread != 4)
        FAIL(h, LBM_EINVAL, "rows_per_thread must be 1, 2 or 4");
    if (t->persistent_wgs < 0) FAIL(h, LBM_EINVAL, "persistent_wgs must be >= 0");
    if (t->use_graph != 0 && t->use_graph != 1) FAIL(h, LBM_EINVAL, "use_graph must be 0 or 1");
    if (t->xcd_remap != 0 && t->xcd_remap != 1) FAIL(h, LBM_EINVAL, "xcd_remap must be 0 or 1");
    if (t->overlap != 0 && t->overlap != 1) FAIL(h, LBM_EINVAL, "overlap must be 0 or 1");
    if (t->adj_fused < 0 || t->adj_fused > 2) FAIL(h, LBM_EINVAL, "adj_fused must be 0, 1 or 2");
    if (t->overlap && !t->vec && (t->tile_w != 64 || t->persistent_wgs != 0))
        FAIL(h, LBM_EINVAL, "overlap = 1 needs tile_w = 64 and persistent_wgs = 0");
    const bool tiles = t->tile_w != h->tune.tile_w || tile_height(*t) != tile_height(h->tune);
    h->tune = *t;
    if (tiles) h->tiles_dirty = true;
    drop_graphs(h);
    return LBM_OK;
}

extern "C" int lbm_get_tuning(const lbm_handle* h, lbm_tuning* t) {
    if (!h || !t) return LBM_EINVAL;
    *t = h->tune;
    return LBM_OK;
}

extern "C" int lbm_time_kernels(lbm_handle* h, int32_t reps, double out_us[3]) {
    if (!h || !out_us || reps < 1) FAIL(h, LBM_EINVAL, "bad argument");
    int r;
    if ((r = finalize(h)) != LBM_OK) return r;
    if (h->tiles_dirty && (r = build_tiles(h)) != LBM_OK) return r;
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    const int par0 = h->cur;
    // The lattice pass adds the IB force in the tiles listed by the force
    // stage of the same step, and each lattice pass clears the other parity's
    // lists; the half read here was cleared by the last step.  So the first
    // force launch runs before the lattice phase, filling the lists as in a
    // step (it is timed with the other force launches), and the lattice
    // launches follow on those lists.  Later force launches append copies,
    // which the lattice pass drops (it sorts and deduplicates).
    float ms_first = 0.0f;
    {
        HIPCHK(h, hipEventRecord(e0, h->stream));
        StepArgs a = make_args(h, h->cur, par0);
        HIPCHK(h, launch_ibm_force(h->store, a, h->stream));
        HIPCHK(h, hipEventRecord(e1, h->stream));
        HIPCHK(h, hipEventSynchronize(e1));
        HIPCHK(h, hipEventElapsedTime(&ms_first, e0, e1));
    }
    const int order[3] = {1, 0, 2};
    for (int kk = 0; kk < 3; ++kk) {
        const int k = order[kk];
        const int n = k == 0 ? reps - 1 : reps;  // the first force launch ran above
        HIPCHK(h, hipEventRecord(e0, h->stream));
        for (int i = 0; i < n; ++i) {
            StepArgs a = make_args(h, h->cur, par0);
            if (k == 0) HIPCHK(h, launch_ibm_force(h->store, a, h->stream));
            if (k == 1) {
                if (h->tune.overlap) {
                    // the combined launch without its particle workgroups
                    a.nwork = 0;
                    HIPCHK(h, launch_lattice_traction(h->store, a, h->tune.rows_per_thread, h->tune.vec, h->stream));
                } else {
                    HIPCHK(h, launch_lattice(h->store, a, h->tune.tile_w, h->tune.rows_per_thread, h->tune.vec, h->stream));
                }
                h->cur = 1 - h->cur;
            }
            if (k == 2) HIPCHK(h, launch_traction(h->store, a, h->stream));
        }
        HIPCHK(h, hipEventRecord(e1, h->stream));
        HIPCHK(h, hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
        if (k == 0) ms += ms_first;
        out_us[k] = (k == 2 && h->nparts == 0) ? 0.0 : 1e3 * ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->steps += reps;  // every phase advanced its part of the state reps times
    return check_flags(h);
}


// ---------------------------------------------------------------------------
// Adjoint.
// ---------------------------------------------------------------------------
static void free_tape2(lbm_handle* h) {
    for (void* p : h->tape2_f)
        if (p) (void)hipFree(p);
    h->tape2_f.clear();
    if (h->tape2_p) (void)hipFree(h->tape2_p);
    if (h->tape2_patch) (void)hipFree(h->tape2_patch);
    h->tape2_p = nullptr;
    h->tape2_patch = nullptr;
}

// Both tapes of the adjoint.
static void free_tapes(lbm_handle* h) {
    free_tape2(h);
    for (void* p : h->tape_f)
        if (p) (void)hipFree(p);
    h->tape_f.clear();
    if (h->tape_p) (void)hipFree(h->tape_p);
    if (h->tape_patch) (void)hipFree(h->tape_patch);
    h->tape_p = nullptr;
    h->tape_patch = nullptr;
    h->tape_np = -1;
    h->tape_cells = -1;
}
// The adjoint state other than the tapes.
static void free_adjoint_state(lbm_handle* h) {
    void* ptrs[] = {h->lam[0], h->dap, h->dapatch, h->dgmk, h->dgwall, h->dgwoff, h->datlist, h->dgout};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    h->lam[0] = h->lam[1] = nullptr;
    h->dap = nullptr;
    h->dapatch = nullptr;
    h->dgmk = h->dgwall = h->dgout = nullptr;
    h->dgwoff = nullptr;
    h->datlist = nullptr;
    h->adj_seg = 0;
    h->adj_pos = -1;
}
static void free_adjoint(lbm_handle* h) {
    free_tapes(h);
    free_adjoint_state(h);
}

static AdjArgs adj_args(lbm_handle* h) {
    AdjArgs a{};
    a.s = make_args(h, h->cur);
    a.s.parity = h->apar;
    a.ap = h->dap;
    a.apatch = h->dapatch;
    a.gmk = h->dgmk;
    a.gwall = h->dgwall;
    a.gw_off = h->dgwoff;
    a.atlist = h->datlist;
    a.lam_in = h->lam[h->lcur];
    a.lam_out = h->lam[1 - h->lcur];
    return a;
}

extern "C" int lbm_adjoint_begin(lbm_handle* h, const double* seed, int32_t max_segment) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    if (max_segment < 1) FAIL(h, LBM_EINVAL, "max_segment must be >= 1");
    int r;
    if ((r = finalize(h)) != LBM_OK) return r;
    if (h->tiles_dirty && (r = build_tiles(h)) != LBM_OK) return r;
    const int np = h->nparts;
    if (np > 0 && !seed) FAIL(h, LBM_EINVAL, "seed is NULL");
    if (np > 0 && !finite_all(seed, 10 * (size_t)np)) FAIL(h, LBM_EINVAL, "non-finite seed");
    const int nch = (int)h->cfg.size();
    // the adjoint populations are addressed like f, with 32-bit byte offsets
    // inside a channel's block, at 8 bytes (FP64 form) or 4 bytes per value
    const size_t lam_elem = h->store == LBM_STORE_F64 ? 8 : 4;
    for (int c = 0; c < nch; ++c) {
        if (9 * (size_t)plane_of(h->cfg[c]) * lam_elem >= ((size_t)1 << 32))
            FAIL(h, LBM_EINVAL, "channel %d: its adjoint populations reach 4 GiB", c);
        if (h->cfg[c].bc_x == LBM_BC_ZOUHE && h->cfg[c].bc_y == LBM_BC_ZOUHE)
            FAIL(h, LBM_EINVAL, "channel %d: the adjoint has no transpose of the closed-box corner closure", c);
    }
    // adjoint patches: the stencils of the markers and of their probes
    std::vector<AdjPart> ap(std::max(np, 1));
    long long acells = 0;
    for (int k = 0; k < np; ++k) {
        const PartHost& P = h->parts[h->user_of_dev[k]];
        const lbm_channel_config& c = h->cfg[P.chan];
        const int side = (int)std::ceil(2.0 * (P.rb + c.probe_dn)) + 6;
        if (side > c.nx || side > c.ny)
            FAIL(h, LBM_EINVAL, "particle %d: probe reach wider than its channel", h->user_of_dev[k]);
        AdjPart& A = ap[k];
        memset(&A, 0, sizeof(A));
        const double* sd = seed + 10 * h->user_of_dev[k];
        A.l[AL_X] = sd[0];
        A.l[AL_X + 1] = sd[1];
        A.l[AL_TH] = sd[2];
        A.l[AL_V] = sd[3];
        A.l[AL_V + 1] = sd[4];
        A.l[AL_OM] = sd[5];
        A.seed[0] = sd[6];
        A.seed[1] = sd[7];
        A.seed[2] = sd[8];
        A.acap = side * side;
        A.aoff = acells;
        acells += A.acap;
    }
    std::vector<long long> gwoff(nch);
    size_t gw = 0;
    for (int c = 0; c < nch; ++c) {
        const lbm_channel_config& cf = h->cfg[c];
        gwoff[c] = (long long)gw;
        const size_t nwall = cf.bc_y == LBM_BC_ZOUHE ? 2 * (size_t)cf.nx : (cf.bc_x == LBM_BC_ZOUHE ? 2 * (size_t)cf.ny : 0);
        gw += 2 * nwall + (size_t)cf.ny;
    }
    // the tapes of a previous adjoint of the same length and particle set
    // are kept: every tape slot is written before it is read
    free_adjoint_state(h);
    if (h->tape_f.size() != (size_t)max_segment || h->tape_np != np || h->tape_cells != h->cells) free_tapes(h);
    size_t planes = 0;
    for (auto& c : h->cfg) planes += 9 * plane_of(c);
    h->lam_bytes = round_up(planes * lam_elem, 4096);
    const size_t nmk = std::max<size_t>(1, [&] {
        size_t m = 0;
        for (auto& p : h->parts) m += p.d.n_markers;
        return m;
    }());
    const size_t nt = h->htiles.size();
    auto alloc = [&](void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 8)) == hipSuccess; };
    if (h->tape_f.empty()) {
        h->tape_f.assign(max_segment, nullptr);
        for (int t = 0; t < max_segment; ++t)
            if (hipMalloc(&h->tape_f[t], h->buf_bytes) != hipSuccess) {
                free_adjoint(h);
                FAIL(h, LBM_ENOMEM, "tape of %d steps (%zu bytes each) does not fit", max_segment, h->buf_bytes);
            }
        if (!alloc((void**)&h->tape_p, sizeof(PartDev) * (size_t)(max_segment + 1) * std::max(np, 1)) ||
            !alloc((void**)&h->tape_patch, sizeof(double2) * (size_t)max_segment * std::max<long long>(h->cells, 1))) {
            free_adjoint(h);
            FAIL(h, LBM_ENOMEM, "allocation of the adjoint tape failed");
        }
        h->tape_np = np;
        h->tape_cells = h->cells;
    }
    bool ok = alloc(&h->lam[0], 2 * h->lam_bytes) && alloc((void**)&h->dap, sizeof(AdjPart) * ap.size()) &&
              alloc((void**)&h->dapatch, sizeof(double) * kAdjCell * std::max<long long>(acells, 1)) &&
              alloc((void**)&h->dgmk, sizeof(double) * 5 * nmk) &&
              alloc((void**)&h->dgwall, sizeof(double) * std::max<size_t>(gw, 1)) &&
              alloc((void**)&h->dgwoff, sizeof(long long) * nch) &&
              alloc((void**)&h->datlist, sizeof(int) * 2 * nt * kTileList) && alloc((void**)&h->dgout, sizeof(double) * 8 * nch);
    if (!ok) {
        free_adjoint(h);
        FAIL(h, LBM_ENOMEM, "allocation of the adjoint state failed");
    }
    h->lam[1] = (char*)h->lam[0] + h->lam_bytes;
    h->adj_seg = max_segment;
    h->gwall_n = gw;
    HIPCHK(h, hipMemsetAsync(h->lam[0], 0, 2 * h->lam_bytes, h->stream));
    HIPCHK(h, hipMemsetAsync(h->dgmk, 0, sizeof(double) * 5 * nmk, h->stream));
    HIPCHK(h, hipMemsetAsync(h->dgwall, 0, sizeof(double) * std::max<size_t>(gw, 1), h->stream));
    HIPCHK(h, hipMemsetAsync(h->datlist, 0, sizeof(int) * 2 * nt * kTileList, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->dap, ap.data(), sizeof(AdjPart) * ap.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(h->dgwoff, gwoff.data(), sizeof(long long) * nch, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->lcur = 0;
    h->apar = 0;
    h->adj_pos = h->steps;
    h->adj_first = true;
    return LBM_OK;
}

// One tape: the recomputed states of a segment of up to adj_seg steps.
struct TapeRef {
    const std::vector<void*>* f;  // [n] post-collision populations
    PartDev* p;                   // [n + 1][nparts] particle snapshots
    double2* patch;               // [n][cells] summed force patches
};

// Recomputes the n steps that start at checkpoint ck into tape T, on stream
// s, with no host wait: the particle state and step counter start from the
// checkpoint, and the first step reads the checkpoint's populations in
// place.  Writes the handle's particle state, step counter, tile lists,
// partial patches and surface-stress scratch, none of which the reverse
// kernels read.
static int tape_segment(lbm_handle* h, const Checkpoint& ck, int n, const TapeRef& T, hipStream_t s) {
    const int np = h->nparts;
    const size_t cells = (size_t)std::max<long long>(h->cells, 1);
    if (np) HIPCHK(h, hipMemcpyAsync(h->dparts, ck.p, sizeof(PartDev) * np, hipMemcpyDeviceToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->dstep, ck.step, sizeof(long long), hipMemcpyDeviceToDevice, s));
    int r;
    for (int t = 0; t < n; ++t) {
        StepArgs a = make_args(h, ck.cur, (ck.cur + t) & 1);
        a.fin = t == 0 ? ck.f : (*T.f)[t - 1];
        a.fout = (*T.f)[t];
        a.patch = T.patch + (size_t)t * cells;
        a.snap = T.p + (size_t)t * np;  // particle snapshot after the force stage
        // the tape keeps the summed patches, which the adjoint kernels read
        a.sum_partials = 0;
        HIPCHK(h, launch_ibm_force(h->store, a, s));
        HIPCHK(h, launch_patch_sum(a, s));
        if ((r = enqueue_rest(h, a, s)) != LBM_OK) return r;
    }
    if (np) HIPCHK(h, hipMemcpyAsync(T.p + (size_t)n * np, h->dparts, sizeof(PartDev) * np, hipMemcpyDeviceToDevice, s));
    return LBM_OK;
}

// Reverses the n taped steps of the segment that starts at checkpoint ck,
// on stream s.
static int reverse_segment(lbm_handle* h, const Checkpoint& ck, int n, const TapeRef& T, hipStream_t s) {
    const int np = h->nparts;
    const size_t cells = (size_t)std::max<long long>(h->cells, 1);
    for (int t = n - 1; t >= 0; --t) {
        AdjArgs a = adj_args(h);
        a.s.fin = t == 0 ? ck.f : (*T.f)[t - 1];
        a.s.parts = T.p + (size_t)t * np;
        a.s.patch = T.patch + (size_t)t * cells;
        a.pnext = T.p + (size_t)(t + 1) * np;
        a.first = h->adj_first ? 1 : 0;
        // channels of at most one particle: the particle kernels as one
        // launch, and with a lattice whose chunks fit the CUs in one pass
        // (a latency-bound step) the adjoint lattice pass in it too
        const int wgs = h->tune.adj_fused == 2 && h->alone ? adj_step_workgroups(a) : -1;
        if (wgs >= 0 && wgs <= h->cus) {
            HIPCHK(h, launch_adj_step(h->store, a, s));
        } else {
            if (h->tune.adj_fused && h->alone) {
                HIPCHK(h, launch_adj_particle(h->store, a, s));
            } else {
                HIPCHK(h, launch_adj_traction(h->store, a, s));
                HIPCHK(h, launch_adj_ibm(h->store, a, s));
            }
            HIPCHK(h, launch_adj_lattice(h->store, a, s));
        }
        h->lcur = 1 - h->lcur;
        h->apar = 1 - h->apar;
        h->adj_first = false;
    }
    return LBM_OK;
}

static int check_segment(lbm_handle* h, int32_t slot, int32_t n, long long end) {
    if (slot < 0 || slot >= kCheckpoints) FAIL(h, LBM_EINVAL, "slot must be in 0..%d", kCheckpoints - 1);
    if (n < 1 || n > h->adj_seg) FAIL(h, LBM_EINVAL, "segment length must be in 1..%d", h->adj_seg);
    const Checkpoint& ck = h->ck[slot];
    if (!ck.f || ck.nparts != h->nparts) FAIL(h, LBM_ESTATE, "slot %d holds no compatible checkpoint", slot);
    if (ck.steps + n != end)
        FAIL(h, LBM_ESTATE, "checkpoint at step %lld plus %d steps does not reach step %lld", ck.steps, n, end);
    return LBM_OK;
}

extern "C" int lbm_adjoint_segment(lbm_handle* h, int32_t slot, int32_t n) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    if (h->adj_pos < 0) FAIL(h, LBM_ESTATE, "no adjoint in progress (call lbm_adjoint_begin)");
    int r;
    if ((r = check_segment(h, slot, n, h->adj_pos)) != LBM_OK) return r;
    const Checkpoint& ck = h->ck[slot];
    if (h->tiles_dirty && (r = build_tiles(h)) != LBM_OK) return r;
    if ((r = lbm_checkpoint_restore(h, slot)) != LBM_OK) return r;
    const TapeRef T{&h->tape_f, h->tape_p, h->tape_patch};
    if ((r = tape_segment(h, ck, n, T, h->stream)) != LBM_OK) return r;
    if ((r = check_flags(h)) != LBM_OK) return r;
    if ((r = reverse_segment(h, ck, n, T, h->stream)) != LBM_OK) return r;
    const int rf = check_flags(h);
    // leave the forward state at the segment's checkpoint
    if ((r = lbm_checkpoint_restore(h, slot)) != LBM_OK) return r;
    if (rf != LBM_OK) {
        h->adj_pos = -1;  // the adjoint is incomplete: a new lbm_adjoint_begin is needed
        return rf;
    }
    h->adj_pos -= n;
    return LBM_OK;
}

extern "C" int lbm_adjoint_sweep(lbm_handle* h, const int32_t* slots, int32_t nseg, int32_t n) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    if (h->adj_pos < 0) FAIL(h, LBM_ESTATE, "no adjoint in progress (call lbm_adjoint_begin)");
    if (!slots || nseg < 1) FAIL(h, LBM_EINVAL, "need at least one segment");
    int r;
    long long end = h->adj_pos;
    for (int j = 0; j < nseg; ++j) {
        if ((r = check_segment(h, slots[j], n, end)) != LBM_OK) return r;
        end -= n;
    }
    if (nseg == 1) return lbm_adjoint_segment(h, slots[0], n);
    const int np = h->nparts;
    const size_t cells = (size_t)std::max<long long>(h->cells, 1);
    if (h->tape2_f.size() != (size_t)h->adj_seg) {
        // the second tape, as large as the first; where it does not fit the
        // segments are reversed one after the other
        free_tape2(h);
        bool ok = true;
        h->tape2_f.assign(h->adj_seg, nullptr);
        for (int t = 0; t < h->adj_seg && ok; ++t) ok = hipMalloc(&h->tape2_f[t], h->buf_bytes) == hipSuccess;
        ok = ok && hipMalloc((void**)&h->tape2_p, sizeof(PartDev) * (size_t)(h->adj_seg + 1) * std::max(np, 1)) == hipSuccess;
        ok = ok && hipMalloc((void**)&h->tape2_patch, sizeof(double2) * (size_t)h->adj_seg * cells) == hipSuccess;
        if (!ok) {
            free_tape2(h);
            (void)hipGetLastError();
            for (int j = 0; j < nseg; ++j)
                if ((r = lbm_adjoint_segment(h, slots[j], n)) != LBM_OK) return r;
            return LBM_OK;
        }
    }
    if (!h->stream2) HIPCHK(h, hipStreamCreateWithFlags(&h->stream2, hipStreamNonBlocking));
    for (auto& e : h->tape_ev)
        if (!e) HIPCHK(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (h->tiles_dirty && (r = build_tiles(h)) != LBM_OK) return r;
    // clears the flags and waits: the second stream starts after it
    if ((r = lbm_checkpoint_restore(h, slots[0])) != LBM_OK) return r;
    const TapeRef T[2] = {{&h->tape_f, h->tape_p, h->tape_patch}, {&h->tape2_f, h->tape2_p, h->tape2_patch}};
    // Segment j is taped into T[j % 2] on the second stream and reversed
    // from it on the handle's stream; taping segment j + 1 waits only for
    // the reversal of segment j - 1 (which read the same tape), so it runs
    // beside the reversal of segment j.
    if ((r = tape_segment(h, h->ck[slots[0]], n, T[0], h->stream2)) != LBM_OK) return r;
    HIPCHK(h, hipEventRecord(h->tape_ev[0], h->stream2));
    for (int j = 0; j < nseg; ++j) {
        const int x = j & 1;
        if (j + 1 < nseg) {
            if (j >= 1) HIPCHK(h, hipStreamWaitEvent(h->stream2, h->tape_ev[2 + (1 - x)], 0));
            if ((r = tape_segment(h, h->ck[slots[j + 1]], n, T[1 - x], h->stream2)) != LBM_OK) return r;
            HIPCHK(h, hipEventRecord(h->tape_ev[1 - x], h->stream2));
        }
        HIPCHK(h, hipStreamWaitEvent(h->stream, h->tape_ev[x], 0));
        if ((r = reverse_segment(h, h->ck[slots[j]], n, T[x], h->stream)) != LBM_OK) return r;
        HIPCHK(h, hipEventRecord(h->tape_ev[2 + x], h->stream));
    }
    // every taping was waited for by a reversal on the handle's stream, so
    // its synchronisation covers both streams; errors of any segment are
    // reported here
    const int rf = check_flags(h);
    if ((r = lbm_checkpoint_restore(h, slots[nseg - 1])) != LBM_OK) return r;
    if (rf != LBM_OK) {
        h->adj_pos = -1;
        return rf;
    }
    h->adj_pos -= (long long)nseg * n;
    return LBM_OK;
}

extern "C" int lbm_adjoint_gradients(lbm_handle* h, double* part_out, double* marker_out, double* wall_out) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    if (h->adj_pos < 0) FAIL(h, LBM_ESTATE, "no adjoint in progress (call lbm_adjoint_begin)");
    const int np = h->nparts, nch = (int)h->cfg.size();
    AdjArgs a = adj_args(h);
    a.lam_in = h->lam[h->lcur];
    for (int c = 0; c < nch; ++c) {
        const int with_init = h->adj_pos == 0 && !h->pop_modified && h->cfg[c].init == LBM_INIT_COUETTE;
        HIPCHK(h, launch_adj_finish(h->store, a, c, with_init, h->dgout + 8 * c, h->stream));
    }
    std::vector<AdjPart> ap(std::max(np, 1));
    size_t nmk = 0;
    for (auto& p : h->parts) nmk += p.d.n_markers;
    std::vector<double> gmk(5 * std::max<size_t>(nmk, 1)), gout(8 * nch);
    if (np) HIPCHK(h, hipMemcpyAsync(ap.data(), h->dap, sizeof(AdjPart) * np, hipMemcpyDeviceToHost, h->stream));
    if (nmk) HIPCHK(h, hipMemcpyAsync(gmk.data(), h->dgmk, sizeof(double) * 5 * nmk, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(gout.data(), h->dgout, sizeof(double) * 8 * nch, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (part_out)
        for (int u = 0; u < np; ++u) {
            const AdjPart& A = ap[h->dev_of_user[u]];
            const double ratio = h->parts[u].d.density_ratio;
            double* o = part_out + (size_t)u * LBM_AGRAD;
            for (int j = 0; j < AL_N; ++j) o[j] = A.l[j];
            o[AL_N] = A.gm;
            o[AL_N + 1] = A.gI;
            // a start with the history equal to the state: each initial value
            // feeds both its current and its previous slot
            double* g = o + AL_N + 2;
            g[0] = A.l[AL_X] + A.l[AL_XM];
            g[1] = A.l[AL_X + 1] + A.l[AL_XM + 1];
            g[2] = A.l[AL_TH] + A.l[AL_THM];
            g[3] = A.l[AL_V] + A.l[AL_VM];
            g[4] = A.l[AL_V + 1] + A.l[AL_VM + 1];
            g[5] = A.l[AL_OM] + A.l[AL_OMM];
            g[6] = A.gm * ratio;  // m = ratio * area
            g[7] = A.gI * ratio;  // I = ratio * polar moment
        }
    if (marker_out) {
        // device marker order follows the device particle order
        std::vector<size_t> dbeg(np + 1, 0);
        for (int k = 0; k < np; ++k) dbeg[k + 1] = dbeg[k] + h->parts[h->user_of_dev[k]].d.n_markers;
        size_t o = 0;
        for (int u = 0; u < np; ++u) {
            const int k = h->dev_of_user[u];
            const size_t m = h->parts[u].d.n_markers;
            memcpy(marker_out + 5 * o, gmk.data() + 5 * dbeg[k], sizeof(double) * 5 * m);
            o += m;
        }
    }
    if (wall_out) memcpy(wall_out, gout.data(), sizeof(double) * 8 * nch);
    return LBM_OK;
}

extern "C" int lbm_adjoint_field(lbm_handle* h, int32_t ch, double* out) {
    if (!h) FAIL(h, LBM_EINVAL, "handle is NULL");
    if (h->adj_pos < 0) FAIL(h, LBM_ESTATE, "no adjoint in progress (call lbm_adjoint_begin)");
    if (ch < 0 || ch >= (int)h->cfg.size() || !out) FAIL(h, LBM_EINVAL, "bad channel or NULL output");
    const size_t n = (size_t)h->cfg[ch].nx * h->cfg[ch].ny;
    double* d = nullptr;
    HIPCHK(h, hipMalloc(&d, sizeof(double) * 9 * n));
    AdjArgs a = adj_args(h);
    a.lam_in = h->lam[h->lcur];
    hipError_t e = launch_adj_field(h->store, a, ch, d, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d, sizeof(double) * 9 * n, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(d);
    HIPCHK(h, e);
    return LBM_OK;
}

extern "C" int lbm_measure_copy(void* dst, const void* src, size_t bytes, int32_t reps, void* stream,
                                double* gbps) {
    if (!dst || !src || !gbps || reps < 1 || bytes == 0 || bytes % 16 != 0)
        FAIL((lbm_handle*)nullptr, LBM_EINVAL, "lbm_measure_copy: NULL pointer, reps < 1 or bytes not a positive multiple of 16");
    hipStream_t s = (hipStream_t)stream;
    const long long n16 = (long long)(bytes / 16);
    hipEvent_t e0, e1;
    HIPCHK((lbm_handle*)nullptr, hipEventCreate(&e0));
    HIPCHK((lbm_handle*)nullptr, hipEventCreate(&e1));
    HIPCHK((lbm_handle*)nullptr, launch_copy(dst, src, n16, s));  // warm
    HIPCHK((lbm_handle*)nullptr, hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) HIPCHK((lbm_handle*)nullptr, launch_copy(dst, src, n16, s));
    HIPCHK((lbm_handle*)nullptr, hipEventRecord(e1, s));
    HIPCHK((lbm_handle*)nullptr, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK((lbm_handle*)nullptr, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *gbps = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    return LBM_OK;
}

extern "C" int64_t lbm_adjoint_position(const lbm_handle* h) { return h ? h->adj_pos : -1; }

extern "C" int64_t lbm_steps_done(const lbm_handle* h) { return h ? h->steps : -1; }

extern "C" const char* lbm_last_error(const lbm_handle* h) { return h ? h->err.c_str() : g_err.c_str(); }

extern "C" int lbm_destroy(lbm_handle* h) {
    if (!h) return LBM_OK;
    drop_graphs(h);
    if (h->stream2) (void)hipStreamSynchronize(h->stream2);
    free_adjoint(h);
    for (auto& e : h->tape_ev)
        if (e) (void)hipEventDestroy(e);
    if (h->stream2) (void)hipStreamDestroy(h->stream2);
    void* ptrs[] = {h->ws_alloc, h->dchan, h->dtiles, h->dparts, h->dxi, h->dnrm, h->dds, h->dpatch,
                    h->dmscr, h->dflags, h->dtlist, h->dstep, h->drec,
                    h->dwork, h->dpsum, h->dpcount, h->dpartial};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto& c : h->ck) {
        if (c.f) (void)hipFree(c.f);
        if (c.p) (void)hipFree(c.p);
        if (c.step) (void)hipFree(c.step);
    }
    delete h;
    return LBM_OK;
}
