// Host runtime and C ABI of the XY-model hot path (see include/xy.h).
//
// A context owns the device state of a batch of lattices: the colour-split
// angle buffer, the slot<->beta-position permutation, the device counters,
// measurement partials and acceptance counters.  Every sweep, measurement
// and exchange is a short sequence of kernel launches on the context's
// stream; xy_run captures that sequence once as a HIP graph and replays it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "xy.h"
#include "xy_kernels.h"

using namespace xy;

// Device scratch of the allocation-free sampled read-back
// (xy_get_sites_noalloc): the site list of one call, then the gathered
// angles.  One copy per GPU, held until the process ends.  In host code the
// array's name is only a stand-in: its device address is looked up once per
// device (scratch_address) and only that address reaches kernels and copies.
static __device__ __align__(256) unsigned char
    scratch[(size_t)XY_NOALLOC_MAX_SITES * (sizeof(int64_t) + sizeof(double))];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// This device's copy of `scratch`: hipGetSymbolAddress with the device
// current, once per device, the result kept for later contexts.
hipError_t scratch_address(int dev, void **out)
{
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

thread_local std::string g_init_error;

constexpr size_t kMaxLds = 64 * 1024;  // dynamic LDS a launch may ask for without attributes

struct Tiling {
    int TY = 0, TZ = 0, spt = 0;
};

struct GraphKey {
    int n_metro = -1, n_or = -1, exch = -1, batch = 0;
    double *obs = nullptr, *bonds = nullptr;
    bool operator==(const GraphKey &o) const
    {
        return n_metro == o.n_metro && n_or == o.n_or && exch == o.exch && batch == o.batch &&
               obs == o.obs && bonds == o.bonds;
    }
};

// Sweeps captured in one graph when every sweep of a loop is the same
// (exchange after every sweep or never): fewer graph launches, and the gap
// between consecutive graphs is paid once per batch.
constexpr int kSweepsPerGraph = 8;
// Captured graphs kept per context.  Each observable ring is baked into its
// graphs, so a caller that passes a new ring to every call would otherwise
// add graphs without bound; beyond this count the oldest graph of another
// loop shape or ring is released.
constexpr size_t kMaxGraphs = 32;

struct GraphEntry {
    GraphKey key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace

struct xy_ctx_s {
    // configuration
    int n_lat = 0;
    std::vector<int> L, R;
    std::vector<double> beta;
    uint64_t seed = 0;
    int prec = XY_FP32;
    uint32_t flags = 0;
    uint32_t k0 = 0, k1 = 0;
    int R_total = 0, max_R = 0;
    size_t elem = 4;       // bytes per angle
    int64_t n_elems = 0;   // total angles
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;

    // layout
    std::vector<LatDev> lat_sweep;   // tiled (FP32) or plain (FP64) item spaces
    std::vector<LatDev> lat_meas;    // standalone measurement item space
    int items_sweep = 0, items_meas = 0;
    int spt = 0;
    int halo = 1;          // halo entries per thread of the tiled kernel (1 or 4)
    size_t lds_bytes = 0;
    int grid_sweep = 0;    // workgroup cap of the tiled launches; 0: resident capacity
    int n_cu = 0;          // compute units of the context's device
    std::map<uint64_t, int> per_cu;  // resident workgroups per CU, by kernel and LDS size
    size_t partials_cap = 0;

    // device memory
    void *ang = nullptr;
    bool own_ang = false;
    LatDev *d_lat_sweep = nullptr, *d_lat_meas = nullptr;
    double *d_beta = nullptr;
    int32_t *d_pos = nullptr, *d_slot_of = nullptr;
    Ctl *d_ctl = nullptr;
    double *d_partials = nullptr;
    double *d_E = nullptr;
    double *d_obs = nullptr;
    double *d_bonds = nullptr;     // [R_total][6] bond sums of the last eager measurement
    unsigned long long *d_macc = nullptr, *d_sacc = nullptr;
    int *d_bad = nullptr;          // latched by the finalisation on a non-finite observable
    int *h_bad = nullptr;          // pinned host copy taken at the end of every xy_run
    hipEvent_t bad_ev = nullptr;   // completes when that copy has landed
    bool bad_pending = false;      // a copy was enqueued and not yet looked at
    RecheckQueue *d_rq = nullptr;
    RecheckEntry *d_rq_entries = nullptr;
    uint32_t rq_capacity = 0;

    // host mirrors
    uint64_t t = 0, tau = 0;
    bool e_fresh = false;          // d_E matches the current configurations
    bool bonds_fresh = false;      // d_bonds matches the current configurations

    std::vector<GraphEntry> graphs;
    std::vector<Tiling> tiles;  // FP32: per-lattice tile choice of the half-sweep kernels
    std::vector<Tiling> tiles2; // FP32: per-lattice tile choice of the fused over-relaxation
    bool fused_avail = false;   // the fused kernel's layout and second buffer exist (FP32, every L <= kBlock)
    bool fused_or = false;      // over-relaxation substeps run as one fused kernel each (the schedule in use)
    double window = 0.0;        // Metropolis proposal window (radians, 0: uniform)
    std::vector<LatDev> lat_or2;
    int items_or2 = 0, spt2 = 0;
    size_t lds2 = 0;
    LatDev *d_lat_or2 = nullptr;
    void *ang2 = nullptr;       // second configuration buffer for the fused kernel
    int dev = 0;                // device the context was created on
    void *scratch = nullptr;    // that device's copy of the static scratch array
    std::string err;
};

namespace {

xy_status fail(xy_ctx c, xy_status s, const std::string &msg)
{
    if (c)
        c->err = msg;
    else
        g_init_error = msg;
    return s;
}

#define XY_HIP(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), XY_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool valid_L(int L) { return L >= 4 && L <= 1024 && (L % 2) == 0; }

std::vector<int> divisors(int L)
{
    std::vector<int> d;
    for (int i = 1; i <= L; ++i)
        if (L % i == 0) d.push_back(i);
    return d;
}

int spt_for(int sites)
{
    int s = (sites + kBlock - 1) / kBlock;
    if (s <= 6) return std::max(s, 1);
    return 8;
}

// Default tile of the FP32 kernel (xy_autotune refines it by timing): about
// 2.5 sites per thread in the y-tile (measured on gfx950 at L = 160 to balance
// occupancy against halo overhead), and z-chunks of at most 24 planes.
Tiling default_tiling(int L, int R)
{
    (void)R;
    const int half = L / 2;
    Tiling t;
    for (int d : divisors(L))
        if (d * half <= 3 * kBlock) t.TY = d;
    if (t.TY == 0) t.TY = 1;
    t.TZ = 1;
    for (int d : divisors(L))
        if (d <= 24) t.TZ = d;
    t.spt = spt_for(t.TY * half);
    return t;
}

// LDS of the fused over-relaxation kernel for a tile of ty rows of L/2
// sites: two old-colour-1 plane buffers of the kernel's fixed size
// (spt + 2) * kBlock and three new-colour-0 plane buffers of (ty + 2) * L/2
// (cos, sin) pairs (the measuring variants rotate through three, the plain
// substep uses two; one size serves both).  Tiles are limited to five
// columns per thread, so that any batch of admissible tiles fits 64 KiB
// ((5 * 5 + 7) * kBlock pairs).
size_t or2_lds_bytes(int ty, int half)
{
    const int spt = spt_for(ty * half);
    return ((size_t)2 * (spt + 2) * kBlock + (size_t)3 * (ty + 2) * half) * 2 * sizeof(float);
}

bool or2_tile_ok(int ty, int half)
{
    return ty * half <= 5 * kBlock && or2_lds_bytes(ty, half) <= kMaxLds;
}

// Default tile of the fused over-relaxation kernel: up to three tile columns
// per thread and z-chunks of at most 40 planes (measured best at L = 160).
Tiling default_tiling2(int L)
{
    const int half = L / 2;
    Tiling t;
    for (int d : divisors(L))
        if (d * half <= 3 * kBlock && or2_tile_ok(d, half)) t.TY = d;
    if (t.TY == 0) t.TY = 1;
    t.TZ = 1;
    for (int d : divisors(L))
        if (d <= 40) t.TZ = d;
    t.spt = spt_for(t.TY * half);
    return t;
}

xy_status sync_stream(xy_ctx c)
{
    XY_HIP(c, hipStreamSynchronize(c->stream));
    return XY_OK;
}

// Workgroups of one tiled launch over `items` work items: the explicit cap
// when one is set, else as many as the GPU holds at once (compute units x the
// kernel's resident workgroups per CU), each taking items in turn.  Measured
// at L = 160 x 32, launches sized to the resident capacity beat one
// workgroup per item by 3-5 % (no half-empty last round of workgroups).
int launch_grid(xy_ctx c, int items, bool fused, int kind, bool meas, bool full, int spt, size_t lds,
                const SweepArgs &a)
{
    if (c->grid_sweep > 0) return std::min(items, c->grid_sweep);
    const uint64_t key = ((uint64_t)lds << 32) | ((uint64_t)fused << 24) | ((uint64_t)c->halo << 16) |
                         ((uint64_t)spt << 8) | ((uint64_t)full << 6) | ((uint64_t)(a.bonds != 0) << 5) |
                         ((uint64_t)meas << 4) | (uint64_t)kind;
    auto it = c->per_cu.find(key);
    if (it == c->per_cu.end()) {
        int n = 0;
        const hipError_t e = fused ? launch_or2_f32(meas, full, spt, 0, lds, a, c->stream, &n)
                                   : launch_tile_f32(kind, meas, full, spt, c->halo, 0, lds, a, c->stream, &n);
        it = c->per_cu.emplace(key, e == hipSuccess ? n : 0).first;
    }
    const int resident = c->n_cu * it->second;
    return resident > 0 ? std::min(items, resident) : items;
}

xy_status launch_half(xy_ctx c, int kind, int colour, int substep, bool fuse_measure, bool bonds = true)
{
    SweepArgs a{};
    a.n_lat = c->n_lat;
    a.ang = c->ang;
    a.beta = c->d_beta;
    a.pos = c->d_pos;
    a.ctl = c->d_ctl;
    a.k0 = c->k0;
    a.k1 = c->k1;
    a.colour = colour;
    a.substep = substep;
    a.recheck = (c->flags & XY_F_NO_RECHECK) ? 0 : 1;
    a.bonds = bonds ? 1 : 0;
    a.window = c->window;
    a.window_t = (float)(c->window / 6.283185307179586476925286766559);
    a.partials = c->d_partials;
    a.macc = c->d_macc;
    a.rq = c->d_rq;
    hipError_t e;
    if (c->prec == XY_FP32) {
        const bool meas_item_space = (kind == kMeas);
        a.lats = meas_item_space ? c->d_lat_meas : c->d_lat_sweep;
        a.total_items = meas_item_space ? c->items_meas : c->items_sweep;
        // every lattice's tile exactly fills the columns of the launch
        bool full = !meas_item_space;
        for (const LatDev &d : c->lat_sweep) full = full && d.TY * d.half == c->spt * kBlock;
        const int grid = launch_grid(c, a.total_items, false, kind, fuse_measure, full, c->spt, c->lds_bytes, a);
        e = launch_tile_f32(kind, fuse_measure, full, c->spt, c->halo, grid, c->lds_bytes, a, c->stream);
        if (e == hipSuccess && kind == kMetro && a.recheck) e = launch_recheck(a, c->stream);
    } else {
        a.lats = c->d_lat_sweep;
        a.total_items = c->items_sweep;
        e = launch_plain_f64(kind, fuse_measure, a.total_items, a, c->stream);
    }
    if (e != hipSuccess) return fail(c, XY_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return XY_OK;
}

// One fused over-relaxation substep from buffer `from` into buffer `to`.
xy_status launch_or2(xy_ctx c, void *from, void *to, bool fuse_measure, bool bonds = true)
{
    SweepArgs a{};
    a.lats = c->d_lat_or2;
    a.n_lat = c->n_lat;
    a.total_items = c->items_or2;
    a.ang = from;
    a.ang_dst = to;
    a.beta = c->d_beta;
    a.pos = c->d_pos;
    a.ctl = c->d_ctl;
    a.k0 = c->k0;
    a.k1 = c->k1;
    a.partials = c->d_partials;
    a.bonds = bonds ? 1 : 0;
    a.macc = c->d_macc;
    a.rq = c->d_rq;
    // the first spt2 - 1 tile columns of every lattice are populated
    bool lead = true;
    for (const LatDev &d : c->lat_or2) lead = lead && d.TY * d.half > (c->spt2 - 1) * kBlock;
    const int grid = launch_grid(c, a.total_items, true, 0, fuse_measure, lead, c->spt2, c->lds2, a);
    hipError_t e = launch_or2_f32(fuse_measure, lead, c->spt2, grid, c->lds2, a, c->stream);
    if (e != hipSuccess) return fail(c, XY_ERR_HIP, std::string("fused launch: ") + hipGetErrorString(e));
    return XY_OK;
}

// Over-relaxation substeps that run fused: all of them when n_or is even,
// all but the last otherwise, so the configuration ends every sweep back in
// the primary buffer (an even number of buffer swaps).
int fused_substeps(xy_ctx c, int n_or)
{
    return c->fused_or ? n_or - (n_or & 1) : 0;
}

enum PartialsLayout { kPartMeas = 0, kPartSweep = 1, kPartOr2 = 2 };

// A sweep that ends on a float32 Metropolis half-sweep with float64
// re-decision is measured by a separate pass after it: the re-decision may
// still change sites that the half-sweep has already measured.
bool measures_after_sweep(xy_ctx c, int n_or)
{
    return n_or == 0 && c->prec == XY_FP32 && !(c->flags & XY_F_NO_RECHECK);
}

// Which item layout the measurement partials of a sweep come from.
int sweep_partials_layout(xy_ctx c, int n_or)
{
    const int n_fused = fused_substeps(c, n_or);
    if (n_fused > 0 && n_fused == n_or) return kPartOr2;
    return measures_after_sweep(c, n_or) ? kPartMeas : kPartSweep;
}

// Enqueue one sweep; if measure_last, the sweep also produces the
// measurement partials of its final configuration (in the item layout
// sweep_partials_layout() names), with the bond sums of Eq. (6) when
// `bonds` is set.  Without `tick` the caller advances the sweep counter
// itself (after the sweep's last kernel).
xy_status enqueue_sweep(xy_ctx c, int n_metro, int n_or, bool measure_last, bool bonds = true,
                        bool tick = true)
{
    const int n_fused = fused_substeps(c, n_or);
    const int total = 2 * (n_metro + n_or - n_fused) + n_fused;
    const bool meas_after = measure_last && measures_after_sweep(c, n_or);
    const bool meas_fused = measure_last && !meas_after;
    int h = 0;
    for (int s = 0; s < n_metro; ++s)
        for (int col = 0; col < 2; ++col, ++h) {
            xy_status st = launch_half(c, kMetro, col, s, meas_fused && h == total - 1, bonds);
            if (st) return st;
        }
    for (int s = 0; s < n_fused; ++s, ++h) {
        void *from = (s & 1) ? c->ang2 : c->ang;
        void *to = (s & 1) ? c->ang : c->ang2;
        xy_status st = launch_or2(c, from, to, meas_fused && h == total - 1, bonds);
        if (st) return st;
    }
    for (int s = n_fused; s < n_or; ++s)
        for (int col = 0; col < 2; ++col, ++h) {
            xy_status st = launch_half(c, kOver, col, s, meas_fused && h == total - 1, bonds);
            if (st) return st;
        }
    if (meas_after) {
        xy_status st = launch_half(c, kMeas, 1, 0, false, bonds);
        if (st) return st;
    }
    if (tick) XY_HIP(c, launch_tick(c->d_ctl, 1u, 0u, 0u, 0, c->stream));
    return XY_OK;
}

xy_status enqueue_measure_kernel(xy_ctx c)
{
    return launch_half(c, kMeas, 1, 0, false);
}

const LatDev *meas_layout_dev(xy_ctx c, int layout)
{
    if (c->prec == XY_FP64) return c->d_lat_sweep;
    if (layout == kPartOr2) return c->d_lat_or2;
    return layout == kPartSweep ? c->d_lat_sweep : c->d_lat_meas;
}

xy_status enqueue_finalize(xy_ctx c, int layout, double *obs, int use_ring, bool do_sum,
                           bool do_exchange, double *bonds = nullptr)
{
    XY_HIP(c, launch_finalize(meas_layout_dev(c, layout), c->n_lat, c->max_R,
                              c->d_partials, c->d_beta, c->d_pos, c->d_slot_of, c->d_E, obs, bonds,
                              use_ring, (int64_t)5 * c->R_total, (int64_t)6 * c->R_total,
                              do_sum ? 1 : 0, do_exchange ? 1 : 0, c->d_sacc, c->d_ctl, c->k0, c->k1,
                              c->d_bad, c->stream));
    return XY_OK;
}

// The non-finite sentinel, once reported, is cleared (stream-ordered) so
// that it reports again only if a later measurement finds the state bad.
xy_status clear_bad(xy_ctx c)
{
    *c->h_bad = 0;
    XY_HIP(c, hipMemcpyAsync(c->d_bad, c->h_bad, sizeof(int), hipMemcpyHostToDevice, c->stream));
    XY_HIP(c, hipStreamSynchronize(c->stream));
    return XY_OK;
}

xy_status check_bad(xy_ctx c)
{
    c->bad_pending = false;
    XY_HIP(c, hipMemcpyAsync(c->h_bad, c->d_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    XY_HIP(c, hipStreamSynchronize(c->stream));
    if (*c->h_bad) {
        xy_status st = clear_bad(c);
        if (st) return st;
        return fail(c, XY_ERR_STATE, "non-finite energy or magnetisation in the device state");
    }
    return XY_OK;
}

// Without waiting: if the sentinel copy taken at the end of an earlier
// xy_run has landed, report (and clear) what it found.
xy_status poll_bad(xy_ctx c)
{
    if (!c->bad_pending || hipEventQuery(c->bad_ev) != hipSuccess) return XY_OK;
    c->bad_pending = false;
    if (!*c->h_bad) return XY_OK;
    xy_status st = clear_bad(c);
    if (st) return st;
    return fail(c, XY_ERR_STATE, "non-finite energy or magnetisation found by an earlier xy_run");
}

void free_graphs(xy_ctx c)
{
    // a replay may still be in flight on the stream
    if (!c->graphs.empty()) (void)hipStreamSynchronize(c->stream);
    for (auto &g : c->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    c->graphs.clear();
}

void free_all(xy_ctx c)
{
    if (!c) return;
    // wait for this context's own work only (other streams and contexts on
    // the device keep running)
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != c->dev) (void)hipSetDevice(c->dev);
    (void)hipStreamSynchronize(c->stream);
    if (c->cap_stream) (void)hipStreamSynchronize(c->cap_stream);
    free_graphs(c);
    if (c->bad_ev) (void)hipEventDestroy(c->bad_ev);
    if (c->h_bad) (void)hipHostFree(c->h_bad);
    if (c->own_ang && c->ang) (void)hipFree(c->ang);
    void *ptrs[] = {c->d_lat_or2, c->ang2, c->d_lat_sweep, c->d_lat_meas, c->d_beta, c->d_pos, c->d_slot_of, c->d_ctl,
                    c->d_partials, c->d_E, c->d_obs, c->d_bonds, c->d_macc, c->d_sacc, c->d_bad,
                    c->d_rq, c->d_rq_entries};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (cur >= 0 && cur != c->dev) (void)hipSetDevice(cur);
}

xy_status validate(const xy_config *cfg)
{
    if (!cfg) return fail(nullptr, XY_ERR_ARG, "config is NULL");
    if (cfg->n_lattices < 1 || cfg->n_lattices > 64)
        return fail(nullptr, XY_ERR_ARG, "n_lattices must be in [1, 64]");
    if (!cfg->L || !cfg->n_replicas || !cfg->beta)
        return fail(nullptr, XY_ERR_ARG, "L, n_replicas and beta must be non-NULL");
    if (cfg->prec != XY_FP32 && cfg->prec != XY_FP64)
        return fail(nullptr, XY_ERR_ARG, "prec must be XY_FP32 or XY_FP64");
    if (cfg->start != XY_START_RANDOM && cfg->start != XY_START_ORDERED)
        return fail(nullptr, XY_ERR_ARG, "start must be XY_START_RANDOM or XY_START_ORDERED");
    int64_t off = 0;
    for (int l = 0; l < cfg->n_lattices; ++l) {
        const int L = cfg->L[l], R = cfg->n_replicas[l];
        if (!valid_L(L))
            return fail(nullptr, XY_ERR_ODD_L,
                        "lattice " + std::to_string(l) + ": L = " + std::to_string(L) +
                            " must be even with 4 <= L <= 1024");
        if (R < 1 || R > 65535)
            return fail(nullptr, XY_ERR_ARG, "lattice " + std::to_string(l) + ": n_replicas must be in [1, 65535]");
        for (int k = 0; k < R; ++k) {
            const double b = cfg->beta[off + k];
            if (!std::isfinite(b) || b < 0.0)
                return fail(nullptr, XY_ERR_ARG, "beta must be finite and >= 0");
            if (k > 0 && !(b > cfg->beta[off + k - 1]))
                return fail(nullptr, XY_ERR_ARG,
                            "lattice " + std::to_string(l) + ": beta ladder must be strictly ascending");
        }
        off += R;
    }
    return XY_OK;
}

int64_t total_elems(const xy_config *cfg)
{
    int64_t n = 0;
    for (int l = 0; l < cfg->n_lattices; ++l)
        n += (int64_t)cfg->n_replicas[l] * (int64_t)cfg->L[l] * cfg->L[l] * cfg->L[l];
    return n;
}

template <typename T>
xy_status dev_alloc(xy_ctx c, T **p, size_t count)
{
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, e == hipErrorOutOfMemory ? XY_ERR_OOM : XY_ERR_HIP,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return XY_OK;
}

// Build the item spaces.  FP32: tiled sweep (TY x L/2 x TZ per item) and a
// measurement space with the same tiles; FP64: one item per kBlock sites of
// a colour of a slot, for every kernel.
void build_layout(xy_ctx c)
{
    int64_t base = 0;
    int pos_base = 0, item_s = 0, item_m = 0;
    c->spt = 1;
    c->halo = 1;
    c->lat_sweep.clear();
    c->lat_meas.clear();
    for (int l = 0; l < c->n_lat; ++l) {
        LatDev d{};
        d.L = c->L[l];
        d.half = d.L / 2;
        d.R = c->R[l];
        d.lat = l;
        d.base = base;
        d.N = (int64_t)d.L * d.L * d.L;
        d.pos_base = pos_base;
        if (c->prec == XY_FP32) {
            if ((int)c->tiles.size() <= l) c->tiles.push_back(default_tiling(d.L, d.R));
            const Tiling t = c->tiles[l];
            d.TY = t.TY;
            d.TZ = t.TZ;
            d.ny = d.L / t.TY;
            d.nz = d.L / t.TZ;
            d.items_per_slot = d.ny * d.nz;
            c->spt = std::max(c->spt, t.spt);
            if (d.L > kBlock) c->halo = 4;
        } else {
            d.TY = d.TZ = d.ny = d.nz = 0;
            d.items_per_slot = (int)((d.N / 2 + kBlock - 1) / kBlock);
        }
        d.item_base = item_s;
        item_s += d.R * d.items_per_slot;
        c->lat_sweep.push_back(d);
        LatDev m = d;
        m.item_base = item_m;
        item_m += m.R * m.items_per_slot;
        c->lat_meas.push_back(m);
        base += (int64_t)d.R * d.N;
        pos_base += d.R;
    }
    c->items_sweep = item_s;
    c->items_meas = item_m;
    // fused over-relaxation layout (FP32, every lattice with L <= kBlock)
    c->lat_or2.clear();
    c->items_or2 = 0;
    c->spt2 = 1;
    c->lds2 = 0;
    if (c->fused_avail) {
        int item2 = 0;
        size_t p0_elems = 0;
        for (int l = 0; l < c->n_lat; ++l) {
            if ((int)c->tiles2.size() <= l) c->tiles2.push_back(default_tiling2(c->L[l]));
            const Tiling t = c->tiles2[l];
            LatDev d = c->lat_sweep[l];
            d.TY = t.TY;
            d.TZ = t.TZ;
            d.ny = d.L / t.TY;
            d.nz = d.L / t.TZ;
            d.items_per_slot = d.ny * d.nz;
            d.item_base = item2;
            item2 += d.R * d.items_per_slot;
            c->lat_or2.push_back(d);
            c->spt2 = std::max(c->spt2, t.spt);
            p0_elems = std::max(p0_elems, (size_t)(t.TY + 2) * d.half);
        }
        // two old-colour-1 plane buffers at the kernel's fixed size (spt2 + 2) * kBlock,
        // a bound on (TY + 4) * L/2, then three new-colour-0 plane buffers (two used
        // by the plain substep)
        c->lds2 = ((size_t)2 * (c->spt2 + 2) * kBlock + 3 * p0_elems) * 2 * sizeof(float);
        c->items_or2 = item2;
    }
    // two plane buffers of (cos, sin), the second at the kernel's fixed offset
    // (spt + halo) * kBlock elements, which bounds (TY + 2) * L/2 for every lattice
    c->lds_bytes = (size_t)2 * (c->spt + c->halo) * kBlock * 2 * sizeof(float);
}

// Re-derive item spaces after a tiling change and upload them.  Partials
// are indexed by item, so grow that buffer if needed; graphs bake the old
// launch shapes in and are dropped.
xy_status relayout(xy_ctx c)
{
    build_layout(c);
    const int n_items_max = std::max(std::max(c->items_sweep, c->items_meas), c->items_or2);
    if ((size_t)kPartials * n_items_max > c->partials_cap) {
        XY_HIP(c, hipStreamSynchronize(c->stream));
        (void)hipFree(c->d_partials);
        c->d_partials = nullptr;
        xy_status st = dev_alloc(c, &c->d_partials, (size_t)kPartials * n_items_max);
        if (st) return st;
        c->partials_cap = (size_t)kPartials * n_items_max;
    }
    XY_HIP(c, hipMemcpyAsync(c->d_lat_sweep, c->lat_sweep.data(), sizeof(LatDev) * c->n_lat,
                             hipMemcpyHostToDevice, c->stream));
    XY_HIP(c, hipMemcpyAsync(c->d_lat_meas, c->lat_meas.data(), sizeof(LatDev) * c->n_lat,
                             hipMemcpyHostToDevice, c->stream));
    if (c->fused_avail)
        XY_HIP(c, hipMemcpyAsync(c->d_lat_or2, c->lat_or2.data(), sizeof(LatDev) * c->n_lat,
                                 hipMemcpyHostToDevice, c->stream));
    XY_HIP(c, hipStreamSynchronize(c->stream));
    free_graphs(c);
    c->e_fresh = c->bonds_fresh = false;
    return XY_OK;
}

// Device time of one call of `launch`, averaged over `reps` calls after one
// warm-up call, on the context's stream.
template <class F>
xy_status time_launches(xy_ctx c, hipEvent_t e0, hipEvent_t e1, int reps, F &&launch, double *ms)
{
    xy_status st = launch();
    if (st) return st;
    XY_HIP(c, hipEventRecord(e0, c->stream));
    for (int r = 0; r < reps; ++r)
        if ((st = launch())) return st;
    XY_HIP(c, hipEventRecord(e1, c->stream));
    XY_HIP(c, hipEventSynchronize(e1));
    float t = 0.f;
    XY_HIP(c, hipEventElapsedTime(&t, e0, e1));
    *ms = (double)t / reps;
    return XY_OK;
}

// Candidate tile shapes of one lattice: ty and tz divide L, at least half a
// block of sites per plane (unless the tile is the whole plane), at most 2048,
// and z-chunks of 2..64 planes (or the whole lattice).
std::vector<std::pair<int, int>> tile_candidates(int L)
{
    const int half = L / 2;
    std::vector<std::pair<int, int>> out;
    for (int ty : divisors(L)) {
        if (ty * half > 8 * kBlock) continue;
        if (ty * half < kBlock / 2 && ty != L) continue;  // mostly idle lanes
        for (int tz : divisors(L)) {
            if (tz < 2 && L > 2) continue;
            if (tz > 64 && tz != L) continue;
            out.push_back({ty, tz});
        }
    }
    return out;
}

}  // namespace

extern "C" {

size_t xy_angles_bytes(const xy_config *cfg)
{
    if (validate(cfg) != XY_OK) return 0;
    return (size_t)total_elems(cfg) * (cfg->prec == XY_FP32 ? 4 : 8);
}

// A caller buffer that kernels (or device-side copies) of this context use:
// device memory of the context's GPU, managed memory, or host memory pinned
// with hipHostMalloc, which the GPU reaches through its mapped address.
// Pageable host memory and memory of another GPU are rejected here rather
// than faulting inside a kernel, and so is a buffer whose allocation ends
// before `bytes` where HIP reports the allocation's range (a tensor carved
// from a larger pool can only be checked against the pool).  *dev receives
// the address kernels use: p itself (unified addressing gives pinned host
// memory the same address on the device).
static xy_status gpu_buffer(xy_ctx c, void *p, size_t bytes, const char *what, void **dev)
{
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess || a.devicePointer == nullptr) {
        (void)hipGetLastError();
        return fail(c, XY_ERR_ARG, std::string(what) + " is neither device memory nor pinned host memory");
    }
    if (a.type == hipMemoryTypeDevice && a.device != c->dev)
        return fail(c, XY_ERR_ARG, std::string(what) + " is memory of another GPU");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, p) == hipSuccess && base) {
        if ((char *)p + bytes > (char *)base + size)
            return fail(c, XY_ERR_ARG, std::string(what) + " is smaller than the " + std::to_string(bytes) +
                                           " bytes the call writes");
    } else {
        (void)hipGetLastError();
    }
    *dev = p;
    return XY_OK;
}

xy_status xy_init(const xy_config *cfg, xy_ctx *out)
{
    if (!out) return fail(nullptr, XY_ERR_ARG, "out is NULL");
    *out = nullptr;
    xy_status st = validate(cfg);
    if (st) return st;
    if (total_elems(cfg) > ((int64_t)1 << 36))
        return fail(nullptr, XY_ERR_ARG, "total number of angles exceeds 2^36");

    xy_ctx c = new (std::nothrow) xy_ctx_s();
    if (!c) return fail(nullptr, XY_ERR_OOM, "host allocation failed");
    c->n_lat = cfg->n_lattices;
    c->L.assign(cfg->L, cfg->L + c->n_lat);
    c->R.assign(cfg->n_replicas, cfg->n_replicas + c->n_lat);
    for (int l = 0; l < c->n_lat; ++l) {
        c->R_total += c->R[l];
        c->max_R = std::max(c->max_R, c->R[l]);
    }
    c->beta.assign(cfg->beta, cfg->beta + c->R_total);
    c->seed = cfg->seed;
    c->k0 = (uint32_t)(cfg->seed & 0xffffffffu);
    c->k1 = (uint32_t)(cfg->seed >> 32);
    c->prec = cfg->prec;
    c->flags = cfg->flags;
    c->elem = (c->prec == XY_FP32) ? 4 : 8;
    c->n_elems = total_elems(cfg);
    c->stream = (hipStream_t)cfg->stream;
    c->fused_avail = c->prec == XY_FP32 && !(cfg->flags & XY_F_NO_FUSED_OR);
    for (int l = 0; l < c->n_lat; ++l)
        if (c->L[l] > kBlock) c->fused_avail = false;
    c->fused_or = c->fused_avail;
    build_layout(c);

    auto bail = [&](xy_status s) {
        g_init_error = c->err;
        free_all(c);
        delete c;
        return s;
    };

    int dev_count = 0, dev = 0;
    if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1 || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        c->err = "no HIP device available";
        return bail(XY_ERR_HIP);
    }
    c->dev = dev;
    {
        const hipError_t e = scratch_address(dev, &c->scratch);
        if (e != hipSuccess) {
            c->err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return bail(XY_ERR_HIP);
        }
    }
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        c->err = "hipStreamCreateWithFlags failed";
        return bail(XY_ERR_HIP);
    }
    if (cfg->angles_dev) {
        if ((st = gpu_buffer(c, cfg->angles_dev, (size_t)c->n_elems * c->elem, "angles_dev", &c->ang)))
            return bail(st);
        c->own_ang = false;
    } else {
        if ((st = dev_alloc(c, (char **)&c->ang, (size_t)c->n_elems * c->elem))) return bail(st);
        c->own_ang = true;
    }
    const int n_items_max = std::max(std::max(c->items_sweep, c->items_meas), c->items_or2);
    if (c->fused_avail) {
        if ((st = dev_alloc(c, (char **)&c->ang2, (size_t)c->n_elems * c->elem)) ||
            (st = dev_alloc(c, &c->d_lat_or2, c->n_lat)))
            return bail(st);
    }
    if ((st = dev_alloc(c, &c->d_lat_sweep, c->n_lat)) || (st = dev_alloc(c, &c->d_lat_meas, c->n_lat)) ||
        (st = dev_alloc(c, &c->d_beta, c->R_total)) || (st = dev_alloc(c, &c->d_pos, c->R_total)) ||
        (st = dev_alloc(c, &c->d_slot_of, c->R_total)) || (st = dev_alloc(c, &c->d_ctl, 1)) ||
        (st = dev_alloc(c, &c->d_partials, (size_t)kPartials * n_items_max)) ||
        (st = dev_alloc(c, &c->d_E, c->R_total)) || (st = dev_alloc(c, &c->d_obs, (size_t)5 * c->R_total)) ||
        (st = dev_alloc(c, &c->d_bonds, (size_t)6 * c->R_total)) ||
        (st = dev_alloc(c, &c->d_macc, c->R_total)) || (st = dev_alloc(c, &c->d_sacc, c->R_total)) ||
        (st = dev_alloc(c, &c->d_bad, 1)))
        return bail(st);
    if (hipHostMalloc((void **)&c->h_bad, sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->bad_ev, hipEventDisableTiming) != hipSuccess) {
        c->err = "pinned host flag or event creation failed";
        return bail(XY_ERR_HIP);
    }
    *c->h_bad = 0;
    // Near-threshold queue: about 2e-5 of a half-sweep's sites land in the band;
    // capacity allows for 1e-3 of the largest lattice's half-sweep.
    {
        int64_t half_sweep_sites = 0;
        for (int l = 0; l < c->n_lat; ++l) half_sweep_sites += (int64_t)c->R[l] * c->lat_sweep[l].N / 2;
        c->rq_capacity = (uint32_t)std::min<int64_t>(std::max<int64_t>(4096, half_sweep_sites / 1000), 1 << 22);
        if ((st = dev_alloc(c, &c->d_rq, 1)) || (st = dev_alloc(c, &c->d_rq_entries, c->rq_capacity)))
            return bail(st);
    }

    c->partials_cap = (size_t)kPartials * n_items_max;
    std::vector<int32_t> ident(c->R_total);
    {
        int p = 0;
        for (int l = 0; l < c->n_lat; ++l)
            for (int r = 0; r < c->R[l]; ++r) ident[p++] = r;
    }
    std::vector<unsigned long long> zeros(c->R_total, 0ull);
    Ctl ctl{};
    int zero = 0;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpy(c->d_lat_sweep, c->lat_sweep.data(), sizeof(LatDev) * c->n_lat, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_lat_meas, c->lat_meas.data(), sizeof(LatDev) * c->n_lat, hipMemcpyHostToDevice);
    if (e == hipSuccess && c->fused_avail)
        e = hipMemcpy(c->d_lat_or2, c->lat_or2.data(), sizeof(LatDev) * c->n_lat, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_beta, c->beta.data(), sizeof(double) * c->R_total, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_pos, ident.data(), sizeof(int32_t) * c->R_total, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_slot_of, ident.data(), sizeof(int32_t) * c->R_total, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_ctl, &ctl, sizeof(Ctl), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_macc, zeros.data(), sizeof(unsigned long long) * c->R_total, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_sacc, zeros.data(), sizeof(unsigned long long) * c->R_total, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_bad, &zero, sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        RecheckQueue q{0u, 0u, c->rq_capacity, 0u, c->d_rq_entries};  // count, overflow, capacity, done
        e = hipMemcpy(c->d_rq, &q, sizeof(q), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        c->err = std::string("hipMemcpy: ") + hipGetErrorString(e);
        return bail(XY_ERR_HIP);
    }
    e = launch_init(c->prec == XY_FP32, cfg->start == XY_START_ORDERED, c->d_lat_sweep, c->n_lat,
                    c->n_elems, c->ang, c->k0, c->k1, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->err = std::string("init kernel: ") + hipGetErrorString(e);
        return bail(XY_ERR_HIP);
    }
    *out = c;
    return XY_OK;
}

xy_status xy_sweep(xy_ctx c, int32_t n_metro, int32_t n_or)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (n_metro < 0 || n_or < 0 || n_metro + n_or < 1 || n_metro > 255 || n_or > 65535)
        return fail(c, XY_ERR_ARG, "need 0 <= n_metro <= 255, 0 <= n_or, n_metro + n_or >= 1");
    if (c->t >= 0xffffffffull) return fail(c, XY_ERR_STATE, "sweep counter would overflow 32 bits");
    xy_status st = enqueue_sweep(c, n_metro, n_or, false);
    if (st) return st;
    c->t += 1;
    c->e_fresh = c->bonds_fresh = false;
    return XY_OK;
}

xy_status xy_sweep_profiled(xy_ctx c, int32_t n_metro, int32_t n_or, double *ms, int32_t *launches)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (!ms || !launches) return fail(c, XY_ERR_ARG, "ms and launches must be non-NULL");
    if (n_metro < 0 || n_or < 0 || n_metro + n_or < 1 || n_metro > 255 || n_or > 65535)
        return fail(c, XY_ERR_ARG, "need 0 <= n_metro <= 255, 0 <= n_or, n_metro + n_or >= 1");
    if (c->t >= 0xffffffffull) return fail(c, XY_ERR_STATE, "sweep counter would overflow 32 bits");
    const int n_fused = fused_substeps(c, n_or);
    // One event pair per group of consecutive launches of one kind (events
    // between every launch would add their own overhead to each kernel):
    // Metropolis half-sweeps with their re-decision kernels, fused
    // substeps, over-relaxation half-sweeps, and the counter update.
    hipEvent_t ev[8] = {};
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &x : ev)
                if (x) (void)hipEventDestroy(x);
            return fail(c, XY_ERR_HIP, "hipEventCreate failed");
        }
    const int counts[4] = {2 * n_metro, 2 * (n_or - n_fused), n_fused, 1};
    xy_status st = XY_OK;
    (void)hipEventRecord(ev[0], c->stream);
    for (int s = 0; s < n_metro && !st; ++s)
        for (int col = 0; col < 2 && !st; ++col) st = launch_half(c, kMetro, col, s, false);
    (void)hipEventRecord(ev[1], c->stream);
    (void)hipEventRecord(ev[4], c->stream);
    for (int s = 0; s < n_fused && !st; ++s)
        st = launch_or2(c, (s & 1) ? c->ang2 : c->ang, (s & 1) ? c->ang : c->ang2, false);
    (void)hipEventRecord(ev[5], c->stream);
    (void)hipEventRecord(ev[2], c->stream);
    for (int s = n_fused; s < n_or && !st; ++s)
        for (int col = 0; col < 2 && !st; ++col) st = launch_half(c, kOver, col, s, false);
    (void)hipEventRecord(ev[3], c->stream);
    (void)hipEventRecord(ev[6], c->stream);
    if (!st && launch_tick(c->d_ctl, 1u, 0u, 0u, 0, c->stream) != hipSuccess)
        st = fail(c, XY_ERR_HIP, "tick launch failed");
    (void)hipEventRecord(ev[7], c->stream);
    if (!st && hipStreamSynchronize(c->stream) != hipSuccess) st = fail(c, XY_ERR_HIP, "sync failed");
    if (!st) {
        const int pairs[4][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}};
        for (int k = 0; k < 4; ++k) {
            float t = 0.f;
            (void)hipEventElapsedTime(&t, ev[pairs[k][0]], ev[pairs[k][1]]);
            ms[k] = counts[k] ? (double)t : 0.0;
            launches[k] = counts[k];
        }
        c->t += 1;
        c->e_fresh = c->bonds_fresh = false;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return st;
}

xy_status xy_measure(xy_ctx c, double *obs, int32_t obs_on_device)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (!obs) return fail(c, XY_ERR_ARG, "obs is NULL");
    double *dst = c->d_obs;
    xy_status st;
    if (obs_on_device && (st = gpu_buffer(c, obs, sizeof(double) * 5 * c->R_total, "obs", (void **)&dst)))
        return st;
    if ((st = enqueue_measure_kernel(c))) return st;
    if ((st = enqueue_finalize(c, kPartMeas, dst, 0, true, false, c->d_bonds))) return st;
    c->e_fresh = true;
    c->bonds_fresh = true;
    if (!obs_on_device) {
        XY_HIP(c, hipMemcpyAsync(obs, c->d_obs, sizeof(double) * 5 * c->R_total, hipMemcpyDeviceToHost,
                                 c->stream));
        return check_bad(c);
    }
    return XY_OK;
}

xy_status xy_exchange(xy_ctx c, int64_t *n_acc)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (c->tau >= 0xffffffffull) return fail(c, XY_ERR_STATE, "exchange counter would overflow 32 bits");
    xy_status st;
    if (!c->e_fresh) {
        if ((st = enqueue_measure_kernel(c))) return st;
        if ((st = enqueue_finalize(c, kPartMeas, nullptr, 0, true, false, c->d_bonds))) return st;
        c->e_fresh = true;
        c->bonds_fresh = true;
    }
    if ((st = enqueue_finalize(c, kPartMeas, nullptr, 0, false, true))) return st;
    XY_HIP(c, launch_tick(c->d_ctl, 0u, 1u, 0u, 0, c->stream));
    c->tau += 1;
    if (n_acc) {
        std::vector<unsigned long long> v(c->R_total);
        XY_HIP(c, hipMemcpyAsync(v.data(), c->d_sacc, sizeof(unsigned long long) * c->R_total,
                                 hipMemcpyDeviceToHost, c->stream));
        XY_HIP(c, hipStreamSynchronize(c->stream));
        for (int i = 0; i < c->R_total; ++i) n_acc[i] = (int64_t)v[i];
    }
    return XY_OK;
}

xy_status xy_run(xy_ctx c, int32_t n_sweeps, int32_t n_metro, int32_t n_or, int32_t exchange_every,
                 double *obs_dev)
{
    return xy_run_ex(c, n_sweeps, n_metro, n_or, exchange_every, obs_dev, nullptr);
}

xy_status xy_run_ex(xy_ctx c, int32_t n_sweeps, int32_t n_metro, int32_t n_or, int32_t exchange_every,
                    double *obs_dev, double *bonds_dev)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (n_sweeps < 0 || exchange_every < 0) return fail(c, XY_ERR_ARG, "n_sweeps and exchange_every must be >= 0");
    if (n_metro < 0 || n_or < 0 || n_metro + n_or < 1 || n_metro > 255 || n_or > 65535)
        return fail(c, XY_ERR_ARG, "need 0 <= n_metro <= 255, 0 <= n_or, n_metro + n_or >= 1");
    if (c->t + (uint64_t)n_sweeps > 0xffffffffull || c->tau + (uint64_t)n_sweeps > 0xffffffffull)
        return fail(c, XY_ERR_STATE, "counters would overflow 32 bits");
    xy_status st0 = poll_bad(c);
    if (st0) return st0;
    if (n_sweeps == 0) return XY_OK;
    if (obs_dev && (st0 = gpu_buffer(c, obs_dev, sizeof(double) * 5 * c->R_total * (size_t)n_sweeps, "obs_dev",
                                     (void **)&obs_dev)))
        return st0;
    if (bonds_dev && (st0 = gpu_buffer(c, bonds_dev, sizeof(double) * 6 * c->R_total * (size_t)n_sweeps,
                                       "bonds_dev", (void **)&bonds_dev)))
        return st0;

    // Captured graphs of `batch` sweeps, each sweep + measure (+ exchange),
    // then one counter update (t, tau, observable ring).  Nothing in the
    // measurement or the exchange reads t, so it advances with the others.
    auto get_graph = [&](int exch, int batch, hipGraphExec_t *exec) -> xy_status {
        GraphKey key{n_metro, n_or, exch, batch, obs_dev, bonds_dev};
        for (auto &g : c->graphs)
            if (g.key == key) {
                *exec = g.exec;
                return XY_OK;
            }
        if (c->graphs.size() >= kMaxGraphs) {
            // release the oldest graph that this call cannot be using
            for (auto it = c->graphs.begin(); it != c->graphs.end(); ++it) {
                const GraphKey &k = it->key;
                if (k.n_metro == n_metro && k.n_or == n_or && k.obs == obs_dev && k.bonds == bonds_dev) continue;
                (void)hipStreamSynchronize(c->stream);
                if (it->exec) (void)hipGraphExecDestroy(it->exec);
                if (it->graph) (void)hipGraphDestroy(it->graph);
                c->graphs.erase(it);
                break;
            }
        }
        GraphEntry g;
        g.key = key;
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        XY_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        xy_status st = XY_OK;
        for (int b = 0; b < batch && !st; ++b) {
            st = enqueue_sweep(c, n_metro, n_or, true, bonds_dev != nullptr, false);
            if (!st)
                st = enqueue_finalize(c, sweep_partials_layout(c, n_or), obs_dev, 1, true, exch != 0,
                                      bonds_dev);
            if (!st) {
                hipError_t e = launch_tick(c->d_ctl, 1u, exch ? 1u : 0u, (obs_dev || bonds_dev) ? 1u : 0u, 0,
                                           c->cap_stream);
                if (e != hipSuccess) st = fail(c, XY_ERR_HIP, "tick launch failed");
            }
        }
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
        c->stream = user;
        if (st) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return fail(c, XY_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(c, XY_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        g.graph = graph;
        c->graphs.push_back(g);
        *exec = g.exec;
        return XY_OK;
    };

    xy_status st;
    if (exchange_every <= 1) {
        // every sweep alike: batches of kSweepsPerGraph, then single sweeps
        const int ex = exchange_every;
        const int batch = std::min(n_sweeps, kSweepsPerGraph);
        const int n_batches = n_sweeps / batch, rest = n_sweeps - n_batches * batch;
        hipGraphExec_t g_batch = nullptr, g_one = nullptr;
        if ((st = get_graph(ex, batch, &g_batch))) return st;
        if (rest > 0 && (st = get_graph(ex, 1, &g_one))) return st;
        XY_HIP(c, launch_tick(c->d_ctl, 0u, 0u, 0u, 1, c->stream));  // ring <- 0
        for (int b = 0; b < n_batches; ++b) XY_HIP(c, hipGraphLaunch(g_batch, c->stream));
        for (int s = 0; s < rest; ++s) XY_HIP(c, hipGraphLaunch(g_one, c->stream));
        c->t += (uint64_t)n_sweeps;
        if (ex) c->tau += (uint64_t)n_sweeps;
    } else {
        hipGraphExec_t g_plain = nullptr, g_exch = nullptr;
        if ((st = get_graph(0, 1, &g_plain))) return st;
        if ((st = get_graph(1, 1, &g_exch))) return st;
        XY_HIP(c, launch_tick(c->d_ctl, 0u, 0u, 0u, 1, c->stream));  // ring <- 0
        for (int s = 0; s < n_sweeps; ++s) {
            const bool ex = ((s + 1) % exchange_every) == 0;
            XY_HIP(c, hipGraphLaunch(ex ? g_exch : g_plain, c->stream));
            c->t += 1;
            if (ex) c->tau += 1;
        }
    }
    c->e_fresh = true;
    c->bonds_fresh = false;
    // the sentinel as this loop leaves it, looked at (without waiting) by the next xy_run
    XY_HIP(c, hipMemcpyAsync(c->h_bad, c->d_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    XY_HIP(c, hipEventRecord(c->bad_ev, c->stream));
    c->bad_pending = true;
    return XY_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: tiles of each lattice for the Metropolis and over-relaxation
// half-sweeps and for the fused substep, timed on the whole batch
// (coordinate descent over the lattices), then the over-relaxation schedule
// (fused pass or two half-sweeps) and the workgroup cap.  The Metropolis
// launches are timed with their float64 re-decision, as they run in a sweep.
// Angles and acceptance counters are saved before and restored after, and
// the sweep counter is not advanced, so tuning leaves the chain untouched
// (tiles, schedule and cap change the launches, not the result).
// ---------------------------------------------------------------------------
xy_status xy_autotune(xy_ctx c, int32_t n_metro, int32_t n_or, int32_t reps)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (c->prec != XY_FP32) return XY_OK;  // plain kernels have no tile choice
    if (n_metro < 0 || n_or < 0 || n_metro + n_or < 1 || reps < 1 || reps > 100)
        return fail(c, XY_ERR_ARG, "need n_metro, n_or >= 0, n_metro + n_or >= 1, 1 <= reps <= 100");
    XY_HIP(c, hipStreamSynchronize(c->stream));
    // Every lattice of a batch shares one launch, so each candidate is timed
    // on the whole batch: coordinate descent, one lattice at a time, the
    // others keeping their current tiles.  The Metropolis and over-relaxation
    // half-sweeps modify the configuration and the acceptance counters, which
    // are saved first and restored at the end; the fused kernel only writes
    // the second buffer.
    void *save = nullptr;
    unsigned long long *save_acc = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const size_t bytes = (size_t)c->n_elems * c->elem;
    xy_status st = XY_OK;
    if ((st = dev_alloc(c, (char **)&save, bytes)) || (st = dev_alloc(c, &save_acc, c->R_total))) {
        (void)hipFree(save);
        (void)hipFree(save_acc);
        return st;
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        st = fail(c, XY_ERR_HIP, "hipEventCreate failed");
    if (!st && (hipMemcpyAsync(save, c->ang, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
                hipMemcpyAsync(save_acc, c->d_macc, sizeof(unsigned long long) * c->R_total,
                               hipMemcpyDeviceToDevice, c->stream) != hipSuccess))
        st = fail(c, XY_ERR_HIP, "saving the state failed");
    const int grid_cap = c->grid_sweep;
    const int w_metro = n_metro, w_over = n_or - fused_substeps(c, n_or);
    auto half_cost = [&](double *cost) -> xy_status {
        *cost = 0.0;
        for (int kind = 0; kind < 2; ++kind) {
            const int weight = kind == 0 ? w_metro : w_over;
            if (weight == 0) continue;
            double ms = 0.0;
            xy_status s2 = time_launches(c, e0, e1, reps,
                                         [&] { return launch_half(c, kind == 0 ? kMetro : kOver, 0, 0, false); }, &ms);
            if (s2) return s2;
            *cost += weight * ms;
        }
        return XY_OK;
    };
    for (int l = 0; l < c->n_lat && !st && (w_metro + w_over) > 0; ++l) {
        Tiling best = c->tiles[l];
        double best_cost = 1e300;
        for (const auto &cand : tile_candidates(c->L[l])) {
            if (xy_set_tiling(c, l, cand.first, cand.second, grid_cap) != XY_OK) continue;
            double cost = 0.0;
            if ((st = half_cost(&cost))) break;
            if (cost < best_cost) {
                best_cost = cost;
                best = c->tiles[l];
            }
        }
        if (st) break;
        c->tiles[l] = best;
        st = relayout(c);
    }
    if (!st && c->fused_avail && n_or >= 2) {
        c->fused_or = true;
        for (int l = 0; l < c->n_lat && !st; ++l) {
            Tiling best = c->tiles2[l];
            double best_ms = 1e300;
            for (const auto &cand : tile_candidates(c->L[l])) {
                if (xy_set_tiling_fused(c, l, cand.first, cand.second) != XY_OK) continue;
                double ms = 0.0;
                if ((st = time_launches(c, e0, e1, reps, [&] { return launch_or2(c, c->ang, c->ang2, false); },
                                        &ms)))
                    break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c->tiles2[l];
                }
            }
            if (st) break;
            c->tiles2[l] = best;
            st = relayout(c);
        }
    }
    // Sublattice schedule of the over-relaxation substeps: one fused pass
    // over both colours, or the two half-sweep launches (the same result, bit
    // for bit); the faster in the tiles just chosen is kept.
    if (!st && c->fused_avail && n_or >= 2) {
        double ms_fused = 0.0, ms_half = 0.0;
        st = time_launches(c, e0, e1, reps, [&] { return launch_or2(c, c->ang, c->ang2, false); }, &ms_fused);
        if (!st)
            st = time_launches(c, e0, e1, reps, [&] {
                const xy_status s0 = launch_half(c, kOver, 0, 0, false);
                return s0 ? s0 : launch_half(c, kOver, 1, 0, false);
            }, &ms_half);
        if (!st) {
            c->fused_or = ms_fused <= ms_half;
            st = relayout(c);
        }
    }
    // Workgroup cap of the tiled and fused launches: the resident capacity
    // (0) or a fixed multiple of the compute units, timed on whole sweeps
    // (the sweep counter is not advanced; the state is restored below).
    if (!st) {
        int best_cap = c->grid_sweep;
        double best_ms = 1e300;
        for (const int cap : {0, 2 * c->n_cu, 3 * c->n_cu, 4 * c->n_cu, 6 * c->n_cu}) {
            c->grid_sweep = cap;
            double ms = 0.0;
            if ((st = time_launches(c, e0, e1, reps, [&] { return enqueue_sweep(c, n_metro, n_or, false, false, false); },
                                    &ms)))
                break;
            if (ms < best_ms) {
                best_ms = ms;
                best_cap = cap;
            }
        }
        c->grid_sweep = best_cap;
    }
    (void)hipStreamSynchronize(c->stream);
    if (hipMemcpyAsync(c->ang, save, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->d_macc, save_acc, sizeof(unsigned long long) * c->R_total, hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        if (!st) st = fail(c, XY_ERR_HIP, "restoring the state failed");
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(save);
    (void)hipFree(save_acc);
    free_graphs(c);  // captured launches carry the old shapes
    c->e_fresh = c->bonds_fresh = false;
    return st;
}

xy_status xy_set_tiling(xy_ctx c, int32_t lattice, int32_t ty, int32_t tz, int32_t grid_cap)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (c->prec != XY_FP32) return fail(c, XY_ERR_UNSUPPORTED, "tiling applies to FP32 contexts only");
    if (lattice < 0 || lattice >= c->n_lat) return fail(c, XY_ERR_ARG, "lattice out of range");
    const int L = c->L[lattice];
    if (ty < 1 || tz < 1 || L % ty != 0 || L % tz != 0)
        return fail(c, XY_ERR_ARG, "ty and tz must divide L");
    if (ty * (L / 2) > 8 * kBlock) return fail(c, XY_ERR_ARG, "ty * L/2 must be <= 2048");
    if (grid_cap < 0) return fail(c, XY_ERR_ARG, "grid_cap must be >= 0");
    Tiling t;
    t.TY = ty;
    t.TZ = tz;
    t.spt = spt_for(ty * (L / 2));
    c->tiles[lattice] = t;
    c->grid_sweep = grid_cap;
    return relayout(c);
}

xy_status xy_set_proposal_window(xy_ctx c, double window)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (!(window >= 0.0) || window > 6.283185307179586476925286766559)
        return fail(c, XY_ERR_ARG, "window must be in [0, 2 pi]");
    c->window = window;
    free_graphs(c);  // captured launches carry the old value
    return XY_OK;
}

xy_status xy_set_tiling_fused(xy_ctx c, int32_t lattice, int32_t ty, int32_t tz)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (!c->fused_avail) return fail(c, XY_ERR_UNSUPPORTED, "this context cannot use the fused over-relaxation");
    if (lattice < 0 || lattice >= c->n_lat) return fail(c, XY_ERR_ARG, "lattice out of range");
    const int L = c->L[lattice];
    if (ty < 1 || tz < 1 || L % ty != 0 || L % tz != 0)
        return fail(c, XY_ERR_ARG, "ty and tz must divide L");
    if (!or2_tile_ok(ty, L / 2))
        return fail(c, XY_ERR_ARG, "fused tile needs ty * L/2 <= 1280 and at most 64 KiB of LDS");
    Tiling t;
    t.TY = ty;
    t.TZ = tz;
    t.spt = spt_for(ty * (L / 2));
    c->tiles2[lattice] = t;
    c->fused_or = true;  // a fused tile selects the fused schedule
    return relayout(c);
}

xy_status xy_get_tiling_fused(xy_ctx c, int32_t lattice, int32_t *ty, int32_t *tz)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (lattice < 0 || lattice >= c->n_lat) return fail(c, XY_ERR_ARG, "lattice out of range");
    if (ty) *ty = c->fused_or ? c->tiles2[lattice].TY : 0;
    if (tz) *tz = c->fused_or ? c->tiles2[lattice].TZ : 0;
    return XY_OK;
}

xy_status xy_get_tiling(xy_ctx c, int32_t lattice, int32_t *ty, int32_t *tz, int32_t *grid_cap)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (lattice < 0 || lattice >= c->n_lat) return fail(c, XY_ERR_ARG, "lattice out of range");
    if (c->prec != XY_FP32) {
        if (ty) *ty = 0;
        if (tz) *tz = 0;
        if (grid_cap) *grid_cap = 0;
        return XY_OK;
    }
    if (ty) *ty = c->tiles[lattice].TY;
    if (tz) *tz = c->tiles[lattice].TZ;
    if (grid_cap) *grid_cap = c->grid_sweep;
    return XY_OK;
}

xy_status xy_get_bond_sums(xy_ctx c, double *out, int32_t out_on_device)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (!out) return fail(c, XY_ERR_ARG, "out is NULL");
    if (out_on_device) {
        xy_status st = gpu_buffer(c, out, sizeof(double) * 6 * c->R_total, "out", (void **)&out);
        if (st) return st;
    }
    if (!c->bonds_fresh) {
        xy_status st = enqueue_measure_kernel(c);
        if (!st) st = enqueue_finalize(c, kPartMeas, nullptr, 0, true, false, c->d_bonds);
        if (st) return st;
        c->e_fresh = true;
        c->bonds_fresh = true;
    }
    // the runtime tells device memory from pinned host memory (hipMemcpyDefault)
    XY_HIP(c, hipMemcpyAsync(out, c->d_bonds, sizeof(double) * 6 * c->R_total,
                             out_on_device ? hipMemcpyDefault : hipMemcpyDeviceToHost, c->stream));
    if (!out_on_device) XY_HIP(c, hipStreamSynchronize(c->stream));
    return XY_OK;
}

xy_status xy_get_counters(xy_ctx c, uint64_t *t, uint64_t *tau)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (t) *t = c->t;
    if (tau) *tau = c->tau;
    return XY_OK;
}

xy_status xy_get_permutation(xy_ctx c, int32_t lattice, int32_t *slot)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (lattice < 0 || lattice >= c->n_lat || !slot) return fail(c, XY_ERR_ARG, "bad lattice or NULL slot");
    XY_HIP(c, hipMemcpyAsync(slot, c->d_slot_of + c->lat_sweep[lattice].pos_base,
                             sizeof(int32_t) * c->R[lattice], hipMemcpyDeviceToHost, c->stream));
    return sync_stream(c);
}

xy_status xy_get_swap_accepts(xy_ctx c, int64_t *n_acc)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (!n_acc) return fail(c, XY_ERR_ARG, "n_acc is NULL");
    std::vector<unsigned long long> v(c->R_total);
    XY_HIP(c, hipMemcpyAsync(v.data(), c->d_sacc, sizeof(unsigned long long) * c->R_total,
                             hipMemcpyDeviceToHost, c->stream));
    XY_HIP(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < c->R_total; ++i) n_acc[i] = (int64_t)v[i];
    return XY_OK;
}

xy_status xy_get_metro_accepts(xy_ctx c, int64_t *n_acc)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (!n_acc) return fail(c, XY_ERR_ARG, "n_acc is NULL");
    std::vector<unsigned long long> v(c->R_total);
    XY_HIP(c, hipMemcpyAsync(v.data(), c->d_macc, sizeof(unsigned long long) * c->R_total,
                             hipMemcpyDeviceToHost, c->stream));
    XY_HIP(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < c->R_total; ++i) n_acc[i] = (int64_t)v[i];
    return XY_OK;
}

xy_status xy_get_recheck_overflow(xy_ctx c, uint64_t *n)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (!n) return fail(c, XY_ERR_ARG, "n is NULL");
    uint32_t v = 0;
    XY_HIP(c, hipMemcpyAsync(&v, (const char *)c->d_rq + offsetof(RecheckQueue, overflow), sizeof(v),
                             hipMemcpyDeviceToHost, c->stream));
    XY_HIP(c, hipStreamSynchronize(c->stream));
    *n = v;
    return XY_OK;
}

// Angle access by (lattice, beta-position) through the slot permutation.
static xy_status slot_of_position(xy_ctx c, int lattice, int beta_pos, int *slot)
{
    if (lattice < 0 || lattice >= c->n_lat) return fail(c, XY_ERR_ARG, "lattice out of range");
    if (beta_pos < 0 || beta_pos >= c->R[lattice]) return fail(c, XY_ERR_ARG, "beta_pos out of range");
    int32_t s = 0;
    XY_HIP(c, hipMemcpyAsync(&s, c->d_slot_of + c->lat_sweep[lattice].pos_base + beta_pos,
                             sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    XY_HIP(c, hipStreamSynchronize(c->stream));
    *slot = s;
    return XY_OK;
}

// Natural-order radians of the configuration at (lattice, beta_pos) held in
// the angle buffer `buf` (the primary one or the fused pass's second one).
static xy_status read_angles(xy_ctx c, const void *buf, int32_t lattice, int32_t beta_pos, double *host)
{
    if (!host) return fail(c, XY_ERR_ARG, "host is NULL");
    int slot = 0;
    xy_status st = slot_of_position(c, lattice, beta_pos, &slot);
    if (st) return st;
    const LatDev &d = c->lat_sweep[lattice];
    std::vector<char> raw((size_t)d.N * c->elem);
    XY_HIP(c, hipMemcpyAsync(raw.data(), (const char *)buf + (size_t)(d.base + (int64_t)slot * d.N) * c->elem,
                             raw.size(), hipMemcpyDeviceToHost, c->stream));
    XY_HIP(c, hipStreamSynchronize(c->stream));
    const int L = d.L, half = d.half;
    const double twopi = 6.283185307179586476925286766559;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                const int col = (x + y + z) & 1;
                const int64_t src = (int64_t)col * (d.N / 2) + ((int64_t)z * L + y) * half + (x >> 1);
                const int64_t i = x + (int64_t)L * (y + (int64_t)L * z);
                host[i] = (c->prec == XY_FP32) ? (double)((const float *)raw.data())[src] * twopi
                                               : ((const double *)raw.data())[src];
            }
    return XY_OK;
}

xy_status xy_get_angles(xy_ctx c, int32_t lattice, int32_t beta_pos, double *host)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    return read_angles(c, c->ang, lattice, beta_pos, host);
}

xy_status xy_get_angles_fused_mid(xy_ctx c, int32_t lattice, int32_t beta_pos, double *host)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (!c->fused_or || !c->ang2)
        return fail(c, XY_ERR_UNSUPPORTED, "this context does not use the fused over-relaxation");
    return read_angles(c, c->ang2, lattice, beta_pos, host);
}

xy_status xy_get_sites(xy_ctx c, int32_t lattice, int32_t beta_pos, int64_t n, const int64_t *sites,
                       double *host)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (n < 0 || (n > 0 && (!sites || !host))) return fail(c, XY_ERR_ARG, "bad n or NULL array");
    if (n > ((int64_t)1 << 26)) return fail(c, XY_ERR_ARG, "at most 2^26 sites per call");
    int slot = 0;
    xy_status st = slot_of_position(c, lattice, beta_pos, &slot);
    if (st || n == 0) return st;
    const LatDev &d = c->lat_sweep[lattice];
    for (int64_t g = 0; g < n; ++g)
        if (sites[g] < 0 || sites[g] >= d.N) return fail(c, XY_ERR_ARG, "site index out of range");
    int64_t *d_sites = nullptr;
    double *d_out = nullptr;
    if ((st = dev_alloc(c, &d_sites, (size_t)n)) || (st = dev_alloc(c, &d_out, (size_t)n))) {
        (void)hipFree(d_sites);
        return st;
    }
    hipError_t e = hipMemcpyAsync(d_sites, sites, sizeof(int64_t) * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = launch_gather(c->prec == XY_FP32, c->ang, d.base + (int64_t)slot * d.N, d.L, n, d_sites, d_out,
                          c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host, d_out, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d_sites);
    (void)hipFree(d_out);
    if (e != hipSuccess) return fail(c, XY_ERR_HIP, std::string("xy_get_sites: ") + hipGetErrorString(e));
    return XY_OK;
}

// xy_get_sites without allocating: the site list and the gathered angles are
// staged in this device's static scratch array instead of per-call buffers.
xy_status xy_get_sites_noalloc(xy_ctx c, int32_t lattice, int32_t beta_pos, int64_t n,
                               const int64_t *sites, double *host)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (n < 0 || (n > 0 && (!sites || !host))) return fail(c, XY_ERR_ARG, "bad n or NULL array");
    if (n > XY_NOALLOC_MAX_SITES)
        return fail(c, XY_ERR_ARG, "n exceeds the static scratch capacity (XY_NOALLOC_MAX_SITES = 262144 sites)");
    if (!c->scratch) return fail(c, XY_ERR_STATE, "device scratch address not set up");
    int slot = 0;
    xy_status st = slot_of_position(c, lattice, beta_pos, &slot);
    if (st || n == 0) return st;
    const LatDev &d = c->lat_sweep[lattice];
    for (int64_t g = 0; g < n; ++g)
        if (sites[g] < 0 || sites[g] >= d.N) return fail(c, XY_ERR_ARG, "site index out of range");
    int64_t *d_sites = (int64_t *)c->scratch;
    double *d_out = (double *)((char *)c->scratch + (size_t)XY_NOALLOC_MAX_SITES * sizeof(int64_t));
    hipError_t e = hipMemcpyAsync(d_sites, sites, sizeof(int64_t) * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = launch_gather(c->prec == XY_FP32, c->ang, d.base + (int64_t)slot * d.N, d.L, n, d_sites, d_out,
                          c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host, d_out, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, XY_ERR_HIP, std::string("xy_get_sites_noalloc: ") + hipGetErrorString(e));
    return XY_OK;
}

xy_status xy_set_angles(xy_ctx c, int32_t lattice, int32_t beta_pos, const double *host)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (!host) return fail(c, XY_ERR_ARG, "host is NULL");
    int slot = 0;
    xy_status st = slot_of_position(c, lattice, beta_pos, &slot);
    if (st) return st;
    const LatDev &d = c->lat_sweep[lattice];
    const int L = d.L, half = d.half;
    const double twopi = 6.283185307179586476925286766559;
    std::vector<char> raw((size_t)d.N * c->elem);
    for (int64_t i = 0; i < d.N; ++i)
        if (!std::isfinite(host[i])) return fail(c, XY_ERR_ARG, "angles must be finite");
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                const int col = (x + y + z) & 1;
                const int64_t dst = (int64_t)col * (d.N / 2) + ((int64_t)z * L + y) * half + (x >> 1);
                const int64_t i = x + (int64_t)L * (y + (int64_t)L * z);
                double v = std::fmod(host[i], twopi);
                if (v < 0.0) v += twopi;
                if (v >= twopi) v = 0.0;
                if (c->prec == XY_FP32) {
                    float tf = (float)(v / twopi);
                    if (!(tf < 1.0f)) tf = 0.0f;
                    ((float *)raw.data())[dst] = tf;
                } else {
                    ((double *)raw.data())[dst] = v;
                }
            }
    XY_HIP(c, hipMemcpyAsync((char *)c->ang + (size_t)(d.base + (int64_t)slot * d.N) * c->elem, raw.data(),
                             raw.size(), hipMemcpyHostToDevice, c->stream));
    XY_HIP(c, hipStreamSynchronize(c->stream));
    c->e_fresh = c->bonds_fresh = false;
    return XY_OK;
}

// --- checkpoint blob -------------------------------------------------------
namespace {
struct BlobHeader {
    char magic[8];
    uint32_t version, n_lat;
    int32_t prec, R_total;
    uint64_t seed, t, tau;
    int64_t n_elems;
};
constexpr char kMagic[8] = {'X', 'Y', 'S', 'T', 'A', 'T', 'E', '1'};

static size_t blob_size(xy_ctx c)
{
    return sizeof(BlobHeader) + sizeof(int32_t) * 2 * c->n_lat + sizeof(double) * c->R_total +
           sizeof(int32_t) * 2 * c->R_total + sizeof(unsigned long long) * 2 * c->R_total +
           (size_t)c->n_elems * c->elem;
}
}  // namespace

xy_status xy_get_state(xy_ctx c, void *blob, size_t *size)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (!size) return fail(c, XY_ERR_ARG, "size is NULL");
    const size_t need = blob_size(c);
    if (!blob) {
        *size = need;
        return XY_OK;
    }
    if (*size < need) return fail(c, XY_ERR_ARG, "blob too small");
    char *p = (char *)blob;
    BlobHeader h{};
    std::memcpy(h.magic, kMagic, 8);
    h.version = 1;
    h.n_lat = (uint32_t)c->n_lat;
    h.prec = c->prec;
    h.R_total = c->R_total;
    h.seed = c->seed;
    h.t = c->t;
    h.tau = c->tau;
    h.n_elems = c->n_elems;
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    std::memcpy(p, c->L.data(), sizeof(int32_t) * c->n_lat);
    p += sizeof(int32_t) * c->n_lat;
    std::memcpy(p, c->R.data(), sizeof(int32_t) * c->n_lat);
    p += sizeof(int32_t) * c->n_lat;
    std::memcpy(p, c->beta.data(), sizeof(double) * c->R_total);
    p += sizeof(double) * c->R_total;
    XY_HIP(c, hipMemcpyAsync(p, c->d_pos, sizeof(int32_t) * c->R_total, hipMemcpyDeviceToHost, c->stream));
    p += sizeof(int32_t) * c->R_total;
    XY_HIP(c, hipMemcpyAsync(p, c->d_slot_of, sizeof(int32_t) * c->R_total, hipMemcpyDeviceToHost, c->stream));
    p += sizeof(int32_t) * c->R_total;
    XY_HIP(c, hipMemcpyAsync(p, c->d_macc, sizeof(unsigned long long) * c->R_total, hipMemcpyDeviceToHost, c->stream));
    p += sizeof(unsigned long long) * c->R_total;
    XY_HIP(c, hipMemcpyAsync(p, c->d_sacc, sizeof(unsigned long long) * c->R_total, hipMemcpyDeviceToHost, c->stream));
    p += sizeof(unsigned long long) * c->R_total;
    XY_HIP(c, hipMemcpyAsync(p, c->ang, (size_t)c->n_elems * c->elem, hipMemcpyDeviceToHost, c->stream));
    XY_HIP(c, hipStreamSynchronize(c->stream));
    *size = need;
    return XY_OK;
}

xy_status xy_set_state(xy_ctx c, const void *blob, size_t size)
{
    if (!c) return fail(nullptr, XY_ERR_ARG, "ctx is NULL");
    if (!blob) return fail(c, XY_ERR_ARG, "blob is NULL");
    if (size != blob_size(c)) return fail(c, XY_ERR_STATE, "blob size does not match this context");
    const char *p = (const char *)blob;
    BlobHeader h;
    std::memcpy(&h, p, sizeof h);
    p += sizeof h;
    if (std::memcmp(h.magic, kMagic, 8) != 0 || h.version != 1) return fail(c, XY_ERR_STATE, "not a state blob");
    if ((int)h.n_lat != c->n_lat || h.prec != c->prec || h.R_total != c->R_total || h.seed != c->seed ||
        h.n_elems != c->n_elems)
        return fail(c, XY_ERR_STATE, "blob was written by a context with another configuration");
    if (std::memcmp(p, c->L.data(), sizeof(int32_t) * c->n_lat) != 0 ||
        std::memcmp(p + sizeof(int32_t) * c->n_lat, c->R.data(), sizeof(int32_t) * c->n_lat) != 0 ||
        std::memcmp(p + sizeof(int32_t) * 2 * c->n_lat, c->beta.data(), sizeof(double) * c->R_total) != 0)
        return fail(c, XY_ERR_STATE, "blob lattices or ladders differ from this context");
    p += sizeof(int32_t) * 2 * c->n_lat + sizeof(double) * c->R_total;
    // validate the permutation before touching device state
    {
        const int32_t *pos = (const int32_t *)p, *slot_of = pos + c->R_total;
        for (int l = 0; l < c->n_lat; ++l) {
            const int pb = c->lat_sweep[l].pos_base;
            for (int r = 0; r < c->R[l]; ++r) {
                const int32_t k = pos[pb + r];
                if (k < 0 || k >= c->R[l] || slot_of[pb + k] != r)
                    return fail(c, XY_ERR_STATE, "blob permutation is not a bijection");
            }
        }
    }
    if (h.t > 0xffffffffull || h.tau > 0xffffffffull) return fail(c, XY_ERR_STATE, "blob counters out of range");
    XY_HIP(c, hipMemcpyAsync(c->d_pos, p, sizeof(int32_t) * c->R_total, hipMemcpyHostToDevice, c->stream));
    p += sizeof(int32_t) * c->R_total;
    XY_HIP(c, hipMemcpyAsync(c->d_slot_of, p, sizeof(int32_t) * c->R_total, hipMemcpyHostToDevice, c->stream));
    p += sizeof(int32_t) * c->R_total;
    XY_HIP(c, hipMemcpyAsync(c->d_macc, p, sizeof(unsigned long long) * c->R_total, hipMemcpyHostToDevice, c->stream));
    p += sizeof(unsigned long long) * c->R_total;
    XY_HIP(c, hipMemcpyAsync(c->d_sacc, p, sizeof(unsigned long long) * c->R_total, hipMemcpyHostToDevice, c->stream));
    p += sizeof(unsigned long long) * c->R_total;
    XY_HIP(c, hipMemcpyAsync(c->ang, p, (size_t)c->n_elems * c->elem, hipMemcpyHostToDevice, c->stream));
    Ctl ctl{(uint32_t)h.t, (uint32_t)h.tau, 0u, 0u};
    XY_HIP(c, hipMemcpyAsync(c->d_ctl, &ctl, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
    XY_HIP(c, hipStreamSynchronize(c->stream));
    c->t = h.t;
    c->tau = h.tau;
    c->e_fresh = c->bonds_fresh = false;
    return XY_OK;
}

const char *xy_last_error(xy_ctx c)
{
    return c ? c->err.c_str() : g_init_error.c_str();
}

void xy_destroy(xy_ctx c)
{
    if (!c) return;
    free_all(c);
    delete c;
}

}  // extern "C"
