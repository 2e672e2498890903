// Shared host/device declarations of the XY-model kernels and their launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xy {

constexpr int kBlock = 256;  // threads per workgroup of the tiled and plain kernels
// measurement partials per work item: S, Mx, My, C_x, C_y, C_z, I_x, I_y, I_z,
// with S = sum over colour-1 sites of S_i . h_i, so that E = -S (Eq. (1));
// the bond sums are filled only when asked for (SweepArgs::bonds)
constexpr int kPartials = 9;
constexpr int kPartialsNoBonds = 3;  // S, Mx, My: what a measurement without bond sums fills

// One lattice of a batch, as the kernels see it.  All offsets are in angle
// elements (float for FP32, double for FP64).
struct LatDev {
    int32_t L, half, R, lat;   // linear size, L/2, ladder length, lattice index
    int64_t base;              // offset of storage slot 0 of this lattice
    int64_t N;                 // L^3 = elements per slot; each colour holds N/2
    int32_t pos_base;          // first entry of this lattice in position-indexed arrays
    int32_t TY, TZ;            // tile rows (y) and planes (z) of the tiled kernel
    int32_t ny, nz;            // L/TY, L/TZ
    int32_t item_base;         // first work item of this lattice (tiled or plain)
    int32_t items_per_slot;    // work items per storage slot
    int32_t pad_;
};

enum Kind : int { kMetro = 0, kOver = 1, kMeas = 2 };

// Device control block: counters read by every kernel of a sweep.
struct Ctl {
    uint32_t t;     // sweep counter (Philox c1 of Metropolis draws)
    uint32_t tau;   // exchange counter (Philox c1 of exchange draws)
    uint32_t ring;  // next observable record of a running loop
    uint32_t pad_;
};

// Metropolis decisions whose float32 acceptance probability lies within
// max(1e-5, 1.6e-5 beta) of the uniform are queued here by the FP32
// half-sweep and re-taken in float64 by a follow-up kernel (same-colour sites
// do not interact, so the deferral changes nothing).  The follow-up draws the
// site's proposal and uniform again from the same Philox counter.
struct RecheckEntry {
    int32_t li, slot;      // lattice, storage slot
    uint32_t q;            // index within the colour array; bit 31: the float32 decision (accepted)
    float cur;             // old angle (turns)
};

struct RecheckQueue {
    uint32_t count;
    uint32_t overflow;     // entries that did not fit: their float32 decision stands
    uint32_t capacity;
    uint32_t done;         // workgroups of the re-decision kernel that have finished
    RecheckEntry *entries;
};

struct SweepArgs {
    const LatDev *lats;
    int32_t n_lat;
    int32_t total_items;
    void *ang;                 // float* (FP32, turns) or double* (FP64, radians)
    void *ang_dst;             // fused over-relaxation: where the new configuration goes
    const double *beta;        // [R_total] by position index
    const int32_t *pos;        // [R_total] beta-position held by each storage slot
    const Ctl *ctl;
    uint32_t k0, k1;           // Philox key
    int32_t colour;
    int32_t substep;
    int32_t recheck;           // FP32 Metropolis: re-decide in float64 near the threshold
    int32_t bonds;             // measuring: also form the bond sums C_mu, I_mu of Eq. (6)
    float window_t;            // Metropolis proposal window in turns (0: uniform proposal)
    double window;             // the same in radians, for the float64 kernels
    RecheckQueue *rq;          // where those decisions are queued
    double *partials;          // [items][kPartials] when measuring
    unsigned long long *macc;  // [R_total] accepted Metropolis moves by position
};

// Launchers (stream-ordered, no synchronisation).
// With per_cu non-null the tiled launchers launch nothing and report in
// *per_cu how many workgroups of the selected kernel fit on one CU.
// full: every lattice of the launch fills its tile exactly (TY * L/2 = spt * kBlock)
hipError_t launch_tile_f32(int kind, bool fuse_measure, bool full, int spt, int halo, int grid,
                           size_t lds_bytes, const SweepArgs &a, hipStream_t s, int *per_cu = nullptr);
// lead: every lattice of the launch fills the first spt - 1 tile columns (TY * L/2 > (spt - 1) * kBlock)
hipError_t launch_or2_f32(bool fuse_measure, bool lead, int spt, int grid, size_t lds_bytes, const SweepArgs &a,
                          hipStream_t s, int *per_cu = nullptr);
// the plain (non-measuring) fused substep, built in its own translation unit
hipError_t launch_or2_plain(bool lead, int spt, int grid, size_t lds, const SweepArgs &a, hipStream_t s,
                            int *per_cu);
hipError_t launch_recheck(const SweepArgs &a, hipStream_t s);
hipError_t launch_plain_f64(int kind, bool fuse_measure, int grid, const SweepArgs &a, hipStream_t s);
hipError_t launch_init(bool fp32, bool ordered, const LatDev *lats, int n_lat,
                       int64_t total_sites, void *ang, uint32_t k0, uint32_t k1,
                       hipStream_t s);
hipError_t launch_finalize(const LatDev *lats, int n_lat, int max_R, const double *partials,
                           const double *beta, int32_t *pos, int32_t *slot_of, double *E_slot,
                           double *obs, double *bonds, int use_ring, int64_t ring_stride,
                           int64_t bond_stride, int do_sum, int do_exchange,
                           unsigned long long *sacc, Ctl *ctl, uint32_t k0, uint32_t k1, int *bad,
                           hipStream_t s);
hipError_t launch_gather(bool fp32, const void *ang, int64_t slot_base, int L, int64_t n,
                         const int64_t *sites, double *out, hipStream_t s);
hipError_t launch_tick(Ctl *ctl, uint32_t dt, uint32_t dtau, uint32_t dring, int set_ring,
                       hipStream_t s);

}  // namespace xy
