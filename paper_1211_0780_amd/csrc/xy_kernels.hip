// gfx950 kernels of the 3D XY model hot path (arXiv:1211.0780, Sec. II):
// checkerboard Metropolis and over-relaxation half-sweeps, observable
// reductions, parallel-tempering exchange, random start.
//
// Angle storage is colour-split: per storage slot, colour c's N/2 sites are
// ordered (z, y, j) with j = x/2 fastest.  Site (x, y, z) of colour c has
// x = 2j + p with p = (c + y + z) & 1.  Its six neighbours all have the other
// colour and sit at index j in rows (y +- 1, z) and (y, z +- 1), and at
// j and j + (p ? +1 : -1) (mod L/2) in its own row.
//
// The fused over-relaxation substep's kernel template is in
// xy_or2_kernel.h (its plain instantiations are built from xy_or2.hip, the
// measuring ones here); the device helpers both files use are in
// xy_kernel_common.h.
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "xy_device.h"
#include "xy_kernels.h"
#include "xy_kernel_common.h"
#include "xy_or2_kernel.h"

namespace xy {

// ---------------------------------------------------------------------------
// Re-take one queued near-threshold Metropolis decision in float64: the
// site's proposal and acceptance uniform are drawn again from its Philox
// counter (the same block and words as the half-sweep), the six neighbour
// angles (other colour, untouched by this half-sweep) are read again, dE and
// exp(-beta dE) evaluated in double, and the site is corrected where the
// float64 decision differs.
// ---------------------------------------------------------------------------
__device__ void recheck_entry(const SweepArgs &a, const RecheckEntry &en)
{
    const double twopi = 6.283185307179586476925286766559;
    const LatDev d = a.lats[en.li];
    const int L = d.L, half = d.half;
    const int64_t plane = (int64_t)L * half;
    const uint32_t q = en.q & 0x7fffffffu;
    const int fp32_accept = (int)(en.q >> 31);
    const int z = (int)(q / plane);
    const int rem = (int)(q - (int64_t)z * plane);
    const int y = rem / half, j = rem - y * half;
    const int p = (a.colour + y + z) & 1;
    float *angs = (float *)a.ang + d.base + (int64_t)en.slot * d.N;
    float *own = angs + (int64_t)a.colour * (d.N / 2);
    const float *oth = angs + (int64_t)(a.colour ^ 1) * (d.N / 2);
    const int k = a.pos[d.pos_base + en.slot];
    // the pair's block: counter word 0 is the even-plane site of this column
    const uint32_t zb = (uint32_t)(z & ~1);
    const uint32_t pb = (uint32_t)p ^ (uint32_t)(z & 1);
    const uint32_t ib = 2u * (uint32_t)j + pb + (uint32_t)L * ((uint32_t)y + (uint32_t)L * zb);
    const u32x4 r = philox4x32_10(ib, a.ctl->t, ((uint32_t)d.lat << 16) | (uint32_t)k,
                                  (kPhaseMetro << 24) | (uint32_t)a.substep, a.k0, a.k1);
    const uint32_t w0 = (z & 1) ? r.z : r.x, w1 = (z & 1) ? r.w : r.y;
    // the proposal exactly as the float32 half-sweep formed it (turns)
    const float u0 = unit24f(w0);
    const float prop = a.window_t > 0.0f ? frac_turn(__builtin_fmaf(a.window_t, u0 - 0.5f, en.cur)) : u0;
    const int ym = (y == 0) ? L - 1 : y - 1, yp = (y + 1 == L) ? 0 : y + 1;
    const int zm = (z == 0) ? L - 1 : z - 1, zp = (z + 1 == L) ? 0 : z + 1;
    const int jx = p ? ((j + 1 == half) ? 0 : j + 1) : ((j == 0) ? half - 1 : j - 1);
    const int64_t zo = (int64_t)z * plane;
    const int64_t nb[6] = {zo + (int64_t)y * half + j,  zo + (int64_t)y * half + jx,
                           zo + (int64_t)ym * half + j, zo + (int64_t)yp * half + j,
                           (int64_t)zm * plane + (int64_t)y * half + j,
                           (int64_t)zp * plane + (int64_t)y * half + j};
    double hx = 0.0, hy = 0.0;
    for (int m = 0; m < 6; ++m) {
        double sn, cn;
        sincos((double)oth[nb[m]] * twopi, &sn, &cn);
        hx += cn;
        hy += sn;
    }
    double so, co, sp, cp;
    sincos((double)en.cur * twopi, &so, &co);
    sincos((double)prop * twopi, &sp, &cp);
    const double dE = (co - cp) * hx + (so - sp) * hy;
    const bool acc = unit24d(w1) < exp(-a.beta[d.pos_base + k] * dE);
    if ((int)acc != fp32_accept) {
        own[q] = acc ? prop : en.cur;
        atomicAdd(a.macc + d.pos_base + k, acc ? 1ull : ~0ull);  // +1 or -1
    }
}

// The queued decisions of one half-sweep, re-taken by a follow-up launch (the
// kernel boundary orders it after every workgroup of the half-sweep).  The
// last workgroup to finish empties the queue for the next half-sweep.
__global__ __launch_bounds__(kBlock) void k_recheck(SweepArgs a)
{
    const uint32_t n = min(a.rq->count, a.rq->capacity);
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x)
        recheck_entry(a, a.rq->entries[e]);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&a.rq->done, 1u) == gridDim.x - 1) {
            a.rq->count = 0;
            a.rq->done = 0;
            __threadfence();
        }
    }
}

// ---------------------------------------------------------------------------
// Tiled FP32 half-sweep.  A work item is (lattice, slot, y-tile, z-chunk):
// TY rows of L/2 sites of the updated colour, streamed over TZ planes.  Each
// thread owns SPT (y, j) columns of the tile.  The other colour is read once
// per plane, turned into (cos, sin) once, kept in registers for the z
// neighbours (planes z-1, z+1 of the same column) and staged in LDS (plane
// z plus one halo row above and below the tile, double-buffered) for the
// x and y neighbours.  The next plane's loads are issued at the top of each
// plane step and stay in flight while this plane is computed.
//
// KIND = kMetro / kOver updates colour a.colour; kMeas (colour 1) only
// measures.  MEAS accumulates S = sum_{i in colour 1} S_i . h_i (every
// bond has exactly one colour-1 end, E = -S), M = sum over both colours and,
// with a.bonds, the bond sums into the item's partials.  HALO = halo entries
// per thread (2*(L/2) <= HALO*kBlock).  FULL: every lattice of the launch
// fills its tile exactly (TY * L/2 = SPT * kBlock), so no column needs a
// guard.
// ---------------------------------------------------------------------------
// Elements of one plane buffer of the tiled kernel: TY * L/2 <= SPT * kBlock
// tile sites and 2 * L/2 <= HALO * kBlock halo sites.
template <int SPT, int HALO>
constexpr int kTileBufElems = (SPT + HALO) * kBlock;

// The Metropolis half-sweep interleaves its columns' draws, which left to
// itself the compiler pays for with registers (194 at five columns per
// thread, two wavefronts per SIMD); capped, three wavefronts fit.
constexpr int tile_min_waves(int kind, bool meas, int spt) { return (kind == kMetro && !meas && spt <= 5) ? 3 : 1; }

template <int KIND, bool MEAS, int SPT, int HALO, bool FULL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(tile_min_waves(KIND, MEAS, SPT))))
void k_tile_f32(SweepArgs a)
{
    extern __shared__ f2 lds[];
    const int tid = threadIdx.x;
    const uint32_t t_sweep = a.ctl->t;

    for (int v = blockIdx.x; v < a.total_items; v += gridDim.x) {
        const int w = xcd_item(v, a.total_items);
        const int li = uni(find_lattice(a.lats, a.n_lat, w));
        const LatDev d = load_lat_uniform(a.lats + li);
        const int L = d.L, half = d.half, TY = d.TY;
        const int wl = w - d.item_base;
        const int slot = wl / d.items_per_slot;
        const int rem = wl - slot * d.items_per_slot;
        const int ty = rem % d.ny, tz = rem / d.ny;
        const int y0 = ty * TY, z0 = tz * d.TZ;
        const int k = uni(a.pos[d.pos_base + slot]);
        const float beta = __builtin_bit_cast(float, uni(__builtin_bit_cast(int, (float)a.beta[d.pos_base + k])));
        // Re-decision band: the float32 dE (|dE| <= 12) errs by about 2e-6,
        // so p = exp(-beta dE) <= 1 errs by up to beta * 2e-6; the band keeps
        // an 8x margin over that and never drops below 1e-5.
        const float band = __builtin_fmaxf(1e-5f, 1.6e-5f * beta);
        // exp(-beta dE) = 2^(dE * nbl2e)
        const float nbl2e = -beta * 1.44269504088896341f;
        const uint32_t plane_b = (uint32_t)L * (uint32_t)half * 4u;  // bytes per plane
        const float *angs = (const float *)a.ang + d.base + (int64_t)slot * d.N;
        const __amdgpu_buffer_rsrc_t rown = colour_rsrc(angs + (int64_t)a.colour * (d.N / 2), d.N / 2);
        const __amdgpu_buffer_rsrc_t roth = colour_rsrc(angs + (int64_t)(a.colour ^ 1) * (d.N / 2), d.N / 2);
        const __amdgpu_buffer_rsrc_t rnull = colour_rsrc(angs, 0);
        const int nsite = TY * half;
        // the second plane buffer at a compile-time offset (a bound on
        // (TY + 2) * L/2 for every lattice of the launch), so that the
        // alternating steps address it through immediate LDS offsets
        f2 *buf0 = lds;
        f2 *buf1 = lds + kTileBufElems<SPT, HALO>;
        const uint32_t LL = (uint32_t)L * (uint32_t)L;
        const uint32_t c2 = ((uint32_t)d.lat << 16) | (uint32_t)k;
        const uint32_t c3 = (kPhaseMetro << 24) | (uint32_t)a.substep;

        uint32_t voff[SPT], ibase[SPT];
        int lc[SPT], lxm[SPT], lxp[SPT], ypar[SPT];
        bool ok[SPT];
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
            const int f = tid + s * kBlock;
            ok[s] = f < nsite;
            const int fl = ok[s] ? f : 0;
            const int yl = fl / half;
            const int j = fl - yl * half;
            const int y = y0 + yl;
            voff[s] = (uint32_t)(y * half + j) * 4u;
            lc[s] = (yl + 1) * half + j;
            lxm[s] = (yl + 1) * half + ((j == 0) ? half - 1 : j - 1);
            lxp[s] = (yl + 1) * half + ((j + 1 == half) ? 0 : j + 1);
            ypar[s] = (a.colour + y) & 1;
            ibase[s] = 2u * (uint32_t)j + (uint32_t)L * (uint32_t)y;
        }
        const int ym = (y0 == 0) ? L - 1 : y0 - 1;
        const int yp = (y0 + TY == L) ? 0 : y0 + TY;
        uint32_t hvoff[HALO];
        int hl[HALO];
        bool hok[HALO];
#pragma unroll
        for (int h = 0; h < HALO; ++h) {
            const int e = tid + h * kBlock;
            hok[h] = e < 2 * half;
            const int ee = hok[h] ? e : 0;
            const int r = ee >= half;
            const int jj = ee - r * half;
            hvoff[h] = (uint32_t)((r ? yp : ym) * half + jj) * 4u;
            hl[h] = (r ? (TY + 1) : 0) * half + jj;
        }

        // Prologue.  Converted: other colour at z0-1, z0, z0+1; raw (in flight
        // one plane ahead of use): other colour at z0+2, ours at z0+1, halo
        // at z0+1.  Plane z0 of the other colour (tile and halo) goes to the
        // LDS buffer of the first step, plane z0-1 (tile columns only) to the
        // other one: a column's z-1 neighbour is read back from there, and
        // only its z+1 neighbour is held in registers.
        auto wrapz = [L](int z) { return z >= L ? z - L : z; };
        const int zm1 = (z0 == 0) ? L - 1 : z0 - 1;
        f2 ocp[SPT];
        float cur[SPT];
        float a_o[SPT], a_c[SPT], a_h[HALO], b_o[SPT], b_c[SPT], b_h[HALO];
        int lx_even[SPT], lx_odd[SPT];  // LDS index of the x-neighbour on even / odd steps
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
            const bool p_even = ((ypar[s] + z0) & 1) != 0;
            lx_even[s] = p_even ? lxp[s] : lxm[s];
            lx_odd[s] = p_even ? lxm[s] : lxp[s];
            const f2 om = sincos_turns(bload(roth, voff[s], (uint32_t)zm1 * plane_b));
            const f2 o0 = sincos_turns(bload(roth, voff[s], (uint32_t)z0 * plane_b));
            ocp[s] = sincos_turns(bload(roth, voff[s], (uint32_t)wrapz(z0 + 1) * plane_b));
            cur[s] = bload(rown, voff[s], (uint32_t)z0 * plane_b);
            a_o[s] = bload(roth, voff[s], (uint32_t)wrapz(z0 + 2) * plane_b);
            a_c[s] = bload(rown, voff[s], (uint32_t)wrapz(z0 + 1) * plane_b);
            buf0[lc[s]] = o0;
            buf1[lc[s]] = om;
        }
#pragma unroll
        for (int h = 0; h < HALO; ++h) {
            const f2 v = sincos_turns(bload(roth, hvoff[h], (uint32_t)z0 * plane_b));
            if (hok[h]) buf0[hl[h]] = v;
            a_h[h] = bload(roth, hvoff[h], (uint32_t)wrapz(z0 + 1) * plane_b);
        }
        lds_barrier();

        double acc[kPartials];
#pragma unroll
        for (int q = 0; q < kPartials; ++q) acc[q] = 0.0;
        uint32_t nacc_w = 0;  // accepted moves of this wavefront in this item (wave-uniform)
        uint32_t kept0[SPT] = {}, kept1[SPT] = {};  // Metropolis: words 2, 3 of the pair's Philox block

        // One plane.  pre_* were loaded one step ago and are consumed at the
        // end of this step; nxt_* are issued now and consumed next step.  The
        // loop below alternates the two register sets (and the two LDS
        // buffers) so that no in-flight load is ever copied between registers,
        // which would force the wait early.  With FULL the per-column guards
        // drop out and the compiler may interleave the columns.
        auto step = [&](const int zz, const f2 *bc, f2 *bn, const int (&lx)[SPT],
                        float (&pre_o)[SPT], float (&pre_c)[SPT], float (&pre_h)[HALO], float (&nxt_o)[SPT],
                        float (&nxt_c)[SPT], float (&nxt_h)[HALO]) __attribute__((always_inline)) {
            const int z = z0 + zz;
            const uint32_t sz = (uint32_t)z * plane_b;
            {
                // planes past the chunk (needed: other colour up to z0+TZ,
                // ours and the halo up to z0+TZ-1) are read through an empty
                // descriptor: the load returns 0 and moves no data
                const bool need = zz + 3 <= d.TZ;
                const __amdgpu_buffer_rsrc_t ro = need ? roth : rnull;
                const __amdgpu_buffer_rsrc_t rc = need ? rown : rnull;
                const uint32_t s3 = (uint32_t)wrapz(wrapz(z + 1) + 2) * plane_b;
                const uint32_t s2 = (uint32_t)wrapz(wrapz(z + 1) + 1) * plane_b;
#pragma unroll
                for (int s = 0; s < SPT; ++s) {
                    nxt_o[s] = bload(ro, voff[s], s3);
                    nxt_c[s] = bload(rc, voff[s], s2);
                }
#pragma unroll
                for (int h = 0; h < HALO; ++h) nxt_h[h] = bload(ro, hvoff[h], s2);
            }

            if constexpr (KIND == kMetro && !MEAS) {
                // Metropolis: first the draws of every column (independent
                // Philox chains the compiler may interleave), then the
                // decisions column by column, then, rarely, the queue of
                // near-threshold decisions for the float64 re-decision.
                // One Philox block per pair of planes (2m, 2m+1) of a column:
                // drawn at the even plane (or at the tile's first plane when
                // that is odd), its last two words kept for the odd plane.
                uint32_t w0[SPT] = {}, w1[SPT] = {};
                if ((z & 1) == 0 || zz == 0) {
                    const int zb = z & ~1;
#pragma unroll
                    for (int s = 0; s < SPT; ++s) {
                        if (!FULL && !ok[s]) continue;
                        const uint32_t pb = (uint32_t)((ypar[s] + zb) & 1);
                        const uint32_t ib = ibase[s] + pb + LL * (uint32_t)zb;
                        const u32x4 r = philox4x32_10(ib, t_sweep, c2, c3, a.k0, a.k1);
                        w0[s] = (z & 1) ? r.z : r.x;
                        w1[s] = (z & 1) ? r.w : r.y;
                        kept0[s] = r.z;
                        kept1[s] = r.w;
                    }
                } else {
#pragma unroll
                    for (int s = 0; s < SPT; ++s) {
                        w0[s] = kept0[s];
                        w1[s] = kept1[s];
                    }
                }
                // One column's decision: the field from the staged neighbours,
                // the proposal, dE and p = exp(-beta dE) (also used, rarely,
                // to queue a decision: the same arithmetic again, so the same
                // values).
                struct Eval {
                    float prop, u1, pa;
                };
                auto eval = [&](auto win_tag, const int s) __attribute__((always_inline)) {
                    const f2 n1 = bc[lc[s] - half];
                    const f2 n2 = bc[lc[s] + half];
                    const f2 n3 = bc[lc[s]];
                    const f2 n4 = bc[lx[s]];
                    // plane z-1 of this column: still in the other buffer, which
                    // this lane overwrites with plane z+1 only at the end of the step
                    const f2 om = bn[lc[s]];
                    const float hx = ((om.c + ocp[s].c) + (n1.c + n2.c)) + (n3.c + n4.c);
                    const float hy = ((om.s + ocp[s].s) + (n1.s + n2.s)) + (n3.s + n4.s);
                    Eval v;
                    // uniform proposal (exact in turns) or theta + w (u0 - 1/2)
                    v.prop = unit24f(w0[s]);
                    if constexpr (decltype(win_tag)::value)
                        v.prop = frac_turn(__builtin_fmaf(a.window_t, v.prop - 0.5f, cur[s]));
                    v.u1 = unit24f(w1[s]);
                    const f2 so = sincos_turns(cur[s]);
                    const f2 sn = sincos_turns(v.prop);
                    // the multiply-add written out: every instantiation (and the
                    // queueing path's recomputation) forms the same dE
                    const float dE = __builtin_fmaf(so.c - sn.c, hx, (so.s - sn.s) * hy);
                    v.pa = __builtin_amdgcn_exp2f(dE * nbl2e);
                    return v;
                };
                // smallest |u - p| over the columns: a decision within the
                // band anywhere in the wave sends it down the queueing path
                float closest = 1.0f;
                auto column = [&](auto win_tag, const int s) __attribute__((always_inline)) {
                    const Eval v = eval(win_tag, s);
                    const bool acc = v.u1 < v.pa;
                    bstore(acc ? v.prop : cur[s], rown, voff[s], sz);
                    nacc_w += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(acc));
                    closest = __builtin_fminf(closest, __builtin_fabsf(v.u1 - v.pa));
                };
                // near-threshold decisions of the step, queued for the float64
                // re-decision, which draws the proposal and the uniform again
                // from the same counter; it needs the old angle and the float32
                // decision
                auto queue = [&](auto win_tag) __attribute__((always_inline)) {
#pragma unroll
                    for (int s = 0; s < SPT; ++s) {
                        if (!FULL && !ok[s]) continue;
                        const Eval v = eval(win_tag, s);
                        if (!(__builtin_fabsf(v.u1 - v.pa) < band)) continue;
                        const uint32_t idx = atomicAdd(&a.rq->count, 1u);
                        if (idx < a.rq->capacity) {
                            RecheckEntry e;
                            e.li = li;
                            e.slot = slot;
                            e.q = ((sz + voff[s]) >> 2) | ((v.u1 < v.pa ? 1u : 0u) << 31);
                            e.cur = cur[s];
                            a.rq->entries[idx] = e;
                        } else {
                            atomicAdd(&a.rq->overflow, 1u);
                        }
                    }
                };
                if (a.window_t > 0.0f) {
#pragma unroll
                    for (int s = 0; s < SPT; ++s)
                        if (FULL || ok[s]) column(std::true_type{}, s);
                    if (a.recheck && __builtin_amdgcn_ballot_w64(closest < band) != 0) queue(std::true_type{});
                } else {
#pragma unroll
                    for (int s = 0; s < SPT; ++s)
                        if (FULL || ok[s]) column(std::false_type{}, s);
                    if (a.recheck && __builtin_amdgcn_ballot_w64(closest < band) != 0) queue(std::false_type{});
                }
            } else {
            // Columns past the tile (ok false) are skipped: with TY * L/2 not a
            // multiple of the block size whole wavefronts have nothing to do
            // in the last column, and the branch lets them skip it.
#pragma unroll
            for (int s = 0; s < SPT; ++s) {
                if (!FULL && !ok[s]) continue;
                const f2 n1 = bc[lc[s] - half];
                const f2 n2 = bc[lc[s] + half];
                const f2 n3 = bc[lc[s]];
                const f2 n4 = bc[lx[s]];
                // plane z-1 of this column: still in the other buffer, which
                // this lane overwrites with plane z+1 only at the end of the step
                const f2 om = bn[lc[s]];
                const float hx = ((om.c + ocp[s].c) + (n1.c + n2.c)) + (n3.c + n4.c);
                const float hy = ((om.s + ocp[s].s) + (n1.s + n2.s)) + (n3.s + n4.s);
                float nv = cur[s];
                if constexpr (KIND == kOver) {
                    nv = overrelax_turns(cur[s], hx, hy);
                } else if constexpr (KIND == kMetro) {
                    uint32_t w0, w1;
                    if ((z & 1) == 0 || zz == 0) {
                        const int zb = z & ~1;
                        const uint32_t pb = (uint32_t)((ypar[s] + zb) & 1);
                        const uint32_t ib = ibase[s] + pb + LL * (uint32_t)zb;
                        const u32x4 r = philox4x32_10(ib, t_sweep, c2, c3, a.k0, a.k1);
                        w0 = (z & 1) ? r.z : r.x;
                        w1 = (z & 1) ? r.w : r.y;
                        kept0[s] = r.z;
                        kept1[s] = r.w;
                    } else {
                        w0 = kept0[s];
                        w1 = kept1[s];
                    }
                    const float u0 = unit24f(w0), u1 = unit24f(w1);
                    // uniform proposal (exact in turns) or theta + w (u0 - 1/2)
                    const float prop = a.window_t > 0.0f
                                           ? frac_turn(__builtin_fmaf(a.window_t, u0 - 0.5f, cur[s]))
                                           : u0;
                    const f2 so = sincos_turns(cur[s]);
                    const f2 sn = sincos_turns(prop);
                    // the multiply-add written out: every instantiation (and the
                    // queueing path's recomputation) forms the same dE
                    const float dE = __builtin_fmaf(so.c - sn.c, hx, (so.s - sn.s) * hy);
                    const float pa = __builtin_amdgcn_exp2f(dE * nbl2e);
                    const bool acc = u1 < pa;
                    if (a.recheck && __builtin_fabsf(u1 - pa) < band) {
                        const uint32_t idx = atomicAdd(&a.rq->count, 1u);
                        if (idx < a.rq->capacity) {
                            RecheckEntry e;
                            e.li = li;
                            e.slot = slot;
                            e.q = ((sz + voff[s]) >> 2) | ((acc ? 1u : 0u) << 31);
                            e.cur = cur[s];
                            a.rq->entries[idx] = e;
                        } else {
                            atomicAdd(&a.rq->overflow, 1u);
                        }
                    }
                    nv = acc ? prop : cur[s];
                    nacc_w += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(acc));
                }
                if constexpr (MEAS || KIND == kMeas) {
                    const f2 sc = sincos_turns(nv);
                    // x neighbours: same j is +x when x is even (p = 0), -x otherwise
                    const bool podd = ((ypar[s] + z) & 1) != 0;
                    const f2 xp = podd ? n4 : n3, xm = podd ? n3 : n4;
                    const float nc[6] = {xp.c, xm.c, n2.c, n1.c, ocp[s].c, om.c};
                    const float ns[6] = {xp.s, xm.s, n2.s, n1.s, ocp[s].s, om.s};
                    // n3 is the other-colour site with the same storage index
                    measure_site(acc, a.bonds != 0, sc.c, sc.s, n3.c, n3.s, hx, hy, nc, ns);
                }
                if constexpr (KIND != kMeas) bstore(nv, rown, voff[s], sz);
            }
            }

            // Plane z+1 into the other LDS buffer; plane z+2 into registers.
#pragma unroll
            for (int s = 0; s < SPT; ++s) {
                if (!FULL && !ok[s]) continue;
                bn[lc[s]] = ocp[s];
                ocp[s] = sincos_turns(pre_o[s]);
                cur[s] = pre_c[s];
            }
#pragma unroll
            for (int h = 0; h < HALO; ++h)
                if (hok[h]) bn[hl[h]] = sincos_turns(pre_h[h]);
            lds_barrier();
        };

        for (int zz = 0; zz < d.TZ; zz += 2) {
            step(zz, buf0, buf1, lx_even, a_o, a_c, a_h, b_o, b_c, b_h);
            if (zz + 1 < d.TZ) step(zz + 1, buf1, buf0, lx_odd, b_o, b_c, b_h, a_o, a_c, a_h);
        }

        if constexpr (KIND == kMetro)
            block_add_accepts((threadIdx.x & 63) == 0 ? (unsigned long long)nacc_w : 0ull, a.macc + d.pos_base + k);
        if constexpr (MEAS || KIND == kMeas)
            block_store_partials(acc, a.partials + kPartials * (int64_t)w, a.bonds ? kPartials : kPartialsNoBonds);
    }
}

// ---------------------------------------------------------------------------
// Plain FP64 half-sweep: one thread per site of the updated colour, all six
// neighbours read straight from global memory, every transcendental in
// double.  A work item is (lattice, slot, block of kBlock sites).
// ---------------------------------------------------------------------------
template <int KIND, bool MEAS>
__global__ __launch_bounds__(kBlock) void k_plain_f64(SweepArgs a)
{
    const double twopi = 6.283185307179586476925286766559;
    const int w = blockIdx.x;
    const int li = find_lattice(a.lats, a.n_lat, w);
    const LatDev d = a.lats[li];
    const int L = d.L, half = d.half;
    const int wl = w - d.item_base;
    const int slot = wl / d.items_per_slot;
    const int b = wl - slot * d.items_per_slot;
    const int k = a.pos[d.pos_base + slot];
    const double beta = a.beta[d.pos_base + k];
    const int64_t plane = (int64_t)L * half;
    double *angs = (double *)a.ang + d.base + (int64_t)slot * d.N;
    double *own = angs + (int64_t)a.colour * (d.N / 2);
    const double *oth = angs + (int64_t)(a.colour ^ 1) * (d.N / 2);

    const int64_t q = (int64_t)b * kBlock + threadIdx.x;
    const bool ok = q < d.N / 2;
    double acc[kPartials];
#pragma unroll
    for (int m = 0; m < kPartials; ++m) acc[m] = 0.0;
    unsigned long long nacc = 0;
    if (ok) {
        const int j = (int)(q % half);
        const int y = (int)((q / half) % L);
        const int z = (int)(q / plane);
        const int p = (a.colour + y + z) & 1;
        const int ym = (y == 0) ? L - 1 : y - 1, yp = (y + 1 == L) ? 0 : y + 1;
        const int zm = (z == 0) ? L - 1 : z - 1, zp = (z + 1 == L) ? 0 : z + 1;
        const int jx = p ? ((j + 1 == half) ? 0 : j + 1) : ((j == 0) ? half - 1 : j - 1);
        const int64_t zo = (int64_t)z * plane;
        const int64_t nb[6] = {zo + (int64_t)y * half + j,  zo + (int64_t)y * half + jx,
                               zo + (int64_t)ym * half + j, zo + (int64_t)yp * half + j,
                               (int64_t)zm * plane + (int64_t)y * half + j,
                               (int64_t)zp * plane + (int64_t)y * half + j};
        double hx = 0.0, hy = 0.0;
        for (int n = 0; n < 6; ++n) {
            double sn, cn;
            sincos(oth[nb[n]], &sn, &cn);
            hx += cn;
            hy += sn;
        }
        const double th = own[q];
        double nv = th;
        if constexpr (KIND == kOver) {
            if (hx != 0.0 || hy != 0.0) {
                double v = 2.0 * atan2(hy, hx) - th;
                v = fmod(v, twopi);
                if (v < 0.0) v += twopi;
                if (v >= twopi) v = 0.0;
                nv = v;
            }
        } else if constexpr (KIND == kMetro) {
            // the Philox block of the plane pair (z - z mod 2, z - z mod 2 + 1):
            // counter word 0 is the even-plane site of this column, whose x
            // parity is the opposite of ours on an odd plane
            const uint32_t zb = (uint32_t)(z & ~1);
            const uint32_t pb = (uint32_t)p ^ (uint32_t)(z & 1);
            const uint32_t ib = 2u * (uint32_t)j + pb + (uint32_t)L * ((uint32_t)y + (uint32_t)L * zb);
            const u32x4 r = philox4x32_10(ib, a.ctl->t, ((uint32_t)d.lat << 16) | (uint32_t)k,
                                          (kPhaseMetro << 24) | (uint32_t)a.substep, a.k0, a.k1);
            const uint32_t w0 = (z & 1) ? r.z : r.x, w1 = (z & 1) ? r.w : r.y;
            double prop = twopi * unit24d(w0);
            if (a.window > 0.0) {
                prop = fmod(th + a.window * (unit24d(w0) - 0.5), twopi);
                if (prop < 0.0) prop += twopi;
                if (prop >= twopi) prop = 0.0;
            }
            const double u = unit24d(w1);
            double so, co, sp, cp;
            sincos(th, &so, &co);
            sincos(prop, &sp, &cp);
            const double dE = (co - cp) * hx + (so - sp) * hy;
            if (u < exp(-beta * dE)) {
                nv = prop;
                nacc = 1;
            }
        }
        if constexpr (MEAS || KIND == kMeas) {
            double s1, c1, s0, c0;
            sincos(nv, &s1, &c1);
            sincos(oth[q], &s0, &c0);
            // neighbour order (+x, -x, +y, -y, +z, -z); nb[0] (same j) is +x when p = 0
            const int64_t dir[6] = {p ? nb[1] : nb[0], p ? nb[0] : nb[1], nb[3], nb[2], nb[5], nb[4]};
            double nc[6] = {}, ns[6] = {};
            if (a.bonds)
                for (int m = 0; m < 6; ++m) sincos(oth[dir[m]], &ns[m], &nc[m]);
            measure_site(acc, a.bonds != 0, c1, s1, c0, s0, hx, hy, nc, ns);
        }
        if constexpr (KIND != kMeas) own[q] = nv;
    }
    if constexpr (KIND == kMetro) block_add_accepts(nacc, a.macc + d.pos_base + k);
    if constexpr (MEAS || KIND == kMeas)
        block_store_partials(acc, a.partials + kPartials * (int64_t)w, a.bonds ? kPartials : kPartialsNoBonds);
}

// ---------------------------------------------------------------------------
// Random or ordered start.  One thread per (lattice, slot, site), natural
// site order; slot r starts at beta-position r.
// ---------------------------------------------------------------------------
__global__ void k_init(int fp32, int ordered, const LatDev *lats, int n_lat, int64_t total,
                       void *ang, uint32_t k0, uint32_t k1)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        int li = 0;
        int64_t start = 0;
        while (li + 1 < n_lat && g >= start + (int64_t)lats[li].R * lats[li].N) {
            start += (int64_t)lats[li].R * lats[li].N;
            ++li;
        }
        const LatDev d = lats[li];
        const int64_t local = g - start;
        const int slot = (int)(local / d.N);
        const int64_t i = local - (int64_t)slot * d.N;
        const int L = d.L;
        const int x = (int)(i % L), y = (int)((i / L) % L), z = (int)(i / ((int64_t)L * L));
        const int c = (x + y + z) & 1;
        const int64_t dst = d.base + (int64_t)slot * d.N + (int64_t)c * (d.N / 2) +
                            ((int64_t)z * L + y) * d.half + (x >> 1);
        double u = 0.0;
        if (!ordered) {
            const u32x4 r = philox4x32_10((uint32_t)i, 0u, ((uint32_t)d.lat << 16) | (uint32_t)slot,
                                          kPhaseInit << 24, k0, k1);
            u = unit24d(r.x);
        }
        if (fp32)
            ((float *)ang)[dst] = (float)u;
        else
            ((double *)ang)[dst] = 6.283185307179586476925286766559 * u;
    }
}

// ---------------------------------------------------------------------------
// Per-lattice finalisation: sum the measurement partials of each slot in a
// fixed order, publish observables by beta-position, then (optionally) one
// even/odd parallel-tempering exchange step, Eq. (3), on the slot<->position
// permutation.  One workgroup per lattice.
// ---------------------------------------------------------------------------
__global__ void k_finalize(const LatDev *lats, const double *partials, const double *beta,
                           int32_t *pos, int32_t *slot_of, double *E_slot, double *obs,
                           double *bonds, int use_ring, int64_t ring_stride, int64_t bond_stride,
                           int do_sum, int do_exchange, unsigned long long *sacc, Ctl *ctl,
                           uint32_t k0, uint32_t k1, int *bad)
{
    const LatDev d = lats[blockIdx.x];
    const int pb = d.pos_base;
    if (do_sum) {
        // one wavefront per slot: lanes stride over the slot's items, then a
        // fixed butterfly; the order depends only on the item layout
        double *out = obs, *bout = bonds;
        if (out && use_ring) out += (int64_t)ctl->ring * ring_stride;
        if (bout && use_ring) bout += (int64_t)ctl->ring * bond_stride;
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
        for (int r = wv; r < d.R; r += nw) {
            const double *pp = partials + kPartials * ((int64_t)d.item_base + (int64_t)r * d.items_per_slot);
            // without a bond ring only S, Mx, My were filled and are summed
            const int nq = bout ? kPartials : kPartialsNoBonds;
            double v[kPartials];
#pragma unroll
            for (int q = 0; q < kPartials; ++q) v[q] = 0.0;
            for (int it = lane; it < d.items_per_slot; it += 64)
#pragma unroll
                for (int q = 0; q < kPartials; ++q)
                    if (q < nq) v[q] += pp[kPartials * it + q];
#pragma unroll
            for (int q = 0; q < kPartials; ++q)
                if (q < nq) v[q] = wave_sum(v[q]);
            if (lane == 0) {
                const double E = -v[0], mx = v[1], my = v[2];
                E_slot[pb + r] = E;
                if (!isfinite(E) || !isfinite(mx) || !isfinite(my)) atomicOr(bad, 1);
                const int kk = pos[pb + r];
                if (out) {
                    const double n = (double)d.N;
                    const double m = sqrt(mx * mx + my * my) / n;
                    double *o = out + 5 * (int64_t)(pb + kk);
                    o[0] = E;
                    o[1] = E / n;
                    o[2] = m;
                    o[3] = m * m;
                    o[4] = (m * m) * (m * m);
                }
                if (bout) {
                    double *o = bout + 6 * (int64_t)(pb + kk);
#pragma unroll
                    for (int q = 0; q < 6; ++q) o[q] = v[3 + q];
                }
            }
        }
        __syncthreads();
    }
    if (do_exchange) {
        const uint32_t tau = ctl->tau;
        for (int kk = (int)(tau & 1u) + 2 * threadIdx.x; kk + 1 < d.R; kk += 2 * blockDim.x) {
            const int s0 = slot_of[pb + kk], s1 = slot_of[pb + kk + 1];
            const double delta = (beta[pb + kk] - beta[pb + kk + 1]) * (E_slot[pb + s0] - E_slot[pb + s1]);
            const u32x4 r = philox4x32_10((uint32_t)kk, tau, (uint32_t)d.lat << 16, kPhaseExch << 24,
                                          k0, k1);
            if (unit24d(r.x) < exp(delta)) {
                slot_of[pb + kk] = s1;
                slot_of[pb + kk + 1] = s0;
                pos[pb + s0] = kk + 1;
                pos[pb + s1] = kk;
                sacc[pb + kk] += 1ull;
            }
        }
    }
}

// Gather angles of chosen sites (natural index) of one slot, as radians.
__global__ void k_gather(int fp32, const void *ang, int64_t slot_base, int L, int64_t n,
                         const int64_t *sites, double *out)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int64_t i = sites[g];
    const int64_t N = (int64_t)L * L * L;
    const int x = (int)(i % L), y = (int)((i / L) % L), z = (int)(i / ((int64_t)L * L));
    const int c = (x + y + z) & 1;
    const int64_t src = slot_base + (int64_t)c * (N / 2) + ((int64_t)z * L + y) * (L / 2) + (x >> 1);
    out[g] = fp32 ? (double)((const float *)ang)[src] * 6.283185307179586476925286766559
                  : ((const double *)ang)[src];
}

__global__ void k_tick(Ctl *ctl, uint32_t dt, uint32_t dtau, uint32_t dring, int set_ring)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->t += dt;
        ctl->tau += dtau;
        if (set_ring)
            ctl->ring = dring;
        else
            ctl->ring += dring;
    }
}

// ---------------------------------------------------------------------------
// Launchers.  With per_cu set, nothing is launched: *per_cu receives how many
// workgroups of the selected kernel fit on one CU at the given LDS size (the
// resident capacity that persistent launches are sized to).
// ---------------------------------------------------------------------------
template <int KIND, bool MEAS, int HALO, bool FULL>
static hipError_t launch_tile_spt(int spt, int grid, size_t lds, const SweepArgs &a, hipStream_t s,
                                  int *per_cu)
{
    switch (spt) {
    case 1: return launch_or_query(k_tile_f32<KIND, MEAS, 1, HALO, FULL>, grid, lds, a, s, per_cu);
    case 2: return launch_or_query(k_tile_f32<KIND, MEAS, 2, HALO, FULL>, grid, lds, a, s, per_cu);
    case 3: return launch_or_query(k_tile_f32<KIND, MEAS, 3, HALO, FULL>, grid, lds, a, s, per_cu);
    case 4: return launch_or_query(k_tile_f32<KIND, MEAS, 4, HALO, FULL>, grid, lds, a, s, per_cu);
    case 5: return launch_or_query(k_tile_f32<KIND, MEAS, 5, HALO, FULL>, grid, lds, a, s, per_cu);
    case 6: return launch_or_query(k_tile_f32<KIND, MEAS, 6, HALO, FULL>, grid, lds, a, s, per_cu);
    case 8: return launch_or_query(k_tile_f32<KIND, MEAS, 8, HALO, FULL>, grid, lds, a, s, per_cu);
    default: return hipErrorInvalidValue;
    }
}

template <int HALO>
static hipError_t launch_tile_halo(int kind, bool fuse_measure, bool full, int spt, int grid, size_t lds,
                                   const SweepArgs &a, hipStream_t s, int *per_cu)
{
    // the unguarded (FULL) variant exists for the plain Metropolis half-sweep
    if (kind == kMetro && !fuse_measure && full)
        return launch_tile_spt<kMetro, false, HALO, true>(spt, grid, lds, a, s, per_cu);
    if (kind == kMetro)
        return fuse_measure ? launch_tile_spt<kMetro, true, HALO, false>(spt, grid, lds, a, s, per_cu)
                            : launch_tile_spt<kMetro, false, HALO, false>(spt, grid, lds, a, s, per_cu);
    if (kind == kOver)
        return fuse_measure ? launch_tile_spt<kOver, true, HALO, false>(spt, grid, lds, a, s, per_cu)
                            : launch_tile_spt<kOver, false, HALO, false>(spt, grid, lds, a, s, per_cu);
    return launch_tile_spt<kMeas, false, HALO, false>(spt, grid, lds, a, s, per_cu);
}

hipError_t launch_tile_f32(int kind, bool fuse_measure, bool full, int spt, int halo, int grid, size_t lds,
                           const SweepArgs &a, hipStream_t s, int *per_cu)
{
    if (halo == 1) return launch_tile_halo<1>(kind, fuse_measure, full, spt, grid, lds, a, s, per_cu);
    if (halo == 4) return launch_tile_halo<4>(kind, fuse_measure, full, spt, grid, lds, a, s, per_cu);
    return hipErrorInvalidValue;
}

hipError_t launch_or2_f32(bool fuse_measure, bool lead, int spt, int grid, size_t lds, const SweepArgs &a,
                          hipStream_t s, int *per_cu)
{
    if (!fuse_measure) return launch_or2_plain(lead, spt, grid, lds, a, s, per_cu);
    return a.bonds ? launch_or2_lead<kOr2MeasureBonds>(lead, spt, grid, lds, a, s, per_cu)
                   : launch_or2_lead<kOr2Measure>(lead, spt, grid, lds, a, s, per_cu);
}

hipError_t launch_recheck(const SweepArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_recheck, dim3(16), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_plain_f64(int kind, bool fuse_measure, int grid, const SweepArgs &a, hipStream_t s)
{
    if (kind == kMetro && fuse_measure)
        hipLaunchKernelGGL((k_plain_f64<kMetro, true>), dim3(grid), dim3(kBlock), 0, s, a);
    else if (kind == kMetro)
        hipLaunchKernelGGL((k_plain_f64<kMetro, false>), dim3(grid), dim3(kBlock), 0, s, a);
    else if (kind == kOver && fuse_measure)
        hipLaunchKernelGGL((k_plain_f64<kOver, true>), dim3(grid), dim3(kBlock), 0, s, a);
    else if (kind == kOver)
        hipLaunchKernelGGL((k_plain_f64<kOver, false>), dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_plain_f64<kMeas, false>), dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_init(bool fp32, bool ordered, const LatDev *lats, int n_lat, int64_t total,
                       void *ang, uint32_t k0, uint32_t k1, hipStream_t s)
{
    int64_t blocks = (total + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(kBlock), 0, s, (int)fp32, (int)ordered,
                       lats, n_lat, total, ang, k0, k1);
    return hipGetLastError();
}

hipError_t launch_finalize(const LatDev *lats, int n_lat, int max_R, const double *partials,
                           const double *beta, int32_t *pos, int32_t *slot_of, double *E_slot,
                           double *obs, double *bonds, int use_ring, int64_t ring_stride,
                           int64_t bond_stride, int do_sum, int do_exchange,
                           unsigned long long *sacc, Ctl *ctl, uint32_t k0, uint32_t k1, int *bad,
                           hipStream_t s)
{
    int threads = 64;
    while (threads < 64 * max_R && threads < 1024) threads *= 2;
    hipLaunchKernelGGL(k_finalize, dim3(n_lat), dim3(threads), 0, s, lats, partials, beta, pos,
                       slot_of, E_slot, obs, bonds, use_ring, ring_stride, bond_stride, do_sum,
                       do_exchange, sacc, ctl, k0, k1, bad);
    return hipGetLastError();
}

hipError_t launch_gather(bool fp32, const void *ang, int64_t slot_base, int L, int64_t n,
                         const int64_t *sites, double *out, hipStream_t s)
{
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks), dim3(kBlock), 0, s, (int)fp32, ang, slot_base, L, n,
                       sites, out);
    return hipGetLastError();
}

hipError_t launch_tick(Ctl *ctl, uint32_t dt, uint32_t dtau, uint32_t dring, int set_ring,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, ctl, dt, dtau, dring, set_ring);
    return hipGetLastError();
}

}  // namespace xy
