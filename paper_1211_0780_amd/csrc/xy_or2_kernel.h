// The fused over-relaxation substep kernel template and its launch
// dispatch, shared by two translation units: the plain substep is
// instantiated in xy_or2.hip, built with the max-ILP instruction scheduler,
// the measuring variants in xy_kernels.hip with the default one (under
// max-ILP they need more registers, and those at two, four and five
// columns per thread lose a wavefront per SIMD).
#pragma once

#include <hip/hip_runtime.h>

#include "xy_device.h"
#include "xy_kernels.h"
#include "xy_kernel_common.h"

namespace xy {

// ---------------------------------------------------------------------------
// Fused over-relaxation substep: colour 0 then colour 1 of one substep in a
// single streaming pass, reading the old configuration from `ang` and
// writing the new one to `ang_dst` (ping-pong buffers, so no tile ever reads
// a value another tile has already replaced).
//
// At step z the kernel updates colour 0 at plane z ("a") and colour 1 at
// plane z-1 ("b"); b needs colour 0 already updated at planes z-2, z-1, z,
// which a has produced by then, so the pass is the sequential order of the
// two half-sweeps.  Colour 0 is also updated, redundantly and without being
// stored, on the halo rows y0-1, y0+TY and the halo planes z0-1, z0+TZ: the
// same deterministic arithmetic on the same inputs as the tile that owns
// them, so colour 1 at the tile edge sees exactly the values that tile
// writes.  That needs the old colour 1 two rows and two planes out.
//
// Per thread: SPT tile columns ("T", rows y0..y0+TY-1), one halo column
// ("H", rows y0-1 or y0+TY) and one outer column ("O", rows y0-2 or
// y0+TY+1, old colour 1 only); H and O need 2*(L/2) <= kBlock, so L <= 256.
// LDS: P1 = old colour 1 (cos, sin) of plane z on rows y0-2..y0+TY+1 and
// P0 = new colour 0 of plane z on rows y0-1..y0+TY, both double-buffered.
// b reads new colour 0 of plane z-2 only at its own column: the plain
// substep carries that value over in registers from the previous step's
// read of plane z-1 (two P0 buffers, alternating with the step parity, whose
// addresses need no per-step arithmetic: 8 % fewer VALU instructions, 2 %
// less time); the measuring variants, already at their register cap, read
// it from a third P0 buffer in rotation.
// Loads run two planes ahead in alternating register sets, as in
// k_tile_f32.  MEAS (kOr2Measure, kOr2MeasureBonds) adds the measurement of
// the new configuration to b (this substep must then be the last of the
// sweep); kOr2MeasureBonds also forms the bond sums when a.bonds is set.
//
// The measuring pass without the bond terms (the production loop's usual
// case) needs few enough registers that, capped at 128, four wavefronts fit
// per SIMD as in the substeps that do not measure (three otherwise): the
// launch drops from 1.31x to about 1.06x a plain fused substep.  The cap is
// applied only up to three columns per thread, where it costs a few spilled
// registers outside the inner loop.
// ---------------------------------------------------------------------------
enum Or2Measure : int { kOr2Plain = 0, kOr2Measure = 1, kOr2MeasureBonds = 2 };

constexpr int or2_min_waves(int meas, int spt) { return (meas == kOr2Measure && spt <= 3) ? 4 : 1; }

// Elements of one old-colour-1 plane buffer of the fused kernel: a bound on
// (TY + 4) * L/2 (TY * L/2 <= SPT * kBlock tile sites, L/2 <= kBlock/2).
template <int SPT>
constexpr int kOr2P1Elems = SPT * kBlock + 2 * kBlock;

// LEAD: every lattice of the launch fills the tile's first SPT - 1 columns
// (TY * L/2 > (SPT - 1) * kBlock), so only the last column needs a guard.
template <int MEAS, int SPT, bool LEAD>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(or2_min_waves(MEAS, SPT))))
void k_or2_f32(SweepArgs a)
{
    constexpr int P1E = kOr2P1Elems<SPT>;
    constexpr bool P0ROT = MEAS != kOr2Plain;  // three rotating P0 buffers
    constexpr bool BONDS = MEAS == kOr2MeasureBonds;
    extern __shared__ f2 lds[];
    const int tid = threadIdx.x;

    for (int v = blockIdx.x; v < a.total_items; v += gridDim.x) {
        const int w = xcd_item(v, a.total_items);
        const int li = uni(find_lattice(a.lats, a.n_lat, w));
        const LatDev d = load_lat_uniform(a.lats + li);
        const int L = d.L, half = d.half, TY = d.TY, TZ = d.TZ;
        const int wl = w - d.item_base;
        const int slot = wl / d.items_per_slot;
        const int rem = wl - slot * d.items_per_slot;
        const int ty = rem % d.ny, tz = rem / d.ny;
        const int y0 = ty * TY, z0 = tz * TZ;
        const uint32_t plane_b = (uint32_t)L * (uint32_t)half * 4u;
        const int64_t nh = d.N / 2;
        const float *src = (const float *)a.ang + d.base + (int64_t)slot * d.N;
        float *dst = (float *)a.ang_dst + d.base + (int64_t)slot * d.N;
        const __amdgpu_buffer_rsrc_t r0s = colour_rsrc(src, nh);
        const __amdgpu_buffer_rsrc_t r1s = colour_rsrc(src + nh, nh);
        const __amdgpu_buffer_rsrc_t r0d = colour_rsrc(dst, nh);
        const __amdgpu_buffer_rsrc_t r1d = colour_rsrc(dst + nh, nh);
        const __amdgpu_buffer_rsrc_t rnull = colour_rsrc(src, 0);
        // P1 buffers at compile-time offsets (the alternating steps address
        // them through immediate LDS offsets); the P0 buffers after them
        const int rows0 = TY + 2;
        f2 *P1[2] = {lds, lds + P1E};
        f2 *P0base = lds + 2 * P1E;
        auto P0 = [&](int b) { return P0base + b * rows0 * half; };
        auto wrapy = [L](int y) { return y < 0 ? y + L : (y >= L ? y - L : y); };
        auto wrapz = wrapy;
        auto xm = [half](int j) { return j == 0 ? half - 1 : j - 1; };
        auto xp = [half](int j) { return j + 1 == half ? 0 : j + 1; };

        // ---- slot geometry (constant over z) ----
        // A tile column's LDS index is its in-plane index plus a uniform
        // shift (P1 rows start two rows above the tile, P0 rows one), and its
        // x-neighbour is a fixed delta away on even and on odd steps: for
        // colour 0 at (y, z) and colour 1 at (y, z-1) alike it is j+1 when
        // (y + z) is odd, j-1 when even (wrapping within the row).
        uint32_t voffT[SPT];
        int dxe[SPT], dxo[SPT];
        bool okT[SPT], pz0[SPT];
        const int zs = wrapz(z0 - 1);  // first step's plane
        const int sh1 = 2 * half - y0 * half, sh0 = half - y0 * half;
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
            const int f = tid + s * kBlock;
            okT[s] = (LEAD && s < SPT - 1) || f < TY * half;
            const int fl = okT[s] ? f : 0;
            const int yl = fl / half, j = fl - yl * half, y = y0 + yl;
            voffT[s] = (uint32_t)(y * half + j) * 4u;
            const bool podd = ((y + zs) & 1) != 0;
            pz0[s] = podd;
            const int dp = xp(j) - j, dm = xm(j) - j;
            dxe[s] = podd ? dp : dm;
            dxo[s] = podd ? dm : dp;
        }
        auto l1T = [&](int s) { return (int)(voffT[s] >> 2) + sh1; };
        auto l0T = [&](int s) { return (int)(voffT[s] >> 2) + sh0; };
        // halo rows on the last 2 * L/2 threads: the last tile column is
        // populated from the first thread on, so the halo goes to the
        // wavefronts that have fewer tile columns
        const int hbase = kBlock - 2 * half;
        const bool okH = tid >= hbase;
        const int eH = okH ? tid - hbase : 0;
        const int rH = eH >= half, jH = eH - rH * half;
        const int yH = rH ? wrapy(y0 + TY) : wrapy(y0 - 1);
        const uint32_t voffH = (uint32_t)(yH * half + jH) * 4u;
        const int l1H = (rH ? TY + 2 : 1) * half + jH;
        const int l0H = (rH ? TY + 1 : 0) * half + jH;
        const bool poddH = ((yH + zs) & 1) != 0;
        const int l1Hxe = (rH ? TY + 2 : 1) * half + (poddH ? xp(jH) : xm(jH));
        const int l1Hxo = (rH ? TY + 2 : 1) * half + (poddH ? xm(jH) : xp(jH));
        const int yO = rH ? wrapy(y0 + TY + 1) : wrapy(y0 - 2);
        const uint32_t voffO = (uint32_t)(yO * half + jH) * 4u;
        const int l1O = (rH ? TY + 3 : 0) * half + jH;

        // ---- prologue: state for the first step (plane zs = z0-1) ----
        auto pb = [&](int z) { return (uint32_t)wrapz(z) * plane_b; };
        // Old colour 1 of plane z-1 stays in the P1 buffer that is rewritten
        // only at the end of step z and new colour 0 of plane z-1 (and z-2
        // with three P0 buffers) in the other P0 buffers, so only plane z+1
        // (old colour 1), plane z and, with two P0 buffers, plane z-2 at the
        // tile columns (new colour 0) are held in registers.
        f2 c1p[SPT], c0z2[SPT];
        float r1m[SPT], r1c[SPT], r1p[SPT], t0[SPT];
        float aT1[SPT], aT0[SPT], bT1[SPT], bT0[SPT];
        f2 hp;
        float ht0, aH1, aH0, bH1, bH0, aO, bO;
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
            r1m[s] = bload(r1s, voffT[s], pb(z0 - 2));
            r1c[s] = bload(r1s, voffT[s], pb(z0 - 1));
            r1p[s] = bload(r1s, voffT[s], pb(z0));
            t0[s] = bload(r0s, voffT[s], pb(z0 - 1));
            aT1[s] = bload(r1s, voffT[s], pb(z0 + 1));
            aT0[s] = bload(r0s, voffT[s], pb(z0));
            P1[1][l1T(s)] = sincos_turns(r1m[s]);
            P1[0][l1T(s)] = sincos_turns(r1c[s]);
            c1p[s] = sincos_turns(r1p[s]);
        }
        const f2 hm0 = sincos_turns(bload(r1s, voffH, pb(z0 - 2)));
        const f2 hc0 = sincos_turns(bload(r1s, voffH, pb(z0 - 1)));
        hp = sincos_turns(bload(r1s, voffH, pb(z0)));
        ht0 = bload(r0s, voffH, pb(z0 - 1));
        aH1 = bload(r1s, voffH, pb(z0 + 1));
        aH0 = bload(r0s, voffH, pb(z0));
        const f2 o0 = sincos_turns(bload(r1s, voffO, pb(z0 - 1)));
        aO = bload(r1s, voffO, pb(z0));
        if (okH) {
            P1[1][l1H] = hm0;
            P1[0][l1H] = hc0;
            P1[0][l1O] = o0;
        }
        lds_barrier();

        double acc[kPartials];
#pragma unroll
        for (int q = 0; q < kPartials; ++q) acc[q] = 0.0;

        // ---- one step: a at plane z = z0-1+zz, b at plane z-1 ----
        auto step = [&](const int zz, const int par, float (&preT1)[SPT], float (&preT0)[SPT],
                        float &preH1, float &preH0, float &preO, float (&nxtT1)[SPT],
                        float (&nxtT0)[SPT], float &nxtH1, float &nxtH0, float &nxtO) {
            const int z = z0 - 1 + zz;
            const f2 *p1 = P1[par];
            f2 *p1n = P1[par ^ 1];           // plane z-1 until rewritten with z+1 at the end
            const int m3 = P0ROT ? zz % 3 : par;
            f2 *p0w = P0(m3);                  // new colour 0, plane z
            const f2 *p0r = P0ROT ? P0(m3 == 0 ? 2 : m3 - 1) : P0(par ^ 1);  // plane z-1
            const f2 *p0r2 = P0(m3 == 2 ? 0 : m3 + 1);  // plane z-2 (three buffers)
            {
                // last planes needed: old colour 1 at z0+TZ+1 (z neighbour of
                // a at z0+TZ), old colour 0 and the outer rows at z0+TZ; all
                // are issued at step TZ-1
                const bool need = zz <= TZ - 1;
                const __amdgpu_buffer_rsrc_t q1 = need ? r1s : rnull;
                const __amdgpu_buffer_rsrc_t q2 = q1;
                const __amdgpu_buffer_rsrc_t q0 = need ? r0s : rnull;
#pragma unroll
                for (int s = 0; s < SPT; ++s) {
                    nxtT1[s] = bload(q1, voffT[s], pb(z + 3));
                    nxtT0[s] = bload(q0, voffT[s], pb(z + 2));
                }
                nxtH1 = bload(q1, voffH, pb(z + 3));
                nxtH0 = bload(q0, voffH, pb(z + 2));
                nxtO = bload(q2, voffO, pb(z + 2));
            }
            const bool store_a = zz >= 1 && zz <= TZ;
            const uint32_t sz = pb(z), szm = pb(z - 1);
            // a: colour 0 at plane z on tile and halo columns
            // Work on columns past the tile (okT false) or past the halo rows
            // (okH false) is skipped: with TY * L/2 not a multiple of the
            // block size whole wavefronts have nothing to do in the last
            // column, and the branch lets them skip it.
            f2 c0cur[SPT];
#pragma unroll
            for (int s = 0; s < SPT; ++s) {
                if (!okT[s]) continue;
                const int lc = l1T(s), lx = lc + (par ? dxo[s] : dxe[s]);
                const f2 n1 = p1[lc - half], n2 = p1[lc + half], n3 = p1[lc], n4 = p1[lx];
                const f2 c1m = p1n[lc];
                const float hx = ((c1m.c + c1p[s].c) + (n1.c + n2.c)) + (n3.c + n4.c);
                const float hy = ((c1m.s + c1p[s].s) + (n1.s + n2.s)) + (n3.s + n4.s);
                const float nv = overrelax_turns(t0[s], hx, hy);
                if (store_a) bstore(nv, r0d, voffT[s], sz);
                c0cur[s] = sincos_turns(nv);
                p0w[l0T(s)] = c0cur[s];
            }
            if (okH) {
                const int lx = par ? l1Hxo : l1Hxe;
                const f2 n1 = p1[l1H - half], n2 = p1[l1H + half], n3 = p1[l1H], n4 = p1[lx];
                const f2 hm = p1n[l1H];
                const float hx = ((hm.c + hp.c) + (n1.c + n2.c)) + (n3.c + n4.c);
                const float hy = ((hm.s + hp.s) + (n1.s + n2.s)) + (n3.s + n4.s);
                p0w[l0H] = sincos_turns(overrelax_turns(ht0, hx, hy));
            }
            // b: colour 1 at plane z-1 on tile columns (from the third step
            // on); with two P0 buffers the own column's colour 0 of plane z-1
            // read here is kept for the next step's plane z-2
            if (zz >= 2) {
#pragma unroll
                for (int s = 0; s < SPT; ++s) {
                    if (!okT[s]) continue;
                    const int lc = l0T(s), lx = lc + (par ? dxo[s] : dxe[s]);
                    const f2 m1 = p0r[lc - half], m2 = p0r[lc + half], m3 = p0r[lc], m4 = p0r[lx];
                    const f2 c0m2 = P0ROT ? p0r2[lc] : c0z2[s];
                    if constexpr (!P0ROT) c0z2[s] = m3;
                    const float hx = ((c0m2.c + c0cur[s].c) + (m1.c + m2.c)) + (m3.c + m4.c);
                    const float hy = ((c0m2.s + c0cur[s].s) + (m1.s + m2.s)) + (m3.s + m4.s);
                    const float nv = overrelax_turns(r1m[s], hx, hy);
                    bstore(nv, r1d, voffT[s], szm);
                    if constexpr (MEAS != kOr2Plain) {
                        // colour 1 at (y, z-1) has x = 2j + p, p = (y + z) & 1
                        // (L even keeps the parity through the z wrap); the
                        // same-j neighbour is +x when p = 0, -x when p = 1
                        const bool podd = pz0[s] != (par != 0);
                        const f2 xpv = podd ? m4 : m3, xmv = podd ? m3 : m4;
                        const f2 sc = sincos_turns(nv);
                        const float nc[6] = {xpv.c, xmv.c, m2.c, m1.c, c0cur[s].c, c0m2.c};
                        const float ns[6] = {xpv.s, xmv.s, m2.s, m1.s, c0cur[s].s, c0m2.s};
                        // m3 is the colour-0 site with the same storage index
                        measure_site(acc, BONDS && a.bonds != 0, sc.c, sc.s, m3.c, m3.s, hx, hy, nc, ns);
                    }
                }
            } else if (!P0ROT && zz == 1) {
#pragma unroll
                for (int s = 0; s < SPT; ++s)
                    if (okT[s]) c0z2[s] = p0r[l0T(s)];
            }
            // next plane of old colour 1 into LDS (over plane z-1, which
            // every lane must have finished reading) and shift the z windows
            lds_barrier();
#pragma unroll
            for (int s = 0; s < SPT; ++s) {
                if (!okT[s]) continue;
                p1n[l1T(s)] = c1p[s];
                c1p[s] = sincos_turns(preT1[s]);
                r1m[s] = r1c[s];
                r1c[s] = r1p[s];
                r1p[s] = preT1[s];
                t0[s] = preT0[s];
            }
            if (okH) {
                p1n[l1H] = hp;
                p1n[l1O] = sincos_turns(preO);
                hp = sincos_turns(preH1);
                ht0 = preH0;
            }
            lds_barrier();
        };

        const int steps = TZ + 2;
        for (int zz = 0; zz < steps; zz += 2) {
            step(zz, 0, aT1, aT0, aH1, aH0, aO, bT1, bT0, bH1, bH0, bO);
            if (zz + 1 < steps) step(zz + 1, 1, bT1, bT0, bH1, bH0, bO, aT1, aT0, aH1, aH0, aO);
        }
        if constexpr (MEAS != kOr2Plain)
            block_store_partials(acc, a.partials + kPartials * (int64_t)w,
                                 (BONDS && a.bonds) ? kPartials : kPartialsNoBonds);
    }
}


// ---------------------------------------------------------------------------
// Launch dispatch over the compile-time column count and lead guard
// ---------------------------------------------------------------------------
template <int MEAS, bool LEAD>
static hipError_t launch_or2_spt(int spt, int grid, size_t lds, const SweepArgs &a, hipStream_t s,
                                 int *per_cu)
{
    switch (spt) {
    case 1: return launch_or_query(k_or2_f32<MEAS, 1, LEAD>, grid, lds, a, s, per_cu);
    case 2: return launch_or_query(k_or2_f32<MEAS, 2, LEAD>, grid, lds, a, s, per_cu);
    case 3: return launch_or_query(k_or2_f32<MEAS, 3, LEAD>, grid, lds, a, s, per_cu);
    case 4: return launch_or_query(k_or2_f32<MEAS, 4, LEAD>, grid, lds, a, s, per_cu);
    case 5: return launch_or_query(k_or2_f32<MEAS, 5, LEAD>, grid, lds, a, s, per_cu);
    case 6: return launch_or_query(k_or2_f32<MEAS, 6, LEAD>, grid, lds, a, s, per_cu);
    case 8: return launch_or_query(k_or2_f32<MEAS, 8, LEAD>, grid, lds, a, s, per_cu);
    default: return hipErrorInvalidValue;
    }
}

template <int MEAS>
static hipError_t launch_or2_lead(bool lead, int spt, int grid, size_t lds, const SweepArgs &a, hipStream_t s,
                                  int *per_cu)
{
    return lead ? launch_or2_spt<MEAS, true>(spt, grid, lds, a, s, per_cu)
                : launch_or2_spt<MEAS, false>(spt, grid, lds, a, s, per_cu);
}

}  // namespace xy
