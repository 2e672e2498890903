// gfx950 kernels of the 3D XY model hot path (arXiv:1211.0780, Sec. II):
// checkerboard Metropolis and over-relaxation half-sweeps, observable
// reductions, parallel-tempering exchange, random start.
//
// Angle storage is colour-split: per storage slot, colour c's N/2 sites are
// ordered (z, y, j) with j = x/2 fastest.  Site (x, y, z) of colour c has
// x = 2j + p with p = (c + y + z) & 1.  Its six neighbours all have the other
// colour and sit at index j in rows (y +- 1, z) and (y, z +- 1), and at
// j and j + (p ? +1 : -1) (mod L/2) in its own row.
#include <hip/hip_runtime.h>
#include <math.h>

#include "xy_device.h"
#include "xy_kernels.h"

namespace xy {

constexpr int kHaloMax = 4;  // halo entries per thread: 2*(L/2) <= 4*kBlock, i.e. L <= 1024

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum (E, Mx, My) over the workgroup in a fixed order and store the item's
// partials.  Ends with a barrier so the scratch can be reused.
__device__ __forceinline__ void block_store_partials(double e, double mx, double my,
                                                     double *dst)
{
    __shared__ double red[kBlock / 64][3];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    e = wave_sum(e);
    mx = wave_sum(mx);
    my = wave_sum(my);
    if (lane == 0) {
        red[wv][0] = e;
        red[wv][1] = mx;
        red[wv][2] = my;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double se = 0.0, sx = 0.0, sy = 0.0;
        for (int i = 0; i < kBlock / 64; ++i) {
            se += red[i][0];
            sx += red[i][1];
            sy += red[i][2];
        }
        dst[0] = se;
        dst[1] = sx;
        dst[2] = sy;
    }
    __syncthreads();
}

__device__ __forceinline__ void block_add_accepts(unsigned long long n, unsigned long long *dst)
{
    __shared__ unsigned long long red[kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    n = wave_sum_u64(n);
    if (lane == 0) red[wv] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < kBlock / 64; ++i) s += red[i];
        if (s) atomicAdd(dst, s);
    }
    __syncthreads();
}

__device__ __forceinline__ int find_lattice(const LatDev *lats, int n_lat, int item)
{
    int li = 0;
    while (li + 1 < n_lat && item >= lats[li + 1].item_base) ++li;
    return li;
}

// ---------------------------------------------------------------------------
// Tiled FP32 half-sweep.  A work item is (lattice, slot, y-tile, z-chunk):
// TY rows of L/2 sites of the updated colour, streamed over TZ planes.  Each
// thread owns SPT (y, j) columns of the tile.  The other colour is read once
// per plane, turned into (cos, sin) once, kept in registers for the z
// neighbours (planes z-1, z+1 of the same column) and staged in LDS (plane
// z plus one halo row above and below the tile, double-buffered) for the
// x and y neighbours.
//
// KIND = kMetro / kOver updates colour a.colour; kMeas (colour 1) only
// measures.  MEAS accumulates E = -sum_{i in colour 1} S_i . h_i (every
// bond has exactly one colour-1 end) and M = sum over both colours into the
// item's partials.
// ---------------------------------------------------------------------------
template <int KIND, bool MEAS, int SPT>
__global__ __launch_bounds__(kBlock) void k_tile_f32(SweepArgs a)
{
    extern __shared__ f2 lds[];
    const int tid = threadIdx.x;
    const uint32_t t_sweep = a.ctl->t;

    for (int w = blockIdx.x; w < a.total_items; w += gridDim.x) {
        const int li = find_lattice(a.lats, a.n_lat, w);
        const LatDev d = a.lats[li];
        const int L = d.L, half = d.half, TY = d.TY;
        const int wl = w - d.item_base;
        const int slot = wl / d.items_per_slot;
        const int rem = wl - slot * d.items_per_slot;
        const int ty = rem % d.ny, tz = rem / d.ny;
        const int y0 = ty * TY, z0 = tz * d.TZ;
        const int k = a.pos[d.pos_base + slot];
        const float beta = (float)a.beta[d.pos_base + k];
        const int64_t plane = (int64_t)L * half;
        float *angs = (float *)a.ang + d.base + (int64_t)slot * d.N;
        float *own = angs + (int64_t)a.colour * (d.N / 2);
        const float *oth = angs + (int64_t)(a.colour ^ 1) * (d.N / 2);
        const int nsite = TY * half;
        f2 *buf0 = lds;
        f2 *buf1 = lds + (TY + 2) * half;
        const uint32_t LL = (uint32_t)L * (uint32_t)L;
        const uint32_t c2 = ((uint32_t)d.lat << 16) | (uint32_t)k;
        const uint32_t c3 = (kPhaseMetro << 24) | (uint32_t)a.substep;

        int off[SPT], lc[SPT], lxm[SPT], lxp[SPT], ypar[SPT];
        uint32_t ibase[SPT];
        bool ok[SPT];
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
            const int f = tid + s * kBlock;
            ok[s] = f < nsite;
            const int fl = ok[s] ? f : 0;
            const int yl = fl / half;
            const int j = fl - yl * half;
            const int y = y0 + yl;
            off[s] = y * half + j;
            lc[s] = (yl + 1) * half + j;
            lxm[s] = (yl + 1) * half + ((j == 0) ? half - 1 : j - 1);
            lxp[s] = (yl + 1) * half + ((j + 1 == half) ? 0 : j + 1);
            ypar[s] = (a.colour + y) & 1;
            ibase[s] = 2u * (uint32_t)j + (uint32_t)L * (uint32_t)y;
        }
        const int ym = (y0 == 0) ? L - 1 : y0 - 1;
        const int yp = (y0 + TY == L) ? 0 : y0 + TY;
        int hoff[kHaloMax], hl[kHaloMax];
        bool hok[kHaloMax];
#pragma unroll
        for (int h = 0; h < kHaloMax; ++h) {
            const int e = tid + h * kBlock;
            hok[h] = e < 2 * half;
            const int ee = hok[h] ? e : 0;
            const int r = ee >= half;
            const int jj = ee - r * half;
            hoff[h] = (r ? yp : ym) * half + jj;
            hl[h] = (r ? (TY + 1) : 0) * half + jj;
        }

        // prologue: planes z0-1, z0, z0+1 of the other colour, plane z0 of ours
        const int zm1 = (z0 == 0) ? L - 1 : z0 - 1;
        const int zp1 = (z0 + 1 == L) ? 0 : z0 + 1;
        f2 ocm[SPT], oc0[SPT], ocp[SPT];
        float cur[SPT];
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
            float am = 0.f, a0 = 0.f, ap = 0.f, ac = 0.f;
            if (ok[s]) {
                am = oth[(int64_t)zm1 * plane + off[s]];
                a0 = oth[(int64_t)z0 * plane + off[s]];
                ap = oth[(int64_t)zp1 * plane + off[s]];
                ac = own[(int64_t)z0 * plane + off[s]];
            }
            ocm[s] = sincos_turns(am);
            oc0[s] = sincos_turns(a0);
            ocp[s] = sincos_turns(ap);
            cur[s] = ac;
            if (ok[s]) buf0[lc[s]] = oc0[s];
        }
#pragma unroll
        for (int h = 0; h < kHaloMax; ++h)
            if (hok[h]) buf0[hl[h]] = sincos_turns(oth[(int64_t)z0 * plane + hoff[h]]);
        __syncthreads();

        double accE = 0.0, accX = 0.0, accY = 0.0;
        unsigned long long nacc = 0;

        for (int zz = 0; zz < d.TZ; ++zz) {
            const int z = z0 + zz;
            const int zn = (z + 1 == L) ? 0 : z + 1;
            const int zn2 = (zn + 1 == L) ? 0 : zn + 1;
            const f2 *bc = (zz & 1) ? buf1 : buf0;
            f2 *bn = (zz & 1) ? buf0 : buf1;
            const bool more = zz + 1 < d.TZ;

            float rawo[SPT], rawc[SPT], rawh[kHaloMax];
#pragma unroll
            for (int s = 0; s < SPT; ++s) {
                rawo[s] = 0.f;
                rawc[s] = 0.f;
                if (more && ok[s]) {
                    rawo[s] = oth[(int64_t)zn2 * plane + off[s]];
                    rawc[s] = own[(int64_t)zn * plane + off[s]];
                }
            }
#pragma unroll
            for (int h = 0; h < kHaloMax; ++h) {
                rawh[h] = 0.f;
                if (more && hok[h]) rawh[h] = oth[(int64_t)zn * plane + hoff[h]];
            }

#pragma unroll
            for (int s = 0; s < SPT; ++s) {
                if (!ok[s]) continue;
                const int p = (ypar[s] + z) & 1;
                const f2 n1 = bc[lc[s] - half];
                const f2 n2 = bc[lc[s] + half];
                const f2 n3 = bc[lc[s]];
                const f2 n4 = bc[p ? lxp[s] : lxm[s]];
                const float hx = ((ocm[s].c + ocp[s].c) + (n1.c + n2.c)) + (n3.c + n4.c);
                const float hy = ((ocm[s].s + ocp[s].s) + (n1.s + n2.s)) + (n3.s + n4.s);
                float nv = cur[s];
                if constexpr (KIND == kOver) {
                    nv = overrelax_turns(cur[s], hx, hy);
                } else if constexpr (KIND == kMetro) {
                    const uint32_t i = ibase[s] + (uint32_t)p + LL * (uint32_t)z;
                    const u32x4 r = philox4x32_10(i, t_sweep, c2, c3, a.k0, a.k1);
                    const float u0 = unit24f(r.x), u1 = unit24f(r.y);
                    const f2 so = sincos_turns(cur[s]);
                    const f2 sn = sincos_turns(u0);
                    const float dE = (so.c - sn.c) * hx + (so.s - sn.s) * hy;
                    const float pa = __expf(-beta * dE);
                    const bool acc = u1 < pa;
                    if (a.recheck && __builtin_fabsf(u1 - pa) < 1e-5f) {
                        const uint32_t idx = atomicAdd(&a.rq->count, 1u);
                        if (idx < a.rq->capacity) {
                            RecheckEntry e;
                            e.li = li;
                            e.slot = slot;
                            e.q = (int32_t)((int64_t)z * plane + off[s]);
                            e.cur = cur[s];
                            e.u0 = u0;
                            e.u1 = u1;
                            e.fp32_accept = acc ? 1 : 0;
                            e.pad_ = 0;
                            a.rq->entries[idx] = e;
                        } else {
                            atomicAdd(&a.rq->overflow, 1u);
                        }
                    }
                    nv = acc ? u0 : cur[s];
                    nacc += acc ? 1ull : 0ull;
                }
                if constexpr (MEAS || KIND == kMeas) {
                    const f2 sc = sincos_turns(nv);
                    accE -= (double)sc.c * (double)hx + (double)sc.s * (double)hy;
                    accX += (double)sc.c + (double)oc0[s].c;
                    accY += (double)sc.s + (double)oc0[s].s;
                }
                if constexpr (KIND != kMeas) own[(int64_t)z * plane + off[s]] = nv;
            }

            if (more) {
#pragma unroll
                for (int s = 0; s < SPT; ++s) {
                    if (ok[s]) bn[lc[s]] = ocp[s];
                    ocm[s] = oc0[s];
                    oc0[s] = ocp[s];
                    ocp[s] = sincos_turns(rawo[s]);
                    cur[s] = rawc[s];
                }
#pragma unroll
                for (int h = 0; h < kHaloMax; ++h)
                    if (hok[h]) bn[hl[h]] = sincos_turns(rawh[h]);
            }
            __syncthreads();
        }

        if constexpr (KIND == kMetro) block_add_accepts(nacc, a.macc + d.pos_base + k);
        if constexpr (MEAS || KIND == kMeas) block_store_partials(accE, accX, accY, a.partials + 3 * (int64_t)w);
    }
}

// ---------------------------------------------------------------------------
// Re-take the queued near-threshold Metropolis decisions in float64: the six
// neighbour angles (other colour, untouched by this half-sweep) are read
// again, dE and exp(-beta dE) evaluated in double, and the site is corrected
// where the float64 decision differs.  One workgroup; empties the queue.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_recheck(const LatDev *lats, float *ang,
                                                    const double *beta, const int32_t *pos,
                                                    int colour, RecheckQueue *rq,
                                                    unsigned long long *macc)
{
    const double twopi = 6.283185307179586476925286766559;
    const uint32_t n = min(rq->count, rq->capacity);
    for (uint32_t e = threadIdx.x; e < n; e += blockDim.x) {
        const RecheckEntry en = rq->entries[e];
        const LatDev d = lats[en.li];
        const int L = d.L, half = d.half;
        const int64_t plane = (int64_t)L * half;
        const int z = (int)(en.q / plane);
        const int rem = (int)(en.q - (int64_t)z * plane);
        const int y = rem / half, j = rem - y * half;
        const int p = (colour + y + z) & 1;
        float *angs = ang + d.base + (int64_t)en.slot * d.N;
        float *own = angs + (int64_t)colour * (d.N / 2);
        const float *oth = angs + (int64_t)(colour ^ 1) * (d.N / 2);
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
        sincos((double)en.u0 * twopi, &sp, &cp);
        const double dE = (co - cp) * hx + (so - sp) * hy;
        const int k = pos[d.pos_base + en.slot];
        const bool acc = (double)en.u1 < exp(-beta[d.pos_base + k] * dE);
        if ((int)acc != en.fp32_accept) {
            own[en.q] = acc ? en.u0 : en.cur;
            atomicAdd(macc + d.pos_base + k, acc ? 1ull : ~0ull);  // +1 or -1
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) rq->count = 0;
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
    double accE = 0.0, accX = 0.0, accY = 0.0;
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
            const uint32_t i = 2u * (uint32_t)j + (uint32_t)p +
                               (uint32_t)L * ((uint32_t)y + (uint32_t)L * (uint32_t)z);
            const u32x4 r = philox4x32_10(i, a.ctl->t, ((uint32_t)d.lat << 16) | (uint32_t)k,
                                          (kPhaseMetro << 24) | (uint32_t)a.substep, a.k0, a.k1);
            const double prop = twopi * unit24d(r.x);
            const double u = unit24d(r.y);
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
            accE = -(c1 * hx + s1 * hy);
            accX = c1 + c0;
            accY = s1 + s0;
        }
        if constexpr (KIND != kMeas) own[q] = nv;
    }
    if constexpr (KIND == kMetro) block_add_accepts(nacc, a.macc + d.pos_base + k);
    if constexpr (MEAS || KIND == kMeas) block_store_partials(accE, accX, accY, a.partials + 3 * (int64_t)w);
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
                           int use_ring, int64_t ring_stride, int do_sum, int do_exchange,
                           unsigned long long *sacc, Ctl *ctl, uint32_t k0, uint32_t k1,
                           int *bad)
{
    const LatDev d = lats[blockIdx.x];
    const int pb = d.pos_base;
    if (do_sum) {
        double *out = obs;
        if (out && use_ring) out += (int64_t)ctl->ring * ring_stride;
        for (int r = threadIdx.x; r < d.R; r += blockDim.x) {
            const double *pp = partials + 3 * ((int64_t)d.item_base + (int64_t)r * d.items_per_slot);
            double E = 0.0, mx = 0.0, my = 0.0;
            for (int it = 0; it < d.items_per_slot; ++it) {
                E += pp[3 * it + 0];
                mx += pp[3 * it + 1];
                my += pp[3 * it + 2];
            }
            E_slot[pb + r] = E;
            if (!isfinite(E) || !isfinite(mx) || !isfinite(my)) atomicOr(bad, 1);
            if (out) {
                const int kk = pos[pb + r];
                const double n = (double)d.N;
                const double m = sqrt(mx * mx + my * my) / n;
                double *o = out + 5 * (int64_t)(pb + kk);
                o[0] = E;
                o[1] = E / n;
                o[2] = m;
                o[3] = m * m;
                o[4] = (m * m) * (m * m);
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
// Launchers
// ---------------------------------------------------------------------------
template <int KIND, bool MEAS>
static hipError_t launch_tile_spt(int spt, int grid, size_t lds, const SweepArgs &a, hipStream_t s)
{
    switch (spt) {
    case 1: hipLaunchKernelGGL((k_tile_f32<KIND, MEAS, 1>), dim3(grid), dim3(kBlock), lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_tile_f32<KIND, MEAS, 2>), dim3(grid), dim3(kBlock), lds, s, a); break;
    case 3: hipLaunchKernelGGL((k_tile_f32<KIND, MEAS, 3>), dim3(grid), dim3(kBlock), lds, s, a); break;
    case 4: hipLaunchKernelGGL((k_tile_f32<KIND, MEAS, 4>), dim3(grid), dim3(kBlock), lds, s, a); break;
    case 5: hipLaunchKernelGGL((k_tile_f32<KIND, MEAS, 5>), dim3(grid), dim3(kBlock), lds, s, a); break;
    case 6: hipLaunchKernelGGL((k_tile_f32<KIND, MEAS, 6>), dim3(grid), dim3(kBlock), lds, s, a); break;
    case 8: hipLaunchKernelGGL((k_tile_f32<KIND, MEAS, 8>), dim3(grid), dim3(kBlock), lds, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tile_f32(int kind, bool fuse_measure, int spt, int grid, size_t lds,
                           const SweepArgs &a, hipStream_t s)
{
    if (kind == kMetro)
        return fuse_measure ? launch_tile_spt<kMetro, true>(spt, grid, lds, a, s)
                            : launch_tile_spt<kMetro, false>(spt, grid, lds, a, s);
    if (kind == kOver)
        return fuse_measure ? launch_tile_spt<kOver, true>(spt, grid, lds, a, s)
                            : launch_tile_spt<kOver, false>(spt, grid, lds, a, s);
    return launch_tile_spt<kMeas, false>(spt, grid, lds, a, s);
}

hipError_t launch_recheck(const LatDev *lats, void *ang, const double *beta, const int32_t *pos,
                          int colour, RecheckQueue *rq, unsigned long long *macc, hipStream_t s)
{
    hipLaunchKernelGGL(k_recheck, dim3(1), dim3(kBlock), 0, s, lats, (float *)ang, beta, pos, colour,
                       rq, macc);
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
                           double *obs, int use_ring, int64_t ring_stride, int do_sum,
                           int do_exchange, unsigned long long *sacc, Ctl *ctl, uint32_t k0,
                           uint32_t k1, int *bad, hipStream_t s)
{
    int threads = 64;
    while (threads < max_R && threads < 1024) threads *= 2;
    hipLaunchKernelGGL(k_finalize, dim3(n_lat), dim3(threads), 0, s, lats, partials, beta, pos,
                       slot_of, E_slot, obs, use_ring, ring_stride, do_sum, do_exchange, sacc, ctl,
                       k0, k1, bad);
    return hipGetLastError();
}

hipError_t launch_tick(Ctl *ctl, uint32_t dt, uint32_t dtau, uint32_t dring, int set_ring,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, ctl, dt, dtau, dring, set_ring);
    return hipGetLastError();
}

}  // namespace xy
