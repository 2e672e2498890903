// Device helpers shared by the two translation units of the gfx950 kernels
// (the tiled half-sweeps and the rest in xy_kernels.hip, the fused
// over-relaxation substep in xy_or2.hip): wavefront reductions, the
// measurement of one site, wave-uniform loads, the LDS-scoped barrier, the
// XCD-contiguous item map, raw buffer loads and stores, and the launch helper.
#pragma once

#include <hip/hip_runtime.h>

#include "xy_device.h"
#include "xy_kernels.h"

namespace xy {

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

// Sum the first nq measurement accumulators (kPartials with the bond sums,
// kPartialsNoBonds without) over the workgroup in a fixed order and store
// the item's partials.  Ends with a barrier so the scratch can be reused.
__device__ __forceinline__ void block_store_partials(const double (&v)[kPartials], double *dst, int nq)
{
    __shared__ double red[kBlock / 64][kPartials];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kPartials; ++q) {
        if (q < nq) {
            const double t = wave_sum(v[q]);
            if (lane == 0) red[wv][q] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < nq) {
        double acc = 0.0;
        for (int i = 0; i < kBlock / 64; ++i) acc += red[i][threadIdx.x];
        dst[threadIdx.x] = acc;
    }
    __syncthreads();
}

// Measurement terms of one colour-1 site i with unit vector (c, s), the field
// h = (hx, hy) of its six colour-0 neighbours (the sum every update kernel
// forms, in the same order), those neighbours split by direction (+x, -x, +y,
// -y, +z, -z) and the colour-0 partner site at the same storage index (pc, ps):
//   S    += S_i . h_i
//   M    += S_i + S_partner                (each site counted once)
// and, when the bond sums of Eq. (6) are asked for,
//   C_mu += S_i . (S_{i+mu} + S_{i-mu})     bonds (i, i+mu) and (i-mu, i)
//   I_mu += sin(th_i - th_{i+mu}) - sin(th_i - th_{i-mu})
// Every bond has exactly one colour-1 end, so S counts each bond once and the
// energy of Eq. (1) is E = -S (= -(C_x + C_y + C_z) up to rounding).  Each
// site's terms are formed in the precision of its inputs (float32 on the
// float32 path: a few 1e-7 relative, like the inputs themselves) and
// accumulated in float64.
// The fused multiply-adds are written out so that every kernel that inlines
// this forms bit-identical terms (left to the compiler, contraction of the
// products may differ between instantiations).
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ void measure_site(double (&acc)[kPartials], bool bonds, T c, T s, T pc, T ps,
                                             T hx, T hy, const T (&nc)[6], const T (&ns)[6])
{
    acc[0] += (double)fma_t(c, hx, s * hy);
    acc[1] += (double)c + (double)pc;
    acc[2] += (double)s + (double)ps;
    if (bonds) {
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            const T cp = nc[2 * mu], sp = ns[2 * mu];
            const T cm = nc[2 * mu + 1], sm = ns[2 * mu + 1];
            const T ssum = s * (sp + sm), cdif = c * (sp - sm);
            acc[3 + mu] += (double)fma_t(c, cp + cm, ssum);
            acc[6 + mu] += (double)fma_t(s, cp - cm, -cdif);
        }
    }
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

// Values that are the same in every lane, moved to scalar registers (loads
// through kernel-argument pointers otherwise land in vector registers, and
// buffer descriptors built from them would need per-lane loops).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ LatDev load_lat_uniform(const LatDev *p)
{
    LatDev d = *p;
    d.L = uni(d.L);
    d.half = uni(d.half);
    d.R = uni(d.R);
    d.lat = uni(d.lat);
    d.base = uni64(d.base);
    d.N = uni64(d.N);
    d.pos_base = uni(d.pos_base);
    d.TY = uni(d.TY);
    d.TZ = uni(d.TZ);
    d.ny = uni(d.ny);
    d.nz = uni(d.nz);
    d.item_base = uni(d.item_base);
    d.items_per_slot = uni(d.items_per_slot);
    return d;
}

// Workgroup barrier that orders LDS only.  __syncthreads() also fences
// global memory, which on gfx9 waits for every outstanding global load and
// store (one shared counter) and would drain the z-plane prefetch at each
// plane.  The half-sweep kernels exchange data between lanes through LDS
// only, so an LDS-scoped release/acquire around s_barrier is sufficient.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Workgroups are dealt round-robin to the 8 XCDs (block b runs on XCD b mod 8).
// Map block ids so that each XCD walks a contiguous range of items: tiles
// that share halo rows (neighbouring y-tiles of one slot and z-chunk) then run
// at the same time on the same XCD and meet in its L2.  A bijection on
// [0, G); with a persistent grid that is a multiple of 8, every id a block
// visits stays on that block's XCD.
__device__ __forceinline__ int xcd_item(int b, int G)
{
    constexpr int kXcd = 8;
    const int q = G / kXcd, r = G - q * kXcd;
    const int x = b % kXcd, i = b / kXcd;
    return x * q + min(x, r) + i;
}

__device__ __forceinline__ int find_lattice(const LatDev *lats, int n_lat, int item)
{
    int li = 0;
    while (li + 1 < n_lat && item >= lats[li + 1].item_base) ++li;
    return li;
}

// ---------------------------------------------------------------------------
// Raw buffer access to one colour array of one slot: a scalar base and byte
// size, a per-lane byte offset (constant over z) and a scalar byte offset
// for the plane.  Out-of-range accesses read 0 / are dropped by hardware.
// ---------------------------------------------------------------------------
__device__ __forceinline__ __amdgpu_buffer_rsrc_t colour_rsrc(const float *base, int64_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)(uint32_t)(n * 4), 0x00020000);
}

__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

// Stores carry the non-temporal hint (cache-policy bit 1, `nt`): no kernel
// reads back what it writes in the same launch, and keeping the new angles
// out of the way in L2 leaves it to the halo rows that neighbouring tiles
// re-read (A/B on the L = 160 x 32 sweep: 1.5 % less time; the same hint on
// the loads cost 6 %).
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, 2);
}

// ---------------------------------------------------------------------------
// Launch helper.  With per_cu set, nothing is launched: *per_cu receives how
// many workgroups of k fit on one CU at the given LDS size (the resident
// capacity that persistent launches are sized to).
// ---------------------------------------------------------------------------
typedef void (*SweepKernel)(SweepArgs);

static inline hipError_t launch_or_query(SweepKernel k, int grid, size_t lds, const SweepArgs &a, hipStream_t s,
                                         int *per_cu)
{
    if (per_cu) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k, kBlock, lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

}  // namespace xy
