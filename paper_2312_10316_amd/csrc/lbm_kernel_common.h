// lbm_kernel_common.h -- device helpers shared by the D2Q9 and D3Q19 kernel files: storage/math
// traits, wave-uniform addressing, the XCD-aware tile order and the compensated block reduction.
#pragma once

#include "lbm_internal.h"

namespace lbm {

template <int MODE>
struct ModeTraits;
template <>
struct ModeTraits<MODE_F64_F64> {
    using St = StoreF64;
    using M = double;
};
template <>
struct ModeTraits<MODE_F64_F32> {
    using St = StoreF64;
    using M = float;
};
template <>
struct ModeTraits<MODE_F32_F32> {
    using St = StoreF32;
    using M = float;
};
template <>
struct ModeTraits<MODE_F16S_F32> {
    using St = StoreF16S;
    using M = float;
};
template <>
struct ModeTraits<MODE_F16SR_F32> {
    using St = StoreF16SR;
    using M = float;
};

// The flux form of the auxiliary term at one node (Sec. 2.3): d_b(phi u_a u_b) - u_a d_b(phi u_b) by
// central differences, from phi and u at the west, east, south and north neighbours (same time level)
// and u at the node.  Every kernel that uses the flux form calls this one expression sequence, so they
// all round alike.
template <class M>
__device__ __forceinline__ void flux_aux(M pw, M pe, M ps, M pn, M uxw, M uyw, M uxe, M uye, M uxs, M uys, M uxn,
                                         M uyn, M uxc, M uyc, M &Ax, M &Ay)
{
    const M fwx = pw * uxw, fex = pe * uxe;  // phi u_x at the west and east neighbours
    const M fsy = ps * uys, fny = pn * uyn;  // phi u_y at the south and north neighbours
    const M div = (fex - fwx) * M(0.5) + (fny - fsy) * M(0.5);
    Ax = (fex * uxe - fwx * uxw) * M(0.5) + (fny * uxn - fsy * uxs) * M(0.5) - uxc * div;
    Ay = (fex * uye - fwx * uyw) * M(0.5) + (fny * uyn - fsy * uys) * M(0.5) - uyc * div;
}

// Time level of the state a launch reads (stochastic rounding only; 0 otherwise).  The counter pair
// lives in device memory so that graph replays see the level advance: a launch reads clock[parity],
// which no thread of it writes, and one thread of it writes clock[parity ^ 1] for the next launch.
template <class C>
__device__ __forceinline__ int64_t launch_level(const InstDesc &d, int parity)
{
    if constexpr (C::kStochastic) {
        const int64_t v = __hip_atomic_load(d.clock + parity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
        return (int64_t)(((uint64_t)hi << 32) | lo);
    } else {
        return 0;
    }
}
template <class C>
__device__ __forceinline__ void advance_level(const InstDesc &d, int parity, int64_t level, int steps, bool writer)
{
    if constexpr (C::kStochastic) {
        if (writer) __hip_atomic_store(d.clock + (parity ^ 1), level + steps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __forceinline__ int wrap_dec(int v, int n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ int wrap_inc(int v, int n) { return v == n - 1 ? 0 : v + 1; }

// Element at a 32-bit byte offset from a wave-uniform base: lets the compiler use the scalar-base +
// 32-bit-lane-offset addressing form instead of per-lane 64-bit address arithmetic.
template <class T>
__device__ __forceinline__ T ld_at(const T *base, unsigned byte_off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}
// Stores of the new state: non-temporal ones stream it to HBM; cached ones leave it in L2 and the
// Infinity Cache, where the next step finds it when the step's working set fits there.
template <class T>
__device__ __forceinline__ void st_nt_at(T *base, unsigned byte_off, T v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off));
}
template <class T>
__device__ __forceinline__ void st_at(T *base, unsigned byte_off, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off) = v;
}

// Block b -> tile t (tiles numbered row-major, ntx per row).  The hardware hands block b to XCD
// b % 8, and each XCD has its own L2.
//   remap 0: t = b, so the XCDs interleave tile by tile along each row;
//   remap 1: XCD j takes one contiguous range of tiles (a band of whole tile rows);
//   remap 2: XCD j takes one band of ntx/8 tile columns and walks it row by row, so the 8 XCDs
//            sweep the same rows together while each shares tile edges with at most two others
//            (needs ntx % 8 == 0; otherwise it is remap 0);
//   remap 3: XCD j takes row blocks j, j + 8, ... of h tile rows each, so the XCDs sweep a window
//            of about 8h tile rows together and every strip edge of a row stays in one L2.
__device__ __forceinline__ int tile_of_block(int b, int nb, int remap, int ntx, int h)
{
    if (remap == 3) {
        // Blocks of hb tiles (h tile rows) dealt round-robin to the XCDs.  The first `full` blocks
        // (a multiple of 8 blocks) are permuted among themselves; the rest keep their tile.
        const int hb = max(h, 1) * ntx, full = nb - nb % (8 * hb);
        if (b < full) {
            const int i = b >> 3;
            return ((i / hb) * 8 + (b & 7)) * hb + i % hb;
        }
        return b;
    }
    if (remap == 1) {
        const int q = nb >> 3, r = nb & 7, j = b & 7;
        return j * q + min(j, r) + (b >> 3);
    }
    if (remap == 2 && (ntx & 7) == 0) {
        const int bw = ntx >> 3, i = b >> 3;
        return (i / bw) * ntx + (b & 7) * bw + i % bw;
    }
    return b;
}

// ---- diagnostics ------------------------------------------------------------------------------

__device__ __forceinline__ CSum csum_shfl_xor(CSum v, int m)
{
    CSum o;
    o.s = __shfl_xor(v.s, m);
    o.c = __shfl_xor(v.c, m);
    return o;
}

// Reduces (3 compensated sums, 2 maxima, 1 count) over the block; thread 0 gets the result.
// Within a wave: butterfly shuffles with TwoSum merges; across the 4 waves: LDS.
__device__ inline void block_reduce(CSum (&cs)[3], double &mx0, double &mx1, double &cnt)
{
    __shared__ double sh[4][10];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) cs[k] = csum_merge(cs[k], csum_shfl_xor(cs[k], m));
        mx0 = fmax(mx0, __shfl_xor(mx0, m));
        mx1 = fmax(mx1, __shfl_xor(mx1, m));
        cnt += __shfl_xor(cnt, m);
    }
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) {
        for (int k = 0; k < 3; ++k) {
            sh[wave][2 * k] = cs[k].s;
            sh[wave][2 * k + 1] = cs[k].c;
        }
        sh[wave][6] = mx0;
        sh[wave][7] = mx1;
        sh[wave][8] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x / 64); ++w) {
            for (int k = 0; k < 3; ++k) cs[k] = csum_merge(cs[k], CSum{sh[w][2 * k], sh[w][2 * k + 1]});
            mx0 = fmax(mx0, sh[w][6]);
            mx1 = fmax(mx1, sh[w][7]);
            cnt += sh[w][8];
        }
    }
}

inline int grid_for(int64_t n, int block, int cap)
{
    int64_t g = (n + block - 1) / block;
    if (g > cap) g = cap;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace lbm
