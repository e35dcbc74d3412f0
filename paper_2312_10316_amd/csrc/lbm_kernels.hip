// lbm_kernels.hip -- HIP kernels of the TRT-R D2Q9 step for gfx950.
//
// State convention (pull scheme): buffer A holds, at node y, the post-collision values P_i(y)
// computed there in the previous step.  The pre-collision population at x is therefore
// g_i(x) = A_i(x - e_i) (streaming of Sec. 2.2, Eq. (14)), and one step reads A with those shifts
// and writes P_i(x) to buffer B at x.  The initial buffer is written pre-shifted
// (A_i(x - e_i) = g_eq_i(phi0(x), u(x))) so that the first pull yields g = g_eq(phi0, u).
//
// The step is a bandwidth-bound stencil: per node it moves 9 populations in and 9 out plus the
// velocity (and D when it is a field), against ~250 flops that stay in registers, so it is written
// for coalesced streaming: lane = column (a wave reads 64 consecutive elements of each row segment),
// each wave walks a few rows so the velocity stencil's y-neighbours stay in registers, stores are
// non-temporal, and the tile order can be remapped so neighbouring tiles share an XCD's L2.
#include <type_traits>

#include "lbm_internal.h"
#include "lbm_kernel_common.h"

namespace lbm {
namespace {



// g_i(x, y) = buf_i(x - e_i).  rm, rc, rp: the row blocks (9 segments) of rows y-1, y, y+1 (wrapped);
// xm, xp: columns x-1, x+1 (wrapped).
template <class St, class M>
__device__ __forceinline__ void pull(const typename St::T *__restrict__ rm, const typename St::T *__restrict__ rc,
                                     const typename St::T *__restrict__ rp, int64_t pitch, int xm, int x, int xp,
                                     const F16Params &f, M (&g)[9])
{
    using C = Codec<St, M>;
    g[0] = C::dec(rc[0 * pitch + x], 0, f);
    g[1] = C::dec(rc[1 * pitch + xm], 1, f);
    g[2] = C::dec(rm[2 * pitch + x], 2, f);
    g[3] = C::dec(rc[3 * pitch + xp], 3, f);
    g[4] = C::dec(rp[4 * pitch + x], 4, f);
    g[5] = C::dec(rm[5 * pitch + xm], 5, f);
    g[6] = C::dec(rm[6 * pitch + xp], 6, f);
    g[7] = C::dec(rp[7 * pitch + xp], 7, f);
    g[8] = C::dec(rp[8 * pitch + xm], 8, f);
}

template <class T>
__device__ __forceinline__ const T *row_block(const T *base, const Layout &L, int y)
{
    return base + (int64_t)y * 9 * L.pitch;
}

template <class St, class M>
__device__ __forceinline__ void pull_node(const typename St::T *__restrict__ src, const Layout &L, int x, int y,
                                          const F16Params &f, M (&g)[9])
{
    pull<St, M>(row_block(src, L, wrap_dec(y, L.ny)), row_block(src, L, y), row_block(src, L, wrap_inc(y, L.ny)),
                L.pitch, wrap_dec(x, L.nx), x, wrap_inc(x, L.nx), f, g);
}

// Dirichlet node (x, y) of a non-equilibrium-extrapolation edge (Guo, Zheng & Shi 2002; the boundary
// scheme of the benchmark of Sec. 3): g = g_eq(phi_b, u) + [g(x_f) - g_eq(phi(x_f), u(x_f))], x_f the
// interior neighbour along the inward normal (diagonal at a corner).
__device__ __forceinline__ bool on_edge(int x, int y, const Layout &L)
{
    return x == 0 || y == 0 || x == L.nx - 1 || y == L.ny - 1;
}

template <class St, class M>
__device__ __forceinline__ void nee_replace(const typename St::T *__restrict__ src, const M *__restrict__ u,
                                            const M *__restrict__ bc, const Layout &L, int x, int y,
                                            const F16Params &f, M (&g)[9])
{
    const int xf = x + (x == 0) - (x == L.nx - 1), yf = y + (y == 0) - (y == L.ny - 1);
    M gf[9];
    pull_node<St, M>(src, L, xf, yf, f, gf);
    const M phif = gf[0] + gf[1] + gf[2] + gf[3] + gf[4] + gf[5] + gf[6] + gf[7] + gf[8];
    M ef[9], eb[9];
    equilibrium<M>(phif, u[(int64_t)yf * 2 * L.pitch + xf], u[((int64_t)yf * 2 + 1) * L.pitch + xf], ef);
    equilibrium<M>(bc[(int64_t)y * L.pitch + x], u[(int64_t)y * 2 * L.pitch + x], u[((int64_t)y * 2 + 1) * L.pitch + x], eb);
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = eb[i] + (gf[i] - ef[i]);
}

// Walls (halfway anti-bounce-back) below row 0 and above row ny - 1: a population that crossed the
// wall returns to its node reversed, g_i = -P_opp(i) + 2 g_eq_i^+(phi_w, u), with
// 2 g_eq_i^+ = g_eq_i + g_eq_opp(i), P_opp(i) the node's own post-collision value of the previous step
// (element (y, opp(i), x)) and phi_w the wall value stored in row y of bc.  Applies to y = 0
// (i = 2, 5, 6 arrive from below) and y = ny - 1 (i = 4, 7, 8 arrive from above).
template <class St, class M>
__device__ __forceinline__ void wall_replace(const typename St::T *__restrict__ row, unsigned boff, M phiw, M ux,
                                             M uy, bool bottom, const F16Params &f, int64_t pitch, M (&g)[9])
{
    using C = Codec<St, M>;
    M e[9];
    equilibrium<M>(phiw, ux, uy, e);
    // every slot is written through a select (no slot-dependent branches), which keeps g in registers
    const int o2 = bottom ? 4 : 2, o5 = bottom ? 7 : 5, o6 = bottom ? 8 : 6;  // stored slot reflected
    const M p2 = C::dec(ld_at(row + o2 * pitch, boff), o2, f);
    const M p5 = C::dec(ld_at(row + o5 * pitch, boff), o5, f);
    const M p6 = C::dec(ld_at(row + o6 * pitch, boff), o6, f);
    const M a = (bottom ? e[2] + e[4] : e[4] + e[2]) - p2;
    const M b = (bottom ? e[5] + e[7] : e[7] + e[5]) - p5;
    const M c = (bottom ? e[6] + e[8] : e[8] + e[6]) - p6;
    g[2] = bottom ? a : g[2];
    g[5] = bottom ? b : g[5];
    g[6] = bottom ? c : g[6];
    g[4] = bottom ? g[4] : a;
    g[7] = bottom ? g[7] : b;
    g[8] = bottom ? g[8] : c;
}

// The state of node (x, y) as the step sees it before collision: the pull, then the boundary rule.
template <class St, class M>
__device__ __forceinline__ void state_node(const typename St::T *__restrict__ src, const EdgeArgs &edge, const Layout &L,
                                           int x, int y, const F16Params &f, M (&g)[9])
{
    if (edge.kind == 3) {  // one buffer after its streaming step: g_i of the node sits in its slot opp(i)
        const typename St::T *row = src + (int64_t)y * 9 * L.pitch;
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = Codec<St, M>::dec(row[kOpp[i] * L.pitch + x], i, f);
        return;
    }
    pull_node<St, M>(src, L, x, y, f, g);
    const M *u = static_cast<const M *>(edge.u);
    const M *bc = static_cast<const M *>(edge.bc);
    if (edge.kind == 1 && on_edge(x, y, L)) {
        nee_replace<St, M>(src, u, bc, L, x, y, f, g);
    } else if (edge.kind == 2 && (y == 0 || y == L.ny - 1)) {
        const int64_t p = L.pitch;
        wall_replace<St, M>(src + (int64_t)y * 9 * p, (unsigned)x * (unsigned)sizeof(typename St::T),
                            bc[(int64_t)y * p + x], u[(int64_t)y * 2 * p + x], u[((int64_t)y * 2 + 1) * p + x],
                            y == 0, f, p, g);
    }
}

// Value of v in lane k (uniform k), broadcast to the wave.
template <class M>
__device__ __forceinline__ M lane_read(M v, int k);
template <>
__device__ __forceinline__ float lane_read<float>(float v, int k)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
template <>
__device__ __forceinline__ double lane_read<double>(double v, int k)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}



// One tile of one step with the local auxiliary term (or none).  Block (64, 4): lane = column of a
// 64-wide tile, wave `wave` walks `rows` rows.  The wave's row is uniform (taken with readfirstlane), so row and segment bases live in
// scalar registers and each load or store needs only a 32-bit lane offset (x, x-1 or x+1).
// ROWS > 0 fixes the walk length at compile time (the common one-row launch then has no loop, and
// every access keeps the scalar-base + 32-bit-offset form); 0 takes it from the launch shape.
// IP: 0 two buffers (pull from buf[parity], store to buf[parity ^ 1]); 1 and 2: one buffer updated in
// place (Bailey et al.'s AA pattern, one-row launches only).  In the standard state every node's
// post-collision values sit at the node (slot i holds P_i), exactly the two-buffer layout.  Step 1
// (streaming) pulls as usual and writes each P_j back to the address g_opp(j) came from, i.e. into
// slot opp(j) of the node x + e_j; step 2 (local) reads g_j from the node's own slot opp(j) and writes
// P_j to slot j, which restores the standard state.  A thread reads and writes only its own set of
// addresses in either step, so no two threads touch one address.
template <int MODE, int AUX, bool HAS_K, bool HAS_S, int BC = 0, bool MRT = false, int ROWS = 0, bool CST = false,
          int IP = 0>
__device__ __forceinline__ void process_tile(const InstDesc &a, int parity, int t, int wave)
{
    using St = typename ModeTraits<MODE>::St;
    using M = typename ModeTraits<MODE>::M;
    using T = typename St::T;
    using C = Codec<St, M>;
    const int nx = a.L.nx, ny = a.L.ny;
    const int64_t pitch = a.L.pitch;
    const int rows = ROWS > 0 ? ROWS : a.lc.rows;
    int x0, y0;
    tile_origin(a.L, a.lc, t, wave, x0, y0);
    if (y0 >= ny || x0 >= nx) return;
    const int64_t level = launch_level<C>(a, parity) + 1;  // time level written (stochastic rounding)
    advance_level<C>(a, parity, level - 1, 1, t == 0 && wave == 0 && threadIdx.x == 0);
    const unsigned x = (unsigned)x0 + threadIdx.x;
    const bool live = x < (unsigned)nx;
    const unsigned xc = live ? x : 0u;  // dead lanes of a ragged tile read column 0 and store nothing
    const unsigned xm = xc == 0 ? (unsigned)nx - 1 : xc - 1;
    const unsigned xp = xc == (unsigned)nx - 1 ? 0u : xc + 1;
    const int y1 = min(y0 + rows, ny);
    // in place, source and destination are one buffer: no restrict on the population pointers
    using SrcP = std::conditional_t<IP == 0, const T *__restrict__, const T *>;
    using DstP = std::conditional_t<IP == 0, T *__restrict__, T *>;
    const SrcP src = static_cast<const T *>(a.buf[parity]);
    const DstP dst = static_cast<T *>(a.buf[parity ^ 1]);
    const M *__restrict__ u = static_cast<const M *>(a.u);
    const M *__restrict__ kf = static_cast<const M *>(a.k);
    const M *__restrict__ sf = static_cast<const M *>(a.s);
    const M lam = (M)a.lambda;
    Relax<M> rconst;
    rconst.w1 = (M)a.w1;
    rconst.w2 = (M)a.w2;
    rconst.beta = (M)a.beta;
    rconst.w3 = (M)a.w3;

    // velocity in this column at rows y-1 and y, rolled down the walk
    const int yprev = wrap_dec(y0, ny);
    const M *__restrict__ u_m = u + (int64_t)yprev * 2 * pitch;
    const M *__restrict__ u_c = u + (int64_t)y0 * 2 * pitch;
    // byte offsets of columns x, x-1, x+1 for population and field element sizes
    const unsigned bc = xc * (unsigned)sizeof(T), bm = xm * (unsigned)sizeof(T), bp = xp * (unsigned)sizeof(T);
    const unsigned fc = xc * (unsigned)sizeof(M), fm = xm * (unsigned)sizeof(M), fp = xp * (unsigned)sizeof(M);
    M ux_m = ld_at(u_m, fc), uy_m = ld_at(u_m + pitch, fc);
    M ux_c = ld_at(u_c, fc), uy_c = ld_at(u_c + pitch, fc);

    for (int y = y0; y < y1; ++y) {
        const int ym = wrap_dec(y, ny), yn = wrap_inc(y, ny);
        const SrcP rm = src + (int64_t)ym * 9 * pitch;
        const SrcP rc = src + (int64_t)y * 9 * pitch;
        const SrcP rp = src + (int64_t)yn * 9 * pitch;
        M g[9];
        if constexpr (IP == 2) {
#pragma unroll
            for (int i = 0; i < 9; ++i) g[i] = C::dec(ld_at(rc + kOpp[i] * pitch, bc), i, a.f16);
        } else {
            g[0] = C::dec(ld_at(rc, bc), 0, a.f16);
            g[1] = C::dec(ld_at(rc + pitch, bm), 1, a.f16);
            g[2] = C::dec(ld_at(rm + 2 * pitch, bc), 2, a.f16);
            g[3] = C::dec(ld_at(rc + 3 * pitch, bp), 3, a.f16);
            g[4] = C::dec(ld_at(rp + 4 * pitch, bc), 4, a.f16);
            g[5] = C::dec(ld_at(rm + 5 * pitch, bm), 5, a.f16);
            g[6] = C::dec(ld_at(rm + 6 * pitch, bp), 6, a.f16);
            g[7] = C::dec(ld_at(rp + 7 * pitch, bp), 7, a.f16);
            g[8] = C::dec(ld_at(rp + 8 * pitch, bm), 8, a.f16);
        }
        if constexpr (BC == 1) {
            if (y == 0 || y == ny - 1 || xc == 0 || xc == (unsigned)nx - 1)
                nee_replace<St, M>(src, u, static_cast<const M *>(a.bc), a.L, (int)xc, y, a.f16, g);
        } else if constexpr (BC == 2) {
            if (y == 0 || y == ny - 1)
                wall_replace<St, M>(rc, bc, ld_at(static_cast<const M *>(a.bc) + (int64_t)y * pitch, fc), ux_c, uy_c,
                                    y == 0, a.f16, pitch, g);
        }
        const M *__restrict__ un = u + (int64_t)yn * 2 * pitch;
        const M *__restrict__ uc = u + (int64_t)y * 2 * pitch;
        const M ux_p = ld_at(un, fc), uy_p = ld_at(un + pitch, fc);

        M Ax = M(0), Ay = M(0);
        if (AUX == 0) {  // Eq. (16): phi u_b d_b u_a, central differences of u
            const M phi = g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8];
            // across a Dirichlet edge the difference is one-sided (the wrapped neighbour is not adjacent)
            unsigned fl = fm, fr = fp;
            M hx = M(0.5), hy = M(0.5), uxl = ux_m, uyl = uy_m, uxr = ux_p, uyr = uy_p;
            if constexpr (BC == 1) {
                if (xc == 0) { fl = fc; hx = M(1); } else if (xc == (unsigned)nx - 1) { fr = fc; hx = M(1); }
            }
            if constexpr (BC != 0) {
                if (y == 0) { uxl = ux_c; uyl = uy_c; hy = M(1); }
                else if (y == ny - 1) { uxr = ux_c; uyr = uy_c; hy = M(1); }
            }
            const M dxux = (ld_at(uc, fr) - ld_at(uc, fl)) * hx;
            const M dxuy = (ld_at(uc + pitch, fr) - ld_at(uc + pitch, fl)) * hx;
            const M dyux = (uxr - uxl) * hy;
            const M dyuy = (uyr - uyl) * hy;
            Ax = phi * (ux_c * dxux + uy_c * dyux);
            Ay = phi * (ux_c * dxuy + uy_c * dyuy);
        }
        const Relax<M> r = HAS_K ? relax_from_k<M>(ld_at(kf + (int64_t)y * pitch, fc), lam, rconst.w3) : rconst;
        const M s = HAS_S ? ld_at(sf + (int64_t)y * pitch, fc) : M(0);
        M P[9];
        collide<M, MRT>(g, ux_c, uy_c, r, Ax, Ay, s, P);
        const auto rb = C::bits(a.f16, level, (int64_t)y * nx, xc);
        if (live && IP == 1) {
            // P_j to the address of g_opp(j): slot opp(j) of node x + e_j (every value is a function of
            // all nine loads, so no store can move ahead of them)
            T *wm = dst + (int64_t)ym * 9 * pitch, *wc = dst + (int64_t)y * 9 * pitch, *wp = dst + (int64_t)yn * 9 * pitch;
            st_at(wc, bc, C::enc(P[0], 0, a.f16, rb));
            st_at(wc + 3 * pitch, bp, C::enc(P[1], 1, a.f16, rb));
            st_at(wp + 4 * pitch, bc, C::enc(P[2], 2, a.f16, rb));
            st_at(wc + pitch, bm, C::enc(P[3], 3, a.f16, rb));
            st_at(wm + 2 * pitch, bc, C::enc(P[4], 4, a.f16, rb));
            st_at(wp + 7 * pitch, bp, C::enc(P[5], 5, a.f16, rb));
            st_at(wp + 8 * pitch, bm, C::enc(P[6], 6, a.f16, rb));
            st_at(wm + 5 * pitch, bm, C::enc(P[7], 7, a.f16, rb));
            st_at(wm + 6 * pitch, bp, C::enc(P[8], 8, a.f16, rb));
        } else if (live) {
            // one scalar row base and 32-bit lane offsets keep every store in the saddr form
            const DstP out = dst + (int64_t)y * 9 * pitch;
            const unsigned pb = (unsigned)(pitch * (int64_t)sizeof(T));
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if constexpr (CST || IP != 0) st_at(out, bc + (unsigned)i * pb, C::enc(P[i], i, a.f16, rb));
                else st_nt_at(out, bc + (unsigned)i * pb, C::enc(P[i], i, a.f16, rb));
            }
        }
        ux_m = ux_c;
        uy_m = uy_c;
        ux_c = ux_p;
        uy_c = uy_p;
    }
}

// One tile of one step with the flux form of the auxiliary term, which needs phi at the four axis
// neighbours at the same time level.  The walk down the rows is software-pipelined: the pull of row
// y+1 gives both the next node's populations and phi(x, y+1), phi(x, y-1) is kept from the previous
// row, and phi(x-1, y), phi(x+1, y) come from the neighbouring lanes (wave shuffles).  The two halo
// nodes just outside the wave (west of its first lane, east of its last live lane, wrapped at the
// periodic seam) are pulled cooperatively: lanes 0-8 load the nine populations of the west node and
// lanes 9-17 those of the east node in one gather, and their sums come back by lane reads, in the
// same order as every other phi.
template <int MODE, bool HAS_K, bool HAS_S, bool MRT = false, bool CST = false>
__device__ __forceinline__ void process_tile_flux(const InstDesc &a, int parity, int t, int wave)
{
    using St = typename ModeTraits<MODE>::St;
    using M = typename ModeTraits<MODE>::M;
    using T = typename St::T;
    using C = Codec<St, M>;
    const int nx = a.L.nx, ny = a.L.ny;
    const int64_t pitch = a.L.pitch;
    const int rows = a.lc.rows;
    const unsigned lane = threadIdx.x;
    int x0t, y0;  // the wave's first column and first row
    tile_origin(a.L, a.lc, t, wave, x0t, y0);
    if (y0 >= ny || x0t >= nx) return;
    const int64_t level = launch_level<C>(a, parity) + 1;  // time level written (stochastic rounding)
    advance_level<C>(a, parity, level - 1, 1, t == 0 && wave == 0 && lane == 0);
    const unsigned x = (unsigned)x0t + lane;
    const bool live = x < (unsigned)nx;
    const unsigned xc = live ? x : 0u;
    const unsigned xm = xc == 0 ? (unsigned)nx - 1 : xc - 1;
    const unsigned xp = xc == (unsigned)nx - 1 ? 0u : xc + 1;
    // byte offsets of columns x, x-1, x+1 (population and field element sizes): scalar bases + 32-bit offsets
    const unsigned bc = xc * (unsigned)sizeof(T), bm = xm * (unsigned)sizeof(T), bp = xp * (unsigned)sizeof(T);
    const unsigned fc = xc * (unsigned)sizeof(M), fm = xm * (unsigned)sizeof(M), fp = xp * (unsigned)sizeof(M);
    const int y1 = min(y0 + rows, ny);
    // halo gather set-up: lane l < 18 loads population l % 9 of the west (l < 9) or east halo node
    const int last = min(63, nx - 1 - x0t);              // last live lane of this wave
    const int xw = x0t == 0 ? nx - 1 : x0t - 1;           // west halo column
    const int xe = x0t + last + 1 == nx ? 0 : x0t + last + 1;  // east halo column
    const int hi = (int)(lane % 9u);
    const int hex = hi == 1 || hi == 5 || hi == 8 ? 1 : (hi == 3 || hi == 6 || hi == 7 ? -1 : 0);
    const int hey = hi == 2 || hi == 5 || hi == 6 ? 1 : (hi == 4 || hi == 7 || hi == 8 ? -1 : 0);
    int hxs = (lane < 9u ? xw : xe) - hex;
    hxs = hxs < 0 ? hxs + nx : (hxs >= nx ? hxs - nx : hxs);
    M hwref = M(0);
    if constexpr (is_f16_mode(MODE)) {
        const F16Params &f = a.f16;
        hwref = hi == 0 ? f.wref[0] : hi == 1 ? f.wref[1] : hi == 2 ? f.wref[2] : hi == 3 ? f.wref[3]
              : hi == 4 ? f.wref[4] : hi == 5 ? f.wref[5] : hi == 6 ? f.wref[6] : hi == 7 ? f.wref[7] : f.wref[8];
    }
    const T *__restrict__ src = static_cast<const T *>(a.buf[parity]);
    T *__restrict__ dst = static_cast<T *>(a.buf[parity ^ 1]);
    const M *__restrict__ u = static_cast<const M *>(a.u);
    const M *__restrict__ kf = static_cast<const M *>(a.k);
    const M *__restrict__ sf = static_cast<const M *>(a.s);
    const M lam = (M)a.lambda;
    Relax<M> rconst;
    rconst.w1 = (M)a.w1;
    rconst.w2 = (M)a.w2;
    rconst.beta = (M)a.beta;
    rconst.w3 = (M)a.w3;
    auto row_pull = [&](int yy, M (&g)[9]) {
        const T *__restrict__ rm = src + (int64_t)wrap_dec(yy, ny) * 9 * pitch;
        const T *__restrict__ rc = src + (int64_t)yy * 9 * pitch;
        const T *__restrict__ rp = src + (int64_t)wrap_inc(yy, ny) * 9 * pitch;
        g[0] = C::dec(ld_at(rc, bc), 0, a.f16);
        g[1] = C::dec(ld_at(rc + pitch, bm), 1, a.f16);
        g[2] = C::dec(ld_at(rm + 2 * pitch, bc), 2, a.f16);
        g[3] = C::dec(ld_at(rc + 3 * pitch, bp), 3, a.f16);
        g[4] = C::dec(ld_at(rp + 4 * pitch, bc), 4, a.f16);
        g[5] = C::dec(ld_at(rm + 5 * pitch, bm), 5, a.f16);
        g[6] = C::dec(ld_at(rm + 6 * pitch, bp), 6, a.f16);
        g[7] = C::dec(ld_at(rp + 7 * pitch, bp), 7, a.f16);
        g[8] = C::dec(ld_at(rp + 8 * pitch, bm), 8, a.f16);
    };
    auto sum9 = [](const M (&g)[9]) { return g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8]; };

    M g[9], gn[9];
    row_pull(y0, g);
    M phi_c = sum9(g);
    M phi_m;
    {
        M gm[9];
        row_pull(wrap_dec(y0, ny), gm);
        phi_m = sum9(gm);
    }
    const int yprev = wrap_dec(y0, ny);
    M ux_m = ld_at(u + (int64_t)yprev * 2 * pitch, fc), uy_m = ld_at(u + ((int64_t)yprev * 2 + 1) * pitch, fc);
    M ux_c = ld_at(u + (int64_t)y0 * 2 * pitch, fc), uy_c = ld_at(u + ((int64_t)y0 * 2 + 1) * pitch, fc);
    for (int y = y0; y < y1; ++y) {
        const int yn = wrap_inc(y, ny);
        row_pull(yn, gn);
        const M phi_p = sum9(gn);
        const M *__restrict__ uc = u + (int64_t)y * 2 * pitch;
        const M *__restrict__ un = u + (int64_t)yn * 2 * pitch;
        const M ux_p = ld_at(un, fc), uy_p = ld_at(un + pitch, fc);
        M pw = __shfl_up(phi_c, 1, 64), pe = __shfl_down(phi_c, 1, 64);
        {
            int hys = y - hey;
            hys = hys < 0 ? hys + ny : (hys >= ny ? hys - ny : hys);
            M hv = M(0);
            if (lane < 18u) {
                const T raw = src[((int64_t)hys * 9 + hi) * pitch + hxs];
                if constexpr (is_f16_mode(MODE)) hv = (float)raw * a.f16.inv_scale + hwref;
                else hv = C::dec(raw, 0, a.f16);
            }
            M phw = lane_read<M>(hv, 0), phe = lane_read<M>(hv, 9);
#pragma unroll
            for (int k = 1; k < 9; ++k) {
                phw += lane_read<M>(hv, k);
                phe += lane_read<M>(hv, 9 + k);
            }
            if (lane == 0u) pw = phw;
            if ((int)lane == last) pe = phe;
        }
        const M uxw = ld_at(uc, fm), uyw = ld_at(uc + pitch, fm), uxe = ld_at(uc, fp), uye = ld_at(uc + pitch, fp);
        M Ax, Ay;
        flux_aux<M>(pw, pe, phi_m, phi_p, uxw, uyw, uxe, uye, ux_m, uy_m, ux_p, uy_p, ux_c, uy_c, Ax, Ay);
        const Relax<M> r = HAS_K ? relax_from_k<M>(ld_at(kf + (int64_t)y * pitch, fc), lam, rconst.w3) : rconst;
        const M s = HAS_S ? ld_at(sf + (int64_t)y * pitch, fc) : M(0);
        M P[9];
        collide<M, MRT>(g, ux_c, uy_c, r, Ax, Ay, s, P);
        if (live) {
            T *__restrict__ out = dst + (int64_t)y * 9 * pitch;
            const unsigned pb = (unsigned)(pitch * (int64_t)sizeof(T));
            const auto rb = C::bits(a.f16, level, (int64_t)y * nx, xc);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if constexpr (CST) st_at(out, bc + (unsigned)i * pb, C::enc(P[i], i, a.f16, rb));
                else st_nt_at(out, bc + (unsigned)i * pb, C::enc(P[i], i, a.f16, rb));
            }
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = gn[i];
        phi_m = phi_c;
        phi_c = phi_p;
        ux_m = ux_c;
        uy_m = uy_c;
        ux_c = ux_p;
        uy_c = uy_p;
    }
}

// Dispatch of one tile to the aux-term form.
template <int MODE, int AUX, bool HAS_K, bool HAS_S, int BC = 0, bool MRT = false, int ROWS = 0, bool CST = false,
          int IP = 0>
__device__ __forceinline__ void run_tile(const InstDesc &d, int parity, int t, int wave)
{
    if constexpr (AUX == 1) process_tile_flux<MODE, HAS_K, HAS_S, MRT, CST>(d, parity, t, wave);
    else process_tile<MODE, AUX, HAS_K, HAS_S, BC, MRT, ROWS, CST, IP>(d, parity, t, wave);
}

// Single instance: block b -> tile (XCD-remapped if requested).
template <int MODE, int AUX, bool HAS_K, bool HAS_S, int BC, bool MRT, int ROWS, bool CST, int IP>
__global__ __launch_bounds__(256) void step_kernel(const StepArgs a)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int t = tile_of_block(blockIdx.x, gridDim.x, a.d.lc.xcd_remap, tiles_per_row(a.d.L, a.d.lc), a.d.lc.xcd_rows);
    run_tile<MODE, AUX, HAS_K, HAS_S, BC, MRT, ROWS, CST, IP>(a.d, a.parity, t, wave);
}

// Many instances in one launch: each block runs a range of (instance, tile) work items; the
// instance descriptor is wave-uniform and read with scalar loads.
template <int MODE, int AUX, int ROWS>
__global__ __launch_bounds__(256) void batched_step_kernel(const BatchArgs a)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
    int beg, end;
    if (a.block_start) {
        beg = a.block_start[blockIdx.x];
        end = a.block_start[blockIdx.x + 1];
    } else {
        beg = tile_of_block(blockIdx.x, gridDim.x, 1, 0, 0);
        end = beg + 1;
    }
    for (int it = beg; it < end; ++it) {
        const WorkItem w = a.items[it];
        const InstDesc &d = a.inst[w.inst];
        if (d.has_k) {
            if (d.has_s) run_tile<MODE, AUX, true, true, 0, false, ROWS>(d, a.parity, w.tile, wave);
            else run_tile<MODE, AUX, true, false, 0, false, ROWS>(d, a.parity, w.tile, wave);
        } else {
            if (d.has_s) run_tile<MODE, AUX, false, true, 0, false, ROWS>(d, a.parity, w.tile, wave);
            else run_tile<MODE, AUX, false, false, 0, false, ROWS>(d, a.parity, w.tile, wave);
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(256) void init_kernel(const InitArgs a)
{
    using St = typename ModeTraits<MODE>::St;
    using M = typename ModeTraits<MODE>::M;
    using T = typename St::T;
    using C = Codec<St, M>;
    const int nx = a.L.nx, ny = a.L.ny;
    const int64_t N = (int64_t)nx * ny, pitch = a.L.pitch;
    T *dst = static_cast<T *>(a.dst);
    const M *u = static_cast<const M *>(a.u);
    bool bad = false;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(n % nx), y = (int)(n / nx);
        M P[9];
        equilibrium<M>((M)a.phi0[n], u[(int64_t)y * 2 * pitch + x], u[((int64_t)y * 2 + 1) * pitch + x], P);
        const auto rb = C::bits(a.f16, 0, (int64_t)y * nx, (unsigned)x);  // time level 0
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int xd = x - kEx[i], yd = y - kEy[i];
            xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
            const bool across = yd < 0 || yd >= ny;
            yd = yd < 0 ? yd + ny : (yd >= ny ? yd - ny : yd);
            if (is_f16_mode(MODE)) {
                const float v = ((float)P[i] - a.f16.wref[i]) * a.f16.scale;
                bad |= !(fabsf(v) <= 65504.0f);
            }
            if (a.walls && across) {
                // No node lies beyond the wall.  Instead this node's own slot of the opposite,
                // wall-bound direction (read only by the reflection) takes g_eq_opp(i), so that the
                // reflection returns g_eq_i while the wall value is phi0's.
                const int o = kOpp[i];
                dst[((int64_t)y * 9 + o) * pitch + x] = C::enc(P[o], o, a.f16, rb);
                continue;
            }
            dst[((int64_t)yd * 9 + i) * pitch + xd] = C::enc(P[i], i, a.f16, rb);
        }
    }
    if (bad) *a.range_flag = 1;  // every writer stores the same value
}

template <class M>
__global__ __launch_bounds__(256) void prep_kernel(const PrepArgs a)
{
    const int nx = a.L.nx;
    const int64_t N = (int64_t)nx * rows_of(a.L);
    M *out = static_cast<M *>(a.out);
    bool bad = false;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(n % nx);
        const int64_t y = n / nx;  // row: y, or z*ny + y on D3Q19
        double v = a.ca * a.a[n];
        if (a.b) v += a.cb * a.b[n];
        if (a.check_positive) bad |= !(v > 0.0 && v < INFINITY);
        out[((int64_t)y * a.stride + a.comp) * a.L.pitch + x] = (M)v;
    }
    if (bad) *a.flag = 1;  // every writer stores the same value
}

// ---- diagnostics -------------------------------------------------------------------------------

template <int MODE>
__global__ __launch_bounds__(256) void macros_kernel(const MacroArgs a)
{
    using St = typename ModeTraits<MODE>::St;
    using M = typename ModeTraits<MODE>::M;
    using T = typename St::T;
    const int nx = a.L.nx, ny = a.L.ny;
    const int64_t N = (int64_t)nx * ny;
    const T *src = static_cast<const T *>(a.src);
    CSum cs[3] = {{0, 0}, {0, 0}, {0, 0}};  // mass, sum err^2, sum ref^2
    double maxerr = 0, maxphi = 0, nonfinite = 0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(n % nx), y = (int)(n / nx);
        M g[9];
        state_node<St, M>(src, a.edge, a.L, x, y, a.f16, g);
        double phi = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) phi += (double)g[i];
        if (a.phi_out) a.phi_out[n] = phi;
        if (!isfinite(phi)) {
            nonfinite += 1;
            continue;
        }
        csum_add(cs[0], phi);
        maxphi = fmax(maxphi, fabs(phi));
        if (a.ref) {
            const double r = a.ref[n], d = phi - r;
            csum_add(cs[1], d * d);
            csum_add(cs[2], r * r);
            maxerr = fmax(maxerr, fabs(d));
        }
    }
    block_reduce(cs, maxerr, maxphi, nonfinite);
    if (threadIdx.x == 0) {
        double *p = a.partials + (int64_t)blockIdx.x * kMacroPartialDoubles;
        for (int k = 0; k < 3; ++k) {
            p[2 * k] = cs[k].s;
            p[2 * k + 1] = cs[k].c;
        }
        p[6] = maxerr;
        p[7] = maxphi;
        p[8] = nonfinite;
    }
}

// Single block: merges the per-block partials; result[0..2] = mass, sum err^2, sum ref^2 (s + c),
// result[3] = max err, result[4] = max |phi|, result[5] = non-finite count.
__global__ __launch_bounds__(256) void macros_finalize(const double *partials, int nblocks, double *result)
{
    CSum cs[3] = {{0, 0}, {0, 0}, {0, 0}};
    double mx0 = 0, mx1 = 0, cnt = 0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        const double *p = partials + (int64_t)b * kMacroPartialDoubles;
        for (int k = 0; k < 3; ++k) cs[k] = csum_merge(cs[k], CSum{p[2 * k], p[2 * k + 1]});
        mx0 = fmax(mx0, p[6]);
        mx1 = fmax(mx1, p[7]);
        cnt += p[8];
    }
    block_reduce(cs, mx0, mx1, cnt);
    if (threadIdx.x == 0) {
        for (int k = 0; k < 3; ++k) result[k] = cs[k].s + cs[k].c;
        result[3] = mx0;
        result[4] = mx1;
        result[5] = cnt;
    }
}

template <int MODE>
__global__ __launch_bounds__(256) void populations_kernel(const PopArgs a)
{
    using St = typename ModeTraits<MODE>::St;
    using M = typename ModeTraits<MODE>::M;
    using T = typename St::T;
    const int nx = a.L.nx, ny = a.L.ny;
    const int64_t N = (int64_t)nx * ny;
    const T *src = static_cast<const T *>(a.src);
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(n % nx), y = (int)(n / nx);
        M g[9];
        state_node<St, M>(src, a.edge, a.L, x, y, a.f16, g);
#pragma unroll
        for (int i = 0; i < 9; ++i) a.out[i * N + n] = (double)g[i];
    }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Bandwidth reference: a 16-byte-per-lane copy with non-temporal loads and stores, the fastest of the
// copy forms measured on MI355X (6.6 TB/s at 2 GiB; 6.3 with cached loads, 5.6-5.9 unrolled or
// grid-stride).
__global__ __launch_bounds__(256) void copy_kernel(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// The same copy with the default cache policy: buffers that fit in the 256 MiB Infinity Cache stay
// there across repetitions, so it measures the rate a cache-resident step can reach.
__global__ __launch_bounds__(256) void copy_cached_kernel(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst,
                                                          int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Between the standard state (slot j of node z holds P_j(z)) and the one-buffer state after its
// streaming step (P_j(z) in slot opp(j) of node z + e_j): dst[z][j] = src[z + e_j][opp(j)], a map that
// is its own inverse.  Raw storage elements (E: their size); padding columns are written as zero.
template <class E>
__global__ __launch_bounds__(256) void relayout_kernel(const E *__restrict__ src, E *__restrict__ dst, Layout L)
{
    const int64_t n = (int64_t)L.ny * L.pitch;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(k % L.pitch), y = (int)(k / L.pitch);
        const bool live = x < L.nx;
        const int xm = x == 0 ? L.nx - 1 : x - 1, xp = x == L.nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? L.ny - 1 : y - 1, yp = y == L.ny - 1 ? 0 : y + 1;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int xs = kEx[j] < 0 ? xm : (kEx[j] > 0 ? xp : x);
            const int ys = kEy[j] < 0 ? ym : (kEy[j] > 0 ? yp : y);
            dst[((int64_t)y * 9 + j) * L.pitch + x] = live ? src[((int64_t)ys * 9 + kOpp[j]) * L.pitch + xs] : E(0);
        }
    }
}


template <int MODE, int AUX, int BC, bool MRT, int ROWS, bool CST = false, int IP = 0>
hipError_t launch_step_rows(const StepArgs &a, hipStream_t st)
{
    dim3 block(64, 4);
    const int nblocks = tiles_of(a.d.L, a.d.lc.rows, a.d.lc.wide);
    const size_t lds = (size_t)a.d.lc.lds_reserve;  // unused LDS that caps the resident waves
    const bool hk = a.d.has_k, hs = a.d.has_s;
    if (hk && hs) step_kernel<MODE, AUX, true, true, BC, MRT, ROWS, CST, IP><<<nblocks, block, lds, st>>>(a);
    else if (hk) step_kernel<MODE, AUX, true, false, BC, MRT, ROWS, CST, IP><<<nblocks, block, lds, st>>>(a);
    else if (hs) step_kernel<MODE, AUX, false, true, BC, MRT, ROWS, CST, IP><<<nblocks, block, lds, st>>>(a);
    else step_kernel<MODE, AUX, false, false, BC, MRT, ROWS, CST, IP><<<nblocks, block, lds, st>>>(a);
    return hipGetLastError();
}

// The local/no-aux kernels (periodic, Dirichlet edges, walls; TRT-R and MRT-R) have a one-row
// instantiation for the default shape: with no loop left, every load keeps the scalar-base +
// 32-bit-offset form (the walking loop's strength-reduced 64-bit vector addresses cost ~160
// instructions and ~28 VGPRs per wave); every other shape walks the launch's row count.  The one-row
// kernels and the flux form come with non-temporal or cached stores (Launch::stores; a compile-time
// choice: a run-time branch between two store loops that differ only in the hint is merged by the
// compiler, which drops the hint); the walking loop of the local form stores non-temporally.
template <int MODE, int AUX, int BC, bool MRT>
hipError_t launch_step_var(const StepArgs &a, hipStream_t st)
{
    if constexpr (AUX == 1) {
        return a.d.lc.stores ? launch_step_rows<MODE, AUX, BC, MRT, 0, true>(a, st)
                             : launch_step_rows<MODE, AUX, BC, MRT, 0, false>(a, st);
    } else {
        if constexpr (BC == 0) {  // one buffer in place (stores == 2): alternate the two steps
            if (a.d.lc.stores == 2) {
                if (a.d.lc.rows != 1) return hipErrorInvalidValue;
                return a.parity == 0 ? launch_step_rows<MODE, AUX, BC, MRT, 1, true, 1>(a, st)
                                     : launch_step_rows<MODE, AUX, BC, MRT, 1, true, 2>(a, st);
            }
        }
        if (a.d.lc.rows == 1)
            return a.d.lc.stores ? launch_step_rows<MODE, AUX, BC, MRT, 1, true>(a, st)
                                 : launch_step_rows<MODE, AUX, BC, MRT, 1, false>(a, st);
        return launch_step_rows<MODE, AUX, BC, MRT, 0>(a, st);
    }
}

// MRT-R (w3 != 0) is a separate instantiation so that the TRT-R kernels keep their registers.
template <int MODE, int AUX, int BC>
hipError_t launch_step_bc(const StepArgs &a, hipStream_t st)
{
    return a.d.w3 != 0.0 ? launch_step_var<MODE, AUX, BC, true>(a, st) : launch_step_var<MODE, AUX, BC, false>(a, st);
}

template <int MODE, int AUX>
hipError_t launch_step_aux(const StepArgs &a, hipStream_t st)
{
    if constexpr (AUX == 1) {
        if (a.d.bckind != 0) return hipErrorInvalidValue;  // the flux form is periodic only
        return launch_step_bc<MODE, AUX, 0>(a, st);
    } else {
        switch (a.d.bckind) {
        case 0: return launch_step_bc<MODE, AUX, 0>(a, st);
        case 1: return launch_step_bc<MODE, AUX, 1>(a, st);
        case 2: return launch_step_bc<MODE, AUX, 2>(a, st);
        default: return hipErrorInvalidValue;
        }
    }
}

template <int MODE>
hipError_t launch_step_mode(int aux, const StepArgs &a, hipStream_t st)
{
    switch (aux) {
    case 0: return launch_step_aux<MODE, 0>(a, st);
    case 1: return launch_step_aux<MODE, 1>(a, st);
    default: return launch_step_aux<MODE, 2>(a, st);
    }
}

template <int MODE>
hipError_t launch_batched_mode(int aux, const BatchArgs &a, int nblocks, size_t lds, hipStream_t st)
{
    dim3 block(64, 4);  // lds: unused LDS that caps the resident waves
    switch (aux) {
    case 0:
        if (a.one_row) batched_step_kernel<MODE, 0, 1><<<nblocks, block, lds, st>>>(a);
        else batched_step_kernel<MODE, 0, 0><<<nblocks, block, lds, st>>>(a);
        break;
    case 1: batched_step_kernel<MODE, 1, 0><<<nblocks, block, lds, st>>>(a); break;
    default:
        if (a.one_row) batched_step_kernel<MODE, 2, 1><<<nblocks, block, lds, st>>>(a);
        else batched_step_kernel<MODE, 2, 0><<<nblocks, block, lds, st>>>(a);
        break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step(int mode, int aux, const StepArgs &a, hipStream_t st)
{
    if (a.d.lc.rows < 1 || a.d.lc.rows > 64 || a.d.lc.lds_reserve < 0 || a.d.lc.lds_reserve > 65536)
        return hipErrorInvalidValue;
    switch (mode) {
    case MODE_F64_F64: return launch_step_mode<MODE_F64_F64>(aux, a, st);
    case MODE_F64_F32: return launch_step_mode<MODE_F64_F32>(aux, a, st);
    case MODE_F32_F32: return launch_step_mode<MODE_F32_F32>(aux, a, st);
    case MODE_F16S_F32: return launch_step_mode<MODE_F16S_F32>(aux, a, st);
    case MODE_F16SR_F32: return launch_step_mode<MODE_F16SR_F32>(aux, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batched_step(int mode, int aux, const BatchArgs &a, int nblocks, int lds_reserve, hipStream_t st)
{
    if (nblocks < 1 || lds_reserve < 0 || lds_reserve > 65536) return hipErrorInvalidValue;
    const size_t lds = (size_t)lds_reserve;
    switch (mode) {
    case MODE_F64_F64: return launch_batched_mode<MODE_F64_F64>(aux, a, nblocks, lds, st);
    case MODE_F64_F32: return launch_batched_mode<MODE_F64_F32>(aux, a, nblocks, lds, st);
    case MODE_F32_F32: return launch_batched_mode<MODE_F32_F32>(aux, a, nblocks, lds, st);
    case MODE_F16S_F32: return launch_batched_mode<MODE_F16S_F32>(aux, a, nblocks, lds, st);
    case MODE_F16SR_F32: return launch_batched_mode<MODE_F16SR_F32>(aux, a, nblocks, lds, st);
    default: return hipErrorInvalidValue;
    }
}

namespace {
__global__ void set_clock_kernel(int64_t *slot, int64_t level)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *slot = level;
}
}  // namespace

hipError_t launch_set_clock(int64_t *slot, int64_t level, hipStream_t st)
{
    if (!slot || level < 0) return hipErrorInvalidValue;
    set_clock_kernel<<<1, 64, 0, st>>>(slot, level);
    return hipGetLastError();
}

hipError_t launch_init(int mode, const InitArgs &a, hipStream_t st)
{
    const int g = grid_for((int64_t)a.L.nx * a.L.ny, 256, 8192);
    switch (mode) {
    case MODE_F64_F64: init_kernel<MODE_F64_F64><<<g, 256, 0, st>>>(a); break;
    case MODE_F64_F32: init_kernel<MODE_F64_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F32_F32: init_kernel<MODE_F32_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F16S_F32: init_kernel<MODE_F16S_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F16SR_F32: init_kernel<MODE_F16SR_F32><<<g, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_prep(int mode, const PrepArgs &a, hipStream_t st)
{
    const int g = grid_for((int64_t)a.L.nx * rows_of(a.L), 256, 8192);
    if (mode == MODE_F64_F64) prep_kernel<double><<<g, 256, 0, st>>>(a);
    else prep_kernel<float><<<g, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_macros(int mode, const MacroArgs &a, double *result, hipStream_t st)
{
    const int g = grid_for((int64_t)a.L.nx * a.L.ny, 256, kMacroBlocks);
    switch (mode) {
    case MODE_F64_F64: macros_kernel<MODE_F64_F64><<<g, 256, 0, st>>>(a); break;
    case MODE_F64_F32: macros_kernel<MODE_F64_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F32_F32: macros_kernel<MODE_F32_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F16S_F32:
    case MODE_F16SR_F32: macros_kernel<MODE_F16S_F32><<<g, 256, 0, st>>>(a); break;  // one code format
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_macros_finalize(a.partials, g, result, st);
}

hipError_t launch_macros_finalize(const double *partials, int nblocks, double *result, hipStream_t st)
{
    macros_finalize<<<1, 256, 0, st>>>(partials, nblocks, result);
    return hipGetLastError();
}

hipError_t launch_populations(int mode, const PopArgs &a, hipStream_t st)
{
    const int g = grid_for((int64_t)a.L.nx * a.L.ny, 256, 8192);
    switch (mode) {
    case MODE_F64_F64: populations_kernel<MODE_F64_F64><<<g, 256, 0, st>>>(a); break;
    case MODE_F64_F32: populations_kernel<MODE_F64_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F32_F32: populations_kernel<MODE_F32_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F16S_F32:
    case MODE_F16SR_F32: populations_kernel<MODE_F16S_F32><<<g, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_relayout(size_t elem_bytes, const void *src, void *dst, const Layout &L, hipStream_t st)
{
    if (L.q != 9 || src == dst) return hipErrorInvalidValue;
    const int g = grid_for((int64_t)L.ny * L.pitch, 256, 8192);
    switch (elem_bytes) {
    case 2: relayout_kernel<uint16_t><<<g, 256, 0, st>>>(static_cast<const uint16_t *>(src), static_cast<uint16_t *>(dst), L); break;
    case 4: relayout_kernel<uint32_t><<<g, 256, 0, st>>>(static_cast<const uint32_t *>(src), static_cast<uint32_t *>(dst), L); break;
    case 8: relayout_kernel<uint64_t><<<g, 256, 0, st>>>(static_cast<const uint64_t *>(src), static_cast<uint64_t *>(dst), L); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, bool cached, hipStream_t st)
{
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (cached)
        copy_cached_kernel<<<(unsigned)blocks, 256, 0, st>>>(static_cast<const f32x4 *>(src), static_cast<f32x4 *>(dst), n);
    else
        copy_kernel<<<(unsigned)blocks, 256, 0, st>>>(static_cast<const f32x4 *>(src), static_cast<f32x4 *>(dst), n);
    return hipGetLastError();
}

}  // namespace lbm
