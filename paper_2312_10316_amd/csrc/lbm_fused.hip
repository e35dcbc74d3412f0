// lbm_fused.hip -- two time steps of the D2Q9 TRT-R update per launch (temporal blocking, gfx950): a
// block walks its tile row by row and passes the intermediate state through an LDS ring.
//
// A step is bound by memory traffic: every population is read once and written once per step
// (Sec. 2.2, Eq. (14) pulls nine values and stores nine).  Fusing two steps halves that traffic: a
// block reads the state at t_n for its tile plus a halo, computes the intermediate state t_{n+1} of
// the tile and a one-node frame around it into LDS, and writes only the state at t_{n+2}.  Every node
// of both steps is evaluated by the same per-node arithmetic as the single-step kernel (the same
// inlined collision), and the intermediate populations go through the storage codec exactly as if
// they had been written to and read back from memory, so two fused steps are bitwise two single
// steps.
//
// Block: NW "interior" waves (lane = column, W = 64 NW output columns x0 .. x0 + W - 1) and one
// "frame" wave whose lanes 0 and 1 compute the intermediate nodes just left and right of the tile
// (columns x0 - 1 and x0 + W, wrapped; where it measured faster, the frame wave computes them for 4 or
// 32 rows at a time, one node per lane, and hands them out row by row).  The block walks its H output rows top to bottom (the
// single-instance kernel walks odd tile rows bottom to top): iteration r computes intermediate row r
// (from state rows r - 1 .. r + 1 in HBM/L2) and, one row behind, output row r - 1 (from intermediate
// rows r - 2 .. r; r + 1 and rows r .. r + 2 walking up).  Intermediate populations that move
// along x (i = 1, 3, 5, 6, 7, 8) are exchanged through a four-row LDS ring; those with e_x = 0
// (i = 0, 2, 4) stay in the registers of the lane that computed them.  Four ring rows let the next
// intermediate row be written while the previous output row is still being read, so one barrier
// per row suffices.
#include "lbm_internal.h"
#include "lbm_kernel_common.h"

namespace lbm {
namespace {

// LDS ring plane of each population that moves along x (-1: kept in registers).
constexpr int kPlane[9] = {-1, 0, -1, 1, -1, 2, 3, 4, 5};

// Resident waves per SIMD that the registers of the two-step kernels are allocated for (see below).
constexpr int step2_waves(int mode, int nw, bool batched)
{
    if (mode == MODE_F64_F64 || mode == MODE_F64_F32) return nw == 2 ? 4 : (nw == 4 ? 3 : 2);
    if (batched) return 6;
    return mode == MODE_F16S_F32 && nw <= 4 ? 8 : 6;
}

// amdgpu_waves_per_eu: register allocation for as many resident waves per SIMD as the blocks of the
// default shapes can use, or as the LDS ring of FP64 storage lets 160 KB hold (2 to 4): FP32 six
// (80 VGPRs), FP16 eight on tiles of up to 256 columns (64; with a D field the walk had grown to 65 and
// lost a wave per SIMD: 8192^2 162k -> 169k MLUPS with the cap), the 9-wave blocks of 512-column tiles,
// stochastic rounding (capped at seven it spilled and lost 2-6 %) and the batched kernel six.
// The walk is bound by the loads each wave keeps in flight, so resident waves count more than registers.
// The LDS ring of a block: four rows of the six x-moving intermediate populations, W + 2 columns and
// one more that the frame wave's idle lanes write (and nothing reads).
template <int MODE, int NW>
using Ring = typename ModeTraits<MODE>::St::T[4][6][64 * NW + 3];

// Value of v in lane l of the wave (l wave-uniform), for 2-, 4- and 8-byte storage types.
template <class T>
__device__ __forceinline__ T read_lane(T v, int l)
{
    if constexpr (sizeof(T) == 8) {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    } else if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    } else {
        const int b = (int)__builtin_bit_cast(uint16_t, v);
        return __builtin_bit_cast(T, (uint16_t)__builtin_amdgcn_readlane(b, l));
    }
}

// Two steps of tile t of one instance (tiles numbered row-major, ceil(nx / W) per row, d.lcf.rows high),
// reading buf[parity] and writing buf[parity ^ 1]; called by every thread of the block.
// PF: issue each row's global loads one row ahead.  Single-instance kernels with FP32 or FP64 storage
// take it; the FP16 codecs (more arithmetic per value, already issue-bound) and the batched kernel
// (four inlined variants within one register budget) measure faster without.  BATCH: called by the
// batched kernel, which keeps the frame wave's nodes in step with the walk (below).
template <int MODE, int AUX, bool HAS_K, bool HAS_S, bool MRT, int NW, bool CST, bool PF, bool UP, bool BATCH>
__device__ __forceinline__ void fused_tile(const InstDesc &d, int parity, int t, Ring<MODE, NW> &ring)
{
    using St = typename ModeTraits<MODE>::St;
    using M = typename ModeTraits<MODE>::M;
    using T = typename St::T;
    using C = Codec<St, M>;
    constexpr int W = 64 * NW, WC = W + 3;

    const int nx = d.L.nx, ny = d.L.ny;
    const int64_t pitch = d.L.pitch;
    const int H = d.lcf.rows;
    const int ntx = (nx + W - 1) / W;
    const int x0 = (t % ntx) * W, y0 = (t / ntx) * H;
    const int y1 = min(y0 + H, ny);  // output rows y0 .. y1 - 1
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63u);
    const bool frame = wave == NW;
    // ring column of this thread's intermediate node (column x0 - 1 + c of the lattice, wrapped)
    const int c = frame ? (lane == 0 ? 0 : (lane == 1 ? W + 1 : -1)) : 1 + wave * 64 + lane;
    const bool act = c >= 0;
    // every lane runs the intermediate node's loads and collision (no divergent branch, whose merges had
    // cost copies and waits); the frame wave's idle lanes take column x0 and write the spare ring column
    const int cw = act ? c : W + 2;
    int xi = x0 - 1 + (act ? c : 1);
    xi = xi % nx;
    xi = xi < 0 ? xi + nx : xi;
    const bool live = !frame && x0 + wave * 64 + lane < nx;  // an output column of this tile
    const unsigned ux_ = (unsigned)xi;
    const unsigned uxm = ux_ == 0 ? (unsigned)nx - 1 : ux_ - 1;
    const unsigned uxp = ux_ == (unsigned)nx - 1 ? 0u : ux_ + 1;
    unsigned bc = ux_ * (unsigned)sizeof(T), bm = uxm * (unsigned)sizeof(T), bp = uxp * (unsigned)sizeof(T);
    unsigned fc = ux_ * (unsigned)sizeof(M), fm = uxm * (unsigned)sizeof(M), fp = uxp * (unsigned)sizeof(M);
    const unsigned pb = (unsigned)(pitch * (int64_t)sizeof(T));

    const T *__restrict__ src = static_cast<const T *>(d.buf[parity]);
    T *__restrict__ dst = static_cast<T *>(d.buf[parity ^ 1]);
    const M *__restrict__ u = static_cast<const M *>(d.u);
    const M *__restrict__ kf = static_cast<const M *>(d.k);
    const M *__restrict__ sf = static_cast<const M *>(d.s);
    const M lam = (M)d.lambda;
    Relax<M> rconst;
    rconst.w1 = (M)d.w1;
    rconst.w2 = (M)d.w2;
    rconst.beta = (M)d.beta;
    rconst.w3 = (M)d.w3;

    auto wrapr = [ny](int r) { return r < 0 ? r + ny : (r >= ny ? r - ny : r); };
    // Walk direction: top to bottom (dir = +1), or with UP bottom to top (dir = -1).  The single-instance
    // kernel walks odd tile rows up, so that two vertically adjacent tiles reach the state rows they both
    // read (two each way) at about the same time (both at their first rows, or both at their last) and
    // the second read finds them in L2: 2048^2 FP32 reads 1.01x its algorithmic bytes instead of 1.15x.
    // A compile-time direction keeps the row arithmetic free of selects.
    constexpr int dir = UP ? -1 : 1;
    constexpr bool up = UP;
    // The global loads of walk row r: u at (xi, r + dir); for the intermediate node (xi, r) its nine
    // pulls from state rows r - 1 .. r + 1, u at its x-neighbours and the k and s fields.  With PF, row
    // r + 1's loads are issued before row r is computed, so they are in flight through row r's two
    // collisions and the barrier instead of stalling the block once per row.
    struct RowLoads {
        T g[9];
        M uxp, uyp, uxe, uxw, uye, uyw, k, s;
    };
    auto load_row = [&](int r, RowLoads &o) {
        // row indices through readfirstlane: uniform values the compiler cannot strength-reduce into
        // per-lane 64-bit address recurrences, so every access keeps the scalar-base + 32-bit-offset form
        const int rw = __builtin_amdgcn_readfirstlane(wrapr(r));
        const int rwm = __builtin_amdgcn_readfirstlane(wrapr(r - 1));
        const int rwp = __builtin_amdgcn_readfirstlane(wrapr(r + 1));
        const int rwa = __builtin_amdgcn_readfirstlane(wrapr(r + dir));
        // the lane offsets are re-read every row (an empty asm that claims to update them), so the compiler
        // keeps each access as one scalar row base plus a 32-bit lane offset instead of hoisting 64-bit
        // per-lane addresses out of the walk
        asm volatile("" : "+v"(bc), "+v"(bm), "+v"(bp), "+v"(fc), "+v"(fm), "+v"(fp));
        const M *__restrict__ un = u + (int64_t)rwa * 2 * pitch;
        o.uxp = ld_at(un, fc);
        o.uyp = ld_at(un + pitch, fc);
        const T *__restrict__ rm = src + (int64_t)rwm * 9 * pitch;
        const T *__restrict__ rc = src + (int64_t)rw * 9 * pitch;
        const T *__restrict__ rp = src + (int64_t)rwp * 9 * pitch;
        o.g[0] = ld_at(rc, bc);
        o.g[1] = ld_at(rc + pitch, bm);
        o.g[2] = ld_at(rm + 2 * pitch, bc);
        o.g[3] = ld_at(rc + 3 * pitch, bp);
        o.g[4] = ld_at(rp + 4 * pitch, bc);
        o.g[5] = ld_at(rm + 5 * pitch, bm);
        o.g[6] = ld_at(rm + 6 * pitch, bp);
        o.g[7] = ld_at(rp + 7 * pitch, bp);
        o.g[8] = ld_at(rp + 8 * pitch, bm);
    };
    // the rest of row r's loads, for the node at (xi, r) (rw: the wrapped row, wave-uniform)
    auto load_aux = [&](int rw, RowLoads &o) {
        const M *__restrict__ uc = u + (int64_t)rw * 2 * pitch;
        if (AUX == 0) {
            o.uxe = ld_at(uc, fp);
            o.uxw = ld_at(uc, fm);
            o.uye = ld_at(uc + pitch, fp);
            o.uyw = ld_at(uc + pitch, fm);
        }
        if (HAS_K) o.k = ld_at(kf + (int64_t)rw * pitch, fc);
        if (HAS_S) o.s = ld_at(sf + (int64_t)rw * pitch, fc);
    };
    // the walk: intermediate rows rs, rs + dir, ..., nk of them; output row r - dir one iteration behind
    const int rs = up ? y1 : y0 - 1;
    const int nk = y1 - y0 + 2;
    // velocity at this column, rows r - 2 dir .. r + dir of the walk (mm, m, c, p)
    M ux_mm = M(0), uy_mm = M(0);
    M ux_m = ld_at(u + (int64_t)wrapr(rs - dir) * 2 * pitch, fc), uy_m = ld_at(u + ((int64_t)wrapr(rs - dir) * 2 + 1) * pitch, fc);
    M ux_c = ld_at(u + (int64_t)wrapr(rs) * 2 * pitch, fc), uy_c = ld_at(u + ((int64_t)wrapr(rs) * 2 + 1) * pitch, fc);
    // x-differences of u, the relaxation and the source of the previous intermediate row (reused by
    // the output node of that row, which sits in the same column)
    M dxux_m = M(0), dxuy_m = M(0);
    Relax<M> r_m = rconst;
    M s_m = M(0);
    // e_x = 0 populations of earlier intermediate rows at this column, as a reader would decode them:
    // p0 of the previous row, and the one moving against the walk (i = 2 walking down, 4 walking up)
    // of the two previous rows
    M p0_m = M(0), pb_m = M(0), pb_mm = M(0);

    // stochastic rounding: time level of the state this launch reads; it writes levels + 1 and + 2
    const int64_t level = launch_level<C>(d, parity);
    advance_level<C>(d, parity, level, 2, t == 0 && threadIdx.x == 0);

    // Frame pass: the frame wave computes the intermediate nodes of columns x0 - 1 (lanes 0-31) and
    // x0 + W (lanes 32-63), wrapped, for FR walk rows at a time, one node per lane (lane l: walk row
    // k0 + min(l % 32, FR - 1)), and holds them in registers; each iteration lanes 0 and 1 copy that
    // row's pair into the ring's frame columns (the other lanes write the spare column).  The nodes run
    // the interior waves' arithmetic, with their pulls and u neighbours addressed per lane.  The frame
    // wave then runs one collision per FR rows instead of one per row, which pays where the walk is
    // bound by VALU issue and the pass does not fetch rows far ahead of the walk:
    //  - FP16 storage on 512-column tiles, 32 rows (2048^2 194.5k -> 204.4k MLUPS); with a D field
    //    (whose relaxation costs three divisions per node) 4 rows;
    //  - with a D field, FP16 storage on 256-column tiles (8192^2 172.1k -> 180.0k), FP16 with
    //    stochastic rounding on 256- and 512-column tiles (8192^2 132.0k -> 139.7k, 2048^2 128.1k ->
    //    137.4k) and FP64 storage on 256-column tiles (2048^2 56.2k -> 58.2k), 4 rows;
    //  - FP16 with stochastic rounding and streaming stores on 256-column tiles, 4 rows, its registers
    //    capped for seven resident waves (8192^2 168.4k -> 171.9k, 4096^2 155.0k -> 158.2k).
    // Elsewhere the frame wave keeps computing its two nodes in step with the walk: FP32 was level,
    // FP64 on 512-column tiles 1 % slower; without a D field 256-column FP16 tiles lost 6-9 % in
    // streaming (32 rows: edge lines fetched a whole tile ahead are evicted from L2 before the walk
    // reaches them) and were level with 4 rows; stochastic rounding with 32 rows and no cap lost a
    // resident wave to one more VGPR (8192^2 169k -> 143k), and the batched kernel (128-column tiles)
    // lost 2 % (0.5 % with 4 rows).
    constexpr bool kFramePass = !BATCH && (MODE == MODE_F16S_F32 ? (NW == 8 || (NW == 4 && HAS_K))
                                           : MODE == MODE_F16SR_F32 ? ((NW >= 4 && HAS_K) || (NW == 4 && !CST))
                                                                    : MODE == MODE_F64_F64 && NW == 4 && HAS_K);
    constexpr int FR = HAS_K || MODE == MODE_F16SR_F32 ? 4 : 32;
    if (kFramePass && frame) {
        int xf = lane < 32 ? x0 - 1 + nx : x0 + W;
        xf %= nx;
        const int xfm = xf == 0 ? nx - 1 : xf - 1, xfp = xf == nx - 1 ? 0 : xf + 1;
        const int col = lane == 0 ? 0 : (lane == 1 ? W + 1 : W + 2);
        T fv[6];
        for (int k = 0; k < nk; ++k) {
            if (k % FR == 0) {
                const int r = rs + dir * (k + min(min(lane & 31, FR - 1), nk - 1 - k));
                const int rw = wrapr(r), rwm = wrapr(r - 1), rwp = wrapr(r + 1);
                const T *__restrict__ rm = src + (int64_t)rwm * 9 * pitch;
                const T *__restrict__ rc = src + (int64_t)rw * 9 * pitch;
                const T *__restrict__ rp = src + (int64_t)rwp * 9 * pitch;
                T gt[9];
                gt[0] = rc[xf];
                gt[1] = rc[pitch + xfm];
                gt[2] = rm[2 * pitch + xf];
                gt[3] = rc[3 * pitch + xfp];
                gt[4] = rp[4 * pitch + xf];
                gt[5] = rm[5 * pitch + xfm];
                gt[6] = rm[6 * pitch + xfp];
                gt[7] = rp[7 * pitch + xfp];
                gt[8] = rp[8 * pitch + xfm];
                const M *__restrict__ uc = u + (int64_t)rw * 2 * pitch;
                const M fux = uc[xf], fuy = uc[pitch + xf];
                M uxe = M(0), uxw = M(0), uye = M(0), uyw = M(0), uxn = M(0), uxs = M(0), uyn = M(0), uys = M(0);
                if (AUX == 0) {
                    const M *__restrict__ us = u + (int64_t)rwm * 2 * pitch;
                    const M *__restrict__ un = u + (int64_t)rwp * 2 * pitch;
                    uxe = uc[xfp];
                    uxw = uc[xfm];
                    uye = uc[pitch + xfp];
                    uyw = uc[pitch + xfm];
                    uxn = un[xf];
                    uyn = un[pitch + xf];
                    uxs = us[xf];
                    uys = us[pitch + xf];
                }
                const M kv = HAS_K ? kf[(int64_t)rw * pitch + xf] : M(0);
                const M sv = HAS_S ? sf[(int64_t)rw * pitch + xf] : M(0);
                M g[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) g[i] = C::dec(gt[i], i, d.f16);
                M Ax = M(0), Ay = M(0);
                if (AUX == 0) {  // as the interior node: u at rows r + 1 and r - 1 for the y-differences
                    const M phi = g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8];
                    const M dxux = (uxe - uxw) * M(0.5);
                    const M dxuy = (uye - uyw) * M(0.5);
                    const M dyux = (uxn - uxs) * M(0.5);
                    const M dyuy = (uyn - uys) * M(0.5);
                    Ax = phi * (fux * dxux + fuy * dyux);
                    Ay = phi * (fux * dxuy + fuy * dyuy);
                }
                const Relax<M> rr = HAS_K ? relax_from_k<M>(kv, lam, rconst.w3) : rconst;
                M P[9];
                collide<M, MRT>(g, fux, fuy, rr, Ax, Ay, sv, P);
                const auto rb = C::bits(d.f16, level + 1, (int64_t)rw * nx, (unsigned)xf);
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    if (kPlane[i] >= 0) fv[kPlane[i]] = C::enc(P[i], i, d.f16, rb);
            }
            const int j = k % FR;
            T(*slot)[WC] = ring[(rs + dir * k) & 3];
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const T left = read_lane(fv[p], j), right = read_lane(fv[p], 32 + j);
                slot[p][col] = lane == 0 ? left : right;
            }
            __syncthreads();
        }
        return;
    }

    RowLoads nxt;
    if (PF) {
        load_row(rs, nxt);
        load_aux(__builtin_amdgcn_readfirstlane(wrapr(rs)), nxt);
    }
    // FP16 with stochastic rounding raises the issue priority of its waves for the output node (after the
    // barrier) and lowers it for the intermediate node: 2048^2 146k -> 158k, 8192^2 156k -> 168k MLUPS.
    // Round-to-nearest FP16 gained with 512-column tiles (2048^2 188k -> 195k) and lost with 256-column
    // ones (8192^2 201k -> 190k); FP32 and FP64 were level or slower.
    constexpr bool kPrio = MODE == MODE_F16SR_F32 || (MODE == MODE_F16S_F32 && NW == 8);
    // one row of the walk; with PF the walk is unrolled by two, so the values rolled from row to row are
    // renamed instead of copied
    auto walk_row = [&](const int k) __attribute__((always_inline)) {
        if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
        const int r = __builtin_amdgcn_readfirstlane(rs + dir * k);
        const int rw = __builtin_amdgcn_readfirstlane(wrapr(r));
        const auto rb1 = C::bits(d.f16, level + 1, (int64_t)rw * nx, (unsigned)xi);  // intermediate node (xi, r)
        RowLoads cur;
        if (PF) {
            cur = nxt;
            if (k + 1 < nk) {
                load_row(r + dir, nxt);
                load_aux(__builtin_amdgcn_readfirstlane(wrapr(r + dir)), nxt);
            }
        } else {
            load_row(r, cur);
        }
        const M ux_p = cur.uxp, uy_p = cur.uyp;
        // ---- phase 1: intermediate node (xi, r) of step n + 1 -----------------------------------------
        M dxux = M(0), dxuy = M(0), s = M(0);
        Relax<M> rr = rconst;
        M P[9];
        {
            M g[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) g[i] = C::dec(cur.g[i], i, d.f16);
            if (!PF) load_aux(rw, cur);
            M Ax = M(0), Ay = M(0);
            if (AUX == 0) {  // Eq. (16): phi u_b d_b u_a, central differences of u
                const M phi = g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8];
                dxux = (cur.uxe - cur.uxw) * M(0.5);
                dxuy = (cur.uye - cur.uyw) * M(0.5);
                // u at rows r + 1 and r - 1 (ahead and behind, or behind and ahead walking up)
                const M dyux = ((up ? ux_m : ux_p) - (up ? ux_p : ux_m)) * M(0.5);
                const M dyuy = ((up ? uy_m : uy_p) - (up ? uy_p : uy_m)) * M(0.5);
                Ax = phi * (ux_c * dxux + uy_c * dyux);
                Ay = phi * (ux_c * dxuy + uy_c * dyuy);
            }
            rr = HAS_K ? relax_from_k<M>(cur.k, lam, rconst.w3) : rconst;
            s = HAS_S ? cur.s : M(0);
            collide<M, MRT>(g, ux_c, uy_c, rr, Ax, Ay, s, P);
            T(*slot)[WC] = ring[r & 3];
#pragma unroll
            for (int i = 0; i < 9; ++i)
                if (kPlane[i] >= 0) slot[kPlane[i]][cw] = C::enc(P[i], i, d.f16, rb1);
        }
        __syncthreads();
        if constexpr (kPrio) __builtin_amdgcn_s_setprio(1);
        // ---- phase 2: output node (x, y = r - dir) of step n + 2 -------------------------------------
        const M p2 = C::dec(C::enc(P[2], 2, d.f16, rb1), 2, d.f16);
        const M p4 = C::dec(C::enc(P[4], 4, d.f16, rb1), 4, d.f16);
        if (!frame && k >= 2) {
            const int y = __builtin_amdgcn_readfirstlane(r - dir);
            M g[9];
            T(*const sy)[WC] = ring[y & 3];
            T(*const sm)[WC] = ring[(y - 1) & 3];
            T(*const sp)[WC] = ring[(y + 1) & 3];
            g[0] = p0_m;
            g[1] = C::dec(sy[kPlane[1]][c - 1], 1, d.f16);
            g[2] = up ? p2 : pb_mm;  // from row y - 1
            g[3] = C::dec(sy[kPlane[3]][c + 1], 3, d.f16);
            g[4] = up ? pb_mm : p4;  // from row y + 1
            g[5] = C::dec(sm[kPlane[5]][c - 1], 5, d.f16);
            g[6] = C::dec(sm[kPlane[6]][c + 1], 6, d.f16);
            g[7] = C::dec(sp[kPlane[7]][c + 1], 7, d.f16);
            g[8] = C::dec(sp[kPlane[8]][c - 1], 8, d.f16);
            M Ax = M(0), Ay = M(0);
            if (AUX == 0) {
                const M phi = g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8];
                const M dyux = ((up ? ux_mm : ux_c) - (up ? ux_c : ux_mm)) * M(0.5);  // u at y + 1 and y - 1
                const M dyuy = ((up ? uy_mm : uy_c) - (up ? uy_c : uy_mm)) * M(0.5);
                Ax = phi * (ux_m * dxux_m + uy_m * dyux);
                Ay = phi * (ux_m * dxuy_m + uy_m * dyuy);
            }
            M Q[9];
            collide<M, MRT>(g, ux_m, uy_m, r_m, Ax, Ay, s_m, Q);
            if (live) {
                T *__restrict__ out = dst + (int64_t)y * 9 * pitch;
                const auto rb2 = C::bits(d.f16, level + 2, (int64_t)y * nx, (unsigned)xi);  // output node (xi, y)
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    if constexpr (CST) st_at(out, bc + (unsigned)i * pb, C::enc(Q[i], i, d.f16, rb2));
                    else st_nt_at(out, bc + (unsigned)i * pb, C::enc(Q[i], i, d.f16, rb2));
                }
            }
        }
        // roll the walk on by one row
        pb_mm = pb_m;
        pb_m = up ? p4 : p2;
        p0_m = C::dec(C::enc(P[0], 0, d.f16, rb1), 0, d.f16);
        dxux_m = dxux;
        dxuy_m = dxuy;
        r_m = rr;
        s_m = s;
        ux_mm = ux_m;
        uy_mm = uy_m;
        ux_m = ux_c;
        uy_m = uy_c;
        ux_c = ux_p;
        uy_c = uy_p;
    };
    int k = 0;
    if constexpr (PF) {
        for (; k + 1 < nk; k += 2) {
            walk_row(k);
            walk_row(k + 1);
        }
    }
    for (; k < nk; ++k) walk_row(k);
}

// ---- two steps with the flux form of the auxiliary term ----------------------------------------------
//
// The flux form needs phi at the four axis neighbours, at the time level of the step.  A two-step tile of
// W output columns therefore carries three frame columns on each side (ring column cc holds lattice
// column x0 - 3 + cc, wrapped): phi at level n + 1 for all W + 6 columns (each the sum of the node's pulls
// from the state at n), intermediate nodes (level n + 1) for the inner W + 4, phi at level n + 2 for the
// inner W + 2 (the sums of the pulls from the intermediate state) and outputs for the W interior
// columns.  Iteration r of the walk (top to bottom; odd tile rows bottom to top, with r + 1 read as the
// row ahead) pulls state row r + 1 (its phi into a ring, its populations kept for the next iteration),
// computes intermediate row r (the x-moving populations into a ring); after the block's one barrier it
// pulls intermediate rows r - 2 .. r for the node of row r - 1 (its phi into a ring, its populations
// kept) and computes output row r - 2.  Frame wave lanes 0-2 and 3-5 take the
// three frame columns on the left and on the right.  Every node runs the arithmetic of the one-step flux
// kernel (the same pulls, sums in index order, flux_aux, collide) and the intermediate populations go
// through the storage codec, so the results are bitwise those of two single steps.
template <int MODE, int NW>
struct FluxRings {  // W + 6 columns and a spare one that lanes without a node of that kind write
    typename ModeTraits<MODE>::St::T pop[4][6][64 * NW + 7];  // intermediate x-moving populations
    typename ModeTraits<MODE>::M phi1[4][64 * NW + 7];        // phi at level n + 1
    typename ModeTraits<MODE>::M phi2[4][64 * NW + 7];        // phi at level n + 2
};

template <int MODE, bool HAS_K, bool HAS_S, int NW, bool CST, bool PF, bool UP>
__device__ __forceinline__ void flux_tile(const InstDesc &d, int parity, int t, FluxRings<MODE, NW> &R)
{
    using St = typename ModeTraits<MODE>::St;
    using M = typename ModeTraits<MODE>::M;
    using T = typename St::T;
    using C = Codec<St, M>;
    constexpr int W = 64 * NW;

    const int nx = d.L.nx, ny = d.L.ny;
    const int64_t pitch = d.L.pitch;
    const int H = d.lcf.rows;
    const int ntx = (nx + W - 1) / W;
    const int x0 = (t % ntx) * W, y0 = (t / ntx) * H;
    const int y1 = min(y0 + H, ny);  // output rows y0 .. y1 - 1
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63u);
    const bool frame = wave == NW;
    const int cc = frame ? (lane < 3 ? lane : (lane < 6 ? W + lane : -1)) : 3 + wave * 64 + lane;
    const bool act = cc >= 0;                         // pulls the state (phi at n + 1)
    const bool inter = act && cc >= 1 && cc < W + 5;  // an intermediate node
    const bool mid = act && cc >= 2 && cc < W + 4;    // phi at n + 2
    const bool live = !frame && x0 + wave * 64 + lane < nx;  // an output node
    int xi = x0 - 3 + (act ? cc : 3);
    xi = xi % nx;
    xi = xi < 0 ? xi + nx : xi;
    const unsigned ux_ = (unsigned)xi;
    const unsigned uxm = ux_ == 0 ? (unsigned)nx - 1 : ux_ - 1;
    const unsigned uxp = ux_ == (unsigned)nx - 1 ? 0u : ux_ + 1;
    unsigned bc = ux_ * (unsigned)sizeof(T), bm = uxm * (unsigned)sizeof(T), bp = uxp * (unsigned)sizeof(T);
    unsigned fc = ux_ * (unsigned)sizeof(M), fm = uxm * (unsigned)sizeof(M), fp = uxp * (unsigned)sizeof(M);
    const unsigned pb = (unsigned)(pitch * (int64_t)sizeof(T));
    // Every lane runs the pulls, the intermediate node and the phi at n + 2 (no divergent branches):
    // lanes without such a node read the ring at a column inside it and write the spare column W + 6.
    const int c1w = act ? cc : W + 6;
    const int ci = inter ? cc : 1, ciw = inter ? cc : W + 6;
    const int cm = mid ? cc : 2, cmw = mid ? cc : W + 6;

    const T *__restrict__ src = static_cast<const T *>(d.buf[parity]);
    T *__restrict__ dst = static_cast<T *>(d.buf[parity ^ 1]);
    const M *__restrict__ u = static_cast<const M *>(d.u);
    const M *__restrict__ kf = static_cast<const M *>(d.k);
    const M *__restrict__ sf = static_cast<const M *>(d.s);
    const M lam = (M)d.lambda;
    Relax<M> rconst;
    rconst.w1 = (M)d.w1;
    rconst.w2 = (M)d.w2;
    rconst.beta = (M)d.beta;
    rconst.w3 = (M)d.w3;

    // rows y0 - 4 .. y1 + 3 wrapped (twice at most: ny >= 3)
    auto wrapr = [ny](int r) {
        r = r < 0 ? r + ny : (r >= ny ? r - ny : r);
        return r < 0 ? r + ny : (r >= ny ? r - ny : r);
    };
    auto sum9 = [](const M (&g)[9]) { return g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8]; };
    // the nine populations node (xi, row) pulls from the state
    auto pull = [&](int row, M (&g)[9]) {
        const T *__restrict__ rm = src + (int64_t)__builtin_amdgcn_readfirstlane(wrapr(row - 1)) * 9 * pitch;
        const T *__restrict__ rc = src + (int64_t)__builtin_amdgcn_readfirstlane(wrapr(row)) * 9 * pitch;
        const T *__restrict__ rp = src + (int64_t)__builtin_amdgcn_readfirstlane(wrapr(row + 1)) * 9 * pitch;
        g[0] = C::dec(ld_at(rc, bc), 0, d.f16);
        g[1] = C::dec(ld_at(rc + pitch, bm), 1, d.f16);
        g[2] = C::dec(ld_at(rm + 2 * pitch, bc), 2, d.f16);
        g[3] = C::dec(ld_at(rc + 3 * pitch, bp), 3, d.f16);
        g[4] = C::dec(ld_at(rp + 4 * pitch, bc), 4, d.f16);
        g[5] = C::dec(ld_at(rm + 5 * pitch, bm), 5, d.f16);
        g[6] = C::dec(ld_at(rm + 6 * pitch, bp), 6, d.f16);
        g[7] = C::dec(ld_at(rp + 7 * pitch, bp), 7, d.f16);
        g[8] = C::dec(ld_at(rp + 8 * pitch, bm), 8, d.f16);
    };
    auto urow = [&](int row) { return u + (int64_t)__builtin_amdgcn_readfirstlane(wrapr(row)) * 2 * pitch; };
    // with PF the state pulls of row r + 2 and u at (xi, r + 2) are loaded during iteration r, one row
    // ahead of their decoding, so the loads stay in flight through the row's collisions and barrier
    // (FP64 storage: +2-3 %; FP32 storage measured slower with the extra registers)
    struct Fetched {
        T g[9];
        M ux, uy;
    };
    auto fetch = [&](int row, Fetched &o) {
        const T *__restrict__ rm = src + (int64_t)__builtin_amdgcn_readfirstlane(wrapr(row - 1)) * 9 * pitch;
        const T *__restrict__ rc = src + (int64_t)__builtin_amdgcn_readfirstlane(wrapr(row)) * 9 * pitch;
        const T *__restrict__ rp = src + (int64_t)__builtin_amdgcn_readfirstlane(wrapr(row + 1)) * 9 * pitch;
        o.g[0] = ld_at(rc, bc);
        o.g[1] = ld_at(rc + pitch, bm);
        o.g[2] = ld_at(rm + 2 * pitch, bc);
        o.g[3] = ld_at(rc + 3 * pitch, bp);
        o.g[4] = ld_at(rp + 4 * pitch, bc);
        o.g[5] = ld_at(rm + 5 * pitch, bm);
        o.g[6] = ld_at(rm + 6 * pitch, bp);
        o.g[7] = ld_at(rp + 7 * pitch, bp);
        o.g[8] = ld_at(rp + 8 * pitch, bm);
        const M *__restrict__ un = urow(row);
        o.ux = ld_at(un, fc);
        o.uy = ld_at(un + pitch, fc);
    };

    const int64_t level = launch_level<C>(d, parity);  // stochastic rounding: writes levels + 1 and + 2
    advance_level<C>(d, parity, level, 2, t == 0 && threadIdx.x == 0);

    // The walk goes top to bottom (dir = +1) or, with UP, bottom to top (dir = -1; the kernel walks odd
    // tile rows up, so that adjacent tiles read the rows they share at about the same time).  Iteration k
    // handles intermediate row r = rs + k dir; "behind" is r - dir, "ahead" r + dir, and the south and
    // north neighbours of a node are the behind and ahead ones walking down, the other way round up.
    constexpr int dir = UP ? -1 : 1;
    const int rs = UP ? y1 + 1 : y0 - 2;
    const int nk = y1 - y0 + 4;
    // the walk starts with the state pulls of rows rs - dir (phi only) and rs
    M gc[9], p1_m, p1_c;
    {
        M gm[9];
        pull(rs - dir, gm);
        p1_m = sum9(gm);
        pull(rs, gc);
        p1_c = sum9(gc);
        R.phi1[(rs - dir) & 3][c1w] = p1_m;
        R.phi1[rs & 3][c1w] = p1_c;
    }
    // u at this column, rows r - 3 dir .. r + dir of the walk
    M ux3 = M(0), uy3 = M(0), ux2 = M(0), uy2 = M(0);
    M ux1 = ld_at(urow(rs - dir), fc), uy1 = ld_at(urow(rs - dir) + pitch, fc);
    M ux0 = ld_at(urow(rs), fc), uy0 = ld_at(urow(rs) + pitch, fc);
    // e_x = 0 intermediate populations of this column as a reader decodes them: p0 of the row behind,
    // and the one moving against the walk (i = 2 walking down, 4 up) of the two rows behind
    M p0_m = M(0), pb_m = M(0), pb_mm = M(0);
    // phi at n + 2 of this column, rows r - 3 dir and r - 2 dir, and the populations node (xi, r - 2 dir)
    // pulled
    M q_m3 = M(0), q_m2 = M(0);
    M g2[9] = {};
    Fetched nxt;
    if (PF) fetch(rs + dir, nxt);
    __syncthreads();  // phi1 of the first two rows

    // FP32 and FP16 storage raise the waves' issue priority for the work after the barrier (2048^2 FP32
    // 95k -> 98k, FP16S 120k -> 133k MLUPS; FP64 storage level)
    constexpr bool kPrio = !(MODE == MODE_F64_F64 || MODE == MODE_F64_F32);
    for (int k = 0; k < nk; ++k) {
        const int r = rs + dir * k;
        if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
        asm volatile("" : "+v"(bc), "+v"(bm), "+v"(bp), "+v"(fc), "+v"(fm), "+v"(fp));
        // ---- the state pulls of row r + dir and their phi ----------------------------------------------
        M gn[9], uxp1, uyp1;
        if (PF) {
            const Fetched cur = nxt;
            if (k + 1 < nk) fetch(r + 2 * dir, nxt);
#pragma unroll
            for (int i = 0; i < 9; ++i) gn[i] = C::dec(cur.g[i], i, d.f16);
            uxp1 = cur.ux;
            uyp1 = cur.uy;
        } else {
            pull(r + dir, gn);
            const M *__restrict__ un = urow(r + dir);
            uxp1 = ld_at(un, fc);
            uyp1 = ld_at(un + pitch, fc);
        }
        const M p1_p = sum9(gn);
        R.phi1[(r + dir) & 3][c1w] = p1_p;
        // ---- intermediate node (xi, r), level n + 1 -------------------------------------------------------
        const int rw = __builtin_amdgcn_readfirstlane(wrapr(r));
        M P[9];
        const auto rb1 = C::bits(d.f16, level + 1, (int64_t)rw * nx, (unsigned)xi);
        {
            const M *__restrict__ uc = u + (int64_t)rw * 2 * pitch;
            const M uxw = ld_at(uc, fm), uyw = ld_at(uc + pitch, fm), uxe = ld_at(uc, fp), uye = ld_at(uc + pitch, fp);
            M Ax, Ay;
            if constexpr (UP)  // south: the row ahead, north: the row behind
                flux_aux<M>(R.phi1[r & 3][ci - 1], R.phi1[r & 3][ci + 1], p1_p, p1_m, uxw, uyw, uxe, uye, uxp1, uyp1, ux1,
                            uy1, ux0, uy0, Ax, Ay);
            else
                flux_aux<M>(R.phi1[r & 3][ci - 1], R.phi1[r & 3][ci + 1], p1_m, p1_p, uxw, uyw, uxe, uye, ux1, uy1, uxp1,
                            uyp1, ux0, uy0, Ax, Ay);
            const Relax<M> rr = HAS_K ? relax_from_k<M>(ld_at(kf + (int64_t)rw * pitch, fc), lam, rconst.w3) : rconst;
            const M s = HAS_S ? ld_at(sf + (int64_t)rw * pitch, fc) : M(0);
            collide<M, false>(gc, ux0, uy0, rr, Ax, Ay, s, P);
#pragma unroll
            for (int i = 0; i < 9; ++i)
                if (kPlane[i] >= 0) R.pop[r & 3][kPlane[i]][ciw] = C::enc(P[i], i, d.f16, rb1);
        }
        const M p2 = C::dec(C::enc(P[2], 2, d.f16, rb1), 2, d.f16);
        const M p4 = C::dec(C::enc(P[4], 4, d.f16, rb1), 4, d.f16);
        __syncthreads();
        if constexpr (kPrio) __builtin_amdgcn_s_setprio(1);
        // ---- phi at n + 2 of node (xi, y = r - dir), from intermediate rows y - 1 .. y + 1 -----------------
        M q_m1 = M(0);
        M gq[9] = {};
        if (k >= 2) {
            const int y = r - dir;
            gq[0] = p0_m;
            gq[1] = C::dec(R.pop[y & 3][kPlane[1]][cm - 1], 1, d.f16);
            gq[2] = UP ? p2 : pb_mm;  // from row y - 1
            gq[3] = C::dec(R.pop[y & 3][kPlane[3]][cm + 1], 3, d.f16);
            gq[4] = UP ? pb_mm : p4;  // from row y + 1
            gq[5] = C::dec(R.pop[(y - 1) & 3][kPlane[5]][cm - 1], 5, d.f16);
            gq[6] = C::dec(R.pop[(y - 1) & 3][kPlane[6]][cm + 1], 6, d.f16);
            gq[7] = C::dec(R.pop[(y + 1) & 3][kPlane[7]][cm + 1], 7, d.f16);
            gq[8] = C::dec(R.pop[(y + 1) & 3][kPlane[8]][cm - 1], 8, d.f16);
            q_m1 = sum9(gq);
            R.phi2[y & 3][cmw] = q_m1;
        }
        // ---- output node (xi, r - 2 dir), level n + 2 -----------------------------------------------------
        if (k >= 4 && live) {
            const int y = __builtin_amdgcn_readfirstlane(wrapr(r - 2 * dir));
            const M *__restrict__ uc = u + (int64_t)y * 2 * pitch;
            const M uxw = ld_at(uc, fm), uyw = ld_at(uc + pitch, fm), uxe = ld_at(uc, fp), uye = ld_at(uc + pitch, fp);
            M Ax, Ay;
            if constexpr (UP)  // south: row r + dir (phi2 of this iteration), north: row r + 3
                flux_aux<M>(R.phi2[(r - 2 * dir) & 3][cc - 1], R.phi2[(r - 2 * dir) & 3][cc + 1], q_m1, q_m3, uxw, uyw, uxe,
                            uye, ux1, uy1, ux3, uy3, ux2, uy2, Ax, Ay);
            else
                flux_aux<M>(R.phi2[(r - 2 * dir) & 3][cc - 1], R.phi2[(r - 2 * dir) & 3][cc + 1], q_m3, q_m1, uxw, uyw, uxe,
                            uye, ux3, uy3, ux1, uy1, ux2, uy2, Ax, Ay);
            const Relax<M> rr = HAS_K ? relax_from_k<M>(ld_at(kf + (int64_t)y * pitch, fc), lam, rconst.w3) : rconst;
            const M s = HAS_S ? ld_at(sf + (int64_t)y * pitch, fc) : M(0);
            M Q[9];
            collide<M, false>(g2, ux2, uy2, rr, Ax, Ay, s, Q);
            T *__restrict__ out = dst + (int64_t)y * 9 * pitch;
            const auto rb2 = C::bits(d.f16, level + 2, (int64_t)y * nx, (unsigned)xi);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if constexpr (CST) st_at(out, bc + (unsigned)i * pb, C::enc(Q[i], i, d.f16, rb2));
                else st_nt_at(out, bc + (unsigned)i * pb, C::enc(Q[i], i, d.f16, rb2));
            }
        }
        // ---- roll the walk on by one row -------------------------------------------------------------------
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            gc[i] = gn[i];
            g2[i] = gq[i];
        }
        p1_m = p1_c;
        p1_c = p1_p;
        q_m3 = q_m2;
        q_m2 = q_m1;
        pb_mm = pb_m;
        pb_m = UP ? p4 : p2;
        p0_m = C::dec(C::enc(P[0], 0, d.f16, rb1), 0, d.f16);
        ux3 = ux2;
        uy3 = uy2;
        ux2 = ux1;
        uy2 = uy1;
        ux1 = ux0;
        uy1 = uy0;
        ux0 = uxp1;
        uy0 = uyp1;
    }
}

// One instance: block b -> tile (XCD-remapped as the launch says).  FP16 with stochastic rounding on
// 256-column tiles with streaming stores and no D field runs the frame pass (above) within registers for
// seven resident waves (72 VGPRs; one value is spilled before the walk and reloaded after it, once
// per tile).
template <int MODE, int AUX, bool HAS_K, bool HAS_S, bool MRT, int NW, bool CST>
__global__ __launch_bounds__(64 * (NW + 1))
__attribute__((amdgpu_waves_per_eu(MODE == MODE_F16SR_F32 && NW == 4 && !HAS_K && !CST ? 7 : step2_waves(MODE, NW, false))))
void step2_kernel(const StepArgs a)
{
    const InstDesc &d = a.d;
    const int ntx = (d.L.nx + 64 * NW - 1) / (64 * NW);
    const int t = tile_of_block(blockIdx.x, gridDim.x, d.lcf.xcd_remap, ntx, d.lcf.xcd_rows);
    __shared__ Ring<MODE, NW> ring;
    constexpr bool PF = !is_f16_mode(MODE);
    if ((t / ntx) & 1) fused_tile<MODE, AUX, HAS_K, HAS_S, MRT, NW, CST, PF, true, false>(d, a.parity, t, ring);
    else fused_tile<MODE, AUX, HAS_K, HAS_S, MRT, NW, CST, PF, false, false>(d, a.parity, t, ring);
}

// One instance, flux form: block b -> tile.
// FP32 storage on 128-column tiles (the default shape): registers for six resident waves per SIMD (80
// VGPRs), which a 2048^2 lattice in 16-row tiles needs for every block to be resident at once
template <int MODE, bool HAS_K, bool HAS_S, int NW, bool CST>
__global__ __launch_bounds__(64 * (NW + 1))
__attribute__((amdgpu_waves_per_eu(MODE == MODE_F32_F32 && NW == 2 ? 6 : 1))) void flux2_kernel(const StepArgs a)
{
    const InstDesc &d = a.d;
    const int ntx = (d.L.nx + 64 * NW - 1) / (64 * NW);
    const int t = tile_of_block(blockIdx.x, gridDim.x, d.lcf.xcd_remap, ntx, d.lcf.xcd_rows);
    __shared__ FluxRings<MODE, NW> rings;
    constexpr bool PF = MODE == MODE_F64_F64 || MODE == MODE_F64_F32;
    if ((t / ntx) & 1) flux_tile<MODE, HAS_K, HAS_S, NW, CST, PF, true>(d, a.parity, t, rings);
    else flux_tile<MODE, HAS_K, HAS_S, NW, CST, PF, false>(d, a.parity, t, rings);
}

// Many instances (periodic D2Q9 TRT-R, one storage form and aux form): each block runs a range of
// (instance, fused tile) work items, non-temporal stores; the descriptor is wave-uniform (scalar loads).
template <int MODE, int AUX, int NW>
__global__ __launch_bounds__(64 * (NW + 1))
__attribute__((amdgpu_waves_per_eu(step2_waves(MODE, NW, true)))) void batched_step2_kernel(const BatchArgs a)
{
    int beg, end;
    if (a.block_start) {
        beg = a.block_start[blockIdx.x];
        end = a.block_start[blockIdx.x + 1];
    } else {
        beg = tile_of_block(blockIdx.x, gridDim.x, 1, 0, 0);
        end = beg + 1;
    }
    __shared__ Ring<MODE, NW> ring;
    for (int it = beg; it < end; ++it) {
        const WorkItem w = a.items[it];
        const InstDesc &d = a.inst[w.inst];
        if (d.has_k) {
            if (d.has_s) fused_tile<MODE, AUX, true, true, false, NW, false, false, false, true>(d, a.parity, w.tile, ring);
            else fused_tile<MODE, AUX, true, false, false, NW, false, false, false, true>(d, a.parity, w.tile, ring);
        } else {
            if (d.has_s) fused_tile<MODE, AUX, false, true, false, NW, false, false, false, true>(d, a.parity, w.tile, ring);
            else fused_tile<MODE, AUX, false, false, false, NW, false, false, false, true>(d, a.parity, w.tile, ring);
        }
        __syncthreads();  // the next tile rewrites the ring the last rows of this one were read from
    }
}

template <int MODE, int AUX, bool MRT, int NW, bool CST>
hipError_t launch_fused_nw(const StepArgs &a, hipStream_t st)
{
    const int W = 64 * NW, H = a.d.lcf.rows;
    const int nblocks = ((a.d.L.nx + W - 1) / W) * ((a.d.L.ny + H - 1) / H);
    const size_t lds = (size_t)a.d.lcf.lds_reserve;  // unused LDS that caps the resident waves
    const dim3 block(64 * (NW + 1));
    const bool hk = a.d.has_k, hs = a.d.has_s;
    if (hk && hs) step2_kernel<MODE, AUX, true, true, MRT, NW, CST><<<nblocks, block, lds, st>>>(a);
    else if (hk) step2_kernel<MODE, AUX, true, false, MRT, NW, CST><<<nblocks, block, lds, st>>>(a);
    else if (hs) step2_kernel<MODE, AUX, false, true, MRT, NW, CST><<<nblocks, block, lds, st>>>(a);
    else step2_kernel<MODE, AUX, false, false, MRT, NW, CST><<<nblocks, block, lds, st>>>(a);
    return hipGetLastError();
}

template <int MODE, int AUX, bool MRT>
hipError_t launch_fused_var(const StepArgs &a, hipStream_t st)
{
    const bool cst = a.d.lcf.stores == 1;
    switch (a.d.lcf.fuse_width) {
    case 128: return cst ? launch_fused_nw<MODE, AUX, MRT, 2, true>(a, st) : launch_fused_nw<MODE, AUX, MRT, 2, false>(a, st);
    case 256: return cst ? launch_fused_nw<MODE, AUX, MRT, 4, true>(a, st) : launch_fused_nw<MODE, AUX, MRT, 4, false>(a, st);
    case 512: return cst ? launch_fused_nw<MODE, AUX, MRT, 8, true>(a, st) : launch_fused_nw<MODE, AUX, MRT, 8, false>(a, st);
    default: return hipErrorInvalidValue;
    }
}

// TRT-R only (the MRT-R operator runs single steps).
template <int MODE, int AUX>
hipError_t launch_fused_aux(const StepArgs &a, hipStream_t st)
{
    return a.d.w3 != 0.0 ? hipErrorInvalidValue : launch_fused_var<MODE, AUX, false>(a, st);
}

template <int MODE, int NW, bool CST>
hipError_t launch_flux2_nw(const StepArgs &a, hipStream_t st)
{
    const int W = 64 * NW, H = a.d.lcf.rows;
    const int nblocks = ((a.d.L.nx + W - 1) / W) * ((a.d.L.ny + H - 1) / H);
    const dim3 block(64 * (NW + 1));
    const bool hk = a.d.has_k, hs = a.d.has_s;
    if (hk && hs) flux2_kernel<MODE, true, true, NW, CST><<<nblocks, block, 0, st>>>(a);
    else if (hk) flux2_kernel<MODE, true, false, NW, CST><<<nblocks, block, 0, st>>>(a);
    else if (hs) flux2_kernel<MODE, false, true, NW, CST><<<nblocks, block, 0, st>>>(a);
    else flux2_kernel<MODE, false, false, NW, CST><<<nblocks, block, 0, st>>>(a);
    return hipGetLastError();
}

// The flux form: TRT-R, tiles of 128 or 256 columns.
template <int MODE>
hipError_t launch_flux2(const StepArgs &a, hipStream_t st)
{
    if (a.d.w3 != 0.0) return hipErrorInvalidValue;
    const bool cst = a.d.lcf.stores == 1;
    switch (a.d.lcf.fuse_width) {
    case 128: return cst ? launch_flux2_nw<MODE, 2, true>(a, st) : launch_flux2_nw<MODE, 2, false>(a, st);
    case 256: return cst ? launch_flux2_nw<MODE, 4, true>(a, st) : launch_flux2_nw<MODE, 4, false>(a, st);
    default: return hipErrorInvalidValue;
    }
}

template <int MODE>
hipError_t launch_fused_mode(int aux, const StepArgs &a, hipStream_t st)
{
    switch (aux) {
    case 0: return launch_fused_aux<MODE, 0>(a, st);
    case 1: return launch_flux2<MODE>(a, st);
    case 2: return launch_fused_aux<MODE, 2>(a, st);
    default: return hipErrorInvalidValue;
    }
}

template <int MODE, int AUX>
hipError_t launch_batched_fused_aux(const BatchArgs &a, int nblocks, int width, hipStream_t st)
{
    switch (width) {
    case 128: batched_step2_kernel<MODE, AUX, 2><<<nblocks, 64 * 3, 0, st>>>(a); break;
    case 256: batched_step2_kernel<MODE, AUX, 4><<<nblocks, 64 * 5, 0, st>>>(a); break;
    case 512: batched_step2_kernel<MODE, AUX, 8><<<nblocks, 64 * 9, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_batched_fused_mode(int aux, const BatchArgs &a, int nblocks, int width, hipStream_t st)
{
    switch (aux) {
    case 0: return launch_batched_fused_aux<MODE, 0>(a, nblocks, width, st);
    case 2: return launch_batched_fused_aux<MODE, 2>(a, nblocks, width, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_batched_step2(int mode, int aux, const BatchArgs &a, int nblocks, int width, hipStream_t st)
{
    if (nblocks < 1) return hipErrorInvalidValue;
    switch (mode) {
    case MODE_F64_F64: return launch_batched_fused_mode<MODE_F64_F64>(aux, a, nblocks, width, st);
    case MODE_F64_F32: return launch_batched_fused_mode<MODE_F64_F32>(aux, a, nblocks, width, st);
    case MODE_F32_F32: return launch_batched_fused_mode<MODE_F32_F32>(aux, a, nblocks, width, st);
    case MODE_F16S_F32: return launch_batched_fused_mode<MODE_F16S_F32>(aux, a, nblocks, width, st);
    case MODE_F16SR_F32: return launch_batched_fused_mode<MODE_F16SR_F32>(aux, a, nblocks, width, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step2(int mode, int aux, const StepArgs &a, hipStream_t st)
{
    if (a.d.L.q != 9 || a.d.bckind != 0 || a.d.lcf.fuse != 2 || a.d.lcf.stores == 2) return hipErrorInvalidValue;
    if (a.d.lcf.rows < 1 || a.d.lcf.rows > 1024 || a.d.lcf.lds_reserve < 0 || a.d.lcf.lds_reserve > 65536)
        return hipErrorInvalidValue;
    switch (mode) {
    case MODE_F64_F64: return launch_fused_mode<MODE_F64_F64>(aux, a, st);
    case MODE_F64_F32: return launch_fused_mode<MODE_F64_F32>(aux, a, st);
    case MODE_F32_F32: return launch_fused_mode<MODE_F32_F32>(aux, a, st);
    case MODE_F16S_F32: return launch_fused_mode<MODE_F16S_F32>(aux, a, st);
    case MODE_F16SR_F32: return launch_fused_mode<MODE_F16SR_F32>(aux, a, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lbm
