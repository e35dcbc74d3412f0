// lbm_kernels3d.hip -- HIP kernels of the TRT-R step on the D3Q19 and D3Q27 lattices for gfx950
// (the three-dimensional extension of Sec. 2.2).
//
// Velocities (lattice units), in this order: 0:(0,0,0); 1,2:(+-1,0,0); 3,4:(0,+-1,0); 5,6:(0,0,+-1);
// 7:(1,1,0) 8:(-1,-1,0) 9:(1,-1,0) 10:(-1,1,0); 11:(1,0,1) 12:(-1,0,-1) 13:(1,0,-1) 14:(-1,0,1);
// 15:(0,1,1) 16:(0,-1,-1) 17:(0,1,-1) 18:(0,-1,1) (D3Q19: weights 1/3, 1/18, 1/36); D3Q27 adds
// 19:(1,1,1) 20:(-1,-1,-1) 21:(1,1,-1) 22:(-1,-1,1) 23:(1,-1,1) 24:(-1,1,-1) 25:(-1,1,1)
// 26:(1,-1,-1) (weights 8/27, 2/27, 1/54, 1/216).  i and i + 1 (odd i) are opposite.  One step of
// Eq. (14) in moment form (c_s^2 = 1/3):
//
//   P_i = w_i [ a0 + 3 e_i.a1 + 9/2 (e_i.a2.e_i - tr a2 / 3) + 9/2 phi ((e_i.u)^3 - (e_i.u) |u|^2) ]
//
// with a0 = phi + s, a1 = phi u + w1 (j - phi u) + beta (A + u s), a2 = phi u u + w2 (Pi - phi I/3
// - phi u u) exactly as on D2Q9 (Eqs. (3), (8), (12), (13), (16)), and the last term H3 : phi u u u,
// the third-order part of the equilibrium (Eq. (6)) contracted in closed form.  H_xxx-type tensors
// vanish at every velocity of both lattices and H_xyz at every D3Q19 velocity, so the closed form
// carries exactly the components each lattice supports (D3Q27 keeps the xyz one).
//
// Layout: row r = z*ny + y holds the Q segments of that lattice row; a wave owns one row of a
// 64-column tile, so the row bases of the nine rows (y, z), (y+-1, z), (y, z+-1), (y+-1, z+-1) it
// pulls from are wave-uniform scalars and every access is base + 32-bit lane offset.  Stores are
// non-temporal and tiles follow the XCD-contiguous order of the D2Q9 kernels.
#include <algorithm>
#include <type_traits>

#include "lbm_internal.h"
#include "lbm_kernel_common.h"

namespace lbm {
namespace {

constexpr int kEx3[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
constexpr int kEy3[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1};
constexpr int kEz3[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, 1, -1};
// Opposite velocity: the tables keep i and i + 1 (odd i) opposite.
__host__ __device__ constexpr int opp3(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Weights of the rest, face (axis), edge and corner velocities.
template <int Q>
struct Weights3;
template <>
struct Weights3<19> {
    static constexpr double rest = 1.0 / 3.0, face = 1.0 / 18.0, edge = 1.0 / 36.0;
};
template <>
struct Weights3<27> {
    static constexpr double rest = 8.0 / 27.0, face = 2.0 / 27.0, edge = 1.0 / 54.0, corner = 1.0 / 216.0;
};

template <class M>
struct Coef3 {
    M a0, a1x, a1y, a1z, axx, ayy, azz, axy, axz, ayz;  // post-collision Hermite coefficients
    M phi, ux, uy, uz;                                  // for the third-order equilibrium term
};

template <int Q, class M>
__device__ __forceinline__ void reconstruct3(const Coef3<M> &c, M (&P)[Q])
{
    using Wt = Weights3<Q>;
    const M usq = c.ux * c.ux + c.uy * c.uy + c.uz * c.uz;
    const M tr = c.axx + c.ayy + c.azz;
    const M base = c.a0 - M(1.5) * tr;
    P[0] = M(Wt::rest) * base;
    auto pair = [&](int i, M w, M eu, M ea, M eae) {
        const M ev = w * (base + M(4.5) * eae);
        const M od = w * (M(3) * ea + M(4.5) * c.phi * eu * (eu * eu - usq));
        P[i] = ev + od;
        P[i + 1] = ev - od;
    };
    const M wa = M(Wt::face), wd = M(Wt::edge);
    pair(1, wa, c.ux, c.a1x, c.axx);
    pair(3, wa, c.uy, c.a1y, c.ayy);
    pair(5, wa, c.uz, c.a1z, c.azz);
    pair(7, wd, c.ux + c.uy, c.a1x + c.a1y, c.axx + c.ayy + M(2) * c.axy);
    pair(9, wd, c.ux - c.uy, c.a1x - c.a1y, c.axx + c.ayy - M(2) * c.axy);
    pair(11, wd, c.ux + c.uz, c.a1x + c.a1z, c.axx + c.azz + M(2) * c.axz);
    pair(13, wd, c.ux - c.uz, c.a1x - c.a1z, c.axx + c.azz - M(2) * c.axz);
    pair(15, wd, c.uy + c.uz, c.a1y + c.a1z, c.ayy + c.azz + M(2) * c.ayz);
    pair(17, wd, c.uy - c.uz, c.a1y - c.a1z, c.ayy + c.azz - M(2) * c.ayz);
    if constexpr (Q == 27) {  // corners (1,1,1), (1,1,-1), (1,-1,1), (-1,1,1) and their opposites
        const M wc = M(Wt::corner);
        pair(19, wc, c.ux + c.uy + c.uz, c.a1x + c.a1y + c.a1z, tr + M(2) * (c.axy + c.axz + c.ayz));
        pair(21, wc, c.ux + c.uy - c.uz, c.a1x + c.a1y - c.a1z, tr + M(2) * (c.axy - c.axz - c.ayz));
        pair(23, wc, c.ux - c.uy + c.uz, c.a1x - c.a1y + c.a1z, tr + M(2) * (c.axz - c.axy - c.ayz));
        pair(25, wc, c.uy + c.uz - c.ux, c.a1y + c.a1z - c.a1x, tr + M(2) * (c.ayz - c.axy - c.axz));
    }
}

template <int Q, class M>
__device__ __forceinline__ void equilibrium3(M phi, M ux, M uy, M uz, M (&P)[Q])
{
    Coef3<M> c;
    c.a0 = phi;
    c.a1x = phi * ux;
    c.a1y = phi * uy;
    c.a1z = phi * uz;
    c.axx = c.a1x * ux;
    c.ayy = c.a1y * uy;
    c.azz = c.a1z * uz;
    c.axy = c.a1x * uy;
    c.axz = c.a1x * uz;
    c.ayz = c.a1y * uz;
    c.phi = phi;
    c.ux = ux;
    c.uy = uy;
    c.uz = uz;
    reconstruct3<Q, M>(c, P);
}

// TRT-R collision plus source and auxiliary term (A = phi u.grad u, lattice units).
template <int Q, class M>
__device__ __forceinline__ void collide3(const M (&g)[Q], M ux, M uy, M uz, const Relax<M> &r, M Ax, M Ay, M Az,
                                         M s, M (&P)[Q])
{
    M phi = g[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) phi += g[i];
    M jx = (g[1] - g[2]) + (g[7] - g[8]) + (g[9] - g[10]) + (g[11] - g[12]) + (g[13] - g[14]);
    M jy = (g[3] - g[4]) + (g[7] - g[8]) - (g[9] - g[10]) + (g[15] - g[16]) + (g[17] - g[18]);
    M jz = (g[5] - g[6]) + (g[11] - g[12]) - (g[13] - g[14]) + (g[15] - g[16]) - (g[17] - g[18]);
    const M sxy = (g[7] + g[8]) + (g[9] + g[10]);
    const M sxz = (g[11] + g[12]) + (g[13] + g[14]);
    const M syz = (g[15] + g[16]) + (g[17] + g[18]);
    M pxx = (g[1] + g[2]) + sxy + sxz;
    M pyy = (g[3] + g[4]) + sxy + syz;
    M pzz = (g[5] + g[6]) + sxz + syz;
    M pxy = (g[7] + g[8]) - (g[9] + g[10]);
    M pxz = (g[11] + g[12]) - (g[13] + g[14]);
    M pyz = (g[15] + g[16]) - (g[17] + g[18]);
    if constexpr (Q == 27) {
        // differences and sums of the opposite corner pairs along (1,1,1), (1,1,-1), (1,-1,1), (-1,1,1)
        const M da = g[19] - g[20], db = g[21] - g[22], dc = g[23] - g[24], dd = g[25] - g[26];
        const M sa = g[19] + g[20], sb = g[21] + g[22], sc = g[23] + g[24], sd = g[25] + g[26];
        jx += (da + db) + (dc - dd);
        jy += (da + db) - (dc - dd);
        jz += (da - db) + (dc + dd);
        const M sall = (sa + sb) + (sc + sd);
        pxx += sall;
        pyy += sall;
        pzz += sall;
        pxy += (sa + sb) - (sc + sd);
        pxz += (sa - sb) + (sc - sd);
        pyz += (sa - sb) - (sc - sd);
    }
    const M pux = phi * ux, puy = phi * uy, puz = phi * uz, third = phi * M(1.0 / 3.0);
    Coef3<M> c;
    c.a0 = phi + s;
    c.a1x = pux + r.w1 * (jx - pux) + r.beta * (Ax + ux * s);
    c.a1y = puy + r.w1 * (jy - puy) + r.beta * (Ay + uy * s);
    c.a1z = puz + r.w1 * (jz - puz) + r.beta * (Az + uz * s);
    const M exx = pux * ux, eyy = puy * uy, ezz = puz * uz, exy = pux * uy, exz = pux * uz, eyz = puy * uz;
    c.axx = exx + r.w2 * (pxx - third - exx);
    c.ayy = eyy + r.w2 * (pyy - third - eyy);
    c.azz = ezz + r.w2 * (pzz - third - ezz);
    c.axy = exy + r.w2 * (pxy - exy);
    c.axz = exz + r.w2 * (pxz - exz);
    c.ayz = eyz + r.w2 * (pyz - eyz);
    c.phi = phi;
    c.ux = ux;
    c.uy = uy;
    c.uz = uz;
    reconstruct3<Q, M>(c, P);
}

// g_i(x, y, z) = buf_i(x - e_i) for one node (diagnostics).
template <int Q, class St, class M>
__device__ __forceinline__ void pull_node3(const typename St::T *__restrict__ src, const Layout &L, int x, int y, int z,
                                           const F16Params &f, M (&g)[Q])
{
    using C = Codec<St, M>;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int xs = x - kEx3[i], ys = y - kEy3[i], zs = z - kEz3[i];
        xs = xs < 0 ? xs + L.nx : (xs >= L.nx ? xs - L.nx : xs);
        ys = ys < 0 ? ys + L.ny : (ys >= L.ny ? ys - L.ny : ys);
        zs = zs < 0 ? zs + L.nz : (zs >= L.nz ? zs - L.nz : zs);
        g[i] = C::dec(src[(((int64_t)zs * L.ny + ys) * Q + i) * L.pitch + xs], i, f);
    }
}

// The state of a node before collision: the pull, or for a one-buffer state after its streaming step
// (edge kind 3) the node's own slots opp(i).
template <int Q, class St, class M>
__device__ __forceinline__ void state3(const typename St::T *__restrict__ src, const Layout &L, int kind, int x, int y,
                                       int z, const F16Params &f, M (&g)[Q])
{
    if (kind == 3) {
        const typename St::T *row = src + ((int64_t)z * L.ny + y) * Q * L.pitch;
#pragma unroll
        for (int i = 0; i < Q; ++i) g[i] = Codec<St, M>::dec(row[opp3(i) * L.pitch + x], i, f);
        return;
    }
    pull_node3<Q, St, M>(src, L, x, y, z, f, g);
}

// ROWS > 0 fixes the walk length at compile time, 0 takes it from the launch shape.  Only FP16
// storage uses the one-row instantiation: at 256^3 it is +19 % (D3Q19) and +24 % (D3Q27) over the
// walking loop, while FP32 and FP64 are 1-2 % faster with the loop.
// IP: 0 two buffers; 1 and 2: one buffer updated in place, as in the D2Q9 kernel (step 1 pulls and
// writes each P_j back to the address g_opp(j) came from; step 2 reads g_j from the node's own slot
// opp(j) and writes P_j to slot j).  Every node owns its own set of addresses, so the walking loop
// stays race-free as well.
template <int Q, int MODE, int AUX, bool HAS_K, bool HAS_S, int ROWS, bool CST, int IP>
__global__ __launch_bounds__(256) void step3_kernel(const StepArgs sa)
{
    using St = typename ModeTraits<MODE>::St;
    using M = typename ModeTraits<MODE>::M;
    using T = typename St::T;
    using C = Codec<St, M>;
    const InstDesc &a = sa.d;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int t = tile_of_block(blockIdx.x, gridDim.x, a.lc.xcd_remap, tiles_per_row(a.L, a.lc), a.lc.xcd_rows);
    const int nx = a.L.nx, ny = a.L.ny, nz = a.L.nz;
    const int R = ny * nz;
    const int64_t pitch = a.L.pitch;
    const int rows = ROWS > 0 ? ROWS : a.lc.rows;
    int x0, r0;
    tile_origin(a.L, a.lc, t, wave, x0, r0);
    if (r0 >= R || x0 >= nx) return;
    const unsigned x = (unsigned)x0 + threadIdx.x;
    const bool live = x < (unsigned)nx;
    const unsigned xc = live ? x : 0u;  // dead lanes of a ragged tile read column 0 and store nothing
    const unsigned xm = xc == 0 ? (unsigned)nx - 1 : xc - 1;
    const unsigned xp = xc == (unsigned)nx - 1 ? 0u : xc + 1;
    const unsigned bc = xc * (unsigned)sizeof(T), bm = xm * (unsigned)sizeof(T), bp = xp * (unsigned)sizeof(T);
    const unsigned fc = xc * (unsigned)sizeof(M), fm = xm * (unsigned)sizeof(M), fp = xp * (unsigned)sizeof(M);
    // in place, source and destination are one buffer: no restrict on the population pointers
    using SrcP = std::conditional_t<IP == 0, const T *__restrict__, const T *>;
    using DstP = std::conditional_t<IP == 0, T *__restrict__, T *>;
    const SrcP src = static_cast<const T *>(a.buf[sa.parity]);
    const DstP dst = static_cast<T *>(a.buf[sa.parity ^ 1]);
    const M *__restrict__ u = static_cast<const M *>(a.u);
    const M *__restrict__ kf = static_cast<const M *>(a.k);
    const M *__restrict__ sf = static_cast<const M *>(a.s);
    Relax<M> rconst;
    rconst.w1 = (M)a.w1;
    rconst.w2 = (M)a.w2;
    rconst.beta = (M)a.beta;
    rconst.w3 = M(0);
    const int r1 = min(r0 + rows, R);
    for (int r = r0; r < r1; ++r) {
        const int z = r / ny, y = r - z * ny;
        const int ym = wrap_dec(y, ny), yp = wrap_inc(y, ny), zm = wrap_dec(z, nz), zp = wrap_inc(z, nz);
        auto blk = [&](int yy, int zz) { return src + ((int64_t)zz * ny + yy) * Q * pitch; };
        const SrcP b00 = blk(y, z);
        const SrcP bm0 = blk(ym, z);
        const SrcP bp0 = blk(yp, z);
        const SrcP b0m = blk(y, zm);
        const SrcP b0p = blk(y, zp);
        const F16Params &f = a.f16;
        // slot i of the node x - e_i (the pull's source) and its byte offset in the row segment
        auto from = [&](int i) {
            return blk(kEy3[i] > 0 ? ym : (kEy3[i] < 0 ? yp : y), kEz3[i] > 0 ? zm : (kEz3[i] < 0 ? zp : z)) + i * pitch;
        };
        auto from_off = [&](int i) { return kEx3[i] > 0 ? bm : (kEx3[i] < 0 ? bp : bc); };
        M g[Q];
        if constexpr (IP == 2) {
#pragma unroll
            for (int i = 0; i < Q; ++i) g[i] = C::dec(ld_at(b00 + opp3(i) * pitch, bc), i, f);
        } else if constexpr (IP == 1) {
#pragma unroll
            for (int i = 0; i < Q; ++i) g[i] = C::dec(ld_at(from(i), from_off(i)), i, f);
        } else {
        g[0] = C::dec(ld_at(b00, bc), 0, f);
        g[1] = C::dec(ld_at(b00 + 1 * pitch, bm), 1, f);
        g[2] = C::dec(ld_at(b00 + 2 * pitch, bp), 2, f);
        g[3] = C::dec(ld_at(bm0 + 3 * pitch, bc), 3, f);
        g[4] = C::dec(ld_at(bp0 + 4 * pitch, bc), 4, f);
        g[5] = C::dec(ld_at(b0m + 5 * pitch, bc), 5, f);
        g[6] = C::dec(ld_at(b0p + 6 * pitch, bc), 6, f);
        g[7] = C::dec(ld_at(bm0 + 7 * pitch, bm), 7, f);
        g[8] = C::dec(ld_at(bp0 + 8 * pitch, bp), 8, f);
        g[9] = C::dec(ld_at(bp0 + 9 * pitch, bm), 9, f);
        g[10] = C::dec(ld_at(bm0 + 10 * pitch, bp), 10, f);
        g[11] = C::dec(ld_at(b0m + 11 * pitch, bm), 11, f);
        g[12] = C::dec(ld_at(b0p + 12 * pitch, bp), 12, f);
        g[13] = C::dec(ld_at(b0p + 13 * pitch, bm), 13, f);
        g[14] = C::dec(ld_at(b0m + 14 * pitch, bp), 14, f);
        g[15] = C::dec(ld_at(blk(ym, zm) + 15 * pitch, bc), 15, f);
        g[16] = C::dec(ld_at(blk(yp, zp) + 16 * pitch, bc), 16, f);
        g[17] = C::dec(ld_at(blk(ym, zp) + 17 * pitch, bc), 17, f);
        g[18] = C::dec(ld_at(blk(yp, zm) + 18 * pitch, bc), 18, f);
        if constexpr (Q == 27) {  // corners: pulled from (x - e_x, y - e_y, z - e_z)
            g[19] = C::dec(ld_at(blk(ym, zm) + 19 * pitch, bm), 19, f);
            g[20] = C::dec(ld_at(blk(yp, zp) + 20 * pitch, bp), 20, f);
            g[21] = C::dec(ld_at(blk(ym, zp) + 21 * pitch, bm), 21, f);
            g[22] = C::dec(ld_at(blk(yp, zm) + 22 * pitch, bp), 22, f);
            g[23] = C::dec(ld_at(blk(yp, zm) + 23 * pitch, bm), 23, f);
            g[24] = C::dec(ld_at(blk(ym, zp) + 24 * pitch, bp), 24, f);
            g[25] = C::dec(ld_at(blk(ym, zm) + 25 * pitch, bp), 25, f);
            g[26] = C::dec(ld_at(blk(yp, zp) + 26 * pitch, bm), 26, f);
        }
        }

        auto vrow = [&](int yy, int zz) { return u + ((int64_t)zz * ny + yy) * 3 * pitch; };
        const M *__restrict__ uc = vrow(y, z);
        const M ux = ld_at(uc, fc), uy = ld_at(uc + pitch, fc), uz = ld_at(uc + 2 * pitch, fc);
        M Ax = M(0), Ay = M(0), Az = M(0);
        if (AUX == 0) {  // Eq. (16): phi u_b d_b u_a, central differences of u
            M phi = g[0];
#pragma unroll
            for (int i = 1; i < Q; ++i) phi += g[i];
            const M *__restrict__ uym = vrow(ym, z), *__restrict__ uyp = vrow(yp, z);
            const M *__restrict__ uzm = vrow(y, zm), *__restrict__ uzp = vrow(y, zp);
            M dd[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const M dxc = ld_at(uc + c * pitch, fp) - ld_at(uc + c * pitch, fm);
                const M dyc = ld_at(uyp + c * pitch, fc) - ld_at(uym + c * pitch, fc);
                const M dzc = ld_at(uzp + c * pitch, fc) - ld_at(uzm + c * pitch, fc);
                dd[c] = M(0.5) * (ux * dxc + uy * dyc + uz * dzc);
            }
            Ax = phi * dd[0];
            Ay = phi * dd[1];
            Az = phi * dd[2];
        }
        const Relax<M> rr = HAS_K ? relax_from_k<M>(ld_at(kf + (int64_t)r * pitch, fc), (M)a.lambda, M(0)) : rconst;
        const M s = HAS_S ? ld_at(sf + (int64_t)r * pitch, fc) : M(0);
        M P[Q];
        collide3<Q, M>(g, ux, uy, uz, rr, Ax, Ay, Az, s, P);
        if (live && IP == 1) {  // P_j to the address of g_opp(j) (each value depends on all Q loads)
#pragma unroll
            for (int j = 0; j < Q; ++j) st_at(const_cast<T *>(from(opp3(j))), from_off(opp3(j)), C::enc(P[j], j, f));
        } else if (live) {
            const DstP out = dst + (int64_t)r * Q * pitch;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if constexpr (CST || IP != 0) st_at(out + i * pitch, bc, C::enc(P[i], i, f));
                else st_nt_at(out + i * pitch, bc, C::enc(P[i], i, f));
            }
        }
    }
}

template <int Q, int MODE>
__global__ __launch_bounds__(256) void init3_kernel(const InitArgs a)
{
    using St = typename ModeTraits<MODE>::St;
    using M = typename ModeTraits<MODE>::M;
    using T = typename St::T;
    using C = Codec<St, M>;
    const int nx = a.L.nx, ny = a.L.ny, nz = a.L.nz;
    const int64_t N = (int64_t)nx * ny * nz, pitch = a.L.pitch;
    T *dst = static_cast<T *>(a.dst);
    const M *u = static_cast<const M *>(a.u);
    bool bad = false;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(n % nx);
        const int64_t r = n / nx;
        const int y = (int)(r % ny), z = (int)(r / ny);
        const M *ur = u + r * 3 * pitch;
        M P[Q];
        equilibrium3<Q, M>((M)a.phi0[n], ur[x], ur[pitch + x], ur[2 * pitch + x], P);
#pragma unroll
        for (int i = 0; i < Q; ++i) {  // written pre-shifted: buf_i(x - e_i) = g_eq_i(x)
            int xd = x - kEx3[i], yd = y - kEy3[i], zd = z - kEz3[i];
            xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
            yd = yd < 0 ? yd + ny : (yd >= ny ? yd - ny : yd);
            zd = zd < 0 ? zd + nz : (zd >= nz ? zd - nz : zd);
            if (MODE == MODE_F16S_F32) {
                const float v = ((float)P[i] - a.f16.wref[i]) * a.f16.scale;
                bad |= !(fabsf(v) <= 65504.0f);
            }
            dst[(((int64_t)zd * ny + yd) * Q + i) * pitch + xd] = C::enc(P[i], i, a.f16);
        }
    }
    if (bad) *a.range_flag = 1;  // every writer stores the same value
}

template <int Q, int MODE>
__global__ __launch_bounds__(256) void macros3_kernel(const MacroArgs a)
{
    using St = typename ModeTraits<MODE>::St;
    using M = typename ModeTraits<MODE>::M;
    using T = typename St::T;
    const int nx = a.L.nx, ny = a.L.ny;
    const int64_t N = (int64_t)nx * ny * a.L.nz;
    const T *src = static_cast<const T *>(a.src);
    CSum cs[3] = {{0, 0}, {0, 0}, {0, 0}};  // mass, sum err^2, sum ref^2
    double maxerr = 0, maxphi = 0, nonfinite = 0;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(n % nx);
        const int64_t r = n / nx;
        M g[Q];
        state3<Q, St, M>(src, a.L, a.edge.kind, x, (int)(r % ny), (int)(r / ny), a.f16, g);
        double phi = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) phi += (double)g[i];
        if (a.phi_out) a.phi_out[n] = phi;
        if (!isfinite(phi)) {
            nonfinite += 1;
            continue;
        }
        csum_add(cs[0], phi);
        maxphi = fmax(maxphi, fabs(phi));
        if (a.ref) {
            const double rv = a.ref[n], d = phi - rv;
            csum_add(cs[1], d * d);
            csum_add(cs[2], rv * rv);
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

template <int Q, int MODE>
__global__ __launch_bounds__(256) void populations3_kernel(const PopArgs a)
{
    using St = typename ModeTraits<MODE>::St;
    using M = typename ModeTraits<MODE>::M;
    using T = typename St::T;
    const int nx = a.L.nx, ny = a.L.ny;
    const int64_t N = (int64_t)nx * ny * a.L.nz;
    const T *src = static_cast<const T *>(a.src);
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(n % nx);
        const int64_t r = n / nx;
        M g[Q];
        state3<Q, St, M>(src, a.L, a.edge.kind, x, (int)(r % ny), (int)(r / ny), a.f16, g);
#pragma unroll
        for (int i = 0; i < Q; ++i) a.out[i * N + n] = (double)g[i];
    }
}

template <int Q, int MODE, int AUX, int ROWS, bool CST, int IP = 0>
hipError_t launch_step3_rows(const StepArgs &a, hipStream_t st)
{
    dim3 block(64, 4);
    const int nblocks = tiles_of(a.d.L, a.d.lc.rows, a.d.lc.wide);
    const size_t lds = (size_t)a.d.lc.lds_reserve;  // unused LDS that caps the resident waves
    const bool hk = a.d.has_k, hs = a.d.has_s;
    if (hk && hs) step3_kernel<Q, MODE, AUX, true, true, ROWS, CST, IP><<<nblocks, block, lds, st>>>(a);
    else if (hk) step3_kernel<Q, MODE, AUX, true, false, ROWS, CST, IP><<<nblocks, block, lds, st>>>(a);
    else if (hs) step3_kernel<Q, MODE, AUX, false, true, ROWS, CST, IP><<<nblocks, block, lds, st>>>(a);
    else step3_kernel<Q, MODE, AUX, false, false, ROWS, CST, IP><<<nblocks, block, lds, st>>>(a);
    return hipGetLastError();
}

// Non-temporal or cached stores of the new state (Launch::stores 0 / 1), a compile-time choice.
template <int Q, int MODE, int AUX, int ROWS>
hipError_t launch_step3_st(const StepArgs &a, hipStream_t st)
{
    return a.d.lc.stores ? launch_step3_rows<Q, MODE, AUX, ROWS, true>(a, st)
                         : launch_step3_rows<Q, MODE, AUX, ROWS, false>(a, st);
}

// One buffer in place (stores 2; one row per wave): the one-row instantiation, whose Q loads and
// stores keep the scalar-base + 32-bit-offset form (the walking loop's 64-bit addresses would keep
// up to 27 store addresses in vector registers).
template <int Q, int MODE, int AUX>
hipError_t launch_step3_aux(const StepArgs &a, hipStream_t st)
{
    if (a.d.lc.stores == 2) {  // never chosen with FP64 math (its in-place collision rounds differently)
        if constexpr (MODE != MODE_F64_F64) {
            if (a.d.lc.rows != 1) return hipErrorInvalidValue;
            return a.parity == 0 ? launch_step3_rows<Q, MODE, AUX, 1, true, 1>(a, st)
                                 : launch_step3_rows<Q, MODE, AUX, 1, true, 2>(a, st);
        }
        return hipErrorInvalidValue;
    }
    if constexpr (MODE == MODE_F16S_F32) {
        if (a.d.lc.rows == 1) return launch_step3_st<Q, MODE, AUX, 1>(a, st);
    }
    return launch_step3_st<Q, MODE, AUX, 0>(a, st);
}

template <int Q, int MODE>
hipError_t launch_step3_mode(int aux, const StepArgs &a, hipStream_t st)
{
    switch (aux) {
    case 0: return launch_step3_aux<Q, MODE, 0>(a, st);
    case 2: return launch_step3_aux<Q, MODE, 2>(a, st);
    default: return hipErrorInvalidValue;  // the flux form is two-dimensional only
    }
}

}  // namespace

hipError_t launch_step3(int mode, int aux, const StepArgs &a, hipStream_t st)
{
    if (a.d.lc.rows < 1 || a.d.lc.rows > 64 || a.d.lc.lds_reserve < 0 || a.d.lc.lds_reserve > 65536)
        return hipErrorInvalidValue;
    if (a.d.L.q != 19 && a.d.L.q != 27) return hipErrorInvalidValue;
    const bool q27 = a.d.L.q == 27;
    switch (mode) {
    case MODE_F64_F64:
        return q27 ? launch_step3_mode<27, MODE_F64_F64>(aux, a, st) : launch_step3_mode<19, MODE_F64_F64>(aux, a, st);
    case MODE_F64_F32:
        return q27 ? launch_step3_mode<27, MODE_F64_F32>(aux, a, st) : launch_step3_mode<19, MODE_F64_F32>(aux, a, st);
    case MODE_F32_F32:
        return q27 ? launch_step3_mode<27, MODE_F32_F32>(aux, a, st) : launch_step3_mode<19, MODE_F32_F32>(aux, a, st);
    case MODE_F16S_F32:
        return q27 ? launch_step3_mode<27, MODE_F16S_F32>(aux, a, st) : launch_step3_mode<19, MODE_F16S_F32>(aux, a, st);
    default: return hipErrorInvalidValue;
    }
}

namespace {

template <int Q>
hipError_t launch_init3_q(int mode, const InitArgs &a, hipStream_t st)
{
    const int g = grid_for((int64_t)a.L.nx * a.L.ny * a.L.nz, 256, 8192);
    switch (mode) {
    case MODE_F64_F64: init3_kernel<Q, MODE_F64_F64><<<g, 256, 0, st>>>(a); break;
    case MODE_F64_F32: init3_kernel<Q, MODE_F64_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F32_F32: init3_kernel<Q, MODE_F32_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F16S_F32: init3_kernel<Q, MODE_F16S_F32><<<g, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int Q>
hipError_t launch_macros3_q(int mode, const MacroArgs &a, double *result, hipStream_t st)
{
    const int g = grid_for((int64_t)a.L.nx * a.L.ny * a.L.nz, 256, kMacroBlocks);
    switch (mode) {
    case MODE_F64_F64: macros3_kernel<Q, MODE_F64_F64><<<g, 256, 0, st>>>(a); break;
    case MODE_F64_F32: macros3_kernel<Q, MODE_F64_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F32_F32: macros3_kernel<Q, MODE_F32_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F16S_F32: macros3_kernel<Q, MODE_F16S_F32><<<g, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_macros_finalize(a.partials, g, result, st);
}

template <int Q>
hipError_t launch_populations3_q(int mode, const PopArgs &a, hipStream_t st)
{
    const int g = grid_for((int64_t)a.L.nx * a.L.ny * a.L.nz, 256, 8192);
    switch (mode) {
    case MODE_F64_F64: populations3_kernel<Q, MODE_F64_F64><<<g, 256, 0, st>>>(a); break;
    case MODE_F64_F32: populations3_kernel<Q, MODE_F64_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F32_F32: populations3_kernel<Q, MODE_F32_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F16S_F32: populations3_kernel<Q, MODE_F16S_F32><<<g, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_init3(int mode, const InitArgs &a, hipStream_t st)
{
    if (a.L.q == 27) return launch_init3_q<27>(mode, a, st);
    if (a.L.q == 19) return launch_init3_q<19>(mode, a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_macros3(int mode, const MacroArgs &a, double *result, hipStream_t st)
{
    if (a.L.q == 27) return launch_macros3_q<27>(mode, a, result, st);
    if (a.L.q == 19) return launch_macros3_q<19>(mode, a, result, st);
    return hipErrorInvalidValue;
}

hipError_t launch_populations3(int mode, const PopArgs &a, hipStream_t st)
{
    if (a.L.q == 27) return launch_populations3_q<27>(mode, a, st);
    if (a.L.q == 19) return launch_populations3_q<19>(mode, a, st);
    return hipErrorInvalidValue;
}

namespace {

// The 3D form of the D2Q9 relayout: dst[z][j] = src[z + e_j][opp(j)] (its own inverse); raw storage
// elements, padding columns written as zero.
template <int Q, class E>
__global__ __launch_bounds__(256) void relayout3_kernel(const E *__restrict__ src, E *__restrict__ dst, Layout L)
{
    const int64_t n = rows_of(L) * L.pitch;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(k % L.pitch);
        const int64_t r = k / L.pitch;
        const int y = (int)(r % L.ny), z = (int)(r / L.ny);
        const bool live = x < L.nx;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            int xs = x + kEx3[j], ys = y + kEy3[j], zs = z + kEz3[j];
            xs = xs < 0 ? L.nx - 1 : (xs == L.nx ? 0 : xs);
            ys = ys < 0 ? L.ny - 1 : (ys == L.ny ? 0 : ys);
            zs = zs < 0 ? L.nz - 1 : (zs == L.nz ? 0 : zs);
            dst[(r * Q + j) * L.pitch + x] =
                live ? src[(((int64_t)zs * L.ny + ys) * Q + opp3(j)) * L.pitch + xs] : E(0);
        }
    }
}

template <int Q>
hipError_t relayout3_q(size_t elem_bytes, const void *src, void *dst, const Layout &L, hipStream_t st)
{
    const int64_t n = rows_of(L) * L.pitch;
    const int g = (int)std::min<int64_t>((n + 255) / 256, 8192);
    switch (elem_bytes) {
    case 2: relayout3_kernel<Q, uint16_t><<<g, 256, 0, st>>>(static_cast<const uint16_t *>(src), static_cast<uint16_t *>(dst), L); break;
    case 4: relayout3_kernel<Q, uint32_t><<<g, 256, 0, st>>>(static_cast<const uint32_t *>(src), static_cast<uint32_t *>(dst), L); break;
    case 8: relayout3_kernel<Q, uint64_t><<<g, 256, 0, st>>>(static_cast<const uint64_t *>(src), static_cast<uint64_t *>(dst), L); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_relayout3(size_t elem_bytes, const void *src, void *dst, const Layout &L, hipStream_t st)
{
    if (src == dst) return hipErrorInvalidValue;
    if (L.q == 27) return relayout3_q<27>(elem_bytes, src, dst, L, st);
    if (L.q == 19) return relayout3_q<19>(elem_bytes, src, dst, L, st);
    return hipErrorInvalidValue;
}

}  // namespace lbm
