// lbm_adjoint.hip -- adjoint (reverse-mode) kernels of the TRT-R D2Q9 step for gfx950.
//
// With u, D and S fixed, one step of Sec. 2.2, Eq. (14) is affine in the pre-collision populations:
//   g^{n+1}_i(x + e_i) = sum_j M_ij(x) g^n_j(x) + c_i(x),   M(x) = dP(x)/dg(x),
// because the equilibrium (Eq. (6)) and the auxiliary term (Eq. (16), with phi at the node) are linear
// in phi = sum_j g_j, and the non-equilibrium projections (Eqs. (8), (13)) are linear in g.  The
// adjoint step is therefore
//   lam^n_j(x) = sum_i M_ij(x) mu_i(x),   mu_i(x) = lam^{n+1}_i(x + e_i),
// and, since D(x) enters only the collision at x (through tau1, tau2 and beta, Sec. 2.4),
//   dL/dD(x) += sum_i mu_i(x) dP_i(x)/dD(x) |_{g^n(x)}.
// M = H C R factorises through moments (R: raw moments phi, j, Pi of g; C: the post-collision Hermite
// coefficients a0..a3 as functions of those moments; H: the reconstruction w_i h_m(e_i)), so M^T mu
// is computed as R^T C^T H^T mu without forming M.  All in lattice units, like the forward kernel.
#include "lbm_internal.h"
#include "lbm_kernel_common.h"

namespace lbm {
namespace {

template <int MODE>
struct AdjTraits;
template <>
struct AdjTraits<MODE_F64_F64> {
    using St = StoreF64;
    using M = double;
};
template <>
struct AdjTraits<MODE_F64_F32> {
    using St = StoreF64;
    using M = float;
};
template <>
struct AdjTraits<MODE_F32_F32> {
    using St = StoreF32;
    using M = float;
};

__device__ __forceinline__ int wdec(int v, int n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ int winc(int v, int n) { return v == n - 1 ? 0 : v + 1; }

// Block (64, 4): lane = column, wave = row.
template <int MODE, bool HAS_K, bool HAS_S, bool LOCAL>
__global__ __launch_bounds__(256) void adjoint_kernel(const AdjArgs a)
{
    using St = typename AdjTraits<MODE>::St;
    using M = typename AdjTraits<MODE>::M;
    using T = typename St::T;
    using C = Codec<St, M>;
    // Tiles of 256 columns (the block's four waves side by side, lane = column) by one row, in row bands
    // over the XCDs (each XCD's rows and their neighbours in one L2); the row is uniform, so every
    // access is a scalar row base plus a 32-bit lane offset.
    const int nx = a.L.nx, ny = a.L.ny;
    const int64_t pitch = a.L.pitch;
    const int ntx = (nx + 255) / 256;
    const int t = tile_of_block(blockIdx.x, gridDim.x, 1, ntx, 0);
    const int y = __builtin_amdgcn_readfirstlane(t / ntx);
    const int x = (t % ntx) * 256 + __builtin_amdgcn_readfirstlane((int)threadIdx.y) * 64 + (int)threadIdx.x;
    if (x >= nx) return;
    const unsigned xc = (unsigned)x, xm = (unsigned)wdec(x, nx), xp = (unsigned)winc(x, nx);
    const int ym = __builtin_amdgcn_readfirstlane(wdec(y, ny)), yp = __builtin_amdgcn_readfirstlane(winc(y, ny));
    const unsigned bc = xc * (unsigned)sizeof(T), bm = xm * (unsigned)sizeof(T), bp = xp * (unsigned)sizeof(T);
    const unsigned fc = xc * (unsigned)sizeof(M), fm = xm * (unsigned)sizeof(M), fp = xp * (unsigned)sizeof(M);
    const T *st = static_cast<const T *>(a.state);
    const M *lin = static_cast<const M *>(a.lam_in);
    M *lout = static_cast<M *>(a.lam_out);
    const M *u = static_cast<const M *>(a.u);

    // forward pre-collision state g^n(x) = buf_i(x - e_i)
    M g[9];
    {
        const T *rm = st + (int64_t)ym * 9 * pitch, *rc = st + (int64_t)y * 9 * pitch, *rp = st + (int64_t)yp * 9 * pitch;
        g[0] = C::dec(ld_at(rc, bc), 0, a.f16);
        g[1] = C::dec(ld_at(rc + 1 * pitch, bm), 1, a.f16);
        g[2] = C::dec(ld_at(rm + 2 * pitch, bc), 2, a.f16);
        g[3] = C::dec(ld_at(rc + 3 * pitch, bp), 3, a.f16);
        g[4] = C::dec(ld_at(rp + 4 * pitch, bc), 4, a.f16);
        g[5] = C::dec(ld_at(rm + 5 * pitch, bm), 5, a.f16);
        g[6] = C::dec(ld_at(rm + 6 * pitch, bp), 6, a.f16);
        g[7] = C::dec(ld_at(rp + 7 * pitch, bp), 7, a.f16);
        g[8] = C::dec(ld_at(rp + 8 * pitch, bm), 8, a.f16);
    }
    // mu_i(x) = lam^{n+1}_i(x + e_i)
    M mu[9];
    {
        const M *lm = lin + (int64_t)ym * 9 * pitch, *lc = lin + (int64_t)y * 9 * pitch, *lp = lin + (int64_t)yp * 9 * pitch;
        mu[0] = ld_at(lc, fc);
        mu[1] = ld_at(lc + 1 * pitch, fp);
        mu[2] = ld_at(lp + 2 * pitch, fc);
        mu[3] = ld_at(lc + 3 * pitch, fm);
        mu[4] = ld_at(lm + 4 * pitch, fc);
        mu[5] = ld_at(lp + 5 * pitch, fp);
        mu[6] = ld_at(lp + 6 * pitch, fm);
        mu[7] = ld_at(lm + 7 * pitch, fm);
        mu[8] = ld_at(lm + 8 * pitch, fp);
    }
    const M *uc = u + (int64_t)y * 2 * pitch;
    const M ux = ld_at(uc, fc), uy = ld_at(uc + pitch, fc);
    M ahx = M(0), ahy = M(0);  // u_b d_b u_a (central differences), Eq. (16) without phi
    if (LOCAL) {
        const M *um = u + (int64_t)ym * 2 * pitch, *up = u + (int64_t)yp * 2 * pitch;
        ahx = ux * (ld_at(uc, fp) - ld_at(uc, fm)) * M(0.5) + uy * (ld_at(up, fc) - ld_at(um, fc)) * M(0.5);
        ahy = ux * (ld_at(uc + pitch, fp) - ld_at(uc + pitch, fm)) * M(0.5) +
              uy * (ld_at(up + pitch, fc) - ld_at(um + pitch, fc)) * M(0.5);
    }
    const M k = HAS_K ? ld_at(static_cast<const M *>(a.k) + (int64_t)y * pitch, fc) : (M)a.k_const;
    const M s = HAS_S ? ld_at(static_cast<const M *>(a.s) + (int64_t)y * pitch, fc) : M(0);
    const M lam = (M)a.lambda;
    const M tau1 = M(0.5) + k, tau2 = M(0.5) + lam / k;
    const M w1 = M(1) - M(1) / tau1, w2 = M(1) - M(1) / tau2, beta = M(1) - M(0.5) / tau1;

    // q = H^T mu: the Hermite "moments" of mu weighted as in the reconstruction
    M q0 = 0, q1x = 0, q1y = 0, q2xx = 0, q2yy = 0, q2xy = 0, q3xxy = 0, q3xyy = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const M wm = M(kW[i]) * mu[i];
        const int ex = kEx[i], ey = kEy[i];
        q0 += wm;
        if (ex) q1x += M(3 * ex) * wm;
        if (ey) q1y += M(3 * ey) * wm;
        q2xx += M(4.5 * (ex * ex - 1.0 / 3.0)) * wm;
        q2yy += M(4.5 * (ey * ey - 1.0 / 3.0)) * wm;
        if (ex * ey) q2xy += M(9 * ex * ey) * wm;
        if (ey) q3xxy += M(13.5 * (ex * ex * ey - ey / 3.0)) * wm;
        if (ex) q3xyy += M(13.5 * (ex * ey * ey - ex / 3.0)) * wm;
    }
    // t = C^T q (derivatives of the Hermite coefficients with respect to phi, j, Pi)
    const M uxx = ux * ux, uyy = uy * uy, uxy = ux * uy;
    const M tphi = q0 + q1x * (ux * (M(1) - w1) + beta * ahx) + q1y * (uy * (M(1) - w1) + beta * ahy) +
                   q2xx * (uxx * (M(1) - w2) - w2 * M(1.0 / 3.0)) + q2yy * (uyy * (M(1) - w2) - w2 * M(1.0 / 3.0)) +
                   q2xy * uxy * (M(1) - w2) + q3xxy * uxx * uy + q3xyy * ux * uyy;
    const M tjx = w1 * q1x, tjy = w1 * q1y, tpxx = w2 * q2xx, tpyy = w2 * q2yy, tpxy = w2 * q2xy;
    // lam^n = R^T t
    M *lo = lout + (int64_t)y * 9 * pitch;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const int ex = kEx[j], ey = kEy[j];
        M v = tphi;
        if (ex) v += M(ex) * tjx + tpxx;
        if (ey) v += M(ey) * tjy + tpyy;
        if (ex * ey) v += M(ex * ey) * tpxy;
        st_at(lo + j * pitch, fc, v);
    }

    // dP/dk at g^n(x): tau1 = 1/2 + k, tau2 = 1/2 + Lambda/k
    const M phi = g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8];
    const M jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const M jy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const M sd = (g[5] + g[6]) + (g[7] + g[8]);
    const M nxx = g[1] + g[3] + sd - phi * M(1.0 / 3.0) - phi * uxx;
    const M nyy = g[2] + g[4] + sd - phi * M(1.0 / 3.0) - phi * uyy;
    const M nxy = (g[5] + g[7]) - (g[6] + g[8]) - phi * uxy;
    const M dw1 = M(1) / (tau1 * tau1), dbeta = M(0.5) / (tau1 * tau1), dw2 = -lam / (k * k * tau2 * tau2);
    const M dk = q1x * (dw1 * (jx - phi * ux) + dbeta * (phi * ahx + ux * s)) +
                 q1y * (dw1 * (jy - phi * uy) + dbeta * (phi * ahy + uy * s)) +
                 dw2 * (q2xx * nxx + q2yy * nyy + q2xy * nxy);
    double *gr = a.grad + (int64_t)y * nx;
    gr[x] += a.dk_dD * (double)dk;
}

// lam_i(x) = dL/dphi(x) for every i (adjoint of phi = sum_i g_i)
template <class M>
__global__ __launch_bounds__(256) void adjoint_seed_kernel(const double *dphi, M *lam, Layout L)
{
    const int64_t N = (int64_t)L.nx * L.ny;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(n % L.nx), y = (int)(n / L.nx);
        const M v = (M)dphi[n];
#pragma unroll
        for (int i = 0; i < 9; ++i) lam[((int64_t)y * 9 + i) * L.pitch + x] = v;
    }
}

// dL/dphi0(x) = sum_i lam0_i(x) dg_eq_i/dphi0(x) (adjoint of the initial condition g = g_eq(phi0, u))
template <class M>
__global__ __launch_bounds__(256) void adjoint_init_kernel(const M *lam, const M *u, double *dphi0, Layout L)
{
    const int64_t N = (int64_t)L.nx * L.ny;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(n % L.nx), y = (int)(n / L.nx);
        M e[9];
        equilibrium<M>(M(1), u[(int64_t)y * 2 * L.pitch + x], u[((int64_t)y * 2 + 1) * L.pitch + x], e);
        double acc = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) acc += (double)(e[i] * lam[((int64_t)y * 9 + i) * L.pitch + x]);
        dphi0[n] = acc;
    }
}

template <int MODE, bool LOCAL>
hipError_t launch_adj_aux(const AdjArgs &a, hipStream_t st)
{
    dim3 block(64, 4);
    const int grid = ((a.L.nx + 255) / 256) * a.L.ny;  // 256-column tiles of one row
    const bool hk = a.k != nullptr, hs = a.s != nullptr;
    if (hk && hs) adjoint_kernel<MODE, true, true, LOCAL><<<grid, block, 0, st>>>(a);
    else if (hk) adjoint_kernel<MODE, true, false, LOCAL><<<grid, block, 0, st>>>(a);
    else if (hs) adjoint_kernel<MODE, false, true, LOCAL><<<grid, block, 0, st>>>(a);
    else adjoint_kernel<MODE, false, false, LOCAL><<<grid, block, 0, st>>>(a);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_adj_mode(int aux, const AdjArgs &a, hipStream_t st)
{
    return aux == 0 ? launch_adj_aux<MODE, true>(a, st) : launch_adj_aux<MODE, false>(a, st);
}

int adj_grid(const Layout &L)
{
    int64_t g = ((int64_t)L.nx * L.ny + 255) / 256;
    return (int)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

}  // namespace

hipError_t launch_adjoint(int mode, int aux, const AdjArgs &a, hipStream_t st)
{
    switch (mode) {
    case MODE_F64_F64: return launch_adj_mode<MODE_F64_F64>(aux, a, st);
    case MODE_F64_F32: return launch_adj_mode<MODE_F64_F32>(aux, a, st);
    case MODE_F32_F32: return launch_adj_mode<MODE_F32_F32>(aux, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_seed(int mode, const double *dphi, void *lam, const Layout &L, hipStream_t st)
{
    if (mode == MODE_F64_F64) adjoint_seed_kernel<double><<<adj_grid(L), 256, 0, st>>>(dphi, static_cast<double *>(lam), L);
    else adjoint_seed_kernel<float><<<adj_grid(L), 256, 0, st>>>(dphi, static_cast<float *>(lam), L);
    return hipGetLastError();
}

hipError_t launch_adjoint_init(int mode, const void *lam, const void *u, double *dphi0, const Layout &L, hipStream_t st)
{
    if (mode == MODE_F64_F64)
        adjoint_init_kernel<double><<<adj_grid(L), 256, 0, st>>>(static_cast<const double *>(lam), static_cast<const double *>(u), dphi0, L);
    else
        adjoint_init_kernel<float><<<adj_grid(L), 256, 0, st>>>(static_cast<const float *>(lam), static_cast<const float *>(u), dphi0, L);
    return hipGetLastError();
}

}  // namespace lbm
