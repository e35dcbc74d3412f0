// lbm_kernels.hip -- HIP kernels of the TRT-R D2Q9 step for gfx950.
//
// State convention (pull scheme): buffer A holds, at node y, the post-collision values P_i(y)
// computed there in the previous step.  The pre-collision population at x is therefore
// g_i(x) = A_i(x - e_i) (streaming of Sec. 2.2, Eq. (14)), and one step reads A with those shifts
// and writes P_i(x) to buffer B at x.  The initial buffer is written pre-shifted
// (A_i(x - e_i) = g_eq_i(phi0(x), u(x))) so that the first pull yields g = g_eq(phi0, u).
#include "lbm_internal.h"

namespace lbm {
namespace {

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

__device__ __forceinline__ int wrap_dec(int v, int n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ int wrap_inc(int v, int n) { return v == n - 1 ? 0 : v + 1; }

// g_i(x, y) = buf_i(x - e_i): row offsets rm = (y-1)*pitch, rc = y*pitch, rp = (y+1)*pitch (wrapped)
// and columns xm = x-1, xp = x+1 (wrapped).
template <class St, class M>
__device__ __forceinline__ void pull(const typename St::T *__restrict__ src, int64_t plane, int64_t rm,
                                     int64_t rc, int64_t rp, int xm, int x, int xp,
                                     const F16Params &f, M (&g)[9])
{
    using C = Codec<St, M>;
    g[0] = C::dec(src[0 * plane + rc + x], 0, f);
    g[1] = C::dec(src[1 * plane + rc + xm], 1, f);
    g[2] = C::dec(src[2 * plane + rm + x], 2, f);
    g[3] = C::dec(src[3 * plane + rc + xp], 3, f);
    g[4] = C::dec(src[4 * plane + rp + x], 4, f);
    g[5] = C::dec(src[5 * plane + rm + xm], 5, f);
    g[6] = C::dec(src[6 * plane + rm + xp], 6, f);
    g[7] = C::dec(src[7 * plane + rp + xp], 7, f);
    g[8] = C::dec(src[8 * plane + rp + xm], 8, f);
}

template <class St, class M>
__device__ __forceinline__ M phi_at(const typename St::T *__restrict__ src, const Layout &L, int x, int y,
                                    const F16Params &f)
{
    const int xm = wrap_dec(x, L.nx), xp = wrap_inc(x, L.nx);
    const int64_t rm = (int64_t)wrap_dec(y, L.ny) * L.pitch, rc = (int64_t)y * L.pitch,
                  rp = (int64_t)wrap_inc(y, L.ny) * L.pitch;
    M g[9];
    pull<St, M>(src, L.plane, rm, rc, rp, xm, x, xp, f, g);
    return g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8];
}

// One step.  Block (64, 4): lane x covers one column, each of the 4 waves walks `rows` rows.
template <int MODE, int AUX, bool HAS_K, bool HAS_S>
__global__ __launch_bounds__(256) void step_kernel(const StepArgs a)
{
    using St = typename ModeTraits<MODE>::St;
    using M = typename ModeTraits<MODE>::M;
    using T = typename St::T;
    using C = Codec<St, M>;
    const int nx = a.L.nx, ny = a.L.ny;
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y0 = (blockIdx.y * 4 + threadIdx.y) * a.rows;
    if (x >= nx || y0 >= ny) return;
    const int y1 = min(y0 + a.rows, ny);
    const int xm = wrap_dec(x, nx), xp = wrap_inc(x, nx);
    const int64_t pitch = a.L.pitch, plane = a.L.plane;
    const T *__restrict__ src = static_cast<const T *>(a.src);
    T *__restrict__ dst = static_cast<T *>(a.dst);
    const M *__restrict__ ux = static_cast<const M *>(a.ux);
    const M *__restrict__ uy = static_cast<const M *>(a.uy);
    const M *__restrict__ kf = static_cast<const M *>(a.k);
    const M *__restrict__ sf = static_cast<const M *>(a.s);
    const M lam = (M)a.lambda;
    Relax<M> rconst{};
    if (!HAS_K) rconst = relax_from_k<M>((M)a.k_const, lam);

    // u in this column at y-1 and y (rolled down the walk)
    int yprev = wrap_dec(y0, ny);
    M ux_m = ux[(int64_t)yprev * pitch + x], uy_m = uy[(int64_t)yprev * pitch + x];
    M ux_c = ux[(int64_t)y0 * pitch + x], uy_c = uy[(int64_t)y0 * pitch + x];

    for (int y = y0; y < y1; ++y) {
        const int yn = wrap_inc(y, ny);
        const int64_t rm = (int64_t)wrap_dec(y, ny) * pitch, rc = (int64_t)y * pitch, rp = (int64_t)yn * pitch;
        M g[9];
        pull<St, M>(src, plane, rm, rc, rp, xm, x, xp, a.f16, g);
        const M ux_p = ux[rp + x], uy_p = uy[rp + x];

        M Ax = M(0), Ay = M(0);
        if (AUX == 0) {  // Eq. (16): phi u_b d_b u_a, central differences of u
            const M phi = g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8];
            const M dxux = (ux[rc + xp] - ux[rc + xm]) * M(0.5);
            const M dxuy = (uy[rc + xp] - uy[rc + xm]) * M(0.5);
            const M dyux = (ux_p - ux_m) * M(0.5);
            const M dyuy = (uy_p - uy_m) * M(0.5);
            Ax = phi * (ux_c * dxux + uy_c * dyux);
            Ay = phi * (ux_c * dxuy + uy_c * dyuy);
        } else if (AUX == 1) {  // d_b(phi u_a u_b) - u_a d_b(phi u_b), phi at the axis neighbours
            const M pw = phi_at<St, M>(src, a.L, xm, y, a.f16);
            const M pe = phi_at<St, M>(src, a.L, xp, y, a.f16);
            const M ps = phi_at<St, M>(src, a.L, x, wrap_dec(y, ny), a.f16);
            const M pn = phi_at<St, M>(src, a.L, x, yn, a.f16);
            const M uxw = ux[rc + xm], uyw = uy[rc + xm], uxe = ux[rc + xp], uye = uy[rc + xp];
            const M fwx = pw * uxw, fex = pe * uxe;    // phi u_x at the west and east neighbours
            const M fsy = ps * uy_m, fny = pn * uy_p;  // phi u_y at the south and north neighbours
            const M div = (fex - fwx) * M(0.5) + (fny - fsy) * M(0.5);
            Ax = (fex * uxe - fwx * uxw) * M(0.5) + (fny * ux_p - fsy * ux_m) * M(0.5) - ux_c * div;
            Ay = (fex * uye - fwx * uyw) * M(0.5) + (fny * uy_p - fsy * uy_m) * M(0.5) - uy_c * div;
        }
        const Relax<M> r = HAS_K ? relax_from_k<M>(kf[rc + x], lam) : rconst;
        const M s = HAS_S ? sf[rc + x] : M(0);
        M P[9];
        collide<M>(g, ux_c, uy_c, r, Ax, Ay, s, P);
#pragma unroll
        for (int i = 0; i < 9; ++i) dst[i * plane + rc + x] = C::enc(P[i], i, a.f16);
        ux_m = ux_c;
        uy_m = uy_c;
        ux_c = ux_p;
        uy_c = uy_p;
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
    const int64_t N = (int64_t)nx * ny;
    T *dst = static_cast<T *>(a.dst);
    const M *ux = static_cast<const M *>(a.ux);
    const M *uy = static_cast<const M *>(a.uy);
    bool bad = false;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(n % nx), y = (int)(n / nx);
        const int64_t q = (int64_t)y * a.L.pitch + x;
        M P[9];
        equilibrium<M>((M)a.phi0[n], ux[q], uy[q], P);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int xd = x - kEx[i], yd = y - kEy[i];
            xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
            yd = yd < 0 ? yd + ny : (yd >= ny ? yd - ny : yd);
            if (MODE == MODE_F16S_F32) {
                const float v = ((float)P[i] - a.f16.wref[i]) * a.f16.scale;
                bad |= !(fabsf(v) <= 65504.0f);
            }
            dst[i * a.L.plane + (int64_t)yd * a.L.pitch + xd] = C::enc(P[i], i, a.f16);
        }
    }
    if (bad) *a.range_flag = 1;  // every writer stores the same value
}

template <class M>
__global__ __launch_bounds__(256) void prep_kernel(const PrepArgs a)
{
    const int nx = a.L.nx;
    const int64_t N = (int64_t)nx * a.L.ny;
    M *out = static_cast<M *>(a.out);
    bool bad = false;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(n % nx), y = (int)(n / nx);
        double v = a.ca * a.a[n];
        if (a.b) v += a.cb * a.b[n];
        if (a.check_positive) bad |= !(v > 0.0 && v < INFINITY);
        out[(int64_t)y * a.L.pitch + x] = (M)v;
    }
    if (bad) *a.flag = 1;  // every writer stores the same value
}

// ---- diagnostics -------------------------------------------------------------------------------

__device__ __forceinline__ CSum csum_shfl_xor(CSum v, int m)
{
    CSum o;
    o.s = __shfl_xor(v.s, m);
    o.c = __shfl_xor(v.c, m);
    return o;
}

// Reduces (3 compensated sums, 2 maxima, 1 count) over the block; thread 0 gets the result.
__device__ void block_reduce(CSum (&cs)[3], double &mx0, double &mx1, double &cnt)
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
        const int xm = wrap_dec(x, nx), xp = wrap_inc(x, nx);
        const int64_t rm = (int64_t)wrap_dec(y, ny) * a.L.pitch, rc = (int64_t)y * a.L.pitch,
                      rp = (int64_t)wrap_inc(y, ny) * a.L.pitch;
        M g[9];
        pull<St, M>(src, a.L.plane, rm, rc, rp, xm, x, xp, a.f16, g);
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
        const int xm = wrap_dec(x, nx), xp = wrap_inc(x, nx);
        const int64_t rm = (int64_t)wrap_dec(y, ny) * a.L.pitch, rc = (int64_t)y * a.L.pitch,
                      rp = (int64_t)wrap_inc(y, ny) * a.L.pitch;
        M g[9];
        pull<St, M>(src, a.L.plane, rm, rc, rp, xm, x, xp, a.f16, g);
#pragma unroll
        for (int i = 0; i < 9; ++i) a.out[i * N + n] = (double)g[i];
    }
}

int grid_for(int64_t n, int block, int cap)
{
    int64_t g = (n + block - 1) / block;
    if (g > cap) g = cap;
    return (int)(g < 1 ? 1 : g);
}

template <int MODE, int AUX>
hipError_t launch_step_aux(const StepArgs &a, hipStream_t st)
{
    dim3 block(64, 4);
    const int waves_y = (a.L.ny + a.rows - 1) / a.rows;
    dim3 grid((a.L.nx + 63) / 64, (waves_y + 3) / 4);
    const bool hk = a.k != nullptr, hs = a.s != nullptr;
    if (hk && hs) step_kernel<MODE, AUX, true, true><<<grid, block, 0, st>>>(a);
    else if (hk) step_kernel<MODE, AUX, true, false><<<grid, block, 0, st>>>(a);
    else if (hs) step_kernel<MODE, AUX, false, true><<<grid, block, 0, st>>>(a);
    else step_kernel<MODE, AUX, false, false><<<grid, block, 0, st>>>(a);
    return hipGetLastError();
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

}  // namespace

hipError_t launch_step(int mode, int aux, const StepArgs &a, hipStream_t st)
{
    switch (mode) {
    case MODE_F64_F64: return launch_step_mode<MODE_F64_F64>(aux, a, st);
    case MODE_F64_F32: return launch_step_mode<MODE_F64_F32>(aux, a, st);
    case MODE_F32_F32: return launch_step_mode<MODE_F32_F32>(aux, a, st);
    case MODE_F16S_F32: return launch_step_mode<MODE_F16S_F32>(aux, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init(int mode, const InitArgs &a, hipStream_t st)
{
    const int g = grid_for((int64_t)a.L.nx * a.L.ny, 256, 8192);
    switch (mode) {
    case MODE_F64_F64: init_kernel<MODE_F64_F64><<<g, 256, 0, st>>>(a); break;
    case MODE_F64_F32: init_kernel<MODE_F64_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F32_F32: init_kernel<MODE_F32_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F16S_F32: init_kernel<MODE_F16S_F32><<<g, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_prep(int mode, const PrepArgs &a, hipStream_t st)
{
    const int g = grid_for((int64_t)a.L.nx * a.L.ny, 256, 8192);
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
    case MODE_F16S_F32: macros_kernel<MODE_F16S_F32><<<g, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    macros_finalize<<<1, 256, 0, st>>>(a.partials, g, result);
    return hipGetLastError();
}

hipError_t launch_populations(int mode, const PopArgs &a, hipStream_t st)
{
    const int g = grid_for((int64_t)a.L.nx * a.L.ny, 256, 8192);
    switch (mode) {
    case MODE_F64_F64: populations_kernel<MODE_F64_F64><<<g, 256, 0, st>>>(a); break;
    case MODE_F64_F32: populations_kernel<MODE_F64_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F32_F32: populations_kernel<MODE_F32_F32><<<g, 256, 0, st>>>(a); break;
    case MODE_F16S_F32: populations_kernel<MODE_F16S_F32><<<g, 256, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm
