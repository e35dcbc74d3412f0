// lbm_internal.h -- memory layout, argument blocks and launchers shared by the C-ABI layer and the
// kernels.
//
// HBM layout of one instance (element = storage type for populations, math type for fields):
//   populations  [ny][9][pitch]   element (i, y, x) at (y*9 + i)*pitch + x   ("row-interleaved")
//   velocity     [ny][2][pitch]   u_x at (y*2)*pitch + x, u_y at (y*2 + 1)*pitch + x
//   k, s         [ny][pitch]      scalar fields at y*pitch + x
// A D3Q19 (D3Q27) instance has ny*nz rows, row r = z*ny + y: populations [nz][ny][19 (27)][pitch],
// velocity [nz][ny][3][pitch], k and s [nz][ny][pitch].
// pitch = nx rounded up to a multiple of 64 elements, so every row segment starts 128-byte aligned for
// every element size.  Keeping the nine segments of one lattice row next to each other turns the 18
// concurrent streams of a step (9 reads at rows y-1, y, y+1 and 9 writes at row y) into accesses to
// three neighbouring ~9*pitch windows, which the HBM serves closer to copy bandwidth than nine separate
// planes.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lbm_device.h"

namespace lbm {

// Storage x arithmetic combinations that have kernels.
enum Mode : int {
    MODE_F64_F64 = 0,  // FP64 storage, FP64 math
    MODE_F64_F32 = 1,  // FP64 storage, FP32 math
    MODE_F32_F32 = 2,  // FP32 storage, FP32 math
    MODE_F16S_F32 = 3,  // shifted/scaled FP16 storage, FP32 math
    MODE_F16SR_F32 = 4  // the same FP16 code written with stochastic rounding (D2Q9 only)
};
constexpr bool is_f16_mode(int mode) { return mode == MODE_F16S_F32 || mode == MODE_F16SR_F32; }

struct Layout {
    int32_t nx, ny;
    int64_t pitch;  // elements per row segment (multiple of 64)
    int32_t nz;     // 1 for D2Q9
    int32_t q;      // velocities: 9 (D2Q9), 19 (D3Q19) or 27 (D3Q27)
};

__host__ __device__ __forceinline__ int64_t rows_of(const Layout &L) { return (int64_t)L.ny * L.nz; }
__host__ __device__ __forceinline__ int dim_of(const Layout &L) { return L.q == 9 ? 2 : 3; }
__host__ __device__ __forceinline__ int64_t pop_elems(const Layout &L) { return rows_of(L) * L.q * L.pitch; }
__host__ __device__ __forceinline__ int64_t vel_elems(const Layout &L) { return rows_of(L) * dim_of(L) * L.pitch; }
__host__ __device__ __forceinline__ int64_t fld_elems(const Layout &L) { return rows_of(L) * L.pitch; }

// Launch shape of the step kernel: a block is 4 waves of 64 lanes; lane = column, each wave walks
// `rows` consecutive rows.  Narrow tiles stack the waves along the rows (64 columns x 4*rows rows);
// wide tiles put them side by side (256 columns x rows rows).
struct Launch {
    int32_t rows;         // 1..64
    int32_t xcd_remap;    // tile order over the XCDs: 0 hardware, 1 row bands, 2 column bands, 3 row blocks
    int32_t wide;         // 1: 256-column tiles; 0: 64-column tiles
    int32_t max_waves;    // cap on resident waves per SIMD (0: none)
    int32_t lds_reserve;  // dynamic LDS bytes reserved per block to enforce max_waves (0: none)
    int32_t xcd_rows;     // tile rows per block of order 3
    int32_t stores;       // 0: non-temporal stores of the new state; 1: cached; 2: one buffer in place, cached
    int32_t fuse;         // time steps per launch: 1 (0 reads as 1), or 2 (step2_kernel, lbm_fused.hip)
    int32_t fuse_width;   // fused launches: output columns per tile (128, 256 or 512); rows = tile height
    int32_t pad_;
};

// Everything a step kernel needs about one instance.  Single-instance launches pass it by value;
// the batched kernel reads an array of them from device memory (wave-uniform, scalar loads).
struct InstDesc {
    void *buf[2];       // population buffers; a step reads buf[parity] and writes buf[parity ^ 1]
    const void *u;      // velocity, math type, lattice units (u dt / dx)
    const void *k;      // math type, tau1 - 1/2 per node (used when has_k)
    const void *s;      // math type, dt S + dt^2/2 dS/dt per node (used when has_s)
    Layout L;
    Launch lc;          // one step per launch (every one-step kernel, single or batched)
    Launch lcf;         // two steps per launch (lcf.fuse == 2): fuse_width x rows tiles, tile order
    int32_t has_k, has_s;
    const void *bc;     // Dirichlet values (math type, [ny][pitch]): phi_b of the edge nodes (NEE), or
                        // the wall values of the walls below row 0 / above row ny - 1 (walls)
    int32_t bckind;     // 0 periodic, 1 NEE edges, 2 walls (lbm_boundary)
    double w1, w2, beta;  // relaxation when !has_k: 1 - 1/tau1, 1 - 1/tau2, 1 - 1/(2 tau1)
    double w3;          // 1 - 1/tau3 (MRT-R); 0 for TRT-R
    double lambda;
    F16Params f16;
    int64_t *clock;     // F16SR: time level of the state in buf[0] and buf[1] (a launch reads
                        // clock[parity] and its first thread writes clock[parity ^ 1]); else unused
};

struct StepArgs {
    InstDesc d;
    int32_t parity;
};

// Work item of the batched step: tile `tile` of instance `inst`.
struct WorkItem {
    int32_t inst, tile;
};

struct BatchArgs {
    const InstDesc *inst;     // [n_inst]
    const WorkItem *items;    // grouped by block when block_start is given
    const int32_t *block_start;  // [nblocks + 1], or nullptr: block b runs item b (XCD-contiguous order)
    int32_t parity;
    int32_t one_row;             // every instance walks one row per wave (the loop-free instantiation)
};

// Number of tiles of one instance: 64 columns x (4 * rows) rows, or (wide) 256 columns x rows rows.
__host__ __device__ __forceinline__ int tiles_of(const Layout &L, int rows, int wide)
{
    const int waves_y = (int)((rows_of(L) + rows - 1) / rows);
    return wide ? ((L.nx + 255) / 256) * waves_y : ((L.nx + 63) / 64) * ((waves_y + 3) / 4);
}

// Tiles per lattice row.
__host__ __device__ __forceinline__ int tiles_per_row(const Layout &L, const Launch &lc)
{
    return lc.wide ? (L.nx + 255) >> 8 : (L.nx + 63) >> 6;
}

// First column and first row of the strip that wave `wave` (0..3) of tile t walks.  The wave has
// nothing to do when x0 >= nx or r0 >= rows_of(L).
__host__ __device__ __forceinline__ void tile_origin(const Layout &L, const Launch &lc, int t, int wave, int &x0,
                                                     int &r0)
{
    const int ntx = tiles_per_row(L, lc);
    if (lc.wide) {
        x0 = (t % ntx) * 256 + wave * 64;
        r0 = (t / ntx) * lc.rows;
    } else {
        x0 = (t % ntx) * 64;
        r0 = ((t / ntx) * 4 + wave) * lc.rows;
    }
}

struct InitArgs {
    const double *phi0;  // dense FP64 [ny][nx]
    const void *u;       // velocity, math type
    void *dst;           // populations
    Layout L;
    F16Params f16;
    int *range_flag;     // set to 1 if an F16S value does not fit
    int32_t walls;       // 1: no node lies across y = -1/2 or y = ny - 1/2 (walls)
};

struct PrepArgs {
    const double *a;   // dense FP64 [ny][nx]
    const double *b;   // second input (nullable)
    void *out;         // math type
    Layout L;
    int32_t stride;    // row stride of out in units of pitch (1 for scalar fields, 2 for velocity)
    int32_t comp;      // component offset in units of pitch (velocity: 0 or 1)
    double ca, cb;     // out = ca * a + cb * b
    int *flag;         // set to 1 if check_positive and a value is not finite and > 0
    int check_positive;
};

// Boundary data the diagnostics need to report the extrapolated Dirichlet nodes.
struct EdgeArgs {
    const void *u;     // velocity (math type)
    const void *bc;    // Dirichlet values (math type), or nullptr for a periodic instance
    int32_t kind;      // lbm_boundary: 1 NEE edges, 2 walls; 3: a one-buffer state after its streaming step
};

struct MacroArgs {
    const void *src;   // populations holding the current state
    const double *ref; // nullable
    double *phi_out;   // nullable
    Layout L;
    F16Params f16;
    EdgeArgs edge;
    double *partials;  // per block: kMacroPartialDoubles
};

constexpr int kMacroPartialDoubles = 10;  // mass(s,c) err2(s,c) ref2(s,c) maxerr maxphi nonfinite pad
constexpr int kMacroBlocks = 1024;

struct PopArgs {
    const void *src;
    double *out;  // dense FP64 [q][ny][nx] ([q][nz][ny][nx] on the 3D lattices)
    Layout L;
    F16Params f16;
    EdgeArgs edge;
};

// Adjoint of one step (lbm_adjoint.hip).
struct AdjArgs {
    const void *state;   // state image (storage type, population layout) holding g^n
    const void *lam_in;  // dL/dg^{n+1}: math type, [ny][9][pitch], lam_i(x) at (y*9 + i)*pitch + x
    void *lam_out;       // dL/dg^n, same layout
    const void *u;       // velocity (math type, lattice units)
    const void *k;       // tau1 - 1/2 per node, or nullptr: k_const
    const void *s;       // dt S + dt^2/2 dS/dt per node, or nullptr
    Layout L;
    double k_const, lambda;
    double dk_dD;        // d(tau1 - 1/2)/dD = 3 dt / dx^2
    F16Params f16;
    double *grad;        // dL/dD, FP64 [ny][nx], accumulated
};

// Launchers (lbm_kernels.hip, lbm_adjoint.hip).  All return the hipError_t of the launch.
hipError_t launch_step(int mode, int aux, const StepArgs &a, hipStream_t st);
// Two steps per launch (lbm_fused.hip): D2Q9, periodic, aux LOCAL or NONE, two buffers (reads
// buf[parity], writes buf[parity ^ 1] two steps later).  lcf.fuse_width columns x lcf.rows rows per tile.
hipError_t launch_step2(int mode, int aux, const StepArgs &a, hipStream_t st);
// The same for many instances in one launch: block b runs work items (instance, fused tile) as the
// one-step batched kernel does; every instance has tiles of `width` columns (128, 256 or 512).
hipError_t launch_batched_step2(int mode, int aux, const BatchArgs &a, int nblocks, int width, hipStream_t st);
hipError_t launch_batched_step(int mode, int aux, const BatchArgs &a, int nblocks, int lds_reserve, hipStream_t st);
hipError_t launch_init(int mode, const InitArgs &a, hipStream_t st);
// F16SR: sets *slot = level (one lane of one block; kept out of graph captures by the callers).
hipError_t launch_set_clock(int64_t *slot, int64_t level, hipStream_t st);
hipError_t launch_prep(int mode, const PrepArgs &a, hipStream_t st);
hipError_t launch_macros(int mode, const MacroArgs &a, double *result, hipStream_t st);
hipError_t launch_macros_finalize(const double *partials, int nblocks, double *result, hipStream_t st);
hipError_t launch_populations(int mode, const PopArgs &a, hipStream_t st);
// D2Q9 state images between the standard layout and the one-buffer layout after a streaming step
// (either way: the map is its own inverse); src and dst must differ.
hipError_t launch_relayout(size_t elem_bytes, const void *src, void *dst, const Layout &L, hipStream_t st);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, bool cached, hipStream_t st);
hipError_t launch_adjoint(int mode, int aux, const AdjArgs &a, hipStream_t st);
// D3Q19 and D3Q27 (lbm_kernels3d.hip, chosen by L.q): storage modes F64_F64, F64_F32, F32_F32; aux
// LOCAL or NONE; periodic.
hipError_t launch_step3(int mode, int aux, const StepArgs &a, hipStream_t st);
hipError_t launch_init3(int mode, const InitArgs &a, hipStream_t st);
hipError_t launch_macros3(int mode, const MacroArgs &a, double *result, hipStream_t st);
hipError_t launch_populations3(int mode, const PopArgs &a, hipStream_t st);
hipError_t launch_relayout3(size_t elem_bytes, const void *src, void *dst, const Layout &L, hipStream_t st);
hipError_t launch_adjoint_seed(int mode, const double *dphi, void *lam, const Layout &L, hipStream_t st);
hipError_t launch_adjoint_init(int mode, const void *lam, const void *u, double *dphi0, const Layout &L, hipStream_t st);

}  // namespace lbm
