// lbm_internal.h -- argument blocks and launchers shared by the C-ABI layer and the kernels.
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
    MODE_F16S_F32 = 3  // shifted/scaled FP16 storage, FP32 math
};

// Layout of one instance in the workspace.  Population planes and fields share the row pitch
// (in elements, a multiple of 64 so every row starts 128-byte aligned for every element size).
struct Layout {
    int32_t nx, ny;
    int64_t pitch;  // elements per row
    int64_t plane;  // elements per population plane (>= ny * pitch)
};

struct StepArgs {
    const void *src;  // 9 planes, storage type
    void *dst;        // 9 planes, storage type
    const void *ux;   // math type, lattice units (u dt / dx), pitched
    const void *uy;
    const void *k;    // math type, tau1 - 1/2 per node (nullptr: k_const)
    const void *s;    // math type, dt S + dt^2/2 dS/dt per node (nullptr: no source)
    Layout L;
    int32_t rows;     // rows walked by one thread
    double k_const;
    double lambda;
    F16Params f16;
};

struct InitArgs {
    const double *phi0;  // dense FP64 [ny][nx]
    const void *ux, *uy; // math type, pitched, lattice units
    void *dst;           // population buffer (storage type)
    Layout L;
    F16Params f16;
    int *range_flag;     // set to 1 if an F16S value does not fit
};

struct PrepArgs {
    const double *a;   // dense FP64 [ny][nx]
    const double *b;   // second input (nullable)
    void *out;         // math type, pitched
    Layout L;
    double ca, cb;     // out = ca * a + cb * b
    int *flag;         // set to 1 if check_positive and a value is not finite and > 0
    int check_positive;
};

struct MacroArgs {
    const void *src;   // population buffer holding the current state
    const double *ref; // nullable
    double *phi_out;   // nullable
    Layout L;
    F16Params f16;
    double *partials;  // per block: see kMacroPartialDoubles
};

constexpr int kMacroPartialDoubles = 10;  // mass(s,c) err2(s,c) ref2(s,c) maxerr maxphi nonfinite pad
constexpr int kMacroBlocks = 1024;

struct PopArgs {
    const void *src;
    double *out;  // dense FP64 [9][ny][nx]
    Layout L;
    F16Params f16;
};

// Launchers (lbm_kernels.hip).  All return the hipError_t of the launch.
hipError_t launch_step(int mode, int aux, const StepArgs &a, hipStream_t st);
hipError_t launch_init(int mode, const InitArgs &a, hipStream_t st);
hipError_t launch_prep(int mode, const PrepArgs &a, hipStream_t st);
hipError_t launch_macros(int mode, const MacroArgs &a, double *result, hipStream_t st);
hipError_t launch_populations(int mode, const PopArgs &a, hipStream_t st);

}  // namespace lbm
