/*
 * lbm.h -- C ABI of the MI355X (gfx950) TRT-R lattice Boltzmann library (D2Q9; D3Q19 and D3Q27).
 *
 * The library advances the two-relaxation-time regularized (TRT-R) lattice Boltzmann model for the
 * convection-diffusion equation with variable coefficients (Y. Yu, Z. Qin, H. Yuan, S. Shu,
 * arXiv:2312.10316):
 *
 *     d_t phi + d_a(phi u_a) = d_a(kappa d_a phi) + S                     (Sec. 2.1, Eq. (1))
 *
 * on D2Q9 lattices, periodic or with Dirichlet edges or walls, and on periodic D3Q19 / D3Q27 lattices
 * (enum lbm_lattice).  One step is the evolution equation of Sec. 2.2, Eq. (14): the TRT-R
 * collision of Eq. (12) (third-order Hermite equilibrium, Eq. (6); Hermite-regularized first- and
 * second-order non-equilibrium moments, Eqs. (8) and (13), relaxed with tau1 and tau2), the
 * first-order discrete-velocity source of Eq. (3) with its time derivative, and the space-derivative
 * auxiliary term of Sec. 2.3, Eq. (16), followed by streaming.  tau1 follows from kappa by
 * kappa = (tau1 - 1/2) c_s^2 dt and tau2 from the magic parameter Lambda = (tau1 - 1/2)(tau2 - 1/2)
 * (Sec. 2.4).  D2Q9: e_i in {(0,0), (+-c,0), (0,+-c), (+-c,+-c)}, c = dx/dt, c_s^2 = c^2/3 (Sec. 2.2).
 *
 * Conventions shared by every entry point:
 *   - Memory: every pointer marked "device" is HIP device memory of the current device; pointers
 *     marked "host" are host memory.  The caller owns every buffer it passes.  Fields are FP64,
 *     row-major [ny][nx] (node (j, k) at index k*nx + j), with no padding; on the 3D lattices
 *     [nz][ny][nx].
 *   - Streams: all work is enqueued on the stream given to lbm_init (a hipStream_t; NULL is the
 *     default stream).  Calls are asynchronous unless stated otherwise.  Input fields must stay
 *     valid until the stream has passed the call that reads them.
 *   - Errors: every function returns an int status (LBM_OK = 0, or a negative LBM_E_* code);
 *     nothing throws across the ABI.  Arguments are validated before anything is launched;
 *     lbm_last_error() returns a message for the calling thread's most recent failure.
 *   - Threads: a context is used by one host thread at a time.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 9

enum lbm_status {
    LBM_OK = 0,
    LBM_E_ARG = -1,        /* invalid argument; nothing was launched */
    LBM_E_HIP = -2,        /* a HIP runtime call or kernel launch failed */
    LBM_E_STATE = -3,      /* NULL or unusable context, instance index out of range */
    LBM_E_NONFINITE = -4,  /* lbm_macros found a non-finite phi: the run blew up (the stability
                              criterion of Sec. 3); the statistics are still written */
    LBM_E_UNSUPPORTED = -5 /* valid request that this build does not implement */
};

/* Population storage.  F16S stores h = f16_rne((g_i - w_i phi_ref) * 2^scale_log2) and decodes
 * g_i = h * 2^-scale_log2 + w_i phi_ref; collision arithmetic is then FP32.
 * F16SR (D2Q9 only) stores the same code, rounded stochastically instead of to nearest (an addition
 * to the paper, after Croci & Giles 2020, who showed that round-to-nearest stagnates in low-precision
 * time stepping of diffusion and stochastic rounding does not): with v the FP32 value
 * (g_i - w_i phi_ref) * 2^scale_log2, lo <= |v| < lo + ulp its FP16 neighbours and r a 13-bit integer,
 * |v| rounds up to lo + ulp iff r < floor(2^13 (|v| - lo) / ulp) (probability (|v| - lo) / ulp exactly
 * for FP16 normal values; bits below 2^-13 ulp, which exist only in the FP16 subnormal range, are
 * dropped); rounding up from 65504, or |v| >= 65536, gives infinity.  The r of population i of node
 * j = y nx + x written at time level t (the step count of the new state; 0 at init) is bits
 * 13 i .. 13 i + 12 of the 128-bit value hi:lo, where lo and hi are outputs 2(t nx ny + j) and
 * 2(t nx ny + j) + 1 (counted from 0) of SplitMix64 (Steele, Lea & Flood 2014: output k is
 * mix(seed + (k + 1) * 0x9e3779b97f4a7c15)) started at seed = (uint32_t)round_seed.  The codes are
 * therefore a pure function of the state, the step count and the seed: bitwise independent of the
 * launch shape, and a state saved at step n resumes bitwise when loaded with step n. */
enum lbm_store { LBM_STORE_F64 = 0, LBM_STORE_F32 = 1, LBM_STORE_F16S = 2, LBM_STORE_F16SR = 3 };
/* Collision arithmetic.  LBM_MATH_F64 requires LBM_STORE_F64. */
enum lbm_math { LBM_MATH_F64 = 0, LBM_MATH_F32 = 1 };
/* Auxiliary term G_i (Sec. 2.3):
 *   LOCAL: Eq. (16), phi u_b d_b u_a with phi at the node and d_b the central difference of u;
 *   FLUX:  d_b(phi u_a u_b) - u_a d_b(phi u_b) with phi at the four axis neighbours (same time
 *          level), central differences -- equal to Eq. (16) by the product rule;
 *   NONE:  G_i = 0 (ablation). */
enum lbm_aux { LBM_AUX_LOCAL = 0, LBM_AUX_FLUX = 1, LBM_AUX_NONE = 2 };

/* Boundary treatment.  PERIODIC: both axes wrap.  NEE: the first and last rows and columns are
 * Dirichlet nodes handled by non-equilibrium extrapolation (the boundary scheme of the benchmark of
 * Sec. 3; Guo, Zheng & Shi 2002): before each collision, every boundary node x_b takes
 * g_i(x_b) = g_eq_i(phi_b(x_b), u(x_b)) + [g_i(x_f) - g_eq_i(phi(x_f), u(x_f))], x_f its interior
 * neighbour along the inward normal (diagonal at corners), phi_b set by lbm_set_dirichlet.  The
 * differences of u in the LOCAL auxiliary term are one-sided across an edge.  NEE is available with
 * aux LOCAL or NONE, runs one launch per instance, and has no adjoint.
 * WALLS: x wraps; Dirichlet walls lie halfway below row 0 and above row ny - 1 (at y = -dx/2 and
 * y = (ny - 1/2) dx), by halfway anti-bounce-back (the wall scheme of Sec. 3.3): a population that
 * would cross a wall returns to its node reversed, g_opp(i) = -P_i + 2 g_eq_i^+(phi_w, u(node)),
 * with g_eq^+ the even part of the equilibrium and phi_w from row 0 (bottom wall) or row ny - 1 (top
 * wall) of lbm_set_dirichlet's array.  The y-differences of u in the LOCAL auxiliary term are
 * one-sided on those rows.  Available with aux LOCAL or NONE; one launch per instance; no adjoint. */
enum lbm_boundary { LBM_BC_PERIODIC = 0, LBM_BC_NEE = 1, LBM_BC_WALLS = 2 };

/* Lattice.  D2Q9 (Sec. 2.2).  D3Q19 and D3Q27: the three-dimensional extension (Sec. 2.2 calls it
 * straightforward) with the same operator written over three axes: velocities 0:(0,0,0);
 * 1,2:(+-1,0,0); 3,4:(0,+-1,0); 5,6:(0,0,+-1); 7:(1,1,0) 8:(-1,-1,0) 9:(1,-1,0) 10:(-1,1,0);
 * 11:(1,0,1) 12:(-1,0,-1) 13:(1,0,-1) 14:(-1,0,1); 15:(0,1,1) 16:(0,-1,-1) 17:(0,1,-1) 18:(0,-1,1),
 * weights 1/3, 1/18, 1/36 (D3Q19); D3Q27 adds the corners 19:(1,1,1) 20:(-1,-1,-1) 21:(1,1,-1)
 * 22:(-1,-1,1) 23:(1,-1,1) 24:(-1,1,-1) 25:(-1,1,1) 26:(1,-1,-1), with weights 8/27, 2/27, 1/54,
 * 1/216; c_s^2 = c^2/3.  The third-order equilibrium keeps every Hermite component the lattice
 * supports (D3Q27 keeps H_xyz, D3Q19 does not).  3D instances are periodic, use any storage mode
 * (FP64, FP32 or shifted FP16, with the lattice's own weights in w_i phi_ref), aux LOCAL or NONE
 * and TRT-R (tau3 0 or 1), run one launch per instance and have no adjoint. */
enum lbm_lattice { LBM_LATTICE_D2Q9 = 0, LBM_LATTICE_D3Q19 = 1, LBM_LATTICE_D3Q27 = 2 };

/* One problem instance: the paper's problem statement on a lattice. */
typedef struct lbm_params {
    int32_t nx, ny;       /* lattice size, each >= 3; nx <= 2^24, nodes <= 2^31 */
    double dx, dt;        /* lattice spacing and time step, finite and > 0 */
    double lambda;        /* magic parameter Lambda > 0 */
    double D_const;       /* kappa when lbm_fields.D is NULL (> 0); ignored otherwise */
    int32_t store;        /* enum lbm_store */
    int32_t math;         /* enum lbm_math */
    int32_t aux;          /* enum lbm_aux */
    int32_t scale_log2;   /* F16S and F16SR only: 0..24 */
    double phi_ref;       /* F16S and F16SR only: background value removed before encoding */
    int32_t boundary;     /* enum lbm_boundary */
    int32_t round_seed;   /* F16SR: seed of the rounding stream (any value); must be 0 for the other stores */
    double tau3;          /* MRT-R (Sec. 2.2, Eq. (11), truncated after third order): relaxation time of
                             the third-order Hermite non-equilibrium moments, finite and > 1/2;
                             0 (or 1) selects the TRT-R operator of Eq. (12), which drops them */
    int32_t lattice;      /* enum lbm_lattice */
    int32_t nz;           /* 3D lattices: size in z, >= 3 (nx * ny * nz <= 2^31); D2Q9: 0 or 1 */
} lbm_params;

/* Fields of one instance (device, FP64, [ny][nx]; 3D lattices: [nz][ny][nx]).  u is in physical units;
 * D > 0 everywhere.  They are read during lbm_init only (copied to the library's own layout). */
typedef struct lbm_fields {
    const double *phi0;   /* initial phi, required */
    const double *ux;     /* velocity x-component, required */
    const double *uy;     /* velocity y-component, required */
    const double *D;      /* diffusion coefficient kappa(x), or NULL for D_const */
    const double *uz;     /* velocity z-component: required on 3D lattices, ignored on D2Q9 */
} lbm_fields;

/* Diagnostics of one instance (host struct filled by lbm_macros). */
typedef struct lbm_stats {
    double mass;          /* sum_x phi, FP64 compensated summation */
    double rms_err;       /* E_r = sqrt(sum (phi - ref)^2 / (nx ny)) (Sec. 3, Eq. (33)); 0 without ref */
    double l2_rel_err;    /* ||phi - ref||_2 / ||ref||_2; 0 without ref */
    double max_abs_err;   /* max |phi - ref|; 0 without ref */
    double max_abs_phi;   /* max |phi| over finite values */
    int64_t nonfinite;    /* number of nodes whose phi is NaN or infinite */
    int64_t step;         /* time steps taken since lbm_init (or set by lbm_state_load) */
} lbm_stats;

typedef struct lbm_ctx lbm_ctx;

/* Bytes of device workspace that lbm_init needs for n_inst instances (p: host array [n_inst]).
 * Returns LBM_E_ARG for invalid parameters. */
int lbm_workspace_size(int32_t n_inst, const lbm_params *p, size_t *bytes);

/* Creates a context for n_inst instances (p, f: host arrays [n_inst]; the pointers inside f are
 * device pointers) and writes the initial state g_i = g_eq_i(phi0, u) (Sec. 3 set-up).
 * workspace: device buffer of at least lbm_workspace_size() bytes, 256-byte aligned, borrowed until
 * lbm_free; or NULL, in which case the library allocates (and later frees) its own.
 * stream: hipStream_t for all later work, or NULL.  Synchronizes the stream once (to check the
 * F16S range: LBM_E_ARG if |g_eq - w_i phi_ref| * 2^scale_log2 would overflow FP16).
 * On success *ctx is set; on failure *ctx is NULL and nothing is owned. */
int lbm_init(lbm_ctx **ctx, int32_t n_inst, const lbm_params *p, const lbm_fields *f,
             void *workspace, size_t workspace_bytes, void *stream);

/* Advances every instance by nsteps >= 0 steps of Eq. (14).  Asynchronous.
 * ux, uy: host arrays [n_inst] of device FP64 [ny][nx] velocity fields that replace u from this
 *         call on, or NULL (both) to keep the current u.  Not for 3D instances (LBM_E_ARG): their
 *         velocity is replaced with lbm_set_velocity.
 * S, dSdt: host arrays [n_inst] of device FP64 [ny][nx] source S and its time derivative, held
 *         constant over this call's steps, or NULL (both) for no source.  An entry may be NULL for an
 *         instance without a source; dSdt entries may be NULL (zero derivative).
 * If a launch fails (LBM_E_HIP), the step counters include only the steps enqueued in full before
 * the failure, and the populations of an instance are unspecified from then on (reload a state with
 * lbm_state_load). */
int lbm_step(lbm_ctx *ctx, int32_t nsteps, const double *const *ux, const double *const *uy,
             const double *const *S, const double *const *dSdt);

/* Replaces the velocity of instance inst from the next step on (device FP64 fields in the layout of
 * lbm_fields; uz required on 3D lattices, ignored on D2Q9).  Asynchronous (stream order). */
int lbm_set_velocity(lbm_ctx *ctx, int32_t inst, const double *ux, const double *uy, const double *uz);

/* Replaces the diffusion field kappa(x) of instance inst from the next step on (device FP64, layout of
 * lbm_fields; tau1 = 1/2 + kappa / (c_s^2 dt) per node, Sec. 2.4).  The instance must have been created
 * with a D field (LBM_E_STATE otherwise: a constant-D instance keeps no per-node field).  Synchronizes
 * the stream to check the values: LBM_E_ARG if one is not finite and > 0, after which the instance's
 * D is unspecified until a successful call.  With lbm_state_load this lets one context run the
 * forward passes of a gradient loop over D without a new lbm_init per pass. */
int lbm_set_diffusion(lbm_ctx *ctx, int32_t inst, const double *D);

/* Dirichlet values of an LBM_BC_NEE or LBM_BC_WALLS instance: phi_b (device FP64 [ny][nx], copied;
 * only its boundary entries take effect: the edge nodes for NEE, rows 0 and ny - 1 as the bottom and
 * top wall values for WALLS).  They are the values of the current time level: the next step applies
 * them to the state it starts from, and lbm_macros / lbm_populations report that state with them
 * (NEE: phi = phi_b on the edges; WALLS: the reflected populations of rows 0 and ny - 1).  Before the
 * first call the values are phi0's, for which the initial state is g_eq(phi0, u) everywhere.
 * Asynchronous (stream order).  LBM_E_STATE for a periodic instance. */
int lbm_set_dirichlet(lbm_ctx *ctx, int32_t inst, const double *phi_b);

/* Diagnostics of instance inst: phi = sum_i g_i at the current time.  phi_out (device FP64
 * [ny][nx], 3D [nz][ny][nx], nullable) receives phi; ref (same shape, nullable) is the field the error
 * statistics are taken against; out (host) receives the statistics.  Synchronizes the stream.
 * Returns LBM_E_NONFINITE if any phi is NaN or infinite (out is still filled). */
int lbm_macros(lbm_ctx *ctx, int32_t inst, double *phi_out, const double *ref, lbm_stats *out);

/* lbm_macros for callers that cannot allocate or use a library workspace while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): the same diagnostics and
 * arguments, with the reduction's partial sums and result in a static device array of the library
 * (82,000 bytes per GPU, allocated with the code object and held until the process ends) instead of
 * the context's workspace.  Calls no hipMalloc or hipFree.  The array is shared by every context on a
 * GPU and keeps the last call's contents (each call writes every entry it reads, so nothing needs
 * clearing): calls that overlap on one GPU (from several host threads or streams) race.  The
 * reduction needs at most 1024 x 10 doubles of it for any lattice the ABI accepts; a larger need
 * would be refused with LBM_E_ARG.  LBM_E_STATE if the device's array address could not be resolved
 * (it is resolved at the first lbm_init on each device).  Synchronizes the stream. */
int lbm_macros_static(lbm_ctx *ctx, int32_t inst, double *phi_out, const double *ref, lbm_stats *out);

/* Pre-collision populations g_i(x, t) of instance inst, decoded to FP64, into g_out (device FP64
 * [9][ny][nx], velocity order 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1)
 * 8:(1,-1); D3Q19 / D3Q27: [19 / 27][nz][ny][nx] in the order of enum lbm_lattice).  Asynchronous. */
int lbm_populations(lbm_ctx *ctx, int32_t inst, double *g_out);

/* Checkpoint of instance inst: the raw population state in the library's storage format.
 * lbm_state_bytes gives its size; save copies it to dst (device), load restores it from src
 * (device) and sets the step counter.  Asynchronous.  A run resumed from a checkpoint is bitwise
 * identical to the uninterrupted run.
 * Image layout: [ny][9][pitch] elements of the storage type (FP64, FP32 or FP16 code), pitch as
 * returned by lbm_pitch, padding zero.  Element (y, i, x) holds the post-collision value
 * P_i of node (x, y) from the previous step, so that g_i(x, y) = element (y - e_iy, i, x - e_ix)
 * (periodic); after lbm_init it holds g_eq_i of node (x + e_ix, y + e_iy).  D3Q19 / D3Q27:
 * [nz][ny][19 / 27][pitch], element (z, y, i, x) likewise. */
int lbm_state_bytes(lbm_ctx *ctx, int32_t inst, size_t *bytes);
/* Row pitch (elements) of an instance's layouts (state image, adjoint arrays): nx rounded up to a
 * multiple of 64, plus 64 when that many storage elements span a multiple of 4 KiB.  Host only (no
 * device work, no context).  LBM_E_ARG for invalid parameters. */
int lbm_pitch(const lbm_params *p, int64_t *pitch);
int lbm_state_save(lbm_ctx *ctx, int32_t inst, void *dst);
int lbm_state_load(lbm_ctx *ctx, int32_t inst, const void *src, int64_t step);

/* Launch shape of the step kernel.  A tuning knob only: results are bitwise independent of it.
 * A block is 4 waves of 64 lanes (lane = column); each wave walks `rows` consecutive lattice rows.
 * tile_width 64 stacks the block's waves along y (tiles of 64 columns x 4*rows rows); 256 puts them
 * side by side along x (256 columns x rows rows), so that each population row segment a block
 * reads or writes is 1 KiB (FP32) of contiguous memory.  max_waves caps the waves resident on each
 * SIMD (3..8; 0: as many as the registers allow) by reserving unused LDS per block (no effect if
 * the device does not report its LDS size); it applies to one-instance launches (the SERIAL policy);
 * the batched launch has its own cap (lbm_batch).  Defaults depend on the lattice, storage, aux form,
 * boundary, tiles per row and on whether what the context's steps touch fits in the 256 MiB Infinity
 * Cache (lbm_get_launch reports them). */
typedef struct lbm_launch {
    int32_t rows;        /* 1..64 */
    int32_t xcd_remap;   /* tile order over the 8 XCDs (each has its own L2): 0 hardware order (tiles of a row
                            interleave over the XCDs); 1 row bands (XCD j takes one contiguous range of
                            tiles); 2 column bands (XCD j takes 1/8 of the tile columns, row by row;
                            as 0 when the tiles per row are not a multiple of 8); 3 row blocks (the tile
                            rows are cut into blocks of xcd_rows tile rows and XCD j takes blocks j,
                            j + 8, j + 16, ...; the last blocks, where fewer than 8 remain, go in
                            hardware order) */
    int32_t tile_width;  /* 64 or 256 */
    int32_t max_waves;   /* 0 or 3..8 */
    int32_t xcd_rows;    /* tile rows per block of order 3 (1..64); ignored with the other orders, where
                            lbm_get_launch reports 0 */
    int32_t stores;      /* how the new state is written: 0 non-temporal (streamed to HBM); 1 cached (left
                            in L2 and the 256 MiB Infinity Cache, where the next step reads it back);
                            2 one buffer updated in place, cached.
                            1 is honoured by launches of one instance (the SERIAL policy) except the
                            walking loop (rows > 1) of D2Q9 instances with the local or no auxiliary
                            term; those and the batched policies store non-temporally.  Default: 1
                            for honouring instances when both population buffers and the per-node
                            fields of every instance of the context fit in 256 MiB, else 0.
                            2: a context of one periodic instance (D2Q9 with the local or no aux
                            term; D3Q19 or D3Q27 without FP64 math) updates a single population buffer
                            in place: a streaming step (pull, then each P_i written back where the
                            opposite population was read) alternates with a local step (the node's
                            own slots), the AA pattern of Bailey et al. (2009).  Results are bitwise
                            those of two buffers, and so are its state images (lbm_state_save and
                            lbm_state_load convert after an odd number of steps).  lbm_init chooses 2
                            for such a context that fits in 256 MiB only with a single buffer (unless
                            it defaults to fuse = 2); lbm_set_launch may switch between one and two
                            buffers at any step (the state is carried over; the workspace always
                            holds both); with stores = 2 it takes only rows = 1 and fuse 0 or 1. */
    int32_t fuse;        /* time steps per launch: 1 (0 reads as 1), or 2: two steps of Eq. (14) fused in one
                            launch (temporal blocking), each block computing the intermediate state of its
                            tile and a one-node frame around it in LDS, so every population crosses memory
                            once per two steps; bitwise the same results.  2 needs periodic D2Q9 TRT-R
                            instances (tau3 0 or 1) and two population buffers: a context of one such
                            instance (any auxiliary term), or every instance of a uniform batch with the
                            local or no auxiliary term at once (inst = -1; one batched launch per two
                            steps, tiles of every instance in the batch schedule, non-temporal stores).
                            Tiles are then tile_width = 128, 256 or 512 columns by rows = 1..256 rows,
                            in the tile order xcd_remap (xcd_rows), with stores 0 or 1 and max_waves 0.
                            An odd step count
                            ends with one single step in the context's one-step shape.  Default: 2 for
                            such a single instance of at least 2^18 nodes (2^21 with FP16 storage) and
                            for such a uniform batch (128 x 16 tiles). */
} lbm_launch;

/* Sets (inst = -1: every instance) or reads the launch shape; captured step graphs are dropped.
 * lbm_set_launch synchronizes the stream.  LBM_E_ARG for a field outside its range (xcd_rows only
 * with xcd_remap 3), LBM_E_STATE for a bad context or instance. */
int lbm_set_launch(lbm_ctx *ctx, int32_t inst, const lbm_launch *cfg);
int lbm_get_launch(lbm_ctx *ctx, int32_t inst, lbm_launch *cfg);

/* How a multi-instance context advances its instances each step.
 *   SERIAL:  one kernel launch per instance.
 *   FLAT:    one launch for all instances, one 256-thread block per tile (tiles of all instances in
 *            one XCD-contiguous list).
 *   STRIDED: one launch, `blocks` persistent blocks taking the tiles round-robin.
 *   LPT:     one launch, `blocks` persistent blocks; tiles go longest-first to the least-loaded block.
 * Batched policies need every instance to share store, math and aux (else LBM_E_UNSUPPORTED).
 * Default: FLAT when possible with more than one instance, else SERIAL.  Results are bitwise
 * independent of the policy. */
enum lbm_batch_policy { LBM_BATCH_SERIAL = 0, LBM_BATCH_FLAT = 1, LBM_BATCH_STRIDED = 2, LBM_BATCH_LPT = 3 };
typedef struct lbm_batch {
    int32_t policy;     /* enum lbm_batch_policy */
    int32_t blocks;     /* persistent blocks for STRIDED / LPT (>= 1; capped at the number of tiles) */
    int32_t max_waves;  /* cap on the batched launch's resident waves per SIMD, as lbm_launch.max_waves
                           (0 or 3..8); the default batch of FP32 instances uses 6 */
} lbm_batch;

/* Sets or reads the batch policy; captured step graphs are dropped.  Synchronizes the stream. */
int lbm_set_batch(lbm_ctx *ctx, const lbm_batch *cfg);
int lbm_get_batch(lbm_ctx *ctx, lbm_batch *cfg);

/* ---- Adjoint (reverse mode) of the step, for gradients with respect to D(x) ------------------
 * With u, D and S fixed, one step is affine in the populations: g^{n+1}_i(x + e_i) = sum_j M_ij(x)
 * g^n_j(x) + c_i(x) (Eq. (14); the equilibrium, Eq. (6), and the auxiliary term, Eq. (16), are linear in
 * phi).  Adjoint arrays ("lam") hold dL/dg in the arithmetic type (FP64 for LBM_MATH_F64, else FP32),
 * layout [ny][9][pitch] (pitch as in the state image), element (y, i, x) = dL/dg_i(x, y).
 * Supported for FP64 and FP32 storage with aux LOCAL or NONE (else LBM_E_UNSUPPORTED).  All
 * asynchronous on the context's stream; the caller owns every buffer. */

/* Bytes of one adjoint array of instance inst. */
int lbm_adjoint_bytes(lbm_ctx *ctx, int32_t inst, size_t *bytes);

/* lam_i(x) = dLdphi(x) for every i: the adjoint of phi = sum_i g_i.  dLdphi: device FP64 [ny][nx]. */
int lbm_adjoint_seed(lbm_ctx *ctx, int32_t inst, const double *dLdphi, void *lam);

/* One step backwards: lam_out_j(x) = sum_i M_ij(x) lam_in_i(x + e_i) (lam_in = dL/dg^{n+1},
 * lam_out = dL/dg^n; they must not alias), and dLdD(x) += sum_i lam_in_i(x + e_i) dP_i(x)/dD(x)
 * evaluated at g^n, which `state` holds as a state image (lbm_state_save format).  dLdD: device FP64
 * [ny][nx], accumulated.  u, D and the source are the instance's current ones. */
int lbm_adjoint_step(lbm_ctx *ctx, int32_t inst, const void *state, const void *lam_in, void *lam_out,
                     double *dLdD);

/* The backward pass over one checkpoint segment of nsteps >= 1 steps, enqueued by the library in one
 * call.  states: device buffer of nsteps state images (lbm_state_bytes each, consecutive); image 0
 * must hold g^{t0} (a checkpoint copied there by the caller).  The call first recomputes images
 * 1 .. nsteps - 1 (image j + 1 = one step of image j, with the instance's current u, D and source;
 * the context's own state is not touched; padding columns of those images are left as they were),
 * then applies nsteps adjoint steps (lbm_adjoint_step) from
 * lam = dL/dg^{t0 + nsteps} down to dL/dg^{t0}, which it writes back into lam; lam_tmp (same size,
 * must not alias lam) is scratch.  dLdD accumulates as in lbm_adjoint_step.  Asynchronous. */
int lbm_adjoint_segment(lbm_ctx *ctx, int32_t inst, void *states, int32_t nsteps, void *lam, void *lam_tmp,
                        double *dLdD);

/* dLdphi0(x) = sum_i lam0_i(x) dg_eq_i/dphi0(x): the adjoint of the initial condition
 * g = g_eq(phi0, u).  dLdphi0: device FP64 [ny][nx] (overwritten). */
int lbm_adjoint_init(lbm_ctx *ctx, int32_t inst, const void *lam0, double *dLdphi0);

/* Plain streaming copy of `bytes` bytes (multiple of 16; both pointers device, 16-byte aligned) on
 * `stream`: 16-byte non-temporal vector loads and stores, one pass.  Not part of the method: it is
 * the reference kernel against which achievable HBM bandwidth and traffic counters are calibrated. */
int lbm_bench_copy(void *dst, const void *src, size_t bytes, void *stream);
/* The same copy with the default cache policy for loads and stores: buffers that together fit in
 * the 256 MiB Infinity Cache stay resident across repeated calls, so it calibrates the rate that a
 * step whose state is held in that cache can reach.  Same arguments and errors. */
int lbm_bench_copy_cached(void *dst, const void *src, size_t bytes, void *stream);

/* Synchronizes the context's stream and releases everything the library allocated (never caller
 * memory).  NULL is accepted. */
int lbm_free(lbm_ctx *ctx);

/* Message for the calling thread's most recent failed call ("" if none).  Never NULL. */
const char *lbm_last_error(void);

/* LBM_ABI_VERSION of the loaded library. */
int lbm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
