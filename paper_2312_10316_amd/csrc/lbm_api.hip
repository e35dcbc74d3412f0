// lbm_api.hip -- C ABI of the TRT-R D2Q9 library (declared in include/lbm.h).
//
// Host side only: argument validation, the workspace layout, the batch schedule, graph capture and
// the order of kernel launches on the caller's stream.  Every arithmetic step of the method runs in
// the kernels of lbm_kernels.hip.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <queue>
#include <utility>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what) { return fail(LBM_E_HIP, "%s: %s", what, hipGetErrorString(e)); }

constexpr size_t kAlign = 256;
constexpr size_t kInfinityCacheBytes = (size_t)256 << 20;  // MI355X's memory-side cache in front of HBM
constexpr size_t kL2Bytes = (size_t)32 << 20;               // the eight XCDs' L2 caches together
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int mode_of(const lbm_params &p)
{
    if (p.store == LBM_STORE_F64) return p.math == LBM_MATH_F64 ? MODE_F64_F64 : MODE_F64_F32;
    if (p.store == LBM_STORE_F32) return MODE_F32_F32;
    return p.store == LBM_STORE_F16SR ? MODE_F16SR_F32 : MODE_F16S_F32;
}
size_t store_bytes(int mode) { return mode == MODE_F32_F32 ? 4 : (is_f16_mode(mode) ? 2 : 8); }
size_t math_bytes(int mode) { return mode == MODE_F64_F64 ? 8 : 4; }

// Row pitch: nx rounded up to 64 elements, plus 64 more when the population row segment would be a
// multiple of 4 KiB long.  The nine segments of a row (and the rows above and below) are read at
// once; at 4 KiB multiples they fall on the same HBM channels, which costs 4-10 % of FP32 throughput
// on MI355X (measured at 1024^2 ... 8192^2).
int64_t pitch_of(const lbm_params &p)
{
    size_t pitch = align_up((size_t)p.nx, 64);
    if (pitch * store_bytes(mode_of(p)) % 4096 == 0) pitch += 64;
    return (int64_t)pitch;
}

Layout layout_of(const lbm_params &p)
{
    Layout L;
    L.nx = p.nx;
    L.ny = p.ny;
    L.pitch = pitch_of(p);
    L.nz = p.lattice == LBM_LATTICE_D2Q9 ? 1 : p.nz;
    L.q = p.lattice == LBM_LATTICE_D3Q27 ? 27 : (p.lattice == LBM_LATTICE_D3Q19 ? 19 : 9);
    return L;
}

// Dynamic LDS that a 256-thread block must reserve so that at most max_waves of its waves are
// resident per SIMD (4 waves per block, 4 SIMDs per CU: max_waves blocks per CU): half-way between
// the per-block sizes that fit max_waves + 1 and max_waves blocks in the CU's LDS, so allocation
// granularity cannot tip the count.  0 (no cap) when the LDS size is unknown.
int lds_reserve_for(int max_waves, int lds_per_cu)
{
    if (max_waves <= 0 || lds_per_cu <= 0) return 0;
    const int lo = lds_per_cu / (max_waves + 1), hi = lds_per_cu / max_waves;
    return ((lo + hi) / 2) & ~511;
}

// Default launch shape, from sweeps on MI355X over 1024^2..8192^2 (2049^2, 3000^2 and 6000^2 among
// them) and 256^3 (the autotuner in the Python package can override it per instance).
// ntx = 256-column tiles per row.
// D2Q9, periodic, local or no aux: one row per wave (the one-row kernels have no walking loop) on
// 256-column tiles, at most 5 waves per SIMD for FP32 storage (6 with a D(x) field) and 4 for FP64
// storage (+1-5 %), FP16 uncapped (a cap costs it 4-20 %).  With ntx >= 4 the XCDs take row blocks
// (order 3): FP32 h = 64 / ntx tile rows, FP64 storage h = 32 / ntx (both clamped to 2..8), FP16
// h = 32 / ntx clamped to 2..4, except at ntx = 8 and 16, where column bands are as fast for FP16.
// Against column bands (ntx a multiple of 8) or row bands: FP32 +2-9 %, FP64 +1-5 %, FP16 +2-6 %
// (2048^2 FP32: 82k MLUPS).  Narrower lattices: row bands, FP64 storage on 64-column tiles in
// hardware order.
// Flux form: two rows per wave on 256-column tiles, FP32 in row bands with 4 waves (+16 % over 8 rows
// of 64-column tiles), FP64 in column bands (ntx a multiple of 8) or row bands, uncapped (row blocks
// measured slower).
// Dirichlet edges and walls with ntx >= 8: FP32 on 256-column tiles in row blocks of 4 tile rows capped
// at 5 waves (2049^2 NEE: 76k against 72k MLUPS in row bands), FP64 the same with h = 2, uncapped;
// FP16 in row bands, uncapped.  Narrower lattices: FP32 and FP16 in row bands, FP64 on 64-column tiles
// in hardware order.
// D3Q19 and D3Q27: 256-column tiles in hardware order; one row per wave, FP32 capped at 4 waves (+17 %
// on D3Q19 and +14 % on D3Q27 over 64-column tiles at full occupancy); FP16 storage in its one-row
// instantiation capped at 5 waves (+3 %).  (256^3; row blocks measured level or slower.)
// A context of several instances keeps 64-column tiles in row bands, which the batched kernel prefers
// (a 256-column tile of a small lattice leaves waves idle).
Launch default_launch(const lbm_params &p, int mode, bool has_D, int n_inst, int lds_per_cu)
{
    Launch lc{1, 0, 1, 0, 0, 0};
    const bool f32 = mode == MODE_F32_F32, f16 = is_f16_mode(mode);
    const int ntx = (p.nx + 255) / 256;
    const int bands = ntx % 8 == 0 ? 2 : 1;
    const auto row_blocks = [&lc](int h) {
        lc.xcd_remap = 3;
        lc.xcd_rows = h;
    };
    if (p.lattice != LBM_LATTICE_D2Q9) {
        lc.max_waves = f32 ? 4 : (f16 ? 5 : 0);
    } else if (p.boundary != LBM_BC_PERIODIC) {
        if (f32 || f16) {
            lc.xcd_remap = 1;
            lc.max_waves = f32 ? 5 : 0;
            if (f32 && ntx >= 8) row_blocks(4);
        } else if (ntx >= 8) {
            row_blocks(2);
        } else {
            lc.wide = 0;
        }
    } else if (p.aux == LBM_AUX_FLUX) {
        lc.rows = 2;
        lc.xcd_remap = f32 ? 1 : bands;
        lc.max_waves = f32 ? 4 : 0;
    } else {
        lc.xcd_remap = 1;
        lc.max_waves = f16 ? 0 : (f32 ? (has_D ? 6 : 5) : 4);
        if (ntx >= 4) {
            if (f32) row_blocks(std::clamp(64 / ntx, 2, 8));
            else if (!f16) row_blocks(std::clamp(32 / ntx, 2, 8));
            else if (ntx == 8 || ntx == 16) lc.xcd_remap = 2;
            else row_blocks(std::clamp(32 / ntx, 2, 4));
        } else if (!f16 && !f32) {  // FP64 storage on narrow lattices
            lc.wide = 0;
            lc.xcd_remap = 0;
        }
    }
    if (n_inst > 1 && p.lattice == LBM_LATTICE_D2Q9) {
        lc.rows = 1;
        lc.wide = 0;
        lc.xcd_remap = 1;
        lc.xcd_rows = 0;
    }
    lc.lds_reserve = lds_reserve_for(lc.max_waves, lds_per_cu);
    return lc;
}

// An instance whose steps can be fused (a periodic D2Q9 TRT-R instance, any aux form).  A context fuses
// its one instance, or every instance of a uniform batch at once (local or no aux term).
bool fusable(const lbm_params &p)
{
    return p.lattice == LBM_LATTICE_D2Q9 && p.boundary == LBM_BC_PERIODIC && (p.tau3 == 0.0 || p.tau3 == 1.0);
}

// Nodes from which one periodic instance takes two steps per launch.  A fused launch walks each tile's
// rows one after the other, which small lattices do not hide; measured (MLUPS, one step / two steps per
// launch): FP64 384^2 26.5k / 26.4k, 512^2 34.4k / 44.8k; FP32 384^2 40.3k / 37.7k, 512^2 59.3k /
// 63.0k; FP16 1024^2 117.2k / 107.4k, 2048^2 about 163k / 203k (its one-step state stays in the
// Infinity Cache longer).
int64_t fuse_min_nodes(int mode)
{
    return is_f16_mode(mode) ? ((int64_t)1 << 21) : ((int64_t)1 << 18);
}

// Two steps per launch (temporal blocking, lbm_fused.hip) for a single periodic D2Q9 TRT-R instance.
// Tile shapes from sweeps at 2048^2, 4096^2 and 8192^2 (widths 128/256/512 x 8..64 rows x stores):
// FP32 storage 512 x 16 (2048^2 131k, 4096^2 131k, 8192^2 140k MLUPS); FP16 storage with at most 8
// tiles of 256 columns per row 512 x 16 (203k), wider 256 x 24 (3072^2 177k, 8192^2 206k, 2 % above
// 256 x 16; stochastic rounding 167k); FP64 storage 512 x 16 (8192^2 69k; FP32 math 76k), on narrow
// lattices 256 x 32 (FP32 math 512 x 32).  Tiles never wider than the lattice needs (at least 128
// columns); rows halved (down to 4) until there are 512 tiles, 256 where a CU holds one block, then
// the width halved (down to 128) until there are 256 (a 512^2 lattice in 512 x 4 tiles kept half the
// CUs idle).  The flux form (128/256 columns x 8..64 rows x stores):
// 128-column tiles, 16 rows for FP32 up to 2048 columns (2048^2: 99k MLUPS), FP16 there 256 x 24 (133k),
// else 32 rows (8192^2 FP32 113k, FP16 136k, FP64 57k).  Row bands over the XCDs, so that the frame
// rows a tile shares with the next tile down sit in the same L2.  (MRT-R stays on single steps: with
// FP64 math the compiler had fused its third-order multiply-adds otherwise in the fused kernel.)
Launch fused_default(const lbm_params &p, int mode)
{
    Launch lc{};
    lc.fuse = 2;
    const bool narrow = (p.nx + 255) / 256 <= 8;
    int width, rows;
    if (mode == MODE_F32_F32) {
        width = 512;
        rows = 16;
    } else if (is_f16_mode(mode)) {
        width = narrow ? 512 : 256;
        rows = narrow ? 16 : 24;
    } else {  // FP64 storage: one 512-column block per CU (98.7 KB of ring) beats narrower tiles
        width = narrow && mode == MODE_F64_F64 ? 256 : 512;
        rows = narrow ? 32 : 16;
    }
    if (p.aux == LBM_AUX_FLUX) {  // 128-column tiles: FP32 16 rows up to 2048 columns, else 32 rows
        width = is_f16_mode(mode) && narrow ? 256 : 128;
        rows = narrow && mode == MODE_F32_F32 ? 16 : (narrow && is_f16_mode(mode) ? 24 : 32);
    }
    while (width > 128 && width / 2 >= p.nx) width /= 2;
    auto tiles = [&](int h) { return (int64_t)((p.nx + width - 1) / width) * ((p.ny + h - 1) / h); };
    // rows halved until every CU has two tiles (one where a CU holds a single block: FP64 storage on
    // 512-column tiles; and the flux form, not measured otherwise): 1024^2 FP32 512 x 8 -> 512 x 4
    // 122.4k -> 135.4k MLUPS, FP64 256 x 16 -> 256 x 8 71.9k -> 73.3k
    const bool one_block = (mode == MODE_F64_F64 || mode == MODE_F64_F32) && width == 512;
    const int64_t want = one_block || p.aux == LBM_AUX_FLUX ? 256 : 512;
    while (rows > 4 && tiles(rows) < want) rows /= 2;
    while (width > 128 && tiles(rows) < 256) width /= 2;  // small lattices: narrower tiles fill the CUs
    lc.fuse_width = width;
    lc.rows = rows;
    lc.xcd_remap = 1;
    return lc;
}

// One buffer updated in place (AA pattern): a context of one periodic instance, D2Q9 with the local or
// no aux term, or D3Q19/D3Q27 except FP64 math (whose one-row in-place kernels fuse the collision's
// multiply-adds otherwise than the two-buffer walking loop: equal to rounding, not bitwise).
bool in_place_ok(const lbm_params &p, int mode, int n_inst)
{
    if (n_inst != 1 || p.boundary != LBM_BC_PERIODIC) return false;
    if (p.lattice != LBM_LATTICE_D2Q9) return mode != MODE_F64_F64;
    return p.aux != LBM_AUX_FLUX;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate(const lbm_params &p, int k)
{
    if (p.nx < 3 || p.ny < 3) return fail(LBM_E_ARG, "instance %d: nx=%d, ny=%d must be >= 3", k, p.nx, p.ny);
    if (p.lattice != LBM_LATTICE_D2Q9 && p.lattice != LBM_LATTICE_D3Q19 && p.lattice != LBM_LATTICE_D3Q27)
        return fail(LBM_E_ARG, "instance %d: unknown lattice %d", k, p.lattice);
    const bool three_d = p.lattice != LBM_LATTICE_D2Q9;
    if (!three_d && p.nz != 0 && p.nz != 1)
        return fail(LBM_E_ARG, "instance %d: nz=%d on a D2Q9 lattice (0 or 1)", k, p.nz);
    if (three_d && p.nz < 3) return fail(LBM_E_ARG, "instance %d: nz=%d must be >= 3", k, p.nz);
    const int64_t nodes = (int64_t)p.nx * p.ny * (three_d ? p.nz : 1);
    if (nodes > ((int64_t)1 << 31)) return fail(LBM_E_ARG, "instance %d: more than 2^31 nodes", k);
    if ((int64_t)p.nx > ((int64_t)1 << 24))  // kernels address a lattice row's segments with 32-bit byte offsets
        return fail(LBM_E_ARG, "instance %d: nx=%d exceeds 2^24", k, p.nx);
    if (!finite_pos(p.dx) || !finite_pos(p.dt)) return fail(LBM_E_ARG, "instance %d: dx and dt must be finite and > 0", k);
    if (!finite_pos(p.lambda)) return fail(LBM_E_ARG, "instance %d: lambda must be finite and > 0", k);
    if (p.store < LBM_STORE_F64 || p.store > LBM_STORE_F16SR) return fail(LBM_E_ARG, "instance %d: unknown store %d", k, p.store);
    if (p.math != LBM_MATH_F64 && p.math != LBM_MATH_F32) return fail(LBM_E_ARG, "instance %d: unknown math %d", k, p.math);
    if (p.math == LBM_MATH_F64 && p.store != LBM_STORE_F64)
        return fail(LBM_E_ARG, "instance %d: FP64 math needs FP64 storage", k);
    if (p.aux < LBM_AUX_LOCAL || p.aux > LBM_AUX_NONE) return fail(LBM_E_ARG, "instance %d: unknown aux %d", k, p.aux);
    if (p.boundary < LBM_BC_PERIODIC || p.boundary > LBM_BC_WALLS)
        return fail(LBM_E_ARG, "instance %d: unknown boundary %d", k, p.boundary);
    if (p.round_seed != 0 && p.store != LBM_STORE_F16SR)
        return fail(LBM_E_ARG, "instance %d: round_seed is for LBM_STORE_F16SR only (0 otherwise)", k);
    if (p.boundary != LBM_BC_PERIODIC && p.aux == LBM_AUX_FLUX)
        return fail(LBM_E_UNSUPPORTED, "instance %d: the flux form of the aux term is periodic only", k);
    if (p.tau3 != 0.0 && !(std::isfinite(p.tau3) && p.tau3 > 0.5))
        return fail(LBM_E_ARG, "instance %d: tau3 must be 0 (TRT-R) or finite and > 1/2", k);
    if (three_d) {
        if (p.aux == LBM_AUX_FLUX) return fail(LBM_E_UNSUPPORTED, "instance %d: the flux form is D2Q9 only", k);
        if (p.boundary != LBM_BC_PERIODIC) return fail(LBM_E_UNSUPPORTED, "instance %d: 3D lattices are periodic only", k);
        if (p.tau3 != 0.0 && p.tau3 != 1.0) return fail(LBM_E_UNSUPPORTED, "instance %d: no MRT-R on 3D lattices", k);
        if (p.store == LBM_STORE_F16SR)
            return fail(LBM_E_UNSUPPORTED, "instance %d: stochastic rounding is D2Q9 only", k);
    }
    if (p.store == LBM_STORE_F16S || p.store == LBM_STORE_F16SR) {
        if (p.scale_log2 < 0 || p.scale_log2 > 24)
            return fail(LBM_E_ARG, "instance %d: scale_log2=%d outside 0..24", k, p.scale_log2);
        if (!std::isfinite(p.phi_ref)) return fail(LBM_E_ARG, "instance %d: phi_ref is not finite", k);
    }
    return LBM_OK;
}

// Lattice weight w_i of velocity i on the 3D lattices (rest, 6 faces, 12 edges, 8 corners).
double weight3(int q, int i)
{
    if (i == 0) return q == 27 ? 8.0 / 27.0 : 1.0 / 3.0;
    if (i <= 6) return q == 27 ? 2.0 / 27.0 : 1.0 / 18.0;
    if (i <= 18) return q == 27 ? 1.0 / 54.0 : 1.0 / 36.0;
    return 1.0 / 216.0;
}

F16Params f16_of(const lbm_params &p)
{
    F16Params f{};
    if (p.store == LBM_STORE_F16S || p.store == LBM_STORE_F16SR) {
        f.scale = std::ldexp(1.0f, p.scale_log2);
        f.inv_scale = std::ldexp(1.0f, -p.scale_log2);
        const int q = layout_of(p).q;
        for (int i = 0; i < q; ++i) f.wref[i] = (float)((q == 9 ? kW[i] : weight3(q, i)) * p.phi_ref);
        f.seed = (uint64_t)(uint32_t)p.round_seed;
        f.nodes = (int64_t)p.nx * p.ny;
    } else {
        f.scale = f.inv_scale = 1.0f;
    }
    return f;
}

struct Instance {
    lbm_params p;
    int mode;
    Layout L;
    Launch lc;   // the configured launch (lc.fuse == 2: two steps per launch)
    Launch lc1;  // the one-step launch used for single steps of a context whose lc is fused
    char *buf[2];
    char *alt;   // the workspace's second population buffer (buf[1] unless the instance runs in place)
    void *u, *k, *s, *bc;
    bool has_D;
    bool has_src;
    int64_t step;
    F16Params f16;
    int64_t *clock;  // device pair: time level of the state in each buffer slot (stochastic rounding)
};

// Per instance: 2 population buffers, the velocity pair, and the k and s fields (math type).
size_t pops_bytes(const lbm_params &p) { return align_up((size_t)pop_elems(layout_of(p)) * store_bytes(mode_of(p)), kAlign); }
size_t vel_bytes(const lbm_params &p) { return align_up((size_t)vel_elems(layout_of(p)) * math_bytes(mode_of(p)), kAlign); }
size_t field_bytes(const lbm_params &p) { return align_up((size_t)fld_elems(layout_of(p)) * math_bytes(mode_of(p)), kAlign); }
size_t instance_bytes(const lbm_params &p)
{
    return 2 * pops_bytes(p) + vel_bytes(p) + (p.boundary != LBM_BC_PERIODIC ? 3 : 2) * field_bytes(p);
}

size_t max_items_of(int32_t n_inst, const lbm_params *p)
{
    size_t items = 0;  // one row per wave gives the most tiles, of either width
    for (int k = 0; k < n_inst; ++k) {
        const Layout L = layout_of(p[k]);
        items += (size_t)std::max(tiles_of(L, 1, 0), tiles_of(L, 1, 1));
    }
    return items;
}
// Two steps per launch: tiles of at least 128 columns and one row.
size_t max_items2_of(int32_t n_inst, const lbm_params *p)
{
    size_t items = 0;
    for (int k = 0; k < n_inst; ++k) items += (size_t)((p[k].nx + 127) / 128) * (size_t)p[k].ny;
    return items;
}

// Shared scratch: macro partials, the macro result, two flag words; then the batch tables
// (instance descriptors, work items, block ranges).
constexpr size_t kPartialBytes = (size_t)kMacroBlocks * kMacroPartialDoubles * sizeof(double);
constexpr size_t kScratchBytes = kPartialBytes + 256 + 256;

size_t tables_bytes(int32_t n_inst, const lbm_params *p)
{
    size_t b = align_up((size_t)n_inst * sizeof(InstDesc), kAlign) + align_up((size_t)n_inst * 2 * sizeof(int64_t), kAlign);
    for (size_t items : {max_items_of(n_inst, p), n_inst > 1 ? max_items2_of(n_inst, p) : (size_t)0})
        b += align_up(items * sizeof(WorkItem), kAlign) + align_up((items + 1) * sizeof(int32_t), kAlign);
    return b;
}

// Constant-D relaxation: tau1 - 1/2 = kappa / (cs^2 dt) = 3 kappa dt / dx^2 (Sec. 2.4), and
// tau2 - 1/2 = Lambda / (tau1 - 1/2) (magic parameter, Sec. 2.4).
void const_relax(const lbm_params &p, double &w1, double &w2, double &beta)
{
    const double k = 3.0 * p.D_const * p.dt / (p.dx * p.dx);
    const double tau1 = 0.5 + k, tau2 = 0.5 + p.lambda / k;
    w1 = 1.0 - 1.0 / tau1;
    w2 = 1.0 - 1.0 / tau2;
    beta = 1.0 - 0.5 / tau1;
}

// The launch of a single step: the configured one, or the one kept beside a fused configuration.
const Launch &one_step(const Instance &in) { return in.lc.fuse == 2 ? in.lc1 : in.lc; }

InstDesc desc_of(const Instance &in)
{
    InstDesc d{};
    d.buf[0] = in.buf[0];
    d.buf[1] = in.buf[1];
    d.u = in.u;
    d.k = in.k;
    d.s = in.s;
    d.L = in.L;
    d.lc = one_step(in);
    if (in.lc.fuse == 2) d.lcf = in.lc;
    d.has_k = in.has_D ? 1 : 0;
    d.has_s = in.has_src ? 1 : 0;
    d.bc = in.bc;
    d.bckind = in.p.boundary;
    if (!in.has_D) const_relax(in.p, d.w1, d.w2, d.beta);
    d.w3 = in.p.tau3 == 0.0 ? 0.0 : 1.0 - 1.0 / in.p.tau3;
    d.lambda = in.p.lambda;
    d.f16 = in.f16;
    d.clock = in.clock;
    return d;
}

}  // namespace

// Long runs replay a captured graph of kGraphSteps steps (an even count, so every buffer returns
// to its role); one graph per buffer parity, dropped whenever a descriptor or the schedule changes.
constexpr int kGraphSteps = 32;
static_assert(kGraphSteps % 2 == 0, "a graph replay must keep the buffer parity");

// Device scratch of lbm_macros_static: the per-block partial sums of the diagnostics reduction
// (kMacroBlocks x kMacroPartialDoubles) and its final result (8 doubles).  One copy per GPU, held until
// the process ends; host code never passes `scratch` itself (in host code the name is a stand-in, not
// a device address) but the address hipGetSymbolAddress returns for the current device, resolved once
// per device at its first lbm_init.
constexpr size_t kStaticScratchDoubles = (size_t)kMacroBlocks * kMacroPartialDoubles + 8;  // 82,000 bytes
static __device__ __align__(256) double scratch[kStaticScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Work list of a batched launch: (instance, tile) items, either one per block (flat) or in ranges.
struct Schedule {
    WorkItem *d_items = nullptr;      // device (in the workspace)
    int32_t *d_block_start = nullptr;
    int nblocks = 0;                  // grid of the launch
    bool use_block_start = false;
    std::vector<WorkItem> h_items;    // host staging
    std::vector<int32_t> h_block_start;
};

struct lbm_ctx {
    std::vector<Instance> inst;
    int parity = 0;                   // the buffer every instance currently reads (they step together)
    bool uniform = false;             // all instances share mode and aux (a batched launch is possible)
    bool l2_streams = false;          // steps stream their stores although the state fits the caches
    lbm_batch batch = {LBM_BATCH_SERIAL, 0, 0};
    InstDesc *d_desc = nullptr;       // device tables (in the workspace)
    std::vector<InstDesc> h_desc;     // host staging of the descriptors
    Schedule sched[2];                // batched work lists: one step per launch, two steps per launch
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;    // private stream used only to record graphs
    int lds_per_cu = 0;               // LDS bytes per CU of the device (for the wave cap)
    char *ws = nullptr;
    bool owns_ws = false;
    double *partials = nullptr;
    double *result = nullptr;
    int *flag = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int device = -1;                  // the device current at lbm_init (its stream's device)
};

namespace {

bool check_inst(lbm_ctx *c, int32_t inst) { return c && inst >= 0 && inst < (int32_t)c->inst.size(); }

void drop_graphs(lbm_ctx *c)
{
    for (int k = 0; k < 2; ++k) {
        if (c->graph[k]) (void)hipGraphExecDestroy(c->graph[k]);
        c->graph[k] = nullptr;
    }
}

bool batched(const lbm_ctx *c) { return c->inst.size() > 1 && c->uniform && c->batch.policy != LBM_BATCH_SERIAL; }

// A context whose instances all run two steps per launch (one instance, or a whole uniform batch).
bool fused(const lbm_ctx *c)
{
    for (const Instance &in : c->inst)
        if (in.lc.fuse != 2) return false;
    return !c->inst.empty();
}

// Builds and uploads the work list of the batched one-step launch (two = false) or of the batched
// two-step launch (two = true): items in instance order, costed by the live nodes of their tile, then
// one per block (flat), dealt round-robin (strided) or longest first to the least-loaded block (LPT).
int build_schedule(lbm_ctx *c, bool two)
{
    Schedule &sc = c->sched[two ? 1 : 0];
    const int n = (int)c->inst.size();
    std::vector<WorkItem> items;
    std::vector<int64_t> cost;
    for (int k = 0; k < n; ++k) {
        const Layout &L = c->inst[k].L;
        const Launch &lc = two ? c->inst[k].lc : one_step(c->inst[k]);
        if (two) {
            const int W = lc.fuse_width, H = lc.rows, ntx = (L.nx + W - 1) / W, nt = ntx * ((L.ny + H - 1) / H);
            for (int t = 0; t < nt; ++t) {
                const int x0 = (t % ntx) * W, y0 = (t / ntx) * H;
                items.push_back(WorkItem{k, t});
                cost.push_back((int64_t)std::min(W, L.nx - x0) * std::min(H, L.ny - y0));
            }
        } else {
            const int nt = tiles_of(L, lc.rows, lc.wide);
            const int tw = lc.wide ? 256 : 64, th = lc.wide ? lc.rows : 4 * lc.rows;  // tile extent
            for (int t = 0; t < nt; ++t) {
                int x0, y0;
                tile_origin(L, lc, t, 0, x0, y0);
                items.push_back(WorkItem{k, t});
                cost.push_back((int64_t)std::min(tw, L.nx - x0) * std::min(th, L.ny - y0));
            }
        }
    }
    const int ni = (int)items.size();
    const lbm_batch &b = c->batch;
    if (b.policy == LBM_BATCH_FLAT) {
        sc.h_items = items;
        sc.use_block_start = false;
        sc.nblocks = ni;
    } else {
        const int P = std::min(b.blocks, ni);
        std::vector<std::vector<int>> per(P);
        if (b.policy == LBM_BATCH_STRIDED) {
            for (int i = 0; i < ni; ++i) per[i % P].push_back(i);
        } else {  // LPT: longest tile first, to the least-loaded block
            std::vector<int> order(ni);
            for (int i = 0; i < ni; ++i) order[i] = i;
            std::stable_sort(order.begin(), order.end(), [&](int a, int z) { return cost[a] > cost[z]; });
            using Load = std::pair<int64_t, int>;
            std::priority_queue<Load, std::vector<Load>, std::greater<Load>> pq;
            for (int j = 0; j < P; ++j) pq.push({0, j});
            for (int i : order) {
                Load l = pq.top();
                pq.pop();
                per[l.second].push_back(i);
                pq.push({l.first + cost[i], l.second});
            }
            for (auto &v : per) std::sort(v.begin(), v.end());  // each block walks its tiles in memory order
        }
        sc.h_items.clear();
        sc.h_block_start.assign(P + 1, 0);
        for (int j = 0; j < P; ++j) {
            sc.h_block_start[j] = (int32_t)sc.h_items.size();
            for (int i : per[j]) sc.h_items.push_back(items[i]);
        }
        sc.h_block_start[P] = (int32_t)sc.h_items.size();
        sc.use_block_start = true;
        sc.nblocks = P;
        hipError_t e = hipMemcpyAsync(sc.d_block_start, sc.h_block_start.data(), (P + 1) * sizeof(int32_t),
                                      hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(e, "uploading block ranges");
    }
    hipError_t e = hipMemcpyAsync(sc.d_items, sc.h_items.data(), sc.h_items.size() * sizeof(WorkItem),
                                  hipMemcpyHostToDevice, c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "uploading work items");
}

// Rebuilds the descriptors and (for a batched policy) the work list, and uploads them.  The host
// staging vectors are only rewritten after the stream has drained.
int refresh_tables(lbm_ctx *c)
{
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "synchronizing before a table update");
    drop_graphs(c);
    const int n = (int)c->inst.size();
    c->h_desc.resize(n);
    for (int k = 0; k < n; ++k) c->h_desc[k] = desc_of(c->inst[k]);
    e = hipMemcpyAsync(c->d_desc, c->h_desc.data(), n * sizeof(InstDesc), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "uploading instance descriptors");
    if (batched(c)) {
        int rc = build_schedule(c, false);
        if (rc == LBM_OK && fused(c)) rc = build_schedule(c, true);
        if (rc) return rc;
    }
    e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "synchronizing after a table update");
}

int prep_field(lbm_ctx *c, Instance &in, const double *a, const double *b, double ca, double cb, void *out,
               int check_positive, int stride = 1, int comp = 0)
{
    PrepArgs pa;
    pa.a = a;
    pa.b = b;
    pa.out = out;
    pa.L = in.L;
    pa.stride = stride;
    pa.comp = comp;
    pa.ca = ca;
    pa.cb = cb;
    pa.flag = c->flag + 1;
    pa.check_positive = check_positive;
    hipError_t e = launch_prep(in.mode, pa, c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "prep kernel launch");
}

int set_velocity(lbm_ctx *c, Instance &in, const double *ux, const double *uy, const double *uz = nullptr)
{
    const double s = in.p.dt / in.p.dx;  // lattice units: u dt / dx
    const int d = dim_of(in.L);
    int rc = prep_field(c, in, ux, nullptr, s, 0.0, in.u, 0, d, 0);
    if (rc == LBM_OK) rc = prep_field(c, in, uy, nullptr, s, 0.0, in.u, 0, d, 1);
    if (rc == LBM_OK && d == 3) rc = prep_field(c, in, uz, nullptr, s, 0.0, in.u, 0, d, 2);
    return rc;
}

bool is3d(const Instance &in) { return in.L.q != 9; }

// Stochastic rounding indexes its random bits by the time level, which the kernels advance in device
// memory (graph replays included).  Where the host sets a state or moves it to the other buffer slot,
// it writes the level of the slot that now holds the state.
int sync_clock(lbm_ctx *c, Instance &in)
{
    if (in.mode != MODE_F16SR_F32) return LBM_OK;
    hipError_t e = launch_set_clock(in.clock + c->parity, in.step, c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "setting the time level of a stochastically rounded state");
}

// Enqueues one step of every instance on stream st.
int enqueue_step(lbm_ctx *c, hipStream_t st)
{
    if (batched(c)) {
        const Schedule &sc = c->sched[0];
        BatchArgs a;
        a.inst = c->d_desc;
        a.items = sc.d_items;
        a.block_start = sc.use_block_start ? sc.d_block_start : nullptr;
        a.parity = c->parity;
        a.one_row = 1;
        for (const Instance &in : c->inst) a.one_row &= one_step(in).rows == 1 ? 1 : 0;
        hipError_t e = launch_batched_step(c->inst[0].mode, c->inst[0].p.aux, a, sc.nblocks,
                                           lds_reserve_for(c->batch.max_waves, c->lds_per_cu), st);
        if (e != hipSuccess) return hip_fail(e, "batched step kernel launch");
    } else {
        for (size_t k = 0; k < c->inst.size(); ++k) {
            StepArgs a;
            a.d = c->h_desc[k];  // its lc is the one-step launch, also in a fused context
            a.parity = c->parity;
            hipError_t e = is3d(c->inst[k]) ? launch_step3(c->inst[k].mode, c->inst[k].p.aux, a, st)
                                             : launch_step(c->inst[k].mode, c->inst[k].p.aux, a, st);
            if (e != hipSuccess) return hip_fail(e, "step kernel launch");
        }
    }
    c->parity ^= 1;
    return LBM_OK;
}

// Enqueues two steps of every instance (fused contexts): one launch for a batch, else one per instance.
int enqueue_fused(lbm_ctx *c, hipStream_t st)
{
    if (batched(c)) {
        const Schedule &sc = c->sched[1];
        BatchArgs a;
        a.inst = c->d_desc;
        a.items = sc.d_items;
        a.block_start = sc.use_block_start ? sc.d_block_start : nullptr;
        a.parity = c->parity;
        a.one_row = 0;
        hipError_t e = launch_batched_step2(c->inst[0].mode, c->inst[0].p.aux, a, sc.nblocks, c->inst[0].lc.fuse_width, st);
        if (e != hipSuccess) return hip_fail(e, "batched fused step kernel launch");
    } else {
        for (size_t k = 0; k < c->inst.size(); ++k) {
            StepArgs a;
            a.d = c->h_desc[k];
            a.parity = c->parity;
            hipError_t e = launch_step2(c->inst[k].mode, c->inst[k].p.aux, a, st);
            if (e != hipSuccess) return hip_fail(e, "fused step kernel launch");
        }
    }
    c->parity ^= 1;
    return LBM_OK;
}

// Returns the graph of kGraphSteps steps for the current buffer parity, capturing it if needed.
int graph_for(lbm_ctx *c, hipGraphExec_t *out)
{
    const int par = c->parity;
    if (c->graph[par]) {
        *out = c->graph[par];
        return LBM_OK;
    }
    if (!c->capture) {
        hipError_t e = hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "creating the capture stream");
    }
    hipError_t e = hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    int rc = LBM_OK;
    if (fused(c))
        for (int t = 0; t < kGraphSteps / 2 && rc == LBM_OK; ++t) rc = enqueue_fused(c, c->capture);
    else
        for (int t = 0; t < kGraphSteps && rc == LBM_OK; ++t) rc = enqueue_step(c, c->capture);
    // Capturing runs nothing: the buffer parity is the one the graph starts from, on every path out
    // (a failed capture may have flipped it an odd number of times).
    c->parity = par;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->capture, &g);
    if (rc != LBM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    c->graph[par] = x;
    *out = x;
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_abi_version(void) { return LBM_ABI_VERSION; }

int lbm_pitch(const lbm_params *p, int64_t *pitch)
{
    g_err[0] = 0;
    if (!p || !pitch) return fail(LBM_E_ARG, "lbm_pitch: p and pitch are required");
    int rc = validate(*p, 0);
    if (rc) return rc;
    *pitch = pitch_of(*p);
    return LBM_OK;
}

const char *lbm_last_error(void) { return g_err; }

int lbm_workspace_size(int32_t n_inst, const lbm_params *p, size_t *bytes)
{
    g_err[0] = 0;
    if (n_inst < 1 || !p || !bytes) return fail(LBM_E_ARG, "lbm_workspace_size: n_inst >= 1, p and bytes required");
    size_t total = align_up(kScratchBytes, kAlign);
    for (int k = 0; k < n_inst; ++k) {
        int rc = validate(p[k], k);
        if (rc) return rc;
        total += instance_bytes(p[k]);
    }
    *bytes = total + tables_bytes(n_inst, p);
    return LBM_OK;
}

int lbm_init(lbm_ctx **out, int32_t n_inst, const lbm_params *p, const lbm_fields *f, void *workspace,
             size_t workspace_bytes, void *stream)
{
    g_err[0] = 0;
    if (!out) return fail(LBM_E_ARG, "lbm_init: ctx pointer is NULL");
    *out = nullptr;
    if (!f) return fail(LBM_E_ARG, "lbm_init: fields are NULL");
    size_t need = 0;
    int rc = lbm_workspace_size(n_inst, p, &need);
    if (rc) return rc;
    for (int k = 0; k < n_inst; ++k) {
        if (!f[k].phi0 || !f[k].ux || !f[k].uy) return fail(LBM_E_ARG, "instance %d: phi0, ux and uy are required", k);
        if (p[k].lattice != LBM_LATTICE_D2Q9 && !f[k].uz)
            return fail(LBM_E_ARG, "instance %d: uz is required on 3D lattices", k);
        if (!f[k].D && !finite_pos(p[k].D_const))
            return fail(LBM_E_ARG, "instance %d: D_const must be finite and > 0 when D is NULL", k);
    }
    if (workspace) {
        if (workspace_bytes < need) return fail(LBM_E_ARG, "lbm_init: workspace of %zu bytes, %zu needed", workspace_bytes, need);
        if ((uintptr_t)workspace % kAlign) return fail(LBM_E_ARG, "lbm_init: workspace not 256-byte aligned");
    }
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_E_ARG, "lbm_init: out of host memory");
    c->stream = static_cast<hipStream_t>(stream);
    {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            c->device = dev;
            if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess)
                c->lds_per_cu = lds;
        }
        // the address of this device's copy of the static scratch array (once per device, with it current)
        if (dev >= 0 && dev < kMaxDevices) {
            std::lock_guard<std::mutex> lock(g_scratch_mu);
            if (!g_scratch_ptr[dev]) {
                void *ptr = nullptr;
                hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
                if (e != hipSuccess) {
                    delete c;
                    return hip_fail(e, "lbm_init: hipGetSymbolAddress of the static scratch array");
                }
                g_scratch_ptr[dev] = static_cast<double *>(ptr);
            }
        }
    }
    if (workspace) {
        c->ws = static_cast<char *>(workspace);
    } else {
        hipError_t e = hipMalloc(&c->ws, need);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "lbm_init: hipMalloc of the workspace");
        }
        c->owns_ws = true;
    }
    char *w = c->ws;
    c->partials = reinterpret_cast<double *>(w);
    c->result = reinterpret_cast<double *>(w + kPartialBytes);
    c->flag = reinterpret_cast<int *>(w + kPartialBytes + 256);
    w += align_up(kScratchBytes, kAlign);
    c->inst.resize(n_inst);
    c->uniform = true;
    for (int k = 0; k < n_inst; ++k) {
        Instance &in = c->inst[k];
        in.p = p[k];
        in.mode = mode_of(p[k]);
        in.L = layout_of(p[k]);
        in.lc1 = default_launch(in.p, in.mode, f[k].D != nullptr, n_inst, c->lds_per_cu);
        in.lc = n_inst == 1 && fusable(in.p) && (int64_t)in.p.nx * in.p.ny >= fuse_min_nodes(in.mode)
                    ? fused_default(in.p, in.mode)
                    : in.lc1;
        const size_t pb = pops_bytes(p[k]), vb = vel_bytes(p[k]), fb = field_bytes(p[k]);
        in.buf[0] = w;
        in.buf[1] = w + pb;
        in.alt = w + pb;
        w += 2 * pb;
        in.u = w;
        w += vb;
        in.k = w;
        in.s = w + fb;
        w += 2 * fb;
        in.bc = nullptr;
        if (p[k].boundary != LBM_BC_PERIODIC) {
            in.bc = w;
            w += fb;
        }
        in.has_D = f[k].D != nullptr;
        in.has_src = false;
        in.step = 0;
        in.f16 = f16_of(p[k]);
        if (in.mode != c->inst[0].mode || in.p.aux != c->inst[0].p.aux || in.p.boundary != LBM_BC_PERIODIC ||
            (in.p.tau3 != 0.0 && in.p.tau3 != 1.0) || in.p.lattice != LBM_LATTICE_D2Q9)
            c->uniform = false;  // batched launches cover periodic D2Q9 TRT-R instances of one storage/aux form
    }
    // A uniform batch of instances that can be fused runs two steps per launch, in one batched launch of
    // 128 x 16 tiles (the 256-instance C4 batch, N = 32..508, FP32: 99k MLUPS against 67k for the
    // best one-step schedule; 256-column tiles and 8 or 32 rows, flat or LPT, measured slower).
    bool batch_fuses = n_inst > 1 && c->uniform;
    for (const Instance &in : c->inst) batch_fuses &= fusable(in.p) && in.p.aux != LBM_AUX_FLUX;
    if (batch_fuses)
        for (Instance &in : c->inst) {
            in.lc = Launch{};
            in.lc.rows = 16;
            in.lc.xcd_remap = 1;
            in.lc.fuse = 2;
            in.lc.fuse_width = 128;
        }
    // Cached stores (honoured by every one-instance launch but the local form's walking loop) when what
    // the steps touch (both population buffers and the per-node fields of every instance, padding
    // columns excluded) fits in the 256 MiB Infinity Cache: the next step then reads the new state back
    // from it (1024^2-1792^2: FP32 +7-11 %, FP64 +10-14 %; FP16 up to 2304^2: +2-9 %; flux form
    // +12-21 %; D3Q19/D3Q27 96^3-128^3 +8-23 %).  Beyond that, the old buffer, the new one and the
    // fields cycle through the cache and every line is evicted before its next use (-2 to -9 %), so
    // the new state streams to HBM.  Served from the cache, the step no longer depends on DRAM page
    // locality: row bands (each XCD's rows and their edges in one L2) with every wave resident beat the
    // streaming orders and caps (2048^2 FP16 162k against 140k MLUPS, 1024^2 FP32 +6 %, D3Q19/D3Q27
    // 96^3-128^3 +24-30 %, flux form and walls +1-3 %).
    size_t touched = 0;
    for (const Instance &in : c->inst)
        touched += (size_t)in.L.nx * rows_of(in.L) *
                   (2 * in.L.q * store_bytes(in.mode) + (dim_of(in.L) + (in.has_D ? 1 : 0)) * math_bytes(in.mode));
    // One periodic instance (D2Q9 TRT-R or MRT-R with the local or no aux term, or D3Q19/D3Q27) that
    // fits only with a single population buffer is updated in place (stores = 2, both buffer slots name
    // one buffer): 2048^2 FP32 then
    // touches 185 MB per step instead of 335 MB (89.9k against 82.3k MLUPS).
    const Instance &i0 = c->inst[0];
    const size_t one_buffer = (size_t)i0.L.nx * rows_of(i0.L) * i0.L.q * store_bytes(i0.mode);
    const bool inplace = touched > kInfinityCacheBytes && touched - one_buffer <= kInfinityCacheBytes &&
                         in_place_ok(i0.p, i0.mode, n_inst) && i0.lc.rows == 1 && i0.lc.fuse != 2;
    // One FP32 instance that takes two steps per launch and whose steps touch no more than the L2 caches
    // hold together streams its stores, in both of its launches: 512^2 with a D field, two steps 55.6k ->
    // 60.4k and one step 56.8k -> 65.7k MLUPS (the adjoint's forward pass and recomputation); FP64 at
    // 512^2 (44 MB) and FP32 from 724^2 (38 MB) measured faster with cached stores, FP32 at 384^2 (one
    // step per launch) level.
    const bool l2_streams = n_inst == 1 && c->inst[0].mode == MODE_F32_F32 && c->inst[0].lc.fuse == 2 &&
                            touched <= kL2Bytes;
    c->l2_streams = l2_streams;
    for (Instance &in : c->inst) {
        for (Launch *lc : {&in.lc, &in.lc1}) {
            lc->stores = touched <= kInfinityCacheBytes && !l2_streams &&
                         (in.p.lattice != LBM_LATTICE_D2Q9 || in.p.aux == LBM_AUX_FLUX || lc->rows == 1 || lc->fuse == 2);
            if (inplace) lc->stores = 2;
            if (lc->stores) {
                lc->xcd_remap = 1;
                lc->xcd_rows = 0;
                lc->max_waves = 0;
                lc->lds_reserve = 0;
            }
        }
        if (inplace) in.buf[1] = in.buf[0];
    }
    const size_t items = max_items_of(n_inst, p);
    c->d_desc = reinterpret_cast<InstDesc *>(w);
    w += align_up((size_t)n_inst * sizeof(InstDesc), kAlign);
    for (int j = 0; j < 2; ++j) {
        const size_t ni = j == 0 ? items : (n_inst > 1 ? max_items2_of(n_inst, p) : 0);
        c->sched[j].d_items = reinterpret_cast<WorkItem *>(w);
        w += align_up(ni * sizeof(WorkItem), kAlign);
        c->sched[j].d_block_start = reinterpret_cast<int32_t *>(w);
        w += align_up((ni + 1) * sizeof(int32_t), kAlign);
    }
    for (int k = 0; k < n_inst; ++k) c->inst[k].clock = reinterpret_cast<int64_t *>(w) + 2 * k;  // zeroed below
    // a uniform batch defaults to one flat launch; FP32 runs it with at most 6 waves per SIMD (+2 %)
    if (n_inst > 1 && c->uniform) c->batch = lbm_batch{LBM_BATCH_FLAT, 0, c->inst[0].mode == MODE_F32_F32 ? 6 : 0};

    // Zero everything the library owns (padding columns included) so that a state is a
    // deterministic byte image; this also clears the flags.
    hipError_t e = hipMemsetAsync(c->ws, 0, need, c->stream);
    if (e != hipSuccess) {
        lbm_free(c);
        return hip_fail(e, "lbm_init: clearing the workspace");
    }
    for (int k = 0; k < n_inst && rc == LBM_OK; ++k) {
        Instance &in = c->inst[k];
        rc = set_velocity(c, in, f[k].ux, f[k].uy, f[k].uz);
        if (rc == LBM_OK && in.has_D)  // k = tau1 - 1/2 = kappa / (cs^2 dt) = 3 kappa dt / dx^2
            rc = prep_field(c, in, f[k].D, nullptr, 3.0 * in.p.dt / (in.p.dx * in.p.dx), 0.0, in.k, 1);
        if (rc == LBM_OK && in.bc)  // Dirichlet (edge or wall) values start as phi0's
            rc = prep_field(c, in, f[k].phi0, nullptr, 1.0, 0.0, in.bc, 0);
        if (rc == LBM_OK) {
            InitArgs ia;
            ia.phi0 = f[k].phi0;
            ia.u = in.u;
            ia.dst = in.buf[0];
            ia.L = in.L;
            ia.f16 = in.f16;
            ia.range_flag = c->flag;
            ia.walls = in.p.boundary == LBM_BC_WALLS ? 1 : 0;
            e = is3d(in) ? launch_init3(in.mode, ia, c->stream) : launch_init(in.mode, ia, c->stream);
            if (e != hipSuccess) rc = hip_fail(e, "init kernel launch");
        }
    }
    int flag[2] = {0, 0};
    if (rc == LBM_OK) {
        e = hipMemcpyAsync(flag, c->flag, sizeof flag, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = hip_fail(e, "lbm_init: synchronizing");
    }
    if (rc == LBM_OK && flag[0]) rc = fail(LBM_E_ARG, "lbm_init: an F16S population does not fit FP16 at this scale_log2");
    if (rc == LBM_OK && flag[1]) rc = fail(LBM_E_ARG, "lbm_init: D field has a value that is not finite and > 0");
    if (rc == LBM_OK) rc = refresh_tables(c);
    if (rc != LBM_OK) {
        char keep[512];
        std::memcpy(keep, g_err, sizeof keep);
        lbm_free(c);
        std::memcpy(g_err, keep, sizeof keep);
        return rc;
    }
    *out = c;
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, int32_t nsteps, const double *const *ux, const double *const *uy, const double *const *S,
             const double *const *dSdt)
{
    g_err[0] = 0;
    if (!c) return fail(LBM_E_STATE, "lbm_step: NULL context");
    if (nsteps < 0) return fail(LBM_E_ARG, "lbm_step: nsteps < 0");
    if ((ux == nullptr) != (uy == nullptr)) return fail(LBM_E_ARG, "lbm_step: give both ux and uy or neither");
    if (!S && dSdt) return fail(LBM_E_ARG, "lbm_step: dSdt without S");
    const int n = (int)c->inst.size();
    if (ux)
        for (int k = 0; k < n; ++k) {
            if (!ux[k] || !uy[k]) return fail(LBM_E_ARG, "lbm_step: instance %d: NULL velocity entry", k);
            if (is3d(c->inst[k])) return fail(LBM_E_ARG, "lbm_step: instance %d is three-dimensional: use lbm_set_velocity", k);
        }
    int rc = LBM_OK;
    bool changed = false;
    for (int k = 0; k < n && rc == LBM_OK; ++k) {
        Instance &in = c->inst[k];
        if (ux) rc = set_velocity(c, in, ux[k], uy[k]);
        const bool src = S && S[k];
        changed |= src != in.has_src;
        in.has_src = src;
        if (rc == LBM_OK && src)  // s = dt S + dt^2/2 dS/dt (Eq. (14), source terms)
            rc = prep_field(c, in, S[k], dSdt ? dSdt[k] : nullptr, in.p.dt, 0.5 * in.p.dt * in.p.dt, in.s, 0);
    }
    if (rc == LBM_OK && changed) rc = refresh_tables(c);
    if (rc) return rc;
    // The step counters advance by the steps actually enqueued, also when a launch fails part-way
    // (graph replays keep the buffer parity: a graph holds an even number of steps).
    int left = nsteps;
    auto account = [&](int status) {
        for (Instance &in : c->inst) in.step += nsteps - left;
        return status;
    };
    if (left >= 2 * kGraphSteps) {
        hipGraphExec_t x = nullptr;
        rc = graph_for(c, &x);
        if (rc) return rc;
        for (; left >= kGraphSteps; left -= kGraphSteps) {
            hipError_t e = hipGraphLaunch(x, c->stream);
            if (e != hipSuccess) return account(hip_fail(e, "hipGraphLaunch"));
        }
    }
    if (fused(c))
        for (; left >= 2; left -= 2) {
            rc = enqueue_fused(c, c->stream);
            if (rc) return account(rc);
        }
    for (; left > 0; --left) {
        rc = enqueue_step(c, c->stream);
        if (rc) return account(rc);
    }
    return account(LBM_OK);
}

namespace {
// The diagnostics of lbm_macros with the reduction's per-block partials and result in `partials` and
// `result` (device).
int macros_into(lbm_ctx *c, int32_t inst, double *phi_out, const double *ref, lbm_stats *out, double *partials,
                double *result)
{
    Instance &in = c->inst[inst];
    MacroArgs a;
    a.src = in.buf[c->parity];
    a.ref = ref;
    a.phi_out = phi_out;
    a.L = in.L;
    a.f16 = in.f16;
    a.edge.u = in.u;
    a.edge.bc = in.bc;
    a.edge.kind = in.lc.stores == 2 && c->parity == 1 ? 3 : in.p.boundary;  // 3: one buffer after a streaming step
    a.partials = partials;
    hipError_t e = is3d(in) ? launch_macros3(in.mode, a, result, c->stream)
                            : launch_macros(in.mode, a, result, c->stream);
    if (e != hipSuccess) return hip_fail(e, "macros kernel launch");
    double r[6];
    e = hipMemcpyAsync(r, result, sizeof r, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_macros: reading the result");
    const double nn = (double)in.L.nx * in.L.ny * in.L.nz;
    out->mass = r[0];
    out->rms_err = ref ? std::sqrt(r[1] / nn) : 0.0;
    out->l2_rel_err = (ref && r[2] > 0) ? std::sqrt(r[1] / r[2]) : 0.0;
    out->max_abs_err = ref ? r[3] : 0.0;
    out->max_abs_phi = r[4];
    out->nonfinite = (int64_t)r[5];
    out->step = in.step;
    if (out->nonfinite > 0)
        return fail(LBM_E_NONFINITE, "instance %d: %lld non-finite phi values (blow-up)", inst, (long long)out->nonfinite);
    return LBM_OK;
}
}  // namespace

int lbm_macros(lbm_ctx *c, int32_t inst, double *phi_out, const double *ref, lbm_stats *out)
{
    g_err[0] = 0;
    if (!check_inst(c, inst)) return fail(LBM_E_STATE, "lbm_macros: bad context or instance %d", inst);
    if (!out) return fail(LBM_E_ARG, "lbm_macros: out is NULL");
    return macros_into(c, inst, phi_out, ref, out, c->partials, c->result);
}

int lbm_macros_static(lbm_ctx *c, int32_t inst, double *phi_out, const double *ref, lbm_stats *out)
{
    g_err[0] = 0;
    if (!check_inst(c, inst)) return fail(LBM_E_STATE, "lbm_macros_static: bad context or instance %d", inst);
    if (!out) return fail(LBM_E_ARG, "lbm_macros_static: out is NULL");
    double *sp = c->device >= 0 && c->device < kMaxDevices ? g_scratch_ptr[c->device] : nullptr;
    if (!sp) return fail(LBM_E_STATE, "lbm_macros_static: no static scratch on device %d", c->device);
    // the reduction runs at most kMacroBlocks blocks (each writes its partials before the single-block
    // pass reads them), so nothing needs clearing; refuse a grid that would not fit all the same
    const Instance &in = c->inst[inst];
    const int64_t nodes = (int64_t)in.L.nx * in.L.ny * in.L.nz;
    const int64_t blocks = std::min<int64_t>(std::max<int64_t>((nodes + 255) / 256, 1), kMacroBlocks);
    if ((size_t)blocks * kMacroPartialDoubles + 8 > kStaticScratchDoubles)
        return fail(LBM_E_ARG, "lbm_macros_static: %lld reduction blocks exceed the static scratch of %zu bytes",
                    (long long)blocks, kStaticScratchDoubles * sizeof(double));
    return macros_into(c, inst, phi_out, ref, out, sp, sp + (size_t)kMacroBlocks * kMacroPartialDoubles);
}

int lbm_set_velocity(lbm_ctx *c, int32_t inst, const double *ux, const double *uy, const double *uz)
{
    g_err[0] = 0;
    if (!check_inst(c, inst)) return fail(LBM_E_STATE, "lbm_set_velocity: bad context or instance %d", inst);
    Instance &in = c->inst[inst];
    if (!ux || !uy || (is3d(in) && !uz)) return fail(LBM_E_ARG, "lbm_set_velocity: a velocity component is NULL");
    return set_velocity(c, in, ux, uy, uz);
}

int lbm_set_dirichlet(lbm_ctx *c, int32_t inst, const double *phi_b)
{
    g_err[0] = 0;
    if (!check_inst(c, inst)) return fail(LBM_E_STATE, "lbm_set_dirichlet: bad context or instance %d", inst);
    if (!phi_b) return fail(LBM_E_ARG, "lbm_set_dirichlet: phi_b is NULL");
    Instance &in = c->inst[inst];
    if (in.p.boundary == LBM_BC_PERIODIC) return fail(LBM_E_STATE, "lbm_set_dirichlet: instance %d is periodic", inst);
    return prep_field(c, in, phi_b, nullptr, 1.0, 0.0, in.bc, 0);
}

int lbm_populations(lbm_ctx *c, int32_t inst, double *g_out)
{
    g_err[0] = 0;
    if (!check_inst(c, inst)) return fail(LBM_E_STATE, "lbm_populations: bad context or instance %d", inst);
    if (!g_out) return fail(LBM_E_ARG, "lbm_populations: g_out is NULL");
    Instance &in = c->inst[inst];
    PopArgs a;
    a.src = in.buf[c->parity];
    a.out = g_out;
    a.L = in.L;
    a.f16 = in.f16;
    a.edge.u = in.u;
    a.edge.bc = in.bc;
    a.edge.kind = in.lc.stores == 2 && c->parity == 1 ? 3 : in.p.boundary;  // 3: one buffer after a streaming step
    hipError_t e = is3d(in) ? launch_populations3(in.mode, a, c->stream) : launch_populations(in.mode, a, c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "populations kernel launch");
}

int lbm_state_bytes(lbm_ctx *c, int32_t inst, size_t *bytes)
{
    g_err[0] = 0;
    if (!check_inst(c, inst)) return fail(LBM_E_STATE, "lbm_state_bytes: bad context or instance %d", inst);
    if (!bytes) return fail(LBM_E_ARG, "lbm_state_bytes: bytes is NULL");
    *bytes = pops_bytes(c->inst[inst].p);
    return LBM_OK;
}

int lbm_state_save(lbm_ctx *c, int32_t inst, void *dst)
{
    g_err[0] = 0;
    if (!check_inst(c, inst)) return fail(LBM_E_STATE, "lbm_state_save: bad context or instance %d", inst);
    if (!dst) return fail(LBM_E_ARG, "lbm_state_save: dst is NULL");
    Instance &in = c->inst[inst];
    hipError_t e;
    if (in.lc.stores == 2 && c->parity == 1) {  // one buffer after a streaming step: write the standard image
        const size_t used = (size_t)pop_elems(in.L) * store_bytes(in.mode);
        e = is3d(in) ? launch_relayout3(store_bytes(in.mode), in.buf[0], dst, in.L, c->stream)
                     : launch_relayout(store_bytes(in.mode), in.buf[0], dst, in.L, c->stream);
        if (e == hipSuccess && pops_bytes(in.p) > used)
            e = hipMemsetAsync(static_cast<char *>(dst) + used, 0, pops_bytes(in.p) - used, c->stream);
    } else {
        e = hipMemcpyAsync(dst, in.buf[c->parity], pops_bytes(in.p), hipMemcpyDeviceToDevice, c->stream);
    }
    return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_state_save");
}

int lbm_state_load(lbm_ctx *c, int32_t inst, const void *src, int64_t step)
{
    g_err[0] = 0;
    if (!check_inst(c, inst)) return fail(LBM_E_STATE, "lbm_state_load: bad context or instance %d", inst);
    if (!src) return fail(LBM_E_ARG, "lbm_state_load: src is NULL");
    if (step < 0) return fail(LBM_E_ARG, "lbm_state_load: step < 0");
    Instance &in = c->inst[inst];
    hipError_t e = in.lc.stores == 2 && c->parity == 1  // one buffer after a streaming step: its layout
                       ? (is3d(in) ? launch_relayout3(store_bytes(in.mode), src, in.buf[0], in.L, c->stream)
                                   : launch_relayout(store_bytes(in.mode), src, in.buf[0], in.L, c->stream))
                       : hipMemcpyAsync(in.buf[c->parity], src, pops_bytes(in.p), hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_state_load");
    in.step = step;
    return sync_clock(c, in);
}

int lbm_set_launch(lbm_ctx *c, int32_t inst, const lbm_launch *cfg)
{
    g_err[0] = 0;
    if (!c || inst < -1 || inst >= (int32_t)c->inst.size())
        return fail(LBM_E_STATE, "lbm_set_launch: bad context or instance %d", inst);
    if (!cfg) return fail(LBM_E_ARG, "lbm_set_launch: cfg is NULL");
    if (cfg->fuse < 0 || cfg->fuse > 2) return fail(LBM_E_ARG, "lbm_set_launch: fuse=%d must be 0, 1 or 2", cfg->fuse);
    const bool two = cfg->fuse == 2;
    const int max_rows = two ? 256 : 64;
    if (cfg->rows < 1 || cfg->rows > max_rows)
        return fail(LBM_E_ARG, "lbm_set_launch: rows=%d outside 1..%d", cfg->rows, max_rows);
    if (cfg->xcd_remap < 0 || cfg->xcd_remap > 3) return fail(LBM_E_ARG, "lbm_set_launch: xcd_remap must be 0..3");
    if (cfg->xcd_remap == 3 && (cfg->xcd_rows < 1 || cfg->xcd_rows > 64))
        return fail(LBM_E_ARG, "lbm_set_launch: xcd_rows=%d outside 1..64 (xcd_remap 3)", cfg->xcd_rows);
    if (cfg->stores < 0 || cfg->stores > 2) return fail(LBM_E_ARG, "lbm_set_launch: stores=%d must be 0, 1 or 2", cfg->stores);
    const bool want_one = cfg->stores == 2;
    for (int k = 0; k < (int)c->inst.size(); ++k) {
        if (inst != -1 && inst != k) continue;
        const Instance &in = c->inst[k];
        if (want_one && !in_place_ok(in.p, in.mode, (int)c->inst.size()))
            return fail(LBM_E_ARG, "lbm_set_launch: stores=2 (one buffer in place) needs a context of one periodic "
                                   "instance: D2Q9 with the local or no auxiliary term, or D3Q19/D3Q27 without FP64 math");
        if (want_one && (cfg->rows != 1 || two))
            return fail(LBM_E_ARG, "lbm_set_launch: stores=2 (one buffer in place) needs rows=1 and fuse 0 or 1");
        if (two && (!fusable(in.p) ||
                    (c->inst.size() > 1 && (!c->uniform || inst != -1 || in.p.aux == LBM_AUX_FLUX))))
            return fail(LBM_E_ARG, "lbm_set_launch: fuse=2 needs periodic D2Q9 TRT-R instances: one instance, or every "
                                   "instance of a uniform batch at once (inst -1) with the local or no auxiliary term");
        if (two && in.p.aux == LBM_AUX_FLUX && cfg->tile_width == 512)
            return fail(LBM_E_ARG, "lbm_set_launch: the flux form's two-step tiles are 128 or 256 columns wide");
    }
    if (two ? (cfg->tile_width != 128 && cfg->tile_width != 256 && cfg->tile_width != 512)
            : (cfg->tile_width != 64 && cfg->tile_width != 256))
        return fail(LBM_E_ARG, "lbm_set_launch: tile_width=%d must be %s", cfg->tile_width,
                    two ? "128, 256 or 512 with fuse=2" : "64 or 256");
    if (cfg->max_waves != 0 && (two || cfg->max_waves < 3 || cfg->max_waves > 8))
        return fail(LBM_E_ARG, "lbm_set_launch: max_waves=%d must be 0 or 3..8 (0 with fuse=2)", cfg->max_waves);
    Launch lc{};
    lc.rows = cfg->rows;
    lc.xcd_remap = cfg->xcd_remap;
    lc.wide = cfg->tile_width == 256 ? 1 : 0;
    lc.max_waves = cfg->max_waves;
    lc.lds_reserve = lds_reserve_for(cfg->max_waves, c->lds_per_cu);
    lc.xcd_rows = cfg->xcd_remap == 3 ? cfg->xcd_rows : 0;
    lc.stores = cfg->stores;
    lc.fuse = two ? 2 : 1;
    lc.fuse_width = two ? cfg->tile_width : 0;
    for (int k = 0; k < (int)c->inst.size(); ++k) {
        if (inst != -1 && inst != k) continue;
        Instance &in = c->inst[k];
        const bool was_one = in.buf[1] == in.buf[0];
        if (was_one && !want_one) {
            // one buffer -> two: after an odd number of steps the state is in the streaming step's layout;
            // its standard image goes to the second buffer, which then holds the state (parity 1)
            if (c->parity == 1) {
                hipError_t e = is3d(in) ? launch_relayout3(store_bytes(in.mode), in.buf[0], in.alt, in.L, c->stream)
                                        : launch_relayout(store_bytes(in.mode), in.buf[0], in.alt, in.L, c->stream);
                if (e != hipSuccess) return hip_fail(e, "lbm_set_launch: converting the one-buffer state");
            }
            in.buf[1] = in.alt;
        } else if (!was_one && want_one) {
            // two buffers -> one: the state must sit in buffer 0 in the standard layout (parity 0)
            if (c->parity == 1) {
                hipError_t e = hipMemcpyAsync(in.buf[0], in.buf[1], pops_bytes(in.p), hipMemcpyDeviceToDevice, c->stream);
                if (e != hipSuccess) return hip_fail(e, "lbm_set_launch: moving the state to one buffer");
                c->parity = 0;
                const int rc = sync_clock(c, in);
                if (rc) return rc;
            }
            in.buf[1] = in.buf[0];
        }
        in.lc = lc;
        if (!two) in.lc1 = lc;  // fused: single steps keep a one-step launch of the same store kind
        else in.lc1.stores = lc.stores;
    }
    c->l2_streams = false;  // the caller's store kind holds for the adjoint's recomputation too
    return refresh_tables(c);
}

int lbm_get_launch(lbm_ctx *c, int32_t inst, lbm_launch *cfg)
{
    g_err[0] = 0;
    if (!check_inst(c, inst)) return fail(LBM_E_STATE, "lbm_get_launch: bad context or instance %d", inst);
    if (!cfg) return fail(LBM_E_ARG, "lbm_get_launch: cfg is NULL");
    const Launch &lc = c->inst[inst].lc;
    const bool two = lc.fuse == 2;
    cfg->rows = lc.rows;
    cfg->xcd_remap = lc.xcd_remap;
    cfg->tile_width = two ? lc.fuse_width : (lc.wide ? 256 : 64);
    cfg->max_waves = lc.max_waves;
    cfg->xcd_rows = lc.xcd_rows;
    cfg->stores = lc.stores;
    cfg->fuse = two ? 2 : 1;
    return LBM_OK;
}

int lbm_set_batch(lbm_ctx *c, const lbm_batch *cfg)
{
    g_err[0] = 0;
    if (!c) return fail(LBM_E_STATE, "lbm_set_batch: NULL context");
    if (!cfg) return fail(LBM_E_ARG, "lbm_set_batch: cfg is NULL");
    if (cfg->policy < LBM_BATCH_SERIAL || cfg->policy > LBM_BATCH_LPT)
        return fail(LBM_E_ARG, "lbm_set_batch: unknown policy %d", cfg->policy);
    if ((cfg->policy == LBM_BATCH_STRIDED || cfg->policy == LBM_BATCH_LPT) && cfg->blocks < 1)
        return fail(LBM_E_ARG, "lbm_set_batch: persistent policies need blocks >= 1");
    if (cfg->max_waves != 0 && (cfg->max_waves < 3 || cfg->max_waves > 8))
        return fail(LBM_E_ARG, "lbm_set_batch: max_waves=%d must be 0 or 3..8", cfg->max_waves);
    if (cfg->policy != LBM_BATCH_SERIAL && !c->uniform)
        return fail(LBM_E_UNSUPPORTED, "lbm_set_batch: instances differ in storage/arithmetic or aux form");
    c->batch = *cfg;
    return refresh_tables(c);
}

int lbm_get_batch(lbm_ctx *c, lbm_batch *cfg)
{
    g_err[0] = 0;
    if (!c) return fail(LBM_E_STATE, "lbm_get_batch: NULL context");
    if (!cfg) return fail(LBM_E_ARG, "lbm_get_batch: cfg is NULL");
    *cfg = c->batch;
    return LBM_OK;
}

namespace {
int adjoint_ok(lbm_ctx *c, int32_t inst, const char *who)
{
    if (!check_inst(c, inst)) return fail(LBM_E_STATE, "%s: bad context or instance %d", who, inst);
    const Instance &in = c->inst[inst];
    if (is_f16_mode(in.mode)) return fail(LBM_E_UNSUPPORTED, "%s: no adjoint for FP16 storage", who);
    if (in.p.aux == LBM_AUX_FLUX) return fail(LBM_E_UNSUPPORTED, "%s: no adjoint for the flux form of the aux term", who);
    if (in.p.boundary != LBM_BC_PERIODIC) return fail(LBM_E_UNSUPPORTED, "%s: no adjoint for Dirichlet edges or walls", who);
    if (in.p.tau3 != 0.0 && in.p.tau3 != 1.0) return fail(LBM_E_UNSUPPORTED, "%s: no adjoint for the MRT-R operator", who);
    if (is3d(in)) return fail(LBM_E_UNSUPPORTED, "%s: no adjoint on 3D lattices", who);
    return LBM_OK;
}
}  // namespace

int lbm_adjoint_bytes(lbm_ctx *c, int32_t inst, size_t *bytes)
{
    g_err[0] = 0;
    int rc = adjoint_ok(c, inst, "lbm_adjoint_bytes");
    if (rc) return rc;
    if (!bytes) return fail(LBM_E_ARG, "lbm_adjoint_bytes: bytes is NULL");
    const Instance &in = c->inst[inst];
    *bytes = (size_t)pop_elems(in.L) * math_bytes(in.mode);
    return LBM_OK;
}

int lbm_adjoint_seed(lbm_ctx *c, int32_t inst, const double *dLdphi, void *lam)
{
    g_err[0] = 0;
    int rc = adjoint_ok(c, inst, "lbm_adjoint_seed");
    if (rc) return rc;
    if (!dLdphi || !lam) return fail(LBM_E_ARG, "lbm_adjoint_seed: NULL pointer");
    const Instance &in = c->inst[inst];
    hipError_t e = launch_adjoint_seed(in.mode, dLdphi, lam, in.L, c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "adjoint seed kernel launch");
}

namespace {
AdjArgs adj_args(const Instance &in, double *dLdD)
{
    AdjArgs a;
    a.state = nullptr;
    a.lam_in = nullptr;
    a.lam_out = nullptr;
    a.u = in.u;
    a.k = in.has_D ? in.k : nullptr;
    a.s = in.has_src ? in.s : nullptr;
    a.L = in.L;
    a.k_const = 3.0 * in.p.D_const * in.p.dt / (in.p.dx * in.p.dx);
    a.lambda = in.p.lambda;
    a.dk_dD = 3.0 * in.p.dt / (in.p.dx * in.p.dx);
    a.f16 = in.f16;
    a.grad = dLdD;
    return a;
}
}  // namespace

int lbm_adjoint_step(lbm_ctx *c, int32_t inst, const void *state, const void *lam_in, void *lam_out, double *dLdD)
{
    g_err[0] = 0;
    int rc = adjoint_ok(c, inst, "lbm_adjoint_step");
    if (rc) return rc;
    if (!state || !lam_in || !lam_out || !dLdD) return fail(LBM_E_ARG, "lbm_adjoint_step: NULL pointer");
    if (lam_in == lam_out) return fail(LBM_E_ARG, "lbm_adjoint_step: lam_in and lam_out must not alias");
    AdjArgs a = adj_args(c->inst[inst], dLdD);
    a.state = state;
    a.lam_in = lam_in;
    a.lam_out = lam_out;
    hipError_t e = launch_adjoint(c->inst[inst].mode, c->inst[inst].p.aux, a, c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "adjoint kernel launch");
}

int lbm_adjoint_segment(lbm_ctx *c, int32_t inst, void *states, int32_t nsteps, void *lam, void *lam_tmp, double *dLdD)
{
    g_err[0] = 0;
    int rc = adjoint_ok(c, inst, "lbm_adjoint_segment");
    if (rc) return rc;
    if (!states || !lam || !lam_tmp || !dLdD) return fail(LBM_E_ARG, "lbm_adjoint_segment: NULL pointer");
    if (nsteps < 1) return fail(LBM_E_ARG, "lbm_adjoint_segment: nsteps must be >= 1");
    if (lam == lam_tmp) return fail(LBM_E_ARG, "lbm_adjoint_segment: lam and lam_tmp must not alias");
    const Instance &in = c->inst[inst];
    const size_t sb = pops_bytes(in.p);
    char *img = static_cast<char *>(states);
    // Recomputation: image j + 1 = one step of image j, image to image with two buffers whatever the
    // context's own store kind (state images are always in the two-buffer layout).  The next launch
    // reads each new image at once, so a context whose steps stream only because they fit the L2 caches
    // recomputes with cached stores (512^2 FP32: 5.3 us per step against 6.2 us streaming).
    StepArgs a;
    a.d = c->h_desc[inst];
    if (a.d.lc.stores == 2 || c->l2_streams) a.d.lc.stores = 1;  // its lc is the one-step launch
    a.parity = 0;
    for (int32_t j = 0; j + 1 < nsteps; ++j) {
        a.d.buf[0] = img + (size_t)j * sb;
        a.d.buf[1] = img + (size_t)(j + 1) * sb;
        hipError_t e = launch_step(in.mode, in.p.aux, a, c->stream);
        if (e != hipSuccess) return hip_fail(e, "step kernel launch (adjoint segment)");
    }
    // Reverse sweep: dL/dg^{j} from dL/dg^{j+1}, j = nsteps - 1 .. 0, alternating the two arrays.
    AdjArgs g = adj_args(in, dLdD);
    void *cur = lam, *nxt = lam_tmp;
    for (int32_t j = nsteps - 1; j >= 0; --j) {
        g.state = img + (size_t)j * sb;
        g.lam_in = cur;
        g.lam_out = nxt;
        hipError_t e = launch_adjoint(in.mode, in.p.aux, g, c->stream);
        if (e != hipSuccess) return hip_fail(e, "adjoint kernel launch (adjoint segment)");
        std::swap(cur, nxt);
    }
    if (cur != lam) {
        hipError_t e = hipMemcpyAsync(lam, cur, (size_t)pop_elems(in.L) * math_bytes(in.mode), hipMemcpyDeviceToDevice,
                                      c->stream);
        if (e != hipSuccess) return hip_fail(e, "lbm_adjoint_segment: copying the result");
    }
    return LBM_OK;
}

int lbm_adjoint_init(lbm_ctx *c, int32_t inst, const void *lam0, double *dLdphi0)
{
    g_err[0] = 0;
    int rc = adjoint_ok(c, inst, "lbm_adjoint_init");
    if (rc) return rc;
    if (!lam0 || !dLdphi0) return fail(LBM_E_ARG, "lbm_adjoint_init: NULL pointer");
    const Instance &in = c->inst[inst];
    hipError_t e = launch_adjoint_init(in.mode, lam0, in.u, dLdphi0, in.L, c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "adjoint init kernel launch");
}

namespace {
int bench_copy(void *dst, const void *src, size_t bytes, void *stream, bool cached, const char *who)
{
    g_err[0] = 0;
    if (!dst || !src) return fail(LBM_E_ARG, "%s: NULL pointer", who);
    if (bytes % 16 || (uintptr_t)dst % 16 || (uintptr_t)src % 16)
        return fail(LBM_E_ARG, "%s: bytes and pointers must be multiples of 16", who);
    if (bytes / 16 > (size_t)UINT32_MAX * 256) return fail(LBM_E_ARG, "%s: too large", who);
    hipError_t e = launch_copy(dst, src, bytes, cached, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LBM_OK : hip_fail(e, "copy kernel launch");
}
}  // namespace

int lbm_bench_copy(void *dst, const void *src, size_t bytes, void *stream)
{
    return bench_copy(dst, src, bytes, stream, false, "lbm_bench_copy");
}

int lbm_bench_copy_cached(void *dst, const void *src, size_t bytes, void *stream)
{
    return bench_copy(dst, src, bytes, stream, true, "lbm_bench_copy_cached");
}

int lbm_set_diffusion(lbm_ctx *c, int32_t inst, const double *D)
{
    g_err[0] = 0;
    if (!check_inst(c, inst)) return fail(LBM_E_STATE, "lbm_set_diffusion: bad context or instance %d", inst);
    if (!D) return fail(LBM_E_ARG, "lbm_set_diffusion: D is NULL");
    Instance &in = c->inst[inst];
    if (!in.has_D) return fail(LBM_E_STATE, "lbm_set_diffusion: instance %d was created with a constant D", inst);
    hipError_t e = hipMemsetAsync(c->flag + 1, 0, sizeof(int), c->stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_set_diffusion: clearing the range flag");
    // k = tau1 - 1/2 = kappa / (cs^2 dt) = 3 kappa dt / dx^2, as at lbm_init
    int rc = prep_field(c, in, D, nullptr, 3.0 * in.p.dt / (in.p.dx * in.p.dx), 0.0, in.k, 1);
    if (rc) return rc;
    int flag = 0;
    e = hipMemcpyAsync(&flag, c->flag + 1, sizeof flag, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_set_diffusion: synchronizing");
    if (flag) return fail(LBM_E_ARG, "lbm_set_diffusion: D has a value that is not finite and > 0");
    return LBM_OK;
}

int lbm_free(lbm_ctx *c)
{
    if (!c) return LBM_OK;
    int rc = LBM_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = hip_fail(e, "lbm_free: synchronizing");
    drop_graphs(c);
    if (c->capture) (void)hipStreamDestroy(c->capture);
    if (c->owns_ws && c->ws) {
        e = hipFree(c->ws);
        if (e != hipSuccess && rc == LBM_OK) rc = hip_fail(e, "lbm_free: hipFree");
    }
    delete c;
    return rc;
}

}  // extern "C"
