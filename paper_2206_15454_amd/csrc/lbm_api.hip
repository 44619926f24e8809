// lbm_api.hip -- host runtime and C ABI (include/lbm.h) of the fused
// lattice-Boltzmann LES canopy step on MI355X (gfx950).
//
// One context owns one device allocation carved into: the in-place population
// buffer (19 planes, stride padded), the moment planes of the latest step,
// the canopy table, and the FP64 accumulators of the deterministic
// reductions.  Every step is one kernel launch on the context's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_device.h"
#include "mlp_device.h"

using namespace lbmx;

struct lbm_ctx {
    lbm_params p{};
    int device = 0;
    hipStream_t stream = nullptr;
    long long n = 0;     // cells
    size_t elt = 0;      // bytes per stored population
    size_t celt = 0;     // bytes per arithmetic value
    long long qs = 0;    // population plane stride, elements
    int px = 0;          // population row pitch, cells (>= nx)
    int zp = 0;          // population z-layer pitch, cells (>= px ny)
    // launch geometry
    int bx = 256, bz = 1, nbx = 1, nbz = 1, ntiles = 1, tpp = 1;
    bool xcd_remap = true;    // plain step: contiguous tile ranges per XCD (FLAG_XCD_REMAP)
    bool mlp_remap = true;    // the same for the learned-closure kernel's walk
    int xcd_run = 0;          // plain step: runs of tiles per XCD (0: one range)
    bool force_wide = false;  // 64-bit population addresses even for small planes
    bool fx = true;           // the x-only-force kernels when the force is along x (VAR_FX)
    bool streaming = false;   // non-temporal accesses on aligned rows (FLAG_STREAMING)
    bool memorder = false;    // tiles in memory order (FLAG_MEMORDER)
    // device memory
    void *base = nullptr;
    bool owns = false;
    size_t bytes = 0;
    void *f = nullptr;
    void *mom = nullptr;
    double *lad = nullptr;
    uint16_t *fidx = nullptr;  // per-cell forest table index (forest_map only)
    double *ftab = nullptr;    // forest LAD table
    float *ftabf = nullptr;    // the same in FP32
    bool forest = false;       // lbm_set_forest active
    double *imp = nullptr;
    double *dg = nullptr;    // per-wavefront diagnostics of the last moments step
    double *stats = nullptr;
    double *red = nullptr;   // diag partials [kDiagRedDoubles] + final [16]
    double *prof = nullptr;  // [ny*10]
    void *mlp = nullptr;     // learned closure parameters
    // host state
    int64_t t = 0;
    int parity = 0;
    bool inited = false;
    bool unstable = false;
    int stats_every = 0;
    int64_t stats_n = 0;
    double cd = 0.0;
    int vector_drag = 0;
    int closure = LBM_CLOSURE_SMAG;
    int closure_every = 1;   // learned closure evaluated every this many steps
    int closure_lag = 0;     // steps since its last evaluation (0: evaluate next)
    int64_t evals = 0;       // evaluations so far (fallback counter slot = evals & 1)
    int last_fb_slot = 0;    // slot of the last evaluation
    int64_t fb_rows_cells = 0;  // cells of the rows the last evaluation gave the plain step
    bool mlp_split = true;   // evaluating steps: network rows in the learned kernel, the rest
                             // in the plain step (LBMX_MLP_SPLIT=0: one learned launch)
    MlpConst mc{};           // learned closure scalars (kernel arguments)
    int mlp_grid[8] = {};    // persistent grid of the learned-closure kernel per variant
    // evaluating steps with a row split: the plain rows run on a second
    // stream beside the learned kernel, which then takes this many blocks
    // per CU (0: one stream, the launches one after the other).  Two blocks
    // (2 of its 3 waves per SIMD) leave each SIMD room for plain-step waves,
    // which keep HBM busy while the network keeps the vector unit busy:
    // measured on 512x128x256 with the canopy-layer network every step,
    // BF16SR 39.1k -> 44.0k MLUPS, F16S 41.2k -> 46.6k (one block per CU
    // 31.7k, three 43.0k)
    int mlp_overlap = 2;
    int ncu = 0;  // compute units (queried with the second stream, once)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool diag_fresh = false; // dg holds the diagnostics of the moments lbm_moments reads
    std::string err;
};

namespace lbmx {  // forest.hip
bool forest_table(const uint32_t *codes, long long n, double afm, bool constant,
                  std::vector<uint16_t> &idx, std::vector<double> &table, std::string *why);
}

namespace {

constexpr size_t kAlign = 256;
const char *kNoCtx = "lbm: NULL context";

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t storage_bytes(int st) {
    switch (st) {
    case LBM_F64: return 8;
    case LBM_F32: return 4;
    case LBM_F16S:
    case LBM_BF16S:
    case LBM_BF16SR: return 2;
    default: return 0;
    }
}

bool valid_params(const lbm_params *p, std::string *why) {
    auto fail = [&](const char *m) {
        if (why) *why = m;
        return false;
    };
    if (!p) return fail("NULL params");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail("every dimension must be >= 1");
    if ((long long)p->nx * p->ny * p->nz >= (1LL << 31)) return fail("nx*ny*nz must be < 2^31");
    if (storage_bytes(p->storage) == 0) return fail("unknown storage type");
    if (!(p->tau0 > 0.5) || !std::isfinite(p->tau0)) return fail("tau0 must be > 0.5");
    if (!(p->c_smag >= 0.0) || !std::isfinite(p->c_smag)) return fail("c_smag must be >= 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->g[a])) return fail("g must be finite");
    if (p->bc_ylo < 0 || p->bc_ylo > 3 || p->bc_yhi < 0 || p->bc_yhi > 3)
        return fail("unknown boundary condition");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->u_wall[a])) return fail("u_wall must be finite");
    if ((p->bc_ylo == LBM_BC_PERIODIC) != (p->bc_yhi == LBM_BC_PERIODIC))
        return fail("periodic y must be set on both ends");
    return true;
}

// launch geometry: tiles of BX x 1 x BZ cells (BX*BZ = 256), one row each.
// BX is the widest of 256/128/64 that pads a row least (idle lanes of a
// ragged last tile cost bandwidth: 350 cells in 256-wide tiles leave 32% of
// the lanes idle, in 128-wide tiles 9%).  32-wide tiles, which pad less, were
// measured slower (their short rows split cache lines) and are not offered:
// the step takes a wave's z row as uniform, which needs tiles of 64 cells or
// more.  Narrow tiles are slower than 256-wide ones at equal work
// (512x140x280 FP32: 0.699 of the roofline in 128-wide tiles against 0.733;
// tiles of two adjacent y rows instead of two z rows measured the same).
// Packing the tails of several rows into one wave (350 cells in 5.5 waves
// instead of 6) was built and measured: no faster at 350x140x280, slower
// for FP32 at 200x80x160 (a wave of eight 8-cell tails touches eight
// lines), and its mapping cost the BF16SR step 2 % on other grids.
void geometry(const lbm_params *p, int *bx, int *bz, int *nbx, int *nbz) {
    int BX = 256;
    long long best = -1;
    for (int cand : {256, 128, 64}) {
        const long long waste = (long long)(p->nx + cand - 1) / cand * cand - p->nx;
        if (best < 0 || waste < best) {
            best = waste;
            BX = cand;
        }
    }
    if (const char *e = std::getenv("LBMX_BX")) {
        int v = std::atoi(e);
        if (v == 64 || v == 128 || v == 256) BX = v;
    }
    *bx = BX;
    *bz = 256 / BX;
    *nbx = (p->nx + BX - 1) / BX;
    *nbz = (p->nz + *bz - 1) / *bz;
}

// population plane stride: rounded to 256 B plus a pad that staggers the 19
// plane starts across HBM channels (a power-of-two-aligned stride makes the 19
// concurrent streams of a wave start in the same channel).  1 KiB for FP32
// and FP64, 2 KiB for the 16-bit types: measured best over 0.5-4 KiB at
// 512x128x256 (16-bit: 0.695 -> 0.708 of the roofline with 2 KiB) and no
// worse at 1024x256x512, 350x140x280 and the forest case; for FP32, 2 KiB
// was better at 512x128x256 and worse at the other two, FP64 unchanged.
long long plane_stride(long long n, size_t elt) {
    long long per = (long long)(kAlign / elt);
    long long qs = (n + per - 1) / per * per;
    long long pad_bytes = elt == 2 ? 2048 : 1024;
    if (const char *e = std::getenv("LBMX_QPAD")) {
        const long long v = std::atoll(e);
        if (v >= 0 && v <= (1LL << 30)) pad_bytes = v;
    }
    qs += (long long)(align_up((size_t)pad_bytes, kAlign) / elt);
    return qs;
}

// Whether the population accesses stream (non-temporal) by default: only for
// population arrays larger than the 256 MiB Infinity Cache.  Smaller arrays
// keep lines there from one step to the next with the default policy;
// streaming them was measured slower (200x80x160 FP32, 195 MB: 32.6k against
// 41.5k MLUPS; 250x100x200 BF16SR, 190 MB: 61.2k against 74.1k), larger ones
// faster (250x100x200 FP32, 380 MB: 34.5k against 32.7k; 350x140x280
// BF16SR, 522 MB: 60.0k against 56.4k; 512x128x256 BF16S, 637 MB: 72.0k
// against 61.3k).
constexpr long long kStreamMinBytes = 256LL << 20;

bool large_array(const lbm_params *p) {
    const long long elt = (long long)storage_bytes(p->storage);
    return (long long)NQ * p->nx * p->ny * p->nz * elt > kStreamMinBytes;
}

// Population row pitch: for the arrays that stream, rows padded to whole
// 128-byte lines, so that every row starts on a line and the row-aligned
// accesses can stream (rows of 350 FP32 cells, 1 400 B, otherwise share
// their end lines with the next row).  The step stores values of no meaning
// to the padding cells (whole lines are written; no cell of the grid reads
// them).  No padding when a row is already whole lines, for arrays that do
// not stream, or when the padded array would not be indexable in 32 bits.
// LBMX_PITCH=0|1 forces dense rows or padded rows (the populations are
// bit-identical either way).
int row_pitch(const lbm_params *p) {
    const long long elt = (long long)storage_bytes(p->storage);
    const long long per_line = 128 / elt;
    bool pad = large_array(p);
    if (const char *e = std::getenv("LBMX_PITCH")) pad = std::atoi(e) != 0;
    long long px = pad ? (p->nx + per_line - 1) / per_line * per_line : p->nx;
    if (px * p->ny * p->nz >= (1LL << 31)) px = p->nx;
    return (int)px;
}

// population z-layer pitch (cells): px ny, or, for tuning, rounded up to a
// multiple of LBMX_ZALIGN bytes and/or widened by LBMX_ZPAD bytes (multiples
// of 128, so that rows stay on cache lines).  The padding cells are never
// read or written.  No padding when the padded array would not be indexable
// in 32 bits.
int z_pitch(const lbm_params *p, int px) {
    const long long elt = (long long)storage_bytes(p->storage);
    long long bytes = (long long)px * p->ny * elt;
    if (const char *e = std::getenv("LBMX_ZALIGN")) {
        const long long v = std::atoll(e);
        if (v > 0 && v <= (1LL << 30) && v % 128 == 0) bytes = (bytes + v - 1) / v * v;
    }
    if (const char *e = std::getenv("LBMX_ZPAD")) {
        const long long v = std::atoll(e);
        if (v > 0 && v <= (1LL << 30) && v % 128 == 0) bytes += v;
    }
    long long zp = bytes / elt;
    if (zp * p->nz >= (1LL << 31)) zp = (long long)px * p->ny;
    return (int)zp;
}

struct Layout {
    size_t f, mom, lad, imp, dg, stats, red, prof, mlp, fidx, ftab, ftabf, total;
};

Layout layout(const lbm_params *p) {
    Layout L{};
    const long long n = (long long)p->nx * p->ny * p->nz;
    const size_t elt = storage_bytes(p->storage);
    const size_t celt = p->storage == LBM_F64 ? 8 : 4;
    int bx, bz, nbx, nbz;
    geometry(p, &bx, &bz, &nbx, &nbz);
    const long long ntiles = (long long)nbx * nbz * p->ny;
    const long long qs = plane_stride((long long)z_pitch(p, row_pitch(p)) * p->nz, elt);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, kAlign);
        return at;
    };
    L.f = take((size_t)NQ * qs * elt);
    L.mom = take((size_t)5 * n * celt);
    L.lad = take((size_t)p->ny * 8);
    L.imp = take((size_t)ntiles * 4 * 3 * 8);  // one triple per wavefront of a tile
    L.dg = take((size_t)ntiles * 4 * 6 * 8);   // one diagnostics record per wavefront
    L.stats = take((size_t)p->ny * nbx * nbz * 10 * 8);
    L.red = take((size_t)(kDiagRedDoubles + 16) * 8);
    L.prof = take((size_t)p->ny * 10 * 8);
    L.mlp = take(kMlpDeviceBytes);
    L.fidx = take(p->forest_map ? (size_t)n * 2 : 0);
    L.ftab = take(p->forest_map ? (size_t)kForestTable * 8 : 0);
    L.ftabf = take(p->forest_map ? (size_t)kForestTable * 4 : 0);
    L.total = off;
    return L;
}

lbm_status fail(lbm_ctx *c, lbm_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

lbm_status hip_fail(lbm_ctx *c, hipError_t e, const char *what) {
    return fail(c, LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, call, what)                          \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

lbm_status reset_accumulators(lbm_ctx *c) {
    HIPCHK(c, launch_fill(c->imp, 0.0, (size_t)c->ntiles * 4 * 3, c->stream), "clear impulse");
    HIPCHK(c, launch_fill(c->stats, 0.0, (size_t)c->p.ny * c->tpp * 10, c->stream),
           "clear statistics");
    c->stats_n = 0;
    return LBM_OK;
}

}  // namespace

extern "C" {

int32_t lbm_lattice(int32_t *c, double *w) {
    for (int q = 0; q < NQ; ++q) {
        if (c) {
            c[3 * q + 0] = CX[q];
            c[3 * q + 1] = CY[q];
            c[3 * q + 2] = CZ[q];
        }
        if (w) w[q] = weight(q);
    }
    return NQ;
}

size_t lbm_required_bytes(const lbm_params *p) {
    if (!valid_params(p, nullptr)) return 0;
    return layout(p).total;
}

lbm_status lbm_create(const lbm_params *p, void *dev_buf, size_t dev_bytes, lbm_ctx **out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    std::string why;
    if (!valid_params(p, &why)) return LBM_EINVAL;
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return LBM_ENOMEM;
    c->p = *p;
    c->stream = static_cast<hipStream_t>(p->stream);
    c->n = (long long)p->nx * p->ny * p->nz;
    c->elt = storage_bytes(p->storage);
    c->celt = p->storage == LBM_F64 ? 8 : 4;
    c->px = row_pitch(p);
    c->zp = z_pitch(p, c->px);
    c->qs = plane_stride((long long)c->zp * p->nz, c->elt);
    geometry(p, &c->bx, &c->bz, &c->nbx, &c->nbz);
    c->tpp = c->nbx * c->nbz;
    c->ntiles = c->tpp * p->ny;
    if (const char *e = std::getenv("LBMX_WIDE")) c->force_wide = std::atoi(e) != 0;
    if (const char *e = std::getenv("LBMX_FX")) c->fx = std::atoi(e) != 0;
    if (const char *e = std::getenv("LBMX_MLP_SPLIT")) c->mlp_split = std::atoi(e) != 0;
    if (const char *e = std::getenv("LBMX_MLP_OVERLAP")) c->mlp_overlap = std::max(0, std::atoi(e));
    // streaming (non-temporal) accesses for arrays beyond the Infinity Cache
    // whose rows are whole 128-byte lines (the planes start on 256-byte
    // boundaries); LBMX_STREAMING=0/1 overrides
    c->streaming = large_array(p) && ((long long)c->px * (long long)c->elt) % 128 == 0;
    if (const char *e = std::getenv("LBMX_STREAMING")) c->streaming = std::atoi(e) != 0;
    // tile order: the tiles that run at the same time span the fewest pages in
    // memory order.  The row-major order measured faster only for streaming
    // rows with planes of up to 64 MiB (512x128x256 in FP32 and 16-bit);
    // memory order was faster for 128 MiB planes and more (FP64 at that
    // size, every type at 1024x256x512) and for rows that are not whole
    // cache lines (350x140x280: +7 %).  The switch is at 96 MiB.
    // LBMX_TILE_ORDER=0/1 overrides.
    c->memorder = !c->streaming || (unsigned long long)c->qs * c->elt > (96ULL << 20);
    // FP32 and FP64 arrays beyond the Infinity Cache: memory order, with the
    // XCDs taking turns in short runs of consecutive tiles (2 for FP32, 4 for
    // FP64), so that they work side by side in one stretch of each plane
    // instead of in eight distant ones.  Measured against the better order
    // with one contiguous range per XCD, single tiles taking turns gained
    // 4.8 % (FP32) and 6.6 % (FP64) at 512x128x256, 4.3 % at 1024x256x512,
    // 3.6 / 4.6 % at 350x140x280 and 7.5 / 9 % at 250x100x200.  Of runs of
    // 1 to 16 tiles, the chosen lengths came within 1 % of the best on each
    // of these grids (single tiles: FP32 -1.6 % at 512x128x256, FP64 -6 % at
    // 1024x256x512; runs of 8: FP32 -3.7 % at 1024x256x512).  The 16-bit
    // types measured best with the choice above and one range per XCD, and
    // so did FP32 on arrays that fit the cache (200x80x160).  The
    // learned-closure kernel keeps its remapped walk.  LBMX_TILE_ORDER=0/1,
    // LBMX_XCD_REMAP=0/1 and LBMX_XCD_RUN=tiles override.
    c->xcd_remap = true;
    if (large_array(p) && c->elt >= 4) {
        c->memorder = true;
        c->xcd_run = c->elt == 8 ? 4 : 2;
    }
    if (const char *e = std::getenv("LBMX_TILE_ORDER")) c->memorder = std::atoi(e) != 0;
    if (const char *e = std::getenv("LBMX_XCD_REMAP")) {
        c->xcd_remap = c->mlp_remap = std::atoi(e) != 0;
        c->xcd_run = 0;
    }
    if (const char *e = std::getenv("LBMX_XCD_RUN")) {
        const int v = std::atoi(e);
        if (v > 0) {
            c->xcd_run = v;
            c->xcd_remap = true;
        }
    }
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return LBM_EDEVICE;
    }
    const Layout L = layout(p);
    c->bytes = L.total;
    if (dev_buf) {
        if (dev_bytes < L.total || (reinterpret_cast<uintptr_t>(dev_buf) % kAlign) != 0) {
            delete c;
            return LBM_ENOMEM;
        }
        c->base = dev_buf;
        c->owns = false;
    } else {
        if (hipMalloc(&c->base, L.total) != hipSuccess) {
            (void)hipGetLastError();
            delete c;
            return LBM_ENOMEM;
        }
        c->owns = true;
    }
    char *b = static_cast<char *>(c->base);
    c->f = b + L.f;
    c->mom = b + L.mom;
    c->lad = reinterpret_cast<double *>(b + L.lad);
    c->imp = reinterpret_cast<double *>(b + L.imp);
    c->dg = reinterpret_cast<double *>(b + L.dg);
    c->stats = reinterpret_cast<double *>(b + L.stats);
    c->red = reinterpret_cast<double *>(b + L.red);
    c->prof = reinterpret_cast<double *>(b + L.prof);
    c->mlp = b + L.mlp;
    if (p->forest_map) {
        c->fidx = reinterpret_cast<uint16_t *>(b + L.fidx);
        c->ftab = reinterpret_cast<double *>(b + L.ftab);
        c->ftabf = reinterpret_cast<float *>(b + L.ftabf);
    }
    if (launch_fill(c->lad, 0.0, (size_t)p->ny, c->stream) != hipSuccess ||
        reset_accumulators(c) != LBM_OK) {
        if (c->owns) (void)hipFree(c->base);
        delete c;
        return LBM_EDEVICE;
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx *c) {
    if (!c) return LBM_EINVAL;
    if (c->side) {  // the second stream's work ends before the memory goes
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
        (void)hipEventDestroy(c->ev_fork);
        (void)hipEventDestroy(c->ev_join);
    }
    if (c->owns && c->base) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(c->base);
    }
    delete c;
    return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err.c_str() : kNoCtx; }

lbm_status lbm_set_stream(lbm_ctx *c, void *stream) {
    if (!c) return LBM_EINVAL;
    c->stream = static_cast<hipStream_t>(stream);
    c->p.stream = stream;
    return LBM_OK;
}

lbm_status lbm_set_canopy(lbm_ctx *c, double cd, const double *lad, int32_t ny,
                          int32_t vector_drag) {
    if (!c) return LBM_EINVAL;
    if (!lad) return fail(c, LBM_EINVAL, "lbm_set_canopy: NULL lad");
    if (ny != c->p.ny) return fail(c, LBM_EINVAL, "lbm_set_canopy: lad length must equal ny");
    if (!std::isfinite(cd)) return fail(c, LBM_EINVAL, "lbm_set_canopy: cd must be finite");
    for (int j = 0; j < ny; ++j)
        if (!(lad[j] >= 0.0) || !std::isfinite(lad[j]))
            return fail(c, LBM_EINVAL, "lbm_set_canopy: lad values must be finite and >= 0");
    HIPCHK(c, hipMemcpyAsync(c->lad, lad, (size_t)ny * 8, hipMemcpyHostToDevice, c->stream),
           "lbm_set_canopy: copy");
    HIPCHK(c, hipStreamSynchronize(c->stream), "lbm_set_canopy: sync");
    c->cd = cd;
    c->vector_drag = vector_drag ? 1 : 0;
    c->forest = false;
    return LBM_OK;
}

lbm_status lbm_set_forest(lbm_ctx *c, double cd, double afm, int32_t constant_lad,
                          const uint32_t *codes, int32_t vector_drag) {
    if (!c) return LBM_EINVAL;
    if (!c->fidx)
        return fail(c, LBM_ESTATE, "lbm_set_forest: context created without forest_map");
    if (!codes) return fail(c, LBM_EINVAL, "lbm_set_forest: NULL codes");
    if (!std::isfinite(cd) || !std::isfinite(afm) || afm < 0.0)
        return fail(c, LBM_EINVAL, "lbm_set_forest: cd and afm must be finite, afm >= 0");
    std::vector<uint16_t> idx;
    std::vector<double> table;
    std::string why;
    if (!forest_table(codes, c->n, afm, constant_lad != 0, idx, table, &why))
        return fail(c, LBM_EINVAL, "lbm_set_forest: " + why);
    HIPCHK(c, hipMemcpyAsync(c->fidx, idx.data(), idx.size() * 2, hipMemcpyHostToDevice, c->stream),
           "lbm_set_forest: copy");
    std::vector<float> tablef(table.begin(), table.end());
    HIPCHK(c, hipMemcpyAsync(c->ftab, table.data(), table.size() * 8, hipMemcpyHostToDevice,
                             c->stream), "lbm_set_forest: copy");
    HIPCHK(c, hipMemcpyAsync(c->ftabf, tablef.data(), tablef.size() * 4, hipMemcpyHostToDevice,
                             c->stream), "lbm_set_forest: copy");
    HIPCHK(c, hipStreamSynchronize(c->stream), "lbm_set_forest: sync");
    c->cd = cd;
    c->vector_drag = vector_drag ? 1 : 0;
    c->forest = true;
    return LBM_OK;
}

lbm_status lbm_set_closure(lbm_ctx *c, int32_t closure, const void *blob, size_t nbytes) {
    if (!c) return LBM_EINVAL;
    if (closure == LBM_CLOSURE_SMAG) {
        c->closure = LBM_CLOSURE_SMAG;
        return LBM_OK;
    }
    if (closure != LBM_CLOSURE_MLP) return fail(c, LBM_EINVAL, "lbm_set_closure: unknown closure");
    std::vector<unsigned char> dev(kMlpDeviceBytes);
    std::string why;
    MlpConst mc{};
    if (!mlp_pack_blob(blob, nbytes, dev.data(), &mc, &why))
        return fail(c, LBM_EINVAL, "lbm_set_closure: " + why);
    HIPCHK(c, hipMemcpyAsync(c->mlp, dev.data(), dev.size(), hipMemcpyHostToDevice, c->stream),
           "lbm_set_closure: copy");
    HIPCHK(c, hipStreamSynchronize(c->stream), "lbm_set_closure: sync");
    c->closure = LBM_CLOSURE_MLP;
    c->mc = mc;
    c->closure_lag = 0;
    c->evals = 0;
    c->fb_rows_cells = 0;
    c->last_fb_slot = 0;
    return LBM_OK;
}

lbm_status lbm_set_closure_interval(lbm_ctx *c, int32_t every) {
    if (!c) return LBM_EINVAL;
    if (every < 1 || every > 1024)
        return fail(c, LBM_EINVAL, "lbm_set_closure_interval: every must be in [1, 1024]");
    c->closure_every = every;
    c->closure_lag = 0;
    return LBM_OK;
}

lbm_status lbm_init(lbm_ctx *c, const double *rho, const double *u, int32_t on_device) {
    if (!c) return LBM_EINVAL;
    if (!rho || !u) return fail(c, LBM_EINVAL, "lbm_init: NULL rho or u");
    const long long n = c->n;
    const double *drho = rho, *du = u;
    double *tmp = nullptr;
    if (!on_device) {
        HIPCHK(c, hipMallocAsync(reinterpret_cast<void **>(&tmp), (size_t)4 * n * 8, c->stream),
               "lbm_init: staging");
        HIPCHK(c, hipMemcpyAsync(tmp, rho, (size_t)n * 8, hipMemcpyHostToDevice, c->stream),
               "lbm_init: copy rho");
        HIPCHK(c, hipMemcpyAsync(tmp + n, u, (size_t)3 * n * 8, hipMemcpyHostToDevice, c->stream),
               "lbm_init: copy u");
        drho = tmp;
        du = tmp + n;
    }
    HIPCHK(c, launch_init(c->p.storage, c->f, c->qs, c->p.nx, c->px, c->p.ny, c->zp, c->mom, drho, du, (int)n, c->stream),
           "lbm_init: kernel");
    if (tmp) HIPCHK(c, hipFreeAsync(tmp, c->stream), "lbm_init: free staging");
    lbm_status s = reset_accumulators(c);
    if (s != LBM_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream), "lbm_init: sync");
    c->t = 0;
    c->parity = 0;
    c->inited = true;
    c->diag_fresh = false;
    c->closure_lag = 0;  // the next step evaluates the learned closure
    c->unstable = false;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *c, int64_t nsteps) {
    if (!c) return LBM_EINVAL;
    if (nsteps < 0) return fail(c, LBM_EINVAL, "lbm_step: n must be >= 0");
    if (!c->inited) return fail(c, LBM_ESTATE, "lbm_step: call lbm_init first");
    if (c->unstable) return fail(c, LBM_ESTATE, "lbm_step: the state is unstable; re-initialise");
    StepArgs a{};
    a.f = c->f;
    a.qs = c->qs;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.nz = c->p.nz;
    a.px = c->px;
    a.zp = c->zp;
    a.nbx = c->nbx;
    a.nbz = c->nbz;
    div_magic((uint32_t)a.nbx, &a.m_nbx, &a.s_nbx);
    div_magic((uint32_t)a.nbz, &a.m_nbz, &a.s_nbz);
    a.j0 = 0;
    a.nrows = c->p.ny;
    div_magic((uint32_t)c->p.ny, &a.m_ny, &a.s_ny);
    a.ntiles = c->ntiles;
    a.xcd_run = c->xcd_run;
    a.bc_lo = c->p.bc_ylo;
    a.bc_hi = c->p.bc_yhi;
    a.tau0 = c->p.tau0;
    a.ksmag = 18.0 * std::sqrt(2.0) * c->p.c_smag;
    for (int d = 0; d < 3; ++d) {
        a.g[d] = c->p.g[d];
        a.u_wall[d] = c->p.u_wall[d];
        a.gf[d] = (float)a.g[d];
        a.u_wallf[d] = (float)a.u_wall[d];
    }
    a.cd = c->cd;
    a.tau0f = (float)a.tau0;
    a.ksmagf = (float)a.ksmag;
    a.cdf = (float)a.cd;
    a.lad = c->lad;
    a.fidx = c->fidx;
    a.ftab = c->ftab;
    a.ftabf = c->ftabf;
    a.mom = c->mom;
    a.imp = c->imp;
    a.dg = c->dg;
    a.stats = c->stats;
    a.mlp = c->mlp;
    a.mc = c->mc;
    int base_flags = FLAG_IMPULSE;
    if (c->vector_drag) base_flags |= FLAG_VECTOR_DRAG;
    if (c->p.g[1] == 0.0 && c->p.g[2] == 0.0 && !c->vector_drag) {
        base_flags |= FLAG_IMPULSE_X;
        if (c->fx) base_flags |= FLAG_FX;
    }
    if (c->xcd_remap) base_flags |= FLAG_XCD_REMAP;
    if (c->forest) base_flags |= FLAG_FOREST;
    if (c->streaming) base_flags |= FLAG_STREAMING;
    if (c->memorder) base_flags |= FLAG_MEMORDER;
    // arrays too large for buffer resources take 64-bit addresses
    // (LBMX_WIDE=1 forces the 64-bit path, for tests)
    if (pop_wide(c->p.storage, (unsigned long long)c->qs * c->elt) || c->force_wide)
        base_flags |= FLAG_WIDE;
    for (int64_t s = 0; s < nsteps; ++s) {
        a.parity = c->parity;
        a.seed = (uint32_t)(c->t * 0x9E3779B97F4A7C15ULL >> 32) ^ 0x5bd1e995u;
        a.flags = base_flags;
        if (s == nsteps - 1) a.flags |= FLAG_MOMENTS;
        const bool sample = c->stats_every > 0 && (c->t + 1) % c->stats_every == 0;
        if (sample) a.flags |= FLAG_STATS;
        // learned closure: the network runs on evaluating steps (and keeps
        // its nu_t when later steps reuse it); the steps between read nu_t
        const bool learned = c->closure == LBM_CLOSURE_MLP;
        const bool evaluate = learned && c->closure_lag == 0;
        if (evaluate) {
            a.flags |= FLAG_MLP;
            a.flags = c->mlp_remap ? (a.flags | FLAG_XCD_REMAP) : (a.flags & ~FLAG_XCD_REMAP);
            // the learned-closure kernel addresses the array through the two
            // array resources for every type (FP32 included)
            if (!pop_array_fits((unsigned long long)c->qs * c->elt)) a.flags |= FLAG_WIDE;
            if (c->closure_every > 1) a.flags |= FLAG_NUT_OUT;
            a.fb_slot = (int)(c->evals & 1);
        } else if (learned) {
            a.flags |= FLAG_NUT_IN;
        }
        hipError_t e = hipSuccess;
        // one launch over the rows j0 .. j0 + nrows - 1, whose tiles take the
        // records from tile 'off' on (the launches of a step fill them once)
        auto launch_rows = [&](StepArgs r, int j0, int nrows, long long off, bool mlp,
                               hipStream_t st, int grid_cap) {
            r.j0 = j0;
            r.nrows = nrows;
            div_magic((uint32_t)nrows, &r.m_ny, &r.s_ny);
            r.ntiles = c->nbx * c->nbz * nrows;
            r.imp = c->imp + 12 * off;
            r.dg = c->dg + 24 * off;
            if (!mlp) {
                r.flags &= ~FLAG_MLP;
                r.flags = (r.flags & ~FLAG_WIDE) | (base_flags & FLAG_WIDE);
                r.flags = c->xcd_remap ? (r.flags | FLAG_XCD_REMAP) : (r.flags & ~FLAG_XCD_REMAP);
                return launch_step(c->p.storage, r, c->bx, c->bz, st);
            }
            // the persistent grid depends on the kernel variant only: the
            // occupancy query runs once per variant and context
            const int v = ((r.flags & FLAG_FOREST) ? 1 : 0) | ((r.flags & FLAG_WIDE) ? 2 : 0) |
                          ((r.flags & FLAG_FX) ? 4 : 0);
            hipError_t e2 = hipSuccess;
            if (c->mlp_grid[v] == 0)
                e2 = mlp_launch_grid(c->p.storage, r.flags, c->ntiles, &c->mlp_grid[v]);
            if (e2 != hipSuccess) return e2;
            int grid = std::min(c->mlp_grid[v], r.ntiles);
            if (grid_cap > 0) grid = std::min(grid, grid_cap);
            return launch_step_mlp(c->p.storage, r, c->bx, c->bz, grid, st);
        };
        if (evaluate) {
            // Rows whose y/h lies outside the network's trained range fall
            // back to Smagorinsky in every cell: the plain step takes them
            // (bit for bit the learned kernel's fallback, at the plain step's
            // rate), the learned kernel the rows in between.  The test is the
            // kernel's own, in FP32.
            int ja = 0, jb = c->p.ny;
            if (c->mlp_split) {
                ja = c->p.ny;
                jb = 0;
                for (int j = 0; j < c->p.ny; ++j) {
                    const float yh = ((float)j + 0.5f) * c->mc.inv_h;
                    if (yh >= c->mc.lo[6] && yh <= c->mc.hi[6]) {
                        ja = std::min(ja, j);
                        jb = j + 1;
                    }
                }
                if (ja >= jb) {  // no row in range: one learned launch as usual
                    ja = 0;
                    jb = c->p.ny;
                }
            }
            const long long rows_tiles = (long long)c->nbx * c->nbz;
            // the plain rows on the second stream: the launches of one step
            // touch disjoint slots and records, and the next step waits for
            // both (the fork and join events)
            const bool overlap = c->mlp_overlap > 0 && (ja > 0 || jb < c->p.ny);
            hipStream_t ps = c->stream;
            int cap = 0;
            if (overlap) {
                if (!c->side) {  // set up once; kept only when every part succeeded
                    hipStream_t st = nullptr;
                    hipEvent_t ef = nullptr, ej = nullptr;
                    int ncu = 0;
                    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
                    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
                    if (e == hipSuccess) e = hipEventCreateWithFlags(&ef, hipEventDisableTiming);
                    if (e == hipSuccess) e = hipEventCreateWithFlags(&ej, hipEventDisableTiming);
                    if (e != hipSuccess) {
                        if (ej) (void)hipEventDestroy(ej);
                        if (ef) (void)hipEventDestroy(ef);
                        if (st) (void)hipStreamDestroy(st);
                        return hip_fail(c, e, "lbm_step: second stream");
                    }
                    c->side = st;
                    c->ev_fork = ef;
                    c->ev_join = ej;
                    c->ncu = ncu;
                }
                e = hipEventRecord(c->ev_fork, c->stream);
                if (e == hipSuccess) e = hipStreamWaitEvent(c->side, c->ev_fork, 0);
                if (e != hipSuccess) return hip_fail(c, e, "lbm_step: fork");
                cap = std::max(8, c->mlp_overlap * c->ncu / 8 * 8);
                ps = c->side;
            }
            e = launch_rows(a, ja, jb - ja, 0, true, c->stream, cap);
            if (e == hipSuccess && ja > 0)
                e = launch_rows(a, 0, ja, rows_tiles * (jb - ja), false, ps, 0);
            if (e == hipSuccess && jb < c->p.ny)
                e = launch_rows(a, jb, c->p.ny - jb, rows_tiles * jb, false, ps, 0);
            if (overlap) {  // joined after a failed launch too: no work left behind
                hipError_t ej = hipEventRecord(c->ev_join, c->side);
                if (ej == hipSuccess) ej = hipStreamWaitEvent(c->stream, c->ev_join, 0);
                if (e == hipSuccess) e = ej;
            }
            c->fb_rows_cells = (long long)(c->p.ny - (jb - ja)) * c->p.nx * c->p.nz;
        } else {
            e = launch_step(c->p.storage, a, c->bx, c->bz, c->stream);
        }
        if (e != hipSuccess) return hip_fail(c, e, "lbm_step: launch");
        if (evaluate) {
            c->last_fb_slot = a.fb_slot;
            c->evals += 1;
        }
        if (learned) c->closure_lag = (c->closure_lag + 1) % c->closure_every;
        c->parity ^= 1;
        c->t += 1;
        if (sample) c->stats_n += 1;
    }
    if (nsteps > 0) c->diag_fresh = true;
    return LBM_OK;
}

lbm_status lbm_moments(lbm_ctx *c, double *rho, double *u, double *nut, int32_t on_device,
                       lbm_diag *d) {
    if (!c) return LBM_EINVAL;
    if (!c->inited) return fail(c, LBM_ESTATE, "lbm_moments: call lbm_init first");
    const long long n = c->n;
    if (rho || u || nut) {
        if (on_device) {
            HIPCHK(c, launch_moments_out(c->p.storage, c->mom, rho, u, nut, (int)n, c->stream),
                   "lbm_moments: convert");
        } else if (c->celt == 8) {
            const double *m = static_cast<const double *>(c->mom);
            if (rho) HIPCHK(c, hipMemcpyAsync(rho, m, n * 8, hipMemcpyDeviceToHost, c->stream), "copy");
            if (u) HIPCHK(c, hipMemcpyAsync(u, m + n, 3 * n * 8, hipMemcpyDeviceToHost, c->stream), "copy");
            if (nut) HIPCHK(c, hipMemcpyAsync(nut, m + 4 * n, n * 8, hipMemcpyDeviceToHost, c->stream), "copy");
        } else {
            std::vector<float> h((size_t)5 * n);
            HIPCHK(c, hipMemcpyAsync(h.data(), c->mom, (size_t)5 * n * 4, hipMemcpyDeviceToHost,
                                     c->stream), "lbm_moments: copy");
            HIPCHK(c, hipStreamSynchronize(c->stream), "lbm_moments: sync");
            for (long long x = 0; x < n; ++x) {
                if (rho) rho[x] = h[x];
                if (u) {
                    u[x] = h[n + x];
                    u[n + x] = h[2 * n + x];
                    u[2 * n + x] = h[3 * n + x];
                }
                if (nut) nut[x] = h[4 * n + x];
            }
        }
    }
    // FP64 diagnostics: from the per-wavefront records of the last step, or
    // from the moment planes when no step ran since lbm_init / lbm_set_f
    double out[9] = {0};
    double *dout = c->red + kDiagRedDoubles;
    HIPCHK(c, launch_diag(c->p.storage, c->mom, (int)n, c->diag_fresh ? c->dg : nullptr, c->imp,
                          4 * c->ntiles, c->red, dout, c->stream), "lbm_moments: reduce");
    HIPCHK(c, hipMemcpyAsync(out, dout, sizeof(out), hipMemcpyDeviceToHost, c->stream),
           "lbm_moments: copy diag");
    HIPCHK(c, hipStreamSynchronize(c->stream), "lbm_moments: sync");
    int64_t fb = 0;
    if (c->closure == LBM_CLOSURE_MLP) {
        lbm_status s = mlp_fallback_count(c->mlp, c->last_fb_slot, &fb, c->stream);
        if (s != LBM_OK) return fail(c, s, "lbm_moments: fallback count");
        fb += c->fb_rows_cells;  // the rows outside the network's range
    }
    if (d) {
        d->mass = out[0];
        d->mom[0] = out[1];
        d->mom[1] = out[2];
        d->mom[2] = out[3];
        d->impulse[0] = out[4];
        d->impulse[1] = out[5];
        d->impulse[2] = out[6];
        d->max_u = out[7];
        d->t = c->t;
        d->nonfinite = (int64_t)out[8];
        d->mlp_fallback = fb;
    }
    if (out[8] > 0 || out[7] > 0.35 || !std::isfinite(out[7])) {
        c->unstable = true;
        return fail(c, LBM_EUNSTABLE, "lbm_moments: non-finite values or max |u| > 0.35");
    }
    return LBM_OK;
}

lbm_status lbm_stats(lbm_ctx *c, int32_t op, int32_t every, double *prof, int64_t *nsamples) {
    if (!c) return LBM_EINVAL;
    if (op == 0) {
        lbm_status s = reset_accumulators(c);
        if (s != LBM_OK) return s;
    } else if (op == 1) {
        if (every < 0) return fail(c, LBM_EINVAL, "lbm_stats: every must be >= 0");
        c->stats_every = every;
    } else if (op == 2) {
        if (!prof) return fail(c, LBM_EINVAL, "lbm_stats: NULL prof");
        std::vector<double> h((size_t)c->p.ny * 10);
        HIPCHK(c, launch_stats_read(c->stats, c->p.ny, c->tpp, c->prof, c->stream),
               "lbm_stats: reduce");
        HIPCHK(c, hipMemcpyAsync(h.data(), c->prof, h.size() * 8, hipMemcpyDeviceToHost,
                                 c->stream), "lbm_stats: copy");
        HIPCHK(c, hipStreamSynchronize(c->stream), "lbm_stats: sync");
        const double denom = (double)c->stats_n * c->p.nx * c->p.nz;
        for (size_t k = 0; k < h.size(); ++k) prof[k] = c->stats_n ? h[k] / denom : 0.0;
    } else {
        return fail(c, LBM_EINVAL, "lbm_stats: op must be 0 (reset), 1 (enable) or 2 (read)");
    }
    if (nsamples) *nsamples = c->stats_n;
    return LBM_OK;
}

lbm_status lbm_set_f(lbm_ctx *c, const double *fin, int32_t on_device) {
    if (!c) return LBM_EINVAL;
    if (!fin) return fail(c, LBM_EINVAL, "lbm_set_f: NULL f");
    const long long n = c->n;
    const double *src = fin;
    double *tmp = nullptr;
    if (!on_device) {
        HIPCHK(c, hipMallocAsync(reinterpret_cast<void **>(&tmp), (size_t)NQ * n * 8, c->stream),
               "lbm_set_f: staging");
        HIPCHK(c, hipMemcpyAsync(tmp, fin, (size_t)NQ * n * 8, hipMemcpyHostToDevice, c->stream),
               "lbm_set_f: copy");
        src = tmp;
    }
    // stored where the next step reads it: the AA parity of the context
    // continues (before the first step after lbm_init it is 0)
    HIPCHK(c, launch_set_f(c->p.storage, c->f, c->qs, src, c->p.nx, c->px, c->zp, c->p.ny, c->p.nz, c->parity,
                           c->p.bc_ylo, c->p.bc_yhi, c->stream), "lbm_set_f: kernel");
    if (tmp) HIPCHK(c, hipFreeAsync(tmp, c->stream), "lbm_set_f: free staging");
    HIPCHK(c, hipStreamSynchronize(c->stream), "lbm_set_f: sync");
    c->inited = true;
    c->diag_fresh = false;
    c->closure_lag = 0;  // the next step evaluates the learned closure
    c->unstable = false;
    return LBM_OK;
}

lbm_status lbm_get_f(lbm_ctx *c, double *fout, int32_t on_device) {
    if (!c) return LBM_EINVAL;
    if (!fout) return fail(c, LBM_EINVAL, "lbm_get_f: NULL f");
    if (!c->inited) return fail(c, LBM_ESTATE, "lbm_get_f: call lbm_init first");
    const long long n = c->n;
    double *dst = fout;
    double *tmp = nullptr;
    if (!on_device) {
        HIPCHK(c, hipMallocAsync(reinterpret_cast<void **>(&tmp), (size_t)NQ * n * 8, c->stream),
               "lbm_get_f: staging");
        dst = tmp;
    }
    HIPCHK(c, launch_get_f(c->p.storage, c->f, c->qs, dst, c->p.nx, c->px, c->zp, c->p.ny, c->p.nz, c->parity,
                           c->p.bc_ylo, c->p.bc_yhi, c->stream), "lbm_get_f: kernel");
    if (tmp) {
        HIPCHK(c, hipMemcpyAsync(fout, tmp, (size_t)NQ * n * 8, hipMemcpyDeviceToHost, c->stream),
               "lbm_get_f: copy");
        HIPCHK(c, hipFreeAsync(tmp, c->stream), "lbm_get_f: free staging");
    }
    HIPCHK(c, hipStreamSynchronize(c->stream), "lbm_get_f: sync");
    return LBM_OK;
}

}  // extern "C"

namespace {

// Arguments shared by lbm_closure_samples and its allocation-free variant;
// *ncc receives the coarse cell count.
lbm_status closure_samples_args(lbm_ctx *c, const char *who, double tau0_coarse, double canopy_h,
                                const double *lad_coarse, const float *X, const float *y,
                                int64_t nc, long long *ncc) {
    if (!c) return LBM_EINVAL;
    if (!c->inited) return fail(c, LBM_ESTATE, std::string(who) + ": call lbm_init first");
    const int nx = c->p.nx, ny = c->p.ny, nz = c->p.nz;
    if ((nx | ny | nz) & 1) return fail(c, LBM_EINVAL, std::string(who) + ": dimensions must be even");
    if (!X || !y || !lad_coarse) return fail(c, LBM_EINVAL, std::string(who) + ": NULL pointer");
    *ncc = (long long)(nx / 2) * (ny / 2) * (nz / 2);
    if (nc != *ncc)
        return fail(c, LBM_EINVAL, std::string(who) + ": nc must be (nx/2)(ny/2)(nz/2)");
    if (!(canopy_h > 0.0) || !(tau0_coarse > 0.5))
        return fail(c, LBM_EINVAL, std::string(who) + ": canopy_h > 0 and tau0_coarse > 0.5");
    return LBM_OK;
}

// Work area of lbm_closure_samples_noalloc: the coarse LAD (FP64, at most
// LBM_NOALLOC_MAX_LAD rows) followed by the filtered velocity and subfilter
// stress (9 FP32 per coarse cell, at most LBM_NOALLOC_MAX_COARSE cells).
// Every device the library runs on holds its own copy for the life of the
// process.  Nothing in it needs clearing: every call writes all of the part
// it reads.
constexpr size_t kNoallocLadBytes = (size_t)LBM_NOALLOC_MAX_LAD * 8;
constexpr size_t kNoallocBytes = kNoallocLadBytes + (size_t)9 * LBM_NOALLOC_MAX_COARSE * 4;
static_assert(kNoallocLadBytes % 256 == 0, "work part 256-byte aligned");
__device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, taken once per device with that
// device current (host code never passes the symbol itself to a kernel).
hipError_t scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        hipError_t e2 = prev != dev ? hipSetDevice(prev) : hipSuccess;
        if (e != hipSuccess) return e;
        if (e2 != hipSuccess) return e2;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

lbm_status lbm_closure_samples(lbm_ctx *c, double tau0_coarse, double canopy_h,
                               const double *lad_coarse, float *X, float *y, int64_t nc) {
    long long ncc = 0;
    const lbm_status st = closure_samples_args(c, "lbm_closure_samples", tau0_coarse, canopy_h,
                                               lad_coarse, X, y, nc, &ncc);
    if (st != LBM_OK) return st;
    const int nx = c->p.nx, ny = c->p.ny, nz = c->p.nz;
    float *work = nullptr;
    double *lad_d = nullptr;
    HIPCHK(c, hipMallocAsync(reinterpret_cast<void **>(&work), (size_t)9 * ncc * 4, c->stream),
           "lbm_closure_samples: work");
    HIPCHK(c, hipMallocAsync(reinterpret_cast<void **>(&lad_d), (size_t)(ny / 2) * 8, c->stream),
           "lbm_closure_samples: lad");
    HIPCHK(c, hipMemcpyAsync(lad_d, lad_coarse, (size_t)(ny / 2) * 8, hipMemcpyHostToDevice, c->stream),
           "lbm_closure_samples: copy lad");
    HIPCHK(c, launch_closure_samples(c->p.storage, c->mom, nx, ny, nz, work, tau0_coarse,
                                     1.0 / canopy_h, lad_d, X, y, c->stream),
           "lbm_closure_samples: kernels");
    HIPCHK(c, hipFreeAsync(work, c->stream), "lbm_closure_samples: free");
    HIPCHK(c, hipFreeAsync(lad_d, c->stream), "lbm_closure_samples: free");
    HIPCHK(c, hipStreamSynchronize(c->stream), "lbm_closure_samples: sync");
    return LBM_OK;
}

lbm_status lbm_closure_samples_noalloc(lbm_ctx *c, double tau0_coarse, double canopy_h,
                                       const double *lad_coarse, float *X, float *y, int64_t nc) {
    long long ncc = 0;
    const lbm_status st = closure_samples_args(c, "lbm_closure_samples_noalloc", tau0_coarse,
                                               canopy_h, lad_coarse, X, y, nc, &ncc);
    if (st != LBM_OK) return st;
    const int nx = c->p.nx, ny = c->p.ny, nz = c->p.nz;
    if (ncc > LBM_NOALLOC_MAX_COARSE || ny / 2 > LBM_NOALLOC_MAX_LAD)
        return fail(c, LBM_EINVAL,
                    "lbm_closure_samples_noalloc: at most " +
                        std::to_string(LBM_NOALLOC_MAX_COARSE) + " coarse cells and " +
                        std::to_string(LBM_NOALLOC_MAX_LAD) + " coarse rows (got " +
                        std::to_string(ncc) + " cells, " + std::to_string(ny / 2) + " rows)");
    void *base = nullptr;
    HIPCHK(c, scratch_address(c->device, &base), "lbm_closure_samples_noalloc: scratch address");
    double *lad_d = static_cast<double *>(base);
    float *work = reinterpret_cast<float *>(static_cast<unsigned char *>(base) + kNoallocLadBytes);
    HIPCHK(c, hipMemcpyAsync(lad_d, lad_coarse, (size_t)(ny / 2) * 8, hipMemcpyHostToDevice, c->stream),
           "lbm_closure_samples_noalloc: copy lad");
    HIPCHK(c, launch_closure_samples(c->p.storage, c->mom, nx, ny, nz, work, tau0_coarse,
                                     1.0 / canopy_h, lad_d, X, y, c->stream),
           "lbm_closure_samples_noalloc: kernels");
    return LBM_OK;
}

lbm_status lbm_lad_lalic(double h, double ym, double afm, double lai, int32_t ny, double *out) {
    if (!out || ny < 1 || !(h > 0.0) || !(ym >= 0.0) || !(ym < h) || !std::isfinite(h))
        return LBM_EINVAL;
    double sum = 0.0;
    for (int j = 0; j < ny; ++j) {
        const double y = j + 0.5;
        double a = 0.0;
        if (y < h) {
            const double nexp = y < ym ? 6.0 : 0.5;
            const double r = (h - ym) / (h - y);
            a = std::exp(nexp * (std::log(r) + 1.0 - r));
        }
        out[j] = a;
        sum += a;
    }
    double scale = afm;
    if (lai > 0.0) {
        if (!(sum > 0.0)) return LBM_EINVAL;
        scale = lai / sum;
    }
    for (int j = 0; j < ny; ++j) out[j] *= scale;
    return LBM_OK;
}

}  // extern "C"
