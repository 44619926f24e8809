// lbm_device.h -- internal definitions shared by the HIP translation units of
// the fused lattice-Boltzmann LES canopy step (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace lbmx {

constexpr int NQ = 19;

// D3Q19 in the interface direction order: rest; +x,-x,+y,-y,+z,-z; edge
// vectors in opposite pairs (q odd, q+1).  Weights 1/3, 1/18, 1/36.
constexpr int CX[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }

// direction with the y component of c_q reversed (specular reflection off a
// y = const plane)
constexpr int mir(int q) {
    for (int p = 0; p < NQ; ++p)
        if (CX[p] == CX[q] && CY[p] == -CY[q] && CZ[p] == CZ[q]) return p;
    return -1;
}

constexpr double weight(int q) {
    return q == 0 ? 1.0 / 3.0 : (q < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}

enum { BC_PERIODIC = 0, BC_BOUNCEBACK = 1, BC_FREESLIP = 2, BC_EQUILIBRIUM = 3 };
enum { ST_F64 = 0, ST_F32 = 1, ST_F16S = 2, ST_BF16S = 3, ST_BF16SR = 4 };

// step flags
enum : int {
    FLAG_MOMENTS = 1,      // write rho, u, nu_t of this collision
    FLAG_STATS = 2,        // accumulate the plane statistics of this step
    FLAG_VECTOR_DRAG = 4,  // canopy drag on all three components
    FLAG_XCD_REMAP = 8,    // keep consecutive tiles on one XCD
    FLAG_IMPULSE = 16,     // accumulate the body-force impulse
    FLAG_MLP = 32,         // learned closure
    FLAG_FOREST = 64,      // per-cell LAD: ftab[fidx[cell]] instead of lad[row]
    FLAG_NUT_IN = 128,     // nu_t read from the moments' nu_t plane (learned closure reused)
    FLAG_NUT_OUT = 256,    // nu_t written to that plane on every step of the launch
    FLAG_WIDE = 512,       // the population array has 2^32 bytes or more
    FLAG_IMPULSE_X = 1024, // g_y = g_z = 0 and x-only drag: the y, z forces are 0
    FLAG_STREAMING = 2048, // rows start on cache lines: aligned accesses are non-temporal
    FLAG_MEMORDER = 4096,  // tiles numbered in memory order (rows not streaming, or planes above 96 MiB)
    FLAG_FX = 8192         // driving force and drag along x only: F_y = F_z = 0 (VAR_FX)
};

// Compile-time variants of the step (a bit set; chosen at launch from the flags)
enum : int {
    VAR_FOREST = 1,        // FLAG_FOREST
    VAR_NUT_IN = 2,        // FLAG_NUT_IN
    VAR_WIDE = 4,          // FLAG_WIDE: population arrays of 4 GiB or more (64-bit addresses)
    VAR_STREAM = 8,        // FLAG_STREAMING (plain step kernel)
    VAR_FX = 16            // FLAG_FX: the y and z forces are zero at compile time
};

// Population loads and stores of the auxiliary kernels (plain cached accesses).
template <class T> __device__ __forceinline__ T pop_ld(const T *p) { return *p; }
template <class T> __device__ __forceinline__ void pop_st(T *p, T v) { *p = v; }

// Cache policy of the step kernel's population accesses: 0 = default, 2 =
// non-temporal (streaming: the lines are not kept for reuse).  A step
// touches every population once (2.5 GB per step at 512x128x256 in FP32, far
// more than the caches).  With FLAG_STREAMING (set when a row of the grid is
// a whole number of 128-byte lines) the accesses that cover whole aligned
// rows stream: every access of the local step of the AA pattern, and the
// neighbour step's planes with c_x = 0.  The neighbour step's planes with
// c_x != 0 are shifted by one cell: the lines at a wavefront's ends are
// shared with the adjacent wavefront, which finds them in L2 only with the
// default policy.  Rows that are not whole lines share their end lines with
// the next row: they keep the default policy (streaming them was measured
// slower in either tile order).
template <bool STREAM> constexpr int policy_local() { return STREAM ? 2 : 0; }
template <bool STREAM> constexpr int policy_neigh(int q) { return STREAM && CX[q] == 0 ? 2 : 0; }

// Reciprocal and square root in the arithmetic type of a step.  FP32 uses
// the hardware instructions (v_rcp_f32, v_sqrt_f32: within 1 ulp of the
// correctly rounded result, one instruction each instead of a refinement
// sequence); FP64 keeps the correctly rounded operations.
template <class C> __device__ __forceinline__ C arith_rcp(C x) {
    if constexpr (std::is_same_v<C, float>)
        return __builtin_amdgcn_rcpf(x);
    else
        return C(1) / x;
}
template <class C> __device__ __forceinline__ C arith_sqrt(C x) {
    if constexpr (std::is_same_v<C, float>)
        return __builtin_amdgcn_sqrtf(x);
    else
        return sqrt(x);
}

// Storage codecs: T is the element type in HBM, C the arithmetic type.
// Stored values are shifted populations f_q - w_q.  st() takes 32 random bits
// (used only by the stochastically rounded type).
template <int ST> struct Codec;
template <> struct Codec<ST_F64> {
    using T = double;
    using C = double;
    static __device__ __forceinline__ C dec(T t) { return t; }
    static __device__ __forceinline__ T enc(C v, uint32_t = 0) { return v; }
    static __device__ __forceinline__ C ld(const T *p) { return pop_ld(p); }
    static __device__ __forceinline__ void st(T *p, C v, uint32_t = 0) { pop_st(p, v); }
};
template <> struct Codec<ST_F32> {
    using T = float;
    using C = float;
    static __device__ __forceinline__ C dec(T t) { return t; }
    static __device__ __forceinline__ T enc(C v, uint32_t = 0) { return v; }
    static __device__ __forceinline__ C ld(const T *p) { return pop_ld(p); }
    static __device__ __forceinline__ void st(T *p, C v, uint32_t = 0) { pop_st(p, v); }
};
template <> struct Codec<ST_F16S> {
    using T = _Float16;
    using C = float;
    static __device__ __forceinline__ C dec(T t) { return (float)t; }
    static __device__ __forceinline__ T enc(C v, uint32_t = 0) { return (_Float16)v; }  // nearest even
    static __device__ __forceinline__ C ld(const T *p) { return dec(pop_ld(p)); }
    static __device__ __forceinline__ void st(T *p, C v, uint32_t = 0) { pop_st(p, enc(v)); }
};
template <> struct Codec<ST_BF16S> {
    using T = __bf16;
    using C = float;
    static __device__ __forceinline__ C dec(T t) { return (float)t; }
    static __device__ __forceinline__ T enc(C v, uint32_t = 0) { return (__bf16)v; }  // nearest even
    static __device__ __forceinline__ C ld(const T *p) { return dec(pop_ld(p)); }
    static __device__ __forceinline__ void st(T *p, C v, uint32_t = 0) { pop_st(p, enc(v)); }
};
// BF16 with stochastic rounding: adding 16 uniform random bits below the kept
// mantissa and truncating rounds up with probability equal to the dropped
// fraction, so the rounding error has zero mean (finite values).
template <> struct Codec<ST_BF16SR> {
    using T = __bf16;
    using C = float;
    static __device__ __forceinline__ C dec(T t) { return (float)t; }
    static __device__ __forceinline__ T enc(C v, uint32_t r) {
        const uint32_t b = __float_as_uint(v) + (r & 0xFFFFu);
        return __builtin_bit_cast(__bf16, (unsigned short)(b >> 16));
    }
    static __device__ __forceinline__ C ld(const T *p) { return dec(pop_ld(p)); }
    static __device__ __forceinline__ void st(T *p, C v, uint32_t r) { pop_st(p, enc(v, r)); }
};

// Population access of the step kernel, by direction plane q and cell index.
// Three forms, chosen per storage type and size (measured on MI355X):
// PopArray: two buffer resources for the population array (planes 0-9 and
// 10-18), built once in scalar registers; the plane enters as the scalar
// offset (q - first plane of its half) * plane bytes and the cell as a 32-bit
// byte offset, so an access costs no scalar work beyond the plane offset.
// Needs 10 planes below 2^32 bytes.  Used for the 16-bit and FP64 storage
// types (16-bit: 5 % faster than PopPlanes).
// PopPlanes: one buffer resource per plane (base f + q qs, the plane's size)
// and a 32-bit byte offset per cell.  Needs plane bytes below 2^32.  Used for
// FP32 (2 % faster than PopArray there).
// PopGlobal: plain 64-bit addresses, for larger arrays.
constexpr int kArraySplit = 10;  // PopArray: planes 0-9 and 10-18, one resource each
template <int ST> struct PopArray {
    using CD = Codec<ST>;
    using T = typename CD::T;
    using C = typename CD::C;
    static constexpr int kSplit = kArraySplit;
    __amdgpu_buffer_rsrc_t r0, r1;
    uint32_t plane;  // bytes per plane (the plane stride)
    __device__ __forceinline__ void init(T *f, long long qs) {
        plane = (uint32_t)(qs * (long long)sizeof(T));
        r0 = __builtin_amdgcn_make_buffer_rsrc(f, 0, (int)(plane * (uint32_t)kSplit), 0x00020000);
        r1 = __builtin_amdgcn_make_buffer_rsrc(f + kSplit * qs, 0,
                                               (int)(plane * (uint32_t)(NQ - kSplit)), 0x00020000);
    }
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t rs(int q) const { return q < kSplit ? r0 : r1; }
    __device__ __forceinline__ uint32_t so(int q) const {
        return (uint32_t)(q < kSplit ? q : q - kSplit) * plane;
    }
};
template <int ST> struct PopPlanes {
    using CD = Codec<ST>;
    using T = typename CD::T;
    using C = typename CD::C;
    T *f;
    long long qs;
    uint32_t bytes;  // plane size in bytes
    __device__ __forceinline__ void init(T *f_, long long qs_) {
        f = f_;
        qs = qs_;
        bytes = (uint32_t)(qs * (long long)sizeof(T));
    }
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t rs(int q) const {
        return __builtin_amdgcn_make_buffer_rsrc(f + q * qs, 0, (int)bytes, 0x00020000);
    }
    __device__ __forceinline__ uint32_t so(int) const { return 0u; }
};
// loads and stores through a buffer resource (PopArray or PopPlanes)
template <class Base> struct PopBuf : Base {
    using CD = typename Base::CD;
    using T = typename CD::T;
    using C = typename CD::C;
    template <int AUX = 0> __device__ __forceinline__ C ld(int q, int x) const {
        const uint32_t off = (uint32_t)x * (uint32_t)sizeof(T);
        if constexpr (sizeof(T) == 8)
            return CD::dec(__builtin_bit_cast(
                T, __builtin_amdgcn_raw_buffer_load_b64(this->rs(q), off, this->so(q), AUX)));
        else if constexpr (sizeof(T) == 4)
            return CD::dec(__builtin_bit_cast(
                T, __builtin_amdgcn_raw_buffer_load_b32(this->rs(q), off, this->so(q), AUX)));
        else
            return CD::dec(__builtin_bit_cast(
                T, __builtin_amdgcn_raw_buffer_load_b16(this->rs(q), off, this->so(q), AUX)));
    }
    template <int AUX = 0> __device__ __forceinline__ void st(int q, int x, C v, uint32_t r) const {
        const uint32_t off = (uint32_t)x * (uint32_t)sizeof(T);
        const T t = CD::enc(v, r);
        if constexpr (sizeof(T) == 8) {
            using R = decltype(__builtin_amdgcn_raw_buffer_load_b64(this->rs(q), 0, 0, 0));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(R, t), this->rs(q), off,
                                                  this->so(q), AUX);
        } else if constexpr (sizeof(T) == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, t), this->rs(q), off,
                                                  this->so(q), AUX);
        } else {
            __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, t), this->rs(q),
                                                  off, this->so(q), AUX);
        }
    }
};
// the buffer form of a storage type, and whether a population array of
// 'plane_bytes' per plane needs 64-bit addresses instead
constexpr bool pop_planes(int st) { return st == ST_F32; }
template <int ST>
using PopBufOf = PopBuf<std::conditional_t<pop_planes(ST), PopPlanes<ST>, PopArray<ST>>>;
constexpr bool pop_array_fits(unsigned long long plane_bytes) {
    return plane_bytes * kArraySplit < (1ULL << 32);
}
constexpr bool pop_wide(int st, unsigned long long plane_bytes) {
    return pop_planes(st) ? plane_bytes >= (1ULL << 32) : !pop_array_fits(plane_bytes);
}

template <int ST> struct PopGlobal {
    using CD = Codec<ST>;
    using T = typename CD::T;
    using C = typename CD::C;
    T *f;
    long long qs;
    __device__ __forceinline__ void init(T *f_, long long qs_) {
        f = f_;
        qs = qs_;
    }
    template <int AUX = 0> __device__ __forceinline__ C ld(int q, int x) const {
        const T *p = f + q * qs + x;
        if constexpr (AUX != 0)
            return CD::dec(__builtin_nontemporal_load(p));
        else
            return CD::dec(*p);
    }
    template <int AUX = 0> __device__ __forceinline__ void st(int q, int x, C v, uint32_t r) const {
        T *p = f + q * qs + x;
        if constexpr (AUX != 0)
            __builtin_nontemporal_store(CD::enc(v, r), p);
        else
            *p = CD::enc(v, r);
    }
};

// 32-bit integer hash for the rounding bits: the xorshift-multiply finaliser
// with the shifts and multipliers of C. Wellons' "lowbias32" (published
// 2018 with his hash-prospector search, public domain)
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// storage handled by the auxiliary (init/import/export) kernels: the
// stochastically rounded type is read and written there like BF16S
constexpr int aux_storage(int st) { return st == ST_BF16SR ? ST_BF16S : st; }

// entries of the per-cell forest LAD table (16-bit index; entry 0 = no forest)
constexpr int kForestTable = 65536;

// Scalars of the learned closure that every cell reads: the standardisation
// z = x zs + zo (zs = 1/std, zo = -mean/std), the trained range [lo, hi] of
// the raw features, 1/h, the output scale and the output bias.  Passed in the
// step's kernel arguments; the learned-closure kernel stages them in LDS.
struct MlpConst {
    float zs[9], zo[9], lo[9], hi[9];
    float inv_h, scale, b3;
};

// Arguments of one fused step launch (passed by value as kernel arguments).
struct StepArgs {
    void *f;          // population buffer, q-plane stride qs elements
    long long qs;
    int nx, ny, nz;
    int px;           // population row pitch (cells, >= nx)
    int zp;           // population z-layer pitch (cells, >= px ny): cell (i,j,k) at k zp + j px + i
    int nbx, nbz;     // tiles per row (x) and per column (z); tile = BX x 1 x BZ cells
    int j0, nrows;    // the launch covers rows j0 .. j0 + nrows - 1 (all: 0, ny)
    // division by nbx, nbz and nrows as multiply and shift (div_magic)
    uint32_t m_nbx, m_nbz, m_ny;
    int s_nbx, s_nbz, s_ny;
    int ntiles;       // nbx * nbz * nrows = grid size
    int xcd_run;      // FLAG_XCD_REMAP: 0 = one contiguous range per XCD, else runs of this many tiles
    int parity;       // 0: neighbour step, 1: local step (in-place AA pattern)
    int bc_lo, bc_hi;
    int flags;
    int fb_slot;      // learned closure: fallback counter slot of this evaluation (0/1)
    uint32_t seed;    // stochastic rounding: hash of (seed, step, cell, direction)
    double tau0;      // molecular relaxation time
    double ksmag;     // 18 sqrt(2) C_smag
    double g[3];      // driving acceleration
    double u_wall[3]; // velocity of a forced-equilibrium boundary (density 1)
    double cd;        // canopy drag coefficient
    // the same scalars in FP32 (the arithmetic type of every storage but F64)
    float gf[3], u_wallf[3], tau0f, ksmagf, cdf;
    const double *lad;  // [ny]
    const uint16_t *fidx;  // [nz][ny][nx] forest table index per cell (FLAG_FOREST)
    const double *ftab;    // LAD of each forest table entry; entry 0 is 0
    const float *ftabf;    // the same in FP32 (FP32 arithmetic)
    void *mom;        // moments in the arithmetic type: rho, ux, uy, uz, nu_t planes of N
    double *imp;      // [ntiles][4][3] body-force impulse accumulators (per wavefront; this
                      // launch's share when a step is split over row ranges)
    double *dg;       // [ntiles][4][6] diagnostics of the last FLAG_MOMENTS step (per
                      // wavefront; likewise)
    double *stats;    // [ny][nbx*nbz][10] statistics accumulators
    const void *mlp;  // learned closure parameters on the device
    MlpConst mc;      // learned closure scalars (FLAG_MLP)
};

// compile-time loop
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F> __device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Blocks are handed to the 8 XCDs round robin (block b runs on XCD b % 8).
// Remap so that XCD x processes one contiguous range of tiles: tiles that
// share cache lines (x neighbours) then meet in the same L2.  A bijection
// of [0, n).
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = b & 7, local = b >> 3;
    return x * q + (x < r ? x : r) + local;
}

// The same with runs of c consecutive tiles: XCD x takes the runs x, x + 8,
// x + 16, ... of the first n - n % (8 c) tiles, in order; the tiles after
// them keep their block (a bijection of [0, n)).
__device__ __forceinline__ int xcd_remap_runs(int b, int n, int c) {
    const int full = n - n % (8 * c);
    if (b >= full) return b;
    const int x = b & 7, local = b >> 3;
    const int run = local / c;
    return (run * 8 + x) * c + (local - run * c);
}

// Division of 0 <= n < 2^31 by a constant d >= 1 as n * m >> s (Granlund and
// Montgomery, "Division by invariant integers using multiplication", 1994,
// Thm. 4.2 with N = 31): l = ceil(log2 d), m = ceil(2^(31+l) / d) < 2^32.
inline void div_magic(uint32_t d, uint32_t *m, int *s) {
    int l = 0;
    while ((1ULL << l) < d) ++l;
    *s = 31 + l;
    *m = (uint32_t)(((1ULL << (31 + l)) + d - 1) / d);
}
__device__ __forceinline__ uint32_t div_by(uint32_t n, uint32_t m, int s) {
    return (uint32_t)(((unsigned long long)n * m) >> s);
}

// Launchers (defined in lbm_kernels.hip).
hipError_t launch_step(int storage, const StepArgs &a, int bx, int bz, hipStream_t s);
// population arrays: rows of pitch px >= nx cells, z-layers of pitch zp >= px ny
// cells (cell (i,j,k) at k zp + j px + i)
hipError_t launch_init(int storage, void *f, long long qs, int nx, int px, int ny, int zp,
                       void *mom, const double *rho, const double *u, int n, hipStream_t s);
// populations [19][N] into the slots the next step of the given AA parity reads
hipError_t launch_set_f(int storage, void *f, long long qs, const double *fin, int nx, int px,
                        int zp, int ny, int nz, int parity, int bc_lo, int bc_hi, hipStream_t s);
hipError_t launch_get_f(int storage, const void *f, long long qs, double *fout, int nx, int px,
                        int zp, int ny, int nz, int parity, int bc_lo, int bc_hi, hipStream_t s);  // EQ stores like BB
hipError_t launch_moments_out(int storage, const void *mom, double *rho, double *u,
                              double *nut, int n, hipStream_t s);
// FP64 diagnostics into out[9] (mass, mom[3], impulse[3], max|u|, nonfinite):
// from the per-wavefront records dg and imp (nrec each), or, with dg null,
// mass to non-finite count from the moment planes.  red: scratch of
// kDiagRedDoubles doubles.
constexpr int kDiagPlaneBlocks = 1024, kDiagRecordBlocks = 512;
constexpr int kDiagRedDoubles = kDiagPlaneBlocks * 6 + kDiagRecordBlocks * 9;
hipError_t launch_diag(int storage, const void *mom, int n, const double *dg, const double *imp,
                       int nrec, double *red, double *out, hipStream_t s);
hipError_t launch_stats_read(const double *stats, int ny, int tpp, double *prof,
                             hipStream_t s);
hipError_t launch_fill(double *p, double v, size_t n, hipStream_t s);
// closure_data.hip: work holds 9 planes of (nx/2)(ny/2)(nz/2) floats
hipError_t launch_closure_samples(int storage, const void *mom, int nx, int ny, int nz,
                                  float *work, double tau0_coarse, double inv_h,
                                  const double *lad_coarse, float *X, float *Y, hipStream_t s);

}  // namespace lbmx
