// mlp_closure.h -- device side of the learned eddy-viscosity closure
// (internal).  A 9-64-64-1 network on the matrix cores (layer 1 BF16, layer 2
// FP16 operands, FP32 accumulation), evaluated for the 64 cells of a
// wavefront at once; the activations are computed in packed FP16.
//
// Formulation: activations are kept transposed (units x cells), so that one
// 16x16 MFMA output tile (lane l holds rows 4*(l/16)+r, r = 0..3, of column
// l%16) is directly the B operand of the next 16x16x32 MFMA (lane l holds
// rows 8*(l/16)+t, t = 0..7, of column l%16) once the k index is permuted the
// same way in the weights: no data moves between lanes from layer to layer.
//   layer 1: mfma 16x16x16 bf16, A = [W1 | b1_hi b1_lo | 0] (16 units x 16 k),
//            B = [z0..z8, 1, 1, 0..] of 16 cells
//   layer 2: mfma 16x16x32 f16 (two k steps), A = W2 (FP16) with permuted
//            k, C initialised with b2 (the inputs are gelu(h1), FP16)
//   output : mfma 16x16x32 f16 (two k steps), A = w3 in every row (permuted
//            k), B = gelu(h2), C initialised with b3: every row of the
//            result holds o of its column
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmx {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef short short4v __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 9, kMlpH1 = 64, kMlpH2 = 64;
constexpr int kMlpParams = kMlpH1 * kMlpIn + kMlpH1 + kMlpH2 * kMlpH1 + kMlpH2 + kMlpH2 + 1;

// Packed device parameters (written by mlp_pack_blob on the host).  The
// standardisation, range and output scalars also travel in the step's kernel
// arguments (MlpConst), where the kernel reads them with scalar loads.
struct MlpParams {
    float mean[12], istd[12], lo[12], hi[12];  // raw-feature standardisation and range
    float scale, inv_h, b3, pad0;
    short4v w1f[4][64];      // layer-1 A fragments [unit tile][lane]
    half8 w2f[4][2][64];     // layer-2 A fragments (FP16) [unit tile][k step][lane]
    floatx4 b2f[4][4];       // layer-2 bias in output layout [unit tile][lane quarter]
    half8 w3a[2][4];         // output layer A fragments (w3 in every row) [k step][lane quarter]
    unsigned long long fallback[2];  // cells that fell back, per step parity
};

// input unit of layer 2 that k slot (k step ks, lane quarter h, element t)
// of the B operand holds: the layer-1 output tiles 2ks and 2ks+1 side by side
__host__ __device__ constexpr int mlp_l2_unit_in(int ks, int h, int t) {
    return 32 * ks + (t < 4 ? 4 * h + t : 16 + 4 * h + (t - 4));
}

// per-lane weight fragments held in registers for the life of a wave; the
// layer-2 fragments (8 KB per block) live in LDS and are read per MFMA
struct MlpFrag {
    short4v w1[4];
    floatx4 b2[4];
    half8 w3[2];
    const half8 *w2;  // LDS copy of MlpParams::w2f, [unit tile][k step][lane]
};

__device__ __forceinline__ MlpFrag mlp_load_frag(const MlpParams *p, int lane,
                                                 const half8 *w2_lds) {
    MlpFrag f;
    const int h = lane >> 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        f.w1[u] = p->w1f[u][lane];
        f.b2[u] = p->b2f[u][h];
    }
    f.w3[0] = p->w3a[0][h];
    f.w3[1] = p->w3a[1][h];
    f.w2 = w2_lds;
    return f;
}

// copy the layer-2 fragments into LDS (all threads of the block; the caller
// synchronises before use)
__device__ __forceinline__ void mlp_stage_w2(const MlpParams *p, half8 *w2_lds, int tid,
                                             int nthreads) {
    const half8 *src = &p->w2f[0][0][0];
    for (int i = tid; i < 4 * 2 * 64; i += nthreads) w2_lds[i] = src[i];
}

// GELU (tanh form x/2 (1 + tanh(a)), a = sqrt(2/pi)(x + 0.044715 x^3)) in
// packed FP16, two values per instruction: gelu(x) = x s(x) with the gate
// s = (1 + tanh a)/2 in [0, 1], written s = clamp(1/2 + x P(x^2), 0, 1).  P
// is a degree-4 polynomial fitted on |x| <= 3 (minimax-weighted least
// squares of the gelu error; coefficients rounded to FP16 from the top down,
// the lower ones refitted after each rounding).  Beyond the fit the odd
// polynomial x P(x^2) grows past 1/2 in magnitude (its leading coefficient
// is positive), so the clamp saturates the gate at 1 or 0; where x^2
// overflows FP16 it does so through infinities, never NaN for finite x.  The
// clamp is the instruction's clamp bit.  Max |error| of gelu over every
// finite FP16 input, in FP16 arithmetic: 3.3e-3 (at x = 3.03), below the
// FP16/BF16 rounding of the activations near 3.  Seven instructions per
// pair.  The degree-4 coefficient is an FP16 subnormal (FP16 denormals are
// preserved on this target).
__device__ __forceinline__ half2v mlp_gelu_h2(half2v x) {
    auto k = [](float v) { return half2v{(_Float16)v, (_Float16)v}; };
    const half2v y = x * x;
    half2v p = __builtin_elementwise_fma(y, k(1.710653305053711e-05f), k(-5.578994750976562e-04f));
    p = __builtin_elementwise_fma(p, y, k(7.762908935546875e-03f));
    p = __builtin_elementwise_fma(p, y, k(-6.2744140625e-02f));
    p = __builtin_elementwise_fma(p, y, k(3.96728515625e-01f));
    half2v s = __builtin_elementwise_fma(x, p, k(0.5f));
    s = __builtin_elementwise_min(__builtin_elementwise_max(s, k(0.0f)), k(1.0f));
    return x * s;
}

// Two independent pairs at once, the two evaluations step by step side by
// side: each instruction of one separates the dependent instructions of the
// other (a lone chain waits between its dependent packed instructions).
__device__ __forceinline__ void mlp_gelu_h2x2(half2v &xa, half2v &xb) {
    auto k = [](float v) { return half2v{(_Float16)v, (_Float16)v}; };
    const half2v ya = xa * xa, yb = xb * xb;
    half2v pa = __builtin_elementwise_fma(ya, k(1.710653305053711e-05f), k(-5.578994750976562e-04f));
    half2v pb = __builtin_elementwise_fma(yb, k(1.710653305053711e-05f), k(-5.578994750976562e-04f));
    pa = __builtin_elementwise_fma(pa, ya, k(7.762908935546875e-03f));
    pb = __builtin_elementwise_fma(pb, yb, k(7.762908935546875e-03f));
    pa = __builtin_elementwise_fma(pa, ya, k(-6.2744140625e-02f));
    pb = __builtin_elementwise_fma(pb, yb, k(-6.2744140625e-02f));
    pa = __builtin_elementwise_fma(pa, ya, k(3.96728515625e-01f));
    pb = __builtin_elementwise_fma(pb, yb, k(3.96728515625e-01f));
    half2v sa = __builtin_elementwise_fma(xa, pa, k(0.5f));
    half2v sb = __builtin_elementwise_fma(xb, pb, k(0.5f));
    sa = __builtin_elementwise_min(__builtin_elementwise_max(sa, k(0.0f)), k(1.0f));
    sb = __builtin_elementwise_min(__builtin_elementwise_max(sb, k(0.0f)), k(1.0f));
    xa = xa * sa;
    xb = xb * sb;
}

__device__ __forceinline__ float mlp_softplus(float x) {
    return x > 20.0f ? x : __logf(1.0f + __expf(x));
}

__device__ __forceinline__ short bf16_bits(float x) {
    __bf16 b = (__bf16)x;  // round to nearest even
    return __builtin_bit_cast(short, b);
}

// Raw features of one cell from Pi_neq (6 components), rho, row data.
// P = Pi_neq / (rho/3); n = e_y.
__device__ __forceinline__ void mlp_features(float nxx, float nyy, float nzz, float nxy,
                                             float nxz, float nyz, float rho, float yh,
                                             float lad, float (&x)[9]) {
    const float s = 3.0f / rho;
    const float a = nxx * s, b = nyy * s, c = nzz * s, d = nxy * s, e = nxz * s, f = nyz * s;
    // P^2 (symmetric)
    const float q_xx = a * a + d * d + e * e;
    const float q_yy = d * d + b * b + f * f;
    const float q_zz = e * e + f * f + c * c;
    const float q_xy = a * d + d * b + e * f;
    const float q_xz = a * e + d * f + e * c;
    const float q_yz = d * e + b * f + f * c;
    const float tr2 = q_xx + q_yy + q_zz;
    const float tr3 = q_xx * a + q_yy * b + q_zz * c + 2.0f * (q_xy * d + q_xz * e + q_yz * f);
    x[0] = a + b + c;
    x[1] = tr2;
    x[2] = tr3;
    x[3] = b;
    x[4] = q_yy;
    x[5] = sqrtf(tr2);
    x[6] = yh;
    x[7] = lad;
    x[8] = 1.0f;
}

// Learned nu_t for the 64 cells of this wave (one cell per lane).  z: this
// lane's 16 standardised inputs as bf16 bits (z0..z8, 1, 1, 0...), lds: 64 x 16
// shorts of this wave's scratch.  The caller orders the LDS write/read.
__device__ __forceinline__ void mlp_stage_inputs(short *lds, int lane, const short (&z)[16]) {
    typedef short short8v __attribute__((ext_vector_type(8)));
    short8v lo = {z[0], z[1], z[2], z[3], z[4], z[5], z[6], z[7]};
    short8v hi = {z[8], z[9], z[10], z[11], z[12], z[13], z[14], z[15]};
    *reinterpret_cast<short8v *>(lds + lane * 16) = lo;
    *reinterpret_cast<short8v *>(lds + lane * 16 + 8) = hi;
}

// o (pre-softplus output) for this lane's cell.  Layer 1 runs for the four
// 16-cell column tiles first (their FP16 activations stay in registers), so
// that each layer-2 weight fragment is read from LDS once per 64 cells and
// serves the four column tiles.  The output layer is a third product on the
// matrix cores: with w3 in every row of A, every row of a column tile's
// result holds o of that column, and lane quarter h keeps column tile h.
__device__ __forceinline__ float mlp_forward_wave(const MlpFrag &f, const short *lds, int lane,
                                                  float b3) {
    const int h = lane >> 4, col = lane & 15;
    half8 x2[4][2];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const short4v zb = *reinterpret_cast<const short4v *>(lds + (16 * ct + col) * 16 + 4 * h);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const floatx4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
            floatx4 d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(f.w1[u], zb, zero, 0, 0, 0);
            half2v g0 = half2v{(_Float16)d[0], (_Float16)d[1]};
            half2v g1 = half2v{(_Float16)d[2], (_Float16)d[3]};
            mlp_gelu_h2x2(g0, g1);
            const int o = (u & 1) * 4;
            x2[ct][u >> 1][o] = g0[0];
            x2[ct][u >> 1][o + 1] = g0[1];
            x2[ct][u >> 1][o + 2] = g1[0];
            x2[ct][u >> 1][o + 3] = g1[1];
        }
    }
    floatx4 acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = floatx4{b3, b3, b3, b3};
    // layer 2 by pairs of unit tiles (one k step of the output layer each):
    // both tiles of the pair for a column tile, then the output product
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        half8 w[2][2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            w[p][0] = f.w2[(2 * (2 * ks + p)) * 64 + lane];
            w[p][1] = f.w2[(2 * (2 * ks + p) + 1) * 64 + lane];
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            half8 x3;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int u = 2 * ks + p;
                floatx4 e = __builtin_amdgcn_mfma_f32_16x16x32_f16(w[p][0], x2[ct][0], f.b2[u], 0, 0, 0);
                e = __builtin_amdgcn_mfma_f32_16x16x32_f16(w[p][1], x2[ct][1], e, 0, 0, 0);
                half2v g0 = half2v{(_Float16)e[0], (_Float16)e[1]};
                half2v g1 = half2v{(_Float16)e[2], (_Float16)e[3]};
                mlp_gelu_h2x2(g0, g1);
                x3[4 * p] = g0[0];
                x3[4 * p + 1] = g0[1];
                x3[4 * p + 2] = g1[0];
                x3[4 * p + 3] = g1[1];
            }
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(f.w3[ks], x3, acc[ct], 0, 0, 0);
        }
    }
    return h == 0 ? acc[0][0] : h == 1 ? acc[1][0] : h == 2 ? acc[2][0] : acc[3][0];
}

}  // namespace lbmx
