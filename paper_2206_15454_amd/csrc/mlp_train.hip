// mlp_train.hip -- training of the learned eddy-viscosity closure on the GPU:
// forward and backward passes of the 9-64-64-1 network with BF16 operands on
// the matrix cores (FP32 accumulation), a deterministic reduction of the
// gradient, and Adam on FP32 master weights.
//
// Loss (the closure's design, identical in the FP64 oracle):
//   L = (1/n) sum_s (softplus(o_s) - y_s / scale)^2,
//   o = w3 . gelu(W2 gelu(W1 z + b1) + b2) + b3,  z = (x - mean) / std,
// gelu the tanh form (evaluated here through one FP32 sigmoid per
// activation, which also gives its derivative; only inference uses the FP16
// polynomial).  Flat parameter order: W1[64][9], b1[64], W2[64][64], b2[64],
// w3[64], b3.
//
// A wavefront handles 64 samples at a time as four 16-sample tiles ct, and
// walks many such chunks.  Activations are transposed (units x samples) as in
// inference, so the layer-1 output tile is the B operand of layer 2 and the
// layer-2 gradient tile is the B operand of the backward product W2^T g2 (A
// fragments of W2^T packed with the same k permutation).  The weight
// gradients contract over samples: h1, g2, g1 and z are staged in LDS as
// [unit][sample] so that 8 consecutive samples are one 16-byte MFMA operand,
// and the products accumulate across the wavefront's chunks in the matrix
// accumulators.  Because inputs 9 and 10 of layer 1 are the constant 1
// carrying b1, the dW1 product also yields db1.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "mlp_closure.h"

namespace lbmx {

namespace {

constexpr int P_W1 = 0, P_B1 = 576, P_W2 = 640, P_B2 = 4736, P_W3 = 4800, P_B3 = 4864;
constexpr int NP = kMlpParams;  // 4865
constexpr int NPL = NP + 1;     // + loss

struct TrainFrag {
    short4v w1f[4][64];
    bf16x8 w2f[4][2][64];   // forward: A[u2][k = u1 (permuted)]
    bf16x8 w2tf[4][2][64];  // backward: A[u1][k = u2 (permuted)] = W2^T
    floatx4 b2f[4][4];
    floatx4 w3f[4][4];      // bf16-rounded w3 (as stored in a blob)
    float b3;
    float mean[9], istd[9];
    float inv_scale;
};

// GELU (tanh form) through one sigmoid: 0.5 (1 + tanh a) = sig(2a),
// 2a = 2 sqrt(2/pi) (x + 0.044715 x^3); gelu = x sig, and its derivative
// gelu' = sig + x sig (1 - sig) d(2a)/dx with d(2a)/dx = 2 sqrt(2/pi)
// (1 + 3 0.044715 x^2).
__device__ __forceinline__ float gelu_sig(float x) {
    const float a2 = 1.5957691216057308f * x * (1.0f + 0.044715f * x * x);
    return 1.0f / (1.0f + __expf(-a2));
}
__device__ __forceinline__ float gelu_grad_sig(float x, float sg) {
    return sg + x * sg * (1.0f - sg) * 1.5957691216057308f * (1.0f + 0.134145f * x * x);
}

__device__ __forceinline__ float softplus_f(float x) {
    return x > 20.0f ? x : log1pf(__expf(x));
}

__device__ __forceinline__ short bf16s(float x) { return __builtin_bit_cast(short, (__bf16)x); }

__device__ __forceinline__ float wave_sum16(float v) {  // sum over the 16 columns of a quarter
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    return v;
}

__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// per-wavefront staging of one 64-sample chunk, [unit or k][sample] in BF16
struct GradLds {
    short zs[64 * 16];   // [sample][k]
    short zT[16 * 64];   // [k][sample]
    short h1T[64 * 64];  // [unit][sample]
    short g2T[64 * 64];
    short g1T[64 * 64];
};
constexpr int kGradWaves = 4;          // wavefronts per block
constexpr int kGradBlocksMax = 256;    // one block per CU (LDS: 4 x 28 KiB)
static_assert(sizeof(GradLds) * kGradWaves >= sizeof(float) * kGradWaves * NPL,
              "the block reduction reuses the staging area");

// Gradient of the loss over n samples.  Each wavefront walks the 64-sample
// chunks c = wave id, wave id + waves in grid, ... in order and keeps its
// weight-gradient sums in the matrix-core accumulators (dW2, dW1) and in
// registers (dw3, db2, db3, loss) across chunks; the four wavefronts of a
// block are then summed in LDS in wave order and the block writes one
// partial part[blockIdx.x][NPL] (parameters in flat order, then the loss
// sum).  The chunk assignment and every summation order are fixed, so the
// result is deterministic.
__global__ __launch_bounds__(256) void mlp_grad_kernel(const TrainFrag *__restrict__ F,
                                                       const float *__restrict__ X,
                                                       const float *__restrict__ Y, int n,
                                                       float inv_n, float *__restrict__ part) {
    __shared__ __attribute__((aligned(16))) GradLds lds[kGradWaves];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, h = lane >> 4, col = lane & 15;
    GradLds &L = lds[wave];
    const int nch = (n + 63) / 64;
    typedef short short8v __attribute__((ext_vector_type(8)));
    auto frag8 = [&](const short *base, int row, int ks) -> bf16x8 {
        return __builtin_bit_cast(bf16x8,
                                  *reinterpret_cast<const short8v *>(base + row * 64 + 32 * ks + 8 * h));
    };

    floatx4 dW2[16], dW1[4];
    #pragma unroll
    for (int i = 0; i < 16; ++i) dW2[i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    #pragma unroll
    for (int i = 0; i < 4; ++i) dW1[i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    float dw3[16], db2[16];
    #pragma unroll
    for (int i = 0; i < 16; ++i) dw3[i] = db2[i] = 0.0f;
    float loss = 0.0f, db3 = 0.0f;

    for (int c = blockIdx.x * kGradWaves + wave; c < nch; c += gridDim.x * kGradWaves) {
        const int s0 = c * 64;
        wave_lds_fence();  // the previous chunk's reads of the staging area are done
        {
            const int s = s0 + lane;
            short z[16];
            #pragma unroll
            for (int k = 0; k < 9; ++k) {
                const float x = s < n ? X[(long long)s * 9 + k] : 0.0f;
                z[k] = bf16s((x - F->mean[k]) * F->istd[k]);
            }
            z[9] = z[10] = bf16s(1.0f);
            #pragma unroll
            for (int k = 11; k < 16; ++k) z[k] = 0;
            #pragma unroll
            for (int k = 0; k < 16; ++k) {
                L.zs[lane * 16 + k] = z[k];
                L.zT[k * 64 + lane] = z[k];
            }
        }
        wave_lds_fence();
        for (int ct = 0; ct < 4; ++ct) {
            const int s = s0 + 16 * ct + col;  // this lane's sample (column) in the tile
            const float m = s < n ? 1.0f : 0.0f;
            const float yt = s < n ? Y[s] * F->inv_scale : 0.0f;
            const short4v zb = *reinterpret_cast<const short4v *>(L.zs + (16 * ct + col) * 16 + 4 * h);
            floatx4 a1[4], sg1[4];
            bf16x8 x2[2];
            #pragma unroll
            for (int u = 0; u < 4; ++u) {
                const floatx4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
                a1[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(F->w1f[u][lane], zb, zero, 0, 0, 0);
                #pragma unroll
                for (int r = 0; r < 4; ++r) {
                    sg1[u][r] = gelu_sig(a1[u][r]);
                    const short hb = bf16s(a1[u][r] * sg1[u][r]);
                    x2[u >> 1][(u & 1) * 4 + r] = __builtin_bit_cast(__bf16, hb);
                    L.h1T[(16 * u + 4 * h + r) * 64 + 16 * ct + col] = hb;
                }
            }
            floatx4 a2[4], sg2[4];
            float part_o = 0.0f;
            #pragma unroll
            for (int u = 0; u < 4; ++u) {
                a2[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F->w2f[u][0][lane], x2[0], F->b2f[u][h], 0, 0, 0);
                a2[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F->w2f[u][1][lane], x2[1], a2[u], 0, 0, 0);
                #pragma unroll
                for (int r = 0; r < 4; ++r) {
                    sg2[u][r] = gelu_sig(a2[u][r]);
                    part_o += F->w3f[u][h][r] * (a2[u][r] * sg2[u][r]);
                }
            }
            part_o += __shfl_xor(part_o, 16, 64);
            part_o += __shfl_xor(part_o, 32, 64);
            const float o = part_o + F->b3;
            const float e = softplus_f(o) - yt;
            const float go = m * 2.0f * e * inv_n / (1.0f + __expf(-o));  // dL/do
            if (h == 0) {
                loss += m * e * e;
                db3 += go;
            }
            // layer-2 gradient g2 = go * w3 * gelu'(a2), in the output layout
            bf16x8 g2b[2];
            #pragma unroll
            for (int u = 0; u < 4; ++u)
                #pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * u + r;
                    dw3[i] += go * (a2[u][r] * sg2[u][r]);
                    const float g2 = go * F->w3f[u][h][r] * gelu_grad_sig(a2[u][r], sg2[u][r]);
                    db2[i] += g2;
                    const short gb = bf16s(g2);
                    g2b[u >> 1][(u & 1) * 4 + r] = __builtin_bit_cast(__bf16, gb);
                    L.g2T[(16 * u + 4 * h + r) * 64 + 16 * ct + col] = gb;
                }
            // layer-1 gradient g1 = (W2^T g2) * gelu'(a1)
            #pragma unroll
            for (int u = 0; u < 4; ++u) {
                const floatx4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
                floatx4 b = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F->w2tf[u][0][lane], g2b[0], zero, 0, 0, 0);
                b = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F->w2tf[u][1][lane], g2b[1], b, 0, 0, 0);
                #pragma unroll
                for (int r = 0; r < 4; ++r)
                    L.g1T[(16 * u + 4 * h + r) * 64 + 16 * ct + col] =
                        bf16s(b[r] * gelu_grad_sig(a1[u][r], sg1[u][r]));
            }
        }
        wave_lds_fence();
        // weight gradients: contractions over the chunk's 64 samples, added to
        // the accumulators.  dW2[u2][u1] = sum_s g2[u2,s] h1[u1,s];
        // dW1[u1][k] = sum_s g1[u1,s] z[k,s] (column k = 9 is db1)
        #pragma unroll
        for (int ut2 = 0; ut2 < 4; ++ut2)
            #pragma unroll
            for (int ut1 = 0; ut1 < 4; ++ut1)
                #pragma unroll
                for (int ks = 0; ks < 2; ++ks)
                    dW2[4 * ut2 + ut1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        frag8(L.g2T, 16 * ut2 + col, ks), frag8(L.h1T, 16 * ut1 + col, ks),
                        dW2[4 * ut2 + ut1], 0, 0, 0);
        #pragma unroll
        for (int ut1 = 0; ut1 < 4; ++ut1)
            #pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                dW1[ut1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    frag8(L.g1T, 16 * ut1 + col, ks), frag8(L.zT, col, ks), dW1[ut1], 0, 0, 0);
    }

    // ---- the wave's sums into LDS (flat parameter order), then the block's
    __syncthreads();  // every wave is done with its staging area
    float *st = reinterpret_cast<float *>(&lds[0]) + wave * NPL;
    #pragma unroll
    for (int ut2 = 0; ut2 < 4; ++ut2)
        #pragma unroll
        for (int ut1 = 0; ut1 < 4; ++ut1)
            #pragma unroll
            for (int r = 0; r < 4; ++r)
                st[P_W2 + (16 * ut2 + 4 * h + r) * 64 + 16 * ut1 + col] = dW2[4 * ut2 + ut1][r];
    #pragma unroll
    for (int ut1 = 0; ut1 < 4; ++ut1)
        #pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int u1 = 16 * ut1 + 4 * h + r;
            if (col < 9) st[P_W1 + u1 * 9 + col] = dW1[ut1][r];
            if (col == 9) st[P_B1 + u1] = dW1[ut1][r];
        }
    #pragma unroll
    for (int i = 0; i < 16; ++i) {
        const float a = wave_sum16(dw3[i]);
        const float b = wave_sum16(db2[i]);
        const int u = 16 * (i >> 2) + 4 * h + (i & 3);
        if (col == 0) {
            st[P_W3 + u] = a;
            st[P_B2 + u] = b;
        }
    }
    const float lsum = wave_sum16(loss);
    const float b3sum = wave_sum16(db3);
    if (lane == 0) {
        st[P_B3] = b3sum;
        st[NP] = lsum;
    }
    __syncthreads();
    const float *s0p = reinterpret_cast<const float *>(&lds[0]);
    float *out = part + (long long)blockIdx.x * NPL;
    #pragma unroll
    for (int i = tid; i < NPL; i += 256)
        out[i] = ((s0p[i] + s0p[NPL + i]) + s0p[2 * NPL + i]) + s0p[3 * NPL + i];
}

// grad[i] = sum over blocks of part[b][i] (fixed order, FP64), then with
// update != 0 one Adam step on the FP32 master parameter i
__global__ __launch_bounds__(256) void mlp_reduce_adam_kernel(
    const float *__restrict__ part, int nb, float *__restrict__ grad, int update,
    float *__restrict__ p, float *__restrict__ m, float *__restrict__ v, float lr, float b1,
    float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPL) return;
    // fixed summation order; the loads of a group of 8 are issued together
    double s = 0.0;
    int b = 0;
    for (; b + 8 <= nb; b += 8) {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = part[(long long)(b + k) * NPL + i];
#pragma unroll
        for (int k = 0; k < 8; ++k) s += v[k];
    }
    for (; b < nb; ++b) s += part[(long long)b * NPL + i];
    const float gi = (float)s;
    grad[i] = gi;
    if (!update || i >= NP) return;
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 MFMA fragments of the current master parameters (one thread per
// fragment element)
__global__ __launch_bounds__(256) void mlp_pack_kernel(const float *__restrict__ p,
                                                       TrainFrag *__restrict__ F) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    constexpr int N1 = 4 * 64 * 4, N2 = 4 * 2 * 64 * 8;
    if (i < N1) {
        const int u = i / 256, l = (i / 4) % 64, t = i % 4;
        const int unit = 16 * u + l % 16, k = 4 * (l / 16) + t;
        float val = 0.0f;
        if (k < 9) {
            val = p[P_W1 + unit * 9 + k];
        } else if (k == 9 || k == 10) {
            const float b = p[P_B1 + unit];
            const float hi = (float)(__bf16)b;
            val = (k == 9) ? hi : b - hi;
        }
        F->w1f[u][l][t] = bf16s(val);
    } else if (i < N1 + N2) {
        const int j = i - N1;
        const int u = j / 1024, ks = (j / 512) % 2, l = (j / 8) % 64, t = j % 8;
        const int uo = 16 * u + l % 16, ui = mlp_l2_unit_in(ks, l / 16, t);
        F->w2f[u][ks][l][t] = (__bf16)p[P_W2 + uo * 64 + ui];
        F->w2tf[u][ks][l][t] = (__bf16)p[P_W2 + ui * 64 + uo];
    } else if (i < N1 + N2 + 64) {
        const int u = i - N1 - N2;  // unit 16 ut + 4 hq + r
        F->b2f[u / 16][(u / 4) % 4][u % 4] = p[P_B2 + u];
        F->w3f[u / 16][(u / 4) % 4][u % 4] = (float)(__bf16)p[P_W3 + u];
    } else if (i == N1 + N2 + 64) {
        F->b3 = p[P_B3];
    }
}

}  // namespace

}  // namespace lbmx

using namespace lbmx;

struct lbm_trainer {
    lbm_train_params prm{};
    hipStream_t stream = nullptr;
    int max_batch = 0;
    float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *part = nullptr;
    TrainFrag *frag = nullptr;
    void *base = nullptr;
    int64_t t = 0;
    std::string err;
};

namespace {

lbm_status tfail(lbm_trainer *tr, lbm_status s, const std::string &m) {
    if (tr) tr->err = m;
    return s;
}

#define TCHK(tr, call, what)                                                              \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return tfail(tr, LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

// gradient blocks for n samples: one 64-sample chunk per wavefront while
// they last, at most one block per CU's worth of the device
int grad_blocks(int64_t n) {
    const int64_t chunks = (n + 63) / 64;
    const int64_t b = (chunks + kGradWaves - 1) / kGradWaves;
    return (int)(b < kGradBlocksMax ? (b > 0 ? b : 1) : kGradBlocksMax);
}

lbm_status repack(lbm_trainer *tr) {
    constexpr int total = 4 * 64 * 4 + 4 * 2 * 64 * 8 + 64 + 1;
    hipLaunchKernelGGL(mlp_pack_kernel, dim3((total + 255) / 256), dim3(256), 0, tr->stream, tr->p,
                       tr->frag);
    TCHK(tr, hipGetLastError(), "pack");
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_train_create(const lbm_train_params *prm, const float *params, lbm_trainer **out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (!prm || !params || prm->max_batch < 1 || !(prm->out_scale > 0.0f) || !(prm->lr > 0.0f))
        return LBM_EINVAL;
    for (int i = 0; i < 9; ++i)
        if (!(prm->std[i] > 0.0f) || !std::isfinite(prm->mean[i])) return LBM_EINVAL;
    lbm_trainer *tr = new (std::nothrow) lbm_trainer();
    if (!tr) return LBM_ENOMEM;
    tr->prm = *prm;
    tr->stream = static_cast<hipStream_t>(prm->stream);
    tr->max_batch = prm->max_batch;
    const int nw = grad_blocks(prm->max_batch);
    const size_t a = 256;
    auto up = [&](size_t x) { return (x + a - 1) / a * a; };
    const size_t o_p = 0, o_m = o_p + up(NP * 4), o_v = o_m + up(NP * 4), o_g = o_v + up(NP * 4),
                 o_f = o_g + up(NPL * 4), o_part = o_f + up(sizeof(TrainFrag)),
                 total = o_part + up((size_t)nw * NPL * 4);
    if (hipMalloc(&tr->base, total) != hipSuccess) {
        (void)hipGetLastError();
        delete tr;
        return LBM_ENOMEM;
    }
    char *b = static_cast<char *>(tr->base);
    tr->p = reinterpret_cast<float *>(b + o_p);
    tr->m = reinterpret_cast<float *>(b + o_m);
    tr->v = reinterpret_cast<float *>(b + o_v);
    tr->grad = reinterpret_cast<float *>(b + o_g);
    tr->frag = reinterpret_cast<TrainFrag *>(b + o_f);
    tr->part = reinterpret_cast<float *>(b + o_part);
    TrainFrag host;
    std::memset(&host, 0, sizeof(host));
    for (int i = 0; i < 9; ++i) {
        host.mean[i] = prm->mean[i];
        host.istd[i] = 1.0f / prm->std[i];
    }
    host.inv_scale = 1.0f / prm->out_scale;
    bool ok = hipMemcpyAsync(tr->frag, &host, sizeof(host), hipMemcpyHostToDevice, tr->stream) == hipSuccess &&
              hipMemcpyAsync(tr->p, params, NP * 4, hipMemcpyHostToDevice, tr->stream) == hipSuccess &&
              hipMemsetAsync(tr->m, 0, NP * 4, tr->stream) == hipSuccess &&
              hipMemsetAsync(tr->v, 0, NP * 4, tr->stream) == hipSuccess &&
              repack(tr) == LBM_OK && hipStreamSynchronize(tr->stream) == hipSuccess;
    if (!ok) {
        (void)hipFree(tr->base);
        delete tr;
        return LBM_EDEVICE;
    }
    *out = tr;
    return LBM_OK;
}

lbm_status lbm_train_step(lbm_trainer *tr, const float *X, const float *Y, int64_t n,
                          int32_t update, float *loss_out) {
    if (!tr) return LBM_EINVAL;
    if (!X || !Y || n < 1 || n > tr->max_batch)
        return tfail(tr, LBM_EINVAL, "lbm_train_step: need device X, y and 1 <= n <= max_batch");
    const int nb = grad_blocks(n);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(nb), dim3(256), 0, tr->stream, tr->frag, X, Y, (int)n,
                       1.0f / (float)n, tr->part);
    TCHK(tr, hipGetLastError(), "lbm_train_step: gradient");
    float c1 = 1.0f, c2 = 1.0f;
    if (update) {
        tr->t += 1;
        c1 = 1.0f - std::pow(tr->prm.beta1, (float)tr->t);
        c2 = 1.0f - std::pow(tr->prm.beta2, (float)tr->t);
    }
    hipLaunchKernelGGL(mlp_reduce_adam_kernel, dim3((NPL + 255) / 256), dim3(256), 0, tr->stream,
                       tr->part, nb, tr->grad, (int)(update != 0), tr->p, tr->m, tr->v,
                       tr->prm.lr, tr->prm.beta1, tr->prm.beta2, tr->prm.eps, c1, c2);
    TCHK(tr, hipGetLastError(), "lbm_train_step: reduce");
    if (update) {
        lbm_status s = repack(tr);
        if (s != LBM_OK) return s;
    }
    if (loss_out) {
        float l = 0.0f;
        TCHK(tr, hipMemcpyAsync(&l, tr->grad + NP, 4, hipMemcpyDeviceToHost, tr->stream), "loss copy");
        TCHK(tr, hipStreamSynchronize(tr->stream), "lbm_train_step: sync");
        *loss_out = l / (float)n;
    }
    return LBM_OK;
}

lbm_status lbm_train_get(lbm_trainer *tr, float *params, float *grad) {
    if (!tr) return LBM_EINVAL;
    if (params) TCHK(tr, hipMemcpyAsync(params, tr->p, NP * 4, hipMemcpyDeviceToHost, tr->stream), "copy");
    if (grad) TCHK(tr, hipMemcpyAsync(grad, tr->grad, NP * 4, hipMemcpyDeviceToHost, tr->stream), "copy");
    TCHK(tr, hipStreamSynchronize(tr->stream), "lbm_train_get: sync");
    return LBM_OK;
}

lbm_status lbm_train_destroy(lbm_trainer *tr) {
    if (!tr) return LBM_EINVAL;
    (void)hipStreamSynchronize(tr->stream);
    (void)hipFree(tr->base);
    delete tr;
    return LBM_OK;
}

const char *lbm_train_last_error(const lbm_trainer *tr) {
    return tr ? tr->err.c_str() : "lbm: NULL trainer";
}

}  // extern "C"
