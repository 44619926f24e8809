// mlp_kernels.hip -- learned eddy-viscosity closure: closure-blob validation
// and packing into the device layout of mlp_closure.h, the fallback counter.
#include <cmath>
#include <cstring>
#include <vector>

#include "mlp_closure.h"
#include "mlp_device.h"

namespace lbmx {

static_assert(sizeof(MlpParams) <= kMlpDeviceBytes, "closure parameters exceed their region");

namespace {

constexpr size_t kBlobBytes = 10184;

float f32_at(const unsigned char *b, size_t off) {
    float v;
    std::memcpy(&v, b + off, 4);
    return v;
}

uint16_t u16_at(const unsigned char *b, size_t off) {
    uint16_t v;
    std::memcpy(&v, b + off, 2);
    return v;
}

uint16_t to_bf16_bits(float x) {  // round to nearest even (finite inputs)
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// IEEE half, round to nearest even (finite inputs; overflow saturates to
// the largest finite half, which the weights never reach)
uint16_t to_f16_bits(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    const uint32_t sign = (u >> 16) & 0x8000u;
    const uint32_t ax = u & 0x7FFFFFFFu;
    if (ax >= 0x477FF000u) return (uint16_t)(sign | 0x7BFFu);  // >= 65520: saturate
    if (ax < 0x38800000u) {                                    // below 2^-14: subnormal
        float a;
        std::memcpy(&a, &ax, 4);
        const float q = std::nearbyint(a * 16777216.0f);       // units of 2^-24
        return (uint16_t)(sign | (uint32_t)q);
    }
    uint32_t m = ax + 0xC8000FFFu + ((ax >> 13) & 1u);  // rebias (-112 << 23), round
    return (uint16_t)(sign | (m >> 13));
}

float from_bf16_bits(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

}  // namespace

bool mlp_pack_blob(const void *blob, size_t nbytes, void *dev, MlpConst *mc, std::string *why) {
    auto fail = [&](const char *m) {
        if (why) *why = m;
        return false;
    };
    const unsigned char *b = static_cast<const unsigned char *>(blob);
    if (!b) return fail("NULL closure blob");
    if (nbytes != kBlobBytes) return fail("closure blob must be 10184 bytes");
    if (std::memcmp(b, "LBMC", 4) != 0) return fail("bad closure blob magic");
    uint32_t hdr[5];
    std::memcpy(hdr, b + 4, sizeof(hdr));
    if (hdr[0] != 1) return fail("unsupported closure blob version");
    if (hdr[1] != kMlpIn || hdr[2] != kMlpH1 || hdr[3] != kMlpH2)
        return fail("closure blob shape must be 9-64-64-1");
    MlpParams P;
    std::memset(&P, 0, sizeof(P));
    for (int i = 0; i < kMlpIn; ++i) {
        P.mean[i] = f32_at(b, 24 + 4 * i);
        const float sd = f32_at(b, 60 + 4 * i);
        if (!(sd > 0.0f) || !std::isfinite(sd)) return fail("feature std must be > 0");
        P.istd[i] = 1.0f / sd;
        P.lo[i] = f32_at(b, 96 + 4 * i);
        P.hi[i] = f32_at(b, 132 + 4 * i);
        if (!std::isfinite(P.mean[i])) return fail("feature mean must be finite");
    }
    P.scale = f32_at(b, 168);
    const float h = f32_at(b, 172);
    if (!(h > 0.0f) || !std::isfinite(h)) return fail("canopy height must be > 0");
    if (!(P.scale >= 0.0f) || !std::isfinite(P.scale)) return fail("output scale must be >= 0");
    P.inv_h = 1.0f / h;
    P.b3 = f32_at(b, 184 + 512);
    const size_t w1o = 712, w2o = w1o + 2 * kMlpH1 * kMlpIn, w3o = w2o + 2 * kMlpH2 * kMlpH1;
    // layer 1, augmented with the bias split into two bf16 halves (inputs 9, 10 are 1)
    std::vector<uint16_t> W1a(kMlpH1 * 16, 0);
    for (int u = 0; u < kMlpH1; ++u) {
        for (int k = 0; k < kMlpIn; ++k) W1a[u * 16 + k] = u16_at(b, w1o + 2 * (u * kMlpIn + k));
        const float b1 = f32_at(b, 184 + 4 * u);
        const uint16_t hi = to_bf16_bits(b1);
        W1a[u * 16 + 9] = hi;
        W1a[u * 16 + 10] = to_bf16_bits(b1 - from_bf16_bits(hi));
    }
    for (int ut = 0; ut < 4; ++ut)
        for (int l = 0; l < 64; ++l)
            for (int t = 0; t < 4; ++t)
                P.w1f[ut][l][t] = (short)W1a[(16 * ut + l % 16) * 16 + 4 * (l / 16) + t];
    for (int ut = 0; ut < 4; ++ut)
        for (int ks = 0; ks < 2; ++ks)
            for (int l = 0; l < 64; ++l)
                for (int t = 0; t < 8; ++t) {
                    const int uo = 16 * ut + l % 16, ui = mlp_l2_unit_in(ks, l / 16, t);
                    // FP16 holds every BF16 weight of magnitude in [2^-14, 65504]
                    // exactly
                    const float wv = from_bf16_bits(u16_at(b, w2o + 2 * (uo * kMlpH1 + ui)));
                    P.w2f[ut][ks][l][t] = __builtin_bit_cast(_Float16, to_f16_bits(wv));
                }
    for (int ut = 0; ut < 4; ++ut)
        for (int hq = 0; hq < 4; ++hq)
            for (int r = 0; r < 4; ++r)
                P.b2f[ut][hq][r] = f32_at(b, 184 + 256 + 4 * (16 * ut + 4 * hq + r));
    // output layer: w3 of layer-2 unit mlp_l2_unit_in(ks, hq, t) in every row
    for (int ks = 0; ks < 2; ++ks)
        for (int hq = 0; hq < 4; ++hq)
            for (int t = 0; t < 8; ++t) {
                const float wv = from_bf16_bits(u16_at(b, w3o + 2 * mlp_l2_unit_in(ks, hq, t)));
                P.w3a[ks][hq][t] = __builtin_bit_cast(_Float16, to_f16_bits(wv));
            }
    std::memcpy(dev, &P, sizeof(P));
    for (int i = 0; i < kMlpIn; ++i) {
        mc->zs[i] = P.istd[i];
        mc->zo[i] = -P.mean[i] * P.istd[i];
        mc->lo[i] = P.lo[i];
        mc->hi[i] = P.hi[i];
    }
    mc->inv_h = P.inv_h;
    mc->scale = P.scale;
    mc->b3 = P.b3;
    return true;
}

lbm_status mlp_fallback_count(const void *dev, int parity, int64_t *count, hipStream_t s) {
    const MlpParams *P = static_cast<const MlpParams *>(dev);
    unsigned long long v = 0;
    if (hipMemcpyAsync(&v, &P->fallback[parity & 1], sizeof(v), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return LBM_EDEVICE;
    *count = (int64_t)v;
    return LBM_OK;
}

}  // namespace lbmx
