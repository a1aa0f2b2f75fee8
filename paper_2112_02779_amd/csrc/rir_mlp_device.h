// Learned per-pixel robust weight (replaces the pseudo-Huber weight of
// Eq. (7)): features of a correspondence and the 14-64-64-1 network evaluated
// by one wavefront for its 64 lanes on the matrix cores (bf16 operands, FP32
// accumulation).
//
// The layers are computed transposed, H^T = W X^T, with the weights as the A
// operand and activations as the B operand of v_mfma_f32_16x16x16_bf16: the
// accumulator layout of that instruction (lane l holds rows 4(l/16)+j, column
// l%16 of a 16x16 tile) is exactly its B-operand layout, so the output of one
// layer feeds the next without moving data between lanes.
#pragma once

#include "rir_internal.h"

namespace rir {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint32_t f2bf(float f)
{
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7f800000u) == 0x7f800000u)
        return (b | ((b & 0x007fffffu) ? 0x00400000u : 0u)) >> 16;
    return (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ float round_bf(float f) { return bf2f(f2bf(f)); }

typedef __bf16 bf16x2v_t __attribute__((ext_vector_type(2)));
typedef float f32x2v_t __attribute__((ext_vector_type(2)));
typedef short s16x2v_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2v_t __attribute__((ext_vector_type(2)));

// Two floats rounded to bfloat16 (to nearest even, one hardware conversion)
// and packed, the first in the low half.
__device__ __forceinline__ uint32_t pack_bf2(float lo, float hi)
{
    const f32x2v_t f = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2v_t));
}

// ReLU of two packed bfloat16 values.  Read as int16, every negative value
// (and -0) lies below 0 and every positive one above, so the integer maximum
// with 0 is the ReLU; ReLU after rounding equals rounding after ReLU.
__device__ __forceinline__ uint32_t relu_bf2(uint32_t x)
{
    const s16x2v_t z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2v_t, x), z));
}

__device__ __forceinline__ bf16x4_t bf4(uint32_t lo, uint32_t hi)
{
    const u32x2v_t v = {lo, hi};
    return __builtin_bit_cast(bf16x4_t, v);
}

// The K = 32 matrix-core product (gfx950): lane l holds A[l % 16][8 (l / 16) + j]
// and B[8 (l / 16) + j][l % 16] for j < 8, and D as in the K = 16 form.
typedef __bf16 bf16x8v_t __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4v_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4_t mfma32(bf16x8v_t a, bf16x8v_t b, f32x4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Two K = 16 operands of one lane as one K = 32 operand: j < 4 from lo, j >= 4 from hi.
__device__ __forceinline__ bf16x8v_t cat8(bf16x4_t lo, bf16x4_t hi)
{
    const u32x2v_t a = __builtin_bit_cast(u32x2v_t, lo), b = __builtin_bit_cast(u32x2v_t, hi);
    const u32x4v_t v = {a.x, a.y, b.x, b.y};
    return __builtin_bit_cast(bf16x8v_t, v);
}

__device__ __forceinline__ f32x4_t mfma16(bf16x4_t a, bf16x4_t b, f32x4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Per-lane operand fragments of the network (lane l: r = l % 16, g = l / 16).
//  a1[mt]      W1 rows mt*16 + r, inputs 4g..4g+3 (inputs >= 14 are zero)
//  a2[mt][kt]  W2 rows mt*16 + r, inputs kt*16 + 4g..+3
//  b1, b2, w3  [mt][j] for hidden unit mt*16 + 4g + j
struct MlpFrag {
    bf16x4_t a1[4];
    bf16x4_t a2[4][4];
    float b1[4][4], b2[4][4], w3[4][4];
    float b3;
};

__device__ __forceinline__ void mlp_load(const MlpDev &m, MlpFrag &F)
{
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * g + j;
            F.a1[mt][j] = (short)(k < 14 ? m.w[kMlpW1 + (mt * 16 + r) * 14 + k] : 0);
            F.b1[mt][j] = m.b[kMlpB1 + mt * 16 + k];
            F.b2[mt][j] = m.b[kMlpB2 + mt * 16 + k];
            F.w3[mt][j] = bf2f(m.w[kMlpW3 + mt * 16 + k]);
        }
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                F.a2[mt][kt][j] = (short)m.w[kMlpW2 + (mt * 16 + r) * 64 + kt * 16 + 4 * g + j];
    }
    F.b3 = m.b[kMlpB3];
}

// Inference fragments (lane l: r = l % 16, g = l / 16).  Layer 1 uses K = 16
// products (a1, b1 as in MlpFrag).  Layers 2 and 3 use K = 32 products whose
// chunk c covers hidden units 32 c .. 32 c + 31 in the order that makes a
// chunk of B the two K = 16 output tiles 2c and 2c + 1 of the lane itself:
// operand index 8 g + j is unit (2 c + j / 4) * 16 + 4 g + j % 4.  a2[mt][c]
// holds W2 row mt * 16 + r over chunk c; a3[c] holds W3 over chunk c in the A
// rows r = 0, 4, 8, 12 and zeros in the others, so the output layer's result
// row 4 g (held by the lanes of group g) is z of pixel column r.
struct MlpInfer {
    bf16x4_t a1[4];
    bf16x8v_t a2[4][2];
    bf16x8v_t a3[2];
    float b1[4][4], b2[4][4];
    float b3;
};

__device__ __forceinline__ int chunk_unit(int c, int g, int j) { return (2 * c + (j >> 2)) * 16 + 4 * g + (j & 3); }

__device__ __forceinline__ void mlp_infer_load(const MlpDev &m, MlpInfer &F)
{
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * g + j;
            F.a1[mt][j] = (short)(k < 14 ? m.w[kMlpW1 + (mt * 16 + r) * 14 + k] : 0);
            F.b1[mt][j] = m.b[kMlpB1 + mt * 16 + k];
            F.b2[mt][j] = m.b[kMlpB2 + mt * 16 + k];
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            u32x4v_t v;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                v[q] = (uint32_t)m.w[kMlpW2 + (mt * 16 + r) * 64 + chunk_unit(c, g, 2 * q)] |
                       ((uint32_t)m.w[kMlpW2 + (mt * 16 + r) * 64 + chunk_unit(c, g, 2 * q + 1)] << 16);
            F.a2[mt][c] = __builtin_bit_cast(bf16x8v_t, v);
        }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        u32x4v_t v;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            v[q] = (r & 3) == 0 ? (uint32_t)m.w[kMlpW3 + chunk_unit(c, g, 2 * q)] |
                                      ((uint32_t)m.w[kMlpW3 + chunk_unit(c, g, 2 * q + 1)] << 16)
                                : 0u;
        F.a3[c] = __builtin_bit_cast(bf16x8v_t, v);
    }
    F.b3 = m.b[kMlpB3];
}

// Packs 14 features (rounded to bf16) into 8 dwords, two per dword, low half first.
__device__ __forceinline__ void pack_features(const float (&f)[14], uint32_t (&fp)[8])
{
#pragma unroll
    for (int k = 0; k < 7; ++k)
        fp[k] = pack_bf2(f[2 * k], f[2 * k + 1]);
    fp[7] = 0u;
}

// Logit z of the network for the wave's 64 pixels: lane l passes its pixel's
// packed features and receives z of that pixel.  `lds` is this wave's private
// 64 x 8-dword staging area (the feature transpose into B-operand layout).
// Layers 1 and 2 start from their biases in the accumulators; activations
// are rounded to bf16 two at a time and ReLU'd in packed form; layers 2 and 3
// are K = 32 products.  Must be called by all 64 lanes.
__device__ __forceinline__ float mlp_wave(const MlpInfer &F, const uint32_t (&fp)[8], uint32_t *lds)
{
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    uint4 *row = reinterpret_cast<uint4 *>(lds + lane * 8);
    row[0] = make_uint4(fp[0], fp[1], fp[2], fp[3]);
    row[1] = make_uint4(fp[4], fp[5], fp[6], fp[7]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float zsel = 0.f;
    // column tiles two at a time, layer by layer: two independent chains of
    // matrix-core products, so that one tile's products run while the
    // other's results are converted
#pragma unroll
    for (int np = 0; np < 4; np += 2) {
        bf16x4_t B[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const uint2 bb = *reinterpret_cast<const uint2 *>(lds + ((np + q) * 16 + r) * 8 + 2 * g);
            B[q] = bf4(bb.x, bb.y);
        }
        bf16x4_t h1[2][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                f32x4_t c = {F.b1[mt][0], F.b1[mt][1], F.b1[mt][2], F.b1[mt][3]};
                c = mfma16(F.a1[mt], B[q], c);
                h1[q][mt] = bf4(relu_bf2(pack_bf2(c[0], c[1])), relu_bf2(pack_bf2(c[2], c[3])));
            }
        bf16x4_t h2[2][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                f32x4_t c = {F.b2[mt][0], F.b2[mt][1], F.b2[mt][2], F.b2[mt][3]};
                c = mfma32(F.a2[mt][0], cat8(h1[q][0], h1[q][1]), c);
                c = mfma32(F.a2[mt][1], cat8(h1[q][2], h1[q][3]), c);
                h2[q][mt] = bf4(relu_bf2(pack_bf2(c[0], c[1])), relu_bf2(pack_bf2(c[2], c[3])));
            }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            f32x4_t z = {0.f, 0.f, 0.f, 0.f};
            z = mfma32(F.a3[0], cat8(h2[q][0], h2[q][1]), z);
            z = mfma32(F.a3[1], cat8(h2[q][2], h2[q][3]), z);
            zsel = g == np + q ? z[0] + F.b3 : zsel;
        }
    }
    __builtin_amdgcn_wave_barrier();
    return zsel;
}

__device__ __forceinline__ float clamp4(float x) { return fminf(fmaxf(x, -4.f), 4.f); }

// Features of a correspondence (target pixel (ul, vl) of level l, residual e,
// projected source range xr, target normal n):
//  f0 = target range / r_max, f1..f8 = clamp((neighbour - centre) / delta, +-4)
//  for the 8 level-l neighbours in raster order (u wraps; rows outside the
//  image or neighbours without return give +4), f9..f11 = n,
//  f12 = clamp(e / delta), f13 = clamp((target range - xr) / delta) (the
//  projective signed distance of Eq. (8)-(9)).  Unspecified when !valid (the
//  weight of such a pixel is zero; store_features writes zeros).
template <typename T>
__device__ __forceinline__ void compute_features(const StepArgs &a, const LevelImage &L, bool valid, int ul,
                                                 int vl, T e, T xr, T n0, T n1, T n2, float (&f)[14])
{
    const int Wl = L.Wl, Hl = L.Hl;
    const rsrc_t img = make_rsrc(L.rng, (uint32_t)(Hl * Wl) * 4u);
    const T rc = (T)bld1<float>(img, valid ? 4u * (uint32_t)(vl * Wl + ul) : kNoLoad);
    const T inv_delta = (T)(1.0 / a.delta), inv_rmax = (T)(1.0 / (double)a.r_max);
    f[0] = (float)(rc * inv_rmax);
    int k = 1;
#pragma unroll
    for (int dv = -1; dv <= 1; ++dv)
#pragma unroll
        for (int du = -1; du <= 1; ++du) {
            if (du == 0 && dv == 0)
                continue;
            const int vv = vl + dv;
            int uu = ul + du;
            uu = uu < 0 ? uu + Wl : (uu >= Wl ? uu - Wl : uu);
            const bool in = valid && vv >= 0 && vv < Hl;
            const float rn = bld1<float>(img, in ? 4u * (uint32_t)(vv * Wl + uu) : kNoLoad);
            f[k++] = range_ok(rn) ? clamp4((float)(((T)rn - rc) * inv_delta)) : 4.f;
        }
    f[9] = (float)n0;
    f[10] = (float)n1;
    f[11] = (float)n2;
    f[12] = clamp4((float)(e * inv_delta));
    f[13] = clamp4((float)((rc - xr) * inv_delta));
}

template <typename T>
__device__ __forceinline__ void store_features(const StepArgs &a, const LevelImage &L, bool valid, int ul,
                                               int vl, T e, T xr, T n0, T n1, T n2, float *out)
{
    float f[14];
    compute_features<T>(a, L, valid, ul, vl, e, xr, n0, n1, n2, f);
#pragma unroll
    for (int k = 0; k < 14; ++k)
        out[k] = valid ? f[k] : 0.f;
}

// The 8 neighbour features of target pixel i of a level image, as packed
// bf16 (the layout of PairDesc::nbf): the same FP32 arithmetic as
// compute_features, rounded once.  rc is the pixel's range.
template <typename T>
__device__ __forceinline__ uint4 neighbour_features(const float *img, int Hl, int Wl, int ul, int vl, T rc,
                                                    T inv_delta)
{
    float f[8];
    int k = 0;
#pragma unroll
    for (int dv = -1; dv <= 1; ++dv)
#pragma unroll
        for (int du = -1; du <= 1; ++du) {
            if (du == 0 && dv == 0)
                continue;
            const int vv = vl + dv;
            int uu = ul + du;
            uu = uu < 0 ? uu + Wl : (uu >= Wl ? uu - Wl : uu);
            const float rn = vv >= 0 && vv < Hl ? img[(size_t)vv * Wl + uu] : 0.f;
            f[k++] = range_ok(rn) ? clamp4((float)(((T)rn - rc) * inv_delta)) : 4.f;
        }
    return make_uint4(pack_bf2(f[0], f[1]), pack_bf2(f[2], f[3]), pack_bf2(f[4], f[5]), pack_bf2(f[6], f[7]));
}

// Target-side inputs of one correspondence's features (FP32 path): the
// target range at the associated pixel and its precomputed neighbour record
// (PairDesc::nbf, 8 packed bf16 features).  Loaded as soon as the pixel is
// known (right after the projection, beside the target record gather), so
// that the features cost no extra dependent memory step; lanes with on =
// false load nothing and get zeros.
struct NbrRec {
    float rc;
    uint32_t d0, d1, d2, d3;
};

__device__ __forceinline__ NbrRec load_nbr(const LevelImage &L, const uint32_t *nbf, bool on, int ul, int vl)
{
    const uint32_t npx = (uint32_t)(L.Hl * L.Wl);
    const uint32_t pix = (uint32_t)(vl * L.Wl + ul);
    const rsrc_t img = make_rsrc(L.rng, npx * 4u);
    const rsrc_t nb = make_rsrc(nbf, npx * 16u);
    NbrRec r;
    r.rc = bld1<float>(img, on ? 4u * pix : kNoLoad);
    const uint32_t o = on ? 16u * pix : kNoLoad;
    r.d0 = bld_u32(nb, o);
    r.d1 = bld_u32(nb, o + 4u);
    r.d2 = bld_u32(nb, o + 8u);
    r.d3 = bld_u32(nb, o + 12u);
    return r;
}

// This wavefront's 64 x 8-dword feature staging area (one per wave of a
// 256-thread workgroup).
__device__ __forceinline__ uint32_t *mlp_stage()
{
    __shared__ uint32_t s_stage[4][64 * 8];
    return s_stage[threadIdx.x >> 6];
}

// Logistic of the network's logit.
__device__ __forceinline__ float logistic(float z) { return d_rcp(1.f + __expf(-z)); }

// Learned weight sigmoid(z) of this lane's correspondence from its loaded
// target-side record (FP32): f0 | f1, f2 | f3, ..., f8 | f9 with f1..f8 from
// the record, then n, e and the projective signed distance.  All lanes of the
// wave must call it; the result of a lane without a correspondence is
// unspecified (its weight is masked by the caller).
__device__ __forceinline__ float learned_weight_rec(const StepArgs &a, const MlpInfer &F, const NbrRec &R, float e,
                                                    float xr, float n0, float n1, float n2)
{
    const float inv_delta = (float)(1.0 / a.delta), inv_rmax = (float)(1.0 / (double)a.r_max);
    uint32_t fp[8];
    fp[0] = (pack_bf2(R.rc * inv_rmax, 0.f) & 0xffffu) | (R.d0 << 16);
    fp[1] = __builtin_amdgcn_alignbit(R.d1, R.d0, 16);
    fp[2] = __builtin_amdgcn_alignbit(R.d2, R.d1, 16);
    fp[3] = __builtin_amdgcn_alignbit(R.d3, R.d2, 16);
    fp[4] = (R.d3 >> 16) | (pack_bf2(n0, 0.f) << 16);
    fp[5] = pack_bf2(n1, n2);
    fp[6] = pack_bf2(clamp4(e * inv_delta), clamp4((R.rc - xr) * inv_delta));
    fp[7] = 0u;
    return logistic(mlp_wave(F, fp, mlp_stage()));
}

// Learned weight sigmoid(z) of this lane's correspondence, features gathered
// here from the level's range image (FP64 path and debug dumps); all lanes of
// the wave must call it (lanes without a correspondence pass valid = false).
// dump (nullable) receives the features of pixel dump_index (>= 0).
template <typename T>
__device__ __forceinline__ T learned_weight(const StepArgs &a, const MlpInfer &F, const LevelImage &L,
                                            bool valid, int ul, int vl, T e, T xr, T n0, T n1, T n2, float *dump,
                                            int dump_index)
{
    uint32_t fp[8];
    float f[14];
    compute_features<T>(a, L, valid, ul, vl, e, xr, n0, n1, n2, f);
    if (dump && dump_index >= 0)
        for (int k = 0; k < 14; ++k)
            dump[14 * (size_t)dump_index + k] = valid ? f[k] : 0.f;
    pack_features(f, fp);
    return (T)logistic(mlp_wave(F, fp, mlp_stage()));
}

}  // namespace rir
