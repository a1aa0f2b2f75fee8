// Learned per-pixel robust weight: standalone forward, training gradient and
// Adam update on gfx950.  Every product runs on the matrix cores
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation) with these bfloat16 rounding
// points, shared with the FP64 test oracle:
//   forward  inputs f, hidden activations h1 = relu(a1), h2 = relu(a2);
//   backward dz = (sigmoid(z) - y) / B, g2 = relu'(a2) W3 dz and
//            g1 = relu'(a1) W2^T g2 (relu'(0) = 0); bias gradients are sums
//            of these rounded deltas.
// Gradients are reduced without atomics: every wavefront writes one record,
// and the update kernel sums the records in a fixed order.
#include <mutex>

#include "rir_internal.h"
#include "rir_mlp_device.h"

namespace rir {

constexpr int kMlpGradWaves = 4;  // wavefronts per workgroup of the gradient kernel

__global__ __launch_bounds__(256) void k_mlp_forward(MlpDev m, const float *feats, int64_t B, float *w_out)
{
    __shared__ uint32_t stage[4][64 * 8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    MlpInfer F;
    mlp_infer_load(m, F);
    const int64_t stride = (int64_t)gridDim.x * 4 * 64;
    for (int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 64; base < B; base += stride) {
        const int64_t i = base + lane;
        float f[14];
#pragma unroll
        for (int k = 0; k < 14; ++k)
            f[k] = i < B ? feats[14 * i + k] : 0.f;
        uint32_t fp[8];
        pack_features(f, fp);
        const float z = mlp_wave(F, fp, stage[wave]);
        if (i < B)
            w_out[i] = 1.f / (1.f + __expf(-z));
    }
}

__device__ __forceinline__ bf16x4_t lds_bf4(const uint16_t *p)
{
    const uint2 v = *reinterpret_cast<const uint2 *>(p);
    bf16x4_t b;
    b[0] = (short)(v.x & 0xffffu);
    b[1] = (short)(v.x >> 16);
    b[2] = (short)(v.y & 0xffffu);
    b[3] = (short)(v.y >> 16);
    return b;
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Gradient of the summed loss over this wavefront's samples.  Record layout:
// W1[64][14], b1[64], W2[64][64], b2[64], W3[64], b3, loss.
__global__ __launch_bounds__(256) void k_mlp_grad(MlpDev m, const float *feats, const float *labels, int64_t B,
                                                  float *gpart)
{
    __shared__ uint32_t s_feat[kMlpGradWaves][64 * 8];    // [pixel][16 bf16]
    __shared__ uint16_t s_g2[kMlpGradWaves][64 * 16];     // [h2][px of the tile]
    __shared__ uint16_t s_h1[kMlpGradWaves][64 * 16];     // [h1][px]
    __shared__ uint16_t s_g1[kMlpGradWaves][64 * 16];     // [h1][px]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
    MlpFrag F;
    mlp_load(m, F);
    // W2^T fragments: rows h1 = mt*16 + r, inputs h2 = kt*16 + 4g + j
    bf16x4_t a2t[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                a2t[mt][kt][j] = (short)m.w[kMlpW2 + (kt * 16 + 4 * g + j) * 64 + mt * 16 + r];
    f32x4_t dW2[4][4], dW1[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        dW1[a] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b)
            dW2[a][b] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
    }
    float dW3[4][4], db2[4][4], db1[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            dW3[a][j] = db2[a][j] = db1[a][j] = 0.f;
    float db3 = 0.f, loss = 0.f;
    const float invB = 1.f / (float)B;
    uint32_t *sf = s_feat[wave];
    uint16_t *sfh = reinterpret_cast<uint16_t *>(sf);
    uint16_t *sg2 = s_g2[wave], *sh1 = s_h1[wave], *sg1 = s_g1[wave];
    const int64_t stride = (int64_t)gridDim.x * kMlpGradWaves * 64;
    for (int64_t base = ((int64_t)blockIdx.x * kMlpGradWaves + wave) * 64; base < B; base += stride) {
        {
            const int64_t i = base + lane;
            float f[14];
#pragma unroll
            for (int k = 0; k < 14; ++k)
                f[k] = i < B ? feats[14 * i + k] : 0.f;
            uint32_t fp[8];
            pack_features(f, fp);
            uint4 *row = reinterpret_cast<uint4 *>(sf + lane * 8);
            row[0] = make_uint4(fp[0], fp[1], fp[2], fp[3]);
            row[1] = make_uint4(fp[4], fp[5], fp[6], fp[7]);
        }
        wave_lds_sync();
#pragma unroll 1
        for (int nt = 0; nt < 4; ++nt) {
            const int64_t smp = base + nt * 16 + r;  // sample of this lane's column
            const bool ok = smp < B;
            // ---- forward
            const bf16x4_t Bf = lds_bf4(sfh + (nt * 16 + r) * 16 + 4 * g);
            bf16x4_t hb[4];
            bool m1[4][4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                f32x4_t c = {F.b1[mt][0], F.b1[mt][1], F.b1[mt][2], F.b1[mt][3]};
                c = mfma16(F.a1[mt], Bf, c);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    m1[mt][j] = c[j] > 0.f;
                    hb[mt][j] = (short)f2bf(fmaxf(c[j], 0.f));
                }
            }
            float h2[4][4];
            bool m2[4][4];
            float part = 0.f;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                f32x4_t c = {F.b2[mt][0], F.b2[mt][1], F.b2[mt][2], F.b2[mt][3]};
#pragma unroll
                for (int kt = 0; kt < 4; ++kt)
                    c = mfma16(F.a2[mt][kt], hb[kt], c);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    m2[mt][j] = c[j] > 0.f;
                    h2[mt][j] = round_bf(fmaxf(c[j], 0.f));
                    part += F.w3[mt][j] * h2[mt][j];
                }
            }
            part += __shfl_xor(part, 16, 64);
            part += __shfl_xor(part, 32, 64);
            const float z = part + F.b3;
            // ---- loss and output delta
            const float y = ok ? labels[smp] : 0.f;
            const float sp = z > 0.f ? z + log1pf(__expf(-z)) : log1pf(__expf(z));
            if (ok && g == 0)
                loss += sp - y * z;
            const float dz = ok ? round_bf((1.f / (1.f + __expf(-z)) - y) * invB) : 0.f;
            if (g == 0)
                db3 += dz;
            // ---- layer 3 and hidden-2 deltas (accumulator layout)
            bf16x4_t g2b[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    dW3[mt][j] += dz * h2[mt][j];
                    const float d2 = round_bf(m2[mt][j] ? F.w3[mt][j] * dz : 0.f);
                    db2[mt][j] += d2;
                    g2b[mt][j] = (short)f2bf(d2);
                    sg2[(mt * 16 + 4 * g + j) * 16 + r] = (uint16_t)f2bf(d2);
                    sh1[(mt * 16 + 4 * g + j) * 16 + r] = (uint16_t)hb[mt][j];
                }
            // ---- hidden-1 deltas: W2^T g2
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                f32x4_t c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kt = 0; kt < 4; ++kt)
                    c = mfma16(a2t[mt][kt], g2b[kt], c);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float d1 = round_bf(m1[mt][j] ? c[j] : 0.f);
                    db1[mt][j] += d1;
                    sg1[(mt * 16 + 4 * g + j) * 16 + r] = (uint16_t)f2bf(d1);
                }
            }
            wave_lds_sync();
            // ---- weight gradients, contracting over the 16 samples of the tile
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const bf16x4_t A2 = lds_bf4(sg2 + (mt * 16 + r) * 16 + 4 * g);
#pragma unroll
                for (int n = 0; n < 4; ++n)
                    dW2[mt][n] = mfma16(A2, lds_bf4(sh1 + (n * 16 + r) * 16 + 4 * g), dW2[mt][n]);
                const bf16x4_t A1 = lds_bf4(sg1 + (mt * 16 + r) * 16 + 4 * g);
                bf16x4_t Bx;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    Bx[j] = (short)sfh[(nt * 16 + 4 * g + j) * 16 + r];
                dW1[mt] = mfma16(A1, Bx, dW1[mt]);
            }
            wave_lds_sync();
        }
    }
    // ---- write this wavefront's record
    float *rec = gpart + ((size_t)blockIdx.x * kMlpGradWaves + wave) * kMlpGradRecord;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int h = mt * 16 + 4 * g + j;
#pragma unroll
            for (int n = 0; n < 4; ++n)
                rec[960 + h * 64 + n * 16 + r] = dW2[mt][n][j];
            if (r < 14)
                rec[h * 14 + r] = dW1[mt][j];
            float a = dW3[mt][j], b2 = db2[mt][j], b1 = db1[mt][j];
#pragma unroll
            for (int s = 1; s < 16; s <<= 1) {
                a += __shfl_xor(a, s, 64);
                b2 += __shfl_xor(b2, s, 64);
                b1 += __shfl_xor(b1, s, 64);
            }
            if (r == 0) {
                rec[5120 + h] = a;
                rec[5056 + h] = b2;
                rec[896 + h] = b1;
            }
        }
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        db3 += __shfl_xor(db3, s, 64);
        loss += __shfl_xor(loss, s, 64);
    }
    if (lane == 0) {
        rec[5184] = db3;
        rec[5185] = loss;
    }
}

// Sums the gradient records in a fixed order (FP64) and applies one Adam step
// (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) to the FP32 master
// weights and the biases; the bf16 weights are re-rounded from the masters.
__global__ __launch_bounds__(256) void k_mlp_adam(const float *gpart, int nrec, int64_t B, float lr, int step,
                                                  float *master, float *bias, float *m1, float *m2, uint16_t *wbf,
                                                  float *loss_out, float *grads_out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 5185 && loss_out) {
        double s = 0.0;
        for (int k = 0; k < nrec; ++k)
            s += (double)gpart[(size_t)k * kMlpGradRecord + 5185];
        loss_out[0] = (float)(s / (double)B);
    }
    if (j >= 5185)
        return;
    double s = 0.0;
    for (int k = 0; k < nrec; ++k)
        s += (double)gpart[(size_t)k * kMlpGradRecord + j];
    const float gj = (float)s;
    if (grads_out)
        grads_out[j] = gj;
    const float b1 = 0.9f, b2 = 0.999f;
    const float mm = b1 * m1[j] + (1.f - b1) * gj;
    const float vv = b2 * m2[j] + (1.f - b2) * gj * gj;
    m1[j] = mm;
    m2[j] = vv;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    const float upd = lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
    // parameter j of the record layout -> weight or bias slot
    int wi = -1, bi = -1;
    if (j < 896)
        wi = kMlpW1 + j;
    else if (j < 960)
        bi = kMlpB1 + (j - 896);
    else if (j < 5056)
        wi = kMlpW2 + (j - 960);
    else if (j < 5120)
        bi = kMlpB2 + (j - 5056);
    else if (j < 5184)
        wi = kMlpW3 + (j - 5120);
    else
        bi = kMlpB3;
    if (wi >= 0) {
        const float nw = master[wi] - upd;
        master[wi] = nw;
        wbf[wi] = (uint16_t)f2bf(nw);
    } else {
        bias[bi] -= upd;
    }
}

// Gradient records of the allocation-free training step: a fixed device array
// of kMlpScratchRecords records (10.1 MiB), one copy per GPU for the life of
// the process.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device, with that
// device current.
static __device__ __align__(256) float scratch[(size_t)kMlpScratchRecords * kMlpGradRecord];
static std::mutex g_scratch_mu;
static float *g_scratch_ptr[kMlpMaxDevices] = {};

hipError_t mlp_scratch(int device, float **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMlpMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_scratch_ptr[device] = static_cast<float *>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

int mlp_grad_blocks(int64_t B)
{
    int64_t nb = (B + 64 * kMlpGradWaves - 1) / (64 * kMlpGradWaves);
    return (int)(nb < 1 ? 1 : (nb > 512 ? 512 : nb)) * kMlpGradWaves;
}

hipError_t launch_mlp_forward(const MlpDev &m, const float *feats, int64_t B, float *w_out, hipStream_t stream)
{
    int64_t nb = (B + 255) / 256;
    nb = nb < 1 ? 1 : (nb > 4096 ? 4096 : nb);
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)nb), dim3(256), 0, stream, m, feats, B, w_out);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpDev &m, const float *feats, const float *labels, int64_t B, float *gpart,
                           int nrec, hipStream_t stream)
{
    hipLaunchKernelGGL(k_mlp_grad, dim3(nrec / kMlpGradWaves), dim3(64 * kMlpGradWaves), 0, stream, m, feats, labels,
                       B, gpart);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(const float *gpart, int nrec, int64_t B, float lr, int step, float *master, float *bias,
                           float *m1, float *m2, uint16_t *wbf, float *loss_out, float *grads_out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_mlp_adam, dim3((5186 + 255) / 256), dim3(256), 0, stream, gpart, nrec, B, lr, step, master,
                       bias, m1, m2, wbf, loss_out, grads_out);
    return hipGetLastError();
}

}  // namespace rir
