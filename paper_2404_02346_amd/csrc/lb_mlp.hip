// MLP surrogate of the radiation force: BF16 MFMA forward and backward
// kernels, Adam, and the C ABI of include/lb_mlp.h.
//
// Matrix products use v_mfma_f32_16x16x32_bf16: per 64-lane wavefront,
// A (16 x 32) has lane l holding row l % 16, k = 8 (l / 16) .. + 7;
// B (32 x 16) has lane l holding column l % 16, the same k range;
// D (16 x 16) has lane l holding column l % 16, rows 4 (l / 16) .. + 3.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/lb_mlp.h"
#include "../../include/lb_wave.h"

int lbw_fail_msg(int code, const char *msg);  // lb_wave.hip

namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kLayers = 5;
constexpr int kIn = 4;
constexpr int kDims[kLayers + 1] = {kIn, 256, 256, 256, 256, 1};
constexpr int kHidden = 256;

constexpr int param_offset_w(int l)
{
    int off = 0;
    for (int i = 0; i < l; ++i) off += kDims[i + 1] * kDims[i] + kDims[i + 1];
    return off;
}
constexpr int param_offset_b(int l) { return param_offset_w(l) + kDims[l + 1] * kDims[l]; }
constexpr int kParams = param_offset_w(kLayers);

__device__ inline float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
// FP32 -> BF16, round to nearest even (one hardware conversion on gfx950)
__device__ inline uint16_t to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
// two at once: a in the low half, b in the high half.  The pair is converted as
// one vector and split by the caller with shifts: reading a single element of a
// BF16 vector is lowered wrongly by this compiler (element 1 reads element 0).
__device__ inline uint32_t to_bf16x2(float a, float b)
{
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2{a, b}), bf16x2));
}

// Standard normal distribution in the tail, h = Phi(-|z|) = (1 - erf(|z| / sqrt 2)) / 2,
// from Hastings' rational-exponential form of erf (Abramowitz & Stegun 7.1.26,
// |error| <= 1.5e-7): for x >= 0, 1 - erf(x) ~ t (a1 + t (a2 + t (a3 + t (a4 + t a5))))
// exp(-x^2), t = 1 / (1 + p x).  Here x = |z| / sqrt 2, with 1/sqrt 2 folded into p and
// the factor 1/2 into the a_i.  In FP32 h is within 3e-7 of Phi(-|z|); e = exp(-z^2 / 2)
// is returned for the derivative.  About a dozen instructions against some 35 for the
// library erf, which evaluates both of its branches.
__device__ inline float normal_tail(float z, float &e)
{
    const float t = __builtin_amdgcn_rcpf(fmaf(0.23164188826636f, fabsf(z), 1.0f));
    float q = fmaf(t, 0.5307027145f, -0.7265760135f);
    q = fmaf(t, q, 0.7107068705f);
    q = fmaf(t, q, -0.142248368f);
    q = fmaf(t, q, 0.127414796f);
    e = __builtin_amdgcn_exp2f(z * (z * -0.72134752044448f));  // exp(-z^2 / 2)
    return (q * t) * e;
}

// max(z, 0) as one instruction (the compiler's fmaxf first quiets a possible
// signalling NaN with a second one; a NaN z still gives a NaN GELU below)
__device__ inline float relu(float z)
{
    float r;
    asm("v_max_f32 %0, 0, %1" : "=v"(r) : "v"(z));
    return r;
}

// exact GELU g(z) = z Phi(z) = max(z, 0) - |z| Phi(-|z|), and its derivative
// g'(z) = Phi(z) + z phi(z)
__device__ inline float gelu(float z)
{
    float e;
    return fmaf(-fabsf(z), normal_tail(z, e), relu(z));
}
__device__ inline float gelu_d(float z)
{
    float e;
    const float h = normal_tail(z, e);
    return fmaf(z * 0.39894228040143268f, e, z >= 0.0f ? 1.0f - h : h);
}

enum Epi { EPI_BIAS_GELU = 0, EPI_BIAS = 1, EPI_STORE = 2, EPI_GELU_BWD = 3 };

struct GemmArgs {
    int M, N, K;
    const uint16_t *A;  // A(m, k) = A[m * sam + k * sak]
    int64_t sam, sak;
    const uint16_t *B;  // B(k, n) = B[k * sbk + n * sbn]
    int64_t sbk, sbn;
    int epi;
    const float *bias;   // N (EPI_BIAS_GELU, EPI_BIAS)
    float *outf;         // FP32 output, row stride ldo
    int64_t ldo;
    uint16_t *outb;      // BF16 output (EPI_BIAS_GELU, EPI_GELU_BWD), row stride ldo
    const float *zprev;  // pre-activation for GELU' (EPI_GELU_BWD), row stride ldo
};

constexpr int TM = 64, TN = 64, TK = 32, LDK = TK + 8;

// C (M x N) = A (M x K) B (K x N), 64 x 64 per block, 4 wavefronts of 32 x 32
// (2 x 2 MFMA tiles each), K in steps of 32 through LDS; then the epilogue.
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[TM][LDK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][LDK];
    // M (up to the batch) on x, whose grid dimension is the large one; N (<= 256) on y
    const int m_blk = blockIdx.x * TM, n_blk = blockIdx.y * TN;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    // with a bias the sums start from it, as in the fused inference kernel, so that
    // both forwards round every activation identically
    const bool has_bias = g.epi == EPI_BIAS_GELU || g.epi == EPI_BIAS;
    f32x4 acc[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int n = n_blk + wn * 32 + j * 16 + (lane & 15);
        const float b0 = (has_bias && n < g.N) ? g.bias[n] : 0.f;
#pragma unroll
        for (int i = 0; i < 2; ++i) acc[i][j] = f32x4{b0, b0, b0, b0};
    }

    for (int k0 = 0; k0 < g.K; k0 += TK) {
#pragma unroll
        for (int e = 0; e < (TM * TK) / 256; ++e) {
            const int idx = tid + 256 * e;
            const int r = idx >> 5, kk = idx & 31;
            const int k = k0 + kk;
            const int m = m_blk + r, n = n_blk + r;
            As[r][kk] = (m < g.M && k < g.K) ? g.A[(int64_t)m * g.sam + (int64_t)k * g.sak] : 0;
            Bs[r][kk] = (n < g.N && k < g.K) ? g.B[(int64_t)k * g.sbk + (int64_t)n * g.sbn] : 0;
        }
        __syncthreads();
        const int kk = 8 * (lane >> 4);
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int row = wm * 32 + i * 16 + (lane & 15);
            af[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const s16x8 *>(&As[row][kk]));
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = wn * 32 + j * 16 + (lane & 15);
            bfr[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const s16x8 *>(&Bs[col][kk]));
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m_blk + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
                const int n = n_blk + wn * 32 + j * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                const float c = acc[i][j][v];
                const int64_t o = (int64_t)m * g.ldo + n;
                switch (g.epi) {
                case EPI_BIAS_GELU:
                    g.outf[o] = c;
                    g.outb[o] = to_bf16(gelu(c));
                    break;
                case EPI_BIAS: g.outf[o] = c; break;
                case EPI_STORE: g.outf[o] = c; break;
                default: {
                    const float d = c * gelu_d(g.zprev[o]);
                    g.outf[o] = d;
                    g.outb[o] = to_bf16(d);
                }
                }
            }
}

__global__ void to_bf16_kernel(const float *x, uint16_t *y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = to_bf16(x[i]);
}

// delta = 2 (y - t) / B (FP32 and BF16), loss = sum (y - t)^2 / B in FP64 (one block)
__global__ void __launch_bounds__(256) loss_kernel(const float *y, const float *t, int B,
                                                   float *df, uint16_t *db, double *loss)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < B; b += 256) {
        const float e = y[b] - t[b];
        const float d = 2.0f * e / (float)B;
        df[b] = d;
        db[b] = to_bf16(d);
        s += (double)e * (double)e;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (double)B;
}

// db[n] = sum_b delta[b, n] in two deterministic passes.  Pass 1: block
// (s, cg) (chunk s on x, the long grid dimension) sums rows 256 s .. 256 s + 255
// of columns 64 cg .. 64 cg + 63;
// thread (c, g) takes rows g, g + 4, ... of column c, then the four row
// groups are added in order.  Pass 2: partials added in chunk order.
constexpr int kColRows = 256;
constexpr int kMaxTrainBatch = 1 << 24;  // training batch limit (workspace about 11 KB per sample)
__global__ void __launch_bounds__(256) colsum_part_kernel(const float *delta, int B, int N,
                                                          float *part)
{
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int n = blockIdx.y * 64 + c;
    const int b0 = blockIdx.x * kColRows;
    const int b1 = min(b0 + kColRows, B);
    float s = 0.f;
    if (n < N)
        for (int b = b0 + g; b < b1; b += 4) s += delta[(int64_t)b * N + n];
    red[g][c] = s;
    __syncthreads();
    if (g == 0 && n < N)
        part[(int64_t)blockIdx.x * N + n] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

__global__ void colsum_final_kernel(const float *part, int n_chunks, int N, float *db)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int k = 0; k < n_chunks; ++k) s += part[(int64_t)k * N + n];
    db[n] = s;
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, uint16_t *pb, int n,
                            float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    pb[i] = to_bf16(pi);
}

__global__ void mirror_kernel(const float *p, uint16_t *pb, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pb[i] = to_bf16(p[i]);
}

__global__ void zero_f32_kernel(float *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

__global__ void activation_kernel(const float *z, int64_t n, int derivative, float *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = derivative ? gelu_d(z[i]) : gelu(z[i]);
}

// one MFMA tile with the network's fragment mapping (lane-layout check)
__global__ void __launch_bounds__(64) mfma_probe_kernel(const uint16_t *A, const uint16_t *B,
                                                        float *D)
{
    const int lane = threadIdx.x;
    const int kk = 8 * (lane >> 4);
    s16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = (short)A[(lane & 15) * 32 + kk + e];
        b[e] = (short)B[(kk + e) * 16 + (lane & 15)];
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                  __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) D[(4 * (lane >> 4) + v) * 16 + (lane & 15)] = acc[v];
}

// Fused inference: one block carries kInferRows samples through all layers,
// their activations staying in LDS (BF16, rows padded by 8 elements so that
// the 16-byte fragment reads of 16 consecutive rows spread over the banks).
// Every layer runs on MFMA with the same operand roundings as the training
// forward: BF16 weights and activations, FP32 accumulation and bias, GELU in
// FP32 rounded to BF16.  The first layer's K = 4 is one 32-wide MFMA step with
// the other 28 k zero, and the last layer's single output is column 0 of a
// 16-column tile whose other columns have zero weights.  In the first four
// layers each of the kInferWaves wavefronts owns 256 / kInferWaves output
// columns for all kInferRows rows and its accumulators start at the bias; the
// weight fragments come from global memory (every block reads the same
// 128 KiB per layer, so they are L2 hits) one K step ahead of use.  The LDS
// tile (67.6 KB) allows two blocks per CU.
constexpr int kInferRows = 128;
constexpr int kInferWaves = 8;
constexpr int kInferThreads = 64 * kInferWaves;
// the 1D grid of ceil(B / kInferRows) blocks must hold fewer than 2^32 threads
constexpr int kMaxInferBatch = 1 << 30;
constexpr int kActLd = kHidden + 8;

__global__ void __launch_bounds__(kInferThreads, kInferWaves / 2)
    infer_kernel(const float *__restrict__ x, int B, const float *__restrict__ p,
                 const uint16_t *__restrict__ pb, float *__restrict__ y)
{
    constexpr int RT = kInferRows / 16;        // row tiles
    constexpr int CW = kHidden / kInferWaves;  // columns per wavefront
    constexpr int JT = CW / 16;                // column tiles per wavefront
    constexpr int OT = RT / kInferWaves;       // output-layer row tiles per wavefront
    static_assert(JT >= 1 && OT >= 1, "wavefront count");
    __shared__ __attribute__((aligned(16))) uint16_t act[kInferRows][kActLd];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int kl = 8 * (lane >> 4);  // this lane's k offset within a 32-wide step
    const int64_t row0 = (int64_t)blockIdx.x * kInferRows;
    f32x4 acc[RT][JT];

    auto start = [&](int l) {
        const float *bias = p + param_offset_b(l);
#pragma unroll
        for (int j = 0; j < JT; ++j) {
            const float bn = bias[w * CW + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < RT; ++i) acc[i][j] = f32x4{bn, bn, bn, bn};
        }
    };
    // GELU of the accumulators, rounded to BF16 in pairs, into this wavefront's columns
    auto finish = [&]() {
#pragma unroll
        for (int j = 0; j < JT; ++j) {
            const int col = w * CW + j * 16 + (lane & 15);
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int v = 0; v < 4; v += 2) {
                    const uint32_t g = to_bf16x2(gelu(acc[i][j][v]), gelu(acc[i][j][v + 1]));
                    const int r = i * 16 + 4 * (lane >> 4) + v;
                    act[r][col] = (uint16_t)g;
                    act[r + 1][col] = (uint16_t)(g >> 16);
                }
        }
    };

    // layer 0 (K = kIn): lanes 0..15 carry k = 0..3 of their row (A) or column (B)
    {
        const uint16_t *W = pb + param_offset_w(0);
        start(0);
        bf16x8 bfr[JT];
#pragma unroll
        for (int j = 0; j < JT; ++j) {
            s16x8 b = {0, 0, 0, 0, 0, 0, 0, 0};
            if (lane < 16) {
                const int col = w * CW + j * 16 + lane;
#pragma unroll
                for (int k = 0; k < kIn; ++k) b[k] = (short)W[col * kIn + k];
            }
            bfr[j] = __builtin_bit_cast(bf16x8, b);
        }
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            s16x8 a = {0, 0, 0, 0, 0, 0, 0, 0};
            const int64_t r = row0 + i * 16 + lane;
            if (lane < 16 && r < B) {
#pragma unroll
                for (int k = 0; k < kIn; ++k) a[k] = (short)to_bf16(x[r * kIn + k]);
            }
            const bf16x8 af = __builtin_bit_cast(bf16x8, a);
#pragma unroll
            for (int j = 0; j < JT; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr[j], acc[i][j], 0, 0, 0);
        }
        finish();
        __syncthreads();
    }

    // hidden layers 1 .. kLayers-2 (256 x 256)
    for (int l = 1; l < kLayers - 1; ++l) {
        const uint16_t *W = pb + param_offset_w(l);  // W[n][k], k fastest
        start(l);
        s16x8 bnext[JT];
#pragma unroll
        for (int j = 0; j < JT; ++j) {
            const int col = w * CW + j * 16 + (lane & 15);
            bnext[j] = *reinterpret_cast<const s16x8 *>(W + col * kHidden + kl);
        }
        for (int k0 = 0; k0 < kHidden; k0 += 32) {
            bf16x8 bfr[JT];
#pragma unroll
            for (int j = 0; j < JT; ++j) bfr[j] = __builtin_bit_cast(bf16x8, bnext[j]);
            if (k0 + 32 < kHidden) {
#pragma unroll
                for (int j = 0; j < JT; ++j) {
                    const int col = w * CW + j * 16 + (lane & 15);
                    bnext[j] = *reinterpret_cast<const s16x8 *>(W + col * kHidden + k0 + 32 + kl);
                }
            }
#pragma unroll
            for (int i = 0; i < RT; ++i) {
                const bf16x8 af = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const s16x8 *>(&act[i * 16 + (lane & 15)][k0 + kl]));
#pragma unroll
                for (int j = 0; j < JT; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();  // every wavefront has read this layer's input
        finish();
        __syncthreads();
    }

    // output layer (256 -> 1): wavefront w takes row tiles OT w .. OT w + OT - 1; the B
    // fragment is nonzero only in column 0 (lanes 0, 16, 32, 48)
    {
        const uint16_t *W = pb + param_offset_w(kLayers - 1);
        const float bias = p[param_offset_b(kLayers - 1)];
        f32x4 o[OT];
#pragma unroll
        for (int ii = 0; ii < OT; ++ii) o[ii] = f32x4{bias, bias, bias, bias};
#pragma unroll
        for (int k0 = 0; k0 < kHidden; k0 += 32) {
            s16x8 b = {0, 0, 0, 0, 0, 0, 0, 0};
            if ((lane & 15) == 0) b = *reinterpret_cast<const s16x8 *>(W + k0 + kl);
            const bf16x8 bf = __builtin_bit_cast(bf16x8, b);
#pragma unroll
            for (int ii = 0; ii < OT; ++ii) {
                const int rt = OT * w + ii;
                const bf16x8 af = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const s16x8 *>(&act[rt * 16 + (lane & 15)][k0 + kl]));
                o[ii] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, o[ii], 0, 0, 0);
            }
        }
        if ((lane & 15) == 0) {
#pragma unroll
            for (int ii = 0; ii < OT; ++ii)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t r = row0 + (OT * w + ii) * 16 + 4 * (lane >> 4) + v;
                    if (r < B) y[r] = o[ii][v];
                }
        }
    }
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t p, g, m, v, pb;           // parameters, gradients, Adam moments, BF16 mirror
    size_t xb;                       // BF16 input (B x kIn)
    size_t act[kLayers];             // BF16 activations a_1..a_4 (B x 256); act[0] unused
    size_t z[kLayers];               // FP32 pre-activations z_0..z_3 (B x 256)
    size_t y;                        // FP32 output (B)
    size_t df[2], dbf[2];            // FP32 / BF16 errors, ping-pong (B x 256)
    size_t part;                     // FP32 column-sum partials (ceil(B / 256) x 256)
    size_t loss;                     // FP64
    size_t total;
};

Layout plan(int Bm)
{
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.p = take(4 * (size_t)kParams);
    L.g = take(4 * (size_t)kParams);
    L.m = take(4 * (size_t)kParams);
    L.v = take(4 * (size_t)kParams);
    L.pb = take(2 * (size_t)kParams);
    L.xb = take(2 * kIn * (size_t)Bm);
    for (int l = 0; l < kLayers; ++l) {
        L.act[l] = take(2 * (size_t)kHidden * Bm);
        L.z[l] = take(4 * (size_t)kHidden * Bm);
    }
    L.y = take(4 * (size_t)Bm);
    for (int i = 0; i < 2; ++i) {
        L.df[i] = take(4 * (size_t)kHidden * Bm);
        L.dbf[i] = take(2 * (size_t)kHidden * Bm);
    }
    L.part = take(4 * (size_t)kHidden * (((size_t)Bm + kColRows - 1) / kColRows));
    L.loss = take(8);
    L.total = off;
    return L;
}

}  // namespace mlp

using namespace mlp;

struct lb_mlp {
    int Bm = 0;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    Layout L;
    int64_t step = 0;
    template <typename T> T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

namespace {

#define MLP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return lbw_fail_msg(LB_EDEVICE, hipGetErrorString(e_));   \
    } while (0)

void gemm(const lb_mlp *h, const GemmArgs &g)
{
    const dim3 grid((g.M + TM - 1) / TM, (g.N + TN - 1) / TN);
    hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, h->stream, g);
}

GemmArgs base_args() { GemmArgs g; std::memset(&g, 0, sizeof g); return g; }

// forward for B samples; keeps activations and pre-activations for backward
void forward(const lb_mlp *h, const float *x, int B, float *y)
{
    const int64_t nx = kIn * (int64_t)B;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, h->stream,
                       x, h->at<uint16_t>(h->L.xb), nx);
    const uint16_t *a = h->at<uint16_t>(h->L.xb);
    for (int l = 0; l < kLayers; ++l) {
        const int K = kDims[l], N = kDims[l + 1];
        GemmArgs g = base_args();
        g.M = B;
        g.N = N;
        g.K = K;
        g.A = a;
        g.sam = K;
        g.sak = 1;
        g.B = h->at<uint16_t>(h->L.pb) + param_offset_w(l);  // B(k, n) = W[n][k]
        g.sbk = 1;
        g.sbn = K;
        g.bias = h->at<float>(h->L.p) + param_offset_b(l);
        g.ldo = N;
        if (l < kLayers - 1) {
            g.epi = EPI_BIAS_GELU;
            g.outf = h->at<float>(h->L.z[l]);
            g.outb = h->at<uint16_t>(h->L.act[l + 1]);
            a = g.outb;
        } else {
            g.epi = EPI_BIAS;
            g.outf = y;
        }
        gemm(h, g);
    }
}

// loss, gradients of every parameter into L.g
void backward(const lb_mlp *h, const float *t, int B)
{
    float *y = h->at<float>(h->L.y);
    int cur = 0;
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, h->stream, y, t, B,
                       h->at<float>(h->L.df[cur]), h->at<uint16_t>(h->L.dbf[cur]),
                       h->at<double>(h->L.loss));
    for (int l = kLayers - 1; l >= 0; --l) {
        const int K = kDims[l], N = kDims[l + 1];
        const uint16_t *a_in = (l == 0) ? h->at<uint16_t>(h->L.xb) : h->at<uint16_t>(h->L.act[l]);
        const uint16_t *dl = h->at<uint16_t>(h->L.dbf[cur]);
        // dW_l (N x K) = delta_l^T (N x B) a_l (B x K)
        GemmArgs g = base_args();
        g.M = N;
        g.N = K;
        g.K = B;
        g.A = dl;
        g.sam = 1;
        g.sak = N;
        g.B = a_in;
        g.sbk = K;
        g.sbn = 1;
        g.epi = EPI_STORE;
        g.outf = h->at<float>(h->L.g) + param_offset_w(l);
        g.ldo = K;
        gemm(h, g);
        const int n_chunks = (B + kColRows - 1) / kColRows;
        hipLaunchKernelGGL(colsum_part_kernel, dim3(n_chunks, (N + 63) / 64), dim3(256), 0,
                           h->stream, h->at<float>(h->L.df[cur]), B, N, h->at<float>(h->L.part));
        hipLaunchKernelGGL(colsum_final_kernel, dim3((N + 255) / 256), dim3(256), 0, h->stream,
                           h->at<float>(h->L.part), n_chunks, N,
                           h->at<float>(h->L.g) + param_offset_b(l));
        if (l == 0) break;
        // delta_{l-1} (B x K) = (delta_l (B x N) W_l (N x K)) * gelu'(z_{l-1})
        GemmArgs d = base_args();
        d.M = B;
        d.N = K;
        d.K = N;
        d.A = dl;
        d.sam = N;
        d.sak = 1;
        d.B = h->at<uint16_t>(h->L.pb) + param_offset_w(l);  // B(k, n) = W[k][n]
        d.sbk = K;
        d.sbn = 1;
        d.epi = EPI_GELU_BWD;
        d.zprev = h->at<float>(h->L.z[l - 1]);
        d.outf = h->at<float>(h->L.df[1 - cur]);
        d.outb = h->at<uint16_t>(h->L.dbf[1 - cur]);
        d.ldo = K;
        gemm(h, d);
        cur = 1 - cur;
    }
}

int check_batch(const lb_mlp *h, int B)
{
    if (!h) return lbw_fail_msg(LB_EINVAL, "handle is NULL");
    if (B < 1 || B > h->Bm) return lbw_fail_msg(LB_EINVAL, "batch outside 1 .. max_batch");
    return LB_OK;
}

}  // namespace

extern "C" {

int32_t lb_mlp_num_params(void) { return kParams; }

size_t lb_mlp_workspace_bytes(int32_t max_batch)
{
    if (max_batch < 1 || max_batch > kMaxTrainBatch) return 0;
    return plan(max_batch).total;
}

int lb_mlp_create(int32_t max_batch, void *dev_workspace, size_t workspace_bytes, void *hip_stream,
                  lb_mlp **out)
{
    if (!out) return lbw_fail_msg(LB_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_batch < 1 || max_batch > kMaxTrainBatch)
        return lbw_fail_msg(LB_EINVAL, "max_batch must be in 1 .. 2^24");
    Layout L = plan(max_batch);
    if (!dev_workspace || reinterpret_cast<uintptr_t>(dev_workspace) % kAlign)
        return lbw_fail_msg(LB_ENOMEM, "workspace must be 256-byte aligned device memory");
    if (workspace_bytes < L.total) return lbw_fail_msg(LB_ENOMEM, "workspace too small");
    lb_mlp *h = new lb_mlp();
    h->Bm = max_batch;
    h->ws = static_cast<char *>(dev_workspace);
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->L = L;
    const int64_t nz = (int64_t)(L.pb - L.p) / 4;  // parameters, gradients, moments
    hipLaunchKernelGGL(zero_f32_kernel, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, h->stream,
                       h->at<float>(L.p), nz);
    hipLaunchKernelGGL(mirror_kernel, dim3((kParams + 255) / 256), dim3(256), 0, h->stream,
                       h->at<float>(L.p), h->at<uint16_t>(L.pb), kParams);
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        delete h;
        return lbw_fail_msg(LB_EDEVICE, hipGetErrorString(e));
    }
    *out = h;
    return LB_OK;
}

int lb_mlp_destroy(lb_mlp *h)
{
    delete h;
    return LB_OK;
}

int lb_mlp_set_params(lb_mlp *h, const float *host_params)
{
    if (!h || !host_params) return lbw_fail_msg(LB_EINVAL, "NULL argument");
    MLP_TRY(hipMemcpyAsync(h->at<float>(h->L.p), host_params, 4 * (size_t)kParams,
                           hipMemcpyHostToDevice, h->stream));
    for (size_t off : {h->L.m, h->L.v})
        hipLaunchKernelGGL(zero_f32_kernel, dim3((kParams + 255) / 256), dim3(256), 0, h->stream,
                           h->at<float>(off), (int64_t)kParams);
    hipLaunchKernelGGL(mirror_kernel, dim3((kParams + 255) / 256), dim3(256), 0, h->stream,
                       h->at<float>(h->L.p), h->at<uint16_t>(h->L.pb), kParams);
    MLP_TRY(hipGetLastError());
    MLP_TRY(hipStreamSynchronize(h->stream));
    h->step = 0;
    return LB_OK;
}

int lb_mlp_get_params(lb_mlp *h, float *host_params)
{
    if (!h || !host_params) return lbw_fail_msg(LB_EINVAL, "NULL argument");
    MLP_TRY(hipMemcpyAsync(host_params, h->at<float>(h->L.p), 4 * (size_t)kParams,
                           hipMemcpyDeviceToHost, h->stream));
    MLP_TRY(hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_mlp_forward(lb_mlp *h, const float *dev_x, int32_t B, float *dev_y)
{
    if (!h) return lbw_fail_msg(LB_EINVAL, "handle is NULL");
    if (B < 1) return lbw_fail_msg(LB_EINVAL, "batch must be >= 1");
    if (B > kMaxInferBatch) return lbw_fail_msg(LB_EINVAL, "batch above 2^30");
    if (!dev_x || !dev_y) return lbw_fail_msg(LB_EINVAL, "NULL argument");
    const unsigned blocks = (unsigned)(((int64_t)B + kInferRows - 1) / kInferRows);
    hipLaunchKernelGGL(infer_kernel, dim3(blocks), dim3(kInferThreads), 0, h->stream, dev_x, B,
                       h->at<float>(h->L.p), h->at<uint16_t>(h->L.pb), dev_y);
    MLP_TRY(hipGetLastError());
    return LB_OK;
}

int lb_mlp_forward_layered(lb_mlp *h, const float *dev_x, int32_t B, float *dev_y)
{
    int st = check_batch(h, B);
    if (st) return st;
    if (!dev_x || !dev_y) return lbw_fail_msg(LB_EINVAL, "NULL argument");
    forward(h, dev_x, B, dev_y);
    MLP_TRY(hipGetLastError());
    return LB_OK;
}

int lb_mlp_grad(lb_mlp *h, const float *dev_x, const float *dev_t, int32_t B, float *host_grads,
                double *host_loss)
{
    int st = check_batch(h, B);
    if (st) return st;
    if (!dev_x || !dev_t || !host_grads) return lbw_fail_msg(LB_EINVAL, "NULL argument");
    forward(h, dev_x, B, h->at<float>(h->L.y));
    backward(h, dev_t, B);
    MLP_TRY(hipGetLastError());
    MLP_TRY(hipMemcpyAsync(host_grads, h->at<float>(h->L.g), 4 * (size_t)kParams,
                           hipMemcpyDeviceToHost, h->stream));
    if (host_loss)
        MLP_TRY(hipMemcpyAsync(host_loss, h->at<double>(h->L.loss), 8, hipMemcpyDeviceToHost,
                               h->stream));
    MLP_TRY(hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_mlp_train_step(lb_mlp *h, const float *dev_x, const float *dev_t, int32_t B, float lr,
                      float beta1, float beta2, float eps)
{
    int st = check_batch(h, B);
    if (st) return st;
    if (!dev_x || !dev_t) return lbw_fail_msg(LB_EINVAL, "NULL argument");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return lbw_fail_msg(LB_EINVAL, "bad Adam hyper-parameters");
    forward(h, dev_x, B, h->at<float>(h->L.y));
    backward(h, dev_t, B);
    h->step++;
    const float c1 = 1.f - std::pow(beta1, (float)h->step);
    const float c2 = 1.f - std::pow(beta2, (float)h->step);
    hipLaunchKernelGGL(adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, h->stream,
                       h->at<float>(h->L.p), h->at<float>(h->L.g), h->at<float>(h->L.m),
                       h->at<float>(h->L.v), h->at<uint16_t>(h->L.pb), kParams, lr, beta1, beta2,
                       eps, c1, c2);
    MLP_TRY(hipGetLastError());
    return LB_OK;
}

int lb_mlp_last_loss(lb_mlp *h, double *loss)
{
    if (!h || !loss) return lbw_fail_msg(LB_EINVAL, "NULL argument");
    MLP_TRY(hipMemcpyAsync(loss, h->at<double>(h->L.loss), 8, hipMemcpyDeviceToHost, h->stream));
    MLP_TRY(hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_mlp_mfma_probe(const uint16_t *dev_A, const uint16_t *dev_B, float *dev_D, void *hip_stream)
{
    if (!dev_A || !dev_B || !dev_D) return lbw_fail_msg(LB_EINVAL, "NULL argument");
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(hip_stream),
                       dev_A, dev_B, dev_D);
    MLP_TRY(hipGetLastError());
    return LB_OK;
}

int lb_mlp_activation(const float *dev_z, int64_t n, int32_t derivative, float *dev_out,
                      void *hip_stream)
{
    if (n < 0 || (n > 0 && (!dev_z || !dev_out)))
        return lbw_fail_msg(LB_EINVAL, "activation: bad arguments");
    // one thread per value in a 1D grid, whose thread count must fit 32 bits
    if (n > ((int64_t)1 << 31)) return lbw_fail_msg(LB_EINVAL, "activation: n above 2^31");
    if (n == 0) return LB_OK;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(activation_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), dev_z, n, derivative ? 1 : 0, dev_out);
    MLP_TRY(hipGetLastError());
    return LB_OK;
}

}  // extern "C"
