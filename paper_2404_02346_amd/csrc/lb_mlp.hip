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

// ---------------------------------------------------------------------------
// Training products.  Every product is C (M x N) = A (M x K) B (N x K)^T with
// both operands stored K-contiguous (A row m at A + m s_am, B row n at B + n
// s_bn), so a lane's MFMA fragment (8 consecutive k of one row) is one 16-byte
// load straight into registers:
//   forward  z_l     = a_l W_l^T          A = a_l (B x K_l),     B = W_l (N_l x K_l)
//   errors   e_{l-1} = delta_l W_l        A = delta_l (B x N_l), B = W_l^T (K_l x N_l)
//   weights  dW_l    = delta_l^T a_l      A = delta_l^T (N_l x B), B = a_l^T (K_l x B)
// The forward and error epilogues therefore also write BF16 transposed copies
// (batch-contiguous, rows padded with zeros to a multiple of 64 samples), and
// the optimizer keeps a transposed BF16 mirror of every weight matrix.  The
// weight products have K = batch (4096): K is split into at most kMaxSplit
// chunks so that some 256 workgroups run, each chunk's sum goes to its own
// slot, and finish_kernel adds the slots in chunk order (deterministic).
// Bias gradients (column sums of the FP32 errors) and the loss are summed per
// 64-sample block in the epilogues and finished the same way.
// ---------------------------------------------------------------------------

enum Epi { EPI_FWD = 0, EPI_OUT = 1, EPI_DX = 2, EPI_PART = 3 };
// operand storage: 16-byte BF16 vectors, or elementwise BF16 / FP32 with any strides
enum OpMode { OP_VEC = 0, OP_BF16 = 1, OP_F32 = 2 };

constexpr int kTile = 64;      // 64 x 64 output tile per workgroup, 4 wavefronts of 32 x 32
constexpr int kStepsAhead = 8; // K steps of 32 whose fragments are loaded before use
constexpr int kMaxSplit = 16;  // K chunks of a weight-gradient product
constexpr int kMaxTrainBatch = 1 << 24;  // training batch limit (workspace about 14 KB per sample)

struct GemmNT {
    int M, N, K;       // K: true length (elementwise operands mask k >= K)
    int Kp;            // K rounded up to 32: the loop bound (vector operands read zeros there)
    int k_chunk;       // K range of chunk z: [z k_chunk, min(Kp, (z + 1) k_chunk))
    int tiles_m, tiles_n, chunks;  // grid of this product: tile (mt, nt) of chunk z
    const void *A;     // A(m, k) = A[m s_am + k s_ak]  (s_ak = 1 for OP_VEC)
    int64_t s_am, s_ak;
    const void *B;     // B(n, k) = B[n s_bn + k s_bk]  (s_bk = 1 for OP_VEC)
    int64_t s_bn, s_bk;
    int epi;
    const float *bias;   // N (EPI_FWD, EPI_OUT)
    float *outf;         // EPI_FWD: z (row stride ldo); EPI_OUT: y; EPI_PART: chunk z at outf + z M ldo
    int64_t ldo;
    uint16_t *outb;      // BF16 row-major output (EPI_FWD: GELU(z); EPI_DX: error), may be NULL
    uint16_t *outt;      // BF16 transposed output outt[n ldt + m] for m < m_pad (zero for m >= M)
    int64_t ldt;
    int m_pad;
    const float *zprev;  // EPI_DX: pre-activation of the layer below (row stride ldo)
    const float *target; // EPI_OUT: targets (training), or NULL (inference)
    float inv_b2;        // EPI_OUT: 2 / batch
    float *colpart;      // EPI_OUT (training), EPI_DX: per-64-row column sums [mt][N]
    double *losspart;    // EPI_OUT (training): per-64-row sum of squared errors [mt]
};

template <int MODE>
__device__ inline s16x8 load_frag(const void *base, int64_t s_row, int64_t s_k, int row, int nrows,
                                  int k, int K)
{
    s16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    if (row >= nrows) return v;
    if constexpr (MODE == OP_VEC) {
        v = *reinterpret_cast<const s16x8 *>(static_cast<const uint16_t *>(base) +
                                             (int64_t)row * s_row + k);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (k + e < K) {
                const int64_t o = (int64_t)row * s_row + (int64_t)(k + e) * s_k;
                if constexpr (MODE == OP_BF16)
                    v[e] = (short)static_cast<const uint16_t *>(base)[o];
                else
                    v[e] = (short)to_bf16(static_cast<const float *>(base)[o]);
            }
        }
    }
    return v;
}

// one 64 x 64 output tile (mt, nt) of K chunk kz
template <int AM, int BM>
__device__ inline void gemm_tile(const GemmNT &g, int mt, int nt, int kz, float (*red)[kTile],
                                 double *lred)
{
    const int m_blk = mt * kTile, n_blk = nt * kTile;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int kl = 8 * (lane >> 4);
    const int k_beg = kz * g.k_chunk;
    const int k_end = min(g.Kp, k_beg + g.k_chunk);
    int ra[2], rb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        ra[i] = m_blk + wm * 32 + i * 16 + (lane & 15);
        rb[i] = n_blk + wn * 32 + i * 16 + (lane & 15);
    }
    // lane holds column rb[j], rows mrow + 16 i + v (v = 0..3) of the result
    const int mrow = m_blk + wm * 32 + 4 * (lane >> 4);
    // with a bias the sums start from it, as in the fused inference kernel, so that
    // both forwards round every activation identically
    const bool has_bias = g.epi == EPI_FWD || g.epi == EPI_OUT;
    f32x4 acc[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const float b0 = (has_bias && rb[j] < g.N) ? g.bias[rb[j]] : 0.f;
#pragma unroll
        for (int i = 0; i < 2; ++i) acc[i][j] = f32x4{b0, b0, b0, b0};
    }
    // the epilogue's other inputs are fetched before the product, so that their
    // latency overlaps it: z of the layer below (EPI_DX), the targets (EPI_OUT)
    float pre[2][2][4];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = mrow + 16 * i + v;
                float q = 0.f;
                if (g.epi == EPI_DX && m < g.M && rb[j] < g.N) q = g.zprev[(int64_t)m * g.ldo + rb[j]];
                if (g.epi == EPI_OUT && g.target && j == 0 && m < g.M) q = g.target[m];
                pre[j][i][v] = q;
            }

    for (int kb = k_beg; kb < k_end; kb += 32 * kStepsAhead) {
        s16x8 a[kStepsAhead][2], b[kStepsAhead][2];
#pragma unroll
        for (int s = 0; s < kStepsAhead; ++s) {
            const int k = kb + 32 * s;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[s][i] = s16x8{0, 0, 0, 0, 0, 0, 0, 0};
                b[s][i] = s16x8{0, 0, 0, 0, 0, 0, 0, 0};
            }
            if (k < k_end) {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    a[s][i] = load_frag<AM>(g.A, g.s_am, g.s_ak, ra[i], g.M, k + kl, g.K);
                    b[s][i] = load_frag<BM>(g.B, g.s_bn, g.s_bk, rb[i], g.N, k + kl, g.K);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < kStepsAhead; ++s) {
            if (kb + 32 * s < k_end) {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf16x8, a[s][i]), __builtin_bit_cast(bf16x8, b[s][j]),
                            acc[i][j], 0, 0, 0);
            }
        }
    }

    if (g.epi == EPI_PART) {
        float *o = g.outf + (int64_t)kz * g.M * g.ldo;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = mrow + 16 * i + v;
                    if (m < g.M && rb[j] < g.N) o[(int64_t)m * g.ldo + rb[j]] = acc[i][j][v];
                }
        return;
    }
    float csum[2] = {0.f, 0.f};
    double lsum = 0.0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int n = rb[j];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            float tv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = mrow + 16 * i + v;
                const bool ok = m < g.M && n < g.N;
                const float c = acc[i][j][v];
                const int64_t o = (int64_t)m * g.ldo + n;
                float t = 0.f;
                if (g.epi == EPI_FWD) {
                    if (ok) {
                        t = gelu(c);
                        g.outf[o] = c;
                        g.outb[o] = to_bf16(t);
                    }
                } else if (g.epi == EPI_OUT) {
                    if (ok) {
                        g.outf[m] = c;
                        if (g.target) {
                            const float e = c - pre[0][i][v];
                            t = e * g.inv_b2;
                            lsum += (double)e * (double)e;
                            csum[j] += t;
                        }
                    }
                } else {  // EPI_DX
                    if (ok) {
                        t = c * gelu_d(pre[j][i][v]);
                        if (g.outb) g.outb[o] = to_bf16(t);
                        csum[j] += t;
                    }
                }
                tv[v] = t;
            }
            const int m0 = mrow + 16 * i;
            if (g.outt && n < g.N && m0 < g.m_pad) {
                const uint32_t lo = to_bf16x2(tv[0], tv[1]), hi = to_bf16x2(tv[2], tv[3]);
                *reinterpret_cast<uint2 *>(g.outt + (int64_t)n * g.ldt + m0) = make_uint2(lo, hi);
            }
        }
    }
    if (g.colpart) {
        // column sums over this block's 64 rows: a lane's 8 rows in order, then the four
        // lane groups of a column (butterfly), then the two wavefront rows
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            float s = csum[j];
            s += __shfl_xor(s, 16);
            s += __shfl_xor(s, 32);
            if (lane < 16) red[wm][wn * 32 + j * 16 + lane] = s;
        }
        if (g.losspart) {
            lsum += __shfl_xor(lsum, 16);
            lsum += __shfl_xor(lsum, 32);
            if (wn == 0 && lane == 0) lred[wm] = lsum;
        }
        __syncthreads();
        if (threadIdx.x < kTile) {
            const int n = n_blk + threadIdx.x;
            if (n < g.N)
                g.colpart[(int64_t)mt * g.N + n] = red[0][threadIdx.x] + red[1][threadIdx.x];
        }
        if (g.losspart && threadIdx.x == 0) g.losspart[mt] = lred[0] + lred[1];
    }
}

// One launch runs two independent products: blocks [0, n0) take tiles of g0, the
// rest tiles of g1 (a single product passes n0 = its block count).  Block b of a
// product is tile (b mod tiles_m, (b / tiles_m) mod tiles_n) of chunk
// b / (tiles_m tiles_n).
template <int AM0, int BM0, int AM1, int BM1>
__global__ void __launch_bounds__(256) gemm_nt_kernel(GemmNT g0, GemmNT g1, int n0)
{
    __shared__ float red[2][kTile];
    __shared__ double lred[2];
    const int b = blockIdx.x;
    if (b < n0) {
        gemm_tile<AM0, BM0>(g0, b % g0.tiles_m, (b / g0.tiles_m) % g0.tiles_n,
                            b / (g0.tiles_m * g0.tiles_n), red, lred);
    } else {
        const int c = b - n0;
        gemm_tile<AM1, BM1>(g1, c % g1.tiles_m, (c / g1.tiles_m) % g1.tiles_n,
                            c / (g1.tiles_m * g1.tiles_n), red, lred);
    }
}

struct FinishArgs {
    float *p, *g, *m, *v;
    uint16_t *pb, *pbT;
    const float *wpart[kLayers];  // chunk sums of dW_l: [chunk][N_l][K_l]
    int wsplit[kLayers];
    const float *bpart[kLayers];  // block sums of db_l: [block][N_l]
    int nblk;
    const double *losspart;
    double *loss;
    int B;
    int adam;
    float lr, b1, b2, eps, c1, c2;
};

// gradient of every parameter from its partial sums (chunk or block order), the
// loss, and (adam != 0) one Adam step with the BF16 mirrors W and W^T refreshed
__global__ void __launch_bounds__(256) finish_kernel(FinishArgs f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        double s = 0.0;
        for (int b0 = 0; b0 < f.nblk; b0 += 16) {
            double q[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) q[u] = b0 + u < f.nblk ? f.losspart[b0 + u] : 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (b0 + u < f.nblk) s += q[u];
        }
        *f.loss = s / (double)f.B;
    }
    if (i >= kParams) return;
    int l = 0;
#pragma unroll
    for (int q = 1; q < kLayers; ++q)
        if (i >= param_offset_w(q)) l = q;
    int K = kDims[0], N = kDims[1], S = f.wsplit[0];
    const float *wp = f.wpart[0], *bp = f.bpart[0];
#pragma unroll
    for (int q = 1; q < kLayers; ++q)
        if (l == q) {
            K = kDims[q];
            N = kDims[q + 1];
            S = f.wsplit[q];
            wp = f.wpart[q];
            bp = f.bpart[q];
        }
    const int local = i - param_offset_w(l);
    const bool weight = local < N * K;
    // every partial is loaded before the first add (a runtime-length loop would wait
    // for each load in turn); the sums still run in chunk or block order
    float gi = 0.f;
    if (weight) {
        float q[kMaxSplit];
#pragma unroll
        for (int s = 0; s < kMaxSplit; ++s) q[s] = s < S ? wp[(int64_t)s * N * K + local] : 0.f;
#pragma unroll
        for (int s = 0; s < kMaxSplit; ++s)
            if (s < S) gi += q[s];
    } else {
        const int n = local - N * K;
        for (int b0 = 0; b0 < f.nblk; b0 += 16) {
            float q[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) q[u] = b0 + u < f.nblk ? bp[(int64_t)(b0 + u) * N + n] : 0.f;
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (b0 + u < f.nblk) gi += q[u];
        }
    }
    f.g[i] = gi;
    if (!f.adam) return;
    const float mi = f.b1 * f.m[i] + (1.f - f.b1) * gi;
    const float vi = f.b2 * f.v[i] + (1.f - f.b2) * gi * gi;
    f.m[i] = mi;
    f.v[i] = vi;
    const float pi = f.p[i] - f.lr * (mi / f.c1) / (sqrtf(vi / f.c2) + f.eps);
    f.p[i] = pi;
    const uint16_t pbi = to_bf16(pi);
    f.pb[i] = pbi;
    if (weight) f.pbT[param_offset_w(l) + (local % K) * N + local / K] = pbi;
}

// BF16 mirrors W and W^T of the FP32 parameters (after they are set)
__global__ void mirror_kernel(const float *p, uint16_t *pb, uint16_t *pbT)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kParams) return;
    const uint16_t b = to_bf16(p[i]);
    pb[i] = b;
    int l = 0;
#pragma unroll
    for (int q = 1; q < kLayers; ++q)
        if (i >= param_offset_w(q)) l = q;
    int K = kDims[0], N = kDims[1];
#pragma unroll
    for (int q = 1; q < kLayers; ++q)
        if (l == q) {
            K = kDims[q];
            N = kDims[q + 1];
        }
    const int local = i - param_offset_w(l);
    if (local < N * K) pbT[param_offset_w(l) + (local % K) * N + local / K] = b;
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
inline int round_up(int v, int q) { return (v + q - 1) / q * q; }

struct Layout {
    size_t p, g, m, v, pb, pbT;      // parameters, gradients, Adam moments, BF16 mirrors W and W^T
    size_t act[kLayers];             // BF16 activations a_1..a_4, row-major (B x 256); act[0] unused
    size_t actT[kLayers];            // the same transposed (256 x ldt)
    size_t z[kLayers];               // FP32 pre-activations z_0..z_3 (B x 256)
    size_t y;                        // FP32 output (B)
    size_t drm[2], dT[2];            // BF16 errors of the hidden layers, row-major and transposed
    size_t d4;                       // BF16 error of the output layer (ldt)
    size_t wpart[kLayers];           // FP32 chunk sums of the weight gradients
    size_t bpart[kLayers];           // FP32 block sums of the bias gradients
    size_t lpart;                    // FP64 block sums of the squared errors
    size_t loss;                     // FP64
    size_t total;
    int64_t ldt;                     // row stride of the transposed copies (max batch padded to 64)
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
    const size_t Bp = (size_t)round_up(Bm, kTile);
    const size_t nblk = Bp / kTile;
    L.ldt = (int64_t)Bp;
    L.p = take(4 * (size_t)kParams);
    L.g = take(4 * (size_t)kParams);
    L.m = take(4 * (size_t)kParams);
    L.v = take(4 * (size_t)kParams);
    L.pb = take(2 * (size_t)kParams);
    L.pbT = take(2 * (size_t)kParams);
    for (int l = 0; l < kLayers; ++l) {
        L.act[l] = take(2 * (size_t)kHidden * Bm);
        L.actT[l] = take(2 * (size_t)kHidden * Bp);
        L.z[l] = take(4 * (size_t)kHidden * Bm);
    }
    L.y = take(4 * (size_t)Bm);
    for (int i = 0; i < 2; ++i) {
        L.drm[i] = take(2 * (size_t)kHidden * Bm);
        L.dT[i] = take(2 * (size_t)kHidden * Bp);
    }
    L.d4 = take(2 * Bp);
    for (int l = 0; l < kLayers; ++l) {
        const size_t nk = (size_t)kDims[l + 1] * kDims[l];
        L.wpart[l] = take(4 * nk * kMaxSplit);
        L.bpart[l] = take(4 * (size_t)kDims[l + 1] * nblk);
    }
    L.lpart = take(8 * nblk);
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

GemmNT base_args()
{
    GemmNT g;
    std::memset(&g, 0, sizeof g);
    return g;
}

// K split into chunks of whole 32-steps: at most `want` chunks, equal but the last
int split_chunks(int steps, int want, int *per_out = nullptr)
{
    want = std::max(1, std::min(want, steps));
    const int per = (steps + want - 1) / want;
    if (per_out) *per_out = per;
    return (steps + per - 1) / per;
}

// the grid of one product: ceil(M/64) x ceil(N/64) tiles, split_chunks(., want) K chunks
void plan_gemm(GemmNT &g, int want)
{
    g.Kp = round_up(g.K, 32);
    int per = 0;
    g.chunks = split_chunks(g.Kp / 32, want, &per);
    g.k_chunk = 32 * per;
    g.tiles_m = (g.M + kTile - 1) / kTile;
    g.tiles_n = (g.N + kTile - 1) / kTile;
}

int blocks_of(const GemmNT &g) { return g.tiles_m * g.tiles_n * g.chunks; }

// one product C = A B^T in one launch
template <int AM, int BM>
void gemm(const lb_mlp *h, GemmNT g, int want = 1)
{
    plan_gemm(g, want);
    const int n = blocks_of(g);
    hipLaunchKernelGGL((gemm_nt_kernel<AM, BM, AM, BM>), dim3(n), dim3(256), 0, h->stream, g, g, n);
}

// two independent products in one launch
template <int AM0, int BM0, int AM1, int BM1>
void gemm2(const lb_mlp *h, GemmNT g0, int want0, GemmNT g1, int want1)
{
    plan_gemm(g0, want0);
    plan_gemm(g1, want1);
    const int n0 = blocks_of(g0), n1 = blocks_of(g1);
    hipLaunchKernelGGL((gemm_nt_kernel<AM0, BM0, AM1, BM1>), dim3(n0 + n1), dim3(256), 0,
                       h->stream, g0, g1, n0);
}

// requested K chunks of a weight-gradient product: about 256 workgroups in all,
// each chunk at least 4 steps of 32, at most kMaxSplit chunks
int weight_split(int l, int B)
{
    const int tiles = ((kDims[l + 1] + kTile - 1) / kTile) * ((kDims[l] + kTile - 1) / kTile);
    const int steps = round_up(B, 32) / 32;
    const int want = std::min(kMaxSplit, std::max(1, 256 / tiles));
    return std::max(1, std::min(want, steps / 4));
}

// forward for B samples; keeps activations (both layouts) and pre-activations for
// the backward pass.  With targets t the output layer also forms the output error
// 2 (y - t) / B, its block sums and the blocks' squared errors.
void forward(const lb_mlp *h, const float *x, int B, float *y, const float *t)
{
    const Layout &L = h->L;
    const int m_pad = round_up(B, kTile);
    for (int l = 0; l < kLayers; ++l) {
        const int K = kDims[l], N = kDims[l + 1];
        GemmNT g = base_args();
        g.M = B;
        g.N = N;
        g.K = K;
        g.B = h->at<uint16_t>(L.pb) + param_offset_w(l);  // W_l (N x K)
        g.s_bn = K;
        g.s_bk = 1;
        g.bias = h->at<float>(L.p) + param_offset_b(l);
        g.ldo = N;
        g.ldt = L.ldt;
        g.m_pad = m_pad;
        if (l < kLayers - 1) {
            g.epi = EPI_FWD;
            g.outf = h->at<float>(L.z[l]);
            g.outb = h->at<uint16_t>(L.act[l + 1]);
            g.outt = h->at<uint16_t>(L.actT[l + 1]);
        } else {
            g.epi = EPI_OUT;
            g.outf = y;
            if (t) {
                g.target = t;
                g.inv_b2 = 2.0f / (float)B;
                g.outt = h->at<uint16_t>(L.d4);
                g.colpart = h->at<float>(L.bpart[l]);
                g.losspart = h->at<double>(L.lpart);
            }
        }
        if (l == 0) {
            g.A = x;  // FP32 input, converted to BF16 on load
            g.s_am = K;
            g.s_ak = 1;
            gemm<OP_F32, OP_BF16>(h, g);
        } else {
            g.A = h->at<uint16_t>(L.act[l]);
            g.s_am = K;
            g.s_ak = 1;
            gemm<OP_VEC, OP_VEC>(h, g);
        }
    }
}

// weight gradients (chunk sums) of every layer and block sums of the errors.  The
// weight gradient of layer l and the error of layer l - 1 both read only layer
// l's error, so they share one launch.
void backward(const lb_mlp *h, const float *x, int B)
{
    const Layout &L = h->L;
    const int m_pad = round_up(B, kTile);
    int cur = 0;
    for (int l = kLayers - 1; l >= 0; --l) {
        const int K = kDims[l], N = kDims[l + 1];
        // this layer's error: transposed (N x ldt) and row-major (B x N)
        const uint16_t *eT = (l == kLayers - 1) ? h->at<uint16_t>(L.d4) : h->at<uint16_t>(L.dT[cur]);
        const uint16_t *erm = (l == kLayers - 1) ? h->at<uint16_t>(L.d4) : h->at<uint16_t>(L.drm[cur]);
        // dW_l (N x K) = delta_l^T a_l
        GemmNT g = base_args();
        g.M = N;
        g.N = K;
        g.K = B;
        g.A = eT;
        g.s_am = L.ldt;
        g.s_ak = 1;
        g.epi = EPI_PART;
        g.outf = h->at<float>(L.wpart[l]);
        g.ldo = K;
        const int split = weight_split(l, B);
        if (l == 0) {
            g.B = x;  // FP32 input: B(n, k) = x[k][n]
            g.s_bn = 1;
            g.s_bk = kIn;
            gemm<OP_VEC, OP_F32>(h, g, split);
            break;
        }
        g.B = h->at<uint16_t>(L.actT[l]);
        g.s_bn = L.ldt;
        g.s_bk = 1;
        // delta_{l-1} (B x K) = (delta_l W_l) * gelu'(z_{l-1}), with its block column sums
        GemmNT d = base_args();
        d.M = B;
        d.N = K;
        d.K = N;
        d.A = erm;
        d.s_am = N;
        d.s_ak = 1;
        d.B = h->at<uint16_t>(L.pbT) + param_offset_w(l);  // W_l^T (K x N)
        d.s_bn = N;
        d.s_bk = 1;
        d.epi = EPI_DX;
        d.zprev = h->at<float>(L.z[l - 1]);
        d.ldo = K;
        d.outb = (l > 1) ? h->at<uint16_t>(L.drm[1 - cur]) : nullptr;
        d.outt = h->at<uint16_t>(L.dT[1 - cur]);
        d.ldt = L.ldt;
        d.m_pad = m_pad;
        d.colpart = h->at<float>(L.bpart[l - 1]);
        if (N < 32)
            gemm2<OP_VEC, OP_VEC, OP_BF16, OP_BF16>(h, g, split, d, 1);  // the output layer's K = 1
        else
            gemm2<OP_VEC, OP_VEC, OP_VEC, OP_VEC>(h, g, split, d, 1);
        cur = 1 - cur;
    }
}

FinishArgs finish_args(const lb_mlp *h, int B)
{
    const Layout &L = h->L;
    FinishArgs f;
    std::memset(&f, 0, sizeof f);
    f.p = h->at<float>(L.p);
    f.g = h->at<float>(L.g);
    f.m = h->at<float>(L.m);
    f.v = h->at<float>(L.v);
    f.pb = h->at<uint16_t>(L.pb);
    f.pbT = h->at<uint16_t>(L.pbT);
    for (int l = 0; l < kLayers; ++l) {
        f.wpart[l] = h->at<float>(L.wpart[l]);
        f.wsplit[l] = split_chunks(round_up(B, 32) / 32, weight_split(l, B));
        f.bpart[l] = h->at<float>(L.bpart[l]);
    }
    f.nblk = round_up(B, kTile) / kTile;
    f.losspart = h->at<double>(L.lpart);
    f.loss = h->at<double>(L.loss);
    f.B = B;
    return f;
}

void finish(const lb_mlp *h, const FinishArgs &f)
{
    hipLaunchKernelGGL(finish_kernel, dim3((kParams + 255) / 256), dim3(256), 0, h->stream, f);
}

int check_batch(const lb_mlp *h, int B)
{
    if (!h) return lbw_fail_msg(LB_EINVAL, "handle is NULL");
    if (B < 1 || B > h->Bm) return lbw_fail_msg(LB_EINVAL, "batch outside 1 .. max_batch");
    return LB_OK;
}

int check_adam(float lr, float beta1, float beta2, float eps)
{
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return lbw_fail_msg(LB_EINVAL, "bad Adam hyper-parameters");
    return LB_OK;
}

// one Adam step (the caller has checked the arguments)
void adam_step(lb_mlp *h, const float *x, const float *t, int B, float lr, float beta1,
               float beta2, float eps)
{
    forward(h, x, B, h->at<float>(h->L.y), t);
    backward(h, x, B);
    h->step++;
    FinishArgs f = finish_args(h, B);
    f.adam = 1;
    f.lr = lr;
    f.b1 = beta1;
    f.b2 = beta2;
    f.eps = eps;
    f.c1 = 1.f - std::pow(beta1, (float)h->step);
    f.c2 = 1.f - std::pow(beta2, (float)h->step);
    finish(h, f);
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
                       h->at<float>(L.p), h->at<uint16_t>(L.pb), h->at<uint16_t>(L.pbT));
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
                       h->at<float>(h->L.p), h->at<uint16_t>(h->L.pb), h->at<uint16_t>(h->L.pbT));
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
    forward(h, dev_x, B, dev_y, nullptr);
    MLP_TRY(hipGetLastError());
    return LB_OK;
}

int lb_mlp_grad(lb_mlp *h, const float *dev_x, const float *dev_t, int32_t B, float *host_grads,
                double *host_loss)
{
    int st = check_batch(h, B);
    if (st) return st;
    if (!dev_x || !dev_t || !host_grads) return lbw_fail_msg(LB_EINVAL, "NULL argument");
    forward(h, dev_x, B, h->at<float>(h->L.y), dev_t);
    backward(h, dev_x, B);
    finish(h, finish_args(h, B));
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
    if ((st = check_adam(lr, beta1, beta2, eps))) return st;
    adam_step(h, dev_x, dev_t, B, lr, beta1, beta2, eps);
    MLP_TRY(hipGetLastError());
    return LB_OK;
}

int lb_mlp_train_steps(lb_mlp *h, const float *dev_x, const float *dev_t, int32_t B,
                       int32_t n_steps, const float *host_lr, float beta1, float beta2, float eps)
{
    int st = check_batch(h, B);
    if (st) return st;
    if (!dev_x || !dev_t || n_steps < 0 || (n_steps > 0 && !host_lr))
        return lbw_fail_msg(LB_EINVAL, "bad argument");
    for (int s = 0; s < n_steps; ++s)
        if ((st = check_adam(host_lr[s], beta1, beta2, eps))) return st;
    for (int s = 0; s < n_steps; ++s) adam_step(h, dev_x, dev_t, B, host_lr[s], beta1, beta2, eps);
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
