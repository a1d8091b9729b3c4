// mlp_kernels.hip -- kernels of the learned surrogate (gfx950).
//
// The surrogate is a multilayer perceptron 66 -> 512 -> 512 -> 512 -> 2806
// with GELU activations that predicts a coarse 61 x 46 map of a frame: for
// each 20 cm cell, the best exact score among the 5 cm points that a
// re-score of that cell visits.  Its top-64 cells are then re-scored exactly
// at 5 cm.  Weights and
// activations are bfloat16, products accumulate in float32 on the matrix
// cores (v_mfma_f32_16x16x32_bf16); biases, pre-activations, gradients and
// the Adam state are float32.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "mlp_internal.h"

namespace dpps {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(4))) float f32x4_t;

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest even
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float x)
{
    float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
    float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
    return cdf + x * pdf;
}

// ---------------------------------------------------------------------------
// GEMM: C[M][N] = sum_k A(m, k) B(k, n), bf16 operands, f32 accumulation.
// A(m, k) = A[m*lda + k] when A_K (k contiguous), else A[k*lda + m].
// B(k, n) = B[n*ldb + k] when B_K (k contiguous), else B[k*ldb + n].
// M, N, K are multiples of 8 (vectors of 8 never straddle an edge).
// Block tile BM x BN (128 x 128 or 64 x 64), K step 32, 256 threads: four
// waves in a 2 x 2 arrangement, each owning a (BM/2) x (BN/2) quarter as
// (BM/32) x (BN/32) MFMA tiles of 16 x 16 (v_mfma_f32_16x16x32_bf16).  The
// next K step is fetched into registers while the current one multiplies
// out of LDS, into the other of two LDS buffers, one barrier per step.
// blockIdx.z splits K into slices of g.k_slice; with EPI_PARTIAL slice z
// writes its partial product to Cf + z * M * ldc (summed by gemm_reduce).
// ---------------------------------------------------------------------------
#define GK 32
#define LDSK (GK + 8)   // padded row (bf16 elements) to spread LDS banks

template <int BM, bool A_K>
__device__ __forceinline__ void fetch_tile(const uint16_t *__restrict__ A, int lda, int M, int K,
                                           int m0, int k0, uint4 (&r)[BM / 64])
{
#pragma unroll
    for (int i = 0; i < BM / 64; ++i) {
        const int idx = threadIdx.x + i * 256;
        int m, kk;
        if (A_K) {
            m = idx >> 2;
            kk = (idx & 3) * 8;
        } else {
            kk = idx / (BM / 8);
            m = (idx % (BM / 8)) * 8;
        }
        uint4 v = make_uint4(0, 0, 0, 0);
        if (m0 + m < M && k0 + kk < K)
            v = A_K ? *(const uint4 *)(A + (size_t)(m0 + m) * lda + k0 + kk)
                    : *(const uint4 *)(A + (size_t)(k0 + kk) * lda + m0 + m);
        r[i] = v;
    }
}

// Tiles are kept in LDS as [row][k] (rows = m for A, n for B).
template <int BM, bool A_K>
__device__ __forceinline__ void store_tile(const uint4 (&r)[BM / 64], uint16_t *As)
{
#pragma unroll
    for (int i = 0; i < BM / 64; ++i) {
        const int idx = threadIdx.x + i * 256;
        if (A_K) {
            *(uint4 *)(As + (idx >> 2) * LDSK + (idx & 3) * 8) = r[i];
        } else {
            const int kk = idx / (BM / 8), m = (idx % (BM / 8)) * 8;
            const uint16_t *e = (const uint16_t *)&r[i];
#pragma unroll
            for (int j = 0; j < 8; ++j) As[(m + j) * LDSK + kk] = e[j];
        }
    }
}

template <int BM, int BN, bool A_K, bool B_K, int EPI>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g)
{
    constexpr int TM = BM / 32, TN = BN / 32;
    __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * LDSK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * LDSK];
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int kb = blockIdx.z * g.k_slice;
    const int ke = min(kb + g.k_slice, g.K);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int wm = (w >> 1) * (BM / 2), wn = (w & 1) * (BN / 2);
    f32x4_t acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
    const int fr = l & 15, fk = (l >> 4) * 8;  // fragment row/col and k offset
    uint4 ra[BM / 64], rb[BN / 64];
    fetch_tile<BM, A_K>(g.A, g.lda, g.M, g.K, m0, kb, ra);
    fetch_tile<BN, B_K>(g.B, g.ldb, g.N, g.K, n0, kb, rb);
    store_tile<BM, A_K>(ra, As[0]);
    store_tile<BN, B_K>(rb, Bs[0]);
    __syncthreads();
    int cur = 0;
    for (int k0 = kb; k0 < ke; k0 += GK) {
        const bool more = k0 + GK < ke;
        if (more) {
            fetch_tile<BM, A_K>(g.A, g.lda, g.M, g.K, m0, k0 + GK, ra);
            fetch_tile<BN, B_K>(g.B, g.ldb, g.N, g.K, n0, k0 + GK, rb);
        }
        bf16x8_t af[TM], bfr[TN];
#pragma unroll
        for (int a = 0; a < TM; ++a)
            af[a] = *(const bf16x8_t *)(As[cur] + (wm + a * 16 + fr) * LDSK + fk);
#pragma unroll
        for (int b = 0; b < TN; ++b)
            bfr[b] = *(const bf16x8_t *)(Bs[cur] + (wn + b * 16 + fr) * LDSK + fk);
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        if (more) {
            // the other buffer was last read before the previous barrier
            store_tile<BM, A_K>(ra, As[cur ^ 1]);
            store_tile<BN, B_K>(rb, Bs[cur ^ 1]);
        }
        __syncthreads();
        cur ^= 1;
    }
    // epilogue: lane holds D[(l/16)*4 + i][l%16] of each 16 x 16 tile
    float *part = g.Cf + (size_t)blockIdx.z * g.M * g.ldc;
#pragma unroll
    for (int a = 0; a < TM; ++a) {
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int n = n0 + wn + b * 16 + (l & 15);
            if (n >= g.N) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + wm + a * 16 + (l >> 4) * 4 + i;
                if (m >= g.M) continue;
                float v = acc[a][b][i];
                const size_t o = (size_t)m * g.ldc + n;
                if (EPI == EPI_BIAS_GELU) {
                    v += g.bias[n];
                    g.Cf[o] = v;                    // pre-activation (f32)
                    g.Cb[o] = f2bf(gelu(v));        // activation (bf16)
                } else if (EPI == EPI_BIAS) {
                    g.Cf[o] = v + g.bias[n];
                } else if (EPI == EPI_GELU_GRAD) {
                    // v = dA; dZ = dA * gelu'(Z)
                    g.Cb[o] = f2bf(v * gelu_grad(g.Zin[o]));
                } else if (EPI == EPI_PARTIAL) {
                    part[o] = v;
                } else {
                    g.Cf[o] = v;
                }
            }
        }
    }
}

// out[m][n] = sum over z of part[z][m][n], in order of z.
__global__ void gemm_reduce_kernel(const float *__restrict__ part, int splits, int64_t n_el,
                                   float *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_el) return;
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += part[(size_t)z * n_el + e];
    out[e] = s;
}

template <int BM, int BN, bool A_K, bool B_K, int EPI>
static void launch_gemm(const GemmArgs &g, int splits, hipStream_t st)
{
    dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, splits);
    hipLaunchKernelGGL((gemm_kernel<BM, BN, A_K, B_K, EPI>), grid, dim3(256), 0, st, g);
}

template <bool A_K, bool B_K, int EPI>
static void launch_shape(GemmArgs g, hipStream_t st)
{
    const int64_t t128 = (int64_t)((g.M + 127) / 128) * ((g.N + 127) / 128);
    const int64_t t64 = (int64_t)((g.M + 63) / 64) * ((g.N + 63) / 64);
    if (EPI == EPI_NONE && g.work && t64 < 512 && g.K >= 1024) {
        // few output tiles and a long reduction (weight gradients over the
        // batch): split K into slices of a multiple of the K step, partial
        // products into the workspace, then a fixed-order sum
        int splits = (int)((512 + t64 - 1) / t64);
        splits = min(splits, g.K / 256);
        const int64_t mn = (int64_t)g.M * g.ldc;
        while (splits > 1 && (int64_t)splits * mn > g.work_elems) --splits;
        if (splits > 1) {
            const int slice = ((g.K + splits - 1) / splits + GK - 1) / GK * GK;
            splits = (g.K + slice - 1) / slice;
            GemmArgs h = g;
            h.k_slice = slice;
            h.Cf = g.work;
            launch_gemm<64, 64, A_K, B_K, EPI_PARTIAL>(h, splits, st);
            hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0,
                               st, (const float *)g.work, splits, mn, g.Cf);
            return;
        }
    }
    g.k_slice = g.K;
    if (t128 >= 256)
        launch_gemm<128, 128, A_K, B_K, EPI>(g, 1, st);
    else
        launch_gemm<64, 64, A_K, B_K, EPI>(g, 1, st);
}

// Few-row GEMM for inference on small batches (A and B k-contiguous): one
// wave per 16 x 16 output tile, operands loaded straight from global memory,
// the same v_mfma_f32_16x16x32_bf16 sequence over K (K steps of 32 from 0,
// zero-filled past K) and the same epilogue as gemm_kernel, so each output
// element is computed exactly as gemm_kernel computes it.
#define ROWS_KSTEPS 16   // K <= 512 for the few-row GEMM

template <int EPI>
__global__ void __launch_bounds__(64) gemm_rows_kernel(GemmArgs g)
{
    const int n0 = blockIdx.x * 16, m0 = blockIdx.y * 16;
    const int l = threadIdx.x;
    const int fr = l & 15, fk = (l >> 4) * 8;
    const bool arow = m0 + fr < g.M, brow = n0 + fr < g.N;
    const uint16_t *pa = g.A + (size_t)(m0 + fr) * g.lda + fk;
    const uint16_t *pb = g.B + (size_t)(n0 + fr) * g.ldb + fk;
    // every K step's operands are loaded before the first product
    uint4 va[ROWS_KSTEPS], vb[ROWS_KSTEPS];
#pragma unroll
    for (int s = 0; s < ROWS_KSTEPS; ++s) {
        const int k0 = s * GK;
        const bool kin = k0 + fk < g.K;
        va[s] = make_uint4(0, 0, 0, 0);
        vb[s] = make_uint4(0, 0, 0, 0);
        if (arow && kin) va[s] = *(const uint4 *)(pa + k0);
        if (brow && kin) vb[s] = *(const uint4 *)(pb + k0);
    }
    f32x4_t acc = (f32x4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < ROWS_KSTEPS; ++s)
        if (s * GK < g.K)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, va[s]),
                                                          __builtin_bit_cast(bf16x8_t, vb[s]), acc,
                                                          0, 0, 0);
    const int n = n0 + (l & 15);
    if (n >= g.N) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + (l >> 4) * 4 + i;
        if (m >= g.M) continue;
        const float v = acc[i];
        const size_t o = (size_t)m * g.ldc + n;
        if (EPI == EPI_BIAS_GELU) {
            const float z = v + g.bias[n];
            g.Cf[o] = z;
            g.Cb[o] = f2bf(gelu(z));
        } else {
            g.Cf[o] = v + g.bias[n];
        }
    }
}

int gemm_rows(const GemmArgs &g, int epi, void *stream)
{
    if ((g.M | g.N | g.K) & 7 || g.M < 1 || g.K > ROWS_KSTEPS * GK) return -1;
    const dim3 grid((unsigned)((g.N + 15) / 16), (unsigned)((g.M + 15) / 16));
    if (epi == EPI_BIAS_GELU)
        hipLaunchKernelGGL(gemm_rows_kernel<EPI_BIAS_GELU>, grid, dim3(64), 0, (hipStream_t)stream, g);
    else if (epi == EPI_BIAS)
        hipLaunchKernelGGL(gemm_rows_kernel<EPI_BIAS>, grid, dim3(64), 0, (hipStream_t)stream, g);
    else
        return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int gemm(const GemmArgs &g, bool a_k, bool b_k, int epi, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    if ((g.M | g.N | g.K) & 7) return -1;
#define GEMM_CASE(AK, BK)                                                          \
    if (a_k == AK && b_k == BK) {                                                  \
        switch (epi) {                                                             \
        case EPI_NONE: launch_shape<AK, BK, EPI_NONE>(g, st); break;               \
        case EPI_BIAS: launch_shape<AK, BK, EPI_BIAS>(g, st); break;               \
        case EPI_BIAS_GELU: launch_shape<AK, BK, EPI_BIAS_GELU>(g, st); break;     \
        case EPI_GELU_GRAD: launch_shape<AK, BK, EPI_GELU_GRAD>(g, st); break;     \
        default: return -1;                                                        \
        }                                                                          \
        return hipGetLastError() == hipSuccess ? 0 : -1;                           \
    }
    GEMM_CASE(true, true)
    GEMM_CASE(false, false)
    GEMM_CASE(true, false)
    GEMM_CASE(false, true)
#undef GEMM_CASE
    return -1;
}

// ---------------------------------------------------------------------------
// elementwise and reduction kernels
// ---------------------------------------------------------------------------

// Column sums of dz [M][ld] (bias gradients), in two deterministic passes:
// block (x, y) sums rows [y * COLSUM_ROWS, (y + 1) * COLSUM_ROWS) of columns
// [64 x, 64 x + 64) (lanes = columns, four row phases, combined in a fixed
// order) into part[y][n]; then each column adds its chunks in order.
#define COLSUM_ROWS 128
__global__ void __launch_bounds__(256) colsum_part_kernel(const uint16_t *__restrict__ dz, int M,
                                                          int N, int ld, float *__restrict__ part)
{
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, r = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    const int m0 = blockIdx.y * COLSUM_ROWS;
    const int m1 = min(m0 + COLSUM_ROWS, M);
    float s = 0.0f;
    if (n < N)
        for (int m = m0 + r; m < m1; m += 4) s += bf2f(dz[(size_t)m * ld + n]);
    red[r][c] = s;
    __syncthreads();
    if (r == 0 && n < N)
        part[(size_t)blockIdx.y * N + n] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

__global__ void colsum_final_kernel(const float *__restrict__ part, int chunks, int N,
                                    float *__restrict__ db)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int k = 0; k < chunks; ++k) s += part[(size_t)k * N + n];
    db[n] = s;
}

__device__ __forceinline__ float block_reduce(float v, float *red, bool is_max)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            red[threadIdx.x] = is_max ? fmaxf(red[threadIdx.x], red[threadIdx.x + s])
                                      : red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    float r = red[0];
    __syncthreads();
    return r;
}

// Training loss of one row (one block per row, 256 threads):
//   sum_c w_c (y_c - t_c)^2 / (rows * outs)        weighted squared error,
//   + ce_weight * CE(softmax(t / tau) || softmax(y / tau)) / rows
// Targets are score maps with infeasible cells (-inf): read as 0 in the
// squared error, excluded from the target distribution of the cross-entropy
// (which ranks the best cells first).  w_c = 1 + pos_weight * t_c.  Writes
// dZ as bf16 (zero in padding) and, per row, the squared-error sum and the
// cross-entropy.
__global__ void __launch_bounds__(256) loss_kernel(const float *__restrict__ y, int ldy,
                                                   const float *__restrict__ tgt, int ldt, int rows,
                                                   int outs, int rows_pad, int outs_pad,
                                                   float pos_weight, float ce_weight, float tau,
                                                   uint16_t *__restrict__ dz,
                                                   float *__restrict__ partial)
{
    __shared__ float red[256];
    const int r = blockIdx.x;
    const bool real = r < rows;
    const float itau = 1.0f / tau;
    float my = -INFINITY, mt = -INFINITY;
    if (real && ce_weight > 0.0f) {
        for (int n = threadIdx.x; n < outs; n += blockDim.x) {
            float t = tgt[(size_t)r * ldt + n];
            my = fmaxf(my, y[(size_t)r * ldy + n] * itau);
            if (t > -INFINITY) mt = fmaxf(mt, t * itau);
        }
    }
    my = block_reduce(my, red, true);
    mt = block_reduce(mt, red, true);
    const bool ce = real && ce_weight > 0.0f && mt > -INFINITY;
    float sy = 0.0f, st = 0.0f;
    if (ce) {
        for (int n = threadIdx.x; n < outs; n += blockDim.x) {
            float t = tgt[(size_t)r * ldt + n];
            sy += expf(y[(size_t)r * ldy + n] * itau - my);
            if (t > -INFINITY) st += expf(t * itau - mt);
        }
    }
    sy = block_reduce(sy, red, false);
    st = block_reduce(st, red, false);
    const float lsy = ce ? logf(sy) : 0.0f;
    const float scale = 2.0f / ((float)rows * (float)outs);
    const float cscale = ce_weight * itau / (float)rows;
    float acc = 0.0f, ent = 0.0f;
    for (int n = threadIdx.x; n < outs_pad; n += blockDim.x) {
        float g = 0.0f;
        if (real && n < outs) {
            float traw = tgt[(size_t)r * ldt + n];
            float t = traw > -INFINITY ? traw : 0.0f;
            float yy = y[(size_t)r * ldy + n];
            float wgt = 1.0f + pos_weight * t;
            float d = yy - t;
            acc += wgt * d * d;
            g = scale * wgt * d;
            if (ce) {
                float lp = yy * itau - my - lsy;
                float p = expf(lp);
                float q = traw > -INFINITY ? expf(traw * itau - mt) / st : 0.0f;
                ent -= q * lp;
                g += cscale * (p - q);
            }
        }
        dz[(size_t)r * outs_pad + n] = f2bf(g);
    }
    acc = block_reduce(acc, red, false);
    ent = block_reduce(ent, red, false);
    if (threadIdx.x == 0 && r < rows_pad) {
        partial[2 * r] = acc;
        partial[2 * r + 1] = ent;
    }
}

// Coarse-cell labels from a fine score map (one thread per coarse cell):
// cell (ci, cj) takes the largest score of the fine points
// {4 ci - 2 .. 4 ci + 1} x {4 cj - 2 .. 4 cj + 1} inside the fine lattice
// (the points a re-score of that cell would visit); -inf if none is feasible.
__global__ void pool_kernel(const float *__restrict__ fine, int n_frames, int fnx, int fny,
                            float *__restrict__ coarse, int cnx, int cny)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)cnx * cny;
    if (i >= per * n_frames) return;
    const int f = (int)(i / per);
    const int c = (int)(i - (int64_t)f * per);
    const int ci = c % cnx, cj = c / cnx;
    const float *src = fine + (size_t)f * fnx * fny;
    float m = -INFINITY;
    for (int J = max(4 * cj - 2, 0); J <= min(4 * cj + 1, fny - 1); ++J)
        for (int I = max(4 * ci - 2, 0); I <= min(4 * ci + 1, fnx - 1); ++I)
            m = fmaxf(m, src[(size_t)J * fnx + I]);
    coarse[i] = m;
}

// Adam on one parameter tensor (f32 master), then refresh its bf16 copies:
// the weight as stored [out][in] and, for matrices, transposed [in][out].
__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2, float wd, uint16_t *__restrict__ wb,
                            uint16_t *__restrict__ wbt, int rows, int cols)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i] + wd * w[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) {
        uint16_t h = f2bf(wi);
        wb[i] = h;
        if (wbt) {
            int r = (int)(i / cols), c = (int)(i - (int64_t)r * cols);
            wbt[(size_t)c * rows + r] = h;
        }
    }
}

// bf16 copies of a weight matrix [rows][cols] and its transpose.
__global__ void cast_kernel(const float *__restrict__ w, int64_t n, uint16_t *__restrict__ wb,
                            uint16_t *__restrict__ wbt, int rows, int cols)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint16_t h = f2bf(w[i]);
    wb[i] = h;
    if (wbt) {
        int r = (int)(i / cols), c = (int)(i - (int64_t)r * cols);
        wbt[(size_t)c * rows + r] = h;
    }
}

// Feature vector of a frame (one wave per row): teammates with the passer
// first and the rest by distance to the ball, zero-padded to 8 slots; then
// the opponents by distance to the ball in slots 8-15; then the ball.
// Positions are divided by the field's half length / half width, velocities
// by 3.25 m/s.  Columns 66..in_pad-1 are zero; rows >= n_frames are zero.
// Lanes 0-15 rank the team, lanes 16-31 the opponents (ties to the lower
// robot index); the slot table goes through LDS; each lane then writes
// columns l and l + 64 of the row.
__global__ void __launch_bounds__(64) featurize_kernel(const FrameDev *__restrict__ frames,
                                                       const dpps_robot *__restrict__ robots,
                                                       int n_frames, int rows_pad, int in_pad,
                                                       float inv_hl, float inv_hw, float inv_v,
                                                       uint16_t *__restrict__ x)
{
    __shared__ int slot_robot[16];
    const int f = blockIdx.x;
    const int l = threadIdx.x;
    if (f >= rows_pad) return;
    uint16_t *row = x + (size_t)f * in_pad;
    const bool real = f < n_frames;
    FrameDev F;
    if (real) F = frames[f];
    if (l < 16) slot_robot[l] = -1;
    __syncthreads();
    if (real) {
        const int side = l >> 4, r = l & 15;
        const int cnt = side == 0 ? F.n_team : F.n_opp;
        const int base = side == 0 ? 0 : F.n_team;
        const bool have = l < 32 && r < cnt;
        float key = INFINITY;
        if (have) {
            const dpps_robot R = robots[F.robot_off + base + r];
            const float dx = R.x - F.ball_x, dy = R.y - F.ball_y;
            key = (side == 0 && r == F.passer) ? -1.0f : dx * dx + dy * dy;
        }
        int rank = 0;
        for (int j = 0; j < 16; ++j) {
            const float kj = __shfl(key, (l & 48) | j, 64);
            rank += (kj < key || (kj == key && j < r)) ? 1 : 0;
        }
        if (have && rank < 8) slot_robot[side * 8 + rank] = base + r;
    }
    __syncthreads();
    for (int c = l; c < in_pad; c += 64) {
        float v = 0.0f;
        if (real && c < 64) {
            const int rb = slot_robot[c >> 2];
            if (rb >= 0) {
                const dpps_robot R = robots[F.robot_off + rb];
                const int comp = c & 3;
                v = comp == 0 ? R.x * inv_hl : comp == 1 ? R.y * inv_hw
                                             : comp == 2 ? R.vx * inv_v : R.vy * inv_v;
            }
        } else if (real && c == 64) {
            v = F.ball_x * inv_hl;
        } else if (real && c == 65) {
            v = F.ball_y * inv_hw;
        }
        row[c] = f2bf(v);
    }
}

// Top-k cells of each frame's predicted map (one 256-thread workgroup per
// frame), ordered by (score, index) descending with ties to the lower index.
// The cells' keys (order-preserving score bits) stay in registers (thread t
// holds cells t, t + 256, ...).  Radix passes of 8 bits narrow down the bin
// of key prefixes that holds the k-th largest key: each pass histograms the
// next digit of the keys in the current bin and picks the digit where the
// count of larger keys reaches k.  Keys above the bin are all taken; once the
// bin holds at most 256 keys, its best ones are found by ranking them
// (composite key: score bits, then the inverted index); a bin of more than
// 256 exactly equal keys gives its lowest indices.  The k winners are
// ordered by their ranks among themselves.
constexpr int TOPK_THREADS = 256;
static_assert(TOPK_MAX <= TOPK_THREADS, "one thread per top-k winner");

// Inclusive prefix sum over the 256 threads of a workgroup (sh: 4 ints):
// DPP row shifts within each row of 16 lanes (lanes without a source add 0),
// the row totals carried by lane reads, then the wave totals through LDS.
template <int N>
__device__ __forceinline__ int row_shr_add(int v)
{
    return v + __builtin_amdgcn_update_dpp(0, v, 0x110 + N, 0xf, 0xf, false);
}

__device__ __forceinline__ int block_scan_256(int v, int *sh)
{
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = row_shr_add<1>(v);
    v = row_shr_add<2>(v);
    v = row_shr_add<4>(v);
    v = row_shr_add<8>(v);
    const int r0 = __builtin_amdgcn_readlane(v, 15);
    const int r1 = __builtin_amdgcn_readlane(v, 31);
    const int r2 = __builtin_amdgcn_readlane(v, 47);
    v += (l >= 16 ? r0 : 0) + (l >= 32 ? r1 : 0) + (l >= 48 ? r2 : 0);
    if (l == 63) sh[w] = v;
    __syncthreads();
    int add = 0;
    for (int i = 0; i < w; ++i) add += sh[i];
    __syncthreads();
    return v + add;
}

// Re-score tables of frame f from its top-k cells (the whole workgroup;
// thread t < k holds cell t): each coarse cell (ci, cj) becomes the window
// of fine points {4 ci - 2 .. 4 ci + 1} x {4 cj - 2 .. 4 cj + 1} clipped to
// the fine lattice, one tile per window, and the frame's copy points at
// its k windows.
__device__ void rescore_windows(const RescoreTables &rt, int f, int k, int cell, int *scan_sh)
{
    const FrameDev F = rt.src[f];
    const int t = threadIdx.x;
    int i0 = 0, j0 = 0, nx = 0, ny = 0;
    if (t < k) {
        const int ci = cell % rt.coarse_nx, cj = cell / rt.coarse_nx;
        const int a0 = max(4 * ci - 2, 0), b0 = max(4 * cj - 2, 0);
        const int a1 = min(4 * ci + 1, rt.fine_nx - 1), b1 = min(4 * cj + 1, rt.fine_ny - 1);
        i0 = a0;
        j0 = b0;
        nx = max(a1 - a0 + 1, 0);
        ny = max(b1 - b0 + 1, 0);
    }
    // element offsets: windows in rank order, each with all the frame's variants
    const int incl = block_scan_256(nx * ny, scan_sh);
    if (t < k) {
        WinDev W;
        W.h = rt.fine_h;
        W.i0 = i0;
        W.j0 = j0;
        W.nx = nx;
        W.ny = ny;
        W.halfNx = 0.5f * (float)(rt.fine_nx - 1);
        W.halfNy = 0.5f * (float)(rt.fine_ny - 1);
        W.frame = f;
        W.npts = nx * ny;
        W.elem_base = (incl - nx * ny) * F.n_variants;
        W.out_base = 0;
        rt.wins[(size_t)f * k + t] = W;
        TileDev T;
        T.win = f * k + t;
        T.p0 = 0;
        rt.tiles[(size_t)f * k + t] = T;
    }
    if (t == 0) {
        FrameDev G = F;
        G.n_windows = k;
        G.win_off = f * k;
        G.tile_begin = f * k;
        G.tile_count = k;
        rt.frames[f] = G;
    }
}

__global__ void __launch_bounds__(TOPK_THREADS) topk_kernel(const float *__restrict__ y, int ldy,
                                                            int n_cells, int k,
                                                            int32_t *__restrict__ out, RescoreTables rt)
{
    constexpr int PER = TOPK_SORT / TOPK_THREADS;
    constexpr int RANK_MAX = TOPK_THREADS;
    __shared__ int hist[256];
    __shared__ int scan_sh[4];
    __shared__ int pick[3];   // digit, keys still to take at it, keys at it
    __shared__ int n_sel, n_cand;
    __shared__ unsigned long long cand[RANK_MAX];
    __shared__ unsigned long long buf[TOPK_MAX];
    __shared__ unsigned long long sorted[TOPK_MAX];
    const int f = blockIdx.x;
    const int t = threadIdx.x;
    const int lane = t & 63;
    uint32_t u[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int i = j * TOPK_THREADS + t;
        uint32_t b = 0u;
        if (i < n_cells) {
            b = __float_as_uint(y[(size_t)f * ldy + i]);
            b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
        }
        u[j] = b;
    }
    uint32_t prefix = 0u, pmask = 0u;
    int rem = k, at_T = 0;
    bool ranked = false;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        hist[t] = 0;
        __syncthreads();
        // a wave whose counted keys share one digit (typical of the leading
        // digits: sign and exponent) adds them with one atomic
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const bool act = j * TOPK_THREADS + t < n_cells && (u[j] & pmask) == prefix;
            const uint32_t dg = (u[j] >> shift) & 255u;
            const unsigned long long am = __ballot(act);
            if (am == 0ull) continue;
            const int first = __builtin_ctzll(am);
            const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)dg, first);
            if (__ballot(act && dg != d0) == 0ull) {
                if (lane == first) atomicAdd(&hist[d0], (int)__popcll(am));
            } else if (act) {
                atomicAdd(&hist[dg], 1);
            }
        }
        __syncthreads();
        // thread t holds digit 255 - t: the inclusive scan counts the keys
        // whose digit is >= that digit
        const int d = 255 - t;
        const int c = hist[d];
        const int incl = block_scan_256(c, scan_sh);
        const int excl = incl - c;
        if (excl < rem && incl >= rem) {
            pick[0] = d;
            pick[1] = rem - excl;
            pick[2] = c;
        }
        __syncthreads();
        prefix |= (uint32_t)pick[0] << shift;
        pmask |= 255u << shift;
        rem = pick[1];
        at_T = pick[2];
        __syncthreads();
        if (at_T <= RANK_MAX) {
            ranked = true;
            break;
        }
    }
    if (t == 0) {
        n_sel = 0;
        n_cand = 0;
    }
    __syncthreads();
    // keys above the bin are taken, the bin's keys are candidates
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int i = j * TOPK_THREADS + t;
        if (i >= n_cells) continue;
        const uint32_t m = u[j] & pmask;
        const unsigned long long ck =
            ((unsigned long long)u[j] << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)i);
        if (m > prefix)
            buf[atomicAdd(&n_sel, 1)] = ck;
        else if (ranked && m == prefix)
            cand[atomicAdd(&n_cand, 1)] = ck;
    }
    if (!ranked) {
        // more than RANK_MAX keys equal the k-th largest: the rem lowest
        // indices among them, in index order (row j holds indices 256 j + t)
        int before = 0;
        for (int j = 0; j < PER; ++j) {
            const int i = j * TOPK_THREADS + t;
            const int e = (i < n_cells && u[j] == prefix) ? 1 : 0;
            const int incl = block_scan_256(e, scan_sh);
            if (e && before + incl <= rem)
                buf[atomicAdd(&n_sel, 1)] = ((unsigned long long)u[j] << 32) |
                                            (unsigned long long)(0xFFFFFFFFu - (uint32_t)i);
            if (t == TOPK_THREADS - 1) scan_sh[0] = incl;
            __syncthreads();
            before += scan_sh[0];
            __syncthreads();
        }
    }
    __syncthreads();
    if (ranked && t < at_T) {
        // composite keys are unique: the rem highest candidates
        const unsigned long long my = cand[t];
        int r = 0;
        for (int q = 0; q < at_T; ++q) r += cand[q] > my ? 1 : 0;
        if (r < rem) buf[atomicAdd(&n_sel, 1)] = my;
    }
    __syncthreads();
    // the k winners in order: each one's rank among them
    if (t < k) {
        const unsigned long long my = buf[t];
        int r = 0;
        for (int q = 0; q < k; ++q) r += buf[q] > my ? 1 : 0;
        sorted[r] = my;
    }
    __syncthreads();
    int cell = 0;
    if (t < k) {
        cell = (int32_t)(0xFFFFFFFFu - (uint32_t)sorted[t]);
        out[(size_t)f * k + t] = cell;
    }
    if (rt.frames) rescore_windows(rt, f, k, cell, scan_sh);
    if (rt.zero_word && f == 0 && threadIdx.x == 0) *rt.zero_word = 0;
}

// host launchers -------------------------------------------------------------

int colsum_chunks(int M) { return (M + COLSUM_ROWS - 1) / COLSUM_ROWS; }

int launch_colsum(const uint16_t *dz, int M, int N, int ld, float *db, float *part, void *st)
{
    const int chunks = colsum_chunks(M);
    if (M > 0 && N > 0) {
        hipLaunchKernelGGL(colsum_part_kernel, dim3((N + 63) / 64, chunks), dim3(256), 0,
                           (hipStream_t)st, dz, M, N, ld, part);
        hipLaunchKernelGGL(colsum_final_kernel, dim3((N + 255) / 256), dim3(256), 0,
                           (hipStream_t)st, part, chunks, N, db);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_loss(const float *y, int ldy, const float *tgt, int ldt, int rows, int outs, int rows_pad,
                int outs_pad, float pos_weight, float ce_weight, float tau, uint16_t *dz,
                float *partial, void *st)
{
    hipLaunchKernelGGL(loss_kernel, dim3(rows_pad), dim3(256), 0, (hipStream_t)st, y, ldy, tgt, ldt,
                       rows, outs, rows_pad, outs_pad, pos_weight, ce_weight, tau, dz, partial);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pool(const float *fine, int n_frames, int fnx, int fny, float *coarse, int cnx, int cny,
                void *st)
{
    int64_t n = (int64_t)n_frames * cnx * cny;
    if (n == 0) return 0;
    hipLaunchKernelGGL(pool_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)st, fine, n_frames, fnx, fny, coarse, cnx, cny);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                float eps, float c1, float c2, float wd, uint16_t *wb, uint16_t *wbt, int rows,
                int cols, void *st)
{
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)st, w, g, m, v, n, lr, b1, b2, eps, c1, c2, wd, wb, wbt, rows,
                       cols);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_cast(const float *w, int64_t n, uint16_t *wb, uint16_t *wbt, int rows, int cols, void *st)
{
    hipLaunchKernelGGL(cast_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)st, w, n, wb, wbt, rows, cols);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_featurize(const FrameDev *frames, const dpps_robot *robots, int n_frames, int rows_pad,
                     int in_pad, float inv_hl, float inv_hw, float inv_v, uint16_t *x, void *st)
{
    if (rows_pad == 0) return 0;
    hipLaunchKernelGGL(featurize_kernel, dim3(rows_pad), dim3(64), 0, (hipStream_t)st, frames,
                       robots, n_frames, rows_pad, in_pad, inv_hl, inv_hw, inv_v, x);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_topk(const float *y, int ldy, int n_frames, int n_cells, int k, int32_t *out,
                const RescoreTables *rt, void *st)
{
    if (n_cells > TOPK_SORT || k > n_cells || k > TOPK_MAX) return -1;
    RescoreTables r;
    memset(&r, 0, sizeof r);
    if (rt) r = *rt;
    hipLaunchKernelGGL(topk_kernel, dim3(n_frames), dim3(TOPK_THREADS), 0, (hipStream_t)st, y, ldy,
                       n_cells, k, out, r);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace dpps
