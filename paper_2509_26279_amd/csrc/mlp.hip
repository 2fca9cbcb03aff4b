// Vetting MLP 32 -> 128 -> 128 -> 1 on gfx950: bf16 operands on the matrix
// cores (v_mfma_f32_16x16x32_bf16), FP32 accumulation.
//
// Forward:   a0 = q((x - mu) / sd);  h1 = q(relu(a0 q(W1) + b1));
//            h2 = q(relu(h1 q(W2) + b2));  z = h2 q(W3) + b3
// Backward:  dz = (sigmoid(z) (pw y + 1 - y) - pw y) / B;  g3 = q(dz)
//            dW3 = h2^T g3;  d2 = q((g3 q(W3)^T) [h2 > 0]);  dW2 = h1^T d2
//            d1 = q((d2 q(W2)^T) [h1 > 0]);  dW1 = a0^T d1;  db = column sums
// with q = round to bfloat16 (nearest even).  Weight gradients reduce over
// the batch in two stages (per-chunk partials, then a fixed-order sum), so
// the result is the same on every run.  AdamW keeps FP32 master weights and
// refreshes the bf16 working copies.
#include "internal.h"

namespace sas {
namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Store parameter i (packed index) into the bf16 working copies.
__device__ inline void mlp_store_working(const MlpWeights &w, int64_t i, float v) {
    if (i < kMlpOffB1) {
        w.w1[i] = f2bf(v);
    } else if (i >= kMlpOffW2 && i < kMlpOffB2) {
        w.w2[i - kMlpOffW2] = f2bf(v);
    } else if (i >= kMlpOffW3 && i < kMlpOffB3) {
        w.w3[(i - kMlpOffW3) * 16] = f2bf(v);
    } else if (i == kMlpOffB3) {
        w.b3pad[0] = v;
    }
}

enum Epi : int {
    kEpiBiasReluBf16 = 0,  // C = q(relu(acc + bias[n]))
    kEpiBiasF32 = 1,       // C = acc + bias[n]
    kEpiMaskBf16 = 2,      // C = q(acc [mask[m][n] > 0])
    kEpiPartialF32 = 3,    // C[kz] = acc (split over K)
};

struct Gemm {
    const uint16_t *A;
    int64_t sam, sak;  // A[m][k] = A[m sam + k sak]
    const uint16_t *B;
    int64_t sbk, sbn;  // B[k][n] = B[k sbk + n sbn]
    int M, N, K, k_chunk;
    const float *bias;
    const uint16_t *mask;
    int64_t smm;
    void *C;
    int64_t scm;
};

constexpr int GT = 256;  // 4 waves, each a 32 x 32 quarter of the 64 x 64 tile

constexpr int GK = 32;   // K of one v_mfma_f32_16x16x32_bf16

template <int EPI>
__global__ void __launch_bounds__(GT) k_gemm(Gemm g) {
    __shared__ uint16_t As[64][GK + 2];
    __shared__ uint16_t Bs[GK][64 + 2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int kb = blockIdx.z * g.k_chunk, ke = min(g.K, kb + g.k_chunk);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int r16 = lane & 15, q4 = lane >> 4;
    v4f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += GK) {
        for (int q = tid; q < 64 * GK; q += GT) {
            const int r = q / GK, kk = q % GK, m = m0 + r, k = k0 + kk;
            As[r][kk] = (m < g.M && k < ke) ? g.A[(int64_t)m * g.sam + (int64_t)k * g.sak] : 0;
        }
        for (int q = tid; q < GK * 64; q += GT) {
            const int kk = q >> 6, cc = q & 63, k = k0 + kk, n = n0 + cc;
            Bs[kk][cc] = (k < ke && n < g.N) ? g.B[(int64_t)k * g.sbk + (int64_t)n * g.sbn] : 0;
        }
        __syncthreads();
        // operands of a 16 x 16 x 32 product: lane holds row (or column)
        // lane % 16 at k = 8 (lane / 16) + j, j < 8
#pragma unroll
        for (int ti = 0; ti < 2; ++ti) {
            v8bf a;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                a[j] = __builtin_bit_cast(__bf16, As[wm + 16 * ti + r16][8 * q4 + j]);
#pragma unroll
            for (int tj = 0; tj < 2; ++tj) {
                v8bf b;
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    b[j] = __builtin_bit_cast(__bf16, Bs[8 * q4 + j][wn + 16 * tj + r16]);
                acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[ti][tj], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // result layout of a 16 x 16 tile: lane holds rows 4 (lane / 16) + i, column lane % 16
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + wm + 16 * ti + 4 * q4 + i, n = n0 + wn + 16 * tj + r16;
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[ti][tj][i];
                const int64_t o = (int64_t)m * g.scm + n;
                if (EPI == kEpiBiasReluBf16) {
                    ((uint16_t *)g.C)[o] = f2bf(fmaxf(v + g.bias[n], 0.0f));
                } else if (EPI == kEpiBiasF32) {
                    ((float *)g.C)[o] = v + g.bias[n];
                } else if (EPI == kEpiMaskBf16) {
                    const float h = bf2f(g.mask[(int64_t)m * g.smm + n]);
                    ((uint16_t *)g.C)[o] = f2bf(h > 0.0f ? v : 0.0f);
                } else {
                    ((float *)g.C)[(int64_t)blockIdx.z * g.M * g.scm + o] = v;
                }
            }
}

// a0 = q((x - mu) / sd) for rows [0, n) of x (row-major, 32 features)
__global__ void k_norm_cast(const float *__restrict__ x, int64_t n, const float *__restrict__ mu,
                            const float *__restrict__ sd, uint16_t *__restrict__ a0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * 32) return;
    const int k = (int)(i & 31);
    const float s = sd[k] == 0.0f ? 1.0f : sd[k];
    a0[i] = f2bf((x[i] - mu[k]) / s);
}

// Per-row loss and logit gradient; g3 is [B][16] with column 0 the gradient.
__global__ void k_loss(const float *__restrict__ z16, const float *__restrict__ y, int64_t B,
                       float pw, uint16_t *__restrict__ g3, float *__restrict__ row_loss) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    const float z = z16[i * 16], yi = y[i];
    const float sp_pos = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));    // softplus(z)
    const float sp_neg = fmaxf(-z, 0.0f) + log1pf(expf(-fabsf(z)));   // softplus(-z)
    row_loss[i] = pw * yi * sp_neg + (1.0f - yi) * sp_pos;
    const float sig = 1.0f / (1.0f + expf(-z));
    const float dz = (sig * (pw * yi + 1.0f - yi) - pw * yi) / (float)B;
#pragma unroll
    for (int c = 0; c < 16; ++c) g3[i * 16 + c] = c == 0 ? f2bf(dz) : (uint16_t)0;
}

constexpr int RT = 256;

// out[c] = sum over rows r of in[r][c] (bf16 matrix, row stride ld), in a
// fixed order: thread t sums rows t, t + RT, ...; then a fixed tree.
__global__ void __launch_bounds__(RT) k_colsum_bf16(const uint16_t *__restrict__ in, int64_t rows,
                                                    int64_t ld, float *__restrict__ out) {
    __shared__ float red[RT];
    const int c = blockIdx.x;
    float s = 0.0f;
    for (int64_t r = threadIdx.x; r < rows; r += RT) s += bf2f(in[r * ld + c]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = RT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}

__global__ void __launch_bounds__(RT) k_sum_f32(const float *__restrict__ in, int64_t n,
                                                float scale, float *__restrict__ out) {
    __shared__ float red[RT];
    float s = 0.0f;
    for (int64_t r = threadIdx.x; r < n; r += RT) s += in[r];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = RT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// out[j] = sum over kz of part[kz][j] (j < n), kz in order; column col of
// a [rows][ld] partial when pick >= 0 (out[j] = sum part[kz][j * ld + pick]).
__global__ void k_reduce_partials(const float *__restrict__ part, int nz, int64_t stride,
                                  int64_t n, int64_t ld, int pick, float *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t o = pick >= 0 ? j * ld + pick : j;
    float s = 0.0f;
    for (int z = 0; z < nz; ++z) s += part[(int64_t)z * stride + o];
    out[j] = s;
}

// AdamW over the packed FP32 parameters; refreshes the bf16 working copies.
__global__ void k_adamw(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                        const float *__restrict__ g, int64_t n, float lr, float b1, float b2,
                        float eps, float wd, float c1, float c2, MlpWeights w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * ((mi * c1) / (sqrtf(vi * c2) + eps) + wd * p[i]);
    p[i] = pi;
    mlp_store_working(w, i, pi);
}

__global__ void k_refresh(const float *__restrict__ p, int64_t n, MlpWeights w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) mlp_store_working(w, i, p[i]);
}

__global__ void k_pick_col0(const float *__restrict__ z16, int64_t n, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = z16[i * 16];
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <int EPI>
hipError_t gemm(const Gemm &g, int nz, hipStream_t s) {
    const dim3 grid((unsigned)((g.N + 63) / 64), (unsigned)((g.M + 63) / 64), (unsigned)nz);
    hipLaunchKernelGGL(k_gemm<EPI>, grid, dim3(GT), 0, s, g);
    return hipGetLastError();
}

Gemm mk(const uint16_t *A, int64_t sam, int64_t sak, const uint16_t *B, int64_t sbk, int64_t sbn,
        int M, int N, int K, void *C, int64_t scm) {
    Gemm g{};
    g.A = A;
    g.sam = sam;
    g.sak = sak;
    g.B = B;
    g.sbk = sbk;
    g.sbn = sbn;
    g.M = M;
    g.N = N;
    g.K = K;
    g.k_chunk = K;
    g.C = C;
    g.scm = scm;
    return g;
}

}  // namespace

// Forward of rows [0, n) (n <= the buffers' batch): a0, h1, h2, z16.
hipError_t mlp_forward(const MlpBuffers &b, const float *x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_norm_cast, dim3(nblk(n * 32, 256)), dim3(256), 0, s, x, n, b.mu, b.sd,
                       b.a0);
    Gemm g = mk(b.a0, kMlpIn, 1, b.w.w1, kMlpHidden, 1, (int)n, kMlpHidden, kMlpIn, b.h1,
                kMlpHidden);
    g.bias = b.p + kMlpOffB1;
    hipError_t e = gemm<kEpiBiasReluBf16>(g, 1, s);
    if (e != hipSuccess) return e;
    g = mk(b.h1, kMlpHidden, 1, b.w.w2, kMlpHidden, 1, (int)n, kMlpHidden, kMlpHidden, b.h2,
           kMlpHidden);
    g.bias = b.p + kMlpOffB2;
    if ((e = gemm<kEpiBiasReluBf16>(g, 1, s)) != hipSuccess) return e;
    g = mk(b.h2, kMlpHidden, 1, b.w.w3, 16, 1, (int)n, 16, kMlpHidden, b.z16, 16);
    g.bias = b.w.b3pad;
    return gemm<kEpiBiasF32>(g, 1, s);
}

hipError_t mlp_logits(const MlpBuffers &b, const float *x, int64_t n, float *out, hipStream_t s) {
    hipError_t e = mlp_forward(b, x, n, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pick_col0, dim3(nblk(n, 256)), dim3(256), 0, s, b.z16, n, out);
    return hipGetLastError();
}

// Loss (mean) and gradient (packed like the parameters) of a batch of B rows.
hipError_t mlp_grad(const MlpBuffers &b, const float *x, const float *y, int64_t B, float pw,
                    float *loss, float *grad, hipStream_t s) {
    hipError_t e = mlp_forward(b, x, B, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_loss, dim3(nblk(B, 256)), dim3(256), 0, s, b.z16, y, B, pw, b.g3,
                       b.row_loss);
    hipLaunchKernelGGL(k_sum_f32, dim3(1), dim3(RT), 0, s, b.row_loss, B, 1.0f / (float)B, loss);
    const int chunk = kMlpSplitK;
    const int nz = (int)((B + chunk - 1) / chunk);
    // dW3 = h2^T g3 (column 0 of a 128 x 16 product)
    Gemm g = mk(b.h2, 1, kMlpHidden, b.g3, 16, 1, kMlpHidden, 16, (int)B, b.part, 16);
    g.k_chunk = chunk;
    if ((e = gemm<kEpiPartialF32>(g, nz, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_partials, dim3(nblk(kMlpHidden, 256)), dim3(256), 0, s, b.part, nz,
                       (int64_t)kMlpHidden * 16, (int64_t)kMlpHidden, (int64_t)16, 0,
                       grad + kMlpOffW3);
    hipLaunchKernelGGL(k_colsum_bf16, dim3(1), dim3(RT), 0, s, b.g3, B, (int64_t)16,
                       grad + kMlpOffB3);
    // d2 = q((g3 q(W3)^T) [h2 > 0])
    g = mk(b.g3, 16, 1, b.w.w3, 1, 16, (int)B, kMlpHidden, 16, b.d2, kMlpHidden);
    g.mask = b.h2;
    g.smm = kMlpHidden;
    if ((e = gemm<kEpiMaskBf16>(g, 1, s)) != hipSuccess) return e;
    // dW2 = h1^T d2, db2
    g = mk(b.h1, 1, kMlpHidden, b.d2, kMlpHidden, 1, kMlpHidden, kMlpHidden, (int)B, b.part,
           kMlpHidden);
    g.k_chunk = chunk;
    if ((e = gemm<kEpiPartialF32>(g, nz, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_partials, dim3(nblk(kMlpHidden * kMlpHidden, 256)), dim3(256), 0,
                       s, b.part, nz, (int64_t)kMlpHidden * kMlpHidden,
                       (int64_t)kMlpHidden * kMlpHidden, (int64_t)0, -1, grad + kMlpOffW2);
    hipLaunchKernelGGL(k_colsum_bf16, dim3(kMlpHidden), dim3(RT), 0, s, b.d2, B,
                       (int64_t)kMlpHidden, grad + kMlpOffB2);
    // d1 = q((d2 q(W2)^T) [h1 > 0])
    g = mk(b.d2, kMlpHidden, 1, b.w.w2, 1, kMlpHidden, (int)B, kMlpHidden, kMlpHidden, b.d1,
           kMlpHidden);
    g.mask = b.h1;
    g.smm = kMlpHidden;
    if ((e = gemm<kEpiMaskBf16>(g, 1, s)) != hipSuccess) return e;
    // dW1 = a0^T d1, db1
    g = mk(b.a0, 1, kMlpIn, b.d1, kMlpHidden, 1, kMlpIn, kMlpHidden, (int)B, b.part, kMlpHidden);
    g.k_chunk = chunk;
    if ((e = gemm<kEpiPartialF32>(g, nz, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_partials, dim3(nblk(kMlpIn * kMlpHidden, 256)), dim3(256), 0, s,
                       b.part, nz, (int64_t)kMlpIn * kMlpHidden, (int64_t)kMlpIn * kMlpHidden,
                       (int64_t)0, -1, grad + kMlpOffW1);
    hipLaunchKernelGGL(k_colsum_bf16, dim3(kMlpHidden), dim3(RT), 0, s, b.d1, B,
                       (int64_t)kMlpHidden, grad + kMlpOffB1);
    return hipGetLastError();
}

hipError_t mlp_adamw(const MlpBuffers &b, const float *grad, float lr, float b1, float b2,
                     float eps, float wd, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adamw, dim3(nblk(kMlpParams, 256)), dim3(256), 0, s, b.p, b.m, b.v, grad,
                       (int64_t)kMlpParams, lr, b1, b2, eps, wd, c1, c2, b.w);
    return hipGetLastError();
}

hipError_t mlp_refresh(const MlpBuffers &b, hipStream_t s) {
    hipLaunchKernelGGL(k_refresh, dim3(nblk(kMlpParams, 256)), dim3(256), 0, s, b.p,
                       (int64_t)kMlpParams, b.w);
    return hipGetLastError();
}

}  // namespace sas
