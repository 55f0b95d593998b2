// Learned-proposal form: a small MLP that proposes the rows of h_eps(Ax),
// trained and run with hand-written gfx950 kernels.
//
//   features    f = H_d x / sqrt(d) (the coefficients of x in the first
//               Kerdock basis, M_0 = 0: the Walsh-Hadamard basis);
//   MLP         z = W3 relu(W2 relu(W1 f + b1) + b2) + b3 with BF16 weights
//               and activations as GEMM inputs and FP32 accumulation (MFMA
//               16x16x16 BF16); FP32 master weights, Adam;
//   loss        binary cross-entropy with logits, positive weight w+:
//               mean over all entries of -[w+ y log s(z) + (1-y) log(1-s(z))].
// (The energy check of the learned apply is in energy.hip.)
//
// GEMM convention: C[M x N] = Ahat Bhat^T with Ahat M x K and Bhat N x K.  An
// operand is either "row" (element (i, k) at P[i ld + k]) or "k-major"
// (element (i, k) at P[k ld + i]); the tile loader turns both into [row][k]
// LDS tiles.  Tails in M, N and K are zero-filled.
#include <hip/hip_runtime.h>
#include <math.h>

#include "common.hpp"

namespace kd {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;          // output tile (GT x GT) per workgroup of 256 threads

enum { EPI_NONE = 0, EPI_BIAS = 1, EPI_RELU = 2, EPI_MASK = 4 };

__device__ __forceinline__ uint16_t bf16_rne(float f) { return f32_to_bf16_rne(f); }
__device__ __forceinline__ float bf16f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------ BF16 GEMM --
// K tile 32; each wave owns a 32 x 32 quarter of the 64 x 64 output tile as
// 2 x 2 MFMA tiles.  MFMA 16x16x16 BF16 operand layout: lane l holds rows
// (or columns) l % 16 and k = 4 (l / 16) .. 4 (l / 16) + 3; the result holds
// C[4 (l / 16) + v][l % 16], v < 4.
template <bool AK, bool BK>
__global__ __launch_bounds__(256) void k_gemm_bf16(const uint16_t *__restrict__ A, int lda,
                                                   const uint16_t *__restrict__ B, int ldb, int M, int N,
                                                   int K, int epi, const float *__restrict__ bias,
                                                   const uint16_t *__restrict__ mask, int ldm,
                                                   float *__restrict__ C32, uint16_t *__restrict__ C16, int ldc) {
    constexpr int KT = 32, KP = KT + 4;      // pitch keeps 8-byte alignment of 4-element reads
    __shared__ uint16_t As[GT][KP];
    __shared__ uint16_t Bs[GT][KP];
    const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < K; k0 += KT) {
        // tiles: 64 rows x 32 k = 2048 elements, 8 per thread
        if (!AK) {
            const int r = tid >> 2, seg = (tid & 3) * 8, i = i0 + r;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + seg + e;
                As[r][seg + e] = (i < M && k < K) ? A[(size_t)i * lda + k] : (uint16_t)0;
            }
        } else {
            const int kr = tid >> 3, seg = (tid & 7) * 8, k = k0 + kr;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int i = i0 + seg + e;
                As[seg + e][kr] = (i < M && k < K) ? A[(size_t)k * lda + i] : (uint16_t)0;
            }
        }
        if (!BK) {
            const int r = tid >> 2, seg = (tid & 3) * 8, j = j0 + r;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + seg + e;
                Bs[r][seg + e] = (j < N && k < K) ? B[(size_t)j * ldb + k] : (uint16_t)0;
            }
        } else {
            const int kr = tid >> 3, seg = (tid & 7) * 8, k = k0 + kr;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int j = j0 + seg + e;
                Bs[seg + e][kr] = (j < N && k < K) ? B[(size_t)k * ldb + j] : (uint16_t)0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KT; kk += 16) {
            s16x4 fa[2], fb[2];
            const int kq = kk + 4 * (lane >> 4);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const uint16_t *p = &As[wi + a * 16 + (lane & 15)][kq];
                fa[a] = s16x4{(short)p[0], (short)p[1], (short)p[2], (short)p[3]};
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const uint16_t *p = &Bs[wj + b * 16 + (lane & 15)][kq];
                fb[b] = s16x4{(short)p[0], (short)p[1], (short)p[2], (short)p[3]};
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wi + a * 16 + 4 * (lane >> 4) + v;
                const int j = j0 + wj + b * 16 + (lane & 15);
                if (i >= M || j >= N) continue;
                float c = acc[a][b][v];
                if (epi & EPI_BIAS) c += bias[j];
                if (epi & EPI_RELU) c = fmaxf(c, 0.f);
                if (epi & EPI_MASK) c = (mask[(size_t)i * ldm + j] != 0 && !(mask[(size_t)i * ldm + j] & 0x8000)) ? c : 0.f;
                if (C32) C32[(size_t)i * ldc + j] = c;
                if (C16) C16[(size_t)i * ldc + j] = bf16_rne(c);
            }
}

// ---------------------------------------------------------- small kernels --
__global__ void k_to_bf16(const float *__restrict__ x, uint16_t *__restrict__ y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = bf16_rne(x[i]);
}

// db[j] = sum_b dz[b][j] (fixed order: one thread per column)
__global__ void k_colsum(const float *__restrict__ dz, int B, int N, float *__restrict__ db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += dz[(size_t)b * N + j];
    db[j] = s;
}

// BCE with logits and positive weight: per-entry loss terms (summed by
// k_loss_sum) and dL/dz = [s(z)(w+ y + 1 - y) - w+ y] / (B N).
__global__ void k_bce(const float *__restrict__ z, const uint8_t *__restrict__ y, size_t n, float pos_w,
                      float inv_count, float *__restrict__ dz, uint16_t *__restrict__ dz16,
                      float *__restrict__ loss_terms) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float zi = z[i];
        const float yi = y[i] ? 1.f : 0.f;
        const float s = 1.f / (1.f + expf(-zi));
        // log s(z) = -softplus(-z), log(1 - s(z)) = -softplus(z)
        const float sp_pos = fmaxf(zi, 0.f) + log1pf(expf(-fabsf(zi)));      // softplus(z)
        const float sp_neg = sp_pos - zi;                                      // softplus(-z)
        loss_terms[i] = pos_w * yi * sp_neg + (1.f - yi) * sp_pos;
        const float g = (s * (pos_w * yi + 1.f - yi) - pos_w * yi) * inv_count;
        dz[i] = g;
        dz16[i] = bf16_rne(g);
    }
}

// out[0] = sum(terms) / n  (one workgroup, fixed order)
__global__ __launch_bounds__(256) void k_loss_sum(const float *__restrict__ terms, size_t n, float *__restrict__ out) {
    __shared__ float sh[256];
    float s = 0.f;
    for (size_t i = threadIdx.x; i < n; i += 256) s += terms[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0] / (float)n;
}

// Adam (Kingma and Ba 2015) on FP32 masters; refreshes the BF16 copy.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, uint16_t *__restrict__ w16, size_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float mh = mi / c1, vh = vi / c2;
        const float wi = w[i] - lr * mh / (sqrtf(vh) + eps);
        w[i] = wi;
        if (w16) w16[i] = bf16_rne(wi);
    }
}

// f = H x / sqrt(d): one wave per vector, element x = q*64 + lane in
// register q, the transform over register bits in registers and over lane
// bits with cross-lane swizzles.
template <int H> __device__ __forceinline__ float lane_xor_f(float v) {
    if constexpr (H < 32)
        return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), (H << 10) | 0x1f));
    else
        return __shfl_xor(v, 32);
}

template <int LOGD>
__global__ __launch_bounds__(256) void k_features(const float *__restrict__ X, int B, int n,
                                                  float *__restrict__ F, uint16_t *__restrict__ F16) {
    constexpr int D = 1 << LOGD;
    constexpr int R = D >= 64 ? D / 64 : 1;
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= B) return;
    float v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int x = q * 64 + lane;
        v[q] = (x < n && (D >= 64 || lane < D)) ? X[(size_t)t * n + x] : 0.f;
    }
#pragma unroll
    for (int h = 1; h < R; h <<= 1)
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (q & h) continue;
            const float a = v[q], b = v[q + h];
            v[q] = a + b;
            v[q + h] = a - b;
        }
#define KD_FSTAGE(HH)                                                  \
    if constexpr ((HH) < D) {                                          \
        const bool up = (lane & (HH)) != 0;                            \
        _Pragma("unroll") for (int q = 0; q < R; ++q) {                \
            const float p = lane_xor_f<(HH)>(v[q]);                    \
            v[q] = up ? (p - v[q]) : (v[q] + p);                       \
        }                                                              \
    }
    KD_FSTAGE(1) KD_FSTAGE(2) KD_FSTAGE(4) KD_FSTAGE(8) KD_FSTAGE(16) KD_FSTAGE(32)
#undef KD_FSTAGE
    const float s = 1.0f / sqrtf((float)D);
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int w = q * 64 + lane;
        if (D >= 64 || lane < D) {
            const float f = v[q] * s;
            if (F) F[(size_t)t * D + w] = f;
            if (F16) F16[(size_t)t * D + w] = bf16_rne(f);
        }
    }
}

// --------------------------------------------------------------- launchers --

int gemm_bf16(bool ak, bool bk, const uint16_t *A, int lda, const uint16_t *B, int ldb, int M, int N, int K,
              int epi, const float *bias, const uint16_t *mask, int ldm, float *C32, uint16_t *C16, int ldc,
              hipStream_t s) {
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
    if (!ak && !bk) hipLaunchKernelGGL((k_gemm_bf16<false, false>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, epi, bias, mask, ldm, C32, C16, ldc);
    else if (!ak && bk) hipLaunchKernelGGL((k_gemm_bf16<false, true>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, epi, bias, mask, ldm, C32, C16, ldc);
    else if (ak && !bk) hipLaunchKernelGGL((k_gemm_bf16<true, false>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, epi, bias, mask, ldm, C32, C16, ldc);
    else hipLaunchKernelGGL((k_gemm_bf16<true, true>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, epi, bias, mask, ldm, C32, C16, ldc);
    KD_LAUNCH("k_gemm_bf16");
    return KERDOCK_OK;
}

static dim3 grid1d(size_t n) {
    size_t b = (n + 255) / 256;
    return dim3((unsigned)(b < 8192 ? (b ? b : 1) : 8192));
}

int launch_to_bf16(const float *x, uint16_t *y, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, grid1d(n), dim3(256), 0, s, x, y, n);
    KD_LAUNCH("k_to_bf16");
    return KERDOCK_OK;
}

int launch_colsum(const float *dz, int B, int N, float *db, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, s, dz, B, N, db);
    KD_LAUNCH("k_colsum");
    return KERDOCK_OK;
}

int launch_bce(const float *z, const uint8_t *y, size_t n, float pos_w, float *dz, uint16_t *dz16,
               float *terms, float *loss, hipStream_t s) {
    hipLaunchKernelGGL(k_bce, grid1d(n), dim3(256), 0, s, z, y, n, pos_w, 1.0f / (float)n, dz, dz16, terms);
    hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(256), 0, s, terms, n, loss);
    KD_LAUNCH("k_bce");
    return KERDOCK_OK;
}

int launch_adam(float *w, const float *g, float *m, float *v, uint16_t *w16, size_t n, float lr, float b1,
                float b2, float eps, int step, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, grid1d(n), dim3(256), 0, s, w, g, m, v, w16, n, lr, b1, b2, eps, c1, c2);
    KD_LAUNCH("k_adam");
    return KERDOCK_OK;
}

int launch_features(int k, const float *X, int B, int n, float *F, uint16_t *F16, hipStream_t s) {
    dim3 grid((B + 3) / 4), block(256);
    switch (k) {
    case 2: hipLaunchKernelGGL(k_features<2>, grid, block, 0, s, X, B, n, F, F16); break;
    case 4: hipLaunchKernelGGL(k_features<4>, grid, block, 0, s, X, B, n, F, F16); break;
    case 6: hipLaunchKernelGGL(k_features<6>, grid, block, 0, s, X, B, n, F, F16); break;
    case 8: hipLaunchKernelGGL(k_features<8>, grid, block, 0, s, X, B, n, F, F16); break;
    case 10: hipLaunchKernelGGL(k_features<10>, grid, block, 0, s, X, B, n, F, F16); break;
    case 12: hipLaunchKernelGGL(k_features<12>, grid, block, 0, s, X, B, n, F, F16); break;
    default: return fail(KERDOCK_ERR_UNSUPPORTED_N, "features: unsupported k");
    }
    KD_LAUNCH("k_features");
    return KERDOCK_OK;
}

}  // namespace kd
