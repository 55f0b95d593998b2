// Shared-draw form of the streaming step.
//
// The rows of X are taken in groups of KERDOCK_SHARED_TILE consecutive
// vectors; every vector of group g uses the same N = J K draws, those of the
// Philox stream at counter words (floor(j/4), t0 + g, 1, 0).  The draws do not
// depend on x, so each vector still sees N independent uniform draws and
// Theorem 5 holds for it as before.  What changes is the shape of the work:
// with one draw list per group, the batch sums of a group,
//     Y_k[i][t] = sum_{j in batch k} T[l_j][i] c_j(x_t),
// form the matrix product of the m x J gathered table columns T_{S_k} and the
// J x 64 coefficient block C_k.  Each table column is then read once per
// group instead of once per vector, and the product runs on the FP32 matrix
// cores (16 x 16 x 4 MFMA), with BF16 and FP8 entries widened to FP32 on the
// way into LDS.  The batch means, median, selection and survivor dots are
// those of the per-vector form (partials with one chunk per batch).
#include "apply_device.hpp"

namespace kd {

constexpr int ST = KERDOCK_SHARED_TILE;       // vectors per draw group
constexpr int SH_CHUNK = MAX_CHUNK;           // draws per coefficient workgroup
constexpr int SG_BM = 128;                    // table rows per GEMM workgroup
constexpr int SG_BK = 32;                     // draws per LDS stage

// k_shared_coef: grid (batch, ceil(N / SH_CHUNK)).  Vector t, draws jbeg ..
// jbeg + cnt - 1 of its group: l_j to ell[g][j] (written by the group's first
// vector), s_l^T x_t to coef[g][t mod 64][j].
template <int P>
__global__ __launch_bounds__(GATHER_THREADS) void k_shared_coef(const float *__restrict__ X, int n, int k, int64_t L,
                                                                const uint32_t *__restrict__ signs, uint64_t seed,
                                                                int64_t t0, int N, uint32_t *__restrict__ ell,
                                                                float *__restrict__ coef,
                                                                uint32_t *__restrict__ dbg_samples,
                                                                float *__restrict__ dbg_coef) {
    __shared__ uint32_t s_ell[SH_CHUNK];
    __shared__ float s_coef[SH_CHUNK];
    const int t = blockIdx.x, g = t / ST, tt = t % ST;
    const int jbeg = blockIdx.y * SH_CHUNK;
    const int cnt = min(SH_CHUNK, N - jbeg);
    draws_coefs<P>(X + (size_t)t * n, n, k, L, signs, seed, (uint64_t)(t0 + g), 1, jbeg, cnt, s_ell, s_coef);
    __syncthreads();
    for (int r = threadIdx.x; r < cnt; r += GATHER_THREADS) {
        const size_t j = (size_t)jbeg + r;
        coef[((size_t)g * ST + tt) * N + j] = s_coef[r];
        if (tt == 0) ell[(size_t)g * N + j] = s_ell[r];
        if (dbg_samples) {
            dbg_samples[(size_t)t * N + j] = s_ell[r];
            dbg_coef[(size_t)t * N + j] = s_coef[r];
        }
    }
}

// 16 bytes of table entries widened to FP32
template <int DT>
__device__ __forceinline__ void widen(const u32x4 raw, float *v) {
    const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
    if constexpr (DT == KERDOCK_F32) {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = __uint_as_float(w[e]);
    } else if constexpr (DT == KERDOCK_BF16) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v[2 * e] = __uint_as_float(w[e] << 16);
            v[2 * e + 1] = __uint_as_float(w[e] & 0xFFFF0000u);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[e], false);
            const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[e], true);
            v[4 * e + 0] = lo[0];
            v[4 * e + 1] = lo[1];
            v[4 * e + 2] = hi[0];
            v[4 * e + 3] = hi[1];
        }
    }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// k_shared_gemm: grid (ceil(pitch / 128), K, groups), 256 threads.  Rows
// i0 .. i0 + 127 of Y_k for the (up to) 64 vectors of group g:
// partial[t][k][i] = sum_{j < J} T[ell[g][k J + j]][i] coef[g][t][k J + j].
// Wave w owns rows i0 + 32 w .. + 31, all 64 vectors: 2 x 4 MFMA blocks.
template <int DT>
__global__ __launch_bounds__(256) void k_shared_gemm(const unsigned char *__restrict__ table, int col_bytes, int pitch,
                                                     int batch, int J, int K, int N,
                                                     const uint32_t *__restrict__ ell,
                                                     const float *__restrict__ coef,
                                                     float *__restrict__ partial) {
    constexpr int E = Elems<DT>::N;           // entries per 16 bytes
    constexpr int TPC = SG_BM / E;            // threads per column slice
    constexpr int CPP = 256 / TPC;            // column slices per pass
    static_assert(SG_BK % CPP == 0, "whole passes");
    __shared__ float As[SG_BK][SG_BM + 16];   // [draw][row]; row stride = 16 mod 64 banks
    __shared__ float Bs[SG_BK][ST + 16];      // [draw][vector]
    const int g = blockIdx.z, kb = blockIdx.y, i0 = blockIdx.x * SG_BM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nx = min(ST, batch - g * ST);
    const uint32_t *__restrict__ el = ell + (size_t)g * N + (size_t)kb * J;
    const float *__restrict__ cf = coef + (size_t)g * ST * N + (size_t)kb * J;
    const int wi = wave * 32;
    f32x4 acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int j0 = 0; j0 < J; j0 += SG_BK) {
        // A stage: SG_BK gathered column slices of SG_BM rows, 16 bytes a thread
#pragma unroll
        for (int c0 = 0; c0 < SG_BK; c0 += CPP) {
            const int cc = c0 + tid / TPC, r = (tid % TPC) * E;
            {
                const int jj = j0 + cc;
                float v[E];
                if (jj < J && i0 + r < pitch) {
                    const unsigned char *src = table + (size_t)el[jj] * (size_t)col_bytes + (size_t)(i0 + r) * (size_t)(16 / E);
                    widen<DT>(__builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(src)), v);
                } else {
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e] = 0.f;
                }
#pragma unroll
                for (int e = 0; e < E; e += 4)
                    *reinterpret_cast<f32x4 *>(&As[cc][r + e]) = f32x4{v[e], v[e + 1], v[e + 2], v[e + 3]};
            }
        }
        // B stage: SG_BK draws x 64 vectors, eight consecutive draws a thread
        {
            const int tt = tid >> 2, q = (tid & 3) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int jj = j0 + q + e;
                Bs[q + e][tt] = (tt < nx && jj < J) ? cf[(size_t)tt * N + jj] : 0.f;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < SG_BK; kk += 4) {
            float fa[2], fb[4];
#pragma unroll
            for (int a = 0; a < 2; ++a) fa[a] = As[kk + (lane >> 4)][wi + a * 16 + (lane & 15)];
#pragma unroll
            for (int b = 0; b < 4; ++b) fb[b] = Bs[kk + (lane >> 4)][b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // D block (a, b): lane holds rows 4 (lane / 16) + v, v < 4, of column lane % 16
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int row = i0 + wi + a * 16 + 4 * (lane >> 4);
            const int tt = b * 16 + (lane & 15);
            if (tt < nx && row < pitch)
                *reinterpret_cast<f32x4 *>(partial + ((size_t)(g * ST + tt) * K + kb) * pitch + row) = acc[a][b];
        }
}

int launch_shared_coef(const float *X, int batch, int n, int k, int64_t L, const uint32_t *signs, uint64_t seed,
                       int64_t t0, int N, uint32_t *ell, float *coef, uint32_t *dbg_samples, float *dbg_coef,
                       hipStream_t s) {
    const int ny = (N + SH_CHUNK - 1) / SH_CHUNK;
    if (ny > 65535) return fail(KERDOCK_ERR_INVALID_ARG, "shared form: J K must stay below 2^26");
    dim3 grid(batch, ny);
    if (n <= 2048)
        hipLaunchKernelGGL(k_shared_coef<1>, grid, dim3(GATHER_THREADS), 0, s, X, n, k, L, signs, seed, t0, N, ell,
                           coef, dbg_samples, dbg_coef);
    else
        hipLaunchKernelGGL(k_shared_coef<2>, grid, dim3(GATHER_THREADS), 0, s, X, n, k, L, signs, seed, t0, N, ell,
                           coef, dbg_samples, dbg_coef);
    KD_LAUNCH("k_shared_coef");
    return KERDOCK_OK;
}

int launch_shared_gemm(kerdock_dtype dt, const void *table, int pitch, int batch, int J, int K, const uint32_t *ell,
                       const float *coef, float *partial, hipStream_t s) {
    const int groups = (batch + ST - 1) / ST;
    if (groups > 65535) return fail(KERDOCK_ERR_INVALID_ARG, "shared form: batch too large");
    dim3 grid((pitch + SG_BM - 1) / SG_BM, K, groups);
    const unsigned char *tb = reinterpret_cast<const unsigned char *>(table);
    const int cb = pitch * (int)dtype_bytes(dt), N = J * K;
    switch (dt) {
    case KERDOCK_F32:
        hipLaunchKernelGGL(k_shared_gemm<KERDOCK_F32>, grid, dim3(256), 0, s, tb, cb, pitch, batch, J, K, N, ell,
                           coef, partial);
        break;
    case KERDOCK_BF16:
        hipLaunchKernelGGL(k_shared_gemm<KERDOCK_BF16>, grid, dim3(256), 0, s, tb, cb, pitch, batch, J, K, N, ell,
                           coef, partial);
        break;
    case KERDOCK_FP8E4M3:
        hipLaunchKernelGGL(k_shared_gemm<KERDOCK_FP8E4M3>, grid, dim3(256), 0, s, tb, cb, pitch, batch, J, K, N, ell,
                           coef, partial);
        break;
    }
    KD_LAUNCH("k_shared_gemm");
    return KERDOCK_OK;
}

}  // namespace kd
