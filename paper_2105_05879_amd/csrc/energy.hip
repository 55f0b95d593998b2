// Certified energy check of the learned-proposal form.
//
// The learned apply accepts the proposal C for a vector x only when the
// energy |Ax|^2 left outside C is provably below eps^2: a row of h_eps(Ax)
// outside C would leave at least eps^2.  Everything runs in FP32 with
// compensated (double-word) sums, and every quantity carries a rigorous
// rounding bound, so the decision is sound in floating point too:
//
//   G = A^T A          every entry a compensated dot product over the m rows
//                      (Ogita, Rump, Oishi, "Accurate sum and dot product",
//                      SIAM J. Sci. Comput. 2005, Dot2), kept unrounded as a
//                      normalised pair G = Ghi + Glo with |Glo| <= u |Ghi|:
//                      |G - A^T A| <= gamma_m^2 |A|^T |A|;
//   z = G x            per output a sequential Dot2 over the n columns for
//                      Ghi and a plain sum for Glo, kept as a pair:
//                      |z - G x| <= 2 gamma_n^2 |G| |x|;
//   E = x^T z          Dot2 over the n products, then one rounding:
//                      |E - |Ax|^2| <= u |E| + (gamma_m^2 + 4 gamma_n^2) Q
//                      with Q = |x|^T |A|^T |A| |x| <= |A|_F^2 |x|^2;
//   S = sum_C v_i^2    from the survivor values (Dot2, |v - a.x| <= u |v| +
//                      2 gamma_n^2 |a| |x|) squared and summed in FP32:
//                      |S - sum_C (a_i.x)^2| <= (3u + gamma_{c+1}) S +
//                      4 gamma_n^2 sqrt(S Q).
// With B >= |E - |Ax|^2| + |S - sum_C (a_i.x)^2| evaluated from these terms
// (doubled, for the rounding of the bound itself), a vector falls back to
// the plain estimator unless E - S <= eps^2 / 2 and B < eps^2 / 2; then
// |Ax|^2 - sum_C (a_i.x)^2 < eps^2, so no row with |(Ax)_i| >= eps is
// outside C.  (u = 2^-24, gamma_k = k u / (1 - k u).)
#include <hip/hip_runtime.h>
#include <math.h>

#include "common.hpp"

namespace kd {

// error-free transformations (FMA and TwoSum) and one Dot2 step
__device__ __forceinline__ void e_two_sum(float a, float b, float &s, float &e) {
#pragma clang fp contract(off)
    s = a + b;
    const float z = s - a;
    e = (a - (s - z)) + (b - z);
}

__device__ __forceinline__ void e_dot_step(float &p, float &e, float a, float b) {
#pragma clang fp contract(off)
    const float h = a * b;
    const float r = fmaf(a, b, -h);
    float s, q;
    e_two_sum(p, h, s, q);
    p = s;
    e = e + (q + r);
}

constexpr int ET = 64;           // output tile (ET x ET) per workgroup
constexpr int EK = 32;           // k step staged in LDS
constexpr int EP = EK + 1;       // LDS pitch (conflict-free column reads)

// G = A^T A as (Ghi, Glo), both [n][n]; grid (ceil(n/64), ceil(n/64)),
// 256 threads, each a 4 x 4 block of entries (j, k), a Dot2 over the rows i.
__global__ __launch_bounds__(256) void k_gram2(const float *__restrict__ A, int m, int n, float *__restrict__ Ghi,
                                               float *__restrict__ Glo) {
    __shared__ float Aj[EK][ET + 1];
    __shared__ float Ak[EK][ET + 1];
    const int j0 = blockIdx.y * ET, k0 = blockIdx.x * ET;
    const int tj = (threadIdx.x >> 4) * 4, tk = (threadIdx.x & 15) * 4;
    float p[4][4], e[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) p[a][b] = e[a][b] = 0.f;
    for (int i0 = 0; i0 < m; i0 += EK) {
        // stage rows i0 .. i0 + 31 of columns j0 .. j0 + 63 and k0 .. k0 + 63
        for (int q = threadIdx.x; q < EK * ET; q += 256) {
            const int r = q / ET, c = q % ET, i = i0 + r;
            Aj[r][c] = (i < m && j0 + c < n) ? A[(size_t)i * n + j0 + c] : 0.f;
            Ak[r][c] = (i < m && k0 + c < n) ? A[(size_t)i * n + k0 + c] : 0.f;
        }
        __syncthreads();
        const int rows = min(EK, m - i0);
        for (int r = 0; r < rows; ++r) {
            float aj[4], ak[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                aj[a] = Aj[r][tj + a];
                ak[a] = Ak[r][tk + a];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) e_dot_step(p[a][b], e[a][b], aj[a], ak[b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int j = j0 + tj + a, k = k0 + tk + b;
            if (j < n && k < n) {
                float hi, lo;
                e_two_sum(p[a][b], e[a][b], hi, lo);
                Ghi[(size_t)j * n + k] = hi;
                Glo[(size_t)j * n + k] = lo;
            }
        }
}

// |A|_F^2 by one workgroup of 1024 threads (Dot2 per thread, TwoSum tree),
// rounded up by a relative 2^-20 so that it bounds the exact value.
__global__ __launch_bounds__(1024) void k_frobenius2(const float *__restrict__ A, size_t count,
                                                     float *__restrict__ out) {
    __shared__ float sp[1024], se[1024];
    float p = 0.f, e = 0.f;
    for (size_t i = threadIdx.x; i < count; i += 1024) e_dot_step(p, e, A[i], A[i]);
    sp[threadIdx.x] = p;
    se[threadIdx.x] = e;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            float s, q;
            e_two_sum(sp[threadIdx.x], sp[threadIdx.x + h], s, q);
            sp[threadIdx.x] = s;
            se[threadIdx.x] = se[threadIdx.x] + se[threadIdx.x + h] + q;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (sp[0] + se[0]) * (1.0f + 0x1p-20f);
}

// z = X G^T (G symmetric) as pairs (Zp, Ze), [B][n] each; grid
// (ceil(n/64), ceil(B/64)), 256 threads, each 4 vectors x 4 outputs with a
// sequential Dot2 over k for Ghi and a plain FP32 sum for Glo.
__global__ __launch_bounds__(256) void k_energy_z(const float *__restrict__ X, int B, int n,
                                                  const float *__restrict__ Ghi, const float *__restrict__ Glo,
                                                  float *__restrict__ Zp, float *__restrict__ Ze) {
    __shared__ float Xs[ET][EP];
    __shared__ float Hs[ET][EP];
    __shared__ float Ls[ET][EP];
    const int t0 = blockIdx.y * ET, j0 = blockIdx.x * ET;
    const int tt = (threadIdx.x >> 4) * 4, tj = (threadIdx.x & 15) * 4;
    float p[4][4], e[4][4], el[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) p[a][b] = e[a][b] = el[a][b] = 0.f;
    for (int k0 = 0; k0 < n; k0 += EK) {
        for (int q = threadIdx.x; q < ET * EK; q += 256) {
            const int r = q / EK, c = q % EK, k = k0 + c;
            const int t = t0 + r, j = j0 + r;
            Xs[r][c] = (t < B && k < n) ? X[(size_t)t * n + k] : 0.f;
            Hs[r][c] = (j < n && k < n) ? Ghi[(size_t)j * n + k] : 0.f;
            Ls[r][c] = (j < n && k < n) ? Glo[(size_t)j * n + k] : 0.f;
        }
        __syncthreads();
        const int cols = min(EK, n - k0);
        for (int c = 0; c < cols; ++c) {
            float xv[4], hv[4], lv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                xv[a] = Xs[tt + a][c];
                hv[a] = Hs[tj + a][c];
                lv[a] = Ls[tj + a][c];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    e_dot_step(p[a][b], e[a][b], xv[a], hv[b]);
                    el[a][b] = fmaf(xv[a], lv[b], el[a][b]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int t = t0 + tt + a, j = j0 + tj + b;
            if (t < B && j < n) {
                Zp[(size_t)t * n + j] = p[a][b];
                Ze[(size_t)t * n + j] = e[a][b] + el[a][b];
            }
        }
}

// One wave per vector: E = x^T z (Dot2 over x_j Zp_j plus a plain sum of
// x_j Ze_j, compensated lane tree), |x|^2, the bound B of the header, and
// the fallback flag.  vsum2 = sum over C of the FP32 survivor values squared.
__global__ __launch_bounds__(256) void k_energy_flags(const float *__restrict__ X, int B, int n, int m, int c,
                                                      const float *__restrict__ Zp, const float *__restrict__ Ze,
                                                      const float *__restrict__ vsum2, const float *__restrict__ fro2,
                                                      float eps, int32_t *__restrict__ flags,
                                                      float *__restrict__ dbg_energy) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= B) return;
    const float *x = X + (size_t)t * n;
    float p = 0.f, e = 0.f, xx = 0.f;
    for (int j = lane; j < n; j += 64) {
        const float xj = x[j];
        e_dot_step(p, e, xj, Zp[(size_t)t * n + j]);
        e = fmaf(xj, Ze[(size_t)t * n + j], e);
        xx = fmaf(xj, xj, xx);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float p2 = __shfl_xor(p, off), e2 = __shfl_xor(e, off);
        float s, q;
        e_two_sum(p, p2, s, q);
        p = s;
        e = e + e2 + q;
        xx += __shfl_xor(xx, off);
    }
    if (lane != 0) return;
    const float u = 0x1p-24f;
    const float gn = (float)n * u / (1.0f - (float)n * u);
    const float gm = (float)m * u / (1.0f - (float)m * u);
    const float gc = (float)(c + 1) * u / (1.0f - (float)(c + 1) * u);
    const float E = p + e;
    const float S = vsum2[t];
    const float xx_up = xx * (1.0f + 2.0f * gn + 0x1p-20f);      // >= |x|^2
    const float Q = fro2[0] * xx_up;                             // >= |x|^T |A|^T |A| |x|
    const float bound = 2.0f * (u * fabsf(E) + (gm * gm + 4.0f * gn * gn) * Q + (3.0f * u + gc) * S +
                                4.0f * gn * gn * sqrtf(S * Q));
    const float half = 0.5f * eps * eps;
    // NaN anywhere (x, the values) makes both comparisons false: fall back
    const bool accept = (E - S <= half) && (bound < half);
    flags[t] = accept ? 0 : 1;
    if (dbg_energy) {
        dbg_energy[(size_t)t * m + 0] = E;
        dbg_energy[(size_t)t * m + 1] = S;
        dbg_energy[(size_t)t * m + 2] = bound;
    }
}

// ------------------------------------------------------------ launchers --

int launch_gram2(const float *A, int m, int n, float *Ghi, float *Glo, float *fro2, hipStream_t s) {
    const int g = (n + ET - 1) / ET;
    hipLaunchKernelGGL(k_gram2, dim3(g, g), dim3(256), 0, s, A, m, n, Ghi, Glo);
    KD_LAUNCH("k_gram2");
    hipLaunchKernelGGL(k_frobenius2, dim3(1), dim3(1024), 0, s, A, (size_t)m * n, fro2);
    KD_LAUNCH("k_frobenius2");
    return KERDOCK_OK;
}

int launch_energy_flags(const float *X, int B, int n, int m, int c, const float *Ghi, const float *Glo,
                        const float *fro2, const float *vsum2, float eps, float *Zp, float *Ze, int32_t *flags,
                        float *dbg_energy, hipStream_t s) {
    if ((B + ET - 1) / ET > 65535) return fail(KERDOCK_ERR_INVALID_ARG, "energy check: batch above 4194240");
    hipLaunchKernelGGL(k_energy_z, dim3((n + ET - 1) / ET, (B + ET - 1) / ET), dim3(256), 0, s, X, B, n, Ghi, Glo,
                       Zp, Ze);
    KD_LAUNCH("k_energy_z");
    hipLaunchKernelGGL(k_energy_flags, dim3((B + 3) / 4), dim3(256), 0, s, X, B, n, m, c, Zp, Ze, vsum2, fro2, eps,
                       flags, dbg_energy);
    KD_LAUNCH("k_energy_flags");
    return KERDOCK_OK;
}

}  // namespace kd
