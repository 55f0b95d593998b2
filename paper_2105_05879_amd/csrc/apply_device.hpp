// Device code of the streaming step (Algorithm 1 streaming step, Theorem 5),
// shared by the single-handle kernels and the persistent multi-handle kernels
// so that both run the same arithmetic in the same order.
//
//   draw_gather    draws l_j (Philox4x64-10), coefficients s_l^T x, and the
//                  hot loop that streams the drawn table columns from HBM and
//                  accumulates c_j T[l_j] per chunk of draws of one batch;
//   select_vec     batch means, entrywise median over the K batches, and the
//                  s_max rows of largest |mu| (ties: smaller index) by an
//                  LDS radix select, compacted in ascending row order;
//   survivors_*    exact a_i.x on the selected rows (compensated FP32 dot
//                  product, Ogita-Rump-Oishi Dot2) and the eps threshold:
//                  one workgroup per vector, one wave per row of S (small
//                  batches), or the rows of S of a block of vectors merged
//                  so each row of A is read once per block (large batches).
#pragma once

#include "common.hpp"

namespace kd {

// ----------------------------------------------------------------- Philox --
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64 x 64 -> 128-bit products with a Weyl key schedule.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// bit q of the result is parity(q & v), q < 32 (Walsh functions on 5 bits)
__device__ __forceinline__ uint32_t walsh32(uint32_t v) {
    uint32_t w = 0;
    if (v & 1u) w ^= 0xAAAAAAAAu;
    if (v & 2u) w ^= 0xCCCCCCCCu;
    if (v & 4u) w ^= 0xF0F0F0F0u;
    if (v & 8u) w ^= 0xFF00FF00u;
    if (v & 16u) w ^= 0xFFFF0000u;
    return w;
}

// -------------------------------------------------- draws + gather (fused) --
// One workgroup owns one chunk of the draws of one batch of one vector and
// TILES x 4 KiB of every column (the whole column up to 16 KiB).
//
// Phase 1, draws and coefficients.  Draw j of vector t is block floor(j/4)
// of Philox4x64-10 at counter (floor(j/4), t0 + t, 0, 0), key (seed, 0),
// word j mod 4, and l = floor(r L / 2^64).  The coefficient c = s_l^T x is,
// for a Kerdock vector, a signed sum of x: lane `ln` holds x[e] for
// e = (ln + 64 p) * 32 + q (q < 32), so that bit q of sign word (ln + 64 p)
// of basis b is Q_b(e), and with w = (w_hi, w_lo) the Walsh sign of e is
// parity((ln + 64 p) & w_hi) ^ parity(q & w_lo).  The sum is exact: x is
// converted once to fixed point x_int = x 2^E with sum |x_int| <= 2^30, and
// -x_int = (x_int ^ -1) + 1, so sum_q s_q x_q = sum_q (x_q ^ m_q) + popcount
// of the negative signs, with m_q in {0, -1}; the only roundings are that of
// x to the 2^-E grid and of the final integer to FP32.  An identity vector
// gives sqrt(d) x[w] (zero for w >= n).  The (l, c) pairs go to LDS.
//
// Phase 2, the hot loop: stream the columns T[l] and accumulate c T[l] in
// FP32 registers; each thread owns TILES x 16 bytes (4 FP32, 8 BF16 or 16
// FP8 entries per 16 bytes), UNROLL draws (UNROLL x TILES loads) in flight.
// Columns shorter than 4 KiB split the workgroup into groups of `tpc`
// threads that take interleaved draws and are summed in LDS.  The FP8 row
// scale is applied once, in k_select.
template <int DT> struct Elems { static constexpr int N = DT == KERDOCK_F32 ? 4 : DT == KERDOCK_BF16 ? 8 : 16; };

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

template <int DT>
__device__ __forceinline__ void accumulate(float *acc, const u32x4 raw, float c) {
    const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
    if constexpr (DT == KERDOCK_F32) {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = fmaf(c, __uint_as_float(w[e]), acc[e]);
    } else if constexpr (DT == KERDOCK_BF16) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            acc[2 * e] = fmaf(c, __uint_as_float(w[e] << 16), acc[2 * e]);
            acc[2 * e + 1] = fmaf(c, __uint_as_float(w[e] & 0xFFFF0000u), acc[2 * e + 1]);
        }
    } else {
        // gfx950 converts OCP E4M3 in hardware, two entries per instruction
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[e], false);
            const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[e], true);
            acc[4 * e + 0] = fmaf(c, lo[0], acc[4 * e + 0]);
            acc[4 * e + 1] = fmaf(c, lo[1], acc[4 * e + 1]);
            acc[4 * e + 2] = fmaf(c, hi[0], acc[4 * e + 2]);
            acc[4 * e + 3] = fmaf(c, hi[1], acc[4 * e + 3]);
        }
    }
}

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

constexpr int GATHER_THREADS = 256;
constexpr int TILE_BYTES = GATHER_THREADS * 16;
constexpr int MAX_CHUNK = 1024;

// Geometry and pointers of one draws + gather problem (one handle, one call).
struct DGArgs {
    const unsigned char *table;
    int col_bytes;            // bytes per column (pitch x element size)
    const float *X;           // [batch][n]
    int n, k;
    int64_t L;
    const uint32_t *signs;    // [d/2][max(d/32, 1)]
    uint64_t seed;
    const int64_t *t0_dev;    // stream position of row 0 in device memory, or NULL
    int64_t t0;               // stream position of row 0 when t0_dev is NULL
    int N, J, chunk, chunks_per_batch, groups, tpc, pitch;
    float *partial;           // [batch][K chunks_per_batch][pitch]
    uint32_t *dbg_samples;    // optional [batch][N]
    float *dbg_coef;          // optional [batch][N]
    const int32_t *active;    // optional [batch]: vectors with 0 are skipped
};

// x in fixed point, x_int = rint(x 2^E2) with sum |x_int| <= 2^30 (so every
// signed sum of x_int is an exact int32); lane `lane` of one wave holds the
// elements (lane + 64 p) * 32 + q, q < 32, zero beyond n.  finite is false
// when x holds an inf or NaN (then x_int = 0).
template <int P>
__device__ __forceinline__ void fixed_point(const float *__restrict__ x, int n, int lane, int (&xi)[P][32], int &E2,
                                            bool &finite) {
    float xf[P][32];
    float asum = 0.f;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            const int e = (lane + 64 * p) * 32 + q;
            xf[p][q] = e < n ? x[e] : 0.f;
            asum += fabsf(xf[p][q]);
        }
    asum = wave_sum_f32(asum);
    // scale 2^E2 with asum 2^E2 <= 2^30: asum < 2^(ea + 1), E2 = 29 - ea
    finite = asum < INFINITY;          // false for inf and NaN
    E2 = 0;
    if (finite && asum > 0.f) E2 = 29 - ((int)((__float_as_uint(asum) >> 23) & 0xFF) - 127);
    E2 = max(-120, min(E2, 120));
    const float up = ldexpf(1.0f, E2);
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int q = 0; q < 32; ++q) xi[p][q] = finite ? (int)rintf(xf[p][q] * up) : 0;
}

// Draws jbeg .. jbeg + cnt - 1 (cnt <= MAX_CHUNK) of the Philox stream with
// counter words (floor(j/4), pos, word2, 0) and their coefficients s_l^T x,
// into s_ell / s_coef; all four waves of the workgroup take part, and the
// caller synchronises before reading them.  The method is described at
// draw_gather below.
template <int P>
__device__ __forceinline__ void draws_coefs(const float *__restrict__ x, int n, int k, int64_t L,
                                            const uint32_t *__restrict__ signs, uint64_t seed, uint64_t pos,
                                            uint64_t word2, int jbeg, int cnt, uint32_t *s_ell,
                                            float *s_coef) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    {
        const int d = 1 << k;
        const int words = d >= 32 ? d / 32 : 1;
        int xi[P][32];
        int E2;
        bool finite;
        fixed_point<P>(x, n, lane, xi, E2, finite);
        const float down = ldexpf(1.0f, -E2);
        const float sqrt_d = sqrtf((float)d);

        // the four waves take equal runs of the chunk's draws (a multiple of
        // four each), 64 at a time, one draw per lane for the Philox block
        const int per = ((cnt + 3) / 4 + 3) & ~3;
        const int rend = min(cnt, (wave + 1) * per);
        for (int r0 = wave * per; r0 < rend; r0 += 64) {
            const int jn = min(64, rend - r0);
            uint32_t my_l = 0;
            if (lane < jn) {
                const int j = jbeg + r0 + lane;
                uint64_t c4[4] = {(uint64_t)(j >> 2), pos, word2, 0};
                philox4x64_10(c4, seed, 0);
                const uint64_t rr = (j & 3) == 0 ? c4[0] : (j & 3) == 1 ? c4[1] : (j & 3) == 2 ? c4[2] : c4[3];
                my_l = (uint32_t)__umul64hi(rr, (uint64_t)L);
            }
            float my_c = 0.f;
            for (int jj0 = 0; jj0 < jn; jj0 += 4) {
                uint32_t lq[4], sw[4][P];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    lq[u] = __builtin_amdgcn_readlane(my_l, min(jj0 + u, jn - 1));
                    const uint32_t b = lq[u] >> k;
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const int word = lane + 64 * p;
                        sw[u][p] = ((int)b < d / 2 && word < words) ? signs[(size_t)b * words + word] : 0u;
                    }
                }
                // per-lane partial sums of the four draws, then one
                // transposed butterfly for all four: bits 5 and 4 of the lane
                // pick the draw, bits 3..0 finish the sums (exact integers)
                int part[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t w = lq[u] & (uint32_t)(d - 1);
                    const uint32_t wlo = walsh32(w & 31u);
                    int acc = 0;
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const uint32_t word = (uint32_t)(lane + 64 * p);
                        if ((int)word < words) {
                            const uint32_t par = __popc(word & (w >> 5)) & 1u;
                            const uint32_t mask = sw[u][p] ^ wlo ^ (0u - par);
#pragma unroll
                            for (int q = 0; q < 32; ++q)
                                acc += xi[p][q] ^ (int)__builtin_amdgcn_sbfe(mask, q, 1);
                            acc += __popc(mask);
                        }
                    }
                    part[u] = acc;
                }
                const bool h5 = (lane & 32) != 0, h4 = (lane & 16) != 0;
                const int k0 = (h5 ? part[2] : part[0]) + __shfl_xor(h5 ? part[0] : part[2], 32);
                const int k1 = (h5 ? part[3] : part[1]) + __shfl_xor(h5 ? part[1] : part[3], 32);
                int z = (h4 ? k1 : k0) + __shfl_xor(h4 ? k0 : k1, 16);
#pragma unroll
                for (int off = 8; off > 0; off >>= 1) z += __shfl_xor(z, off);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (jj0 + u >= jn) break;
                    const uint32_t b = lq[u] >> k, w = lq[u] & (uint32_t)(d - 1);
                    float c;
                    if ((int)b == d / 2) {
                        c = ((int)w < n) ? sqrt_d * x[w] : 0.f;
                    } else {
                        const int tot = __builtin_amdgcn_readlane(z, ((u >> 1) << 5) | ((u & 1) << 4));
                        c = finite ? (float)tot * down : __builtin_nanf("");
                    }
                    if (lane == jj0 + u) my_c = c;
                }
            }
            if (lane < jn) {
                s_ell[r0 + lane] = my_l;
                s_coef[r0 + lane] = my_c;
            }
        }
    }

}

template <int DT, int TILES, int UNROLL, bool GROUPED, int P>
__device__ __forceinline__ void draw_gather(const DGArgs &a, int t, int cid, int seg, int nchunks,
                                            uint32_t *s_ell, float *s_coef, float *red) {
    const unsigned char *__restrict__ table = a.table;
    const int col_bytes = a.col_bytes, n = a.n, k = a.k, N = a.N, J = a.J, chunk = a.chunk;
    const int chunks_per_batch = a.chunks_per_batch, groups = a.groups, tpc = a.tpc, pitch = a.pitch;
    const float *__restrict__ X = a.X;
    const int64_t L = a.L;
    const uint32_t *__restrict__ signs = a.signs;
    const uint64_t seed = a.seed;
    const int64_t t0 = a.t0_dev ? *a.t0_dev : a.t0;
    float *__restrict__ partial = a.partial;
    uint32_t *__restrict__ dbg_samples = a.dbg_samples;
    float *__restrict__ dbg_coef = a.dbg_coef;
    constexpr int E = Elems<DT>::N;
    if (a.active && !a.active[t]) return;      // uniform over the workgroup
    const int kb = cid / chunks_per_batch, cj = cid % chunks_per_batch;
    const int jbeg = kb * J + cj * chunk;
    const int cnt = min(chunk, (kb + 1) * J - jbeg);

    // ---------------------------------------------------------- phase 1
    draws_coefs<P>(X + (size_t)t * n, n, k, L, signs, seed, (uint64_t)(t0 + t), 0, jbeg, cnt, s_ell, s_coef);
    __syncthreads();
    if (dbg_samples && seg == 0)
        for (int r = threadIdx.x; r < cnt; r += GATHER_THREADS) {
            dbg_samples[(size_t)t * N + jbeg + r] = s_ell[r];
            dbg_coef[(size_t)t * N + jbeg + r] = s_coef[r];
        }

    // ---------------------------------------------------------- phase 2
    const int g = GROUPED ? (int)threadIdx.x / tpc : 0;
    const int r = GROUPED ? (int)threadIdx.x % tpc : (int)threadIdx.x;
    const int gstride = GROUPED ? groups : 1;
    const size_t seg_off = (size_t)seg * TILES * TILE_BYTES;
    bool tile_on[TILES];
    bool active = false;
#pragma unroll
    for (int ti = 0; ti < TILES; ++ti) {
        tile_on[ti] = (g < gstride) && seg_off + (size_t)ti * TILE_BYTES + (size_t)r * 16 < (size_t)col_bytes;
        active |= tile_on[ti];
    }

    float acc[TILES][E];
#pragma unroll
    for (int ti = 0; ti < TILES; ++ti)
#pragma unroll
        for (int e = 0; e < E; ++e) acc[ti][e] = 0.f;

    if (active) {
        const unsigned char *base = table + seg_off + (size_t)r * 16;
        int j = g;
        for (; j + (UNROLL - 1) * gstride < cnt; j += UNROLL * gstride) {
            u32x4 raw[UNROLL][TILES];
            float cc[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const uint32_t l = s_ell[j + u * gstride];
                cc[u] = s_coef[j + u * gstride];
                const unsigned char *colp = base + (size_t)l * (size_t)col_bytes;
#pragma unroll
                for (int ti = 0; ti < TILES; ++ti)
                    raw[u][ti] = tile_on[ti] ? __builtin_nontemporal_load(
                                                   reinterpret_cast<const u32x4 *>(colp + ti * TILE_BYTES))
                                             : u32x4{0u, 0u, 0u, 0u};
            }
#pragma unroll
            for (int u = 0; u < UNROLL; ++u)
#pragma unroll
                for (int ti = 0; ti < TILES; ++ti) accumulate<DT>(acc[ti], raw[u][ti], cc[u]);
        }
        for (; j < cnt; j += gstride) {
            const uint32_t l = s_ell[j];
            const float c = s_coef[j];
            const unsigned char *colp = base + (size_t)l * (size_t)col_bytes;
#pragma unroll
            for (int ti = 0; ti < TILES; ++ti)
                if (tile_on[ti])
                    accumulate<DT>(acc[ti], __builtin_nontemporal_load(
                                                reinterpret_cast<const u32x4 *>(colp + ti * TILE_BYTES)), c);
        }
    }

    if constexpr (GROUPED) {
#pragma unroll
        for (int e = 0; e < E; ++e) red[e * GATHER_THREADS + threadIdx.x] = acc[0][e];
        __syncthreads();
        if (g != 0 || !active) return;
        for (int gg = 1; gg < groups; ++gg)
#pragma unroll
            for (int e = 0; e < E; ++e) acc[0][e] += red[e * GATHER_THREADS + gg * tpc + r];
    } else {
        if (!active) return;
    }
    float *dst = partial + ((size_t)t * nchunks + cid) * pitch;
#pragma unroll
    for (int ti = 0; ti < TILES; ++ti) {
        if (!tile_on[ti]) continue;
        float *dti = dst + (seg_off + (size_t)ti * TILE_BYTES + (size_t)r * 16) / (16 / E);
#pragma unroll
        for (int e = 0; e < E; e += 4)
            *reinterpret_cast<float4 *>(dti + e) = make_float4(acc[ti][e], acc[ti][e + 1], acc[ti][e + 2], acc[ti][e + 3]);
    }
}

// ---------------------------------------------------------------- select --
// One workgroup per vector.  Row i: ybar_k = (sum of the chunk partials of
// batch k) / J, mu_i = median_k ybar_k (bitonic sort over KMAX >= K slots
// padded with +inf; even K: mean of the two middle values), times the FP8
// row scale.  Then the s_max largest |mu| are found by a radix select over
// the FP32 bit patterns of |mu| (non-negative floats order like their bits)
// and written in ascending row order.
constexpr int SELECT_THREADS = 1024;

__device__ __forceinline__ int block_exclusive_scan(int v, int *total, int *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(incl, off);
        if (lane >= off) incl += u;
    }
    if (lane == 63) sh[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int w = 0; w < SELECT_THREADS / 64; ++w) {
            const int c = sh[w];
            sh[w] = run;
            run += c;
        }
        sh[SELECT_THREADS / 64] = run;
    }
    __syncthreads();
    const int res = sh[wave] + incl - v;
    *total = sh[SELECT_THREADS / 64];
    __syncthreads();
    return res;
}

// The s_max largest keys (ties: smaller index), optionally only keys >=
// tau_bits, written in ascending index order to surv_row (padded with -1),
// their number to *nsurv_out.  Radix select over the 32-bit keys in LDS
// (8 bits per round, histogram in LDS), then two block-wide scans.
__device__ __forceinline__ void select_top(const uint32_t *key, int m, int s_max, uint32_t tau_bits,
                                           int32_t *surv_row, int32_t *nsurv_out, uint32_t *hist,
                                           int *scan_sh, uint32_t *sel_state) {
    uint32_t &sel_prefix = sel_state[0], &sel_want = sel_state[1];
    // radix select of the s_max-th largest key
    uint32_t prefix = 0, fixed = 0, want = (uint32_t)s_max;
    const bool take_all = s_max >= m;
    if (!take_all) {
        for (int shift = 24; shift >= 0; shift -= 8) {
            if (threadIdx.x < 256) hist[threadIdx.x] = 0;
            __syncthreads();
            for (int i = threadIdx.x; i < m; i += SELECT_THREADS) {
                const uint32_t kk = key[i];
                if (((kk ^ prefix) & fixed) == 0) atomicAdd(&hist[(kk >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (threadIdx.x < 64) {
                const int lane = threadIdx.x;
                // lane owns bins 4*lane .. 4*lane+3; suffix sums from the top
                uint32_t hb[4], tot = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    hb[q] = hist[4 * lane + q];
                    tot += hb[q];
                }
                // inclusive suffix scan over lanes: incl = sum of tot over lanes >= lane
                uint32_t incl = tot;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const uint32_t u = __shfl_down(incl, off);
                    if (lane + off < 64) incl += u;
                }
                uint32_t above = incl - tot;   // keys in the bins of higher lanes
#pragma unroll
                for (int q = 3; q >= 0; --q) {
                    if (above < want && want <= above + hb[q]) {
                        sel_prefix = prefix | ((uint32_t)(4 * lane + q) << shift);
                        sel_want = want - above;
                    }
                    above += hb[q];
                }
            }
            __syncthreads();
            prefix = sel_prefix;
            want = sel_want;
            fixed |= 255u << shift;
            __syncthreads();
        }
    }
    const uint32_t theta = prefix;

    // ascending compaction: thread owns rows [i0, i1)
    const int per = (m + SELECT_THREADS - 1) / SELECT_THREADS;
    const int i0 = min(m, (int)threadIdx.x * per), i1 = min(m, i0 + per);
    int eq_local = 0;
    if (!take_all)
        for (int i = i0; i < i1; ++i) eq_local += key[i] == theta;
    int eq_total;
    int eq_rank = block_exclusive_scan(eq_local, &eq_total, scan_sh);
    int sel_local = 0;
    {
        int er = eq_rank;
        for (int i = i0; i < i1; ++i) {
            const uint32_t kk = key[i];
            bool sel = take_all || kk > theta || (kk == theta && (uint32_t)er < want);
            if (!take_all && kk == theta) ++er;
            sel = sel && kk >= tau_bits;
            sel_local += sel;
        }
    }
    int total;
    int pos = block_exclusive_scan(sel_local, &total, scan_sh);
    {
        int er = eq_rank;
        for (int i = i0; i < i1; ++i) {
            const uint32_t kk = key[i];
            bool sel = take_all || kk > theta || (kk == theta && (uint32_t)er < want);
            if (!take_all && kk == theta) ++er;
            sel = sel && kk >= tau_bits;
            if (sel && pos < s_max) surv_row[pos++] = i;
        }
    }
    total = min(total, s_max);
    for (int s = total + threadIdx.x; s < s_max; s += SELECT_THREADS) surv_row[s] = -1;
    if (threadIdx.x == 0) *nsurv_out = total;
}


// Inputs and outputs of the selection for one handle.
struct SelArgs {
    const float *partial;
    int m, pitch, K, chunks_per_batch, J;
    const float *scales;
    int s_max;
    float tau;
    float *mu_out;            // optional [batch][m]
    int32_t *surv;            // [batch][s_max]
    int32_t *nsurv;           // [batch]
    const int32_t *active;    // optional [batch]: vectors with 0 are skipped
};

// shared memory: key[m], hist[256], scan_sh[SELECT_THREADS/64 + 1], sel_state[2]
template <int KMAX>
__device__ __forceinline__ void select_vec(const SelArgs &a, int t, uint32_t *key, uint32_t *hist,
                                           int *scan_sh, uint32_t *sel_state) {
    const float *__restrict__ partial = a.partial;
    const int m = a.m, pitch = a.pitch, K = a.K, chunks_per_batch = a.chunks_per_batch, J = a.J;
    const int s_max = a.s_max;
    const float tau = a.tau;
    const float *__restrict__ scales = a.scales;
    float *__restrict__ mu_out = a.mu_out;
    int32_t *__restrict__ surv = a.surv;
    int32_t *__restrict__ nsurv = a.nsurv;
    if (a.active && !a.active[t]) return;      // uniform over the workgroup
    const int nchunks = K * chunks_per_batch;
    const float *pt = partial + (size_t)t * nchunks * pitch;
    for (int i = threadIdx.x; i < m; i += SELECT_THREADS) {
        float v[KMAX];
#pragma unroll
        for (int a = 0; a < KMAX; ++a) {
            float s = INFINITY;
            if (a < K) {
                // partials of batch a summed in chunk order; eight loads in
                // flight at a time
                const float *pa = pt + (size_t)a * chunks_per_batch * pitch + i;
                s = 0.f;
                int c = 0;
                for (; c + 8 <= chunks_per_batch; c += 8) {
                    float q[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) q[u] = pa[(size_t)(c + u) * pitch];
#pragma unroll
                    for (int u = 0; u < 8; ++u) s += q[u];
                }
                for (; c < chunks_per_batch; ++c) s += pa[(size_t)c * pitch];
                s = s / (float)J;
            }
            v[a] = s;
        }
        // bitonic sort, ascending
#pragma unroll
        for (int size = 2; size <= KMAX; size <<= 1)
#pragma unroll
            for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
                for (int a = 0; a < KMAX; ++a) {
                    const int bb = a ^ stride;
                    if (bb > a) {
                        const bool up = (a & size) == 0;
                        const float lo = fminf(v[a], v[bb]), hi = fmaxf(v[a], v[bb]);
                        v[a] = up ? lo : hi;
                        v[bb] = up ? hi : lo;
                    }
                }
        float lo_mid = 0.f, hi_mid = 0.f;
#pragma unroll
        for (int a = 0; a < KMAX; ++a) {
            if (a == (K - 1) / 2) lo_mid = v[a];
            if (a == K / 2) hi_mid = v[a];
        }
        float med = (K & 1) ? hi_mid : 0.5f * (lo_mid + hi_mid);
        med *= scales[i];
        if (mu_out) mu_out[(size_t)t * m + i] = med;
        key[i] = __float_as_uint(fabsf(med));
    }
    __syncthreads();
    select_top(key, m, s_max, __float_as_uint(fmaxf(tau, 0.f)), surv + (size_t)t * s_max, nsurv + t, hist,
               scan_sh, sel_state);
}

// ------------------------------------------------------------- survivors --
// Inputs and outputs of the survivor dots and threshold for one handle.
struct SurvArgs {
    const float *A;
    int n;
    const float *X;
    const int32_t *surv, *nsurv;
    int s_max;
    float eps;
    int32_t *out_idx;
    float *out_val;
    int32_t *out_cnt;
    float *dbg_values;        // optional [batch][s_max]
    const int32_t *active;    // optional [batch]: vectors with 0 are skipped
    float *vsum2;             // optional [batch]: sum over S of (a_i.x)^2
    float *svals;             // [batch][s_max] survivor values (split launches)
    int vec4;                 // rows of A and X may be read as 16-byte pieces
    int m;                    // rows of A (row-merged launch)
    int *row_ws;              // row-merged launch workspace (survivor_rows_bytes)
};

// Row-merged survivor step: the (vector, row) pairs of SURV_SBLOCK
// consecutive vectors are grouped by row, so each row of A is read once per
// block of vectors and kept in registers while the vectors that selected it
// are dotted against it; a block's vectors (SURV_SBLOCK n 4 bytes) stay in
// the L2 of the one XCD that processes the block.
constexpr int SURV_SBLOCK = 64;
inline size_t survivor_rows_bytes(int batch, int m, int s_max) {
    const size_t nblk = ((size_t)batch + SURV_SBLOCK - 1) / SURV_SBLOCK;
    return (nblk * m + nblk * (m + 1) + (size_t)batch * s_max) * sizeof(int);
}

// 16-byte pieces are legal when n is a multiple of 4 and X is 16-byte
// aligned (A is a device allocation of m x n floats).
inline int surv_vec4(const float *X, int n) {
    return (n % 4 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
}

constexpr int SURV_THREADS = 256;
constexpr int SURV_SPLIT_BATCH = 2048;   // below this many vectors use the split form

// Survivor dots: compensated FP32 dot product (Ogita, Rump, Oishi, "Accurate
// sum and dot product", SIAM J. Sci. Comput. 2005, Dot2): error-free products
// (FMA) and sums (TwoSum), so the result is as accurate as if computed in
// twice the working precision and then rounded.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
#pragma clang fp contract(off)
    s = a + b;
    const float z = s - a;
    e = (a - (s - z)) + (b - z);
}

// one Dot2 step: (p, e) += a b
__device__ __forceinline__ void dot_step(float &p, float &e, float a, float b) {
#pragma clang fp contract(off)
    const float h = a * b;
    const float rr = fmaf(a, b, -h);
    float sum, err;
    two_sum(p, h, sum, err);
    p = sum;
    e = e + (err + rr);
}

// four cascades (one per element position of a 16-byte piece) joined with
// TwoSum, then a compensated butterfly over the wave; every lane returns the
// rounded total
__device__ __forceinline__ float dot_finish(const float (&p)[4], const float (&e)[4]) {
#pragma clang fp contract(off)
    float pp = p[0], ee = e[0];
#pragma unroll
    for (int c = 1; c < 4; ++c) {
        float sum, err;
        two_sum(pp, p[c], sum, err);
        pp = sum;
        ee = ee + (e[c] + err);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float p2 = __shfl_xor(pp, off), e2 = __shfl_xor(ee, off);
        float sum, err;
        two_sum(pp, p2, sum, err);
        pp = sum;
        ee = ee + e2 + err;
    }
    return pp + ee;
}

// a_i.x by one wave.  Lane l takes the 16-byte pieces l, l + 64, ..., one
// Dot2 cascade per element position of a piece (or, when rows cannot be read
// in pieces, elements l, l + 64, ... into one cascade).
__device__ __forceinline__ float survivor_dot(const float *__restrict__ row, const float *__restrict__ x,
                                              int n, int vec4) {
    const int lane = threadIdx.x & 63;
    float p[4] = {0.f, 0.f, 0.f, 0.f}, e[4] = {0.f, 0.f, 0.f, 0.f};
    if (vec4) {
        const float4 *__restrict__ r4 = reinterpret_cast<const float4 *>(row);
        const float4 *__restrict__ x4 = reinterpret_cast<const float4 *>(x);
        const int n4 = n >> 2;
#pragma unroll 4
        for (int q = lane; q < n4; q += 64) {
            const float4 a = r4[q], b = x4[q];
            dot_step(p[0], e[0], a.x, b.x);
            dot_step(p[1], e[1], a.y, b.y);
            dot_step(p[2], e[2], a.z, b.z);
            dot_step(p[3], e[3], a.w, b.w);
        }
    } else {
        for (int q = lane; q < n; q += 64) dot_step(p[0], e[0], row[q], x[q]);
    }
    return dot_finish(p, e);
}

// The same dot (16-byte path) with the row already in registers: rr[i] is
// the piece lane + 64 i of the row (n <= 4096).
__device__ __forceinline__ float survivor_dot_regs(const float4 (&rr)[16], const float *__restrict__ x, int n) {
    const int lane = threadIdx.x & 63;
    const float4 *__restrict__ x4 = reinterpret_cast<const float4 *>(x);
    const int n4 = n >> 2;
    float p[4] = {0.f, 0.f, 0.f, 0.f}, e[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int q = lane + 64 * i;
        if (q < n4) {
            const float4 b = x4[q];
            dot_step(p[0], e[0], rr[i].x, b.x);
            dot_step(p[1], e[1], rr[i].y, b.y);
            dot_step(p[2], e[2], rr[i].z, b.z);
            dot_step(p[3], e[3], rr[i].w, b.w);
        }
    }
    return dot_finish(p, e);
}

// Threshold and compaction of the values of vector t by one wave: rows of S
// with |a_i.x| >= eps, in ascending row order, then padding; optional debug
// values and sum of squares.
__device__ __forceinline__ void survivors_compact(const SurvArgs &a, int t, const float *vals) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const int s_max = a.s_max;
    const int ns = min(a.nsurv[t], s_max);
    // a non-finite survivor value (inf or NaN in x or in a selected row of
    // A) marks the whole vector: count -1, rows all padding
    bool bad = false;
    for (int s0 = 0; s0 < ns; s0 += 64) {
        const int s = s0 + lane;
        bad = bad || (s < ns && !isfinite(vals[s]));
    }
    const bool invalid = __ballot(bad) != 0;
    int base = 0;
    for (int s0 = 0; s0 < s_max; s0 += 64) {
        const int s = s0 + lane;
        const bool keep = !invalid && s < ns && fabsf(vals[s]) >= a.eps;
        const uint64_t mask = __ballot(keep);
        const int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (keep) {
            a.out_idx[(size_t)t * s_max + pos] = a.surv[(size_t)t * s_max + s];
            a.out_val[(size_t)t * s_max + pos] = vals[s];
        }
        base += __popcll(mask);
    }
    for (int s = base + lane; s < s_max; s += 64) {
        a.out_idx[(size_t)t * s_max + s] = -1;
        a.out_val[(size_t)t * s_max + s] = 0.f;
    }
    if (a.dbg_values)
        for (int s = lane; s < s_max; s += 64) a.dbg_values[(size_t)t * s_max + s] = s < ns ? vals[s] : 0.f;
    if (a.vsum2) {
        float e2 = 0.f;
        for (int s = lane; s < ns; s += 64) e2 += vals[s] * vals[s];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off);
        if (lane == 0) a.vsum2[t] = e2;
    }
    if (lane == 0) a.out_cnt[t] = invalid ? -1 : base;
}

// Whole survivor step of vector t in one workgroup (shared memory:
// vals[s_max]): waves take rows of S in turn, then wave 0 compacts.
__device__ __forceinline__ void survivors_vec(const SurvArgs &a, int t, float *vals) {
    if (a.active && !a.active[t]) return;      // uniform over the workgroup
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ns = min(a.nsurv[t], a.s_max);
    const float *x = a.X + (size_t)t * a.n;
    for (int s = wave; s < ns; s += SURV_THREADS / 64) {
        const float v = survivor_dot(a.A + (size_t)a.surv[(size_t)t * a.s_max + s] * a.n, x, a.n, a.vec4);
        if (lane == 0) vals[s] = v;
    }
    __syncthreads();
    if (wave == 0) survivors_compact(a, t, vals);
}

// Split form, for small batches: one wave per row of S across many
// workgroups (values to a.svals), then one wave per vector compacts.
__device__ __forceinline__ void survivor_dots_split(const SurvArgs &a, int t, int s) {
    if (a.active && !a.active[t]) return;
    if (s >= min(a.nsurv[t], a.s_max)) return;
    const float v = survivor_dot(a.A + (size_t)a.surv[(size_t)t * a.s_max + s] * a.n,
                                 a.X + (size_t)t * a.n, a.n, a.vec4);
    if ((threadIdx.x & 63) == 0) a.svals[(size_t)t * a.s_max + s] = v;
}

}  // namespace kd
