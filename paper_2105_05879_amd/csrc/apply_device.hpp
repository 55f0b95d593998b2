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

// ------------------------------------------- draws, buckets and gather --
// Three stages per batch of J draws of one vector.
//
// Draws and buckets (draw_sort, one workgroup per (vector, batch)).  Draw j
// of vector t is word j mod 4 of Philox4x64-10 at counter (floor(j/4),
// t0 + t, 0, 0), key (seed, 0), and l = floor(r L / 2^64).  The draws of
// the batch are sorted by their basis b = l >> k with a counting sort:
// per-wave histograms of b in LDS, one scan over (basis, wave), then every
// wave places its draws in drawing order, ranking equal bases within 64
// draws by ballots over the bits of b.  The batch's draws thus come grouped
// by basis, in drawing order within a basis; only the summation order of the
// batch sum depends on this.
//
// Coefficients (draw_gather phase 1).  One workgroup owns `chunk`
// consecutive sorted draws of one batch of one vector and TILES x 4 KiB of
// every column (the whole column up to 16 KiB).  c = s_l^T x is, for a
// Kerdock vector, a signed sum of x: lane `ln` holds x[e] for
// e = (ln + 64 p) * 32 + q (q < 32), so that bit q of sign word (ln + 64 p)
// of basis b is Q_b(e), and with w = (w_hi, w_lo) the Walsh sign of e is
// parity((ln + 64 p) & w_hi) ^ parity(q & w_lo).  The sums are exact: x is
// converted once to fixed point x_int = x 2^E with sum |x_int| <= 2^30, so
// every partial sum is an exact int32; the only roundings are that of x to
// the 2^-E grid and of the final integer to FP32.  A run of at least
// BUCKET_MIN draws of one Kerdock basis (Lemma 8's per-basis transform)
// forms y = sigma_b x once and its 32-point Walsh-Hadamard transform
// Y[v] = sum_q y_q (-1)^{q.v} per lane, so a draw costs one register pick
// Y[w_lo], a lane sign and the wave sum; other draws sum directly,
// sum_q s_q x_q = sum_q (x_q ^ m_q) + popcount of the negative signs with
// m_q in {0, -1}.  Both give the same integer.  An identity vector gives
// sqrt(d) x[w] (zero for w >= n).  The (l, c) pairs go to LDS.
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
    int bucket;               // 1: draws grouped by basis (draw_sort ran), 0: drawn here in order
    uint32_t *jlist;          // bucket: [batch][N] draws in drawing order (written by draw_sort)
    uint32_t *sorted;         // bucket: [batch][N] draws of each batch grouped by basis
    int32_t *perm;            // bucket, optional [batch][N]: draw index j of each sorted entry
    uint32_t *dbg_samples;    // no bucket, optional [batch][N] draws
    float *dbg_coef;          // optional [batch][N] (with bucket it needs perm)
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

// ------------------------------------------------------------ draw_sort --
constexpr int SORT_THREADS = 256;

// exclusive scan over the SORT_THREADS threads of a workgroup (sh holds
// SORT_THREADS / 64 + 1 ints); *total receives the sum
__device__ __forceinline__ int sort_block_scan(int v, int *total, int *sh) {
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
        for (int w = 0; w < SORT_THREADS / 64; ++w) {
            const int c = sh[w];
            sh[w] = run;
            run += c;
        }
        sh[SORT_THREADS / 64] = run;
    }
    __syncthreads();
    const int res = sh[wave] + incl - v;
    *total = sh[SORT_THREADS / 64];
    __syncthreads();
    return res;
}

// Draws of batch kb of vector t into a.jlist (drawing order) and a.sorted
// (grouped by basis, drawing order within a basis), and with a.perm the draw
// index of every sorted entry.  cur: LDS [(d/2 + 1) * 4] counters, indexed
// basis * 4 + wave; sh: SORT_THREADS / 64 + 1 ints.
__device__ __forceinline__ void draw_sort(const DGArgs &a, int t, int kb, uint32_t *cur, int *sh) {
    if (a.active && !a.active[t]) return;      // uniform over the workgroup
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int k = a.k, nbin = (1 << (k - 1)) + 1, J = a.J;
    const int64_t t0 = a.t0_dev ? *a.t0_dev : a.t0;
    const uint64_t pos = (uint64_t)(t0 + t);
    const uint64_t L = (uint64_t)a.L;
    const int J0 = kb * J;
    uint32_t *jl = a.jlist + (size_t)t * a.N + J0;
    uint32_t *so = a.sorted + (size_t)t * a.N + J0;
    int32_t *pm = a.perm ? a.perm + (size_t)t * a.N + J0 : nullptr;
    for (int i = threadIdx.x; i < nbin * 4; i += SORT_THREADS) cur[i] = 0;
    __syncthreads();

    // pass 1: Philox blocks c (draws 4c .. 4c + 3) of the batch, a
    // contiguous range of blocks per wave, one block per lane; histogram of
    // the bases per wave
    const int c_lo = J0 >> 2, c_hi = (J0 + J + 3) >> 2;
    const int bpw = (c_hi - c_lo + 3) / 4;
    const int wb = min(c_hi, c_lo + wave * bpw), we = min(c_hi, wb + bpw);
    for (int c0 = wb; c0 < we; c0 += 64) {
        const int c = c0 + lane;
        if (c < we) {
            uint64_t w4[4] = {(uint64_t)c, pos, 0, 0};
            philox4x64_10(w4, a.seed, 0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = 4 * c + u;
                if (j >= J0 && j < J0 + J) {
                    const uint32_t l = (uint32_t)__umul64hi(w4[u], L);
                    jl[j - J0] = l;
                    atomicAdd(&cur[(l >> k) * 4 + wave], 1u);
                }
            }
        }
    }
    __syncthreads();

    // start of every (basis, wave) range: exclusive scan in (basis, wave) order
    {
        const int tot = nbin * 4;
        const int per = (tot + SORT_THREADS - 1) / SORT_THREADS;
        const int i0 = min(tot, (int)threadIdx.x * per), i1 = min(tot, i0 + per);
        int local = 0;
        for (int i = i0; i < i1; ++i) local += (int)cur[i];
        int total;
        int run = sort_block_scan(local, &total, sh);
        for (int i = i0; i < i1; ++i) {
            const int c = (int)cur[i];
            cur[i] = (uint32_t)run;
            run += c;
        }
    }
    __syncthreads();

    // pass 2: every wave places its draws (the ones it drew, re-read in
    // drawing order, 64 at a time); lanes with equal bases are ranked by the
    // ballots of the bits of b, and the lowest of them advances the counter
    const int rb = max(4 * wb, J0) - J0, re = min(4 * we, J0 + J) - J0;
    constexpr int PF = 8;              // steps whose draws are loaded at once
    uint32_t lbuf[PF];
    for (int r0 = rb; r0 < re; r0 += 64) {
        const int step = ((r0 - rb) >> 6) % PF;
        if (step == 0)
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                const int rr = r0 + 64 * u + lane;
                lbuf[u] = rr < re ? jl[rr] : 0u;
            }
        const int r = r0 + lane;
        const bool valid = r < re;
        uint32_t l = lbuf[0];
#pragma unroll
        for (int u = 1; u < PF; ++u)
            if (step == u) l = lbuf[u];
        const uint32_t b = l >> k;
        uint64_t peers = __ballot(valid);
        for (int bit = 0; bit < k; ++bit) {
            const bool on = (b >> bit) & 1u;
            const uint64_t bal = __ballot(on);
            peers &= on ? bal : ~bal;
        }
        if (valid) {
            const int rank = __popcll(peers & ((1ull << lane) - 1ull));
            const uint32_t base = cur[b * 4 + wave];
            so[base + rank] = l;
            if (pm) pm[base + rank] = J0 + r;
            if (rank == 0) cur[b * 4 + wave] = base + (uint32_t)__popcll(peers);
        }
    }
}

// ------------------------------------------------------- coefficients --
// Runs of at least this many draws of one Kerdock basis use the per-basis
// transform; shorter runs sum directly (the transform costs about as much as
// three direct sums).
constexpr int BUCKET_MIN = 4;

// x in fixed point in LDS, shared by the waves of a workgroup: word p of
// lane `lane` (elements (lane + 64 p) 32 + q, q < 32) as eight 16-byte
// pieces, piece j at ((p 8 + j) 64 + lane) 16 bytes (consecutive lanes,
// consecutive pieces: no bank conflicts).
constexpr int XI_INTS_PER_P = 32 * 64;

__device__ __forceinline__ void load_xi_word(const int *s_xi, int p, int lane, int (&y)[32]) {
    const int4 *src = reinterpret_cast<const int4 *>(s_xi) + (size_t)p * 8 * 64 + lane;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int4 v = src[j * 64];
        y[4 * j] = v.x;
        y[4 * j + 1] = v.y;
        y[4 * j + 2] = v.z;
        y[4 * j + 3] = v.w;
    }
}

template <int P>
__device__ __forceinline__ void load_xi(const int *s_xi, int lane, int (&xi)[P][32]) {
#pragma unroll
    for (int p = 0; p < P; ++p) load_xi_word(s_xi, p, lane, xi[p]);
}

// fixed_point by one wave, written straight to LDS in the layout above;
// s_fx receives E2 and finite (0 / 1)
template <int P>
__device__ __forceinline__ void fixed_point_lds(const float *__restrict__ x, int n, int lane, int *s_xi, int *s_fx) {
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
    // the same scale as fixed_point: 2^E2 with asum 2^E2 <= 2^30
    const bool finite = asum < INFINITY;
    int E2 = 0;
    if (finite && asum > 0.f) E2 = 29 - ((int)((__float_as_uint(asum) >> 23) & 0xFF) - 127);
    E2 = max(-120, min(E2, 120));
    const float up = ldexpf(1.0f, E2);
    int4 *dst = reinterpret_cast<int4 *>(s_xi) + lane;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            int v[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = finite ? (int)rintf(xf[p][4 * j + c] * up) : 0;
            dst[(p * 8 + j) * 64] = make_int4(v[0], v[1], v[2], v[3]);
        }
    if (lane == 0) {
        s_fx[0] = E2;
        s_fx[1] = finite ? 1 : 0;
    }
}

// Direct signed sums of the draws at LDS positions list[0 .. cnt), or
// base .. base + cnt - 1 when list is NULL (one
// wave; four draws at a time so that the sign-word loads overlap).
template <int P>
__device__ __forceinline__ void direct_coefs(const int (&xi)[P][32], float down, bool finite,
                                             const float *__restrict__ x, int n, int k,
                                             const uint32_t *__restrict__ signs, const int *list, int base, int cnt,
                                             const uint32_t *s_ell, float *s_coef) {
    const int lane = threadIdx.x & 63;
    const int d = 1 << k;
    const int words = d >= 32 ? d / 32 : 1;
    const float sqrt_d = sqrtf((float)d);
    for (int jj0 = 0; jj0 < cnt; jj0 += 4) {
        uint32_t lq[4], sw[4][P];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int jp = min(jj0 + u, cnt - 1);
            lq[u] = s_ell[list ? list[jp] : base + jp];
            const uint32_t b = lq[u] >> k;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int word = lane + 64 * p;
                sw[u][p] = ((int)b < d / 2 && word < words) ? signs[(size_t)b * words + word] : 0u;
            }
        }
        // per-lane partial sums of the four draws, then one transposed
        // butterfly for all four: bits 5 and 4 of the lane pick the draw,
        // bits 3..0 finish the sums (exact integers)
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
                    for (int q = 0; q < 32; ++q) acc += xi[p][q] ^ (int)__builtin_amdgcn_sbfe(mask, q, 1);
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
            if (jj0 + u >= cnt) break;
            const uint32_t b = lq[u] >> k, w = lq[u] & (uint32_t)(d - 1);
            float c;
            if ((int)b == d / 2) {
                c = ((int)w < n) ? sqrt_d * x[w] : 0.f;
            } else {
                const int tot = __builtin_amdgcn_readlane(z, ((u >> 1) << 5) | ((u & 1) << 4));
                c = finite ? (float)tot * down : __builtin_nanf("");
            }
            if (lane == 0) s_coef[list ? list[jj0 + u] : base + jj0 + u] = c;
        }
    }
}

// A run of cnt >= 1 draws of Kerdock basis b at LDS positions i0 .. i0 + cnt
// (one wave): y = sigma_b x, Y = the 32-point Walsh-Hadamard transform of
// each lane's word, then c = sum over lanes and words of
// (-1)^{parity(word & w_hi)} Y[w_lo] for each draw.
template <int P>
__device__ __forceinline__ void transform_run(const int *s_xi, float down, bool finite, int k, uint32_t b,
                                              const uint32_t *__restrict__ signs, int i0, int cnt,
                                              const uint32_t *s_ell, float *s_coef) {
    typedef int i32x32 __attribute__((ext_vector_type(32)));
    const int lane = threadIdx.x & 63;
    const int d = 1 << k;
    const int words = d >= 32 ? d / 32 : 1;
    i32x32 Y[P];        // vectors, so that a wave-uniform index picks a register
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int word = lane + 64 * p;
        const uint32_t sw = word < words ? signs[(size_t)b * words + word] : 0u;
        int y[32];
        load_xi_word(s_xi, p, lane, y);
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            const int m = (int)__builtin_amdgcn_sbfe(sw, q, 1);
            y[q] = (y[q] ^ m) - m;
        }
#pragma unroll
        for (int h = 1; h < 32; h <<= 1)
#pragma unroll
            for (int q = 0; q < 32; ++q)
                if ((q & h) == 0) {
                    const int u = y[q], v = y[q + h];
                    y[q] = u + v;
                    y[q + h] = u - v;
                }
#pragma unroll
        for (int q = 0; q < 32; ++q) Y[p][q] = y[q];
    }
    for (int jj0 = 0; jj0 < cnt; jj0 += 4) {
        int part[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t l = __builtin_amdgcn_readfirstlane(s_ell[i0 + min(jj0 + u, cnt - 1)]);
            const uint32_t w = l & (uint32_t)(d - 1);
            const int wlo = (int)__builtin_amdgcn_readfirstlane(w & 31u);
            int acc = 0;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const uint32_t word = (uint32_t)(lane + 64 * p);
                const int neg = -(int)(__popc(word & (w >> 5)) & 1u);
                acc += (Y[p][wlo] ^ neg) - neg;
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
            if (jj0 + u >= cnt) break;
            const int tot = __builtin_amdgcn_readlane(z, ((u >> 1) << 5) | ((u & 1) << 4));
            if (lane == 0) s_coef[i0 + jj0 + u] = finite ? (float)tot * down : __builtin_nanf("");
        }
    }
}

// Coefficients of the cnt (<= MAX_CHUNK) sorted draws in s_ell into s_coef;
// the four waves take equal contiguous runs of positions, split them into
// runs of one basis, transform the long Kerdock runs and collect the other
// positions in s_list (same positions, so the waves' lists never overlap)
// for the direct sums.  The caller synchronises before and after.
template <int P>
__device__ __forceinline__ void bucket_coefs(const float *__restrict__ x, int n, int k,
                                             const uint32_t *__restrict__ signs, int cnt, const uint32_t *s_ell,
                                             float *s_coef, int *s_list, const int *s_xi, int E2, bool finite) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int d = 1 << k;
    const float down = ldexpf(1.0f, -E2);
    const int per = ((cnt + 3) / 4 + 3) & ~3;
    const int r0 = min(cnt, wave * per), r1 = min(cnt, r0 + per);
    int nd = 0;
    for (int i = r0; i < r1;) {
        const uint32_t b = __builtin_amdgcn_readfirstlane(s_ell[i] >> k);
        int run = 0;
        for (;;) {
            const int q = i + run + lane;
            const uint64_t same = __ballot(q < r1 && (s_ell[q] >> k) == b);
            const int c = same == ~0ull ? 64 : __ffsll((long long)~same) - 1;
            run += c;
            if (c < 64) break;
        }
        if ((int)b < d / 2 && run >= BUCKET_MIN) {
            transform_run<P>(s_xi, down, finite, k, b, signs, i, run, s_ell, s_coef);
        } else {
            for (int q = lane; q < run; q += 64) s_list[r0 + nd + q] = i + q;
            nd += run;
        }
        i += run;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (nd > 0) {
        int xi[P][32];
        load_xi<P>(s_xi, lane, xi);
        direct_coefs<P>(xi, down, finite, x, n, k, signs, s_list + r0, 0, nd, s_ell, s_coef);
    }
}

// LDS of one draws + gather workgroup: the draws, coefficients, direct-sum
// list and fixed-point x of phase 1, then (aliasing them once phase 2 has
// read the last pair) the group sums of short columns.
// BK: the kernel can take draws grouped by basis (their list and x in
// fixed point live in LDS); without it only (l, c) pairs are staged
template <int DT, bool GROUPED, int P, bool BK = true> struct DGSmem {
    static constexpr size_t PHASE1 =
        BK ? 3 * MAX_CHUNK * 4 + (size_t)P * XI_INTS_PER_P * 4 + 16 : 2 * MAX_CHUNK * 4;
    static constexpr size_t RED = GROUPED ? (size_t)GATHER_THREADS * Elems<DT>::N * 4 : 0;
    static constexpr size_t BYTES = PHASE1 > RED ? PHASE1 : RED;
};

// BK = false: a kernel that never takes grouped draws (a.bucket must be 0);
// it leaves out that path and its registers
template <int DT, int TILES, int UNROLL, bool GROUPED, int P, bool BK = true>
__device__ __forceinline__ void draw_gather(const DGArgs &a, int t, int cid, int seg, int nchunks,
                                            unsigned char *smem) {
    uint32_t *s_ell = reinterpret_cast<uint32_t *>(smem);
    float *s_coef = reinterpret_cast<float *>(smem + MAX_CHUNK * 4);
    int *s_list = reinterpret_cast<int *>(smem + 2 * MAX_CHUNK * 4);
    int *s_xi = reinterpret_cast<int *>(smem + 3 * MAX_CHUNK * 4);
    int *s_fx = s_xi + P * XI_INTS_PER_P;             // E2, finite
    float *red = reinterpret_cast<float *>(smem);
    const unsigned char *__restrict__ table = a.table;
    const int col_bytes = a.col_bytes, n = a.n, k = a.k, N = a.N, J = a.J, chunk = a.chunk;
    const int chunks_per_batch = a.chunks_per_batch, groups = a.groups, tpc = a.tpc, pitch = a.pitch;
    const float *__restrict__ X = a.X;
    const uint32_t *__restrict__ signs = a.signs;
    float *__restrict__ partial = a.partial;
    float *__restrict__ dbg_coef = a.dbg_coef;
    constexpr int E = Elems<DT>::N;
    if (a.active && !a.active[t]) return;      // uniform over the workgroup
    const int kb = cid / chunks_per_batch, cj = cid % chunks_per_batch;
    const int jbeg = kb * J + cj * chunk;
    const int cnt = min(chunk, (kb + 1) * J - jbeg);

    // ---------------------------------------------------------- phase 1
    const int per = ((cnt + 3) / 4 + 3) & ~3;          // the waves' runs of positions
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r0 = min(cnt, wave * per), r1 = min(cnt, r0 + per);
    if (BK && a.bucket) {
        // the batch's draws grouped by basis (draw_sort), x in fixed point
        // shared through LDS by wave 0, then the four waves' runs
        const uint32_t *src = a.sorted + (size_t)t * N + jbeg;
        for (int r = threadIdx.x; r < cnt; r += GATHER_THREADS) s_ell[r] = src[r];
        if (threadIdx.x < 64) fixed_point_lds<P>(X + (size_t)t * n, n, threadIdx.x, s_xi, s_fx);
        __syncthreads();
        bucket_coefs<P>(X + (size_t)t * n, n, k, signs, cnt, s_ell, s_coef, s_list, s_xi, s_fx[0], s_fx[1] != 0);
    } else {
        // every wave on its own run of positions: x in fixed point (in
        // registers), draw j = jbeg + r as word j mod 4 of Philox4x64-10 at
        // counter (floor(j/4), t0 + t, 0, 0), key (seed, 0), l = floor(r L /
        // 2^64), and the direct sums
        int xi[P][32];
        int E2;
        bool finite;
        fixed_point<P>(X + (size_t)t * n, n, lane, xi, E2, finite);
        const int64_t t0 = a.t0_dev ? *a.t0_dev : a.t0;
        for (int r = r0 + lane; r < r1; r += 64) {
            const int j = jbeg + r;
            uint64_t c4[4] = {(uint64_t)(j >> 2), (uint64_t)(t0 + t), 0, 0};
            philox4x64_10(c4, a.seed, 0);
            const uint64_t rr = (j & 3) == 0 ? c4[0] : (j & 3) == 1 ? c4[1] : (j & 3) == 2 ? c4[2] : c4[3];
            s_ell[r] = (uint32_t)__umul64hi(rr, (uint64_t)a.L);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        direct_coefs<P>(xi, ldexpf(1.0f, -E2), finite, X + (size_t)t * n, n, k, signs, nullptr, r0, r1 - r0, s_ell,
                        s_coef);
    }
    __syncthreads();
    if (dbg_coef && seg == 0) {
        if (BK && a.bucket) {
            for (int r = threadIdx.x; r < cnt; r += GATHER_THREADS)
                dbg_coef[(size_t)t * N + a.perm[(size_t)t * N + jbeg + r]] = s_coef[r];
        } else {
            for (int r = threadIdx.x; r < cnt; r += GATHER_THREADS) {
                a.dbg_samples[(size_t)t * N + jbeg + r] = s_ell[r];
                dbg_coef[(size_t)t * N + jbeg + r] = s_coef[r];
            }
        }
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
        if (j < cnt) {
            // the last draws (fewer than UNROLL): their loads issued
            // together, accumulated in the same order
            u32x4 raw[UNROLL][TILES];
            float cc[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const bool on = j + u * gstride < cnt;
                const uint32_t l = on ? s_ell[j + u * gstride] : 0u;
                cc[u] = on ? s_coef[j + u * gstride] : 0.f;
                const unsigned char *colp = base + (size_t)l * (size_t)col_bytes;
#pragma unroll
                for (int ti = 0; ti < TILES; ++ti)
                    raw[u][ti] = (on && tile_on[ti]) ? __builtin_nontemporal_load(
                                                           reinterpret_cast<const u32x4 *>(colp + ti * TILE_BYTES))
                                                     : u32x4{0u, 0u, 0u, 0u};
            }
#pragma unroll
            for (int u = 0; u < UNROLL; ++u)
                if (j + u * gstride < cnt)
#pragma unroll
                    for (int ti = 0; ti < TILES; ++ti) accumulate<DT>(acc[ti], raw[u][ti], cc[u]);
        }
    }

    if constexpr (GROUPED) {
        __syncthreads();               // every (l, c) pair read: red reuses their LDS
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

// TH threads (a multiple of 64); sh holds TH / 64 + 1 ints
template <int TH = SELECT_THREADS>
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
        for (int w = 0; w < TH / 64; ++w) {
            const int c = sh[w];
            sh[w] = run;
            run += c;
        }
        sh[TH / 64] = run;
    }
    __syncthreads();
    const int res = sh[wave] + incl - v;
    *total = sh[TH / 64];
    __syncthreads();
    return res;
}

// The s_max largest keys (ties: smaller index), optionally only keys >=
// tau_bits, written in ascending index order to surv_row (padded with -1),
// their number to *nsurv_out.  Radix select over the 32-bit keys in LDS
// (8 bits per round, histogram in LDS), then two block-wide scans; TH >= 256
// threads (the result does not depend on TH).
template <int TH = SELECT_THREADS>
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
            for (int i = threadIdx.x; i < m; i += TH) {
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
    const int per = (m + TH - 1) / TH;
    const int i0 = min(m, (int)threadIdx.x * per), i1 = min(m, i0 + per);
    int eq_local = 0;
    if (!take_all)
        for (int i = i0; i < i1; ++i) eq_local += key[i] == theta;
    int eq_total;
    int eq_rank = block_exclusive_scan<TH>(eq_local, &eq_total, scan_sh);
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
    int pos = block_exclusive_scan<TH>(sel_local, &total, scan_sh);
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
    for (int s = total + threadIdx.x; s < s_max; s += TH) surv_row[s] = -1;
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

// shared memory: key[m], hist[256], scan_sh[TH/64 + 1], sel_state[2]; TH
// threads (the result does not depend on TH)
template <int KMAX, int TH = SELECT_THREADS>
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
    // R rows per thread (i0 + r TH) with all their loads of a round issued
    // together; each row's partials are still summed in chunk order
    constexpr int R = KMAX <= 8 ? 4 : 1;
    for (int i0 = threadIdx.x; i0 < m; i0 += R * TH) {
        float v[R][KMAX];
#pragma unroll
        for (int a = 0; a < KMAX; ++a) {
            float sr[R];
#pragma unroll
            for (int r = 0; r < R; ++r) sr[r] = INFINITY;
            if (a < K) {
                const float *pa = pt + (size_t)a * chunks_per_batch * pitch;
#pragma unroll
                for (int r = 0; r < R; ++r) sr[r] = 0.f;
                int c = 0;
                for (; c + 8 <= chunks_per_batch; c += 8) {
                    float q[R][8];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int i = min(i0 + r * TH, m - 1);
#pragma unroll
                        for (int u = 0; u < 8; ++u) q[r][u] = pa[(size_t)(c + u) * pitch + i];
                    }
#pragma unroll
                    for (int r = 0; r < R; ++r)
#pragma unroll
                        for (int u = 0; u < 8; ++u) sr[r] += q[r][u];
                }
                for (; c < chunks_per_batch; ++c) {
#pragma unroll
                    for (int r = 0; r < R; ++r) sr[r] += pa[(size_t)c * pitch + min(i0 + r * TH, m - 1)];
                }
#pragma unroll
                for (int r = 0; r < R; ++r) sr[r] = sr[r] / (float)J;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) v[r][a] = sr[r];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = i0 + r * TH;
            if (i >= m) break;
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
                            const float lo = fminf(v[r][a], v[r][bb]), hi = fmaxf(v[r][a], v[r][bb]);
                            v[r][a] = up ? lo : hi;
                            v[r][bb] = up ? hi : lo;
                        }
                    }
            float lo_mid = 0.f, hi_mid = 0.f;
#pragma unroll
            for (int a = 0; a < KMAX; ++a) {
                if (a == (K - 1) / 2) lo_mid = v[r][a];
                if (a == K / 2) hi_mid = v[r][a];
            }
            float med = (K & 1) ? hi_mid : 0.5f * (lo_mid + hi_mid);
            med *= scales[i];
            if (mu_out) mu_out[(size_t)t * m + i] = med;
            key[i] = __float_as_uint(fabsf(med));
        }
    }
    __syncthreads();
    select_top<TH>(key, m, s_max, __float_as_uint(fmaxf(tau, 0.f)), surv + (size_t)t * s_max, nsurv + t, hist,
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
// in pieces, elements l, l + 64, ... into one cascade).  For waves that take
// many dots in turn (few registers, so more waves hide the loads).
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

// The same dot with all pieces of the row and of x loaded before the steps
// (n <= 4096: at most 16 pieces per lane), for a wave that takes one dot:
// one round of loads instead of four.  Same steps in the same order.
__device__ __forceinline__ float survivor_dot_once(const float *__restrict__ row, const float *__restrict__ x,
                                                   int n, int vec4) {
    const int lane = threadIdx.x & 63;
    if (!vec4) return survivor_dot(row, x, n, vec4);
    float p[4] = {0.f, 0.f, 0.f, 0.f}, e[4] = {0.f, 0.f, 0.f, 0.f};
    const float4 *__restrict__ r4 = reinterpret_cast<const float4 *>(row);
    const float4 *__restrict__ x4 = reinterpret_cast<const float4 *>(x);
    const int n4 = n >> 2;
    float4 ra[16], xa[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int q = lane + 64 * i;
        ra[i] = q < n4 ? r4[q] : make_float4(0.f, 0.f, 0.f, 0.f);
        xa[i] = q < n4 ? x4[q] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (lane + 64 * i < n4) {
            dot_step(p[0], e[0], ra[i].x, xa[i].x);
            dot_step(p[1], e[1], ra[i].y, xa[i].y);
            dot_step(p[2], e[2], ra[i].z, xa[i].z);
            dot_step(p[3], e[3], ra[i].w, xa[i].w);
        }
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
    const float v = survivor_dot_once(a.A + (size_t)a.surv[(size_t)t * a.s_max + s] * a.n,
                                      a.X + (size_t)t * a.n, a.n, a.vec4);
    if ((threadIdx.x & 63) == 0) a.svals[(size_t)t * a.s_max + s] = v;
}

}  // namespace kd
