// Streaming-step kernels (Algorithm 1 streaming step, Theorem 5) for gfx950.
//
//   k_sample_coef  draw l_j uniformly from [L] (Philox4x64-10) and compute the
//                  coefficient c_j = s_{l_j}^T x: a signed Walsh sum of x for
//                  Kerdock vectors, sqrt(d) x[w] for identity vectors;
//   k_gather       the hot loop: stream the drawn table columns from HBM and
//                  accumulate c_j T[l_j] per chunk of draws of one batch;
//   k_select       batch means, entrywise median over the K batches, and the
//                  s_max rows of largest |mu| (ties: smaller index) by an
//                  LDS radix select, compacted in ascending row order;
//   k_survivors    exact a_i.x on the selected rows (compensated FP32 dot
//                  product, Ogita-Rump-Oishi Dot2) and the eps threshold.
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

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ------------------------------------------------------------ draws + c_j --
// Draw j of vector t: block floor(j/4) of Philox4x64-10 at counter
// (floor(j/4), t0 + t, 0, 0), key (seed, 0), word j mod 4; l = floor(r L / 2^64).
// One wave handles 64 consecutive draws.  Lane l holds x[e] for
// e = (l + 64 p) * 32 + q, q < 32, so that the sign word (l + 64 p) of basis b
// carries Q_b(e) in bit q; with w = (w_hi, w_lo) the Walsh sign is
// parity((l + 64 p) & w_hi) ^ parity(q & w_lo).
template <int P>
__global__ __launch_bounds__(256) void k_sample_coef(const float *__restrict__ X, int n, int k,
                                                     int64_t L, const uint32_t *__restrict__ signs,
                                                     uint64_t seed, int64_t t0, int N,
                                                     uint32_t *__restrict__ samples,
                                                     float *__restrict__ coef) {
    const int t = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int j0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 64;
    if (j0 >= N) return;
    const int d = 1 << k;
    const int words = d >= 32 ? d / 32 : 1;
    const float *x = X + (size_t)t * n;

    float xv[P][32];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            const int e = (lane + 64 * p) * 32 + q;
            xv[p][q] = e < n ? x[e] : 0.f;
        }

    uint32_t ell[4];
    {
        uint64_t c[4] = {(uint64_t)(j0 / 4 + lane), (uint64_t)(t0 + t), 0, 0};
        philox4x64_10(c, seed, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) ell[q] = (uint32_t)__umul64hi(c[q], (uint64_t)L);
    }

    const float sqrt_d = sqrtf((float)d);
    float my_coef = 0.f;
    uint32_t my_ell = 0;
    const int jcount = min(64, N - j0);
    for (int jb = 0; jb * 4 < jcount; ++jb) {
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
            const int jj = jb * 4 + q4;
            if (jj >= jcount) continue;
            const uint32_t l = __builtin_amdgcn_readlane(ell[q4], jb);
            const uint32_t b = l >> k, w = l & (uint32_t)(d - 1);
            float c;
            if ((int)b == d / 2) {
                c = ((int)w < n) ? sqrt_d * x[w] : 0.f;
            } else {
                const uint32_t wlo = walsh32(w & 31u);
                float part = 0.f;
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const uint32_t word = (uint32_t)(lane + 64 * p);
                    if ((int)word < words) {
                        const uint32_t sw = signs[(size_t)b * words + word];
                        const uint32_t par = __popc(word & (w >> 5)) & 1u;
                        const uint32_t mask = sw ^ wlo ^ (0u - par);
#pragma unroll
                        for (int q = 0; q < 32; ++q)
                            part += ((mask >> q) & 1u) ? -xv[p][q] : xv[p][q];
                    }
                }
                c = wave_sum(part);
            }
            if (lane == jj) {
                my_coef = c;
                my_ell = l;
            }
        }
    }
    if (j0 + lane < N) {
        samples[(size_t)t * N + j0 + lane] = my_ell;
        coef[(size_t)t * N + j0 + lane] = my_coef;
    }
}

// ----------------------------------------------------------------- gather --
// Each workgroup owns one 4 KiB segment of every column and one chunk of the
// draws of one batch of one vector; each thread owns 16 bytes of the segment
// (4 FP32, 8 BF16 or 16 FP8 elements) and keeps FP32 accumulators in
// registers.  UNROLL independent 16-byte loads are in flight per thread.
// When a column is shorter than 4 KiB, the workgroup splits into `groups`
// groups of `tpc` threads that take interleaved draws and are summed in LDS
// at the end.  The FP8 row scale is applied once, in k_select.
template <int DT> struct Elems { static constexpr int N = DT == KERDOCK_F32 ? 4 : DT == KERDOCK_BF16 ? 8 : 16; };

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

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
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc[4 * e + s] = fmaf(c, e4m3_to_f32((w[e] >> (8 * s)) & 0xFFu), acc[4 * e + s]);
    }
}

constexpr int GATHER_THREADS = 256;
constexpr int SEG_BYTES = GATHER_THREADS * 16;

template <int DT, int UNROLL, bool GROUPED>
__global__ __launch_bounds__(GATHER_THREADS) void k_gather(
    const unsigned char *__restrict__ table, int col_bytes, const uint32_t *__restrict__ samples,
    const float *__restrict__ coef, int N, int J, int chunk, int chunks_per_batch, int groups,
    int tpc, int pitch, float *__restrict__ partial) {
    constexpr int E = Elems<DT>::N;
    const int t = blockIdx.z;
    const int seg = blockIdx.y;
    const int cid = blockIdx.x;
    const int kb = cid / chunks_per_batch, cj = cid % chunks_per_batch;
    const int jbeg = kb * J + cj * chunk;
    const int jend = min(jbeg + chunk, (kb + 1) * J);
    const int g = GROUPED ? (int)threadIdx.x / tpc : 0;
    const int r = GROUPED ? (int)threadIdx.x % tpc : (int)threadIdx.x;
    const int gstride = GROUPED ? groups : 1;
    const size_t byte_off = (size_t)seg * SEG_BYTES + (size_t)r * 16;
    const bool active = (g < gstride) && byte_off < (size_t)col_bytes;

    float acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = 0.f;

    const uint32_t *sp = samples + (size_t)t * N;
    const float *cp = coef + (size_t)t * N;
    if (active) {
        const unsigned char *base = table + byte_off;
        int j = jbeg + g;
        for (; j + (UNROLL - 1) * gstride < jend; j += UNROLL * gstride) {
            u32x4 raw[UNROLL];
            float cc[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const uint32_t l = sp[j + u * gstride];
                cc[u] = cp[j + u * gstride];
                raw[u] = __builtin_nontemporal_load(
                    reinterpret_cast<const u32x4 *>(base + (size_t)l * (size_t)col_bytes));
            }
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) accumulate<DT>(acc, raw[u], cc[u]);
        }
        for (; j < jend; j += gstride) {
            const uint32_t l = sp[j];
            const u32x4 raw = __builtin_nontemporal_load(
                reinterpret_cast<const u32x4 *>(base + (size_t)l * (size_t)col_bytes));
            accumulate<DT>(acc, raw, cp[j]);
        }
    }

    if constexpr (GROUPED) {
        __shared__ float red[GATHER_THREADS * E];
#pragma unroll
        for (int e = 0; e < E; ++e) red[e * GATHER_THREADS + threadIdx.x] = acc[e];
        __syncthreads();
        if (g != 0 || !active) return;
        for (int gg = 1; gg < groups; ++gg)
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] += red[e * GATHER_THREADS + gg * tpc + r];
    } else {
        if (!active) return;
    }
    const size_t nchunks = (size_t)gridDim.x;
    float *dst = partial + ((size_t)t * nchunks + cid) * pitch + byte_off / (16 / E);
#pragma unroll
    for (int e = 0; e < E; e += 4)
        *reinterpret_cast<float4 *>(dst + e) = make_float4(acc[e], acc[e + 1], acc[e + 2], acc[e + 3]);
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

template <int KMAX>
__global__ __launch_bounds__(SELECT_THREADS) void k_select(
    const float *__restrict__ partial, int m, int pitch, int K, int chunks_per_batch, int J,
    const float *__restrict__ scales, int s_max, float tau, float *__restrict__ mu_out,
    int32_t *__restrict__ surv, int32_t *__restrict__ nsurv) {
    extern __shared__ uint32_t key[];          // [m] bits of |mu|
    __shared__ uint32_t hist[256];
    __shared__ int scan_sh[SELECT_THREADS / 64 + 1];
    __shared__ uint32_t sel_prefix, sel_want;

    const int t = blockIdx.x;
    const int nchunks = K * chunks_per_batch;
    const float *pt = partial + (size_t)t * nchunks * pitch;
    for (int i = threadIdx.x; i < m; i += SELECT_THREADS) {
        float v[KMAX];
#pragma unroll
        for (int a = 0; a < KMAX; ++a) {
            float s = INFINITY;
            if (a < K) {
                s = 0.f;
                for (int c = 0; c < chunks_per_batch; ++c)
                    s += pt[(size_t)(a * chunks_per_batch + c) * pitch + i];
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
    const uint32_t tau_bits = __float_as_uint(fmaxf(tau, 0.f));

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
            if (sel && pos < s_max) surv[(size_t)t * s_max + pos++] = i;
        }
    }
    total = min(total, s_max);
    for (int s = total + threadIdx.x; s < s_max; s += SELECT_THREADS) surv[(size_t)t * s_max + s] = -1;
    if (threadIdx.x == 0) nsurv[t] = total;
}

// ------------------------------------------------------------- survivors --
// Dot2 (Ogita, Rump, Oishi, "Accurate sum and dot product", SIAM J. Sci.
// Comput. 2005): error-free products and sums, so the FP32 result is as
// accurate as if computed in twice the working precision.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
#pragma clang fp contract(off)
    s = a + b;
    const float z = s - a;
    e = (a - (s - z)) + (b - z);
}

__global__ __launch_bounds__(256) void k_survivors(
    const float *__restrict__ A, int n, const float *__restrict__ X,
    const int32_t *__restrict__ surv, const int32_t *__restrict__ nsurv, int s_max, float eps,
    int32_t *__restrict__ out_idx, float *__restrict__ out_val, int32_t *__restrict__ out_cnt,
    float *__restrict__ dbg_values) {
#pragma clang fp contract(off)
    extern __shared__ float vals[];
    const int t = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ns = min(nsurv[t], s_max);
    const float *x = X + (size_t)t * n;
    for (int s = wave; s < ns; s += 4) {
        const int i = surv[(size_t)t * s_max + s];
        const float *row = A + (size_t)i * n;
        float p = 0.f, e = 0.f;
        for (int q = lane; q < n; q += 64) {
            const float a = row[q], b = x[q];
            const float h = a * b;
            const float rr = fmaf(a, b, -h);
            float sum, err;
            two_sum(p, h, sum, err);
            p = sum;
            e = e + (err + rr);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float p2 = __shfl_xor(p, off), e2 = __shfl_xor(e, off);
            float sum, err;
            two_sum(p, p2, sum, err);
            p = sum;
            e = e + e2 + err;
        }
        if (lane == 0) vals[s] = p + e;
    }
    __syncthreads();
    if (wave != 0) return;
    int base = 0;
    for (int s0 = 0; s0 < s_max; s0 += 64) {
        const int s = s0 + lane;
        const bool keep = s < ns && fabsf(vals[s]) >= eps;
        const uint64_t mask = __ballot(keep);
        const int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (keep) {
            out_idx[(size_t)t * s_max + pos] = surv[(size_t)t * s_max + s];
            out_val[(size_t)t * s_max + pos] = vals[s];
        }
        base += __popcll(mask);
    }
    for (int s = base + lane; s < s_max; s += 64) {
        out_idx[(size_t)t * s_max + s] = -1;
        out_val[(size_t)t * s_max + s] = 0.f;
    }
    if (dbg_values)
        for (int s = lane; s < s_max; s += 64) dbg_values[(size_t)t * s_max + s] = s < ns ? vals[s] : 0.f;
    if (lane == 0) out_cnt[t] = base;
}

// -------------------------------------------------------------- launchers --

int launch_sample_coef(const float *X, int batch, int n, int k, int64_t L, const uint32_t *signs,
                       uint64_t seed, int64_t t0, int N, uint32_t *samples, float *coef,
                       hipStream_t s) {
    const int waves = (N + 63) / 64;
    dim3 grid((waves + 3) / 4, batch);
    if (n <= 2048)
        hipLaunchKernelGGL(k_sample_coef<1>, grid, dim3(256), 0, s, X, n, k, L, signs, seed, t0, N, samples, coef);
    else
        hipLaunchKernelGGL(k_sample_coef<2>, grid, dim3(256), 0, s, X, n, k, L, signs, seed, t0, N, samples, coef);
    KD_LAUNCH("k_sample_coef");
    return KERDOCK_OK;
}

// geometry of the gather for one handle
struct GatherShape {
    int col_bytes, segs, groups, tpc, grouped;
};

GatherShape gather_shape(kerdock_dtype dt, int pitch) {
    GatherShape g;
    g.col_bytes = pitch * (int)dtype_bytes(dt);
    g.segs = (g.col_bytes + SEG_BYTES - 1) / SEG_BYTES;
    if (g.col_bytes >= SEG_BYTES) {
        g.groups = 1;
        g.tpc = GATHER_THREADS;
        g.grouped = 0;
    } else {
        g.tpc = g.col_bytes / 16;
        g.groups = GATHER_THREADS / g.tpc;
        g.grouped = 1;
    }
    return g;
}

template <int DT, int U>
static void gather_dt(dim3 grid, const GatherShape &g, const void *table, const uint32_t *samples,
                      const float *coef, int N, int J, int chunk, int cpb, int pitch, float *partial,
                      hipStream_t s) {
    const unsigned char *tb = reinterpret_cast<const unsigned char *>(table);
    if (g.grouped)
        hipLaunchKernelGGL((k_gather<DT, U, true>), grid, dim3(GATHER_THREADS), 0, s, tb, g.col_bytes,
                           samples, coef, N, J, chunk, cpb, g.groups, g.tpc, pitch, partial);
    else
        hipLaunchKernelGGL((k_gather<DT, U, false>), grid, dim3(GATHER_THREADS), 0, s, tb, g.col_bytes,
                           samples, coef, N, J, chunk, cpb, g.groups, g.tpc, pitch, partial);
}

int launch_gather(kerdock_dtype dt, const void *table, int pitch, const uint32_t *samples,
                  const float *coef, int batch, int N, int J, int K, int chunk, int unroll,
                  float *partial, hipStream_t s) {
    const GatherShape g = gather_shape(dt, pitch);
    const int cpb = (J + chunk - 1) / chunk;
    dim3 grid(K * cpb, g.segs, batch);
#define KD_GATHER_U(DT)                                                                       \
    switch (unroll) {                                                                         \
    case 4: gather_dt<DT, 4>(grid, g, table, samples, coef, N, J, chunk, cpb, pitch, partial, s); break; \
    case 16: gather_dt<DT, 16>(grid, g, table, samples, coef, N, J, chunk, cpb, pitch, partial, s); break; \
    default: gather_dt<DT, 8>(grid, g, table, samples, coef, N, J, chunk, cpb, pitch, partial, s); break; \
    }
    switch (dt) {
    case KERDOCK_F32: KD_GATHER_U(KERDOCK_F32) break;
    case KERDOCK_BF16: KD_GATHER_U(KERDOCK_BF16) break;
    case KERDOCK_FP8E4M3: KD_GATHER_U(KERDOCK_FP8E4M3) break;
    }
#undef KD_GATHER_U
    KD_LAUNCH("k_gather");
    return KERDOCK_OK;
}

int launch_select(const float *partial, int batch, int m, int pitch, int K, int cpb, int J,
                  const float *scales, int s_max, float tau, float *mu_out, int32_t *surv,
                  int32_t *nsurv, hipStream_t s) {
    const size_t shmem = (size_t)m * sizeof(uint32_t);
    dim3 grid(batch), block(SELECT_THREADS);
#define KD_SEL(KM)                                                                            \
    hipLaunchKernelGGL(k_select<KM>, grid, block, shmem, s, partial, m, pitch, K, cpb, J, scales, \
                       s_max, tau, mu_out, surv, nsurv)
    if (K <= 1) KD_SEL(1);
    else if (K <= 2) KD_SEL(2);
    else if (K <= 4) KD_SEL(4);
    else if (K <= 8) KD_SEL(8);
    else if (K <= 16) KD_SEL(16);
    else KD_SEL(32);
#undef KD_SEL
    KD_LAUNCH("k_select");
    return KERDOCK_OK;
}

int launch_survivors(const float *A, int n, const float *X, int batch, const int32_t *surv,
                     const int32_t *nsurv, int s_max, float eps, int32_t *out_idx, float *out_val,
                     int32_t *out_cnt, float *dbg_values, hipStream_t s) {
    hipLaunchKernelGGL(k_survivors, dim3(batch), dim3(256), (size_t)s_max * sizeof(float), s, A, n,
                       X, surv, nsurv, s_max, eps, out_idx, out_val, out_cnt, dbg_values);
    KD_LAUNCH("k_survivors");
    return KERDOCK_OK;
}

}  // namespace kd
