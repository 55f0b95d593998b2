// Preprocessing kernels (Algorithm 1 preprocessing step, Lemma 8) for gfx950.
//
// For every Kerdock basis b < d/2 and row i of A the table holds the
// unnormalised Walsh-Hadamard transform of the signed, zero-padded row:
//   T[b d + w][i] = sum_{x < n} A[i][x] (-1)^{Q_b(x)} (-1)^{popcount(x & w)},
// which equals (A sqrt(d) Pi u_{M_b, w})_i because sqrt(d) 2^{-k/2} = 1
// (equation (3) and the proof of Lemma 8: columns of A sqrt(d) Pi D_M H^k).
// The identity block b = d/2 holds sqrt(d) A e_w (zero for w >= n).
//
// Layout in HBM: column l = b d + w is `pitch` contiguous elements (rows
// i = 0..pitch-1, rows >= m are zero), so that the streaming step reads one
// contiguous column per draw.
#include <stdlib.h>

#include "common.hpp"

namespace kd {

// ------------------------------------------------------------------ signs --
// Bit x mod 32 of word x/32 of basis b is Q_b(x) = sum_{i<j} M_ij x_i x_j,
// evaluated as parity( sum_{i : x_i = 1} popcount(x & U_b[i]) ) where U_b[i]
// holds the strict upper triangle of row i.
__global__ void k_signs(const uint16_t *__restrict__ masks, int k, int words_per_basis,
                        int nbases, uint32_t *__restrict__ signs) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nbases * words_per_basis) return;
    const int b = gid / words_per_basis;
    const int word = gid % words_per_basis;
    uint32_t U[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) U[i] = (i < k) ? masks[b * k + i] : 0u;
    uint32_t bits = 0;
    const int d = 1 << k;
    for (int q = 0; q < 32; ++q) {
        const uint32_t x = (uint32_t)(word * 32 + q);
        if ((int)x >= d) break;
        uint32_t acc = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if ((x >> i) & 1u) acc += __popc(x & U[i]);
        bits |= (acc & 1u) << q;
    }
    signs[gid] = bits;
}

// ------------------------------------------------------------- row scales --
// FP8 tables: scale_i = max(|a_i|_1, sqrt(d) |a_i|_inf) / 448 bounds every
// |T[l]_i| (a Kerdock entry is a signed sum of a_i, an identity entry is
// sqrt(d) a_i[w]), so a single pass can quantise.  Other dtypes: 1.
__global__ void k_row_scales(const float *__restrict__ A, int m, int n, int pitch, float sqrt_d,
                             int fp8, float *__restrict__ scales, float *__restrict__ norm2) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= pitch) return;
    float l1 = 0.f, linf = 0.f, l2 = 0.f;
    if (row < m) {
        for (int x = lane; x < n; x += 64) {
            float a = fabsf(A[(size_t)row * n + x]);
            l1 += a;
            l2 += a * a;
            linf = fmaxf(linf, a);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        l1 += __shfl_xor(l1, off);
        l2 += __shfl_xor(l2, off);
        linf = fmaxf(linf, __shfl_xor(linf, off));
    }
    if (lane == 0 && norm2) norm2[row] = row < m ? l2 : 0.f;
    if (lane == 0) {
        float s = 1.0f;
        if (fp8 && row < m) {
            float bound = fmaxf(l1, sqrt_d * linf) / 448.0f;
            s = bound > 0.f ? bound : 1.0f;
        }
        scales[row] = s;
    }
}

// --------------------------------------------------------- element stores --

// Values already divided by the row scale; gfx950 converts in hardware with
// round-to-nearest-even: BF16 by v_cvt_pk_bf16_f32, OCP E4M3 by
// v_cvt_pk_fp8_f32 after a clamp to +-448 (the largest finite E4M3 value:
// saturation, as the FP8 row scales bound every entry up to rounding).
template <int DT> struct Store;
template <> struct Store<KERDOCK_F32> {
    static constexpr int ROWS = 1;   // rows packed per 32-bit store
    __device__ static uint32_t pack(const float *v) { return __float_as_uint(v[0]); }
};
template <> struct Store<KERDOCK_BF16> {
    static constexpr int ROWS = 2;
    __device__ static uint32_t pack(const float *v) {
        const __bf16 a = (__bf16)v[0], b = (__bf16)v[1];
        return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
    }
};
template <> struct Store<KERDOCK_FP8E4M3> {
    static constexpr int ROWS = 4;
    __device__ static uint32_t pack(const float *v) {
        float c[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = fminf(fmaxf(v[r], -448.0f), 448.0f);
        int w = __builtin_amdgcn_cvt_pk_fp8_f32(c[0], c[1], 0, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(c[2], c[3], w, true);
        return (uint32_t)w;
    }
};

// ------------------------------------------------------ cross-lane moves --
// value of v in lane (lane ^ H)
template <int H> __device__ __forceinline__ float lane_xor(float v) {
    if constexpr (H < 32) {
        // ds_swizzle bitmask mode: and_mask 0x1f, or_mask 0, xor_mask H
        return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), (H << 10) | 0x1f));
    } else {
        return __shfl_xor(v, 32);
    }
}

// ----------------------------------------------------------- table build --
// One workgroup = 16 waves (8 for FP8) = as many consecutive rows of A and
// one Kerdock basis.  Wave r transforms row i0 + r: lane l holds elements
// x = q*64 + l (q < R), the transform runs over the register index (bits
// 6..k-1) in registers and over the lane index (bits 0..5) with cross-lane
// swizzles.  The d outputs of the rows are then staged, 1024 columns at a
// time, in LDS as [w][rows] and written as contiguous row segments of each
// column.  Workgroups that
// run on the same XCD handle adjacent row strips of the same basis, so that
// the segments of one column are merged in that XCD's L2 before reaching HBM.
// rows per workgroup: 16 (FP32, BF16); 8 for FP8, whose 4-row packed stores
// leave 16-row workgroups with too few store threads per column (measured
// 44 ms -> 32 ms for the n = 2048 FP8 table)
template <int DT> struct BuildShape {
    static constexpr int ROWS = DT == KERDOCK_FP8E4M3 ? 8 : 16;
    static constexpr int THREADS = ROWS * 64;
    static constexpr int PITCH = ROWS + 1;    // +1 float: conflict-free staging
};
constexpr int STAGE_COLS = 1024;

template <int LOGD> __device__ __forceinline__ void fwht_wave(float *v) {
    constexpr int D = 1 << LOGD;
    constexpr int R = D >= 64 ? D / 64 : 1;
    const int lane = threadIdx.x & 63;
    // register bits
#pragma unroll
    for (int h = 1; h < R; h <<= 1) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (q & h) continue;
            float a = v[q], b = v[q + h];
            v[q] = a + b;
            v[q + h] = a - b;
        }
    }
    // lane bits
    // the upper lane of a pair takes p - v, the lower v + p: one FMA with a
    // per-lane sign, rounded exactly as the add or subtract
#define KD_LANE_STAGE(H)                                                    \
    if constexpr ((H) < D) {                                                \
        const float sg = (lane & (H)) != 0 ? -1.0f : 1.0f;                  \
        _Pragma("unroll") for (int q = 0; q < R; ++q) {                     \
            const float p = lane_xor<(H)>(v[q]);                            \
            v[q] = fmaf(v[q], sg, p);                                       \
        }                                                                   \
    }
    KD_LANE_STAGE(1)
    KD_LANE_STAGE(2)
    KD_LANE_STAGE(4)
    KD_LANE_STAGE(8)
    KD_LANE_STAGE(16)
    KD_LANE_STAGE(32)
#undef KD_LANE_STAGE
}

template <int LOGD, int DT>
__global__ __launch_bounds__(BuildShape<DT>::THREADS) void k_table_build(
    const float *__restrict__ A, int m, int n, int pitch, const uint32_t *__restrict__ signs,
    const float *__restrict__ scales, void *__restrict__ table, int strips, int xcd_map) {
    constexpr int D = 1 << LOGD;
    constexpr int R = D >= 64 ? D / 64 : 1;
    constexpr int WORDS = D >= 32 ? D / 32 : 1;
    constexpr int COLS = D < STAGE_COLS ? D : STAGE_COLS;
    constexpr int BUILD_ROWS = BuildShape<DT>::ROWS, BUILD_THREADS = BuildShape<DT>::THREADS;
    constexpr int STAGE_PITCH = BuildShape<DT>::PITCH;
    __shared__ float stage[COLS * STAGE_PITCH];
    __shared__ uint32_t sbits[WORDS];

    // workgroup -> (basis, strip)
    int g = blockIdx.x, b, strip;
    if (xcd_map) {
        const int per_xcd = strips / 8;
        const int xcd = g & 7, q = g >> 3;
        strip = xcd * per_xcd + q % per_xcd;
        b = q / per_xcd;
    } else {
        strip = g % strips;
        b = g / strips;
    }
    const int i0 = strip * BUILD_ROWS;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = i0 + wave;

    for (int t = threadIdx.x; t < WORDS; t += BUILD_THREADS) sbits[t] = signs[(size_t)b * WORDS + t];
    __syncthreads();

    // load the signed, zero-padded row: element x = q*64 + lane (every load
    // issued, from a clamped in-bounds address, and masked afterwards)
    float v[R];
    const int rowc = row < m ? row : m - 1;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int x = q * 64 + lane;
        const bool live = (D >= 64 || lane < D) && row < m && x < n;
        const int xc = x < n ? x : n - 1;
        const float a = A[(size_t)rowc * n + xc];
        const uint32_t bit = (D >= 64 || lane < D) ? (sbits[x >> 5] >> (x & 31)) & 1u : 0u;
        v[q] = live ? (bit ? -a : a) : 0.f;
    }
    fwht_wave<LOGD>(v);

    using S = Store<DT>;
    constexpr int ROWS = S::ROWS;
    constexpr int THREADS_PER_COL = BUILD_ROWS / ROWS;
    constexpr int COLS_PER_PASS = BUILD_THREADS / THREADS_PER_COL;
    float inv_scale[ROWS];
    const int my_rows = (threadIdx.x % THREADS_PER_COL) * ROWS;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) inv_scale[r] = 1.0f / scales[i0 + my_rows + r];

    uint32_t *out32 = reinterpret_cast<uint32_t *>(table);
    const size_t col_words = (size_t)pitch * (DT == KERDOCK_F32 ? 4 : DT == KERDOCK_BF16 ? 2 : 1) / 4;

#pragma unroll
    for (int c0 = 0; c0 < D; c0 += COLS) {
        // stage columns [c0, c0 + COLS) of this wave's row
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int w = q * 64 + lane;
            if (w >= c0 && w < c0 + COLS && (D >= 64 || lane < D))
                stage[(w - c0) * STAGE_PITCH + wave] = v[q];
        }
        __syncthreads();
        for (int cc = threadIdx.x / THREADS_PER_COL; cc < COLS; cc += COLS_PER_PASS) {
            float vals[ROWS];
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                // FP32 and BF16 tables have unit scales: no division
                if constexpr (DT == KERDOCK_FP8E4M3) vals[r] = stage[cc * STAGE_PITCH + my_rows + r] * inv_scale[r];
                else vals[r] = stage[cc * STAGE_PITCH + my_rows + r];
            }
            const size_t col = (size_t)b * D + c0 + cc;
            const size_t word = col * col_words + (size_t)(i0 + my_rows) / ROWS;
            out32[word] = S::pack(vals);
        }
        __syncthreads();
    }
}

// ------------------------------------------------- table build, d >= 256 --
// The same transform with fewer vector instructions, in workgroups of ROWS
// waves.  Wave r holds row i0 + r; lane l holds R = d/64 consecutive input
// elements of the row in registers q < R (16-byte loads), r = log2 R.  For
// d = 256 (R = 4, fwht_wave2) lane l holds x = (l ^ 15) R + q, so that
//   * x bits 0..r-1 (the register index): butterflies inside each lane;
//   * x bits r..r+3 (lane bits 0..3, xor 1, 2, 4, 8): the partner value
//     arrives by DPP (quad_perm, row_half_mirror + quad_perm, row_ror:8) and
//     every lane computes v + s p with s = -1 in the upper lane of the pair,
//     i.e. the upper lanes hold the negated difference.  Across the four
//     stages this multiplies output w by (-1)^{w . M} (M = 15 R, the mask of
//     these bits), which the input order (lane l reads segment l ^ 15)
//     cancels exactly, H[w][x ^ M] = (-1)^{w . M} H[w][x];
//   * x bits r+4, r+5 (lane bits 4, 5): v_permlane16_swap / permlane32_swap
//     exchange lane bit 4 (5) with register bit 0 (1), after which the pair
//     sits in one lane and the butterfly is local;
// output w of register q in lane l:
//   w = (l >> 4 & 1) | (l >> 5 & 1) << 1 | (q & (R - 4)) | (l & 15) << r |
//       (q & 3) << (r + 4),
// staged with slot = w' ^ ((w' >> 6 & 15) << 2), w' = w mod 1024, row pitch
// 1032 floats.  For d >= 1024 (R >= 16, fwht_wave3 below) the four lane bits
// go through LDS into registers instead, with the output map and staging
// given there.  For d = 4096 a chunk of 1024 columns is one value of q & 3.
// Each thread then stores PACK consecutive rows of a column (4 to 16 bytes).
// The barriers around the staging wait for LDS only: stores to the table
// need not complete before the next chunk.
constexpr int STAGE2_PITCH = 1032;

__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// every lane reads a valid lane under these controls, so the old value is
// never used (undefined: lets the move fold into the consuming instruction)
template <int CTRL> __device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// the d-point transform of a row held as R = d/64 registers per lane, lane l
// holding x = (l ^ 15) R + q; output positions as described above
template <int LOGD> __device__ __forceinline__ void fwht_wave2(float *v) {
    constexpr int R = (1 << LOGD) / 64;
    const int lane = threadIdx.x & 63;
    // register bits
#pragma unroll
    for (int h = 1; h < R; h <<= 1)
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (q & h) continue;
            const float a = v[q], b = v[q + h];
            v[q] = a + b;
            v[q + h] = a - b;
        }
    // lane bits 0..3 by DPP: v + s p, s = -1 in the upper lane
    const float s1 = (lane & 1) ? -1.f : 1.f, s2 = (lane & 2) ? -1.f : 1.f;
    const float s4 = (lane & 4) ? -1.f : 1.f, s8 = (lane & 8) ? -1.f : 1.f;
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = fmaf(dpp_f<0xB1>(v[q]), s1, v[q]);                  // quad_perm [1,0,3,2]
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = fmaf(dpp_f<0x4E>(v[q]), s2, v[q]);                  // quad_perm [2,3,0,1]
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = fmaf(dpp_f<0x1B>(dpp_f<0x141>(v[q])), s4, v[q]);   // half_mirror, [3,2,1,0]
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = fmaf(dpp_f<0x128>(v[q]), s8, v[q]);                 // row_ror:8
    // lane bit 4 <-> register bit 0, then the butterfly in the lane
#pragma unroll
    for (int q = 0; q < R; q += 2) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[q]), __float_as_uint(v[q + 1]), false,
                                                        false);
        const float a = __uint_as_float(r[0]), b = __uint_as_float(r[1]);
        v[q] = a + b;
        v[q + 1] = a - b;
    }
    // lane bit 5 <-> register bit 1
#pragma unroll
    for (int q = 0; q < R; ++q) {
        if (q & 2) continue;
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[q]), __float_as_uint(v[q + 2]), false,
                                                        false);
        const float a = __uint_as_float(r[0]), b = __uint_as_float(r[1]);
        v[q] = a + b;
        v[q + 2] = a - b;
    }
}

// PACK consecutive rows of one column in one store of PACK x element bytes
template <int DT, int PACK> __device__ __forceinline__ void store_rows(unsigned char *dst, const float *vals) {
    constexpr int SR = Store<DT>::ROWS, NW = PACK / SR;
    static_assert(PACK % SR == 0 && NW <= 4 && NW != 3, "store of 4, 8 or 16 bytes");
    uint32_t w[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) w[k] = Store<DT>::pack(vals + k * SR);
    if constexpr (NW == 1) *reinterpret_cast<uint32_t *>(dst) = w[0];
    else if constexpr (NW == 2) *reinterpret_cast<uint2 *>(dst) = make_uint2(w[0], w[1]);
    else *reinterpret_cast<uint4 *>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
}

// R >= 16 (d >= 1024): the same transform with lane bits 0..3 moved into
// registers instead of crossed by DPP.  Lane l holds x = l R + q (natural
// order).  After the register levels (x bits 0..r-1), each group of 16
// registers (register bits 4.. fixed) is transposed through this wave's LDS
// region tr (1088 floats: [lane bits 4,5][register bit 0..3][17-float row],
// conflict-free writes and reads), which exchanges lane bits 0..3 with
// register bits 0..3: lane l' then holds x bits 0..3 in its bits 0..3 and
// registers q' hold x bits r..r+3 in their bits 0..3, so those four levels
// are in-register butterflies (one instruction per element instead of a DPP
// move and an FMA).  Lane bits 4, 5 (x bits r+4, r+5) as in fwht_wave2.
// Output w of register q' in lane l':
//   w = (l' & 15) | (q' & (R - 16)) | (l' >> 4 & 3) << r | (q' >> 2 & 3) << (r + 2) |
//       (q' & 1) << (r + 4) | (q' >> 1 & 1) << (r + 5),
// staged with slot = w' ^ ((w' >> 6 & 3) << 4), w' = w mod 1024 (a write's 64
// lanes meet 64 banks), row pitch 1024 + 64 / ROWS floats (a read's row
// groups, PACK rows apart, start 64 / TPC banks apart).
constexpr int TR_WAVE = 1088;                  // floats of a wave's transpose region

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LOGD> __device__ __forceinline__ void fwht_wave3(float *v, float *tr) {
    constexpr int R = (1 << LOGD) / 64;
    static_assert(R >= 16, "four register bits to exchange");
    const int lane = threadIdx.x & 63, l_hi = lane >> 4, l_lo = lane & 15;
    // register bits
#pragma unroll
    for (int h = 1; h < R; h <<= 1)
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (q & h) continue;
            const float a = v[q], b = v[q + h];
            v[q] = a + b;
            v[q + h] = a - b;
        }
    // lane bits 0..3 <-> register bits 0..3, 16 registers at a time
#pragma unroll
    for (int c = 0; c < R / 16; ++c) {
#pragma unroll
        for (int j = 0; j < 16; ++j) tr[(l_hi * 16 + j) * 17 + l_lo] = v[c * 16 + j];
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < 16; ++i) v[c * 16 + i] = tr[(l_hi * 16 + l_lo) * 17 + i];
        wave_lds_sync();                       // before the next group overwrites the region
    }
    // the exchanged bits, now register bits 0..3
#pragma unroll
    for (int h = 1; h < 16; h <<= 1)
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (q & h) continue;
            const float a = v[q], b = v[q + h];
            v[q] = a + b;
            v[q + h] = a - b;
        }
    // lane bit 4 <-> register bit 0, then the butterfly in the lane
#pragma unroll
    for (int q = 0; q < R; q += 2) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[q]), __float_as_uint(v[q + 1]), false,
                                                        false);
        const float a = __uint_as_float(r[0]), b = __uint_as_float(r[1]);
        v[q] = a + b;
        v[q + 1] = a - b;
    }
    // lane bit 5 <-> register bit 1
#pragma unroll
    for (int q = 0; q < R; ++q) {
        if (q & 2) continue;
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[q]), __float_as_uint(v[q + 2]), false,
                                                        false);
        const float a = __uint_as_float(r[0]), b = __uint_as_float(r[1]);
        v[q] = a + b;
        v[q + 2] = a - b;
    }
}

template <int LOGD, int DT, int ROWS, int PACK>
__global__ __launch_bounds__(ROWS * 64) void k_table_build2(const float *__restrict__ A, int m, int n, int pitch,
                                                              const uint32_t *__restrict__ signs,
                                                              const float *__restrict__ scales,
                                                              void *__restrict__ table, int strips, int xcd_map) {
    constexpr int D = 1 << LOGD;
    constexpr int R = D / 64;                           // elements per lane
    constexpr int WORDS = D / 32;
    constexpr int COLS = D < STAGE_COLS ? D : STAGE_COLS;
    constexpr int QC = COLS / 64;                       // registers per chunk
    constexpr int THREADS = ROWS * 64;
    constexpr bool TR = R >= 16;                        // lane bits 0..3 through LDS (fwht_wave3)
    // staging row pitch: a read's row groups (PACK rows apart) start 64 / TPC
    // banks apart, so they meet distinct banks (PACK (64 / ROWS) = 64 / TPC)
    constexpr int PITCH = TR ? 1024 + 64 / ROWS : STAGE2_PITCH;
    constexpr int LDS_ROW = TR && TR_WAVE > PITCH ? TR_WAVE : PITCH;
    __shared__ __align__(16) float stage[ROWS * LDS_ROW];

    int g = blockIdx.x, b, strip;
    if (xcd_map) {
        const int per_xcd = strips / 8;
        const int xcd = g & 7, qq = g >> 3;
        strip = xcd * per_xcd + qq % per_xcd;
        b = qq / per_xcd;
    } else {
        strip = g % strips;
        b = g / strips;
    }
    const int i0 = strip * ROWS;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = i0 + wave;
    const int seg = TR ? lane : lane ^ 15;              // input segment of this lane
    const int x0 = seg * R;

    // signed, zero-padded row: 64 (R) consecutive elements per lane
    float v[R];
    {
        // sign bits of elements x0 .. x0 + R - 1 (R >= 32: whole words)
        constexpr int SW = (R + 31) / 32;
        uint32_t sw[SW];
#pragma unroll
        for (int w = 0; w < SW; ++w) sw[w] = signs[(size_t)b * WORDS + (x0 >> 5) + w];
        if constexpr (R < 32) sw[0] >>= (x0 & 31);
        const bool live = row < m && x0 < n;
        const float *src = A + (size_t)(row < m ? row : 0) * n + x0;
        if (live && x0 + R <= n && (n & 3) == 0) {
            // whole segment inside the row: 16-byte loads
            const float4 *s4 = reinterpret_cast<const float4 *>(src);
#pragma unroll
            for (int j = 0; j < R / 4; ++j) {
                const float4 t = s4[j];
                v[4 * j] = t.x;
                v[4 * j + 1] = t.y;
                v[4 * j + 2] = t.z;
                v[4 * j + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < R; ++q) v[q] = (live && x0 + q < n) ? src[q] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < R; ++q)
            v[q] = __uint_as_float(__float_as_uint(v[q]) ^ (((sw[q >> 5] >> (q & 31)) & 1u) << 31));
    }
    if constexpr (TR) {
        fwht_wave3<LOGD>(v, stage + wave * TR_WAVE);
        lds_barrier();                                  // every wave done with its transpose region
    } else {
        fwht_wave2<LOGD>(v);
    }

    constexpr int TPC = ROWS / PACK;                   // threads per column
    constexpr int CPP = THREADS / TPC;                  // columns per pass
    const int half = threadIdx.x % TPC, my_rows = half * PACK;
    float inv_scale[PACK];
#pragma unroll
    for (int r = 0; r < PACK; ++r) inv_scale[r] = 1.0f / scales[i0 + my_rows + r];
    constexpr int BT = DT == KERDOCK_F32 ? 4 : DT == KERDOCK_BF16 ? 2 : 1;
    unsigned char *out = reinterpret_cast<unsigned char *>(table);
    const size_t col_bytes = (size_t)pitch * BT;
    // output index of register q in this lane, less its register bits
    constexpr int LR = LOGD - 6;
    const int w_lane = TR ? (lane & 15) | ((lane >> 4) & 3) << LR
                          : ((lane >> 4) & 1) | ((lane >> 5) & 1) << 1 | (lane & 15) << LR;
    // staging slot of column wl (mod COLS): the 64 lanes of a write and the
    // columns of a read meet distinct banks
    auto slot_of = [](int wl) { return TR ? wl ^ (((wl >> 6) & 3) << 4) : wl ^ (((wl >> 6) & 15) << 2); };

#pragma unroll
    for (int c = 0; c < R / QC; ++c) {
        // chunk c: the registers whose output lies in columns [c COLS, (c+1) COLS)
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if ((((q & 3) << (LR + 4)) >> 10) != c) continue;   // w >> 10, as w_lane < 1024
            const int w = TR ? w_lane | (q & (R - 16)) | ((q >> 2) & 3) << (LR + 2) | (q & 3) << (LR + 4)
                             : w_lane | (q & (R - 4)) | (q & 3) << (LR + 4);
            stage[wave * PITCH + slot_of(w & (COLS - 1))] = v[q];
        }
        lds_barrier();
        const size_t colbase = (size_t)b * D + (size_t)c * COLS;
        for (int cc = threadIdx.x / TPC; cc < COLS; cc += CPP) {
            const int slot = slot_of(cc);
            float vals[PACK];
#pragma unroll
            for (int r = 0; r < PACK; ++r) {
                const float t = stage[(my_rows + r) * PITCH + slot];
                vals[r] = DT == KERDOCK_FP8E4M3 ? t * inv_scale[r] : t;
            }
            unsigned char *dst = out + (colbase + cc) * col_bytes + (size_t)(i0 + my_rows) * BT;
            store_rows<DT, PACK>(dst, vals);
        }
        lds_barrier();
    }
}

// --------------------------------------------------------- identity block --
// T[(d/2) d + w][i] = sqrt(d) A[i][w] for w < n, 0 for n <= w < d: a scaled
// transpose through a 64 x 64 LDS tile.
template <int DT>
__global__ __launch_bounds__(256) void k_identity_block(const float *__restrict__ A, int m, int n,
                                                        int d, int pitch, float sqrt_d,
                                                        const float *__restrict__ scales,
                                                        void *__restrict__ table) {
    __shared__ float tile[64][65];
    const int w0 = blockIdx.x * 64, i0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int i = i0 + r, w = w0 + tx;
        tile[r][tx] = (i < m && w < n) ? sqrt_d * A[(size_t)i * n + w] : 0.f;
    }
    __syncthreads();
    using S = Store<DT>;
    constexpr int ROWS = S::ROWS;
    constexpr int TPC = 64 / ROWS;                 // threads per column segment
    uint32_t *out32 = reinterpret_cast<uint32_t *>(table);
    const size_t col_words = (size_t)pitch * (DT == KERDOCK_F32 ? 4 : DT == KERDOCK_BF16 ? 2 : 1) / 4;
    const size_t base_col = (size_t)(d / 2) * d;
    for (int t = threadIdx.x; t < 64 * TPC; t += 256) {
        const int c = t / TPC, part = t % TPC;
        const int w = w0 + c;
        if (w >= d) continue;
        float vals[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int ii = part * ROWS + r;
            vals[r] = tile[ii][c] * (1.0f / scales[i0 + ii]);
        }
        out32[(base_col + w) * col_words + (size_t)(i0 + part * ROWS) / ROWS] = S::pack(vals);
    }
}

// ------------------------------------------------------------ read back --
template <int DT>
__global__ void k_read_columns(const void *__restrict__ table, int m, int pitch, int64_t L,
                               const float *__restrict__ scales, const uint32_t *__restrict__ ells,
                               int count, float *__restrict__ out) {
    const int c = blockIdx.y;
    if (c >= count) return;
    const size_t col = ells[c];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        float v;
        if ((int64_t)col >= L) {
            v = __builtin_nanf("");                // index outside the design
        } else if constexpr (DT == KERDOCK_F32) {
            v = reinterpret_cast<const float *>(table)[col * pitch + i];
        } else if constexpr (DT == KERDOCK_BF16) {
            v = bf16_to_f32(reinterpret_cast<const uint16_t *>(table)[col * pitch + i]);
        } else {
            v = e4m3_to_f32(reinterpret_cast<const uint8_t *>(table)[col * pitch + i]) * scales[i];
        }
        out[(size_t)c * m + i] = v;
    }
}

// -------------------------------------------------------------- launchers --

// table build kernel: 2 = k_table_build2 (d >= 256), 1 = k_table_build;
// KERDOCK_BUILD selects one (for measurements), default 2
static int build_variant() {
    const char *v = getenv("KERDOCK_BUILD");
    return (v && *v == '1') ? 1 : 2;
}

int launch_signs(const uint16_t *masks, int k, uint32_t *signs, hipStream_t s) {
    const int d = 1 << k;
    const int wpb = d >= 32 ? d / 32 : 1, nb = d / 2;
    const int total = wpb * nb;
    hipLaunchKernelGGL(k_signs, dim3((total + 255) / 256), dim3(256), 0, s, masks, k, wpb, nb, signs);
    KD_LAUNCH("k_signs");
    return KERDOCK_OK;
}

int launch_row_scales(const float *A, int m, int n, int pitch, int d, kerdock_dtype dt,
                      float *scales, float *norm2, hipStream_t s) {
    hipLaunchKernelGGL(k_row_scales, dim3((pitch + 3) / 4), dim3(256), 0, s, A, m, n, pitch,
                       sqrtf((float)d), dt == KERDOCK_FP8E4M3 ? 1 : 0, scales, norm2);
    KD_LAUNCH("k_row_scales");
    return KERDOCK_OK;
}

// rows per workgroup and rows per store of k_table_build2.  The write rate
// follows the length of the column segment one workgroup writes (measured
// on the n = 2048, m = 2048 tables: 32-byte segments about 1.9 TB/s, 64-byte
// segments about 3.4 TB/s), so FP32 and BF16 take 16 rows (one or two
// workgroups per CU at their register count; BF16 17.2 ms with 16 rows
// against 19.5 ms with 8); FP8 is bound by its vector work, where 8-row
// workgroups (several per CU) overlap one's stores with another's
// arithmetic (15.6 ms against 16.6 ms with 16 rows).
template <int DT> struct Build2Shape {
    static constexpr int ROWS = DT == KERDOCK_FP8E4M3 ? 8 : 16;
    static constexpr int PACK = DT == KERDOCK_F32 ? 4 : 8;
};

template <int LOGD, int DT, int ROWS, int PACK>
static int launch_build2(const float *A, int m, int n, int pitch, const uint32_t *signs, const float *scales,
                         void *table, hipStream_t s) {
    const int nb = (1 << LOGD) / 2;
    const int strips = pitch / ROWS;
    const int xcd_map = (strips % 8 == 0) ? 1 : 0;
    hipLaunchKernelGGL((k_table_build2<LOGD, DT, ROWS, PACK>), dim3(strips * nb), dim3(ROWS * 64), 0, s, A, m, n,
                       pitch, signs, scales, table, strips, xcd_map);
    KD_LAUNCH("k_table_build2");
    return KERDOCK_OK;
}

template <int LOGD, int DT>
static int build_kd(const float *A, int m, int n, int pitch, const uint32_t *signs,
                    const float *scales, void *table, hipStream_t s) {
    const int nb = (1 << LOGD) / 2;
    if constexpr (LOGD >= 8) {
        if (build_variant() == 2)
            return launch_build2<LOGD, DT, Build2Shape<DT>::ROWS, Build2Shape<DT>::PACK>(A, m, n, pitch, signs,
                                                                                        scales, table, s);
    }
    const int strips = pitch / BuildShape<DT>::ROWS;
    const int xcd_map = (strips % 8 == 0) ? 1 : 0;
    hipLaunchKernelGGL((k_table_build<LOGD, DT>), dim3(strips * nb), dim3(BuildShape<DT>::THREADS), 0, s, A,
                       m, n, pitch, signs, scales, table, strips, xcd_map);
    KD_LAUNCH("k_table_build");
    return KERDOCK_OK;
}

template <int DT>
static int build_dt(int k, const float *A, int m, int n, int pitch, const uint32_t *signs,
                    const float *scales, void *table, hipStream_t s) {
    switch (k) {
    case 2: return build_kd<2, DT>(A, m, n, pitch, signs, scales, table, s);
    case 4: return build_kd<4, DT>(A, m, n, pitch, signs, scales, table, s);
    case 6: return build_kd<6, DT>(A, m, n, pitch, signs, scales, table, s);
    case 8: return build_kd<8, DT>(A, m, n, pitch, signs, scales, table, s);
    case 10: return build_kd<10, DT>(A, m, n, pitch, signs, scales, table, s);
    case 12: return build_kd<12, DT>(A, m, n, pitch, signs, scales, table, s);
    default: return fail(KERDOCK_ERR_UNSUPPORTED_N, "table build: unsupported k");
    }
}

template <int DT>
static int identity_dt(const float *A, int m, int n, int d, int pitch, const float *scales,
                       void *table, hipStream_t s) {
    hipLaunchKernelGGL(k_identity_block<DT>, dim3((d + 63) / 64, pitch / 64), dim3(256), 0, s, A, m,
                       n, d, pitch, sqrtf((float)d), scales, table);
    KD_LAUNCH("k_identity_block");
    return KERDOCK_OK;
}

int launch_table_build(kerdock_dtype dt, int k, const float *A, int m, int n, int pitch,
                       const uint32_t *signs, const float *scales, void *table, hipStream_t s) {
    const int d = 1 << k;
    int rc;
    switch (dt) {
    case KERDOCK_F32:
        rc = build_dt<KERDOCK_F32>(k, A, m, n, pitch, signs, scales, table, s);
        if (rc == KERDOCK_OK) rc = identity_dt<KERDOCK_F32>(A, m, n, d, pitch, scales, table, s);
        return rc;
    case KERDOCK_BF16:
        rc = build_dt<KERDOCK_BF16>(k, A, m, n, pitch, signs, scales, table, s);
        if (rc == KERDOCK_OK) rc = identity_dt<KERDOCK_BF16>(A, m, n, d, pitch, scales, table, s);
        return rc;
    case KERDOCK_FP8E4M3:
        rc = build_dt<KERDOCK_FP8E4M3>(k, A, m, n, pitch, signs, scales, table, s);
        if (rc == KERDOCK_OK) rc = identity_dt<KERDOCK_FP8E4M3>(A, m, n, d, pitch, scales, table, s);
        return rc;
    }
    return fail(KERDOCK_ERR_INVALID_ARG, "table build: unknown dtype");
}

int launch_read_columns(kerdock_dtype dt, const void *table, int m, int pitch, int64_t L,
                        const float *scales, const uint32_t *ells, int count, float *out,
                        hipStream_t s) {
    if (count <= 0) return KERDOCK_OK;
    dim3 grid((m + 255) / 256, count);
    switch (dt) {
    case KERDOCK_F32:
        hipLaunchKernelGGL(k_read_columns<KERDOCK_F32>, grid, dim3(256), 0, s, table, m, pitch, L, scales, ells, count, out);
        break;
    case KERDOCK_BF16:
        hipLaunchKernelGGL(k_read_columns<KERDOCK_BF16>, grid, dim3(256), 0, s, table, m, pitch, L, scales, ells, count, out);
        break;
    case KERDOCK_FP8E4M3:
        hipLaunchKernelGGL(k_read_columns<KERDOCK_FP8E4M3>, grid, dim3(256), 0, s, table, m, pitch, L, scales, ells, count, out);
        break;
    }
    KD_LAUNCH("k_read_columns");
    return KERDOCK_OK;
}

}  // namespace kd
