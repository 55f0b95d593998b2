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
// group instead of once per vector.  With an FP32 table the product runs on
// the FP32 matrix cores (16 x 16 x 4 MFMA).  BF16 and FP8 entries are exact
// BF16 values, so there it runs on the BF16 matrix cores (16 x 16 x 32 MFMA)
// with every coefficient split exactly into three BF16 parts: each product
// of an entry and a part is exact in FP32, and only the FP32 accumulation
// rounds, as in the FP32 product.  The batch means, median, selection and
// survivor dots are those of the per-vector form (partials with one chunk
// per batch).
#include "apply_device.hpp"

namespace kd {

// coordinates of the digit rows: n rounded up to a multiple of 64
int shared_n_pad(int n) { return (n + 63) / 64 * 64; }

constexpr int ST = KERDOCK_SHARED_TILE;       // vectors per draw group

// Digits in the order the coefficient MFMAs read them: for group g, digit
// plane b and step s (coordinates 64 s .. + 63), a 4 KiB block of 4 wave
// blocks (vectors 16 w .. + 15) of 1 KiB, each [coordinate quarter (16
// coordinates)][vector][16 coordinate bytes], so that lane l of wave w reads
// bytes 16 l .. + 15 of its wave block as its B operand.
__device__ __forceinline__ size_t digit_offset(int g, int b, int steps, int s, int tv, int c) {
    return ((((size_t)g * 4 + b) * steps + s) << 12) + ((size_t)(tv >> 4) << 10) + ((size_t)(c >> 4) << 8) +
           ((size_t)(tv & 15) << 4) + (size_t)(c & 15);
}
size_t shared_digit_bytes(int batch, int n) {
    return (size_t)((batch + ST - 1) / ST) * ST * 4 * (size_t)shared_n_pad(n);
}
constexpr int SG_BM = 128;                    // table rows per GEMM workgroup
constexpr int SG_BK = 32;                     // draws per LDS stage

// ------------------------------------------------------- coefficients --
// With one draw list per group the coefficients of a group form the product
// C = S X_g of the N x n sign matrix S (rows s_l restricted to the first n
// coordinates, entries +-1) and the n x 64 block of the group's vectors.  In
// the fixed point of the per-vector form, x_int = rint(x 2^E2) with
// sum |x_int| <= 2^30, each x_int is split into four balanced base-256 digits
// in [-128, 127], and C is accumulated digit by digit on the int8 matrix cores
// (16 x 16 x 64 MFMA, int32 accumulators): every step is integer arithmetic,
// so c = (sum_b 256^b C_b) 2^-E2 equals the per-vector form's exact signed sum.
// Identity draws (basis d/2) give sqrt(d) x[w] directly.

// Workgroups are dealt to the 8 XCDs in turn by id; this numbering gives each
// XCD one contiguous range of [0, total) instead, taken in order.
__device__ __forceinline__ int xcd_contiguous(int id, int total) {
    const int q = total / 8, r = total % 8, x = id % 8;
    return x * q + min(x, r) + id / 8;
}

// k_x_digits: grid (batch), one wave.  The digits of x_t at digit_offset
// (coordinates q < n_pad, zero beyond n) and xscale[t] = (scale exponent,
// flags): bit 0 x_t is finite, bit 1 its top digit plane (b = 3) has a
// nonzero digit.  Vectors are numbered contiguously per XCD: the 16 vectors
// whose 16-byte pieces share a 256-byte digit block then write through one
// L2, where the pieces merge into whole lines.
template <int P>
__global__ __launch_bounds__(64) void k_x_digits(const float *__restrict__ X, int n, int n_pad,
                                                 int8_t *__restrict__ digits, int2 *__restrict__ xscale) {
    const int t = xcd_contiguous(blockIdx.x, gridDim.x), lane = threadIdx.x;
    int xi[P][32];
    int E2;
    bool finite;
    fixed_point<P>(X + (size_t)t * n, n, lane, xi, E2, finite);
    const int g = t / ST, tv = t % ST, steps = n_pad / 64;
    uint32_t top = 0u;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int e0 = (lane + 64 * p) * 32;
        if (e0 >= n_pad) continue;
        uint32_t packed[4][8];
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            int v = xi[p][q];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int dg = ((v & 255) ^ 128) - 128;        // balanced digit
                v = (v - dg) >> 8;                              // exact
                if (q % 4 == 0) packed[b][q / 4] = 0u;
                packed[b][q / 4] |= (uint32_t)(uint8_t)dg << (8 * (q % 4));
            }
        }
        // coordinates e0 .. e0 + 31: two 16-coordinate quarters of step e0 / 64
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int c = (e0 & 63) + 16 * h;
                *reinterpret_cast<u32x4 *>(digits + digit_offset(g, b, steps, e0 / 64, tv, c)) =
                    u32x4{packed[b][4 * h], packed[b][4 * h + 1], packed[b][4 * h + 2], packed[b][4 * h + 3]};
            }
#pragma unroll
        for (int w = 0; w < 8; ++w) top |= packed[3][w];
    }
    const bool top_any = __ballot(top != 0u) != 0;
    if (lane == 0) xscale[t] = make_int2(E2, (finite ? 1 : 0) | (top_any ? 2 : 0));
}

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int SC_DRAWS = 64;                  // draws per coefficient workgroup

// Sign bits to +-1 bytes: bit q of the 4-bit value m goes to byte q (the
// four shifted copies m << 7 q do not overlap), then 0 -> 0x01, 1 -> 0xFF.
__device__ __forceinline__ int sign_bytes4(uint32_t m) {
    const uint32_t bits = (m * 0x00204081u) & 0x01010101u;
    return (int)(0x01010101u + bits * 0xFEu);
}

// k_shared_coef: grid (K ceil(J / 64), groups), 256 threads; block x takes
// draws kb J + 64 jb .. + 63 of batch kb = x / ceil(J / 64) (never past the
// batch).  Output layout: by_vector == 0, coef[g][j][t mod 64] (the 64
// vectors of a draw contiguous); by_vector != 0, coef[g][t mod 64][kb JP + j
// - kb J] with JP = J rounded up to 64 (the draws of a vector and batch
// contiguous).  Wave w takes the group's vectors 16 w .. + 15 (the 16
// columns of its MFMA blocks) against all 64 draws of the block (4 row
// blocks) and the 3 or 4 digit planes: 16 accumulators.  The sign rows of
// the 64 draws are staged in LDS once (dynamic LDS: 64 (d/32 + 1) words, a
// padded row per draw so that the 16 draws of a read meet distinct banks).
// Per step of 64 coordinates wave w makes the +-1 sign operands of row
// block w (from the staged sign words and the Walsh pattern of w) into a
// double-buffered LDS tile that every wave then reads, one barrier per step;
// a lane reads its 16-byte digit operands straight from memory (one
// contiguous 1 KiB per wave and plane, in digit_offset order; a group's
// digits stay in L2).  The next step's digits and sign operands are loaded
// and made before this step's MFMAs.
__global__ __launch_bounds__(256) void k_shared_coef(const float *__restrict__ X, int n, int n_pad, int k, int64_t L,
                                                     const uint32_t *__restrict__ signs, uint64_t seed, int64_t t0,
                                                     int batch, int J, int K, int by_vector,
                                                     const int8_t *__restrict__ digits,
                                                     const int2 *__restrict__ xscale, uint32_t *__restrict__ ell,
                                                     float *__restrict__ coef, uint32_t *__restrict__ dbg_samples,
                                                     float *__restrict__ dbg_coef) {
    extern __shared__ uint32_t s_sign[];             // [64][words + 1]
    __shared__ uint32_t s_l[SC_DRAWS];
    __shared__ __align__(16) i32x4 s_a[2][4][64];   // sign operands [buffer][row block][lane]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = blockIdx.y, nx = min(ST, batch - g * ST);
    const int d = 1 << k, words = d >= 32 ? d / 32 : 1, wp = words + 1;
    const int row = lane & 15;                       // draw row of a block / vector column
    const int N = J * K, JP = (J + 63) & ~63, jblocks = JP / SC_DRAWS;
    const int kb = blockIdx.x / jblocks, jb0 = (blockIdx.x % jblocks) * SC_DRAWS;
    const int kq = (lane >> 4) * 16;                 // this lane's 16 coordinates within a step
    const int tv = wave * 16 + row;                  // this lane's vector column

    // the block's draws (wave 0, one per lane) and their sign rows
    if (tid < SC_DRAWS) {
        const int jl = jb0 + tid;
        uint32_t l = 0;
        if (jl < J) {
            const int j = kb * J + jl;
            uint64_t c4[4] = {(uint64_t)(j >> 2), (uint64_t)(t0 + g), 1, 0};
            philox4x64_10(c4, seed, 0);
            const uint64_t rr = (j & 3) == 0 ? c4[0] : (j & 3) == 1 ? c4[1] : (j & 3) == 2 ? c4[2] : c4[3];
            l = (uint32_t)__umul64hi(rr, (uint64_t)L);
        }
        s_l[tid] = l;
    }
    __syncthreads();
    // only the words of coordinates below n_pad are read
    const int wn = min(words, (n_pad + 31) / 32);
    for (int i = tid; i < SC_DRAWS * wn; i += 256) {
        const int r = i / wn, wi = i % wn;
        const uint32_t bb = s_l[r] >> k;
        s_sign[r * wp + wi] = (jb0 + r < J && (int)bb < d / 2) ? signs[bb * (uint32_t)words + wi] : 0u;
    }
    // the draw whose sign operands this lane makes: row `row` of block `wave`
    const uint32_t my_l = s_l[wave * 16 + row];
    const uint32_t ww = my_l & (uint32_t)(d - 1);
    const bool krow = jb0 + wave * 16 + row < J && (int)(my_l >> k) < d / 2;
    const uint32_t w16 = (ww & 1u ? 0xAAAAu : 0u) ^ (ww & 2u ? 0xCCCCu : 0u) ^ (ww & 4u ? 0xF0F0u : 0u) ^
                         (ww & 8u ? 0xFF00u : 0u);
    const uint32_t *srow = s_sign + (wave * 16 + row) * wp;

    i32x4 acc[4][4];                                 // [digit][row block]
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[b][c] = i32x4{0, 0, 0, 0};

    // The top digit plane is skipped for a group whose vectors all have it
    // zero (typical for unit vectors: it only holds entries beyond about
    // 2^23 of the fixed-point scale); its products would all be zero.  (The
    // barrier also completes the sign-row staging.)
    const bool top = __syncthreads_or(tid < nx && (xscale[g * ST + tid].y & 2)) != 0;
    // this lane's digit operands (columns past the batch end read the
    // buffer's padding and are not written)
    const int steps = n_pad / 64;
    const int8_t *dsrc = digits + digit_offset(g, 0, steps, 0, wave * 16, 0) + (size_t)lane * 16;
    i32x4 dg[4];
    auto fetch = [&](int st) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (b < 3 || top) dg[b] = *reinterpret_cast<const i32x4 *>(dsrc + (((size_t)b * steps + st) << 12));
    };
    // sign operand of this lane's draw at step st (coordinates past d, only
    // when n_pad > d, meet zero digits)
    auto make_sign = [&](int st) {
        const int q = st * 64 + kq;
        const uint32_t wd = srow[min(q >> 5, words - 1)];
        const uint32_t par = __popc((uint32_t)q & ww) & 1u;
        const uint32_t m16 = ((wd >> (q & 31)) & 0xFFFFu) ^ w16 ^ (par ? 0xFFFFu : 0u);
        const bool on = krow && (q >> 5) < words;
        s_a[st & 1][wave][lane] = on ? i32x4{sign_bytes4(m16 & 15u), sign_bytes4((m16 >> 4) & 15u),
                                             sign_bytes4((m16 >> 8) & 15u), sign_bytes4(m16 >> 12)}
                                     : i32x4{0, 0, 0, 0};
    };
    fetch(0);
    make_sign(0);
    __syncthreads();
    for (int st = 0; st < steps; ++st) {
        i32x4 a[4], bop[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) a[rb] = s_a[st & 1][rb][lane];
#pragma unroll
        for (int b = 0; b < 4; ++b) bop[b] = dg[b];
        if (st + 1 < steps) {
            fetch(st + 1);
            make_sign(st + 1);
        }
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (b == 3 && !top) continue;        // uniform
                acc[b][rb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[rb], bop[b], acc[b][rb], 0, 0, 0);
            }
        __syncthreads();                             // next buffer written; this one read
    }

    // D block rb: lane holds draws rb 16 + 4 (lane / 16) + v of the block,
    // vector column lane % 16 of this wave
    const float sqrt_d = sqrtf((float)d);
    const bool col_on = tv < nx;
    const int t = g * ST + tv;
    int2 sc = make_int2(0, 0);
    if (col_on) sc = xscale[t];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        float cv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = 4 * (lane >> 4) + v;          // row within the block
            const uint32_t l_r = s_l[rb * 16 + rr];
            const int jl = jb0 + rb * 16 + rr;
            const int jr = kb * J + jl;
            cv[v] = 0.f;
            if (jl >= J) continue;
            const uint32_t b_r = l_r >> k, w_r = l_r & (uint32_t)(d - 1);
            const bool ident = (int)b_r == d / 2;
            if (tv == 0) ell[(size_t)g * N + jr] = l_r;
            if (!col_on) continue;
            float cf;
            if (ident) {
                cf = ((int)w_r < n) ? sqrt_d * X[(size_t)t * n + w_r] : 0.f;
            } else {
                const int64_t tot = (int64_t)acc[0][rb][v] + ((int64_t)acc[1][rb][v] << 8) +
                                    ((int64_t)acc[2][rb][v] << 16) + ((int64_t)acc[3][rb][v] << 24);
                cf = (sc.y & 1) ? (float)(int)tot * ldexpf(1.0f, -sc.x) : __builtin_nanf("");
            }
            cv[v] = cf;
            if (!by_vector) coef[((size_t)g * N + jr) * ST + tv] = cf;
            if (dbg_samples) {
                dbg_samples[(size_t)t * N + jr] = l_r;
                dbg_coef[(size_t)t * N + jr] = cf;
            }
        }
        if (by_vector && col_on) {
            // four consecutive draws of one vector per lane: one 16-byte store
            // (zeros past the batch end, inside the row's padding to JP)
            const size_t pos = (size_t)kb * JP + jb0 + rb * 16 + 4 * (lane >> 4);
            *reinterpret_cast<f32x4 *>(coef + ((size_t)g * ST + tv) * ((size_t)K * JP) + pos) =
                f32x4{cv[0], cv[1], cv[2], cv[3]};
        }
    }
}

// Draws of a batch are split into `splits` consecutive slices (a function of
// J alone, so results never depend on the batch size), each summed by its
// own workgroups; the slices are added in order with the batch mean.
int shared_splits(int J) { return J / 2048 < 1 ? 1 : J / 2048 > 16 ? 16 : J / 2048; }

// k_shared_gemm: the product for FP32 tables.  Grid (ceil(pitch / 128), K
// splits, groups), 256 threads.  Rows i0 .. i0 + 127 of slice sp of Y_k for
// the (up to) 64 vectors of group g: partial[t][k][sp][i] = sum_{j in slice}
// T[ell[g][k J + j]][i] coef[g][k J + j][t mod 64].  Wave w owns rows
// i0 + 32 w .. + 31, all 64 vectors: 2 x 4 MFMA blocks.
__global__ __launch_bounds__(256) void k_shared_gemm(const unsigned char *__restrict__ table, int col_bytes, int pitch,
                                                     int batch, int J, int K, int N, int splits,
                                                     const uint32_t *__restrict__ ell,
                                                     const float *__restrict__ coef,
                                                     float *__restrict__ partial) {
    constexpr int E = 4;                      // FP32 entries per 16 bytes
    constexpr int TPC = SG_BM / E;            // threads per column slice
    constexpr int CPP = 256 / TPC;            // column slices per pass
    static_assert(SG_BK % CPP == 0, "whole passes");
    __shared__ float As[SG_BK][SG_BM + 16];   // [draw][row]; row stride = 16 mod 64 banks
    __shared__ float Bs[SG_BK][ST + 16];      // [draw][vector]
    const int g = blockIdx.z, kb = blockIdx.y / splits, sp = blockIdx.y % splits, i0 = blockIdx.x * SG_BM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nx = min(ST, batch - g * ST);
    const int js = (int)(((long long)J * sp) / splits);
    const int Jl = (int)(((long long)J * (sp + 1)) / splits) - js;     // draws of this slice
    const uint32_t *__restrict__ el = ell + (size_t)g * N + (size_t)kb * J + js;
    const float *__restrict__ cf = coef + ((size_t)g * N + (size_t)kb * J + js) * ST;
    const int wi = wave * 32;
    f32x4 acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    // Global loads of stage j0 + SG_BK are issued before the MFMAs of stage
    // j0 and land in LDS after them (one LDS buffer, register prefetch).  The
    // loads are branch-free (indices clamped, values masked where they are
    // consumed) and the draw indices are loaded one stage ahead, so that a
    // stage's loads are in flight together.
    constexpr int PASSES = SG_BK / CPP;
    u32x4 ra[PASSES];
    f32x4 rb[2];
    uint32_t lv[PASSES];
    const int bj = tid >> 3, bv = (tid & 7) * 8;     // B stage: draw bj, vectors bv .. bv + 7
    const int ar = (tid % TPC) * E;                  // A stage: rows i0 + ar .. + E - 1
    const bool arow_ok = i0 + ar < pitch;            // pitch is a multiple of 64
    const size_t aoff = (size_t)(arow_ok ? i0 + ar : 0) * (size_t)(16 / E);
    auto fetch_ell = [&](int j0) {
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) lv[ps] = el[min(j0 + ps * CPP + tid / TPC, Jl - 1)];
    };
    auto fetch = [&](int j0) {
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps)
            ra[ps] = __builtin_nontemporal_load(
                reinterpret_cast<const u32x4 *>(table + (size_t)lv[ps] * (size_t)col_bytes + aoff));
        const f32x4 *src = reinterpret_cast<const f32x4 *>(cf + (size_t)min(j0 + bj, Jl - 1) * ST + bv);
        rb[0] = src[0];
        rb[1] = src[1];
    };
    fetch_ell(0);
    fetch(0);
    fetch_ell(SG_BK);
    for (int j0 = 0; j0 < Jl; j0 += SG_BK) {
#pragma unroll
        for (int ps = 0; ps < PASSES; ++ps) {
            const int cc = ps * CPP + tid / TPC;
            const bool ok = j0 + cc < Jl && arow_ok;
            *reinterpret_cast<f32x4 *>(&As[cc][ar]) =
                ok ? f32x4{__uint_as_float(ra[ps].x), __uint_as_float(ra[ps].y), __uint_as_float(ra[ps].z),
                           __uint_as_float(ra[ps].w)}
                   : f32x4{0.f, 0.f, 0.f, 0.f};
        }
        {
            const bool ok = j0 + bj < Jl;
#pragma unroll
            for (int e = 0; e < 8; ++e) Bs[bj][bv + e] = (ok && bv + e < nx) ? rb[e >> 2][e & 3] : 0.f;
        }
        __syncthreads();
        // unconditional (indices are clamped; the last stage reloads data it
        // does not use), so that the waits count exactly the loads they need
        fetch(j0 + SG_BK);
        fetch_ell(j0 + 2 * SG_BK);
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
                *reinterpret_cast<f32x4 *>(partial + (((size_t)(g * ST + tt) * K + kb) * splits + sp) * pitch + row) =
                    acc[a][b];
        }
}

// ---------------------------------------------- BF16 matrix-core product --
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
constexpr int SB_BM = 256;                    // table rows per workgroup
constexpr int SB_BK = 64;                     // draws per LDS stage
constexpr int SB_LD = SB_BK + 8;              // LDS row: 144 bytes, an odd number of 16-byte units

// First draw of slice sp: J sp / splits rounded up to a multiple of four
// (the coefficient rows then start 16-byte aligned); slice `splits` ends at J.
__device__ __forceinline__ int slice_begin(int J, int sp, int splits) {
    if (sp >= splits) return J;
    return min(J, (int)((((long long)J * sp) / splits + 3) & ~3ll));
}

__device__ __forceinline__ uint32_t bf16_bits(__bf16 v) { return (uint32_t)__builtin_bit_cast(uint16_t, v); }

// c = hi + mid + lo exactly: each step rounds to BF16 and keeps the rounding
// error, which FP32 holds exactly; after two steps at most 8 significant bits
// of c's 24 are left, so the third part is exact.  The parts come back as
// packed pairs: p[q] = part q of c0 (low half) and of c1 (high half).
__device__ __forceinline__ void split3x2(float c0, float c1, uint32_t p[3]) {
    const __bf16 h0 = (__bf16)c0, h1 = (__bf16)c1;
    const float r0 = c0 - (float)h0, r1 = c1 - (float)h1;
    const __bf16 m0 = (__bf16)r0, m1 = (__bf16)r1;
    const __bf16 l0 = (__bf16)(r0 - (float)m0), l1 = (__bf16)(r1 - (float)m1);
    p[0] = bf16_bits(h0) | (bf16_bits(h1) << 16);
    p[1] = bf16_bits(m0) | (bf16_bits(m1) << 16);
    p[2] = bf16_bits(l0) | (bf16_bits(l1) << 16);
}

// k_shared_gemm16: the product for BF16 and FP8 tables.  Grid (ceil(pitch /
// 256), K splits, groups), 256 threads; output as k_shared_gemm, slice
// bounds slice_begin.  Coefficients in the by-vector layout (k_shared_coef,
// by_vector != 0).  Per stage of 64 draws:
//   A: thread (ad, ar) = (tid % 8, tid / 8) loads rows i0 + 8 ar .. + 7 of draws
//      8 ad .. + 7 (FP8 entries widened to BF16, exact) and transposes the
//      8 x 8 block in registers, so that As[row][draw] holds the draws of a row
//      contiguous, as the MFMA operand wants them (8 draws per lane);
//   B: thread (bt, bq) = (tid % 64, tid / 64) loads draws 16 bq .. + 15 of
//      vector bt and writes the three parts to Bs[part][vector][draw].
// With rows of 9 16-byte units, the 16 lanes of an LDS access always meet 16
// distinct bank groups, on the staging writes and on the operand reads.
// Wave w owns rows 128 (w % 2) .. + 127 and vectors 32 (w / 2) .. + 31: 8 x 2
// MFMA blocks, 3 MFMAs (one per part) per block and 32 draws.
template <int DT>
__global__ __launch_bounds__(256, 2) void k_shared_gemm16(const unsigned char *__restrict__ table, int col_bytes,
                                                       int pitch, int batch, int J, int K, int N, int splits,
                                                       const uint32_t *__restrict__ ell,
                                                       const float *__restrict__ coef,
                                                       float *__restrict__ partial) {
    static_assert(DT == KERDOCK_BF16 || DT == KERDOCK_FP8E4M3, "BF16-exact tables only");
    constexpr int EB = DT == KERDOCK_BF16 ? 2 : 1;   // bytes per entry
    constexpr int LW = 2 * EB;                       // 32-bit words per 8 rows
    __shared__ __align__(16) uint16_t As[SB_BM][SB_LD];
    __shared__ __align__(16) uint16_t Bs[3][ST][SB_LD];
    const int g = blockIdx.z, kb = blockIdx.y / splits, sp = blockIdx.y % splits, i0 = blockIdx.x * SB_BM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nx = min(ST, batch - g * ST);
    const int js = slice_begin(J, sp, splits);
    const int Jl = slice_begin(J, sp + 1, splits) - js;
    const int JP = (J + 63) & ~63;
    const uint32_t *__restrict__ el = ell + (size_t)g * N + (size_t)kb * J + js;
    const int ad = tid & 7, ar = tid >> 3;
    const int arow = i0 + 8 * ar;
    const bool arow_ok = arow < pitch;                // pitch is a multiple of 64
    const int bt = tid & 63, bq = tid >> 6;
    const float *__restrict__ cf = coef + ((size_t)g * ST + bt) * ((size_t)K * JP) + (size_t)kb * JP + js;
    const bool bt_ok = bt < nx;
    const int wr = (wave & 1) * 128, wv = (wave >> 1) * 32;

    f32x4 acc[8][2];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    // The loads are branch-free (indices clamped into the slice, values
    // masked), so that all of a stage's loads are in flight together.  Two
    // stages of table entries are in flight (register sets 0 and 1, taken in
    // turn), and the draw indices of stage s are loaded before the table
    // entries of stage s - 1: vector loads complete in order, so waiting for
    // the indices never waits for table entries still in flight.
    const int Jq = (Jl - 1) & ~3;                  // last aligned quad of the slice
    const float *__restrict__ cfr = bt_ok ? cf : coef + ((size_t)g * ST) * ((size_t)K * JP) + (size_t)kb * JP + js;
    const size_t aoff = (size_t)(arow_ok ? arow : 0) * EB;
    uint32_t lv0[8], lv1[8];
    uint32_t ra0[8][LW], ra1[8][LW];
    f32x4 rb0[4], rb1[4];
    auto fetch_ell = [&](uint32_t (&lv)[8], int j0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) lv[e] = el[min(j0 + 8 * ad + e, Jl - 1)];
    };
    auto fetch = [&](uint32_t (&ra)[8][LW], f32x4 (&rb)[4], const uint32_t (&lv)[8], int j0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const unsigned char *src = table + (size_t)lv[e] * (size_t)col_bytes + aoff;
            if constexpr (DT == KERDOCK_BF16) {
                const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(src));
                ra[e][0] = v.x; ra[e][1] = v.y; ra[e][2] = v.z; ra[e][3] = v.w;
            } else {
                const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(src));
                ra[e][0] = v.x; ra[e][1] = v.y;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            rb[u] = *reinterpret_cast<const f32x4 *>(cfr + min(j0 + 16 * bq + 4 * u, Jq));
    };
    // one stage's operands into LDS
    auto stage = [&](const uint32_t (&ra)[8][LW], const f32x4 (&rb)[4], int j0) {
        {
            // rows as packed BF16 pairs: q[e][w] holds rows 2w, 2w + 1 of draw e
            // (values past the slice end or the last row are masked here,
            // where the loads are consumed)
            uint32_t q[8][4];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const bool ok = j0 + 8 * ad + e < Jl && arow_ok;
                if constexpr (DT == KERDOCK_BF16) {
#pragma unroll
                    for (int w = 0; w < 4; ++w) q[e][w] = ok ? ra[e][w] : 0u;
                } else {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const uint32_t word = ok ? ra[e][h] : 0u;
                        const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)word, false);
                        const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)word, true);
                        q[e][2 * h] = (__float_as_uint(lo[0]) >> 16) | (__float_as_uint(lo[1]) & 0xFFFF0000u);
                        q[e][2 * h + 1] = (__float_as_uint(hi[0]) >> 16) | (__float_as_uint(hi[1]) & 0xFFFF0000u);
                    }
                }
            }
            // transpose: row r gets draws 2 v, 2 v + 1 in word v
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                u32x4 even, odd;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const uint32_t a = q[2 * v][w], b = q[2 * v + 1][w];
                    even[v] = (a & 0xFFFFu) | (b << 16);
                    odd[v] = (a >> 16) | (b & 0xFFFF0000u);
                }
                *reinterpret_cast<u32x4 *>(&As[8 * ar + 2 * w][8 * ad]) = even;
                *reinterpret_cast<u32x4 *>(&As[8 * ar + 2 * w + 1][8 * ad]) = odd;
            }
        }
        {
            uint32_t p[4][2][3];                     // [u][pair][part]
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int jj = j0 + 16 * bq + 4 * u;
                float c[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) c[e] = (bt_ok && jj + e < Jl) ? rb[u][e] : 0.f;
                split3x2(c[0], c[1], p[u][0]);
                split3x2(c[2], c[3], p[u][1]);
            }
#pragma unroll
            for (int part = 0; part < 3; ++part)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    *reinterpret_cast<u32x4 *>(&Bs[part][bt][16 * bq + 8 * h]) =
                        u32x4{p[2 * h][0][part], p[2 * h][1][part], p[2 * h + 1][0][part], p[2 * h + 1][1][part]};
        }
    };
    auto mma = [&]() {
#pragma unroll
        for (int kk = 0; kk < SB_BK; kk += 32) {
            const int kc = kk + 8 * (lane >> 4);
            bf16x8 fa[8];
#pragma unroll
            for (int a = 0; a < 8; ++a)
                fa[a] = *reinterpret_cast<const bf16x8 *>(&As[wr + 16 * a + (lane & 15)][kc]);
#pragma unroll
            for (int part = 0; part < 3; ++part)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const bf16x8 fb = *reinterpret_cast<const bf16x8 *>(&Bs[part][wv + 16 * b + (lane & 15)][kc]);
#pragma unroll
                    for (int a = 0; a < 8; ++a)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb, acc[a][b], 0, 0, 0);
                }
        }
    };

    // (the scheduling barriers keep the loads in this issue order)
    fetch_ell(lv0, 0);
    fetch_ell(lv1, SB_BK);
    __builtin_amdgcn_sched_barrier(0);
    fetch(ra0, rb0, lv0, 0);
    __builtin_amdgcn_sched_barrier(0);
    fetch_ell(lv0, 2 * SB_BK);
    __builtin_amdgcn_sched_barrier(0);
    fetch(ra1, rb1, lv1, SB_BK);
    __builtin_amdgcn_sched_barrier(0);
    // pairs of stages, then a last single one (the loads past the slice end
    // are clamped into it and never used)
    int j0 = 0;
    for (; j0 + SB_BK < Jl; j0 += 2 * SB_BK) {
        stage(ra0, rb0, j0);
        __syncthreads();
        fetch_ell(lv1, j0 + 3 * SB_BK);
        __builtin_amdgcn_sched_barrier(0);
        fetch(ra0, rb0, lv0, j0 + 2 * SB_BK);
        __builtin_amdgcn_sched_barrier(0);
        mma();
        __syncthreads();
        stage(ra1, rb1, j0 + SB_BK);
        __syncthreads();
        fetch_ell(lv0, j0 + 4 * SB_BK);
        __builtin_amdgcn_sched_barrier(0);
        fetch(ra1, rb1, lv1, j0 + 3 * SB_BK);
        __builtin_amdgcn_sched_barrier(0);
        mma();
        __syncthreads();
    }
    if (j0 < Jl) {
        stage(ra0, rb0, j0);
        __syncthreads();
        mma();
    }
    // D block (a, b): lane holds rows 4 (lane / 16) + v, v < 4, of column lane % 16
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int row = i0 + wr + a * 16 + 4 * (lane >> 4);
            const int tt = wv + b * 16 + (lane & 15);
            if (tt < nx && row < pitch)
                *reinterpret_cast<f32x4 *>(partial + (((size_t)(g * ST + tt) * K + kb) * splits + sp) * pitch + row) =
                    acc[a][b];
        }
}

// Coefficient layout of the product for a table type: by vector for the
// BF16 product, by draw for the FP32 one.
bool shared_by_vector(kerdock_dtype dt) { return dt != KERDOCK_F32; }

// floats of the coefficient buffer
size_t shared_coef_floats(kerdock_dtype dt, int batch, int J, int K) {
    const size_t groups = ((size_t)batch + ST - 1) / ST;
    const size_t JP = ((size_t)J + 63) & ~(size_t)63;
    return groups * ST * (shared_by_vector(dt) ? (size_t)K * JP : (size_t)J * K);
}

int launch_shared_coef(kerdock_dtype dt, const float *X, int batch, int n, int k, int64_t L, const uint32_t *signs,
                       uint64_t seed, int64_t t0, int J, int K, int8_t *digits, int2 *xscale, uint32_t *ell,
                       float *coef, uint32_t *dbg_samples, float *dbg_coef, hipStream_t s) {
    const int groups = (batch + ST - 1) / ST;
    const long long nb = (long long)K * ((J + SC_DRAWS - 1) / SC_DRAWS);
    if (nb > 2147483647ll) return fail(KERDOCK_ERR_INVALID_ARG, "shared form: too many draws");
    if (groups > 65535) return fail(KERDOCK_ERR_INVALID_ARG, "shared form: launch too large");
    const int n_pad = shared_n_pad(n);
    if (n <= 2048) hipLaunchKernelGGL(k_x_digits<1>, dim3(batch), dim3(64), 0, s, X, n, n_pad, digits, xscale);
    else hipLaunchKernelGGL(k_x_digits<2>, dim3(batch), dim3(64), 0, s, X, n, n_pad, digits, xscale);
    KD_LAUNCH("k_x_digits");
    const size_t sign_lds = (size_t)SC_DRAWS * ((k >= 5 ? (1 << k) / 32 : 1) + 1) * 4;
    hipLaunchKernelGGL(k_shared_coef, dim3((unsigned)nb, groups), dim3(256), sign_lds, s, X, n, n_pad, k, L, signs, seed, t0,
                       batch, J, K, shared_by_vector(dt) ? 1 : 0, digits, xscale, ell, coef, dbg_samples, dbg_coef);
    KD_LAUNCH("k_shared_coef");
    return KERDOCK_OK;
}

int launch_shared_gemm(kerdock_dtype dt, const void *table, int pitch, int batch, int J, int K, const uint32_t *ell,
                       const float *coef, float *partial, hipStream_t s) {
    const int groups = (batch + ST - 1) / ST;
    if (groups > 65535) return fail(KERDOCK_ERR_INVALID_ARG, "shared form: batch too large");
    const int splits = shared_splits(J);
    dim3 grid((pitch + SG_BM - 1) / SG_BM, K * splits, groups);
    dim3 grid16((pitch + SB_BM - 1) / SB_BM, K * splits, groups);
    const unsigned char *tb = reinterpret_cast<const unsigned char *>(table);
    const int cb = pitch * (int)dtype_bytes(dt), N = J * K;
    switch (dt) {
    case KERDOCK_F32:
        hipLaunchKernelGGL(k_shared_gemm, grid, dim3(256), 0, s, tb, cb, pitch, batch, J, K, N, splits, ell,
                           coef, partial);
        break;
    case KERDOCK_BF16:
        hipLaunchKernelGGL(k_shared_gemm16<KERDOCK_BF16>, grid16, dim3(256), 0, s, tb, cb, pitch, batch, J, K, N, splits,
                           ell, coef, partial);
        break;
    case KERDOCK_FP8E4M3:
        hipLaunchKernelGGL(k_shared_gemm16<KERDOCK_FP8E4M3>, grid16, dim3(256), 0, s, tb, cb, pitch, batch, J, K, N,
                           splits, ell, coef, partial);
        break;
    }
    KD_LAUNCH("k_shared_gemm");
    return KERDOCK_OK;
}

}  // namespace kd
