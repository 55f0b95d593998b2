// Single-handle kernels of the streaming step: thin wrappers around the
// device code in apply_device.hpp, one launch per stage.
#include "apply_device.hpp"

namespace kd {

template <int DT, int TILES, int UNROLL, bool GROUPED, int P>
__global__ __launch_bounds__(GATHER_THREADS) void k_draw_gather(DGArgs a) {
    constexpr int E = Elems<DT>::N;
    __shared__ uint32_t s_ell[MAX_CHUNK];
    __shared__ float s_coef[MAX_CHUNK];
    __shared__ float red[GROUPED ? GATHER_THREADS * E : 1];
    draw_gather<DT, TILES, UNROLL, GROUPED, P>(a, blockIdx.z, blockIdx.x, blockIdx.y, gridDim.x, s_ell,
                                               s_coef, red);
}

template <int KMAX>
__global__ __launch_bounds__(SELECT_THREADS) void k_select(SelArgs a) {
    extern __shared__ uint32_t key[];          // [m] bits of |mu|
    __shared__ uint32_t hist[256];
    __shared__ int scan_sh[SELECT_THREADS / 64 + 1];
    __shared__ uint32_t sel_state[2];
    select_vec<KMAX>(a, blockIdx.x, key, hist, scan_sh, sel_state);
}

__global__ __launch_bounds__(SURV_THREADS) void k_survivors(SurvArgs a) {
    extern __shared__ float vals[];
    survivors_vec(a, blockIdx.x, vals);
}

// split survivor step: grid (ceil(s_max / 4), batch), one row of S per wave
__global__ __launch_bounds__(SURV_THREADS) void k_survivor_dots(SurvArgs a) {
    survivor_dots_split(a, blockIdx.y, blockIdx.x * (SURV_THREADS / 64) + (threadIdx.x >> 6));
}

// grid (batch), one wave
__global__ __launch_bounds__(64) void k_survivor_compact(SurvArgs a) {
    const int t = blockIdx.x;
    if (a.active && !a.active[t]) return;
    survivors_compact(a, t, a.svals + (size_t)t * a.s_max);
}

// Learned form: the c rows of largest logit (ties: smaller index), ascending.
// Keys map floats monotonically to unsigned integers.
__global__ __launch_bounds__(SELECT_THREADS) void k_topc_logits(const float *__restrict__ Z, int m, int c,
                                                                int32_t *__restrict__ cand,
                                                                int32_t *__restrict__ ncand) {
    extern __shared__ uint32_t key[];
    __shared__ uint32_t hist[256];
    __shared__ int scan_sh[SELECT_THREADS / 64 + 1];
    __shared__ uint32_t sel_state[2];
    const int t = blockIdx.x;
    for (int i = threadIdx.x; i < m; i += SELECT_THREADS) {
        const uint32_t u = __float_as_uint(Z[(size_t)t * m + i]);
        key[i] = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    }
    __syncthreads();
    select_top(key, m, c, 0u, cand + (size_t)t * c, ncand + t, hist, scan_sh, sel_state);
}

// fall back when the verified energy sum_{i in C} (a_i.x)^2 falls short of
// the exact energy |Ax|^2 by more than tol (NaN also falls back)
__global__ void k_fallback_flags(const float *__restrict__ E, const float *__restrict__ vsum2, int B, float tol,
                                 int32_t *__restrict__ flags) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B) return;
    const float gap = E[t] - vsum2[t];
    flags[t] = (gap <= tol) ? 0 : 1;
}

// -------------------------------------------------------------- launchers --

int launch_topc_logits(const float *Z, int B, int m, int c, int32_t *cand, int32_t *ncand, hipStream_t s) {
    hipLaunchKernelGGL(k_topc_logits, dim3(B), dim3(SELECT_THREADS), (size_t)m * 4, s, Z, m, c, cand, ncand);
    KD_LAUNCH("k_topc_logits");
    return KERDOCK_OK;
}

int launch_fallback_flags(const float *E, const float *vsum2, int B, float tol, int32_t *flags, hipStream_t s) {
    hipLaunchKernelGGL(k_fallback_flags, dim3((B + 255) / 256), dim3(256), 0, s, E, vsum2, B, tol, flags);
    KD_LAUNCH("k_fallback_flags");
    return KERDOCK_OK;
}


GatherShape gather_shape(kerdock_dtype dt, int pitch, long long work) {
    GatherShape g;
    g.small = 0;
    g.col_bytes = pitch * (int)dtype_bytes(dt);
    if (g.col_bytes >= TILE_BYTES) {
        const int need = (g.col_bytes + TILE_BYTES - 1) / TILE_BYTES;
        g.tiles = need >= 3 ? 4 : need;
        // few chunks in the launch: one 4 KiB tile per workgroup, for more
        // workgroups (each entry still sums its draws in the same order)
        if (work * ((need + g.tiles - 1) / g.tiles) < GATHER_MIN_WGS) {
            g.tiles = 1;
            g.small = 1;
        }
        g.segs = (g.col_bytes + g.tiles * TILE_BYTES - 1) / (g.tiles * TILE_BYTES);
        g.groups = 1;
        g.tpc = GATHER_THREADS;
        g.grouped = 0;
    } else {
        g.tiles = 1;
        g.segs = 1;
        g.tpc = g.col_bytes / 16;
        g.groups = GATHER_THREADS / g.tpc;
        g.grouped = 1;
    }
    return g;
}

int gather_chunk_max() { return MAX_CHUNK; }

template <int DT, int TILES, int U, bool GR>
static void launch_dg(dim3 grid, const DGArgs &a, hipStream_t s) {
    if (a.n <= 2048)
        hipLaunchKernelGGL((k_draw_gather<DT, TILES, U, GR, 1>), grid, dim3(GATHER_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((k_draw_gather<DT, TILES, U, GR, 2>), grid, dim3(GATHER_THREADS), 0, s, a);
}

template <int DT>
static void launch_dt(dim3 grid, const GatherShape &g, int unroll, const DGArgs &a, hipStream_t s) {
    if (g.grouped) {
        if (unroll <= 4) launch_dg<DT, 1, 4, true>(grid, a, s);
        else launch_dg<DT, 1, 8, true>(grid, a, s);
    } else if (g.tiles == 1) {
        if (unroll <= 4) launch_dg<DT, 1, 4, false>(grid, a, s);
        else if (unroll >= 16) launch_dg<DT, 1, 16, false>(grid, a, s);
        else launch_dg<DT, 1, 8, false>(grid, a, s);
    } else if (g.tiles == 2) {
        if (unroll <= 4) launch_dg<DT, 2, 4, false>(grid, a, s);
        else launch_dg<DT, 2, 8, false>(grid, a, s);
    } else {
        if (unroll <= 2) launch_dg<DT, 4, 2, false>(grid, a, s);
        else launch_dg<DT, 4, 4, false>(grid, a, s);
    }
}

int launch_draw_gather(kerdock_dtype dt, const DGArgs &a, int batch, int K, int unroll, hipStream_t s) {
    if (a.chunk < 1 || a.chunk > MAX_CHUNK) return fail(KERDOCK_ERR_INVALID_ARG, "gather chunk out of range");
    const GatherShape g = gather_shape(dt, a.pitch, (long long)batch * K * a.chunks_per_batch);
    // a launch too small to fill the chip is latency-bound: most loads in flight
    if (g.small) unroll = 16;
    dim3 grid(K * a.chunks_per_batch, g.segs, batch);
    switch (dt) {
    case KERDOCK_F32: launch_dt<KERDOCK_F32>(grid, g, unroll, a, s); break;
    case KERDOCK_BF16: launch_dt<KERDOCK_BF16>(grid, g, unroll, a, s); break;
    case KERDOCK_FP8E4M3: launch_dt<KERDOCK_FP8E4M3>(grid, g, unroll, a, s); break;
    }
    KD_LAUNCH("k_draw_gather");
    return KERDOCK_OK;
}

int launch_select(const SelArgs &a, int batch, hipStream_t s) {
    const size_t shmem = (size_t)a.m * sizeof(uint32_t);
    dim3 grid(batch), block(SELECT_THREADS);
    if (a.K <= 1) hipLaunchKernelGGL(k_select<1>, grid, block, shmem, s, a);
    else if (a.K <= 2) hipLaunchKernelGGL(k_select<2>, grid, block, shmem, s, a);
    else if (a.K <= 4) hipLaunchKernelGGL(k_select<4>, grid, block, shmem, s, a);
    else if (a.K <= 8) hipLaunchKernelGGL(k_select<8>, grid, block, shmem, s, a);
    else if (a.K <= 16) hipLaunchKernelGGL(k_select<16>, grid, block, shmem, s, a);
    else hipLaunchKernelGGL(k_select<32>, grid, block, shmem, s, a);
    KD_LAUNCH("k_select");
    return KERDOCK_OK;
}

int launch_survivors(const SurvArgs &a, int batch, hipStream_t s) {
    // One workgroup per vector fills the chip when there are many vectors;
    // otherwise spread the rows of S over one wave each.
    if (a.svals && batch < SURV_SPLIT_BATCH) {
        if (batch > 65535) return fail(KERDOCK_ERR_INVALID_ARG, "batch too large for the split survivor grid");
        const int per = SURV_THREADS / 64;
        hipLaunchKernelGGL(k_survivor_dots, dim3((a.s_max + per - 1) / per, batch), dim3(SURV_THREADS), 0, s, a);
        KD_LAUNCH("k_survivor_dots");
        hipLaunchKernelGGL(k_survivor_compact, dim3(batch), dim3(64), 0, s, a);
        KD_LAUNCH("k_survivor_compact");
        return KERDOCK_OK;
    }
    hipLaunchKernelGGL(k_survivors, dim3(batch), dim3(SURV_THREADS), (size_t)a.s_max * sizeof(float), s, a);
    KD_LAUNCH("k_survivors");
    return KERDOCK_OK;
}

}  // namespace kd
