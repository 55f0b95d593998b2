// Single-handle kernels of the streaming step: thin wrappers around the
// device code in apply_device.hpp, one launch per stage.
#include "apply_device.hpp"

namespace kd {

template <int DT, int TILES, int UNROLL, bool GROUPED, int P>
__global__ __launch_bounds__(GATHER_THREADS) void k_draw_gather(DGArgs a) {
    __shared__ __align__(16) unsigned char smem[DGSmem<DT, GROUPED, P>::BYTES];
    draw_gather<DT, TILES, UNROLL, GROUPED, P>(a, blockIdx.z, blockIdx.x, blockIdx.y, gridDim.x, smem);
}

// grid (K, batch): draws of batch blockIdx.x of vector blockIdx.y, grouped
// by basis (dynamic LDS: (d/2 + 1) * 4 counters)
__global__ __launch_bounds__(SORT_THREADS) void k_draw_sort(DGArgs a) {
    extern __shared__ uint32_t cur[];
    __shared__ int sh[SORT_THREADS / 64 + 1];
    draw_sort(a, blockIdx.y, blockIdx.x, cur, sh);
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

// ---- row-merged survivor step (many vectors): count, scan, scatter, dots
// row_ws: cnt [nblk][m], off [nblk][m + 1], pairs [batch * s_max]
__global__ void k_rows_zero(int *__restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

// grid (batch), one wave: cnt[blk][row] += 1 for every row of S_t
__global__ __launch_bounds__(64) void k_rows_count(SurvArgs a) {
    const int t = blockIdx.x, blk = t / SURV_SBLOCK;
    if (a.active && !a.active[t]) return;
    const int ns = min(a.nsurv[t], a.s_max);
    int *cnt = a.row_ws + (size_t)blk * a.m;
    for (int s = threadIdx.x; s < ns; s += 64) atomicAdd(&cnt[a.surv[(size_t)t * a.s_max + s]], 1);
}

// grid (nblk), SELECT_THREADS: off[blk][i] = sum of cnt[blk][< i], i <= m
__global__ __launch_bounds__(SELECT_THREADS) void k_rows_scan(SurvArgs a, int nblk) {
    __shared__ int scan_sh[SELECT_THREADS / 64 + 1];
    const int blk = blockIdx.x, m = a.m;
    const int *cnt = a.row_ws + (size_t)blk * m;
    int *off = a.row_ws + (size_t)nblk * m + (size_t)blk * (m + 1);
    const int per = (m + SELECT_THREADS - 1) / SELECT_THREADS;
    const int i0 = min(m, (int)threadIdx.x * per), i1 = min(m, i0 + per);
    int local = 0;
    for (int i = i0; i < i1; ++i) local += cnt[i];
    int total;
    int run = block_exclusive_scan(local, &total, scan_sh);
    for (int i = i0; i < i1; ++i) {
        off[i] = run;
        run += cnt[i];
    }
    if (threadIdx.x == 0) off[m] = total;
}

// grid (batch), one wave: pair index t s_max + s placed in its row's range
// (cnt counts back down to zero)
__global__ __launch_bounds__(64) void k_rows_scatter(SurvArgs a, int nblk) {
    const int t = blockIdx.x, blk = t / SURV_SBLOCK, m = a.m;
    if (a.active && !a.active[t]) return;
    const int ns = min(a.nsurv[t], a.s_max);
    int *cnt = a.row_ws + (size_t)blk * m;
    const int *off = a.row_ws + (size_t)nblk * m + (size_t)blk * (m + 1);
    int *pairs = a.row_ws + (size_t)nblk * m + (size_t)nblk * (m + 1) + (size_t)blk * SURV_SBLOCK * a.s_max;
    for (int s = threadIdx.x; s < ns; s += 64) {
        const int row = a.surv[(size_t)t * a.s_max + s];
        const int pos = off[row] + atomicSub(&cnt[row], 1) - 1;
        pairs[pos] = t * a.s_max + s;
    }
}

// grid (8 ceil(nblk / 8) rg), 256 threads, rg = ceil(m / 4): wave = one row
// of A, in registers, dotted with every vector of the block that selected
// it.  Workgroups are dealt to the 8 XCDs in turn, so workgroup id = 8 j + x
// runs on XCD x; XCD x takes blocks x, x + 8, ..., one after another.
__global__ __launch_bounds__(SURV_THREADS) void k_rows_dots(SurvArgs a, int nblk) {
    const int m = a.m, lane = threadIdx.x & 63;
    const int rg = (m + SURV_THREADS / 64 - 1) / (SURV_THREADS / 64);
    const int xcd = blockIdx.x % 8, jx = blockIdx.x / 8;
    const int blk = xcd + 8 * (jx / rg);
    const int row = (jx % rg) * (SURV_THREADS / 64) + (threadIdx.x >> 6);
    if (blk >= nblk || row >= m) return;
    const int *off = a.row_ws + (size_t)nblk * m + (size_t)blk * (m + 1);
    const int beg = off[row], end = off[row + 1];
    if (beg == end) return;
    const int *pairs = a.row_ws + (size_t)nblk * m + (size_t)nblk * (m + 1) + (size_t)blk * SURV_SBLOCK * a.s_max;
    typedef float v4f __attribute__((ext_vector_type(4)));
    const v4f *r4 = reinterpret_cast<const v4f *>(a.A + (size_t)row * a.n);
    const int n4 = a.n >> 2;
    float4 rr[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int q = lane + 64 * i;
        const v4f v = q < n4 ? __builtin_nontemporal_load(r4 + q) : v4f{0.f, 0.f, 0.f, 0.f};
        rr[i] = make_float4(v.x, v.y, v.z, v.w);
    }
    for (int pi = beg; pi < end; ++pi) {
        const int idx = pairs[pi];
        const int t = idx / a.s_max;
        const float v = survivor_dot_regs(rr, a.X + (size_t)t * a.n, a.n);
        if (lane == 0) a.svals[idx] = v;
    }
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

// -------------------------------------------------------------- launchers --

int launch_topc_logits(const float *Z, int B, int m, int c, int32_t *cand, int32_t *ncand, hipStream_t s) {
    hipLaunchKernelGGL(k_topc_logits, dim3(B), dim3(SELECT_THREADS), (size_t)m * 4, s, Z, m, c, cand, ncand);
    KD_LAUNCH("k_topc_logits");
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
        else if (unroll >= 16) launch_dg<DT, 1, 16, true>(grid, a, s);
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

size_t sort_lds_bytes(int k) { return (size_t)((1 << (k - 1)) + 1) * 4 * sizeof(uint32_t); }

int launch_draw_sort(const DGArgs &a, int batch, int K, hipStream_t s) {
    if (batch > 65535) return fail(KERDOCK_ERR_INVALID_ARG, "batch above 65535 (grid y dimension of the draw sort)");
    hipLaunchKernelGGL(k_draw_sort, dim3(K, batch), dim3(SORT_THREADS), sort_lds_bytes(a.k), s, a);
    KD_LAUNCH("k_draw_sort");
    return KERDOCK_OK;
}

int launch_draw_gather(kerdock_dtype dt, const DGArgs &a, int batch, int K, int unroll, hipStream_t s) {
    if (a.chunk < 1 || a.chunk > MAX_CHUNK) return fail(KERDOCK_ERR_INVALID_ARG, "gather chunk out of range");
    const GatherShape g = gather_shape(dt, a.pitch, (long long)batch * K * a.chunks_per_batch);
    // a launch too small to fill the chip is latency-bound: most loads in flight
    if (g.small) unroll = 16;
    if (batch > 65535) return fail(KERDOCK_ERR_INVALID_ARG, "batch above 65535 (grid z dimension of the gather)");
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
    if (a.svals && a.row_ws && a.vec4 && a.n <= 4096) {
        const int nblk = (batch + SURV_SBLOCK - 1) / SURV_SBLOCK;
        hipLaunchKernelGGL(k_rows_zero, dim3(256), dim3(256), 0, s, a.row_ws, (size_t)nblk * a.m);
        hipLaunchKernelGGL(k_rows_count, dim3(batch), dim3(64), 0, s, a);
        hipLaunchKernelGGL(k_rows_scan, dim3(nblk), dim3(SELECT_THREADS), 0, s, a, nblk);
        hipLaunchKernelGGL(k_rows_scatter, dim3(batch), dim3(64), 0, s, a, nblk);
        const int per = SURV_THREADS / 64;
        const long long wgs = 8ll * ((nblk + 7) / 8) * ((a.m + per - 1) / per);
        if (wgs > 2147483647ll) return fail(KERDOCK_ERR_INVALID_ARG, "batch too large for the row-merged survivor grid");
        hipLaunchKernelGGL(k_rows_dots, dim3((unsigned)wgs), dim3(SURV_THREADS), 0, s, a, nblk);
        KD_LAUNCH("k_rows_dots");
        hipLaunchKernelGGL(k_survivor_compact, dim3(batch), dim3(64), 0, s, a);
        KD_LAUNCH("k_survivor_compact");
        return KERDOCK_OK;
    }
    hipLaunchKernelGGL(k_survivors, dim3(batch), dim3(SURV_THREADS), (size_t)a.s_max * sizeof(float), s, a);
    KD_LAUNCH("k_survivors");
    return KERDOCK_OK;
}

}  // namespace kd
