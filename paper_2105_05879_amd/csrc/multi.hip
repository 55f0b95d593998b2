// Batched form: several prepared matrices (possibly of different n) streamed
// in one persistent launch, captured in a HIP graph, with an autotuned
// unroll depth.
//
// A plan binds, for every handle q, its input rows X_q, its outputs and its
// streaming parameters.  One run is six launches on one stream:
//   k_multi_begin        reset the work counter (a kernel, not a memset, so
//                        that graph replays reset it too);
//   k_multi_sort         the draws of every (handle, vector, batch) of the
//                        handles that group them by basis (draw_sort);
//   k_multi_draw_gather  persistent: every workgroup takes work items
//                        (handle, vector, chunk, segment) from the counter,
//                        longest columns first, and runs the same draws +
//                        gather code as the single-handle kernel; it leaves
//                        when the counter passes the item count;
//   k_multi_select       one workgroup per (handle, vector);
//   k_multi_survivors    one workgroup per (handle, vector);
//   k_multi_end          advance every stream position by its batch, so that
//                        consecutive runs (and graph replays) draw for
//                        consecutive stream positions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "apply_device.hpp"

namespace kd {

constexpr int MAX_MULTI = 8;

struct MultiSelect {
    int nh;
    int offset[MAX_MULTI + 1];       // prefix sums of the batches
    const SelArgs *sel;              // device [nh]
};

struct MultiSurv {
    int nh;
    int offset[MAX_MULTI + 1];
    const SurvArgs *surv;            // device [nh]
};

struct MultiSort {
    int nh;
    int offset[MAX_MULTI + 1];       // prefix sums of batch K
    int K[MAX_MULTI];
    const DGArgs *dg;                // device [nh]
};

// item: handle q (4 bits) | segment (4 bits) | chunk id (24 bits) | vector t (32 bits)
__device__ __forceinline__ void unpack_item(uint64_t v, int &q, int &seg, int &cid, int &t) {
    q = (int)(v >> 60);
    seg = (int)((v >> 56) & 0xF);
    cid = (int)((v >> 32) & 0xFFFFFF);
    t = (int)(v & 0xFFFFFFFFu);
}

__global__ void k_multi_begin(int *counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

__global__ void k_multi_end(int64_t *t0, const int *batch, int nh) {
    const int q = threadIdx.x;
    if (q < nh) t0[q] += batch[q];
}

template <int DT, int TILES, int UNROLL, int P, bool BK>
__global__ __launch_bounds__(GATHER_THREADS) void k_multi_draw_gather(
    const DGArgs *__restrict__ hd, const int *__restrict__ nchunks, const int *__restrict__ grouped,
    const uint64_t *__restrict__ items, int nitems, int *counter) {
    constexpr size_t SMEM = DGSmem<DT, true, P, BK>::BYTES > DGSmem<DT, false, P, BK>::BYTES
                                ? DGSmem<DT, true, P, BK>::BYTES
                                : DGSmem<DT, false, P, BK>::BYTES;
    __shared__ __align__(16) unsigned char smem[SMEM];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();                       // the previous item is finished
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = s_item;
        if (it >= nitems) break;               // every workgroup reaches this exit
        int q, seg, cid, t;
        unpack_item(items[it], q, seg, cid, t);
        const DGArgs &a = hd[q];
        if (grouped[q])
            draw_gather<DT, TILES, UNROLL, true, P, BK>(a, t, cid, seg, nchunks[q], smem);
        else
            draw_gather<DT, TILES, UNROLL, false, P, BK>(a, t, cid, seg, nchunks[q], smem);
    }
}

__device__ __forceinline__ int find_handle(const int *offset, int nh, int g) {
    int q = 0;
    while (q + 1 < nh && g >= offset[q + 1]) ++q;
    return q;
}

template <int KMAX>
__global__ __launch_bounds__(SELECT_THREADS) void k_multi_select(MultiSelect ms) {
    extern __shared__ uint32_t key[];
    __shared__ uint32_t hist[256];
    __shared__ int scan_sh[SELECT_THREADS / 64 + 1];
    __shared__ uint32_t sel_state[2];
    const int q = find_handle(ms.offset, ms.nh, blockIdx.x);
    select_vec<KMAX>(ms.sel[q], blockIdx.x - ms.offset[q], key, hist, scan_sh, sel_state);
}

// one workgroup per (handle, vector, batch)
__global__ __launch_bounds__(SORT_THREADS) void k_multi_sort(MultiSort ms) {
    extern __shared__ uint32_t cur[];
    __shared__ int sh[SORT_THREADS / 64 + 1];
    const int q = find_handle(ms.offset, ms.nh, blockIdx.x);
    const int r = blockIdx.x - ms.offset[q];
    if (!ms.dg[q].bucket) return;              // this handle draws inside the gather
    draw_sort(ms.dg[q], r / ms.K[q], r % ms.K[q], cur, sh);
}

__global__ __launch_bounds__(SURV_THREADS) void k_multi_survivors(MultiSurv mv) {
    extern __shared__ float vals[];
    const int q = find_handle(mv.offset, mv.nh, blockIdx.x);
    survivors_vec(mv.surv[q], blockIdx.x - mv.offset[q], vals);
}

}  // namespace kd

// ------------------------------------------------------------------ plan --

struct kerdock_multi_s {
    int nh = 0;
    kerdock_dtype dtype = KERDOCK_F32;
    int batch[kd::MAX_MULTI] = {}, K[kd::MAX_MULTI] = {}, s_max[kd::MAX_MULTI] = {};
    int m[kd::MAX_MULTI] = {};
    int tiles = 1, P = 1, kmax = 1, unroll = 8;
    int any_bucket = 0;               // some handle groups its draws by basis
    int nitems = 0, total_batch = 0, max_m = 1, max_smax = 1, grid = 0;
    kd::MultiSelect msel{};
    kd::MultiSurv msurv{};
    kd::MultiSort msort{};
    int sort_wgs = 0;
    size_t sort_lds = 0;
    void *ws = nullptr;               // device: everything below
    kd::DGArgs *dg_dev = nullptr;
    kd::SelArgs *sel_dev = nullptr;
    kd::SurvArgs *surv_dev = nullptr;
    int *nchunks_dev = nullptr, *grouped_dev = nullptr, *batch_dev = nullptr, *counter = nullptr;
    int64_t *t0_dev = nullptr;
    uint64_t *items = nullptr;
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_def = nullptr;
    int device = 0;
};

namespace kd {

int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
int gather_chunk_max();
size_t sort_lds_bytes(int k);

static size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

template <int DT, int TILES, int U, int P, bool BK>
static void multi_launch_dt(const kerdock_multi_s *pl, hipStream_t s) {
    hipLaunchKernelGGL((k_multi_draw_gather<DT, TILES, U, P, BK>), dim3(pl->grid), dim3(GATHER_THREADS), 0, s,
                       pl->dg_dev, pl->nchunks_dev, pl->grouped_dev, pl->items, pl->nitems, pl->counter);
}

// Plans without a handle that groups its draws run kernels without that path
// (fewer registers, more resident workgroups) at the tuned unroll; plans with
// one use a single unroll per tile count (the unroll never changes results).
template <int DT, int TILES, int P>
static void multi_launch_u(const kerdock_multi_s *pl, hipStream_t s) {
    if constexpr (TILES == 4) {
        if (pl->any_bucket) multi_launch_dt<DT, TILES, 4, P, true>(pl, s);
        else if (pl->unroll <= 2) multi_launch_dt<DT, TILES, 2, P, false>(pl, s);
        else multi_launch_dt<DT, TILES, 4, P, false>(pl, s);
    } else if constexpr (TILES == 2) {
        if (pl->any_bucket) multi_launch_dt<DT, TILES, 8, P, true>(pl, s);
        else if (pl->unroll <= 4) multi_launch_dt<DT, TILES, 4, P, false>(pl, s);
        else multi_launch_dt<DT, TILES, 8, P, false>(pl, s);
    } else {
        if (pl->any_bucket) multi_launch_dt<DT, TILES, 8, P, true>(pl, s);
        else if (pl->unroll <= 4) multi_launch_dt<DT, TILES, 4, P, false>(pl, s);
        else if (pl->unroll >= 16) multi_launch_dt<DT, TILES, 16, P, false>(pl, s);
        else multi_launch_dt<DT, TILES, 8, P, false>(pl, s);
    }
}

template <int DT, int P>
static void multi_launch_t(const kerdock_multi_s *pl, hipStream_t s) {
    if (pl->tiles == 1) multi_launch_u<DT, 1, P>(pl, s);
    else if (pl->tiles == 2) multi_launch_u<DT, 2, P>(pl, s);
    else multi_launch_u<DT, 4, P>(pl, s);
}

template <int DT>
static void multi_launch_p(const kerdock_multi_s *pl, hipStream_t s) {
    if (pl->P == 1) multi_launch_t<DT, 1>(pl, s);
    else multi_launch_t<DT, 2>(pl, s);
}

static void multi_gather(const kerdock_multi_s *pl, hipStream_t s) {
    switch (pl->dtype) {
    case KERDOCK_F32: multi_launch_p<KERDOCK_F32>(pl, s); break;
    case KERDOCK_BF16: multi_launch_p<KERDOCK_BF16>(pl, s); break;
    case KERDOCK_FP8E4M3: multi_launch_p<KERDOCK_FP8E4M3>(pl, s); break;
    }
}

// persistent grid: workgroups resident at once on the device
template <int DT, int TILES, int U, int P, bool BK>
static int resident_dt(int cus) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_multi_draw_gather<DT, TILES, U, P, BK>,
                                                     GATHER_THREADS, 0) != hipSuccess || per < 1)
        per = 1;
    return per * cus;
}

// occupancy of the instantiation that multi_gather would launch
template <int DT, int TILES, int P>
static int resident_u(const kerdock_multi_s *pl, int cus) {
    if constexpr (TILES == 4) {
        if (pl->any_bucket) return resident_dt<DT, TILES, 4, P, true>(cus);
        return pl->unroll <= 2 ? resident_dt<DT, TILES, 2, P, false>(cus) : resident_dt<DT, TILES, 4, P, false>(cus);
    } else if constexpr (TILES == 2) {
        if (pl->any_bucket) return resident_dt<DT, TILES, 8, P, true>(cus);
        return pl->unroll <= 4 ? resident_dt<DT, TILES, 4, P, false>(cus) : resident_dt<DT, TILES, 8, P, false>(cus);
    } else {
        if (pl->any_bucket) return resident_dt<DT, TILES, 8, P, true>(cus);
        return pl->unroll <= 4    ? resident_dt<DT, TILES, 4, P, false>(cus)
               : pl->unroll >= 16 ? resident_dt<DT, TILES, 16, P, false>(cus)
                                  : resident_dt<DT, TILES, 8, P, false>(cus);
    }
}

template <int DT, int P>
static int resident_t(const kerdock_multi_s *pl, int cus) {
    if (pl->tiles == 1) return resident_u<DT, 1, P>(pl, cus);
    if (pl->tiles == 2) return resident_u<DT, 2, P>(pl, cus);
    return resident_u<DT, 4, P>(pl, cus);
}

static int resident(const kerdock_multi_s *pl, int cus) {
    switch (pl->dtype) {
    case KERDOCK_F32: return pl->P == 1 ? resident_t<KERDOCK_F32, 1>(pl, cus) : resident_t<KERDOCK_F32, 2>(pl, cus);
    case KERDOCK_BF16: return pl->P == 1 ? resident_t<KERDOCK_BF16, 1>(pl, cus) : resident_t<KERDOCK_BF16, 2>(pl, cus);
    case KERDOCK_FP8E4M3:
        return pl->P == 1 ? resident_t<KERDOCK_FP8E4M3, 1>(pl, cus) : resident_t<KERDOCK_FP8E4M3, 2>(pl, cus);
    }
    return cus;
}

static int multi_enqueue(kerdock_multi_s *pl, hipStream_t s) {
    hipLaunchKernelGGL(k_multi_begin, dim3(1), dim3(64), 0, s, pl->counter);
    hipLaunchKernelGGL(k_multi_sort, dim3(pl->sort_wgs), dim3(SORT_THREADS), pl->sort_lds, s, pl->msort);
    multi_gather(pl, s);
    const size_t key_bytes = (size_t)pl->max_m * 4;
    dim3 g(pl->total_batch), b(SELECT_THREADS);
    if (pl->kmax <= 1) hipLaunchKernelGGL(k_multi_select<1>, g, b, key_bytes, s, pl->msel);
    else if (pl->kmax <= 2) hipLaunchKernelGGL(k_multi_select<2>, g, b, key_bytes, s, pl->msel);
    else if (pl->kmax <= 4) hipLaunchKernelGGL(k_multi_select<4>, g, b, key_bytes, s, pl->msel);
    else if (pl->kmax <= 8) hipLaunchKernelGGL(k_multi_select<8>, g, b, key_bytes, s, pl->msel);
    else if (pl->kmax <= 16) hipLaunchKernelGGL(k_multi_select<16>, g, b, key_bytes, s, pl->msel);
    else hipLaunchKernelGGL(k_multi_select<32>, g, b, key_bytes, s, pl->msel);
    hipLaunchKernelGGL(k_multi_survivors, dim3(pl->total_batch), dim3(SURV_THREADS),
                       (size_t)pl->max_smax * 4, s, pl->msurv);
    hipLaunchKernelGGL(k_multi_end, dim3(1), dim3(64), 0, s, pl->t0_dev, pl->batch_dev, pl->nh);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "multi launches");
    return KERDOCK_OK;
}

static void free_plan(kerdock_multi_s *pl) {
    if (!pl) return;
    if (pl->graph) (void)hipGraphExecDestroy(pl->graph);
    if (pl->graph_def) (void)hipGraphDestroy(pl->graph_def);
    (void)hipFree(pl->ws);
    delete pl;
}

}  // namespace kd

using namespace kd;

extern "C" {

int kerdock_multi_create(const kerdock_handle *hs, int nh, const float *const *X, const int *batch,
                         const kerdock_apply_params *params, float eps, const int *s_max,
                         int32_t *const *out_idx, float *const *out_val, int32_t *const *out_cnt,
                         kerdock_multi *out) {
    if (!out) return fail(KERDOCK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!hs || nh < 1 || nh > MAX_MULTI || !X || !batch || !params || !s_max || !out_idx || !out_val || !out_cnt)
        return fail(KERDOCK_ERR_INVALID_ARG, "multi: need 1..8 handles and every array");
    if (!(eps > 0.f) || !(eps < INFINITY)) return fail(KERDOCK_ERR_INVALID_ARG, "eps must be > 0");
    kerdock_multi_s *pl = new kerdock_multi_s();
    pl->nh = nh;
    pl->dtype = hs[0] ? hs[0]->dtype : KERDOCK_F32;
    for (int q = 0; q < nh; ++q) {
        const kerdock_handle h = hs[q];
        const kerdock_apply_params *p = &params[q];
        if (!h) { delete pl; return fail(KERDOCK_ERR_NOT_PREPARED, "multi: NULL handle"); }
        if (h->dtype != pl->dtype) { delete pl; return fail(KERDOCK_ERR_INVALID_ARG, "multi: handles must share the table dtype"); }
        if (batch[q] < 1 || !X[q] || !out_idx[q] || !out_val[q] || !out_cnt[q] || s_max[q] < 1 || s_max[q] > h->m ||
            p->J < 1 || p->K < 1 || p->K > 32 || (int64_t)p->J * p->K > ((int64_t)1 << 31) - 64 ||
            (int64_t)batch[q] * s_max[q] >= ((int64_t)1 << 31)) {
            delete pl;
            return fail(KERDOCK_ERR_INVALID_ARG, "multi: invalid batch, pointer, s_max, J or K for handle " + std::to_string(q));
        }
    }
    if (hipGetDevice(&pl->device) != hipSuccess) { delete pl; return fail(KERDOCK_ERR_HIP, "hipGetDevice"); }

    // geometry and workspace layout
    std::vector<DGArgs> dg(nh);
    std::vector<SelArgs> sel(nh);
    std::vector<SurvArgs> sv(nh);
    std::vector<int> nchunks(nh), grouped(nh), chunk(nh), cpb(nh), bucket(nh);
    std::vector<size_t> off_partial(nh), off_jlist(nh), off_sorted(nh), off_surv(nh), off_nsurv(nh);
    size_t off = 0;
    const size_t off_dg = off; off += al(sizeof(DGArgs) * nh);
    const size_t off_sel = off; off += al(sizeof(SelArgs) * nh);
    const size_t off_sv = off; off += al(sizeof(SurvArgs) * nh);
    const size_t off_nch = off; off += al(sizeof(int) * nh);
    const size_t off_grp = off; off += al(sizeof(int) * nh);
    const size_t off_bat = off; off += al(sizeof(int) * nh);
    const size_t off_cnt = off; off += al(sizeof(int));
    const size_t off_t0 = off; off += al(sizeof(int64_t) * nh);
    size_t items = 0;
    pl->total_batch = 0;
    for (int q = 0; q < nh; ++q) {
        const kerdock_handle h = hs[q];
        const int J = params[q].J, K = params[q].K;
        if (params[q].chunk < 0 || params[q].chunk > gather_chunk_max()) {
            delete pl;
            return fail(KERDOCK_ERR_INVALID_ARG, "multi: chunk must lie in [0, 1024]");
        }
        chunk[q] = chunk_for(h, J, params[q].chunk);
        cpb[q] = (J + chunk[q] - 1) / chunk[q];
        nchunks[q] = K * cpb[q];
        if (nchunks[q] > 0xFFFFFF) {       // the chunk id of a work item has 24 bits
            delete pl;
            return fail(KERDOCK_ERR_INVALID_ARG, "multi: K ceil(J / chunk) must stay below 2^24 for handle " +
                                                     std::to_string(q));
        }
        const GatherShape gs = gather_shape(h->dtype, h->pitch);
        grouped[q] = gs.grouped;
        pl->tiles = std::max(pl->tiles, gs.tiles);
        if (gs.segs > 1 || gs.segs * gs.tiles * 4096 > 4 * 4096) { delete pl; return fail(KERDOCK_ERR_INVALID_ARG, "multi: columns longer than 16 KiB"); }
        pl->P = std::max(pl->P, h->n <= 2048 ? 1 : 2);
        pl->kmax = std::max(pl->kmax, K);
        pl->max_m = std::max(pl->max_m, h->m);
        pl->max_smax = std::max(pl->max_smax, s_max[q]);
        pl->batch[q] = batch[q];
        pl->K[q] = K;
        pl->s_max[q] = s_max[q];
        pl->m[q] = h->m;
        off_partial[q] = off; off += al((size_t)batch[q] * nchunks[q] * h->pitch * 4);
        bucket[q] = use_bucket(h, J);
        pl->any_bucket |= bucket[q];
        off_jlist[q] = off; off += bucket[q] ? al((size_t)batch[q] * J * K * 4) : 0;
        off_sorted[q] = off; off += bucket[q] ? al((size_t)batch[q] * J * K * 4) : 0;
        pl->msort.offset[q] = pl->sort_wgs;
        pl->msort.K[q] = K;
        pl->sort_wgs += batch[q] * K;
        pl->sort_lds = std::max(pl->sort_lds, sort_lds_bytes(h->k));
        off_surv[q] = off; off += al((size_t)batch[q] * s_max[q] * 4);
        off_nsurv[q] = off; off += al((size_t)batch[q] * 4);
        items += (size_t)batch[q] * nchunks[q];
        pl->msel.offset[q] = pl->total_batch;
        pl->total_batch += batch[q];
    }
    pl->msel.offset[nh] = pl->total_batch;
    pl->msort.offset[nh] = pl->sort_wgs;
    pl->msort.nh = nh;
    const size_t off_items = off; off += al(sizeof(uint64_t) * items);
    if (items > (size_t)0x7FFFFFFF) { delete pl; return fail(KERDOCK_ERR_INVALID_ARG, "multi: too many work items"); }
    if (hipMalloc(&pl->ws, off) != hipSuccess) { delete pl; return fail(KERDOCK_ERR_OOM, "multi workspace"); }
    char *ws = reinterpret_cast<char *>(pl->ws);
    pl->dg_dev = reinterpret_cast<DGArgs *>(ws + off_dg);
    pl->sel_dev = reinterpret_cast<SelArgs *>(ws + off_sel);
    pl->surv_dev = reinterpret_cast<SurvArgs *>(ws + off_sv);
    pl->nchunks_dev = reinterpret_cast<int *>(ws + off_nch);
    pl->grouped_dev = reinterpret_cast<int *>(ws + off_grp);
    pl->batch_dev = reinterpret_cast<int *>(ws + off_bat);
    pl->counter = reinterpret_cast<int *>(ws + off_cnt);
    pl->t0_dev = reinterpret_cast<int64_t *>(ws + off_t0);
    pl->items = reinterpret_cast<uint64_t *>(ws + off_items);
    pl->nitems = (int)items;

    std::vector<int64_t> t0(nh);
    for (int q = 0; q < nh; ++q) {
        const kerdock_handle h = hs[q];
        const kerdock_apply_params *p = &params[q];
        const GatherShape gs = gather_shape(h->dtype, h->pitch);
        DGArgs &a = dg[q];
        a = DGArgs{};
        a.table = reinterpret_cast<const unsigned char *>(h->table);
        a.col_bytes = gs.col_bytes;
        a.X = X[q];
        a.n = h->n;
        a.k = h->k;
        a.L = h->L;
        a.signs = h->signs;
        a.seed = p->seed;
        a.t0_dev = pl->t0_dev + q;
        a.t0 = 0;
        a.N = p->J * p->K;
        a.J = p->J;
        a.chunk = chunk[q];
        a.chunks_per_batch = cpb[q];
        a.groups = gs.groups;
        a.tpc = gs.tpc;
        a.pitch = h->pitch;
        a.partial = reinterpret_cast<float *>(ws + off_partial[q]);
        a.bucket = bucket[q];
        a.jlist = bucket[q] ? reinterpret_cast<uint32_t *>(ws + off_jlist[q]) : nullptr;
        a.sorted = bucket[q] ? reinterpret_cast<uint32_t *>(ws + off_sorted[q]) : nullptr;
        a.perm = nullptr;
        a.dbg_samples = nullptr;
        a.dbg_coef = nullptr;
        int32_t *sv_ = reinterpret_cast<int32_t *>(ws + off_surv[q]);
        int32_t *ns_ = reinterpret_cast<int32_t *>(ws + off_nsurv[q]);
        sel[q] = SelArgs{a.partial, h->m, h->pitch, p->K, cpb[q], p->J, h->scales, s_max[q], p->tau,
                         nullptr, sv_, ns_};
        sv[q] = SurvArgs{h->A, h->n, X[q], sv_, ns_, s_max[q], eps, out_idx[q], out_val[q], out_cnt[q], nullptr,
                         nullptr, nullptr, nullptr, surv_vec4(X[q], h->n)};
        t0[q] = p->t0;
    }
    // work items, longest columns first
    std::vector<int> order(nh);
    for (int q = 0; q < nh; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return dg[a].col_bytes > dg[b].col_bytes; });
    std::vector<uint64_t> it;
    it.reserve(items);
    for (int q : order)
        for (int t = 0; t < batch[q]; ++t)
            for (int c = 0; c < nchunks[q]; ++c)
                it.push_back(((uint64_t)q << 60) | ((uint64_t)c << 32) | (uint64_t)(uint32_t)t);
    hipError_t e = hipSuccess;
    if ((e = hipMemcpy(pl->dg_dev, dg.data(), sizeof(DGArgs) * nh, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(pl->sel_dev, sel.data(), sizeof(SelArgs) * nh, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(pl->surv_dev, sv.data(), sizeof(SurvArgs) * nh, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(pl->nchunks_dev, nchunks.data(), sizeof(int) * nh, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(pl->grouped_dev, grouped.data(), sizeof(int) * nh, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(pl->batch_dev, batch, sizeof(int) * nh, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(pl->t0_dev, t0.data(), sizeof(int64_t) * nh, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(pl->items, it.data(), sizeof(uint64_t) * items, hipMemcpyHostToDevice)) != hipSuccess) {
        free_plan(pl);
        return hip_fail(e, "multi: upload");
    }
    pl->msel.nh = nh;
    pl->msel.sel = pl->sel_dev;
    pl->msurv.nh = nh;
    for (int q = 0; q <= nh; ++q) pl->msurv.offset[q] = pl->msel.offset[q];
    pl->msurv.surv = pl->surv_dev;
    pl->msort.dg = pl->dg_dev;
    int tuned = 0;
    for (int q = 0; q < nh; ++q) tuned = std::max(tuned, hs[q]->tune_unroll);
    pl->unroll = tuned > 0 ? tuned : 8;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, pl->device)) != hipSuccess) { free_plan(pl); return hip_fail(e, "properties"); }
    pl->grid = resident(pl, prop.multiProcessorCount);
    *out = pl;
    return KERDOCK_OK;
}

int kerdock_multi_run(kerdock_multi plan, void *stream) {
    if (!plan) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL plan");
    return multi_enqueue(plan, reinterpret_cast<hipStream_t>(stream));
}

int kerdock_multi_set_position(kerdock_multi plan, const int64_t *t0) {
    if (!plan) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL plan");
    if (!t0) return fail(KERDOCK_ERR_INVALID_ARG, "t0 is NULL");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(plan->t0_dev, t0, sizeof(int64_t) * plan->nh, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "multi: set position");
    return KERDOCK_OK;
}

int kerdock_multi_graph_launch(kerdock_multi plan, void *stream) {
    if (!plan) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL plan");
    hipError_t e;
    if (!plan->graph) {
        hipStream_t cs;
        if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "capture stream");
        if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
            (void)hipStreamDestroy(cs);
            return hip_fail(e, "begin capture");
        }
        const int rc = multi_enqueue(plan, cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        (void)hipStreamDestroy(cs);
        if (rc != KERDOCK_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        if ((e = hipGraphInstantiate(&plan->graph, g, nullptr, nullptr, 0)) != hipSuccess) {
            (void)hipGraphDestroy(g);
            plan->graph = nullptr;
            return hip_fail(e, "instantiate graph");
        }
        plan->graph_def = g;
    }
    if ((e = hipGraphLaunch(plan->graph, reinterpret_cast<hipStream_t>(stream))) != hipSuccess)
        return hip_fail(e, "graph launch");
    return KERDOCK_OK;
}

int kerdock_multi_autotune(kerdock_multi plan, void *stream, int *best_unroll) {
    if (!plan) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL plan");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int cands_1[] = {4, 8, 16}, cands_2[] = {4, 8}, cands_4[] = {2, 4};
    const int *cands = plan->tiles == 1 ? cands_1 : plan->tiles == 2 ? cands_2 : cands_4;
    const int nc = plan->tiles == 1 ? 3 : 2;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, plan->device);
    if (e != hipSuccess) return hip_fail(e, "properties");
    hipEvent_t a, b;
    if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) return hip_fail(e, "events");
    float best = 1e30f;
    int best_u = plan->unroll;
    // the draws of the current stream positions, grouped by basis (they do
    // not depend on the gather shape that is being timed)
    hipLaunchKernelGGL(k_multi_sort, dim3(plan->sort_wgs), dim3(SORT_THREADS), plan->sort_lds, s, plan->msort);
    for (int i = 0; i < nc; ++i) {
        plan->unroll = cands[i];
        plan->grid = resident(plan, prop.multiProcessorCount);
        float tmin = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
            hipLaunchKernelGGL(k_multi_begin, dim3(1), dim3(64), 0, s, plan->counter);
            (void)hipEventRecord(a, s);
            multi_gather(plan, s);
            (void)hipEventRecord(b, s);
            if ((e = hipEventSynchronize(b)) != hipSuccess) { (void)hipEventDestroy(a); (void)hipEventDestroy(b); return hip_fail(e, "autotune run"); }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, a, b);
            tmin = std::min(tmin, ms);
        }
        if (tmin < best) { best = tmin; best_u = cands[i]; }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    plan->unroll = best_u;
    plan->grid = resident(plan, prop.multiProcessorCount);
    if (plan->graph) {             // a captured graph used the old shape
        (void)hipGraphExecDestroy(plan->graph);
        (void)hipGraphDestroy(plan->graph_def);
        plan->graph = nullptr;
        plan->graph_def = nullptr;
    }
    if (best_unroll) *best_unroll = best_u;
    return KERDOCK_OK;
}

int kerdock_multi_destroy(kerdock_multi plan) {
    if (!plan) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL plan");
    (void)hipSetDevice(plan->device);
    (void)hipDeviceSynchronize();
    free_plan(plan);
    return KERDOCK_OK;
}

int kerdock_sparse_apply_multi(const kerdock_handle *hs, int nh, const float *const *X, const int *batch,
                               const kerdock_apply_params *params, float eps, const int *s_max,
                               int32_t *const *out_idx, float *const *out_val, int32_t *const *out_cnt,
                               void *stream) {
    kerdock_multi plan = nullptr;
    int rc = kerdock_multi_create(hs, nh, X, batch, params, eps, s_max, out_idx, out_val, out_cnt, &plan);
    if (rc != KERDOCK_OK) return rc;
    rc = kerdock_multi_run(plan, stream);
    hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    const int rd = kerdock_multi_destroy(plan);
    if (rc != KERDOCK_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "multi apply");
    return rd;
}

}  // extern "C"
