// C ABI of the Kerdock fast sparsifying transform (include/kerdock.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <stdio.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "apply_device.hpp"

namespace kd {

uint32_t field_polynomial(int D);
std::vector<uint16_t> kerdock_masks(int k, uint32_t *poly_out);

int launch_signs(const uint16_t *masks, int k, uint32_t *signs, hipStream_t s);
int launch_row_scales(const float *A, int m, int n, int pitch, int d, kerdock_dtype dt,
                      float *scales, float *norm2, hipStream_t s);
int launch_table_build(kerdock_dtype dt, int k, const float *A, int m, int n, int pitch,
                       const uint32_t *signs, const float *scales, void *table, hipStream_t s);
int launch_read_columns(kerdock_dtype dt, const void *table, int m, int pitch, int64_t L,
                        const float *scales, const uint32_t *ells, int count, float *out,
                        hipStream_t s);
int launch_draw_gather(kerdock_dtype dt, const DGArgs &a, int batch, int K, int unroll, hipStream_t s);
int launch_draw_sort(const DGArgs &a, int batch, int K, hipStream_t s);
int gather_chunk_max();
int launch_select(const SelArgs &a, int batch, hipStream_t s);
int launch_survivors(const SurvArgs &a, int batch, hipStream_t s);
int launch_shared_coef(kerdock_dtype dt, const float *X, int batch, int n, int k, int64_t L, const uint32_t *signs,
                       uint64_t seed, int64_t t0, int J, int K, int8_t *digits, int2 *xscale, uint32_t *ell,
                       float *coef, uint32_t *dbg_samples, float *dbg_coef, hipStream_t s);
size_t shared_coef_floats(kerdock_dtype dt, int batch, int J, int K);
int shared_n_pad(int n);
size_t shared_digit_bytes(int batch, int n);
int shared_splits(int J);
int launch_shared_gemm(kerdock_dtype dt, const void *table, int pitch, int batch, int J, int K, const uint32_t *ell,
                       const float *coef, float *partial, hipStream_t s);

static thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? KERDOCK_ERR_OOM : KERDOCK_ERR_HIP;
}

// Streaming-step tuning: loads in flight per thread (results do not depend
// on it); overridable with KERDOCK_UNROLL.
static int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    if (!v || !*v) return dflt;
    return atoi(v);
}

// Draws per FP32 partial sum: the caller's value, else the tuned one, else
// about J/8 (so that a single vector still spreads over several chunks per
// batch) between 16 and 512, or 768 for FP8 tables (whose 2-byte-per-row
// columns are short, so a workgroup's coefficient work is amortised over
// more draws); never above J.
int chunk_for(const kerdock_handle_s *h, int J, int requested) {
    int c;
    if (requested > 0) c = requested;
    else if (h->tune_chunk > 0) c = h->tune_chunk;
    else c = std::min(h->dtype == KERDOCK_FP8E4M3 ? 768 : 512, std::max(16, (J + 7) / 8));
    c = std::min(c, gather_chunk_max());
    return c < J ? c : J;
}

// Draws in flight per thread: 16 for short columns (several per workgroup
// step, e.g. 2 KiB FP8 columns: 15.0 -> 14.8 ms at n = m = 2048), 8 otherwise.
static int gather_unroll(const kerdock_handle_s *h, bool grouped) {
    return env_int("KERDOCK_UNROLL", h->tune_unroll > 0 ? h->tune_unroll : grouped ? 16 : 8);
}

// Whether a call groups its draws by basis before the gather (draw_sort and
// the per-basis transform of the coefficients).  It pays only where the
// direct coefficient sums are not hidden behind the column stream: runs of
// at least four draws per basis on average (J >= 4 (d/2 + 1)) and columns
// short against the length of x (m b_T <= 1024 P bytes, P = 1 for n <= 2048,
// else 2).  kerdock_autotune may settle it by timing; KERDOCK_BUCKET=0 / 1
// overrides both.  The summation order of the batch means follows it.
int use_bucket(const kerdock_handle_s *h, int J) {
    const int forced = env_int("KERDOCK_BUCKET", -1);
    if (forced == 0 || forced == 1) return forced;
    if (h->tune_bucket >= 0) return h->tune_bucket;
    const int64_t bases = h->d / 2 + 1;
    const int64_t col = (int64_t)h->pitch * (int64_t)dtype_bytes(h->dtype);
    const int P = h->n <= 2048 ? 1 : 2;
    return ((int64_t)J >= 4 * bases && col <= 1024 * P) ? 1 : 0;
}

// workspace layout of the streaming step (perm only for debug dumps)
struct Workspace {
    size_t partial, jlist, sorted, perm, surv, nsurv, svals, rows, total;
};

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static Workspace workspace_layout(const kerdock_handle_s *h, int batch, int J, int K, int s_max, int chunk,
                                  bool debug = false) {
    const size_t cpb = (J + chunk - 1) / chunk;
    const size_t draws = use_bucket(h, J) ? (size_t)batch * J * K * 4 : 0;
    Workspace w;
    size_t off = 0;
    w.partial = off; off += align256((size_t)batch * K * cpb * h->pitch * 4);
    w.jlist = off;   off += align256(draws);
    w.sorted = off;  off += align256(draws);
    w.perm = off;    off += debug ? align256(draws) : 0;
    w.surv = off;    off += align256((size_t)batch * s_max * 4);
    w.nsurv = off;   off += align256((size_t)batch * 4);
    w.svals = off;   off += align256((size_t)batch * s_max * 4);
    w.rows = off;    off += align256(survivor_rows_bytes(batch, h->m, s_max));
    w.total = off;
    return w;
}

static int ensure_workspace(kerdock_handle_s *h, size_t bytes) {
    if (bytes <= h->ws_bytes) return KERDOCK_OK;
    if (h->ws) {
        KD_HIP(hipDeviceSynchronize());
        KD_HIP(hipFree(h->ws));
        h->ws = nullptr;
        h->ws_bytes = 0;
    }
    hipError_t e = hipMalloc(&h->ws, bytes);
    if (e != hipSuccess) {
        h->ws = nullptr;
        return fail(KERDOCK_ERR_OOM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
    }
    h->ws_bytes = bytes;
    return KERDOCK_OK;
}

static void free_handle(kerdock_handle_s *h) {
    if (!h) return;
    (void)hipFree(h->table);
    (void)hipFree(h->scales);
    (void)hipFree(h->A);
    (void)hipFree(h->signs);
    (void)hipFree(h->masks);
    (void)hipFree(h->ws);
    for (int q = 0; q < 5; ++q)
        if (h->ev[q]) (void)hipEventDestroy(h->ev[q]);
    free_learned(h->learned);
    delete h;
}

// Tuning cache: one line "m n dtype K chunk unroll bucket" per tuned shape, in the
// file named by KERDOCK_TUNE_CACHE (read at prepare, appended by autotune).
static void cache_lookup(kerdock_handle_s *h) {
    const char *path = getenv("KERDOCK_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    int m, n, dt, K, c, u, bk;
    while (fscanf(f, "%d %d %d %d %d %d %d", &m, &n, &dt, &K, &c, &u, &bk) == 7)
        if (m == h->m && n == h->n && dt == (int)h->dtype) {
            h->tune_chunk = c;
            h->tune_unroll = u;
            h->tune_bucket = bk;
        }
    fclose(f);
}

static void cache_store(const kerdock_handle_s *h, int K) {
    const char *path = getenv("KERDOCK_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%d %d %d %d %d %d %d\n", h->m, h->n, (int)h->dtype, K, h->tune_chunk, h->tune_unroll, h->tune_bucket);
    fclose(f);
}

// The streaming step for every row of X; rows t with active[t] == 0 (when
// active is given) are skipped by every kernel and their outputs untouched.
// Argument checks shared by the streaming entry points; 1 = nothing to do.
static int check_apply_args(kerdock_handle h, const float *X, int batch, float eps, int s_max,
                            const kerdock_apply_params *p, const int32_t *out_idx, const float *out_val,
                            const int32_t *out_cnt) {
    if (!h) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL handle");
    if (!p) return fail(KERDOCK_ERR_INVALID_ARG, "params is NULL");
    if (batch < 0) return fail(KERDOCK_ERR_INVALID_ARG, "batch < 0");
    if (!(eps > 0.f) || !isfinite(eps)) return fail(KERDOCK_ERR_INVALID_ARG, "eps must be > 0");
    if (s_max < 1 || s_max > h->m) return fail(KERDOCK_ERR_INVALID_ARG, "s_max must lie in [1, m]");
    if (p->J < 1 || p->K < 1 || p->K > 32) return fail(KERDOCK_ERR_INVALID_ARG, "need J >= 1, 1 <= K <= 32");
    if ((int64_t)p->J * p->K > ((int64_t)1 << 31) - 64)
        return fail(KERDOCK_ERR_INVALID_ARG, "J K must stay below 2^31");
    if (p->chunk < 0 || p->chunk > gather_chunk_max())
        return fail(KERDOCK_ERR_INVALID_ARG, "chunk must lie in [0, 1024]");
    if ((p->dbg_samples == nullptr) != (p->dbg_coef == nullptr))
        return fail(KERDOCK_ERR_INVALID_ARG, "dbg_samples and dbg_coef must be given together");
    if ((int64_t)batch * s_max >= ((int64_t)1 << 31)) return fail(KERDOCK_ERR_INVALID_ARG, "batch s_max must stay below 2^31");
    if (batch == 0) return 1;
    if (!X || !out_idx || !out_val || !out_cnt)
        return fail(KERDOCK_ERR_INVALID_ARG, "NULL input or output pointer");
    return KERDOCK_OK;
}

// The streaming step with the workspace either the handle's own (ext_ws
// NULL: grown with hipMalloc when too small) or a caller-provided device
// buffer of ext_bytes (then nothing is allocated: sizes that do not fit are
// rejected, kernel_ms is not supported).
static int apply_ws(kerdock_handle h, const float *X, int batch, float eps, int s_max,
                    const kerdock_apply_params *p, int32_t *out_idx, float *out_val, int32_t *out_cnt,
                    const int32_t *active, void *stream, void *ext_ws, size_t ext_bytes) {
    {
        const int c = check_apply_args(h, X, batch, eps, s_max, p, out_idx, out_val, out_cnt);
        if (c != KERDOCK_OK) return c == 1 ? KERDOCK_OK : c;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int J = p->J, K = p->K, N = J * K;
    const int chunk = chunk_for(h, J, p->chunk);
    const int cpb = (J + chunk - 1) / chunk;

    const Workspace lay = workspace_layout(h, batch, J, K, s_max, chunk, p->dbg_samples != nullptr);
    char *ws;
    int rc = KERDOCK_OK;
    if (ext_ws) {
        if (lay.total > ext_bytes)
            return fail(KERDOCK_ERR_INVALID_ARG, "this call needs " + std::to_string(lay.total) +
                                                     " bytes of workspace, more than the " + std::to_string(ext_bytes) +
                                                     " bytes of the static scratch (use fewer vectors per call)");
        if (p->kernel_ms) return fail(KERDOCK_ERR_INVALID_ARG, "kernel_ms is not supported without allocation");
        ws = reinterpret_cast<char *>(ext_ws);
    } else {
        rc = ensure_workspace(h, lay.total);
        if (rc != KERDOCK_OK) return rc;
        ws = reinterpret_cast<char *>(h->ws);
    }
    float *partial = reinterpret_cast<float *>(ws + lay.partial);
    int32_t *surv = reinterpret_cast<int32_t *>(ws + lay.surv);
    int32_t *nsurv = reinterpret_cast<int32_t *>(ws + lay.nsurv);
    float *svals = reinterpret_cast<float *>(ws + lay.svals);
    int *row_ws = reinterpret_cast<int *>(ws + lay.rows);

    // kernel_ms slots: [0] grouping of the draws by basis (0 without it),
    // [1] draws, coefficients + gather, [2] select, [3] survivors
    const bool timed = p->kernel_ms != nullptr;
    if (timed && !h->ev[0])
        for (int q = 0; q < 5; ++q) KD_HIP(hipEventCreate(&h->ev[q]));
    if (timed) KD_HIP(hipEventRecord(h->ev[0], s));
    DGArgs dg{};
    dg.table = reinterpret_cast<const unsigned char *>(h->table);
    dg.col_bytes = h->pitch * (int)dtype_bytes(h->dtype);
    dg.X = X;
    dg.n = h->n;
    dg.k = h->k;
    dg.L = h->L;
    dg.signs = h->signs;
    dg.seed = p->seed;
    dg.t0_dev = nullptr;
    dg.t0 = p->t0;
    dg.N = N;
    dg.J = J;
    dg.chunk = chunk;
    dg.chunks_per_batch = cpb;
    bool grouped;
    {
        const GatherShape gs = gather_shape(h->dtype, h->pitch);
        dg.groups = gs.groups;
        dg.tpc = gs.tpc;
        grouped = gs.grouped != 0;
    }
    dg.pitch = h->pitch;
    dg.partial = partial;
    dg.bucket = use_bucket(h, J);
    if (dg.bucket) {
        dg.jlist = p->dbg_samples ? p->dbg_samples : reinterpret_cast<uint32_t *>(ws + lay.jlist);
        dg.sorted = reinterpret_cast<uint32_t *>(ws + lay.sorted);
        dg.perm = p->dbg_samples ? reinterpret_cast<int32_t *>(ws + lay.perm) : nullptr;
    } else {
        dg.dbg_samples = p->dbg_samples;
    }
    dg.dbg_coef = p->dbg_coef;
    dg.active = active;
    SelArgs sa{partial, h->m, h->pitch, K, cpb, J, h->scales, s_max, p->tau, p->dbg_mu, surv, nsurv, active};
    SurvArgs va{h->A, h->n, X, surv, nsurv, s_max, eps, out_idx, out_val, out_cnt, p->dbg_values, active, nullptr,
                svals, surv_vec4(X, h->n), h->m, row_ws};
    if (dg.bucket) rc = launch_draw_sort(dg, batch, K, s);
    if (timed && rc == KERDOCK_OK) KD_HIP(hipEventRecord(h->ev[1], s));
    if (rc == KERDOCK_OK) rc = launch_draw_gather(h->dtype, dg, batch, K, gather_unroll(h, grouped), s);
    if (timed && rc == KERDOCK_OK) KD_HIP(hipEventRecord(h->ev[2], s));
    if (rc == KERDOCK_OK) rc = launch_select(sa, batch, s);
    if (timed && rc == KERDOCK_OK) KD_HIP(hipEventRecord(h->ev[3], s));
    if (rc == KERDOCK_OK) rc = launch_survivors(va, batch, s);
    if (timed && rc == KERDOCK_OK) KD_HIP(hipEventRecord(h->ev[4], s));
    if (rc != KERDOCK_OK) return rc;
    if (timed) {
        KD_HIP(hipEventSynchronize(h->ev[4]));
        for (int q = 0; q < 4; ++q) KD_HIP(hipEventElapsedTime(&p->kernel_ms[q], h->ev[q], h->ev[q + 1]));
    }
    if (p->dbg_survivors)
        KD_HIP(hipMemcpyAsync(p->dbg_survivors, surv, (size_t)batch * s_max * 4, hipMemcpyDeviceToDevice, s));
    return KERDOCK_OK;
}

int apply_internal(kerdock_handle h, const float *X, int batch, float eps, int s_max,
                   const kerdock_apply_params *p, int32_t *out_idx, float *out_val, int32_t *out_cnt,
                   const int32_t *active, void *stream) {
    return apply_ws(h, X, batch, eps, s_max, p, out_idx, out_val, out_cnt, active, stream, nullptr, 0);
}

// ---------------------------------------------------- static scratch ----
// Device scratch of fixed size for kerdock_sparse_apply_static (callers that
// cannot allocate).  In host code `scratch` names a host-side stand-in, not
// a device address: its address on each device is looked up once, with that
// device current, and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[KERDOCK_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES];

static int static_scratch(int device, void **out) {
    if (device < 0 || device >= MAX_DEVICES) return fail(KERDOCK_ERR_INVALID_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return KERDOCK_OK;
}

}  // namespace kd

using namespace kd;

extern "C" {

int kerdock_autotune(kerdock_handle h, const float *X, int batch, int J, int K, void *stream,
                     int *best_chunk, int *best_unroll, float *best_ms) {
    if (!h) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL handle");
    if (!X || batch < 1 || J < 1 || K < 1 || K > 32) return fail(KERDOCK_ERR_INVALID_ARG, "autotune: bad arguments");
    if ((int64_t)J * K > ((int64_t)1 << 31) - 64) return fail(KERDOCK_ERR_INVALID_ARG, "J K must stay below 2^31");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const GatherShape gs = gather_shape(h->dtype, h->pitch);
    std::vector<int> unrolls;
    if (gs.grouped) unrolls = {4, 8, 16};
    else if (gs.tiles == 1) unrolls = {4, 8, 16};
    else if (gs.tiles == 2) unrolls = {4, 8};
    else unrolls = {2, 4};
    const int chunks[] = {256, 512, 1024};
    size_t need = 0;
    for (int c : chunks) {
        const size_t cc = std::min(c, J);
        need = std::max(need, (size_t)batch * K * ((J + cc - 1) / cc) * h->pitch * 4);
    }
    const size_t draws = align256((size_t)batch * J * K * 4);
    need = align256(need);
    int rc = ensure_workspace(h, need + 2 * draws);
    if (rc != KERDOCK_OK) return rc;
    uint32_t *jlist = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(h->ws) + need);
    uint32_t *sorted = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(h->ws) + need + draws);
    if (!h->ev[0])
        for (int q = 0; q < 5; ++q) KD_HIP(hipEventCreate(&h->ev[q]));
    float best = 1e30f;
    int bc = 512, bu = 8, bb = 0;
    // grouping by basis is worth timing only with runs of several draws
    const int nbk = (int64_t)J >= 2 * (int64_t)(h->d / 2 + 1) ? 2 : 1;
    for (int bk = 0; bk < nbk; ++bk)
    for (int c : chunks) {
        const int chunk = std::min(c, J);
        if (c > J && c != chunks[0]) continue;
        for (int u : unrolls) {
            DGArgs dg{};
            dg.table = reinterpret_cast<const unsigned char *>(h->table);
            dg.col_bytes = gs.col_bytes;
            dg.X = X;
            dg.n = h->n;
            dg.k = h->k;
            dg.L = h->L;
            dg.signs = h->signs;
            dg.seed = 12345;
            dg.t0 = 0;
            dg.N = J * K;
            dg.J = J;
            dg.chunk = chunk;
            dg.chunks_per_batch = (J + chunk - 1) / chunk;
            dg.groups = gs.groups;
            dg.tpc = gs.tpc;
            dg.pitch = h->pitch;
            dg.partial = reinterpret_cast<float *>(h->ws);
            dg.bucket = bk;
            dg.jlist = jlist;
            dg.sorted = sorted;
            float tmin = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                KD_HIP(hipEventRecord(h->ev[0], s));
                rc = bk ? launch_draw_sort(dg, batch, K, s) : KERDOCK_OK;
                if (rc == KERDOCK_OK) rc = launch_draw_gather(h->dtype, dg, batch, K, u, s);
                if (rc != KERDOCK_OK) return rc;
                KD_HIP(hipEventRecord(h->ev[1], s));
                KD_HIP(hipEventSynchronize(h->ev[1]));
                float ms = 0.f;
                KD_HIP(hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
                if (rep > 0) tmin = std::min(tmin, ms);     // first run warms up
            }
            if (tmin < best) {
                best = tmin;
                bc = chunk;
                bu = u;
                bb = bk;
            }
        }
    }
    h->tune_chunk = bc;
    h->tune_unroll = bu;
    h->tune_bucket = bb;
    cache_store(h, K);
    if (best_chunk) *best_chunk = bc;
    if (best_unroll) *best_unroll = bu;
    if (best_ms) *best_ms = best;
    return KERDOCK_OK;
}


const char *kerdock_last_error(void) { return g_error.c_str(); }

int kerdock_prepare(const float *A, int m, int n, kerdock_dtype dtype, void *stream,
                    kerdock_handle *out) {
    if (!out) return fail(KERDOCK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!A) return fail(KERDOCK_ERR_INVALID_ARG, "A is NULL");
    if (m < 1 || m > 16384) return fail(KERDOCK_ERR_INVALID_ARG, "m must lie in [1, 16384]");
    if (n < 1 || n > 4096)
        return fail(KERDOCK_ERR_UNSUPPORTED_N, "n must lie in [1, 4096] (n > 4096 needs d = 16384)");
    if (dtype != KERDOCK_F32 && dtype != KERDOCK_BF16 && dtype != KERDOCK_FP8E4M3)
        return fail(KERDOCK_ERR_INVALID_ARG, "unknown dtype");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    kerdock_handle_s *h = new kerdock_handle_s();
    h->m = m;
    h->n = n;
    h->k = 2;
    while ((1 << h->k) < n) h->k += 2;
    h->d = 1 << h->k;
    h->L = (int64_t)h->d * (h->d / 2 + 1);
    h->pitch = column_pitch(m);
    h->dtype = dtype;
    {
        hipError_t e0 = hipGetDevice(&h->device);
        if (e0 != hipSuccess) {
            delete h;
            return hip_fail(e0, "hipGetDevice");
        }
    }

    std::vector<uint16_t> masks = kerdock_masks(h->k, &h->poly);
    const size_t nb = (size_t)h->d / 2;
    const size_t wpb = h->d >= 32 ? (size_t)h->d / 32 : 1;
    h->table_bytes = (size_t)h->L * h->pitch * dtype_bytes(dtype);

    size_t free_b = 0, total_b = 0;
    {
        hipError_t e0 = hipMemGetInfo(&free_b, &total_b);
        if (e0 != hipSuccess) {
            delete h;
            return hip_fail(e0, "hipMemGetInfo");
        }
    }
    const size_t side = (size_t)m * n * 4 + nb * wpb * 4 + masks.size() * 2 + (size_t)h->pitch * 4;
    if (h->table_bytes + side + ((size_t)1 << 28) > free_b) {
        const std::string msg = "table of " + std::to_string(h->table_bytes) + " bytes does not fit in free device memory";
        delete h;
        return fail(KERDOCK_ERR_OOM, msg);
    }
#define KD_ALLOC(ptr, bytes)                                                      \
    do {                                                                          \
        hipError_t e_ = hipMalloc((void **)&(ptr), (bytes));                      \
        if (e_ != hipSuccess) {                                                   \
            free_handle(h);                                                       \
            return fail(KERDOCK_ERR_OOM, std::string("allocation failed: ") + #ptr); \
        }                                                                         \
    } while (0)
    KD_ALLOC(h->table, h->table_bytes);
    KD_ALLOC(h->scales, (size_t)h->pitch * 4);
    KD_ALLOC(h->A, (size_t)m * n * 4);
    KD_ALLOC(h->signs, nb * wpb * 4);
    KD_ALLOC(h->masks, masks.size() * 2);
#undef KD_ALLOC

    int rc = KERDOCK_OK;
    hipError_t e;
    if ((e = hipMemcpyAsync(h->A, A, (size_t)m * n * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(h->masks, masks.data(), masks.size() * 2, hipMemcpyHostToDevice, s)) !=
            hipSuccess) {
        rc = hip_fail(e, "prepare copies");
    }
    if (rc == KERDOCK_OK) rc = launch_signs(h->masks, h->k, h->signs, s);
    float *norm2 = nullptr;
    if (rc == KERDOCK_OK && (e = hipMalloc((void **)&norm2, (size_t)h->pitch * 4)) != hipSuccess)
        rc = fail(KERDOCK_ERR_OOM, "row norms");
    if (rc == KERDOCK_OK) rc = launch_row_scales(h->A, m, n, h->pitch, h->d, dtype, h->scales, norm2, s);
    // the construction kernels are timed with a pair of events (their
    // failure to be created only leaves build_ms at 0)
    hipEvent_t tb[2] = {nullptr, nullptr};
    const bool timed = hipEventCreate(&tb[0]) == hipSuccess && hipEventCreate(&tb[1]) == hipSuccess;
    if (rc == KERDOCK_OK && timed && (e = hipEventRecord(tb[0], s)) != hipSuccess) rc = hip_fail(e, "event");
    if (rc == KERDOCK_OK)
        rc = launch_table_build(dtype, h->k, h->A, m, n, h->pitch, h->signs, h->scales, h->table, s);
    if (rc == KERDOCK_OK && timed && (e = hipEventRecord(tb[1], s)) != hipSuccess) rc = hip_fail(e, "event");
    if (rc == KERDOCK_OK && (e = hipStreamSynchronize(s)) != hipSuccess) rc = hip_fail(e, "prepare");
    if (rc == KERDOCK_OK && timed) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, tb[0], tb[1]) == hipSuccess) h->build_ms = ms;
    }
    for (hipEvent_t ev : tb)
        if (ev) (void)hipEventDestroy(ev);
    if (rc == KERDOCK_OK) {
        std::vector<float> rn((size_t)m);
        if ((e = hipMemcpy(rn.data(), norm2, (size_t)m * 4, hipMemcpyDeviceToHost)) != hipSuccess)
            rc = hip_fail(e, "row norms");
        for (float v : rn) h->row_norm2_max = std::max(h->row_norm2_max, v);
    }
    (void)hipFree(norm2);
    if (rc != KERDOCK_OK) {
        free_handle(h);
        return rc;
    }
    cache_lookup(h);
    *out = h;
    return KERDOCK_OK;
}

int kerdock_reserve(kerdock_handle h, int batch, int J, int K, int s_max) {
    if (!h) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL handle");
    if (batch < 0 || J < 1 || K < 1 || K > 32 || s_max < 1 || s_max > h->m)
        return fail(KERDOCK_ERR_INVALID_ARG, "reserve: invalid sizes");
    if ((int64_t)J * K > ((int64_t)1 << 31) - 64) return fail(KERDOCK_ERR_INVALID_ARG, "J K must stay below 2^31");
    KD_HIP(hipSetDevice(h->device));
    return ensure_workspace(h, workspace_layout(h, batch, J, K, s_max, chunk_for(h, J, 0)).total);
}

int kerdock_sparse_apply(kerdock_handle h, const float *X, int batch, float eps, int s_max,
                         const kerdock_apply_params *p, int32_t *out_idx, float *out_val,
                         int32_t *out_cnt, void *stream) {
    return kd::apply_internal(h, X, batch, eps, s_max, p, out_idx, out_val, out_cnt, nullptr, stream);
}

int kerdock_sparse_apply_static(kerdock_handle h, const float *X, int batch, float eps, int s_max,
                                const kerdock_apply_params *p, int32_t *out_idx, float *out_val,
                                int32_t *out_cnt, void *stream) {
    if (!h) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL handle");
    void *ws = nullptr;
    const int rc = static_scratch(h->device, &ws);
    if (rc != KERDOCK_OK) return rc;
    return kd::apply_ws(h, X, batch, eps, s_max, p, out_idx, out_val, out_cnt, nullptr, stream, ws,
                        KERDOCK_STATIC_SCRATCH_BYTES);
}

int kerdock_sparse_apply_shared(kerdock_handle h, const float *X, int batch, float eps, int s_max,
                                const kerdock_apply_params *p, int32_t *out_idx, float *out_val,
                                int32_t *out_cnt, void *stream) {
    {
        const int c = check_apply_args(h, X, batch, eps, s_max, p, out_idx, out_val, out_cnt);
        if (c != KERDOCK_OK) return c == 1 ? KERDOCK_OK : c;
    }
    const int J = p->J, K = p->K, N = J * K;
    if (N > (1 << 26)) return fail(KERDOCK_ERR_INVALID_ARG, "shared form: J K must stay below 2^26");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t groups = ((size_t)batch + KERDOCK_SHARED_TILE - 1) / KERDOCK_SHARED_TILE;
    size_t off = 0;
    const int splits = shared_splits(J);
    const size_t o_partial = off; off += align256((size_t)batch * K * splits * h->pitch * 4);
    const size_t o_coef = off;    off += align256(shared_coef_floats(h->dtype, batch, J, K) * 4);
    const size_t o_ell = off;     off += align256(groups * N * 4);
    const size_t o_surv = off;    off += align256((size_t)batch * s_max * 4);
    const size_t o_nsurv = off;   off += align256((size_t)batch * 4);
    const size_t o_svals = off;   off += align256((size_t)batch * s_max * 4);
    const size_t o_digits = off;  off += align256(shared_digit_bytes(batch, h->n));
    const size_t o_xscale = off;  off += align256((size_t)batch * 8);
    const size_t o_rows = off;    off += align256(survivor_rows_bytes(batch, h->m, s_max));
    int rc = ensure_workspace(h, off);
    if (rc != KERDOCK_OK) return rc;
    char *ws = reinterpret_cast<char *>(h->ws);
    float *partial = reinterpret_cast<float *>(ws + o_partial);
    float *coef = reinterpret_cast<float *>(ws + o_coef);
    uint32_t *ell = reinterpret_cast<uint32_t *>(ws + o_ell);
    int32_t *surv = reinterpret_cast<int32_t *>(ws + o_surv);
    int32_t *nsurv = reinterpret_cast<int32_t *>(ws + o_nsurv);
    float *svals = reinterpret_cast<float *>(ws + o_svals);
    int8_t *digits = reinterpret_cast<int8_t *>(ws + o_digits);
    int2 *xscale = reinterpret_cast<int2 *>(ws + o_xscale);
    int *row_ws = reinterpret_cast<int *>(ws + o_rows);

    // kernel_ms: [0] draws + coefficients, [1] matrix product, [2] select,
    // [3] survivors
    const bool timed = p->kernel_ms != nullptr;
    if (timed && !h->ev[0])
        for (int q = 0; q < 5; ++q) KD_HIP(hipEventCreate(&h->ev[q]));
    if (timed) KD_HIP(hipEventRecord(h->ev[0], s));
    rc = launch_shared_coef(h->dtype, X, batch, h->n, h->k, h->L, h->signs, p->seed, p->t0, J, K, digits, xscale, ell,
                            coef, p->dbg_samples, p->dbg_coef, s);
    if (timed && rc == KERDOCK_OK) KD_HIP(hipEventRecord(h->ev[1], s));
    if (rc == KERDOCK_OK) rc = launch_shared_gemm(h->dtype, h->table, h->pitch, batch, J, K, ell, coef, partial, s);
    if (timed && rc == KERDOCK_OK) KD_HIP(hipEventRecord(h->ev[2], s));
    SelArgs sa{partial, h->m, h->pitch, K, splits, J, h->scales, s_max, p->tau, p->dbg_mu, surv, nsurv, nullptr};
    if (rc == KERDOCK_OK) rc = launch_select(sa, batch, s);
    if (timed && rc == KERDOCK_OK) KD_HIP(hipEventRecord(h->ev[3], s));
    SurvArgs va{h->A, h->n, X, surv, nsurv, s_max, eps, out_idx, out_val, out_cnt, p->dbg_values, nullptr, nullptr,
                svals, surv_vec4(X, h->n), h->m, row_ws};
    if (rc == KERDOCK_OK) rc = launch_survivors(va, batch, s);
    if (timed && rc == KERDOCK_OK) KD_HIP(hipEventRecord(h->ev[4], s));
    if (rc != KERDOCK_OK) return rc;
    if (timed) {
        KD_HIP(hipEventSynchronize(h->ev[4]));
        for (int q = 0; q < 4; ++q) KD_HIP(hipEventElapsedTime(&p->kernel_ms[q], h->ev[q], h->ev[q + 1]));
    }
    if (p->dbg_survivors)
        KD_HIP(hipMemcpyAsync(p->dbg_survivors, surv, (size_t)batch * s_max * 4, hipMemcpyDeviceToDevice, s));
    return KERDOCK_OK;
}

int kerdock_theory_params(kerdock_handle h, float eps, float delta, float eta, int32_t *J, int32_t *K,
                          float *tau, float *norm2inf) {
    if (!h) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL handle");
    if (!(eps > delta) || !(delta >= 0.f) || !(eta > 0.f) || !(eta < 1.f) || !J || !K)
        return fail(KERDOCK_ERR_INVALID_ARG, "need eps > delta >= 0, 0 < eta < 1 and outputs");
    const double gamma = 0.5 * ((double)eps - (double)delta);
    const double e = 2.718281828459045;
    const double Jd = ceil(4.0 * e * e * (double)h->row_norm2_max / (gamma * gamma));
    const double Kd = ceil(2.0 * log((double)h->m / (double)eta));
    if (Jd > 2147483647.0 || Kd > 32.0 || Jd * Kd > 2147483583.0)
        return fail(KERDOCK_ERR_INVALID_ARG, "Theorem 5's J or K exceeds the supported range (J K < 2^31, K <= 32)");
    *J = (int32_t)(Jd < 1 ? 1 : Jd);
    *K = (int32_t)(Kd < 1 ? 1 : Kd);
    if (tau) *tau = 0.5f * (eps + delta);
    if (norm2inf) *norm2inf = h->row_norm2_max;
    return KERDOCK_OK;
}

int kerdock_query(kerdock_handle h, kerdock_info *info) {
    if (!h) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL handle");
    if (!info) return fail(KERDOCK_ERR_INVALID_ARG, "info is NULL");
    info->m = h->m;
    info->n = h->n;
    info->k = h->k;
    info->d = h->d;
    info->L = h->L;
    info->pitch = h->pitch;
    info->field_poly = h->poly;
    info->dtype = h->dtype;
    info->table_bytes = h->table_bytes;
    info->build_ms = h->build_ms;
    return KERDOCK_OK;
}

int kerdock_read_columns(kerdock_handle h, const uint32_t *ells, int count, float *out, void *stream) {
    if (!h) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL handle");
    if (count < 0 || (count > 0 && (!ells || !out))) return fail(KERDOCK_ERR_INVALID_ARG, "bad arguments");
    return launch_read_columns(h->dtype, h->table, h->m, h->pitch, h->L, h->scales, ells, count, out,
                               reinterpret_cast<hipStream_t>(stream));
}

int kerdock_debug_signs(kerdock_handle h, int b, uint32_t *out_bits) {
    if (!h) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL handle");
    if (b < 0 || b >= h->d / 2 || !out_bits) return fail(KERDOCK_ERR_INVALID_ARG, "bad basis or pointer");
    const size_t wpb = h->d >= 32 ? (size_t)h->d / 32 : 1;
    KD_HIP(hipMemcpy(out_bits, h->signs + (size_t)b * wpb, wpb * 4, hipMemcpyDeviceToHost));
    return KERDOCK_OK;
}

int kerdock_row_scales(kerdock_handle h, float *out, void *stream) {
    if (!h) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL handle");
    if (!out) return fail(KERDOCK_ERR_INVALID_ARG, "out is NULL");
    KD_HIP(hipMemcpyAsync(out, h->scales, (size_t)h->m * 4, hipMemcpyDeviceToDevice,
                          reinterpret_cast<hipStream_t>(stream)));
    return KERDOCK_OK;
}

int kerdock_destroy(kerdock_handle h) {
    if (!h) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL handle");
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    free_handle(h);
    return KERDOCK_OK;
}

}  // extern "C"
