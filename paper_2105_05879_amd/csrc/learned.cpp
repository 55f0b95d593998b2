// Learned-proposal form (host side): the MLP object, its training step, and
// the learned apply with exact verification and fallback to the plain
// randomized estimator.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <string>
#include <vector>

#include "apply_device.hpp"

namespace kd {

int gemm_bf16(bool ak, bool bk, const uint16_t *A, int lda, const uint16_t *B, int ldb, int M, int N, int K,
              int epi, const float *bias, const uint16_t *mask, int ldm, float *C32, uint16_t *C16, int ldc,
              hipStream_t s);
int launch_to_bf16(const float *x, uint16_t *y, size_t n, hipStream_t s);
int launch_colsum(const float *dz, int B, int N, float *db, hipStream_t s);
int launch_bce(const float *z, const uint8_t *y, size_t n, float pos_w, float *dz, uint16_t *dz16,
               float *terms, float *loss, hipStream_t s);
int launch_adam(float *w, const float *g, float *m, float *v, uint16_t *w16, size_t n, float lr, float b1,
                float b2, float eps, int step, hipStream_t s);
int launch_features(int k, const float *X, int B, int n, float *F, uint16_t *F16, hipStream_t s);
int launch_topc_logits(const float *Z, int B, int m, int c, int32_t *cand, int32_t *ncand, hipStream_t s);
int launch_gram2(const float *A, int m, int n, float *Ghi, float *Glo, float *fro2, hipStream_t s);
int launch_energy_flags(const float *X, int B, int n, int m, int c, const float *Ghi, const float *Glo,
                        const float *fro2, const float *vsum2, float eps, float *Zp, float *Ze, int32_t *flags,
                        float *dbg_energy, hipStream_t s);
int launch_survivors(const SurvArgs &a, int batch, hipStream_t s);
int apply_internal(kerdock_handle h, const float *X, int batch, float eps, int s_max,
                   const kerdock_apply_params *p, int32_t *out_idx, float *out_val, int32_t *out_cnt,
                   const int32_t *active, void *stream);

enum { EPI_NONE = 0, EPI_BIAS = 1, EPI_RELU = 2, EPI_MASK = 4 };

}  // namespace kd

// parameters, FP32 masters: W1 [d1][d0], b1 [d1], W2 [d2][d1], b2 [d2], W3 [d3][d2], b3 [d3]
struct kerdock_mlp_s {
    int d0 = 0, d1 = 0, d2 = 0, d3 = 0;
    int device = 0;
    size_t off[6] = {}, count = 0;
    float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;   // masters, grads, Adam moments
    uint16_t *P16 = nullptr;                                        // BF16 copy (same layout)
    int step = 0;
    int cap = 0;                                                    // rows the activations hold
    uint16_t *F16 = nullptr, *H1 = nullptr, *H2 = nullptr, *dZ16 = nullptr, *dH2_16 = nullptr, *dH1_16 = nullptr;
    float *Z = nullptr, *dZ = nullptr, *dH2 = nullptr, *dH1 = nullptr, *terms = nullptr;
    void *act = nullptr;
};

// the learned state attached to a handle
struct kerdock_learned_s {
    kerdock_mlp net = nullptr;
    float *Gram = nullptr;            // [2][n][n]: A^T A = Ghi + Glo (compensated), then |A|_F^2
    void *ws = nullptr;
    size_t ws_bytes = 0;
};

namespace kd {

static size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

static void free_act(kerdock_mlp_s *net) {
    (void)hipFree(net->act);
    net->act = nullptr;
    net->cap = 0;
}

// grow the activation buffers to hold B rows
static int ensure_act(kerdock_mlp_s *net, int B) {
    if (B <= net->cap) return KERDOCK_OK;
    (void)hipDeviceSynchronize();
    free_act(net);
    const size_t b = (size_t)B;
    size_t off = 0;
    const size_t oF16 = off; off += al(b * net->d0 * 2);
    const size_t oH1 = off; off += al(b * net->d1 * 2);
    const size_t oH2 = off; off += al(b * net->d2 * 2);
    const size_t odZ16 = off; off += al(b * net->d3 * 2);
    const size_t odH2_16 = off; off += al(b * net->d2 * 2);
    const size_t odH1_16 = off; off += al(b * net->d1 * 2);
    const size_t oZ = off; off += al(b * net->d3 * 4);
    const size_t odZ = off; off += al(b * net->d3 * 4);
    const size_t odH2 = off; off += al(b * net->d2 * 4);
    const size_t odH1 = off; off += al(b * net->d1 * 4);
    const size_t oT = off; off += al(b * net->d3 * 4);
    if (hipMalloc(&net->act, off) != hipSuccess) {
        net->act = nullptr;
        return fail(KERDOCK_ERR_OOM, "mlp activations");
    }
    char *p = reinterpret_cast<char *>(net->act);
    net->F16 = reinterpret_cast<uint16_t *>(p + oF16);
    net->H1 = reinterpret_cast<uint16_t *>(p + oH1);
    net->H2 = reinterpret_cast<uint16_t *>(p + oH2);
    net->dZ16 = reinterpret_cast<uint16_t *>(p + odZ16);
    net->dH2_16 = reinterpret_cast<uint16_t *>(p + odH2_16);
    net->dH1_16 = reinterpret_cast<uint16_t *>(p + odH1_16);
    net->Z = reinterpret_cast<float *>(p + oZ);
    net->dZ = reinterpret_cast<float *>(p + odZ);
    net->dH2 = reinterpret_cast<float *>(p + odH2);
    net->dH1 = reinterpret_cast<float *>(p + odH1);
    net->terms = reinterpret_cast<float *>(p + oT);
    net->cap = B;
    return KERDOCK_OK;
}

// logits Z (FP32, net->Z or Zout) from BF16 inputs already in net->F16
static int mlp_forward16(kerdock_mlp_s *n, int B, float *Zout, hipStream_t s) {
    const uint16_t *W1 = n->P16 + n->off[0], *W2 = n->P16 + n->off[2], *W3 = n->P16 + n->off[4];
    const float *b1 = n->P + n->off[1], *b2 = n->P + n->off[3], *b3 = n->P + n->off[5];
    int rc = gemm_bf16(false, false, n->F16, n->d0, W1, n->d0, B, n->d1, n->d0, EPI_BIAS | EPI_RELU, b1, nullptr, 0,
                       nullptr, n->H1, n->d1, s);
    if (rc == KERDOCK_OK)
        rc = gemm_bf16(false, false, n->H1, n->d1, W2, n->d1, B, n->d2, n->d1, EPI_BIAS | EPI_RELU, b2, nullptr, 0,
                       nullptr, n->H2, n->d2, s);
    if (rc == KERDOCK_OK)
        rc = gemm_bf16(false, false, n->H2, n->d2, W3, n->d2, B, n->d3, n->d2, EPI_BIAS, b3, nullptr, 0,
                       Zout ? Zout : n->Z, nullptr, n->d3, s);
    return rc;
}

// 64-bit splitmix (Steele, Lea, Flood 2014) for the initial weights
static uint64_t splitmix(uint64_t &x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void free_mlp(kerdock_mlp_s *n) {
    if (!n) return;
    (void)hipFree(n->P);
    (void)hipFree(n->G);
    (void)hipFree(n->M);
    (void)hipFree(n->V);
    (void)hipFree(n->P16);
    free_act(n);
    delete n;
}

static int upload_params(kerdock_mlp_s *n, const float *host) {
    hipError_t e;
    if ((e = hipMemcpy(n->P, host, n->count * 4, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "mlp params");
    if ((e = hipMemset(n->M, 0, n->count * 4)) != hipSuccess) return hip_fail(e, "mlp adam");
    if ((e = hipMemset(n->V, 0, n->count * 4)) != hipSuccess) return hip_fail(e, "mlp adam");
    n->step = 0;
    int rc = launch_to_bf16(n->P, n->P16, n->count, nullptr);
    if (rc != KERDOCK_OK) return rc;
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "mlp params");
    return KERDOCK_OK;
}

}  // namespace kd

using namespace kd;

extern "C" {

int kerdock_mlp_create(int d_in, int h1, int h2, int d_out, uint64_t seed, kerdock_mlp *out) {
    if (!out) return fail(KERDOCK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (d_in < 1 || h1 < 1 || h2 < 1 || d_out < 1 || d_in > 16384 || h1 > 16384 || h2 > 16384 || d_out > 16384)
        return fail(KERDOCK_ERR_INVALID_ARG, "mlp sizes must lie in [1, 16384]");
    kerdock_mlp_s *n = new kerdock_mlp_s();
    n->d0 = d_in;
    n->d1 = h1;
    n->d2 = h2;
    n->d3 = d_out;
    const size_t sz[6] = {(size_t)h1 * d_in, (size_t)h1, (size_t)h2 * h1, (size_t)h2, (size_t)d_out * h2, (size_t)d_out};
    size_t c = 0;
    for (int q = 0; q < 6; ++q) {
        n->off[q] = c;
        c += sz[q];
    }
    n->count = c;
    if (hipGetDevice(&n->device) != hipSuccess) { delete n; return fail(KERDOCK_ERR_HIP, "hipGetDevice"); }
    if (hipMalloc((void **)&n->P, c * 4) != hipSuccess || hipMalloc((void **)&n->G, c * 4) != hipSuccess ||
        hipMalloc((void **)&n->M, c * 4) != hipSuccess || hipMalloc((void **)&n->V, c * 4) != hipSuccess ||
        hipMalloc((void **)&n->P16, c * 2) != hipSuccess) {
        free_mlp(n);
        return fail(KERDOCK_ERR_OOM, "mlp parameters");
    }
    // He initialisation: weights uniform in +-sqrt(6 / fan_in), biases 0
    std::vector<float> host(c, 0.f);
    uint64_t st = seed;
    const int fan[3] = {d_in, h1, h2};
    for (int layer = 0; layer < 3; ++layer) {
        const float a = sqrtf(6.0f / (float)fan[layer]);
        for (size_t i = 0; i < sz[2 * layer]; ++i) {
            const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
            host[n->off[2 * layer] + i] = (float)((2.0 * u - 1.0) * a);
        }
    }
    const int rc = upload_params(n, host.data());
    if (rc != KERDOCK_OK) { free_mlp(n); return rc; }
    *out = n;
    return KERDOCK_OK;
}

int kerdock_mlp_param_count(kerdock_mlp net, size_t *count) {
    if (!net) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL mlp");
    if (!count) return fail(KERDOCK_ERR_INVALID_ARG, "count is NULL");
    *count = net->count;
    return KERDOCK_OK;
}

int kerdock_mlp_get_params(kerdock_mlp net, float *host) {
    if (!net) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL mlp");
    if (!host) return fail(KERDOCK_ERR_INVALID_ARG, "host is NULL");
    KD_HIP(hipDeviceSynchronize());
    KD_HIP(hipMemcpy(host, net->P, net->count * 4, hipMemcpyDeviceToHost));
    return KERDOCK_OK;
}

int kerdock_mlp_set_params(kerdock_mlp net, const float *host) {
    if (!net) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL mlp");
    if (!host) return fail(KERDOCK_ERR_INVALID_ARG, "host is NULL");
    KD_HIP(hipDeviceSynchronize());
    return upload_params(net, host);
}

int kerdock_mlp_forward(kerdock_mlp net, const float *F, int B, float *Z, void *stream) {
    if (!net) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL mlp");
    if (B < 0 || (B > 0 && (!F || !Z))) return fail(KERDOCK_ERR_INVALID_ARG, "bad arguments");
    if (B == 0) return KERDOCK_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int rc = ensure_act(net, B);
    if (rc == KERDOCK_OK) rc = launch_to_bf16(F, net->F16, (size_t)B * net->d0, s);
    if (rc == KERDOCK_OK) rc = mlp_forward16(net, B, Z, s);
    return rc;
}

int kerdock_mlp_train_step(kerdock_mlp net, const float *F, const uint8_t *Y, int B, float lr, float pos_weight,
                           float *loss, float *grads, void *stream) {
    if (!net) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL mlp");
    if (B < 1 || !F || !Y || !loss || !(lr >= 0.f) || !(pos_weight > 0.f))
        return fail(KERDOCK_ERR_INVALID_ARG, "train step: bad arguments");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    kerdock_mlp_s *n = net;
    int rc = ensure_act(n, B);
    if (rc != KERDOCK_OK) return rc;
    const uint16_t *W2 = n->P16 + n->off[2], *W3 = n->P16 + n->off[4];
    float *G = n->G;
    rc = launch_to_bf16(F, n->F16, (size_t)B * n->d0, s);
    if (rc == KERDOCK_OK) rc = mlp_forward16(n, B, nullptr, s);
    if (rc == KERDOCK_OK) rc = launch_bce(n->Z, Y, (size_t)B * n->d3, pos_weight, n->dZ, n->dZ16, n->terms, loss, s);
    // layer 3: dW3 = dZ^T H2, db3 = colsum dZ, dH2 = (dZ W3) masked by H2 > 0
    if (rc == KERDOCK_OK)
        rc = gemm_bf16(true, true, n->dZ16, n->d3, n->H2, n->d2, n->d3, n->d2, B, EPI_NONE, nullptr, nullptr, 0,
                       G + n->off[4], nullptr, n->d2, s);
    if (rc == KERDOCK_OK) rc = launch_colsum(n->dZ, B, n->d3, G + n->off[5], s);
    if (rc == KERDOCK_OK)
        rc = gemm_bf16(false, true, n->dZ16, n->d3, W3, n->d2, B, n->d2, n->d3, EPI_MASK, nullptr, n->H2, n->d2,
                       n->dH2, n->dH2_16, n->d2, s);
    // layer 2
    if (rc == KERDOCK_OK)
        rc = gemm_bf16(true, true, n->dH2_16, n->d2, n->H1, n->d1, n->d2, n->d1, B, EPI_NONE, nullptr, nullptr, 0,
                       G + n->off[2], nullptr, n->d1, s);
    if (rc == KERDOCK_OK) rc = launch_colsum(n->dH2, B, n->d2, G + n->off[3], s);
    if (rc == KERDOCK_OK)
        rc = gemm_bf16(false, true, n->dH2_16, n->d2, W2, n->d1, B, n->d1, n->d2, EPI_MASK, nullptr, n->H1, n->d1,
                       n->dH1, n->dH1_16, n->d1, s);
    // layer 1
    if (rc == KERDOCK_OK)
        rc = gemm_bf16(true, true, n->dH1_16, n->d1, n->F16, n->d0, n->d1, n->d0, B, EPI_NONE, nullptr, nullptr, 0,
                       G + n->off[0], nullptr, n->d0, s);
    if (rc == KERDOCK_OK) rc = launch_colsum(n->dH1, B, n->d1, G + n->off[1], s);
    if (rc != KERDOCK_OK) return rc;
    if (grads) KD_HIP(hipMemcpyAsync(grads, G, n->count * 4, hipMemcpyDeviceToDevice, s));
    if (lr > 0.f) {
        n->step += 1;
        rc = launch_adam(n->P, G, n->M, n->V, n->P16, n->count, lr, 0.9f, 0.999f, 1e-8f, n->step, s);
    }
    return rc;
}

int kerdock_mlp_destroy(kerdock_mlp net) {
    if (!net) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL mlp");
    (void)hipSetDevice(net->device);
    (void)hipDeviceSynchronize();
    free_mlp(net);
    return KERDOCK_OK;
}

int kerdock_features(kerdock_handle h, const float *X, int B, float *F, void *stream) {
    if (!h) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL handle");
    if (B < 0 || (B > 0 && (!X || !F))) return fail(KERDOCK_ERR_INVALID_ARG, "bad arguments");
    if (B == 0) return KERDOCK_OK;
    return launch_features(h->k, X, B, h->n, F, nullptr, reinterpret_cast<hipStream_t>(stream));
}

int kerdock_learned_attach(kerdock_handle h, kerdock_mlp net) {
    if (!h || !net) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL handle or mlp");
    if (net->d0 != h->d || net->d3 != h->m)
        return fail(KERDOCK_ERR_INVALID_ARG, "mlp input must be d = " + std::to_string(h->d) +
                                                 " and output m = " + std::to_string(h->m));
    kerdock_learned_s *L = h->learned;
    if (!L) {
        L = new kerdock_learned_s();
        const size_t nn = (size_t)h->n * h->n;
        if (hipMalloc((void **)&L->Gram, (2 * nn + 64) * 4) != hipSuccess) {
            delete L;
            return fail(KERDOCK_ERR_OOM, "Gram matrix");
        }
        // G = A^T A as a compensated pair, and |A|_F^2
        int rc = launch_gram2(h->A, h->m, h->n, L->Gram, L->Gram + nn, L->Gram + 2 * nn, nullptr);
        hipError_t e = hipDeviceSynchronize();
        if (rc != KERDOCK_OK || e != hipSuccess) {
            (void)hipFree(L->Gram);
            delete L;
            return rc != KERDOCK_OK ? rc : hip_fail(e, "Gram matrix");
        }
        h->learned = L;
    }
    L->net = net;
    return KERDOCK_OK;
}

int kerdock_learned_apply(kerdock_handle h, const float *X, int B, float eps, int s_max,
                          const kerdock_apply_params *p, int32_t *out_idx, float *out_val, int32_t *out_cnt,
                          int32_t *fallback, void *stream) {
    if (!h) return fail(KERDOCK_ERR_NOT_PREPARED, "NULL handle");
    kerdock_learned_s *L = h->learned;
    if (!L || !L->net) return fail(KERDOCK_ERR_NOT_PREPARED, "no network attached (kerdock_learned_attach)");
    if (!p) return fail(KERDOCK_ERR_INVALID_ARG, "params is NULL");
    if (B < 0 || !(eps > 0.f) || !(eps < INFINITY) || s_max < 1 || s_max > h->m)
        return fail(KERDOCK_ERR_INVALID_ARG, "bad batch, eps or s_max");
    if ((int64_t)B * s_max >= ((int64_t)1 << 31)) return fail(KERDOCK_ERR_INVALID_ARG, "batch s_max must stay below 2^31");
    if (B == 0) return KERDOCK_OK;
    if (!X || !out_idx || !out_val || !out_cnt || !fallback) return fail(KERDOCK_ERR_INVALID_ARG, "NULL pointer");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    kerdock_mlp_s *n = L->net;
    int rc = ensure_act(n, B);
    if (rc != KERDOCK_OK) return rc;
    // workspace: candidates, counts, verified energies, G x as pairs
    const size_t oc = 0, onc = al((size_t)B * s_max * 4), ov = onc + al((size_t)B * 4), oz = ov + al((size_t)B * 4),
                 total = oz + 2 * al((size_t)B * h->n * 4);
    if (total > L->ws_bytes) {
        (void)hipDeviceSynchronize();
        (void)hipFree(L->ws);
        L->ws = nullptr;
        L->ws_bytes = 0;
        if (hipMalloc(&L->ws, total) != hipSuccess) return fail(KERDOCK_ERR_OOM, "learned workspace");
        L->ws_bytes = total;
    }
    char *w = reinterpret_cast<char *>(L->ws);
    int32_t *cand = reinterpret_cast<int32_t *>(w + oc);
    int32_t *ncand = reinterpret_cast<int32_t *>(w + onc);
    float *vs2 = reinterpret_cast<float *>(w + ov);
    float *Zp = reinterpret_cast<float *>(w + oz);
    float *Ze = reinterpret_cast<float *>(w + oz + al((size_t)B * h->n * 4));

    // L1 features, L2 MLP, L3 top-s_max logits, L4 exact dots + threshold
    rc = launch_features(h->k, X, B, h->n, nullptr, n->F16, s);
    if (rc == KERDOCK_OK) rc = mlp_forward16(n, B, nullptr, s);
    if (rc == KERDOCK_OK) rc = launch_topc_logits(n->Z, B, h->m, s_max, cand, ncand, s);
    SurvArgs va{h->A, h->n, X, cand, ncand, s_max, eps, out_idx, out_val, out_cnt, nullptr, nullptr, vs2,
                nullptr, surv_vec4(X, h->n)};
    if (rc == KERDOCK_OK) rc = launch_survivors(va, B, s);
    // L5 certified energy check: |Ax|^2 = x^T G x against the verified energy
    const size_t nn = (size_t)h->n * h->n;
    float *dbg_energy = (p->dbg_mu && h->m >= 3) ? p->dbg_mu : nullptr;
    if (rc == KERDOCK_OK)
        rc = launch_energy_flags(X, B, h->n, h->m, s_max, L->Gram, L->Gram + nn, L->Gram + 2 * nn, vs2, eps, Zp, Ze,
                                 fallback, dbg_energy, s);
    // debug: the candidate set C of every row (ascending, padded with -1)
    if (rc == KERDOCK_OK && p->dbg_survivors) {
        hipError_t e = hipMemcpyAsync(p->dbg_survivors, cand, (size_t)B * s_max * 4, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) rc = hip_fail(e, "candidate dump");
    }
    // fallback: the plain streaming step on the flagged rows only (its own
    // debug dumps are not requested)
    kerdock_apply_params pf = *p;
    pf.dbg_samples = nullptr;
    pf.dbg_coef = nullptr;
    pf.dbg_mu = nullptr;
    pf.dbg_survivors = nullptr;
    pf.dbg_values = nullptr;
    pf.kernel_ms = nullptr;
    if (rc == KERDOCK_OK) rc = apply_internal(h, X, B, eps, s_max, &pf, out_idx, out_val, out_cnt, fallback, stream);
    return rc;
}

}  // extern "C"

namespace kd {
void free_learned(kerdock_learned_s *L) {
    if (!L) return;
    (void)hipFree(L->Gram);
    (void)hipFree(L->ws);
    delete L;
}
}  // namespace kd
