// Shared definitions of the gfx950 Kerdock library: table element codecs,
// launch-error plumbing and the handle layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/kerdock.h"

namespace kd {

// ---------------------------------------------------------------- errors --

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define KD_HIP(call)                                                        \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) return ::kd::hip_fail(e_, #call);             \
    } while (0)

#define KD_LAUNCH(what)                                                     \
    do {                                                                    \
        hipError_t e_ = hipGetLastError();                                  \
        if (e_ != hipSuccess) return ::kd::hip_fail(e_, what);              \
    } while (0)

// ------------------------------------------------------------ geometry --

// Table columns are stored with a pitch rounded up to 64 elements so that
// every column starts on a 64-byte boundary for every element type.
inline int column_pitch(int m) { return (m + 63) & ~63; }

inline size_t dtype_bytes(kerdock_dtype t) {
    return t == KERDOCK_F32 ? 4 : (t == KERDOCK_BF16 ? 2 : 1);
}

// -------------------------------------------------------- element codecs --

// bfloat16: the upper half of an FP32 word, rounded to nearest even.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint32_t h16) {
    return __uint_as_float(h16 << 16);
}

// E4M3 byte -> FP32.  Normal codes: move exponent and mantissa into an FP32
// word and add 120 to the exponent (bias 127 - 7).  Subnormal codes (exponent
// field 0): mantissa * 2^-9.  No FP32 denormal is ever formed.
__device__ __forceinline__ float e4m3_to_f32(uint32_t byte) {
    uint32_t em = byte & 0x7Fu;
    float normal = __uint_as_float((em << 20) + (120u << 23));
    float sub = (float)em * 0.001953125f;                       // 2^-9
    float mag = (em >= 8u) ? normal : sub;
    return (byte & 0x80u) ? -mag : mag;
}

// geometry of the gather for one table: bytes per column, 4 KiB tiles per
// workgroup, segments per column, and the draw groups of short columns
struct GatherShape {
    int col_bytes, tiles, segs, groups, tpc, grouped;
    int small;    // launch below GATHER_MIN_WGS workgroups: single tiles
};
// work: chunks of draws in the launch (vectors x batches x chunks); below
// GATHER_MIN_WGS workgroups the columns are split into single tiles
constexpr long long GATHER_MIN_WGS = 2048;
GatherShape gather_shape(kerdock_dtype dt, int pitch, long long work = 1ll << 40);
// draws per FP32 partial sum for a call with J draws per batch
int chunk_for(const kerdock_handle_s *h, int J, int requested);
// whether a call with J draws per batch groups its draws by basis
int use_bucket(const kerdock_handle_s *h, int J);

}  // namespace kd

// --------------------------------------------------------------- handle --

struct kerdock_learned_s;
namespace kd {
void free_learned(kerdock_learned_s *L);
}

struct kerdock_handle_s {
    int m = 0, n = 0, k = 0, d = 0, pitch = 0;
    int64_t L = 0;
    uint32_t poly = 0;
    kerdock_dtype dtype = KERDOCK_F32;
    int device = 0;
    void *table = nullptr;        // [L][pitch] elements of dtype
    size_t table_bytes = 0;
    float *scales = nullptr;      // [pitch] row scales (1 unless FP8)
    float *A = nullptr;           // [m][n] copy of A
    uint32_t *signs = nullptr;    // [d/2][d/32] sign bitmaps of the Kerdock bases
    uint16_t *masks = nullptr;    // [d/2][k] strict-upper-triangle row masks
    void *ws = nullptr;           // growable workspace of the streaming step
    size_t ws_bytes = 0;
    hipEvent_t ev[5] = {};        // kernel timing events (created on first use)
    int tune_chunk = 0;           // draws per gather workgroup (0: default)
    int tune_unroll = 0;          // draws in flight per thread (0: default)
    int tune_bucket = -1;         // group draws by basis: 1 / 0, -1: the default rule
    kerdock_learned_s *learned = nullptr;   // attached learned-proposal state
    float row_norm2_max = 0.f;    // |A|_{2->inf}^2: largest squared row norm
    float build_ms = 0.f;         // device time of the table construction kernels
};
