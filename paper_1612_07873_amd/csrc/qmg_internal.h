// Internal helpers of the qmg library: error reporting, HIP checks, complex
// arithmetic on interleaved pairs.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../../include/qmg.h"

namespace qmg {

qmg_status fail(qmg_status st, const char* fmt, ...);
void clear_error();
const char* last_error();

#define QMG_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::qmg::fail(e_ == hipErrorOutOfMemory ? QMG_ERR_NOMEM : QMG_ERR_HIP, \
                               "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),   \
                               __FILE__, __LINE__);                                     \
    } while (0)

#define QMG_TRY(...)                       \
    do {                                   \
        qmg_status s_ = (__VA_ARGS__);     \
        if (s_ != QMG_OK) return s_;       \
    } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Most right-hand sides one call of the field entry points takes (grid dimension y).
constexpr int kMaxFieldBatch = 1024;

inline int64_t volume(const int d[4]) { return (int64_t)d[0] * d[1] * d[2] * d[3]; }

qmg_status check_dims(const int dims[4], int min_extent, const char* what);

// Neighbour table [V][8] (d = 2mu forward, 2mu+1 backward, periodic) on the device.
qmg_status make_neighbour_table(const int dims[4], int** dev_out, hipStream_t s);

// Red-black numbering [2][V/2]: lattice index of each half-lattice site of
// parity 0, then parity 1 (QMG_ERR_SHAPE unless every extent is even).
qmg_status make_half_site_table(const int dims[4], int** dev_out, hipStream_t s);

// Non-finite inputs of the 16-bit encoders: a per-device word that an encoder
// kernel sets (vector atomic OR) when it meets a NaN or Inf input, or a scale
// that does not fit FP32.  nonfinite_flag() is its device address on the
// current device (looked up once per device); take_nonfinite() waits for
// `s`, and if the word is set clears it and returns QMG_ERR_NONFINITE.
qmg_status nonfinite_flag(unsigned** out);
qmg_status take_nonfinite(hipStream_t s, const char* what);

// Launch error check right after a kernel launch.
#define QMG_LAUNCH_CHECK() QMG_HIP(hipGetLastError())

// ---------------------------------------------------------------- complex
template <typename R> struct cpx { R re, im; };

template <typename R>
__host__ __device__ __forceinline__ void cmac(R& ar, R& ai, R xr, R xi, R yr, R yi) {
    // a += x * y
    ar = fma(xr, yr, ar);
    ar = fma(-xi, yi, ar);
    ai = fma(xr, yi, ai);
    ai = fma(xi, yr, ai);
}

template <typename R>
__host__ __device__ __forceinline__ void cmac_conj(R& ar, R& ai, R xr, R xi, R yr, R yi) {
    // a += conj(x) * y
    ar = fma(xr, yr, ar);
    ar = fma(xi, yi, ar);
    ai = fma(xr, yi, ai);
    ai = fma(-xi, yr, ai);
}

}  // namespace qmg
