// Read-stream reference kernel: the achievable HBM read bandwidth the
// read-dominated stencils are measured against (the coarse operator of Eq. (3)
// reads its links once and writes a vector a ninth of their size).  Every
// thread walks the buffer grid-strided with eight independent 16-byte loads
// in flight per step, folds what it reads into one word, and one word per
// work-group is written so the loads cannot be dropped.  The loads are
// non-temporal, as the stencils' link loads are.  16 work-groups of 256
// threads per compute unit; of the shapes measured (4, 8, 16 work-groups per
// CU; 4, 8, 16 loads in flight; with and without the hint) this one read
// fastest, 6.2 TB/s over 2 GiB.
#include "qmg_internal.h"

namespace {

typedef unsigned int u4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_read_stream(const u4v* __restrict__ p, int64_t n, uint32_t* __restrict__ sink) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (; i + 7 * stride < n; i += 8 * stride) {
        u4v v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = __builtin_nontemporal_load(p + i + k * stride);
        u4v e = v[0];
#pragma unroll
        for (int k = 1; k < 8; ++k) e ^= v[k];
        acc ^= e.x ^ e.y ^ e.z ^ e.w;
    }
    for (; i < n; i += stride) {
        const u4v a = __builtin_nontemporal_load(p + i);
        acc ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    __shared__ uint32_t red[4];
    for (int o = 32; o > 0; o >>= 1) acc ^= __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) sink[blockIdx.x] = red[0] ^ red[1] ^ red[2] ^ red[3];
}

}  // namespace

using namespace qmg;

extern "C" qmg_status qmg_stream_read(const void* buf, long long bytes, void* sink, int sink_words, void* stream) {
    if (!buf || !sink) return fail(QMG_ERR_ARG, "stream_read: NULL argument");
    if (bytes < 16 || bytes % 16) return fail(QMG_ERR_ARG, "stream_read: %lld bytes (a multiple of 16)", bytes);
    int dev = 0, cus = 0;
    QMG_HIP(hipGetDevice(&dev));
    QMG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const unsigned grid = (unsigned)(cus > 0 ? 16 * cus : 4096);
    if ((long long)sink_words < (long long)grid)
        return fail(QMG_ERR_ARG, "stream_read: the sink needs %u words, has %d", grid, sink_words);
    hipLaunchKernelGGL(k_read_stream, dim3(grid), dim3(256), 0, as_stream(stream), static_cast<const u4v*>(buf),
                       (int64_t)(bytes / 16), static_cast<uint32_t*>(sink));
    QMG_LAUNCH_CHECK();
    return QMG_OK;
}
