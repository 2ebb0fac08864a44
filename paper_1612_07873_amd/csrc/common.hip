// Error state, argument checks and lattice helpers shared by the entry points.
#include "qmg_internal.h"

#include <mutex>
#include <vector>

namespace qmg {

static thread_local char g_err[1024] = "";

qmg_status fail(qmg_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

void clear_error() { g_err[0] = 0; }

qmg_status check_dims(const int dims[4], int min_extent, const char* what) {
    if (!dims) return fail(QMG_ERR_ARG, "%s: dims is NULL", what);
    for (int m = 0; m < 4; ++m)
        if (dims[m] < min_extent || dims[m] > (1 << 12))
            return fail(QMG_ERR_SHAPE, "%s: extent %d of dimension %d outside [%d, 4096]", what,
                        dims[m], m, min_extent);
    if (volume(dims) > (int64_t)1 << 30) return fail(QMG_ERR_SHAPE, "%s: volume too large", what);
    return QMG_OK;
}

qmg_status make_neighbour_table(const int dims[4], int** dev_out, hipStream_t s) {
    const int64_t V = volume(dims);
    std::vector<int> h(V * 8);
    for (int64_t i = 0; i < V; ++i) {
        int x[4];
        int64_t t = i;
        for (int m = 0; m < 4; ++m) { x[m] = (int)(t % dims[m]); t /= dims[m]; }
        for (int d = 0; d < 8; ++d) {
            int mu = d / 2, step = (d & 1) ? -1 : 1;
            int y[4] = {x[0], x[1], x[2], x[3]};
            y[mu] = (y[mu] + step + dims[mu]) % dims[mu];
            h[i * 8 + d] = y[0] + dims[0] * (y[1] + dims[1] * (y[2] + dims[2] * y[3]));
        }
    }
    int* d = nullptr;
    QMG_HIP(hipMalloc(&d, sizeof(int) * V * 8));
    hipError_t e = hipMemcpyAsync(d, h.data(), sizeof(int) * V * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(QMG_ERR_HIP, "neighbour table upload: %s", hipGetErrorString(e));
    }
    *dev_out = d;
    return QMG_OK;
}

// Red-black numbering: for each parity p (of x0 + x1 + x2 + x3) the lattice
// indices of its sites in lattice order, [2][V/2].  With every extent even
// the half-lattice index of site x is x >> 1 (x0 runs fastest), which the
// kernels use for neighbours; that is checked here.
qmg_status make_half_site_table(const int dims[4], int** dev_out, hipStream_t s) {
    for (int m = 0; m < 4; ++m)
        if (dims[m] % 2) return fail(QMG_ERR_SHAPE, "red-black form: extent %d of dimension %d is odd", dims[m], m);
    const int64_t V = volume(dims), Vh = V / 2;
    std::vector<int> h(V);
    int64_t cnt[2] = {0, 0};
    for (int64_t i = 0; i < V; ++i) {
        int64_t t = i, par = 0;
        for (int m = 0; m < 4; ++m) { par += t % dims[m]; t /= dims[m]; }
        const int p = (int)(par & 1);
        if (cnt[p] != (i >> 1)) return fail(QMG_ERR_SHAPE, "red-black form: half-lattice numbering mismatch");
        h[p * Vh + cnt[p]++] = (int)i;
    }
    int* d = nullptr;
    QMG_HIP(hipMalloc(&d, sizeof(int) * V));
    hipError_t e = hipMemcpyAsync(d, h.data(), sizeof(int) * V, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(QMG_ERR_HIP, "half-site table upload: %s", hipGetErrorString(e));
    }
    *dev_out = d;
    return QMG_OK;
}

namespace {
__device__ unsigned g_nonfinite = 0;   // one word per device: see nonfinite_flag()
std::mutex g_nf_mu;
std::vector<unsigned*> g_nf_ptr;
}  // namespace

qmg_status nonfinite_flag(unsigned** out) {
    int dev = 0;
    QMG_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_nf_mu);
    if ((int)g_nf_ptr.size() <= dev) g_nf_ptr.resize(dev + 1, nullptr);
    if (!g_nf_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_nonfinite));
        if (e != hipSuccess || !p)
            return fail(QMG_ERR_HIP, "non-finite flag address on device %d: %s", dev, hipGetErrorString(e));
        g_nf_ptr[dev] = static_cast<unsigned*>(p);
    }
    *out = g_nf_ptr[dev];
    return QMG_OK;
}

qmg_status take_nonfinite(hipStream_t s, const char* what) {
    unsigned* f = nullptr;
    QMG_TRY(nonfinite_flag(&f));
    unsigned h = 0;
    QMG_HIP(hipMemcpyAsync(&h, f, sizeof h, hipMemcpyDeviceToHost, s));
    QMG_HIP(hipStreamSynchronize(s));
    if (!h) return QMG_OK;
    const unsigned zero = 0;
    QMG_HIP(hipMemcpyAsync(f, &zero, sizeof zero, hipMemcpyHostToDevice, s));
    QMG_HIP(hipStreamSynchronize(s));
    return fail(QMG_ERR_NONFINITE, "%s: a 16-bit encoder met a NaN or Inf input (or a scale beyond FP32)", what);
}

const char* last_error() { return g_err; }

}  // namespace qmg

extern "C" const char* qmg_last_error(void) { return qmg::last_error(); }

extern "C" int qmg_version(void) { return 100; }

extern "C" qmg_status qmg_sync(void* stream) {
    QMG_HIP(hipStreamSynchronize(qmg::as_stream(stream)));
    return qmg::take_nonfinite(qmg::as_stream(stream), "sync");
}
