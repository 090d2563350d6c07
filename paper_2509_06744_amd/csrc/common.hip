// Errors, dtype helpers, deterministic reductions and small utilities.
#include <cmath>
#include <cstring>

#include "internal.h"
#include "kernels_common.h"

namespace chf {

static thread_local std::string g_last_error;
static thread_local std::vector<void*>* g_free_deferral = nullptr;

void set_free_deferral(std::vector<void*>* list) { g_free_deferral = list; }

void dev_free(void* p) {
    if (!p) return;
    if (g_free_deferral)
        g_free_deferral->push_back(p);
    else
        (void)hipFree(p);
}

void set_error(const std::string& msg) { g_last_error = msg; }

void fail(int code, const std::string& msg) { throw Error(code, msg); }

size_t dtype_size(chf_dtype t) {
    switch (t) {
        case CHF_F64: return 8;
        case CHF_F32: return 4;
        case CHF_BF16: return 2;
    }
    fail(CHF_EINVAL, "unknown dtype");
}

size_t vec_size(chf_dtype t) { return t == CHF_F64 ? 8 : 4; }

int device_cu_count() {
    int dev = 0;
    CHF_HIP(hipGetDevice(&dev));
    int cus = 0;
    CHF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return cus;
}

// ------------------------------------------------------------- fill / cast --
__global__ void k_fill_zero_u32(uint32_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_fill_zero_u8(uint8_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

void fill_zero(void* p, size_t bytes, hipStream_t s) {
    if (!bytes) return;
    if ((reinterpret_cast<uintptr_t>(p) & 3) == 0 && (bytes & 3) == 0) {
        int64_t n = bytes / 4;
        int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
        hipLaunchKernelGGL(k_fill_zero_u32, dim3(grid), dim3(256), 0, s, (uint32_t*)p, n);
    } else {
        int64_t n = bytes;
        int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
        hipLaunchKernelGGL(k_fill_zero_u8, dim3(grid), dim3(256), 0, s, (uint8_t*)p, n);
    }
    CHF_LAUNCH_CHECK();
}

template <typename TI, typename TO>
__global__ void k_cast(const TI* __restrict__ x, TO* __restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (TO)x[i];
}

void cast_vec(chf_dtype from, const void* x, chf_dtype to, void* y, int64_t n, hipStream_t s) {
    int grid = (int)std::min<int64_t>((n + 255) / 256, 16384);
    if (grid < 1) return;
    bool f64i = from == CHF_F64, f64o = to == CHF_F64;
    if (f64i && !f64o)
        hipLaunchKernelGGL((k_cast<double, float>), dim3(grid), dim3(256), 0, s, (const double*)x, (float*)y, n);
    else if (!f64i && f64o)
        hipLaunchKernelGGL((k_cast<float, double>), dim3(grid), dim3(256), 0, s, (const float*)x, (double*)y, n);
    else if (f64i)
        hipLaunchKernelGGL((k_cast<double, double>), dim3(grid), dim3(256), 0, s, (const double*)x, (double*)y, n);
    else
        hipLaunchKernelGGL((k_cast<float, float>), dim3(grid), dim3(256), 0, s, (const float*)x, (float*)y, n);
    CHF_LAUNCH_CHECK();
}

// ------------------------------------------------------------ reductions --
// Stage 1: a fixed grid of RED_BLOCKS blocks, grid-stride partial sums in
// FP64, then a fixed LDS tree per block. Stage 2: one block sums the
// partials with the same tree. Results are bit-reproducible for a given n.
template <typename T>
__global__ __launch_bounds__(256) void k_dot_partial(const T* __restrict__ x, const T* __restrict__ y,
                                                     int64_t n, double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        acc += (double)x[i] * (double)y[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, int np,
                                                      double* __restrict__ out) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

void dot(chf_dtype vec, const void* x, const void* y, int64_t n, double* d_out, double* d_partials,
         hipStream_t s) {
    if (vec == CHF_F64)
        hipLaunchKernelGGL((k_dot_partial<double>), dim3(RED_BLOCKS), dim3(256), 0, s, (const double*)x,
                           (const double*)y, n, d_partials);
    else
        hipLaunchKernelGGL((k_dot_partial<float>), dim3(RED_BLOCKS), dim3(256), 0, s, (const float*)x,
                           (const float*)y, n, d_partials);
    CHF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, d_partials, RED_BLOCKS, d_out);
    CHF_LAUNCH_CHECK();
}

// ------------------------------------------------- tridiagonal eigenvalue --
// Largest eigenvalue of the symmetric tridiagonal matrix (alpha, beta) by
// bisection on the Sturm count (number of eigenvalues below x).
static int sturm_below(const std::vector<double>& a, const std::vector<double>& b, double x) {
    int cnt = 0;
    double q = 1.0;
    const double tiny = 1e-300;
    for (size_t i = 0; i < a.size(); ++i) {
        double bb = i ? b[i - 1] * b[i - 1] : 0.0;
        q = (a[i] - x) - (i ? bb / q : 0.0);
        if (q == 0.0) q = -tiny;
        if (q < 0) ++cnt;
    }
    return cnt;
}

double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
    size_t m = a.size();
    if (m == 0) return 0.0;
    double lo = a[0], hi = a[0];
    for (size_t i = 0; i < m; ++i) {
        double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    double span = std::max(std::fabs(lo), std::fabs(hi));
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_below(a, b, mid) == (int)m) hi = mid; else lo = mid;
        if (hi - lo <= 4e-16 * span) break;
    }
    return 0.5 * (lo + hi);
}

}  // namespace chf

extern "C" const char* chf_last_error(void) { return chf::g_last_error.c_str(); }
extern "C" const char* chf_version(void) { return "chf 0.1 gfx950"; }
