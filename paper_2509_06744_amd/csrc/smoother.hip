// Polynomial smoothers with M = G^T G, all written as the same two-term step
//   r = b - A x,  p = a_i p + M r,  x += c_i p        (step 1: p = M r)
// with per-step scalars formed on the host, so nothing is read back:
//   - Algorithm 3 (Chebyshev iteration of the fourth kind) on [0, beta];
//   - Algorithm 2 (Chebyshev iteration of the first kind), preconditioned,
//     on a smoothing interval [alpha, beta] (Sec. 3.1);
//   - Richardson smoothing S = (I - omega M A)^k (Sec. 3.1, omega = 1 there).
//
// Each step is three kernels: r = b - A x (skipped in the first step when x
// starts at zero), t = G r, and z = G^T t fused with the update of p and x.
// With a nested factor (Sec. 2.2), M = G0^T G1^T G1 G0 and the middle of the
// step becomes t = G0 r, t' = G1 t, t = G1^T t' (five kernels).
#include <cmath>
#include <mutex>
#include <vector>

#include "internal.h"

// Work space of chf_cheb4_smooth_noalloc: the three vectors r, t, p of the
// smoother step in one file-scope device array, so that the call allocates
// nothing. Each device the library runs on holds its own copy until the
// process ends. Host code must not pass `scratch` itself to a kernel (on the
// host it is only a stand-in symbol): its device address comes from
// hipGetSymbolAddress, taken once per device.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

namespace chf {

struct StepCoef {
    std::vector<double> a;   // a[i]: weight of the previous p in step i (a[0] unused)
    std::vector<double> c;   // c[i]: x += c[i] p
};

// Algorithm 3: mu_1 = 1/3, p_i = mu_{i-1}^2 p_{i-1} + M r_i, mu_i = 1/(2 - mu_{i-1}),
// x += (4 / beta) mu_i p_i.
static StepCoef cheb4_coef(double beta, int k) {
    StepCoef s;
    const double d = 4.0 / beta;
    double mu = 1.0 / 3.0;
    s.a.push_back(0.0);
    s.c.push_back(d * mu);
    for (int i = 2; i <= k; ++i) {
        const double alpha = mu * mu;
        mu = 1.0 / (2.0 - mu);
        s.a.push_back(alpha);
        s.c.push_back(d * mu);
    }
    return s;
}

// Algorithm 2 with the preconditioner: c = (alpha + beta) / 2,
// d = (beta - alpha) / 2, omega_1 = 1 / c, psi_1 = (d omega_1)^2 / 2; then
// p_i = M r_i + psi_{i-1} p_{i-1}, omega_i = 1 / (c - psi_{i-1} / omega_{i-1}),
// psi_i = (d omega_i / 2)^2, x += omega_i p_i.
static StepCoef cheb1_coef(double alpha, double beta, int k) {
    StepCoef s;
    const double c = 0.5 * (alpha + beta), d = 0.5 * (beta - alpha);
    double omega = 1.0 / c;
    double psi = 0.5 * (d * omega) * (d * omega);
    s.a.push_back(0.0);
    s.c.push_back(omega);
    for (int i = 2; i <= k; ++i) {
        s.a.push_back(psi);
        omega = 1.0 / (c - psi / omega);
        psi = (0.5 * d * omega) * (0.5 * d * omega);
        s.c.push_back(omega);
    }
    return s;
}

static StepCoef richardson_coef(double omega, int k) {
    StepCoef s;
    for (int i = 1; i <= k; ++i) {
        s.a.push_back(0.0);
        s.c.push_back(omega);
    }
    return s;
}

static void poly_smooth_impl(const Sell& A, const Sell& G, const Sell& Gt, const Sell* Gi, const Sell* Git,
                             chf_dtype vec, const StepCoef& cf, const void* b, void* x, bool x_is_zero, void* work,
                             hipStream_t s) {
    const int k = (int)cf.c.size();
    const int64_t n = A.ndof;
    const size_t es = vec_size(vec);
    char* w = static_cast<char*>(work);
    void* r = w;
    void* t = w + n * es;
    void* p = w + 2 * n * es;
    // step 1: r = b - A x0 (or b), p = M r, x = x0 + c_1 p
    const void* r0 = b;
    if (!x_is_zero) {
        sell_spmv(A, vec, x, r, b, EPI_RES, nullptr, nullptr, 0, 0, s);
        r0 = r;
    }
    // t = G r (nested: t = G1^T G1 G0 r, with r's buffer as the spare)
    auto gmid = [&](const void* rin) {
        sell_spmv(G, vec, rin, t, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
        if (Gi) {
            sell_spmv(*Gi, vec, t, r, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
            sell_spmv(*Git, vec, r, t, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
        }
    };
    gmid(r0);
    sell_spmv(Gt, vec, t, nullptr, nullptr, x_is_zero ? EPI_CHEB_FIRST0 : EPI_CHEB_FIRST, p, x, 0.0, cf.c[0], s);
    for (int i = 1; i < k; ++i) {
        sell_spmv(A, vec, x, r, b, EPI_RES, nullptr, nullptr, 0, 0, s);
        gmid(r);
        sell_spmv(Gt, vec, t, nullptr, nullptr, EPI_CHEB, p, x, cf.a[i], cf.c[i], s);
    }
}

static void check_degree(int degree) { CHF_CHECK(degree >= 1, CHF_EINVAL, "degree must be >= 1"); }

void cheb4_impl(const Sell& A, const FactorOps& G, chf_dtype vec, double beta, int degree, const void* b, void* x,
                bool x_is_zero, void* work, hipStream_t s) {
    check_degree(degree);
    CHF_CHECK(beta > 0 && std::isfinite(beta), CHF_EINVAL, "beta must be positive and finite");
    poly_smooth_impl(A, *G.g, *G.gt, G.gi, G.git, vec, cheb4_coef(beta, degree), b, x, x_is_zero, work, s);
}

void cheb1_impl(const Sell& A, const FactorOps& G, chf_dtype vec, double alpha, double beta, int degree,
                const void* b, void* x, bool x_is_zero, void* work, hipStream_t s) {
    check_degree(degree);
    CHF_CHECK(alpha > 0 && beta > alpha && std::isfinite(beta), CHF_EINVAL, "need 0 < alpha < beta < inf");
    poly_smooth_impl(A, *G.g, *G.gt, G.gi, G.git, vec, cheb1_coef(alpha, beta, degree), b, x, x_is_zero, work, s);
}

void richardson_impl(const Sell& A, const FactorOps& G, chf_dtype vec, double omega, int degree, const void* b,
                     void* x, bool x_is_zero, void* work, hipStream_t s) {
    check_degree(degree);
    CHF_CHECK(omega > 0 && std::isfinite(omega), CHF_EINVAL, "omega must be positive and finite");
    poly_smooth_impl(A, *G.g, *G.gt, G.gi, G.git, vec, richardson_coef(omega, degree), b, x, x_is_zero, work, s);
}

}  // namespace chf

using namespace chf;

namespace {
// resolve the operand layouts for a smoother call on (A, G) in `dtype`
template <class F>
int with_operands(chf_bsr A, chf_fsai G, chf_dtype dtype, const void* b, void* x, void* work, hipStream_t stream,
                  F&& f) {
    return guarded([&] {
        CHF_CHECK(A && G && b && x && work, CHF_EINVAL, "NULL argument");
        CHF_CHECK(A->nb == G->nb && A->b == G->b && A->vb == G->base().vb, CHF_EINVAL, "A and G sizes differ");
        CHF_CHECK(dtype == CHF_F64 || dtype == G->store || (dtype == CHF_F64_BF16G && G->store == CHF_BF16),
                  CHF_EINVAL, "dtype must be F64, the factor's storage dtype, or F64_BF16G for a BF16 factor");
        const chf_dtype vec = mode_vec(dtype);
        const Sell& sa = A->sell(vec, stream);
        f(sa, factor_ops(*G, mode_g(dtype)), vec);
    });
}
}  // namespace

extern "C" int chf_cheb4_smooth(chf_bsr A, chf_fsai G, chf_dtype dtype, double beta, int degree, const void* b,
                                void* x, int x_is_zero, void* work, hipStream_t stream) {
    return with_operands(A, G, dtype, b, x, work, stream, [&](const Sell& sa, const FactorOps& g, chf_dtype vec) {
        cheb4_impl(sa, g, vec, beta, degree, b, x, x_is_zero != 0, work, stream);
    });
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call made with that device current, then cached).
void* noalloc_scratch() {
    int dev = 0;
    CHF_HIP(hipGetDevice(&dev));
    CHF_CHECK(dev >= 0 && dev < kMaxDevices, CHF_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        CHF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        CHF_CHECK(p != nullptr, CHF_EDEVICE, "no device address for the smoother scratch");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" int chf_cheb4_smooth_noalloc(chf_bsr A, chf_fsai G, chf_dtype dtype, double beta, int degree,
                                        const void* b, void* x, int x_is_zero, hipStream_t stream) {
    return guarded([&] {
        CHF_CHECK(A && G && b && x, CHF_EINVAL, "NULL argument");
        CHF_CHECK(A->nb == G->nb && A->b == G->b && A->vb == G->base().vb, CHF_EINVAL, "A and G sizes differ");
        CHF_CHECK(dtype == CHF_F64 || dtype == G->store || (dtype == CHF_F64_BF16G && G->store == CHF_BF16),
                  CHF_EINVAL, "dtype must be F64, the factor's storage dtype, or F64_BF16G for a BF16 factor");
        const chf_dtype vec = mode_vec(dtype);
        const int64_t n = A->ndof;
        CHF_CHECK((size_t)n * 3 * vec_size(vec) <= kNoallocScratchBytes, CHF_EINVAL,
                  "chf_cheb4_smooth_noalloc: 3 vectors of " + std::to_string(n) +
                      " elements exceed its 64 MiB scratch");
        // the FP32 layout of A is built on first use, which allocates
        CHF_CHECK(vec == CHF_F64 || !A->vb, CHF_EINVAL, "variable block sizes: FP64 only");
        CHF_CHECK(vec == CHF_F64 || A->nb == 0 || A->sell32.nslices > 0, CHF_EINVAL,
                  "chf_cheb4_smooth_noalloc: the FP32 layout of A does not exist yet (make one FP32 call of "
                  "chf_cheb4_smooth or chf_bsr_spmv first)");
        const Sell& sa = vec == CHF_F64 ? A->sell64 : A->sell32;
        cheb4_impl(sa, factor_ops(*G, mode_g(dtype)), vec, beta, degree, b, x, x_is_zero != 0, noalloc_scratch(),
                   stream);
    });
}

extern "C" int chf_cheb1_smooth(chf_bsr A, chf_fsai G, chf_dtype dtype, double alpha, double beta, int degree,
                                const void* b, void* x, int x_is_zero, void* work, hipStream_t stream) {
    return with_operands(A, G, dtype, b, x, work, stream, [&](const Sell& sa, const FactorOps& g, chf_dtype vec) {
        cheb1_impl(sa, g, vec, alpha, beta, degree, b, x, x_is_zero != 0, work, stream);
    });
}

extern "C" int chf_richardson_smooth(chf_bsr A, chf_fsai G, chf_dtype dtype, double omega, int degree,
                                     const void* b, void* x, int x_is_zero, void* work, hipStream_t stream) {
    return with_operands(A, G, dtype, b, x, work, stream, [&](const Sell& sa, const FactorOps& g, chf_dtype vec) {
        richardson_impl(sa, g, vec, omega, degree, b, x, x_is_zero != 0, work, stream);
    });
}
