// Fourth-kind Chebyshev smoothing (Algorithm 3) with M = G^T G.
//
// Each step is three kernels: r = b - A x (skipped in the first step when x
// starts at zero), t = G r, and z = G^T t fused with the recurrence
// p = mu^2 p + z; mu <- 1 / (2 - mu); x += d mu p (first step: p = z). The
// scalars mu_i and d mu_i are formed on the host, so nothing is read back.
#include <cmath>

#include "internal.h"

namespace chf {

void cheb4_impl(const Sell& A, const Sell& G, const Sell& Gt, chf_dtype vec, double beta, int degree,
                const void* b, void* x, bool x_is_zero, void* work, hipStream_t s) {
    CHF_CHECK(degree >= 1, CHF_EINVAL, "degree must be >= 1");
    CHF_CHECK(beta > 0 && std::isfinite(beta), CHF_EINVAL, "beta must be positive and finite");
    const int64_t n = A.nb * (int64_t)A.b;
    const size_t es = vec_size(vec);
    char* w = static_cast<char*>(work);
    void* r = w;
    void* t = w + n * es;
    void* p = w + 2 * n * es;
    const double d = 4.0 / beta;
    double mu = 1.0 / 3.0;
    // step 1: r = b - A x0 (or b), p = M r, x = x0 + d mu p
    const void* r0 = b;
    if (!x_is_zero) {
        sell_spmv(A, vec, x, r, b, EPI_RES, nullptr, nullptr, 0, 0, s);
        r0 = r;
    }
    sell_spmv(G, vec, r0, t, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
    sell_spmv(Gt, vec, t, nullptr, nullptr, x_is_zero ? EPI_CHEB_FIRST0 : EPI_CHEB_FIRST, p, x, 0.0, d * mu, s);
    for (int i = 2; i <= degree; ++i) {
        // r = b - A x ; p = mu^2 p + M r ; mu = 1/(2 - mu) ; x += d mu p
        sell_spmv(A, vec, x, r, b, EPI_RES, nullptr, nullptr, 0, 0, s);
        sell_spmv(G, vec, r, t, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
        const double alpha = mu * mu;
        mu = 1.0 / (2.0 - mu);
        sell_spmv(Gt, vec, t, nullptr, nullptr, EPI_CHEB, p, x, alpha, d * mu, s);
    }
}

}  // namespace chf

using namespace chf;

extern "C" int chf_cheb4_smooth(chf_bsr A, chf_fsai G, chf_dtype dtype, double beta, int degree, const void* b,
                                void* x, int x_is_zero, void* work, hipStream_t stream) {
    return guarded([&] {
        CHF_CHECK(A && G && b && x && work, CHF_EINVAL, "NULL argument");
        CHF_CHECK(A->nb == G->nb && A->b == G->b, CHF_EINVAL, "A and G sizes differ");
        CHF_CHECK(dtype == CHF_F64 || dtype == G->store, CHF_EINVAL,
                  "dtype must be F64 or the factor's storage dtype");
        chf_dtype vec = dtype == CHF_F64 ? CHF_F64 : CHF_F32;
        const Sell& sa = A->sell(vec, stream);
        cheb4_impl(sa, G->g(dtype), G->gt(dtype), vec, beta, degree, b, x, x_is_zero != 0, work, stream);
    });
}
