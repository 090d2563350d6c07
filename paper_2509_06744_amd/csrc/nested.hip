// Nested block-FSAI with one nesting level (Sec. 2.2).
//
// The inner factor is built for A~_1 = G_0 A G_0^T, where G_0 = J_0 F_0 is
// the (scaled) outer factor; block-FSAI and Algorithm 1 are invariant under
// this block-diagonal congruence, so M = G_0^T G~_1^T G~_1 G_0 is the
// preconditioner F^T S^{-1} F (F = F_1 F_0) of Sec. 2.2.
//
// The triple product C = G A G^T is formed in two products, T = G A and
// C = T G^T. The structures and the list of contributing block pairs of
// every output block are index work done on the host; the block arithmetic
// runs on the GPU, one workgroup per output block, summing its pairs in list
// order (so the result does not depend on the launch).
#include <algorithm>
#include <memory>
#include <vector>

#include "internal.h"

namespace chf {

// out[o] = sum over pairs k of X[px[k]] op(Y[py[k]]), with op(Y) = Y
// (TRANS_Y = false) or Y^T; threads run over the b x b entries of a block.
template <bool TRANS_Y>
__global__ __launch_bounds__(128) void k_block_pairs(int64_t nout, int b, const int64_t* __restrict__ ptr,
                                                     const int* __restrict__ px, const int* __restrict__ py,
                                                     const double* __restrict__ X, const double* __restrict__ Y,
                                                     double* __restrict__ out) {
    const int bb = b * b;
    for (int64_t o = blockIdx.x; o < nout; o += gridDim.x) {
        const int64_t k0 = ptr[o], k1 = ptr[o + 1];
        for (int e = threadIdx.x; e < bb; e += blockDim.x) {
            const int r = e / b, c = e - r * b;
            double acc = 0.0;
            for (int64_t k = k0; k < k1; ++k) {
                const double* x = X + (int64_t)px[k] * bb + r * b;
                const double* y = Y + (int64_t)py[k] * bb;
                if (TRANS_Y) {
                    for (int s = 0; s < b; ++s) acc += x[s] * y[c * b + s];
                } else {
                    for (int s = 0; s < b; ++s) acc += x[s] * y[s * b + c];
                }
            }
            out[o * bb + e] = acc;
        }
    }
}

chf_bsr_s* bsr_triple_impl(chf_bsr A, const chf_fsai_s& G, hipStream_t s) {
    const int64_t nb = A->nb;
    const int b = A->b;
    // structure of G^T: for each column q, the entries (row j, index e) of G
    std::vector<int64_t> gtp(nb + 1, 0);
    for (int64_t e = 0; e < G.nnz; ++e) gtp[G.colidx[e] + 1]++;
    for (int64_t q = 0; q < nb; ++q) gtp[q + 1] += gtp[q];
    std::vector<int32_t> gtr(G.nnz), gte(G.nnz);
    {
        std::vector<int64_t> fill(gtp.begin(), gtp.end() - 1);
        for (int64_t j = 0; j < nb; ++j)
            for (int64_t e = G.rowptr[j]; e < G.rowptr[j + 1]; ++e) {
                const int64_t at = fill[G.colidx[e]]++;
                gtr[at] = (int32_t)j;
                gte[at] = (int32_t)e;
            }
    }
    std::vector<int64_t> mark(nb, -1), pos(nb, 0);
    // T = G A: row i is the union of the rows A_p, p in G_i
    std::vector<int64_t> tptr(nb + 1, 0), tpp(1, 0);
    std::vector<int32_t> tcol, tpx, tpy;
    std::vector<int32_t> row;
    std::vector<int64_t> cnt;
    for (int64_t i = 0; i < nb; ++i) {
        row.clear();
        for (int64_t e = G.rowptr[i]; e < G.rowptr[i + 1]; ++e) {
            const int64_t p = G.colidx[e];
            for (int64_t f = A->rowptr[p]; f < A->rowptr[p + 1]; ++f) {
                const int32_t q = A->colidx[f];
                if (mark[q] != i) {
                    mark[q] = i;
                    row.push_back(q);
                }
            }
        }
        std::sort(row.begin(), row.end());
        const int64_t t0 = (int64_t)tcol.size();
        for (size_t u = 0; u < row.size(); ++u) pos[row[u]] = (int64_t)u;
        cnt.assign(row.size() + 1, 0);
        for (int64_t e = G.rowptr[i]; e < G.rowptr[i + 1]; ++e) {
            const int64_t p = G.colidx[e];
            for (int64_t f = A->rowptr[p]; f < A->rowptr[p + 1]; ++f) cnt[pos[A->colidx[f]] + 1]++;
        }
        for (size_t u = 0; u < row.size(); ++u) cnt[u + 1] += cnt[u];
        const int64_t base = (int64_t)tpx.size();
        tpx.resize(base + cnt[row.size()]);
        tpy.resize(base + cnt[row.size()]);
        std::vector<int64_t> at(cnt.begin(), cnt.end() - 1);
        for (int64_t e = G.rowptr[i]; e < G.rowptr[i + 1]; ++e) {
            const int64_t p = G.colidx[e];
            for (int64_t f = A->rowptr[p]; f < A->rowptr[p + 1]; ++f) {
                const int64_t k = base + at[pos[A->colidx[f]]]++;
                tpx[k] = (int32_t)e;   // G_ip
                tpy[k] = (int32_t)f;   // A_pq
            }
        }
        for (size_t u = 0; u < row.size(); ++u) {
            tcol.push_back(row[u]);
            tpp.push_back(base + cnt[u + 1]);
        }
        tptr[i + 1] = t0 + (int64_t)row.size();
    }
    const int64_t nt = (int64_t)tcol.size();
    CHF_CHECK(nt < (1ll << 31) && (int64_t)tpx.size() < (1ll << 31), CHF_EINVAL, "triple product too large");
    // C = T G^T: row i is the union over q in T_i of the rows j of G with column q
    std::fill(mark.begin(), mark.end(), -1);
    std::unique_ptr<chf_bsr_s> C(new chf_bsr_s);
    C->nb = nb;
    C->b = b;
    C->ndof = nb * (int64_t)b;
    C->rowptr.assign(nb + 1, 0);
    std::vector<int64_t> cpp(1, 0);
    std::vector<int32_t> cpx, cpy;
    for (int64_t i = 0; i < nb; ++i) {
        row.clear();
        for (int64_t t = tptr[i]; t < tptr[i + 1]; ++t) {
            const int64_t q = tcol[t];
            for (int64_t g = gtp[q]; g < gtp[q + 1]; ++g) {
                const int32_t j = gtr[g];
                if (mark[j] != i) {
                    mark[j] = i;
                    row.push_back(j);
                }
            }
        }
        std::sort(row.begin(), row.end());
        for (size_t u = 0; u < row.size(); ++u) pos[row[u]] = (int64_t)u;
        cnt.assign(row.size() + 1, 0);
        for (int64_t t = tptr[i]; t < tptr[i + 1]; ++t) {
            const int64_t q = tcol[t];
            for (int64_t g = gtp[q]; g < gtp[q + 1]; ++g) cnt[pos[gtr[g]] + 1]++;
        }
        for (size_t u = 0; u < row.size(); ++u) cnt[u + 1] += cnt[u];
        const int64_t base = (int64_t)cpx.size();
        cpx.resize(base + cnt[row.size()]);
        cpy.resize(base + cnt[row.size()]);
        std::vector<int64_t> at(cnt.begin(), cnt.end() - 1);
        for (int64_t t = tptr[i]; t < tptr[i + 1]; ++t) {
            const int64_t q = tcol[t];
            for (int64_t g = gtp[q]; g < gtp[q + 1]; ++g) {
                const int64_t k = base + at[pos[gtr[g]]]++;
                cpx[k] = (int32_t)t;        // T_iq
                cpy[k] = gte[g];            // G_jq (transposed in the product)
            }
        }
        for (size_t u = 0; u < row.size(); ++u) {
            C->colidx.push_back(row[u]);
            cpp.push_back(base + cnt[u + 1]);
        }
        C->rowptr[i + 1] = (int64_t)C->colidx.size();
    }
    C->nnzb = (int64_t)C->colidx.size();
    CHF_CHECK(C->nnzb < (1ll << 31) && (int64_t)cpx.size() < (1ll << 31), CHF_EINVAL, "triple product too large");
    // numeric phase
    const int64_t bb = (int64_t)b * b;
    DevBuf<int64_t> d_tpp(tpp.size()), d_cpp(cpp.size());
    DevBuf<int> d_tpx(std::max<size_t>(1, tpx.size())), d_tpy(std::max<size_t>(1, tpy.size()));
    DevBuf<int> d_cpx(std::max<size_t>(1, cpx.size())), d_cpy(std::max<size_t>(1, cpy.size()));
    DevBuf<double> d_t(std::max<int64_t>(1, nt * bb));
    d_tpp.upload(tpp.data(), tpp.size(), s);
    d_cpp.upload(cpp.data(), cpp.size(), s);
    if (!tpx.empty()) {
        d_tpx.upload(tpx.data(), tpx.size(), s);
        d_tpy.upload(tpy.data(), tpy.size(), s);
    }
    if (!cpx.empty()) {
        d_cpx.upload(cpx.data(), cpx.size(), s);
        d_cpy.upload(cpy.data(), cpy.size(), s);
    }
    C->d_vals.alloc(std::max<int64_t>(1, C->nnzb * bb));
    const int cus = device_cu_count();
    if (nt > 0) {
        const int64_t grid = std::min<int64_t>(nt, (int64_t)cus * 64);
        hipLaunchKernelGGL(k_block_pairs<false>, dim3((unsigned)grid), dim3(128), 0, s, nt, b, d_tpp.p, d_tpx.p,
                           d_tpy.p, G.d_vals.p, A->d_vals.p, d_t.p);
        CHF_LAUNCH_CHECK();
    }
    if (C->nnzb > 0) {
        const int64_t grid = std::min<int64_t>(C->nnzb, (int64_t)cus * 64);
        hipLaunchKernelGGL(k_block_pairs<true>, dim3((unsigned)grid), dim3(128), 0, s, C->nnzb, b, d_cpp.p, d_cpx.p,
                           d_cpy.p, (const double*)d_t.p, G.d_vals.p, C->d_vals.p);
        CHF_LAUNCH_CHECK();
    }
    std::vector<int> rp32(nb + 1);
    for (int64_t i = 0; i <= nb; ++i) rp32[i] = (int)C->rowptr[i];
    C->d_rowptr.alloc(nb + 1);
    C->d_rowptr.upload(rp32.data(), nb + 1, s);
    C->d_colidx.alloc(std::max<int64_t>(1, C->nnzb));
    if (C->nnzb) C->d_colidx.upload(C->colidx.data(), C->nnzb, s);
    C->plan = sell_plan(nb, b, C->rowptr, C->colidx, nullptr);
    sell_build(C->sell64, C->plan, C->d_vals.p, false, CHF_F64, s);
    CHF_HIP(hipStreamSynchronize(s));   // the pair lists are released on return
    return C.release();
}

}  // namespace chf

using namespace chf;

extern "C" int chf_bsr_triple(chf_bsr A, chf_fsai G, chf_bsr* out) {
    return guarded([&] {
        CHF_CHECK(A && G && out, CHF_EINVAL, "NULL argument");
        *out = nullptr;
        CHF_CHECK(!G->nest_outer, CHF_EINVAL, "G is a nested factor: pass its outer factor");
        CHF_CHECK(!A->vb && !G->vb, CHF_EINVAL, "nested FSAI supports uniform block sizes only");
        CHF_CHECK(A->nb == G->nb && A->b == G->b, CHF_EINVAL, "A and G sizes differ");
        *out = bsr_triple_impl(A, *G, 0);
    });
}

extern "C" int chf_fsai_nest(chf_fsai G0, chf_fsai G1, chf_fsai* out) {
    return guarded([&] {
        CHF_CHECK(G0 && G1 && out, CHF_EINVAL, "NULL argument");
        *out = nullptr;
        CHF_CHECK(!G0->nest_outer && !G1->nest_outer, CHF_EINVAL, "one nesting level only");
        CHF_CHECK(!G0->vb && !G1->vb, CHF_EINVAL, "nested FSAI supports uniform block sizes only");
        CHF_CHECK(G0->nb == G1->nb && G0->b == G1->b, CHF_EINVAL, "G0 and G1 sizes differ");
        CHF_CHECK(G0->store == G1->store, CHF_EINVAL, "G0 and G1 storage dtypes differ");
        std::unique_ptr<chf_fsai_s> N(new chf_fsai_s);
        N->nb = G0->nb;
        N->b = G0->b;
        N->store = G0->store;
        N->nest_outer = G0;
        N->nest_inner = G1;
        *out = N.release();
    });
}
