// Variable block sizes (Def. 2.1 with unequal m_i): creation of the matrix,
// its SpMV layout and kernel, and the block-FSAI set-up (Def. 2.2 with
// m_k x m_j blocks). FP64 only.
//
// SpMV layout. A slice is 64 consecutive unknowns, one wavefront, lane =
// unknown. The slice's unknowns belong to block rows i0..i1 (nl local rows; a
// block row may continue in the next slice). Slot j of the slice holds, for
// every lane, row a of the j-th stored block of the lane's block row: W_j
// values, W_j the widest of these blocks over the slice rounded up to even,
// stored as W_j / 2 runs of 128 doubles with lane l's pair at 2 l, so every
// matrix load is a 16-byte load and each run is 1 KB contiguous. Columns past
// a block's width, and slots past a block row's last block, hold zeros; their
// x index is clamped to the vector. cols[] holds, per (slot, local row), the
// first unknown of the column block.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace chf {

struct VSellLayout {
    int64_t nslices = 0, nslots = 0, ndof = 0;
    DevBuf<int> slot_off;       // nslices + 1: first slot of each slice
    DevBuf<int> slot_w;         // nslots: values per lane (even)
    DevBuf<int64_t> slot_voff;  // nslots: first value of the slot
    DevBuf<int> lane_lr;        // nslices * 64: local block row of each lane (-1 past ndof)
    DevBuf<int> col_off;        // nslices + 1: start of the slice's column table
    DevBuf<int> nlr;            // nslices: local block rows of the slice
    DevBuf<int> cols;           // slots x local rows per slice: first unknown of the column block
    DevBuf<double> vals;
};

typedef double vd2 __attribute__((ext_vector_type(2)));

__device__ inline int64_t vxcd_block() {
    // gridDim.x is a multiple of 8; block id b runs on XCD b % 8
    const int64_t per = gridDim.x / 8;
    return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// Pack: one thread per (slot, lane); meta = a | mrow << 8 | mcol << 16.
__global__ void k_vsell_pack(int64_t nslots, const int* __restrict__ slot_w, const int64_t* __restrict__ slot_voff,
                             const int64_t* __restrict__ src, const int* __restrict__ meta, int transpose,
                             const double* __restrict__ blocks, double* __restrict__ out) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nslots * 64) return;
    const int64_t slot = t / 64;
    const int lane = (int)(t - slot * 64);
    const int W = slot_w[slot];
    const int64_t sb = src[t];
    const int mt = meta[t];
    const int a = mt & 0xff, mrow = (mt >> 8) & 0xff, mcol = (mt >> 16) & 0xff;
    double* o = out + slot_voff[slot] + 2 * lane;
    for (int c = 0; c < W; ++c) {
        double v = 0.0;
        if (sb >= 0 && c < mcol) v = transpose ? blocks[sb + (int64_t)c * mrow + a] : blocks[sb + (int64_t)a * mcol + c];
        o[(int64_t)(c >> 1) * 128 + (c & 1)] = v;
    }
}

// Build the layout of the matrix whose block row i holds the blocks at
// colidx[rowptr[i] .. rowptr[i+1]) (ascending), block e's values at
// d_blocks + srcoff[e] (row-major bsize[i] x bsize[col], or its transpose
// stored bsize[col] x bsize[i] when `transpose`).
void vsell_build(Sell& out, const std::vector<int32_t>& bsize, const std::vector<int64_t>& boff,
                 const std::vector<int64_t>& rowptr, const std::vector<int32_t>& colidx,
                 const std::vector<int64_t>& srcoff, bool transpose, const double* d_blocks, hipStream_t s) {
    const int64_t nb = (int64_t)bsize.size();
    const int64_t ndof = boff[nb];
    auto L = std::make_shared<VSellLayout>();
    L->ndof = ndof;
    L->nslices = (ndof + 63) / 64;
    std::vector<int> slot_off(L->nslices + 1, 0), slot_w, lane_lr(L->nslices * 64, -1), col_off(L->nslices + 1, 0),
        nlr(L->nslices, 0), cols;
    std::vector<int64_t> slot_voff, src;
    std::vector<int> meta;
    int64_t nvals = 0;
    for (int64_t sl = 0; sl < L->nslices; ++sl) {
        const int64_t d0 = sl * 64, d1 = std::min<int64_t>(ndof, d0 + 64);
        const int64_t i0 = (int64_t)(std::upper_bound(boff.begin(), boff.end(), d0) - boff.begin()) - 1;
        const int64_t i1 = (int64_t)(std::upper_bound(boff.begin(), boff.end(), d1 - 1) - boff.begin()) - 1;
        const int nl = (int)(i1 - i0 + 1);
        nlr[sl] = nl;
        int64_t ns = 0;
        for (int64_t i = i0; i <= i1; ++i) ns = std::max<int64_t>(ns, rowptr[i + 1] - rowptr[i]);
        for (int64_t d = d0; d < d1; ++d) {
            int64_t i = i0;
            while (boff[i + 1] <= d) ++i;
            lane_lr[sl * 64 + (d - d0)] = (int)(i - i0);
        }
        for (int64_t j = 0; j < ns; ++j) {
            int w = 0;
            for (int64_t i = i0; i <= i1; ++i)
                if (j < rowptr[i + 1] - rowptr[i]) w = std::max(w, (int)bsize[colidx[rowptr[i] + j]]);
            w = (w + 1) / 2 * 2;
            slot_w.push_back(w);
            slot_voff.push_back(nvals);
            nvals += (int64_t)w * 64;
            for (int r = 0; r < nl; ++r) {
                const int64_t i = i0 + r;
                cols.push_back((int)(j < rowptr[i + 1] - rowptr[i] ? boff[colidx[rowptr[i] + j]] : boff[i]));
            }
            for (int lane = 0; lane < 64; ++lane) {
                const int64_t d = d0 + lane;
                int64_t sb = -1;
                int mt = 0;
                if (d < d1) {
                    const int64_t i = i0 + lane_lr[sl * 64 + lane];
                    if (j < rowptr[i + 1] - rowptr[i]) {
                        const int64_t e = rowptr[i] + j;
                        sb = srcoff[e];
                        mt = (int)(d - boff[i]) | (bsize[i] << 8) | (bsize[colidx[e]] << 16);
                    }
                }
                src.push_back(sb);
                meta.push_back(mt);
            }
        }
        slot_off[sl + 1] = slot_off[sl] + (int)ns;
        col_off[sl + 1] = col_off[sl] + (int)(ns * nl);
        CHF_CHECK((int64_t)slot_off[sl + 1] < INT_MAX / 64 && (int64_t)cols.size() < INT_MAX, CHF_EINVAL,
                  "matrix too large for the variable-block SpMV layout");
    }
    L->nslots = slot_off[L->nslices];
    L->slot_off.alloc(slot_off.size());
    L->slot_off.upload(slot_off.data(), slot_off.size(), s);
    L->slot_w.alloc(std::max<size_t>(1, slot_w.size()));
    L->slot_w.upload(slot_w.data(), slot_w.size(), s);
    L->slot_voff.alloc(std::max<size_t>(1, slot_voff.size()));
    L->slot_voff.upload(slot_voff.data(), slot_voff.size(), s);
    L->lane_lr.alloc(std::max<size_t>(1, lane_lr.size()));
    L->lane_lr.upload(lane_lr.data(), lane_lr.size(), s);
    L->col_off.alloc(col_off.size());
    L->col_off.upload(col_off.data(), col_off.size(), s);
    L->nlr.alloc(std::max<size_t>(1, nlr.size()));
    L->nlr.upload(nlr.data(), nlr.size(), s);
    L->cols.alloc(std::max<size_t>(1, cols.size()));
    L->cols.upload(cols.data(), cols.size(), s);
    L->vals.alloc(std::max<int64_t>(1, nvals));
    if (L->nslots > 0) {
        DevBuf<int64_t> d_src(src.size());
        DevBuf<int> d_meta(meta.size());
        d_src.upload(src.data(), src.size(), s);
        d_meta.upload(meta.data(), meta.size(), s);
        const int64_t tot = L->nslots * 64;
        hipLaunchKernelGGL(k_vsell_pack, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, L->nslots,
                           L->slot_w.p, L->slot_voff.p, d_src.p, d_meta.p, transpose ? 1 : 0, d_blocks, L->vals.p);
        CHF_LAUNCH_CHECK();
        CHF_HIP(hipStreamSynchronize(s));   // d_src and d_meta are freed at scope exit
    }
    out.nb = nb;
    out.ndof = ndof;
    out.b = bsize.empty() ? 1 : *std::max_element(bsize.begin(), bsize.end());
    out.dtype = CHF_F64;
    out.vb = L;
}

template <int EPI>
__global__ __launch_bounds__(256) void k_vsell_spmv(int64_t nslices, int64_t ndof, const int* __restrict__ slot_off,
                                                    const int* __restrict__ slot_w,
                                                    const int64_t* __restrict__ slot_voff,
                                                    const int* __restrict__ lane_lr, const int* __restrict__ col_off,
                                                    const int* __restrict__ nlr, const int* __restrict__ cols,
                                                    const double* __restrict__ vals, const double* __restrict__ x,
                                                    double* __restrict__ y, const double* __restrict__ bv,
                                                    double* __restrict__ p, double* __restrict__ xo, double alpha,
                                                    double beta) {
    const int64_t slice = vxcd_block() * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (slice >= nslices) return;
    const int64_t d = slice * 64 + lane;
    if (d >= ndof) return;
    const int nl = nlr[slice];
    const int* cp = cols + col_off[slice] + lane_lr[slice * 64 + lane];
    const int64_t last = ndof - 1;
    double acc = 0.0;
    for (int j = slot_off[slice]; j < slot_off[slice + 1]; ++j, cp += nl) {
        const int W = slot_w[j];
        const double* v = vals + slot_voff[j] + 2 * lane;
        const int64_t x0 = *cp;
        for (int c = 0; c < W; c += 2) {
            const vd2 a = __builtin_nontemporal_load(reinterpret_cast<const vd2*>(v + (int64_t)c * 64));
            acc += a.x * x[min(x0 + c, last)] + a.y * x[min(x0 + c + 1, last)];
        }
    }
    if constexpr (EPI == EPI_AX) {
        y[d] = acc;
    } else if constexpr (EPI == EPI_RES) {
        y[d] = bv[d] - acc;
    } else if constexpr (EPI == EPI_CHEB_FIRST0) {
        p[d] = acc;
        xo[d] = beta * acc;
    } else if constexpr (EPI == EPI_CHEB_FIRST) {
        p[d] = acc;
        xo[d] += beta * acc;
    } else {
        const double pn = alpha * p[d] + acc;
        p[d] = pn;
        xo[d] += beta * pn;
    }
}

void vsell_spmv(const Sell& A, chf_dtype vec, const void* x, void* y, const void* bvec, int epi, void* p, void* xo,
                double alpha, double beta, hipStream_t s) {
    CHF_CHECK(vec == CHF_F64, CHF_EINVAL, "variable block sizes: FP64 only");
    const VSellLayout& L = *A.vb;
    const int64_t nblk = (L.nslices + 3) / 4;
    if (nblk == 0) return;
    dim3 grid((unsigned)((nblk + 7) / 8 * 8)), block(256);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, block, 0, s, L.nslices, L.ndof, L.slot_off.p, L.slot_w.p, L.slot_voff.p,
                           L.lane_lr.p, L.col_off.p, L.nlr.p, L.cols.p, L.vals.p, (const double*)x, (double*)y,
                           (const double*)bvec, (double*)p, (double*)xo, alpha, beta);
    };
    switch (epi) {
        case EPI_AX: go(k_vsell_spmv<EPI_AX>); break;
        case EPI_RES: go(k_vsell_spmv<EPI_RES>); break;
        case EPI_CHEB_FIRST0: go(k_vsell_spmv<EPI_CHEB_FIRST0>); break;
        case EPI_CHEB_FIRST: go(k_vsell_spmv<EPI_CHEB_FIRST>); break;
        default: go(k_vsell_spmv<EPI_CHEB>); break;
    }
    CHF_LAUNCH_CHECK();
}

// ------------------------------------------------------------ FSAI set-up --
// Row k of Def. 2.2 with blocks of their own sizes: K = A[idx, idx] with idx =
// P~_k ascending, then k (n = sum of the m_j), K = L L^T, and G's row blocks
// are the last m_k rows of L^{-1}: G[k, idx] = Z^T with L^T Z = the last m_k
// columns of the identity. One workgroup per row (grid-stride); the lower
// triangle of K, packed by rows, and Z live in LDS.
constexpr int VF_MAXN = 160;   // unknowns of a local system
constexpr int VF_MAXM = 16;    // unknowns of the row's own block
constexpr int VF_MAXP = 32;    // blocks of a pattern row

__device__ inline int vtri(int i) { return i * (i + 1) / 2; }

__device__ inline int vfind(const int* __restrict__ rowptr, const int* __restrict__ col, int row, int want) {
    int lo = rowptr[row], hi = rowptr[row + 1];
    const int end = hi;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] < want) lo = mid + 1; else hi = mid;
    }
    return (lo < end && col[lo] == want) ? lo : -1;
}

__global__ __launch_bounds__(256) void k_vfsai_setup(int64_t nb, const int* __restrict__ bsize,
                                                     const int* __restrict__ a_rowptr, const int* __restrict__ a_col,
                                                     const int64_t* __restrict__ a_voff,
                                                     const double* __restrict__ a_vals,
                                                     const int64_t* __restrict__ prow, const int* __restrict__ pcol,
                                                     const int64_t* __restrict__ g_voff, double* __restrict__ g_vals,
                                                     int* __restrict__ err) {
    __shared__ double K[VF_MAXN * (VF_MAXN + 1) / 2];
    __shared__ double Z[VF_MAXM * VF_MAXN];
    __shared__ int off[VF_MAXP + 1];
    __shared__ int ok;
    const int t = threadIdx.x;
    for (int64_t k = blockIdx.x; k < nb; k += gridDim.x) {
        const int64_t p0 = prow[k];
        const int np = (int)(prow[k + 1] - p0);
        if (t == 0) {
            off[0] = 0;
            for (int q = 0; q < np; ++q) off[q + 1] = off[q] + bsize[pcol[p0 + q]];
            ok = 1;
        }
        __syncthreads();
        const int n = off[np];
        const int m = bsize[k];
        // lower triangle of K = A[idx, idx], one block pair (pr >= pc) per thread
        for (int u = t; u < np * np; u += 256) {
            const int pr = u / np, pc = u - pr * np;
            if (pc > pr) continue;
            const int bi = pcol[p0 + pr], bj = pcol[p0 + pc];
            const int mi = off[pr + 1] - off[pr], mj = off[pc + 1] - off[pc];
            const int e = vfind(a_rowptr, a_col, bi, bj);
            for (int a = 0; a < mi; ++a) {
                const int i = off[pr] + a;
                for (int c = 0; c < mj; ++c) {
                    const int j = off[pc] + c;
                    if (j <= i) K[vtri(i) + j] = e >= 0 ? a_vals[a_voff[e] + (int64_t)a * mj + c] : 0.0;
                }
            }
        }
        __syncthreads();
        // right-looking Cholesky in place
        for (int q = 0; q < n; ++q) {
            if (t == 0) {
                const double dq = K[vtri(q) + q];
                if (!(dq > 0.0) || !isfinite(dq)) ok = 0;
                K[vtri(q) + q] = sqrt(fabs(dq));
            }
            __syncthreads();
            if (!ok) break;
            const double piv = K[vtri(q) + q];
            for (int i = q + 1 + t; i < n; i += 256) K[vtri(i) + q] /= piv;
            __syncthreads();
            const int r = n - q - 1;
            for (int u = t; u < r * r; u += 256) {
                const int i = q + 1 + u / r, j = q + 1 + u % r;
                if (j <= i) K[vtri(i) + j] -= K[vtri(i) + q] * K[vtri(j) + q];
            }
            __syncthreads();
        }
        if (!ok) {
            if (t == 0) atomicMin(err, (int)k);
            __syncthreads();
            continue;
        }
        // L^T Z = E (E: the last m columns of I), one column of Z per thread
        if (t < m) {
            double* z = Z + t * VF_MAXN;
            for (int i = n - 1; i >= 0; --i) {
                double v = (i == n - m + t) ? 1.0 : 0.0;
                for (int l = i + 1; l < n; ++l) v -= K[vtri(l) + i] * z[l];
                z[i] = v / K[vtri(i) + i];
            }
        }
        __syncthreads();
        // G[k, idx] = Z^T: block q's entry (a, c) = Z[off[q] + c][a]
        for (int u = t; u < m * n; u += 256) {
            const int a = u / n, i = u - a * n;
            int q = 0;
            while (off[q + 1] <= i) ++q;
            const int c = i - off[q];
            const int mq = off[q + 1] - off[q];
            g_vals[g_voff[p0 + q] + (int64_t)a * mq + c] = Z[a * VF_MAXN + i];
        }
        __syncthreads();
    }
}

chf_fsai_s* vfsai_setup_impl(chf_bsr A, const chf_pattern_s& P, int64_t* bad_row, hipStream_t s) {
    CHF_CHECK(P.nb == A->nb, CHF_EINVAL, "pattern and matrix sizes differ");
    const int64_t nb = A->nb;
    std::unique_ptr<chf_fsai_s> G(new chf_fsai_s);
    G->nb = nb;
    G->b = A->b;
    G->store = CHF_F64;
    G->vb = true;
    G->bsize = A->bsize;
    G->rowptr = P.rowptr;
    G->colidx = P.colidx;
    G->nnz = P.rowptr[nb];
    G->voff.assign(G->nnz + 1, 0);
    for (int64_t k = 0; k < nb; ++k) {
        int64_t n = 0;
        for (int64_t e = P.rowptr[k]; e < P.rowptr[k + 1]; ++e) {
            n += A->bsize[P.colidx[e]];
            G->voff[e + 1] = G->voff[e] + (int64_t)A->bsize[k] * A->bsize[P.colidx[e]];
        }
        CHF_CHECK(P.rowptr[k + 1] - P.rowptr[k] <= VF_MAXP && n <= VF_MAXN && A->bsize[k] <= VF_MAXM, CHF_EINVAL,
                  "variable-block pattern row " + std::to_string(k) + " too large for the local solver (at most " +
                      std::to_string(VF_MAXP) + " blocks, " + std::to_string(VF_MAXN) + " unknowns, own block " +
                      std::to_string(VF_MAXM) + ")");
    }
    std::vector<int> pcol32(P.colidx.begin(), P.colidx.end());
    DevBuf<int64_t> d_prow(nb + 1), d_gvoff(G->nnz + 1);
    DevBuf<int> d_pcol(std::max<int64_t>(1, G->nnz)), d_err(1);
    d_prow.upload(P.rowptr.data(), nb + 1, s);
    d_pcol.upload(pcol32.data(), G->nnz, s);
    d_gvoff.upload(G->voff.data(), G->nnz + 1, s);
    const int init = INT32_MAX;
    d_err.upload(&init, 1, s);
    G->d_vals.alloc(std::max<int64_t>(1, G->voff[G->nnz]));
    if (nb > 0) {
        const int64_t grid = std::min<int64_t>(nb, (int64_t)device_cu_count() * 2);
        hipLaunchKernelGGL(k_vfsai_setup, dim3((unsigned)grid), dim3(256), 0, s, nb, A->d_bsize.p, A->d_rowptr.p,
                           A->d_colidx.p, A->d_voff.p, A->d_vals.p, d_prow.p, d_pcol.p, d_gvoff.p, G->d_vals.p,
                           d_err.p);
        CHF_LAUNCH_CHECK();
        int herr = 0;
        d_err.download(&herr, 1, s);
        CHF_HIP(hipStreamSynchronize(s));
        if (herr != INT32_MAX) {
            if (bad_row) *bad_row = herr;
            fail(CHF_ENOTSPD, "local FSAI system of block row " + std::to_string(herr) + " is not positive definite");
        }
    }
    // SpMV layouts of G and G^T (G^T's block (j, k) is G's block (k, j) transposed)
    vsell_build(G->g64, A->bsize, A->boff, G->rowptr, G->colidx, std::vector<int64_t>(G->voff.begin(), G->voff.end() - 1),
                false, G->d_vals.p, s);
    std::vector<int64_t> trow(nb + 1, 0), tsrc(G->nnz);
    std::vector<int32_t> tcol(G->nnz);
    for (int64_t e = 0; e < G->nnz; ++e) trow[G->colidx[e] + 1]++;
    for (int64_t j = 0; j < nb; ++j) trow[j + 1] += trow[j];
    std::vector<int64_t> fillp(trow.begin(), trow.end() - 1);
    for (int64_t i = 0; i < nb; ++i)
        for (int64_t e = G->rowptr[i]; e < G->rowptr[i + 1]; ++e) {
            const int64_t pos = fillp[G->colidx[e]]++;
            tcol[pos] = (int32_t)i;
            tsrc[pos] = G->voff[e];
        }
    vsell_build(G->gt64, A->bsize, A->boff, trow, tcol, tsrc, true, G->d_vals.p, s);
    CHF_HIP(hipStreamSynchronize(s));
    return G.release();
}

}  // namespace chf

using namespace chf;

extern "C" int chf_vbsr_create(int64_t nb, const int32_t* bsize, const int64_t* rowptr, const int32_t* colidx,
                               const double* vals, chf_bsr* out) {
    return guarded([&] {
        CHF_CHECK(out, CHF_EINVAL, "out is NULL");
        *out = nullptr;
        CHF_CHECK(nb >= 0 && bsize && rowptr && (nb == 0 || (colidx && vals)), CHF_EINVAL, "bad argument");
        CHF_CHECK(rowptr[0] == 0, CHF_EINVAL, "rowptr[0] must be 0");
        const int64_t nnzb = rowptr[nb];
        CHF_CHECK(nnzb >= 0 && nnzb < (1ll << 31), CHF_EINVAL, "bad nnzb");
        std::unique_ptr<chf_bsr_s> A(new chf_bsr_s);
        A->nb = nb;
        A->nnzb = nnzb;
        A->vb = true;
        A->bsize.assign(bsize, bsize + nb);
        A->boff.assign(nb + 1, 0);
        int bmax = 1;
        for (int64_t i = 0; i < nb; ++i) {
            CHF_CHECK(bsize[i] >= 1 && bsize[i] <= 64, CHF_EINVAL, "block sizes must be in [1, 64]");
            A->boff[i + 1] = A->boff[i] + bsize[i];
            bmax = std::max(bmax, (int)bsize[i]);
        }
        A->b = bmax;
        A->ndof = A->boff[nb];
        CHF_CHECK(A->ndof < (1ll << 31), CHF_EINVAL, "too many unknowns");
        A->voff.assign(nnzb + 1, 0);
        for (int64_t i = 0; i < nb; ++i) {
            CHF_CHECK(rowptr[i + 1] >= rowptr[i], CHF_EINVAL, "rowptr not monotone");
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                CHF_CHECK(colidx[e] >= 0 && colidx[e] < nb, CHF_EINVAL, "column index out of range");
                CHF_CHECK(e == rowptr[i] || colidx[e] > colidx[e - 1], CHF_EINVAL,
                          "column indices must ascend strictly within a row");
                A->voff[e + 1] = A->voff[e] + (int64_t)bsize[i] * bsize[colidx[e]];
            }
        }
        A->rowptr.assign(rowptr, rowptr + nb + 1);
        A->colidx.assign(colidx, colidx + nnzb);
        hipStream_t s = 0;
        std::vector<int> rp32(nb + 1);
        for (int64_t i = 0; i <= nb; ++i) rp32[i] = (int)rowptr[i];
        A->d_rowptr.alloc(nb + 1);
        A->d_rowptr.upload(rp32.data(), nb + 1, s);
        A->d_colidx.alloc(std::max<int64_t>(1, nnzb));
        A->d_colidx.upload(colidx, nnzb, s);
        A->d_bsize.alloc(std::max<int64_t>(1, nb));
        A->d_bsize.upload(bsize, nb, s);
        A->d_voff.alloc(nnzb + 1);
        A->d_voff.upload(A->voff.data(), nnzb + 1, s);
        const size_t nv = (size_t)A->voff[nnzb];
        A->d_vals.alloc(std::max<size_t>(1, nv));
        A->d_vals.upload(vals, nv, s);
        std::vector<double> check(vals, vals + nv);
        for (double v : check) CHF_CHECK(std::isfinite(v), CHF_EINVAL, "non-finite matrix value");
        vsell_build(A->sell64, A->bsize, A->boff, A->rowptr, A->colidx,
                    std::vector<int64_t>(A->voff.begin(), A->voff.end() - 1), false, A->d_vals.p, s);
        CHF_HIP(hipStreamSynchronize(s));
        *out = A.release();
    });
}

extern "C" int chf_vbsr_info(chf_bsr A, int64_t* ndof, int64_t* nvals, int32_t* bsize) {
    return guarded([&] {
        CHF_CHECK(A, CHF_EINVAL, "NULL handle");
        if (ndof) *ndof = A->ndof;
        if (nvals) *nvals = A->vb ? A->voff[A->nnzb] : A->nnzb * (int64_t)A->b * A->b;
        if (bsize) {
            if (A->vb)
                std::memcpy(bsize, A->bsize.data(), A->nb * 4);
            else
                for (int64_t i = 0; i < A->nb; ++i) bsize[i] = A->b;
        }
    });
}
