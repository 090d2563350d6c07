// Adaptive block-FSAI pattern (Algorithm 1 with the ratio of Lemma 2.4) on the
// GPU. Block rows evolve independently (row k of F depends only on A and
// P_k), so one workgroup owns one row for all t_max steps.
//
// Per row, with P~ the off-diagonal part of P_k kept in insertion order:
//   L  = chol(A[P~, P~])                (extended by one block row per step)
//   Y_k = L^{-1} A[P~, k],  H_kk = A_kk - Y_k^T Y_k = (F A F^T)_kk
// and for each candidate c (c < k, c not in P_k, (FA)_kc structurally
// nonzero, i.e. c in the pattern of some row A_j with j in P_k):
//   Y_c = L^{-1} A[P~, c],  H_kc = A_kc - Y_k^T Y_c,  W_c = A_cc - Y_c^T Y_c,
//   rho_c = det(W_c - H_kc^T H_kk^{-1} H_kc) / det(W_c) = det(I - X X^T),
//   X = L_W^{-1} H_kc^T L_H^{-T}   (W_c = L_W L_W^T, H_kk = L_H L_H^T),
//   g_c = -log rho_c, evaluated by a Cholesky of I - X X^T with log1p pivots.
// The best candidate c* (largest g; ties within a relative 1e-9 of the best go
// to the smallest block index) enters when g* > -log(tau) + 1e-12. Adding c*
// appends [Y_c*^T, L_W] to L, L_W^{-1} H_kc*^T to Y_k, and updates H_kk.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace chf {

constexpr int AD_MAXP = 32;     // blocks per row (t_max + 1)
constexpr int AD_MAXC = 640;    // candidates per row
constexpr double AD_TIE_REL = 1e-9;
constexpr double AD_GAIN_EPS = 1e-12;

__device__ inline int64_t atri(int64_t i) { return i * (i + 1) / 2; }

__device__ inline int find_block(const int* __restrict__ rowptr, const int* __restrict__ col, int row, int want) {
    int lo = rowptr[row], hi = rowptr[row + 1];
    const int end = hi;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (col[mid] < want) lo = mid + 1; else hi = mid;
    }
    return (lo < end && col[lo] == want) ? lo : -1;
}

struct AdRegion {
    double* L;     // packed lower, Mmax
    double* Yk;    // Mmax x b (row-major)
    double* Hkk;   // b x b
    double* LH;    // b x b (lower)
    double* W;     // NB x b x b  (W_c, then L_W in place)
    double* Hc;    // NB x b x b  (H_kc)
    double* U;     // NB x b x b  (L_W^{-1} H_kc^T)
    double* X;     // NB x b x b
    double* Cm;    // NB x b x b (shares H_kc's storage: H_kc is dead once U is formed)
};

__device__ inline AdRegion ad_region(double* base, int Mmax, int b, int NB) {
    AdRegion r;
    const int bb = b * b;
    r.L = base;
    r.Yk = r.L + atri(Mmax);
    r.Hkk = r.Yk + (int64_t)Mmax * b;
    r.LH = r.Hkk + bb;
    r.W = r.LH + bb;
    r.Hc = r.W + NB * bb;
    r.U = r.Hc + NB * bb;
    r.X = r.U + NB * bb;
    r.Cm = r.Hc;
    return r;
}

__host__ __device__ inline int64_t ad_region_doubles(int Mmax, int b, int NB) {
    return Mmax * (int64_t)(Mmax + 1) / 2 + (int64_t)Mmax * b + 2 * b * b + 4 * (int64_t)NB * b * b;
}

// Lower Cholesky of the b x b matrix in H (row-major) into LH, lanes < b
// each own one row. Returns false (uniformly) if a pivot is not positive.
__device__ bool small_chol(const double* H, double* LH, int b, int lane, int* flag) {
    if (lane < b)
        for (int j = 0; j < b; ++j) LH[lane * b + j] = j <= lane ? H[lane * b + j] : 0.0;
    if (lane == 0) *flag = 1;
    __syncthreads();
    for (int q = 0; q < b; ++q) {
        if (lane == 0) {
            double d = LH[q * b + q];
            if (!(d > 0.0) || !isfinite(d)) *flag = 0;
            LH[q * b + q] = sqrt(fabs(d));
        }
        __syncthreads();
        if (!*flag) return false;
        if (lane > q && lane < b) LH[lane * b + q] /= LH[q * b + q];
        __syncthreads();
        if (lane > q && lane < b)
            for (int j = q + 1; j <= lane; ++j) LH[lane * b + j] -= LH[lane * b + q] * LH[j * b + q];
        __syncthreads();
    }
    return true;
}

// Gains for candidates cand[s0 .. s0+cnt) (cnt <= NB), b <= MAXB. Lane
// (ci, col) owns column col of candidate ci's right-hand-side block
// A[P~, c]; the block is kept at Ybuf[i * NT + lane] (row i). On return
// gain[] is set (when non-null) and R.W / R.U hold L_W and L_W^{-1} H_kc^T
// for each candidate of the batch.
template <int MAXB, int NT>
__device__ void ad_batch(int k, int b, int NB, int m, int M, const int* plist, const int* cand, int s0, int cnt,
                         const int* __restrict__ a_rowptr, const int* __restrict__ a_col,
                         const double* __restrict__ a_vals, const AdRegion& R, double* __restrict__ Ybuf,
                         double* gain, double* part, int* flag, int* err) {
    // NB = (NT / 64) * (64 / b) candidates per batch: every wavefront holds
    // 64 / b groups of b lanes, one group per candidate.
    const int lane = threadIdx.x;
    const int bb = b * b;
    const int gw = 64 / b;
    const int wl = lane & 63;
    const int ci = (lane >> 6) * gw + wl / b;
    const int col = wl - (wl / b) * b;
    const int gl0 = lane - col;                  // first lane of this lane's group
    const bool act = ci < cnt && wl < gw * b;
    const int c = act ? cand[s0 + ci] : 0;
    if (act) {
        // right-hand side A[P~, c][:, col]
        for (int jb = 0; jb < m; ++jb) {
            const int e = find_block(a_rowptr, a_col, plist[jb], c);
            for (int r = 0; r < b; ++r)
                Ybuf[(int64_t)(jb * b + r) * NT + lane] = e >= 0 ? a_vals[(int64_t)e * bb + r * b + col] : 0.0;
        }
        // Y_c = L^{-1} A[P~, c], right-looking by block rows: the b solved
        // values of a block stay in registers and every later row is updated
        // independently of the others.
        for (int jb = 0; jb < m; ++jb) {
            const int i0 = jb * b;
            double yv[MAXB];
#pragma unroll
            for (int r = 0; r < MAXB; ++r) {
                if (r < b) {
                    const double* li = R.L + atri(i0 + r) + i0;
                    double sacc = Ybuf[(int64_t)(i0 + r) * NT + lane];
#pragma unroll
                    for (int q = 0; q < MAXB; ++q)
                        if (q < r) sacc -= li[q] * yv[q];
                    yv[r] = sacc / li[r];
                    Ybuf[(int64_t)(i0 + r) * NT + lane] = yv[r];
                }
            }
            for (int i = i0 + b; i < M; ++i) {
                const double* li = R.L + atri(i) + i0;
                double sacc = Ybuf[(int64_t)i * NT + lane];
#pragma unroll
                for (int q = 0; q < MAXB; ++q)
                    if (q < b) sacc -= li[q] * yv[q];
                Ybuf[(int64_t)i * NT + lane] = sacc;
            }
        }
    }
    __syncthreads();
    // H_kc[:, col] = A_kc[:, col] - Y_k^T y ; W_c[:, col] = A_cc[:, col] - Y_c^T y
    if (act) {
        const int ekc = find_block(a_rowptr, a_col, k, c);
        const int ecc = find_block(a_rowptr, a_col, c, c);
        double h[MAXB], w[MAXB];
#pragma unroll
        for (int rr = 0; rr < MAXB; ++rr) {
            if (rr < b) {
                h[rr] = ekc >= 0 ? a_vals[(int64_t)ekc * bb + rr * b + col] : 0.0;
                w[rr] = ecc >= 0 ? a_vals[(int64_t)ecc * bb + rr * b + col] : 0.0;
            }
        }
        for (int i = 0; i < M; ++i) {
            const double yi = Ybuf[(int64_t)i * NT + lane];
            const double* yk = R.Yk + (int64_t)i * b;
            const double* yg = Ybuf + (int64_t)i * NT + gl0;
#pragma unroll
            for (int rr = 0; rr < MAXB; ++rr) {
                if (rr < b) {
                    h[rr] -= yk[rr] * yi;
                    w[rr] -= yg[rr] * yi;
                }
            }
        }
        double* Hc = R.Hc + ci * bb;
        double* W = R.W + ci * bb;
#pragma unroll
        for (int rr = 0; rr < MAXB; ++rr) {
            if (rr < b) {
                Hc[rr * b + col] = h[rr];
                W[rr * b + col] = w[rr];
            }
        }
    }
    if (lane == 0) *flag = 1;
    __syncthreads();
    // L_W = chol(W_c) in place; lanes of group ci own rows
    for (int q = 0; q < b; ++q) {
        double* W = R.W + ci * bb;
        if (act && col == 0) {
            double d = W[q * b + q];
            if (!(d > 0.0) || !isfinite(d)) *flag = 0;
            W[q * b + q] = sqrt(fabs(d));
        }
        __syncthreads();
        if (act && col > q) W[col * b + q] /= W[q * b + q];
        __syncthreads();
        if (act && col > q)
            for (int j = q + 1; j <= col; ++j) W[col * b + j] -= W[col * b + q] * W[j * b + q];
        __syncthreads();
    }
    if (!*flag) {
        if (lane == 0) atomicMin(err, k);
        return;
    }
    // U = L_W^{-1} H_kc^T (column col of U)
    if (act) {
        const double* W = R.W + ci * bb;
        const double* Hc = R.Hc + ci * bb;
        double* U = R.U + ci * bb;
        for (int i = 0; i < b; ++i) {
            double sacc = Hc[col * b + i];
            for (int q = 0; q < i; ++q) sacc -= W[i * b + q] * U[q * b + col];
            U[i * b + col] = sacc / W[i * b + i];
        }
    }
    __syncthreads();
    // X = U L_H^{-T}: row `col` of X
    if (act) {
        const double* U = R.U + ci * bb;
        double* X = R.X + ci * bb;
        for (int j = 0; j < b; ++j) {
            double sacc = U[col * b + j];
            for (int q = 0; q < j; ++q) sacc -= X[col * b + q] * R.LH[j * b + q];
            X[col * b + j] = sacc / R.LH[j * b + j];
        }
    }
    __syncthreads();
    // N = C = X X^T: row `col`
    if (act) {
        const double* X = R.X + ci * bb;
        double* Cm = R.Cm + ci * bb;
        for (int j = 0; j < b; ++j) {
            double sacc = 0.0;
            for (int q = 0; q < b; ++q) sacc += X[col * b + q] * X[j * b + q];
            Cm[col * b + j] = sacc;
        }
    }
    __syncthreads();
    // g = -log det(I - C): right-looking Cholesky of I - C written on
    // N = C + sum_q l_q l_q^T, whose diagonal is s_q = 1 - pivot_q^2, so each
    // pivot's log is log1p(-s_q); lanes of a group own rows.
    double lg = 0.0;
    for (int q = 0; q < b; ++q) {
        double* N = R.Cm + ci * bb;
        if (act && col == q) {
            const double sq = N[q * b + q];
            if (!(sq < 1.0)) *flag = 0;
            lg += log1p(-sq);
            N[q * b + q] = sqrt(fmax(1.0 - sq, 0.0));
        }
        __syncthreads();
        if (act && col > q) N[col * b + q] = -N[col * b + q] / N[q * b + q];
        __syncthreads();
        if (act && col > q)
            for (int j = q + 1; j <= col; ++j) N[col * b + j] += N[col * b + q] * N[j * b + q];
        __syncthreads();
    }
    part[lane] = lg;
    __syncthreads();
    if (!*flag) {
        if (lane == 0) atomicMin(err, k);
        return;
    }
    if (act && col == 0 && gain) {
        double acc = 0.0;
        for (int q = 0; q < b; ++q) acc += part[lane + q];
        gain[s0 + ci] = -acc;
    }
    __syncthreads();
}

template <int MAXB, int NT>
__device__ void ad_row(int k, int b, int tmax, double thresh, const int* __restrict__ a_rowptr,
                       const int* __restrict__ a_col, const double* __restrict__ a_vals, int* __restrict__ out_cols,
                       int* __restrict__ out_cnt, double* base, double* __restrict__ Ybuf, int* plist, int* cand,
                       double* gain, double* part, int* sh, int* err) {
    const int lane = threadIdx.x;
    const int NB = (NT / 64) * (64 / b);
    const int Mmax = (tmax - 1) * b;   // L, Y_k and Y_c never grow past t_max - 1 blocks
    const int bb = b * b;
    AdRegion R = ad_region(base, Mmax, b, NB);
    // sh[0] = ncand, sh[1] = m, sh[2] = c*, sh[3] = flag, sh[4] = continue
    // init: H_kk = A_kk, candidates = pattern of A_k left of the diagonal
    const int ekk = find_block(a_rowptr, a_col, k, k);
    for (int e = lane; e < bb; e += NT) R.Hkk[e] = ekk >= 0 ? a_vals[(int64_t)ekk * bb + e] : 0.0;
    if (lane == 0) {
        int nc = 0;
        for (int e = a_rowptr[k]; e < a_rowptr[k + 1]; ++e) {
            int c = a_col[e];
            if (c < k && nc < AD_MAXC) cand[nc++] = c;
        }
        sh[0] = nc;
        sh[1] = 0;
    }
    __syncthreads();
    bool ok = small_chol(R.Hkk, R.LH, b, lane, sh + 3);
    if (!ok) {
        if (lane == 0) atomicMin(err, k);
    }
    for (int t = 0; t < tmax && ok; ++t) {
        const int nc = sh[0];
        const int m = sh[1];
        const int M = m * b;
        if (nc == 0) break;
        for (int s0 = 0; s0 < nc; s0 += NB) {
            ad_batch<MAXB, NT>(k, b, NB, m, M, plist, cand, s0, min(NB, nc - s0), a_rowptr, a_col, a_vals, R, Ybuf,
                               gain, part, sh + 3, err);
            if (!sh[3]) { ok = false; break; }
        }
        if (!ok) break;
        // selection: best gain, ties to the smallest block index
        if (lane == 0) {
            double gmax = -1e300;
            for (int i = 0; i < nc; ++i) gmax = fmax(gmax, gain[i]);
            const double lim = gmax - AD_TIE_REL * fabs(gmax);
            int best = -1;
            for (int i = 0; i < nc; ++i)
                if (gain[i] >= lim && (best < 0 || cand[i] < cand[best])) best = i;
            sh[2] = best;
            sh[4] = (gmax > thresh) ? 1 : 0;
        }
        __syncthreads();
        if (!sh[4]) break;
        const int bi = sh[2];
        if (t == tmax - 1) {
            // last step: the pattern grows, nothing else is needed afterwards
            if (lane == 0) {
                plist[m] = cand[bi];
                sh[1] = m + 1;
            }
            __syncthreads();
            break;
        }
        // recompute Y, L_W and U for c* alone (group 0)
        ad_batch<MAXB, NT>(k, b, NB, m, M, plist, cand, bi, 1, a_rowptr, a_col, a_vals, R, Ybuf, nullptr, part,
                           sh + 3, err);
        if (!sh[3]) { ok = false; break; }
        // extend L by [Y_c*^T, L_W], Y_k by U, H_kk -= U^T U
        for (int t2 = lane; t2 < b * (M + b); t2 += NT) {
            int r = t2 / (M + b), i = t2 - r * (M + b);
            double v;
            if (i < M) v = Ybuf[(int64_t)i * NT + r];
            else v = (i - M <= r) ? R.W[r * b + (i - M)] : 0.0;
            if (i <= M + r) R.L[atri(M + r) + i] = v;
        }
        for (int e = lane; e < bb; e += NT) R.Yk[(int64_t)M * b + e] = R.U[e];
        __syncthreads();
        for (int e = lane; e < bb; e += NT) {
            int r = e / b, s = e - r * b;
            double acc = 0.0;
            for (int q = 0; q < b; ++q) acc += R.U[q * b + r] * R.U[q * b + s];
            R.Hkk[e] -= acc;
        }
        __syncthreads();
        ok = small_chol(R.Hkk, R.LH, b, lane, sh + 3);
        if (!ok) {
            if (lane == 0) atomicMin(err, k);
            break;
        }
        // update the pattern and the candidate list
        if (lane == 0) {
            const int cstar = cand[bi];
            plist[m] = cstar;
            sh[1] = m + 1;
            int ncand = nc;
            for (int i = bi; i + 1 < ncand; ++i) cand[i] = cand[i + 1];
            --ncand;
            for (int e = a_rowptr[cstar]; e < a_rowptr[cstar + 1]; ++e) {
                const int c = a_col[e];
                if (c >= k) break;
                bool inp = false;
                for (int q = 0; q <= m; ++q) inp |= plist[q] == c;
                if (inp) continue;
                int pos = 0;
                while (pos < ncand && cand[pos] < c) ++pos;
                if (pos < ncand && cand[pos] == c) continue;
                if (ncand >= AD_MAXC) { atomicMin(err, k); break; }
                for (int i = ncand; i > pos; --i) cand[i] = cand[i - 1];
                cand[pos] = c;
                ++ncand;
            }
            sh[0] = ncand;
        }
        __syncthreads();
    }
    // output: sorted P_k (P~ and k)
    if (lane == 0) {
        const int m = sh[1];
        int tmp[AD_MAXP];
        for (int i = 0; i < m; ++i) tmp[i] = plist[i];
        tmp[m] = k;
        for (int i = 1; i <= m; ++i) {
            int v = tmp[i], j = i - 1;
            while (j >= 0 && tmp[j] > v) { tmp[j + 1] = tmp[j]; --j; }
            tmp[j + 1] = v;
        }
        for (int i = 0; i <= m; ++i) out_cols[(int64_t)k * (tmax + 1) + i] = tmp[i];
        out_cnt[k] = m + 1;
    }
    __syncthreads();
}

template <int MAXB, int NT>
__global__ __launch_bounds__(NT) void k_adaptive(int64_t nb, int b, int tmax, double thresh,
                                                 const int* __restrict__ a_rowptr, const int* __restrict__ a_col,
                                                 const double* __restrict__ a_vals, int* __restrict__ out_cols,
                                                 int* __restrict__ out_cnt, int region_lds, int ybuf_lds,
                                                 int64_t region_doubles, double* scratch, int64_t gstride,
                                                 int* counter, int* err) {
    extern __shared__ double lds[];
    __shared__ int plist[AD_MAXP];
    __shared__ int cand[AD_MAXC];
    __shared__ double gain[AD_MAXC];
    __shared__ int sh[8];
    __shared__ int next;
    __shared__ double part[NT];
    double* greg = scratch + (int64_t)blockIdx.x * gstride;
    double* reg = region_lds ? lds : greg;
    double* Ybuf = ybuf_lds ? lds + (region_lds ? region_doubles : 0) : greg + (region_lds ? 0 : region_doubles);
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int64_t row = next;
        __syncthreads();
        if (row >= nb) break;
        ad_row<MAXB, NT>((int)row, b, tmax, thresh, a_rowptr, a_col, a_vals, out_cols, out_cnt, reg, Ybuf, plist, cand,
                     gain, part, sh, err);
    }
}

chf_pattern_s* adaptive_pattern_impl(chf_bsr A, int tmax, double tau, hipStream_t s) {
    CHF_CHECK(tmax >= 0 && tmax + 1 <= AD_MAXP, CHF_EINVAL, "tmax must be in [0, 31]");
    CHF_CHECK(tau > 0.0 && tau <= 1.0, CHF_EINVAL, "tau must be in (0, 1]");
    const int64_t nb = A->nb;
    const int b = A->b;
    std::unique_ptr<chf_pattern_s> P(new chf_pattern_s);
    P->nb = nb;
    P->rowptr.assign(nb + 1, 0);
    if (tmax == 0 || nb == 0) {
        for (int64_t k = 0; k < nb; ++k) {
            P->colidx.push_back((int32_t)k);
            P->rowptr[k + 1] = k + 1;
        }
        return P.release();
    }
    constexpr int NT = 64;   // one wavefront per row: wider workgroups lose more to barriers than they gain
    const int NB = (NT / 64) * (64 / b);
    const int Mmax = (tmax - 1) * b;
    const int64_t region = ad_region_doubles(Mmax, b, NB);
    const size_t region_bytes = (size_t)region * 8;
    const size_t ybuf_bytes = (size_t)Mmax * NT * 8;
    int dev = 0, lim = 0;
    CHF_HIP(hipGetDevice(&dev));
    CHF_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t static_lds = AD_MAXP * 4 + AD_MAXC * 12 + 64 + NT * 8;
    const size_t avail = (size_t)lim > static_lds + 512 ? (size_t)lim - static_lds - 512 : 0;
    // placement: everything in LDS if it fits, else the right-hand-side buffer
    // (the operand of the forward substitutions) in LDS, else both in a global slot
    // LDS only while at least 4 workgroups still fit on a CU: occupancy
    // matters more than latency for this kernel (measured at 512^2, b = 10:
    // t_max 8 takes 1.19 s with everything in a global slot at 8 workgroups
    // per CU, 1.74 s with the right-hand sides in LDS at 3 per CU)
    const size_t occ = (size_t)lim / 4 > static_lds + 512 ? (size_t)lim / 4 - static_lds - 512 : 0;
    bool region_lds = region_bytes + ybuf_bytes <= occ;
    bool ybuf_lds = region_lds || ybuf_bytes <= occ;
    if (const char* env = std::getenv("CHF_ADAPTIVE_PLACEMENT")) {   // tuning knob: "global" or "region"
        if (std::string(env) == "global") region_lds = ybuf_lds = false;
        if (std::string(env) == "region" && region_bytes <= avail) { region_lds = true; ybuf_lds = false; }
    }
    const size_t dyn = (region_lds ? region_bytes : 0) + (ybuf_lds && !region_lds ? ybuf_bytes : 0) +
                       (region_lds && ybuf_lds ? ybuf_bytes : 0);
    const int cus = device_cu_count();
    const int per_cu = std::max<int>(1, (int)std::min<size_t>(8, (size_t)lim / (dyn + static_lds + 512)));
    const int64_t grid = std::min<int64_t>((int64_t)cus * per_cu, nb);
    const int64_t stride = std::max<int64_t>(1, (region_lds ? 0 : region) + (ybuf_lds ? 0 : (int64_t)Mmax * NT));
    DevBuf<double> scratch((size_t)grid * stride);
    CHF_CHECK(b <= 32, CHF_EINVAL, "adaptive pattern supports block sizes up to 32");
    auto kern = b == 10 ? k_adaptive<10, NT> : b == 21 ? k_adaptive<21, NT> : k_adaptive<32, NT>;
    if (dyn > 64 * 1024)
        CHF_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    DevBuf<int> out_cols((size_t)nb * (tmax + 1)), out_cnt(nb), flags(2);
    int init[2] = {0, INT32_MAX};
    flags.upload(init, 2, s);
    const double thresh = -std::log(tau) + AD_GAIN_EPS;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), dyn, s, nb, b, tmax, thresh, A->d_rowptr.p,
                       A->d_colidx.p, A->d_vals.p, out_cols.p, out_cnt.p, (int)region_lds, (int)ybuf_lds, region,
                       scratch.p, stride, flags.p, flags.p + 1);
    CHF_LAUNCH_CHECK();
    std::vector<int> hcols((size_t)nb * (tmax + 1)), hcnt(nb);
    int hflags[2];
    out_cols.download(hcols.data(), hcols.size(), s);
    out_cnt.download(hcnt.data(), nb, s);
    flags.download(hflags, 2, s);
    CHF_HIP(hipStreamSynchronize(s));
    if (hflags[1] != INT32_MAX)
        fail(CHF_ENOTSPD, "adaptive pattern: local matrices of block row " + std::to_string(hflags[1]) +
                              " are not positive definite (or the candidate list overflowed)");
    for (int64_t k = 0; k < nb; ++k) {
        CHF_CHECK(hcnt[k] >= 1 && hcnt[k] <= tmax + 1, CHF_EDEVICE, "adaptive pattern: bad row count");
        for (int i = 0; i < hcnt[k]; ++i) P->colidx.push_back(hcols[(size_t)k * (tmax + 1) + i]);
        P->rowptr[k + 1] = (int64_t)P->colidx.size();
    }
    return P.release();
}

}  // namespace chf

extern "C" int chf_pattern_adaptive(chf_bsr A, int tmax, double tau, chf_pattern* out) {
    return chf::guarded([&] {
        CHF_CHECK(A && out, CHF_EINVAL, "NULL argument");
        *out = chf::adaptive_pattern_impl(A, tmax, tau, 0);
    });
}

// ------------------------------------------------ learned-pattern features --
// For block row k and each candidate c of the strictly lower part of the row
// pattern of A^2, four features: ||A_kc||_F / sqrt(||A_kk||_F ||A_cc||_F),
// ||A_cc^{-1} A_ck||_F, the Euclidean distance of the patch centres, and the
// one-step gain -log rho_c at P_k = {k} (Lemma 2.4 with P~ empty:
// H_kk = A_kk, H_kc = A_kc, W_c = A_cc). The gain uses the same batch code as
// Algorithm 1.
namespace chf {

template <int MAXB>
__global__ __launch_bounds__(64) void k_mlp_features(int64_t nb, int b, int nx, int ny,
                                                     const int* __restrict__ a_rowptr, const int* __restrict__ a_col,
                                                     const double* __restrict__ a_vals,
                                                     const int64_t* __restrict__ c_rowptr,
                                                     const int* __restrict__ c_col, float* __restrict__ feats,
                                                     double* scratch, int64_t region_stride, int* err) {
    extern __shared__ double lds[];
    __shared__ double gain[AD_MAXC];
    __shared__ double part[64];
    __shared__ int sh[8];
    const int lane = threadIdx.x;
    const int NB = 64 / b;
    const int bb = b * b;
    double* base = scratch + (int64_t)blockIdx.x * region_stride;
    AdRegion R = ad_region(lds, 0, b, NB);
    for (int64_t k = blockIdx.x; k < nb; k += gridDim.x) {
        const int ekk = find_block(a_rowptr, a_col, (int)k, (int)k);
        for (int e = lane; e < bb; e += 64) R.Hkk[e] = ekk >= 0 ? a_vals[(int64_t)ekk * bb + e] : 0.0;
        __syncthreads();
        if (!small_chol(R.Hkk, R.LH, b, lane, sh + 3)) {
            if (lane == 0) atomicMin(err, (int)k);
            continue;
        }
        double nkk = 0.0;
        for (int e = 0; e < bb; ++e) nkk += R.Hkk[e] * R.Hkk[e];
        nkk = sqrt(nkk);
        const int64_t c0 = c_rowptr[k];
        const int nc = (int)(c_rowptr[k + 1] - c0);
        const int* cand = c_col + c0;
        const int kx = (int)(k % nx), ky = (int)((k / nx) % ny), kz = (int)(k / ((int64_t)nx * ny));
        for (int s0 = 0; s0 < nc; s0 += NB) {
            const int cnt = min(NB, nc - s0);
            ad_batch<MAXB, 64>((int)k, b, NB, 0, 0, nullptr, cand, s0, cnt, a_rowptr, a_col, a_vals, R, base, gain,
                               part, sh + 3, err);
            if (!sh[3]) break;
            const int ci = lane / b, col = lane - ci * b;
            const bool act = ci < cnt && lane < NB * b;
            // V = L_W^{-T} U = A_cc^{-1} A_ck, column col; partial sums of squares
            double sv = 0.0, skc = 0.0, scc = 0.0;
            if (act) {
                const double* W = R.W + ci * bb;
                const double* U = R.U + ci * bb;
                double* V = R.X + ci * bb;
                for (int i = b - 1; i >= 0; --i) {
                    double s = U[i * b + col];
                    for (int q = i + 1; q < b; ++q) s -= W[q * b + i] * V[q * b + col];
                    V[i * b + col] = s / W[i * b + i];
                    sv += V[i * b + col] * V[i * b + col];
                }
                const int c = cand[s0 + ci];
                const int ekc = find_block(a_rowptr, a_col, (int)k, c);
                const int ecc = find_block(a_rowptr, a_col, c, c);
                for (int rr = 0; rr < b; ++rr) {
                    double v1 = ekc >= 0 ? a_vals[(int64_t)ekc * bb + rr * b + col] : 0.0;
                    double v2 = ecc >= 0 ? a_vals[(int64_t)ecc * bb + rr * b + col] : 0.0;
                    skc += v1 * v1;
                    scc += v2 * v2;
                }
            }
            part[lane] = sv;
            __syncthreads();
            double fv = 0.0;
            if (act && col == 0)
                for (int q = 0; q < b; ++q) fv += part[lane + q];
            __syncthreads();
            part[lane] = skc;
            __syncthreads();
            double fkc = 0.0;
            if (act && col == 0)
                for (int q = 0; q < b; ++q) fkc += part[lane + q];
            __syncthreads();
            part[lane] = scc;
            __syncthreads();
            double fcc = 0.0;
            if (act && col == 0) {
                for (int q = 0; q < b; ++q) fcc += part[lane + q];
                const int c = cand[s0 + ci];
                const int cx = c % nx, cy = (c / nx) % ny, cz = c / (nx * ny);
                const double dx = cx - kx, dy = cy - ky, dz = cz - kz;
                float* f = feats + (c0 + s0 + ci) * 4;
                f[0] = (float)(sqrt(fkc) / sqrt(nkk * sqrt(fcc)));
                f[1] = (float)sqrt(fv);
                f[2] = (float)sqrt(dx * dx + dy * dy + dz * dz);
                f[3] = (float)gain[s0 + ci];
            }
            __syncthreads();
        }
    }
}

// strictly lower part of the row pattern of A^2 (host, index work)
void a2_candidates(chf_bsr A, std::vector<int64_t>& rowptr, std::vector<int32_t>& cols) {
    const int64_t nb = A->nb;
    rowptr.assign(nb + 1, 0);
    cols.clear();
    std::vector<int64_t> mark(nb, -1);
    std::vector<int32_t> tmp;
    for (int64_t k = 0; k < nb; ++k) {
        tmp.clear();
        for (int64_t e = A->rowptr[k]; e < A->rowptr[k + 1]; ++e) {
            int64_t j = A->colidx[e];
            for (int64_t f = A->rowptr[j]; f < A->rowptr[j + 1]; ++f) {
                int32_t c = A->colidx[f];
                if (c < k && mark[c] != k) { mark[c] = k; tmp.push_back(c); }
            }
        }
        std::sort(tmp.begin(), tmp.end());
        CHF_CHECK((int64_t)tmp.size() <= AD_MAXC, CHF_EINVAL, "too many candidates in a row");
        cols.insert(cols.end(), tmp.begin(), tmp.end());
        rowptr[k + 1] = (int64_t)cols.size();
    }
}

void mlp_features_impl(chf_bsr A, int nx, int ny, const std::vector<int64_t>& crow, const std::vector<int32_t>& ccol,
                       float* feats, hipStream_t s) {
    const int64_t nb = A->nb;
    const int b = A->b;
    if (nb == 0 || ccol.empty()) return;
    const int NB = 64 / b;
    const size_t region_bytes = (size_t)ad_region_doubles(0, b, NB) * 8;
    DevBuf<int64_t> d_crow(nb + 1);
    DevBuf<int> d_ccol(ccol.size());
    d_crow.upload(crow.data(), nb + 1, s);
    d_ccol.upload(ccol.data(), ccol.size(), s);
    DevBuf<int> err(1);
    int init = INT32_MAX;
    err.upload(&init, 1, s);
    const int64_t grid = std::min<int64_t>((int64_t)device_cu_count() * 8, nb);
    DevBuf<double> scratch(1);
    CHF_CHECK(b <= 32, CHF_EINVAL, "features support block sizes up to 32");
    auto kern = b == 10 ? k_mlp_features<10> : b == 21 ? k_mlp_features<21> : k_mlp_features<32>;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64), region_bytes, s, nb, b, nx, ny, A->d_rowptr.p,
                       A->d_colidx.p, A->d_vals.p, d_crow.p, d_ccol.p, feats, scratch.p, (int64_t)0, err.p);
    CHF_LAUNCH_CHECK();
    int herr = 0;
    err.download(&herr, 1, s);
    CHF_HIP(hipStreamSynchronize(s));
    CHF_CHECK(herr == INT32_MAX, CHF_ENOTSPD, "features: block row " + std::to_string(herr) + " not positive definite");
}

}  // namespace chf

extern "C" int chf_mlp_candidates(chf_bsr A, int64_t* ncand, int64_t* rowptr, int32_t* cols) {
    return chf::guarded([&] {
        CHF_CHECK(A && ncand, CHF_EINVAL, "NULL argument");
        std::vector<int64_t> r;
        std::vector<int32_t> c;
        chf::a2_candidates(A, r, c);
        *ncand = (int64_t)c.size();
        if (rowptr) std::memcpy(rowptr, r.data(), r.size() * 8);
        if (cols) std::memcpy(cols, c.data(), c.size() * 4);
    });
}

extern "C" int chf_mlp_features(chf_bsr A, int32_t nx, int32_t ny, float* feats, hipStream_t stream) {
    return chf::guarded([&] {
        CHF_CHECK(A && feats, CHF_EINVAL, "NULL argument");
        CHF_CHECK(nx >= 1 && ny >= 1 && A->nb % ((int64_t)nx * ny) == 0, CHF_EINVAL, "grid does not match nb");
        std::vector<int64_t> r;
        std::vector<int32_t> c;
        chf::a2_candidates(A, r, c);
        chf::mlp_features_impl(A, nx, ny, r, c, feats, stream);
    });
}
