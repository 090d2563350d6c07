// Adaptive block-FSAI pattern (Algorithm 1 with the ratio of Lemma 2.4) on the
// GPU. Block rows evolve independently (row k of F depends only on A and
// P_k), so one single-wavefront workgroup owns one row for all t_max steps.
//
// For a row k with current pattern P_k = P~ + {k} and a candidate c (c < k,
// c not in P_k, (FA)_kc structurally nonzero, i.e. c in the pattern of some
// row A_j with j in P_k):
//   H_kk = A_kk - A[k,P~] A[P~,P~]^{-1} A[P~,k]   (= (F A F^T)_kk),
//   H_kc = A_kc - A[k,P~] A[P~,P~]^{-1} A[P~,c]   (= (F A)_kc),
//   W_c  = A_cc - A[c,P~] A[P~,P~]^{-1} A[P~,c],
//   rho_c = det(W_c - H_kc^T H_kk^{-1} H_kc) / det(W_c) = det(I - X X^T),
//   X = L_W^{-1} H_kc^T L_H^{-T}   (W_c = L_W L_W^T, H_kk = L_H L_H^T),
//   g_c = -log rho_c, evaluated by a Cholesky of I - X X^T with log1p pivots.
// The best candidate c* (largest g; ties within a relative 1e-9 of the best go
// to the smallest block index) enters when g* > -log(tau) + 1e-12.
//
// Two evaluations live here. ad_batch forms H_kc and W_c from scratch for a
// batch of candidates (Y_c = L^{-1} A[P~,c] with L = chol(A[P~,P~])); the
// learned-pattern features use it with P~ empty. The pattern kernel
// (ai_row) keeps A[P~,P~]^{-1} and every candidate's H_kc, W_c across the
// steps and updates them when a block enters (described at ai_row).
#include <algorithm>
#include <climits>
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

// ------------------------------------------------------ Algorithm 1 rows --
// Incremental form. State of a row, with P~ in insertion order and
// M = b |P~|:
//   Kinv = A[P~,P~]^{-1}                       (packed lower, M x M)
//   H_kk = A_kk - A[k,P~] Kinv A[P~,k],  L_H = chol(H_kk)
//   per candidate c:  W_c  = A_cc - A[c,P~] Kinv A[P~,c]
//                     H_kc = A_kc - A[k,P~] Kinv A[P~,c]
//                     the (position in P~, block index of A_jc) of every
//                     j in P~ with A_jc structurally nonzero.
// Adding c* (S = W_c* = L_S L_S^T is the Schur complement of A[P~,P~] in
// A[P~ + c*, P~ + c*]) changes them by the bordering identities
//   V = Kinv A[P~,c*],  U = L_S^{-1} H_kc*^T,  H_kk -= U^T U,
//   E_c = A_c*c - V^T A[P~,c],  e_c = L_S^{-1} E_c,
//   W_c -= e_c^T e_c,  H_kc -= U^T e_c,
//   Kinv <- [[Kinv + Vt Vt^T, -Vt L_S^{-1}], [-L_S^{-T} Vt^T, L_S^{-T} L_S^{-1}]],
//   Vt = V L_S^{-T},
// so a step costs O(b^3) per candidate (A[P~,c] has few nonzero blocks)
// plus O(M^2 b) once, instead of a triangular solve with L per candidate.
// Candidates that c* brings in start from W_c = A_cc, H_kc = A_kc (their
// A[P~,c] was empty) and receive the same update.

__host__ __device__ inline int64_t ai_tri(int64_t i) { return i * (i + 1) / 2; }

__device__ inline int64_t kidx(int i, int j) { return i >= j ? ai_tri(i) + j : ai_tri(j) + i; }

struct AiState {
    double* kinv;   // atri(Mmax)
    double* V;      // Mmax x b
    double* Vt;     // Mmax x b
    double* W;      // cap x b x b
    double* H;      // cap x b x b
    double* gain;   // cap
    int* cand;      // cap
    int* nzn;       // cap
    int* ecs;       // cap: block index of A_c*c for the block added last (-1 if none)
    int* nzp;       // cap x AD_MAXP
    int* nze;       // cap x AD_MAXP
};

__host__ __device__ inline int64_t ai_global_doubles(int Mmax, int b, int cap) {
    const int64_t ints = (int64_t)cap * (3 + 2 * AD_MAXP);
    return ai_tri(Mmax) + 2 * (int64_t)Mmax * b + 2 * (int64_t)cap * b * b + cap + (ints + 1) / 2;
}

// LDS: the row's b x b work matrices with the pivot buffers of group_chol,
// then one buffer per group of b lanes (the group's own pivot buffers only
// where its Cholesky factors run in LDS, i.e. for block sizes not fixed at
// compile time).
__host__ __device__ inline int64_t ai_small_doubles(int b) { return 5 * (int64_t)b * b + 4 * b; }
__host__ __device__ inline int64_t ai_group_doubles(int b, bool reg) {
    return 3 * (int64_t)b * b + (reg ? b : 3 * b);
}

__host__ __device__ inline int64_t ai_lds_doubles(int b, int maxrow, bool reg) {
    const int NB = 64 / b;
    return ai_small_doubles(b) + (int64_t)NB * ai_group_doubles(b, reg) + (maxrow + 1) / 2;
}

// threadIdx.x behind an empty asm: values derived from it are formed where a
// phase uses them instead of being hoisted out of the row and step loops,
// which would keep every phase's lane addresses live through all the others.
__device__ __forceinline__ int ai_lane() {
    int l = threadIdx.x;
    asm volatile("" : "+v"(l));
    return l;
}

// Cholesky of a b x b SPD matrix held row-major in LDS (Mx) by the b lanes of
// one group: lane r owns row r and ends with row r of the factor in
// Mx[r][0..r] and 1 / L_rr in rd[r]. One barrier per pivot: the pivot column
// is published to cb (two alternating buffers of b doubles) and every lane
// forms its own multipliers. The loops stay rolled so that the square root
// and the division are emitted once. All lanes of the workgroup call it; it
// ends with a barrier.
__device__ inline void group_chol(double* Mx, double* rd, double* cb, int b, int r, bool act, bool& ok) {
#pragma unroll 1
    for (int q = 0; q < b; ++q) {
        double* c = cb + (q & 1) * b;
        if (act && r >= q) c[r] = Mx[r * b + q];
        __syncthreads();
        if (act && r >= q) {
            const double d = c[q];
            ok = ok && d > 0.0 && isfinite(d);
            const double sd = sqrt(fmax(d, 1e-300));
            const double isd = 1.0 / sd;
            const double cr = c[r] * isd;   // L_rq
            Mx[r * b + q] = r == q ? sd : cr;
            if (r == q) rd[r] = isd;
            const double crs = cr * isd;    // c_r / d
#pragma unroll 1
            for (int j = q + 1; j <= r; ++j) Mx[r * b + j] -= crs * c[j];
        }
    }
    __syncthreads();
}

// One pass over the candidates in slots [s0, s0 + cnt): apply the pending
// update of the block added last (when `pending`), then g_c = -log rho_c.
// Lane (ci, r) works on candidate s0 + ci, row/column r of its blocks. BC > 0
// fixes the block size at compile time.
template <int MAXB, int BC>
__device__ __forceinline__ void ai_batch(int k, int b, int s0, int cnt, bool pending, int cstar, int mold,
                                         const int* __restrict__ a_rowptr, const int* __restrict__ a_col,
                                         const double* __restrict__ a_vals, const AiState& S, const double* V,
                                         const double* LSinv, const double* U, const double* LH,
                                         const double* LHrd, double* gbufs, int* flag) {
    if (BC > 0) b = BC;
    const int lane = ai_lane();
    const int bb = b * b;
    const int ci = lane / b, r = lane - ci * b;
    const bool act = ci < cnt;
    const int slot = s0 + ci;
    double* cb = gbufs + (act ? ci : 0) * ai_group_doubles(b, BC > 0);   // pivot buffers (LDS Cholesky)
    double* rd = BC > 0 ? cb : cb + 2 * b;   // 1 / diagonal of L_W
    double* BW = rd + b;       // W_c by rows, then L_W
    double* B1 = BW + bb;      // e_c by columns, then Z by columns, then N by rows
    double* BX = B1 + bb;      // X by columns
    double w[MAXB], h[MAXB];
    __syncthreads();
    if (act) {
#pragma unroll
        for (int i = 0; i < MAXB; ++i)
            if (i < b) {
                w[i] = S.W[(int64_t)slot * bb + i * b + r];
                h[i] = S.H[(int64_t)slot * bb + i * b + r];
            }
    }
    if (pending) {
        double et[MAXB], e[MAXB];
        int ecs = -1, nn = 0;
        // lane r of a group holds list entry r (entries past b are loaded
        // where they are used), loaded with the rest of the slot's state
        int my_pos = 0, my_ea = 0;
        if (act) {
            ecs = S.ecs[slot];
            nn = S.nzn[slot];
            my_pos = S.nzp[(int64_t)slot * AD_MAXP + r];
            my_ea = S.nze[(int64_t)slot * AD_MAXP + r];
#pragma unroll
            for (int i = 0; i < MAXB; ++i)
                if (i < b) e[i] = ecs >= 0 ? a_vals[(int64_t)ecs * bb + i * b + r] : 0.0;
        }
        // E_c -= V_j^T A_jc over the blocks j of P~ next to c, two list entries
        // per pass: each V_j block (b x b) is staged through the group's LDS
        // buffers by rows (the trip count is made uniform across the wavefront
        // for the barriers); lane r loads row r of V_j and column r of A_jc,
        // both entries' loads issued together
        int nmax = act ? nn : 0;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) nmax = max(nmax, __shfl_xor(nmax, o, 64));
        const int g0l = lane - r;
        auto entry = [&](int t, int& pos, int& ea) {
            pos = __shfl(my_pos, g0l + min(t, b - 1), 64);
            ea = __shfl(my_ea, g0l + min(t, b - 1), 64);
            if (t >= b && act && t < nn) {
                pos = S.nzp[(int64_t)slot * AD_MAXP + t];
                ea = S.nze[(int64_t)slot * AD_MAXP + t];
            }
        };
#pragma unroll 1
        for (int t = 0; t < nmax; t += 2) {
            int pos0, ea0, pos1, ea1;
            entry(t, pos0, ea0);
            entry(t + 1, pos1, ea1);
            const bool live0 = act && t < nn, live1 = act && t + 1 < nn;
            double vr0[MAXB], ac0[MAXB], vr1[MAXB], ac1[MAXB];
            if (live0) {
                const double* vp = V + (int64_t)(pos0 * b + r) * b;
                const double* ap = a_vals + (int64_t)ea0 * bb + r;
#pragma unroll
                for (int i = 0; i < MAXB; ++i)
                    if (i < b) {
                        vr0[i] = vp[i];
                        ac0[i] = ap[i * b];
                    }
            }
            if (live1) {
                const double* vp = V + (int64_t)(pos1 * b + r) * b;
                const double* ap = a_vals + (int64_t)ea1 * bb + r;
#pragma unroll
                for (int i = 0; i < MAXB; ++i)
                    if (i < b) {
                        vr1[i] = vp[i];
                        ac1[i] = ap[i * b];
                    }
            }
            if (live0) {
#pragma unroll
                for (int i = 0; i < MAXB; ++i)
                    if (i < b) BX[r * b + i] = vr0[i];
            }
            if (live1) {
#pragma unroll
                for (int i = 0; i < MAXB; ++i)
                    if (i < b) BW[r * b + i] = vr1[i];
            }
            __syncthreads();
            if (live0) {
#pragma unroll
                for (int q = 0; q < MAXB; ++q)
                    if (q < b) {
#pragma unroll
                        for (int i = 0; i < MAXB; ++i)
                            if (i < b) e[i] -= BX[q * b + i] * ac0[q];
                    }
            }
            if (live1) {
#pragma unroll
                for (int q = 0; q < MAXB; ++q)
                    if (q < b) {
#pragma unroll
                        for (int i = 0; i < MAXB; ++i)
                            if (i < b) e[i] -= BW[q * b + i] * ac1[q];
                    }
            }
            __syncthreads();
        }
        if (act) {
#pragma unroll
            for (int i = 0; i < MAXB; ++i)
                if (i < b) {
                    double s = 0.0;
#pragma unroll
                    for (int q = 0; q < MAXB; ++q)
                        if (q <= i) s += LSinv[i * b + q] * e[q];
                    et[i] = s;
                    B1[i * b + r] = s;
                }
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int i = 0; i < MAXB; ++i)
                if (i < b) {
                    double sw = 0.0, sh = 0.0;
#pragma unroll
                    for (int q = 0; q < MAXB; ++q)
                        if (q < b) {
                            sw += B1[q * b + i] * et[q];
                            sh += U[q * b + i] * et[q];
                        }
                    w[i] -= sw;
                    h[i] -= sh;
                    S.W[(int64_t)slot * bb + i * b + r] = w[i];
                    S.H[(int64_t)slot * bb + i * b + r] = h[i];
                }
            if (r == 0 && ecs >= 0) {
                S.nzp[(int64_t)slot * AD_MAXP + nn] = mold;
                S.nze[(int64_t)slot * AD_MAXP + nn] = ecs;
                S.nzn[slot] = nn + 1;
            }
        }
    }
    // L_W = chol(W_c); W_c is symmetric, so column r is row r
    bool ok = true;
    const int g0l = lane - r;
    if constexpr (BC > 0) {
        // in registers: lane r keeps row r and takes the pivot column from the
        // group by shuffles; the arithmetic is group_chol's, element by element
        double rdv = 0.0;
#pragma unroll
        for (int q = 0; q < MAXB; ++q)
            if (q < b) {
                const double cr = w[q];
                const double d = __shfl(cr, g0l + q, 64);
                if (r >= q) ok = ok && d > 0.0 && isfinite(d);
                const double sd = sqrt(fmax(d, 1e-300));
                const double isd = 1.0 / sd;
                const double lrq = cr * isd;
                const double crs = lrq * isd;
#pragma unroll
                for (int j = q + 1; j < MAXB; ++j)
                    if (j < b) {
                        const double cj = __shfl(cr, g0l + j, 64);
                        if (j <= r) w[j] -= crs * cj;
                    }
                if (r >= q) w[q] = r == q ? sd : lrq;
                if (r == q) rdv = isd;
            }
        if (act) {
#pragma unroll
            for (int i = 0; i < MAXB; ++i)
                if (i < b) BW[r * b + i] = w[i];
            rd[r] = rdv;
        }
    } else {
        if (act) {
#pragma unroll
            for (int i = 0; i < MAXB; ++i)
                if (i < b) BW[r * b + i] = w[i];
        }
        group_chol(BW, rd, cb, b, r, act, ok);
    }
    if (act) {
        // Z = L_H^{-1} H_kc, column r
        double z[MAXB];
#pragma unroll
        for (int i = 0; i < MAXB; ++i)
            if (i < b) {
                double s = h[i];
#pragma unroll
                for (int q = 0; q < MAXB; ++q)
                    if (q < i) s -= LH[i * b + q] * z[q];
                z[i] = s * LHrd[i];
                B1[i * b + r] = z[i];
            }
    }
    __syncthreads();
    if (act) {
        // X = L_W^{-1} Z^T, column r (X = L_W^{-1} H_kc^T L_H^{-T})
        double x[MAXB];
#pragma unroll
        for (int i = 0; i < MAXB; ++i)
            if (i < b) {
                double s = B1[r * b + i];
#pragma unroll
                for (int q = 0; q < MAXB; ++q)
                    if (q < i) s -= BW[i * b + q] * x[q];
                x[i] = s * rd[i];
                BX[i * b + r] = x[i];
            }
    }
    __syncthreads();
    // row r of N = X X^T, lower part (in registers for compile-time b)
    double nrow[MAXB];
#pragma unroll
    for (int s = 0; s < MAXB; ++s) nrow[s] = 0.0;
    if (act) {
        double xr[MAXB];
#pragma unroll
        for (int q = 0; q < MAXB; ++q)
            if (q < b) xr[q] = BX[r * b + q];
#pragma unroll
        for (int s = 0; s < MAXB; ++s)
            if (s < b && s <= r) {
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < MAXB; ++q)
                    if (q < b) acc += xr[q] * BX[s * b + q];
                if constexpr (BC > 0) nrow[s] = acc;
                else B1[r * b + s] = acc;
            }
    }
    // -log det(I - N): Cholesky of I - N carried on N (the pivot of step q is
    // 1 - s_q with s_q the current N_qq, logged as log1p(-s_q)); every lane
    // sees every pivot and accumulates the sum itself
    double lg = 0.0;
    if constexpr (BC > 0) {
        // in registers, the pivot column by shuffles (same arithmetic)
#pragma unroll
        for (int q = 0; q < MAXB; ++q)
            if (q < b) {
                const double c0 = nrow[q];
                const double sq = __shfl(c0, g0l + q, 64);
                ok = ok && sq < 1.0;
                lg += log1p(-sq);
                const double cr = c0 / fmax(1.0 - sq, 1e-300);
#pragma unroll
                for (int j = q + 1; j < MAXB; ++j)
                    if (j < b) {
                        const double cj = __shfl(c0, g0l + j, 64);
                        if (r > q && j <= r) nrow[j] += cr * cj;
                    }
            }
    } else
#pragma unroll 1
    for (int q = 0; q < b; ++q) {
        double* c = cb + (q & 1) * b;
        if (act && r >= q) c[r] = B1[r * b + q];
        __syncthreads();
        if (act) {
            const double sq = c[q];
            ok = ok && sq < 1.0;
            lg += log1p(-sq);
            if (r > q) {
                const double cr = c[r] / fmax(1.0 - sq, 1e-300);
#pragma unroll 1
                for (int j = q + 1; j <= r; ++j) B1[r * b + j] += cr * c[j];
            }
        }
    }
    if (act && r == 0) S.gain[slot] = -lg;
    if (act && !ok) *flag = 0;
}

// W_c = A_cc, H_kc = A_kc for the candidates in slots [s0, s1): one search
// of row c and row k per candidate, then the blocks are copied by all lanes.
__device__ inline void ai_init_slots(int k, int b, int s0, int s1, const int* __restrict__ a_rowptr,
                                     const int* __restrict__ a_col, const double* __restrict__ a_vals,
                                     const AiState& S, int* tmp_a, int* tmp_b) {
    const int lane = ai_lane();
    const int bb = b * b;
#pragma unroll 1
    for (int c0 = s0; c0 < s1; c0 += 64) {
        const int n = min(64, s1 - c0);
        if (lane < n) {
            const int c = S.cand[c0 + lane];
            tmp_a[lane] = find_block(a_rowptr, a_col, c, c);
            tmp_b[lane] = find_block(a_rowptr, a_col, k, c);
        }
        __syncthreads();
        // four elements per pass, their loads issued together
#pragma unroll 1
        for (int t0 = lane; t0 < n * bb; t0 += 256) {
            double wv[4], hv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + 64 * u;
                wv[u] = hv[u] = 0.0;
                if (t < n * bb) {
                    const int sl = t / bb, e = t - sl * bb;
                    const int ecc = tmp_a[sl], ekc = tmp_b[sl];
                    if (ecc >= 0) wv[u] = a_vals[(int64_t)ecc * bb + e];
                    if (ekc >= 0) hv[u] = a_vals[(int64_t)ekc * bb + e];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + 64 * u;
                if (t < n * bb) {
                    const int sl = t / bb, e = t - sl * bb;
                    S.W[(int64_t)(c0 + sl) * bb + e] = wv[u];
                    S.H[(int64_t)(c0 + sl) * bb + e] = hv[u];
                }
            }
        }
        __syncthreads();
    }
}

// P0 (Algorithm 1's initial pattern): when p0_rowptr is given, the blocks of
// row k of P0 other than k enter first, in ascending order, through the same
// bordering update as an adaptive choice (a block that is not yet a candidate
// is structurally decoupled from the current P~, so its W = A_cc, H_kc = 0 are
// exact and it is appended as one); the t_max adaptive steps follow.
template <int MAXB, int BC>
__device__ __forceinline__ void ai_row(int k, int b, int tmax, double thresh, int cap, const int* __restrict__ a_rowptr,
                       const int* __restrict__ a_col, const double* __restrict__ a_vals,
                       const int* __restrict__ p0_rowptr, const int* __restrict__ p0_col, int out_stride,
                       int* __restrict__ out_cols,
                       int* __restrict__ out_cnt, const AiState& S, double* sm, double* gbufs, int* mark,
                       int* plist, int* tmp_a, int* tmp_b, int* sh, int* err) {
    if (BC > 0) b = BC;
    const int lane = threadIdx.x;
    const int bb = b * b;
    const int NB = 64 / b;
    double* Hkk = sm;
    double* LH = Hkk + bb;
    double* LS = LH + bb;
    double* LSinv = LS + bb;
    double* U = LSinv + bb;
    double* LHrd = U + bb;      // 1 / diagonal of L_H
    double* LSrd = LHrd + b;    // 1 / diagonal of L_S
    double* scb = LSrd + b;     // pivot buffers of the row's own factorisations
    const bool g0 = lane < b;   // group 0 does the single b x b factorisations
    const int r = lane;
    // H_kk = A_kk, L_H; candidates: A_kc != 0, c < k, with W_c = A_cc, H_kc = A_kc
    const int ekk = find_block(a_rowptr, a_col, k, k);
    #pragma unroll 1
    for (int e = lane; e < bb; e += 64) Hkk[e] = ekk >= 0 ? a_vals[(int64_t)ekk * bb + e] : 0.0;
    int ncand = 0;
    {
        const int r0 = a_rowptr[k], r1 = a_rowptr[k + 1];
        #pragma unroll 1
        for (int base = r0; base < r1; base += 64) {
            const int e = base + lane;
            const bool f = e < r1 && a_col[e] < k;
            const unsigned long long m = __ballot(f);
            if (f) {
                const int slot = ncand + __popcll(m & ((1ull << lane) - 1));
                if (slot < cap) {
                    S.cand[slot] = a_col[e];
                    S.nzn[slot] = 0;
                }
            }
            ncand += __popcll(m);
        }
    }
    if (lane == 0) sh[3] = 1;
    __syncthreads();
    if (ncand > cap) {
        if (lane == 0) atomicMin(err, k);
        ncand = 0;
    }
    ai_init_slots(k, b, 0, ncand, a_rowptr, a_col, a_vals, S, tmp_a, tmp_b);
    bool ok = true;
    if (g0)
#pragma unroll 1
        for (int j = 0; j < b; ++j) LH[r * b + j] = Hkk[r * b + j];
    group_chol(LH, LHrd, scb, b, r, g0, ok);
    if (g0 && !ok) sh[3] = 0;
    __syncthreads();
    if (!sh[3]) {
        if (lane == 0) atomicMin(err, k);
    }
    int m = 0;
    bool pending = false;
    int cstar = -1;
    const int* forced = nullptr;
    int nforced = 0;
    if (p0_rowptr) {
        forced = p0_col + p0_rowptr[k];
        nforced = p0_rowptr[k + 1] - p0_rowptr[k] - 1;   // the diagonal is the row's last entry
    }
    const int total = nforced + tmax;
    #pragma unroll 1
    for (int step = 0; step < total && sh[3]; ++step) {
        const int lane = ai_lane(), r = lane;
        const bool g0 = lane < b;
        const bool is_forced = step < nforced;
        if (ncand == 0 && !is_forced) break;
        #pragma unroll 1
        for (int s0 = 0; s0 < ncand; s0 += NB)
            ai_batch<MAXB, BC>(k, b, s0, min(NB, ncand - s0), pending, cstar, m - 1, a_rowptr, a_col, a_vals, S, S.V,
                               LSinv, U, LH, LHrd, gbufs, sh + 3);
        __syncthreads();
        if (!sh[3]) {
            if (lane == 0) atomicMin(err, k);
            break;
        }
        int bs;
        if (is_forced) {
            cstar = forced[step];
            int found = INT_MAX;
            #pragma unroll 1
            for (int i = lane; i < ncand; i += 64)
                if (S.cand[i] == cstar) found = min(found, i);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) found = min(found, __shfl_xor(found, o, 64));
            if (found == INT_MAX) {
                if (ncand >= cap) {
                    if (lane == 0) { atomicMin(err, k); sh[3] = 0; }
                    __syncthreads();
                    break;
                }
                if (lane == 0) {
                    S.cand[ncand] = cstar;
                    S.nzn[ncand] = 0;
                }
                __syncthreads();
                ai_init_slots(k, b, ncand, ncand + 1, a_rowptr, a_col, a_vals, S, tmp_a, tmp_b);
                found = ncand++;
            }
            bs = found;
        } else {
        // selection: largest gain; ties within a relative AD_TIE_REL of it go
        // to the smallest block index
        double gm = -1e300;
        #pragma unroll 1
        for (int i = lane; i < ncand; i += 64) gm = fmax(gm, S.gain[i]);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) gm = fmax(gm, __shfl_xor(gm, o, 64));
        const double lim = gm - AD_TIE_REL * fabs(gm);
        long long best = LLONG_MAX;
        #pragma unroll 1
        for (int i = lane; i < ncand; i += 64)
            if (S.gain[i] >= lim) best = min(best, ((long long)S.cand[i] << 32) | (long long)i);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) best = min(best, (long long)__shfl_xor(best, o, 64));
        if (!(gm > thresh)) break;
        bs = (int)(best & 0xffffffffLL);
        cstar = (int)(best >> 32);
        }
        if (step == total - 1) {
            if (lane == 0) plist[m] = cstar;
            ++m;
            pending = false;
            break;
        }
        const int M = m * b;
        // L_S = chol(W_c*); U = L_S^{-1} H_kc*^T; L_S^{-1}
        {
            if (g0)
#pragma unroll 1
                for (int j = 0; j < b; ++j) LS[r * b + j] = S.W[(int64_t)bs * bb + j * b + r];
            bool okS = true;
            group_chol(LS, LSrd, scb, b, r, g0, okS);
            if (g0 && !okS) sh[3] = 0;
            if (g0) {
                double x[MAXB], u[MAXB];
#pragma unroll
                for (int i = 0; i < MAXB; ++i)
                    if (i < b) {
                        double sx = i == r ? 1.0 : 0.0;
                        double su = S.H[(int64_t)bs * bb + r * b + i];
#pragma unroll
                        for (int q = 0; q < MAXB; ++q)
                            if (q < i) {
                                sx -= LS[i * b + q] * x[q];
                                su -= LS[i * b + q] * u[q];
                            }
                        x[i] = sx * LSrd[i];
                        u[i] = su * LSrd[i];
                        LSinv[i * b + r] = x[i];
                        U[i * b + r] = u[i];
                        __builtin_amdgcn_sched_barrier(0);
                    }
            }
            __syncthreads();
        }
        if (!sh[3]) {
            if (lane == 0) atomicMin(err, k);
            break;
        }
        // H_kk -= U^T U, L_H = chol(H_kk)
        #pragma unroll 1
        for (int e = lane; e < bb; e += 64) {
            const int i = e / b, j = e - i * b;
            double acc = 0.0;
                        for (int q = 0; q < b; ++q) acc += U[q * b + i] * U[q * b + j];
            Hkk[e] -= acc;
        }
        __syncthreads();
        {
            if (g0)
#pragma unroll 1
                for (int j = 0; j < b; ++j) LH[r * b + j] = Hkk[r * b + j];
            bool okH = true;
            group_chol(LH, LHrd, scb, b, r, g0, okH);
            if (g0 && !okH) sh[3] = 0;
        }
        // V = Kinv A[P~, c*] (c*'s list holds its nonzero blocks A_jc*) and
        // Vt = V L_S^{-T}, one row i of both per lane. c*'s blocks A_jc* are
        // staged in LDS (the group buffers are free here) in chunks of list
        // entries; a lane's Kinv elements of an entry are loaded together.
        {
            const int nn = S.nzn[bs];
            if (lane < nn) {
                tmp_a[lane] = S.nzp[(int64_t)bs * AD_MAXP + lane];
                tmp_b[lane] = S.nze[(int64_t)bs * AD_MAXP + lane];
            }
            const int ln = ai_lane();
            const int per = (int)((NB * ai_group_doubles(b, BC > 0)) / bb);   // entries per chunk
#pragma unroll 1
            for (int i0 = 0; i0 < M; i0 += 64) {
                const int i = i0 + ln;
                const bool live = i < M;
                double acc[MAXB];
#pragma unroll
                for (int s2 = 0; s2 < MAXB; ++s2) acc[s2] = 0.0;
#pragma unroll 1
                for (int t0 = 0; t0 < nn; t0 += per) {
                    const int t1 = min(nn, t0 + per);
                    __syncthreads();
#pragma unroll 1
                    for (int e = ln; e < (t1 - t0) * bb; e += 64) {
                        const int tt = e / bb;
                        gbufs[e] = a_vals[(int64_t)tmp_b[t0 + tt] * bb + (e - tt * bb)];
                    }
                    __syncthreads();
#pragma unroll 1
                    for (int t = t0; t < t1; ++t) {
                        const int pos = tmp_a[t];
                        const double* at = gbufs + (t - t0) * bb;
                        double kc[MAXB];
#pragma unroll
                        for (int q = 0; q < MAXB; ++q)
                            if (q < b) kc[q] = live ? S.kinv[kidx(i, pos * b + q)] : 0.0;
#pragma unroll
                        for (int q = 0; q < MAXB; ++q)
                            if (q < b) {
#pragma unroll
                                for (int s2 = 0; s2 < MAXB; ++s2)
                                    if (s2 < b) acc[s2] += kc[q] * at[q * b + s2];
                            }
                    }
                }
                if (live) {
#pragma unroll
                    for (int s2 = 0; s2 < MAXB; ++s2)
                        if (s2 < b) {
                            S.V[(int64_t)i * b + s2] = acc[s2];
                            double vt = 0.0;
#pragma unroll
                            for (int q = 0; q < MAXB; ++q)
                                if (q < b && q <= s2) vt += acc[q] * LSinv[s2 * b + q];
                            S.Vt[(int64_t)i * b + s2] = vt;
                        }
                }
            }
        }
        __syncthreads();
        if (!sh[3]) {
            if (lane == 0) atomicMin(err, k);
            break;
        }
        // candidate list: drop c* (the last slot moves into its place)
        const int last = ncand - 1;
        if (bs != last) {
            for (int e = lane; e < bb; e += 64) {
                S.W[(int64_t)bs * bb + e] = S.W[(int64_t)last * bb + e];
                S.H[(int64_t)bs * bb + e] = S.H[(int64_t)last * bb + e];
            }
            for (int t = lane; t < AD_MAXP; t += 64) {
                S.nzp[(int64_t)bs * AD_MAXP + t] = S.nzp[(int64_t)last * AD_MAXP + t];
                S.nze[(int64_t)bs * AD_MAXP + t] = S.nze[(int64_t)last * AD_MAXP + t];
            }
        }
        const int r0 = a_rowptr[cstar], r1 = a_rowptr[cstar + 1];
#pragma unroll 1
        for (int e = lane; e < r1 - r0; e += 64) mark[e] = 0;
        __syncthreads();   // V, Vt complete; reads of c*'s slot done; marks clear
        if (bs != last && lane == 0) {
            S.cand[bs] = S.cand[last];
            S.nzn[bs] = S.nzn[last];
        }
        ncand = last;
        __syncthreads();
        // A_c*c for every remaining candidate (one search of row c* each);
        // the entries of row c* found this way are marked
#pragma unroll 1
        for (int q = lane; q < ncand; q += 64) {
            const int e = find_block(a_rowptr, a_col, cstar, S.cand[q]);
            S.ecs[q] = e;
            if (e >= 0) mark[e - r0] = 1;
        }
        // Kinv <- bordered inverse (packed rows keep their offsets as M grows).
        // Rows i < M: Kinv_ij += Vt_i . Vt_j; each lane walks its elements of
        // the packed rows with (i, j) advanced incrementally.
        {
            const int64_t top = ai_tri(M);
            const int ln = ai_lane();
            int i = 0, j = ln;
            while (j > i) {
                j -= i + 1;
                ++i;
            }
            // compile-time block sizes up to 10: two elements (idx and idx + 64)
            // per pass and the border rows unrolled; otherwise one element per
            // pass (register budget). Each element's loads are issued together.
            constexpr bool wide = !(BC > 0 && MAXB <= 10);
            constexpr int KE = wide ? 1 : 2;
#pragma unroll 1
            for (int64_t idx = ln; idx < top; idx += 64 * KE) {
                int ie[KE], je[KE];
                ie[0] = i;
                je[0] = j;
#pragma unroll
                for (int u = 1; u < KE; ++u) {
                    ie[u] = ie[u - 1];
                    je[u] = je[u - 1] + 64;
                    while (je[u] > ie[u]) {
                        je[u] -= ie[u] + 1;
                        ++ie[u];
                    }
                }
                double vi[KE][MAXB], vj[KE][MAXB], kk[KE];
#pragma unroll
                for (int u = 0; u < KE; ++u) {
                    const bool in = idx + 64 * u < top;
#pragma unroll
                    for (int q = 0; q < MAXB; ++q)
                        if (q < b) {
                            vi[u][q] = in ? S.Vt[(int64_t)ie[u] * b + q] : 0.0;
                            vj[u][q] = in ? S.Vt[(int64_t)je[u] * b + q] : 0.0;
                        }
                    kk[u] = in ? S.kinv[idx + 64 * u] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < KE; ++u) {
                    double acc = 0.0;
#pragma unroll
                    for (int q = 0; q < MAXB; ++q)
                        if (q < b) acc += vi[u][q] * vj[u][q];
                    if (idx + 64 * u < top) S.kinv[idx + 64 * u] = kk[u] + acc;
                }
                i = ie[KE - 1];
                j = je[KE - 1] + 64;
                while (j > i) {
                    j -= i + 1;
                    ++i;
                }
            }
            // border rows i = M + rr, columns j < M: -(L_S^{-T} Vt_j^T)_rr,
            // one lane per column
#pragma unroll 1
            for (int jj = ln; jj < M; jj += 64) {
                double vr[MAXB];
#pragma unroll
                for (int q = 0; q < MAXB; ++q)
                    if (q < b) vr[q] = S.Vt[(int64_t)jj * b + q];
                if constexpr (!wide) {
#pragma unroll
                    for (int rr = 0; rr < MAXB; ++rr)
                        if (rr < b) {
                            double acc = 0.0;
#pragma unroll
                            for (int q = 0; q < MAXB; ++q)
                                if (q < b && q >= rr) acc -= LSinv[q * b + rr] * vr[q];
                            S.kinv[ai_tri(M + rr) + jj] = acc;
                        }
                } else {
#pragma unroll 1
                    for (int rr = 0; rr < b; ++rr) {
                        double acc = 0.0;
#pragma unroll
                        for (int q = 0; q < MAXB; ++q)
                            if (q < b && q >= rr) acc -= LSinv[q * b + rr] * vr[q];
                        S.kinv[ai_tri(M + rr) + jj] = acc;
                    }
                }
            }
            // corner: L_S^{-T} L_S^{-1}, lower part
#pragma unroll 1
            for (int e = lane; e < (b * (b + 1)) / 2; e += 64) {
                int rr = 0, ss = e;
                while (ss > rr) {
                    ss -= rr + 1;
                    ++rr;
                }
                double acc = 0.0;
                for (int q = rr; q < b; ++q) acc += LSinv[q * b + rr] * LSinv[q * b + ss];
                S.kinv[ai_tri(M + rr) + M + ss] = acc;
            }
        }
        __syncthreads();
        // candidates brought in by c*: unmarked entries of row c* left of k,
        // other than c* and the blocks of P~
        {
            const int nold = ncand;
#pragma unroll 1
            for (int base = r0; base < r1; base += 64) {
                const int e = base + lane;
                bool f = false;
                int c = -1;
                if (e < r1) {
                    c = a_col[e];
                    f = c < k && c != cstar && !mark[e - r0];
#pragma unroll 1
                    for (int q = 0; q < m && f; ++q) f = plist[q] != c;
                }
                const unsigned long long mk = __ballot(f);
                if (f) {
                    const int slot = ncand + __popcll(mk & ((1ull << lane) - 1));
                    if (slot < cap) {
                        S.cand[slot] = c;
                        S.nzn[slot] = 0;
                        S.ecs[slot] = e;
                    }
                }
                ncand += __popcll(mk);
            }
            if (ncand > cap) {
                if (lane == 0) { atomicMin(err, k); sh[3] = 0; }
                ncand = cap;
            }
            __syncthreads();
            ai_init_slots(k, b, nold, ncand, a_rowptr, a_col, a_vals, S, tmp_a, tmp_b);
        }
        if (lane == 0) plist[m] = cstar;
        ++m;
        pending = true;
        __syncthreads();
    }
    // output: sorted P_k (P~ and k)
    if (lane == 0) {
        int tmp[AD_MAXP];
        #pragma unroll 1
        for (int i = 0; i < m; ++i) tmp[i] = plist[i];
        tmp[m] = k;
        #pragma unroll 1
        for (int i = 1; i <= m; ++i) {
            int v = tmp[i], j = i - 1;
            while (j >= 0 && tmp[j] > v) { tmp[j + 1] = tmp[j]; --j; }
            tmp[j + 1] = v;
        }
        #pragma unroll 1
        for (int i = 0; i <= m; ++i) out_cols[(int64_t)k * out_stride + i] = tmp[i];
        out_cnt[k] = m + 1;
    }
    __syncthreads();
}

template <int MAXB, int BC>
__device__ __forceinline__ void ai_kernel(int64_t nb, int b, int tmax, double thresh, int cap,
                                                 const int* __restrict__ a_rowptr, const int* __restrict__ a_col,
                                                 const double* __restrict__ a_vals, const int* __restrict__ p0_rowptr,
                                                 const int* __restrict__ p0_col, int out_stride,
                                                 int* __restrict__ out_cols,
                                                 int* __restrict__ out_cnt, int Mmax, double* scratch,
                                                 int64_t gstride, int* counter,
                                                 int* err) {
    if (BC > 0) b = BC;
    extern __shared__ double lds[];
    __shared__ int plist[AD_MAXP];
    __shared__ int sh[8];
    __shared__ int next;
    __shared__ int tmp_a[64], tmp_b[64];
    const int bb = b * b;
    const int NB = 64 / b;
    double* sm = lds;
    double* gbufs = sm + ai_small_doubles(b);
    int* mark = reinterpret_cast<int*>(gbufs + NB * ai_group_doubles(b, BC > 0));
    // the row's state lives in the workgroup's global slot
    double* g = scratch + (int64_t)blockIdx.x * gstride;
    AiState S;
    S.kinv = g;
    S.V = g + ai_tri(Mmax);
    S.Vt = S.V + (int64_t)Mmax * b;
    S.W = S.Vt + (int64_t)Mmax * b;
    S.H = S.W + (int64_t)cap * bb;
    S.gain = S.H + (int64_t)cap * bb;
    int* gi = reinterpret_cast<int*>(S.gain + cap);
    S.cand = gi;
    S.nzn = gi + cap;
    S.ecs = gi + 2 * cap;
    S.nzp = gi + 3 * cap;
    S.nze = S.nzp + (int64_t)cap * AD_MAXP;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int64_t row = next;
        __syncthreads();
        if (row >= nb) break;
        ai_row<MAXB, BC>((int)row, b, tmax, thresh, cap, a_rowptr, a_col, a_vals, p0_rowptr, p0_col, out_stride,
                         out_cols, out_cnt, S, sm, gbufs, mark, plist, tmp_a, tmp_b, sh, err);
    }
}

// Block sizes up to 4, and 10 (compile-time), run two wavefronts per SIMD;
// the others take the registers they need.
#define CHF_AI_PARAMS                                                                                        \
    int64_t nb, int b, int tmax, double thresh, int cap, const int* __restrict__ a_rowptr,                   \
        const int* __restrict__ a_col, const double* __restrict__ a_vals, const int* __restrict__ p0_rowptr, \
        const int* __restrict__ p0_col, int out_stride, int* __restrict__ out_cols, int* __restrict__ out_cnt,   \
        int Mmax, double* scratch, int64_t gstride, int* counter, int* err
#define CHF_AI_ARGS \
    nb, b, tmax, thresh, cap, a_rowptr, a_col, a_vals, p0_rowptr, p0_col, out_stride, out_cols, out_cnt, Mmax, \
        scratch, gstride, counter, err
template <int MAXB, int BC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_adaptive(CHF_AI_PARAMS) {
    ai_kernel<MAXB, BC>(CHF_AI_ARGS);
}
template <int MAXB, int BC>
__global__ __launch_bounds__(64) void k_adaptive_wide(CHF_AI_PARAMS) {
    ai_kernel<MAXB, BC>(CHF_AI_ARGS);
}
#undef CHF_AI_PARAMS
#undef CHF_AI_ARGS

template <int MAXB, int BC>
static void ai_launch(int64_t grid, size_t dyn, hipStream_t s, int64_t nb, int b, int tmax, double thresh, int cap,
                      chf_bsr A, const int* p0_rowptr, const int* p0_col, int out_stride, int* out_cols, int* out_cnt,
                      int Mmax, double* scratch, int64_t stride, int* counter, int* err) {
    void (*kern)(int64_t, int, int, double, int, const int*, const int*, const double*, const int*, const int*, int,
                 int*, int*, int, double*, int64_t, int*, int*);
    if constexpr (MAXB <= 4 || (BC > 0 && MAXB <= 10)) kern = k_adaptive<MAXB, BC>;
    else kern = k_adaptive_wide<MAXB, BC>;
    if (dyn > 64 * 1024)
        CHF_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64), dyn, s, nb, b, tmax, thresh, cap,
                       A->d_rowptr.p, A->d_colidx.p, A->d_vals.p, p0_rowptr, p0_col, out_stride, out_cols, out_cnt,
                       Mmax, scratch, stride, counter, err);
    CHF_LAUNCH_CHECK();
}

chf_pattern_s* adaptive_pattern_impl(chf_bsr A, const chf_pattern_s* P0, int tmax, double tau, hipStream_t s) {
    CHF_CHECK(tau > 0.0 && tau <= 1.0, CHF_EINVAL, "tau must be in (0, 1]");
    CHF_CHECK(!A->vb, CHF_EINVAL, "the adaptive pattern supports uniform block sizes only");
    const int64_t nb = A->nb;
    const int b = A->b;
    int maxp0 = 1;   // blocks per row of P0 (diagonal when P0 is NULL)
    if (P0) {
        CHF_CHECK(P0->nb == nb, CHF_EINVAL, "P0 has a different number of block rows than A");
        for (int64_t k = 0; k < nb; ++k) maxp0 = (int)std::max<int64_t>(maxp0, P0->rowptr[k + 1] - P0->rowptr[k]);
    }
    CHF_CHECK(tmax >= 0 && (int64_t)maxp0 + tmax <= AD_MAXP, CHF_EINVAL,
              "tmax plus the longest row of P0 must not exceed 32 blocks");
    const int width = maxp0 + tmax;   // blocks per output row at most
    std::unique_ptr<chf_pattern_s> P(new chf_pattern_s);
    P->nb = nb;
    P->rowptr.assign(nb + 1, 0);
    if (tmax == 0 || nb == 0) {
        if (P0) {
            P->rowptr = P0->rowptr;
            P->colidx = P0->colidx;
            return P.release();
        }
        for (int64_t k = 0; k < nb; ++k) {
            P->colidx.push_back((int32_t)k);
            P->rowptr[k + 1] = k + 1;
        }
        return P.release();
    }
    CHF_CHECK(b >= 1 && b <= 32, CHF_EINVAL, "adaptive pattern supports block sizes up to 32");
    // every candidate lies in the union of the rows A_j, j in P_k
    int64_t maxrow = 1;
    for (int64_t k = 0; k < nb; ++k) maxrow = std::max<int64_t>(maxrow, A->rowptr[k + 1] - A->rowptr[k]);
    const int cap = (int)std::min<int64_t>((int64_t)width * maxrow, 1 << 20);
    // Kinv and V never grow past width - 2 blocks (the last block enters
    // without a bordering update)
    const int Mmax = std::max(1, width - 2) * b;
    DevBuf<int> d_p0_rowptr, d_p0_col;
    if (P0) {
        std::vector<int> rp(nb + 1);
        for (int64_t k = 0; k <= nb; ++k) rp[k] = (int)P0->rowptr[k];
        d_p0_rowptr.alloc(nb + 1);
        d_p0_rowptr.upload(rp.data(), nb + 1, s);
        d_p0_col.alloc(std::max<size_t>(1, P0->colidx.size()));
        d_p0_col.upload(P0->colidx.data(), P0->colidx.size(), s);
    }
    int dev = 0, lim = 0;
    CHF_HIP(hipGetDevice(&dev));
    CHF_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t static_lds = AD_MAXP * 4 + 8 * 4 + 64 + 2 * 64 * 4;
    // the row's state (Kinv, V, Vt and the candidates) lives in the
    // workgroup's global slot; LDS holds the b x b work buffers
    // (block sizes 10 and 21 run their own instantiation, whose candidate
    // factorisations are register-resident)
    const bool reg = b == 10 || b == 21;
    const size_t dyn = (size_t)ai_lds_doubles(b, (int)maxrow, reg) * 8;
    CHF_CHECK(dyn + static_lds <= (size_t)lim, CHF_EINVAL, "adaptive pattern: block size too large for LDS");
    const int cus = device_cu_count();
    // LDS is allocated in 512-byte granules
    int per_cu = std::max<int>(1, (int)std::min<size_t>(8, (size_t)lim / ((dyn + static_lds + 511) / 512 * 512)));
    // CHF_AI_WG_PER_CU=<n> lowers the number of resident rows per CU (fewer
    // row states in flight, each more likely to stay in the caches)
    if (const char* e = std::getenv("CHF_AI_WG_PER_CU")) per_cu = std::max(1, std::min(per_cu, std::atoi(e)));
    const int64_t grid = std::min<int64_t>((int64_t)cus * per_cu, nb);
    const int64_t stride = (ai_global_doubles(Mmax, b, cap) + 31) / 32 * 32;
    DevBuf<double> scratch((size_t)grid * stride);
    DevBuf<int> out_cols((size_t)nb * width), out_cnt(nb), flags(2);
    int init[2] = {0, INT32_MAX};
    flags.upload(init, 2, s);
    const double thresh = -std::log(tau) + AD_GAIN_EPS;
    // the block sizes of the workloads get their own instantiation (block
    // offsets are compile-time constants); others share one per size class
#define CHF_AI_LAUNCH(MB, BCV)                                                                                   \
    ai_launch<MB, BCV>(grid, dyn, s, nb, b, tmax, thresh, cap, A, P0 ? d_p0_rowptr.p : nullptr,                  \
                       P0 ? d_p0_col.p : nullptr, width, out_cols.p, out_cnt.p, Mmax, scratch.p, stride, flags.p, \
                       flags.p + 1)
    if (b == 10) CHF_AI_LAUNCH(10, 10);
    else if (b == 21) CHF_AI_LAUNCH(21, 21);
    else if (b <= 4) CHF_AI_LAUNCH(4, 0);
    else if (b <= 10) CHF_AI_LAUNCH(10, 0);
    else if (b <= 16) CHF_AI_LAUNCH(16, 0);
    else if (b <= 21) CHF_AI_LAUNCH(21, 0);
    else CHF_AI_LAUNCH(32, 0);
#undef CHF_AI_LAUNCH
    std::vector<int> hcols((size_t)nb * width), hcnt(nb);
    int hflags[2];
    out_cols.download(hcols.data(), hcols.size(), s);
    out_cnt.download(hcnt.data(), nb, s);
    flags.download(hflags, 2, s);
    CHF_HIP(hipStreamSynchronize(s));
    if (hflags[1] != INT32_MAX)
        fail(CHF_ENOTSPD, "adaptive pattern: local matrices of block row " + std::to_string(hflags[1]) +
                              " are not positive definite");
    for (int64_t k = 0; k < nb; ++k) {
        CHF_CHECK(hcnt[k] >= 1 && hcnt[k] <= width, CHF_EDEVICE, "adaptive pattern: bad row count");
        for (int i = 0; i < hcnt[k]; ++i) P->colidx.push_back(hcols[(size_t)k * width + i]);
        P->rowptr[k + 1] = (int64_t)P->colidx.size();
    }
    return P.release();
}
}  // namespace chf

extern "C" int chf_pattern_adaptive(chf_bsr A, chf_pattern P0, int tmax, double tau, chf_pattern* out) {
    return chf::guarded([&] {
        CHF_CHECK(A && out, CHF_EINVAL, "NULL argument");
        *out = chf::adaptive_pattern_impl(A, P0, tmax, tau, 0);
    });
}

// ------------------------------------------------ learned-pattern features --
// For block row k and each candidate c of the strictly lower part of the row
// pattern of A^2, six features: ||A_kc||_F / sqrt(||A_kk||_F ||A_cc||_F),
// ||A_cc^{-1} A_ck||_F, the signed patch offset (dx, dy, dz) of c from k on
// the grid, and the one-step gain -log rho_c at P_k = {k} (Lemma 2.4 with P~ empty:
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
                float* f = feats + (c0 + s0 + ci) * MLP_NIN;
                f[0] = (float)(sqrt(fkc) / sqrt(nkk * sqrt(fcc)));
                f[1] = (float)sqrt(fv);
                f[2] = (float)dx;
                f[3] = (float)dy;
                f[4] = (float)dz;
                f[5] = (float)gain[s0 + ci];
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
        CHF_CHECK(!A || !A->vb, CHF_EINVAL, "the learned proposer supports uniform block sizes only");
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
        CHF_CHECK(!A || !A->vb, CHF_EINVAL, "the learned proposer supports uniform block sizes only");
        CHF_CHECK(A && feats, CHF_EINVAL, "NULL argument");
        CHF_CHECK(nx >= 1 && ny >= 1 && A->nb % ((int64_t)nx * ny) == 0, CHF_EINVAL, "grid does not match nb");
        std::vector<int64_t> r;
        std::vector<int32_t> c;
        chf::a2_candidates(A, r, c);
        chf::mlp_features_impl(A, nx, ny, r, c, feats, stream);
    });
}
