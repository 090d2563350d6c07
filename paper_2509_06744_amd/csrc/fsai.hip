// Static patterns and the batched block-FSAI set-up (Def. 2.2): one dense SPD
// system A[P_k, P_k] per block row k, all rows in one persistent launch.
//
// With the row's blocks ordered as P~_k ascending followed by k, the
// Cholesky factor L of K = A[P_k, P_k] has as its last block row
// [L_kP, L_kk] with L_kk L_kk^T = S_kk (Eq. schur_complement_fsai) and
// L_kP L_PP^{-1} = -F[k, P~_k] (Eq. fsai_f_definition). The last b rows of
// L^{-1} are therefore [L_kk^{-1} F_kP, L_kk^{-1}] = J F with J = L_kk^{-1}:
// the factor G = S^{-1/2} F with the inverse Cholesky root as S^{-1/2}.
// They are obtained from L^T Z = E (E the last b columns of I), G_k = Z^T.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>

#include "internal.h"
#include "kernels_common.h"

namespace chf {

constexpr int FSAI_MAXM = 32;    // blocks per pattern row
constexpr int FSAI_MAXN = 320;   // local system size b * |P_k|

__device__ inline int64_t tri(int64_t i) { return i * (i + 1) / 2; }

// Per-row work of the set-up kernel. K: packed lower triangle (row-major),
// Z: n x b right-hand sides; both either in LDS or in a global scratch slot.
template <int NT>
__device__ void fsai_row(int64_t k, int b, const int* __restrict__ a_rowptr, const int* __restrict__ a_col,
                         const double* __restrict__ a_vals, const int64_t* __restrict__ p_rowptr,
                         const int* __restrict__ p_col, double* __restrict__ g_vals, double* K, double* Z,
                         int* idx, double* sh_scal, int* sh_flag, int* bad_row) {
    const int tid = threadIdx.x;
    const int64_t p0 = p_rowptr[k];
    const int m = (int)(p_rowptr[k + 1] - p0);
    const int n = m * b;
    const int* cols = p_col + p0;
    // block lookup table idx[a * m + c] (a >= c): position of A[P_a, P_c] or -1
    for (int t = tid; t < m * m; t += NT) {
        int a = t / m, c = t - a * m;
        int e = -1;
        if (c <= a) {
            int row = cols[a], want = cols[c];
            int lo = a_rowptr[row], hi = a_rowptr[row + 1];
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                int v = a_col[mid];
                if (v < want) lo = mid + 1; else hi = mid;
            }
            if (lo < a_rowptr[row + 1] && a_col[lo] == want) e = lo;
        }
        idx[t] = e;
    }
    __syncthreads();
    // gather K = A[P_k, P_k] (lower triangle)
    const int64_t nn = (int64_t)n * n;
    for (int64_t t = tid; t < nn; t += NT) {
        int i = (int)(t / n), j = (int)(t - (int64_t)i * n);
        if (j > i) continue;
        int a = i / b, ra = i - a * b, c = j / b, rc = j - c * b;
        int e = idx[a * m + c];
        K[tri(i) + j] = e >= 0 ? a_vals[(int64_t)e * b * b + ra * b + rc] : 0.0;
    }
    if (tid == 0) sh_flag[0] = 1;
    __syncthreads();
    // right-looking Cholesky, one column at a time
    for (int q = 0; q < n; ++q) {
        if (tid == 0) {
            double d = K[tri(q) + q];
            if (!(d > 0.0) || !isfinite(d)) {
                sh_flag[0] = 0;
            } else {
                double l = sqrt(d);
                K[tri(q) + q] = l;
                sh_scal[0] = 1.0 / l;
            }
        }
        __syncthreads();
        if (!sh_flag[0]) break;
        const double inv = sh_scal[0];
        for (int i = q + 1 + tid; i < n; i += NT) K[tri(i) + q] *= inv;
        __syncthreads();
        for (int i = q + 1 + tid; i < n; i += NT) {
            const double liq = K[tri(i) + q];
            double* ki = K + tri(i);
            for (int j = q + 1; j <= i; ++j) ki[j] -= liq * K[tri(j) + q];
        }
        __syncthreads();
    }
    const bool ok = sh_flag[0] != 0;
    __syncthreads();
    if (!ok) {
        if (tid == 0) atomicMin(bad_row, (int)k);
        for (int64_t t = tid; t < (int64_t)m * b * b; t += NT) g_vals[p0 * b * b + t] = 0.0;
        __syncthreads();
        return;
    }
    // back substitution L^T Z = E_last (right-looking over rows of Z)
    for (int64_t t = tid; t < (int64_t)n * b; t += NT) {
        int i = (int)(t / b), c = (int)(t - (int64_t)i * b);
        Z[t] = (i == n - b + c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int q = n - 1; q >= 0; --q) {
        const double lqq = K[tri(q) + q];
        if (tid < b) Z[(int64_t)q * b + tid] /= lqq;
        __syncthreads();
        const double* lrow = K + tri(q);
        for (int t = tid; t < q * b; t += NT) {
            int pidx = t / b, c = t - pidx * b;
            Z[t] -= lrow[pidx] * Z[(int64_t)q * b + c];
        }
        __syncthreads();
    }
    // G[k, P_k] = Z^T, block a of the row = Z[a*b:(a+1)*b, :]^T
    for (int64_t t = tid; t < (int64_t)m * b * b; t += NT) {
        int a = (int)(t / (b * b));
        int rem = (int)(t - (int64_t)a * b * b);
        int r = rem / b, c = rem - r * b;
        g_vals[(p0 + a) * b * b + rem] = Z[(int64_t)(a * b + c) * b + r];
    }
    __syncthreads();
}

// ------------------------------------------------- tiled MFMA local solver --
// For larger local systems (n > ntile, b <= 16) the factorisation works on
// 16 x 16 tiles of the lower triangle, held in the workgroup's global scratch
// slot (L2/MALL resident), right-looking by pairs of tile columns. Per column,
// one wavefront factors the diagonal tile and inverts its factor in registers
// (the only sequential step); the panel L_ik = A_ik L_kk^{-T} and the
// trailing update A_IJ -= L_Ik L_Jk^T + L_I,k+1 L_J,k+1^T are FP64 MFMA
// products over the four wavefronts (v_mfma_f64_16x16x4: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[4 r + l / 16][l % 16]
// in register r). The b right-hand sides of L^T Z = E are solved by tile
// rows, Z_I = L_II^{-T}(E_I - sum L_JI^T Z_J), also on MFMA. Padding rows of
// the last tile are identity rows.
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline v4d mfma16(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// Broadcast of lane l's value to the wavefront through scalar registers
// (v_readlane), cheaper than an LDS permute when l is a compile-time constant.
__device__ inline double lane_bcast(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

__device__ inline double* tile_at(double* base, int I, int J) { return base + ((int64_t)I * (I + 1) / 2 + J) * 256; }

__device__ inline void tri_decode(int t, int& I, int& J) {
    int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    I = i;
    J = t - i * (i + 1) / 2;
}

// One wavefront: Cholesky factor L of the 16 x 16 SPD tile Dt (row-major; lane
// l works on row l % 16 in registers) and its inverse X = L^{-1}, written to X
// and to inv. Row r of X is finished once the rows above it are, so rows
// complete in order and are broadcast by readlane. Returns false if a pivot is
// not positive and finite.
__device__ inline bool diag_tile_inv(const double* Dt, double* X, double* inv, int lane) {
    const int r = lane & 15;
    double row[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) row[c] = Dt[r * 16 + c];
    bool ok = true;
    double rinv[16];   // 1 / L[q][q], the same on every lane
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const double dq = lane_bcast(row[q], q);
        ok = ok && (dq > 0.0) && isfinite(dq);
        const double lqq = sqrt(fmax(dq, 1e-300));
        rinv[q] = 1.0 / lqq;
        const double lrq = (r > q) ? row[q] * rinv[q] : (r == q ? lqq : 0.0);
        row[q] = lrq;
#pragma unroll
        for (int j = q + 1; j < 16; ++j) {
            const double ljq = lane_bcast(lrq, j);
            if (j <= r) row[j] -= lrq * ljq;
        }
    }
    double acc[16], xr[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) { acc[c] = 0.0; xr[c] = 0.0; }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const double dinv = rinv[q];
#pragma unroll
        for (int c = 0; c <= q; ++c) {
            const double xq = ((q == c ? 1.0 : 0.0) - acc[c]) * dinv;   // X[q][c] on lane q
            const double v = lane_bcast(xq, q);
            if (r == q) xr[c] = v;
            if (r > q) acc[c] += row[q] * v;
        }
    }
    if (lane < 16) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const double v = c <= r ? xr[c] : 0.0;
            X[r * 16 + c] = v;
            inv[r * 16 + c] = v;
        }
    }
    return ok;
}

__device__ void fsai_row_tiled(int64_t k, int b, const int* __restrict__ a_rowptr, const int* __restrict__ a_col,
                               const double* __restrict__ a_vals, const int64_t* __restrict__ p_rowptr,
                               const int* __restrict__ p_col, double* __restrict__ g_vals, double* tiles,
                               double* panel, double* invs, double* part, int* idx, int* sh_flag,
                               int* bad_row) {
    constexpr int NT = 256;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t p0 = p_rowptr[k];
    const int m = (int)(p_rowptr[k + 1] - p0);
    const int n = m * b;
    const int T = (n + 15) / 16;
    const int* cols = p_col + p0;
    // block map idx[a m + c] = position of A[P_k[a], P_k[c]] in A (or -1), c <= a;
    // each thread runs IS binary searches side by side so their loads overlap
    constexpr int IS = 4;
    for (int t0 = tid; t0 < m * m; t0 += IS * NT) {
        int lo[IS], hi[IS], end[IS], want[IS];
#pragma unroll
        for (int s = 0; s < IS; ++s) {
            const int t = t0 + s * NT;
            const int a = t / m, c = t - a * m;
            lo[s] = hi[s] = end[s] = 0;
            want[s] = -1;
            if (t < m * m && c <= a) {
                const int row = cols[a];
                lo[s] = a_rowptr[row];
                hi[s] = end[s] = a_rowptr[row + 1];
                want[s] = cols[c];
            }
        }
        for (;;) {
            bool any = false;
#pragma unroll
            for (int s = 0; s < IS; ++s) {
                if (lo[s] < hi[s]) {
                    any = true;
                    const int mid = (lo[s] + hi[s]) >> 1;
                    if (a_col[mid] < want[s]) lo[s] = mid + 1; else hi[s] = mid;
                }
            }
            if (!any) break;
        }
#pragma unroll
        for (int s = 0; s < IS; ++s) {
            const int t = t0 + s * NT;
            if (t < m * m) idx[t] = (want[s] >= 0 && lo[s] < end[s] && a_col[lo[s]] == want[s]) ? lo[s] : -1;
        }
    }
    __syncthreads();
    const int ntiles = T * (T + 1) / 2;
    // tiles of the lower triangle: one lane fills 8 entries of a tile row, with
    // its 8 gathers from A issued before any is used (unused lanes read entry 0);
    // entries above the diagonal are 0, padding rows and columns are identity
    for (int u = tid; u < ntiles * 32; u += NT) {
        int I, J;
        tri_decode(u >> 5, I, J);
        const int r = (u >> 1) & 15, c0 = (u & 1) << 3;
        const int i = 16 * I + r, j0 = 16 * J + c0;
        const bool row_in = i < n;
        const int a = row_in ? i / b : 0, ra = row_in ? i - a * b : 0;
        int cb = j0 / b, rc = j0 - cb * b;
        double v[8];
        bool take[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = j0 + q;
            const int ee = (row_in && j < n && j <= i) ? idx[a * m + cb] : -1;
            take[q] = ee >= 0;
            v[q] = a_vals[take[q] ? (int64_t)ee * b * b + ra * b + rc : 0];
            if (++rc == b) { rc = 0; ++cb; }
        }
        double2* dst = reinterpret_cast<double2*>(tile_at(tiles, I, J) + r * 16 + c0);
#pragma unroll
        for (int q = 0; q < 8; q += 2) {
            const double d0 = (i == j0 + q) ? 1.0 : 0.0, d1 = (i == j0 + q + 1) ? 1.0 : 0.0;
            dst[q >> 1] = make_double2(take[q] ? v[q] : d0, take[q + 1] ? v[q + 1] : d1);
        }
    }
    if (tid == 0) sh_flag[0] = 1;
    __syncthreads();
    // Right-looking by pairs of tile columns k, k + 1, so that each trailing
    // tile is read and written once per two columns:
    //   (a) one wavefront factors A_kk and inverts the factor, X = L_kk^{-1};
    //   (b) L_ik = A_ik X^T (i > k) to the slot and to LDS;
    //   (c1) column k + 1 alone: A_{i,k+1} -= L_ik L_{k+1,k}^T (i > k);
    //   (a2), (b2) the same two steps for column k + 1 (panel to the slot only);
    //   (c) A_IJ -= L_Ik L_Jk^T + L_{I,k+1} L_{J,k+1}^T (J, I > k + 1), with
    //       column k from LDS and column k + 1 read back through L2.
    // The wavefront taking the sequential step rotates with the column and the
    // workgroup, spreading it over the SIMDs.
    for (int kt = 0; kt < T; kt += 2) {
        for (int h = 0; h < 2 && kt + h < T; ++h) {
            const int kc = kt + h;   // the column factored in this step: (a), (b) for h = 0; (a2), (b2) for h = 1
            if (wave == ((kc + (int)blockIdx.x) & 3)) {
                if (!diag_tile_inv(tile_at(tiles, kc, kc), panel, invs + kc * 256, lane) && lane == 0) sh_flag[0] = 0;
            }
            __syncthreads();
            if (!sh_flag[0]) break;
            // L_ic = A_ic X^T: step q takes A_ic[l % 16][4q + l / 16] and
            // X^T[4q + l / 16][l % 16] = X[l % 16][4q + l / 16]; column k also to LDS
            for (int ti = kc + 1 + wave; ti < T; ti += 4) {
                double* Tt = tile_at(tiles, ti, kc);
                v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc = mfma16(Tt[(lane & 15) * 16 + 4 * q + (lane >> 4)], panel[(lane & 15) * 16 + 4 * q + (lane >> 4)],
                                 acc);
                double* pt = panel + (ti - kt) * 256;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int o = (4 * rr + (lane >> 4)) * 16 + (lane & 15);
                    Tt[o] = acc[rr];
                    if (h == 0) pt[o] = acc[rr];
                }
            }
            __syncthreads();
            if (h == 0) {
                // (c1) column k + 1 alone: A_{i,k+1} -= L_ik L_{k+1,k}^T, L_{k+1,k} in LDS slot 1
                for (int ti = kt + 1 + wave; ti < T; ti += 4) {
                    double* Ct = tile_at(tiles, ti, kt + 1);
                    v4d acc;
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) acc[rr] = Ct[(4 * rr + (lane >> 4)) * 16 + (lane & 15)];
                    const double* Li = panel + (ti - kt) * 256;
                    const double* Lj = panel + 256;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        acc = mfma16(-Li[(lane & 15) * 16 + 4 * q + (lane >> 4)], Lj[(lane & 15) * 16 + 4 * q + (lane >> 4)],
                                     acc);
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) Ct[(4 * rr + (lane >> 4)) * 16 + (lane & 15)] = acc[rr];
                }
                __syncthreads();
            }
        }
        if (!sh_flag[0] || kt + 1 >= T) break;
        // (c) trailing tiles, k + 1 < J <= I < T; each wavefront keeps U tiles in flight
        const int nt = T - kt - 2;
        const int npairs = nt * (nt + 1) / 2;
        constexpr int U = 2;
        for (int base = wave * U; base < npairs; base += 4 * U) {
            v4d acc[U];
            double li2[U][4], lj2[U][4];
            double* Ct[U];
            int ii[U], jj[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int pidx = min(base + u, npairs - 1);
                tri_decode(pidx, ii[u], jj[u]);
                Ct[u] = tile_at(tiles, kt + 2 + ii[u], kt + 2 + jj[u]);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) acc[u][rr] = Ct[u][(4 * rr + (lane >> 4)) * 16 + (lane & 15)];
                const double* Li2 = tile_at(tiles, kt + 2 + ii[u], kt + 1);
                const double* Lj2 = tile_at(tiles, kt + 2 + jj[u], kt + 1);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    li2[u][q] = Li2[(lane & 15) * 16 + 4 * q + (lane >> 4)];
                    lj2[u][q] = Lj2[(lane & 15) * 16 + 4 * q + (lane >> 4)];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double* Li = panel + (ii[u] + 2) * 256;   // L_{I,k}: LDS slot I - k
                const double* Lj = panel + (jj[u] + 2) * 256;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc[u] = mfma16(-Li[(lane & 15) * 16 + 4 * q + (lane >> 4)], Lj[(lane & 15) * 16 + 4 * q + (lane >> 4)],
                                    acc[u]);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[u] = mfma16(-li2[u][q], lj2[u][q], acc[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (base + u < npairs) {
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) Ct[u][(4 * rr + (lane >> 4)) * 16 + (lane & 15)] = acc[u][rr];
                }
            }
        }
        __syncthreads();
    }
    if (!sh_flag[0]) {
        if (tid == 0) atomicMin(bad_row, (int)k);
        for (int64_t t = tid; t < (int64_t)m * b * b; t += NT) g_vals[p0 * b * b + t] = 0.0;
        __syncthreads();
        return;
    }
    // L^T Z = E (Z: 16T x 16, columns c < b carry the last b unit vectors),
    // by tile rows: Z_I = X_II^T (E_I - sum_{J > I} L_JI^T Z_J) on MFMA. Z is
    // kept in LDS, in the space of the panel, which is free from here on.
    double* Zs = panel;
    for (int I = T - 1; I >= 0; --I) {
        // the single-wavefront step of this tile row rotates like (a)
        const bool own = wave == ((I + (int)blockIdx.x) & 3);
        double xa[4];
        if (own) {
#pragma unroll
            for (int q = 0; q < 4; ++q) xa[q] = invs[I * 256 + (4 * q + (lane >> 4)) * 16 + (lane & 15)];   // X^T
        }
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        // wavefront w takes J = I + 1 + w + 4 s; four L_JI tiles are loaded before use
        for (int J0 = I + 1 + wave; J0 < T; J0 += 16) {
            double av[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double* LJI = tile_at(tiles, min(J0 + 4 * u, T - 1), I);
#pragma unroll
                for (int q = 0; q < 4; ++q) av[u][q] = LJI[(4 * q + (lane >> 4)) * 16 + (lane & 15)];   // L_JI^T
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int J = J0 + 4 * u;
                if (J < T) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        acc = mfma16(av[u][q], Zs[(16 * J + 4 * q + (lane >> 4)) * 16 + (lane & 15)], acc);   // Z_J
                }
            }
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) part[wave * 256 + (4 * rr + (lane >> 4)) * 16 + (lane & 15)] = acc[rr];
        __syncthreads();
        // R = E_I - S, stored row-major in part[4 * 256 ...]
        for (int e = tid; e < 256; e += NT) {
            const int r = e >> 4, c = e & 15;
            const double ev = (c < b && 16 * I + r == n - b + c) ? 1.0 : 0.0;
            part[1024 + e] = ev - (part[e] + part[256 + e] + part[512 + e] + part[768 + e]);
        }
        __syncthreads();
        if (own) {
            v4d z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 4; ++q)
                z = mfma16(xa[q], part[1024 + (4 * q + (lane >> 4)) * 16 + (lane & 15)], z);   // R[4q+k][col]
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) Zs[(16 * I + 4 * rr + (lane >> 4)) * 16 + (lane & 15)] = z[rr];
        }
        __syncthreads();
    }
    for (int64_t t = tid; t < (int64_t)m * b * b; t += NT) {
        const int a = (int)(t / (b * b));
        const int rem = (int)(t - (int64_t)a * b * b);
        const int r = rem / b, c = rem - r * b;
        g_vals[(p0 + a) * b * b + rem] = Zs[(a * b + c) * 16 + r];
    }
    __syncthreads();
}

// ---------------------------------------------------- register-resident --
// Rows with 16 < n <= 240 (at most 15 x 15 tiles) can keep the whole upper
// triangle of the padded local matrix in the registers of one workgroup of 8
// wavefronts (one workgroup per CU, 15 tiles of 8 registers per lane each),
// so nothing but A, the block map and G crosses the memory hierarchy. The
// padding rows come first here (identity, decoupled from the rest), which
// puts block row k in the last b rows of the last tile row.
//
// The factorisation is block LDL^T over 16 x 16 tiles, U_ab = Kpad tile (a, b)
// for a <= b, D_c the diagonal tile after the updates of the steps before c:
//   step c:  Dinv = D_c^{-1}, W_cb = Dinv U_cb (b > c),
//            U_ab -= U_ca^T W_cb (c < a <= b).
// With Lt the block unit lower factor (Lt_bc = W_cb^T) and R_c = chol(D_c),
// the Cholesky factor is L = Lt blockdiag(R_c); the last tile row of L^{-1}
// is X V with X = R_{T-1}^{-1} and V the last tile row of Lt^{-1}:
//   V_{T-1} = I,  V_a = -sum_{b > a} V_b W_ab^T,
// and G_k is the last b rows of X V. The sequential work per step is one
// 16 x 16 inverse on one wavefront, done by block sweeps on MFMA; the other
// wavefronts update their tiles meanwhile.
//
// MFMA operand layouts (v_mfma_f64_16x16x4f64, lane l, g = l / 16, j = l % 16):
// step q reads A[j][4q + g] and B[4q + g][j]; accumulator element rr holds
// row 4 rr + g, column j. A tile held in accumulator layout therefore serves
// directly as B, and as A for its transpose.
constexpr int RR_WAVES = 8;
constexpr int RR_NT = 64 * RR_WAVES;
constexpr int RR_TMAX = 15;
constexpr int RR_MAXN = 16 * RR_TMAX;
constexpr int RR_SLOTS = (RR_TMAX * (RR_TMAX + 1) / 2 + RR_WAVES - 1) / RR_WAVES;   // 15

__device__ __forceinline__ double sel4(int i, double a0, double a1, double a2, double a3) {
    double r = a3;
    r = i == 2 ? a2 : r;
    r = i == 1 ? a1 : r;
    r = i == 0 ? a0 : r;
    return r;
}

// 1 / x to double precision, likewise: y <- y + y (1 - x y).
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) y = fma(y, fma(-x, y, 1.0), y);
    return y;
}

// 1 / sqrt(x) to double precision: the hardware estimate refined by two
// Newton steps y <- y + y (1 - x y^2) / 2 (each at least doubles the correct
// bits), in place of a square root and a division on the sequential path.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// One block step of a 4 x 4 SPD pivot P (the same on every lane; lower
// triangle used), by P = L D L^T with L unit lower: X = D^{-1/2} L^{-1} is
// chol(P)^{-1} and P^{-1} = X^T X. Returned as the entries this lane needs
// for the padded 16 x 4 MFMA operands, pin = P^{-1}[j][g] and xin = X[j][g]
// (zero for j >= 4). False if a pivot is not positive and finite.
__device__ __forceinline__ bool chol_inv4(const double (&P)[4][4], int g, int j, double& pin, double& xin) {
    double L[4][4], e[4][4], sq[4];
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        // e[i][c] = L[i][c] d_c (the unscaled column), d_c = P_cc - sum_t L[c][t] e[c][t]
        double d = P[c][c];
#pragma unroll
        for (int t = 0; t < c; ++t) d -= L[c][t] * e[c][t];
        ok = ok && (d > 0.0) && isfinite(d);
        sq[c] = rsqrt_nr(fmax(d, 1e-300));
        const double r = sq[c] * sq[c];
#pragma unroll
        for (int i = c + 1; i < 4; ++i) {
            double v = P[i][c];
#pragma unroll
            for (int t = 0; t < c; ++t) v -= L[i][t] * e[c][t];
            e[i][c] = v;
            L[i][c] = v * r;
        }
    }
    // Y = L^{-1} (unit lower), X[i][c] = Y[i][c] / sqrt(d_i)
    double Y[4][4], X[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int c = 0; c < 4; ++c) Y[i][c] = c == i ? 1.0 : 0.0;
#pragma unroll
        for (int c = 0; c < i; ++c) {
            double v = L[i][c];
#pragma unroll
            for (int t = c + 1; t < i; ++t) v += L[i][t] * Y[t][c];
            Y[i][c] = -v;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) X[i][c] = Y[i][c] * sq[i];
    }
    // columns j and g of X on this lane; P^{-1}[j][g] = sum_t X[t][j] X[t][g]
    double xj[4], xg[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        xj[t] = sel4(j, X[t][0], X[t][1], X[t][2], X[t][3]);
        xg[t] = sel4(g, X[t][0], X[t][1], X[t][2], X[t][3]);
    }
    double pi = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) pi += xj[t] * xg[t];
    pin = j < 4 ? pi : 0.0;
    xin = j < 4 ? sel4(j, xg[0], xg[1], xg[2], xg[3]) : 0.0;
    return ok;
}

// P^{-1}[j][g] of a 4 x 4 SPD pivot P (the same on every lane; lower triangle
// used) for the padded operand (zero for j >= 4), by P = L D L^T with L unit
// lower: P^{-1} = Y^T D^{-1} Y with Y = L^{-1}; reciprocals only, no square
// roots. (Closed-form 2 x 2 block inverses are shorter but lose up to three
// more digits on ill-conditioned pivots.) False if a pivot is not positive
// and finite.
__device__ __forceinline__ bool spd_inv4(const double (&P)[4][4], int g, int j, double& pin) {
    double L[4][4], e[4][4], r[4];
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double d = P[c][c];
#pragma unroll
        for (int t = 0; t < c; ++t) d -= L[c][t] * e[c][t];
        ok = ok && (d > 0.0) && isfinite(d);
        r[c] = rcp_nr(fmax(d, 1e-300));
#pragma unroll
        for (int i = c + 1; i < 4; ++i) {
            double v = P[i][c];
#pragma unroll
            for (int t = 0; t < c; ++t) v -= L[i][t] * e[c][t];
            e[i][c] = v;
            L[i][c] = v * r[c];
        }
    }
    double Y[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int c = 0; c < 4; ++c) Y[i][c] = c == i ? 1.0 : 0.0;
#pragma unroll
        for (int c = 0; c < i; ++c) {
            double v = L[i][c];
#pragma unroll
            for (int t = c + 1; t < i; ++t) v += L[i][t] * Y[t][c];
            Y[i][c] = -v;
        }
    }
    double pi = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double yj = sel4(j, Y[t][0], Y[t][1], Y[t][2], Y[t][3]);
        const double yg = sel4(g, Y[t][0], Y[t][1], Y[t][2], Y[t][3]);
        pi = fma(yj * r[t], yg, pi);
    }
    pin = j < 4 ? pi : 0.0;
    return ok;
}

// In place on an SPD tile M in accumulator layout (one wavefront), by 4 x 4
// blocks p with pivot P (entry (i, c) of P sits in element p of lane
// 16 i + 4 p + c):
//  - chol = false: M <- M^{-1} by block sweeps. Sweeping p maps M_pp to
//    -P^{-1}, M_pj to P^{-1} M_pj, M_ip to M_ip P^{-1} and M_ij to
//    M_ij - M_ip P^{-1} M_pj. With a = M[:, p] - lam E_p (E_p the identity
//    columns of p), M - a P^{-1} a^T gives all four at once up to scale:
//    lam P^{-1} M_pj, lam M_ip P^{-1} and 2 lam I - lam^2 P^{-1}; so -2 lam
//    on the diagonal of P and 1 / lam on the rows and columns of p finish the
//    step. lam = trace(P) / 4 keeps the row and column terms free of the
//    cancellation a unit shift suffers when P is far from the identity in
//    scale. Sweeping every block leaves -M^{-1}.
//  - chol = true: M <- chol(M)^{-1} (lower), by forward elimination of
//    [M | I]: the rows below p take -= M[i, p] P^{-1} [M | Y][p, :], then
//    Y[p, :] <- chol(P)^{-1} Y[p, :].
// M stays symmetric in the part still read (all of it for the sweep, the
// trailing part for the elimination), so column p of M is row p read across
// lanes: element p of this lane's accumulator.
template <bool chol>
__device__ inline bool tile_inverse(v4d& m, int lane) {
    const int g = lane >> 4, j = lane & 15;
    v4d y = {0.0, 0.0, 0.0, 0.0};
    if constexpr (chol) {
#pragma unroll
        for (int q = 0; q < 4; ++q) y[q] = (4 * q + g == j) ? 1.0 : 0.0;
    }
    bool ok = true;
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) {
        double P[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c <= i; ++c) P[i][c] = lane_bcast(m[blk], 16 * i + 4 * blk + c);
        double pin, xin = 0.0;
        if constexpr (chol)
            ok = chol_inv4(P, g, j, pin, xin) && ok;
        else
            ok = spd_inv4(P, g, j, pin) && ok;
        const bool dg = j == 4 * blk + g;
        const double lam = 0.25 * (P[0][0] + P[1][1] + P[2][2] + P[3][3]);
        const double sw = m[blk] - (dg ? lam : 0.0);
        const double av = chol ? (j >= 4 * blk + 4 ? m[blk] : 0.0) : sw;   // A: column p (rows i)
        const double bv = chol ? m[blk] : sw;                               // B: row p
        v4d t = {0.0, 0.0, 0.0, 0.0};
        t = mfma16(pin, bv, t);   // rows 0..3: P^{-1} B
        if constexpr (chol) {
            v4d ty = {0.0, 0.0, 0.0, 0.0}, ts = ty;
            ty = mfma16(pin, y[blk], ty);
            ts = mfma16(xin, y[blk], ts);
            y = mfma16(-av, ty[0], y);
            y[blk] = ts[0];
        }
        m = mfma16(-av, t[0], m);
        if constexpr (!chol) {
            const double rl = rcp_nr(lam);
            if (dg) m[blk] -= 2.0 * lam;
            m[blk] *= rl;                         // rows of p
            if (j >= 4 * blk && j < 4 * blk + 4) {   // columns of p
#pragma unroll
                for (int q = 0; q < 4; ++q) m[q] *= rl;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) m[q] = chol ? y[q] : -m[q];
    return ok;
}

// The slot word, opaque to the optimiser at each use: keeps the per-slot LDS
// addresses from being hoisted out of the step loops (15 slots x 2 arrays of
// live addresses would not fit beside the tiles). For the same reason the
// slot loops below end each slot with a scheduling barrier: the operands of
// all slots loaded together would not fit either.
__device__ __forceinline__ int slot_word(int v) {
    asm volatile("" : "+s"(v));
    return v;
}

// The constants a tile element takes where it has no entry of A: 0, or 1 on
// the diagonal of the padding.
__device__ double rr_zero_one[2] = {0.0, 1.0};   // global, like A, so the loads stay global loads

// Persistent: one workgroup per CU pops rows of order[0 .. nrows). The order
// is cut into chunks of RR_CHUNK consecutive rows (neighbours in space, which
// share most blocks of A), and chunk c goes to XCD c % nx (workgroups are
// dealt to the XCDs in turn; nx = min(8, grid)), each XCD popping from its
// own counter, so that a chunk's rows meet in one L2.
// bmul = ceil(2^16 / b): x / b = (x * bmul) >> 16 for 0 <= x < 2^16 / b.
constexpr int RR_CHUNK = 32;
__global__ __launch_bounds__(RR_NT) void k_fsai_setup_rr(int64_t nrows, const int64_t* __restrict__ order, int b,
                                                         int bmul, const int* __restrict__ a_rowptr,
                                                         const int* __restrict__ a_col,
                                                         const double* __restrict__ a_vals,
                                                         const int64_t* __restrict__ p_rowptr,
                                                         const int* __restrict__ p_col, double* __restrict__ g_vals,
                                                         int* xcd_counters, int* bad_row) {
    constexpr int PANEL = RR_TMAX * 256;
    // panel row c in buffer c & 1 (-U_c. and W_c.); the block map lives in pw's
    // buffer 1 during the fill, V in pw's buffer 0 and S in pu's buffer 0
    // during the back-substitution
    __shared__ double pu[2 * PANEL];
    __shared__ double pw[2 * PANEL];
    __shared__ double dg[PANEL];        // the diagonal tiles U_aa
    __shared__ double dinv[2 * 256];    // D_a^{-1} in buffer a & 1; X = R_{T-1}^{-1} for a = T - 1
    __shared__ int sh_flag, f_dinv, f_wcrit, f_diag, v_done;
    __shared__ int s_next[RR_TMAX];
    __shared__ int64_t sh_next;
    int* idx = reinterpret_cast<int*>(pw + PANEL);
    double* vv = pw;
    static_assert(FSAI_MAXM * FSAI_MAXM * sizeof(int) <= PANEL * sizeof(double), "block map must fit");
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, j = lane & 15;
    const int nx = min((int)gridDim.x, 8), xcd = (int)blockIdx.x % nx;
    for (;;) {
        if (tid == 0) {
            const int64_t i = atomicAdd(xcd_counters + xcd, 1);
            const int64_t it = ((i / RR_CHUNK) * nx + xcd) * RR_CHUNK + i % RR_CHUNK;
            sh_next = it < nrows ? it : -1;
        }
        __syncthreads();
        const int64_t it = sh_next;
        __syncthreads();
        if (it < 0) break;
        const int64_t k = order[it];
        const int64_t p0 = p_rowptr[k];
        const int m = __builtin_amdgcn_readfirstlane((int)(p_rowptr[k + 1] - p0));
        const int n = m * b;
        const int T = (n + 15) >> 4;
        const int pad = 16 * T - n;
        const int* cols = p_col + p0;
        // block map idx[x m + y] = position of A[P_x, P_y] in A (or -1), all x, y
        constexpr int IS = 4;
        for (int t0 = tid; t0 < m * m; t0 += IS * RR_NT) {
            int lo[IS], hi[IS], end[IS], want[IS];
#pragma unroll
            for (int s = 0; s < IS; ++s) {
                const int t = t0 + s * RR_NT;
                lo[s] = hi[s] = end[s] = 0;
                want[s] = -1;
                if (t < m * m) {
                    const int x = t / m, y = t - x * m;
                    const int row = cols[x];
                    lo[s] = a_rowptr[row];
                    hi[s] = end[s] = a_rowptr[row + 1];
                    want[s] = cols[y];
                }
            }
            for (;;) {
                bool any = false;
#pragma unroll
                for (int s = 0; s < IS; ++s) {
                    if (lo[s] < hi[s]) {
                        any = true;
                        const int mid = (lo[s] + hi[s]) >> 1;
                        if (a_col[mid] < want[s]) lo[s] = mid + 1; else hi[s] = mid;
                    }
                }
                if (!any) break;
            }
#pragma unroll
            for (int s = 0; s < IS; ++s) {
                const int t = t0 + s * RR_NT;
                if (t < m * m) idx[t] = (want[s] >= 0 && lo[s] < end[s] && a_col[lo[s]] == want[s]) ? lo[s] : -1;
            }
        }
        if (tid == 0) {
            sh_flag = 1;
            f_dinv = f_wcrit = f_diag = -1;
            v_done = T - 1;
            for (int a = 0; a < T; ++a) s_next[a] = T - 1;
        }
        __syncthreads();
        // Element (4q + g, j) of tile U_ab is Kpad[16 a + 4q + g][16 b + j].
        // Each element is one load straight into its register, from A or, for
        // a missing block, a padding entry or an unused slot, from the
        // constants {0, 1}: no branches and nothing to do after the loads.
        // fill_map looks up the block map for a tile's 4 elements (clamped
        // positions are in range), fill_load issues its loads; the callers
        // run the lookups of several tiles before their loads, so that the
        // LDS latency is paid once per group and the loads overlap.
        auto fill_map = [&](int a, int bt, int (&e)[4]) {
            const int pcc = max(16 * bt + j - pad, 0);
            const int y = (pcc * bmul) >> 16;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int prc = max(16 * a + 4 * q + g - pad, 0);
                e[q] = idx[((prc * bmul) >> 16) * m + y];
            }
        };
        auto fill_load = [&](int a, int bt, bool use, const int (&e)[4], v4d& t) {
            const int pc = 16 * bt + j - pad;
            const int pcc = max(pc, 0);
            const int ry = pcc - ((pcc * bmul) >> 16) * b;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int pr = 16 * a + 4 * q + g - pad;
                const int prc = max(pr, 0);
                const int rx = prc - ((prc * bmul) >> 16) * b;
                const bool real = pr >= 0 && pc >= 0;
                const double* src = use && real && e[q] >= 0
                                        ? a_vals + ((int64_t)e[q] * b * b + rx * b + ry)
                                        : rr_zero_one + ((use && !real && pr == pc) ? 1 : 0);
                t[q] = *src;
            }
        };
        // Roles. Wavefront 0 runs the chain of diagonal inverses and holds no
        // tile. The diagonal tiles sit in LDS, tile a updated by wavefront
        // 1 + a % 7. The off-diagonal tiles, listed by tile row descending and
        // column ascending, are dealt in turn to wavefronts 1..7: slot s of
        // wavefront w holds list entry 7 s + w - 1. The two roles run separate
        // loops that cross the same barriers in the same order (every count
        // below depends on T only), so that the tiles' registers are not live
        // in the chain's code and the inverse's temporaries not in the tiles'.
        //
        // Steps c = -1 .. T - 2 (block LDL^T with a look-ahead of one step),
        // one barrier each; n1 = c + 1, n2 = c + 2. At the start of step c,
        // panel row c is in buffer c & 1 and D_{n1}^{-1} is ready (step -1
        // makes D_0^{-1} itself). In step c:
        //  - the owner of U_{n1,n2} updates it with panel row c, forms
        //    W_{n1,n2} = D_{n1}^{-1} U_{n1,n2} at once and publishes it
        //    (f_wcrit); the updater of U_{n2,n2} updates it with panel row c
        //    and publishes that (f_diag);
        //  - the chain takes D_{n2} = U_{n2,n2} - U_{n1,n2}^T W_{n1,n2} (its
        //    last update) and inverts it, the last one (T - 1) by its Cholesky
        //    factor, while
        //  - the others update their tiles with panel row c and then write
        //    panel row n1 to buffer n1 & 1, their tiles becoming W^T.
        // D^{-1} is stored symmetrised: its rounding asymmetry would otherwise
        // grow step by step through the Schur updates.
        auto wait_eq = [&](int* f, int v) {   // bounded; a wait that runs out fails the row
            for (int spin = 0; __hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != v; ++spin) {
                if (spin > (1 << 14)) {
                    if (lane == 0) sh_flag = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        };
        auto publish = [&](int* f, int v) { __hip_atomic_store(f, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP); };
        auto wait_le = [&](int* f, int v) {   // bounded, for the decreasing counter of finished V tiles
            for (int spin = 0; __hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) > v; ++spin) {
                if (spin > (1 << 14)) {
                    if (lane == 0) sh_flag = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        };
        for (int a = w; a < T; a += RR_WAVES) {
            int e[4];
            v4d d;
            fill_map(a, a, e);
            fill_load(a, a, true, e, d);
#pragma unroll
            for (int q = 0; q < 4; ++q) dg[a * 256 + 64 * q + lane] = d[q];
        }
        bool ok_row;
        if (w == 0) {
            // ----------------------------------------------------- the chain
            __syncthreads();
            for (int c = -1; c + 1 < T; ++c) {
                const int n2 = c + 2;
                // step -1 inverts D_0 (and publishes it), then D_1; later steps D_{n2}
#pragma unroll 1
                for (int a = c < 0 ? 0 : n2; a <= n2 && a < T; ++a) {
                    const double* pua = pu + ((a - 1) & 1) * PANEL;   // panel row a - 1
                    const double* pwa = pw + ((a - 1) & 1) * PANEL;
                    if (a > 0) {
                        wait_eq(&f_wcrit, a - 1);
                        wait_eq(&f_diag, a);
                    }
                    v4d d;   // read only once its updater has published it
#pragma unroll
                    for (int q = 0; q < 4; ++q) d[q] = dg[a * 256 + 64 * q + lane];
                    if (a > 0) {
#pragma unroll
                        for (int q = 0; q < 4; ++q)   // the panel holds -U
                            d = mfma16(pua[a * 256 + 64 * q + lane], pwa[a * 256 + 64 * q + lane], d);
                    }
                    double* di = dinv + (a & 1) * 256;   // D_a^{-1}, or X for a = T - 1
                    bool ok;
                    if (a + 1 < T) {
                        ok = tile_inverse<false>(d, lane);
#pragma unroll
                        for (int q = 0; q < 4; ++q) di[64 * q + lane] = d[q];
                        double dt[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) dt[q] = di[j * 16 + 4 * q + g];
#pragma unroll
                        for (int q = 0; q < 4; ++q) di[64 * q + lane] = 0.5 * (d[q] + dt[q]);
                    } else {
                        ok = tile_inverse<true>(d, lane);
#pragma unroll
                        for (int q = 0; q < 4; ++q) di[64 * q + lane] = d[q];
                    }
                    if (!ok && lane == 0) sh_flag = 0;
                    if (a == 0) publish(&f_dinv, 0);
                }
                __syncthreads();
            }
            ok_row = sh_flag != 0;
            if (ok_row) {
                // Y_a = X V_a as soon as V_a is out (V_{T-1} = I), to dg
                const double* xl = dinv + ((T - 1) & 1) * 256;   // X = R_{T-1}^{-1}
                for (int a = T - 1; a >= 0; --a) {
                    v4d y = {0.0, 0.0, 0.0, 0.0};
                    if (a == T - 1) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) y[q] = xl[64 * q + lane];
                    } else {
                        wait_le(&v_done, a);
#pragma unroll
                        for (int q = 0; q < 4; ++q) y = mfma16(xl[j * 16 + 4 * q + g], vv[a * 256 + 64 * q + lane], y);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) dg[a * 256 + 64 * q + lane] = y[q];
                }
            }
        } else {
            // ------------------------------------------------------ the tiles
            int ab[RR_SLOTS];   // slot s: tile (ab[s] >> 8, ab[s] & 255); < 0 if unused
            {
                const int noff = T * (T - 1) / 2;
#pragma unroll
                for (int s = 0; s < RR_SLOTS; ++s) {
                    int v = -1;
                    const int i = 7 * s + w - 1;
                    if (i < noff) {
                        int r, o;
                        tri_decode(i, r, o);
                        v = (T - 2 - r) * 256 + (T - 1 - r + o);
                    }
                    ab[s] = __builtin_amdgcn_readfirstlane(v);
                }
            }
            v4d t[RR_SLOTS];
            constexpr int FG = 5;   // slots per fill group
            static_assert(RR_SLOTS % FG == 0, "fill groups");
#pragma unroll
            for (int s0 = 0; s0 < RR_SLOTS; s0 += FG) {
                int e[FG][4];
#pragma unroll
                for (int s = s0; s < s0 + FG; ++s) {   // unused slots read zeros through tile (0, 0)
                    const bool use = ab[s] >= 0;
                    fill_map(use ? ab[s] >> 8 : 0, use ? ab[s] & 255 : 0, e[s - s0]);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int s = s0; s < s0 + FG; ++s) {
                    const bool use = ab[s] >= 0;
                    fill_load(use ? ab[s] >> 8 : 0, use ? ab[s] & 255 : 0, use, e[s - s0], t[s]);
                }
            }
            __syncthreads();
            for (int c = -1; c + 1 < T; ++c) {
                const int n1 = c + 1, n2 = c + 2;
                const double* puc = pu + (c & 1) * PANEL;
                const double* pwc = pw + (c & 1) * PANEL;
                double* pun = pu + (n1 & 1) * PANEL;
                double* pwn = pw + (n1 & 1) * PANEL;
                const double* din1 = dinv + (n1 & 1) * 256;
                if (c < 0) wait_eq(&f_dinv, 0);
                // panel tile of row n1: W = Dinv U and W^T = U^T Dinv
                auto panel = [&](v4d& tt, int bt) {
                    double xa[4];   // D_{n1}^{-1}[j][4q+g] (symmetric)
#pragma unroll
                    for (int q = 0; q < 4; ++q) xa[q] = din1[64 * q + lane];
                    v4d wv = {0.0, 0.0, 0.0, 0.0}, wt = wv;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        wv = mfma16(xa[q], tt[q], wv);
                        wt = mfma16(tt[q], xa[q], wt);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        pun[bt * 256 + 64 * q + lane] = -tt[q];   // -U: the updates then accumulate
                        pwn[bt * 256 + 64 * q + lane] = wv[q];
                    }
                    tt = wt;
                };
                // U_ab -= U_ca^T W_cb with panel row c (its U held negated)
                auto update = [&](v4d& tt, int a, int bt) {
                    double pa[4], pb[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        pa[q] = puc[a * 256 + 64 * q + lane];    // -U_ca^T[j][4q+g]
                        pb[q] = pwc[bt * 256 + 64 * q + lane];   // W_cb[4q+g][j]
                    }
                    __builtin_amdgcn_sched_barrier(0);   // all 8 operands in flight together
#pragma unroll
                    for (int q = 0; q < 4; ++q) tt = mfma16(pa[q], pb[q], tt);
                };
                if (n2 < T) {
                    // the critical tile (n1, n2) first
#pragma unroll
                    for (int s = 0; s < RR_SLOTS; ++s) {
                        if (slot_word(ab[s]) == n1 * 256 + n2) {
                            if (c >= 0) update(t[s], n1, n2);
                            panel(t[s], n2);
                            publish(&f_wcrit, n1);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    // then the diagonal tile n2
                    if (w == 1 + n2 % 7) {
                        if (c >= 0) {
                            v4d d;
#pragma unroll
                            for (int q = 0; q < 4; ++q) d[q] = dg[n2 * 256 + 64 * q + lane];
                            update(d, n2, n2);
#pragma unroll
                            for (int q = 0; q < 4; ++q) dg[n2 * 256 + 64 * q + lane] = d[q];
                        }
                        publish(&f_diag, n2);
                    }
                }
                if (c >= 0) {
                    // the other diagonal tiles still to come (a > n2)
                    for (int a = n2 + 1; a < T; ++a) {
                        if (w != 1 + a % 7) continue;
                        v4d d;
#pragma unroll
                        for (int q = 0; q < 4; ++q) d[q] = dg[a * 256 + 64 * q + lane];
                        update(d, a, a);
#pragma unroll
                        for (int q = 0; q < 4; ++q) dg[a * 256 + 64 * q + lane] = d[q];
                    }
                    // the off-diagonal tiles
#pragma unroll
                    for (int s = 0; s < RR_SLOTS; ++s) {
                        const int v = slot_word(ab[s]);
                        const int a = v >> 8, bt = v & 255;
                        if (v >= 0 && a > c && v != n1 * 256 + n2) update(t[s], a, bt);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                // panel row n1 (but the critical tile)
#pragma unroll
                for (int s = 0; s < RR_SLOTS; ++s) {
                    const int v = slot_word(ab[s]);
                    const int a = v >> 8, bt = v & 255;
                    if (v >= 0 && a == n1 && bt > n2) panel(t[s], bt);
                    __builtin_amdgcn_sched_barrier(0);
                }
                __syncthreads();
            }
            // a failed pivot is reported after all steps: the steps only ever
            // address tiles by slot, so values gone bad are harmless
            ok_row = sh_flag != 0;
            if (ok_row) {
                // V_{T-1} = I, V_a = -S_a with S_a = sum_{b > a} V_b W_ab^T, as a
                // dataflow: each tile (a, b), by b descending, waits for V_b
                // (v_done <= b) and for row a's sum to hold the terms above b
                // (s_next[a] == b), adds its term in pu (a fixed order) and
                // publishes; the tile (a, a + 1) finishes V_a. Every wait is on
                // a tile of larger b, so the waits end.
                for (int jt = T - 1; jt >= 1; --jt) {
#pragma unroll
                    for (int s = 0; s < RR_SLOTS; ++s) {
                        const int v = slot_word(ab[s]);
                        const int a = v >> 8, bt = v & 255;
                        if (v >= 0 && bt == jt && a < jt) {
                            v4d acc;
                            if (jt == T - 1) {
                                acc = t[s];
                            } else {
                                wait_le(&v_done, jt);
                                wait_eq(&s_next[a], jt);
#pragma unroll
                                for (int q = 0; q < 4; ++q) acc[q] = pu[a * 256 + 64 * q + lane];
#pragma unroll
                                for (int q = 0; q < 4; ++q)
                                    acc = mfma16(vv[jt * 256 + j * 16 + 4 * q + g], t[s][q], acc);   // V_jt[j][4q+g]
                            }
                            if (a == jt - 1) {
#pragma unroll
                                for (int q = 0; q < 4; ++q) vv[a * 256 + 64 * q + lane] = -acc[q];
                                publish(&v_done, a);
                            } else {
#pragma unroll
                                for (int q = 0; q < 4; ++q) pu[a * 256 + 64 * q + lane] = acc[q];
                                publish(&s_next[a], jt - 1);
                            }
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
        }
        if (ok_row) {
            __syncthreads();
            ok_row = sh_flag != 0;   // a wait of the back-substitution that ran out
        }
        if (!ok_row) {
            if (tid == 0) atomicMin(bad_row, (int)k);
            for (int64_t e = tid; e < (int64_t)m * b * b; e += RR_NT) g_vals[p0 * b * b + e] = 0.0;
            __syncthreads();
            continue;
        }
        // G_k[t][x b + cc] = row 16 - b + t of the last tile row, column pad + x b + cc
        const int bb = b * b;
        for (int e = tid; e < m * bb; e += RR_NT) {
            const int x = e / bb, rem = e - x * bb;
            const int tr = rem / b, cc = rem - tr * b;
            const int p = pad + x * b + cc;
            g_vals[(p0 + x) * bb + rem] = dg[(p >> 4) * 256 + (16 - b + tr) * 16 + (p & 15)];
        }
        __syncthreads();
    }
}

// Persistent kernel: each workgroup pops rows (ordered by decreasing local
// size, less the range [skip_lo, skip_lo + skip_len) of the order) from a
// global counter until the queue is empty. Per row, by size:
// the tiled MFMA solver (n > ntile, 256-wide workgroups, b <= 16), the
// scalar solver in LDS (n <= nlds), or the scalar solver in the workgroup's
// global scratch slot.
template <int NT>
__global__ __launch_bounds__(NT) void k_fsai_setup(int64_t nrows, const int64_t* __restrict__ order, int b,
                                                   const int* __restrict__ a_rowptr, const int* __restrict__ a_col,
                                                   const double* __restrict__ a_vals,
                                                   const int64_t* __restrict__ p_rowptr, const int* __restrict__ p_col,
                                                   double* __restrict__ g_vals, int nlds, int ntile, int tmaxtiles,
                                                   double* scratch, int64_t scratch_stride, int* counter,
                                                   int* bad_row, int64_t skip_lo, int64_t skip_len) {
    extern __shared__ double lds[];
    __shared__ int idx[FSAI_MAXM * FSAI_MAXM];
    __shared__ double sh_scal[1];
    __shared__ int sh_flag[1];
    __shared__ int sh_next;
    double* lds_K = lds;
    double* lds_Z = lds + (int64_t)nlds * (nlds + 1) / 2;
    double* gK = scratch + (int64_t)blockIdx.x * scratch_stride;
    double* gZ = gK + (int64_t)FSAI_MAXN * (FSAI_MAXN + 1) / 2;
    for (;;) {
        if (threadIdx.x == 0) sh_next = atomicAdd(counter, 1);
        __syncthreads();
        int64_t it = sh_next;
        __syncthreads();
        if (it >= nrows) break;
        if (it >= skip_lo) it += skip_len;   // order[skip_lo .. skip_lo + skip_len) went to another kernel
        const int64_t k = order[it];
        const int n = (int)(p_rowptr[k + 1] - p_rowptr[k]) * b;
        if constexpr (NT == 256) {
            if (n > ntile && b <= 16) {
                double* panel = lds;
                double* part = panel + (int64_t)tmaxtiles * 256;
                // inverses of the diagonal tiles: global, after the tiles
                double* invs = gK + (int64_t)tmaxtiles * (tmaxtiles + 1) / 2 * 256;
                fsai_row_tiled(k, b, a_rowptr, a_col, a_vals, p_rowptr, p_col, g_vals, gK, panel, invs, part,
                               idx, sh_flag, bad_row);
                continue;
            }
        }
        if (n <= nlds)
            fsai_row<NT>(k, b, a_rowptr, a_col, a_vals, p_rowptr, p_col, g_vals, lds_K, lds_Z, idx, sh_scal,
                         sh_flag, bad_row);
        else
            fsai_row<NT>(k, b, a_rowptr, a_col, a_vals, p_rowptr, p_col, g_vals, gK, gZ, idx, sh_scal, sh_flag,
                         bad_row);
    }
}

// ------------------------------------------------------------ autotuning --
// A configuration is a workgroup width (64, 128, 256), a size threshold
// above which rows take the tiled MFMA path (256-wide only), and a threshold
// above which rows of at most RR_MAXN take the register-resident kernel. The
// best one for (b, largest local size) is picked by timing the set-up on an
// evenly strided sample of the rows, and cached for the process.
struct TuneKey {
    int b, nmax;
    bool operator<(const TuneKey& o) const { return b != o.b ? b < o.b : nmax < o.nmax; }
};
struct TuneVal {
    int nt, ntile, rr_lo;
};
static std::map<TuneKey, TuneVal> g_tuned;
static std::mutex g_tune_mu;
constexpr int NO_TILES = 1 << 30;

struct SetupArgs {
    int64_t nrows;
    const int64_t* order;
    int b;
    const int* a_rowptr;
    const int* a_col;
    const double* a_vals;
    const int64_t* p_rowptr;
    const int* p_col;
    double* g_vals;
    int nlds;
    int* counter;
    int* bad_row;
    int nmax;
    const int* nsz;      // host: local size of order[i], non-increasing
    int* xcd_counters;   // 8 counters of the register-resident kernel
};

static size_t lds_bytes(int nlds, int b) {
    return ((size_t)nlds * (nlds + 1) / 2 + (size_t)nlds * b) * sizeof(double);
}

// Launches the persistent set-up kernel on s and returns without waiting;
// `scratch` (the workgroups' global slots) must outlive the launch.
static void launch_setup(TuneVal cfg, const SetupArgs& a, hipStream_t s, DevBuf<double>& scratch) {
    const int cus = device_cu_count();
    const bool tiled = cfg.nt == 256 && a.b <= 16 && a.nmax > cfg.ntile;
    const int tmaxtiles = (a.nmax + 15) / 16;
    // rows above the tile threshold never use the scalar LDS solver, so its
    // buffer only needs the threshold's size (more workgroups per CU)
    const int nlds = tiled ? std::min(a.nlds, cfg.ntile) : a.nlds;
    size_t shm = lds_bytes(nlds, a.b);
    if (tiled) shm = std::max(shm, ((size_t)tmaxtiles * 256 + 5 * 256) * sizeof(double));
    int dev = 0, lim = 0;
    CHF_HIP(hipGetDevice(&dev));
    CHF_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    int per_cu = std::max<int>(1, (int)std::min<size_t>(8, (size_t)lim / (shm + 4096 + 64)));
    int64_t grid = std::min<int64_t>((int64_t)cus * per_cu, std::max<int64_t>(1, a.nrows));
    int64_t stride = (int64_t)FSAI_MAXN * (FSAI_MAXN + 1) / 2 + (int64_t)FSAI_MAXN * a.b;
    if (tiled)
        stride = std::max<int64_t>(stride, (int64_t)tmaxtiles * (tmaxtiles + 1) / 2 * 256 + (int64_t)tmaxtiles * 256);
    // global scratch only when some row exceeds the LDS limit or is tiled;
    // the buffer only grows, so repeated launches (the autotuner) reuse it
    const size_t need = (a.nmax > nlds || tiled) ? (size_t)grid * stride : 1;
    if (scratch.n < need) scratch.alloc(need);
    double* scr = scratch.p;
    // rows with rr_lo < n <= RR_MAXN: one contiguous range of the size-sorted order
    int64_t rr0 = 0, rr1 = 0;
    if (cfg.rr_lo < NO_TILES && a.b <= 16) {
        rr0 = std::partition_point(a.nsz, a.nsz + a.nrows, [](int v) { return v > RR_MAXN; }) - a.nsz;
        rr1 = std::partition_point(a.nsz, a.nsz + a.nrows, [&](int v) { return v > cfg.rr_lo; }) - a.nsz;
        rr1 = std::max(rr1, rr0);
    }
    if (rr1 > rr0) {
        fill_zero(a.xcd_counters, 8 * sizeof(int), s);
        const int bmul = (65536 + a.b - 1) / a.b;
        hipLaunchKernelGGL(k_fsai_setup_rr, dim3((unsigned)std::min<int64_t>(cus, rr1 - rr0)), dim3(RR_NT), 0, s,
                           rr1 - rr0, a.order + rr0, a.b, bmul, a.a_rowptr, a.a_col, a.a_vals, a.p_rowptr, a.p_col,
                           a.g_vals, a.xcd_counters, a.bad_row);
        CHF_LAUNCH_CHECK();
    }
    const int64_t rest = a.nrows - (rr1 - rr0);
    if (rest == 0) return;
    grid = std::min<int64_t>(grid, rest);
    fill_zero(a.counter, sizeof(int), s);
    if (shm > 64 * 1024) {
        CHF_HIP(hipFuncSetAttribute((const void*)k_fsai_setup<64>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        CHF_HIP(hipFuncSetAttribute((const void*)k_fsai_setup<128>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        CHF_HIP(hipFuncSetAttribute((const void*)k_fsai_setup<256>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    }
    auto go = [&](auto kern, int nt) {
        // the queue holds the `rest` rows outside [rr0, rr1): popped indices
        // at or above rr0 are shifted past that range, so stay below nrows
        hipLaunchKernelGGL(kern, dim3(grid), dim3(nt), shm, s, rest, a.order, a.b, a.a_rowptr, a.a_col, a.a_vals,
                           a.p_rowptr, a.p_col, a.g_vals, nlds, cfg.ntile, tmaxtiles, scr, stride, a.counter,
                           a.bad_row, rr0, rr1 - rr0);
    };
    switch (cfg.nt) {
        case 64: go(k_fsai_setup<64>, 64); break;
        case 128: go(k_fsai_setup<128>, 128); break;
        default: go(k_fsai_setup<256>, 256); break;
    }
    CHF_LAUNCH_CHECK();
}

static TuneVal pick_config(const SetupArgs& a, const std::vector<int64_t>& order_host, hipStream_t s) {
    const int nmax = a.nmax;
    if (const char* env = std::getenv("CHF_FSAI_CONFIG")) {   // "<width>,<tile threshold>[,<rr threshold>]"
        int w = 0, t = 0, r = -1;
        const int got = std::sscanf(env, "%d,%d,%d", &w, &t, &r);
        if (got >= 2 && (w == 64 || w == 128 || w == 256))
            return TuneVal{w, t > 0 ? t : NO_TILES, got == 3 && r >= 0 ? r : NO_TILES};
    }
    TuneKey key{a.b, nmax};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) return it->second;
    }
    std::vector<TuneVal> cands = {{64, NO_TILES, NO_TILES}, {128, NO_TILES, NO_TILES}, {256, NO_TILES, NO_TILES}};
    if (a.b <= 16 && nmax > 32) {
        cands.push_back({256, 32, NO_TILES});
        if (nmax > 48) cands.push_back({256, 48, NO_TILES});
        if (nmax > 96) cands.push_back({256, 96, NO_TILES});
        if (nmax > 160) cands.push_back({256, 160, NO_TILES});
        // the register-resident kernel for the rows above 96 or 160, the rest as tuned above
        const size_t nbase = cands.size();
        for (int lo : {96, 160}) {
            if (nmax <= lo) continue;
            for (size_t i = 0; i < nbase; ++i) cands.push_back({cands[i].nt, cands[i].ntile, lo});
        }
    }
    TuneVal best = nmax > 64 ? TuneVal{128, NO_TILES, NO_TILES} : TuneVal{64, NO_TILES, NO_TILES};
    if (a.nrows >= 4096) {
        // evenly strided samples of the size-sorted order keep the size mix
        auto sample = [&](int64_t ns, std::vector<int>& sz) {
            std::vector<int64_t> o(std::min<int64_t>(ns, a.nrows));
            sz.resize(o.size());
            for (size_t i = 0; i < o.size(); ++i) {
                const int64_t pos = (int64_t)i * a.nrows / (int64_t)o.size();
                o[i] = order_host[pos];
                sz[i] = a.nsz[pos];
            }
            return o;
        };
        DevBuf<double> scratch;
        // seconds of one launch on `rows` (device order), after a warm-up launch
        auto time_on = [&](const TuneVal& c, const DevBuf<int64_t>& rows, int64_t n, const std::vector<int>& sz) {
            SetupArgs smp = a;
            smp.nrows = n;
            smp.order = rows.p;
            smp.nsz = sz.data();
            launch_setup(c, smp, s, scratch);
            CHF_HIP(hipStreamSynchronize(s));
            auto t0 = std::chrono::steady_clock::now();
            launch_setup(c, smp, s, scratch);
            CHF_HIP(hipStreamSynchronize(s));
            return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        };
        // screening on 1,024 rows drops candidates more than twice as slow as
        // the best one (the scalar solvers on wide rows are tens of times slower)
        std::vector<int> sz_small, sz_full;
        const std::vector<int64_t> small = sample(1024, sz_small), full = sample(8192, sz_full);
        DevBuf<int64_t> d_small(small.size()), d_full(full.size());
        d_small.upload(small.data(), small.size(), s);
        d_full.upload(full.data(), full.size(), s);
        std::vector<double> ts(cands.size());
        double ts_best = 1e30;
        for (size_t i = 0; i < cands.size(); ++i) {
            ts[i] = time_on(cands[i], d_small, (int64_t)small.size(), sz_small);
            ts_best = std::min(ts_best, ts[i]);
        }
        double best_t = 1e30;
        for (size_t i = 0; i < cands.size(); ++i) {
            if (ts[i] > 2.0 * ts_best) continue;
            const double dt = time_on(cands[i], d_full, (int64_t)full.size(), sz_full);
            if (dt < best_t) { best_t = dt; best = cands[i]; }
        }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = best;
    return best;
}

static int max_lds_n(int b) {
    int dev = 0;
    CHF_HIP(hipGetDevice(&dev));
    int lim = 0;
    CHF_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // static LDS: index table + scalars
    size_t avail = (size_t)lim - (FSAI_MAXM * FSAI_MAXM * 4 + 64);
    int n = FSAI_MAXN;
    while (n > 0 && lds_bytes(n, b) > avail) --n;
    return n;
}

// ----------------------------------------------------------- G^T builder --
static void build_transpose_structure(const chf_fsai_s& G, std::vector<int64_t>& trow, std::vector<int32_t>& tcol,
                                      std::vector<int64_t>& tsrc) {
    int64_t nb = G.nb;
    trow.assign(nb + 1, 0);
    for (int64_t e = 0; e < G.nnz; ++e) trow[G.colidx[e] + 1]++;
    for (int64_t j = 0; j < nb; ++j) trow[j + 1] += trow[j];
    tcol.assign(G.nnz, 0);
    tsrc.assign(G.nnz, 0);
    std::vector<int64_t> fillp(trow.begin(), trow.end() - 1);
    for (int64_t i = 0; i < nb; ++i)          // rows ascending -> stable, columns of G^T ascend
        for (int64_t e = G.rowptr[i]; e < G.rowptr[i + 1]; ++e) {
            int64_t j = G.colidx[e];
            int64_t pos = fillp[j]++;
            tcol[pos] = (int32_t)i;
            tsrc[pos] = e;
        }
}

// SpMV layouts of G and G^T: their structure depends on the pattern only
// (host work), the packing of the values needs the factor (device work).
static void fsai_plan_layouts(chf_fsai_s& G) {
    G.plan_g = sell_plan(G.nb, G.b, G.rowptr, G.colidx, nullptr);
    std::vector<int64_t> trow, tsrc;
    std::vector<int32_t> tcol;
    build_transpose_structure(G, trow, tcol, tsrc);
    G.plan_gt = sell_plan(G.nb, G.b, trow, tcol, &tsrc);
}

static void fsai_pack_layouts(chf_fsai_s& G, hipStream_t s) {
    sell_build(G.g64, G.plan_g, G.d_vals.p, false, CHF_F64, s);
    sell_build(G.gt64, G.plan_gt, G.d_vals.p, true, CHF_F64, s);
    if (G.store != CHF_F64) {
        sell_build(G.g_lo, G.plan_g, G.d_vals.p, false, G.store, s);
        sell_build(G.gt_lo, G.plan_gt, G.d_vals.p, true, G.store, s);
    }
}

void validate_pattern(int64_t nb, const int64_t* rowptr, const int32_t* colidx) {
    CHF_CHECK(rowptr && rowptr[0] == 0, CHF_EINVAL, "pattern rowptr[0] must be 0");
    for (int64_t k = 0; k < nb; ++k) {
        int64_t lo = rowptr[k], hi = rowptr[k + 1];
        CHF_CHECK(hi > lo, CHF_EINVAL, "pattern row " + std::to_string(k) + " is empty (diagonal missing)");
        CHF_CHECK(colidx[hi - 1] == k, CHF_EINVAL,
                  "pattern row " + std::to_string(k) + ": diagonal missing or entry above the diagonal");
        for (int64_t e = lo; e < hi; ++e) {
            CHF_CHECK(colidx[e] >= 0, CHF_EINVAL, "negative pattern column");
            CHF_CHECK(e == lo || colidx[e] > colidx[e - 1], CHF_EINVAL,
                      "pattern row " + std::to_string(k) + ": columns not strictly ascending");
        }
    }
}

chf_fsai_s* fsai_setup_impl(chf_bsr A, const chf_pattern_s& P, chf_dtype g_store, int64_t* bad_row,
                            hipStream_t s) {
    CHF_CHECK(P.nb == A->nb, CHF_EINVAL, "pattern and matrix sizes differ");
    const int b = A->b;
    const int64_t nb = A->nb;
    std::unique_ptr<chf_fsai_s> G(new chf_fsai_s);
    G->nb = nb;
    G->b = b;
    G->store = g_store;
    G->rowptr = P.rowptr;
    G->colidx = P.colidx;
    G->nnz = P.rowptr[nb];
    int nmax = 0;
    for (int64_t k = 0; k < nb; ++k) {
        int64_t m = P.rowptr[k + 1] - P.rowptr[k];
        CHF_CHECK(m <= FSAI_MAXM && m * b <= FSAI_MAXN, CHF_EINVAL,
                  "pattern row " + std::to_string(k) + " too large for the local solver");
        nmax = std::max<int>(nmax, (int)(m * b));
    }
    // queue order: local size descending, then row index
    std::vector<int64_t> order(nb);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
        return P.rowptr[x + 1] - P.rowptr[x] > P.rowptr[y + 1] - P.rowptr[y];
    });
    std::vector<int> nsz(nb);
    for (int64_t i = 0; i < nb; ++i) nsz[i] = (int)(P.rowptr[order[i] + 1] - P.rowptr[order[i]]) * b;
    std::vector<int> pcol32(P.colidx.begin(), P.colidx.end());
    DevBuf<int64_t> d_order(std::max<int64_t>(1, nb)), d_prow(nb + 1);
    DevBuf<int> d_pcol(std::max<int64_t>(1, G->nnz)), d_flags(10);   // counter, bad row, 8 XCD counters
    d_order.upload(order.data(), nb, s);
    d_prow.upload(P.rowptr.data(), nb + 1, s);
    d_pcol.upload(pcol32.data(), G->nnz, s);
    int init[2] = {0, INT32_MAX};
    d_flags.upload(init, 2, s);
    G->d_vals.alloc(std::max<int64_t>(1, G->nnz * b * b));
    if (nb > 0) {
        SetupArgs args{nb, d_order.p, b, A->d_rowptr.p, A->d_colidx.p, A->d_vals.p, d_prow.p, d_pcol.p,
                       G->d_vals.p, std::min(max_lds_n(b), nmax), d_flags.p, d_flags.p + 1, nmax, nsz.data(),
                       d_flags.p + 2};
        TuneVal cfg = pick_config(args, order, s);
        DevBuf<double> scratch;
        launch_setup(cfg, args, s, scratch);
        // the host plans the layouts while the factorisation runs
        try {
            fsai_plan_layouts(*G);
        } catch (...) {
            (void)hipStreamSynchronize(s);   // the kernel still reads buffers freed on unwinding
            throw;
        }
        int flags[2];
        d_flags.download(flags, 2, s);
        CHF_HIP(hipStreamSynchronize(s));
        if (flags[1] != INT32_MAX) {
            if (bad_row) *bad_row = flags[1];
            fail(CHF_ENOTSPD, "local FSAI system of block row " + std::to_string(flags[1]) +
                                  " is not positive definite");
        }
    }
    if (nb == 0) fsai_plan_layouts(*G);
    fsai_pack_layouts(*G, s);
    CHF_HIP(hipStreamSynchronize(s));
    return G.release();
}

// ---------------------------------------------------------------- Lanczos --
// alpha_j = v . w, w <- w - alpha_j v - beta_{j-1} v_prev, beta_j = ||w||,
// v_next = w / beta_j. Scalars stay on the device; the host reads them once.
__global__ void k_lz_update(int64_t n, double* __restrict__ w, const double* __restrict__ v,
                            const double* __restrict__ vprev, const double* __restrict__ alpha_j,
                            const double* __restrict__ beta_prev) {
    const double a = alpha_j[0];
    const double bp = beta_prev ? beta_prev[0] : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        w[i] = w[i] - a * v[i] - bp * vprev[i];
}

__global__ void k_lz_scale(int64_t n, const double* __restrict__ w, double* __restrict__ vout,
                           const double* __restrict__ nrm2, double* __restrict__ beta_j) {
    const double bj = sqrt(nrm2[0]);
    const double inv = bj > 0.0 ? 1.0 / bj : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) beta_j[0] = bj;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        vout[i] = w[i] * inv;
}

__global__ void k_scale_by_rsqrt(int64_t n, const double* __restrict__ x, double* __restrict__ y,
                                 const double* __restrict__ nrm2) {
    const double inv = 1.0 / sqrt(nrm2[0]);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i] * inv;
}

void lanczos_impl(chf_bsr A, const chf_fsai_s& G, chf_dtype dt, int iters, const double* v0, double safety,
                  double* beta_out, double* theta_out, hipStream_t s) {
    const int64_t n = A->ndof;
    CHF_CHECK(iters >= 1, CHF_EINVAL, "iters must be >= 1");
    CHF_CHECK(!A->vb || dt == CHF_F64, CHF_EINVAL, "variable block sizes: FP64 only");
    const int m = (int)std::min<int64_t>(iters, n);
    const Sell& sa = A->sell(mode_vec(dt), s);
    const FactorOps fo = factor_ops(G, mode_g(dt));
    DevBuf<double> vbuf(3 * n), w(n), t1(n), scal(2 * m + 4), part(RED_BLOCKS);
    double* va = vbuf.p;
    double* vb = vbuf.p + n;
    double* vc = vbuf.p + 2 * n;
    double* alphas = scal.p;
    double* betas = scal.p + m;
    double* tmp = scal.p + 2 * m;
    int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
    dot(CHF_F64, v0, v0, n, tmp, part.p, s);
    hipLaunchKernelGGL(k_scale_by_rsqrt, dim3(grid), dim3(256), 0, s, n, v0, va, (const double*)tmp);
    CHF_LAUNCH_CHECK();
    fill_zero(vb, n * 8, s);
    double* v = va;
    double* vprev = vb;
    double* spare = vc;
    for (int j = 0; j < m; ++j) {
        // w = G A G^T v in FP64 arithmetic on the stored operators (nested:
        // G = G1 G0, so w = G1 G0 A G0^T G1^T v)
        if (fo.gi) {
            sell_spmv(*fo.git, CHF_F64, v, t1.p, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
            sell_spmv(*fo.gt, CHF_F64, t1.p, w.p, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
        } else {
            sell_spmv(*fo.gt, CHF_F64, v, w.p, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
        }
        sell_spmv(sa, CHF_F64, w.p, t1.p, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
        sell_spmv(*fo.g, CHF_F64, t1.p, w.p, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
        if (fo.gi) {
            sell_spmv(*fo.gi, CHF_F64, w.p, t1.p, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
            CHF_HIP(hipMemcpyAsync(w.p, t1.p, n * 8, hipMemcpyDeviceToDevice, s));
        }
        dot(CHF_F64, v, w.p, n, alphas + j, part.p, s);
        hipLaunchKernelGGL(k_lz_update, dim3(grid), dim3(256), 0, s, n, w.p, (const double*)v,
                           (const double*)vprev, (const double*)(alphas + j),
                           (const double*)(j > 0 ? betas + j - 1 : nullptr));
        CHF_LAUNCH_CHECK();
        if (j == m - 1) break;
        dot(CHF_F64, w.p, w.p, n, tmp, part.p, s);
        hipLaunchKernelGGL(k_lz_scale, dim3(grid), dim3(256), 0, s, n, (const double*)w.p, spare,
                           (const double*)tmp, betas + j);
        CHF_LAUNCH_CHECK();
        double* nv = spare;
        spare = vprev;
        vprev = v;
        v = nv;
    }
    std::vector<double> h(2 * m);
    CHF_HIP(hipMemcpyAsync(h.data(), scal.p, 2 * m * 8, hipMemcpyDeviceToHost, s));
    CHF_HIP(hipStreamSynchronize(s));
    std::vector<double> al, be;
    double amax = 0;
    for (int j = 0; j < m; ++j) {
        al.push_back(h[j]);
        amax = std::max(amax, std::fabs(h[j]));
        if (j == m - 1) break;
        double bj = h[m + j];
        if (!(bj >= 1e-12 * amax)) break;
        be.push_back(bj);
    }
    double theta = al.size() == 1 ? al[0] : tridiag_max_eig(al, be);
    CHF_CHECK(std::isfinite(theta) && theta > 0, CHF_EINVAL, "Lanczos produced a non-positive estimate");
    if (theta_out) *theta_out = theta;
    if (beta_out) *beta_out = safety * theta;
}

}  // namespace chf

using namespace chf;

extern "C" int chf_pattern_lower(chf_bsr A, chf_pattern* out) {
    return guarded([&] {
        CHF_CHECK(A && out, CHF_EINVAL, "NULL argument");
        std::unique_ptr<chf_pattern_s> P(new chf_pattern_s);
        P->nb = A->nb;
        P->rowptr.assign(A->nb + 1, 0);
        for (int64_t k = 0; k < A->nb; ++k) {
            bool diag = false;
            for (int64_t e = A->rowptr[k]; e < A->rowptr[k + 1]; ++e) {
                int32_t j = A->colidx[e];
                if (j < k) P->colidx.push_back(j);
                if (j == k) diag = true;
            }
            (void)diag;
            P->colidx.push_back((int32_t)k);
            P->rowptr[k + 1] = (int64_t)P->colidx.size();
        }
        *out = P.release();
    });
}

extern "C" int chf_pattern_from_csr(int64_t nb, const int64_t* rowptr, const int32_t* colidx, chf_pattern* out) {
    return guarded([&] {
        CHF_CHECK(out && nb >= 0 && rowptr && (nb == 0 || colidx), CHF_EINVAL, "bad argument");
        validate_pattern(nb, rowptr, colidx);
        std::unique_ptr<chf_pattern_s> P(new chf_pattern_s);
        P->nb = nb;
        P->rowptr.assign(rowptr, rowptr + nb + 1);
        P->colidx.assign(colidx, colidx + rowptr[nb]);
        *out = P.release();
    });
}

extern "C" int chf_pattern_template(int64_t nx, int64_t ny, int64_t nz, int32_t noff, const int32_t* offsets,
                                    chf_pattern* out) {
    return guarded([&] {
        CHF_CHECK(out && nx >= 1 && ny >= 1 && nz >= 1 && noff >= 0 && (noff == 0 || offsets), CHF_EINVAL,
                  "bad argument");
        std::vector<int64_t> lin(noff);
        for (int32_t t = 0; t < noff; ++t) {
            const int64_t dx = offsets[3 * t], dy = offsets[3 * t + 1], dz = offsets[3 * t + 2];
            lin[t] = dx + nx * (dy + ny * dz);
            CHF_CHECK(lin[t] < 0, CHF_EINVAL, "template offsets must point to smaller block indices");
        }
        const int64_t nb = nx * ny * nz;
        std::unique_ptr<chf_pattern_s> P(new chf_pattern_s);
        P->nb = nb;
        P->rowptr.assign(nb + 1, 0);
        std::vector<int32_t> row;
        for (int64_t k = 0; k < nb; ++k) {
            const int64_t kx = k % nx, ky = (k / nx) % ny, kz = k / (nx * ny);
            row.clear();
            for (int32_t t = 0; t < noff; ++t) {
                const int64_t cx = kx + offsets[3 * t], cy = ky + offsets[3 * t + 1], cz = kz + offsets[3 * t + 2];
                if (cx < 0 || cx >= nx || cy < 0 || cy >= ny || cz < 0 || cz >= nz) continue;
                row.push_back((int32_t)(k + lin[t]));
            }
            std::sort(row.begin(), row.end());
            row.erase(std::unique(row.begin(), row.end()), row.end());
            P->colidx.insert(P->colidx.end(), row.begin(), row.end());
            P->colidx.push_back((int32_t)k);
            P->rowptr[k + 1] = (int64_t)P->colidx.size();
        }
        *out = P.release();
    });
}

extern "C" int chf_pattern_info(chf_pattern P, int64_t* nb, int64_t* nnz) {
    return guarded([&] {
        CHF_CHECK(P, CHF_EINVAL, "NULL handle");
        if (nb) *nb = P->nb;
        if (nnz) *nnz = P->rowptr[P->nb];
    });
}

extern "C" int chf_pattern_export(chf_pattern P, int64_t* rowptr, int32_t* colidx) {
    return guarded([&] {
        CHF_CHECK(P, CHF_EINVAL, "NULL handle");
        if (rowptr) std::memcpy(rowptr, P->rowptr.data(), (P->nb + 1) * 8);
        if (colidx) std::memcpy(colidx, P->colidx.data(), P->colidx.size() * 4);
    });
}

extern "C" int chf_pattern_destroy(chf_pattern P) {
    return guarded([&] { delete P; });
}

extern "C" int chf_fsai_setup(chf_bsr A, chf_pattern P, chf_dtype g_store, chf_fsai* out, int64_t* bad_row) {
    return guarded([&] {
        CHF_CHECK(A && P && out, CHF_EINVAL, "NULL argument");
        CHF_CHECK(g_store == CHF_F64 || g_store == CHF_F32 || g_store == CHF_BF16, CHF_EINVAL, "bad dtype");
        *out = nullptr;
        if (bad_row) *bad_row = -1;
        if (A->vb) {
            CHF_CHECK(g_store == CHF_F64, CHF_EINVAL, "variable block sizes: FP64 only");
            *out = vfsai_setup_impl(A, *P, bad_row, 0);
            return;
        }
        *out = fsai_setup_impl(A, *P, g_store, bad_row, 0);
    });
}

extern "C" int chf_fsai_destroy(chf_fsai G) {
    return guarded([&] { delete G; });
}

extern "C" int chf_fsai_export(chf_fsai G, double* vals) {
    return guarded([&] {
        CHF_CHECK(G && vals, CHF_EINVAL, "NULL argument");
        CHF_CHECK(!G->nest_outer, CHF_EINVAL, "nested factor: export its outer and inner factors");
        G->d_vals.download(vals, G->vb ? (size_t)G->voff[G->nnz] : (size_t)G->nnz * G->b * G->b, 0);
        CHF_HIP(hipStreamSynchronize(0));
    });
}

extern "C" int chf_fsai_apply(chf_fsai G, chf_dtype dtype, const void* r, void* z, void* work,
                              hipStream_t stream) {
    return guarded([&] {
        CHF_CHECK(G && r && z && work, CHF_EINVAL, "NULL argument");
        CHF_CHECK(dtype == CHF_F64 || G->store == dtype || (dtype == CHF_F32 && G->store == CHF_BF16) ||
                      (dtype == CHF_F64_BF16G && G->store == CHF_BF16),
                  CHF_EINVAL, "dtype does not match the factor's storage");
        chf_dtype vec = mode_vec(dtype);
        chf_dtype use = dtype == CHF_F64 ? CHF_F64 : G->store;
        const FactorOps fo = factor_ops(*G, use);
        sell_spmv(*fo.g, vec, r, work, nullptr, EPI_AX, nullptr, nullptr, 0, 0, stream);
        if (fo.gi) {   // z is the spare: work = G1^T G1 work
            sell_spmv(*fo.gi, vec, work, z, nullptr, EPI_AX, nullptr, nullptr, 0, 0, stream);
            sell_spmv(*fo.git, vec, z, work, nullptr, EPI_AX, nullptr, nullptr, 0, 0, stream);
        }
        sell_spmv(*fo.gt, vec, work, z, nullptr, EPI_AX, nullptr, nullptr, 0, 0, stream);
    });
}

extern "C" int chf_lmax_lanczos(chf_bsr A, chf_fsai G, chf_dtype dtype, int iters, const double* v0,
                                double safety, double* beta, double* theta, hipStream_t stream) {
    return guarded([&] {
        CHF_CHECK(A && G && v0, CHF_EINVAL, "NULL argument");
        CHF_CHECK(A->nb == G->nb && A->b == G->b, CHF_EINVAL, "A and G sizes differ");
        CHF_CHECK(dtype == CHF_F64 || dtype == G->store || (dtype == CHF_F64_BF16G && G->store == CHF_BF16),
                  CHF_EINVAL, "dtype does not match the factor's storage");
        CHF_CHECK(A->vb == G->base().vb, CHF_EINVAL, "A and G block structures differ");
        lanczos_impl(A, *G, dtype, iters, v0, safety, beta, theta, stream);
    });
}
