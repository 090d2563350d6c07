// Galerkin hierarchy, transfers, exact coarsest-level solve, the V(k,k)
// cycle and the outer FP64 preconditioned CG (Sec. 5, opening paragraphs;
// Sec. 6 on CG with symmetric cycles).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>

#include <functional>
#include <memory>
#include <thread>

#include "internal.h"
#include "kernels_common.h"

namespace chf {

void cheb4_impl(const Sell& A, const FactorOps& G, chf_dtype vec, double beta, int degree, const void* b, void* x,
                bool x_is_zero, void* work, hipStream_t s);
void cheb1_impl(const Sell& A, const FactorOps& G, chf_dtype vec, double alpha, double beta, int degree,
                const void* b, void* x, bool x_is_zero, void* work, hipStream_t s);
void richardson_impl(const Sell& A, const FactorOps& G, chf_dtype vec, double omega, int degree, const void* b,
                     void* x, bool x_is_zero, void* work, hipStream_t s);
chf_fsai_s* fsai_setup_impl(chf_bsr A, const chf_pattern_s& P, chf_dtype g_store, int64_t* bad_row,
                            hipStream_t s);
chf_bsr_s* bsr_triple_impl(chf_bsr A, const chf_fsai_s& G, hipStream_t s);
void lanczos_impl(chf_bsr A, const chf_fsai_s& G, chf_dtype dt, int iters, const double* v0, double safety,
                  double* beta_out, double* theta_out, hipStream_t s);
chf_pattern_s* adaptive_pattern_impl(chf_bsr A, const chf_pattern_s* P0, int tmax, double tau, hipStream_t s);
void validate_pattern(int64_t nb, const int64_t* rowptr, const int32_t* colidx);

// ------------------------------------------------- host structure products --
// Runs f(c) for c = 0 .. ntask-1, one host thread per task.
// The first exception a task throws is rethrown here after all have joined.
static void run_tasks(int ntask, const std::function<void(int)>& f) {
    if (ntask <= 1) {
        if (ntask == 1) f(0);
        return;
    }
    std::vector<std::exception_ptr> err(ntask);
    std::vector<std::thread> th;
    for (int c = 0; c < ntask; ++c)
        th.emplace_back([&, c] {
            try {
                f(c);
            } catch (...) {
                err[c] = std::current_exception();
            }
        });
    for (auto& x : th) x.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
}

// Structure of the product X Y of two CSR patterns (X: nr rows, Y: columns
// < ncol): row r = the sorted union of the rows Y(k), k in X(r).
static void struct_product(int64_t nr, const int64_t* xr, const int32_t* xc, const int64_t* yr, const int32_t* yc,
                           int64_t ncol, std::vector<int64_t>& orow, std::vector<int32_t>& ocol) {
    const int64_t hw = std::max<unsigned>(1u, std::thread::hardware_concurrency());
    const int nchunk = (int)std::min<int64_t>(std::min<int64_t>(hw, 16), std::max<int64_t>(1, nr / 2048));
    std::vector<std::vector<int32_t>> cols(nchunk);
    std::vector<int64_t> len(nr + 1, 0);
    run_tasks(nchunk, [&](int c) {
        std::vector<int32_t> mark((size_t)ncol, -1), tmp;
        const int64_t lo = nr * c / nchunk, hi = nr * (c + 1) / nchunk;
        for (int64_t r = lo; r < hi; ++r) {
            tmp.clear();
            for (int64_t e = xr[r]; e < xr[r + 1]; ++e) {
                const int64_t k = xc[e];
                for (int64_t f = yr[k]; f < yr[k + 1]; ++f) {
                    const int32_t j = yc[f];
                    if (mark[j] != (int32_t)r) { mark[j] = (int32_t)r; tmp.push_back(j); }
                }
            }
            std::sort(tmp.begin(), tmp.end());
            cols[c].insert(cols[c].end(), tmp.begin(), tmp.end());
            len[r + 1] = (int64_t)tmp.size();
        }
    });
    orow.assign(nr + 1, 0);
    for (int64_t r = 0; r < nr; ++r) orow[r + 1] = orow[r] + len[r + 1];
    ocol.resize((size_t)orow[nr]);
    run_tasks(nchunk, [&](int c) { std::copy(cols[c].begin(), cols[c].end(), ocol.begin() + orow[nr * c / nchunk]); });
}

// ------------------------------------------------------------- Galerkin --
// A_c[I, J] = sum_{i in P^T(I)} sum_{j in A(i)} sum_{J in P(j)} P_iI A_ij P_jJ.
// One workgroup per coarse block row; thread e owns entry e of every block of
// that row, so accumulation order is fixed and no two threads share an output.
__global__ void k_galerkin(int64_t nc, int b, const int64_t* __restrict__ pt_rowptr,
                           const int* __restrict__ pt_col, const double* __restrict__ pt_val,
                           const int64_t* __restrict__ p_rowptr, const int* __restrict__ p_col,
                           const double* __restrict__ p_val, const int* __restrict__ a_rowptr,
                           const int* __restrict__ a_col, const double* __restrict__ a_vals,
                           const int64_t* __restrict__ c_rowptr, const int* __restrict__ c_col,
                           double* __restrict__ c_vals) {
    const int64_t I = blockIdx.x;
    if (I >= nc) return;
    const int bb = b * b;
    const int64_t c0 = c_rowptr[I], c1 = c_rowptr[I + 1];
    for (int e = threadIdx.x; e < bb; e += blockDim.x)
        for (int64_t q = c0; q < c1; ++q) c_vals[q * bb + e] = 0.0;
    for (int64_t ti = pt_rowptr[I]; ti < pt_rowptr[I + 1]; ++ti) {
        const int i = pt_col[ti];
        const double wi = pt_val[ti];
        for (int ea = a_rowptr[i]; ea < a_rowptr[i + 1]; ++ea) {
            const int j = a_col[ea];
            for (int64_t tj = p_rowptr[j]; tj < p_rowptr[j + 1]; ++tj) {
                const int J = p_col[tj];
                const double w = wi * p_val[tj];
                int64_t lo = c0, hi = c1;
                while (lo < hi) {
                    int64_t mid = (lo + hi) >> 1;
                    if (c_col[mid] < J) lo = mid + 1; else hi = mid;
                }
                const double* src = a_vals + (int64_t)ea * bb;
                double* dst = c_vals + lo * bb;
                for (int e = threadIdx.x; e < bb; e += blockDim.x) dst[e] += w * src[e];
            }
        }
    }
}

// Congruence with a block-diagonal basis change: out_e = T_i^T A_e T_j for
// every stored block e = (i, j). One workgroup per block row.
__global__ void k_congruence(int64_t nb, int b, const int* __restrict__ rowptr, const int* __restrict__ col,
                             const double* __restrict__ vals, const double* __restrict__ T,
                             double* __restrict__ out) {
    extern __shared__ double sm[];
    const int64_t i = blockIdx.x;
    if (i >= nb) return;
    const int bb = b * b;
    double* tmp = sm;
    const double* Ti = T + i * bb;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const double* Ae = vals + (int64_t)e * bb;
        const double* Tj = T + (int64_t)col[e] * bb;
        for (int t = threadIdx.x; t < bb; t += blockDim.x) {
            int r = t / b, c = t - r * b;
            double acc = 0.0;
            for (int q = 0; q < b; ++q) acc += Ae[r * b + q] * Tj[q * b + c];
            tmp[t] = acc;                                  // (A_e T_j)[r][c]
        }
        __syncthreads();
        for (int t = threadIdx.x; t < bb; t += blockDim.x) {
            int r = t / b, c = t - r * b;
            double acc = 0.0;
            for (int p = 0; p < b; ++p) acc += Ti[p * b + r] * tmp[p * b + c];
            out[(int64_t)e * bb + t] = acc;                // (T_i^T A_e T_j)[r][c]
        }
        __syncthreads();
    }
}

// y_i = T_i^T r_i for every block row
template <typename TV>
__global__ void k_basis_t(int64_t nb, int b, const TV* __restrict__ T, const TV* __restrict__ r,
                          TV* __restrict__ y) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nb * b) return;
    const int64_t i = t / b;
    const int c = (int)(t - i * b);
    const TV* Ti = T + i * b * b;
    const TV* ri = r + i * b;
    TV acc = 0;
    for (int q = 0; q < b; ++q) acc += Ti[q * b + c] * ri[q];
    y[t] = acc;
}

// x_i += T_i z_i with z_i = sum_{(I, w) in P(i)} w x_c[I]. A wavefront holds
// S = 64 / b block rows, lane = local_row * b + r: the lane forms component r
// of z_i once, and the row's b lanes exchange their components by shuffles.
// BT > 0 fixes b at compile time, so the lane's row of T_i is loaded at once.
template <int BT, typename TV>
__global__ void k_prolong_add_basis(int64_t nf, int brt, const int64_t* __restrict__ p_rowptr,
                                    const int* __restrict__ p_col, const double* __restrict__ p_val,
                                    const TV* __restrict__ T, const TV* __restrict__ xc, TV* __restrict__ x) {
    const int b = BT ? BT : brt;
    const int S = 64 / b;
    const int lane = threadIdx.x & 63;
    const int64_t wv = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int lr = lane / b, r = lane - lr * b;
    const int64_t i = wv * S + lr;
    const bool active = lr < S && i < nf;
    TV z = 0;
    if (active)
        for (int64_t e = p_rowptr[i]; e < p_rowptr[i + 1]; ++e) z += (TV)p_val[e] * xc[(int64_t)p_col[e] * b + r];
    const TV* Ti = T + (active ? i : 0) * b * b + r * b;
    TV acc = 0;
    if constexpr (BT > 0) {
        TV t[BT];
#pragma unroll
        for (int c = 0; c < BT; ++c) t[c] = active ? Ti[c] : (TV)0;
#pragma unroll
        for (int c = 0; c < BT; ++c) acc += t[c] * __shfl(z, lr * BT + c, 64);   // lanes past S * b: unused
    } else {
        for (int c = 0; c < b; ++c) {
            const TV zc = __shfl(z, lr * b + c, 64);   // lanes past S * b read a wrapped lane, unused
            if (active) acc += Ti[c] * zc;
        }
    }
    if (active) x[i * b + r] += acc;
}

// ------------------------------------------------------------- transfers --
// restriction b_c[I] = sum_{(i, w) in P^T(I)} w r[i], per scalar component
template <typename TV>
__global__ void k_restrict(int64_t nc, int b, const int64_t* __restrict__ pt_rowptr, const int* __restrict__ pt_col,
                           const double* __restrict__ pt_val, const TV* __restrict__ r, TV* __restrict__ bc) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nc * b) return;
    const int64_t I = t / b;
    const int c = (int)(t - I * b);
    TV acc = 0;
    for (int64_t e = pt_rowptr[I]; e < pt_rowptr[I + 1]; ++e) acc += (TV)pt_val[e] * r[(int64_t)pt_col[e] * b + c];
    bc[t] = acc;
}

// prolongation x[i] += sum_{(I, w) in P(i)} w x_c[I]
template <typename TV>
__global__ void k_prolong_add(int64_t nf, int b, const int64_t* __restrict__ p_rowptr, const int* __restrict__ p_col,
                              const double* __restrict__ p_val, const TV* __restrict__ xc, TV* __restrict__ x) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nf * b) return;
    const int64_t i = t / b;
    const int c = (int)(t - i * b);
    TV acc = 0;
    for (int64_t e = p_rowptr[i]; e < p_rowptr[i + 1]; ++e) acc += (TV)p_val[e] * xc[(int64_t)p_col[e] * b + c];
    x[t] += acc;
}

// ---------------------------------------------------- dense coarse solve --
// The coarsest operator is inverted once by a blocked Gauss-Jordan sweep on
// 32 x 32 tiles: for each pivot tile k, P = A_kk^{-1}; A_kj <- P A_kj;
// A_ij <- A_ij - A_ik A_kj; A_ik <- -A_ik P; A_kk <- P. The pivot tile is
// inverted by the scalar sweep whose pivots are the Cholesky pivots of the
// SPD matrix (Schur complements), so a non-positive pivot reports a matrix
// that is not positive definite. Each V-cycle then applies the inverse with
// one dense matrix-vector product.
constexpr int GJ = 32;

__global__ void k_scatter_dense(int64_t nb, int b, int64_t ld, const int* __restrict__ rowptr,
                                const int* __restrict__ col, const double* __restrict__ vals,
                                double* __restrict__ d) {
    const int64_t i = blockIdx.x;
    const int bb = b * b;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const int64_t j = col[e];
        for (int t = threadIdx.x; t < bb; t += blockDim.x) {
            int r = t / b, c = t - r * b;
            d[(i * b + r) * ld + j * b + c] = vals[(int64_t)e * bb + t];
        }
    }
}

__global__ void k_set_identity_tail(int64_t n, int64_t ld, double* __restrict__ d) {
    const int64_t i = n + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < ld) d[i * ld + i] = 1.0;
}

__global__ __launch_bounds__(256) void k_gj_pivot(int64_t ld, int64_t k0, double* __restrict__ d, int* bad) {
    __shared__ double t[GJ][GJ + 1];
    __shared__ double piv;
    __shared__ int ok;
    const int tid = threadIdx.x;
    for (int e = tid; e < GJ * GJ; e += 256) t[e / GJ][e % GJ] = d[(k0 + e / GJ) * ld + k0 + e % GJ];
    if (tid == 0) ok = 1;
    __syncthreads();
    for (int k = 0; k < GJ; ++k) {
        if (tid == 0) {
            double p = t[k][k];
            if (!(p > 0.0) || !isfinite(p)) ok = 0;
            piv = 1.0 / p;
        }
        __syncthreads();
        if (!ok) break;
        const double ip = piv;
        // a_ij -= a_ik a_kj / p for i, j != k (uses old row k and column k)
        double upd[4];
        int cnt = 0;
        for (int e = tid; e < GJ * GJ; e += 256, ++cnt) {
            int i = e / GJ, j = e % GJ;
            upd[cnt] = (i != k && j != k) ? t[i][j] - t[i][k] * t[k][j] * ip : t[i][j];
        }
        __syncthreads();
        cnt = 0;
        for (int e = tid; e < GJ * GJ; e += 256, ++cnt) {
            int i = e / GJ, j = e % GJ;
            if (i != k && j != k) t[i][j] = upd[cnt];
        }
        __syncthreads();
        if (tid < GJ && tid != k) {
            t[k][tid] *= ip;      // row k
            t[tid][k] *= -ip;     // column k
        }
        if (tid == 0) t[k][k] = ip;
        __syncthreads();
    }
    if (!ok) {
        if (tid == 0) bad[0] = 1;
        return;
    }
    for (int e = tid; e < GJ * GJ; e += 256) d[(k0 + e / GJ) * ld + k0 + e % GJ] = t[e / GJ][e % GJ];
}

// C = op: mode 0: A_kj <- P A_kj (tile j = blockIdx.x, skipping k)
//         mode 1: A_ik <- -A_ik P (tile i = blockIdx.x, skipping k)
__global__ __launch_bounds__(256) void k_gj_panel(int64_t ld, int64_t nt, int64_t kt, int mode,
                                                  double* __restrict__ d) {
    __shared__ double P[GJ][GJ + 1];
    __shared__ double X[GJ][GJ + 1];
    int64_t o = blockIdx.x;
    if (o >= kt) ++o;
    if (o >= nt) return;
    const int tid = threadIdx.x;
    const int64_t k0 = kt * GJ, o0 = o * GJ;
    for (int e = tid; e < GJ * GJ; e += 256) {
        int r = e / GJ, c = e % GJ;
        P[r][c] = d[(k0 + r) * ld + k0 + c];
        X[r][c] = mode == 0 ? d[(k0 + r) * ld + o0 + c] : d[(o0 + r) * ld + k0 + c];
    }
    __syncthreads();
    for (int e = tid; e < GJ * GJ; e += 256) {
        int r = e / GJ, c = e % GJ;
        double acc = 0.0;
        if (mode == 0) {
            for (int q = 0; q < GJ; ++q) acc += P[r][q] * X[q][c];
            d[(k0 + r) * ld + o0 + c] = acc;
        } else {
            for (int q = 0; q < GJ; ++q) acc += X[r][q] * P[q][c];
            d[(o0 + r) * ld + k0 + c] = -acc;
        }
    }
}

// A_ij -= A_ik A_kj for all tiles i, j != k; one workgroup per output tile,
// each thread 2 x 2 outputs.
__global__ __launch_bounds__(256) void k_gj_update(int64_t ld, int64_t nt, int64_t kt, double* __restrict__ d) {
    __shared__ double Ck[GJ][GJ + 1];   // A_ik
    __shared__ double Rk[GJ][GJ + 1];   // A_kj
    int64_t ti = blockIdx.y, tj = blockIdx.x;
    if (ti >= kt) ++ti;
    if (tj >= kt) ++tj;
    if (ti >= nt || tj >= nt) return;
    const int tid = threadIdx.x;
    const int64_t i0 = ti * GJ, j0 = tj * GJ, k0 = kt * GJ;
    for (int e = tid; e < GJ * GJ; e += 256) {
        int r = e / GJ, c = e % GJ;
        Ck[r][c] = d[(i0 + r) * ld + k0 + c];
        Rk[r][c] = d[(k0 + r) * ld + j0 + c];
    }
    __syncthreads();
    const int r0 = (tid / 16) * 2, c0 = (tid % 16) * 2;
    double a00 = 0, a01 = 0, a10 = 0, a11 = 0;
    for (int q = 0; q < GJ; ++q) {
        double x0 = Ck[r0][q], x1 = Ck[r0 + 1][q];
        double y0 = Rk[q][c0], y1 = Rk[q][c0 + 1];
        a00 += x0 * y0;
        a01 += x0 * y1;
        a10 += x1 * y0;
        a11 += x1 * y1;
    }
    d[(i0 + r0) * ld + j0 + c0] -= a00;
    d[(i0 + r0) * ld + j0 + c0 + 1] -= a01;
    d[(i0 + r0 + 1) * ld + j0 + c0] -= a10;
    d[(i0 + r0 + 1) * ld + j0 + c0 + 1] -= a11;
}

// y = Ainv x (dense, FP64 arithmetic); one wavefront per row.
template <typename TV>
__global__ __launch_bounds__(256) void k_dense_gemv(int64_t n, int64_t ld, const double* __restrict__ d,
                                                    const TV* __restrict__ x, TV* __restrict__ y) {
    const int64_t row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const double* a = d + row * ld;
    double acc = 0.0;
    for (int64_t j = lane; j < n; j += 64) acc += a[j] * (double)x[j];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) y[row] = (TV)acc;
}

// --------------------------------------------------------------- PCG ops --
// scal layout (device doubles): 0 rz, 1 pq, 2 rr, 3 rz_new, 4 num
__global__ void k_pcg_xr(int64_t n, const double* __restrict__ scal, const double* __restrict__ p,
                         const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r,
                         double* __restrict__ rold) {
    // breakdown (p^T A p <= 0 or r^T z <= 0, NaN included): leave x and r at
    // the last good iterate; the host reads the same scalars and stops
    if (!(scal[1] > 0.0) || !(scal[0] > 0.0)) return;
    const double alpha = scal[0] / scal[1];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * p[i];
        const double ri = r[i];
        if (rold) rold[i] = ri;
        r[i] = ri - alpha * q[i];
    }
}

__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ c) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c[i] = a[i] - b[i];
}

// p = z + (num / rz) p ; rz <- rz_new
__global__ void k_pcg_p(int64_t n, double* __restrict__ scal, const double* __restrict__ z, double* __restrict__ p) {
    const double beta = scal[4] / scal[0];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + beta * p[i];
}

__global__ void k_copy_scalar(double* __restrict__ scal, int from, int to) {
    if (threadIdx.x == 0 && blockIdx.x == 0) scal[to] = scal[from];
}

// ---------------------------------------------------------- BiCGStab ops --
// bs layout (device doubles): 0 rho, 1 rho_old, 2 alpha, 3 omega, 4 (r^, v),
// 5 (t, s), 6 (t, t), 7 squared norm of the residual checked last
__global__ void k_bicg_p(int64_t n, const double* __restrict__ bs, const double* __restrict__ r,
                         const double* __restrict__ v, double* __restrict__ p, int first) {
    const double beta = first ? 0.0 : (bs[0] / bs[1]) * (bs[2] / bs[3]);
    const double om = first ? 0.0 : bs[3];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = first ? r[i] : r[i] + beta * (p[i] - om * v[i]);
}

// alpha = rho / (r^, v); s = r - alpha v
__global__ void k_bicg_s(int64_t n, double* __restrict__ bs, const double* __restrict__ r,
                         const double* __restrict__ v, double* __restrict__ s) {
    const double alpha = bs[0] / bs[4];
    if (blockIdx.x == 0 && threadIdx.x == 0) bs[2] = alpha;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s[i] = r[i] - alpha * v[i];
}

// omega = (t, s) / (t, t); x += alpha p^ + omega s^; r = s - omega t
__global__ void k_bicg_xr(int64_t n, double* __restrict__ bs, const double* __restrict__ ph,
                          const double* __restrict__ sh, const double* __restrict__ s, const double* __restrict__ t,
                          double* __restrict__ x, double* __restrict__ r) {
    const double alpha = bs[0] / bs[4];
    const double omega = bs[5] / bs[6];
    if (blockIdx.x == 0 && threadIdx.x == 0) bs[3] = omega;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * ph[i] + omega * sh[i];
        r[i] = s[i] - omega * t[i];
    }
}

// x += alpha p^ (convergence at the half step)
__global__ void k_bicg_half(int64_t n, const double* __restrict__ bs, const double* __restrict__ ph,
                            double* __restrict__ x) {
    const double alpha = bs[0] / bs[4];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += alpha * ph[i];
}

}  // namespace chf

using namespace chf;

struct chf_level_s {
    chf_bsr A = nullptr;
    bool own_A = false;
    chf_pattern P = nullptr;
    bool preset = false;                // P given by the caller

    chf_fsai G = nullptr;               // the smoother's factor (nested handle when nesting)
    chf_fsai G0 = nullptr, G1 = nullptr; // outer and inner factors of a nested G
    chf_pattern P1 = nullptr;           // inner pattern
    double beta = 0.0;
    // prolongation from the next coarser level (host + device CSR)
    int64_t nc = 0;
    std::vector<int64_t> p_rowptr, pt_rowptr;
    std::vector<int32_t> p_col, pt_col;
    std::vector<double> p_val, pt_val;
    bool has_T = false;                 // P = T (P_s (x) I_b) with T block diagonal
    DevBuf<double> d_T64;
    DevBuf<float> d_T32;
    DevBuf<int64_t> d_p_rowptr, d_pt_rowptr;
    DevBuf<int> d_p_col, d_pt_col;
    DevBuf<double> d_p_val, d_pt_val;
    // working vectors in the hierarchy's vector dtype
    DevBuf<char> bvec, xvec, rvec, work;
    // coarsest level: dense inverse
    DevBuf<double> dense;
    int64_t ld = 0;
};

struct chf_levels_s {
    std::vector<chf_level_s> lev;
    chf_level_opts opts{};
    bool ready = false;
    chf_dtype vec = CHF_F64;
    DevBuf<double> bicg_buf, bicg_scal;
    int64_t bicg_n = 0;
    int smoother = CHF_SMOOTH_CHEB4;   // smoother of every level but the coarsest
    double sm_param = 0.0;             // rho (first kind: alpha_l = rho beta_l) or omega (Richardson)
    int cycle = CHF_CYCLE_VKK;
    int nest = 0;                      // 1: nested block-FSAI with one level (Sec. 2.2)
    DevBuf<double> pcg_buf, scal, part;
    int64_t pcg_n = 0;
    ~chf_levels_s() {
        for (auto& l : lev) {
            if (l.G) delete l.G;
            if (l.G0) delete l.G0;
            if (l.G1) delete l.G1;
            if (l.P1) delete l.P1;
            if (l.P) delete l.P;
            if (l.own_A && l.A) delete l.A;
        }
    }
};

namespace chf {

static const Sell& level_A(chf_levels_s& H, int l, hipStream_t s) {
    return H.lev[l].A->sell(H.vec, s);
}

static void coarse_apply(chf_levels_s& H, int l, const void* b, void* x, hipStream_t s) {
    chf_level_s& L = H.lev[l];
    int64_t n = L.A->nb * (int64_t)L.A->b;
    dim3 grid((unsigned)((n + 3) / 4));
    if (H.vec == CHF_F64)
        hipLaunchKernelGGL((k_dense_gemv<double>), grid, dim3(256), 0, s, n, L.ld, L.dense.p, (const double*)b,
                           (double*)x);
    else
        hipLaunchKernelGGL((k_dense_gemv<float>), grid, dim3(256), 0, s, n, L.ld, L.dense.p, (const float*)b,
                           (float*)x);
    CHF_LAUNCH_CHECK();
}

static void restrict_to(chf_levels_s& H, int l, const void* r, void* bc, hipStream_t s) {
    chf_level_s& L = H.lev[l];
    int b = L.A->b;
    if (L.has_T) {
        int64_t nf = L.A->nb * (int64_t)b;
        dim3 g((unsigned)((nf + 255) / 256));
        if (H.vec == CHF_F64)
            hipLaunchKernelGGL((k_basis_t<double>), g, dim3(256), 0, s, L.A->nb, b, (const double*)L.d_T64.p,
                               (const double*)r, (double*)L.work.p);
        else
            hipLaunchKernelGGL((k_basis_t<float>), g, dim3(256), 0, s, L.A->nb, b, (const float*)L.d_T32.p,
                               (const float*)r, (float*)L.work.p);
        CHF_LAUNCH_CHECK();
        r = L.work.p;
    }
    int64_t tot = L.nc * b;
    dim3 grid((unsigned)((tot + 255) / 256));
    if (H.vec == CHF_F64)
        hipLaunchKernelGGL((k_restrict<double>), grid, dim3(256), 0, s, L.nc, b, L.d_pt_rowptr.p, L.d_pt_col.p,
                           L.d_pt_val.p, (const double*)r, (double*)bc);
    else
        hipLaunchKernelGGL((k_restrict<float>), grid, dim3(256), 0, s, L.nc, b, L.d_pt_rowptr.p, L.d_pt_col.p,
                           L.d_pt_val.p, (const float*)r, (float*)bc);
    CHF_LAUNCH_CHECK();
}

static void prolong_add(chf_levels_s& H, int l, const void* xc, void* x, hipStream_t s) {
    chf_level_s& L = H.lev[l];
    int b = L.A->b;
    int64_t nf = L.A->nb;
    int64_t tot = nf * b;
    dim3 grid((unsigned)((tot + 255) / 256));
    if (L.has_T) {
        const int64_t waves = (nf + 64 / b - 1) / (64 / b);
        dim3 gw((unsigned)((waves + 3) / 4));   // four wavefronts per 256-wide workgroup
        if (H.vec == CHF_F64) {
            if (b == 10)
                hipLaunchKernelGGL((k_prolong_add_basis<10, double>), gw, dim3(256), 0, s, nf, b, L.d_p_rowptr.p,
                                   L.d_p_col.p, L.d_p_val.p, (const double*)L.d_T64.p, (const double*)xc, (double*)x);
            else
                hipLaunchKernelGGL((k_prolong_add_basis<0, double>), gw, dim3(256), 0, s, nf, b, L.d_p_rowptr.p,
                                   L.d_p_col.p, L.d_p_val.p, (const double*)L.d_T64.p, (const double*)xc, (double*)x);
        } else {
            if (b == 10)
                hipLaunchKernelGGL((k_prolong_add_basis<10, float>), gw, dim3(256), 0, s, nf, b, L.d_p_rowptr.p,
                                   L.d_p_col.p, L.d_p_val.p, (const float*)L.d_T32.p, (const float*)xc, (float*)x);
            else
                hipLaunchKernelGGL((k_prolong_add_basis<0, float>), gw, dim3(256), 0, s, nf, b, L.d_p_rowptr.p,
                                   L.d_p_col.p, L.d_p_val.p, (const float*)L.d_T32.p, (const float*)xc, (float*)x);
        }
        CHF_LAUNCH_CHECK();
        return;
    }
    if (H.vec == CHF_F64)
        hipLaunchKernelGGL((k_prolong_add<double>), grid, dim3(256), 0, s, nf, b, L.d_p_rowptr.p, L.d_p_col.p,
                           L.d_p_val.p, (const double*)xc, (double*)x);
    else
        hipLaunchKernelGGL((k_prolong_add<float>), grid, dim3(256), 0, s, nf, b, L.d_p_rowptr.p, L.d_p_col.p,
                           L.d_p_val.p, (const float*)xc, (float*)x);
    CHF_LAUNCH_CHECK();
}

// One smoother application of the given degree on level l.
static void smooth_level(chf_levels_s& H, int l, int degree, const void* b, void* x, bool x_is_zero, hipStream_t s) {
    chf_level_s& L = H.lev[l];
    const Sell& A = level_A(H, l, s);
    const chf_dtype gdt = H.vec == CHF_F64 ? mode_g(H.opts.dtype) : L.G->store;
    const FactorOps G = factor_ops(*L.G, gdt);
    switch (H.smoother) {
        case CHF_SMOOTH_CHEB1:
            cheb1_impl(A, G, H.vec, H.sm_param * L.beta, L.beta, degree, b, x, x_is_zero, L.work.p, s);
            break;
        case CHF_SMOOTH_RICHARDSON:
            richardson_impl(A, G, H.vec, H.sm_param, degree, b, x, x_is_zero, L.work.p, s);
            break;
        default:
            cheb4_impl(A, G, H.vec, L.beta, degree, b, x, x_is_zero, L.work.p, s);
    }
}

// V(k,k) on level l: pre-smooth, residual, restrict, recurse, prolongate,
// post-smooth. V(2k,0): one pre-smoothing application of degree 2k and no
// post-smoothing (the non-symmetric cycle of Sec. 5).
static void vcycle_rec(chf_levels_s& H, int l, const void* b, void* x, bool x_is_zero, hipStream_t s) {
    const int nl = (int)H.lev.size();
    chf_level_s& L = H.lev[l];
    if (l == nl - 1) {
        coarse_apply(H, l, b, x, s);
        return;
    }
    const Sell& A = level_A(H, l, s);
    const int k = H.opts.degree;
    const bool v2k0 = H.cycle == CHF_CYCLE_V2K0;
    smooth_level(H, l, v2k0 ? 2 * k : k, b, x, x_is_zero, s);
    sell_spmv(A, H.vec, x, L.rvec.p, b, EPI_RES, nullptr, nullptr, 0, 0, s);
    chf_level_s& C = H.lev[l + 1];
    restrict_to(H, l, L.rvec.p, C.bvec.p, s);
    vcycle_rec(H, l + 1, C.bvec.p, C.xvec.p, true, s);
    prolong_add(H, l, C.xvec.p, x, s);
    if (!v2k0) smooth_level(H, l, k, b, x, false, s);
}

static void build_coarse_dense(chf_level_s& L, hipStream_t s) {
    chf_bsr A = L.A;
    const int64_t n = A->nb * (int64_t)A->b;
    const int64_t ld = (n + GJ - 1) / GJ * GJ;
    const int64_t nt = ld / GJ;
    L.ld = ld;
    L.dense.alloc((size_t)ld * ld);
    fill_zero(L.dense.p, (size_t)ld * ld * 8, s);
    if (A->nb > 0) {
        hipLaunchKernelGGL(k_scatter_dense, dim3((unsigned)A->nb), dim3(128), 0, s, A->nb, A->b, ld, A->d_rowptr.p,
                           A->d_colidx.p, A->d_vals.p, L.dense.p);
        CHF_LAUNCH_CHECK();
    }
    if (ld > n) {
        hipLaunchKernelGGL(k_set_identity_tail, dim3(1), dim3(64), 0, s, n, ld, L.dense.p);
        CHF_LAUNCH_CHECK();
    }
    DevBuf<int> bad(1);
    fill_zero(bad.p, 4, s);
    for (int64_t kt = 0; kt < nt; ++kt) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, s, ld, kt * GJ, L.dense.p, bad.p);
        CHF_LAUNCH_CHECK();
        if (nt > 1) {
            hipLaunchKernelGGL(k_gj_panel, dim3((unsigned)(nt - 1)), dim3(256), 0, s, ld, nt, kt, 0, L.dense.p);
            CHF_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_gj_update, dim3((unsigned)(nt - 1), (unsigned)(nt - 1)), dim3(256), 0, s, ld, nt,
                               kt, L.dense.p);
            CHF_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_gj_panel, dim3((unsigned)(nt - 1)), dim3(256), 0, s, ld, nt, kt, 1, L.dense.p);
            CHF_LAUNCH_CHECK();
        }
    }
    int hbad = 0;
    bad.download(&hbad, 1, s);
    CHF_HIP(hipStreamSynchronize(s));
    CHF_CHECK(hbad == 0, CHF_ENOTSPD, "coarsest-level operator is not positive definite");
}

static void alloc_vectors(chf_levels_s& H) {
    const size_t es = vec_size(H.vec);
    for (auto& L : H.lev) {
        int64_t n = L.A->nb * (int64_t)L.A->b;
        L.bvec.alloc(std::max<int64_t>(1, n) * es);
        L.xvec.alloc(std::max<int64_t>(1, n) * es);
        L.rvec.alloc(std::max<int64_t>(1, n) * es);
        L.work.alloc(std::max<int64_t>(1, 3 * n) * es);
    }
}

}  // namespace chf

extern "C" int chf_levels_create(chf_bsr A0, chf_levels* out) {
    return guarded([&] {
        CHF_CHECK(A0 && out, CHF_EINVAL, "NULL argument");
        CHF_CHECK(!A0->vb, CHF_EINVAL, "the hierarchy supports uniform block sizes only");
        std::unique_ptr<chf_levels_s> H(new chf_levels_s);
        H->lev.emplace_back();
        H->lev[0].A = A0;
        *out = H.release();
    });
}

extern "C" int chf_levels_add_coarse(chf_levels H, int64_t nc, const int64_t* p_rowptr, const int32_t* p_colidx,
                                     const double* p_vals, const double* basis) {
    return guarded([&] {
        CHF_CHECK(H && p_rowptr && p_colidx && p_vals, CHF_EINVAL, "NULL argument");
        CHF_CHECK(!H->ready, CHF_EINVAL, "hierarchy already set up");
        chf_level_s& F = H->lev.back();
        chf_bsr A = F.A;
        const int64_t nf = A->nb;
        const int b = A->b;
        CHF_CHECK(nc > 0 && nc <= nf, CHF_EINVAL, "bad coarse size");
        CHF_CHECK(p_rowptr[0] == 0, CHF_EINVAL, "bad prolongation rowptr");
        const int64_t nnzp = p_rowptr[nf];
        for (int64_t i = 0; i < nf; ++i) {
            CHF_CHECK(p_rowptr[i + 1] >= p_rowptr[i], CHF_EINVAL, "bad prolongation rowptr");
            for (int64_t e = p_rowptr[i]; e < p_rowptr[i + 1]; ++e) {
                CHF_CHECK(p_colidx[e] >= 0 && p_colidx[e] < nc, CHF_EINVAL, "prolongation column out of range");
                CHF_CHECK(std::isfinite(p_vals[e]), CHF_EINVAL, "non-finite prolongation weight");
            }
        }
        F.nc = nc;
        F.p_rowptr.assign(p_rowptr, p_rowptr + nf + 1);
        F.p_col.assign(p_colidx, p_colidx + nnzp);
        F.p_val.assign(p_vals, p_vals + nnzp);
        // transpose (rows ascending -> stable)
        F.pt_rowptr.assign(nc + 1, 0);
        for (int64_t e = 0; e < nnzp; ++e) F.pt_rowptr[F.p_col[e] + 1]++;
        for (int64_t I = 0; I < nc; ++I) F.pt_rowptr[I + 1] += F.pt_rowptr[I];
        F.pt_col.assign(nnzp, 0);
        F.pt_val.assign(nnzp, 0.0);
        std::vector<int64_t> fillp(F.pt_rowptr.begin(), F.pt_rowptr.end() - 1);
        for (int64_t i = 0; i < nf; ++i)
            for (int64_t e = F.p_rowptr[i]; e < F.p_rowptr[i + 1]; ++e) {
                int64_t pos = fillp[F.p_col[e]]++;
                F.pt_col[pos] = (int32_t)i;
                F.pt_val[pos] = F.p_val[e];
            }
        // coarse structure struct(P^T A P) = struct(P^T T) with T = struct(A P)
        std::vector<int64_t> trow, crow;
        std::vector<int32_t> tcol, ccol;
        struct_product(nf, A->rowptr.data(), A->colidx.data(), F.p_rowptr.data(), F.p_col.data(), nc, trow, tcol);
        struct_product(nc, F.pt_rowptr.data(), F.pt_col.data(), trow.data(), tcol.data(), nc, crow, ccol);
        hipStream_t s = 0;
        auto up64 = [&](DevBuf<int64_t>& d, const std::vector<int64_t>& h) {
            d.alloc(std::max<size_t>(1, h.size())); d.upload(h.data(), h.size(), s); };
        auto up32 = [&](DevBuf<int>& d, const std::vector<int32_t>& h) {
            d.alloc(std::max<size_t>(1, h.size())); d.upload(h.data(), h.size(), s); };
        auto upd = [&](DevBuf<double>& d, const std::vector<double>& h) {
            d.alloc(std::max<size_t>(1, h.size())); d.upload(h.data(), h.size(), s); };
        up64(F.d_p_rowptr, F.p_rowptr);
        up32(F.d_p_col, F.p_col);
        upd(F.d_p_val, F.p_val);
        up64(F.d_pt_rowptr, F.pt_rowptr);
        up32(F.d_pt_col, F.pt_col);
        upd(F.d_pt_val, F.pt_val);
        DevBuf<int64_t> d_crow;
        DevBuf<int> d_ccol;
        up64(d_crow, crow);
        up32(d_ccol, ccol);
        const int64_t cnnz = crow[nc];
        DevBuf<double> cvals(std::max<int64_t>(1, cnnz * b * b));
        const double* avals = A->d_vals.p;
        DevBuf<double> tvals;
        if (basis) {
            const size_t nt = (size_t)nf * b * b;
            const int nchunk = (int)std::min<size_t>(16, std::max<size_t>(1, nt >> 20));
            std::vector<char> bad(nchunk, 0);
            run_tasks(nchunk, [&](int c) {
                for (size_t q = nt * c / nchunk, q1 = nt * (c + 1) / nchunk; q < q1; ++q)
                    if (!std::isfinite(basis[q])) { bad[c] = 1; break; }
            });
            for (char f : bad) CHF_CHECK(!f, CHF_EINVAL, "non-finite basis value");
            F.has_T = true;
            F.d_T64.alloc(nt);
            F.d_T64.upload(basis, nt, s);
            F.d_T32.alloc(nt);
            cast_vec(CHF_F64, F.d_T64.p, CHF_F32, F.d_T32.p, (int64_t)nt, s);
            tvals.alloc(std::max<int64_t>(1, A->nnzb * b * b));
            int ntc = std::min(256, ((b * b + 63) / 64) * 64);
            hipLaunchKernelGGL(k_congruence, dim3((unsigned)nf), dim3(ntc), (size_t)b * b * 8, s, nf, b, A->d_rowptr.p,
                               A->d_colidx.p, A->d_vals.p, F.d_T64.p, tvals.p);
            CHF_LAUNCH_CHECK();
            avals = tvals.p;
            CHF_HIP(hipStreamSynchronize(s));
        }
        int nt = std::min(256, ((b * b + 63) / 64) * 64);
        hipLaunchKernelGGL(k_galerkin, dim3((unsigned)nc), dim3(nt), 0, s, nc, b, F.d_pt_rowptr.p, F.d_pt_col.p,
                           F.d_pt_val.p, F.d_p_rowptr.p, F.d_p_col.p, F.d_p_val.p, A->d_rowptr.p, A->d_colidx.p,
                           avals, d_crow.p, d_ccol.p, cvals.p);
        CHF_LAUNCH_CHECK();
        CHF_HIP(hipStreamSynchronize(s));
        chf_bsr C = nullptr;
        int st = chf_bsr_create(nc, b, crow.data(), ccol.data(), cvals.p, 1, &C);
        if (st != CHF_OK) fail(st, std::string("coarse operator: ") + chf_last_error());
        H->lev.emplace_back();
        H->lev.back().A = C;
        H->lev.back().own_A = true;
    });
}

extern "C" int chf_levels_setup(chf_levels H, const chf_level_opts* opts, const double* const* v0,
                                int64_t* bad_row) {
    return guarded([&] {
        CHF_CHECK(H && opts, CHF_EINVAL, "NULL argument");
        CHF_CHECK(!H->ready, CHF_EINVAL, "hierarchy already set up");
        CHF_CHECK(opts->degree >= 1, CHF_EINVAL, "degree must be >= 1");
        CHF_CHECK(opts->pattern >= 0 && opts->pattern <= 2, CHF_EINVAL, "bad pattern mode");
        CHF_CHECK(!H->nest || opts->pattern == 1, CHF_EINVAL, "nesting needs the adaptive pattern (pattern = 1)");
        CHF_CHECK(opts->dtype == CHF_F64 || opts->dtype == CHF_F32 || opts->dtype == CHF_BF16 ||
                      opts->dtype == CHF_F64_BF16G, CHF_EINVAL,
                  "bad dtype");
        if (bad_row) *bad_row = -1;
        H->opts = *opts;
        H->vec = mode_vec(opts->dtype);
        const chf_dtype gstore = opts->dtype == CHF_F64_BF16G ? CHF_BF16 : opts->dtype;   // G's storage
        hipStream_t s = 0;
        const int nl = (int)H->lev.size();
        // pattern and factor of level l on stream st
        auto factor_level = [&](int l, hipStream_t st, int64_t* br) {
            chf_level_s& L = H->lev[l];
            if (L.preset) {
                // caller-supplied pattern (e.g. a learned proposal)
            } else if (opts->pattern == 1) {
                L.P = adaptive_pattern_impl(L.A, nullptr, opts->tmax, opts->tau, st);
            } else {
                chf_pattern P = nullptr;
                int rc = opts->pattern == 0 ? chf_pattern_lower(L.A, &P) : CHF_OK;
                if (opts->pattern == 2) {
                    P = new chf_pattern_s;
                    P->nb = L.A->nb;
                    P->rowptr.resize(P->nb + 1);
                    P->colidx.resize(P->nb);
                    for (int64_t k = 0; k <= P->nb; ++k) P->rowptr[k] = k;
                    for (int64_t k = 0; k < P->nb; ++k) P->colidx[k] = (int32_t)k;
                }
                if (rc != CHF_OK) fail(rc, chf_last_error());
                L.P = P;
            }
            if (H->nest) {
                // outer factor for A_l, inner factor for G0 A_l G0^T with
                // Algorithm 1's pattern (same t_max and tau)
                L.G0 = fsai_setup_impl(L.A, *L.P, gstore, br, st);
                std::unique_ptr<chf_bsr_s> A1(bsr_triple_impl(L.A, *L.G0, st));
                L.P1 = adaptive_pattern_impl(A1.get(), nullptr, opts->tmax, opts->tau, st);
                L.G1 = fsai_setup_impl(A1.get(), *L.P1, gstore, br, st);
                L.G = new chf_fsai_s;
                L.G->nb = L.G0->nb;
                L.G->b = L.G0->b;
                L.G->store = L.G0->store;
                L.G->nest_outer = L.G0;
                L.G->nest_inner = L.G1;
            } else {
                L.G = fsai_setup_impl(L.A, *L.P, gstore, br, st);
            }
        };
        // the coarsest level's dense factorisation; a non-SPD operator reports -2
        auto coarse_level = [&](hipStream_t st, int64_t* br) {
            try {
                build_coarse_dense(H->lev[nl - 1], st);
            } catch (const Error& e) {
                if (e.code == CHF_ENOTSPD && br) *br = -2;
                throw;
            }
        };
        auto bound_level = [&](int l, hipStream_t st) {
            chf_level_s& L = H->lev[l];
            if (v0 && v0[l])
                lanczos_impl(L.A, *L.G, opts->dtype, opts->lanczos_iters, v0[l], opts->safety, &L.beta, nullptr, st);
        };
        // Level 0 is factored first. Its Lanczos bound (bandwidth-bound SpMVs)
        // then runs on the caller's stream while a host thread sets up the
        // coarser levels (latency-bound pattern and factor kernels) and the
        // coarsest solve on a stream of its own; the levels share no data.
        // Frees inside the overlapped part are deferred to its end (a free
        // would synchronise the device and so wait for the other stream).
        if (nl > 1) factor_level(0, s, bad_row);
        hipStream_t s1 = nullptr;
        std::thread worker;
        std::exception_ptr werr, merr;
        int64_t wbad = -1;
        std::vector<void*> defer_main, defer_worker;
        if (nl > 2) {
            int dev = 0;
            CHF_HIP(hipGetDevice(&dev));
            CHF_HIP(hipStreamCreateWithFlags(&s1, hipStreamNonBlocking));
            auto work = [&, dev] {
                set_free_deferral(&defer_worker);
                try {
                    CHF_HIP(hipSetDevice(dev));   // the current device is per host thread
                    for (int l = 1; l < nl - 1; ++l) {
                        factor_level(l, s1, &wbad);
                        bound_level(l, s1);
                    }
                    coarse_level(s1, &wbad);
                    CHF_HIP(hipStreamSynchronize(s1));
                } catch (...) {
                    werr = std::current_exception();
                }
                set_free_deferral(nullptr);
            };
            try {
                worker = std::thread(work);
            } catch (...) {
                (void)hipStreamDestroy(s1);
                throw;
            }
            set_free_deferral(&defer_main);
        }
        try {
            if (nl > 1) bound_level(0, s);
            if (nl <= 2) coarse_level(s, bad_row);
        } catch (...) {
            merr = std::current_exception();
        }
        set_free_deferral(nullptr);
        if (worker.joinable()) worker.join();
        if (s1) (void)hipStreamDestroy(s1);
        for (void* q : defer_main) dev_free(q);
        for (void* q : defer_worker) dev_free(q);
        if (merr) std::rethrow_exception(merr);
        if (werr) {
            if (bad_row && wbad != -1) *bad_row = wbad;
            std::rethrow_exception(werr);
        }
        if (H->vec != CHF_F64)
            for (int l = 0; l < nl; ++l) (void)H->lev[l].A->sell(CHF_F32, s);
        alloc_vectors(*H);
        H->ready = true;
        CHF_HIP(hipStreamSynchronize(s));
    });
}

extern "C" int chf_levels_set_pattern(chf_levels H, int level, chf_pattern P) {
    return guarded([&] {
        CHF_CHECK(H && P && level >= 0 && level + 1 < (int)H->lev.size(), CHF_EINVAL, "bad level or pattern");
        CHF_CHECK(!H->ready, CHF_EINVAL, "hierarchy already set up");
        chf_level_s& L = H->lev[level];
        CHF_CHECK(P->nb == L.A->nb, CHF_EINVAL, "pattern and level sizes differ");
        validate_pattern(P->nb, P->rowptr.data(), P->colidx.data());
        if (L.P) delete L.P;
        L.P = new chf_pattern_s(*P);
        L.preset = true;
    });
}

extern "C" int chf_levels_destroy(chf_levels H) {
    return guarded([&] { delete H; });
}

extern "C" int chf_levels_info(chf_levels H, int* nlevels, int64_t* nb_per_level) {
    return guarded([&] {
        CHF_CHECK(H, CHF_EINVAL, "NULL handle");
        if (nlevels) *nlevels = (int)H->lev.size();
        if (nb_per_level)
            for (size_t l = 0; l < H->lev.size(); ++l) nb_per_level[l] = H->lev[l].A->nb;
    });
}

extern "C" int chf_levels_get(chf_levels H, int level, chf_bsr* A, chf_fsai* G, chf_pattern* P) {
    return guarded([&] {
        CHF_CHECK(H && level >= 0 && level < (int)H->lev.size(), CHF_EINVAL, "bad level");
        if (A) *A = H->lev[level].A;
        if (G) *G = H->lev[level].G;
        if (P) *P = H->lev[level].P;
    });
}

extern "C" int chf_levels_get_beta(chf_levels H, int level, double* beta) {
    return guarded([&] {
        CHF_CHECK(H && beta && level >= 0 && level < (int)H->lev.size(), CHF_EINVAL, "bad level");
        *beta = H->lev[level].beta;
    });
}

extern "C" int chf_levels_set_beta(chf_levels H, int level, double beta) {
    return guarded([&] {
        CHF_CHECK(H && level >= 0 && level < (int)H->lev.size(), CHF_EINVAL, "bad level");
        CHF_CHECK(beta > 0 && std::isfinite(beta), CHF_EINVAL, "beta must be positive and finite");
        H->lev[level].beta = beta;
    });
}

static void check_ready(chf_levels_s* H) {
    CHF_CHECK(H && H->ready, CHF_EINVAL, "hierarchy not set up");
    for (size_t l = 0; l + 1 < H->lev.size(); ++l)
        CHF_CHECK(H->lev[l].beta > 0, CHF_EINVAL, "level " + std::to_string(l) + " has no spectral bound");
}

extern "C" int chf_vcycle(chf_levels H, const void* b, void* x, int x_is_zero, hipStream_t stream) {
    return guarded([&] {
        check_ready(H);
        CHF_CHECK(b && x, CHF_EINVAL, "NULL vector");
        vcycle_rec(*H, 0, b, x, x_is_zero != 0, stream);
    });
}

extern "C" int chf_levels_set_nesting(chf_levels H, int nest) {
    return guarded([&] {
        CHF_CHECK(H, CHF_EINVAL, "NULL hierarchy");
        CHF_CHECK(!H->ready, CHF_EINVAL, "hierarchy already set up");
        CHF_CHECK(nest == 0 || nest == 1, CHF_EINVAL, "nesting depth must be 0 or 1");
        H->nest = nest;
    });
}

extern "C" int chf_levels_set_cycle(chf_levels H, chf_smoother smoother, double param, chf_cycle cycle) {
    return guarded([&] {
        CHF_CHECK(H, CHF_EINVAL, "NULL hierarchy");
        CHF_CHECK(smoother == CHF_SMOOTH_CHEB4 || smoother == CHF_SMOOTH_CHEB1 || smoother == CHF_SMOOTH_RICHARDSON,
                  CHF_EINVAL, "unknown smoother");
        CHF_CHECK(cycle == CHF_CYCLE_VKK || cycle == CHF_CYCLE_V2K0, CHF_EINVAL, "unknown cycle");
        if (smoother == CHF_SMOOTH_CHEB1)
            CHF_CHECK(param > 0.0 && param < 1.0, CHF_EINVAL, "first-kind smoothing needs 0 < rho < 1");
        if (smoother == CHF_SMOOTH_RICHARDSON)
            CHF_CHECK(param > 0.0 && std::isfinite(param), CHF_EINVAL, "Richardson needs omega > 0");
        H->smoother = smoother;
        H->sm_param = param;
        H->cycle = cycle;
    });
}

extern "C" int chf_levels_energy_factor(chf_levels H, const double* e0, double tol, int maxit, double* rho,
                                        int* cycles, hipStream_t stream) {
    return guarded([&] {
        check_ready(H);
        CHF_CHECK(e0 && rho && maxit >= 1 && tol >= 0, CHF_EINVAL, "bad argument");
        hipStream_t s = stream;
        chf_level_s& L0 = H->lev[0];
        const int64_t n = L0.A->nb * (int64_t)L0.A->b;
        if (H->pcg_n != n) {
            H->pcg_buf.alloc((size_t)std::max<int64_t>(1, 6 * n));
            H->scal.alloc(8);
            H->part.alloc(RED_BLOCKS);
            H->pcg_n = n;
        }
        double* e64 = H->pcg_buf.p;        // the error in FP64
        double* ae = e64 + n;              // A e
        void* ew = e64 + 2 * n;            // the error in the working dtype
        void* zw = e64 + 3 * n;            // zero right-hand side, working dtype
        double* sc = H->scal.p;
        const Sell& A64 = L0.A->sell(CHF_F64, s);
        const bool mixed = H->vec != CHF_F64;
        fill_zero(zw, n * vec_size(H->vec), s);
        cast_vec(CHF_F64, e0, H->vec, mixed ? ew : (void*)e64, n, s);
        // e^T A e of the current iterate, in FP64
        auto energy = [&]() {
            if (mixed) cast_vec(H->vec, ew, CHF_F64, e64, n, s);
            sell_spmv(A64, CHF_F64, e64, ae, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
            dot(CHF_F64, e64, ae, n, sc, H->part.p, s);
            double v;
            CHF_HIP(hipMemcpyAsync(&v, sc, 8, hipMemcpyDeviceToHost, s));
            CHF_HIP(hipStreamSynchronize(s));
            return v;
        };
        const double en0 = energy();
        CHF_CHECK(std::isfinite(en0) && en0 > 0, CHF_EINVAL, "e0 must be nonzero and finite");
        double en = en0;
        int cyc = 0;
        while (cyc < maxit) {
            vcycle_rec(*H, 0, zw, mixed ? ew : (void*)e64, false, s);
            ++cyc;
            en = energy();
            CHF_CHECK(std::isfinite(en), CHF_EBREAKDOWN, "energy norm of the error is not finite");
            if (std::sqrt(en / en0) < tol) break;
        }
        *rho = std::pow(en / en0, 1.0 / (2.0 * cyc));
        if (cycles) *cycles = cyc;
    });
}

extern "C" int chf_pcg_solve(chf_levels H, const double* b, double* x, double rtol, int maxit, int flexible,
                             int* iters, double* relres_hist, double* true_relres, hipStream_t stream) {
    int status = CHF_OK;
    int rc = guarded([&] {
        check_ready(H);
        CHF_CHECK(b && x && maxit >= 0 && rtol >= 0, CHF_EINVAL, "bad argument");
        CHF_CHECK(flexible || H->cycle == CHF_CYCLE_VKK, CHF_EINVAL,
                  "a V(2k,0) cycle is not symmetric: use the flexible form");
        hipStream_t s = stream;
        chf_level_s& L0 = H->lev[0];
        const int64_t n = L0.A->nb * (int64_t)L0.A->b;
        if (H->pcg_n != n) {
            H->pcg_buf.alloc((size_t)std::max<int64_t>(1, 6 * n));
            H->scal.alloc(8);
            H->part.alloc(RED_BLOCKS);
            H->pcg_n = n;
        }
        double* r = H->pcg_buf.p;
        double* z = r + n;
        double* p = z + n;
        double* q = p + n;
        double* rold = q + n;
        double* tmp = rold + n;
        double* sc = H->scal.p;
        const Sell& A64 = L0.A->sell(CHF_F64, s);
        const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
        auto precond = [&](const double* rin, double* zout) {
            if (H->vec == CHF_F64) {
                vcycle_rec(*H, 0, rin, zout, true, s);
            } else {
                cast_vec(CHF_F64, rin, CHF_F32, L0.bvec.p, n, s);
                vcycle_rec(*H, 0, L0.bvec.p, L0.xvec.p, true, s);
                cast_vec(CHF_F32, L0.xvec.p, CHF_F64, zout, n, s);
            }
        };
        auto read = [&](int idx) {
            double v;
            CHF_HIP(hipMemcpyAsync(&v, sc + idx, 8, hipMemcpyDeviceToHost, s));
            CHF_HIP(hipStreamSynchronize(s));
            return v;
        };
        fill_zero(x, n * 8, s);
        cast_vec(CHF_F64, b, CHF_F64, r, n, s);
        dot(CHF_F64, b, b, n, sc + 2, H->part.p, s);
        const double bnorm = std::sqrt(read(2));
        CHF_CHECK(std::isfinite(bnorm), CHF_EINVAL, "non-finite right-hand side");
        int it = 0;
        if (relres_hist) relres_hist[0] = bnorm > 0 ? 1.0 : 0.0;
        if (bnorm == 0.0 || 1.0 <= rtol) {
            if (iters) *iters = 0;
            if (true_relres) *true_relres = 0.0;
            return;
        }
        precond(r, z);
        cast_vec(CHF_F64, z, CHF_F64, p, n, s);
        dot(CHF_F64, r, z, n, sc + 0, H->part.p, s);
        bool converged = false;
        for (it = 1; it <= maxit; ++it) {
            sell_spmv(A64, CHF_F64, p, q, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
            dot(CHF_F64, p, q, n, sc + 1, H->part.p, s);
            hipLaunchKernelGGL(k_pcg_xr, dim3(grid), dim3(256), 0, s, n, (const double*)sc, (const double*)p,
                               (const double*)q, x, r, flexible ? rold : nullptr);
            CHF_LAUNCH_CHECK();
            dot(CHF_F64, r, r, n, sc + 2, H->part.p, s);
            double hs[3];
            CHF_HIP(hipMemcpyAsync(hs, sc, 24, hipMemcpyDeviceToHost, s));
            CHF_HIP(hipStreamSynchronize(s));
            if (!(hs[1] > 0)) { status = CHF_EBREAKDOWN; set_error("PCG breakdown: p^T A p <= 0"); break; }
            if (!(hs[0] > 0)) { status = CHF_EBREAKDOWN; set_error("PCG breakdown: r^T z <= 0"); break; }
            const double rel = std::sqrt(hs[2]) / bnorm;
            if (relres_hist) relres_hist[it] = rel;
            if (!std::isfinite(rel)) { status = CHF_EBREAKDOWN; set_error("PCG produced a non-finite residual"); break; }
            if (rel <= rtol) { converged = true; break; }
            precond(r, z);
            dot(CHF_F64, r, z, n, sc + 3, H->part.p, s);
            if (flexible) {
                hipLaunchKernelGGL(k_sub, dim3(grid), dim3(256), 0, s, n, (const double*)r, (const double*)rold, tmp);
                CHF_LAUNCH_CHECK();
                dot(CHF_F64, z, tmp, n, sc + 4, H->part.p, s);
            } else {
                hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, s, sc, 3, 4);
                CHF_LAUNCH_CHECK();
            }
            hipLaunchKernelGGL(k_pcg_p, dim3(grid), dim3(256), 0, s, n, sc, (const double*)z, p);
            CHF_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, s, sc, 3, 0);
            CHF_LAUNCH_CHECK();
        }
        if (iters) *iters = std::min(it, maxit);
        if (true_relres) {
            sell_spmv(A64, CHF_F64, x, tmp, b, EPI_RES, nullptr, nullptr, 0, 0, s);
            dot(CHF_F64, tmp, tmp, n, sc + 2, H->part.p, s);
            *true_relres = std::sqrt(read(2)) / bnorm;
        }
        if (status == CHF_OK && !converged) {
            status = CHF_ENOCONV;
            set_error("PCG did not reach rtol within maxit iterations");
        }
    });
    return rc != CHF_OK ? rc : status;
}

extern "C" int chf_bicgstab_solve(chf_levels H, const double* b, double* x, double rtol, int maxit, int* iters,
                                  double* relres_hist, double* true_relres, hipStream_t stream) {
    int status = CHF_OK;
    int rc = guarded([&] {
        check_ready(H);
        CHF_CHECK(b && x && maxit >= 0 && rtol >= 0, CHF_EINVAL, "bad argument");
        hipStream_t s = stream;
        chf_level_s& L0 = H->lev[0];
        const int64_t n = L0.A->nb * (int64_t)L0.A->b;
        if (H->bicg_n != n) {
            H->bicg_buf.alloc((size_t)std::max<int64_t>(1, 8 * n));
            H->bicg_scal.alloc(16);
            H->part.alloc(RED_BLOCKS);
            H->bicg_n = n;
        }
        double* r = H->bicg_buf.p;
        double* rh = r + n;
        double* p = rh + n;
        double* v = p + n;
        double* ph = v + n;
        double* sv = ph + n;
        double* sh = sv + n;
        double* t = sh + n;
        double* bs = H->bicg_scal.p;
        const Sell& A64 = L0.A->sell(CHF_F64, s);
        const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
        auto precond = [&](const double* rin, double* zout) {
            if (H->vec == CHF_F64) {
                vcycle_rec(*H, 0, rin, zout, true, s);
            } else {
                cast_vec(CHF_F64, rin, CHF_F32, L0.bvec.p, n, s);
                vcycle_rec(*H, 0, L0.bvec.p, L0.xvec.p, true, s);
                cast_vec(CHF_F32, L0.xvec.p, CHF_F64, zout, n, s);
            }
        };
        auto read = [&](int idx) {
            double val;
            CHF_HIP(hipMemcpyAsync(&val, bs + idx, 8, hipMemcpyDeviceToHost, s));
            CHF_HIP(hipStreamSynchronize(s));
            return val;
        };
        fill_zero(x, n * 8, s);
        cast_vec(CHF_F64, b, CHF_F64, r, n, s);
        cast_vec(CHF_F64, b, CHF_F64, rh, n, s);
        dot(CHF_F64, b, b, n, bs + 7, H->part.p, s);
        const double bnorm = std::sqrt(read(7));
        CHF_CHECK(std::isfinite(bnorm), CHF_EINVAL, "non-finite right-hand side");
        int it = 0, nh = 0;
        if (relres_hist) relres_hist[nh++] = bnorm > 0 ? 1.0 : 0.0;
        if (bnorm == 0.0 || 1.0 <= rtol) {
            if (iters) *iters = 0;
            if (true_relres) *true_relres = 0.0;
            return;
        }
        bool converged = false;
        for (it = 1; it <= maxit; ++it) {
            dot(CHF_F64, rh, r, n, bs + 0, H->part.p, s);
            hipLaunchKernelGGL(k_bicg_p, dim3(grid), dim3(256), 0, s, n, (const double*)bs, (const double*)r,
                               (const double*)v, p, it == 1 ? 1 : 0);
            CHF_LAUNCH_CHECK();
            precond(p, ph);
            sell_spmv(A64, CHF_F64, ph, v, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
            dot(CHF_F64, rh, v, n, bs + 4, H->part.p, s);
            hipLaunchKernelGGL(k_bicg_s, dim3(grid), dim3(256), 0, s, n, bs, (const double*)r, (const double*)v, sv);
            CHF_LAUNCH_CHECK();
            dot(CHF_F64, sv, sv, n, bs + 7, H->part.p, s);
            double hs[8];
            CHF_HIP(hipMemcpyAsync(hs, bs, 64, hipMemcpyDeviceToHost, s));
            CHF_HIP(hipStreamSynchronize(s));
            if (hs[0] == 0.0 || hs[4] == 0.0 || !std::isfinite(hs[2])) {
                status = CHF_EBREAKDOWN;
                set_error("BiCGStab breakdown: (r^, r) or (r^, v) vanished");
                break;
            }
            double rel = std::sqrt(hs[7]) / bnorm;
            if (relres_hist) relres_hist[nh++] = rel;
            if (rel <= rtol) {
                hipLaunchKernelGGL(k_bicg_half, dim3(grid), dim3(256), 0, s, n, (const double*)bs,
                                   (const double*)ph, x);
                CHF_LAUNCH_CHECK();
                converged = true;
                break;
            }
            precond(sv, sh);
            sell_spmv(A64, CHF_F64, sh, t, nullptr, EPI_AX, nullptr, nullptr, 0, 0, s);
            dot(CHF_F64, t, sv, n, bs + 5, H->part.p, s);
            dot(CHF_F64, t, t, n, bs + 6, H->part.p, s);
            hipLaunchKernelGGL(k_bicg_xr, dim3(grid), dim3(256), 0, s, n, bs, (const double*)ph, (const double*)sh,
                               (const double*)sv, (const double*)t, x, r);
            CHF_LAUNCH_CHECK();
            dot(CHF_F64, r, r, n, bs + 7, H->part.p, s);
            CHF_HIP(hipMemcpyAsync(hs, bs, 64, hipMemcpyDeviceToHost, s));
            CHF_HIP(hipStreamSynchronize(s));
            if (!(hs[6] > 0.0) || !std::isfinite(hs[3]) || hs[3] == 0.0) {
                status = CHF_EBREAKDOWN;
                set_error("BiCGStab breakdown: omega vanished");
                break;
            }
            rel = std::sqrt(hs[7]) / bnorm;
            if (relres_hist) relres_hist[nh++] = rel;
            if (!std::isfinite(rel)) {
                status = CHF_EBREAKDOWN;
                set_error("BiCGStab produced a non-finite residual");
                break;
            }
            if (rel <= rtol) {
                converged = true;
                break;
            }
            hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, s, bs, 0, 1);
            CHF_LAUNCH_CHECK();
        }
        if (iters) *iters = std::min(it, maxit);
        if (true_relres) {
            sell_spmv(A64, CHF_F64, x, t, b, EPI_RES, nullptr, nullptr, 0, 0, s);
            dot(CHF_F64, t, t, n, bs + 7, H->part.p, s);
            *true_relres = std::sqrt(read(7)) / bnorm;
        }
        if (status == CHF_OK && !converged) {
            status = CHF_ENOCONV;
            set_error("BiCGStab did not reach rtol within maxit iterations");
        }
    });
    return rc != CHF_OK ? rc : status;
}
