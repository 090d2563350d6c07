// Block-sparse matrices: creation, the slice-interleaved SpMV layout and the
// SpMV kernels with their fused epilogues (residual, fourth-kind Chebyshev
// update of Algorithm 3).
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "internal.h"
#include "kernels_common.h"

namespace chf {

// ---------------------------------------------------------------- layout --
SellPlan sell_plan(int64_t nb, int b, const std::vector<int64_t>& rowptr,
                   const std::vector<int32_t>& colidx, const std::vector<int64_t>* srcmap) {
    SellPlan p;
    p.nb = nb;
    p.b = b;
    p.S = std::max(1, 64 / b);
    p.L = p.S * b;
    p.nslices = (nb + p.S - 1) / p.S;
    p.slice_off.assign(p.nslices + 1, 0);
    for (int64_t s = 0; s < p.nslices; ++s) {
        int64_t w = 0;
        for (int64_t r = s * p.S; r < std::min<int64_t>(nb, (s + 1) * p.S); ++r)
            w = std::max<int64_t>(w, rowptr[r + 1] - rowptr[r]);
        CHF_CHECK(p.slice_off[s] + w < (1ll << 31), CHF_EINVAL, "matrix too large for the SpMV layout");
        p.slice_off[s + 1] = (int)(p.slice_off[s] + w);
    }
    p.nslots = p.slice_off[p.nslices];
    CHF_CHECK(p.nslots * (int64_t)p.S < (1ll << 31), CHF_EINVAL, "matrix too large for the SpMV layout");
    p.cols.assign(p.nslots * p.S, 0);
    p.src.assign(p.nslots * p.S, -1);
    for (int64_t s = 0; s < p.nslices; ++s) {
        int64_t off = p.slice_off[s], w = p.slice_off[s + 1] - off;
        for (int lr = 0; lr < p.S; ++lr) {
            int64_t row = s * p.S + lr;
            for (int64_t j = 0; j < w; ++j) {
                int64_t e = (off + j) * p.S + lr;
                if (row < nb && j < rowptr[row + 1] - rowptr[row]) {
                    int64_t idx = rowptr[row] + j;
                    p.cols[e] = colidx[idx];
                    p.src[e] = srcmap ? (*srcmap)[idx] : idx;
                } else {
                    p.cols[e] = row < nb ? (int)row : 0;
                    p.src[e] = -1;
                }
            }
        }
    }
    return p;
}

// Column runs of one slot row: run q covers columns start[q] .. start[q+1]-1.
struct SellRuns {
    int n = 0;
    int start[65] = {};
};

// Run widths of the layouts with a specialised SpMV (16-byte loads where the
// block width allows):
//   b = 10: FP64 2 x 5; FP32 4, 4, 2; BF16 8, 2;
//   b = 21: FP64 2 x 10, 1; FP32 4 x 5, 1; BF16 8, 8, 4, 1;
// every other b: single columns. The id V is the widest run.
static SellRuns sell_runs(int b, chf_dtype t, int* V) {
    std::vector<int> w;
    if (b == 10) {
        if (t == CHF_F64) w = {2, 2, 2, 2, 2};
        else if (t == CHF_F32) w = {4, 4, 2};
        else w = {8, 2};
    } else if (b == 21) {
        if (t == CHF_F64) w = {2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 1};
        else if (t == CHF_F32) w = {4, 4, 4, 4, 4, 1};
        else w = {8, 8, 4, 1};
    } else {
        w.assign(b, 1);
    }
    SellRuns r;
    r.n = (int)w.size();
    int v = 1;
    for (int q = 0; q < r.n; ++q) {
        r.start[q + 1] = r.start[q] + w[q];
        v = std::max(v, w[q]);
    }
    if (V) *V = v;
    return r;
}

// Elements per slot: b * L, padded to a multiple of 16 bytes when runs are
// loaded 16 bytes at a time (keeps every run of every slot aligned).
__host__ __device__ constexpr int sell_slot_stride(int b, int L, int V, int elem) {
    return V == 1 ? b * L : (b * L * elem + 15) / 16 * 16 / elem;
}

template <typename T>
__global__ void k_sell_pack(int64_t total, int b, int S, int L, int stride, SellRuns runs,
                            const int64_t* __restrict__ src, const double* __restrict__ blocks, int transpose,
                            T* __restrict__ out) {
    const int bl = b * L;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t slot = e / stride;
        const int rem = (int)(e - slot * stride);
        double v = 0.0;
        if (rem < bl) {
            int q = 0;
            while (q + 1 < runs.n && L * runs.start[q + 1] <= rem) ++q;
            const int w = runs.start[q + 1] - runs.start[q];
            const int rem2 = rem - L * runs.start[q];
            const int lane = rem2 / w;
            const int c = runs.start[q] + (rem2 - lane * w);
            const int lr = lane / b, r = lane - lr * b;
            const int64_t sb = src[slot * S + lr];
            if (sb >= 0) {
                const double* blk = blocks + sb * b * b;
                v = transpose ? blk[c * b + r] : blk[r * b + c];
            }
        }
        store_from_f64<T>(out + e, v);
    }
}

static int sell_vec_width(int b, chf_dtype t) {
    int v = 1;
    sell_runs(b, t, &v);
    return v;
}

void sell_build(Sell& out, const SellPlan& plan, const double* d_src_blocks, bool transpose,
                chf_dtype dtype, hipStream_t s) {
    out.nb = plan.nb;
    out.ndof = plan.nb * (int64_t)plan.b;
    out.b = plan.b;
    out.S = plan.S;
    out.L = plan.L;
    const SellRuns runs = sell_runs(plan.b, dtype, &out.V);
    out.stride = sell_slot_stride(plan.b, plan.L, out.V, (int)dtype_size(dtype));
    out.nslices = plan.nslices;
    out.nslots = plan.nslots;
    out.dtype = dtype;
    out.slice_off.alloc(plan.slice_off.size());
    out.slice_off.upload(plan.slice_off.data(), plan.slice_off.size(), s);
    out.cols.alloc(std::max<size_t>(1, plan.cols.size()));
    out.cols.upload(plan.cols.data(), plan.cols.size(), s);
    DevBuf<int64_t> src(std::max<size_t>(1, plan.src.size()));
    src.upload(plan.src.data(), plan.src.size(), s);
    int64_t total = plan.nslots * (int64_t)out.stride;
    out.vals.alloc(std::max<int64_t>(1, total) * dtype_size(dtype));
    if (total > 0) {
        int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
        if (dtype == CHF_F64)
            hipLaunchKernelGGL((k_sell_pack<double>), dim3(grid), dim3(256), 0, s, total, plan.b, plan.S, plan.L,
                               out.stride, runs, src.p, d_src_blocks, (int)transpose, (double*)out.vals.p);
        else if (dtype == CHF_F32)
            hipLaunchKernelGGL((k_sell_pack<float>), dim3(grid), dim3(256), 0, s, total, plan.b, plan.S, plan.L,
                               out.stride, runs, src.p, d_src_blocks, (int)transpose, (float*)out.vals.p);
        else
            hipLaunchKernelGGL((k_sell_pack<bf16_t>), dim3(grid), dim3(256), 0, s, total, plan.b, plan.S, plan.L,
                               out.stride, runs, src.p, d_src_blocks, (int)transpose, (bf16_t*)out.vals.p);
        CHF_LAUNCH_CHECK();
    }
    // src is freed at scope exit; make sure the pack has consumed it.
    CHF_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ SpMV --
// One 64-wide wavefront per slice; lane = local_row * b + r owns output
// scalar r of block row slice*S + local_row and accumulates
// sum_j sum_c block_j[r][c] * x[col_j * b + c] in TV precision. Each matrix
// load instruction reads L * V contiguous elements; x is gathered V values at
// a time. Workgroups are mapped so that each of the 8 XCDs (which receive
// workgroups round-robin) works on one contiguous range of slices, keeping the
// x gathers of neighbouring block rows in that XCD's L2.
// Matrix values are streamed once per product; with NTL they are loaded with
// the non-temporal hint so that they do not displace the x gathers in L2.
typedef double d2v __attribute__((ext_vector_type(2)));
template <int V, typename TA, typename TV, bool NTL = false>
struct Pair;
template <typename TA, typename TV, bool NTL>
struct Pair<1, TA, TV, NTL> {
    __device__ static inline TV dot(const TA* v, const TV* x) {
        if constexpr (NTL && !std::is_same<TA, bf16_t>::value)
            return (TV)__builtin_nontemporal_load(v) * x[0];
        else
            return load_as<TV>(v) * x[0];
    }
};
template <typename TV, bool NTL>
struct Pair<2, double, TV, NTL> {
    __device__ static inline TV dot(const double* v, const TV* x) {
        d2v a;
        if constexpr (NTL)
            a = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(v));
        else
            a = *reinterpret_cast<const d2v*>(v);
        if constexpr (sizeof(TV) == 8) {
            const double2 y = *reinterpret_cast<const double2*>(x);
            return a.x * y.x + a.y * y.y;
        } else {
            return (TV)a.x * x[0] + (TV)a.y * x[1];
        }
    }
};
typedef float f2v __attribute__((ext_vector_type(2)));
template <typename TV, bool NTL>
struct Pair<2, float, TV, NTL> {
    __device__ static inline TV dot(const float* v, const TV* x) {
        f2v a;
        if constexpr (NTL)
            a = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(v));
        else
            a = *reinterpret_cast<const f2v*>(v);
        if constexpr (sizeof(TV) == 4) {
            const float2 y = *reinterpret_cast<const float2*>(x);
            return a.x * y.x + a.y * y.y;
        } else {
            return (TV)a.x * x[0] + (TV)a.y * x[1];
        }
    }
};
template <typename TV, bool NTL>
struct Pair<2, bf16_t, TV, NTL> {
    __device__ static inline TV dot(const bf16_t* v, const TV* x) {
        uint32_t u;
        if constexpr (NTL)
            u = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(v));
        else
            u = *reinterpret_cast<const uint32_t*>(v);
        return (TV)bf16_bits_to_f32((uint16_t)(u & 0xffffu)) * x[0] + (TV)bf16_bits_to_f32((uint16_t)(u >> 16)) * x[1];
    }
};

typedef float f4v __attribute__((ext_vector_type(4)));
template <typename TV, bool NTL>
struct Pair<4, float, TV, NTL> {
    __device__ static inline TV dot(const float* v, const TV* x) {
        f4v a;
        if constexpr (NTL)
            a = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(v));
        else
            a = *reinterpret_cast<const f4v*>(v);
        if constexpr (sizeof(TV) == 4) {
            const float2 y0 = *reinterpret_cast<const float2*>(x);
            const float2 y1 = *reinterpret_cast<const float2*>(x + 2);
            return (a.x * y0.x + a.y * y0.y) + (a.z * y1.x + a.w * y1.y);
        } else {
            return ((TV)a.x * x[0] + (TV)a.y * x[1]) + ((TV)a.z * x[2] + (TV)a.w * x[3]);
        }
    }
};
typedef unsigned int u2v __attribute__((ext_vector_type(2)));
template <typename TV, bool NTL>
struct Pair<4, bf16_t, TV, NTL> {
    __device__ static inline TV dot(const bf16_t* v, const TV* x) {
        u2v u;
        if constexpr (NTL)
            u = __builtin_nontemporal_load(reinterpret_cast<const u2v*>(v));
        else
            u = *reinterpret_cast<const u2v*>(v);
        return ((TV)bf16_bits_to_f32((uint16_t)(u.x & 0xffffu)) * x[0] +
                (TV)bf16_bits_to_f32((uint16_t)(u.x >> 16)) * x[1]) +
               ((TV)bf16_bits_to_f32((uint16_t)(u.y & 0xffffu)) * x[2] +
                (TV)bf16_bits_to_f32((uint16_t)(u.y >> 16)) * x[3]);
    }
};

typedef unsigned int u4v __attribute__((ext_vector_type(4)));
template <typename TV, bool NTL>
struct Pair<8, bf16_t, TV, NTL> {
    __device__ static inline TV dot(const bf16_t* v, const TV* x) {
        u4v u;
        if constexpr (NTL)
            u = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(v));
        else
            u = *reinterpret_cast<const u4v*>(v);
        auto lo = [](unsigned w) { return (TV)bf16_bits_to_f32((uint16_t)(w & 0xffffu)); };
        auto hi = [](unsigned w) { return (TV)bf16_bits_to_f32((uint16_t)(w >> 16)); };
        return ((lo(u.x) * x[0] + hi(u.x) * x[1]) + (lo(u.y) * x[2] + hi(u.y) * x[3])) +
               ((lo(u.z) * x[4] + hi(u.z) * x[5]) + (lo(u.w) * x[6] + hi(u.w) * x[7]));
    }
};

__device__ inline int64_t xcd_slice_block(int64_t nwork_blocks) {
    // gridDim.x is a multiple of 8; block id b runs on XCD b % 8
    const int64_t per = gridDim.x / 8;
    return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// Sum over the slots j = j_first, j_first + STEP, ... < j1 of one lane's row r
// of its block row: sum_c block_j[r][c] x[col_j b + c].
template <int BT, int V, typename TA, typename TV, bool NTL, int STEP>
__device__ inline TV sell_lane_sum(int b, int S, int L, int lane, int lr, int j_first, int j1,
                                   const int* __restrict__ cols, const TA* __restrict__ vals,
                                   const TV* __restrict__ x) {
    TV acc = 0;
    if constexpr (BT == 10 && V == 8) {
        // runs of 8 and 2 columns per slot (BF16: 16- and 4-byte loads)
        const int64_t stride = (int64_t)10 * L;
        const TA* v = vals + (int64_t)j_first * stride;
        const int* cp = cols + (int64_t)j_first * S + lr;
#pragma unroll 2
        for (int j = j_first; j < j1; j += STEP) {
            const TV* xc = x + (int64_t)(*cp) * 10;
            acc += Pair<8, TA, TV, NTL>::dot(v + lane * 8, xc);
            acc += Pair<2, TA, TV, NTL>::dot(v + 8 * L + lane * 2, xc + 8);
            v += STEP * stride;
            cp += STEP * S;
        }
    } else if constexpr (BT == 10 && V == 4) {
        // runs of 4, 4 and 2 columns per slot (16-, 16- and 8-byte loads)
        const int64_t stride = (int64_t)10 * L;
        const TA* v = vals + (int64_t)j_first * stride;
        const int* cp = cols + (int64_t)j_first * S + lr;
#pragma unroll 2
        for (int j = j_first; j < j1; j += STEP) {
            const TV* xc = x + (int64_t)(*cp) * 10;
            acc += Pair<4, TA, TV, NTL>::dot(v + lane * 4, xc);
            acc += Pair<4, TA, TV, NTL>::dot(v + 4 * L + lane * 4, xc + 4);
            acc += Pair<2, TA, TV, NTL>::dot(v + 8 * L + lane * 2, xc + 8);
            v += STEP * stride;
            cp += STEP * S;
        }
    } else if constexpr (BT == 21) {
        // FP64: ten runs of 2 and one of 1 column; FP32: five runs of 4 and
        // one of 1; BF16: runs of 8, 8, 4 and 1 (16-byte loads but for the
        // last column); slots padded to 16 bytes
        constexpr int SS = sell_slot_stride(21, 63, V, (int)sizeof(TA));
        const TA* v = vals + (int64_t)j_first * SS;
        const int* cp = cols + (int64_t)j_first * S + lr;
#pragma unroll 1
        for (int j = j_first; j < j1; j += STEP) {
            // x + 21 col is only 8- (FP64) or 4-byte (FP32) aligned: x is read
            // one value at a time, the matrix runs 16 bytes at a time
            const TV* xc = x + (int64_t)(*cp) * 21;
            if constexpr (sizeof(TA) == 8) {
#pragma unroll
                for (int q = 0; q < 10; ++q) {
                    d2v a;
                    if constexpr (NTL)
                        a = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(v + q * 2 * L + lane * 2));
                    else
                        a = *reinterpret_cast<const d2v*>(v + q * 2 * L + lane * 2);
                    acc += (TV)a.x * xc[2 * q] + (TV)a.y * xc[2 * q + 1];
                }
            } else if constexpr (sizeof(TA) == 4) {
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    f4v a;
                    if constexpr (NTL)
                        a = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(v + q * 4 * L + lane * 4));
                    else
                        a = *reinterpret_cast<const f4v*>(v + q * 4 * L + lane * 4);
                    acc += ((TV)a.x * xc[4 * q] + (TV)a.y * xc[4 * q + 1]) +
                           ((TV)a.z * xc[4 * q + 2] + (TV)a.w * xc[4 * q + 3]);
                }
            } else {
                acc += Pair<8, TA, TV, NTL>::dot(v + lane * 8, xc);
                acc += Pair<8, TA, TV, NTL>::dot(v + 8 * L + lane * 8, xc + 8);
                acc += Pair<4, TA, TV, NTL>::dot(v + 16 * L + lane * 4, xc + 16);
            }
            acc += Pair<1, TA, TV, NTL>::dot(v + 20 * L + lane, xc + 20);
            v += STEP * SS;
            cp += STEP * S;
        }
    } else if constexpr (BT > 0) {
        constexpr int NQ = BT / V;
        const int64_t stride = (int64_t)NQ * L * V;
        const TA* v = vals + (int64_t)j_first * stride + lane * V;
        const int* cp = cols + (int64_t)j_first * S + lr;
#pragma unroll 1
        for (int j = j_first; j < j1; j += STEP) {
            const TV* xc = x + (int64_t)(*cp) * BT;
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc += Pair<V, TA, TV, NTL>::dot(v + q * L * V, xc + q * V);
            v += STEP * stride;
            cp += STEP * S;
        }
    } else {
        for (int j = j_first; j < j1; j += STEP) {
            const int col = cols[(int64_t)j * S + lr];
            const TA* v = vals + (int64_t)j * b * L + lane;
            const TV* xc = x + (int64_t)col * b;
            for (int c = 0; c < b; ++c) acc += Pair<1, TA, TV, NTL>::dot(v + c * L, xc + c);
        }
    }
    return acc;
}

template <int EPI, typename TV>
__device__ inline void sell_epilogue(int64_t o, TV acc, TV* __restrict__ y, const TV* __restrict__ bv,
                                     TV* __restrict__ p, TV* __restrict__ xo, TV alpha, TV beta) {
    if constexpr (EPI == EPI_AX) {
        y[o] = acc;
    } else if constexpr (EPI == EPI_RES) {
        y[o] = bv[o] - acc;
    } else if constexpr (EPI == EPI_CHEB_FIRST0) {
        p[o] = acc;
        xo[o] = beta * acc;
    } else if constexpr (EPI == EPI_CHEB_FIRST) {
        p[o] = acc;
        xo[o] += beta * acc;
    } else {
        const TV pn = alpha * p[o] + acc;
        p[o] = pn;
        xo[o] += beta * pn;
    }
}

template <int BT, int V, typename TA, typename TV, int EPI, bool NTL>
__global__ __launch_bounds__(256) void k_sell_spmv(int64_t nslices, int64_t nb, int brt,
                                                   const int* __restrict__ soff, const int* __restrict__ cols,
                                                   const TA* __restrict__ vals, const TV* __restrict__ x,
                                                   TV* __restrict__ y, const TV* __restrict__ bv,
                                                   TV* __restrict__ p, TV* __restrict__ xo, TV alpha, TV beta) {
    const int b = BT ? BT : brt;
    const int S = 64 / b;
    const int L = S * b;
    const int64_t slice = xcd_slice_block((nslices + 3) / 4) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (slice >= nslices || lane >= L) return;
    const int lr = lane / b;
    const int r = lane - lr * b;
    const int64_t row = slice * S + lr;
    if (row >= nb) return;
    const TV acc = sell_lane_sum<BT, V, TA, TV, NTL, 1>(b, S, L, lane, lr, soff[slice], soff[slice + 1], cols, vals, x);
    sell_epilogue<EPI>(row * b + r, acc, y, bv, p, xo, alpha, beta);
}

// Small matrices (few slices, so too few wavefronts to cover the latency of
// their slots): one workgroup per slice, wavefront w takes the slots
// j0 + w, j0 + w + 4, ..., and the four partial sums meet in LDS.
template <int BT, int V, typename TA, typename TV, int EPI, bool NTL>
__global__ __launch_bounds__(256) void k_sell_spmv_split(int64_t nslices, int64_t nb, int brt,
                                                         const int* __restrict__ soff, const int* __restrict__ cols,
                                                         const TA* __restrict__ vals, const TV* __restrict__ x,
                                                         TV* __restrict__ y, const TV* __restrict__ bv,
                                                         TV* __restrict__ p, TV* __restrict__ xo, TV alpha, TV beta) {
    __shared__ TV part[3][64];
    const int b = BT ? BT : brt;
    const int S = 64 / b;
    const int L = S * b;
    const int64_t slice = blockIdx.x;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane / b;
    const int r = lane - lr * b;
    const int64_t row = slice * S + lr;
    const bool act = slice < nslices && lane < L && row < nb;
    TV acc = 0;
    if (act)
        acc = sell_lane_sum<BT, V, TA, TV, NTL, 4>(b, S, L, lane, lr, soff[slice] + w, soff[slice + 1], cols, vals, x);
    if (w > 0) part[w - 1][lane] = acc;
    __syncthreads();
    if (w == 0 && act) {
        acc += (part[0][lane] + part[1][lane]) + part[2][lane];
        sell_epilogue<EPI>(row * b + r, acc, y, bv, p, xo, alpha, beta);
    }
}

// Matrices with fewer slices than this use the split kernel (one workgroup per
// slice); CHF_SPMV_SPLIT_BELOW overrides it (0: never split).
static int64_t spmv_split_below() {
    const char* e = std::getenv("CHF_SPMV_SPLIT_BELOW");
    return e ? std::atoll(e) : 2048;
}

template <int BT, int V, typename TA, typename TV>
static void launch_spmv_t(const Sell& A, const void* x, void* y, const void* bv, int epi, void* p, void* xo,
                          double alpha, double beta, hipStream_t s) {
    const int64_t nblk = (A.nslices + 3) / 4;
    if (nblk == 0) return;
    const bool split = A.nslices < spmv_split_below();
    dim3 grid(split ? (unsigned)A.nslices : (unsigned)((nblk + 7) / 8 * 8)), block(256);
    auto args = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, block, 0, s, A.nslices, A.nb, A.b, A.slice_off.p, A.cols.p,
                           (const TA*)A.vals.p, (const TV*)x, (TV*)y, (const TV*)bv, (TV*)p, (TV*)xo, (TV)alpha,
                           (TV)beta);
    };
    if (split) {
        switch (epi) {
            case EPI_AX: args(k_sell_spmv_split<BT, V, TA, TV, EPI_AX, true>); break;
            case EPI_RES: args(k_sell_spmv_split<BT, V, TA, TV, EPI_RES, true>); break;
            case EPI_CHEB_FIRST0: args(k_sell_spmv_split<BT, V, TA, TV, EPI_CHEB_FIRST0, true>); break;
            case EPI_CHEB_FIRST: args(k_sell_spmv_split<BT, V, TA, TV, EPI_CHEB_FIRST, true>); break;
            default: args(k_sell_spmv_split<BT, V, TA, TV, EPI_CHEB, true>); break;
        }
        CHF_LAUNCH_CHECK();
        return;
    }
    // non-temporal matrix loads are the default (measured at 512^2, b = 10:
    // residual SpMV 78 % instead of 71 % of HBM peak); CHF_SPMV_NONTEMPORAL=0
    // turns them off
    static const bool ntl = [] {
        const char* e = std::getenv("CHF_SPMV_NONTEMPORAL");
        return !(e && e[0] == '0');
    }();
    if (ntl) {
        switch (epi) {
            case EPI_AX: args(k_sell_spmv<BT, V, TA, TV, EPI_AX, true>); break;
            case EPI_RES: args(k_sell_spmv<BT, V, TA, TV, EPI_RES, true>); break;
            case EPI_CHEB_FIRST0: args(k_sell_spmv<BT, V, TA, TV, EPI_CHEB_FIRST0, true>); break;
            case EPI_CHEB_FIRST: args(k_sell_spmv<BT, V, TA, TV, EPI_CHEB_FIRST, true>); break;
            default: args(k_sell_spmv<BT, V, TA, TV, EPI_CHEB, true>); break;
        }
    } else {
        switch (epi) {
            case EPI_AX: args(k_sell_spmv<BT, V, TA, TV, EPI_AX, false>); break;
            case EPI_RES: args(k_sell_spmv<BT, V, TA, TV, EPI_RES, false>); break;
            case EPI_CHEB_FIRST0: args(k_sell_spmv<BT, V, TA, TV, EPI_CHEB_FIRST0, false>); break;
            case EPI_CHEB_FIRST: args(k_sell_spmv<BT, V, TA, TV, EPI_CHEB_FIRST, false>); break;
            default: args(k_sell_spmv<BT, V, TA, TV, EPI_CHEB, false>); break;
        }
    }
    CHF_LAUNCH_CHECK();
}

template <typename TA, typename TV>
static void launch_spmv_b(const Sell& A, const void* x, void* y, const void* bv, int epi, void* p, void* xo,
                          double alpha, double beta, hipStream_t s) {
    CHF_CHECK(A.V == sell_vec_width(A.b, A.dtype), CHF_EDEVICE, "SpMV layout width mismatch");
    switch (A.b) {
        case 10:
            if constexpr (sizeof(TA) == 8)
                launch_spmv_t<10, 2, TA, TV>(A, x, y, bv, epi, p, xo, alpha, beta, s);
            else if constexpr (sizeof(TA) == 4)
                launch_spmv_t<10, 4, TA, TV>(A, x, y, bv, epi, p, xo, alpha, beta, s);
            else
                launch_spmv_t<10, 8, TA, TV>(A, x, y, bv, epi, p, xo, alpha, beta, s);
            break;
        case 21:
            if constexpr (sizeof(TA) == 8)
                launch_spmv_t<21, 2, TA, TV>(A, x, y, bv, epi, p, xo, alpha, beta, s);
            else if constexpr (sizeof(TA) == 4)
                launch_spmv_t<21, 4, TA, TV>(A, x, y, bv, epi, p, xo, alpha, beta, s);
            else
                launch_spmv_t<21, 8, TA, TV>(A, x, y, bv, epi, p, xo, alpha, beta, s);
            break;
        default: launch_spmv_t<0, 1, TA, TV>(A, x, y, bv, epi, p, xo, alpha, beta, s); break;
    }
}

void sell_spmv(const Sell& A, chf_dtype vec, const void* x, void* y, const void* bvec, int epi, void* p,
               void* xo, double alpha, double beta, hipStream_t s) {
    if (A.vb) {
        vsell_spmv(A, vec, x, y, bvec, epi, p, xo, alpha, beta, s);
        return;
    }
    // b = 10 kernels read x in pairs (8 bytes for FP32 vectors, 16 for FP64)
    if (A.b == 10) {
        const uintptr_t need = vec == CHF_F64 ? 16 : 8;
        CHF_CHECK((uintptr_t)x % need == 0, CHF_EINVAL, "vector not aligned to 16 bytes (FP64) or 8 bytes (FP32)");
    }
    if (A.dtype == CHF_F64) {
        CHF_CHECK(vec == CHF_F64, CHF_EINVAL, "FP64 operator needs FP64 vectors");
        launch_spmv_b<double, double>(A, x, y, bvec, epi, p, xo, alpha, beta, s);
    } else if (A.dtype == CHF_F32) {
        if (vec == CHF_F64)
            launch_spmv_b<float, double>(A, x, y, bvec, epi, p, xo, alpha, beta, s);
        else
            launch_spmv_b<float, float>(A, x, y, bvec, epi, p, xo, alpha, beta, s);
    } else {
        if (vec == CHF_F64)
            launch_spmv_b<bf16_t, double>(A, x, y, bvec, epi, p, xo, alpha, beta, s);
        else
            launch_spmv_b<bf16_t, float>(A, x, y, bvec, epi, p, xo, alpha, beta, s);
    }
}

// ------------------------------------------------------ finiteness check --
__global__ __launch_bounds__(256) void k_nonfinite_partial(const double* __restrict__ v, int64_t n,
                                                           double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        acc += isfinite(v[i]) ? 0.0 : 1.0;
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_sum_partials_ext(const double* __restrict__ part, int np, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double a = 0;
        for (int i = 0; i < np; ++i) a += part[i];
        out[0] = a;
    }
}

static int64_t count_nonfinite(const double* d, int64_t n, hipStream_t s) {
    if (n == 0) return 0;
    DevBuf<double> part(RED_BLOCKS + 1);
    hipLaunchKernelGGL(k_nonfinite_partial, dim3(RED_BLOCKS), dim3(256), 0, s, d, n, part.p);
    CHF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_partials_ext, dim3(1), dim3(64), 0, s, part.p, RED_BLOCKS, part.p + RED_BLOCKS);
    CHF_LAUNCH_CHECK();
    double h = 0;
    CHF_HIP(hipMemcpyAsync(&h, part.p + RED_BLOCKS, 8, hipMemcpyDeviceToHost, s));
    CHF_HIP(hipStreamSynchronize(s));
    return (int64_t)h;
}

}  // namespace chf

using namespace chf;

const Sell& chf_bsr_s::sell(chf_dtype t, hipStream_t s) {
    if (t == CHF_F64) return sell64;
    CHF_CHECK(!vb, CHF_EINVAL, "variable block sizes: FP64 only");
    if (sell32.nslices == 0 && nb > 0) sell_build(sell32, plan, d_vals.p, false, CHF_F32, s);
    return sell32;
}

extern "C" int chf_bsr_create(int64_t nb, int32_t b, const int64_t* rowptr, const int32_t* colidx,
                              const double* vals, int vals_on_device, chf_bsr* out) {
    return guarded([&] {
        CHF_CHECK(out, CHF_EINVAL, "out is NULL");
        *out = nullptr;
        CHF_CHECK(nb >= 0 && b >= 1 && b <= 64, CHF_EINVAL, "need nb >= 0 and 1 <= b <= 64");
        CHF_CHECK(rowptr && (nb == 0 || (colidx && vals)), CHF_EINVAL, "NULL array");
        CHF_CHECK(rowptr[0] == 0, CHF_EINVAL, "rowptr[0] must be 0");
        int64_t nnzb = rowptr[nb];
        CHF_CHECK(nnzb >= 0 && nnzb < (1ll << 31), CHF_EINVAL, "bad nnzb");
        for (int64_t i = 0; i < nb; ++i) {
            CHF_CHECK(rowptr[i + 1] >= rowptr[i], CHF_EINVAL, "rowptr not monotone");
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                CHF_CHECK(colidx[e] >= 0 && colidx[e] < nb, CHF_EINVAL, "column index out of range");
                CHF_CHECK(e == rowptr[i] || colidx[e] > colidx[e - 1], CHF_EINVAL,
                          "column indices must ascend strictly within a row");
            }
        }
        std::unique_ptr<chf_bsr_s> A(new chf_bsr_s);
        A->nb = nb;
        A->b = b;
        A->ndof = nb * (int64_t)b;
        A->nnzb = nnzb;
        A->rowptr.assign(rowptr, rowptr + nb + 1);
        A->colidx.assign(colidx, colidx + nnzb);
        std::vector<int> rp32(nb + 1);
        for (int64_t i = 0; i <= nb; ++i) rp32[i] = (int)rowptr[i];
        hipStream_t s = 0;
        A->d_rowptr.alloc(nb + 1);
        A->d_rowptr.upload(rp32.data(), nb + 1, s);
        A->d_colidx.alloc(std::max<int64_t>(1, nnzb));
        A->d_colidx.upload(colidx, nnzb, s);
        size_t nv = (size_t)nnzb * b * b;
        A->d_vals.alloc(std::max<size_t>(1, nv));
        if (nv) {
            CHF_HIP(hipMemcpyAsync(A->d_vals.p, vals, nv * 8,
                                   vals_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        }
        CHF_CHECK(count_nonfinite(A->d_vals.p, (int64_t)nv, s) == 0, CHF_EINVAL, "non-finite matrix value");
        A->plan = sell_plan(nb, b, A->rowptr, A->colidx, nullptr);
        sell_build(A->sell64, A->plan, A->d_vals.p, false, CHF_F64, s);
        CHF_HIP(hipStreamSynchronize(s));
        *out = A.release();
    });
}

extern "C" int chf_bsr_destroy(chf_bsr A) {
    return guarded([&] { delete A; });
}

extern "C" int chf_bsr_info(chf_bsr A, int64_t* nb, int32_t* b, int64_t* nnzb) {
    return guarded([&] {
        CHF_CHECK(A, CHF_EINVAL, "NULL handle");
        if (nb) *nb = A->nb;
        if (b) *b = A->b;
        if (nnzb) *nnzb = A->nnzb;
    });
}

extern "C" int chf_bsr_export(chf_bsr A, int64_t* rowptr, int32_t* colidx, double* vals) {
    return guarded([&] {
        CHF_CHECK(A, CHF_EINVAL, "NULL handle");
        if (rowptr) std::memcpy(rowptr, A->rowptr.data(), (A->nb + 1) * 8);
        if (colidx) std::memcpy(colidx, A->colidx.data(), A->nnzb * 4);
        if (vals) {
            const size_t nv = A->vb ? (size_t)A->voff[A->nnzb] : (size_t)A->nnzb * A->b * A->b;
            A->d_vals.download(vals, nv, 0);
            CHF_HIP(hipStreamSynchronize(0));
        }
    });
}

extern "C" int chf_bsr_spmv(chf_bsr A, chf_dtype dtype, const void* x, const void* bvec, void* y,
                            int residual, hipStream_t stream) {
    return guarded([&] {
        CHF_CHECK(A && x && y, CHF_EINVAL, "NULL argument");
        CHF_CHECK(!residual || bvec, CHF_EINVAL, "residual needs bvec");
        CHF_CHECK(dtype == CHF_F64 || dtype == CHF_F32, CHF_EINVAL, "vector dtype must be F64 or F32");
        CHF_CHECK(!A->vb || dtype == CHF_F64, CHF_EINVAL, "variable block sizes: FP64 only");
        const Sell& S = A->sell(dtype, stream);
        sell_spmv(S, dtype, x, y, bvec, residual ? EPI_RES : EPI_AX, nullptr, nullptr, 0, 0, stream);
    });
}
