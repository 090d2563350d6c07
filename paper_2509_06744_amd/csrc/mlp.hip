// Learned block-pattern proposer: a 6 -> 64 -> 64 -> 1 ReLU network in FP32
// with hand-written forward, backward (binary cross-entropy with logits) and
// Adam kernels, and a top-t selection that turns scores into a pattern.
//
// Parameter layout (4673 floats): W1[64][6], b1[64], W2[64][64], b2[64],
// W3[64], b3.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace chf {
constexpr int H = 64;
constexpr int NIN = MLP_NIN;
constexpr int OFF_W1 = 0, OFF_B1 = H * NIN, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H, OFF_W3 = OFF_B2 + H,
              OFF_B3 = OFF_W3 + H;
constexpr int NPARAM = OFF_B3 + 1;
static_assert(NPARAM == 4673, "parameter layout");
constexpr int TILE = 32;          // samples per tile
constexpr int MLP_NT = 256;
constexpr int MLP_OWN = (NPARAM + MLP_NT - 1) / MLP_NT;   // owned gradient entries per thread
constexpr int MLP_GRID = 512;

void a2_candidates(chf_bsr A, std::vector<int64_t>& rowptr, std::vector<int32_t>& cols);
void mlp_features_impl(chf_bsr A, int nx, int ny, const std::vector<int64_t>& crow, const std::vector<int32_t>& ccol,
                       float* feats, hipStream_t s);

// Forward pass of one tile: X -> H1 -> H2 (in LDS), returns nothing; logits
// per sample are left in `o`.
__device__ void mlp_tile_forward(const float* P, const float* __restrict__ X, const int64_t* __restrict__ perm,
                                 int64_t off, int64_t s0, int64_t n, float* Xs, float* H1, float* H2, float* o) {
    const int t = threadIdx.x;
    for (int e = t; e < TILE * NIN; e += MLP_NT) {
        int64_t s = s0 + e / NIN;
        int64_t src = perm ? perm[off + s] : off + s;
        Xs[e] = s < n ? X[src * NIN + e % NIN] : 0.0f;
    }
    __syncthreads();
    for (int e = t; e < TILE * H; e += MLP_NT) {
        int s = e / H, j = e % H;
        float a = P[OFF_B1 + j];
        for (int c = 0; c < NIN; ++c) a += P[OFF_W1 + j * NIN + c] * Xs[s * NIN + c];
        H1[e] = a > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    for (int e = t; e < TILE * H; e += MLP_NT) {
        int s = e / H, j = e % H;
        float a = P[OFF_B2 + j];
        const float* w = P + OFF_W2 + j * H;
        const float* h = H1 + s * H;
        for (int i = 0; i < H; ++i) a += w[i] * h[i];
        H2[e] = a > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    if (t < TILE) {
        float a = P[OFF_B3];
        for (int j = 0; j < H; ++j) a += P[OFF_W3 + j] * H2[t * H + j];
        o[t] = a;
    }
    __syncthreads();
}

__global__ __launch_bounds__(MLP_NT) void k_mlp_forward(const float* __restrict__ params, const float* __restrict__ X,
                                                        int64_t n, float* __restrict__ out) {
    __shared__ float P[NPARAM];
    __shared__ float Xs[TILE * NIN], H1[TILE * H], H2[TILE * H], o[TILE];
    for (int e = threadIdx.x; e < NPARAM; e += MLP_NT) P[e] = params[e];
    __syncthreads();
    for (int64_t s0 = (int64_t)blockIdx.x * TILE; s0 < n; s0 += (int64_t)gridDim.x * TILE) {
        mlp_tile_forward(P, X, nullptr, 0, s0, n, Xs, H1, H2, o);
        if (threadIdx.x < TILE && s0 + threadIdx.x < n) out[s0 + threadIdx.x] = o[threadIdx.x];
        __syncthreads();
    }
}

// Gradient of mean BCE-with-logits over n samples. Each thread owns fixed
// parameter entries (p = tid + 256 q) and accumulates their contributions
// tile by tile; per-block partial gradients are summed by k_mlp_reduce in a
// fixed order, so results are reproducible.
__global__ __launch_bounds__(MLP_NT) void k_mlp_grad(const float* __restrict__ params, const float* __restrict__ X,
                                                     const float* __restrict__ Y, const int64_t* __restrict__ perm,
                                                     int64_t off, int64_t n, float inv_n, float* __restrict__ part_g,
                                                     double* __restrict__ part_l) {
    __shared__ float P[NPARAM];
    __shared__ float Xs[TILE * NIN], H1[TILE * H], H2[TILE * H], D1[TILE * H], o[TILE], dout[TILE];
    __shared__ double lsum[TILE];
    const int t = threadIdx.x;
    for (int e = t; e < NPARAM; e += MLP_NT) P[e] = params[e];
    float acc[MLP_OWN];
#pragma unroll
    for (int q = 0; q < MLP_OWN; ++q) acc[q] = 0.0f;
    double lacc = 0.0;
    __syncthreads();
    for (int64_t s0 = (int64_t)blockIdx.x * TILE; s0 < n; s0 += (int64_t)gridDim.x * TILE) {
        mlp_tile_forward(P, X, perm, off, s0, n, Xs, H1, H2, o);
        if (t < TILE) {
            const int64_t s = s0 + t;
            float d = 0.0f;
            if (s < n) {
                const float z = o[t], y = Y[perm ? perm[off + s] : off + s];
                lacc += (double)(fmaxf(z, 0.0f) - z * y + log1pf(expf(-fabsf(z))));
                const float sig = 1.0f / (1.0f + expf(-z));
                d = (sig - y) * inv_n;
            }
            dout[t] = d;
        }
        __syncthreads();
        // gradients that need H2 before it becomes D2: W3, b3
#pragma unroll
        for (int q = 0; q < MLP_OWN; ++q) {
            const int p = t + MLP_NT * q;
            if (p >= OFF_W3 && p < NPARAM) {
                float g = 0.0f;
                if (p == OFF_B3) {
                    for (int s = 0; s < TILE; ++s) g += dout[s];
                } else {
                    const int j = p - OFF_W3;
                    for (int s = 0; s < TILE; ++s) g += dout[s] * H2[s * H + j];
                }
                acc[q] += g;
            }
        }
        __syncthreads();
        // D2 = dout W3 * [H2 > 0], stored over H2
        for (int e = t; e < TILE * H; e += MLP_NT) {
            int s = e / H, j = e % H;
            H2[e] = H2[e] > 0.0f ? dout[s] * P[OFF_W3 + j] : 0.0f;
        }
        __syncthreads();
        // D1 = (D2 W2) * [H1 > 0]
        for (int e = t; e < TILE * H; e += MLP_NT) {
            int s = e / H, j = e % H;
            float a = 0.0f;
            if (H1[e] > 0.0f)
                for (int i = 0; i < H; ++i) a += H2[s * H + i] * P[OFF_W2 + i * H + j];
            D1[e] = a;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < MLP_OWN; ++q) {
            const int p = t + MLP_NT * q;
            float g = 0.0f;
            if (p < OFF_B1) {                       // W1[j][c]
                const int j = p / NIN, c = p % NIN;
                for (int s = 0; s < TILE; ++s) g += D1[s * H + j] * Xs[s * NIN + c];
            } else if (p < OFF_W2) {                // b1[j]
                const int j = p - OFF_B1;
                for (int s = 0; s < TILE; ++s) g += D1[s * H + j];
            } else if (p < OFF_B2) {                // W2[i][j]
                const int i = (p - OFF_W2) / H, j = (p - OFF_W2) % H;
                for (int s = 0; s < TILE; ++s) g += H2[s * H + i] * H1[s * H + j];
            } else if (p < OFF_W3) {                // b2[i]
                const int i = p - OFF_B2;
                for (int s = 0; s < TILE; ++s) g += H2[s * H + i];
            }
            if (p < OFF_W3) acc[q] += g;
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < MLP_OWN; ++q) {
        const int p = t + MLP_NT * q;
        if (p < NPARAM) part_g[(int64_t)blockIdx.x * NPARAM + p] = acc[q];
    }
    if (t < TILE) lsum[t] = lacc;
    __syncthreads();
    if (t == 0) {
        double l = 0.0;
        for (int s = 0; s < TILE; ++s) l += lsum[s];
        part_l[blockIdx.x] = l;
    }
}

__global__ void k_mlp_reduce(const float* __restrict__ part_g, const double* __restrict__ part_l, int nblk,
                             double inv_n, float* __restrict__ grad, double* __restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NPARAM) {
        float g = 0.0f;
        for (int k = 0; k < nblk; ++k) g += part_g[(int64_t)k * NPARAM + p];
        grad[p] = g;
    }
    if (p == 0) {
        double l = 0.0;
        for (int k = 0; k < nblk; ++k) l += part_l[k];
        loss[0] = l * inv_n;
    }
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float bc1, float bc2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.0f - b1) * gi;
    const float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    w[p] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// top-t candidates per row by score (ties to the smaller column), plus k
__global__ void k_topk(int64_t nb, int t, const int64_t* __restrict__ crow, const int* __restrict__ ccol,
                       const float* __restrict__ score, int* __restrict__ out_cols, int* __restrict__ out_cnt) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nb) return;
    const int64_t c0 = crow[k], c1 = crow[k + 1];
    int* out = out_cols + k * (t + 1);
    int cnt = 0;
    for (int r = 0; r < t; ++r) {
        int64_t best = -1;
        for (int64_t e = c0; e < c1; ++e) {
            bool taken = false;
            for (int q = 0; q < cnt; ++q) taken |= out[q] == ccol[e];
            if (taken) continue;
            if (best < 0 || score[e] > score[best] || (score[e] == score[best] && ccol[e] < ccol[best])) best = e;
        }
        if (best < 0) break;
        out[cnt++] = ccol[best];
    }
    out[cnt++] = (int)k;
    for (int i = 1; i < cnt; ++i) {
        int v = out[i], j = i - 1;
        while (j >= 0 && out[j] > v) { out[j + 1] = out[j]; --j; }
        out[j + 1] = v;
    }
    out_cnt[k] = cnt;
}

}  // namespace chf

using namespace chf;

struct chf_mlp_s {
    DevBuf<float> w, m, v, g, part_g;
    DevBuf<double> part_l;
    int64_t step = 0;
};

static void adam_step(chf_mlp_s& net, float lr, float beta1, float beta2, float eps, hipStream_t stream);

static void mlp_grad_impl(chf_mlp_s& net, const float* feats, const float* labels, int64_t n, float* grad_out,
                          double* loss_host, hipStream_t s, const int64_t* perm = nullptr, int64_t off = 0) {
    CHF_CHECK(n >= 1, CHF_EINVAL, "need at least one sample");
    const int64_t tiles = (n + TILE - 1) / TILE;
    const int grid = (int)std::min<int64_t>(MLP_GRID, tiles);
    hipLaunchKernelGGL(k_mlp_grad, dim3(grid), dim3(MLP_NT), 0, s, net.w.p, feats, labels, perm, off, n,
                       (float)(1.0 / n), net.part_g.p, net.part_l.p);
    CHF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NPARAM + 255) / 256), dim3(256), 0, s, net.part_g.p, net.part_l.p, grid,
                       1.0 / n, grad_out, net.part_l.p + MLP_GRID);
    CHF_LAUNCH_CHECK();
    if (loss_host) {
        CHF_HIP(hipMemcpyAsync(loss_host, net.part_l.p + MLP_GRID, 8, hipMemcpyDeviceToHost, s));
        CHF_HIP(hipStreamSynchronize(s));
    }
}

extern "C" int chf_mlp_create(const float* params_host, chf_mlp* out) {
    return guarded([&] {
        CHF_CHECK(params_host && out, CHF_EINVAL, "NULL argument");
        for (int i = 0; i < NPARAM; ++i) CHF_CHECK(std::isfinite(params_host[i]), CHF_EINVAL, "non-finite parameter");
        std::unique_ptr<chf_mlp_s> net(new chf_mlp_s);
        net->w.alloc(NPARAM);
        net->m.alloc(NPARAM);
        net->v.alloc(NPARAM);
        net->g.alloc(NPARAM);
        net->part_g.alloc((size_t)MLP_GRID * NPARAM);
        net->part_l.alloc(MLP_GRID + 1);
        net->w.upload(params_host, NPARAM, 0);
        fill_zero(net->m.p, NPARAM * 4, 0);
        fill_zero(net->v.p, NPARAM * 4, 0);
        CHF_HIP(hipStreamSynchronize(0));
        *out = net.release();
    });
}

extern "C" int chf_mlp_destroy(chf_mlp net) {
    return guarded([&] { delete net; });
}

extern "C" int chf_mlp_get_params(chf_mlp net, float* params_host) {
    return guarded([&] {
        CHF_CHECK(net && params_host, CHF_EINVAL, "NULL argument");
        net->w.download(params_host, NPARAM, 0);
        CHF_HIP(hipStreamSynchronize(0));
    });
}

extern "C" int chf_mlp_forward(chf_mlp net, const float* feats, int64_t n, float* logits, hipStream_t stream) {
    return guarded([&] {
        CHF_CHECK(net && feats && logits && n >= 0, CHF_EINVAL, "bad argument");
        if (n == 0) return;
        const int grid = (int)std::min<int64_t>(4096, (n + TILE - 1) / TILE);
        hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(MLP_NT), 0, stream, net->w.p, feats, n, logits);
        CHF_LAUNCH_CHECK();
    });
}

extern "C" int chf_mlp_loss_grad(chf_mlp net, const float* feats, const float* labels, int64_t n, float* loss_host,
                                 float* grad, hipStream_t stream) {
    return guarded([&] {
        CHF_CHECK(net && feats && labels && grad, CHF_EINVAL, "NULL argument");
        double l = 0.0;
        mlp_grad_impl(*net, feats, labels, n, grad, &l, stream);
        if (loss_host) *loss_host = (float)l;
    });
}

extern "C" int chf_mlp_train_step(chf_mlp net, const float* feats, const float* labels, int64_t n, float lr,
                                  float beta1, float beta2, float eps, float* loss_host, hipStream_t stream) {
    return guarded([&] {
        CHF_CHECK(net && feats && labels, CHF_EINVAL, "NULL argument");
        CHF_CHECK(lr > 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0, CHF_EINVAL,
                  "bad optimiser parameters");
        double l = 0.0;
        mlp_grad_impl(*net, feats, labels, n, net->g.p, loss_host ? &l : nullptr, stream);
        adam_step(*net, lr, beta1, beta2, eps, stream);
        if (loss_host) *loss_host = (float)l;
    });
}

static void adam_step(chf_mlp_s& net, float lr, float beta1, float beta2, float eps, hipStream_t stream) {
    net.step += 1;
    const float bc1 = 1.0f - std::pow(beta1, (float)net.step);
    const float bc2 = 1.0f - std::pow(beta2, (float)net.step);
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, stream, net.w.p, (const float*)net.g.p,
                       net.m.p, net.v.p, lr, beta1, beta2, eps, bc1, bc2);
    CHF_LAUNCH_CHECK();
}

extern "C" int chf_mlp_train(chf_mlp net, const float* feats, const float* labels, int64_t n, const int64_t* perm,
                             int64_t batch, int epochs, float lr, float beta1, float beta2, float eps,
                             float* loss_hist, hipStream_t stream) {
    return guarded([&] {
        CHF_CHECK(net && feats && labels && n >= 1 && batch >= 1 && epochs >= 0, CHF_EINVAL, "bad argument");
        CHF_CHECK(lr > 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0, CHF_EINVAL,
                  "bad optimiser parameters");
        for (int ep = 0; ep < epochs; ++ep) {
            double lsum = 0.0;
            int64_t seen = 0;
            for (int64_t off = 0; off < n; off += batch) {
                const int64_t nb = std::min(batch, n - off);
                double l = 0.0;
                const bool want = loss_hist != nullptr;
                mlp_grad_impl(*net, feats, labels, nb, net->g.p, want ? &l : nullptr, stream, perm, off);
                adam_step(*net, lr, beta1, beta2, eps, stream);
                lsum += l * nb;
                seen += nb;
            }
            if (loss_hist) loss_hist[ep] = (float)(lsum / seen);
        }
        CHF_HIP(hipStreamSynchronize(stream));
    });
}

extern "C" int chf_mlp_labels(chf_bsr A, chf_pattern P, float* labels, hipStream_t stream) {
    return guarded([&] {
        CHF_CHECK(A && P && labels, CHF_EINVAL, "NULL argument");
        CHF_CHECK(P->nb == A->nb, CHF_EINVAL, "pattern and matrix sizes differ");
        std::vector<int64_t> crow;
        std::vector<int32_t> ccol;
        a2_candidates(A, crow, ccol);
        std::vector<float> h(ccol.size(), 0.0f);
        for (int64_t k = 0; k < A->nb; ++k) {
            const int32_t* pb = P->colidx.data() + P->rowptr[k];
            const int32_t* pe = P->colidx.data() + P->rowptr[k + 1];
            for (int64_t e = crow[k]; e < crow[k + 1]; ++e) h[e] = std::binary_search(pb, pe, ccol[e]) ? 1.0f : 0.0f;
        }
        if (!h.empty()) {
            CHF_HIP(hipMemcpyAsync(labels, h.data(), h.size() * 4, hipMemcpyHostToDevice, stream));
            CHF_HIP(hipStreamSynchronize(stream));
        }
    });
}

extern "C" int chf_mlp_propose(chf_bsr A, chf_mlp net, int32_t nx, int32_t ny, int t, chf_pattern* out) {
    return guarded([&] {
        CHF_CHECK(A && net && out, CHF_EINVAL, "NULL argument");
        CHF_CHECK(t >= 0 && t < 32, CHF_EINVAL, "t must be in [0, 31]");
        CHF_CHECK(nx >= 1 && ny >= 1 && A->nb % ((int64_t)nx * ny) == 0, CHF_EINVAL, "grid does not match nb");
        hipStream_t s = 0;
        const int64_t nb = A->nb;
        std::vector<int64_t> crow;
        std::vector<int32_t> ccol;
        a2_candidates(A, crow, ccol);
        const int64_t nc = (int64_t)ccol.size();
        DevBuf<float> feats(std::max<int64_t>(1, nc * NIN)), score(std::max<int64_t>(1, nc));
        mlp_features_impl(A, nx, ny, crow, ccol, feats.p, s);
        if (nc > 0) {
            const int grid = (int)std::min<int64_t>(4096, (nc + TILE - 1) / TILE);
            hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(MLP_NT), 0, s, net->w.p, feats.p, nc, score.p);
            CHF_LAUNCH_CHECK();
        }
        DevBuf<int64_t> d_crow(nb + 1);
        DevBuf<int> d_ccol(std::max<int64_t>(1, nc)), d_out((size_t)std::max<int64_t>(1, nb) * (t + 1)),
            d_cnt(std::max<int64_t>(1, nb));
        d_crow.upload(crow.data(), nb + 1, s);
        d_ccol.upload(ccol.data(), nc, s);
        std::unique_ptr<chf_pattern_s> P(new chf_pattern_s);
        P->nb = nb;
        P->rowptr.assign(nb + 1, 0);
        if (nb > 0) {
            hipLaunchKernelGGL(k_topk, dim3((unsigned)((nb + 127) / 128)), dim3(128), 0, s, nb, t, d_crow.p, d_ccol.p,
                               score.p, d_out.p, d_cnt.p);
            CHF_LAUNCH_CHECK();
            std::vector<int> hout((size_t)nb * (t + 1)), hcnt(nb);
            d_out.download(hout.data(), hout.size(), s);
            d_cnt.download(hcnt.data(), nb, s);
            CHF_HIP(hipStreamSynchronize(s));
            for (int64_t k = 0; k < nb; ++k) {
                for (int i = 0; i < hcnt[k]; ++i) P->colidx.push_back(hout[(size_t)k * (t + 1) + i]);
                P->rowptr[k + 1] = (int64_t)P->colidx.size();
            }
        }
        *out = P.release();
    });
}
