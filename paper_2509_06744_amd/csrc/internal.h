// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "chf.h"

namespace chf {

// ---------------------------------------------------------------- errors --
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_error(const std::string& msg);
[[noreturn]] void fail(int code, const std::string& msg);

#define CHF_HIP(call)                                                            \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess)                                                    \
            ::chf::fail(e_ == hipErrorOutOfMemory ? CHF_ENOMEM : CHF_EDEVICE,    \
                        std::string(#call) + ": " + hipGetErrorString(e_));      \
    } while (0)

#define CHF_CHECK(cond, code, msg)                                               \
    do {                                                                         \
        if (!(cond)) ::chf::fail((code), (msg));                                 \
    } while (0)

#define CHF_LAUNCH_CHECK() CHF_HIP(hipGetLastError())

// C-ABI wrapper: runs f, maps exceptions to status codes.
template <class F>
int guarded(F&& f) {
    try {
        f();
        return CHF_OK;
    } catch (const Error& e) {
        set_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return CHF_ENOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return CHF_EDEVICE;
    }
}

// ------------------------------------------------------------ device mem --
// Frees device memory, or, while the calling thread has a deferral list set,
// records the pointer for the caller to free later. hipFree synchronises the
// whole device, so a free would serialise work overlapped on two streams.
void dev_free(void* p);
void set_free_deferral(std::vector<void*>* list);   // nullptr: free at once

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        n = count;
        if (count) CHF_HIP(hipMalloc(&p, count * sizeof(T)));
    }
    void release() {
        if (p) dev_free(p);
        p = nullptr;
        n = 0;
    }
    void upload(const T* h, size_t count, hipStream_t s = 0) {
        if (count) CHF_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
    }
    void download(T* h, size_t count, hipStream_t s = 0) const {
        if (count) CHF_HIP(hipMemcpyAsync(h, p, count * sizeof(T), hipMemcpyDeviceToHost, s));
    }
};

size_t dtype_size(chf_dtype t);      // storage element size
size_t vec_size(chf_dtype t);        // vector element size (double or float)

// ------------------------------------------------------------- SELL layout --
// Slice-interleaved block-ELL: a slice holds S = 64 / b consecutive block
// rows, so one 64-wide wavefront owns L = S * b output scalars (lane =
// local_row * b + r). Slot j of slice s stores, for every lane, the b entries
// of row r of that lane's j-th block in runs of consecutive columns: run q
// covers columns c0_q .. c0_q + w_q - 1 and is stored as L groups of w_q values,
//   vals[(slot_base + j) * stride + L * c0_q + lane * w_q + v]
//       = block(row, j)[r][c0_q + v].
// One load instruction therefore reads L * w_q contiguous values (16 bytes per
// lane for FP64 with w_q = 2). The run widths depend on b and the storage
// dtype (sell_build); slots are padded to 16 bytes when runs are wider than 1. Column indices are cols[(slot_base + j) * S +
// local_row]; padding slots point at the row's own block with zero values.
struct VSellLayout;   // variable block sizes (vbsr.hip)

struct Sell {
    int64_t nb = 0;
    int64_t ndof = 0;         // rows of the matrix in unknowns (nb * b for uniform blocks)
    int b = 0, S = 0, L = 0;
    int V = 1;                // layout id: widest run of consecutive columns per lane load (see sell_build)
    int stride = 0;           // elements per slot: b * L, padded to 16 bytes for the run layouts
    int64_t nslices = 0, nslots = 0;
    chf_dtype dtype = CHF_F64;
    DevBuf<int> slice_off;    // nslices + 1 (slots)
    DevBuf<int> cols;         // nslots * S
    DevBuf<char> vals;        // nslots * b * L elements of dtype
    std::shared_ptr<VSellLayout> vb;   // set for variable block sizes (then the fields above are unused)
};

// Host description of a block-sparse structure with a map from each stored
// block to a source block (index into a flat array of b*b blocks) and a flag
// telling whether the source block is stored transposed.
struct SellPlan {
    int64_t nb = 0;
    int b = 0, S = 0, L = 0;
    int64_t nslices = 0, nslots = 0;
    std::vector<int> slice_off;   // nslices+1
    std::vector<int> cols;        // nslots*S
    std::vector<int64_t> src;     // nslots*S, -1 for padding
};

SellPlan sell_plan(int64_t nb, int b, const std::vector<int64_t>& rowptr,
                   const std::vector<int32_t>& colidx, const std::vector<int64_t>* srcmap);
// Build a device SELL matrix in `dtype` from FP64 source blocks (device).
void sell_build(Sell& out, const SellPlan& plan, const double* d_src_blocks, bool transpose,
                chf_dtype dtype, hipStream_t s);

// y = A x, y = bvec - A x, or fused Chebyshev updates (see spmv.hip).
enum Epi { EPI_AX = 0, EPI_RES = 1, EPI_CHEB_FIRST0 = 2, EPI_CHEB_FIRST = 3, EPI_CHEB = 4 };
// vec: working vector dtype (CHF_F64 -> double, else float); the matrix is
// read in its own storage dtype and accumulated in the vector's precision.
void sell_spmv(const Sell& A, chf_dtype vec, const void* x, void* y, const void* bvec, int epi,
               void* p, void* xo, double alpha, double beta, hipStream_t s);
// The same for the variable-block layout (vbsr.hip; FP64 only).
void vsell_spmv(const Sell& A, chf_dtype vec, const void* x, void* y, const void* bvec, int epi,
                void* p, void* xo, double alpha, double beta, hipStream_t s);

// ------------------------------------------------------------------ handles --
}  // namespace chf

struct chf_bsr_s {
    int64_t nb = 0, nnzb = 0;
    int b = 0;                          // block size (the largest one with variable blocks)
    int64_t ndof = 0;                   // unknowns: nb * b, or the sum of the block sizes
    // variable block sizes (chf_vbsr_create): block e = (i, j) is the
    // bsize[i] x bsize[j] array at d_vals + voff[e]; unknowns of block row i
    // start at boff[i]
    bool vb = false;
    std::vector<int32_t> bsize;
    std::vector<int64_t> boff, voff;
    chf::DevBuf<int64_t> d_voff;        // device copies (variable block sizes only)
    chf::DevBuf<int> d_bsize;
    std::vector<int64_t> rowptr;        // host structure
    std::vector<int32_t> colidx;
    chf::DevBuf<int> d_rowptr;          // device plain BSR (FP64) for set-up kernels
    chf::DevBuf<int> d_colidx;
    chf::DevBuf<double> d_vals;
    chf::SellPlan plan;
    chf::Sell sell64;                   // SpMV layouts, built on demand
    chf::Sell sell32;
    const chf::Sell& sell(chf_dtype t, hipStream_t s);
};

struct chf_pattern_s {
    int64_t nb = 0;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> colidx;
};

struct chf_fsai_s {
    int64_t nb = 0, nnz = 0;
    int b = 0;
    // variable block sizes: G's block e = (k, j) is bsize[k] x bsize[j] at
    // d_vals + voff[e] (uniform blocks: voff empty, e * b * b)
    bool vb = false;
    std::vector<int32_t> bsize;
    std::vector<int64_t> voff;
    chf_dtype store = CHF_F64;
    std::vector<int64_t> rowptr;        // pattern (lower)
    std::vector<int32_t> colidx;
    chf::DevBuf<double> d_vals;         // FP64 blocks in pattern order
    chf::SellPlan plan_g, plan_gt;
    chf::Sell g64, gt64;                // FP64 copies (Lanczos, F64 smoother)
    chf::Sell g_lo, gt_lo;              // rounded copies (F32 / BF16) for mixed
    const chf::Sell& g(chf_dtype t) const { return t == CHF_F64 ? g64 : g_lo; }
    const chf::Sell& gt(chf_dtype t) const { return t == CHF_F64 ? gt64 : gt_lo; }
    // nested factor (one level, Sec. 2.2): M = G0^T G1^T G1 G0 with G0 = outer,
    // G1 = inner, both borrowed; a plain factor has neither
    const chf_fsai_s* nest_outer = nullptr;
    const chf_fsai_s* nest_inner = nullptr;
    const chf_fsai_s& base() const { return nest_outer ? *nest_outer : *this; }
};

namespace chf {
// The SpMV layouts of a factor in storage dtype t: g/gt the factor (the
// outer one of a nested factor) and gi/git the inner one (null if plain).
struct FactorOps {
    const Sell* g;
    const Sell* gt;
    const Sell* gi;
    const Sell* git;
};
inline FactorOps factor_ops(const chf_fsai_s& G, chf_dtype t) {
    const chf_fsai_s& o = G.base();
    FactorOps f{&o.g(t), &o.gt(t), nullptr, nullptr};
    if (G.nest_inner) {
        f.gi = &G.nest_inner->g(t);
        f.git = &G.nest_inner->gt(t);
    }
    return f;
}
// Inputs per candidate of the learned pattern proposer (features of
// chf_mlp_features).
constexpr int MLP_NIN = 6;
// Block-FSAI factor of a variable-block matrix (vbsr.hip).
chf_fsai_s* vfsai_setup_impl(chf_bsr A, const chf_pattern_s& P, int64_t* bad_row, hipStream_t s);
// Working mode -> (vector dtype, storage dtype of the factor's layouts used).
inline chf_dtype mode_vec(chf_dtype mode) { return (mode == CHF_F64 || mode == CHF_F64_BF16G) ? CHF_F64 : CHF_F32; }
inline chf_dtype mode_g(chf_dtype mode) { return mode == CHF_F64_BF16G ? CHF_BF16 : mode; }
// Deterministic FP64 reductions (fixed grid, fixed tree).
constexpr int RED_BLOCKS = 512;
// out[0] = sum x_i y_i over n doubles/floats (vec dtype), accumulated in FP64.
void dot(chf_dtype vec, const void* x, const void* y, int64_t n, double* d_out, double* d_partials,
         hipStream_t s);
// Bisection for the largest eigenvalue of a symmetric tridiagonal matrix.
double tridiag_max_eig(const std::vector<double>& alpha, const std::vector<double>& beta);
// Elementwise helpers.
void cast_vec(chf_dtype from, const void* x, chf_dtype to, void* y, int64_t n, hipStream_t s);
void fill_zero(void* p, size_t bytes, hipStream_t s);
int device_cu_count();
}  // namespace chf
