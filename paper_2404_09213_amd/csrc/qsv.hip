// qsv.hip -- gfx950 kernels and the C ABI of libqsv.
//
// Kernels (all float32 amplitude arithmetic, float64 reductions):
//   k_coef          gate-matrix cache evaluation: C + cos(t/2) A + sin(t/2) S per
//                   gate (Eq. (1) generalised), products of fused chains, daggers
//   k_init          product-state init from the leading 1-qubit gates (embedding),
//                   for the per-gate method (the fused passes build it in their
//                   first pass instead)
//   k_pg_apply      plain method: one strided sweep of the state per gate
//   k_pg_adj        plain method, backward: gradient partial + uncompute psi, lambda
//   k_pg_apply_vec / k_pg_adj_vec   the same with 16-byte streaming accesses (complex64)
//   k_adj_init      plain method: lambda = (sum_i g_i Z_i) psi_N
//   k_pass_fwd      fused pass: tile of 2^m amplitudes, register stages, LDS re-layout
//   k_pass_bwd      fused pass, backward: same tiles for psi and lambda + gradients
//   k_expval_part / k_expval_final   <Z_i> readout, two deterministic stages
//   k_grad_reduce   gradient partials -> weight (batch-summed) and input gradients
//   k_multi_fwd / k_multi_bwd, k_init_multi, k_expval_part_multi / k_expval_final_multi
//                   many circuits in one plan: fused passes as one launch per round
//                   (k_init_multi only when some circuit has no forward pass)
//   k_pass_copy     measurement aid: a generated pass's loads and stores alone
// The fused passes of single-circuit plans normally run as kernels generated
// for the plan (jit.cpp); k_pass_fwd / k_pass_bwd interpret the same tables.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <unordered_set>

#include "jit.hpp"
#include "plan.hpp"

using namespace qsv;

// ----------------------------------------------------------------------------
// error state
// ----------------------------------------------------------------------------
static thread_local std::string g_last_error;
static thread_local bool g_capturing = false;  // inside qsv_graph_create: no profiling events
static thread_local bool g_noalloc = false;    // inside qsv_forward_expval_noalloc: nothing may be created

namespace qsv {
void set_error(const std::string& msg) { g_last_error = msg; }
}

// A roctx range around one library call (planning, forward, readout,
// backward, graph capture and replay), shown by rocprofv3 --marker-trace.
// None inside the allocation-free call, which must not call into a tool.
struct TraceRange {
    bool on;
    explicit TraceRange(const char* name) : on(!g_noalloc) { if (on) roctxRangePushA(name); }
    ~TraceRange() { if (on) roctxRangePop(); }
};

#define HIP_TRY(expr)                                                            \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess) {                                                  \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));        \
            return QSV_ERR_HIP;                                                  \
        }                                                                        \
    } while (0)

// ----------------------------------------------------------------------------
// device helpers
// ----------------------------------------------------------------------------
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Amplitude types: complex64 (float2, the default) or complex128 (double2,
// the plain method's amp_dtype option); Real<V> is the component type.
template <class V> struct RealOf;
template <> struct RealOf<float2> { using T = float; };
template <> struct RealOf<double2> { using T = double; };
template <class V> using Real = typename RealOf<V>::T;
template <class V> struct CplxOf;
template <> struct CplxOf<float> { using T = float2; };
template <> struct CplxOf<double> { using T = double2; };
template <class R> using Cplx = typename CplxOf<R>::T;

__device__ __forceinline__ float2 mkc(float re, float im) { return make_float2(re, im); }
__device__ __forceinline__ double2 mkc(double re, double im) { return make_double2(re, im); }

template <class V> struct M2T { V m00, m01, m10, m11; };
using M2 = M2T<float2>;

template <class R>
__device__ __forceinline__ const R* mat_ptr(const R* mats, int32_t slot, int b, int n_shared, int n_ps) {
    return slot >= 0 ? mats + 8 * (size_t)slot
                     : mats + 8 * ((size_t)n_shared + (size_t)b * n_ps + (size_t)(-slot - 1));
}

template <class R>
__device__ __forceinline__ M2T<Cplx<R>> load_m2(const R* p) {
    M2T<Cplx<R>> m;
    m.m00 = mkc(p[0], p[1]);
    m.m01 = mkc(p[2], p[3]);
    m.m10 = mkc(p[4], p[5]);
    m.m11 = mkc(p[6], p[7]);
    return m;
}

// Two adjacent amplitudes (index i, i + 1; i even) as one streaming access:
// 16 bytes for complex64, two 16-byte accesses for complex128. `vec` false
// (an array that is only 8-byte aligned) falls back to one access each.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void load_pair(const float2* p, bool vec, float2& a, float2& b) {
    if (vec) {
        const f4v v = __builtin_nontemporal_load((const f4v*)p);
        a = make_float2(v.x, v.y);
        b = make_float2(v.z, v.w);
    } else {
        a = p[0];
        b = p[1];
    }
}
__device__ __forceinline__ void load_pair(const double2* p, bool vec, double2& a, double2& b) {
    const d2v u = __builtin_nontemporal_load((const d2v*)p), v = __builtin_nontemporal_load((const d2v*)p + 1);
    a = make_double2(u.x, u.y);
    b = make_double2(v.x, v.y);
    (void)vec;  // double2 arrays are 16-byte aligned
}
__device__ __forceinline__ void store_pair(float2* p, bool vec, float2 a, float2 b) {
    if (vec) {
        __builtin_nontemporal_store(f4v{a.x, a.y, b.x, b.y}, (f4v*)p);
    } else {
        p[0] = a;
        p[1] = b;
    }
}
__device__ __forceinline__ void store_pair(double2* p, bool vec, double2 a, double2 b) {
    __builtin_nontemporal_store(d2v{a.x, a.y}, (d2v*)p);
    __builtin_nontemporal_store(d2v{b.x, b.y}, (d2v*)p + 1);
    (void)vec;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// float32 sum over the 16 lanes of a DPP row (pairs, quads, half rows, rows);
// every lane of the row ends with the row's total. Fixed order.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float row_sum(float v) {
    v += dpp_f<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f<0x141>(v);  // row_half_mirror
    v += dpp_f<0x140>(v);  // row_mirror
    return v;
}

__device__ __forceinline__ float im_conj_mul(float2 l, float2 p) { return l.x * p.y - l.y * p.x; }
__device__ __forceinline__ float re_conj_mul(float2 l, float2 p) { return l.x * p.x + l.y * p.y; }
__device__ __forceinline__ double im_conj_mul(double2 l, double2 p) { return l.x * p.y - l.y * p.x; }
__device__ __forceinline__ double re_conj_mul(double2 l, double2 p) { return l.x * p.x + l.y * p.y; }

// Bank-conflict swizzle of a tile-local amplitude index (bijection on [0, 2^m)).
__device__ __forceinline__ int swz(int l) { return l ^ (((l >> 5) ^ (l >> 10)) & 31); }

__device__ __forceinline__ int64_t insert_bit(int64_t x, int s, int v) {
    const int64_t lo = x & ((int64_t(1) << s) - 1);
    return ((x >> s) << (s + 1)) | (int64_t(v) << s) | lo;
}

// ----------------------------------------------------------------------------
// gate-matrix cache evaluation
// ----------------------------------------------------------------------------
template <class R>  // R: matrix entry type (float, or double for complex128 states)
__global__ void k_coef(const DGate* __restrict__ gates, const DRecipe* __restrict__ recipes,
                       const int32_t* __restrict__ rg, int n_recipes,
                       const float* __restrict__ weights, const float* __restrict__ inputs,
                       int n_inputs, int n_shared, int n_ps, int remap, R* __restrict__ mats) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (r >= n_recipes) return;
    const DRecipe Rc = recipes[r];
    if (Rc.out >= 0 && b != 0) return;
    double M[8] = {1, 0, 0, 0, 0, 0, 1, 0};
    for (int i = 0; i < Rc.count; ++i) {
        const DGate& G = gates[rg[Rc.first + i]];
        double th = 0.0;
        if (G.src == QSV_SRC_WEIGHT) {
            th = (double)weights[G.idx];
            if (remap) th = M_PI * tanh(th);  // weight remapping into (-pi, pi)
        }
        else if (G.src == QSV_SRC_INPUT) th = (double)inputs[(size_t)b * n_inputs + G.idx];
        double s, c;
        sincos(0.5 * th, &s, &c);
        double g[8];
        for (int e = 0; e < 8; ++e) g[e] = G.C[e] + c * G.A[e] + s * G.S[e];
        // M <- g * M (later gates act on the left)
        double N[8];
        for (int row = 0; row < 2; ++row)
            for (int col = 0; col < 2; ++col) {
                double re = 0, im = 0;
                for (int k = 0; k < 2; ++k) {
                    const double ar = g[(row * 2 + k) * 2], ai = g[(row * 2 + k) * 2 + 1];
                    const double br = M[(k * 2 + col) * 2], bi = M[(k * 2 + col) * 2 + 1];
                    re += ar * br - ai * bi;
                    im += ar * bi + ai * br;
                }
                N[(row * 2 + col) * 2] = re;
                N[(row * 2 + col) * 2 + 1] = im;
            }
        for (int e = 0; e < 8; ++e) M[e] = N[e];
    }
    R out[8];
    if (Rc.dagger) {
        out[0] = (R)M[0]; out[1] = (R)-M[1];  // m00*
        out[2] = (R)M[4]; out[3] = (R)-M[5];  // m10*
        out[4] = (R)M[2]; out[5] = (R)-M[3];  // m01*
        out[6] = (R)M[6]; out[7] = (R)-M[7];  // m11*
    } else {
        for (int e = 0; e < 8; ++e) out[e] = (R)M[e];
    }
    R* dst = Rc.out >= 0 ? mats + 8 * (size_t)Rc.out
                         : mats + 8 * ((size_t)n_shared + (size_t)b * n_ps + (size_t)(-Rc.out - 1));
    for (int e = 0; e < 8; ++e) dst[e] = out[e];
}

// ----------------------------------------------------------------------------
// product-state init: amp(idx) = prod_q v_q[bit_q(idx)], v_q = column 0 of the
// prefix matrix of qubit q. One block per chunk of 2^cb amplitudes (cb =
// min(W, 12)) and sample: the block first tabulates, in LDS, the products
// over the chunk's low h bits (lo, 2^h entries) and over its other cb - h
// bits times the chunk's constant factor from the bits above cb (hi), so
// every amplitude is one complex product lo[.] hi[.], written as 16-byte
// streaming pairs.
// ----------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ Cplx<R> prefix_v(const R* mats, const int32_t* pm, int q, int bit,
                                            int b, int n_shared, int n_ps) {
    const R* M = mat_ptr(mats, pm[q], b, n_shared, n_ps);
    return bit ? mkc(M[4], M[5]) : mkc(M[0], M[1]);
}

template <class V>
__global__ __launch_bounds__(256) void k_init(V* __restrict__ state, int W,
                                              const int32_t* __restrict__ pm,
                                              const Real<V>* __restrict__ mats, int n_shared,
                                              int n_ps, int vec) {
    __shared__ V lo[64], hi[64];
    const int cb = min(W, 12), h = cb / 2, hb = cb - h;
    const int t = threadIdx.x;
    const int b = blockIdx.y;
    const int64_t chunk = blockIdx.x;
    if (t < (1 << h)) {
        V P = mkc(Real<V>(1), Real<V>(0));
        for (int s = 0; s < h; ++s) P = cmul(P, prefix_v(mats, pm, W - 1 - s, (t >> s) & 1, b, n_shared, n_ps));
        lo[t] = P;
    } else if (t >= 64 && t < 64 + (1 << hb)) {
        const int k = t - 64;
        V P = mkc(Real<V>(1), Real<V>(0));
        for (int s = h; s < cb; ++s)
            P = cmul(P, prefix_v(mats, pm, W - 1 - s, (k >> (s - h)) & 1, b, n_shared, n_ps));
        for (int s = cb; s < W; ++s)
            P = cmul(P, prefix_v(mats, pm, W - 1 - s, (int)((chunk >> (s - cb)) & 1), b, n_shared, n_ps));
        hi[k] = P;
    }
    __syncthreads();
    V* st = state + ((size_t)b << W) + ((size_t)chunk << cb);
    const int lm = (1 << h) - 1;
    for (int i = 2 * t; i < (1 << cb); i += 512)
        store_pair(st + i, vec, cmul(lo[i & lm], hi[i >> h]), cmul(lo[(i + 1) & lm], hi[(i + 1) >> h]));
}

// ----------------------------------------------------------------------------
// readout
// ----------------------------------------------------------------------------
// <Z_i> partials of one chunk of 2^cb amplitudes (cb = min(W, 12)) of one
// sample: thread t reads the pairs (2i, 2i + 1), i = t + 2^tb j, so bit 0
// sits in the pair, bits 1..tb come from t and the bits above from j.
// Per-thread float32 sums over at most 16 amplitudes, float64 above.
template <class V>
__global__ __launch_bounds__(256) void k_expval_part(const V* __restrict__ state, int W,
                                                     double* __restrict__ part, int vec) {
    using R = Real<V>;
    __shared__ double red[4][13];
    const int cb = min(W, 12), tb = min(cb - 1, 8), jb = cb - 1 - tb;
    const int t = threadIdx.x;
    const int b = blockIdx.y;
    const int64_t chunk = blockIdx.x;
    const int64_t nchunk = gridDim.x;
    const V* st = state + ((size_t)b << W) + ((size_t)chunk << cb);
    R T = 0, S0 = 0, S[3] = {0, 0, 0};
    if (t < (1 << tb)) {
        for (int j = 0; j < (1 << jb); ++j) {
            V a0, a1;
            load_pair(st + 2 * (((size_t)j << tb) | t), vec != 0, a0, a1);
            const R p0 = a0.x * a0.x + a0.y * a0.y, p1 = a1.x * a1.x + a1.y * a1.y;
            T += p0 + p1;
            S0 += p1;
            for (int i = 0; i < jb; ++i)
                if ((j >> i) & 1) S[i] += p0 + p1;
        }
    }
    // values: [0] total, [1] bit-0 sum, [2..4] j-bit sums, [5..12] thread-bit weighted totals
    double v[13];
    v[0] = T;
    v[1] = S0;
    for (int i = 0; i < 3; ++i) v[2 + i] = S[i];
    for (int k = 0; k < 8; ++k) v[5 + k] = ((t >> k) & 1) ? (double)T : 0.0;
    const int wave = t >> 6, lane = t & 63;
    for (int k = 0; k < 13; ++k) {
        const double r = wave_sum(v[k]);
        if (lane == 0) red[wave][k] = r;
    }
    __syncthreads();
    if (t < W) {
        auto tot = [&](int k) { return red[0][k] + red[1][k] + red[2][k] + red[3][k]; };
        const int sh = W - 1 - t;  // qubit t is index bit sh
        const double Tsum = tot(0);
        double e;
        if (sh == 0) e = Tsum - 2.0 * tot(1);
        else if (sh <= tb) e = Tsum - 2.0 * tot(5 + sh - 1);
        else if (sh < cb) e = Tsum - 2.0 * tot(2 + sh - 1 - tb);
        else e = ((chunk >> (sh - cb)) & 1) ? -Tsum : Tsum;
        part[((size_t)b * nchunk + chunk) * W + t] = e;
    }
}

__global__ __launch_bounds__(256) void k_expval_final(const double* __restrict__ part, int W,
                                                      int64_t nchunk, double* __restrict__ out) {
    __shared__ double red[256];
    const int b = blockIdx.y, i = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (int64_t c = t; c < nchunk; c += 256) s += part[((size_t)b * nchunk + c) * W + i];
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) out[(size_t)b * W + i] = red[0];
}

// ----------------------------------------------------------------------------
// gradient reduction: partials[(ordinal * B + b) * nch + chunk]
// ----------------------------------------------------------------------------
// Partial of ordinal o, sample b, chunk k at part[B * pu[o] + b * nch[o] + k].
__global__ __launch_bounds__(256) void k_grad_reduce(const double* __restrict__ part,
                                                     const int32_t* __restrict__ csr, int n_weights,
                                                     int n_inputs, int B,
                                                     const int64_t* __restrict__ pu,
                                                     const int32_t* __restrict__ nchv,
                                                     double* __restrict__ gw,
                                                     double* __restrict__ gx,
                                                     const float* __restrict__ weights, int remap) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    const int o = blockIdx.x;  // output index: weights first, then (b, input)
    double s = 0.0;
    int j, b0, b1;
    const int32_t* list;
    int nl;
    if (o < n_weights) {
        j = o;
        list = csr + csr[j];
        nl = csr[j + 1] - csr[j];
        b0 = 0;
        b1 = B;
    } else {
        const int r = o - n_weights;
        const int b = r / n_inputs;
        j = r % n_inputs;
        const int32_t* xo = csr + n_weights + 1;
        list = csr + xo[j];
        nl = xo[j + 1] - xo[j];
        b0 = b;
        b1 = b + 1;
    }
    for (int l = 0; l < nl; ++l) {
        const int o = list[l];
        const int64_t nch = nchv[o];
        const int64_t per = (int64_t)(b1 - b0) * nch;
        const double* base = part + (int64_t)B * pu[o] + (int64_t)b0 * nch;
        for (int64_t e = t; e < per; e += 256) s += base[e];
    }
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) {
        if (o < n_weights) {
            double f = 1.0;
            if (remap) {  // d(pi tanh w)/dw
                const double th = tanh((double)weights[j]);
                f = M_PI * (1.0 - th * th);
            }
            gw[j] = red[0] * f;
        }
        else if (gx) gx[(size_t)b0 * n_inputs + j] = red[0];
    }
}

// ----------------------------------------------------------------------------
// plain method (one sweep per gate)
// ----------------------------------------------------------------------------
constexpr int kPgItems = 4;

// Launch shape of a one-dimensional grid of n_blocks blocks. HIP bounds the
// threads of each grid dimension by 2^32, which the whole-batch kernels reach
// from 2^32 amplitudes (32 GiB of complex64), so blocks beyond 2^16 spill into y.
// Kernels launched this way read their block number from block_1d().
static dim3 grid_1d(int64_t n_blocks) {
    n_blocks = std::max<int64_t>(n_blocks, 1);  // every kernel launched this way bounds-checks its items
    const int64_t gx = std::min<int64_t>(n_blocks, int64_t(1) << 16);
    return dim3((unsigned)gx, (unsigned)((n_blocks + gx - 1) / gx));
}
__device__ __forceinline__ int64_t block_1d() { return (int64_t)blockIdx.y * gridDim.x + blockIdx.x; }

template <class V>
__device__ __forceinline__ void pair_apply(int cls, const M2T<V>& M, V& x, V& y) {
    V u, v;
    switch (cls) {
    case OP_SWAP: u = y; v = x; break;
    case OP_REAL:
        u = mkc(M.m00.x * x.x + M.m01.x * y.x, M.m00.x * x.y + M.m01.x * y.y);
        v = mkc(M.m10.x * x.x + M.m11.x * y.x, M.m10.x * x.y + M.m11.x * y.y);
        break;
    case OP_RXL: {
        const Real<V> a = M.m00.x, bb = M.m01.y;
        u = mkc(a * x.x - bb * y.y, a * x.y + bb * y.x);
        v = mkc(a * y.x - bb * x.y, a * y.y + bb * x.x);
        break;
    }
    default: {
        const V p = cmul(M.m00, x), q = cmul(M.m01, y), r = cmul(M.m10, x), s = cmul(M.m11, y);
        u = mkc(p.x + q.x, p.y + q.y);
        v = mkc(r.x + s.x, r.y + s.y);
        break;
    }
    }
    x = u;
    y = v;
}

// Index bits fixed by a per-gate launch: the target bit (0) and the control
// bits (1) of a pair update, or every qubit's bit (1) of a sign flip.
struct PgBits {
    int n;
    int sh[3], val[3];  // ascending shifts
};

__device__ __forceinline__ PgBits pg_bits(const PGate& pg) {
    PgBits r;
    r.n = 0;
    auto add = [&](int sh, int v) {
        if (sh < 0) return;
        int i = r.n++;
        while (i > 0 && r.sh[i - 1] > sh) { r.sh[i] = r.sh[i - 1]; r.val[i] = r.val[i - 1]; --i; }
        r.sh[i] = sh;
        r.val[i] = v;
    };
    if (pg.cls == OP_SIGN) {
        add(pg.tsh, 1);
        add(pg.sh2, 1);
        add(pg.csh2, 1);
    } else {
        add(pg.tsh, 0);
        add(pg.csh, 1);
        add(pg.csh2, 1);
    }
    return r;
}

// index of item `it` among the indices whose fixed bits take their values
__device__ __forceinline__ int64_t pg_index(int64_t it, const PgBits& f) {
    for (int i = 0; i < f.n; ++i) it = insert_bit(it, f.sh[i], f.val[i]);
    return it;
}

// controls of a diagonal gate satisfied at index idx
__device__ __forceinline__ bool pg_ctl_ok(const PGate& pg, int64_t idx) {
    return (pg.csh < 0 || ((idx >> pg.csh) & 1)) && (pg.csh2 < 0 || ((idx >> pg.csh2) & 1));
}

template <class V>
__global__ __launch_bounds__(256) void k_pg_apply(V* __restrict__ state, int W, int64_t B,
                                                  PGate pg, const Real<V>* __restrict__ mats,
                                                  int n_shared, int n_ps) {
    // kPgItems items per thread, 256 apart (coalesced). Items touch disjoint
    // amplitudes, so every load of the thread is issued before the first store:
    // several loads in flight per thread instead of one item at a time.
    const int64_t base = (block_1d() * kPgItems) * 256 + threadIdx.x;
    if (pg.cls == OP_DIAG) {
        const int64_t total = B << W;
        V a[kPgItems];
#pragma unroll
        for (int i = 0; i < kPgItems; ++i) {
            const int64_t it = base + i * 256;
            if (it < total && pg_ctl_ok(pg, it)) a[i] = state[it];
        }
#pragma unroll
        for (int i = 0; i < kPgItems; ++i) {
            const int64_t it = base + i * 256;
            if (it >= total || !pg_ctl_ok(pg, it)) continue;
            const int b = (int)(it >> W);
            const auto M = load_m2(mat_ptr(mats, pg.mat, b, n_shared, n_ps));
            const V ph = ((it >> pg.tsh) & 1) ? M.m11 : M.m00;
            state[it] = cmul(ph, a[i]);
        }
    } else if (pg.cls == OP_SIGN) {
        const PgBits f = pg_bits(pg);
        const int64_t total = B << (W - f.n);
        V a[kPgItems];
        int64_t idx[kPgItems];
#pragma unroll
        for (int i = 0; i < kPgItems; ++i) {
            const int64_t it = base + i * 256;
            idx[i] = it < total ? pg_index(it, f) : -1;
            if (idx[i] >= 0) a[i] = state[idx[i]];
        }
#pragma unroll
        for (int i = 0; i < kPgItems; ++i)
            if (idx[i] >= 0) state[idx[i]] = mkc(-a[i].x, -a[i].y);
    } else {
        const PgBits f = pg_bits(pg);
        const int64_t total = B << (W - f.n);
        const int64_t step = int64_t(1) << pg.tsh;
        V x[kPgItems], y[kPgItems];
        int64_t i0[kPgItems];
#pragma unroll
        for (int i = 0; i < kPgItems; ++i) {
            const int64_t it = base + i * 256;
            i0[i] = it < total ? pg_index(it, f) : -1;
            if (i0[i] >= 0) {
                x[i] = state[i0[i]];
                y[i] = state[i0[i] | step];
            }
        }
#pragma unroll
        for (int i = 0; i < kPgItems; ++i) {
            if (i0[i] < 0) continue;
            M2T<V> M{};
            if (pg.cls != OP_SWAP) M = load_m2(mat_ptr(mats, pg.mat, (int)(i0[i] >> W), n_shared, n_ps));
            pair_apply(pg.cls, M, x[i], y[i]);
            state[i0[i]] = x[i];
            state[i0[i] | step] = y[i];
        }
    }
}

// 16-byte access modes of a complex64 per-gate launch (chosen on the host):
//  PG_VEC_PAIRS  every index bit the gate fixes is above bit 0, so item i covers
//                the gate's items 2i and 2i+1, whose amplitudes sit next to each
//                other (for a pair update: both first and both second amplitudes);
//                a diagonal gate's items are simply consecutive amplitudes;
//  PG_VEC_ADJ    the target is bit 0: a pair's two amplitudes are adjacent.
// Every other launch (a control on bit 0, complex128, a state not 16-byte
// aligned) takes the scalar kernel. Loads and stores are non-temporal: every
// amplitude is touched once per launch.
//  PG_VEC_SWEEP  a sign gate whose lowest fixed bit is 0, 1 or 2: its touched
//                amplitudes come in runs shorter than a cache line, so every line
//                moves anyway; all adjacent pairs are read, the amplitudes whose
//                fixed bits are all 1 negated, and everything written back with
//                full 16-byte stores.
enum { PG_SCALAR = 0, PG_VEC_PAIRS = 1, PG_VEC_ADJ = 2, PG_VEC_SWEEP = 3 };
__device__ __forceinline__ f4v ntl4(const float2* p) { return __builtin_nontemporal_load((const f4v*)p); }
// cached load: for a pair whose two halves share a cache line (target bit <= 3),
// where a streaming load of the second half would fetch the line again
__device__ __forceinline__ f4v ld4(const float2* p, bool cached) {
    return cached ? *(const f4v*)p : __builtin_nontemporal_load((const f4v*)p);
}
__device__ __forceinline__ void nts4(float2* p, f4v v) { __builtin_nontemporal_store(v, (f4v*)p); }
__device__ __forceinline__ float2 lo2(f4v v) { return make_float2(v.x, v.y); }
__device__ __forceinline__ float2 hi2(f4v v) { return make_float2(v.z, v.w); }
__device__ __forceinline__ f4v cat2(float2 a, float2 b) { return f4v{a.x, a.y, b.x, b.y}; }
// every bit a sign gate fixes is 1 at index idx
__device__ __forceinline__ bool sign_on(const PgBits& f, int64_t idx) {
    bool on = true;
    for (int i = 0; i < f.n; ++i) on = on && ((idx >> f.sh[i]) & 1);
    return on;
}

// One item per thread, 16-byte accesses (see PG_VEC_*). Items: diagonal B 2^W / 2,
// sign and pair updates B 2^(W - fixed) / 2 (PAIRS) or B 2^(W - fixed) (ADJ).
__global__ __launch_bounds__(256) void k_pg_apply_vec(float2* __restrict__ state, int W, int64_t items,
                                                      PGate pg, int mode, const float* __restrict__ mats,
                                                      int n_shared, int n_ps, int rev) {
    const int64_t blk = rev ? (int64_t)gridDim.x * gridDim.y - 1 - block_1d() : block_1d();
    const int64_t it = blk * 256 + threadIdx.x;
    if (it >= items) return;
    if (pg.cls == OP_DIAG) {
        const int64_t i0 = 2 * it;
        const int b = (int)(i0 >> W);
        const M2 M = load_m2(mat_ptr(mats, pg.mat, b, n_shared, n_ps));
        const f4v a = ntl4(state + i0);
        float2 u = lo2(a), v = hi2(a);
        if (pg_ctl_ok(pg, i0)) u = cmul(((i0 >> pg.tsh) & 1) ? M.m11 : M.m00, u);
        if (pg_ctl_ok(pg, i0 + 1)) v = cmul((((i0 + 1) >> pg.tsh) & 1) ? M.m11 : M.m00, v);
        nts4(state + i0, cat2(u, v));
        return;
    }
    const PgBits f = pg_bits(pg);
    if (pg.cls == OP_SIGN) {
        if (mode == PG_VEC_SWEEP) {
            const int64_t i0 = 2 * it;
            const bool n0 = sign_on(f, i0), n1 = sign_on(f, i0 + 1);
            const f4v a = ntl4(state + i0);
            nts4(state + i0, f4v{n0 ? -a.x : a.x, n0 ? -a.y : a.y, n1 ? -a.z : a.z, n1 ? -a.w : a.w});
            return;
        }
        const int64_t i0 = pg_index(2 * it, f);  // with its neighbour i0 + 1
        const f4v a = ntl4(state + i0);
        nts4(state + i0, f4v{-a.x, -a.y, -a.z, -a.w});
        return;
    }
    M2 M{};
    if (mode == PG_VEC_ADJ) {
        const int64_t i0 = pg_index(it, f);
        if (pg.cls != OP_SWAP) M = load_m2(mat_ptr(mats, pg.mat, (int)(i0 >> W), n_shared, n_ps));
        const f4v a = ntl4(state + i0);
        float2 x = lo2(a), y = hi2(a);
        pair_apply(pg.cls, M, x, y);
        nts4(state + i0, cat2(x, y));
        return;
    }
    const int64_t i0 = pg_index(2 * it, f), i1 = i0 | (int64_t(1) << pg.tsh);
    if (pg.cls != OP_SWAP) M = load_m2(mat_ptr(mats, pg.mat, (int)(i0 >> W), n_shared, n_ps));
    const bool near = pg.tsh <= 3;
    const f4v a = ld4(state + i0, near), c = ld4(state + i1, near);
    float2 x0 = lo2(a), x1 = hi2(a), y0 = lo2(c), y1 = hi2(c);
    pair_apply(pg.cls, M, x0, y0);
    pair_apply(pg.cls, M, x1, y1);
    nts4(state + i0, cat2(x0, x1));
    nts4(state + i1, cat2(y0, y1));
}

// lambda = D psi_N with D(idx) = sum_i g[b,i] (1 - 2 bit_i(idx)) = G - 2 sum over
// the set bits, psi_N copied to the workspace. One block per chunk of 2^cb
// amplitudes (cb = min(W, 12)) and sample; the block tabulates the set-bit
// sums of its low h bits (lo) and of its other bits (hi, including the
// chunk's bits above cb) in float64, then streams 16-byte pairs.
template <class V>
__global__ __launch_bounds__(256) void k_adj_init(const V* __restrict__ psiN,
                                                  V* __restrict__ psi, V* __restrict__ lam,
                                                  int W, const double* __restrict__ g, int vec) {
    __shared__ double gs[32], lo[64], hi[64], G;
    const int cb = min(W, 12), h = cb / 2, hb = cb - h;
    const int t = threadIdx.x;
    const int b = blockIdx.y;
    const int64_t chunk = blockIdx.x;
    if (t < W) gs[t] = g[(size_t)b * W + t];
    __syncthreads();
    if (t < (1 << h)) {
        double d = 0.0;
        for (int s = 0; s < h; ++s)
            if ((t >> s) & 1) d += gs[W - 1 - s];
        lo[t] = d;
    } else if (t >= 64 && t < 64 + (1 << hb)) {
        const int k = t - 64;
        double d = 0.0;
        for (int s = h; s < cb; ++s)
            if ((k >> (s - h)) & 1) d += gs[W - 1 - s];
        for (int s = cb; s < W; ++s)
            if ((chunk >> (s - cb)) & 1) d += gs[W - 1 - s];
        hi[k] = d;
    } else if (t == 128) {
        double d = 0.0;
        for (int i = 0; i < W; ++i) d += gs[i];
        G = d;
    }
    __syncthreads();
    const size_t base = ((size_t)b << W) + ((size_t)chunk << cb);
    const int lm = (1 << h) - 1;
    for (int i = 2 * t; i < (1 << cb); i += 512) {
        V a0, a1;
        load_pair(psiN + base + i, vec != 0, a0, a1);
        const Real<V> d0 = (Real<V>)(G - 2.0 * (lo[i & lm] + hi[i >> h]));
        const Real<V> d1 = (Real<V>)(G - 2.0 * (lo[(i + 1) & lm] + hi[(i + 1) >> h]));
        store_pair(psi + base + i, true, a0, a1);
        store_pair(lam + base + i, true, mkc(d0 * a0.x, d0 * a0.y), mkc(d1 * a1.x, d1 * a1.y));
    }
}

// Plain-method backward step for one gate: gradient partial at psi_k, lambda_k,
// then psi <- U^dagger psi, lambda <- U^dagger lambda. Grid (nch, B).
template <class V>
__global__ __launch_bounds__(256) void k_pg_adj(V* __restrict__ psi, V* __restrict__ lam,
                                                int W, int B, PGate pg,
                                                const Real<V>* __restrict__ mats, int n_shared,
                                                int n_ps, double* __restrict__ part, int64_t nch) {
    __shared__ double red[4];
    const int t = threadIdx.x;
    const int b = blockIdx.y;
    const int64_t chunk = blockIdx.x;
    const size_t off = (size_t)b << W;
    V* P = psi + off;
    V* L = lam + off;
    Real<V> acc = 0;
    M2T<V> M{};
    if (pg.cls != OP_SWAP && pg.cls != OP_SIGN) M = load_m2(mat_ptr(mats, pg.mat, b, n_shared, n_ps));
    if (pg.cls == OP_DIAG) {
        const int64_t n = int64_t(1) << W, per = n / nch;
        for (int64_t e = t; e < per; e += 256) {
            const int64_t idx = chunk * per + e;
            if (!pg_ctl_ok(pg, idx)) continue;
            const int bit = (idx >> pg.tsh) & 1;
            V p = P[idx], l = L[idx];
            if (pg.grad == OP_GZ) acc += bit ? -im_conj_mul(l, p) : im_conj_mul(l, p);
            const V ph = bit ? M.m11 : M.m00;
            P[idx] = cmul(ph, p);
            L[idx] = cmul(ph, l);
        }
    } else if (pg.cls == OP_SIGN) {
        const PgBits f = pg_bits(pg);
        const int64_t n = int64_t(1) << (W - f.n), per = n / nch;
        for (int64_t e = t; e < per; e += 256) {
            const int64_t idx = pg_index(chunk * per + e, f);
            const V p = P[idx], l = L[idx];
            P[idx] = mkc(-p.x, -p.y);
            L[idx] = mkc(-l.x, -l.y);
        }
    } else {
        const PgBits f = pg_bits(pg);
        const int64_t n = int64_t(1) << (W - f.n), per = n / nch;
        for (int64_t e = t; e < per; e += 256) {
            const int64_t it = chunk * per + e;
            const int64_t i0 = pg_index(it, f);
            const int64_t i1 = i0 | (int64_t(1) << pg.tsh);
            V p0 = P[i0], p1 = P[i1], l0 = L[i0], l1 = L[i1];
            if (pg.grad == OP_GX) acc += im_conj_mul(l0, p1) + im_conj_mul(l1, p0);
            else if (pg.grad == OP_GY) acc += re_conj_mul(l1, p0) - re_conj_mul(l0, p1);
            pair_apply(pg.cls, M, p0, p1);
            pair_apply(pg.cls, M, l0, l1);
            P[i0] = p0; P[i1] = p1; L[i0] = l0; L[i1] = l1;
        }
    }
    if (pg.slot >= 0) {
        const double r = wave_sum((double)acc);
        if ((t & 63) == 0) red[t >> 6] = r;
        __syncthreads();
        if (t == 0) part[((size_t)pg.slot * B + b) * nch + chunk] = red[0] + red[1] + red[2] + red[3];
    }
}

// Plain-method backward step with 16-byte accesses (complex64, PG_VEC_* modes
// as in k_pg_apply_vec): same arithmetic, partials and grid as k_pg_adj.
__global__ __launch_bounds__(256) void k_pg_adj_vec(float2* __restrict__ psi, float2* __restrict__ lam, int W,
                                                    int B, PGate pg, int mode, const float* __restrict__ mats,
                                                    int n_shared, int n_ps, double* __restrict__ part,
                                                    int64_t nch, int rev) {
    __shared__ double red[4];
    constexpr int nt = 256;
    const int t = threadIdx.x;
    const int b = rev ? (int)gridDim.y - 1 - (int)blockIdx.y : (int)blockIdx.y;
    const int64_t chunk = rev ? (int64_t)gridDim.x - 1 - blockIdx.x : (int64_t)blockIdx.x;
    const size_t off = (size_t)b << W;
    float2* P = psi + off;
    float2* L = lam + off;
    float acc = 0.f;
    M2 M{};
    if (pg.cls != OP_SWAP && pg.cls != OP_SIGN) M = load_m2(mat_ptr(mats, pg.mat, b, n_shared, n_ps));
    auto grad_pair = [&](float2 p0, float2 p1, float2 l0, float2 l1) {
        if (pg.grad == OP_GX) acc += im_conj_mul(l0, p1) + im_conj_mul(l1, p0);
        else if (pg.grad == OP_GY) acc += re_conj_mul(l1, p0) - re_conj_mul(l0, p1);
    };
    if (pg.cls == OP_DIAG) {
        const int64_t per = ((int64_t(1) << W) / 2) / nch;  // items of two amplitudes
        for (int64_t e = t; e < per; e += nt) {
            const int64_t i0 = 2 * (chunk * per + e);
            const f4v pa = ntl4(P + i0), la = ntl4(L + i0);
            float2 p[2] = {lo2(pa), hi2(pa)}, l[2] = {lo2(la), hi2(la)};
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int64_t idx = i0 + j;
                if (!pg_ctl_ok(pg, idx)) continue;
                const int bit = (idx >> pg.tsh) & 1;
                if (pg.grad == OP_GZ) acc += bit ? -im_conj_mul(l[j], p[j]) : im_conj_mul(l[j], p[j]);
                const float2 ph = bit ? M.m11 : M.m00;
                p[j] = cmul(ph, p[j]);
                l[j] = cmul(ph, l[j]);
            }
            nts4(P + i0, cat2(p[0], p[1]));
            nts4(L + i0, cat2(l[0], l[1]));
        }
    } else if (pg.cls == OP_SIGN && mode == PG_VEC_SWEEP) {
        const PgBits f = pg_bits(pg);
        const int64_t per = ((int64_t(1) << W) / 2) / nch;
        for (int64_t e = t; e < per; e += nt) {
            const int64_t i0 = 2 * (chunk * per + e);
            const bool n0 = sign_on(f, i0), n1 = sign_on(f, i0 + 1);
            const f4v pa = ntl4(P + i0), la = ntl4(L + i0);
            nts4(P + i0, f4v{n0 ? -pa.x : pa.x, n0 ? -pa.y : pa.y, n1 ? -pa.z : pa.z, n1 ? -pa.w : pa.w});
            nts4(L + i0, f4v{n0 ? -la.x : la.x, n0 ? -la.y : la.y, n1 ? -la.z : la.z, n1 ? -la.w : la.w});
        }
    } else if (pg.cls == OP_SIGN) {
        const PgBits f = pg_bits(pg);
        const int64_t per = ((int64_t(1) << (W - f.n)) / 2) / nch;
        for (int64_t e = t; e < per; e += nt) {
            const int64_t i0 = pg_index(2 * (chunk * per + e), f);
            const f4v pa = ntl4(P + i0), la = ntl4(L + i0);
            nts4(P + i0, f4v{-pa.x, -pa.y, -pa.z, -pa.w});
            nts4(L + i0, f4v{-la.x, -la.y, -la.z, -la.w});
        }
    } else if (mode == PG_VEC_ADJ) {
        const PgBits f = pg_bits(pg);
        const int64_t per = (int64_t(1) << (W - f.n)) / nch;
        for (int64_t e = t; e < per; e += nt) {
            const int64_t i0 = pg_index(chunk * per + e, f);
            const f4v pa = ntl4(P + i0), la = ntl4(L + i0);
            float2 p0 = lo2(pa), p1 = hi2(pa), l0 = lo2(la), l1 = hi2(la);
            grad_pair(p0, p1, l0, l1);
            pair_apply(pg.cls, M, p0, p1);
            pair_apply(pg.cls, M, l0, l1);
            nts4(P + i0, cat2(p0, p1));
            nts4(L + i0, cat2(l0, l1));
        }
    } else {
        const PgBits f = pg_bits(pg);
        const int64_t per = ((int64_t(1) << (W - f.n)) / 2) / nch;
        const int64_t step = int64_t(1) << pg.tsh;
        const bool near = pg.tsh <= 3;
        for (int64_t e = t; e < per; e += nt) {
            const int64_t i0 = pg_index(2 * (chunk * per + e), f), i1 = i0 | step;
            const f4v pa = ld4(P + i0, near), pc = ld4(P + i1, near), la = ld4(L + i0, near), lc = ld4(L + i1, near);
            float2 p00 = lo2(pa), p01 = hi2(pa), p10 = lo2(pc), p11 = hi2(pc);
            float2 l00 = lo2(la), l01 = hi2(la), l10 = lo2(lc), l11 = hi2(lc);
            grad_pair(p00, p10, l00, l10);
            grad_pair(p01, p11, l01, l11);
            pair_apply(pg.cls, M, p00, p10);
            pair_apply(pg.cls, M, p01, p11);
            pair_apply(pg.cls, M, l00, l10);
            pair_apply(pg.cls, M, l01, l11);
            nts4(P + i0, cat2(p00, p01));
            nts4(P + i1, cat2(p10, p11));
            nts4(L + i0, cat2(l00, l01));
            nts4(L + i1, cat2(l10, l11));
        }
    }
    if (pg.slot >= 0) {
        const double r = wave_sum((double)acc);
        if ((t & 63) == 0) red[t >> 6] = r;
        __syncthreads();
        if (t == 0) part[((size_t)pg.slot * B + b) * nch + chunk] = red[0] + red[1] + red[2] + red[3];
    }
}

// ----------------------------------------------------------------------------
// fused passes
// ----------------------------------------------------------------------------
// Register position p of a thread's 16 amplitudes <-> local tile bit reg[p].
// Thread bits fill the other local bits in ascending order.
struct Lay {
    int lT, gT;          // thread part of the local / global index
    int lr[kRegBits];    // 1 << reg[p]
    int gr[kRegBits];    // 1 << lq[reg[p]]
};

__device__ __forceinline__ void make_layout(const DPass* __restrict__ P, int m, const int* reg,
                                            int t, int tile_base, Lay& L) {
    L.lT = 0;
    L.gT = tile_base;
    int i = 0;
    for (int j = 0; j < m; ++j) {
        if (j == reg[0] || j == reg[1] || j == reg[2] || j == reg[3]) continue;
        const int bit = (t >> i) & 1;
        ++i;
        L.lT |= bit << j;
        L.gT |= bit << P->lq[j];
    }
    for (int p = 0; p < kRegBits; ++p) {
        L.lr[p] = 1 << reg[p];
        L.gr[p] = 1 << P->lq[reg[p]];
    }
}

template <int K>
__device__ __forceinline__ int reg_part(const int* parts) {
    return ((K & 1) ? parts[0] : 0) | ((K & 2) ? parts[1] : 0) | ((K & 4) ? parts[2] : 0) |
           ((K & 8) ? parts[3] : 0);
}

template <int K = 0>
__device__ __forceinline__ void lds_store(float2* lds, const Lay& L, const float2 (&a)[kRegs]) {
    if constexpr (K < kRegs) {
        lds[swz(L.lT | reg_part<K>(L.lr))] = a[K];
        lds_store<K + 1>(lds, L, a);
    }
}
template <int K = 0>
__device__ __forceinline__ void lds_load(const float2* lds, const Lay& L, float2 (&a)[kRegs]) {
    if constexpr (K < kRegs) {
        a[K] = lds[swz(L.lT | reg_part<K>(L.lr))];
        lds_load<K + 1>(lds, L, a);
    }
}
template <int K = 0>
__device__ __forceinline__ void g_load(const float2* st, const Lay& L, float2 (&a)[kRegs]) {
    if constexpr (K < kRegs) {
        a[K] = st[L.gT | reg_part<K>(L.gr)];
        g_load<K + 1>(st, L, a);
    }
}
template <int K = 0>
__device__ __forceinline__ void g_store(float2* st, const Lay& L, const float2 (&a)[kRegs]) {
    if constexpr (K < kRegs) {
        st[L.gT | reg_part<K>(L.gr)] = a[K];
        g_store<K + 1>(st, L, a);
    }
}

// The product state at a thread's 16 amplitudes, in place of loading them
// (first forward pass): amp(idx) = prod over amplitude bits s of
// v_{W-1-s}[bit s of idx], v_q = column 0 of qubit q's prefix matrix. The
// factors of the thread's fixed bits (L.gT) are multiplied once, then the
// product is split over the four register bits.
__device__ __forceinline__ void init_regs(const Lay& L, float2 (&a)[kRegs], const int32_t* __restrict__ pm,
                                          const float* __restrict__ mats, int W, int b, int n_shared,
                                          int n_ps) {
    const int rm = L.gr[0] | L.gr[1] | L.gr[2] | L.gr[3];
    float2 P = make_float2(1.f, 0.f);
    for (int s = 0; s < W; ++s)
        if (!((rm >> s) & 1)) P = cmul(P, prefix_v(mats, pm, W - 1 - s, (L.gT >> s) & 1, b, n_shared, n_ps));
    a[0] = P;
#pragma unroll
    for (int p = 0; p < kRegBits; ++p) {
        const int q = W - 1 - (31 - __builtin_clz((unsigned)L.gr[p]));
        const float2 v0 = prefix_v(mats, pm, q, 0, b, n_shared, n_ps);
        const float2 v1 = prefix_v(mats, pm, q, 1, b, n_shared, n_ps);
#pragma unroll
        for (int k = 0; k < (1 << p); ++k) {
            a[k | (1 << p)] = cmul(a[k], v1);
            a[k] = cmul(a[k], v0);
        }
    }
}

// --- register ops, templated on the target's register position P ---
template <int P, bool CTL>
__device__ __forceinline__ void r_u2(float2 (&a)[kRegs], const M2& M, int cm) {
#pragma unroll
    for (int k = 0; k < kRegs; ++k) {
        if (k & (1 << P)) continue;
        const int k1 = k | (1 << P);
        const float2 x = a[k], y = a[k1];
        const float2 p = cmul(M.m00, x), q = cmul(M.m01, y), r = cmul(M.m10, x), s = cmul(M.m11, y);
        const float2 u = make_float2(p.x + q.x, p.y + q.y), v = make_float2(r.x + s.x, r.y + s.y);
        if (CTL) {
            const bool c = (cm >> k) & 1;
            a[k] = c ? u : x;
            a[k1] = c ? v : y;
        } else {
            a[k] = u;
            a[k1] = v;
        }
    }
}

template <int P, bool CTL>
__device__ __forceinline__ void r_real(float2 (&a)[kRegs], const M2& M, int cm) {
#pragma unroll
    for (int k = 0; k < kRegs; ++k) {
        if (k & (1 << P)) continue;
        const int k1 = k | (1 << P);
        const float2 x = a[k], y = a[k1];
        const float2 u = make_float2(M.m00.x * x.x + M.m01.x * y.x, M.m00.x * x.y + M.m01.x * y.y);
        const float2 v = make_float2(M.m10.x * x.x + M.m11.x * y.x, M.m10.x * x.y + M.m11.x * y.y);
        if (CTL) {
            const bool c = (cm >> k) & 1;
            a[k] = c ? u : x;
            a[k1] = c ? v : y;
        } else {
            a[k] = u;
            a[k1] = v;
        }
    }
}

template <int P, bool CTL>
__device__ __forceinline__ void r_rxl(float2 (&a)[kRegs], const M2& M, int cm) {
    const float al = M.m00.x, be = M.m01.y;
#pragma unroll
    for (int k = 0; k < kRegs; ++k) {
        if (k & (1 << P)) continue;
        const int k1 = k | (1 << P);
        const float2 x = a[k], y = a[k1];
        const float2 u = make_float2(al * x.x - be * y.y, al * x.y + be * y.x);
        const float2 v = make_float2(al * y.x - be * x.y, al * y.y + be * x.x);
        if (CTL) {
            const bool c = (cm >> k) & 1;
            a[k] = c ? u : x;
            a[k1] = c ? v : y;
        } else {
            a[k] = u;
            a[k1] = v;
        }
    }
}

template <int P, bool CTL>
__device__ __forceinline__ void r_swap(float2 (&a)[kRegs], int cm) {
#pragma unroll
    for (int k = 0; k < kRegs; ++k) {
        if (k & (1 << P)) continue;
        const int k1 = k | (1 << P);
        const float2 x = a[k], y = a[k1];
        if (CTL) {
            const bool c = (cm >> k) & 1;
            a[k] = c ? y : x;
            a[k1] = c ? x : y;
        } else {
            a[k] = y;
            a[k1] = x;
        }
    }
}

// diagonal ops apply to the registers in cm (the controls' mask; 0xFFFF = all)
template <int P>
__device__ __forceinline__ void r_diag(float2 (&a)[kRegs], const M2& M, int cm) {
#pragma unroll
    for (int k = 0; k < kRegs; ++k) {
        const float2 u = cmul((k & (1 << P)) ? M.m11 : M.m00, a[k]);
        a[k] = ((cm >> k) & 1) ? u : a[k];
    }
}

__device__ __forceinline__ void r_phase_all(float2 (&a)[kRegs], float2 ph, int cm) {
#pragma unroll
    for (int k = 0; k < kRegs; ++k) {
        const float2 u = cmul(ph, a[k]);
        a[k] = ((cm >> k) & 1) ? u : a[k];
    }
}

__device__ __forceinline__ void r_flip(float2 (&a)[kRegs], int flip) {
#pragma unroll
    for (int k = 0; k < kRegs; ++k) {
        const unsigned s = (unsigned)((flip >> k) & 1) << 31;
        a[k] = make_float2(__uint_as_float(__float_as_uint(a[k].x) ^ s),
                           __uint_as_float(__float_as_uint(a[k].y) ^ s));
    }
}

template <int P, bool CTL>
__device__ __forceinline__ float r_gx(const float2 (&ps)[kRegs], const float2 (&lm)[kRegs], int cm) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < kRegs; ++k) {
        if (k & (1 << P)) continue;
        const int k1 = k | (1 << P);
        const float v = im_conj_mul(lm[k], ps[k1]) + im_conj_mul(lm[k1], ps[k]);
        acc += (!CTL || ((cm >> k) & 1)) ? v : 0.f;
    }
    return acc;
}
template <int P>
__device__ __forceinline__ float r_gy(const float2 (&ps)[kRegs], const float2 (&lm)[kRegs], int cm) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < kRegs; ++k) {
        if (k & (1 << P)) continue;
        const int k1 = k | (1 << P);
        const float v = re_conj_mul(lm[k1], ps[k]) - re_conj_mul(lm[k], ps[k1]);
        acc += ((cm >> k) & 1) ? v : 0.f;
    }
    return acc;
}
template <int P>
__device__ __forceinline__ float r_gz(const float2 (&ps)[kRegs], const float2 (&lm)[kRegs], int cm) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < kRegs; ++k) {
        const float v = im_conj_mul(lm[k], ps[k]);
        acc += ((cm >> k) & 1) ? ((k & (1 << P)) ? -v : v) : 0.f;
    }
    return acc;
}
__device__ __forceinline__ float r_gz_all(const float2 (&ps)[kRegs], const float2 (&lm)[kRegs], int cm) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < kRegs; ++k) acc += ((cm >> k) & 1) ? im_conj_mul(lm[k], ps[k]) : 0.f;
    return acc;
}

// 16-bit mask of the registers whose control qubit is 1.
__device__ __forceinline__ int ctl_mask(int ctl, int gT) {
    if (ctl < 0) return 0xFFFF;
    switch (ctl) {
    case 0: return 0xAAAA;
    case 1: return 0xCCCC;
    case 2: return 0xF0F0;
    case 3: return 0xFF00;
    default: return ((gT >> (ctl & 0xFF)) & 1) ? 0xFFFF : 0;
    }
}

#define QSV_DISPATCH_POS(pos, CALL) \
    switch (pos) {                  \
    case 0: CALL(0); break;         \
    case 1: CALL(1); break;         \
    case 2: CALL(2); break;         \
    default: CALL(3); break;        \
    }

// Apply one non-gradient op to one register set (NA = 1) or to two (NA = 2,
// psi and lambda in the backward: one dispatch for both).
template <int NA>
__device__ __forceinline__ void apply_op(const DOp& op, float2 (&a)[kRegs], float2 (&a2)[kRegs], const M2& M,
                                         int gT, const DTerm* __restrict__ terms) {
    const bool ctl = op.ctl >= 0;
    const int cm = ctl_mask(op.ctl, gT) & ctl_mask(op.ctl2, gT);
#define BOTH_(f)        \
    do {                \
        { f(a); }       \
        if (NA == 2) {  \
            f(a2);      \
        }               \
    } while (0)
    switch (op.kind) {
    case OP_U2:
#define U_(x) if (ctl) r_u2<P_, true>(x, M, cm); else r_u2<P_, false>(x, M, cm)
#define C_(P) { constexpr int P_ = P; BOTH_(U_); }
        QSV_DISPATCH_POS(op.pos, C_)
#undef C_
#undef U_
        break;
    case OP_REAL:
#define U_(x) if (ctl) r_real<P_, true>(x, M, cm); else r_real<P_, false>(x, M, cm)
#define C_(P) { constexpr int P_ = P; BOTH_(U_); }
        QSV_DISPATCH_POS(op.pos, C_)
#undef C_
#undef U_
        break;
    case OP_RXL:
#define U_(x) if (ctl) r_rxl<P_, true>(x, M, cm); else r_rxl<P_, false>(x, M, cm)
#define C_(P) { constexpr int P_ = P; BOTH_(U_); }
        QSV_DISPATCH_POS(op.pos, C_)
#undef C_
#undef U_
        break;
    case OP_SWAP:
#define U_(x) if (ctl) r_swap<P_, true>(x, cm); else r_swap<P_, false>(x, cm)
#define C_(P) { constexpr int P_ = P; BOTH_(U_); }
        QSV_DISPATCH_POS(op.pos, C_)
#undef C_
#undef U_
        break;
    case OP_DIAG:
        if (op.pos >= 0) {
#define U_(x) r_diag<P_>(x, M, cm)
#define C_(P) { constexpr int P_ = P; BOTH_(U_); }
            QSV_DISPATCH_POS(op.pos, C_)
#undef C_
#undef U_
        } else {
            const float2 ph = ((gT >> op.sh) & 1) ? M.m11 : M.m00;
#define U_(x) r_phase_all(x, ph, cm)
            BOTH_(U_);
#undef U_
        }
        break;
    case OP_SIGN: {
        int flip = op.pos;
        for (int i = 0; i < op.nterm; ++i) {
            const DTerm tm = terms[op.term0 + i];
            const bool on = ((gT >> tm.s0) & 1) && (tm.s1 < 0 || ((gT >> tm.s1) & 1)) &&
                            (tm.s2 < 0 || ((gT >> tm.s2) & 1));
            if (on) flip ^= tm.mask;
        }
#define U_(x) r_flip(x, flip)
        BOTH_(U_);
#undef U_
        break;
    }
    default: break;
    }
#undef BOTH_
}

__device__ __forceinline__ float grad_op(const DOp& op, const float2 (&ps)[kRegs],
                                         const float2 (&lm)[kRegs], int gT) {
    float v = 0.f;
    const bool ctl = op.ctl >= 0;
    const int cm = ctl_mask(op.ctl, gT) & ctl_mask(op.ctl2, gT);
    if (op.kind == OP_GX) {
#define C_(P) v = ctl ? r_gx<P, true>(ps, lm, cm) : r_gx<P, false>(ps, lm, cm)
        QSV_DISPATCH_POS(op.pos, C_)
#undef C_
    } else if (op.kind == OP_GY) {
#define C_(P) v = r_gy<P>(ps, lm, cm)
        QSV_DISPATCH_POS(op.pos, C_)
#undef C_
    } else {
        if (op.pos >= 0) {
#define C_(P) v = r_gz<P>(ps, lm, cm)
            QSV_DISPATCH_POS(op.pos, C_)
#undef C_
        } else {
            v = r_gz_all(ps, lm, cm);
            if ((gT >> op.sh) & 1) v = -v;
        }
    }
    return v;
}

__device__ __forceinline__ bool same_reg(const int* a, const int* b) {
    return a[0] == b[0] && a[1] == b[1] && a[2] == b[2] && a[3] == b[3];
}

__device__ __forceinline__ int tile_base_of(const DPass* __restrict__ P, int tbits, int64_t tis) {
    int base = 0;
    for (int k = 0; k < tbits; ++k) base |= (int)((tis >> k) & 1) << P->oq[k];
    return base;
}

// One fused forward pass over one tile of one sample. st: the sample's 2^W
// amplitudes; tis: tile index within the sample; lds: 2^m float2.
// An op's 2x2 matrix (ops without one get zeros).
__device__ __forceinline__ M2 op_matrix(const DOp& op, const float* __restrict__ mats, int b, int n_shared,
                                        int n_ps) {
    M2 M{};
    if (op.kind != OP_SIGN && op.kind != OP_SWAP && op.kind < OP_GX)
        M = load_m2(mat_ptr(mats, op.mat, b, n_shared, n_ps));
    return M;
}

__device__ __forceinline__ void pass_fwd_tile(const DPass* __restrict__ P,
                                              const DStage* __restrict__ S,
                                              const DOp* __restrict__ O,
                                              const DTerm* __restrict__ Tm,
                                              const float* __restrict__ mats, int n_shared,
                                              int n_ps, const int32_t* __restrict__ pm,
                                              float2* __restrict__ st, int W, int b, int64_t tis,
                                              float2* lds) {
    const int m = P->m;
    const int t = threadIdx.x;
    const bool act = t < (1 << (m - kRegBits));
    const bool wave_on = (t >> 6) < (((1 << (m - kRegBits)) + 63) >> 6);
    const int base = tile_base_of(P, W - m, tis);

    int cur[kRegBits] = {m - 4, m - 3, m - 2, m - 1};
    Lay L;
    make_layout(P, m, cur, t, base, L);
    float2 a[kRegs];
    if (!act) for (int k = 0; k < kRegs; ++k) a[k] = make_float2(0.f, 0.f);
    else if (P->flags & PF_INIT_FWD) init_regs(L, a, pm, mats, W, b, n_shared, n_ps);
    else g_load(st, L, a);

    for (int s = 0; s < P->n_stages; ++s) {
        const DStage& stg = S[P->stage0 + s];
        if (!same_reg(cur, stg.reg)) {
            if (act) lds_store(lds, L, a);
            __syncthreads();
            for (int p = 0; p < kRegBits; ++p) cur[p] = stg.reg[p];
            make_layout(P, m, cur, t, base, L);
            if (act) lds_load(lds, L, a);
            __syncthreads();
        }
        // waves without an active lane only keep the barrier count (wave-uniform
        // branch). The next op and its matrix are fetched while the current one
        // is applied, so their load latency overlaps the arithmetic.
        if (wave_on && stg.op0 < stg.op1) {
            DOp op = O[stg.op0];
            M2 M = op_matrix(op, mats, b, n_shared, n_ps);
            for (int oi = stg.op0; oi < stg.op1; ++oi) {
                DOp nop = op;
                M2 nM = M;
                if (oi + 1 < stg.op1) {
                    nop = O[oi + 1];
                    nM = op_matrix(nop, mats, b, n_shared, n_ps);
                }
                apply_op<1>(op, a, a, M, L.gT, Tm);
                op = nop;
                M = nM;
            }
        }
    }
    const int nat[kRegBits] = {m - 4, m - 3, m - 2, m - 1};
    if (!same_reg(cur, nat)) {
        if (act) lds_store(lds, L, a);
        __syncthreads();
        make_layout(P, m, nat, t, base, L);
        if (act) lds_load(lds, L, a);
        __syncthreads();
    }
    if (act) g_store(st, L, a);
}

// One fused backward pass over one tile of one sample. psiN_s / psi_s / lam_s:
// the sample's vectors; g: the sample's W upstream gradients. The partial of
// gradient slot j goes to part[B * pu[ord] + b * nch + tis] with ord its
// parametric-gate ordinal. lds: 2^m float2 followed by (blockDim/64) x
// n_gslots doubles.
// Gradient of a gate inside a 1-qubit chain from the chain's components
// cx, cy, cz = Im<l|X|psi>, Im<l|Y|psi>, Im<l|Z|psi> taken after the chain:
// Im<l|H|psi> with H = V P V^dagger, V = the later gates' product (row-major
// 2x2, interleaved re/im), P the gate's generator (axis 0 X, 1 Y, 2 Z).
// H is traceless Hermitian, H = H00 Z + Re(H01) X - Im(H01) Y.
__device__ double chain_grad(const float* V, int axis, double cx, double cy, double cz) {
    const double ar = V[0], ai = V[1], br = V[2], bi = V[3];  // v00, v01
    const double cr = V[4], ci = V[5], dr = V[6], di = V[7];  // v10, v11
    double h00, hr, hi;
    if (axis == 2) {         // V Z V^dagger
        h00 = ar * ar + ai * ai - br * br - bi * bi;
        hr = (ar * cr + ai * ci) - (br * dr + bi * di);   // v00 conj(v10) - v01 conj(v11)
        hi = (ai * cr - ar * ci) - (bi * dr - br * di);
    } else if (axis == 0) {  // V X V^dagger
        h00 = 2.0 * (ar * br + ai * bi);                  // 2 Re(v00 conj(v01))
        hr = (br * cr + bi * ci) + (ar * dr + ai * di);   // v01 conj(v10) + v00 conj(v11)
        hi = (bi * cr - br * ci) + (ai * dr - ar * di);
    } else {                 // V Y V^dagger
        h00 = -2.0 * (bi * ar - br * ai);                 // -2 Im(v01 conj(v00))
        const double ur = (br * cr + bi * ci) - (ar * dr + ai * di);  // v01 conj(v10) - v00 conj(v11)
        const double ui = (bi * cr - br * ci) - (ai * dr - ar * di);
        hr = -ui;                                          // i (ur + i ui)
        hi = ur;
    }
    return h00 * cz + hr * cx - hi * cy;
}

__device__ __forceinline__ void pass_bwd_tile(
    const DPass* __restrict__ P, const DStage* __restrict__ S, const DOp* __restrict__ O,
    const DTerm* __restrict__ Tm, const DGOut* __restrict__ gouts,
    const float* __restrict__ mats, int n_shared, int n_ps, const float2* __restrict__ psiN_s,
    float2* __restrict__ psi_s, float2* __restrict__ lam_s, const double* __restrict__ g, int W,
    int64_t B, int b, int64_t tis, double* __restrict__ part, const int64_t* __restrict__ pu,
    float2* lds) {
    const int m = P->m;
    const int t = threadIdx.x;
    const int nthr = 1 << (m - kRegBits);
    const bool act = t < nthr;
    const int nwaves = (int)(blockDim.x >> 6);
    const int waves_on = (nthr + 63) >> 6;  // waves holding at least one active lane
    const bool wave_on = (t >> 6) < waves_on;
    // float32 partials per 16-lane row and component slot, then float64 sums
    const int ng = P->n_gslots;
    const int nrows = nwaves * 4;
    const int nrows_on = waves_on * 4;
    float* red = reinterpret_cast<float*>(lds + (1 << m));
    double* csum = reinterpret_cast<double*>(lds + (1 << m) + ((nrows * ng + 1) >> 1));
    const int tbits = W - m;
    const int base = tile_base_of(P, tbits, tis);
    const int flags = P->flags;

    int cur[kRegBits] = {m - 4, m - 3, m - 2, m - 1};
    Lay L;
    make_layout(P, m, cur, t, base, L);
    float2 ps[kRegs], lm[kRegs];
    for (int k = 0; k < kRegs; ++k) ps[k] = lm[k] = make_float2(0.f, 0.f);
    if (act) {
        if (flags & PF_FIRST_BWD) {
            g_load(psiN_s, L, ps);
            // lambda = D psi, D(idx) = G0 - 2 sum_{i: bit_i = 1} g_i (additive over bits)
            double G0 = 0.0, DT = 0.0;
            for (int i = 0; i < W; ++i) {
                G0 += g[i];
                if ((L.gT >> (W - 1 - i)) & 1) DT += g[i];
            }
            double gp[kRegBits];
            for (int p = 0; p < kRegBits; ++p) gp[p] = g[W - 1 - P->lq[cur[p]]];
#pragma unroll
            for (int k = 0; k < kRegs; ++k) {
                double dr = DT;
                for (int p = 0; p < kRegBits; ++p)
                    if ((k >> p) & 1) dr += gp[p];
                const float d = (float)(G0 - 2.0 * dr);
                lm[k] = make_float2(d * ps[k].x, d * ps[k].y);
            }
        } else {
            g_load(psi_s, L, ps);
            g_load(lam_s, L, lm);
        }
    }
    const int wave = t >> 6, lane = t & 63;
    for (int s = 0; s < P->n_stages; ++s) {
        const DStage& stg = S[P->stage0 + s];
        if (!same_reg(cur, stg.reg)) {
            Lay Ln;
            for (int p = 0; p < kRegBits; ++p) cur[p] = stg.reg[p];
            make_layout(P, m, cur, t, base, Ln);
            if (act) lds_store(lds, L, ps);
            __syncthreads();
            if (act) lds_load(lds, Ln, ps);
            __syncthreads();
            if (act) lds_store(lds, L, lm);
            __syncthreads();
            if (act) lds_load(lds, Ln, lm);
            __syncthreads();
            L = Ln;
        }
        // waves without an active lane only keep the barrier count (wave-uniform
        // branch); their rows are left out of the sums below
        if (wave_on && stg.op0 < stg.op1) {
            // next op and matrix fetched while the current one is applied
            DOp op = O[stg.op0];
            M2 M = op_matrix(op, mats, b, n_shared, n_ps);
            for (int oi = stg.op0; oi < stg.op1; ++oi) {
                DOp nop = op;
                M2 nM = M;
                if (oi + 1 < stg.op1) {
                    nop = O[oi + 1];
                    nM = op_matrix(nop, mats, b, n_shared, n_ps);
                }
                if (op.kind >= OP_GX) {
                    // every lane of a row stores the row's sum (same value, same address)
                    red[(wave * 4 + (lane >> 4)) * ng + op.slot] = row_sum(grad_op(op, ps, lm, L.gT));
                } else {
                    apply_op<2>(op, ps, lm, M, L.gT, Tm);
                }
                op = nop;
                M = nM;
            }
        }
    }
    if (!(flags & PF_LAST_BWD)) {
        const int nat[kRegBits] = {m - 4, m - 3, m - 2, m - 1};
        if (!same_reg(cur, nat)) {
            Lay Ln;
            make_layout(P, m, nat, t, base, Ln);
            if (act) lds_store(lds, L, ps);
            __syncthreads();
            if (act) lds_load(lds, Ln, ps);
            __syncthreads();
            if (act) lds_store(lds, L, lm);
            __syncthreads();
            if (act) lds_load(lds, Ln, lm);
            L = Ln;
        }
        if (act) {
            g_store(psi_s, L, ps);
            g_store(lam_s, L, lm);
        }
    }
    __syncthreads();
    const int64_t nch = int64_t(1) << tbits;
    for (int j = t; j < ng; j += blockDim.x) {
        double s = 0.0;
        for (int r = 0; r < nrows_on; ++r) s += (double)red[r * ng + j];
        csum[j] = s;
    }
    __syncthreads();
    for (int j = t; j < P->n_gout; j += blockDim.x) {
        const DGOut o = gouts[P->gout0 + j];
        double v;
        if (o.axis < 0) {
            v = csum[o.c0];
        } else {
            const double cx = o.c0 >= 0 ? csum[o.c0] : 0.0, cy = o.c1 >= 0 ? csum[o.c1] : 0.0,
                         cz = o.c2 >= 0 ? csum[o.c2] : 0.0;
            v = chain_grad(mat_ptr(mats, o.mat, b, n_shared, n_ps), o.axis, cx, cy, cz);
        }
        part[B * pu[o.ord] + (int64_t)b * nch + tis] = v;
    }
    __syncthreads();  // red and lds may be reused by the caller's next tile
}

__global__ __launch_bounds__(1024) void k_pass_fwd(const DPass* __restrict__ P,
                                                   const DStage* __restrict__ S,
                                                   const DOp* __restrict__ O,
                                                   const DTerm* __restrict__ Tm,
                                                   const float* __restrict__ mats, int n_shared,
                                                   int n_ps, const int32_t* __restrict__ pm,
                                                   float2* __restrict__ state, int W) {
    extern __shared__ float2 lds[];
    const int tbits = W - P->m;
    const int64_t tile = blockIdx.x;
    const int b = (int)(tile >> tbits);
    const int64_t tis = tile & ((int64_t(1) << tbits) - 1);
    pass_fwd_tile(P, S, O, Tm, mats, n_shared, n_ps, pm, state + ((size_t)b << W), W, b, tis, lds);
}

__global__ __launch_bounds__(256) void k_pass_bwd(
    const DPass* __restrict__ P, const DStage* __restrict__ S, const DOp* __restrict__ O,
    const DTerm* __restrict__ Tm, const DGOut* __restrict__ gouts,
    const float* __restrict__ mats, int n_shared, int n_ps, const float2* __restrict__ psiN,
    float2* __restrict__ psi, float2* __restrict__ lam, const double* __restrict__ gout, int W,
    int B, double* __restrict__ part, const int64_t* __restrict__ pu) {
    extern __shared__ float2 lds[];
    const int tbits = W - P->m;
    const int64_t tile = blockIdx.x;
    const int b = (int)(tile >> tbits);
    const int64_t tis = tile & ((int64_t(1) << tbits) - 1);
    const size_t off = (size_t)b << W;
    pass_bwd_tile(P, S, O, Tm, gouts, mats, n_shared, n_ps, psiN + off, psi + off, lam + off,
                  gout + (size_t)b * W, W, B, b, tis, part, pu, lds);
}

// ----------------------------------------------------------------------------
// many circuits, one launch per round
// ----------------------------------------------------------------------------
// Round r holds tile items of pass r of every circuit that has one; workgroup
// i of the launch processes item i. Pass r + 1 of a circuit only starts in the
// next launch, so kernel boundaries order the passes; no workgroup waits on
// another.
__global__ __launch_bounds__(256) void k_multi_fwd(
    const DCirc* __restrict__ C, const DItem* __restrict__ Q,
    const DPass* __restrict__ passes, const DStage* __restrict__ S, const DOp* __restrict__ O,
    const DTerm* __restrict__ Tm, const float* __restrict__ mats, int n_shared, int n_ps,
    const int32_t* __restrict__ pm, float2* __restrict__ state, int64_t row) {
    extern __shared__ float2 lds[];
    const DItem I = Q[blockIdx.x];
    const DCirc& c = C[I.c];
    const int tbits = c.W - c.m;
    const int b = I.tile >> tbits;
    const int64_t tis = I.tile & ((1 << tbits) - 1);
    pass_fwd_tile(passes + c.fwd0 + I.pass, S, O, Tm, mats, n_shared, n_ps, pm + c.pm0,
                  state + (size_t)b * row + c.amp0, c.W, b, tis, lds);
}

__global__ __launch_bounds__(256) void k_multi_bwd(
    const DCirc* __restrict__ C, const DItem* __restrict__ Q,
    const DPass* __restrict__ passes, const DStage* __restrict__ S, const DOp* __restrict__ O,
    const DTerm* __restrict__ Tm, const DGOut* __restrict__ gouts,
    const float* __restrict__ mats, int n_shared, int n_ps, const float2* __restrict__ psiN,
    float2* __restrict__ psi, float2* __restrict__ lam, const double* __restrict__ gout, int Wtot,
    int64_t row, int B, double* __restrict__ part, const int64_t* __restrict__ pu) {
    extern __shared__ float2 lds[];
    const DItem I = Q[blockIdx.x];
    const DCirc& c = C[I.c];
    const int tbits = c.W - c.m;
    const int b = I.tile >> tbits;
    const int64_t tis = I.tile & ((1 << tbits) - 1);
    const size_t off = (size_t)b * row + c.amp0;
    pass_bwd_tile(passes + c.bwd0 + I.pass, S, O, Tm, gouts, mats, n_shared, n_ps, psiN + off,
                  psi + off, lam + off, gout + (size_t)b * Wtot + c.e0, c.W, B, b, tis, part, pu, lds);
}

// product-state init of every circuit: grid (sum of per-circuit chunks, B)
__global__ __launch_bounds__(256) void k_init_multi(const DCirc* __restrict__ C, int n_circ,
                                                    float2* __restrict__ state, int64_t row,
                                                    const int32_t* __restrict__ pm,
                                                    const float* __restrict__ mats, int n_shared,
                                                    int n_ps) {
    // find the circuit owning this chunk (chunk prefix in DCirc.ic0)
    int lo = 0, hi = n_circ - 1;
    const int x = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (C[mid].ic0 <= x) lo = mid; else hi = mid - 1;
    }
    const DCirc& c = C[lo];
    const int W = c.W;
    const int cb = min(W, 12), tb = min(cb, 8), jb = cb - tb;
    const int t = threadIdx.x;
    if (t >= (1 << tb)) return;
    const int b = blockIdx.y;
    const int64_t chunk = x - c.ic0;
    const int32_t* pmc = pm + c.pm0;
    float2 P = make_float2(1.f, 0.f);
    for (int s = 0; s < tb; ++s) P = cmul(P, prefix_v(mats, pmc, W - 1 - s, (t >> s) & 1, b, n_shared, n_ps));
    for (int s = cb; s < W; ++s)
        P = cmul(P, prefix_v(mats, pmc, W - 1 - s, (int)((chunk >> (s - cb)) & 1), b, n_shared, n_ps));
    float2* st = state + (size_t)b * row + c.amp0;
    for (int j = 0; j < (1 << jb); ++j) {
        float2 Q = P;
        for (int s = tb; s < cb; ++s)
            Q = cmul(Q, prefix_v(mats, pmc, W - 1 - s, (j >> (s - tb)) & 1, b, n_shared, n_ps));
        st[(chunk << cb) | ((int64_t)j << tb) | t] = Q;
    }
}

// readout of every circuit: grid (sum of per-circuit chunks, B); 32 doubles per chunk
__global__ __launch_bounds__(256) void k_expval_part_multi(const DCirc* __restrict__ C, int n_circ,
                                                           const float2* __restrict__ state,
                                                           int64_t row, int64_t nchunk_tot,
                                                           double* __restrict__ part) {
    __shared__ double red[4][14];
    int lo = 0, hi = n_circ - 1;
    const int x = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (C[mid].ic0 <= x) lo = mid; else hi = mid - 1;
    }
    const DCirc& c = C[lo];
    const int W = c.W;
    const int cb = min(W, 12), tb = min(cb, 8), jb = cb - tb;
    const int t = threadIdx.x;
    const int b = blockIdx.y;
    const int64_t chunk = x - c.ic0;
    const float2* st = state + (size_t)b * row + c.amp0;
    float T = 0.f, Sj[4] = {0.f, 0.f, 0.f, 0.f};
    if (t < (1 << tb)) {
        for (int j = 0; j < (1 << jb); ++j) {
            const float2 a = st[(chunk << cb) | ((int64_t)j << tb) | t];
            const float p = a.x * a.x + a.y * a.y;
            T += p;
            for (int i = 0; i < jb; ++i)
                if ((j >> i) & 1) Sj[i] += p;
        }
    }
    double v[13];
    v[0] = T;
    for (int i = 0; i < 4; ++i) v[1 + i] = Sj[i];
    for (int s = 0; s < 8; ++s) v[5 + s] = ((t >> s) & 1) ? (double)T : 0.0;
    const int wave = t >> 6, lane = t & 63;
    for (int k = 0; k < 13; ++k) {
        const double r = wave_sum(v[k]);
        if (lane == 0) red[wave][k] = r;
    }
    __syncthreads();
    if (t < W) {
        auto tot = [&](int k) { return red[0][k] + red[1][k] + red[2][k] + red[3][k]; };
        const int s = W - 1 - t;
        const double Tsum = tot(0);
        double e;
        if (s < tb) e = Tsum - 2.0 * tot(5 + s);
        else if (s < cb) e = Tsum - 2.0 * tot(1 + (s - tb));
        else e = ((chunk >> (s - cb)) & 1) ? -Tsum : Tsum;
        part[((size_t)b * nchunk_tot + x) * 32 + t] = e;
    }
}

// E[b, e0_c + i] = sum over circuit c's chunks; grid (total qubits, B)
__global__ __launch_bounds__(256) void k_expval_final_multi(const DCirc* __restrict__ C, int n_circ,
                                                            const double* __restrict__ part,
                                                            int64_t nchunk_tot, int Wtot,
                                                            double* __restrict__ out) {
    __shared__ double red[256];
    int lo = 0, hi = n_circ - 1;
    const int col = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (C[mid].e0 <= col) lo = mid; else hi = mid - 1;
    }
    const DCirc& c = C[lo];
    const int i = col - c.e0;
    const int b = blockIdx.y, t = threadIdx.x;
    double s = 0.0;
    for (int64_t k = t; k < c.nchunk; k += 256) s += part[((size_t)b * nchunk_tot + c.ic0 + k) * 32 + i];
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) out[(size_t)b * Wtot + col] = red[0];
}

// ----------------------------------------------------------------------------
// memory accesses of a fused pass alone (measurement aid)
// ----------------------------------------------------------------------------
// The global loads and stores of one generated pass kernel with nothing in
// between: the same tiles, 16 amplitudes per thread, register bits (tile bit 0
// when it is amplitude bit 0, else the fourth-highest tile bit, plus the top
// three), thread-index bits on the other tile bits in ascending order,
// 16-byte pairs when tile bit 0 is amplitude bit 0, and the XCD-contiguous
// block order. rd / wr: bit 0 array a, bit 1 array b (read from ra / rb,
// written to wa / wb; b takes a's values where b is not read). A thread reads
// all its amplitudes before it writes any, so ra may be wa and rb may be wb.
struct PassGeom {
    int32_t m, W, tb, pair;
    int32_t lq[kMaxQ];  // tile bit j -> amplitude bit
    int32_t oq[kMaxQ];  // tile-index bit k -> amplitude bit
};

__global__ __launch_bounds__(256) void k_pass_copy(const float2* ra, const float2* rb, float2* wa, float2* wb,
                                                   const PassGeom g, int rd, int wr) {
    const int t = threadIdx.x;
    if (t >= (1 << (g.m - kRegBits))) return;  // no barriers below
    const unsigned tile = (gridDim.x & 7u) ? blockIdx.x : (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const unsigned s = tile >> g.tb, tis = tile & ((1u << g.tb) - 1u);
    size_t base = (size_t)s << g.W;
    for (int k = 0; k < g.tb; ++k) base |= (size_t)((tis >> k) & 1u) << g.oq[k];
    const int r0 = g.pair ? 0 : g.m - 4;
    size_t gT = base;
    for (int j = 0, i = 0; j < g.m; ++j) {
        if (j == r0 || j >= g.m - 3) continue;
        gT |= (size_t)((t >> i) & 1) << g.lq[j];
        ++i;
    }
    const int s0 = g.lq[r0], s1 = g.lq[g.m - 3], s2 = g.lq[g.m - 2], s3 = g.lq[g.m - 1];
    float2 va[kRegs], vb[kRegs];
#pragma unroll
    for (int k = 0; k < kRegs; ++k) va[k] = vb[k] = make_float2(0.f, 0.f);
    // offset of register pair k, k + 1 (k even); array by array, like the passes
    auto off = [&](int k) {
        return gT + ((size_t)((k >> 1) & 1) << s1) + ((size_t)((k >> 2) & 1) << s2) + ((size_t)((k >> 3) & 1) << s3);
    };
    auto load = [&](const float2* x, float2 (&v)[kRegs]) {
#pragma unroll
        for (int k = 0; k < kRegs; k += 2) {
            const size_t o = off(k);
            if (g.pair) {
                const float4 q = *reinterpret_cast<const float4*>(x + o);
                v[k] = make_float2(q.x, q.y);
                v[k + 1] = make_float2(q.z, q.w);
            } else {
                v[k] = x[o];
                v[k + 1] = x[o + ((size_t)1 << s0)];
            }
        }
    };
    auto store = [&](float2* x, const float2 (&v)[kRegs]) {
#pragma unroll
        for (int k = 0; k < kRegs; k += 2) {
            const size_t o = off(k);
            if (g.pair) {
                *reinterpret_cast<float4*>(x + o) = make_float4(v[k].x, v[k].y, v[k + 1].x, v[k + 1].y);
            } else {
                x[o] = v[k];
                x[o + ((size_t)1 << s0)] = v[k + 1];
            }
        }
    };
    if (rd & 1) load(ra, va);
    if (rd & 2) load(rb, vb);
    else {
#pragma unroll
        for (int k = 0; k < kRegs; ++k) vb[k] = va[k];
    }
    if (!wr) {
        // keep the loads: their values feed an empty asm statement
#pragma unroll
        for (int k = 0; k < kRegs; ++k) __asm__ volatile("" ::"v"(va[k].x), "v"(va[k].y), "v"(vb[k].x), "v"(vb[k].y));
        return;
    }
    if (wr & 1) store(wa, va);
    if (wr & 2) store(wb, vb);
}

// ----------------------------------------------------------------------------
// host side: device tables
// ----------------------------------------------------------------------------
namespace {

// ---- profiling: event pairs around launches, per-kernel totals ----
enum KernelId { K_COEF, K_INIT, K_PASS_FWD, K_PASS_BWD, K_PG_APPLY, K_PG_ADJ, K_ADJ_INIT,
                K_EXPVAL_PART, K_EXPVAL_FINAL, K_GRAD_REDUCE, K_MULTI_FWD, K_MULTI_BWD, K_COUNT };
const char* const kKernelNames[K_COUNT] = {"k_coef", "k_init", "k_pass_fwd", "k_pass_bwd",
                                           "k_pg_apply", "k_pg_adj", "k_adj_init",
                                           "k_expval_part", "k_expval_final", "k_grad_reduce",
                                           "k_multi_fwd", "k_multi_bwd"};

struct ProfRec {
    int kid;
    int sub;  // pass index of a generated per-pass kernel, else -1
    hipEvent_t a, b;
    double bytes, flops;
};

struct Profiler {
    bool on = false;
    bool each = false;  // one entry per launch, in launch order
    std::mutex mu;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
};

Profiler* prof_of(const qsv_plan_t* p) { return static_cast<Profiler*>(p->prof); }

// Returns the start event (or nullptr when profiling is off).
hipEvent_t prof_begin(const qsv_plan_t* p, hipStream_t s) {
    Profiler* pr = prof_of(p);
    if (!pr || !pr->on || g_capturing || g_noalloc) return nullptr;
    std::lock_guard<std::mutex> lk(pr->mu);
    hipEvent_t e = nullptr;
    if (!pr->pool.empty()) { e = pr->pool.back(); pr->pool.pop_back(); }
    else if (hipEventCreate(&e) != hipSuccess) return nullptr;
    (void)hipEventRecord(e, s);
    return e;
}

void prof_end(const qsv_plan_t* p, hipStream_t s, hipEvent_t a, int kid, double bytes, double flops,
              int sub = -1) {
    if (!a) return;
    Profiler* pr = prof_of(p);
    std::lock_guard<std::mutex> lk(pr->mu);
    hipEvent_t b = nullptr;
    if (!pr->pool.empty()) { b = pr->pool.back(); pr->pool.pop_back(); }
    else if (hipEventCreate(&b) != hipSuccess) { pr->pool.push_back(a); return; }
    (void)hipEventRecord(b, s);
    pr->recs.push_back({kid, sub, a, b, bytes, flops});
}

template <class T>
size_t bytes_of(const std::vector<T>& v) { return v.size() * sizeof(T); }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int get_tables(const qsv_plan_t* p, DeviceTables** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(p->dev_mu);
    auto it = p->dev.find(dev);
    if (it != p->dev.end()) {
        *out = &it->second;
        return QSV_OK;
    }
    if (g_noalloc) {
        set_error("the plan has no tables on this device yet: an allocation-free call needs an earlier "
                  "call that creates them (any forward, readout or backward call on this device)");
        return QSV_ERR_ARG;
    }
    DeviceTables t;
    const size_t sizes[] = {bytes_of(p->dgates), bytes_of(p->recipes), bytes_of(p->recipe_gates),
                            bytes_of(p->fwd_pass), bytes_of(p->bwd_pass), bytes_of(p->stages),
                            bytes_of(p->ops), bytes_of(p->terms), bytes_of(p->gouts),
                            bytes_of(p->prefix_mat), bytes_of(p->grad_csr), bytes_of(p->pu),
                            bytes_of(p->nchv), bytes_of(p->circ)};
    const void* srcs[] = {p->dgates.data(), p->recipes.data(), p->recipe_gates.data(),
                          p->fwd_pass.data(), p->bwd_pass.data(), p->stages.data(),
                          p->ops.data(), p->terms.data(), p->gouts.data(),
                          p->prefix_mat.data(), p->grad_csr.data(), p->pu.data(), p->nchv.data(),
                          p->circ.data()};
    const int n = (int)(sizeof(sizes) / sizeof(sizes[0]));
    size_t total = 0, offs[16];
    for (int i = 0; i < n; ++i) { offs[i] = total; total += align256(std::max<size_t>(sizes[i], 1)); }
    char* host = (char*)std::calloc(total, 1);
    if (!host) { set_error("host allocation of plan tables failed"); return QSV_ERR_OOM; }
    for (int i = 0; i < n; ++i)
        if (sizes[i]) std::memcpy(host + offs[i], srcs[i], sizes[i]);
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, total);
    if (e != hipSuccess) {
        std::free(host);
        set_error(std::string("hipMalloc of plan tables: ") + hipGetErrorString(e));
        return QSV_ERR_OOM;
    }
    e = hipMemcpy(d, host, total, hipMemcpyHostToDevice);
    std::free(host);
    if (e != hipSuccess) {
        (void)hipFree(d);
        set_error(std::string("hipMemcpy of plan tables: ") + hipGetErrorString(e));
        return QSV_ERR_HIP;
    }
    char* c = (char*)d;
    t.base = d;
    t.gates = (DGate*)(c + offs[0]);
    t.recipes = (DRecipe*)(c + offs[1]);
    t.recipe_gates = (int32_t*)(c + offs[2]);
    t.fwd_pass = (DPass*)(c + offs[3]);
    t.bwd_pass = (DPass*)(c + offs[4]);
    t.stages = (DStage*)(c + offs[5]);
    t.ops = (DOp*)(c + offs[6]);
    t.terms = (DTerm*)(c + offs[7]);
    t.gouts = (DGOut*)(c + offs[8]);
    t.prefix_mat = (int32_t*)(c + offs[9]);
    t.grad_csr = (int32_t*)(c + offs[10]);
    t.pu = (int64_t*)(c + offs[11]);
    t.nchv = (int32_t*)(c + offs[12]);
    t.circ = (DCirc*)(c + offs[13]);
    if (p->opts.method == QSV_METHOD_FUSED && p->opts.codegen && !p->multi &&
        !(p->fwd_pass.empty() && p->bwd_pass.empty())) {
        JitModules jm;
        std::string err;
        int rc = jit_compile(p, "", jm, err);
        if (rc != QSV_OK) {
            (void)hipFree(d);
            set_error(err);
            return rc;
        }
        std::vector<hipModule_t> mods(jm.codes.size());
        for (size_t g = 0; g < jm.codes.size(); ++g) {
            hipError_t le = hipModuleLoadData(&mods[g], jm.codes[g].data());
            if (le != hipSuccess) {
                for (size_t h = 0; h < g; ++h) (void)hipModuleUnload(mods[h]);
                (void)hipFree(d);
                set_error(std::string("hipModuleLoadData: ") + hipGetErrorString(le));
                return QSV_ERR_HIP;
            }
            t.modules.push_back((void*)mods[g]);
        }
        t.fwd_fn.assign(p->fwd_pass.size(), nullptr);
        t.bwd_fn.assign(p->bwd_pass.size(), nullptr);
        for (const JitKernelRef& r : jm.refs) {
            hipFunction_t f = nullptr;
            hipError_t fe = hipModuleGetFunction(&f, mods[r.group], r.name.c_str());
            if (fe != hipSuccess) {
                for (auto m : mods) (void)hipModuleUnload(m);
                (void)hipFree(d);
                set_error("hipModuleGetFunction(" + r.name + "): " + hipGetErrorString(fe));
                return QSV_ERR_HIP;
            }
            (r.which == 0 ? t.fwd_fn : t.bwd_fn)[r.pass] = (void*)f;
        }
    }
    auto res = p->dev.emplace(dev, t);
    *out = &res.first->second;
    return QSV_OK;
}

// complex128 amplitudes (and float64 gate matrices) for the plain method's amp_dtype = 1
bool c128(const qsv_plan_t* p) { return p->opts.amp_dtype == QSV_AMP_C128; }
size_t amp_size(const qsv_plan_t* p) { return c128(p) ? 16 : 8; }

size_t mats_bytes(const qsv_plan_t* p, int64_t B) {
    return align256(((size_t)p->n_shared_mats + (size_t)B * p->n_ps_mats) * 8 * (amp_size(p) / 2) + 32);
}

int64_t grad_nch(const qsv_plan_t* p) {
    return p->opts.method == QSV_METHOD_PER_GATE ? pg_chunks(p->W)
                                                 : int64_t(1) << (p->W - std::min(p->opts.tile_qubits, p->W));
}

int64_t expval_nchunk(const qsv_plan_t* p) { return int64_t(1) << (p->W - std::min(p->W, 12)); }

// amplitudes of one sample (all circuits of a multi-circuit plan)
int64_t row_amps(const qsv_plan_t* p) { return p->multi ? p->row : int64_t(1) << p->W; }

size_t state_bytes(const qsv_plan_t* p, int64_t B) { return (size_t)B * (size_t)row_amps(p) * amp_size(p); }

// The backward's lambda copy starts this many bytes after psi's end, so that an
// amplitude of psi and the same amplitude of lambda (read and written together
// by every backward kernel) are not a power of two apart: per-gate adjoint
// 1-qubit class 0.668 -> 0.681 of 8 TB/s, fused passes unchanged.
constexpr size_t kLamSkew = 4096 + 256;

size_t partial_bytes(const qsv_plan_t* p, int64_t B) {
    return align256((size_t)std::max<int64_t>(p->pu_total, 1) * B * sizeof(double));
}



// Live handles: every plan and graph returned to a caller and not yet
// destroyed. A handle is checked by looking it up here, never by reading
// through it, so a destroyed (freed) handle is rejected without touching
// its memory. A new object that happens to reuse a destroyed one's address
// is live again: the registry cannot tell the two apart.
std::mutex g_handles_mu;
std::unordered_set<const void*> g_live_plans, g_live_graphs;

void handle_add(std::unordered_set<const void*>& set, const void* h) {
    std::lock_guard<std::mutex> lk(g_handles_mu);
    set.insert(h);
}
bool handle_live(const std::unordered_set<const void*>& set, const void* h) {
    std::lock_guard<std::mutex> lk(g_handles_mu);
    return h && set.count(h) != 0;
}
bool handle_remove(std::unordered_set<const void*>& set, const void* h) {
    std::lock_guard<std::mutex> lk(g_handles_mu);
    return h && set.erase(h) != 0;
}

int check_plan(const qsv_plan_t* p) {
    if (!handle_live(g_live_plans, p)) {
        set_error("null or destroyed plan");
        return QSV_ERR_HANDLE;
    }
    return QSV_OK;
}

int run_coef(const qsv_plan_t* p, DeviceTables* T, const float* w, const float* x, int64_t B,
             float* mats, hipStream_t s) {
    const int nr = (int)p->recipes.size();
    if (nr == 0) return QSV_OK;
    dim3 grid((nr + 127) / 128, (unsigned)(p->n_ps_mats ? B : 1));
    hipEvent_t ev = prof_begin(p, s);
    if (c128(p))
        hipLaunchKernelGGL(k_coef<double>, grid, dim3(128), 0, s, T->gates, T->recipes, T->recipe_gates, nr,
                           w, x, p->n_inputs, p->n_shared_mats, p->n_ps_mats, (int)p->opts.weight_remap,
                           (double*)mats);
    else
        hipLaunchKernelGGL(k_coef<float>, grid, dim3(128), 0, s, T->gates, T->recipes, T->recipe_gates, nr,
                           w, x, p->n_inputs, p->n_shared_mats, p->n_ps_mats, (int)p->opts.weight_remap, mats);
    prof_end(p, s, ev, K_COEF, 4.0 * (double)amp_size(p) * ((double)p->n_shared_mats + (double)B * p->n_ps_mats),
             0.0);
    HIP_TRY(hipGetLastError());
    return QSV_OK;
}

int run_init(const qsv_plan_t* p, DeviceTables* T, const float* mats, int64_t B, float2* st,
             hipStream_t s) {
    const int cb = std::min(p->W, 12);
    dim3 grid((unsigned)(int64_t(1) << (p->W - cb)), (unsigned)B);
    hipEvent_t ev = prof_begin(p, s);
    const int vec = ((uintptr_t)st & 15) == 0;
    if (c128(p))
        hipLaunchKernelGGL(k_init<double2>, grid, dim3(256), 0, s, (double2*)st, p->W, T->prefix_mat,
                           (const double*)mats, p->n_shared_mats, p->n_ps_mats, vec);
    else
        hipLaunchKernelGGL(k_init<float2>, grid, dim3(256), 0, s, st, p->W, T->prefix_mat, mats,
                           p->n_shared_mats, p->n_ps_mats, vec);
    const double amps = (double)B * (double)(int64_t(1) << p->W);
    prof_end(p, s, ev, K_INIT, (double)amp_size(p) * amps, 0.0);
    HIP_TRY(hipGetLastError());
    return QSV_OK;
}

int check_batch(const qsv_plan_t* p, int64_t B) {
    if (B <= 0) { set_error("batch must be positive"); return QSV_ERR_ARG; }
    if (B > 65535) { set_error("batch above 65535 is not supported"); return QSV_ERR_ARG; }
    if ((uint64_t)B * (uint64_t)row_amps(p) > (uint64_t(1) << 40)) { set_error("state too large"); return QSV_ERR_TOO_BIG; }
    // a tiled launch has one block per tile; HIP bounds its threads by 2^32
    const uint64_t kMaxGridThreads = 0xffffffffull;
    if (p->multi) {
        uint64_t tiles = 0;
        for (const DCirc& c : p->circ) {
            if ((B << (c.W - c.m)) > (int64_t(1) << 30)) { set_error("too many tiles"); return QSV_ERR_TOO_BIG; }
            tiles += (uint64_t)B << (c.W - c.m);
        }
        if (tiles * 256 > kMaxGridThreads) { set_error("too many tiles in one round"); return QSV_ERR_TOO_BIG; }
    } else if (p->opts.method != QSV_METHOD_PER_GATE) {
        const int m = std::min(p->opts.tile_qubits, p->W);
        const uint64_t threads = (uint64_t)std::max(64, 1 << (m - kRegBits));
        if (((uint64_t)B << (p->W - m)) * threads > kMaxGridThreads) {
            set_error("tile_qubits too small for this state size (tiles x threads above 2^32)");
            return QSV_ERR_TOO_BIG;
        }
    }
    // one gradient-reduction block per weight and per (sample, input)
    if ((uint64_t)p->n_weights + (uint64_t)B * (uint64_t)std::max(p->n_inputs, 0) > (uint64_t(1) << 24)) {
        set_error("more than 2^24 gradient outputs");
        return QSV_ERR_TOO_BIG;
    }
    return QSV_OK;
}

// Work list of one direction (dir 0 forward, 1 backward) of a multi-circuit
// plan at batch B, as rounds (one launch each): rounds[r] is round r's first
// item (and rounds.back() the item count). A circuit with k passes runs them
// in k consecutive rounds s, s+1, ..., s+k-1, so every item's predecessors
// (all tiles of its circuit's previous pass) are in the round before: the
// kernel boundary orders them and no workgroup waits on another. The start
// round s is chosen to balance the rounds: circuits in decreasing order of
// estimated work (tile amplitudes x (the pass's float32 operations per
// amplitude + 16, a byte-traffic allowance)) take the start that keeps the
// busiest of their rounds least loaded (earliest on ties), which fills the
// sparse late rounds with circuits that have fewer passes than the deepest
// one. Within a round the most expensive tiles come first.
void multi_items(const qsv_plan_t* p, int64_t B, int dir, std::vector<DItem>& items, std::vector<int>& rounds) {
    const int nc = (int)p->circ.size();
    auto npass = [&](const DCirc& c) { return dir ? c.n_bwd : c.n_fwd; };
    auto tile_cost = [&](const DCirc& c, int r) {
        const double fl = dir ? p->bwd_pass_flops[c.bwd0 + r] : p->fwd_pass_flops[c.fwd0 + r];
        return (double)(int64_t(1) << c.m) * (fl + 16.0);
    };
    auto ntiles = [&](const DCirc& c) { return (int)(B << (c.W - c.m)); };
    int R = 0;
    for (const DCirc& c : p->circ) R = std::max(R, npass(c));
    std::vector<double> total(nc, 0.0);
    for (int ci = 0; ci < nc; ++ci)
        for (int r = 0; r < npass(p->circ[ci]); ++r) total[ci] += ntiles(p->circ[ci]) * tile_cost(p->circ[ci], r);
    std::vector<int> order(nc);
    for (int i = 0; i < nc; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return total[a] > total[b]; });
    std::vector<double> load(R, 0.0);
    std::vector<int> start(nc, 0);
    for (int ci : order) {
        const DCirc& c = p->circ[ci];
        const int k = npass(c);
        int best = 0;
        double best_max = 0.0;
        for (int s0 = 0; s0 + k <= R; ++s0) {
            double mx = 0.0;
            for (int j = 0; j < k; ++j) mx = std::max(mx, load[s0 + j] + ntiles(c) * tile_cost(c, j));
            if (s0 == 0 || mx < best_max) { best = s0; best_max = mx; }
        }
        start[ci] = best;
        for (int j = 0; j < k; ++j) load[best + j] += ntiles(c) * tile_cost(c, j);
    }
    for (int r = 0; r < R; ++r) {
        rounds.push_back((int)items.size());
        std::vector<std::pair<double, int>> in;  // (tile cost, circuit) of the circuits with a pass in round r
        for (int ci = 0; ci < nc; ++ci) {
            const int j = r - start[ci];
            if (j >= 0 && j < npass(p->circ[ci])) in.emplace_back(tile_cost(p->circ[ci], j), ci);
        }
        std::stable_sort(in.begin(), in.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
            return a.first > b.first;
        });
        for (const auto& e : in) {
            const DCirc& c = p->circ[e.second];
            for (int t = 0; t < ntiles(c); ++t) items.push_back({e.second, r - start[e.second], t, {0, 0, 0}});
        }
    }
    rounds.push_back((int)items.size());
}

// Work lists of the multi-circuit launches for batch B (built once per device
// and batch size, see multi_items).
int get_queue(const qsv_plan_t* p, DeviceTables* T, int64_t B, DeviceTables::Queue** out) {
    std::lock_guard<std::mutex> lk(p->dev_mu);
    for (auto& q : T->queues)
        if (q.B == B) { *out = &q; return QSV_OK; }
    if (g_noalloc) {
        set_error("the multi-circuit plan has no work lists for this batch size on this device yet: an "
                  "allocation-free call needs an earlier call at this batch size");
        return QSV_ERR_ARG;
    }
    std::vector<DItem> items[2];
    std::vector<int> rounds[2];
    for (int dir = 0; dir < 2; ++dir) multi_items(p, B, dir, items[dir], rounds[dir]);
    const size_t b0 = items[0].size() * sizeof(DItem), b1 = items[1].size() * sizeof(DItem);
    void* d = nullptr;
    if (hipMalloc(&d, std::max<size_t>(align256(b0) + b1, 256)) != hipSuccess) {
        set_error("hipMalloc of work lists failed");
        return QSV_ERR_OOM;
    }
    if ((b0 && hipMemcpy(d, items[0].data(), b0, hipMemcpyHostToDevice) != hipSuccess) ||
        (b1 && hipMemcpy((char*)d + align256(b0), items[1].data(), b1, hipMemcpyHostToDevice) != hipSuccess)) {
        (void)hipFree(d);
        set_error("hipMemcpy of work lists failed");
        return QSV_ERR_HIP;
    }
    DeviceTables::Queue q;
    q.B = B;
    q.fwd = (DItem*)d;
    q.n_fwd = (int)items[0].size();
    q.bwd = (DItem*)((char*)d + align256(b0));
    q.n_bwd = (int)items[1].size();
    q.mem = d;
    q.fwd_rounds = rounds[0];
    q.bwd_rounds = rounds[1];
    T->queues.push_back(q);
    *out = &T->queues.back();
    return QSV_OK;
}

// Backward LDS: the tile (8 B per amplitude), float32 row partials
// [rows][slots], then float64 component sums (8-byte aligned).
size_t bwd_lds(int m, int threads, int maxg) {
    const size_t rows = (size_t)(threads / 64) * 4;
    const size_t part = ((rows * maxg + 1) / 2) * 8;
    return (size_t(1) << m) * 8 + part + (size_t)maxg * 8;
}

size_t multi_lds(const qsv_plan_t* p) {
    int maxg = 0;
    for (auto& ps : p->bwd_pass) maxg = std::max(maxg, (int)ps.n_gslots);
    return bwd_lds(kMaxTileQubitsTables, 256, maxg);
}



// Block order of a per-gate launch. When the states exceed the 256 MB
// Infinity Cache, pair kernels alternate between ascending and descending
// order from gate to gate, so that a sweep starts where the previous one
// ended, on lines it has just written (20 qubits at batch 64, 512 MiB: dense
// 1-qubit classes 0.68 -> 0.70 of the HBM peak in the adjoint and 0.70 ->
// 0.74 in the forward). Single-stream sweeps (diagonal gates, sign flips
// over the whole state) always ascend, and so does everything on states that
// fit the cache (16 qubits at batch 256 lost 1% with alternation).
int pg_reverse(const PGate& pg, int vmode, size_t i, int64_t state_bytes) {
    if (state_bytes <= (int64_t(256) << 20) || pg.cls == OP_DIAG || vmode == PG_VEC_SWEEP) return 0;
    return (int)((i + 1) & 1);
}

// Per-gate launches: index bits fixed per item (target + controls, or the
// qubits of a sign flip) and the fraction of the amplitudes a gate changes.
int pg_fixed_bits(const PGate& g) {
    const int nctl = (g.csh >= 0) + (g.csh2 >= 0);
    return g.cls == OP_SIGN ? 2 + (g.csh2 >= 0) : 1 + nctl;
}

double pg_touched(const PGate& g) {
    const int nctl = (g.csh >= 0) + (g.csh2 >= 0);
    if (g.cls == OP_SIGN) return 1.0 / (double)(1 << pg_fixed_bits(g));
    return 1.0 / (double)(1 << nctl);
}

// profiling class of a per-gate launch: 0 dense 1-qubit, 1 diagonal, 2 controlled
// (half or a quarter of the pairs), 3 sign (CZ / Z / CCZ on a fraction of the state)
int pg_prof_class(const PGate& g) {
    if (g.cls == OP_SIGN) return 3;
    if (g.csh >= 0 || g.csh2 >= 0) return 2;
    return g.cls == OP_DIAG ? 1 : 0;
}
constexpr int kPgSub0 = 1000;  // profiler sub-key offset of the per-gate classes

// 16-byte access mode of a per-gate launch on `state` (PG_VEC_*; PG_SCALAR
// for complex128 states, states not 16-byte aligned, or a fixed bit 0 that is
// not a pair's target)
int pg_vec_mode(const qsv_plan_t* p, const PGate& g, const void* state) {
    if (c128(p) || ((uintptr_t)state & 15)) return PG_SCALAR;
    if (g.cls == OP_DIAG) return PG_VEC_PAIRS;
    int lo = 64;
    for (int sh : {g.tsh, g.cls == OP_SIGN ? g.sh2 : g.csh, g.csh2})
        if (sh >= 0) lo = std::min(lo, sh);
    if (g.cls == OP_SIGN && lo <= 2) return PG_VEC_SWEEP;
    if (lo >= 1) return PG_VEC_PAIRS;
    if (g.tsh == 0) return PG_VEC_ADJ;
    return PG_SCALAR;
}
const char* const kPgClassNames[4] = {"1q", "diag", "ctl", "sign"};

size_t pass_lds_fwd(const qsv_plan_t* p) {
    const int m = std::min(p->opts.tile_qubits, p->W);
    return (size_t(1) << m) * 8;
}

size_t pass_lds_bwd(const qsv_plan_t* p) {
    const int m = std::min(p->opts.tile_qubits, p->W);
    const int threads = std::max(64, 1 << (m - kRegBits));
    int maxg = 0;
    for (auto& ps : p->bwd_pass) maxg = std::max(maxg, (int)ps.n_gslots);
    return bwd_lds(m, threads, maxg);
}

}  // namespace

// ----------------------------------------------------------------------------
// C ABI
// ----------------------------------------------------------------------------
extern "C" {

const char* qsv_strerror(int code) {
    switch (code) {
    case QSV_OK: return "ok";
    case QSV_ERR_ARG: return "invalid argument";
    case QSV_ERR_QUBIT: return "qubit index out of range or repeated";
    case QSV_ERR_GATE: return "unknown gate kind";
    case QSV_ERR_PARAM: return "invalid angle source or index";
    case QSV_ERR_TOO_BIG: return "circuit or state too large";
    case QSV_ERR_OOM: return "out of memory";
    case QSV_ERR_HIP: return "HIP runtime error";
    case QSV_ERR_HANDLE: return "invalid plan handle";
    default: return "unknown error";
    }
}

const char* qsv_last_error(void) { return g_last_error.c_str(); }

void qsv_default_opts(qsv_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->method = QSV_METHOD_FUSED;
    o->fuse_width = 1;
    o->tile_qubits = 12;
    o->low_qubits = 4;
    o->max_pass_grads = 256;
    o->codegen = 1;
    o->mfma = 1;
    o->pack_beam = 16;
}

int qsv_plan(int32_t n_qubits, const qsv_gate* gates, int32_t n_gates, int32_t n_weights,
             int32_t n_inputs, const qsv_opts* opts, qsv_plan_t** out) {
    TraceRange trace_("qsv_plan");
    if (!out) { set_error("out is NULL"); return QSV_ERR_ARG; }
    *out = nullptr;
    if (n_qubits < 1) { set_error("n_qubits must be >= 1"); return QSV_ERR_ARG; }
    if (n_qubits > QSV_MAX_QUBITS) { set_error("n_qubits above QSV_MAX_QUBITS"); return QSV_ERR_TOO_BIG; }
    if (n_gates < 0 || n_weights < 0 || n_inputs < 0) { set_error("negative count"); return QSV_ERR_ARG; }
    if (n_gates > 0 && !gates) { set_error("gates is NULL"); return QSV_ERR_ARG; }
    qsv_opts o;
    qsv_default_opts(&o);
    if (opts) o = *opts;
    if (o.method != QSV_METHOD_FUSED && o.method != QSV_METHOD_PER_GATE) { set_error("bad method"); return QSV_ERR_ARG; }
    if (o.codegen != 0 && o.codegen != 1) { set_error("codegen must be 0 or 1"); return QSV_ERR_ARG; }
    if (o.fuse_width < 1 || o.fuse_width > 16) { set_error("fuse_width must be in 1..16"); return QSV_ERR_ARG; }
    if (o.tile_qubits < kRegBits || o.tile_qubits > kMaxTileQubits) { set_error("tile_qubits must be in 4..14"); return QSV_ERR_ARG; }
    if (o.codegen == 0 && o.tile_qubits > kMaxTileQubitsTables) { set_error("table-driven kernels (codegen 0) need tile_qubits <= 12"); return QSV_ERR_ARG; }
    if (o.low_qubits < 0 || o.low_qubits >= o.tile_qubits) { set_error("low_qubits must be in 0..tile_qubits-1"); return QSV_ERR_ARG; }
    if (o.max_pass_grads < 1 || o.max_pass_grads > 256) { set_error("max_pass_grads must be in 1..256"); return QSV_ERR_ARG; }
    if (o.bwd_gate_by_gate != 0 && o.bwd_gate_by_gate != 1) { set_error("bwd_gate_by_gate must be 0 or 1"); return QSV_ERR_ARG; }
    if (o.mfma < 0 || o.mfma > 7) { set_error("mfma must be in 0..7"); return QSV_ERR_ARG; }
    if (o.weight_remap != 0 && o.weight_remap != 1) { set_error("weight_remap must be 0 or 1"); return QSV_ERR_ARG; }
    if (o.splitter != 0 && o.splitter != 1) { set_error("splitter must be 0 or 1"); return QSV_ERR_ARG; }
    if (o.pack_beam < 0 || o.pack_beam > 256) { set_error("pack_beam must be in 0..256"); return QSV_ERR_ARG; }
    if (o.amp_dtype != QSV_AMP_C64 && o.amp_dtype != QSV_AMP_C128) { set_error("amp_dtype must be 0 or 1"); return QSV_ERR_ARG; }
    if (o.amp_dtype == QSV_AMP_C128 && o.method != QSV_METHOD_PER_GATE) {
        set_error("complex128 amplitudes (amp_dtype = 1) need method = per_gate");
        return QSV_ERR_ARG;
    }
    for (int g = 0; g < n_gates; ++g) {
        const qsv_gate& G = gates[g];
        char buf[160];
        if (G.kind < QSV_H || G.kind > QSV_CCRX) {
            std::snprintf(buf, sizeof buf, "gate %d: unknown kind %d", g, G.kind);
            set_error(buf);
            return QSV_ERR_GATE;
        }
        const int nq = 1 + (G.kind == QSV_CNOT || G.kind == QSV_CZ || G.kind == QSV_CRX ||
                            G.kind == QSV_CRY || G.kind == QSV_CRZ)
                     + 2 * (G.kind == QSV_CCX || G.kind == QSV_CCZ || G.kind == QSV_CCRX);
        const int qs[3] = {G.q0, G.q1, G.q2};
        bool ok = true;
        for (int i = 0; i < nq; ++i) {
            ok &= qs[i] >= 0 && qs[i] < n_qubits;
            for (int j = 0; j < i; ++j) ok &= qs[i] != qs[j];
        }
        if (!ok) {
            std::snprintf(buf, sizeof buf, "gate %d: qubits (%d, %d, %d) invalid for W = %d", g, G.q0, G.q1,
                          G.q2, n_qubits);
            set_error(buf);
            return QSV_ERR_QUBIT;
        }
        const bool param = G.kind == QSV_RX || G.kind == QSV_RY || G.kind == QSV_RZ || G.kind == QSV_CRX ||
                           G.kind == QSV_CRY || G.kind == QSV_CRZ || G.kind == QSV_CCRX;
        const bool ok_src = param ? (G.src == QSV_SRC_WEIGHT || G.src == QSV_SRC_INPUT) : G.src == QSV_SRC_NONE;
        const bool ok_idx = G.src == QSV_SRC_WEIGHT ? (G.idx >= 0 && G.idx < n_weights)
                          : G.src == QSV_SRC_INPUT ? (G.idx >= 0 && G.idx < n_inputs) : true;
        if (!ok_src || !ok_idx) {
            std::snprintf(buf, sizeof buf, "gate %d: angle source %d / index %d invalid", g, G.src, G.idx);
            set_error(buf);
            return QSV_ERR_PARAM;
        }
    }
    qsv_plan_t* p = new (std::nothrow) qsv_plan_t();
    if (!p) { set_error("plan allocation failed"); return QSV_ERR_OOM; }
    p->W = n_qubits;
    p->n_gates = n_gates;
    p->n_weights = n_weights;
    p->n_inputs = n_inputs;
    if (o.method == QSV_METHOD_FUSED && n_qubits < kRegBits) o.method = QSV_METHOD_PER_GATE;
    p->opts = o;
    p->gates.assign(gates, gates + n_gates);
    int rc;
    try {
        rc = build_plan(p);
    } catch (const std::bad_alloc&) {
        rc = QSV_ERR_OOM;
        set_error("out of host memory while planning");
    }
    if (rc != QSV_OK) {
        delete p;
        return rc;
    }
    handle_add(g_live_plans, p);
    *out = p;
    return QSV_OK;
}

void qsv_plan_destroy(qsv_plan_t* p) {
    if (!handle_remove(g_live_plans, p)) return;  // NULL, destroyed or never a plan
    // no HIP call at all for a plan that never ran on a device: a host-only
    // user of the library must not initialise the HIP runtime (in a process
    // where another HIP runtime, such as the one bundled with PyTorch, has not
    // opened the GPU yet, that can leave the GPU unusable for the other one)
    if (!p->dev.empty()) {
        int cur = 0;
        const bool have = hipGetDevice(&cur) == hipSuccess;
        for (auto& kv : p->dev) {
            if (hipSetDevice(kv.first) == hipSuccess) {
                for (void* m : kv.second.modules) (void)hipModuleUnload((hipModule_t)m);
                for (auto& q : kv.second.queues) (void)hipFree(q.mem);
                (void)hipFree(kv.second.base);
            }
        }
        if (have) (void)hipSetDevice(cur);
    }
    if (Profiler* pr = prof_of(p)) {
        for (auto& r : pr->recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto e : pr->pool) (void)hipEventDestroy(e);
        delete pr;
    }
    delete p;
}

int qsv_plan_get_info(const qsv_plan_t* p, qsv_plan_info* info) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!info) { set_error("info is NULL"); return QSV_ERR_ARG; }
    std::memset(info, 0, sizeof *info);
    info->n_qubits = p->W;
    info->n_gates = p->n_gates;
    info->n_weights = p->n_weights;
    info->n_inputs = p->n_inputs;
    info->method = p->opts.method;
    info->fuse_width = p->opts.fuse_width;
    info->tile_qubits = std::min(p->opts.tile_qubits, p->W);
    info->low_qubits = p->opts.low_qubits;
    info->n_prefix_gates = (int32_t)p->prefix_gates.size();
    info->n_blocks = (int32_t)p->blocks.size();
    if (p->opts.method == QSV_METHOD_PER_GATE) {
        info->n_fwd_passes = (int32_t)p->pg_fwd.size();
        info->n_bwd_passes = (int32_t)p->pg_bwd.size();
    } else {
        info->n_fwd_passes = (int32_t)p->fwd_pass.size();
        info->n_bwd_passes = (int32_t)p->bwd_pass.size();
    }
    info->n_fwd_stages = p->n_fwd_stages;
    info->n_bwd_stages = p->n_bwd_stages;
    info->n_param_gates = p->n_param;
    info->n_recipes = (int32_t)p->recipes.size();
    info->n_circuits = p->multi ? (int32_t)p->circ.size() : 1;
    if (p->multi) info->n_qubits = p->Wtot;
    return QSV_OK;
}

int qsv_plan_gate_order(const qsv_plan_t* p, int32_t which, int32_t* order) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!order || (which != 0 && which != 1)) { set_error("bad arguments"); return QSV_ERR_ARG; }
    const auto& v = which == 0 ? p->fwd_order : p->bwd_order;
    std::copy(v.begin(), v.end(), order);
    return QSV_OK;
}

int qsv_plan_gate_blocks(const qsv_plan_t* p, int32_t* block_of_gate) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!block_of_gate) { set_error("block_of_gate is NULL"); return QSV_ERR_ARG; }
    std::copy(p->block_of_gate.begin(), p->block_of_gate.end(), block_of_gate);
    return QSV_OK;
}

size_t qsv_workspace_size(const qsv_plan_t* p, int64_t B, int32_t op) {
    if (check_plan(p) || B <= 0) return 0;
    switch (op) {
    case QSV_OP_FORWARD: return mats_bytes(p, B);
    case QSV_OP_EXPVAL:
        if (p->multi) return align256((size_t)B * p->nchunk_tot * 32 * sizeof(double));
        return align256((size_t)B * expval_nchunk(p) * p->W * sizeof(double));
    case QSV_OP_BACKWARD:
        return mats_bytes(p, B) + 2 * align256(state_bytes(p, B)) + kLamSkew + partial_bytes(p, B);
    case QSV_OP_STEP:
        return std::max(qsv_workspace_size(p, B, QSV_OP_BACKWARD), qsv_workspace_size(p, B, QSV_OP_FORWARD_EXPVAL));
    case QSV_OP_FORWARD_EXPVAL: {
        // forward matrices, then readout partials: per generated tile (fused
        // readout) or per readout chunk, whichever is more
        size_t part = qsv_workspace_size(p, B, QSV_OP_EXPVAL);
        if (!p->multi)
            part = std::max(part, align256((size_t)B * ((size_t)1 << (p->W - std::min(p->opts.tile_qubits, p->W))) *
                                           p->W * sizeof(double)));
        return mats_bytes(p, B) + part;
    }
    default: return 0;
    }
}

// true when the last generated forward kernel can write the readout partials
// itself: fused method, generated kernels, at least one pass
static bool fused_readout(const qsv_plan_t* p, const DeviceTables* T) {
    return !p->multi && p->opts.method != QSV_METHOD_PER_GATE && !T->fwd_fn.empty() && !p->fwd_pass.empty();
}

// Forward over validated arguments. epart (used only when fused_readout())
// receives the per-tile readout partials [b][tile][i] of the final state.
static int forward_impl(const qsv_plan_t* p, const float* w, const float* x, int64_t B, void* d_state,
                        void* ws, hipStream_t s, DeviceTables* T, double* epart) {
    int rc;
    float* mats = (float*)ws;
    float2* st = (float2*)d_state;
    if ((rc = run_coef(p, T, w, x, B, mats, s))) return rc;
    if (p->multi) {
        DeviceTables::Queue* Q;
        if ((rc = get_queue(p, T, B, &Q))) return rc;
        const double amps = (double)B * (double)p->row;
        // each circuit's first pass builds its product state, unless a
        // circuit has no forward pass at all
        bool all_init = true;
        for (const DCirc& c : p->circ)
            all_init = all_init && c.n_fwd > 0 && (p->fwd_pass[c.fwd0].flags & PF_INIT_FWD);
        hipEvent_t ev;
        if (!all_init) {
            ev = prof_begin(p, s);
            hipLaunchKernelGGL(k_init_multi, dim3((unsigned)p->nchunk_tot, (unsigned)B), dim3(256), 0, s,
                               (const DCirc*)T->circ, (int)p->circ.size(), st, p->row, T->prefix_mat,
                               (const float*)mats, p->n_shared_mats, p->n_ps_mats);
            prof_end(p, s, ev, K_INIT, 8.0 * amps, 0.0);
        }
        double flops = 0.0, bytes = 0.0;
        for (const DCirc& c : p->circ)
            for (int r = 0; r < c.n_fwd; ++r) {
                flops += p->fwd_pass_flops[c.fwd0 + r] * (double)B * (double)(int64_t(1) << c.W);
                const bool init = p->fwd_pass[c.fwd0 + r].flags & PF_INIT_FWD;
                bytes += (init ? 8.0 : 16.0) * (double)B * (double)(int64_t(1) << c.W);
            }
        ev = prof_begin(p, s);
        for (size_t r = 0; r + 1 < Q->fwd_rounds.size(); ++r) {
            const int i0 = Q->fwd_rounds[r], n = Q->fwd_rounds[r + 1] - i0;
            hipLaunchKernelGGL(k_multi_fwd, dim3((unsigned)n), dim3(256), multi_lds(p), s,
                               (const DCirc*)T->circ, (const DItem*)(Q->fwd + i0), (const DPass*)T->fwd_pass,
                               (const DStage*)T->stages, (const DOp*)T->ops, (const DTerm*)T->terms,
                               (const float*)mats, p->n_shared_mats, p->n_ps_mats, T->prefix_mat, st, p->row);
        }
        prof_end(p, s, ev, K_MULTI_FWD, bytes, flops);
        HIP_TRY(hipGetLastError());
        return QSV_OK;
    }
    // fused passes (generated or table-driven) build the product state in
    // their first pass
    const bool fused_init = p->opts.method != QSV_METHOD_PER_GATE && !p->fwd_pass.empty() &&
                            (p->fwd_pass[0].flags & PF_INIT_FWD);
    if (!fused_init && (rc = run_init(p, T, mats, B, st, s))) return rc;
    const int W = p->W;
    const double amps = (double)B * (double)(int64_t(1) << W);
    if (p->opts.method == QSV_METHOD_PER_GATE) {
        for (size_t i = 0; i < p->pg_fwd.size(); ++i) {
            const PGate& pg = p->pg_fwd[i];
            int64_t items;
            const double touched = pg_touched(pg);  // fraction of the amplitudes the gate changes
            const int nfix = pg_fixed_bits(pg);
            if (pg.cls == OP_DIAG) items = B << W;
            else items = B << (W - nfix);
            const int64_t blocks = (items + 256 * kPgItems - 1) / (256 * kPgItems);
            hipEvent_t ev = prof_begin(p, s);
            const int vmode = pg_vec_mode(p, pg, st);
            if (vmode != PG_SCALAR) {
                // one item per thread: two amplitudes (diagonal), two pairs (PAIRS) or one pair (ADJ)
                const int64_t vitems = (pg.cls == OP_DIAG || vmode == PG_VEC_SWEEP) ? (B << W) / 2
                                     : vmode == PG_VEC_ADJ ? (B << (W - nfix)) : (B << (W - nfix)) / 2;
                hipLaunchKernelGGL(k_pg_apply_vec, grid_1d((vitems + 255) / 256), dim3(256), 0, s, st, W,
                                   vitems, pg, vmode, (const float*)mats, p->n_shared_mats, p->n_ps_mats,
                                   pg_reverse(pg, vmode, i, (int64_t)state_bytes(p, B)));
            } else if (c128(p)) {
                hipLaunchKernelGGL(k_pg_apply<double2>, grid_1d(blocks), dim3(256), 0, s, (double2*)st, W,
                                   B, pg, (const double*)mats, p->n_shared_mats, p->n_ps_mats);
            } else {
                hipLaunchKernelGGL(k_pg_apply<float2>, grid_1d(blocks), dim3(256), 0, s, st, W, B, pg,
                                   (const float*)mats, p->n_shared_mats, p->n_ps_mats);
            }
            prof_end(p, s, ev, K_PG_APPLY, 2.0 * (double)amp_size(p) * touched * amps, p->pg_fwd_flops[i] * amps,
                     kPgSub0 + pg_prof_class(pg));
        }
        HIP_TRY(hipGetLastError());
        return QSV_OK;
    }
    const int m = std::min(p->opts.tile_qubits, W);
    const unsigned threads = (unsigned)std::max(64, 1 << (m - kRegBits));
    const unsigned tiles = (unsigned)(B << (W - m));
    const size_t lds = pass_lds_fwd(p);
    for (size_t i = 0; i < p->fwd_pass.size(); ++i) {
        hipEvent_t ev = prof_begin(p, s);
        if (!T->fwd_fn.empty()) {
            int ns = p->n_shared_mats, np = p->n_ps_mats;
            const float* mp = mats;
            double* ep = epart;
            void* args[] = {&st, &mp, &ns, &np, &ep};  // the last pass takes the readout pointer
            HIP_TRY(hipModuleLaunchKernel((hipFunction_t)T->fwd_fn[i], tiles, 1, 1, threads, 1, 1, 0,
                                          s, args, nullptr));
        } else {
            hipLaunchKernelGGL(k_pass_fwd, dim3(tiles), dim3(threads), lds, s, T->fwd_pass + i,
                               T->stages, T->ops, T->terms, (const float*)mats, p->n_shared_mats,
                               p->n_ps_mats, T->prefix_mat, st, W);
        }
        // a first pass that builds the initial state reads nothing; a last pass
        // with the readout adds its partials
        double bytes = (fused_init && i == 0 ? 8.0 : 16.0) * amps;
        if (epart && i + 1 == p->fwd_pass.size()) bytes += 8.0 * (double)tiles * W;
        prof_end(p, s, ev, K_PASS_FWD, bytes, p->fwd_pass_flops[i] * amps, T->fwd_fn.empty() ? -1 : (int)i);
    }
    HIP_TRY(hipGetLastError());
    return QSV_OK;
}

int qsv_forward(const qsv_plan_t* p, const float* w, const float* x, int64_t B, void* d_state,
                void* ws, size_t ws_bytes, void* stream) {
    TraceRange trace_("qsv_forward");
    int rc = check_plan(p);
    if (rc) return rc;
    if ((rc = check_batch(p, B))) return rc;
    if (!d_state || (p->n_weights && !w) || (p->n_inputs && !x)) { set_error("null pointer"); return QSV_ERR_ARG; }
    const size_t need = qsv_workspace_size(p, B, QSV_OP_FORWARD);
    if (!ws || ws_bytes < need) { set_error("forward workspace too small"); return QSV_ERR_ARG; }
    DeviceTables* T;
    if ((rc = get_tables(p, &T))) return rc;
    return forward_impl(p, w, x, B, d_state, ws, (hipStream_t)stream, T, nullptr);
}

int qsv_forward_expval(const qsv_plan_t* p, const float* w, const float* x, int64_t B, void* d_state,
                       double* out, void* ws, size_t ws_bytes, void* stream) {
    TraceRange trace_("qsv_forward_expval");
    int rc = check_plan(p);
    if (rc) return rc;
    if ((rc = check_batch(p, B))) return rc;
    if (!d_state || !out || (p->n_weights && !w) || (p->n_inputs && !x)) {
        set_error("null pointer");
        return QSV_ERR_ARG;
    }
    const size_t need = qsv_workspace_size(p, B, QSV_OP_FORWARD_EXPVAL);
    if (!ws || ws_bytes < need) { set_error("forward_expval workspace too small"); return QSV_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    DeviceTables* T;
    if ((rc = get_tables(p, &T))) return rc;
    const size_t fwd_bytes = qsv_workspace_size(p, B, QSV_OP_FORWARD);
    char* wsc = (char*)ws;
    if (!fused_readout(p, T)) {
        rc = forward_impl(p, w, x, B, d_state, ws, s, T, nullptr);
        if (!rc) rc = qsv_expval(p, d_state, B, out, wsc + fwd_bytes, ws_bytes - fwd_bytes, stream);
        return rc;
    }
    double* part = (double*)(wsc + fwd_bytes);
    if ((rc = forward_impl(p, w, x, B, d_state, ws, s, T, part))) return rc;
    const int64_t ntiles = int64_t(1) << (p->W - std::min(p->opts.tile_qubits, p->W));
    hipEvent_t ev = prof_begin(p, s);
    hipLaunchKernelGGL(k_expval_final, dim3((unsigned)p->W, (unsigned)B), dim3(256), 0, s, (const double*)part,
                       p->W, ntiles, out);
    prof_end(p, s, ev, K_EXPVAL_FINAL, 8.0 * (double)B * ntiles * p->W, 0.0);
    HIP_TRY(hipGetLastError());
    return QSV_OK;
}

// The workspace of qsv_forward_expval_noalloc: a file-scope device array,
// one copy per GPU, created with the library's code object on that GPU and
// held until the process ends. In host code `scratch` names a host-side
// stand-in, so its device address is looked up once per device (with that
// device current) and only that address is ever passed on.
static __device__ __align__(256) unsigned char scratch[QSV_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;

static int scratch_address(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return QSV_ERR_HIP;
        }
        it = g_scratch_ptr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return QSV_OK;
}

int qsv_forward_expval_noalloc(const qsv_plan_t* p, const float* w, const float* x, int64_t B, void* d_state,
                               double* out, void* stream) {
    int rc = check_plan(p);
    if (rc) return rc;
    if ((rc = check_batch(p, B))) return rc;
    if (!d_state || !out || (p->n_weights && !w) || (p->n_inputs && !x)) {
        set_error("null pointer");
        return QSV_ERR_ARG;
    }
    const size_t need = qsv_workspace_size(p, B, QSV_OP_FORWARD_EXPVAL);
    if (need > (size_t)QSV_NOALLOC_SCRATCH_BYTES) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "this plan and batch need %zu bytes of scratch, above the %zu-byte "
                      "limit of the allocation-free call", need, (size_t)QSV_NOALLOC_SCRATCH_BYTES);
        set_error(buf);
        return QSV_ERR_TOO_BIG;
    }
    void* ws = nullptr;
    if ((rc = scratch_address(&ws))) return rc;
    // the same launches as qsv_forward_expval on the scratch array; g_noalloc
    // turns every lazy creation (tables, kernels, work lists, events) into an error
    g_noalloc = true;
    rc = qsv_forward_expval(p, w, x, B, d_state, out, ws, (size_t)QSV_NOALLOC_SCRATCH_BYTES, stream);
    g_noalloc = false;
    return rc;
}

int qsv_expval(const qsv_plan_t* p, const void* d_state, int64_t B, double* out, void* ws,
               size_t ws_bytes, void* stream) {
    TraceRange trace_("qsv_expval");
    int rc = check_plan(p);
    if (rc) return rc;
    if ((rc = check_batch(p, B))) return rc;
    if (!d_state || !out) { set_error("null pointer"); return QSV_ERR_ARG; }
    const size_t need = qsv_workspace_size(p, B, QSV_OP_EXPVAL);
    if (!ws || ws_bytes < need) { set_error("expval workspace too small"); return QSV_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    if (p->multi) {
        DeviceTables* T;
        if ((rc = get_tables(p, &T))) return rc;
        double* part = (double*)ws;
        const double amps = (double)B * (double)p->row;
        hipEvent_t ev = prof_begin(p, s);
        hipLaunchKernelGGL(k_expval_part_multi, dim3((unsigned)p->nchunk_tot, (unsigned)B), dim3(256), 0, s,
                           (const DCirc*)T->circ, (int)p->circ.size(), (const float2*)d_state, p->row,
                           p->nchunk_tot, part);
        prof_end(p, s, ev, K_EXPVAL_PART, 8.0 * amps, 3.0 * amps);
        ev = prof_begin(p, s);
        hipLaunchKernelGGL(k_expval_final_multi, dim3((unsigned)p->Wtot, (unsigned)B), dim3(256), 0, s,
                           (const DCirc*)T->circ, (int)p->circ.size(), (const double*)part, p->nchunk_tot,
                           p->Wtot, out);
        prof_end(p, s, ev, K_EXPVAL_FINAL, 8.0 * (double)B * p->nchunk_tot * 32, 0.0);
        HIP_TRY(hipGetLastError());
        return QSV_OK;
    }
    const int64_t nchunk = expval_nchunk(p);
    double* part = (double*)ws;
    const double amps = (double)B * (double)(int64_t(1) << p->W);
    hipEvent_t ev = prof_begin(p, s);
    const int vec = ((uintptr_t)d_state & 15) == 0;
    if (c128(p))
        hipLaunchKernelGGL(k_expval_part<double2>, dim3((unsigned)nchunk, (unsigned)B), dim3(256), 0, s,
                           (const double2*)d_state, p->W, part, vec);
    else
        hipLaunchKernelGGL(k_expval_part<float2>, dim3((unsigned)nchunk, (unsigned)B), dim3(256), 0, s,
                           (const float2*)d_state, p->W, part, vec);
    prof_end(p, s, ev, K_EXPVAL_PART, (double)amp_size(p) * amps, 3.0 * amps);
    ev = prof_begin(p, s);
    hipLaunchKernelGGL(k_expval_final, dim3((unsigned)p->W, (unsigned)B), dim3(256), 0, s,
                       (const double*)part, p->W, nchunk, out);
    prof_end(p, s, ev, K_EXPVAL_FINAL, 8.0 * (double)B * nchunk * p->W, 0.0);
    HIP_TRY(hipGetLastError());
    return QSV_OK;
}

int qsv_backward(const qsv_plan_t* p, const float* w, const float* x, int64_t B,
                 const void* d_state, const double* gout, void* ws, size_t ws_bytes, double* gw,
                 double* gx, void* stream) {
    TraceRange trace_("qsv_backward");
    int rc = check_plan(p);
    if (rc) return rc;
    if ((rc = check_batch(p, B))) return rc;
    if (!d_state || !gout || (p->n_weights && !w) || (p->n_inputs && !x) || (p->n_weights && !gw)) {
        set_error("null pointer");
        return QSV_ERR_ARG;
    }
    const size_t need = qsv_workspace_size(p, B, QSV_OP_BACKWARD);
    if (!ws || ws_bytes < need) { set_error("backward workspace too small"); return QSV_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    DeviceTables* T;
    if ((rc = get_tables(p, &T))) return rc;
    const int W = p->W;
    char* c = (char*)ws;
    float* mats = (float*)c;
    c += mats_bytes(p, B);
    float2* psi = (float2*)c;
    c += align256(state_bytes(p, B)) + kLamSkew;
    float2* lam = (float2*)c;
    c += align256(state_bytes(p, B));
    double* part = (double*)c;
    c += partial_bytes(p, B);
    if ((rc = run_coef(p, T, w, x, B, mats, s))) return rc;
    const int64_t nch = grad_nch(p);
    const double amps = (double)B * (double)(int64_t(1) << W);
    if (p->multi) {
        DeviceTables::Queue* Q;
        if ((rc = get_queue(p, T, B, &Q))) return rc;
        double flops = 0.0, bytes = 0.0;
        for (const DCirc& cc : p->circ)
            for (int r = 0; r < cc.n_bwd; ++r) {
                const int fl = p->bwd_pass[cc.bwd0 + r].flags;
                const double a = (double)B * (double)(int64_t(1) << cc.W);
                flops += p->bwd_pass_flops[cc.bwd0 + r] * a;
                bytes += (((fl & PF_FIRST_BWD) ? 8.0 : 16.0) + ((fl & PF_LAST_BWD) ? 0.0 : 16.0)) * a;
            }
        hipEvent_t ev = prof_begin(p, s);
        for (size_t r = 0; r + 1 < Q->bwd_rounds.size(); ++r) {
            const int i0 = Q->bwd_rounds[r], n = Q->bwd_rounds[r + 1] - i0;
            hipLaunchKernelGGL(k_multi_bwd, dim3((unsigned)n), dim3(256), multi_lds(p), s,
                               (const DCirc*)T->circ, (const DItem*)(Q->bwd + i0), (const DPass*)T->bwd_pass,
                               (const DStage*)T->stages, (const DOp*)T->ops, (const DTerm*)T->terms,
                               (const DGOut*)T->gouts, (const float*)mats, p->n_shared_mats,
                               p->n_ps_mats, (const float2*)d_state, psi, lam, gout, p->Wtot, p->row, (int)B,
                               part, (const int64_t*)T->pu);
        }
        prof_end(p, s, ev, K_MULTI_BWD, bytes, flops);
    } else if (p->opts.method == QSV_METHOD_PER_GATE) {
        const dim3 grid((unsigned)expval_nchunk(p), (unsigned)B);  // chunks of 2^min(W, 12) amplitudes
        const int vec = ((uintptr_t)d_state & 15) == 0;
        hipEvent_t ev = prof_begin(p, s);
        if (c128(p))
            hipLaunchKernelGGL(k_adj_init<double2>, grid, dim3(256), 0, s,
                               (const double2*)d_state, (double2*)psi, (double2*)lam, W, gout, vec);
        else
            hipLaunchKernelGGL(k_adj_init<float2>, grid, dim3(256), 0, s,
                               (const float2*)d_state, psi, lam, W, gout, vec);
        prof_end(p, s, ev, K_ADJ_INIT, 3.0 * (double)amp_size(p) * amps, 2.0 * W * amps);
        for (size_t i = 0; i < p->pg_bwd.size(); ++i) {
            const PGate& pg = p->pg_bwd[i];
            const double touched = pg_touched(pg);
            ev = prof_begin(p, s);
            const int vmode = pg_vec_mode(p, pg, psi);
            if (vmode != PG_SCALAR)
                hipLaunchKernelGGL(k_pg_adj_vec, dim3((unsigned)nch, (unsigned)B), dim3(256), 0, s, psi, lam, W,
                                   (int)B, pg, vmode, (const float*)mats, p->n_shared_mats, p->n_ps_mats, part,
                                   nch, pg_reverse(pg, vmode, i, (int64_t)state_bytes(p, B)));
            else if (c128(p))
                hipLaunchKernelGGL(k_pg_adj<double2>, dim3((unsigned)nch, (unsigned)B), dim3(256), 0, s,
                                   (double2*)psi, (double2*)lam, W, (int)B, pg, (const double*)mats,
                                   p->n_shared_mats, p->n_ps_mats, part, nch);
            else
                hipLaunchKernelGGL(k_pg_adj<float2>, dim3((unsigned)nch, (unsigned)B), dim3(256), 0, s, psi,
                                   lam, W, (int)B, pg, (const float*)mats, p->n_shared_mats,
                                   p->n_ps_mats, part, nch);
            prof_end(p, s, ev, K_PG_ADJ, 4.0 * (double)amp_size(p) * touched * amps, p->pg_bwd_flops[i] * amps,
                     kPgSub0 + pg_prof_class(pg));
        }
    } else {
        const int m = std::min(p->opts.tile_qubits, W);
        const unsigned threads = (unsigned)std::max(64, 1 << (m - kRegBits));
        const unsigned tiles = (unsigned)(B << (W - m));
        const size_t lds = pass_lds_bwd(p);
        for (size_t i = 0; i < p->bwd_pass.size(); ++i) {
            const int fl = p->bwd_pass[i].flags;
            // psi_N read (8) or psi, lambda read (16); psi, lambda written (16) unless last
            const double per_amp = ((fl & PF_FIRST_BWD) ? 8.0 : 16.0) + ((fl & PF_LAST_BWD) ? 0.0 : 16.0);
            hipEvent_t ev = prof_begin(p, s);
            if (!T->bwd_fn.empty()) {
                const void* psiN = d_state;
                const float* mp = mats;
                int ns = p->n_shared_mats, np = p->n_ps_mats, bb = (int)B;
                void* args[] = {&psiN, &psi, &lam, &gout, &mp, &ns, &np, &part, &bb};
                HIP_TRY(hipModuleLaunchKernel((hipFunction_t)T->bwd_fn[i], tiles, 1, 1, threads, 1, 1, 0,
                                              s, args, nullptr));
            } else {
                hipLaunchKernelGGL(k_pass_bwd, dim3(tiles), dim3(threads), lds, s, T->bwd_pass + i,
                                   T->stages, T->ops, T->terms, T->gouts, (const float*)mats,
                                   p->n_shared_mats, p->n_ps_mats, (const float2*)d_state, psi, lam,
                                   gout, W, (int)B, part, (const int64_t*)T->pu);
            }
            prof_end(p, s, ev, K_PASS_BWD, per_amp * amps, p->bwd_pass_flops[i] * amps,
                     T->bwd_fn.empty() ? -1 : (int)i);
        }
    }
    const int n_out = p->n_weights + (gx ? (int)B * p->n_inputs : 0);
    if (n_out > 0) {
        hipEvent_t ev = prof_begin(p, s);
        hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)n_out), dim3(256), 0, s,
                           (const double*)part, T->grad_csr, p->n_weights, p->n_inputs, (int)B,
                           (const int64_t*)T->pu, (const int32_t*)T->nchv, gw, gx, w,
                           (int)p->opts.weight_remap);
        prof_end(p, s, ev, K_GRAD_REDUCE, 8.0 * (double)std::max<int64_t>(p->pu_total, 1) * B, 0.0);
    }
    HIP_TRY(hipGetLastError());
    return QSV_OK;
}

// Options of one circuit of a multi-circuit plan, completed and checked.
static int multi_opts(qsv_opts& o) {
    o.method = QSV_METHOD_FUSED;
    o.codegen = 0;
    if (o.fuse_width < 1 || o.fuse_width > 16) { set_error("fuse_width must be in 1..16"); return QSV_ERR_ARG; }
    if (o.tile_qubits < kRegBits || o.tile_qubits > kMaxTileQubitsTables) { set_error("tile_qubits must be in 4..12"); return QSV_ERR_ARG; }
    if (o.low_qubits < 0 || o.low_qubits >= o.tile_qubits) { set_error("low_qubits must be in 0..tile_qubits-1"); return QSV_ERR_ARG; }
    if (o.max_pass_grads < 1 || o.max_pass_grads > 256) { set_error("max_pass_grads must be in 1..256"); return QSV_ERR_ARG; }
    if (o.bwd_gate_by_gate != 0 && o.bwd_gate_by_gate != 1) { set_error("bwd_gate_by_gate must be 0 or 1"); return QSV_ERR_ARG; }
    if (o.mfma < 0 || o.mfma > 7) { set_error("mfma must be in 0..7"); return QSV_ERR_ARG; }
    if (o.weight_remap != 0 && o.weight_remap != 1) { set_error("weight_remap must be 0 or 1"); return QSV_ERR_ARG; }
    if (o.splitter != 0 && o.splitter != 1) { set_error("splitter must be 0 or 1"); return QSV_ERR_ARG; }
    if (o.pack_beam < 0 || o.pack_beam > 256) { set_error("pack_beam must be in 0..256"); return QSV_ERR_ARG; }
    if (o.amp_dtype != QSV_AMP_C64) { set_error("multi-circuit plans use complex64 amplitudes (amp_dtype = 0)"); return QSV_ERR_ARG; }
    return QSV_OK;
}

// A multi-circuit plan from circuits and one completed option set per circuit.
static int plan_multi(const qsv_circuit* circuits, int32_t n_circuits, std::vector<qsv_opts>& per,
                      qsv_plan_t** out) {
    std::vector<CircuitIn> cs;
    int64_t row = 0;
    for (int c = 0; c < n_circuits; ++c) {
        const qsv_circuit& C = circuits[c];
        if (C.n_qubits < kRegBits) { set_error("multi-circuit plans need circuits of at least 4 qubits"); return QSV_ERR_ARG; }
        // validate each circuit like a single plan (host only)
        qsv_plan_t* tmp = nullptr;
        qsv_opts ot = per[c];
        int rc = qsv_plan(C.n_qubits, C.gates, C.n_gates, C.n_weights, C.n_inputs, &ot, &tmp);
        if (rc) return rc;
        qsv_plan_destroy(tmp);
        row += int64_t(1) << C.n_qubits;
        cs.push_back({C.n_qubits, C.gates, C.n_gates, C.n_weights, C.n_inputs, per[c]});
    }
    if (row > (int64_t(1) << 34)) { set_error("circuits too large together"); return QSV_ERR_TOO_BIG; }
    qsv_plan_t* p = new (std::nothrow) qsv_plan_t();
    if (!p) { set_error("plan allocation failed"); return QSV_ERR_OOM; }
    p->opts = per[0];  // plan-wide settings (weight remapping) and what qsv_plan_get_info reports
    int W = 0;
    for (auto& c : cs) W = std::max(W, c.W);
    p->W = W;
    int rc;
    try {
        rc = build_multi(p, cs);
    } catch (const std::bad_alloc&) {
        rc = QSV_ERR_OOM;
        set_error("out of host memory while planning");
    }
    if (rc != QSV_OK) {
        delete p;
        return rc;
    }
    handle_add(g_live_plans, p);
    *out = p;
    return QSV_OK;
}

int qsv_plan_multi(const qsv_circuit* circuits, int32_t n_circuits, const qsv_opts* opts,
                   qsv_plan_t** out) {
    TraceRange trace_("qsv_plan_multi");
    if (!out) { set_error("out is NULL"); return QSV_ERR_ARG; }
    *out = nullptr;
    if (!circuits || n_circuits < 1) { set_error("need at least one circuit"); return QSV_ERR_ARG; }
    qsv_opts o;
    qsv_default_opts(&o);
    if (opts) o = *opts;
    int rc = multi_opts(o);
    if (rc) return rc;
    std::vector<qsv_opts> per((size_t)n_circuits, o);
    return plan_multi(circuits, n_circuits, per, out);
}

int qsv_plan_multi_each(const qsv_circuit* circuits, int32_t n_circuits, const qsv_opts* per_circuit,
                        qsv_plan_t** out) {
    TraceRange trace_("qsv_plan_multi_each");
    if (!out) { set_error("out is NULL"); return QSV_ERR_ARG; }
    *out = nullptr;
    if (!circuits || n_circuits < 1) { set_error("need at least one circuit"); return QSV_ERR_ARG; }
    if (!per_circuit) { set_error("per_circuit is NULL"); return QSV_ERR_ARG; }
    std::vector<qsv_opts> per(per_circuit, per_circuit + n_circuits);
    for (qsv_opts& o : per) {
        int rc = multi_opts(o);
        if (rc) return rc;
        if (o.weight_remap != per[0].weight_remap) {
            set_error("weight_remap must be the same for every circuit");
            return QSV_ERR_ARG;
        }
    }
    return plan_multi(circuits, n_circuits, per, out);
}

int qsv_plan_circuit_offsets(const qsv_plan_t* p, int32_t circuit, int64_t* amp, int32_t* qubit,
                             int32_t* weight, int32_t* input) {
    int rc = check_plan(p);
    if (rc) return rc;
    const int n = p->multi ? (int)p->circ.size() : 1;
    if (circuit < 0 || circuit >= n) { set_error("circuit index out of range"); return QSV_ERR_ARG; }
    int64_t a = 0;
    int32_t q = 0, w = 0, x = 0;
    if (p->multi) {
        a = p->circ[circuit].amp0;
        q = p->circ[circuit].e0;
        w = p->circ_w0[circuit];
        x = p->circ_x0[circuit];
    }
    if (amp) *amp = a;
    if (qubit) *qubit = q;
    if (weight) *weight = w;
    if (input) *input = x;
    return QSV_OK;
}

int qsv_plan_multi_items(const qsv_plan_t* p, int64_t B, int32_t which, int32_t* items, int64_t max_items,
                         int64_t* n_items) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!p->multi) { set_error("not a multi-circuit plan"); return QSV_ERR_ARG; }
    if ((which != 0 && which != 1) || !n_items) { set_error("bad arguments"); return QSV_ERR_ARG; }
    if ((rc = check_batch(p, B))) return rc;
    std::vector<DItem> list;
    std::vector<int> rounds;
    multi_items(p, B, which, list, rounds);
    *n_items = (int64_t)list.size();
    if (items)
        for (int64_t i = 0; i < std::min<int64_t>(max_items, (int64_t)list.size()); ++i) {
            items[3 * i] = list[i].c;
            items[3 * i + 1] = list[i].pass;
            items[3 * i + 2] = list[i].tile;
        }
    return QSV_OK;
}

int64_t qsv_state_offset(const qsv_plan_t* p, int32_t circuit) {
    int64_t amp = 0;
    const int rc = qsv_plan_circuit_offsets(p, circuit, &amp, nullptr, nullptr, nullptr);
    return rc ? (int64_t)rc : amp * (int64_t)sizeof(float2);
}

struct qsv_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};


int qsv_graph_create(const qsv_plan_t* p, int64_t B, const float* w, const float* x, void* d_state,
                     double* d_expval, const double* gout, double* gw, double* gx, void* ws,
                     size_t ws_bytes, void* stream, qsv_graph_t** out) {
    TraceRange trace_("qsv_graph_create");
    int rc = check_plan(p);
    if (rc) return rc;
    if (!out) { set_error("out is NULL"); return QSV_ERR_ARG; }
    *out = nullptr;
    if ((rc = check_batch(p, B))) return rc;
    if (!stream) { set_error("graph capture needs a non-default stream"); return QSV_ERR_ARG; }
    if (!d_state || !d_expval || !ws) { set_error("null pointer"); return QSV_ERR_ARG; }
    if (ws_bytes < qsv_workspace_size(p, B, QSV_OP_STEP)) { set_error("step workspace too small"); return QSV_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    // everything that allocates or copies happens before the capture
    DeviceTables* T;
    if ((rc = get_tables(p, &T))) return rc;
    if (p->multi) {
        DeviceTables::Queue* Q;
        if ((rc = get_queue(p, T, B, &Q))) return rc;
    }
    const size_t bwd_bytes = qsv_workspace_size(p, B, QSV_OP_BACKWARD);
    char* wsc = (char*)ws;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    g_capturing = true;
    // forward with readout, then the backward over the same workspace (stream order)
    rc = qsv_forward_expval(p, w, x, B, d_state, d_expval, wsc, ws_bytes, stream);
    if (!rc && gout) rc = qsv_backward(p, w, x, B, d_state, gout, wsc, bwd_bytes, gw, gx, stream);
    g_capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(s, &graph);
    if (rc || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (!rc) {
            set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
            rc = QSV_ERR_HIP;
        }
        return rc;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
        return QSV_ERR_HIP;
    }
    qsv_graph_t* g = new (std::nothrow) qsv_graph_t{graph, exec};
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        set_error("graph allocation failed");
        return QSV_ERR_OOM;
    }
    handle_add(g_live_graphs, g);
    *out = g;
    return QSV_OK;
}

int qsv_graph_launch(qsv_graph_t* g, void* stream) {
    TraceRange trace_("qsv_graph_launch");
    if (!handle_live(g_live_graphs, g)) { set_error("null or destroyed graph"); return QSV_ERR_HANDLE; }
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return QSV_OK;
}

void qsv_graph_destroy(qsv_graph_t* g) {
    if (!handle_remove(g_live_graphs, g)) return;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
}

int qsv_plan_estimate(const qsv_plan_t* p, int64_t B, double hbm_gbs, double alu_tflops,
                      double launch_us, double* us) {
    int rc = check_plan(p);
    if (rc) return rc;
    if ((rc = check_batch(p, B))) return rc;
    if (!us || !(hbm_gbs > 0.0) || !(alu_tflops > 0.0) || !(launch_us >= 0.0)) {
        set_error("estimate: null output or non-positive rate");
        return QSV_ERR_ARG;
    }
    const double bw = hbm_gbs * 1e3;      // bytes per microsecond
    const double alu = alu_tflops * 1e6;  // operations per microsecond
    auto sweep = [&](double bytes, double flops) { return std::max(bytes / bw, flops / alu); };
    double t = 0.0;
    int64_t launches = 3;  // coefficients, init, readout
    // a first fused pass that builds the product state replaces the init
    // launch and reads nothing
    auto fwd_bytes = [&](const DPass& ps) { return (ps.flags & PF_INIT_FWD) ? 8.0 : 16.0; };
    if (p->multi) {
        int nf = 0, nb = 0;
        bool all_init = true;
        for (const DCirc& c : p->circ) {
            const double a = (double)B * (double)(int64_t(1) << c.W);
            const bool init = c.n_fwd > 0 && (p->fwd_pass[c.fwd0].flags & PF_INIT_FWD);
            all_init = all_init && init;
            t += (init ? 0.0 : sweep(8.0 * a, 0.0)) + sweep(8.0 * a, 0.0);  // init + readout
            for (int r = 0; r < c.n_fwd; ++r)
                t += sweep(fwd_bytes(p->fwd_pass[c.fwd0 + r]) * a, p->fwd_pass_flops[c.fwd0 + r] * a);
            for (int r = 0; r < c.n_bwd; ++r) {
                const int fl = p->bwd_pass[c.bwd0 + r].flags;
                const double pa = ((fl & PF_FIRST_BWD) ? 8.0 : 16.0) + ((fl & PF_LAST_BWD) ? 0.0 : 16.0);
                t += sweep(pa * a, p->bwd_pass_flops[c.bwd0 + r] * a);
            }
            nf = std::max(nf, c.n_fwd);
            nb = std::max(nb, c.n_bwd);
        }
        launches += nf + nb + 2 - (all_init ? 1 : 0);
    } else {
        const double a = (double)B * (double)(int64_t(1) << p->W);
        const double e = (double)amp_size(p);  // bytes per amplitude
        const bool init = p->opts.method != QSV_METHOD_PER_GATE && !p->fwd_pass.empty() &&
                          (p->fwd_pass[0].flags & PF_INIT_FWD);
        t += (init ? 0.0 : sweep(e * a, 0.0)) + sweep(e * a, 0.0);  // init + readout
        if (init) --launches;
        if (p->opts.method == QSV_METHOD_PER_GATE) {
            t += sweep(3.0 * e * a, 0.0);  // adjoint init
            for (size_t i = 0; i < p->pg_fwd.size(); ++i) {
                const PGate& g = p->pg_fwd[i];
                const double touched = pg_touched(g);
                t += sweep(2.0 * e * touched * a, p->pg_fwd_flops[i] * a);
            }
            for (size_t i = 0; i < p->pg_bwd.size(); ++i) {
                const PGate& g = p->pg_bwd[i];
                const double touched = pg_touched(g);
                t += sweep(4.0 * e * touched * a, p->pg_bwd_flops[i] * a);
            }
            launches += (int64_t)(p->pg_fwd.size() + p->pg_bwd.size()) + 2;
        } else {
            for (size_t i = 0; i < p->fwd_pass.size(); ++i)
                t += sweep(fwd_bytes(p->fwd_pass[i]) * a, p->fwd_pass_flops[i] * a);
            for (size_t i = 0; i < p->bwd_pass.size(); ++i) {
                const int fl = p->bwd_pass[i].flags;
                const double pa = ((fl & PF_FIRST_BWD) ? 8.0 : 16.0) + ((fl & PF_LAST_BWD) ? 0.0 : 16.0);
                t += sweep(pa * a, p->bwd_pass_flops[i] * a);
            }
            launches += (int64_t)(p->fwd_pass.size() + p->bwd_pass.size()) + 1;
        }
    }
    *us = t + launch_us * (double)launches;
    return QSV_OK;
}

int qsv_plan_codegen_source(const qsv_plan_t* p, char* buf, size_t buf_size, size_t* needed) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!needed) { set_error("needed is NULL"); return QSV_ERR_ARG; }
    std::vector<JitKernelRef> refs;
    const std::string src = p->opts.method == QSV_METHOD_FUSED ? jit_source(p, refs, 1 << 30) : std::string();
    *needed = src.size() + 1;
    if (buf && buf_size) {
        const size_t n = std::min(buf_size - 1, src.size());
        std::memcpy(buf, src.data(), n);
        buf[n] = 0;
    }
    return QSV_OK;
}

int qsv_plan_codegen_check(const qsv_plan_t* p, const char* arch) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!arch || !*arch) { set_error("arch is empty"); return QSV_ERR_ARG; }
    if (p->opts.method != QSV_METHOD_FUSED) return QSV_OK;
    JitModules jm;
    std::string err;
    rc = jit_compile(p, arch, jm, err);
    if (rc) set_error(err);
    return rc;
}

int qsv_pass_copy(const qsv_plan_t* p, int32_t which, int32_t pass, int64_t B, void* d_state, void* ws,
                  size_t ws_bytes, int32_t lds_bytes, void* stream) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (p->multi || p->opts.method != QSV_METHOD_FUSED || c128(p)) {
        set_error("pass copy: fused complex64 plans of one circuit only");
        return QSV_ERR_ARG;
    }
    if ((rc = check_batch(p, B))) return rc;
    if (which != 0 && which != 1) { set_error("pass copy: which must be 0 or 1"); return QSV_ERR_ARG; }
    const std::vector<DPass>& passes = which == 0 ? p->fwd_pass : p->bwd_pass;
    if (pass < 0 || pass >= (int32_t)passes.size()) { set_error("pass copy: no such pass"); return QSV_ERR_ARG; }
    if (lds_bytes < 0 || lds_bytes > 65536) { set_error("pass copy: lds_bytes outside 0..65536"); return QSV_ERR_ARG; }
    const DPass& ps = passes[pass];
    const int m = ps.m;
    if (m < kRegBits || m > p->W) { set_error("pass copy: tile outside 4..n qubits"); return QSV_ERR_ARG; }
    if (!d_state) { set_error("pass copy: null state"); return QSV_ERR_ARG; }
    // the arrays the pass itself reads and writes: the state (forward, and
    // psi_N for the first backward pass), psi and lambda in the backward workspace
    float2 *ra = nullptr, *rb = nullptr, *wa = nullptr, *wb = nullptr;
    int rd, wr;
    if (which == 0) {
        rd = (ps.flags & PF_INIT_FWD) ? 0 : 1;
        wr = 1;
        ra = wa = (float2*)d_state;
    } else {
        if (!ws || ws_bytes < qsv_workspace_size(p, B, QSV_OP_BACKWARD)) {
            set_error("pass copy: backward workspace too small");
            return QSV_ERR_ARG;
        }
        char* c = (char*)ws + mats_bytes(p, B);
        float2* psi = (float2*)c;
        float2* lam = (float2*)(c + align256(state_bytes(p, B)) + kLamSkew);
        const bool first = ps.flags & PF_FIRST_BWD;
        rd = first ? 1 : 3;
        wr = (ps.flags & PF_LAST_BWD) ? 0 : 3;
        ra = first ? (float2*)d_state : psi;
        rb = lam;
        wa = psi;
        wb = lam;
    }
    const bool pair = ps.lq[0] == 0;
    const uintptr_t al = pair ? 15 : 7;
    if (((uintptr_t)ra & al) || ((uintptr_t)rb & al) || ((uintptr_t)wa & al) || ((uintptr_t)wb & al)) {
        set_error("pass copy: arrays must be 16-byte aligned");
        return QSV_ERR_ARG;
    }
    PassGeom g{};
    g.m = m;
    g.W = p->W;
    g.tb = p->W - m;
    g.pair = pair ? 1 : 0;
    for (int j = 0; j < m; ++j) g.lq[j] = ps.lq[j];
    for (int k = 0; k < g.tb; ++k) g.oq[k] = ps.oq[k];
    const uint64_t tiles = (uint64_t)B << g.tb;
    const int threads = std::max(64, 1 << (m - kRegBits));
    hipLaunchKernelGGL(k_pass_copy, dim3((unsigned)tiles), dim3(threads), (size_t)lds_bytes, (hipStream_t)stream,
                       (const float2*)ra, (const float2*)rb, wa, wb, g, rd, wr);
    HIP_TRY(hipGetLastError());
    return QSV_OK;
}

int qsv_profile_enable(qsv_plan_t* p, int32_t on) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!p->prof) {
        Profiler* pr = new (std::nothrow) Profiler();
        if (!pr) { set_error("profiler allocation failed"); return QSV_ERR_OOM; }
        p->prof = pr;
    }
    if (on < 0 || on > 2) { set_error("profile mode must be 0, 1 or 2"); return QSV_ERR_ARG; }
    prof_of(p)->on = on != 0;
    prof_of(p)->each = on == 2;
    return QSV_OK;
}

int qsv_profile_read(qsv_plan_t* p, qsv_kernel_stat* out, int32_t max_out, int32_t* n_out) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!n_out || (max_out > 0 && !out)) { set_error("null pointer"); return QSV_ERR_ARG; }
    // totals per (kernel, generated pass); ordered by kernel id, then pass.
    // Per-launch mode keys each record by its position instead.
    std::map<std::pair<int, int>, qsv_kernel_stat> tot;
    Profiler* pr = prof_of(p);
    int err = QSV_OK;
    if (pr) {
        std::lock_guard<std::mutex> lk(pr->mu);
        int pos = 0;
        for (auto& r : pr->recs) {
            const std::pair<int, int> key = pr->each ? std::make_pair(pos++, 0) : std::make_pair(r.kid, r.sub);
            float ms = 0.f;
            if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
                set_error("event timing failed");
                err = QSV_ERR_HIP;
            }
            auto it = tot.find(key);
            if (it == tot.end()) {
                qsv_kernel_stat z;
                std::memset(&z, 0, sizeof z);
                if (r.sub >= kPgSub0)  // per-gate kernel, split by gate class
                    std::snprintf(z.name, sizeof z.name, "%s.%s", kKernelNames[r.kid], kPgClassNames[r.sub - kPgSub0]);
                else if (r.sub >= 0)  // the generated kernel's own symbol name
                    std::snprintf(z.name, sizeof z.name, "qsv_%c%d", r.kid == K_PASS_FWD ? 'f' : 'b', r.sub);
                else
                    std::snprintf(z.name, sizeof z.name, "%s", kKernelNames[r.kid]);
                it = tot.emplace(key, z).first;
            }
            it->second.launches++;
            it->second.total_ms += ms;
            it->second.bytes += r.bytes;
            it->second.flops += r.flops;
            pr->pool.push_back(r.a);
            pr->pool.push_back(r.b);
        }
        pr->recs.clear();
    }
    int n = 0;
    for (auto& kv : tot) {
        if (n < max_out) out[n] = kv.second;
        ++n;
    }
    *n_out = std::min(n, max_out);
    return err;
}

}  // extern "C"
