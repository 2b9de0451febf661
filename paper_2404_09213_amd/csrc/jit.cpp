// jit.cpp -- per-plan code generation of the fused pass kernels.
//
// The interpreter kernels in qsv.hip read the pass/stage/op tables at run time;
// every op then ends in a data-dependent branch, and the compiler has to copy
// all register amplitudes back into place after it. Here the same tables are
// turned into HIP source instead: one straight-line kernel per pass, with the
// tile layout, the register position of every gate, the sign masks of CZ
// groups and the gradient slots as constants. Only the gate matrices (which
// depend on the weights and inputs of a call) are read from memory. The
// source is compiled for the device's architecture once per plan and device:
// by the ROCm clang driver in parallel child processes (one per kernel) when it
// is installed, else by hipRTC (which serialises compilations in a process).
//
// Every generated kernel applies the same ops in the same order as the
// matching table-driven kernel; only float32 contraction and the order of the
// per-thread gradient sums differ.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <fcntl.h>
#include <spawn.h>
#include <sys/stat.h>
#include <sys/wait.h>
#include <unistd.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "jit.hpp"

namespace qsv {
namespace {

std::string I(long long v) { return std::to_string(v); }

std::string hex(unsigned v) {
    char b[16];
    std::snprintf(b, sizeof b, "0x%xu", v);
    return b;
}

// Expression placing bit i of `var` at position pos[i] (runs of consecutive
// positions are moved with one shift and mask).
std::string scatter(const std::string& var, const std::vector<int>& pos) {
    std::string s;
    const int n = (int)pos.size();
    int i = 0;
    while (i < n) {
        int j = i;
        while (j + 1 < n && pos[j + 1] == pos[j] + 1) ++j;
        const int len = j - i + 1;
        std::string term = i ? "(" + var + " >> " + I(i) + ")" : var;
        term = "(" + term + " & " + hex((1u << len) - 1) + ")";
        if (pos[i]) term = "(" + term + " << " + I(pos[i]) + ")";
        s += (s.empty() ? "" : " | ") + term;
        i = j + 1;
    }
    return s.empty() ? "0" : s;
}

int swz_host(int l) { return l ^ (((l >> 5) ^ (l >> 10)) & 31); }

struct Layout {
    int reg[kRegBits];
    std::vector<int> nonreg;  // local bits fed by the thread index, ascending
};

Layout make_layout(int m, const int* reg) {
    Layout L;
    for (int p = 0; p < kRegBits; ++p) L.reg[p] = reg[p];
    for (int j = 0; j < m; ++j)
        if (std::find(reg, reg + kRegBits, j) == reg + kRegBits) L.nonreg.push_back(j);
    return L;
}

bool same(const Layout& a, const Layout& b) {
    return std::equal(a.reg, a.reg + kRegBits, b.reg);
}

class Gen {
public:
    Gen(const qsv_plan_t* p) : p_(p) {}

    std::string prelude() const {
        return R"(
typedef float2 f2;
typedef float qsv_v4f __attribute__((ext_vector_type(4)));
typedef __UINTPTR_TYPE__ qsv_uptr;  // pointer-sized integer without any header
// float64 wavefront sum by DPP lane moves: pairs, quads, half rows, rows, then
// row 0 -> 1, 2 -> 3 and rows 0-1 -> 2-3 broadcasts; lane 63 holds the total.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double qsv_dpp(double v) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWMASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, ROWMASK, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double qsv_wave_sum(double v) {
    v += qsv_dpp<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v += qsv_dpp<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    v += qsv_dpp<0x141, 0xF>(v);   // row_half_mirror
    v += qsv_dpp<0x140, 0xF>(v);   // row_mirror
    v += qsv_dpp<0x142, 0xA>(v);   // row_bcast:15 into rows 1, 3
    v += qsv_dpp<0x143, 0xC>(v);   // row_bcast:31 into rows 2, 3
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)x, 63), hi = __builtin_amdgcn_readlane((int)(x >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// float32 sum over the 16 lanes of a DPP row (pairs, quads, half rows, rows);
// every lane of the row ends with the row's total.
template <int CTRL>
__device__ __forceinline__ float qsv_dppf(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float qsv_row_sum(float v) {
    v += qsv_dppf<0xB1>(v);
    v += qsv_dppf<0x4E>(v);
    v += qsv_dppf<0x141>(v);
    v += qsv_dppf<0x140>(v);
    return v;
}
// gradient of a gate inside a 1-qubit chain: Im<l|V P V^dagger|psi> from the
// chain's components cx, cy, cz = Im<l|X|psi>, Im<l|Y|psi>, Im<l|Z|psi>, with
// V the later gates' product (row-major 2x2) and P = X, Y, Z for axis 0, 1, 2;
// V P V^dagger = H00 Z + Re(H01) X - Im(H01) Y
__device__ double qsv_chain_grad(const float* V, int axis, double cx, double cy, double cz) {
    const double ar = V[0], ai = V[1], br = V[2], bi = V[3], cr = V[4], ci = V[5], dr = V[6], di = V[7];
    double h00, hr, hi;
    if (axis == 2) {
        h00 = ar * ar + ai * ai - br * br - bi * bi;
        hr = (ar * cr + ai * ci) - (br * dr + bi * di);
        hi = (ai * cr - ar * ci) - (bi * dr - br * di);
    } else if (axis == 0) {
        h00 = 2.0 * (ar * br + ai * bi);
        hr = (br * cr + bi * ci) + (ar * dr + ai * di);
        hi = (bi * cr - br * ci) + (ai * dr - ar * di);
    } else {
        h00 = -2.0 * (bi * ar - br * ai);
        hr = -((bi * cr - br * ci) - (ai * dr - ar * di));
        hi = (br * cr + bi * ci) - (ar * dr + ai * di);
    }
    return h00 * cz + hr * cx - hi * cy;
}
__device__ __forceinline__ unsigned qsv_sgn(int f, int k) { return ((unsigned)(f >> k) & 1u) << 31; }
__device__ __forceinline__ f2 qsv_flip(f2 a, unsigned s) {
    return make_float2(__uint_as_float(__float_as_uint(a.x) ^ s), __uint_as_float(__float_as_uint(a.y) ^ s));
}
)";
    }

    std::string kernel(int which, int i, std::string& name) {
        const DPass& ps = which == 0 ? p_->fwd_pass[i] : p_->bwd_pass[i];
        name = std::string(which == 0 ? "qsv_f" : "qsv_b") + I(i);
        o_.str("");
        bwd_ = which == 1;
        last_fwd_ = which == 0 && i + 1 == (int)p_->fwd_pass.size();
        ps_ = &ps;
        m_ = ps.m;
        W_ = p_->W;
        T_ = 1 << (m_ - kRegBits);
        threads_ = std::max(64, T_);
        guard_ = threads_ > T_;
        arrays_ = bwd_ ? std::vector<std::string>{"ps", "lm"} : std::vector<std::string>{"a"};
        emit_kernel(name);
        return o_.str();
    }

private:
    const qsv_plan_t* p_;
    const DPass* ps_ = nullptr;
    const Layout* lay_ = nullptr;  // register layout of the ops being emitted
    std::ostringstream o_;
    bool bwd_ = false, guard_ = false, last_fwd_ = false;
    std::string name_;
    int m_ = 0, W_ = 0, T_ = 0, threads_ = 0;
    std::vector<std::string> arrays_;

    std::string act(const std::string& body) const { return guard_ ? "if (act) { " + body + " }" : body; }

    // Matrix-core path for a generic 2x2: only where every lane of the wave
    // executes it (matrix instructions run on all lanes regardless of the
    // execution mask), i.e. not under a control outside the registers.
    // opts.mfma bits: 1 forward kernels, 2 backward psi array, 4 backward lambda array.
    bool use_mfma(const DOp& op) const {
        return (p_->opts.mfma & (bwd_ ? 6 : 1)) && op.kind == OP_U2 && op.ctl < kCtlNonReg &&
               op.ctl2 < kCtlNonReg;
    }
    bool mfma_array(const std::string& A) const {
        if (!bwd_) return p_->opts.mfma & 1;
        return p_->opts.mfma & (A == "ps" ? 2 : 4);
    }

    int lq(int j) const { return ps_->lq[j]; }

    // Register bits of the layout a pass loads and stores in: the top three
    // tile bits, plus tile bit 0 when it is amplitude bit 0 (then a register
    // pair k, k + 1 holds two adjacent amplitudes), else the fourth-highest.
    std::array<int, kRegBits> nat_reg() const {
        return {lq(0) == 0 ? 0 : m_ - 4, m_ - 3, m_ - 2, m_ - 1};
    }

    // global offset of register k (within the sample) in layout L
    int gR(const Layout& L, int k) const {
        int v = 0;
        for (int p = 0; p < kRegBits; ++p)
            if (k >> p & 1) v |= 1 << lq(L.reg[p]);
        return v;
    }
    int lR(const Layout& L, int k) const {
        int v = 0;
        for (int p = 0; p < kRegBits; ++p)
            if (k >> p & 1) v |= 1 << L.reg[p];
        return v;
    }
    std::string gT_expr(const Layout& L) const {
        std::vector<int> pos;
        for (int j : L.nonreg) pos.push_back(lq(j));
        return "base | " + scatter("t", pos);
    }
    std::string lT_expr(const Layout& L) const { return scatter("t", L.nonreg); }

    void emit_exchange(const Layout& from, const Layout& to) {
        // The empty asm statements make each exchange compute its LDS
        // addresses afresh: otherwise the compiler keeps the addresses of
        // every layout alive across the whole kernel (tens of registers).
        o_ << "  {\n    int l0_ = " << lT_expr(from) << ";\n"
           << "    __asm__ volatile(\"\" : \"+v\"(l0_));\n"
           << "    const int s0_ = l0_ ^ (((l0_ >> 5) ^ (l0_ >> 10)) & 31);\n"
           << "    int l1_ = " << lT_expr(to) << ";\n"
           << "    __asm__ volatile(\"\" : \"+v\"(l1_));\n"
           << "    const int s1_ = l1_ ^ (((l1_ >> 5) ^ (l1_ >> 10)) & 31);\n";
        for (size_t ai = 0; ai < arrays_.size(); ++ai) {
            const std::string& A = arrays_[ai];
            std::string w, r;
            for (int k = 0; k < kRegs; ++k) {
                w += "lds[s0_ ^ " + I(swz_host(lR(from, k))) + "] = " + A + "[" + I(k) + "]; ";
                r += A + "[" + I(k) + "] = lds[s1_ ^ " + I(swz_host(lR(to, k))) + "]; ";
            }
            if (ai > 0) o_ << "    __syncthreads();\n";
            o_ << "    " << act(w) << "\n    __syncthreads();\n    " << act(r) << "\n";
        }
        o_ << "    __syncthreads();\n  }\n";
        o_ << "  gT = " << gT_expr(to) << ";\n";
    }

    std::string mat_ptr(int mat) const {
        if (mat >= 0) return "mats + " + I(8LL * mat);
        return "mp + " + I(8LL * (-mat - 1));
    }

    static std::string rk(const std::string& A, int k) { return A + "[" + I(k) + "]"; }

    void emit_matrix(const DOp& op) {
        o_ << "    const float* M_ = " << mat_ptr(op.mat) << ";\n";
        switch (op.kind) {
        case OP_U2:
            if (use_mfma(op)) {
                // row (lane & 3) of the real 4x4 form of [[u00, u01], [u10, u11]] acting
                // on (x.re, x.im, y.re, y.im): rows 0, 1 from u00, u01; rows 2, 3 from u10, u11
                // entries read as wave-uniform values (scalar loads), then selected per lane
                o_ << "    float u_[8];\n"
                   << "    for (int i_ = 0; i_ < 8; ++i_) u_[i_] = __int_as_float(__builtin_amdgcn_readfirstlane("
                      "__float_as_int(M_[i_])));\n"
                   << "    const float ur_ = lo4_ ? u_[0] : u_[4], ui_ = lo4_ ? u_[1] : u_[5], "
                      "vr_ = lo4_ ? u_[2] : u_[6], vi_ = lo4_ ? u_[3] : u_[7];\n"
                   << "    const float a0_ = im4_ ? ui_ : ur_, a1_ = im4_ ? ur_ : -ui_, "
                      "a2_ = im4_ ? vi_ : vr_, a3_ = im4_ ? vr_ : -vi_;\n";
                bool valu_too = false;
                for (const std::string& A : arrays_) valu_too |= !mfma_array(A);
                if (valu_too)
                    o_ << "    const float m0r = u_[0], m0i = u_[1], m1r = u_[2], m1i = u_[3], "
                          "m2r = u_[4], m2i = u_[5], m3r = u_[6], m3i = u_[7];\n";
            } else {
                o_ << "    const float m0r = M_[0], m0i = M_[1], m1r = M_[2], m1i = M_[3], "
                      "m2r = M_[4], m2i = M_[5], m3r = M_[6], m3i = M_[7];\n";
            }
            break;
        case OP_REAL:
            o_ << "    const float m0r = M_[0], m1r = M_[2], m2r = M_[4], m3r = M_[6];\n";
            break;
        case OP_RXL:
            o_ << "    const float al = M_[0], be = M_[3];\n";
            break;
        case OP_DIAG:
            o_ << "    const float m0r = M_[0], m0i = M_[1], m3r = M_[6], m3i = M_[7];\n";
            break;
        default: break;
        }
    }

    // pairs (k, k | 1<<pos) of an op on register position `pos`; with a control
    // on a register position, only pairs where that bit is 1.
    // register k satisfies the op's controls that sit on register positions
    static bool reg_ok(const DOp& op, int k) {
        for (int c : {op.ctl, op.ctl2})
            if (c >= 0 && c < kCtlNonReg && !(k >> c & 1)) return false;
        return true;
    }
    // Whether a control outside the registers sits on an index bit fed by one
    // of the six lane bits of the thread index (the condition then differs
    // between the lanes of a wave). Other controls are uniform over a wave:
    // their bit lies outside the tile or comes from the wave index.
    bool lane_ctl(const DOp& op) const {
        for (int x : {op.ctl, op.ctl2}) {
            if (x < kCtlNonReg) continue;
            for (size_t i = 0; i < lay_->nonreg.size() && i < 6; ++i)
                if (lq(lay_->nonreg[i]) == (x & 0xFF)) return true;
        }
        return false;
    }
    // run-time condition of the op's controls outside the registers ("" if
    // none); a wave-uniform one is read from the first lane, so the compiler
    // branches on a scalar and skips the op for waves where it is false
    std::string nonreg_cond(const DOp& op) const {
        std::string c;
        for (int x : {op.ctl, op.ctl2})
            if (x >= kCtlNonReg) c += std::string(c.empty() ? "" : " && ") + "((gT >> " + I(x & 0xFF) + ") & 1)";
        if (c.empty() || lane_ctl(op)) return c;
        return "__builtin_amdgcn_readfirstlane((int)(" + c + "))";
    }
    std::vector<int> pairs(const DOp& op) const {
        std::vector<int> v;
        for (int k = 0; k < kRegs; ++k) {
            if (k >> op.pos & 1) continue;
            if (!reg_ok(op, k)) continue;
            v.push_back(k);
        }
        return v;
    }

    // Matrix-core form of a generic 2x2 over every pair of every state array:
    // 16 blocks of 4 lanes; lane 4b+j supplies row j of the gate's real 4x4
    // form (A operand) and its own pair (B operand) and receives its pair's
    // four outputs. The four rank-1 steps are issued step by step across all
    // pairs, so consecutive matrix instructions are independent.
    void emit_pairs_mfma(const DOp& op) {
        std::vector<std::pair<std::string, std::string>> xy;
        for (const std::string& A : arrays_)
            if (mfma_array(A))
                for (int k : pairs(op)) xy.emplace_back(rk(A, k), rk(A, k | (1 << op.pos)));
        const int n = (int)xy.size();
        o_ << "    {\n";
        for (int i = 0; i < n; ++i)
            o_ << "      qsv_v4f c" << i << "_ = __builtin_amdgcn_mfma_f32_4x4x1f32(a0_, " << xy[i].first
               << ".x, qsv_v4f{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);\n";
        for (int st = 1; st < 4; ++st)
            for (int i = 0; i < n; ++i) {
                const std::string src = st == 1 ? xy[i].first + ".y" : st == 2 ? xy[i].second + ".x" : xy[i].second + ".y";
                o_ << "      c" << i << "_ = __builtin_amdgcn_mfma_f32_4x4x1f32(a" << st << "_, " << src << ", c" << i
                   << "_, 0, 0, 0);\n";
            }
        for (int i = 0; i < n; ++i)
            o_ << "      " << xy[i].first << " = make_float2(c" << i << "_[0], c" << i << "_[1]); " << xy[i].second
               << " = make_float2(c" << i << "_[2], c" << i << "_[3]);\n";
        o_ << "    }\n";
    }

    void emit_pair_op(const DOp& op, const std::string& A) {
        for (int k : pairs(op)) {
            const int k1 = k | (1 << op.pos);
            const std::string x = rk(A, k), y = rk(A, k1);
            o_ << "      { const f2 x = " << x << ", y = " << y << ";\n";
            switch (op.kind) {
            case OP_U2:
                o_ << "        " << x << " = make_float2(m0r * x.x - m0i * x.y + m1r * y.x - m1i * y.y, "
                   << "m0r * x.y + m0i * x.x + m1r * y.y + m1i * y.x);\n"
                   << "        " << y << " = make_float2(m2r * x.x - m2i * x.y + m3r * y.x - m3i * y.y, "
                   << "m2r * x.y + m2i * x.x + m3r * y.y + m3i * y.x); }\n";
                break;
            case OP_REAL:
                o_ << "        " << x << " = make_float2(m0r * x.x + m1r * y.x, m0r * x.y + m1r * y.y);\n"
                   << "        " << y << " = make_float2(m2r * x.x + m3r * y.x, m2r * x.y + m3r * y.y); }\n";
                break;
            case OP_RXL:
                o_ << "        " << x << " = make_float2(al * x.x - be * y.y, al * x.y + be * y.x);\n"
                   << "        " << y << " = make_float2(al * y.x - be * x.y, al * y.y + be * x.x); }\n";
                break;
            case OP_SWAP:
                o_ << "        " << x << " = y; " << y << " = x; }\n";
                break;
            }
        }
    }

    void emit_apply(const DOp& op) {
        o_ << "  {\n";
        if (op.kind != OP_SIGN && op.kind != OP_SWAP) emit_matrix(op);
        if (op.kind == OP_SIGN) {
            // uniform part folded at compile time, per-thread part from the index bits
            const int nt = op.nterm;
            if (nt) {
                o_ << "    int f_ = 0;\n";
                for (int i = 0; i < nt; ++i) {
                    const DTerm& tm = p_->terms[op.term0 + i];
                    std::string c = "(gT >> " + I(tm.s0) + ")";
                    if (tm.s1 >= 0) c += " & (gT >> " + I(tm.s1) + ")";
                    if (tm.s2 >= 0) c += " & (gT >> " + I(tm.s2) + ")";
                    o_ << "    if ((" << c << ") & 1) f_ ^= " << hex(tm.mask) << ";\n";
                }
            }
            for (const std::string& A : arrays_)
                for (int k = 0; k < kRegs; ++k) {
                    const bool u = op.pos >> k & 1;
                    if (nt) {
                        o_ << "    " << rk(A, k) << " = qsv_flip(" << rk(A, k) << ", qsv_sgn(f_"
                           << (u ? " ^ 0xffff" : "") << ", " << k << "));\n";
                    } else if (u) {
                        o_ << "    " << rk(A, k) << " = make_float2(-" << rk(A, k) << ".x, -" << rk(A, k) << ".y);\n";
                    }
                }
            o_ << "  }\n";
            return;
        }
        if (op.kind == OP_DIAG) {
            const std::string nc = nonreg_cond(op);
            if (!nc.empty()) o_ << "    if (" << nc << ") {\n";
            if (op.pos >= 0) {
                for (const std::string& A : arrays_)
                    for (int k = 0; k < kRegs; ++k) {
                        if (!reg_ok(op, k)) continue;
                        const bool hi = k >> op.pos & 1;
                        const std::string pr = hi ? "m3r" : "m0r", pi = hi ? "m3i" : "m0i";
                        o_ << "    { const f2 x = " << rk(A, k) << "; " << rk(A, k) << " = make_float2(" << pr
                           << " * x.x - " << pi << " * x.y, " << pr << " * x.y + " << pi << " * x.x); }\n";
                    }
            } else {
                o_ << "    const bool hb_ = (gT >> " << op.sh << ") & 1;\n"
                   << "    const float pr = hb_ ? m3r : m0r, pi = hb_ ? m3i : m0i;\n";
                for (const std::string& A : arrays_)
                    for (int k = 0; k < kRegs; ++k) {
                        if (!reg_ok(op, k)) continue;
                        o_ << "    { const f2 x = " << rk(A, k) << "; " << rk(A, k)
                           << " = make_float2(pr * x.x - pi * x.y, pr * x.y + pi * x.x); }\n";
                    }
            }
            if (!nc.empty()) o_ << "    }\n";
            o_ << "  }\n";
            return;
        }
        const std::string nc = nonreg_cond(op);
        if (op.kind == OP_SWAP && !nc.empty() && lane_ctl(op)) {
            // A swap under a per-lane control as selects: written as a branch,
            // the compiler keeps both orders of every pair live across the
            // divergent region (64 more VGPRs for psi and lambda).
            o_ << "    const bool c_ = " << nc << ";\n";
            for (const std::string& A : arrays_)
                for (int k : pairs(op)) {
                    const std::string x = rk(A, k), y = rk(A, k | (1 << op.pos));
                    o_ << "    { const f2 x = " << x << ", y = " << y << "; " << x << " = c_ ? y : x; " << y
                       << " = c_ ? x : y; }\n";
                }
            o_ << "  }\n";
            return;
        }
        if (!nc.empty()) o_ << "    if (" << nc << ") {\n";
        if (use_mfma(op)) emit_pairs_mfma(op);
        for (const std::string& A : arrays_)
            if (!use_mfma(op) || !mfma_array(A)) emit_pair_op(op, A);
        if (!nc.empty()) o_ << "    }\n";
        o_ << "  }\n";
    }

    void emit_grad(const DOp& op) {
        // two float32 accumulators (alternating terms), summed at the end
        const std::string gs = "g" + I(op.slot);
        const std::string g = "ga_";
        o_ << "  {\n    float ga_ = 0.f, gb_ = 0.f;\n";
        const std::string nc = nonreg_cond(op);
        if (op.kind == OP_GZ && op.pos < 0) {
            o_ << "    float h_ = 0.f;\n";
            if (!nc.empty()) o_ << "    if (" << nc << ") {\n";
            for (int k = 0; k < kRegs; ++k) {
                if (!reg_ok(op, k)) continue;
                o_ << "    h_ = fmaf(lm[" << k << "].x, ps[" << k << "].y, h_); h_ = fmaf(-lm[" << k
                   << "].y, ps[" << k << "].x, h_);\n";
            }
            if (!nc.empty()) o_ << "    }\n";
            o_ << "    " << gs << " = ((gT >> " << op.sh << ") & 1) ? -h_ : h_;\n  }\n";
            return;
        }
        if (!nc.empty()) o_ << "    if (" << nc << ") {\n";
        if (op.kind == OP_GZ) {
            for (int k = 0; k < kRegs; ++k) {
                if (!reg_ok(op, k)) continue;
                const std::string g = (k & 1) ? "gb_" : "ga_";
                const char* sg = (k >> op.pos & 1) ? "-" : "";
                o_ << "    " << g << " = fmaf(" << sg << "lm[" << k << "].x, ps[" << k << "].y, " << g << "); "
                   << g << " = fmaf(" << (sg[0] ? "" : "-") << "lm[" << k << "].y, ps[" << k << "].x, " << g
                   << ");\n";
            }
        } else {
            int alt = 0;
            for (int k : pairs(op)) {
                const std::string g = (alt++ & 1) ? "gb_" : "ga_";
                const int k1 = k | (1 << op.pos);
                const std::string l0 = rk("lm", k), l1 = rk("lm", k1), p0 = rk("ps", k), p1 = rk("ps", k1);
                if (op.kind == OP_GX)  // Im(conj(l0) p1) + Im(conj(l1) p0)
                    o_ << "    " << g << " = fmaf(" << l0 << ".x, " << p1 << ".y, " << g << "); " << g << " = fmaf(-"
                       << l0 << ".y, " << p1 << ".x, " << g << "); " << g << " = fmaf(" << l1 << ".x, " << p0
                       << ".y, " << g << "); " << g << " = fmaf(-" << l1 << ".y, " << p0 << ".x, " << g << ");\n";
                else  // GY: Re(conj(l1) p0) - Re(conj(l0) p1)
                    o_ << "    " << g << " = fmaf(" << l1 << ".x, " << p0 << ".x, " << g << "); " << g << " = fmaf("
                       << l1 << ".y, " << p0 << ".y, " << g << "); " << g << " = fmaf(-" << l0 << ".x, " << p1
                       << ".x, " << g << "); " << g << " = fmaf(-" << l0 << ".y, " << p1 << ".y, " << g << ");\n";
            }
        }
        if (!nc.empty()) o_ << "    }\n";
        o_ << "    " << gs << " = ga_ + gb_;\n  }\n";
    }

    // Readout of the last forward pass (when epart is given): per tile and
    // qubit i, sum |a|^2 (1 - 2 bit_i) into epart[(b ntiles + tile) W + i].
    // Reduced values: the thread's total T, its sums S_r over registers with
    // register bit r set, and T on threads with thread-index bit j set; the
    // out-of-tile qubits take the tile total with the tile's sign.
    void emit_readout(const Layout& L) {
        const int nreg = kRegBits, ntb = (int)L.nonreg.size();
        const int nv = 1 + nreg + ntb, nw = threads_ / 64;
        o_ << "  if (epart) {\n    __shared__ double ered_[" << nw * nv << "];\n";
        o_ << "    float T_ = 0.f, S_[" << nreg << "] = {0.f, 0.f, 0.f, 0.f};\n";
        o_ << "    if (" << (guard_ ? "act" : "true") << ") {\n";
        for (int k = 0; k < kRegs; ++k) {
            o_ << "      { const float p_ = a[" << k << "].x * a[" << k << "].x + a[" << k << "].y * a[" << k
               << "].y; T_ += p_;";
            for (int r = 0; r < nreg; ++r)
                if (k >> r & 1) o_ << " S_[" << r << "] += p_;";
            o_ << " }\n";
        }
        o_ << "    }\n";
        o_ << "    double v_[" << nv << "];\n    v_[0] = T_;\n";
        for (int r = 0; r < nreg; ++r) o_ << "    v_[" << 1 + r << "] = S_[" << r << "];\n";
        for (int j = 0; j < ntb; ++j)
            o_ << "    v_[" << 1 + nreg + j << "] = ((t >> " << j << ") & 1) ? (double)T_ : 0.0;\n";
        o_ << "    for (int k = 0; k < " << nv << "; ++k) { const double r_ = qsv_wave_sum(v_[k]); "
           << "if (lane == 0) ered_[wave * " << nv << " + k] = r_; }\n";
        o_ << "    __syncthreads();\n";
        o_ << "    const int* eq_ = " << name_ << "_eq;\n";
        o_ << "    for (int i = t; i < " << W_ << "; i += " << threads_ << ") {\n"
           << "      double tot = 0.0, part_ = 0.0;\n"
           << "      for (int w = 0; w < " << nw << "; ++w) { tot += ered_[w * " << nv << "]; "
           << "if (eq_[2 * i] != 2) part_ += ered_[w * " << nv << " + eq_[2 * i + 1]]; }\n"
           << "      const double e = eq_[2 * i] == 2 ? (((base >> eq_[2 * i + 1]) & 1) ? -tot : tot)"
           << " : tot - 2.0 * part_;\n"
           << "      epart[((size_t)b * " << (1u << (W_ - m_)) << "u + tis) * " << W_ << " + i] = e;\n    }\n  }\n";
    }

    // per qubit of the readout: kind (0 register bit, 1 thread bit, 2 out-of-tile)
    // and the reduced value's index (kinds 0, 1) or the index-bit shift (kind 2)
    std::string readout_table(const Layout& L) const {
        std::ostringstream e;
        e << "__device__ const int " << name_ << "_eq[" << 2 * W_ << "] = {";
        for (int i = 0; i < W_; ++i) {
            const int sh = W_ - 1 - i;
            int kind = 2, idx = sh;
            for (int r = 0; r < kRegBits; ++r)
                if (lq(L.reg[r]) == sh) { kind = 0; idx = 1 + r; }
            for (int j = 0; j < (int)L.nonreg.size(); ++j)
                if (lq(L.nonreg[j]) == sh) { kind = 1; idx = 1 + kRegBits + j; }
            e << (i ? "," : "") << kind << "," << idx;
        }
        e << "};\n";
        return e.str();
    }

    void emit_kernel(const std::string& name) {
        name_ = name;
        const int tb = W_ - m_;
        if (last_fwd_) {
            o_ << readout_table(make_layout(m_, nat_reg().data()));
        }
        if (bwd_ && ps_->n_gout) {
            // gradient outputs of this pass: ordinal, axis, component slots x/y/z, matrix slot
            o_ << "__device__ const int " << name << "_out[" << 6 * ps_->n_gout << "] = {";
            for (int j = 0; j < ps_->n_gout; ++j) {
                const DGOut& go = p_->gouts[ps_->gout0 + j];
                o_ << (j ? "," : "") << go.ord << "," << go.axis << "," << go.c0 << "," << go.c1 << ","
                   << go.c2 << "," << go.mat;
            }
            o_ << "};\n";
        }
        o_ << "extern \"C\" __global__ void __launch_bounds__(" << threads_ << ") " << name << "(";
        if (bwd_)
            o_ << "const f2* __restrict__ psiN, f2* __restrict__ psi, f2* __restrict__ lam, "
                  "const double* __restrict__ gout, const float* __restrict__ mats, int n_shared, int n_ps, "
                  "double* __restrict__ part, int B)\n{\n";
        else
            o_ << "f2* __restrict__ state, const float* __restrict__ mats, int n_shared, int n_ps"
               << (last_fwd_ ? ", double* __restrict__ epart" : "") << ")\n{\n";
        o_ << "  __shared__ f2 lds[" << (1 << m_) << "];\n";
        int ng = bwd_ ? ps_->n_gslots : 0;
        const int nw = threads_ / 64;
        // per-row float32 partials of every gradient slot: [wave * 4 + row][slot]
        if (bwd_ && ng) o_ << "  __shared__ float red[" << nw * 4 * ng << "];\n";
        o_ << "  const int t = threadIdx.x;\n";
        o_ << "  const int q4_ = t & 3; const bool lo4_ = q4_ < 2, im4_ = q4_ & 1; (void)lo4_; (void)im4_;\n";
        if (guard_) o_ << "  const bool act = t < " << T_ << ";\n";
        // Workgroups are dealt to the chip's 8 XCDs in turn (workgroup i to XCD
        // i mod 8), each with its own L2. When the tile count divides by 8, XCD x
        // takes the contiguous tile range [x n/8, (x+1) n/8): the tiles one XCD
        // holds at a time are then neighbours in the state (adjacent runs of the
        // lowest out-of-tile bits), not tiles 8 apart. 28 qubits: 54.2 -> 51.7 ms
        // per step; neutral on the ALU-bound passes.
        o_ << "  const unsigned tile = (gridDim.x & 7u) ? blockIdx.x : (blockIdx.x & 7u) * (gridDim.x >> 3) + "
              "(blockIdx.x >> 3);\n"
           << "  const int b = (int)(tile >> " << tb << ");\n"
           << "  const int tis = (int)(tile & " << hex((1u << tb) - 1) << ");\n";
        {
            std::vector<int> pos;
            for (int k = 0; k < tb; ++k) pos.push_back(ps_->oq[k]);
            o_ << "  const int base = " << (tb ? scatter("tis", pos) : "0") << ";\n";
        }
        o_ << "  const size_t off = (size_t)b << " << W_ << ";\n"
           << "  const float* mp = mats + ((size_t)n_shared + (size_t)b * n_ps) * 8;\n"
           << "  (void)mp;\n";
        Layout nat = make_layout(m_, nat_reg().data());
        // With tile bit 0 = amplitude bit 0 in registers 0 and 1 of each pair,
        // a thread moves its amplitudes as 16-byte pairs when the array is
        // 16-byte aligned (a wave-uniform test; 8-byte aligned arrays take
        // single-amplitude accesses).
        const bool v16 = lq(0) == 0;
        Layout cur = nat;
        o_ << "  int gT = " << gT_expr(cur) << ";\n";
        for (const std::string& A : arrays_) o_ << "  f2 " << A << "[16];\n";
        if (guard_)
            for (const std::string& A : arrays_)
                o_ << "  for (int k = 0; k < 16; ++k) " << A << "[k] = make_float2(0.f, 0.f);\n";
        auto gload = [&](const std::string& A, const std::string& src) {
            std::string s1;
            for (int k = 0; k < kRegs; ++k) s1 += A + "[" + I(k) + "] = " + src + "[gT + " + I(gR(cur, k)) + "]; ";
            if (!v16) return s1;
            std::string s2;
            for (int k = 0; k < kRegs; k += 2)
                s2 += "{ const float4 v_ = *reinterpret_cast<const float4*>(" + src + " + gT + " + I(gR(cur, k)) + "); " +
                      A + "[" + I(k) + "] = make_float2(v_.x, v_.y); " + A + "[" + I(k + 1) +
                      "] = make_float2(v_.z, v_.w); } ";
            return "if (((qsv_uptr)(" + src + ") & 15) == 0) { " + s2 + "} else { " + s1 + "}";
        };
        auto gstore = [&](const std::string& A, const std::string& dst) {
            std::string s1;
            for (int k = 0; k < kRegs; ++k) s1 += dst + "[gT + " + I(gR(cur, k)) + "] = " + A + "[" + I(k) + "]; ";
            if (!v16) return s1;
            std::string s2;
            for (int k = 0; k < kRegs; k += 2)
                s2 += "*reinterpret_cast<float4*>(" + dst + " + gT + " + I(gR(cur, k)) + ") = make_float4(" + A + "[" +
                      I(k) + "].x, " + A + "[" + I(k) + "].y, " + A + "[" + I(k + 1) + "].x, " + A + "[" + I(k + 1) +
                      "].y); ";
            return "if (((qsv_uptr)(" + dst + ") & 15) == 0) { " + s2 + "} else { " + s1 + "}";
        };
        const int flags = ps_->flags;
        if (!bwd_ && (flags & PF_INIT_FWD)) {
            // The first pass generates the product state of the leading 1-qubit
            // gates instead of loading it: amplitude idx is the product over
            // qubits q of column 0 of q's prefix matrix, entry bit_q(idx).
            o_ << "  f2* st = state + off;\n  {\n    f2 P_ = make_float2(1.f, 0.f);\n";
            auto vq = [&](int q) {
                const int slot = p_->prefix_mat[q];
                return slot >= 0 ? "mats + " + I(8LL * slot) : "mp + " + I(8LL * (-slot - 1));
            };
            std::vector<int> reg_shift(kRegBits);
            for (int r = 0; r < kRegBits; ++r) reg_shift[r] = lq(cur.reg[r]);
            for (int q = 0; q < W_; ++q) {
                const int sh = W_ - 1 - q;
                if (std::find(reg_shift.begin(), reg_shift.end(), sh) != reg_shift.end()) continue;
                o_ << "    { const float* v_ = " << vq(q) << "; const int bt_ = (gT >> " << sh << ") & 1;\n"
                   << "      const f2 u_ = bt_ ? make_float2(v_[4], v_[5]) : make_float2(v_[0], v_[1]);\n"
                   << "      P_ = make_float2(P_.x * u_.x - P_.y * u_.y, P_.x * u_.y + P_.y * u_.x); }\n";
            }
            // register qubits: a[k] = P_ * prod_r v_r[bit r of k], built as a doubling tree
            o_ << "    a[0] = P_;\n";
            for (int r = 0; r < kRegBits; ++r) {
                const int q = W_ - 1 - reg_shift[r];
                o_ << "    { const float* v_ = " << vq(q) << ";\n"
                   << "      const f2 u0_ = make_float2(v_[0], v_[1]), u1_ = make_float2(v_[4], v_[5]);\n";
                for (int k = (1 << r) - 1; k >= 0; --k) {
                    const int k1 = k | (1 << r);
                    o_ << "      a[" << k1 << "] = make_float2(a[" << k << "].x * u1_.x - a[" << k << "].y * u1_.y, a["
                       << k << "].x * u1_.y + a[" << k << "].y * u1_.x);\n"
                       << "      a[" << k << "] = make_float2(a[" << k << "].x * u0_.x - a[" << k << "].y * u0_.y, a["
                       << k << "].x * u0_.y + a[" << k << "].y * u0_.x);\n";
                }
                o_ << "    }\n";
            }
            o_ << "  }\n";
        } else if (!bwd_) {
            o_ << "  f2* st = state + off;\n  " << act(gload("a", "st")) << "\n";
        } else if (flags & PF_FIRST_BWD) {
            o_ << "  " << act(gload("ps", "(psiN + off)")) << "\n";
            // lambda = D psi with D(idx) = G0 - 2 sum_{i: bit_i(idx) = 1} g_i
            o_ << "  {\n    const double* g_ = gout + (size_t)b * " << W_ << ";\n"
               << "    double G0 = 0.0, DT = 0.0;\n"
               << "    for (int i = 0; i < " << W_ << "; ++i) { const double gi = g_[i]; G0 += gi; "
               << "if ((gT >> (" << W_ - 1 << " - i)) & 1) DT += gi; }\n";
            for (int p = 0; p < kRegBits; ++p)
                o_ << "    const double gp" << p << " = g_[" << W_ - 1 - lq(cur.reg[p]) << "];\n";
            for (int k = 0; k < kRegs; ++k) {
                std::string dr = "DT";
                for (int p = 0; p < kRegBits; ++p)
                    if (k >> p & 1) dr += " + gp" + I(p);
                o_ << "    { const float d = (float)(G0 - 2.0 * (" << dr << ")); lm[" << k << "] = make_float2(d * ps["
                   << k << "].x, d * ps[" << k << "].y); }\n";
            }
            o_ << "  }\n";
        } else {
            o_ << "  " << act(gload("ps", "(psi + off)") + gload("lm", "(lam + off)")) << "\n";
        }
        if (bwd_ && ng) {
            for (int j = 0; j < ng; ++j) o_ << "  float g" << j << " = 0.f;\n";
        }
        o_ << "  const int wave = t >> 6, lane = t & 63; (void)wave; (void)lane;\n";
        for (int s = 0; s < ps_->n_stages; ++s) {
            const DStage& st = p_->stages[ps_->stage0 + s];
            Layout L = make_layout(m_, st.reg);
            if (!same(L, cur)) {
                emit_exchange(cur, L);
                cur = L;
            }
            lay_ = &cur;
            for (int oi = st.op0; oi < st.op1; ++oi) {
                const DOp& op = p_->ops[oi];
                if (op.kind >= OP_GX) {
                    emit_grad(op);
                    // row reduction of the partial right away (float32 within a
                    // 16-lane row; rows are combined in float64 at the end of the
                    // pass). Every lane of a row holds the row's sum and stores it
                    // (same value, same address): no branch, which keeps the
                    // compiler's register allocation across the kernel intact.
                    o_ << "  { const float r_ = qsv_row_sum(g" << op.slot << "); red[(wave * 4 + (lane >> 4)) * "
                       << ng << " + " << op.slot << "] = r_; }\n";
                } else {
                    emit_apply(op);
                }
            }
        }
        lay_ = nullptr;  // cur goes out of scope with this kernel
        const bool write_back = !bwd_ || !(flags & PF_LAST_BWD);
        if (write_back) {
            if (!same(cur, nat)) {
                emit_exchange(cur, nat);
                cur = nat;
            }
            if (!bwd_) o_ << "  " << act(gstore("a", "st")) << "\n";
            else o_ << "  " << act(gstore("ps", "(psi + off)") + gstore("lm", "(lam + off)")) << "\n";
        }
        if (last_fwd_) emit_readout(cur);
        if (bwd_ && ng) {
            o_ << "  __syncthreads();\n";
            o_ << "  {\n    __shared__ double cs_[" << ng << "];\n";
            o_ << "    for (int j = t; j < " << ng << "; j += " << threads_ << ") {\n"
               << "      double s = 0.0;\n";
            for (int r = 0; r < nw * 4; ++r) o_ << "      s += (double)red[" << r * ng << " + j];\n";
            o_ << "      cs_[j] = s;\n    }\n    __syncthreads();\n";
            o_ << "    const int* out_ = " << name << "_out;\n"
               << "    for (int j = t; j < " << ps_->n_gout << "; j += " << threads_ << ") {\n"
               << "      const int* e = out_ + 6 * j;\n"
               << "      double v;\n"
               << "      if (e[1] < 0) v = cs_[e[2]];\n"
               << "      else v = qsv_chain_grad(e[5] >= 0 ? mats + 8 * (size_t)e[5] : mp + 8 * (size_t)(-e[5] - 1), "
                  "e[1], e[2] >= 0 ? cs_[e[2]] : 0.0, e[3] >= 0 ? cs_[e[3]] : 0.0, e[4] >= 0 ? cs_[e[4]] : 0.0);\n"
               << "      part[((size_t)e[0] * B + b) * " << (1u << tb) << "u + tis] = v;\n    }\n  }\n";
        }
        o_ << "}\n\n";
    }
};

std::string arch_of_device() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
    return prop.gcnArchName;
}

uint64_t fnv1a(const std::string& s) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : s) { h ^= c; h *= 1099511628211ull; }
    return h;
}

const char* const kOpts[] = {"-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};

std::string cache_path(const std::string& src, const std::string& arch) {
    const char* dir = std::getenv("QSV_JIT_CACHE");
    if (!dir || !*dir) return "";
    char b[40];
    // the tag changes whenever the compiler options below change
    std::snprintf(b, sizeof b, "%016llx", (unsigned long long)fnv1a(src + "|" + arch + "|opts2"));
    return std::string(dir) + "/qsv_" + b + ".co";
}

bool read_file(const std::string& path, std::vector<char>& out) {
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    out.assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
    return !out.empty();
}

void write_cache(const std::string& path, const std::vector<char>& code) {
    if (path.empty()) return;
    const std::string tmp = path + ".tmp" + std::to_string((long long)getpid()) + "_" +
                            std::to_string((long long)std::hash<std::thread::id>()(std::this_thread::get_id()));
    std::ofstream f(tmp, std::ios::binary);
    f.write(code.data(), (std::streamsize)code.size());
    f.close();
    std::rename(tmp.c_str(), path.c_str());
}

// The ROCm clang driver, if installed (QSV_JIT_CLANG overrides; "none" disables).
std::string find_clang() {
    const char* env = std::getenv("QSV_JIT_CLANG");
    if (env && *env) return std::string(env) == "none" ? "" : env;
    const char* rp = std::getenv("ROCM_PATH");
    const std::string cands[] = {std::string(rp ? rp : "/opt/rocm") + "/llvm/bin/clang++",
                                 "/opt/rocm/llvm/bin/clang++"};
    for (const auto& c : cands)
        if (access(c.c_str(), X_OK) == 0) return c;
    return "";
}

extern "C" char** environ;

// Compile sources in parallel child processes of the clang driver.
int compile_children(const std::string& clang, const std::vector<std::string>& srcs,
                     const std::string& arch, std::vector<std::vector<char>>& codes,
                     std::vector<int>& todo, std::string& err) {
    const char* tmpenv = std::getenv("TMPDIR");
    std::string tmpl = std::string(tmpenv && *tmpenv ? tmpenv : "/tmp") + "/qsv_jit_XXXXXX";
    std::vector<char> dirbuf(tmpl.begin(), tmpl.end());
    dirbuf.push_back(0);
    if (!mkdtemp(dirbuf.data())) {
        err = "mkdtemp failed";
        return QSV_ERR_HIP;
    }
    const std::string dir = dirbuf.data();
    const int maxpar = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
    const std::string arch_opt = "--offload-arch=" + arch;
    int rc = QSV_OK;
    size_t next = 0;
    std::vector<std::pair<pid_t, int>> running;
    auto paths = [&](int i, const char* ext) { return dir + "/k" + std::to_string(i) + ext; };
    while ((next < todo.size() || !running.empty()) && rc == QSV_OK) {
        while (next < todo.size() && (int)running.size() < maxpar) {
            const int i = todo[next++];
            {
                std::ofstream f(paths(i, ".hip"));
                f << srcs[i];
            }
            const std::string in = paths(i, ".hip"), out = paths(i, ".co"), log = paths(i, ".log");
            std::vector<std::string> args = {clang, "-x", "hip", arch_opt, "--cuda-device-only",
                                             "--no-gpu-bundle-output", "-O3", "-std=c++17",
                                             "-include", "hip/hip_runtime.h",
                                             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                                             "-mllvm", "-amdgpu-mfma-vgpr-form=1", "-o", out, in};
            std::vector<char*> argv;
            for (auto& a : args) argv.push_back(&a[0]);
            argv.push_back(nullptr);
            posix_spawn_file_actions_t fa;
            posix_spawn_file_actions_init(&fa);
            posix_spawn_file_actions_addopen(&fa, 1, log.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
            posix_spawn_file_actions_adddup2(&fa, 1, 2);
            pid_t pid;
            const int e = posix_spawn(&pid, clang.c_str(), &fa, nullptr, argv.data(), environ);
            posix_spawn_file_actions_destroy(&fa);
            if (e != 0) {
                err = "cannot start " + clang;
                rc = QSV_ERR_HIP;
                break;
            }
            running.emplace_back(pid, i);
        }
        if (running.empty()) break;
        int status = 0;
        const pid_t done = waitpid(-1, &status, 0);
        if (done < 0) {
            err = "waitpid failed";
            rc = QSV_ERR_HIP;
            break;
        }
        for (size_t r = 0; r < running.size(); ++r) {
            if (running[r].first != done) continue;
            const int i = running[r].second;
            running.erase(running.begin() + (long)r);
            if (!WIFEXITED(status) || WEXITSTATUS(status) != 0 || !read_file(paths(i, ".co"), codes[i])) {
                std::vector<char> log;
                read_file(paths(i, ".log"), log);
                err = "kernel compile failed: " + std::string(log.begin(), log.end()).substr(0, 2000);
                rc = QSV_ERR_HIP;
            }
            break;
        }
    }
    for (auto& r : running) waitpid(r.first, nullptr, 0);
    for (size_t i = 0; i < srcs.size(); ++i)
        for (const char* ext : {".hip", ".co", ".log"}) std::remove(paths((int)i, ext).c_str());
    rmdir(dir.c_str());
    return rc;
}

}  // namespace

// Compile one group of kernels (source) for `arch` with hipRTC.
static int compile_group(const std::string& src, const std::string& arch, std::vector<char>& code,
                         std::string& log) {
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "qsv_jit.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        log = "hiprtcCreateProgram failed";
        return QSV_ERR_HIP;
    }
    std::vector<const char*> opts(std::begin(kOpts), std::end(kOpts));
    const std::string arch_opt = "--offload-arch=" + arch;
    opts.push_back(arch_opt.c_str());
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    if (n > 1) {
        log.resize(n);
        hiprtcGetProgramLog(prog, &log[0]);
    }
    if (r != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        return QSV_ERR_HIP;
    }
    hiprtcGetCodeSize(prog, &n);
    code.resize(n);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return QSV_OK;
}

std::string jit_source(const qsv_plan_t* p, std::vector<JitKernelRef>& refs, int max_ops_per_group) {
    Gen g(p);
    std::string all;
    refs.clear();
    int group = 0, ops_in_group = 0;
    for (int which = 0; which < 2; ++which) {
        const auto& passes = which == 0 ? p->fwd_pass : p->bwd_pass;
        for (int i = 0; i < (int)passes.size(); ++i) {
            int nops = 0;
            for (int s = passes[i].stage0; s < passes[i].stage0 + passes[i].n_stages; ++s)
                nops += p->stages[s].op1 - p->stages[s].op0;
            if (ops_in_group && ops_in_group + nops > max_ops_per_group) {
                ++group;
                ops_in_group = 0;
            }
            ops_in_group += nops;
            JitKernelRef r;
            r.which = which;
            r.pass = i;
            r.group = group;
            r.source = g.kernel(which, i, r.name);
            refs.push_back(r);
        }
    }
    for (auto& r : refs) all += r.source;
    return g.prelude() + all;
}

int jit_compile(const qsv_plan_t* p, const std::string& arch_in, JitModules& out, std::string& err) {
    std::vector<JitKernelRef> refs;
    Gen g(p);
    jit_source(p, refs, 1);  // one kernel per compilation unit: compiled in parallel
    const std::string arch = arch_in.empty() ? arch_of_device() : arch_in;
    if (arch.empty()) {
        err = "cannot determine the device architecture";
        return QSV_ERR_HIP;
    }
    int ngroups = refs.empty() ? 0 : refs.back().group + 1;
    std::vector<std::string> srcs(ngroups, g.prelude());
    for (auto& r : refs) srcs[r.group] += r.source;
    std::vector<std::vector<char>> codes(ngroups);
    std::vector<int> todo;
    for (int i = 0; i < ngroups; ++i)
        if (!read_file(cache_path(srcs[i], arch), codes[i])) todo.push_back(i);
    const std::string clang = find_clang();
    if (!todo.empty() && !clang.empty()) {
        int rc = compile_children(clang, srcs, arch, codes, todo, err);
        if (rc != QSV_OK) return rc;
    } else {
        for (int i : todo) {
            std::string log;
            if (compile_group(srcs[i], arch, codes[i], log) != QSV_OK) {
                err = "hipRTC compile failed: " + log.substr(0, 2000);
                return QSV_ERR_HIP;
            }
        }
    }
    for (int i : todo) write_cache(cache_path(srcs[i], arch), codes[i]);
    out.codes = std::move(codes);
    out.refs = std::move(refs);
    out.arch = arch;
    return QSV_OK;
}

}  // namespace qsv
