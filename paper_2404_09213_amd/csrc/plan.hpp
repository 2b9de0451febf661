// plan.hpp -- host-side plan: gate-matrix cache, split, pass/stage schedule,
// and the flat tables the kernels read. Shared by planner.cpp and qsv.hip.
#pragma once

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "qsv.h"

namespace qsv {

constexpr int kRegBits = 4;            // amplitudes per thread in a tile = 2^kRegBits
constexpr int kRegs = 1 << kRegBits;
constexpr int kMaxTileQubits = 14;        // generated kernels
constexpr int kMaxTileQubitsTables = 12;  // table-driven kernels (256 threads)
constexpr int kMaxQ = 32;

// ---- device-visible tables (plain old data, copied verbatim to the GPU) ----

// One gate of the cache: its matrix is C + cos(theta/2) A + sin(theta/2) S
// (2x2 complex, row-major, interleaved re/im), the generalisation of Eq. (1)
// to every kind. Fixed gates have A = S = 0.
struct DGate {
    int32_t kind, src, idx, pad;
    double C[8], A[8], S[8];
};

// A recipe: the ordered product of `count` gates (recipe_gates[first ..]),
// optionally daggered. Evaluated once per call (per sample if any gate reads
// an input). out >= 0: shared slot; out < 0: per-sample slot (-out - 1).
struct DRecipe {
    int32_t first, count, dagger, out;
};

enum OpKind : int32_t {
    OP_U2 = 0,     // generic 2x2 on register position `pos`, optional control
    OP_REAL = 1,   // 2x2 with real entries
    OP_RXL = 2,    // [[a, ib], [ib, a]] with real a, b (RX family)
    OP_DIAG = 3,   // diag(m00, m11) on a qubit; pos >= 0 register, else `sh` global shift
    OP_SIGN = 4,   // product of CZ / Z signs (a sign group), see DTerm
    OP_SWAP = 5,   // X / CNOT target: exchange the pair (optional control)
    OP_GX = 6,     // gradient partial, generator X on `pos` (optional control)
    OP_GY = 7,     // gradient partial, generator Y on `pos`
    OP_GZ = 8,     // gradient partial, generator Z; pos >= 0 register, else `sh`
};

// Control encoding: ctl = -1 none; 0..3 register position; 0x100 | shift for
// a qubit outside the registers (thread bit or out-of-tile bit).
constexpr int32_t kCtlNonReg = 0x100;

struct DOp {
    int32_t kind;
    int32_t pos;      // register position of the target, or -1
    int32_t ctl;      // first control, see above (-1 none)
    int32_t mat;      // matrix slot (>= 0 shared, < 0 per-sample: -mat-1)
    int32_t slot;     // local gradient slot within the pass (OP_G*)
    int32_t sh;       // global bit shift for non-register diagonal / GZ ops
    int32_t term0;    // OP_SIGN: first term
    int32_t nterm;    // OP_SIGN: number of terms; uniform 16-bit mask in `pos`
    int32_t ctl2;     // second control, same encoding (-1 none)
    int32_t pad;
};

// Sign term of an OP_SIGN group, for one stage layout: if every listed bit
// (s0, s1, s2; -1 = unused) of the thread's global index is set, flip the
// registers in `mask`. A CZ / CCZ contributes its register-only part to the
// op's uniform mask and its other qubits as a term.
struct DTerm {
    int32_t s0, s1, s2, mask;
};

struct DStage {
    int32_t reg[kRegBits];  // local tile bits held in registers, position p -> local bit
    int32_t op0, op1;       // ops [op0, op1)
    int32_t pad[2];
};

enum PassFlags : int32_t {
    PF_FIRST_BWD = 1,  // backward: read psi_N from the caller's state, build lambda on the fly
    PF_LAST_BWD = 2,   // backward: nothing is written back
    PF_INIT_FWD = 4,   // forward: generate the product-state init instead of loading
};

struct DPass {
    int32_t m;            // tile qubits
    int32_t n_stages;
    int32_t stage0;
    int32_t flags;
    int32_t n_gslots;     // backward: gradient component slots (one float sum each)
    int32_t gout0;        // backward: first gradient output (DGOut) of this pass
    int32_t n_gout;       // backward: gradient outputs of this pass
    int32_t pad;
    int32_t lq[kMaxQ];    // local tile bit j -> global bit shift (W-1-qubit), j < m
    int32_t oq[kMaxQ];    // tile-index bit k -> global bit shift, k < W-m
};

// One parametric gate's gradient partial, formed at the end of a backward
// pass from the pass's component sums c[slot] (slot -1 reads as 0):
//   axis < 0: value = c[c0]                     (the gate's own Im<l|P|psi>)
//   axis 0/1/2 (generator X/Y/Z): with V = matrix slot `mat` (the product of
//   the later gates of the gate's 1-qubit chain) and H = V P V^dagger,
//   value = H00 c[cz] + Re(H01) c[cx] - Im(H01) c[cy], where c[cx], c[cy],
//   c[cz] are Im<l|X|psi>, Im<l|Y|psi>, Im<l|Z|psi> on the chain's qubit taken
//   after the whole chain (c0, c1, c2 = cx, cy, cz).
struct DGOut {
    int32_t ord;          // parametric ordinal (partial row)
    int32_t axis;
    int32_t c0, c1, c2;
    int32_t mat;
    int32_t pad[2];
};

// Per-gate (plain method) launch description.
struct PGate {
    int32_t gate;       // gate index
    int32_t cls;        // OpKind of the apply step (U2/REAL/RXL/DIAG/SIGN/SWAP)
    int32_t tsh, csh;   // target / first control global shifts (-1 none)
    int32_t mat;        // matrix slot
    int32_t grad;       // OP_GX/GY/GZ or -1
    int32_t slot;       // parametric gate ordinal or -1
    int32_t sh2;        // OP_SIGN: second qubit's shift
    int32_t csh2;       // second control shift (OP_SIGN: third qubit of a CCZ), -1 none
    int32_t pad;
};

// One circuit of a multi-circuit plan.
struct DCirc {
    int32_t W, m;           // qubits, tile qubits
    int32_t n_fwd, n_bwd;   // passes
    int32_t fwd0, bwd0;     // first pass in the concatenated pass arrays
    int32_t e0;             // first expectation column (sum of earlier circuits' qubits)
    int32_t pm0;            // first prefix-matrix entry
    int64_t amp0;           // amplitude offset within a sample row
    int32_t ic0;            // first readout / init chunk (chunks of 2^min(W,12) amplitudes)
    int32_t nchunk;         // chunks per sample
};

// A work item of a multi-circuit launch: one tile of one pass of one circuit.
struct DItem {
    int32_t c, pass, tile;  // circuit, pass index within the circuit, tile within the pass
    int32_t pad[3];
};

// ---- host plan ----

struct Block {
    std::vector<int> gates;
    uint32_t Q = 0;   // all qubits touched
};

struct DeviceTables {
    void* base = nullptr;  // one allocation holding everything below
    DGate* gates = nullptr;
    DRecipe* recipes = nullptr;
    int32_t* recipe_gates = nullptr;
    DPass* fwd_pass = nullptr;
    DPass* bwd_pass = nullptr;
    DStage* stages = nullptr;
    DOp* ops = nullptr;
    DTerm* terms = nullptr;
    DGOut* gouts = nullptr;
    int32_t* prefix_mat = nullptr;
    int32_t* grad_csr = nullptr;   // weights then inputs: offsets, then slot lists
    int64_t* pu = nullptr;         // per parametric ordinal: partial offset in units of B
    int32_t* nchv = nullptr;       // per parametric ordinal: partial chunks per sample
    DCirc* circ = nullptr;         // multi-circuit plans
    // multi-circuit work lists per batch size, grouped in rounds (item offsets)
    struct Queue {
        int64_t B;
        DItem* fwd; int n_fwd;
        DItem* bwd; int n_bwd;
        void* mem;
        std::vector<int> fwd_rounds, bwd_rounds;
    };
    std::vector<Queue> queues;
    // generated pass kernels (hipModule_t / hipFunction_t, kept opaque here)
    std::vector<void*> modules;
    std::vector<void*> fwd_fn, bwd_fn;
};

}  // namespace qsv

struct qsv_plan_s {
    int W, n_gates, n_weights, n_inputs;
    qsv_opts opts;
    std::vector<qsv_gate> gates;

    // gate-matrix cache
    std::vector<qsv::DGate> dgates;
    std::vector<qsv::DRecipe> recipes;
    std::vector<int32_t> recipe_gates;
    int n_shared_mats = 0, n_ps_mats = 0;

    // product-state prefix: per qubit a matrix slot (identity recipe if none)
    std::vector<int> prefix_gates;      // gate indices folded into init
    std::vector<int32_t> prefix_mat;    // W entries

    // splitter output over the whole gate list
    std::vector<qsv::Block> blocks;
    std::vector<int32_t> block_of_gate;

    // fused schedule
    std::vector<qsv::DPass> fwd_pass, bwd_pass;
    std::vector<qsv::DStage> stages;
    std::vector<qsv::DOp> ops;
    std::vector<qsv::DTerm> terms;
    std::vector<qsv::DGOut> gouts;      // backward gradient outputs (per pass ranges)

    // per-gate schedule
    std::vector<qsv::PGate> pg_fwd, pg_bwd;

    // parametric gates and gradient gathering
    std::vector<int32_t> param_ordinal;  // gate -> ordinal or -1
    std::vector<int32_t> param_gate;     // ordinal -> gate
    std::vector<int32_t> grad_csr;       // [n_weights+1 offsets][n_inputs+1 offsets][slots...]
    int n_param = 0;

    // gate orders for introspection
    std::vector<int32_t> fwd_order, bwd_order;
    int n_fwd_stages = 0, n_bwd_stages = 0;

    // algorithmic float32 operations per amplitude of each launch (profiling)
    std::vector<double> fwd_pass_flops, bwd_pass_flops, pg_fwd_flops, pg_bwd_flops;

    // profiling state (opaque; owned by the HIP side)
    mutable void* prof = nullptr;

    // gradient partial layout (all methods): ordinal o, sample b, chunk k at
    // part[B * pu[o] + b * nchv[o] + k]
    std::vector<int64_t> pu;
    std::vector<int32_t> nchv;
    int64_t pu_total = 0;

    // multi-circuit plans: circuits simulated together, one launch per round of passes
    bool multi = false;
    std::vector<qsv::DCirc> circ;
    int Wtot = 0;          // expectation columns (sum of qubits)
    int64_t row = 0;       // amplitudes per sample row (sum of 2^W)
    int64_t nchunk_tot = 0;
    int n_fwd_tot = 0, n_bwd_tot = 0;  // passes over all circuits
    std::vector<int32_t> circ_w0, circ_x0;  // first weight / input column of each circuit

    // lazily created device copies, per device ordinal
    mutable std::mutex dev_mu;
    mutable std::map<int, qsv::DeviceTables> dev;
};

namespace qsv {
// chunks per sample of the plain method's gradient partials
inline int64_t pg_chunks(int W) {
    const int64_t q = int64_t(1) << (W - 2 > 0 ? W - 2 : 0);
    return q / 1024 > 1 ? q / 1024 : 1;
}
int build_plan(qsv_plan_t* p);  // planner.cpp
struct CircuitIn { int W; const qsv_gate* gates; int n_gates, n_weights, n_inputs; qsv_opts opts; };
int build_multi(qsv_plan_t* p, const std::vector<CircuitIn>& cs);  // planner.cpp
void set_error(const std::string& msg);       // api
}  // namespace qsv
