/*
 * qsv.h -- C ABI of libqsv: batched state-vector simulation of parameterised
 * quantum circuits on one AMD Instinct MI355X (gfx950), with Pauli-Z readout
 * and adjoint gradients.
 *
 * What is computed (the paper's problem statement, sections "State Vector
 * Simulation", "Hybrid Machine Learning" and "Concept of Shapes"): a circuit
 * of W qubits is a list of gates; every sample b of a batch starts in
 * |0...0>, has the gates applied in order, and is read out as
 * E[b,i] = <psi_b| Z_i |psi_b>. Gate angles come from a shared weight vector
 * (trainable layers) or from a per-sample input row (embedding layers).
 *
 * Conventions:
 *  - MSb-0 ordering (section "Symbols"): qubit w is bit (W-1-w) of a
 *    basis-state index.
 *  - Rotations R_d(theta) = exp(-i theta sigma_d / 2) (Eq. (1) for d = x):
 *    RX = [[c,-is],[-is,c]], RY = [[c,-s],[s,c]], RZ = diag(e^{-i t/2}, e^{i t/2})
 *    with c = cos(theta/2), s = sin(theta/2). H = (X+Z)/sqrt2. CNOT(c,t) flips
 *    t where c = 1; CZ(a,b) negates where both are 1; CRX(c,t) applies RX to t
 *    where c = 1. For 2-qubit gates q0 is the control, q1 the target.
 *  - State layout: sample-major (B, 2^W) complex64, interleaved (re, im) float
 *    pairs; amplitude idx of sample b at float offset 2 * (b * 2^W + idx).
 *    Plans with amp_dtype = QSV_AMP_C128 use complex128 (interleaved double
 *    pairs) in the same order.
 *  - Expectations and gradients are float64; amplitudes and gate arithmetic
 *    are float32 (float64 with amp_dtype = QSV_AMP_C128).
 *
 * Ownership: every d_ pointer is device memory owned by the caller; the
 * library never frees it. A plan owns its host tables and the device copies
 * it makes of them (created on first use on a device, freed by
 * qsv_plan_destroy). Workspaces are caller memory of at least
 * qsv_workspace_size() bytes, 256-byte aligned.
 *
 * Asynchrony: qsv_forward / qsv_forward_expval / qsv_expval / qsv_backward
 * validate on the host, then enqueue kernels on `stream` (a hipStream_t,
 * NULL = default stream) and return; faults show at the caller's next
 * synchronisation. On a non-zero return nothing was enqueued.
 *
 * Errors: functions return 0 or a negative QSV_ERR_* code; qsv_last_error()
 * gives a thread-local message for the last failure in this thread.
 *
 * Thread safety: a plan is immutable after creation except for its lazily
 * created per-device tables, which are guarded by a lock. Concurrent calls
 * on one plan are safe when they use distinct workspaces and outputs.
 */
#ifndef QSV_H_INCLUDED
#define QSV_H_INCLUDED

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* gate kinds. Controlled kinds list their controls first: q0 for one
 * control (target q1), q0 and q1 for two controls (target q2). The target
 * part of a controlled kind is the gate of the same letter: CRY(c,t) applies
 * RY to t where c = 1, CRZ likewise, CCX (Toffoli) flips t where both
 * controls are 1, CCZ negates where all three qubits are 1, CCRX applies RX
 * to t where both controls are 1 (multi-controlled gates, named as future
 * work in section "Conclusion"). */
enum {
    QSV_H = 0, QSV_X = 1, QSV_Y = 2, QSV_Z = 3,
    QSV_RX = 4, QSV_RY = 5, QSV_RZ = 6,
    QSV_CNOT = 7, QSV_CZ = 8, QSV_CRX = 9,
    QSV_CRY = 10, QSV_CRZ = 11, QSV_CCX = 12, QSV_CCZ = 13, QSV_CCRX = 14
};

/* where a gate's angle comes from */
enum { QSV_SRC_NONE = 0, QSV_SRC_WEIGHT = 1, QSV_SRC_INPUT = 2 };

/* return codes */
enum {
    QSV_OK = 0,
    QSV_ERR_ARG = -1,      /* null pointer, batch <= 0, workspace too small, bad option */
    QSV_ERR_QUBIT = -2,    /* qubit index out of range, or a gate naming one qubit twice */
    QSV_ERR_GATE = -3,     /* unknown gate kind */
    QSV_ERR_PARAM = -4,    /* angle source / index invalid for the gate */
    QSV_ERR_TOO_BIG = -5,  /* W > QSV_MAX_QUBITS, the state size overflows, a
                              launch would exceed HIP's grid limit (see
                              tile_qubits) or more than 2^24 gradient outputs */
    QSV_ERR_OOM = -6,      /* host or device allocation failed */
    QSV_ERR_HIP = -7,      /* a HIP runtime call failed; see qsv_last_error() */
    QSV_ERR_HANDLE = -8    /* null or destroyed plan */
};

#define QSV_MAX_QUBITS 30

/* methods */
enum {
    QSV_METHOD_FUSED = 0,   /* circuit splitting + register/LDS tiles (default) */
    QSV_METHOD_PER_GATE = 1 /* the plain method: one strided sweep of the state per gate */
};

/* workspace queries; QSV_OP_STEP = forward + readout + backward (qsv_graph_create),
   QSV_OP_FORWARD_EXPVAL = qsv_forward_expval */
enum { QSV_OP_FORWARD = 0, QSV_OP_EXPVAL = 1, QSV_OP_BACKWARD = 2, QSV_OP_STEP = 3, QSV_OP_FORWARD_EXPVAL = 4 };

typedef struct {
    int32_t kind;  /* QSV_H ... QSV_CCRX */
    int32_t q0;    /* qubit (1-qubit gates) or first control */
    int32_t q1;    /* target of a 1-control gate, second control of a 2-control
                      gate; -1 for 1-qubit gates */
    int32_t src;   /* QSV_SRC_NONE | QSV_SRC_WEIGHT | QSV_SRC_INPUT */
    int32_t idx;   /* weights[idx] or inputs[b * n_inputs + idx]; -1 if src is NONE */
    int32_t q2;    /* target of a 2-control gate; -1 otherwise */
} qsv_gate;

/*
 * Plan options. The paper names one knob, the largest number of qubits of a
 * sub-circuit (section "Circuit Splitting"): fuse_width. The others are this
 * library's. Work-group size is not an option: a fused pass uses
 * max(64, 2^(tile_qubits - 4)) threads, 16 amplitudes each. Matrix-core use
 * is the `mfma` bit mask (there is no dense-block path: a 3-qubit block as one
 * 16x16x4 product measured slower than the 2x2 products it replaces).
 * Choosing options by measurement is the Python tuner's job (tune.py, over
 * qsv_plan_estimate and timed runs), and HIP-graph capture is a call of its
 * own (qsv_graph_create), not an option.
 */
typedef struct {
    int32_t method;      /* QSV_METHOD_FUSED or QSV_METHOD_PER_GATE */
    int32_t fuse_width;  /* k: max qubits of a splitter block (section "Circuit
                            Splitting" suggests 3..6); 1..16. A gate with more
                            qubits than k forms a block by itself, so k = 1
                            packs gate by gate (1-qubit chains, single
                            2-qubit gates), which gives the fewest passes */
    int32_t tile_qubits; /* m: qubits of one tile of amplitudes held by a
                            workgroup, 4..14 (4..12 when codegen = 0); clamped to W.
                            A call whose tiles x threads per tile (max(64, 2^(m-4)))
                            exceed 2^32 returns QSV_ERR_TOO_BIG: below m = 10 that
                            bounds the batch's amplitudes by 2^(26+m) */
    int32_t low_qubits;  /* c: number of lowest-stride qubits every tile keeps
                            (contiguous runs of 2^c amplitudes); 0..m-1 */
    int32_t max_pass_grads; /* cap on parametric gates per backward pass, 1..256 */
    int32_t codegen;     /* fused method: 1 = kernels generated for this plan and
                            compiled with hipRTC on first use on a device (default);
                            0 = table-driven kernels compiled into the library */
    int32_t bwd_gate_by_gate; /* 0 (default): in the backward, a chain of 1-qubit
                            gates on one qubit is uncomputed as one 2x2 product and
                            its gates' gradients are formed from the X, Y, Z
                            components taken after the chain, where that costs
                            fewer operations; 1: every gate is uncomputed on its own */
    int32_t mfma;        /* generated kernels: generic 2x2 products on the matrix
                            cores (v_mfma_f32_4x4x1_16b: each lane multiplies its own
                            amplitude pair, as a real 4-vector, by the gate's real 4x4
                            form). Bit mask, 0..7: 1 forward kernels (default 1),
                            2 backward psi, 4 backward lambda; 0 = everything on the
                            vector ALU */
    int32_t weight_remap; /* 1: every weight angle w enters its gate as pi tanh(w)
                            (quantum weight remapping, section "Additional
                            Optimizations": weights mapped into (-pi, pi) by tanh);
                            weight gradients are then with respect to w. 0 (default): off */
    int32_t splitter;    /* 0 (default): greedy split in program order (section
                            "Circuit Splitting"); 1: list scheduling over the
                            dependency graph (the graph-based split named as future
                            work in section "Conclusion") */
    int32_t amp_dtype;   /* QSV_AMP_C64 (default): complex64 states, float32 gate
                            arithmetic; QSV_AMP_C128: complex128 states and float64
                            gate matrices, for the plain method only (method =
                            QSV_METHOD_PER_GATE; the same kernels instantiated for
                            double precision). State and workspace sizes double. */
    int32_t pack_beam;   /* fused method: width of the beam search that chooses each
                            pass's tile qubits (0..256, default 16); 0 packs passes
                            greedily in program order with no choice of tile */
} qsv_opts;

/* amplitude types (qsv_opts.amp_dtype) */
enum { QSV_AMP_C64 = 0, QSV_AMP_C128 = 1 };

typedef struct {
    int32_t n_qubits, n_gates, n_weights, n_inputs;
    int32_t method, fuse_width, tile_qubits, low_qubits;
    int32_t n_prefix_gates;   /* leading 1-qubit gates folded into the product-state init */
    int32_t n_blocks;         /* splitter blocks over the whole gate list */
    int32_t n_fwd_passes;     /* state sweeps of a forward (fused: tiles; per-gate: gates) */
    int32_t n_bwd_passes;     /* sweeps of a backward */
    int32_t n_fwd_stages;     /* register stages over all forward passes (fused) */
    int32_t n_bwd_stages;
    int32_t n_param_gates;    /* gates with src != NONE */
    int32_t n_recipes;        /* cached gate-matrix products evaluated per call */
    int32_t n_circuits;       /* 1, or the number of circuits of a multi-circuit plan */
} qsv_plan_info;

/* One circuit of a multi-circuit plan. */
typedef struct {
    int32_t n_qubits;         /* 4..QSV_MAX_QUBITS */
    int32_t n_gates;
    const qsv_gate* gates;    /* host memory, read during qsv_plan_multi only */
    int32_t n_weights, n_inputs;
} qsv_circuit;

typedef struct qsv_plan_s qsv_plan_t;

/* Fill *opts with the defaults (fused, k = 1, m = 12, c = 4, 256, codegen 1, chain
 * products in the backward, mfma 1). */
void qsv_default_opts(qsv_opts* opts);

/*
 * Build a plan for a circuit (host only; no device work, no GPU needed).
 * The plan is the gate-matrix cache of section "Gate Matrix Caching" (each
 * gate kept as constant partial matrices plus coefficient functions of its
 * angle, never expanded by Kronecker products) and the split of section
 * "Circuit Splitting" (dependency-graph blocks of at most k qubits, packed
 * into passes over tiles of the state).
 * gates: n_gates entries, host memory, read during the call only.
 * n_weights / n_inputs: lengths of the weight vector and of one input row.
 * opts: NULL for defaults. *out receives the plan.
 */
int qsv_plan(int32_t n_qubits, const qsv_gate* gates, int32_t n_gates, int32_t n_weights,
             int32_t n_inputs, const qsv_opts* opts, qsv_plan_t** out);

/*
 * Plan for many circuits of different sizes and depths simulated together
 * (the uneven batch). Not an operation of the paper: its section "Circuit
 * Splitting" only motivates it (sub-circuits on disjoint qubit sets can be
 * executed in parallel); the call is this library's addition for batches of
 * unrelated circuits. Every circuit is split and scheduled as by qsv_plan
 * (fused method, table-driven kernels, tile_qubits <= 12). qsv_forward and
 * qsv_backward then run the passes of ALL circuits in a few launches
 * ("rounds"), one workgroup per (circuit, tile), in the order of
 * qsv_plan_multi_items: a circuit's passes sit in consecutive rounds, so
 * the number of launches per direction is the largest pass count of any
 * circuit, not the number of circuits. No workgroup waits on another. (A single persistent launch per
 * direction that walks the same list, each item waiting for its circuit's
 * previous pass, stopped making progress on its first device run; it is not
 * used.)
 * Layouts with the plan (c = circuit, prefix sums over earlier circuits):
 *   weights:      concatenation of every circuit's weights;
 *   inputs:       batch x (sum of n_inputs), circuit c's columns after c-1's;
 *   state:        batch x (sum of 2^n_qubits) complex64, circuit c's
 *                 amplitudes at qsv_plan_circuit_offsets(...amp);
 *   expectations, grad_out: batch x (sum of n_qubits), float64;
 *   gradients:    weights and inputs laid out as above.
 * Each circuit's results equal those of a single plan of that circuit.
 */
int qsv_plan_multi(const qsv_circuit* circuits, int32_t n_circuits, const qsv_opts* opts,
                   qsv_plan_t** out);

/*
 * qsv_plan_multi with options chosen per circuit: circuit c is split and
 * scheduled with per_circuit[c] (n_circuits entries, host memory, read during
 * the call only; the same fields and limits as the options of qsv_plan_multi),
 * so that a batch of unrelated circuits can take the fusion width, tile and
 * low qubits that suit each (section "Circuit Splitting" leaves the block
 * size to the user). weight_remap must be the same for every circuit;
 * qsv_plan_get_info reports the options of circuit 0. Layouts, launches and
 * results are as with qsv_plan_multi.
 */
int qsv_plan_multi_each(const qsv_circuit* circuits, int32_t n_circuits, const qsv_opts* per_circuit,
                        qsv_plan_t** out);

/* Offsets of circuit `circuit` in the layouts above (single plans: all 0).
 * Any output pointer may be NULL. */
int qsv_plan_circuit_offsets(const qsv_plan_t* plan, int32_t circuit, int64_t* amp_offset,
                             int32_t* qubit_offset, int32_t* weight_offset, int32_t* input_offset);

/* Byte offset of circuit `circuit`'s amplitudes within one sample's row of
 * the state (8 bytes per complex64 amplitude; single plans: 0), or a
 * negative QSV_ERR_* code (QSV_ERR_HANDLE, QSV_ERR_ARG for an index out of
 * range). */
int64_t qsv_state_offset(const qsv_plan_t* plan, int32_t circuit);

/*
 * Work list of a multi-circuit plan at this batch size, in the order one
 * forward (which = 0) or backward (which = 1) runs it: item i is
 * (circuit, pass, tile) at items[3i .. 3i+2]. The list goes round by round
 * (one launch each); a circuit with k passes takes k consecutive rounds,
 * starting where the rounds stay best balanced, so pass r of a circuit comes
 * after all tiles of its pass r - 1; the costliest tiles of a round come
 * first. (A persistent launch taking items in this order could start an item
 * once every tile of its circuit's previous pass is done.) Copies at most
 * max_items items (items may be NULL) and stores the total count in
 * *n_items. Host only.
 */
int qsv_plan_multi_items(const qsv_plan_t* plan, int64_t batch, int32_t which, int32_t* items,
                         int64_t max_items, int64_t* n_items);

/* Release a plan and its device tables. NULL, an already destroyed plan and
 * any pointer that is not a live plan are ignored: handles are checked
 * against the library's registry of live plans (and graphs), never read
 * through, so every call with a destroyed handle returns QSV_ERR_HANDLE. */
void qsv_plan_destroy(qsv_plan_t* plan);

/* Bytes of workspace one call of kind `op` (QSV_OP_*) needs at this batch size. */
size_t qsv_workspace_size(const qsv_plan_t* plan, int64_t batch, int32_t op);

/*
 * Forward: d_state[b] = U_N ... U_1 |0...0> for b < batch (section "State
 * Vector Simulation": the gates applied in order to the state vector, each as
 * the 2x2 / 4x4 update of section "Concept of Shapes", with the gate matrices
 * of section "Gate Matrix Caching" and the blocks of section "Circuit
 * Splitting").
 * d_weights: n_weights float32 (may be NULL if n_weights == 0).
 * d_inputs:  batch x n_inputs float32, row-major (may be NULL if n_inputs == 0).
 * d_state:   batch x 2^W complex64 (complex128 with amp_dtype = QSV_AMP_C128),
 *            written; 8-byte alignment suffices. The plain method's kernels
 *            and the generated fused kernels use 16-byte accesses when it is
 *            16-byte aligned (any torch allocation is).
 * d_ws:      at least qsv_workspace_size(plan, batch, QSV_OP_FORWARD) bytes of
 *            device memory, 256-byte aligned, owned by the caller. It receives
 *            the gate matrices evaluated for this call (per sample for gates
 *            driven by inputs). The paper's signature has no workspace; it is
 *            taken here so that concurrent calls on one plan share no mutable
 *            device memory and no call allocates.
 */
int qsv_forward(const qsv_plan_t* plan, const float* d_weights, const float* d_inputs,
                int64_t batch, void* d_state, void* d_ws, size_t ws_bytes, void* stream);

/*
 * Readout (the measurement layer of section "Hybrid Machine Learning"):
 * d_out[b * W + i] = sum_idx |psi_b[idx]|^2 (1 - 2 bit_{W-1-i}(idx)), float64.
 * Per-thread float32 partials over at most 16 amplitudes, float64 above.
 */
int qsv_expval(const qsv_plan_t* plan, const void* d_state, int64_t batch, double* d_out,
               void* d_ws, size_t ws_bytes, void* stream);

/*
 * Forward and readout in one call: the same d_state as qsv_forward and the
 * same d_out as qsv_expval (the circuit of section "State Vector
 * Simulation" followed by the measurement layer of section "Hybrid Machine
 * Learning"). With generated kernels (fused method, codegen on) the last
 * forward pass sums |a|^2 (1 - 2 bit) over its tile while the amplitudes are
 * still in registers, so the state is not read back; every other plan runs
 * qsv_forward then qsv_expval. d_ws must hold qsv_workspace_size(plan, batch,
 * QSV_OP_FORWARD_EXPVAL) bytes. Errors as for qsv_forward; d_out may not be
 * NULL.
 */
int qsv_forward_expval(const qsv_plan_t* plan, const float* d_weights, const float* d_inputs,
                       int64_t batch, void* d_state, double* d_out, void* d_ws, size_t ws_bytes,
                       void* stream);

/*
 * qsv_forward_expval without a workspace argument, for callers that cannot
 * allocate device memory where they call it (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc). Same kernels and
 * results as qsv_forward_expval. Its workspace is a file-scope device array of
 * QSV_NOALLOC_SCRATCH_BYTES bytes inside the library: one per GPU the library
 * runs on, held by that GPU until the process ends; the call looks up its
 * address once per device (on its first call there) and never calls hipMalloc,
 * hipFree or anything else that allocates; profiling records nothing.
 *  - The plan's tables must already exist on the current device: an earlier
 *    qsv_forward, qsv_forward_expval, qsv_expval, qsv_backward or
 *    qsv_graph_create call on this device creates them (for a multi-circuit
 *    plan, at this batch size). Otherwise QSV_ERR_ARG, nothing enqueued.
 *  - A plan and batch whose workspace, qsv_workspace_size(plan, batch,
 *    QSV_OP_FORWARD_EXPVAL), exceeds QSV_NOALLOC_SCRATCH_BYTES return
 *    QSV_ERR_TOO_BIG before anything is enqueued.
 *  - Every call on one GPU shares that GPU's array, which keeps the last
 *    call's contents (each call writes everything it reads, so nothing needs
 *    clearing). Calls that may overlap on one GPU (other streams, threads or
 *    plans) race: the caller must order them.
 * Other arguments and errors as for qsv_forward_expval.
 */
#define QSV_NOALLOC_SCRATCH_BYTES (16 * 1024 * 1024)
int qsv_forward_expval_noalloc(const qsv_plan_t* plan, const float* d_weights, const float* d_inputs,
                               int64_t batch, void* d_state, double* d_out, void* stream);

/*
 * Adjoint backward of L = sum_{b,i} g[b,i] E[b,i], g = d_grad_out (batch x W
 * float64). Not the paper's method: it trains through PyTorch's automatic
 * differentiation (section "Hybrid Machine Learning"), which stores every
 * intermediate state; this call is the adjoint method added by this library,
 * which needs two state-sized buffers whatever the depth, and it gives the
 * same gradients up to rounding. d_state holds psi_N from qsv_forward with the same weights and
 * inputs; it is read, not modified. Going back over the gates, the angle
 * derivative of gate k is Im <lambda_k| P_k |psi_k> with lambda = (sum_i g_i
 * Z_i) psi_N and P_k the gate's generator; psi and lambda are then multiplied
 * by U_k^dagger (uncomputed) instead of being stored per gate.
 * d_grad_weights: n_weights float64, overwritten (summed over the batch).
 * d_grad_inputs:  batch x n_inputs float64, overwritten; may be NULL.
 * d_ws: at least qsv_workspace_size(plan, batch, QSV_OP_BACKWARD) bytes,
 *       256-byte aligned: gate matrices, the psi and lambda copies (one state
 *       each) and float64 gradient partials.
 */
int qsv_backward(const qsv_plan_t* plan, const float* d_weights, const float* d_inputs,
                 int64_t batch, const void* d_state, const double* d_grad_out,
                 void* d_ws, size_t ws_bytes, double* d_grad_weights,
                 double* d_grad_inputs, void* stream);

/* Host-side introspection (no GPU needed). */
int qsv_plan_get_info(const qsv_plan_t* plan, qsv_plan_info* info);

/*
 * Cost model of one step (forward + readout + backward) at this batch, for
 * choosing fuse_width / tile_qubits / low_qubits without running anything:
 * each state sweep costs max(algorithmic bytes / hbm_gbs, algorithmic
 * float32 operations / alu_tflops), each launch adds launch_us.
 * *us receives the estimate in microseconds. Host only.
 */
int qsv_plan_estimate(const qsv_plan_t* plan, int64_t batch, double hbm_gbs, double alu_tflops,
                      double launch_us, double* us);

/*
 * Gate order in which a forward (which = 0) or backward (which = 1) applies
 * the gates: order[j] is the index of the j-th gate applied (for the
 * backward, the j-th gate uncomputed). Every gate appears once. order has
 * n_gates entries.
 */
int qsv_plan_gate_order(const qsv_plan_t* plan, int32_t which, int32_t* order);

/* Splitter block of every gate (blocks numbered in execution order). */
int qsv_plan_gate_blocks(const qsv_plan_t* plan, int32_t* block_of_gate);

/*
 * Generated source of a fused plan's pass kernels (codegen = 1). Copies at
 * most buf_size bytes including the terminating NUL into buf (may be NULL)
 * and stores the full size including the NUL in *needed.
 */
int qsv_plan_codegen_source(const qsv_plan_t* plan, char* buf, size_t buf_size, size_t* needed);

/*
 * Compile a fused plan's generated kernels with hipRTC for the named
 * architecture (e.g. "gfx950") without touching any device; on failure the
 * compiler log is available from qsv_last_error(). Host only.
 */
int qsv_plan_codegen_check(const qsv_plan_t* plan, const char* arch);

/*
 * Memory accesses of one fused pass alone, a measurement aid (not part of
 * the paper's method): the global loads and stores of pass `pass` of the
 * forward (which = 0) or backward (which = 1) schedule in a plain copy
 * kernel, with no arithmetic between them, on the arrays the pass itself
 * uses and through the same tiles, thread layout, 16-byte pairs and block
 * order as the pass kernel generated for it. A pass that takes about as long
 * is bound by its accesses (it can also be faster: the copy issues every
 * tile's stores right behind its loads, the pass spreads them out).
 *   which = 0: reads and writes d_state (batch x 2^n complex64) in place,
 *     values unchanged; the first pass, which builds the product state,
 *     only writes it: zeros. d_ws may be NULL.
 *   which = 1: d_ws of at least qsv_workspace_size(plan, batch,
 *     QSV_OP_BACKWARD) bytes, whose psi and lambda copies (where
 *     qsv_backward keeps them) are read and written; the first pass reads
 *     d_state instead and writes its values to both, the last writes
 *     nothing. d_state is not written.
 * lds_bytes (0 to 65536) of LDS are reserved per workgroup without being
 * used, which bounds how many tiles a compute unit holds at once (160 KB
 * each; the pass kernels themselves reserve 32-36 KB, 4-5 tiles). Arrays are
 * 16-byte aligned when the pass's tiles hold amplitude bit 0 (else 8-byte).
 * Fused complex64 plans of one circuit only (QSV_ERR_ARG otherwise).
 * Launches on `stream`.
 */
int qsv_pass_copy(const qsv_plan_t* plan, int32_t which, int32_t pass, int64_t batch, void* d_state,
                  void* d_ws, size_t ws_bytes, int32_t lds_bytes, void* stream);

/*
 * Kernel profiling. While enabled, every kernel launch made by qsv_forward,
 * qsv_forward_expval, qsv_expval and qsv_backward with this plan is bracketed
 * by two HIP events recorded on the call's stream, and the launch's
 * algorithmic traffic and arithmetic are noted:
 *   bytes = 8 bytes per amplitude read or written (complex64) by the
 *           method's definition of the step, not by the cache hierarchy;
 *   flops = float32 operations of the gate arithmetic (complex multiply = 6).
 * qsv_profile_read waits for the recorded events, writes up to max_out
 * per-kernel totals, sets *n_out, and clears the record. Kernels generated
 * for a plan get one entry per pass under their symbol names ("qsv_f<i>",
 * "qsv_b<i>"); the per-gate method's kernels one entry per gate class
 * ("k_pg_apply.1q", ".diag", ".ctl" for controlled gates, ".sign" for CZ / Z /
 * CCZ; likewise "k_pg_adj.*"); other library kernels one entry per kernel.
 * With on = 2 the record is not summed: qsv_profile_read writes one entry
 * per launch (launches = 1) in launch order, under the same names, so that
 * per-dispatch counters of an external profiler can be matched to gate
 * classes. on outside 0..2 is QSV_ERR_ARG. Enabling or reading while another
 * thread calls into the same plan is not supported.
 */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;  /* sum of event-measured launch durations */
    double bytes;     /* sum of algorithmic bytes */
    double flops;     /* sum of algorithmic float32 operations */
} qsv_kernel_stat;

int qsv_profile_enable(qsv_plan_t* plan, int32_t on);
int qsv_profile_read(qsv_plan_t* plan, qsv_kernel_stat* out, int32_t max_out, int32_t* n_out);

/*
 * HIP-graph capture of one step: qsv_forward_expval and (if d_grad_out
 * is not NULL) qsv_backward with these pointers are recorded once on
 * `stream` (a non-default hipStream_t) into a graph; qsv_graph_launch then
 * replays the whole launch sequence with one call. Pointers are fixed in the
 * graph: to run a new step, write new weights / inputs / upstream gradients
 * into the same buffers. d_ws must hold qsv_workspace_size(plan, batch,
 * QSV_OP_STEP) bytes and stay allocated while the graph exists. The plan's
 * device tables (and generated kernels) are created before capturing, so the
 * capture itself contains only kernel launches; no memory-set nodes.
 * Profiling records nothing inside a captured step.
 */
typedef struct qsv_graph_s qsv_graph_t;

int qsv_graph_create(const qsv_plan_t* plan, int64_t batch, const float* d_weights,
                     const float* d_inputs, void* d_state, double* d_expval,
                     const double* d_grad_out, double* d_grad_weights, double* d_grad_inputs,
                     void* d_ws, size_t ws_bytes, void* stream, qsv_graph_t** out);
int qsv_graph_launch(qsv_graph_t* graph, void* stream);
void qsv_graph_destroy(qsv_graph_t* graph);

const char* qsv_strerror(int code);
const char* qsv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QSV_H_INCLUDED */
