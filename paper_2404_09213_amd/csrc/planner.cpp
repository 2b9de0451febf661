// planner.cpp -- host-only plan construction (no device calls).
//
// 1. Gate-matrix cache (section "Gate Matrix Caching", Eq. (1)): every gate is
//    stored as constant partial matrices C, A, S with matrix(theta) =
//    C + cos(theta/2) A + sin(theta/2) S. Nothing is Kronecker-expanded: the
//    kernels apply 2x2 blocks by index arithmetic instead of Eq. (2)'s
//    2^W x 2^W operators.
// 2. Product-state prefix: the 1-qubit gates that precede every multi-qubit
//    gate on their qubit act on |0...0> qubit by qubit, so the forward starts
//    from their tensor product (this covers the angle-embedding layer).
// 3. Splitter (section "Circuit Splitting"): gates are placed greedily, in
//    program order, into blocks of at most k qubits; a gate goes into the
//    first block at or after the last block touching one of its qubits that
//    still has room, else into a new block.
// 4. Pass builder: blocks are packed into passes; a pass is one read and one
//    write of the state in tiles of 2^m amplitudes whose qubits cover every
//    qubit the pass acts on non-diagonally, plus the c lowest-stride qubits.
//    A block may move ahead of blocks it commutes with. Which qubits each
//    pass's tile holds is chosen by a small beam search (see pack_passes).
// 5. Stage builder: inside a pass, each thread keeps 2^4 amplitudes spanning 4
//    tile qubits in registers; ops are grouped into stages whose non-diagonal
//    qubits fit those 4 register bits; between stages the tile is re-laid out
//    through LDS.
//
// Commutation rule used by 4 and 5: a gate acts "densely" on the qubits where
// it is not block-diagonal in the computational basis (1-qubit non-diagonal
// gates, targets of CNOT/CRX) and "diagonally" on the others (RZ, Z, CZ and
// controls). Two gates commute when neither acts densely on a qubit the
// other touches.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "plan.hpp"

namespace qsv {
namespace {

inline int popc(uint32_t x) { return __builtin_popcount(x); }

// Controls of a kind (listed first: q0, then q1); the target follows them.
int n_ctl(int k) {
    switch (k) {
    case QSV_CNOT: case QSV_CZ: case QSV_CRX: case QSV_CRY: case QSV_CRZ: return 1;
    case QSV_CCX: case QSV_CCZ: case QSV_CCRX: return 2;
    default: return 0;
    }
}
bool is_multi(int k) { return n_ctl(k) > 0; }
int target_of(const qsv_gate& g) { return n_ctl(g.kind) == 0 ? g.q0 : n_ctl(g.kind) == 1 ? g.q1 : g.q2; }
bool is_param_kind(int k) {
    return k == QSV_RX || k == QSV_RY || k == QSV_RZ || k == QSV_CRX || k == QSV_CRY || k == QSV_CRZ ||
           k == QSV_CCRX;
}
bool is_zz(int k) { return k == QSV_CZ || k == QSV_CCZ; }  // pure sign flips

uint32_t qmask(const qsv_gate& g) {
    uint32_t m = 1u << g.q0;
    if (n_ctl(g.kind) >= 1) m |= 1u << g.q1;
    if (n_ctl(g.kind) >= 2) m |= 1u << g.q2;
    return m;
}

// Dense (D) and diagonal/control (C) qubit masks of a gate.
void gate_sets(const qsv_gate& g, uint32_t& D, uint32_t& C) {
    switch (g.kind) {
    case QSV_Z: case QSV_RZ: D = 0; C = 1u << g.q0; break;
    case QSV_CZ: case QSV_CCZ: case QSV_CRZ: D = 0; C = qmask(g); break;
    case QSV_CNOT: case QSV_CRX: case QSV_CRY: case QSV_CCX: case QSV_CCRX:
        D = 1u << target_of(g);
        C = qmask(g) & ~D;
        break;
    default: D = 1u << g.q0; C = 0; break;
    }
}

bool conflicts(uint32_t D1, uint32_t C1, uint32_t D2, uint32_t C2) {
    return (D1 & (D2 | C2)) || (D2 & (D1 | C1));
}

void setm(double* M, int r, int c, double re, double im) {
    M[(r * 2 + c) * 2] = re;
    M[(r * 2 + c) * 2 + 1] = im;
}

void fill_partials(DGate& d, const qsv_gate& g) {
    std::memset(&d, 0, sizeof d);
    d.kind = g.kind;
    d.src = g.src;
    d.idx = g.idx;
    const double r = 1.0 / std::sqrt(2.0);
    switch (g.kind) {
    case QSV_H: setm(d.C, 0, 0, r, 0); setm(d.C, 0, 1, r, 0); setm(d.C, 1, 0, r, 0); setm(d.C, 1, 1, -r, 0); break;
    case QSV_X: case QSV_CNOT: case QSV_CCX: setm(d.C, 0, 1, 1, 0); setm(d.C, 1, 0, 1, 0); break;
    case QSV_Y: setm(d.C, 0, 1, 0, -1); setm(d.C, 1, 0, 0, 1); break;
    case QSV_Z: case QSV_CZ: case QSV_CCZ: setm(d.C, 0, 0, 1, 0); setm(d.C, 1, 1, -1, 0); break;
    case QSV_RX: case QSV_CRX: case QSV_CCRX:  // cos I + sin (-i X)
        setm(d.A, 0, 0, 1, 0); setm(d.A, 1, 1, 1, 0);
        setm(d.S, 0, 1, 0, -1); setm(d.S, 1, 0, 0, -1); break;
    case QSV_RY: case QSV_CRY:  // cos I + sin [[0,-1],[1,0]]
        setm(d.A, 0, 0, 1, 0); setm(d.A, 1, 1, 1, 0);
        setm(d.S, 0, 1, -1, 0); setm(d.S, 1, 0, 1, 0); break;
    case QSV_RZ: case QSV_CRZ:  // cos I + sin (-i Z)
        setm(d.A, 0, 0, 1, 0); setm(d.A, 1, 1, 1, 0);
        setm(d.S, 0, 0, 0, -1); setm(d.S, 1, 1, 0, 1); break;
    }
}

// Structural class of a product of gates (for the kernels' cheaper variants).
int recipe_class(const qsv_plan_t* p, const std::vector<int>& gs) {
    bool all_diag = true, all_real = true;
    for (int g : gs) {
        const int k = p->gates[g].kind;
        if (!(k == QSV_Z || k == QSV_RZ || k == QSV_CZ || k == QSV_CRZ || k == QSV_CCZ)) all_diag = false;
        if (!(k == QSV_H || k == QSV_X || k == QSV_Z || k == QSV_RY || k == QSV_CNOT || k == QSV_CZ ||
              k == QSV_CRY || k == QSV_CCX || k == QSV_CCZ))
            all_real = false;
    }
    if (all_diag) return OP_DIAG;
    if (gs.size() == 1) {
        const int k = p->gates[gs[0]].kind;
        if (k == QSV_X || k == QSV_CNOT || k == QSV_CCX) return OP_SWAP;
        if (k == QSV_RX || k == QSV_CRX || k == QSV_CCRX) return OP_RXL;
    }
    return all_real ? OP_REAL : OP_U2;
}

int add_recipe(qsv_plan_t* p, const std::vector<int>& gs, bool dagger) {
    DRecipe r;
    r.first = (int32_t)p->recipe_gates.size();
    r.count = (int32_t)gs.size();
    r.dagger = dagger ? 1 : 0;
    bool per_sample = false;
    for (int g : gs) {
        p->recipe_gates.push_back(g);
        if (p->gates[g].src == QSV_SRC_INPUT) per_sample = true;
    }
    r.out = per_sample ? -(p->n_ps_mats++) - 1 : p->n_shared_mats++;
    p->recipes.push_back(r);
    return r.out;
}

std::vector<Block> split(const qsv_plan_t* p, const std::vector<int>& seq, int k) {
    std::vector<Block> blocks;
    std::vector<int> last(p->W, -1);
    for (int g : seq) {
        const uint32_t q = qmask(p->gates[g]);
        int jstar = -1;
        for (int b = 0; b < p->W; ++b)
            if (q >> b & 1) jstar = std::max(jstar, last[b]);
        int placed = -1;
        for (int j = std::max(jstar, 0); j < (int)blocks.size(); ++j)
            if (popc(blocks[j].Q | q) <= k) { placed = j; break; }
        if (placed < 0) { blocks.emplace_back(); placed = (int)blocks.size() - 1; }
        blocks[placed].gates.push_back(g);
        blocks[placed].Q |= q;
        for (int b = 0; b < p->W; ++b)
            if (q >> b & 1) last[b] = placed;
    }
    return blocks;
}

// Dependency-graph splitter (the graph-based split proposed as future work in
// section "Conclusion"): list scheduling over the circuit's dependency DAG
// (an edge joins consecutive gates on a qubit). A block is filled from the
// gates whose predecessors are all placed, each time taking the ready gate
// that adds the fewest new qubits, then the one with the longest chain of
// dependants behind it, then the earliest; a block closes when no ready gate
// fits within k qubits. Unlike the program-order rule it may place a gate
// before gates it commutes with trivially (disjoint qubits), so it can fill a
// block with gates the program lists far apart.
std::vector<Block> split_dag(const qsv_plan_t* p, const std::vector<int>& seq, int k) {
    const int n = (int)seq.size();
    std::vector<std::vector<int>> succ(n);
    std::vector<int> npred(n, 0), last(p->W, -1);
    std::vector<uint32_t> qm(n);
    for (int i = 0; i < n; ++i) {
        qm[i] = qmask(p->gates[seq[i]]);
        std::vector<int> preds;
        for (int b = 0; b < p->W; ++b)
            if (qm[i] >> b & 1) {
                if (last[b] >= 0 && std::find(preds.begin(), preds.end(), last[b]) == preds.end())
                    preds.push_back(last[b]);
                last[b] = i;
            }
        for (int j : preds) succ[j].push_back(i);
        npred[i] = (int)preds.size();
    }
    std::vector<int> height(n, 0);  // longest chain of dependants
    for (int i = n - 1; i >= 0; --i)
        for (int j : succ[i]) height[i] = std::max(height[i], height[j] + 1);
    std::vector<int> ready;
    for (int i = 0; i < n; ++i)
        if (npred[i] == 0) ready.push_back(i);
    std::vector<Block> blocks;
    int placed = 0;
    while (placed < n) {
        Block blk;
        uint32_t Q = 0;
        for (;;) {
            int best = -1, bgrow = 0;
            for (int r : ready) {
                const uint32_t nq = Q | qm[r];
                if (Q && popc(nq) > k) continue;
                const int grow = popc(nq) - popc(Q);
                if (best < 0 || grow < bgrow || (grow == bgrow && (height[r] > height[best] ||
                                                                   (height[r] == height[best] && r < best)))) {
                    best = r;
                    bgrow = grow;
                }
            }
            if (best < 0) break;
            ready.erase(std::find(ready.begin(), ready.end(), best));
            blk.gates.push_back(seq[best]);
            Q |= qm[best];
            ++placed;
            for (int s2 : succ[best])
                if (--npred[s2] == 0) ready.push_back(s2);
            if (popc(Q) > k) break;  // a gate wider than k stays alone
        }
        blk.Q = Q;
        blocks.push_back(blk);
    }
    return blocks;
}

std::vector<Block> split_with(const qsv_plan_t* p, const std::vector<int>& seq, int k) {
    return p->opts.splitter == 1 ? split_dag(p, seq, k) : split(p, seq, k);
}

struct BlockSets { uint32_t D = 0, C = 0; int nparam = 0; };

BlockSets block_sets(const qsv_plan_t* p, const Block& b) {
    BlockSets s;
    for (int g : b.gates) {
        uint32_t D, C;
        gate_sets(p->gates[g], D, C);
        s.D |= D;
        s.C |= C;
        if (p->gates[g].src != QSV_SRC_NONE) s.nparam++;
    }
    s.C &= ~s.D;
    return s;
}

uint32_t low_mask(int W, int c) {
    uint32_t m = 0;
    for (int i = 0; i < c; ++i) m |= 1u << (W - 1 - i);  // qubit W-1 has stride 1
    return m;
}

// Pack blocks into passes; returns per pass the gate list in execution order.
//
// One pass is one greedy scan of the remaining blocks in order, from a tile
// seed T0: a block joins when it commutes with every block skipped before it,
// its dense qubits fit the tile (with T0 and the c low qubits) and the
// gradient cap allows; the others stay, in order, for later passes. Which
// qubits a pass's tile holds decides how far later passes get, so the seeds
// tried are the empty set (the plain program-order greedy), every window of
// consecutive qubits (in qubit order, wrapping round) and the dense qubits of
// the first remaining blocks; a beam search over those choices keeps the
// `beam` sequences that have packed the most gates after each pass (plus the
// plain greedy sequence) and returns the first that packs everything, i.e.
// the fewest passes it found, never more than the plain greedy needs.
std::vector<std::vector<int>> pack_passes(const qsv_plan_t* p, std::vector<Block> blocks, int m,
                                          int c, int max_grads, std::vector<uint32_t>& pass_dense) {
    const uint32_t low = low_mask(p->W, c);
    // A block wider than a tile, or with more parametric gates than a pass may
    // hold, is packed gate by gate. A single gate always fits an empty pass (it
    // acts densely on at most one qubit, c < m, and max_grads >= 1), so every
    // pass below packs at least the first remaining block.
    std::vector<Block> bl;
    for (auto& b : blocks) {
        const BlockSets s = block_sets(p, b);
        if (popc(s.D | low) <= m && s.nparam <= max_grads) { bl.push_back(b); continue; }
        for (int g : b.gates) {
            Block one;
            one.gates.push_back(g);
            one.Q = qmask(p->gates[g]);
            bl.push_back(one);
        }
    }
    const int nb = (int)bl.size();
    if (nb == 0) return {};
    std::vector<BlockSets> bs(nb);
    for (int i = 0; i < nb; ++i) bs[i] = block_sets(p, bl[i]);

    // A search state: the blocks still to pack and the passes so far (a chain
    // of nodes, so that states share their history).
    struct Node {
        int parent;
        uint32_t T;
        std::vector<int> took;
    };
    struct State {
        int node = -1;
        std::vector<int> rem;  // remaining block indices, in order
        uint64_t hash = 0;     // of rem
        int packed = 0;        // gates packed so far
        bool greedy = true;    // every pass so far from the empty seed
    };
    std::vector<Node> nodes;
    auto hash_of = [](const std::vector<int>& v) {
        uint64_t h = 1469598103934665603ull;
        for (int x : v) h = (h ^ (uint64_t)(uint32_t)x) * 1099511628211ull;
        return h;
    };
    // one pass from seed T0 over st.rem: taken blocks, their dense qubits, the rest
    auto scan = [&](const std::vector<int>& rem, uint32_t T0, std::vector<int>& took, std::vector<int>& left,
                    uint32_t& T, int& ngate) {
        uint32_t Tt = T0, sD = 0, sC = 0;
        int ngrad = 0;
        T = 0;
        ngate = 0;
        took.clear();
        left.clear();
        for (int i : rem) {
            const BlockSets& s = bs[i];
            if (!conflicts(s.D, s.C, sD, sC) && popc(Tt | s.D | low) <= m && ngrad + s.nparam <= max_grads) {
                Tt |= s.D;
                T |= s.D;
                ngrad += s.nparam;
                ngate += (int)bl[i].gates.size();
                took.push_back(i);
            } else {
                left.push_back(i);
                sD |= s.D;
                sC |= s.C;
            }
        }
    };
    std::vector<int> others;
    for (int q = 0; q < p->W; ++q)
        if (!(low >> q & 1)) others.push_back(q);
    const int free_q = m - popc(low), no = (int)others.size();
    std::vector<uint32_t> windows;
    if (free_q > 0 && free_q < no)
        for (int a = 0; a < no; ++a) {
            uint32_t w = 0;
            for (int j = 0; j < free_q; ++j) w |= 1u << others[(a + j) % no];
            windows.push_back(w);
        }
    const int beam = p->opts.pack_beam;
    constexpr int kBlockSeeds = 16;

    State init;
    for (int i = 0; i < nb; ++i) init.rem.push_back(i);
    init.hash = hash_of(init.rem);
    std::vector<State> cur{init};
    int done = -1;
    std::vector<State> next;
    std::vector<uint32_t> cand;
    std::vector<int> took, left;
    // each pass packs at least one block, so at most nb passes
    for (int level = 0; done < 0 && level < nb && !cur.empty(); ++level) {
        next.clear();
        for (const State& st : cur) {
            cand.assign(1, 0u);
            if (beam > 0) {
                cand.insert(cand.end(), windows.begin(), windows.end());
                for (int k = 0; k < (int)st.rem.size() && k < kBlockSeeds; ++k) cand.push_back(bs[st.rem[k]].D & ~low);
                std::sort(cand.begin() + 1, cand.end());
                cand.erase(std::unique(cand.begin() + 1, cand.end()), cand.end());
            }
            for (uint32_t T0 : cand) {
                uint32_t T;
                int n;
                scan(st.rem, T0, took, left, T, n);
                if (n == 0) continue;  // never for seed 0: the first block always fits
                nodes.push_back(Node{st.node, T, took});
                State ns;
                ns.node = (int)nodes.size() - 1;
                ns.rem = left;
                ns.hash = hash_of(ns.rem);
                ns.packed = st.packed + n;
                ns.greedy = st.greedy && T0 == 0;
                next.push_back(std::move(ns));
            }
        }
        // best first (most gates packed; earlier candidate on ties), one state per
        // remaining set; the program-order greedy sequence always stays (or a
        // state with the same remaining blocks), so the result never needs more
        // passes than it
        std::stable_sort(next.begin(), next.end(), [](const State& a, const State& b) { return a.packed > b.packed; });
        cur.clear();
        bool have_greedy = false;
        for (State& ns : next) {
            const bool full = (int)cur.size() >= std::max(beam, 1);
            if (full && (have_greedy || !ns.greedy)) continue;
            bool dup = false;
            for (const State& k : cur)
                if (k.hash == ns.hash && k.rem == ns.rem) { dup = true; break; }
            have_greedy = have_greedy || ns.greedy;
            if (!dup) cur.push_back(std::move(ns));
        }
        for (const State& st : cur)
            if (st.rem.empty()) { done = st.node; break; }
    }
    if (done < 0) return {};  // unreachable (see above); the caller checks coverage
    std::vector<int> chain;
    for (int k = done; k >= 0; k = nodes[k].parent) chain.push_back(k);
    std::reverse(chain.begin(), chain.end());
    std::vector<std::vector<int>> passes;
    for (int k : chain) {
        std::vector<int> gates;
        for (int b : nodes[k].took) gates.insert(gates.end(), bl[b].gates.begin(), bl[b].gates.end());
        passes.push_back(gates);
        pass_dense.push_back(nodes[k].T);
    }
    return passes;
}

// One schedulable unit inside a pass: a fused 1-qubit chain or a 2-qubit gate.
struct Unit {
    std::vector<int> gates;  // in application order
    uint32_t D = 0, C = 0;
    int qubit = -1;          // chain qubit, or target of a 2-qubit gate
    int comps = 0;           // backward chain: Pauli components needed (bit 0 X, 1 Y, 2 Z)
};

// Generator axis of a parametric gate (0 X, 1 Y, 2 Z).
int axis_of(int kind) { return kind == QSV_RY ? 1 : kind == QSV_RZ ? 2 : 0; }

// Pauli support (bit 0 X, 1 Y, 2 Z) of U P U^dagger for P spanned by the
// Paulis in `s`, with U one 1-qubit gate: a rotation about one axis keeps that
// axis and mixes the other two; H swaps X and Z; X, Y, Z only change signs.
int conj_support(int kind, int s) {
    int out = 0;
    for (int a = 0; a < 3; ++a) {
        if (!(s >> a & 1)) continue;
        switch (kind) {
        case QSV_RX: out |= a == 0 ? 1 : 6; break;
        case QSV_RY: out |= a == 1 ? 2 : 5; break;
        case QSV_RZ: out |= a == 2 ? 4 : 3; break;
        case QSV_H: out |= a == 0 ? 4 : a == 2 ? 1 : 2; break;
        default: out |= 1 << a; break;
        }
    }
    return out;
}

// Vector instructions per amplitude pair and state array of one apply op.
int apply_cost(int cls) {
    switch (cls) {
    case OP_U2: return 16;
    case OP_SWAP: return 1;
    default: return 8;
    }
}

std::vector<Unit> fwd_units(const qsv_plan_t* p, const std::vector<int>& gates) {
    std::vector<Unit> units;
    std::vector<int> open(p->W, -1);
    for (int g : gates) {
        const qsv_gate& G = p->gates[g];
        if (!is_multi(G.kind)) {
            int& u = open[G.q0];
            if (u < 0) {
                units.emplace_back();
                u = (int)units.size() - 1;
                units[u].qubit = G.q0;
            }
            units[u].gates.push_back(g);
            uint32_t D, C;
            gate_sets(G, D, C);
            units[u].D |= D;
            units[u].C |= C;
        } else {
            for (int q = 0; q < p->W; ++q)
                if (qmask(G) >> q & 1) open[q] = -1;
            Unit x;
            x.gates.push_back(g);
            gate_sets(G, x.D, x.C);
            x.qubit = target_of(G);
            units.push_back(x);
        }
    }
    for (auto& u : units) u.C &= ~u.D;
    return units;
}

// Backward units, in uncompute order. A run of 1-qubit gates on one qubit
// (with only gates on other qubits in between) becomes one chain unit when
// uncomputing it as a single 2x2 product, with the gradients recovered from
// the chain's X/Y/Z components, takes fewer vector operations than gate by
// gate (and needs no more gradient slots); otherwise every gate is its own
// unit. The gradient of gate j of a chain U_n...U_1 is
// Im<l|V_j P_j V_j^dagger|psi> with V_j = U_n...U_{j+1}, taken after the
// chain: a combination of Im<l|X|psi>, Im<l|Y|psi>, Im<l|Z|psi>.
std::vector<Unit> bwd_units(const qsv_plan_t* p, const std::vector<int>& gates, bool fuse) {
    std::vector<Unit> chains;
    std::vector<int> open(p->W, -1);
    for (auto it = gates.rbegin(); it != gates.rend(); ++it) {
        const int g = *it;
        const qsv_gate& G = p->gates[g];
        uint32_t D, C;
        gate_sets(G, D, C);
        if (!is_multi(G.kind)) {
            int& u = open[G.q0];
            if (u < 0) {
                chains.emplace_back();
                u = (int)chains.size() - 1;
                chains[u].qubit = G.q0;
            }
            chains[u].gates.insert(chains[u].gates.begin(), g);
            chains[u].D |= D;
            chains[u].C |= C;
        } else {
            for (int q = 0; q < p->W; ++q)
                if (qmask(G) >> q & 1) open[q] = -1;
            Unit x;
            x.gates.push_back(g);
            x.D = D;
            x.C = C;
            x.qubit = target_of(G);
            chains.push_back(x);
        }
    }
    std::vector<Unit> units;
    for (Unit& u : chains) {
        u.C &= ~u.D;
        const int n = (int)u.gates.size();
        bool fused = false;
        if (fuse && n >= 2 && !is_multi(p->gates[u.gates[0]].kind)) {
            int comps = 0, nparam = 0, sep = 0;
            for (int j = 0; j < n; ++j) {
                const qsv_gate& G = p->gates[u.gates[j]];
                sep += 2 * apply_cost(recipe_class(p, {u.gates[j]}));
                if (G.src == QSV_SRC_NONE) continue;
                ++nparam;
                sep += 4;
                int sup = 1 << axis_of(G.kind);
                for (int k = j + 1; k < n; ++k) sup = conj_support(p->gates[u.gates[k]].kind, sup);
                comps |= sup;
            }
            const int ncomp = popc((uint32_t)comps);
            const int cost = 2 * apply_cost(recipe_class(p, u.gates)) + 4 * ncomp;
            if (cost < sep && ncomp <= std::max(nparam, 1)) {
                fused = true;
                u.comps = comps;
            }
        }
        if (fused) {
            units.push_back(u);
            continue;
        }
        for (int j = n - 1; j >= 0; --j) {
            Unit x;
            x.gates.push_back(u.gates[j]);
            const qsv_gate& G = p->gates[u.gates[j]];
            gate_sets(G, x.D, x.C);
            x.C &= ~x.D;
            x.qubit = target_of(G);
            units.push_back(x);
        }
    }
    return units;
}

// Greedy stage grouping: each stage's dense qubits fit the register bits.
std::vector<std::pair<uint32_t, std::vector<int>>> group_stages(const std::vector<Unit>& units) {
    std::vector<std::pair<uint32_t, std::vector<int>>> stages;
    std::vector<int> remaining(units.size());
    for (size_t i = 0; i < units.size(); ++i) remaining[i] = (int)i;
    // One stage with register qubits `S`: in order, a unit joins when its dense
    // qubits lie in S and it commutes with every unit left behind so far.
    auto scan = [&](uint32_t S, std::vector<int>* taken, std::vector<int>* skipped) {
        uint32_t sD = 0, sC = 0, R = 0;
        int n = 0;
        for (int u : remaining) {
            const Unit& U = units[u];
            if (!conflicts(U.D, U.C, sD, sC) && !(U.D & ~S)) {
                R |= U.D;
                ++n;
                if (taken) taken->push_back(u);
            } else {
                sD |= U.D;
                sC |= U.C;
                if (skipped) skipped->push_back(u);
            }
        }
        return std::make_pair(n, R);
    };
    while (!remaining.empty()) {
        // Register qubits of the stage: of all kRegBits-subsets of the dense
        // qubits still to come, the one that lets the most units join (every
        // unit needs at most kRegBits dense qubits, so some unit always joins);
        // ties keep the first subset in enumeration order.
        uint32_t pool = 0;
        for (int u : remaining) pool |= units[u].D;
        std::vector<int> bits;
        for (int q = 0; q < 32; ++q)
            if (pool >> q & 1) bits.push_back(q);
        const int k = std::min<int>(kRegBits, (int)bits.size());
        uint32_t bestS = 0;
        int bestN = -1;
        std::vector<int> idx(k);
        for (int i = 0; i < k; ++i) idx[i] = i;
        while (true) {
            uint32_t S = 0;
            for (int i : idx) S |= 1u << bits[i];
            const int n = scan(S, nullptr, nullptr).first;
            if (n > bestN) { bestN = n; bestS = S; }
            // next k-combination of bits
            int i = k - 1;
            while (i >= 0 && idx[i] == (int)bits.size() - k + i) --i;
            if (i < 0) break;
            ++idx[i];
            for (int j = i + 1; j < k; ++j) idx[j] = idx[j - 1] + 1;
        }
        std::vector<int> taken, skipped;
        const uint32_t R = scan(bestS, &taken, &skipped).second;
        stages.emplace_back(R, taken);
        remaining = skipped;
    }
    return stages;
}

// Builds one DPass (tile qubits + stages + ops) from a pass's gate list.
struct PassBuilder {
    qsv_plan_t* p;
    bool backward;
    // backward: first gate (program order) on each qubit. A unit holding the
    // first gate on every qubit it touches needs no uncompute: nothing later
    // in the backward touches those qubits, and Im<l|P|psi> for P on other
    // qubits does not change under a unitary applied to both states on them.
    std::vector<int> first_on;

    void build(const std::vector<int>& gates, uint32_t dense, int m, int c, int flags,
               std::vector<DPass>& out, std::vector<int32_t>& order) {
        const int W = p->W;
        DPass ps;
        std::memset(&ps, 0, sizeof ps);
        ps.m = m;
        ps.flags = flags;
        // tile qubits: dense set + c lowest + fill with the lowest remaining
        uint32_t tile = dense | low_mask(W, c);
        for (int q = W - 1; q >= 0 && popc(tile) < m; --q) tile |= 1u << q;
        // local bits ordered by ascending global shift (qubit W-1 first)
        int local_of_qubit[kMaxQ];
        int j = 0, k = 0;
        for (int q = W - 1; q >= 0; --q) {
            if (tile >> q & 1) { local_of_qubit[q] = j; ps.lq[j++] = W - 1 - q; }
            else { local_of_qubit[q] = -1; ps.oq[k++] = W - 1 - q; }
        }
        std::vector<Unit> units = backward ? bwd_units(p, gates, !p->opts.bwd_gate_by_gate)
                                           : fwd_units(p, gates);
        auto groups = group_stages(units);
        ps.stage0 = (int32_t)p->stages.size();
        ps.n_stages = (int32_t)groups.size();
        ps.gout0 = (int32_t)p->gouts.size();
        int nslot = 0;
        for (auto& grp : groups) {
            DStage st;
            std::memset(&st, 0, sizeof st);
            // register bits: the stage's dense qubits, padded with the top local bits
            std::vector<int> regs;
            for (int q = 0; q < W; ++q)
                if (grp.first >> q & 1) regs.push_back(local_of_qubit[q]);
            for (int lb = m - 1; lb >= 0 && (int)regs.size() < kRegBits; --lb)
                if (std::find(regs.begin(), regs.end(), lb) == regs.end()) regs.push_back(lb);
            std::sort(regs.begin(), regs.end());
            for (int i = 0; i < kRegBits; ++i) st.reg[i] = regs[i];
            auto pos_of = [&](int qubit) -> int {
                const int lb = local_of_qubit[qubit];
                for (int i = 0; i < kRegBits; ++i)
                    if (lb >= 0 && st.reg[i] == lb) return i;
                return -1;
            };
            // control encoding: register position, or kCtlNonReg | index-bit shift
            auto ctl_code = [&](int qubit) {
                const int pc = pos_of(qubit);
                return pc >= 0 ? pc : (kCtlNonReg | (W - 1 - qubit));
            };
            st.op0 = (int32_t)p->ops.size();
            int sign_op = -1;  // open OP_SIGN being extended
            for (int ui : grp.second) {
                const Unit& U = units[ui];
                if (backward) order.insert(order.end(), U.gates.rbegin(), U.gates.rend());
                else order.insert(order.end(), U.gates.begin(), U.gates.end());
                const qsv_gate& G = p->gates[U.gates[0]];
                const bool is_cz = U.gates.size() == 1 && is_zz(G.kind);
                auto starts_timelines = [&]() {
                    if (!backward || first_on.empty()) return false;
                    const qsv_gate& G0 = p->gates[U.gates[0]];
                    for (int b = 0; b < W; ++b)
                        if ((qmask(G0) >> b & 1) && first_on[b] != U.gates[0]) return false;
                    return true;
                };
                if (is_cz && starts_timelines()) continue;
                if (is_cz) {
                    // CZ / CCZ: flip where every qubit is 1. Register qubits select
                    // the flipped registers; the other qubits gate them by index bits.
                    if (sign_op < 0) {
                        DOp o;
                        std::memset(&o, 0, sizeof o);
                        o.kind = OP_SIGN;
                        o.pos = 0;  // uniform mask
                        o.ctl = o.ctl2 = -1;
                        o.term0 = (int32_t)p->terms.size();
                        o.nterm = 0;
                        p->ops.push_back(o);
                        sign_op = (int)p->ops.size() - 1;
                    }
                    DOp& o = p->ops[sign_op];
                    int mask = 0xFFFF;
                    std::vector<int> glob;
                    for (int q = 0; q < W; ++q) {
                        if (!(qmask(G) >> q & 1)) continue;
                        const int pq = pos_of(q);
                        if (pq >= 0) {
                            int m = 0;
                            for (int r = 0; r < kRegs; ++r)
                                if (r >> pq & 1) m |= 1 << r;
                            mask &= m;
                        } else {
                            glob.push_back(W - 1 - q);
                        }
                    }
                    if (glob.empty()) {
                        o.pos ^= mask;
                    } else {
                        DTerm t;
                        t.s0 = glob[0];
                        t.s1 = glob.size() > 1 ? glob[1] : -1;
                        t.s2 = glob.size() > 2 ? glob[2] : -1;
                        t.mask = mask;
                        p->terms.push_back(t);
                        o.nterm++;
                    }
                    continue;
                }
                sign_op = -1;
                auto comp_op = [&](int kind) {
                    DOp o;
                    std::memset(&o, 0, sizeof o);
                    o.kind = kind;
                    o.pos = pos_of(U.qubit);
                    o.sh = W - 1 - U.qubit;
                    o.ctl = o.ctl2 = -1;
                    o.slot = nslot++;
                    p->ops.push_back(o);
                    return o.slot;
                };
                if (backward && U.comps) {
                    // chain: X/Y/Z components after the chain, one output per
                    // parametric gate, then the chain's product uncomputed at once
                    int slot_of[3] = {-1, -1, -1};
                    for (int a = 0; a < 3; ++a)
                        if (U.comps >> a & 1) slot_of[a] = comp_op(OP_GX + a);
                    const int n = (int)U.gates.size();
                    for (int j = 0; j < n; ++j) {
                        const qsv_gate& Gj = p->gates[U.gates[j]];
                        if (Gj.src == QSV_SRC_NONE) continue;
                        DGOut go;
                        std::memset(&go, 0, sizeof go);
                        go.ord = p->param_ordinal[U.gates[j]];
                        if (j == n - 1) {
                            go.axis = -1;
                            go.c0 = slot_of[axis_of(Gj.kind)];
                            go.c1 = go.c2 = -1;
                        } else {
                            go.axis = axis_of(Gj.kind);
                            go.c0 = slot_of[0];
                            go.c1 = slot_of[1];
                            go.c2 = slot_of[2];
                            go.mat = add_recipe(p, std::vector<int>(U.gates.begin() + j + 1, U.gates.end()),
                                                false);
                        }
                        p->gouts.push_back(go);
                    }
                } else if (backward) {
                    // gradient partial (before uncomputing the gate), then U^dagger
                    const int g = U.gates[0];
                    if (G.src != QSV_SRC_NONE) {
                        DOp o;
                        std::memset(&o, 0, sizeof o);
                        o.kind = (G.kind == QSV_RY || G.kind == QSV_CRY)   ? OP_GY
                                 : (G.kind == QSV_RZ || G.kind == QSV_CRZ) ? OP_GZ
                                                                           : OP_GX;
                        o.pos = pos_of(U.qubit);
                        o.sh = W - 1 - U.qubit;
                        o.ctl = o.ctl2 = -1;
                        if (is_multi(G.kind)) {
                            o.ctl = ctl_code(G.q0);
                            if (n_ctl(G.kind) == 2) o.ctl2 = ctl_code(G.q1);
                        }
                        o.mat = 0;
                        o.slot = nslot++;
                        p->ops.push_back(o);
                        DGOut go;
                        std::memset(&go, 0, sizeof go);
                        go.ord = p->param_ordinal[g];
                        go.axis = -1;
                        go.c0 = o.slot;
                        go.c1 = go.c2 = -1;
                        p->gouts.push_back(go);
                    }
                }
                if (starts_timelines()) continue;
                DOp o;
                std::memset(&o, 0, sizeof o);
                o.kind = recipe_class(p, U.gates);
                o.mat = add_recipe(p, U.gates, backward);
                o.pos = pos_of(U.qubit);
                o.sh = W - 1 - U.qubit;
                o.ctl = o.ctl2 = -1;
                o.slot = -1;
                if (is_multi(G.kind) && U.gates.size() == 1) {
                    o.ctl = ctl_code(G.q0);
                    if (n_ctl(G.kind) == 2) o.ctl2 = ctl_code(G.q1);
                }
                p->ops.push_back(o);
            }
            st.op1 = (int32_t)p->ops.size();
            p->stages.push_back(st);
        }
        ps.n_gslots = nslot;
        ps.n_gout = (int32_t)p->gouts.size() - ps.gout0;
        out.push_back(ps);
    }
};

// Float32 operations per amplitude of one op (complex multiply = 6, add = 2).
double op_flops(const DOp& o) {
    // controlled ops touch half of the amplitudes per control
    const double half = (o.ctl >= 0 ? 0.5 : 1.0) * (o.ctl2 >= 0 ? 0.5 : 1.0);
    switch (o.kind) {
    case OP_U2: return 14.0 * half;    // two complex products and a sum per output
    case OP_REAL: case OP_RXL: return 6.0 * half;
    case OP_DIAG: return 6.0 * half;
    case OP_GX: case OP_GY: return 3.5 * half;
    case OP_GZ: return 4.0 * half;
    default: return 0.0;               // sign flips and swaps move data only
    }
}

double pass_flops(const qsv_plan_t* p, const DPass& ps, bool backward) {
    double f = 0.0;
    for (int s = ps.stage0; s < ps.stage0 + ps.n_stages; ++s)
        for (int o = p->stages[s].op0; o < p->stages[s].op1; ++o) {
            const DOp& op = p->ops[o];
            const bool grad = op.kind >= OP_GX;
            f += op_flops(op) * (backward && !grad ? 2.0 : 1.0);
        }
    return f;
}

double pg_flops(const PGate& g, bool backward) {
    DOp o;
    std::memset(&o, 0, sizeof o);
    o.kind = g.cls;
    o.ctl = g.csh >= 0 ? 0 : -1;
    o.ctl2 = g.csh2 >= 0 ? 0 : -1;
    double f = op_flops(o) * (backward ? 2.0 : 1.0);
    if (backward && g.grad >= 0) {
        o.kind = g.grad;
        f += op_flops(o);
    }
    return f;
}

void set_partial_layout(qsv_plan_t* p, int64_t nch) {
    p->pu.resize(p->n_param);
    p->nchv.assign(p->n_param, (int32_t)nch);
    for (int o = 0; o < p->n_param; ++o) p->pu[o] = (int64_t)o * nch;
    p->pu_total = (int64_t)p->n_param * nch;
}

// Index-bit shifts of a per-gate launch: target and controls; a CZ / CCZ
// lists its qubits as tsh, sh2 (and csh2).
void pg_shifts(int W, const qsv_gate& G, PGate& x) {
    const int nc = n_ctl(G.kind);
    x.tsh = W - 1 - target_of(G);
    x.csh = x.csh2 = x.sh2 = -1;
    if (is_zz(G.kind)) {
        x.sh2 = W - 1 - G.q0;
        if (nc == 2) x.csh2 = W - 1 - G.q1;
        return;
    }
    if (nc >= 1) x.csh = W - 1 - G.q0;
    if (nc >= 2) x.csh2 = W - 1 - G.q1;
}

int pg_class(const qsv_plan_t* p, int g) {
    const int k = p->gates[g].kind;
    if (is_zz(k)) return OP_SIGN;
    return recipe_class(p, std::vector<int>{g});
}

}  // namespace

int build_plan(qsv_plan_t* p) {
    const int W = p->W;
    const qsv_opts& o = p->opts;
    // gate cache
    p->dgates.resize(p->n_gates);
    p->param_ordinal.assign(p->n_gates, -1);
    for (int g = 0; g < p->n_gates; ++g) {
        fill_partials(p->dgates[g], p->gates[g]);
        if (p->gates[g].src != QSV_SRC_NONE) {
            p->param_ordinal[g] = p->n_param++;
            p->param_gate.push_back(g);
        }
    }
    // gradient gathering lists
    {
        std::vector<std::vector<int>> wl(p->n_weights), xl(p->n_inputs);
        for (int g = 0; g < p->n_gates; ++g) {
            const qsv_gate& G = p->gates[g];
            if (G.src == QSV_SRC_WEIGHT) wl[G.idx].push_back(p->param_ordinal[g]);
            if (G.src == QSV_SRC_INPUT) xl[G.idx].push_back(p->param_ordinal[g]);
        }
        const int head = p->n_weights + 1 + p->n_inputs + 1;
        p->grad_csr.assign(head, 0);
        int at = head;
        for (int j = 0; j < p->n_weights; ++j) { p->grad_csr[j] = at; at += (int)wl[j].size(); }
        p->grad_csr[p->n_weights] = at;
        for (int j = 0; j < p->n_inputs; ++j) { p->grad_csr[p->n_weights + 1 + j] = at; at += (int)xl[j].size(); }
        p->grad_csr[p->n_weights + 1 + p->n_inputs] = at;
        for (auto& l : wl) p->grad_csr.insert(p->grad_csr.end(), l.begin(), l.end());
        for (auto& l : xl) p->grad_csr.insert(p->grad_csr.end(), l.begin(), l.end());
    }
    // product-state prefix
    std::vector<int> first2(W, p->n_gates);
    for (int g = p->n_gates - 1; g >= 0; --g) {
        const qsv_gate& G = p->gates[g];
        if (is_multi(G.kind))
            for (int q = 0; q < W; ++q)
                if (qmask(G) >> q & 1) first2[q] = g;
    }
    std::vector<char> in_prefix(p->n_gates, 0);
    std::vector<std::vector<int>> pre(W);
    for (int g = 0; g < p->n_gates; ++g) {
        const qsv_gate& G = p->gates[g];
        if (!is_multi(G.kind) && g < first2[G.q0]) {
            in_prefix[g] = 1;
            pre[G.q0].push_back(g);
            p->prefix_gates.push_back(g);
        }
    }
    p->prefix_mat.resize(W);
    for (int q = 0; q < W; ++q) p->prefix_mat[q] = add_recipe(p, pre[q], false);
    std::vector<int> body, all;
    for (int g = 0; g < p->n_gates; ++g) {
        all.push_back(g);
        if (!in_prefix[g]) body.push_back(g);
    }
    p->fwd_order = p->prefix_gates;

    // splitter over the whole list (reported; drives the backward schedule)
    p->blocks = split_with(p, all, o.fuse_width);
    p->block_of_gate.assign(p->n_gates, -1);
    for (size_t b = 0; b < p->blocks.size(); ++b)
        for (int g : p->blocks[b].gates) p->block_of_gate[g] = (int32_t)b;

    if (o.method == QSV_METHOD_PER_GATE) {
        for (int g : body) {
            PGate x;
            std::memset(&x, 0, sizeof x);
            const qsv_gate& G = p->gates[g];
            x.gate = g;
            x.cls = pg_class(p, g);
            pg_shifts(W, G, x);
            x.mat = x.cls == OP_SIGN ? 0 : add_recipe(p, {g}, false);
            x.grad = -1;
            x.slot = -1;
            p->pg_fwd.push_back(x);
            p->fwd_order.push_back(g);
        }
        for (int g = p->n_gates - 1; g >= 0; --g) {
            PGate x;
            std::memset(&x, 0, sizeof x);
            const qsv_gate& G = p->gates[g];
            x.gate = g;
            x.cls = pg_class(p, g);
            pg_shifts(W, G, x);
            x.mat = x.cls == OP_SIGN ? 0 : add_recipe(p, {g}, true);
            x.slot = p->param_ordinal[g];
            x.grad = G.src == QSV_SRC_NONE                      ? -1
                   : (G.kind == QSV_RY || G.kind == QSV_CRY) ? OP_GY
                   : (G.kind == QSV_RZ || G.kind == QSV_CRZ) ? OP_GZ
                                                             : OP_GX;
            p->pg_bwd.push_back(x);
            p->bwd_order.push_back(g);
        }
        for (auto& x : p->pg_fwd) p->pg_fwd_flops.push_back(pg_flops(x, false));
        for (auto& x : p->pg_bwd) p->pg_bwd_flops.push_back(pg_flops(x, true));
        set_partial_layout(p, pg_chunks(W));
        return QSV_OK;
    }

    // fused schedule
    const int m = std::min(o.tile_qubits, W);
    const int c = std::min(o.low_qubits, m - 1);
    // LDS budget for gradient partials per slot: float32 per 16-lane row
    // (generated kernels) or float64 per wave (table-driven) = threads / 4
    // bytes, plus one float64 component sum; 256 bytes kept for the rest
    const int threads = std::max(64, 1 << (m - kRegBits));
    const int exch = (1 << m) * 8;
    int max_grads = std::min(o.max_pass_grads, (160 * 1024 - 256 - exch) / (threads / 4 + 8));
    max_grads = std::max(max_grads, 1);
    // every gate of the packed list must land in exactly one pass
    auto covers = [](const std::vector<std::vector<int>>& passes, size_t n) {
        size_t k = 0;
        for (auto& ps : passes) k += ps.size();
        if (k == n) return true;
        set_error("internal error: pass packing did not place every gate");
        return false;
    };
    {
        std::vector<uint32_t> dense;
        auto passes = pack_passes(p, split_with(p, body, o.fuse_width), m, c, 1 << 30, dense);
        if (!covers(passes, body.size())) return QSV_ERR_GATE;
        PassBuilder pb{p, false, {}};
        for (size_t i = 0; i < passes.size(); ++i)
            pb.build(passes[i], dense[i], m, c, i == 0 ? PF_INIT_FWD : 0, p->fwd_pass, p->fwd_order);
    }
    {
        std::vector<uint32_t> dense;
        auto passes = pack_passes(p, p->blocks, m, c, max_grads, dense);
        if (!covers(passes, (size_t)p->n_gates)) return QSV_ERR_GATE;
        PassBuilder pb{p, true, std::vector<int>(W, p->n_gates)};
        for (int g = p->n_gates - 1; g >= 0; --g) {
            const qsv_gate& G = p->gates[g];
            for (int q = 0; q < W; ++q)
                if (qmask(G) >> q & 1) pb.first_on[q] = g;
        }
        const int n = (int)passes.size();
        for (int i = n - 1; i >= 0; --i) {
            int flags = 0;
            if (i == n - 1) flags |= PF_FIRST_BWD;
            if (i == 0) flags |= PF_LAST_BWD;
            pb.build(passes[i], dense[i], m, c, flags, p->bwd_pass, p->bwd_order);
        }
    }
    for (auto& ps : p->fwd_pass) {
        p->n_fwd_stages += ps.n_stages;
        p->fwd_pass_flops.push_back(pass_flops(p, ps, false));
    }
    for (auto& ps : p->bwd_pass) {
        p->n_bwd_stages += ps.n_stages;
        p->bwd_pass_flops.push_back(pass_flops(p, ps, true));
    }
    set_partial_layout(p, int64_t(1) << (W - m));
    return QSV_OK;
}

// Many circuits in one plan: each circuit is planned on its own (fused,
// table-driven kernels), then the tables are concatenated with every index
// shifted to the combined numbering. Weights and input columns of circuit c
// follow those of circuits 0..c-1; a sample row of the state holds every
// circuit's 2^W amplitudes back to back, and a row of expectations every
// circuit's qubits.
int build_multi(qsv_plan_t* p, const std::vector<CircuitIn>& cs) {
    p->multi = true;
    int w0 = 0, x0 = 0, e0 = 0, ord0 = 0, chunk0 = 0;
    int64_t amp0 = 0;
    std::vector<int> wl_off, xl_off;
    std::vector<std::vector<int>> wl, xl;
    for (size_t c = 0; c < cs.size(); ++c) {
        const CircuitIn& ci = cs[c];
        qsv_plan_t sub;
        sub.W = ci.W;
        sub.n_gates = ci.n_gates;
        sub.n_weights = ci.n_weights;
        sub.n_inputs = ci.n_inputs;
        sub.opts = ci.opts;  // each circuit's own options (validated by the caller)
        sub.opts.method = QSV_METHOD_FUSED;
        sub.opts.codegen = 0;
        sub.opts.tile_qubits = std::min(sub.opts.tile_qubits, (int32_t)kMaxTileQubitsTables);
        sub.gates.assign(ci.gates, ci.gates + ci.n_gates);
        int rc = build_plan(&sub);
        if (rc != QSV_OK) return rc;
        DCirc d;
        std::memset(&d, 0, sizeof d);
        d.W = ci.W;
        d.m = std::min((int)sub.opts.tile_qubits, ci.W);
        d.n_fwd = (int32_t)sub.fwd_pass.size();
        d.n_bwd = (int32_t)sub.bwd_pass.size();
        d.fwd0 = (int32_t)p->fwd_pass.size();
        d.bwd0 = (int32_t)p->bwd_pass.size();
        d.e0 = e0;
        d.pm0 = (int32_t)p->prefix_mat.size();
        d.amp0 = amp0;
        d.ic0 = chunk0;
        d.nchunk = 1 << (ci.W - std::min(ci.W, 12));
        const int g0 = (int)p->dgates.size(), rg0 = (int)p->recipe_gates.size();
        const int st0 = (int)p->stages.size(), op0 = (int)p->ops.size(), t0 = (int)p->terms.size();
        const int go0 = (int)p->gouts.size();
        const int sh0 = p->n_shared_mats, ps0 = p->n_ps_mats;
        auto fix_mat = [&](int32_t mat) { return mat >= 0 ? mat + sh0 : -((-mat - 1) + ps0) - 1; };
        for (DGate g : sub.dgates) {
            if (g.src == QSV_SRC_WEIGHT) g.idx += w0;
            if (g.src == QSV_SRC_INPUT) g.idx += x0;
            p->dgates.push_back(g);
        }
        for (int32_t g : sub.recipe_gates) p->recipe_gates.push_back(g + g0);
        for (DRecipe r : sub.recipes) {
            r.first += rg0;
            r.out = fix_mat(r.out);
            p->recipes.push_back(r);
        }
        p->n_shared_mats += sub.n_shared_mats;
        p->n_ps_mats += sub.n_ps_mats;
        for (int32_t m : sub.prefix_mat) p->prefix_mat.push_back(fix_mat(m));
        for (DStage st : sub.stages) {
            st.op0 += op0;
            st.op1 += op0;
            p->stages.push_back(st);
        }
        for (DOp o : sub.ops) {
            if (o.kind != OP_SIGN && o.kind != OP_SWAP && o.kind < OP_GX) o.mat = fix_mat(o.mat);
            if (o.kind == OP_SIGN) o.term0 += t0;
            p->ops.push_back(o);
        }
        p->terms.insert(p->terms.end(), sub.terms.begin(), sub.terms.end());
        for (DGOut o : sub.gouts) {
            o.ord += ord0;
            if (o.axis >= 0) o.mat = fix_mat(o.mat);
            p->gouts.push_back(o);
        }
        for (DPass ps : sub.fwd_pass) {
            ps.stage0 += st0;
            p->fwd_pass.push_back(ps);
        }
        for (DPass ps : sub.bwd_pass) {
            ps.stage0 += st0;
            ps.gout0 += go0;
            p->bwd_pass.push_back(ps);
        }
        p->fwd_pass_flops.insert(p->fwd_pass_flops.end(), sub.fwd_pass_flops.begin(), sub.fwd_pass_flops.end());
        p->bwd_pass_flops.insert(p->bwd_pass_flops.end(), sub.bwd_pass_flops.begin(), sub.bwd_pass_flops.end());
        // parametric ordinals, gradient lists and partial layout
        const int64_t nch = int64_t(1) << (ci.W - d.m);
        for (int o = 0; o < sub.n_param; ++o) {
            p->pu.push_back(p->pu_total);
            p->nchv.push_back((int32_t)nch);
            p->pu_total += nch;
            const int g = sub.param_gate[o];
            const qsv_gate& G = sub.gates[g];
            p->param_gate.push_back(g0 + g);
            if (G.src == QSV_SRC_WEIGHT) {
                if ((int)wl.size() < w0 + G.idx + 1) wl.resize(w0 + G.idx + 1);
                wl[w0 + G.idx].push_back(ord0 + o);
            } else {
                if ((int)xl.size() < x0 + G.idx + 1) xl.resize(x0 + G.idx + 1);
                xl[x0 + G.idx].push_back(ord0 + o);
            }
        }
        for (int g = 0; g < ci.n_gates; ++g) {
            p->gates.push_back(ci.gates[g]);
            p->param_ordinal.push_back(sub.param_ordinal[g] >= 0 ? sub.param_ordinal[g] + ord0 : -1);
            p->block_of_gate.push_back(sub.block_of_gate[g] + (int32_t)p->blocks.size());
        }
        for (const Block& b : sub.blocks) {
            Block nb = b;
            for (int& g : nb.gates) g += g0;
            p->blocks.push_back(nb);
        }
        for (int32_t g : sub.fwd_order) p->fwd_order.push_back(g + g0);
        for (int32_t g : sub.bwd_order) p->bwd_order.push_back(g + g0);
        for (int g : sub.prefix_gates) p->prefix_gates.push_back(g + g0);
        p->n_fwd_stages += sub.n_fwd_stages;
        p->n_bwd_stages += sub.n_bwd_stages;
        p->circ.push_back(d);
        p->circ_w0.push_back(w0);
        p->circ_x0.push_back(x0);
        w0 += ci.n_weights;
        x0 += ci.n_inputs;
        e0 += ci.W;
        ord0 += sub.n_param;
        chunk0 += d.nchunk;
        amp0 += int64_t(1) << ci.W;
    }
    p->n_param = ord0;
    p->n_gates = (int)p->gates.size();
    p->n_weights = w0;
    p->n_inputs = x0;
    p->Wtot = e0;
    p->row = amp0;
    p->nchunk_tot = chunk0;
    p->n_fwd_tot = (int)p->fwd_pass.size();
    p->n_bwd_tot = (int)p->bwd_pass.size();
    wl.resize(w0);
    xl.resize(x0);
    const int head = w0 + 1 + x0 + 1;
    p->grad_csr.assign(head, 0);
    int at = head;
    for (int j = 0; j < w0; ++j) { p->grad_csr[j] = at; at += (int)wl[j].size(); }
    p->grad_csr[w0] = at;
    for (int j = 0; j < x0; ++j) { p->grad_csr[w0 + 1 + j] = at; at += (int)xl[j].size(); }
    p->grad_csr[w0 + 1 + x0] = at;
    for (auto& l : wl) p->grad_csr.insert(p->grad_csr.end(), l.begin(), l.end());
    for (auto& l : xl) p->grad_csr.insert(p->grad_csr.end(), l.begin(), l.end());
    return QSV_OK;
}

}  // namespace qsv
