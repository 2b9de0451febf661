/*
 * qsv_oracle.c -- plain, slow, obviously correct CPU reference simulator.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may call, link or
 * load this file or the library built from it; only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * Arithmetic: complex128 amplitudes, float64 everywhere. Gates are applied one
 * at a time by the per-gate pair update the paper describes for a single-qubit
 * gate (section "Concept of Shapes": view the state with the gate's qubit as
 * the last axis and multiply by the 2x2 matrix), written as explicit loops.
 *
 * Conventions (readings of the paper, all stated here):
 *  - MSb-0 ordering (section "Symbols"): qubit w of W is bit (W-1-w) of the
 *    basis-state index; |0001> is index 1.
 *  - The expanded operator of Eq. (2) is I_{2^w} (x) R (x) I_{2^(W-w-1)}; the
 *    printed exponent W-w is off by one (the product would have size 2^(W+1)).
 *  - The gate acts on the column vector: psi' = G psi on the qubit's axis.
 *  - Rotations follow Eq. (1)'s family R_d(theta) = exp(-i theta sigma_d / 2):
 *      RX = [[c, -i s], [-i s, c]],  RY = [[c, -s], [s, c]],
 *      RZ = diag(e^{-i theta/2}, e^{+i theta/2}),  c = cos(theta/2), s = sin(theta/2).
 *    H = (X + Z)/sqrt(2). CNOT(c,t) flips t where c = 1. CZ negates where both
 *    are 1. CRX(c,t,theta) applies RX(theta) to t where c = 1; CRY and CRZ
 *    likewise. The multi-qubit gates named as future work (section
 *    "Conclusion": Toffoli and the like) are read as: CCX(c1,c2,t) flips t
 *    where both controls are 1, CCZ negates where all three are 1, CCRX
 *    applies RX to t where both controls are 1.
 *  - Initial state |0...0>; expectation <Z_i> = sum_idx |psi|^2 (1 - 2 bit_i),
 *    no renormalisation (the measurement layer of "Hybrid Machine Learning").
 *  - Gradient by the adjoint recurrence: with lambda = O psi_N and
 *    O = sum_i g_i Z_i, going back over gates k = N..1, the derivative with
 *    respect to gate k's angle is Im <lambda_k | P_k | psi_k>, where P_k is the
 *    gate's generator (dU/dtheta = -(i/2) P U); then psi and lambda are both
 *    multiplied by U_k^dagger. For a controlled rotation, P is the target's
 *    generator where every control is 1 and zero elsewhere (CRX:
 *    P = |1><1|_c (x) X_t).
 *
 * Gate-kind numbering below is private to the oracle.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum { K_H = 0, K_X, K_Y, K_Z, K_RX, K_RY, K_RZ, K_CNOT, K_CZ, K_CRX,
       K_CRY, K_CRZ, K_CCX, K_CCZ, K_CCRX, K_COUNT };

/* number of controls of a kind (listed first: q0, then q1); the target is the
 * next qubit (q0, q1 or q2) */
static int n_controls(int kind)
{
    switch (kind) {
    case K_CNOT: case K_CZ: case K_CRX: case K_CRY: case K_CRZ: return 1;
    case K_CCX: case K_CCZ: case K_CCRX: return 2;
    default: return 0;
    }
}
enum { S_NONE = 0, S_WEIGHT = 1, S_INPUT = 2 };

/* 2x2 matrix of a 1-qubit gate, or the target part of a controlled gate. */
static void gate_matrix(int kind, double th, cplx m[2][2])
{
    const double c = cos(0.5 * th), s = sin(0.5 * th);
    const double r = 1.0 / sqrt(2.0);
    switch (kind) {
    case K_H:   m[0][0] = r;    m[0][1] = r;    m[1][0] = r;    m[1][1] = -r;   break;
    case K_X: case K_CNOT: case K_CCX:
                m[0][0] = 0;    m[0][1] = 1;    m[1][0] = 1;    m[1][1] = 0;    break;
    case K_Y:   m[0][0] = 0;    m[0][1] = -I;   m[1][0] = I;    m[1][1] = 0;    break;
    case K_Z: case K_CZ: case K_CCZ:
                m[0][0] = 1;    m[0][1] = 0;    m[1][0] = 0;    m[1][1] = -1;   break;
    case K_RX: case K_CRX: case K_CCRX:
                m[0][0] = c;    m[0][1] = -I*s; m[1][0] = -I*s; m[1][1] = c;    break;
    case K_RY: case K_CRY:
                m[0][0] = c;    m[0][1] = -s;   m[1][0] = s;    m[1][1] = c;    break;
    case K_RZ: case K_CRZ:
                m[0][0] = cexp(-0.5 * I * th); m[0][1] = 0; m[1][0] = 0;
                m[1][1] = cexp(0.5 * I * th); break;
    default:    m[0][0] = 1;    m[0][1] = 0;    m[1][0] = 0;    m[1][1] = 1;    break;
    }
}

/* Generator P with dU/dtheta = -(i/2) P U (target part for CRX). */
static void gate_generator(int kind, cplx p[2][2])
{
    switch (kind) {
    case K_RX: case K_CRX: case K_CCRX: gate_matrix(K_X, 0.0, p); break;
    case K_RY: case K_CRY:              gate_matrix(K_Y, 0.0, p); break;
    case K_RZ: case K_CRZ:              gate_matrix(K_Z, 0.0, p); break;
    default: p[0][0] = p[0][1] = p[1][0] = p[1][1] = 0; break;
    }
}

static void dagger(cplx m[2][2], cplx d[2][2])
{
    d[0][0] = conj(m[0][0]); d[0][1] = conj(m[1][0]);
    d[1][0] = conj(m[0][1]); d[1][1] = conj(m[1][1]);
}

static int is_param(int kind)
{
    return kind == K_RX || kind == K_RY || kind == K_RZ || kind == K_CRX || kind == K_CRY ||
           kind == K_CRZ || kind == K_CCRX;
}

/* index-bit mask of a gate's controls and the index bit of its target */
static void gate_bits(int W, int kind, int q0, int q1, int q2, int64_t* cmask, int64_t* tbit)
{
    const int nc = n_controls(kind);
    const int t = nc == 0 ? q0 : nc == 1 ? q1 : q2;
    *cmask = 0;
    if (nc >= 1) *cmask |= (int64_t)1 << (W - 1 - q0);
    if (nc >= 2) *cmask |= (int64_t)1 << (W - 1 - q1);
    *tbit = (int64_t)1 << (W - 1 - t);
}

/* Apply m to the target bit bt of one state, only where every control bit in
 * cm is 1. For every index with bit bt clear (and the controls set), the pair
 * (idx, idx | bt) is multiplied by m. */
static void apply_2x2(cplx* psi, int W, int64_t cm, int64_t bt, cplx m[2][2])
{
    const int64_t n = (int64_t)1 << W;
    #pragma omp parallel for if (n >= (1 << 16)) schedule(static)
    for (int64_t i0 = 0; i0 < n; ++i0) {
        if (i0 & bt) continue;
        if ((i0 & cm) != cm) continue;
        const int64_t i1 = i0 | bt;
        const cplx a0 = psi[i0], a1 = psi[i1];
        psi[i0] = m[0][0] * a0 + m[0][1] * a1;
        psi[i1] = m[1][0] * a0 + m[1][1] * a1;
    }
}

/* Apply gate (kind, q0, q1, q2) with angle th, or its inverse when dag != 0:
 * the 2x2 of its target part, where all its controls are 1. */
static void apply_gate(cplx* psi, int W, int kind, int q0, int q1, int q2, double th, int dag)
{
    cplx m[2][2], d[2][2];
    int64_t cm, bt;
    gate_matrix(kind, th, m);
    if (dag) { dagger(m, d); memcpy(m, d, sizeof(m[0][0]) * 4); }
    gate_bits(W, kind, q0, q1, q2, &cm, &bt);
    apply_2x2(psi, W, cm, bt, m);
}

/* Im <lam | P | psi> for the generator of gate (kind, q0, q1, q2): P is the
 * target generator where every control is 1, zero elsewhere. Neumaier-summed. */
static double grad_term(const cplx* lam, const cplx* psi, int W, int kind, int q0, int q1, int q2)
{
    cplx p[2][2];
    gate_generator(kind, p);
    int64_t cm, bt;
    gate_bits(W, kind, q0, q1, q2, &cm, &bt);
    const int64_t n = (int64_t)1 << W;
    double sum = 0.0, comp = 0.0;
    for (int64_t i0 = 0; i0 < n; ++i0) {
        if (i0 & bt) continue;
        if ((i0 & cm) != cm) continue;
        const int64_t i1 = i0 | bt;
        const cplx p0 = p[0][0] * psi[i0] + p[0][1] * psi[i1];
        const cplx p1 = p[1][0] * psi[i0] + p[1][1] * psi[i1];
        const double v = cimag(conj(lam[i0]) * p0 + conj(lam[i1]) * p1);
        const double t2 = sum + v;
        comp += fabs(sum) >= fabs(v) ? (sum - t2) + v : (v - t2) + sum;
        sum = t2;
    }
    return sum + comp;
}

static double angle_of(int src, int idx, const double* weights, const double* inputs,
                       int n_inputs, int b)
{
    if (src == S_WEIGHT) return weights[idx];
    if (src == S_INPUT) return inputs[(int64_t)b * n_inputs + idx];
    return 0.0;
}

/* Checks shared by the entry points; returns 0 or a negative code. */
static int check_gates(int W, int n_gates, const int* kind, const int* q0, const int* q1,
                       const int* src, const int* idx, const int* q2, int n_weights, int n_inputs)
{
    if (W < 1 || W > 34 || n_gates < 0) return -1;
    for (int k = 0; k < n_gates; ++k) {
        if (kind[k] < 0 || kind[k] >= K_COUNT) return -2;
        if (q0[k] < 0 || q0[k] >= W) return -3;
        const int nc = n_controls(kind[k]);
        if (nc >= 1 && (q1[k] < 0 || q1[k] >= W || q1[k] == q0[k])) return -3;
        if (nc >= 2 && (q2[k] < 0 || q2[k] >= W || q2[k] == q0[k] || q2[k] == q1[k])) return -3;
        if (src[k] == S_WEIGHT && (idx[k] < 0 || idx[k] >= n_weights)) return -4;
        if (src[k] == S_INPUT && (idx[k] < 0 || idx[k] >= n_inputs)) return -4;
        if (src[k] != S_NONE && !is_param(kind[k])) return -4;
    }
    return 0;
}

/*
 * Forward: state[b] = U_N ... U_1 |0...0> for every sample b.
 * shift (nullable, n_gates entries) is added to each gate's angle; the
 * parameter-shift and finite-difference checks use it.
 * state: B x 2^W complex128, written.
 */
int orc_forward(int W, int n_gates, const int* kind, const int* q0, const int* q1,
                const int* src, const int* idx, const int* q2, const double* weights, int n_weights,
                const double* inputs, int n_inputs, int B, const double* shift, cplx* state)
{
    int e = check_gates(W, n_gates, kind, q0, q1, src, idx, q2, n_weights, n_inputs);
    if (e) return e;
    const int64_t n = (int64_t)1 << W;
    for (int b = 0; b < B; ++b) {
        cplx* psi = state + (int64_t)b * n;
        memset(psi, 0, sizeof(cplx) * (size_t)n);
        psi[0] = 1.0;
        for (int k = 0; k < n_gates; ++k) {
            double th = angle_of(src[k], idx[k], weights, inputs, n_inputs, b);
            if (shift) th += shift[k];
            apply_gate(psi, W, kind[k], q0[k], q1[k], q2[k], th, 0);
        }
    }
    return 0;
}

/* E[b, i] = sum_idx |psi_b[idx]|^2 (1 - 2 bit_{W-1-i}(idx)), Neumaier-summed. */
int orc_expval(int W, int B, const cplx* state, double* out)
{
    const int64_t n = (int64_t)1 << W;
    for (int b = 0; b < B; ++b) {
        const cplx* psi = state + (int64_t)b * n;
        for (int i = 0; i < W; ++i) {
            const int64_t bit = (int64_t)1 << (W - 1 - i);
            double sum = 0.0, comp = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                const double p = creal(psi[j]) * creal(psi[j]) + cimag(psi[j]) * cimag(psi[j]);
                const double v = (j & bit) ? -p : p;
                const double t = sum + v;
                comp += fabs(sum) >= fabs(v) ? (sum - t) + v : (v - t) + sum;
                sum = t;
            }
            out[(int64_t)b * W + i] = sum + comp;
        }
    }
    return 0;
}

/*
 * Adjoint gradient of L = sum_{b,i} g[b,i] E[b,i].
 * grad_w (n_weights) is summed over samples and over every gate that reads the
 * weight; grad_x (B x n_inputs, nullable) is per sample. Both are overwritten.
 * final_state (nullable, B x 2^W) receives psi_N.
 */
int orc_adjoint(int W, int n_gates, const int* kind, const int* q0, const int* q1,
                const int* src, const int* idx, const int* q2, const double* weights, int n_weights,
                const double* inputs, int n_inputs, int B, const double* g,
                double* grad_w, double* grad_x, cplx* final_state)
{
    int e = check_gates(W, n_gates, kind, q0, q1, src, idx, q2, n_weights, n_inputs);
    if (e) return e;
    const int64_t n = (int64_t)1 << W;
    cplx* psi = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    cplx* lam = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    if (!psi || !lam) { free(psi); free(lam); return -5; }
    for (int j = 0; j < n_weights; ++j) grad_w[j] = 0.0;
    if (grad_x) for (int64_t j = 0; j < (int64_t)B * n_inputs; ++j) grad_x[j] = 0.0;

    for (int b = 0; b < B; ++b) {
        /* forward for this sample */
        memset(psi, 0, sizeof(cplx) * (size_t)n);
        psi[0] = 1.0;
        for (int k = 0; k < n_gates; ++k)
            apply_gate(psi, W, kind[k], q0[k], q1[k], q2[k],
                       angle_of(src[k], idx[k], weights, inputs, n_inputs, b), 0);
        if (final_state) memcpy(final_state + (int64_t)b * n, psi, sizeof(cplx) * (size_t)n);
        /* lambda = O psi_N with O = sum_i g[b,i] Z_i */
        const double* gb = g + (int64_t)b * W;
        for (int64_t j = 0; j < n; ++j) {
            double d = 0.0;
            for (int i = 0; i < W; ++i)
                d += (j >> (W - 1 - i) & 1) ? -gb[i] : gb[i];
            lam[j] = d * psi[j];
        }
        /* backward sweep */
        for (int k = n_gates - 1; k >= 0; --k) {
            const double th = angle_of(src[k], idx[k], weights, inputs, n_inputs, b);
            if (src[k] != S_NONE) {
                const double gk = grad_term(lam, psi, W, kind[k], q0[k], q1[k], q2[k]);
                if (src[k] == S_WEIGHT) grad_w[idx[k]] += gk;
                else if (grad_x) grad_x[(int64_t)b * n_inputs + idx[k]] += gk;
            }
            apply_gate(psi, W, kind[k], q0[k], q1[k], q2[k], th, 1);
            apply_gate(lam, W, kind[k], q0[k], q1[k], q2[k], th, 1);
        }
    }
    free(psi);
    free(lam);
    return 0;
}

/* 2x2 matrix of one gate as the oracle defines it (row-major, 4 complex). */
int orc_gate_matrix(int kind, double theta, cplx* out4)
{
    if (kind < 0 || kind >= K_COUNT) return -2;
    cplx m[2][2];
    gate_matrix(kind, theta, m);
    out4[0] = m[0][0]; out4[1] = m[0][1]; out4[2] = m[1][0]; out4[3] = m[1][1];
    return 0;
}
