/*
 * sv_oracle.c -- plain, slow, obviously-correct FP64 CPU oracle for the
 * state-vector path of "LogosQ" (arxiv 2512.23183).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header, table or
 * helper with the GPU path.
 *
 * Every operation is written from its textbook / paper definition, one gate
 * at a time, with the bit-mask loops of the paper's direct state-vector
 * gates (Sec. "Direct State Vector Gates", Alg. "Direct State Vector CNOT";
 * App. B, Alg. "Direct State Vector Toffoli").  There is no fusion, tiling or
 * reordering.  Arithmetic is C99 double complex throughout.
 *
 * Conventions (Alg. "Direct State Vector CNOT"; App. A and App. B examples):
 *   - state psi has 2^n amplitudes, stored as (re, im) double pairs;
 *   - qubit q corresponds to index bit n-1-q (qubit 0 is the most
 *     significant bit, "MSB-first");
 *   - a 4x4 two-qubit matrix is indexed by 2*bit(q0) + bit(q1), i.e. the first
 *     listed qubit is the more significant (App. C, the printed CNOT matrix).
 *
 * Gate-kind numbers are an interface shared with the C ABI (same numbers,
 * separately declared there).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;

enum {
    OG_H = 0, OG_X = 1, OG_Y = 2, OG_Z = 3,
    OG_RX = 4, OG_RY = 5, OG_RZ = 6, OG_U3 = 7,
    OG_CNOT = 8, OG_CZ = 9, OG_CP = 10, OG_SWAP = 11,
    OG_CRX = 12, OG_CRY = 13, OG_CRZ = 14, OG_CCX = 15,
    OG_RXX = 16, OG_RYY = 17, OG_RZZ = 18,
    OG_MAT1 = 19, OG_MAT2 = 20,
    OG_NKINDS = 21
};

/* Number of qubit operands of each gate kind. */
static int arity(int kind)
{
    switch (kind) {
    case OG_H: case OG_X: case OG_Y: case OG_Z:
    case OG_RX: case OG_RY: case OG_RZ: case OG_U3: case OG_MAT1:
        return 1;
    case OG_CNOT: case OG_CZ: case OG_CP: case OG_SWAP:
    case OG_CRX: case OG_CRY: case OG_CRZ:
    case OG_RXX: case OG_RYY: case OG_RZZ: case OG_MAT2:
        return 2;
    case OG_CCX:
        return 3;
    default:
        return -1;
    }
}

/* Index bit of qubit q: MSB-first (Alg. "Direct State Vector CNOT"). */
static size_t qmask(int n, int q) { return (size_t)1 << (n - 1 - q); }

/* ------------------------------------------------------------------ */
/* Generic bit-mask loops                                               */
/* ------------------------------------------------------------------ */

/*
 * 2x2 matrix u = [u0 u1; u2 u3] on qubit q, applied only where every bit
 * of ctrl is set (ctrl = 0 for an uncontrolled gate).  For every index i
 * with the target bit clear, the pair (psi[i], psi[i|m]) is replaced by
 * u applied to it (Sec. "Direct State Vector Gates": O(2^n) update of
 * amplitude pairs selected by bit masks).
 */
static void apply_1q(cplx *psi, int n, int q, size_t ctrl, const cplx u[4])
{
    const size_t dim = (size_t)1 << n;
    const size_t m = qmask(n, q);
#pragma omp parallel for if (dim >= ((size_t)1 << 16)) schedule(static)
    for (size_t i = 0; i < dim; ++i) {
        if ((i & m) != 0 || (i & ctrl) != ctrl)
            continue;
        cplx a = psi[i], b = psi[i | m];
        psi[i] = u[0] * a + u[1] * b;
        psi[i | m] = u[2] * a + u[3] * b;
    }
}

/*
 * 4x4 matrix on (q0, q1); basis index of the 4-vector is
 * 2*bit(q0) + bit(q1) (App. C: printed CNOT matrix, control listed first).
 */
static void apply_2q(cplx *psi, int n, int q0, int q1, const cplx u[16])
{
    const size_t dim = (size_t)1 << n;
    const size_t m0 = qmask(n, q0), m1 = qmask(n, q1);
#pragma omp parallel for if (dim >= ((size_t)1 << 16)) schedule(static)
    for (size_t i = 0; i < dim; ++i) {
        if ((i & m0) != 0 || (i & m1) != 0)
            continue;
        size_t idx[4] = { i, i | m1, i | m0, i | m0 | m1 };
        cplx v[4], w[4];
        for (int r = 0; r < 4; ++r)
            v[r] = psi[idx[r]];
        for (int r = 0; r < 4; ++r) {
            w[r] = 0;
            for (int c = 0; c < 4; ++c)
                w[r] += u[4 * r + c] * v[c];
        }
        for (int r = 0; r < 4; ++r)
            psi[idx[r]] = w[r];
    }
}

/*
 * Alg. "Direct State Vector CNOT": for every i with the control bit set and
 * the target bit clear, swap psi[i] and psi[i XOR t_mask].  The Toffoli of
 * App. B is the same loop with the combined control mask.
 */
static void apply_cnot_masks(cplx *psi, int n, size_t ctrl, size_t tm)
{
    const size_t dim = (size_t)1 << n;
#pragma omp parallel for if (dim >= ((size_t)1 << 16)) schedule(static)
    for (size_t i = 0; i < dim; ++i) {
        if ((i & ctrl) == ctrl && (i & tm) == 0) {
            size_t j = i ^ tm;
            cplx t = psi[i];
            psi[i] = psi[j];
            psi[j] = t;
        }
    }
}

/* Diagonal phase on every amplitude whose index has all bits of mask set. */
static void apply_phase_masks(cplx *psi, int n, size_t mask, cplx ph)
{
    const size_t dim = (size_t)1 << n;
#pragma omp parallel for if (dim >= ((size_t)1 << 16)) schedule(static)
    for (size_t i = 0; i < dim; ++i)
        if ((i & mask) == mask)
            psi[i] *= ph;
}

/* ------------------------------------------------------------------ */
/* Gate matrices from their definitions                                 */
/* ------------------------------------------------------------------ */

static const cplx PAULI[4][4] = {
    { 1, 0, 0, 1 },        /* I */
    { 0, 1, 1, 0 },        /* X */
    { 0, -I, I, 0 },       /* Y */
    { 1, 0, 0, -1 },       /* Z */
};

/*
 * R_P(theta) = exp(-i theta P / 2) = cos(theta/2) I - i sin(theta/2) P for
 * a Pauli P (the rotation gates whose generator form is given with the
 * parameter-shift rule, Eq. "parameter_shift" and the text after it).
 */
static void pauli_rotation(int p, double theta, cplx u[4])
{
    const double c = cos(0.5 * theta), s = sin(0.5 * theta);
    for (int k = 0; k < 4; ++k)
        u[k] = c * PAULI[0][k] - I * s * PAULI[p][k];
}

/*
 * U3(theta, phi, lambda) is not defined in the paper; the reading taken is
 * the OpenQASM 2 gate (the paper names OpenQASM as its interchange format):
 *   [[cos t/2, -e^{i lambda} sin t/2], [e^{i phi} sin t/2, e^{i(phi+lambda)} cos t/2]].
 */
static void u3_matrix(double theta, double phi, double lam, cplx u[4])
{
    const double c = cos(0.5 * theta), s = sin(0.5 * theta);
    u[0] = c;
    u[1] = -cexp(I * lam) * s;
    u[2] = cexp(I * phi) * s;
    u[3] = cexp(I * (phi + lam)) * c;
}

/* exp(-i theta/2 P (x) P) = cos(theta/2) I4 - i sin(theta/2) (P (x) P). */
static void pauli_pair_rotation(int p, double theta, cplx u[16])
{
    const double c = cos(0.5 * theta), s = sin(0.5 * theta);
    for (int r = 0; r < 4; ++r)
        for (int col = 0; col < 4; ++col) {
            cplx kron = PAULI[p][2 * (r >> 1) + (col >> 1)] *
                        PAULI[p][2 * (r & 1) + (col & 1)];
            u[4 * r + col] = (r == col ? c : 0.0) - I * s * kron;
        }
}

/* ------------------------------------------------------------------ */
/* One gate                                                             */
/* ------------------------------------------------------------------ */

/*
 * Apply one gate of the given kind to psi.  q[] holds the qubit operands
 * (control(s) first for controlled gates), ang[] the effective angles and
 * mat the user matrix for MAT1 (8 doubles) / MAT2 (32 doubles), row-major
 * (re, im) pairs.  Returns 0, or -1 for an invalid gate.
 */
int or_apply_gate(double *psi_d, int n, int kind, const int *q,
                  const double *ang, const double *mat)
{
    cplx *psi = (cplx *)psi_d;
    const int a = arity(kind);
    if (a < 0 || n < 1 || n > 40)
        return -1;
    for (int k = 0; k < a; ++k) {
        if (q[k] < 0 || q[k] >= n)
            return -1;
        for (int j = 0; j < k; ++j)
            if (q[j] == q[k])
                return -1;
    }
    cplx u[16];
    switch (kind) {
    case OG_H: {
        /* H = (1/sqrt 2)[[1,1],[1,-1]] (App. C, Hadamard on qubit 0). */
        const double r = 1.0 / sqrt(2.0);
        u[0] = r; u[1] = r; u[2] = r; u[3] = -r;
        apply_1q(psi, n, q[0], 0, u);
        return 0;
    }
    case OG_X: case OG_Y: case OG_Z:
        apply_1q(psi, n, q[0], 0, PAULI[kind - OG_H]);
        return 0;
    case OG_RX: case OG_RY: case OG_RZ:
        pauli_rotation(kind - OG_RX + 1, ang[0], u);
        apply_1q(psi, n, q[0], 0, u);
        return 0;
    case OG_U3:
        u3_matrix(ang[0], ang[1], ang[2], u);
        apply_1q(psi, n, q[0], 0, u);
        return 0;
    case OG_CNOT:
        apply_cnot_masks(psi, n, qmask(n, q[0]), qmask(n, q[1]));
        return 0;
    case OG_CCX:
        apply_cnot_masks(psi, n, qmask(n, q[0]) | qmask(n, q[1]),
                         qmask(n, q[2]));
        return 0;
    case OG_CZ:
        /* diag(1,1,1,-1): the -1 is applied exactly. */
        apply_phase_masks(psi, n, qmask(n, q[0]) | qmask(n, q[1]), -1.0);
        return 0;
    case OG_CP:
        /* CP(phi) = diag(1,1,1,e^{i phi}) (controlled-phase of Alg.
         * "Gate-Based QFT"; textbook definition, symmetric in its qubits). */
        apply_phase_masks(psi, n, qmask(n, q[0]) | qmask(n, q[1]),
                          cexp(I * ang[0]));
        return 0;
    case OG_SWAP: {
        const size_t m0 = qmask(n, q[0]), m1 = qmask(n, q[1]);
        const size_t dim = (size_t)1 << n;
        for (size_t i = 0; i < dim; ++i)
            if ((i & m0) && !(i & m1)) {
                size_t j = i ^ m0 ^ m1;
                cplx t = psi[i];
                psi[i] = psi[j];
                psi[j] = t;
            }
        return 0;
    }
    case OG_CRX: case OG_CRY: case OG_CRZ:
        /* |0><0|_c (x) I + |1><1|_c (x) R_P(theta)_t */
        pauli_rotation(kind - OG_CRX + 1, ang[0], u);
        apply_1q(psi, n, q[1], qmask(n, q[0]), u);
        return 0;
    case OG_RXX: case OG_RYY: case OG_RZZ:
        pauli_pair_rotation(kind - OG_RXX + 1, ang[0], u);
        apply_2q(psi, n, q[0], q[1], u);
        return 0;
    case OG_MAT1:
        for (int k = 0; k < 4; ++k)
            u[k] = mat[2 * k] + I * mat[2 * k + 1];
        apply_1q(psi, n, q[0], 0, u);
        return 0;
    case OG_MAT2:
        for (int k = 0; k < 16; ++k)
            u[k] = mat[2 * k] + I * mat[2 * k + 1];
        apply_2q(psi, n, q[0], q[1], u);
        return 0;
    default:
        return -1;
    }
}

/* |0...0>: psi[0] = 1 (Sec. "Dense State Vector Representation", zero_state). */
void or_zero_state(double *psi_d, int n)
{
    const size_t dim = (size_t)1 << n;
    memset(psi_d, 0, 2 * dim * sizeof(double));
    psi_d[0] = 1.0;
}

/* ------------------------------------------------------------------ */
/* Circuits                                                             */
/* ------------------------------------------------------------------ */

/*
 * A circuit is a list of G gate records given as flat arrays:
 *   kinds[G], qubits[3G], pidx[3G], angles[3G], mat_idx[G], mats[32*M].
 * The effective angle k of gate g is angles[3g+k] plus, when pidx[3g+k] >= 0,
 * params[pidx[3g+k]] (Sec. "Circuit Rebuilding Architecture": each
 * evaluation builds its gates from the parameter vector).  When shift_gate
 * >= 0, the angle slot shift_slot of that one gate occurrence gets an extra
 * offset shift_val (used by the parameter-shift rule below).
 */
static int run_circuit_shifted(double *psi, int n, int G, const int *kinds,
                               const int *qubits, const int *pidx,
                               const double *angles, const int *mat_idx,
                               const double *mats, int n_mats,
                               const double *params, int n_params,
                               int shift_gate, int shift_slot, double shift_val)
{
    for (int g = 0; g < G; ++g) {
        double ang[3];
        for (int k = 0; k < 3; ++k) {
            int p = pidx[3 * g + k];
            if (p >= n_params)
                return -1;
            ang[k] = angles[3 * g + k] + (p >= 0 ? params[p] : 0.0);
            if (g == shift_gate && k == shift_slot)
                ang[k] += shift_val;
        }
        const double *m = NULL;
        if (kinds[g] == OG_MAT1 || kinds[g] == OG_MAT2) {
            int mi = mat_idx[g];
            if (mi < 0 || mi >= n_mats)
                return -1;
            m = mats + 32 * (size_t)mi;
        }
        if (or_apply_gate(psi, n, kinds[g], qubits + 3 * g, ang, m) != 0)
            return -1;
    }
    return 0;
}

int or_run_circuit(double *psi, int n, int G, const int *kinds,
                   const int *qubits, const int *pidx, const double *angles,
                   const int *mat_idx, const double *mats, int n_mats,
                   const double *params, int n_params)
{
    return run_circuit_shifted(psi, n, G, kinds, qubits, pidx, angles,
                               mat_idx, mats, n_mats, params, n_params,
                               -1, -1, 0.0);
}

/*
 * Alg. "Gate-Based QFT": for i = 0..n-1, H on qubit i, then for j > i the
 * controlled-phase CP(pi / 2^(j-i)) with control i and target j; afterwards
 * SWAP(i, n-1-i) for i < floor(n/2).  Applied here to the dense state.
 */
void or_qft(double *psi, int n)
{
    for (int i = 0; i < n; ++i) {
        int q[3] = { i, 0, 0 };
        double ang[3] = { 0, 0, 0 };
        or_apply_gate(psi, n, OG_H, q, ang, NULL);
        for (int j = i + 1; j < n; ++j) {
            int qq[3] = { i, j, 0 };
            double a[3] = { M_PI / ldexp(1.0, j - i), 0, 0 };
            or_apply_gate(psi, n, OG_CP, qq, a, NULL);
        }
    }
    for (int i = 0; i < n / 2; ++i) {
        int q[3] = { i, n - 1 - i, 0 };
        double ang[3] = { 0, 0, 0 };
        or_apply_gate(psi, n, OG_SWAP, q, ang, NULL);
    }
}

/* ------------------------------------------------------------------ */
/* Expectation values                                                   */
/* ------------------------------------------------------------------ */

/*
 * <psi| P |psi> for one Pauli string P = P_0 (x) ... (x) P_{n-1}, taken from
 * its definition: phi = P psi (each factor applied as a one-qubit gate on a
 * copy), then the inner product sum_k conj(psi[k]) phi[k].  paulis[q] is one
 * of 'I', 'X', 'Y', 'Z' for qubit q (the Pauli-string observables of the VQE
 * and XYZ sections, Eq. "energy_expectation").  Returns 0 or -1.
 */
int or_pauli_expectation(const double *psi_d, int n, const char *paulis,
                         double *re_out, double *im_out)
{
    const size_t dim = (size_t)1 << n;
    cplx *phi = (cplx *)malloc(dim * sizeof(cplx));
    if (!phi)
        return -1;
    memcpy(phi, psi_d, dim * sizeof(cplx));
    for (int q = 0; q < n; ++q) {
        int kind;
        switch (paulis[q]) {
        case 'I': continue;
        case 'X': kind = OG_X; break;
        case 'Y': kind = OG_Y; break;
        case 'Z': kind = OG_Z; break;
        default: free(phi); return -1;
        }
        apply_1q(phi, n, q, 0, PAULI[kind - OG_H]);
    }
    const cplx *psi = (const cplx *)psi_d;
    cplx acc = 0;
    for (size_t k = 0; k < dim; ++k)
        acc += conj(psi[k]) * phi[k];
    free(phi);
    *re_out = creal(acc);
    *im_out = cimag(acc);
    return 0;
}

/*
 * E = sum_t c_t <psi|P_t|psi>, accumulated in term order (Hamiltonian as a
 * linear combination of Pauli strings, VQE "Problem Formulation";
 * Eq. "energy_expectation").  paulis holds n_terms rows of n characters.
 * *max_imag receives the largest |Im <P_t>| seen (must be ~0 for Hermitian P).
 */
int or_energy(const double *psi, int n, int n_terms, const double *coeffs,
              const char *paulis, double *energy, double *max_imag)
{
    double e = 0.0, mi = 0.0;
    for (int t = 0; t < n_terms; ++t) {
        double re, im;
        if (or_pauli_expectation(psi, n, paulis + (size_t)t * n, &re, &im))
            return -1;
        e += coeffs[t] * re;
        if (fabs(im) > mi)
            mi = fabs(im);
    }
    *energy = e;
    if (max_imag)
        *max_imag = mi;
    return 0;
}

/* One full evaluation f(theta): fresh |0..0>, circuit, energy. */
static int evaluate(int n, int G, const int *kinds, const int *qubits,
                    const int *pidx, const double *angles, const int *mat_idx,
                    const double *mats, int n_mats, const double *params,
                    int n_params, int n_terms, const double *coeffs,
                    const char *paulis, int sg, int ss, double sv, double *f)
{
    const size_t dim = (size_t)1 << n;
    double *psi = (double *)malloc(2 * dim * sizeof(double));
    if (!psi)
        return -1;
    or_zero_state(psi, n);
    int rc = run_circuit_shifted(psi, n, G, kinds, qubits, pidx, angles,
                                 mat_idx, mats, n_mats, params, n_params,
                                 sg, ss, sv);
    if (rc == 0)
        rc = or_energy(psi, n, n_terms, coeffs, paulis, f, NULL);
    free(psi);
    return rc;
}

int or_circuit_energy(int n, int G, const int *kinds, const int *qubits,
                      const int *pidx, const double *angles,
                      const int *mat_idx, const double *mats, int n_mats,
                      const double *params, int n_params, int n_terms,
                      const double *coeffs, const char *paulis, double *energy)
{
    return evaluate(n, G, kinds, qubits, pidx, angles, mat_idx, mats, n_mats,
                    params, n_params, n_terms, coeffs, paulis, -1, -1, 0.0,
                    energy);
}

/*
 * Parameter-shift gradient (Eq. "parameter_shift", s = pi/2, and the
 * ParameterShift gradient method of Sec. "Circuit Rebuilding Architecture"):
 * for every parameter i, evaluate f at theta + s e_i and theta - s e_i, each
 * from a fresh |0...0> with a rebuilt circuit, and take half the difference.
 *
 * Readings where the paper is silent:
 *  - a parameter used by several gate occurrences gets the sum over its
 *    occurrences of the rule applied to that occurrence alone (chain rule);
 *    with one occurrence per parameter this is exactly the paper's rule;
 *  - Pauli rotations, CP and the three U3 angles (each enters as a Pauli
 *    rotation or a phase with eigenvalue gap 1) use the two-term rule;
 *  - controlled rotations CRX/CRY/CRZ, whose generator has eigenvalues
 *    {0, +-1/2}, use the four-term rule of the general parameter-shift
 *    rules the paper cites (Wierichs et al.): shifts pi/2 and 3pi/2 with
 *    weights d1 = (sqrt2+1)/(4 sqrt2), d2 = (sqrt2-1)/(4 sqrt2):
 *      df = d1 [f(+pi/2) - f(-pi/2)] - d2 [f(+3pi/2) - f(-3pi/2)].
 * energy_out receives f(theta) (the "+1" evaluation).  Returns 0 or -1.
 */
int or_param_shift(int n, int G, const int *kinds, const int *qubits,
                   const int *pidx, const double *angles, const int *mat_idx,
                   const double *mats, int n_mats, const double *params,
                   int n_params, int n_terms, const double *coeffs,
                   const char *paulis, double *energy_out, double *grad)
{
    const double s = M_PI / 2.0;
    if (evaluate(n, G, kinds, qubits, pidx, angles, mat_idx, mats, n_mats,
                 params, n_params, n_terms, coeffs, paulis, -1, -1, 0.0,
                 energy_out))
        return -1;
    for (int i = 0; i < n_params; ++i) {
        grad[i] = 0.0;
        for (int g = 0; g < G; ++g)
            for (int k = 0; k < 3; ++k) {
                if (pidx[3 * g + k] != i)
                    continue;
                int kind = kinds[g];
                double fp, fm;
#define EVAL(shift, out)                                                       \
    if (evaluate(n, G, kinds, qubits, pidx, angles, mat_idx, mats, n_mats,     \
                 params, n_params, n_terms, coeffs, paulis, g, k, (shift),     \
                 &(out)))                                                      \
        return -1;
                EVAL(+s, fp);
                EVAL(-s, fm);
                if (kind == OG_CRX || kind == OG_CRY || kind == OG_CRZ) {
                    const double d1 = (sqrt(2.0) + 1.0) / (4.0 * sqrt(2.0));
                    const double d2 = (sqrt(2.0) - 1.0) / (4.0 * sqrt(2.0));
                    double fp3, fm3;
                    EVAL(+3.0 * s, fp3);
                    EVAL(-3.0 * s, fm3);
                    grad[i] += d1 * (fp - fm) - d2 * (fp3 - fm3);
                } else if (kind == OG_RX || kind == OG_RY || kind == OG_RZ ||
                           kind == OG_U3 || kind == OG_CP ||
                           kind == OG_RXX || kind == OG_RYY ||
                           kind == OG_RZZ) {
                    grad[i] += 0.5 * (fp - fm);
                } else {
                    return -1; /* no angle to differentiate */
                }
#undef EVAL
            }
    }
    return 0;
}

/*
 * The paper's own gradient loop taken literally (ParameterShift listing of
 * Sec. "Circuit Rebuilding Architecture"): the two-term rule with s = pi/2
 * for every parameter, whatever gate it feeds.  Used only to reproduce the
 * edge-case table of App. D, whose CRY parameter the paper differentiates
 * this way.
 */
int or_param_shift_two_term(int n, int G, const int *kinds, const int *qubits,
                            const int *pidx, const double *angles,
                            const int *mat_idx, const double *mats, int n_mats,
                            const double *params, int n_params, int n_terms,
                            const double *coeffs, const char *paulis,
                            double *grad)
{
    const double s = M_PI / 2.0;
    double *pp = (double *)malloc((size_t)(n_params > 0 ? n_params : 1) *
                                  sizeof(double));
    if (!pp)
        return -1;
    for (int i = 0; i < n_params; ++i) {
        double fp, fm;
        memcpy(pp, params, (size_t)n_params * sizeof(double));
        pp[i] += s;
        if (evaluate(n, G, kinds, qubits, pidx, angles, mat_idx, mats, n_mats,
                     pp, n_params, n_terms, coeffs, paulis, -1, -1, 0.0, &fp))
            goto fail;
        memcpy(pp, params, (size_t)n_params * sizeof(double));
        pp[i] -= s;
        if (evaluate(n, G, kinds, qubits, pidx, angles, mat_idx, mats, n_mats,
                     pp, n_params, n_terms, coeffs, paulis, -1, -1, 0.0, &fm))
            goto fail;
        grad[i] = (fp - fm) / 2.0;
    }
    free(pp);
    return 0;
fail:
    free(pp);
    return -1;
}

/* Squared norm sum_k |psi_k|^2, sequential FP64 sum. */
double or_norm2(const double *psi_d, int n)
{
    const cplx *psi = (const cplx *)psi_d;
    const size_t dim = (size_t)1 << n;
    double s = 0.0;
    for (size_t k = 0; k < dim; ++k)
        s += creal(psi[k]) * creal(psi[k]) + cimag(psi[k]) * cimag(psi[k]);
    return s;
}
