// Host side of the boundary: argument validation, gate lowering (FP64 gate
// matrices from the gate definitions), the QFT gate list, and Pauli-sum
// lowering to bit masks.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include "sv_internal.h"

namespace sv {

static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }
const std::string &last_error() { return g_last_error; }

void fail(int code, const std::string &msg) { throw Error{code, msg}; }

static int arity(int kind) {
    switch (kind) {
    case SV_H: case SV_X: case SV_Y: case SV_Z: case SV_RX: case SV_RY:
    case SV_RZ: case SV_U3: case SV_MAT1:
        return 1;
    case SV_CNOT: case SV_CZ: case SV_CP: case SV_SWAP: case SV_CRX:
    case SV_CRY: case SV_CRZ: case SV_RXX: case SV_RYY: case SV_RZZ:
    case SV_MAT2:
        return 2;
    case SV_CCX:
        return 3;
    default:
        return -1;
    }
}

static int n_angles(int kind) {
    switch (kind) {
    case SV_RX: case SV_RY: case SV_RZ: case SV_CP: case SV_CRX: case SV_CRY:
    case SV_CRZ: case SV_RXX: case SV_RYY: case SV_RZZ:
        return 1;
    case SV_U3:
        return 3;
    default:
        return 0;
    }
}

int gate_arity(int kind) { return arity(kind); }
int gate_n_angles(int kind) { return n_angles(kind); }

// Validation of a circuit and its parameter vector (every rule returns
// SV_EINVAL with a message naming the offending gate).
void check_circuit(const sv_circuit *c, const double *params, size_t n_params) {
    if (!c) fail(SV_EINVAL, "circuit is NULL");
    if (c->n_qubits < 1 || c->n_qubits > SV_MAX_QUBITS)
        fail(SV_EINVAL, "n_qubits must be in 1.." + std::to_string(SV_MAX_QUBITS));
    if (c->n_gates > SV_MAX_GATES) fail(SV_EINVAL, "too many gates");
    if (c->n_gates > 0 && !c->gates) fail(SV_EINVAL, "gates is NULL");
    if (c->n_params < 0) fail(SV_EINVAL, "n_params < 0");
    if ((size_t)c->n_params != n_params)
        fail(SV_EINVAL, "parameter vector has length " + std::to_string(n_params) +
                            ", circuit expects " + std::to_string(c->n_params));
    if (n_params > 0 && !params) fail(SV_EINVAL, "params is NULL");
    for (size_t i = 0; i < n_params; ++i)
        if (!std::isfinite(params[i]))
            fail(SV_EINVAL, "parameter " + std::to_string(i) + " is not finite");
    if (c->n_mats > 0 && !c->mats) fail(SV_EINVAL, "mats is NULL");
    for (size_t i = 0; i < 32 * c->n_mats; ++i)
        if (!std::isfinite(c->mats[i])) fail(SV_EINVAL, "matrix entry not finite");
    const int n = c->n_qubits;
    for (size_t gi = 0; gi < c->n_gates; ++gi) {
        const sv_gate &g = c->gates[gi];
        const std::string where = "gate " + std::to_string(gi) + ": ";
        int a = arity(g.kind);
        if (a < 0) fail(SV_EINVAL, where + "unknown kind " + std::to_string(g.kind));
        for (int k = 0; k < a; ++k) {
            if (g.q[k] < 0 || g.q[k] >= n)
                fail(SV_EINVAL, where + "qubit " + std::to_string(g.q[k]) + " out of range");
            for (int j = 0; j < k; ++j)
                if (g.q[j] == g.q[k]) fail(SV_EINVAL, where + "repeated qubit");
        }
        int na = n_angles(g.kind);
        for (int k = 0; k < 3; ++k) {
            if (k < na) {
                if (!std::isfinite(g.angle[k])) fail(SV_EINVAL, where + "angle not finite");
                if (g.param_idx[k] < -1 || g.param_idx[k] >= (int)n_params)
                    fail(SV_EINVAL, where + "param_idx " + std::to_string(g.param_idx[k]) +
                                        " out of range");
            } else if (g.param_idx[k] != -1) {
                fail(SV_EINVAL, where + "param_idx set on an angle slot the gate does not have");
            }
        }
        if (g.kind == SV_MAT1 || g.kind == SV_MAT2) {
            if (g.mat_idx < 0 || (size_t)g.mat_idx >= c->n_mats)
                fail(SV_EINVAL, where + "mat_idx out of range");
        }
    }
}

void check_pauli_sum(const sv_pauli_sum *h, int n) {
    if (!h) fail(SV_EINVAL, "Pauli sum is NULL");
    if (h->n_qubits != n)
        fail(SV_EINVAL, "Pauli sum has " + std::to_string(h->n_qubits) +
                            " qubits, state has " + std::to_string(n));
    if (h->n_terms > SV_MAX_TERMS) fail(SV_EINVAL, "too many terms");
    if (h->n_terms > 0 && (!h->coeffs || !h->paulis))
        fail(SV_EINVAL, "coeffs or paulis is NULL");
    for (size_t t = 0; t < h->n_terms; ++t) {
        if (!std::isfinite(h->coeffs[t]))
            fail(SV_EINVAL, "coefficient " + std::to_string(t) + " not finite");
        for (int q = 0; q < n; ++q) {
            char ch = h->paulis[t * (size_t)n + q];
            if (ch != 'I' && ch != 'X' && ch != 'Y' && ch != 'Z')
                fail(SV_EINVAL, "term " + std::to_string(t) + ": character not in IXYZ");
        }
    }
}

void effective_angles(const sv_gate &g, const double *params, double out[3]) {
    for (int k = 0; k < 3; ++k)
        out[k] = g.angle[k] + (g.param_idx[k] >= 0 ? params[g.param_idx[k]] : 0.0);
}

// ---------------------------------------------------------------------------
// Gate lowering
// ---------------------------------------------------------------------------

static inline int bitpos(int n, int q) { return n - 1 - q; }

Op lower_gate(int n, const sv_gate &g, const double ang[3], const double *mat,
              int gate_index) {
    Op op;
    op.gate = gate_index;
    for (int k = 0; k < 3; ++k)
        if (g.param_idx[k] >= 0) op.param = true;
    const cd I(0.0, 1.0);
    const double h = ang[0] * 0.5;
    const double c = std::cos(h), s = std::sin(h);
    auto set1 = [&](cd m0, cd m1, cd m2, cd m3) {
        op.m[0] = m0; op.m[1] = m1; op.m[2] = m2; op.m[3] = m3;
    };
    switch (g.kind) {
    case SV_H: {
        const double r = 1.0 / std::sqrt(2.0);
        op.kind = OP_U1; op.a = bitpos(n, g.q[0]);
        set1(r, r, r, -r);
        break;
    }
    case SV_X:
        op.kind = OP_XPERM; op.a = bitpos(n, g.q[0]);
        set1(0.0, 1.0, 1.0, 0.0);
        break;
    case SV_Y:
        op.kind = OP_U1; op.a = bitpos(n, g.q[0]);
        set1(0.0, -I, I, 0.0);
        break;
    case SV_Z:
        op.kind = OP_DIAG; op.a = bitpos(n, g.q[0]); op.b = -1;
        op.m[0] = 1.0; op.m[1] = -1.0;
        break;
    case SV_RX:
        op.kind = OP_U1; op.a = bitpos(n, g.q[0]);
        set1(c, -I * s, -I * s, c);
        break;
    case SV_RY:
        op.kind = OP_U1; op.a = bitpos(n, g.q[0]);
        set1(c, -s, s, c);
        op.real_family = true;
        break;
    case SV_RZ:
        op.kind = OP_DIAG; op.a = bitpos(n, g.q[0]); op.b = -1;
        op.m[0] = std::exp(-I * h); op.m[1] = std::exp(I * h);
        break;
    case SV_U3: {
        const double th = ang[0] * 0.5, ph = ang[1], la = ang[2];
        op.kind = OP_U1; op.a = bitpos(n, g.q[0]);
        set1(std::cos(th), -std::exp(I * la) * std::sin(th),
             std::exp(I * ph) * std::sin(th), std::exp(I * (ph + la)) * std::cos(th));
        break;
    }
    case SV_CNOT:
        op.kind = OP_XPERM; op.a = bitpos(n, g.q[1]);
        op.cmask = 1ull << bitpos(n, g.q[0]);
        set1(0.0, 1.0, 1.0, 0.0);
        break;
    case SV_CCX:
        op.kind = OP_XPERM; op.a = bitpos(n, g.q[2]);
        op.cmask = (1ull << bitpos(n, g.q[0])) | (1ull << bitpos(n, g.q[1]));
        set1(0.0, 1.0, 1.0, 0.0);
        break;
    case SV_CZ:
        op.kind = OP_DIAG; op.a = bitpos(n, g.q[0]); op.b = bitpos(n, g.q[1]);
        op.m[0] = 1.0; op.m[1] = 1.0; op.m[2] = 1.0; op.m[3] = -1.0;
        break;
    case SV_CP:
        op.kind = OP_DIAG; op.a = bitpos(n, g.q[0]); op.b = bitpos(n, g.q[1]);
        op.m[0] = 1.0; op.m[1] = 1.0; op.m[2] = 1.0; op.m[3] = std::exp(I * ang[0]);
        op.ang = ang[0];
        break;
    case SV_SWAP:
        op.kind = OP_SWAP; op.a = bitpos(n, g.q[0]); op.b = bitpos(n, g.q[1]);
        break;
    case SV_CRX:
        op.kind = OP_U1; op.a = bitpos(n, g.q[1]); op.cmask = 1ull << bitpos(n, g.q[0]);
        set1(c, -I * s, -I * s, c);
        break;
    case SV_CRY:
        op.kind = OP_U1; op.a = bitpos(n, g.q[1]); op.cmask = 1ull << bitpos(n, g.q[0]);
        set1(c, -s, s, c);
        op.real_family = true;
        break;
    case SV_CRZ:
        op.kind = OP_DIAG; op.a = bitpos(n, g.q[1]); op.b = -1;
        op.cmask = 1ull << bitpos(n, g.q[0]);
        op.m[0] = std::exp(-I * h); op.m[1] = std::exp(I * h);
        break;
    case SV_RXX: case SV_RYY: {
        // exp(-i t/2 P x P) = c I - i s P x P.  X x X has ones on the
        // anti-diagonal; Y x Y = [[0,0,0,-1],[0,0,1,0],[0,1,0,0],[-1,0,0,0]].
        op.kind = OP_U2; op.a = bitpos(n, g.q[0]); op.b = bitpos(n, g.q[1]);
        for (int k = 0; k < 16; ++k) op.m[k] = 0.0;
        for (int k = 0; k < 4; ++k) op.m[5 * k] = c;
        const double sg = (g.kind == SV_RXX) ? 1.0 : -1.0;
        op.m[3] = -I * s * sg;    // (0,3)
        op.m[12] = -I * s * sg;   // (3,0)
        op.m[6] = -I * s;         // (1,2)
        op.m[9] = -I * s;         // (2,1)
        break;
    }
    case SV_RZZ:
        op.kind = OP_DIAG; op.a = bitpos(n, g.q[0]); op.b = bitpos(n, g.q[1]);
        op.m[0] = std::exp(-I * h); op.m[1] = std::exp(I * h);
        op.m[2] = std::exp(I * h); op.m[3] = std::exp(-I * h);
        break;
    case SV_MAT1:
        op.kind = OP_U1; op.a = bitpos(n, g.q[0]);
        for (int k = 0; k < 4; ++k) op.m[k] = cd(mat[2 * k], mat[2 * k + 1]);
        break;
    case SV_MAT2:
        op.kind = OP_U2; op.a = bitpos(n, g.q[0]); op.b = bitpos(n, g.q[1]);
        for (int k = 0; k < 16; ++k) op.m[k] = cd(mat[2 * k], mat[2 * k + 1]);
        break;
    default:
        fail(SV_EINVAL, "unknown gate kind");
    }
    return op;
}

// Alg. "Gate-Based QFT": for i = 0..n-1: H(i), then CP(pi / 2^(j-i)) with
// control i and target j for every j > i; finally SWAP(i, n-1-i) for
// i < floor(n/2).
std::vector<sv_gate> qft_gates(int n) {
    std::vector<sv_gate> v;
    auto mk = [](int kind, int a, int b, double ang) {
        sv_gate g;
        std::memset(&g, 0, sizeof g);
        g.kind = kind;
        g.q[0] = a; g.q[1] = b; g.q[2] = -1;
        g.param_idx[0] = g.param_idx[1] = g.param_idx[2] = -1;
        g.mat_idx = -1;
        g.angle[0] = ang;
        return g;
    };
    for (int i = 0; i < n; ++i) {
        v.push_back(mk(SV_H, i, -1, 0.0));
        for (int j = i + 1; j < n; ++j)
            v.push_back(mk(SV_CP, i, j, std::ldexp(M_PI, -(j - i))));
    }
    for (int i = 0; i < n / 2; ++i) v.push_back(mk(SV_SWAP, i, n - 1 - i, 0.0));
    return v;
}

// ---------------------------------------------------------------------------
// Pauli sums: term t -> (x, z, ny); grouped by x in order of first appearance.
// ---------------------------------------------------------------------------

TermGroups lower_pauli_sum(const sv_pauli_sum &h) {
    TermGroups tg;
    const int n = h.n_qubits;
    tg.terms.resize(h.n_terms);
    for (size_t t = 0; t < h.n_terms; ++t) {
        Term &T = tg.terms[t];
        T.c = h.coeffs[t];
        for (int q = 0; q < n; ++q) {
            const uint64_t bit = 1ull << (n - 1 - q);
            switch (h.paulis[t * (size_t)n + q]) {
            case 'X': T.x |= bit; break;
            case 'Y': T.x |= bit; T.z |= bit; T.ny++; break;
            case 'Z': T.z |= bit; break;
            default: break;
            }
        }
        T.ny &= 3;
    }
    std::map<uint64_t, int> gid;
    std::vector<std::vector<int>> members;
    for (size_t t = 0; t < h.n_terms; ++t) {
        auto it = gid.find(tg.terms[t].x);
        int g;
        if (it == gid.end()) {
            g = (int)members.size();
            gid[tg.terms[t].x] = g;
            members.emplace_back();
            tg.gx.push_back(tg.terms[t].x);
        } else {
            g = it->second;
        }
        members[g].push_back((int)t);
    }
    for (auto &mb : members) {
        tg.g_begin.push_back((int)tg.order.size());
        for (int t : mb) tg.order.push_back(t);
        tg.g_end.push_back((int)tg.order.size());
    }
    return tg;
}

}  // namespace sv
