// Autotuner for the tile widths of a context: gate tile passes, expectation
// passes and permutation passes, per amplitude precision.  Each candidate is
// timed on synthetic work of the requested size through the public entry
// points (planning included), and the fastest is kept in the context.  An
// optional text cache (one line per device / precision / size) skips the
// timing on later runs.
#include "sv_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <functional>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "sv.h"

namespace sv {
namespace {

struct Gates {
    std::vector<sv_gate> g;
    void add(int kind, int q0, int q1 = -1, double a = 0.0) {
        sv_gate x;
        x.kind = kind;
        x.q[0] = q0;
        x.q[1] = q1;
        x.q[2] = -1;
        x.param_idx[0] = x.param_idx[1] = x.param_idx[2] = -1;
        x.mat_idx = -1;
        x.angle[0] = a;
        x.angle[1] = x.angle[2] = 0.0;
        g.push_back(x);
    }
    sv_circuit circuit(int n) const {
        sv_circuit c;
        c.n_qubits = n;
        c.n_params = 0;
        c.gates = g.data();
        c.n_gates = g.size();
        c.mats = nullptr;
        c.n_mats = 0;
        return c;
    }
};

// Gate-based QFT (H, controlled phases, final swaps) followed by two layers
// of RY / RZ on every qubit and a CNOT ladder: both pass shapes the planner
// produces (ladder tiles + permutation, dense 1q stages + ladder of CNOTs).
Gates tuning_circuit(int n) {
    Gates G;
    for (int j = 0; j < n; ++j) {
        G.add(SV_H, j);
        for (int k = j + 1; k < n; ++k) G.add(SV_CP, k, j, M_PI / std::ldexp(1.0, k - j));
    }
    for (int j = 0; j < n / 2; ++j) G.add(SV_SWAP, j, n - 1 - j);
    for (int l = 0; l < 2; ++l) {
        for (int q = 0; q < n; ++q) G.add(SV_RY, q, -1, 0.1 + 0.01 * q + l);
        for (int q = 0; q < n; ++q) G.add(SV_RZ, q, -1, 0.2 + 0.02 * q + l);
        for (int q = 0; q + 1 < n; ++q) G.add(SV_CNOT, q, q + 1);
    }
    return G;
}

// Sixteen layers of U3 on every qubit and CZ on a random perfect matching
// per layer (a seeded shuffle of the qubits, paired in order): the
// rotation-layer passes, whose tiles the planner searches.  Matchings with
// a regular structure (q with q + 2^k) let the search pack more layers per
// pass than random ones and favoured narrower tiles than the random deep
// circuits run best at.
Gates layers_circuit(int n) {
    Gates G;
    uint64_t x = 0x9e3779b97f4a7c15ull;
    auto next = [&x] {  // splitmix64
        uint64_t z = (x += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    };
    std::vector<int> q(n);
    for (int l = 0; l < 16; ++l) {
        for (int j = 0; j < n; ++j) {
            G.add(SV_U3, j, -1, 0.3 + 0.05 * j + l);
            G.g.back().angle[1] = 0.7 + 0.03 * j;
            G.g.back().angle[2] = 1.1 + 0.02 * j;
        }
        for (int j = 0; j < n; ++j) q[j] = j;
        for (int j = n - 1; j > 0; --j) std::swap(q[j], q[next() % (uint64_t)(j + 1)]);
        for (int j = 0; j + 1 < n; j += 2) G.add(SV_CZ, q[j], q[j + 1]);
    }
    return G;
}

// Layers of fixed dense gates: U3 on every qubit, CZ on (q, q + 1) for even
// q, then RXX and RYY on alternating neighbour pairs, twice (the rotation
// runs are what the planner may fuse into dense four-qubit blocks).
Gates dense_circuit(int n) {
    Gates G;
    for (int l = 0; l < 2; ++l) {
        for (int q = 0; q < n; ++q) {
            G.add(SV_U3, q, -1, 0.3 + 0.05 * q + l);
            G.g.back().angle[1] = 0.7 + 0.03 * q;
            G.g.back().angle[2] = 1.1 + 0.02 * q;
        }
        for (int q = 0; q + 1 < n; q += 2) G.add(SV_CZ, q, q + 1);
        // two-qubit rotations on neighbours: the runs dense blocks are made
        // for (runs of one-qubit gates and diagonals never become blocks)
        for (int q = l % 2; q + 1 < n; q += 2) {
            G.add(SV_RXX, q, q + 1, 0.4 + 0.01 * q);
            G.add(SV_RYY, q, q + 1, 0.5 + 0.01 * q);
        }
    }
    return G;
}

// 2-local Pauli sum with every support pattern of a chain plus long-range
// pairs: (q, q+1) XX / YY / ZZ and (q, q + n/2) XY.
void tuning_hamiltonian(int n, std::vector<double> &coeffs, std::string &paulis) {
    auto term = [&](double c, int a, char pa, int b, char pb) {
        std::string s(n, 'I');
        s[a] = pa;
        s[b] = pb;
        coeffs.push_back(c);
        paulis += s;
    };
    for (int q = 0; q + 1 < n; ++q) {
        term(1.0, q, 'X', q + 1, 'X');
        term(0.8, q, 'Y', q + 1, 'Y');
        term(0.6, q, 'Z', q + 1, 'Z');
    }
    for (int q = 0; q + n / 2 < n; ++q) term(0.3, q, 'X', q + n / 2, 'Y');
}

double time_ms(sv_ctx *ctx, const std::function<void()> &f, int reps) {
    f();  // warm-up (and plan caches)
    if (sv_synchronize(ctx) != SV_OK) fail(SV_EDEVICE, "synchronize failed while tuning");
    double best = 1e300;
    for (int r = 0; r < reps; ++r) {
        const auto t0 = std::chrono::steady_clock::now();
        f();
        if (sv_synchronize(ctx) != SV_OK) fail(SV_EDEVICE, "synchronize failed while tuning");
        const auto t1 = std::chrono::steady_clock::now();
        best = std::min(best, std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
    return best;
}

std::string cache_key(const Ctx *ctx, int dtype, int n) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
    for (char &ch : arch)
        if (ch == ' ') ch = '_';
    std::ostringstream os;
    os << arch << " cu" << ctx->cu_count << " dtype" << dtype << " n" << n;
    return os.str();
}

}  // namespace

// Tunes ctx (handle ctx_ for the public entry points); errors throw.
void autotune(Ctx *ctx, sv_ctx *ctx_, int dtype, int n_qubits, const char *cache_path) {
    // tuned at the requested size up to 2^30 amplitudes: per-pass costs
    // shift with the state size (at 27 qubits complex128 the 11- and 12-bit
    // rotation-layer passes time within 1%, at 30 the 12-bit ones win by 8%)
    const int n = std::max(8, std::min(n_qubits, 30));
    if (n_qubits < 1 || n_qubits > SV_MAX_QUBITS) fail(SV_EINVAL, "n_qubits out of range");
    const std::string key = cache_key(ctx, dtype, n);
    bool hit = false;
    if (cache_path && *cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            if (line.compare(0, key.size() + 1, key + " ") != 0) continue;
            int tb = 0, lb = 0, eb = 0, pb = 0, dn = 0;
            if (std::sscanf(line.c_str() + key.size(), " tile=%d layers=%d expect=%d perm=%d dense=%d", &tb, &lb, &eb,
                            &pb, &dn) == 5 &&
                tb >= 6 && tb <= TILE_MAX[dtype] && lb >= 6 && lb <= TILE_MAX[dtype] && eb >= 6 &&
                eb <= EXPECT_MAX[dtype] && pb >= 6 && pb <= PERM_MAX[dtype] && (dn == 0 || dn == 1)) {
                ctx->tile_bits[dtype] = tb;
                ctx->tile_bits_layers[dtype] = lb;
                ctx->expect_bits[dtype] = eb;
                ctx->perm_bits[dtype] = pb;
                if (dtype == SV_C64) ctx->dense4 = dn == 1;
                hit = true;
            }
        }
    }
    if (!hit) {
        Gates G = tuning_circuit(n);
        const sv_circuit circ = G.circuit(n);
        Gates GL = layers_circuit(n);
        const sv_circuit lcirc = GL.circuit(n);
        std::vector<double> coeffs;
        std::string paulis;
        tuning_hamiltonian(n, coeffs, paulis);
        sv_pauli_sum ham{n, coeffs.size(), coeffs.data(), paulis.data()};
        sv_state *st = nullptr;
        int rc = sv_alloc(ctx_, n, dtype, &st);
        if (rc != SV_OK) fail((sv_status)rc, std::string("tuning state: ") + sv_last_error());
        struct Free {
            sv_state *s;
            ~Free() { sv_free(s); }
        } guard_state{st};
        const int reps = n >= 26 ? 2 : 3;
        auto apply = [&] {
            if (sv_reset(st) != SV_OK || sv_apply_circuit(st, &circ, nullptr, 0) != SV_OK)
                fail(SV_EDEVICE, std::string("tuning run: ") + sv_last_error());
        };
        // layered circuits (their own tile width): U3 + CZ layers
        auto apply_layers = [&] {
            if (sv_reset(st) != SV_OK || sv_apply_circuit(st, &lcirc, nullptr, 0) != SV_OK)
                fail(SV_EDEVICE, std::string("tuning run: ") + sv_last_error());
        };
        auto expect = [&] {
            double e;
            if (sv_expectation(st, &ham, &e, nullptr) != SV_OK)
                fail(SV_EDEVICE, std::string("tuning run: ") + sv_last_error());
        };
        // one width at a time, the others held; a candidate that the device
        // cannot run (an error from its launch) is skipped
        auto sweep = [&](int *field, int lo, int hi, const std::function<void()> &work) {
            double best = 1e300;
            int pick = *field;
            for (int v = lo; v <= hi; ++v) {
                *field = v;
                try {
                    const double t = time_ms(ctx_, work, reps);
                    if (t < best) best = t, pick = v;
                } catch (const Error &) {
                    (void)sv_synchronize(ctx_);
                }
            }
            *field = pick;
            return pick;
        };
        const int best_tb = sweep(&ctx->tile_bits[dtype], TILE_MAX[dtype] - 3, TILE_MAX[dtype], apply);
        const int best_lb = sweep(&ctx->tile_bits_layers[dtype], TILE_MAX[dtype] - 3, TILE_MAX[dtype], apply_layers);
        const int best_pb = sweep(&ctx->perm_bits[dtype], PERM_MAX[dtype] - 2, PERM_MAX[dtype], apply);
        const int best_eb = sweep(&ctx->expect_bits[dtype], EXPECT_MAX[dtype] - 3, EXPECT_MAX[dtype], expect);
        // complex64: dense four-qubit blocks on MFMA or the register stages,
        // whichever runs the dense layers faster
        int best_dn = ctx->dense4 ? 1 : 0;
        if (dtype == SV_C64) {
            Gates D = dense_circuit(n);
            const sv_circuit dc = D.circuit(n);
            auto apply_dense = [&] {
                if (sv_reset(st) != SV_OK || sv_apply_circuit(st, &dc, nullptr, 0) != SV_OK)
                    fail(SV_EDEVICE, std::string("tuning run: ") + sv_last_error());
            };
            int dn = best_dn;
            sweep(&dn, 0, 1, [&] {
                ctx->dense4 = dn == 1;
                apply_dense();
            });
            best_dn = dn;
            ctx->dense4 = best_dn == 1;
        }
        if (cache_path && *cache_path) {
            std::ofstream out(cache_path, std::ios::app);
            out << key << " tile=" << best_tb << " layers=" << best_lb << " expect=" << best_eb << " perm=" << best_pb
                << " dense=" << best_dn << "\n";
        }
    }
}

}  // namespace sv
