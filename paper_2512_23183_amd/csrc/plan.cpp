// Planner: groups lowered ops into passes over the state.
//
// A TILE pass holds every amplitude whose index agrees outside a set S of m
// bit positions ("local bits") in one workgroup's LDS.  S always contains
// the lowest bits so that global loads and stores are coalesced runs.  An op
// joins the pass if the bits it mixes (the target of a 2x2, both bits of a
// 4x4) are in S; diagonal ops (phases, controlled phases, ladders) join any
// pass because their factor is a function of the global index.  Ops that do
// not fit are deferred, and later ops that commute with every deferred op
// may still join (commutation test on bit sets), so layered circuits pack
// several layers' worth of gates per pass.
//
// SWAP gates are absorbed into a relabelling of bit positions; the standard
// layout is restored at the end by at most two in-place involution passes
// (every permutation is a product of two involutions).
#include <algorithm>
#include <cassert>
#include <numeric>
#include <set>

#include "sv_internal.h"

namespace sv {

namespace {

inline uint64_t bit(int b) { return 1ull << b; }

struct OpSets {
    uint64_t target = 0;   // bits mixed by the op (must be local)
    uint64_t control = 0;  // control bits
    uint64_t touch = 0;    // every bit the op depends on
    bool diag = false;
};

OpSets sets_of(const Op &op) {
    OpSets s;
    switch (op.kind) {
    case OP_U1: case OP_XPERM:
        s.target = bit(op.a);
        s.control = op.cmask;
        break;
    case OP_U2: case OP_SWAP:
        s.target = bit(op.a) | bit(op.b);
        s.control = op.cmask;
        break;
    case OP_DIAG:
        s.diag = true;
        s.touch = bit(op.a) | (op.b >= 0 ? bit(op.b) : 0) | op.cmask;
        break;
    case OP_LADDER:
        s.diag = true;
        s.touch = bit(op.a) | op.lmask;
        break;
    }
    if (!s.diag) s.touch = s.target | s.control;
    return s;
}

// Relabel bit positions of an op through phys[] (logical bit -> physical).
Op remap(const Op &op, const std::vector<int> &phys) {
    Op r = op;
    auto mapmask = [&](uint64_t m) {
        uint64_t o = 0;
        for (int b = 0; b < (int)phys.size(); ++b)
            if (m & bit(b)) o |= bit(phys[b]);
        return o;
    };
    if (r.a >= 0) r.a = phys[r.a];
    if (r.b >= 0) r.b = phys[r.b];
    r.cmask = mapmask(op.cmask);
    r.lmask = mapmask(op.lmask);  // ladders are only formed after relabelling
    return r;
}

// Decompose the permutation "data bit at physical position phys[i] must move
// to position i" into <= 2 involutions, each a list of disjoint bit pairs.
// Applying the first involution and then the second realises the move.
std::vector<std::vector<std::pair<int, int>>> involutions(const std::vector<int> &phys) {
    const int n = (int)phys.size();
    // dest[p] = where the bit now at position p must go
    std::vector<int> dest(n);
    for (int i = 0; i < n; ++i) dest[phys[i]] = i;
    std::vector<std::vector<std::pair<int, int>>> out;
    std::vector<std::pair<int, int>> s1, s2;
    std::vector<bool> seen(n, false);
    for (int p0 = 0; p0 < n; ++p0) {
        if (seen[p0] || dest[p0] == p0) { seen[p0] = true; continue; }
        std::vector<int> cyc;
        for (int p = p0; !seen[p]; p = dest[p]) { seen[p] = true; cyc.push_back(p); }
        const int k = (int)cyc.size();
        // cycle c0 -> c1 -> ... -> c_{k-1} -> c0 (position c_i goes to c_{i+1})
        // r1: c_i <-> c_{-i}, r2: c_i <-> c_{1-i};  r2 o r1 maps c_i -> c_{i+1}
        for (int i = 0; i < k; ++i) {
            int j = (k - i) % k;
            if (i < j) s1.push_back({cyc[i], cyc[j]});
            int j2 = ((1 - i) % k + k) % k;
            if (i < j2) s2.push_back({cyc[i], cyc[j2]});
        }
    }
    if (!s1.empty()) out.push_back(s1);
    if (!s2.empty()) out.push_back(s2);
    // verify on positions
    std::vector<int> pos(n);
    std::iota(pos.begin(), pos.end(), 0);  // pos[p] = current position of bit originally at p
    for (auto &inv : out)
        for (int p = 0; p < n; ++p)
            for (auto &pr : inv) {
                if (pos[p] == pr.first) { pos[p] = pr.second; break; }
                if (pos[p] == pr.second) { pos[p] = pr.first; break; }
            }
    for (int p = 0; p < n; ++p)
        if (pos[p] != dest[p]) fail(SV_EDEVICE, "internal: permutation decomposition failed");
    return out;
}

Pass make_perm_pass(int n, const std::vector<std::pair<int, int>> &pairs, int m_target, int l) {
    Pass ps;
    ps.kind = PASS_PERM;
    ps.swaps = pairs;
    std::vector<int> partner(n, -1);
    for (auto &pr : pairs) { partner[pr.first] = pr.second; partner[pr.second] = pr.first; }
    std::vector<bool> in(n, false);
    int cnt = 0;
    auto add = [&](int b) {
        if (!in[b]) { in[b] = true; ++cnt; }
    };
    for (int b = 0; b < l; ++b) {
        add(b);
        if (partner[b] >= 0) add(partner[b]);
    }
    // pad with the lowest bits that are unswapped, or whole pairs
    for (int b = 0; b < n && cnt < m_target; ++b) {
        if (in[b]) continue;
        if (partner[b] < 0) add(b);
        else if (cnt + 2 <= m_target) { add(b); add(partner[b]); }
    }
    for (int b = 0; b < n; ++b) (in[b] ? ps.local_bits : ps.free_bits).push_back(b);
    ps.m = (int)ps.local_bits.size();
    int run = 0;
    while (run < ps.m && ps.local_bits[run] == run) ++run;
    ps.l = run;
    return ps;
}

void finish_tile_pass(int n, Pass &ps, uint64_t S) {
    ps.kind = PASS_TILE;
    ps.local_bits.clear();
    ps.free_bits.clear();
    for (int b = 0; b < n; ++b) (S & bit(b) ? ps.local_bits : ps.free_bits).push_back(b);
    ps.m = (int)ps.local_bits.size();
    int run = 0;
    while (run < ps.m && ps.local_bits[run] == run) ++run;
    ps.l = run;
}

// Order the ops of a layered pass (uncontrolled one-qubit mixing ops and
// diagonals) so that the four-bit stage builder, which closes a stage at a
// fifth register bit, at a second mixing op on one bit, or at a mixing op
// on a bit of a diagonal that follows a mixing op of the stage, forms few
// stages.  Any topological order of the ops' conflict graph (two ops
// conflict unless they act on disjoint bits or are both diagonal) is the
// same product.  List scheduling: each stage first takes every diagonal
// whose predecessors are placed, then up to four ready mixing ops (on
// distinct bits by construction), those heading the longest chains of
// mixing ops first, then program order.
void order_layered_pass(std::vector<Op> &ops) {
    const int N = (int)ops.size();
    if (N < 3) return;
    std::vector<OpSets> st(N);
    for (int i = 0; i < N; ++i) st[i] = sets_of(ops[i]);
    std::vector<std::vector<int>> succ(N);
    std::vector<int> npred(N, 0);
    std::vector<int> last_mix(64, -1);
    std::vector<std::vector<int>> diags(64);
    auto edge = [&](int a, int b) {
        if (a < 0) return;
        succ[a].push_back(b);
        ++npred[b];
    };
    for (int j = 0; j < N; ++j) {
        const uint64_t bits = st[j].touch;
        if (st[j].diag) {
            for (uint64_t m = bits; m; m &= m - 1) {
                const int b = __builtin_ctzll(m);
                edge(last_mix[b], j);
                diags[b].push_back(j);
            }
        } else {
            for (uint64_t m = bits; m; m &= m - 1) {
                const int b = __builtin_ctzll(m);
                edge(last_mix[b], j);
                for (int d : diags[b]) edge(d, j);
                diags[b].clear();
                last_mix[b] = j;
            }
        }
    }
    // longest chain of mixing ops from each op (edges run forward)
    std::vector<int> height(N, 0);
    for (int j = N - 1; j >= 0; --j) {
        int h = 0;
        for (int k : succ[j]) h = std::max(h, height[k]);
        height[j] = h + (st[j].diag ? 0 : 1);
    }
    // ready sets kept up to date as ops are placed: O((N + edges) log N)
    std::vector<int> order, ready_diag;
    order.reserve(N);
    std::set<std::pair<int, int>> ready_mix;  // (-height, index): longest chains first
    auto enqueue = [&](int j) {
        if (st[j].diag) ready_diag.push_back(j);
        else ready_mix.insert({-height[j], j});
    };
    for (int j = 0; j < N; ++j)
        if (npred[j] == 0) enqueue(j);
    auto place = [&](int j) {
        order.push_back(j);
        for (int k : succ[j])
            if (--npred[k] == 0) enqueue(k);
    };
    while ((int)order.size() < N) {
        // every ready diagonal (placing one readies only mixing ops)
        std::vector<int> diag_now;
        diag_now.swap(ready_diag);
        std::sort(diag_now.begin(), diag_now.end());
        for (int j : diag_now) place(j);
        if (ready_mix.empty()) {
            if ((int)order.size() < N) return;  // cannot happen for a DAG; keep program order
            break;
        }
        // then up to four ready mixing ops, in program order
        std::vector<int> take;
        while (!ready_mix.empty() && take.size() < 4) {
            take.push_back(ready_mix.begin()->second);
            ready_mix.erase(ready_mix.begin());
        }
        std::sort(take.begin(), take.end());
        for (int j : take) place(j);
    }
    std::vector<Op> out;
    out.reserve(N);
    for (int j : order) out.push_back(ops[j]);
    ops.swap(out);
}

// ---------------------------------------------------------------------------
// Dense four-bit blocks.  A run of consecutive fixed (parameter-free) ops
// of a tile pass whose bits all lie in one set of at most four local bits
// is multiplied out into one 16 x 16 matrix (OP_DENSE4), applied by one
// MFMA stage (a 32 x 32 real GEMM per 32 groups of 16 amplitudes) instead
// of several register stages.  Only passes without CNOT-like ops are fused
// (their runs may instead be folded into LDS layout maps).
// ---------------------------------------------------------------------------

std::vector<int> mask_bits(uint64_t m) {
    std::vector<int> r;
    for (int b = 0; b < 64; ++b)
        if ((m >> b) & 1) r.push_back(b);
    return r;
}

// Register-engine VALU operations per amplitude of an op (the fusion model).
double op_cost(const Op &o) {
    switch (o.kind) {
    case OP_U1: {
        bool real = true;
        for (int k = 0; k < 4; ++k) real &= o.m[k].imag() == 0.0;
        return real ? 4.0 : 8.0;
    }
    case OP_U2: return 32.0;
    case OP_DIAG: return 2.0;
    default: return 1.0;
    }
}

uint64_t op_bits(const Op &o) {
    uint64_t b = o.cmask;
    if (o.a >= 0) b |= bit(o.a);
    if (o.b >= 0) b |= bit(o.b);
    return b;
}

// Apply op to a vector over the block bits (index bit k = global bit pos[k]).
void apply_op16(const Op &op, const int (&pos)[64], cd *v) {
    auto has = [&](int i, uint64_t mask) {
        for (int b : mask_bits(mask))
            if (!((i >> pos[b]) & 1)) return false;
        return true;
    };
    const int A = op.a >= 0 ? 1 << pos[op.a] : 0, B = op.b >= 0 ? 1 << pos[op.b] : 0;
    switch (op.kind) {
    case OP_U1:
        for (int i = 0; i < 16; ++i)
            if (!(i & A) && has(i, op.cmask)) {
                const cd x = v[i], y = v[i | A];
                v[i] = op.m[0] * x + op.m[1] * y;
                v[i | A] = op.m[2] * x + op.m[3] * y;
            }
        break;
    case OP_XPERM:
        for (int i = 0; i < 16; ++i)
            if (!(i & A) && has(i, op.cmask)) std::swap(v[i], v[i | A]);
        break;
    case OP_SWAP:
        for (int i = 0; i < 16; ++i)
            if ((i & A) && !(i & B) && has(i, op.cmask)) std::swap(v[i], v[i ^ A ^ B]);
        break;
    case OP_DIAG:
        for (int i = 0; i < 16; ++i)
            if (has(i, op.cmask)) {
                const int ba = (i & A) ? 1 : 0, bb = (B && (i & B)) ? 1 : 0;
                v[i] *= op.b >= 0 ? op.m[2 * ba + bb] : op.m[ba];
            }
        break;
    case OP_U2:
        for (int i = 0; i < 16; ++i)
            if (!(i & A) && !(i & B) && has(i, op.cmask)) {
                const int idx[4] = {i, i | B, i | A, i | A | B};  // 2 bit_a + bit_b
                cd x[4], y[4];
                for (int r = 0; r < 4; ++r) x[r] = v[idx[r]];
                for (int r = 0; r < 4; ++r) {
                    y[r] = 0.0;
                    for (int c = 0; c < 4; ++c) y[r] += op.m[4 * r + c] * x[c];
                }
                for (int r = 0; r < 4; ++r) v[idx[r]] = y[r];
            }
        break;
    default: fail(SV_EDEVICE, "internal: op kind cannot join a dense block");
    }
}

// Least total op cost for which a block is replaced by a dense op.
constexpr double DENSE4_MIN_COST = 24.0;

// force (2..4): every run of at least two fusible ops on at most force bits
// becomes a block, whatever its cost and gate kinds (a measurement mode:
// blocks of k = force qubits, each still applied as a padded 16 x 16).
void fuse_dense4(Pass &ps, Plan &plan, int force) {
    const int kmax = force >= 2 && force <= 4 ? force : 4;
    uint64_t local = 0;
    for (int b : ps.local_bits) local |= bit(b);
    for (const Op &o : ps.ops)
        if (o.kind == OP_XPERM || o.kind == OP_SWAP) return;
    auto fusible = [&](const Op &o) {
        return !o.param && (o.kind == OP_U1 || o.kind == OP_U2 || o.kind == OP_DIAG) &&
               (op_bits(o) & ~local) == 0;
    };
    std::vector<Op> out, blk;
    uint64_t B = 0;
    auto flush = [&]() {
        double cost = 0;
        bool two = false;  // a two-qubit gate that mixes amplitudes
        for (const Op &o : blk) {
            cost += op_cost(o);
            two |= o.kind == OP_U2;
        }
        // runs of one-qubit gates and diagonals alone are left to the
        // four-bit register stages (measured faster than the block)
        if (force ? blk.size() >= 2 : (two && blk.size() >= 2 && cost >= DENSE4_MIN_COST)) {
            // pad to four bits with the lowest local bits not in the block
            for (int b : ps.local_bits)
                if (__builtin_popcountll(B) < 4 && !(B & bit(b))) B |= bit(b);
            int pos[64];
            int k = 0;
            for (int b : mask_bits(B)) pos[b] = k++;
            std::vector<cd> U(256);
            for (int c = 0; c < 16; ++c) {
                cd v[16];
                for (int i = 0; i < 16; ++i) v[i] = i == c ? 1.0 : 0.0;
                for (const Op &o : blk) apply_op16(o, pos, v);
                for (int r = 0; r < 16; ++r) U[16 * r + c] = v[r];
            }
            Op d;
            d.kind = OP_DENSE4;
            d.lmask = B;
            d.dense = (int)plan.dense.size();
            plan.dense.push_back(std::move(U));
            out.push_back(d);
        } else {
            out.insert(out.end(), blk.begin(), blk.end());
        }
        blk.clear();
        B = 0;
    };
    for (const Op &o : ps.ops) {
        if (fusible(o)) {
            const uint64_t nb = B | op_bits(o);
            if (__builtin_popcountll(nb) <= kmax) {
                blk.push_back(o);
                B = nb;
                continue;
            }
            flush();
            blk.push_back(o);
            B = op_bits(o);
            continue;
        }
        flush();
        out.push_back(o);
    }
    flush();
    ps.ops.swap(out);
}

// A fixed, uncontrolled one-qubit gate with complex entries is written as
// diag(p0, p1) R diag(q0, q1) with R = [[c, -s], [s, c]] a real rotation
// (c = |u00|, s = |u10|): every 2x2 unitary has this form (U3 and RX are
// the configurations' cases).  Then each fixed uncontrolled one-qubit
// diagonal is merged into the previous one on the same bit when no op in
// between mixes that bit (a diagonal commutes with ops that leave its bit
// unmixed, controls included), and every such diagonal is normalised to
// diag(1, d1 / d0), its d0 going to one global phase kept on the first of
// them.  The register stages apply a real rotation in two FMAs per
// amplitude (its c or s goes to the pass scale) and a diag(1, r) in one
// complex multiply on half of the amplitudes, where a complex 2x2 costs
// eight operations per amplitude.  Exact up to rounding of the factors
// (computed in FP64).
void split_phases(std::vector<Op> &ops) {
    auto unitary = [](const Op &o) {
        const cd a = o.m[0], b = o.m[1], c = o.m[2], d = o.m[3];
        const double e1 = std::abs(std::norm(a) + std::norm(c) - 1.0);
        const double e2 = std::abs(std::norm(b) + std::norm(d) - 1.0);
        const double e3 = std::abs(a * std::conj(b) + c * std::conj(d));
        return e1 <= 1e-12 && e2 <= 1e-12 && e3 <= 1e-12;
    };
    auto diag1 = [](const Op &o) { return o.kind == OP_DIAG && !o.param && o.b < 0 && o.cmask == 0; };
    std::vector<Op> out;
    out.reserve(ops.size() + ops.size() / 2);
    for (const Op &o : ops) {
        bool real = true;
        for (int k = 0; k < 4; ++k) real &= o.m[k].imag() == 0.0;
        if (o.kind != OP_U1 || o.param || o.cmask != 0 || real || !unitary(o)) {
            out.push_back(o);
            continue;
        }
        const cd u00 = o.m[0], u01 = o.m[1], u10 = o.m[2], u11 = o.m[3];
        const double c = std::abs(u00), s = std::abs(u10);
        Op q, r, p;
        q.kind = p.kind = OP_DIAG;
        q.a = p.a = r.a = o.a;
        q.b = p.b = -1;
        q.gate = p.gate = -1;
        r.kind = OP_U1;
        r.gate = o.gate;
        if (s == 0.0) {  // diagonal already
            p.m[0] = u00;
            p.m[1] = u11;
            p.gate = o.gate;
            out.push_back(p);
            continue;
        }
        if (c == 0.0) {  // anti-diagonal: R = [[0, -1], [1, 0]]
            q.m[0] = 1.0;
            q.m[1] = -u01;
            p.m[0] = 1.0;
            p.m[1] = u10;
        } else {
            const cd p0 = u00 / c;
            q.m[0] = 1.0;
            q.m[1] = -u01 * c / (s * u00);
            p.m[0] = p0;
            p.m[1] = u10 / s;
        }
        r.m[0] = c;
        r.m[1] = -s;
        r.m[2] = s;
        r.m[3] = c;
        out.push_back(q);
        out.push_back(r);
        out.push_back(p);
    }
    // merge and normalise the fixed one-qubit diagonals
    std::vector<Op> merged;
    merged.reserve(out.size());
    std::vector<int> last(64, -1);  // per bit: index in merged of a diagonal that can take the next one
    cd phase = 1.0;
    int first = -1;
    for (const Op &o : out) {
        if (diag1(o)) {
            cd d0 = o.m[0], d1 = o.m[1];
            if (d0 == cd(0.0)) {  // singular: keep as it is
                merged.push_back(o);
                last[o.a] = -1;
                continue;
            }
            phase *= d0;
            d1 /= d0;
            if (last[o.a] >= 0) {
                merged[last[o.a]].m[1] *= d1;
                continue;
            }
            Op n = o;
            n.m[0] = 1.0;
            n.m[1] = d1;
            last[o.a] = (int)merged.size();
            if (first < 0) first = (int)merged.size();
            merged.push_back(n);
            continue;
        }
        const OpSets st = sets_of(o);
        if (!st.diag)
            for (int b : mask_bits(st.target)) last[b] = -1;
        merged.push_back(o);
    }
    if (first >= 0) {
        merged[first].m[0] *= phase;
        merged[first].m[1] *= phase;
    }
    ops.swap(merged);
}

}  // namespace

Plan make_plan(int n, const std::vector<Op> &ops_in, const PlanOptions &opt) {
    Plan plan;
    plan.n = n;
    plan.n_gate_ops = (int)ops_in.size();

    // fused passes work on 8-amplitude groups: states of 1-2 qubits (and the
    // plain path) take one sweep per gate
    if (!opt.fuse || n < 3) {
        for (const Op &op : ops_in) {
            Pass ps;
            ps.kind = PASS_SWEEP;
            ps.ops.push_back(op);
            plan.passes.push_back(std::move(ps));
        }
        return plan;
    }

    // 1. absorb SWAPs into a relabelling
    std::vector<int> phys(n);
    std::iota(phys.begin(), phys.end(), 0);
    std::vector<Op> ops;
    ops.reserve(ops_in.size());
    for (const Op &op : ops_in) {
        if (op.kind == OP_SWAP && op.cmask == 0) {
            std::swap(phys[op.a], phys[op.b]);
            continue;
        }
        ops.push_back(remap(op, phys));
    }

    // 1b. phase structure of fixed one-qubit gates (see split_phases)
    split_phases(ops);

    // 2. merge runs of fixed-angle controlled phases with a common control
    //    into ladders when their angles are a common multiple of the
    //    target's binary weight (the controlled-phase cascades of the QFT).
    {
        std::vector<Op> merged;
        merged.reserve(ops.size());
        size_t i = 0;
        while (i < ops.size()) {
            const Op &o = ops[i];
            auto is_cp = [](const Op &p) {
                return p.kind == OP_DIAG && !p.param && p.b >= 0 && p.cmask == 0 &&
                       p.ang > 0.0 && p.m[0] == cd(1) && p.m[1] == cd(1) && p.m[2] == cd(1);
            };
            bool cp = is_cp(o);
            if (!cp) { merged.push_back(o); ++i; continue; }
            // the control is whichever bit is shared by the run: try o.a then o.b
            Op best;
            size_t best_end = i + 1;
            for (int side = 0; side < 2; ++side) {
                const int c = side == 0 ? o.a : o.b;
                double turns = -1.0;
                uint64_t mask = 0;
                size_t j = i;
                for (; j < ops.size(); ++j) {
                    const Op &p = ops[j];
                    if (!is_cp(p) || (p.a != c && p.b != c)) break;
                    const int t = (p.a == c) ? p.b : p.a;
                    if (mask & bit(t)) break;
                    // phase 2 pi * turns * 2^t when bits c and t are set
                    double tu = p.ang / (2.0 * M_PI) / std::ldexp(1.0, t);
                    if (turns < 0) {
                        if (tu <= 0) break;
                        turns = tu;
                    } else if (std::abs(tu - turns) > 1e-15 * turns) {
                        break;
                    }
                    mask |= bit(t);
                }
                if (j - i >= 2 && j > best_end) {
                    best = Op();
                    best.kind = OP_LADDER;
                    best.a = c;
                    best.lmask = mask;
                    best.turns = turns;
                    best.gate = o.gate;
                    best_end = j;
                }
            }
            if (best_end > i + 1) {
                merged.push_back(best);
                i = best_end;
            } else {
                merged.push_back(o);
                ++i;
            }
        }
        ops.swap(merged);
    }

    // 3. greedy tile passes with commutation-aware deferral
    std::vector<Op> rest = ops;
    std::vector<OpSets> rsets(rest.size());
    for (size_t i = 0; i < rest.size(); ++i) rsets[i] = sets_of(rest[i]);
    // Layered circuits -- fixed uncontrolled one-qubit gates and diagonals
    // only, no CP ladders (layers of rotations with CZ / CP: the deep random
    // circuits) -- take their own tile width and search each pass's tile.
    // Elsewhere the search is not used: in a batched gradient a shifted
    // circuit runs the whole pass of its shifted gate, so larger passes
    // repeat more work; passes of two-qubit mixing gates (the Trotter
    // rotations) measured slower when denser; the QFT's ladder passes gain
    // nothing from it and prefer wider tiles than rotation layers.
    bool layered = true;
    for (const OpSets &st : rsets) {
        if (st.diag) continue;
        layered = layered && st.control == 0 && __builtin_popcountll(st.target) == 1;
    }
    for (const Op &o : rest) layered = layered && o.kind != OP_LADDER && !(o.kind != OP_DIAG && o.param);
    const int m = std::min(layered && opt.tile_bits_layers > 0 ? opt.tile_bits_layers : opt.tile_bits, n);
    const int l = std::min(opt.low_bits, m);
    const uint64_t low = (l >= 64) ? ~0ull : (bit(l) - 1);
    const uint64_t all = (n >= 64) ? ~0ull : (bit(n) - 1);
    // One pass over the remaining ops in order: an op joins when no deferred
    // op before it conflicts with it and (mixing ops) its target bits are in
    // the tile, which grows to m bits in program order (grow) or is the
    // fixed set S.  Returns the number of mixing ops that join; taken marks
    // the joining ops.  Stops once every bit is blocked for mixing.
    auto scan = [&](uint64_t &S, bool grow, std::vector<char> *taken) {
        int nS = __builtin_popcountll(S), mixing = 0;
        uint64_t DT = 0, DC = 0, DZ = 0;
        for (size_t i = 0; i < rest.size(); ++i) {
            const OpSets &s = rsets[i];
            bool can;
            if (s.diag) can = (s.touch & DT) == 0;
            else can = (s.target & (DT | DC | DZ)) == 0 && (s.control & DT) == 0;
            if (can && !s.diag) {
                const uint64_t need = s.target & ~S;
                const int add = __builtin_popcountll(need);
                if (!grow) can = add == 0;
                else if (nS + add <= m) { S |= need; nS += add; }
                else can = false;
            }
            if (can) {
                if (taken) (*taken)[i] = 1;
                if (!s.diag) ++mixing;
            } else {
                if (s.diag) DZ |= s.touch;
                else { DT |= s.target; DC |= s.control; }
                if ((DT & all) == all) break;
            }
        }
        return mixing;
    };
    while (!rest.empty()) {
        Pass ps;
        // the tile: grown in program order, then (layered circuits) improved
        // by swapping one chosen bit (the low l stay) for an outside one
        // while that lets more mixing ops join the pass (diagonals never
        // need the tile)
        uint64_t S = low;
        int best = scan(S, true, nullptr);
        if (layered && n > m && m > l) {
            for (int round = 0; round < 32; ++round) {
                int gain = 0;
                uint64_t bestS = S;
                for (int out = l; out < n; ++out) {
                    if (!(S & bit(out))) continue;
                    for (int in = l; in < n; ++in) {
                        if (S & bit(in)) continue;
                        uint64_t T = (S & ~bit(out)) | bit(in);
                        const int c = scan(T, false, nullptr);
                        if (c - best > gain) { gain = c - best; bestS = T; }
                    }
                }
                if (gain <= 0) break;
                best += gain;
                S = bestS;
            }
        }
        std::vector<char> taken(rest.size(), 0);
        {
            uint64_t T = S;
            scan(T, false, &taken);
        }
        int nS = __builtin_popcountll(S);
        std::vector<Op> deferred;
        std::vector<OpSets> dsets;
        for (size_t i = 0; i < rest.size(); ++i) {
            if (taken[i]) {
                ps.ops.push_back(rest[i]);
            } else {
                deferred.push_back(rest[i]);
                dsets.push_back(rsets[i]);
            }
        }
        // A pass of Hadamards and diagonals runs in four-bit stages: when
        // another pass follows anyway, hand its Hadamards beyond a multiple
        // of four (and every op taken after the first of them) to the next
        // pass, where they share stages with that pass's own.
        if (!deferred.empty()) {
            auto is_had = [](const Op &o) {
                return o.kind == OP_U1 && !o.param && o.cmask == 0 && o.m[0] == o.m[1] && o.m[0] == o.m[2] &&
                       o.m[3] == -o.m[0] && o.m[0].imag() == 0.0 && o.m[0].real() > 0.0;
            };
            bool only = true;
            std::vector<int> hbits;
            for (size_t i = 0; i < rest.size() && only; ++i) {
                if (!taken[i]) continue;
                const Op &o = rest[i];
                if (o.kind == OP_U1) {
                    only = is_had(o);
                    if (std::find(hbits.begin(), hbits.end(), o.a) == hbits.end()) hbits.push_back(o.a);
                } else {
                    only = o.kind == OP_LADDER || o.kind == OP_DIAG;
                }
            }
            const int h = (int)hbits.size(), drop = h % 4;
            if (only && h > 4 && drop != 0) {
                const uint64_t dropped = [&] {
                    uint64_t d = 0;
                    for (int k = h - drop; k < h; ++k) d |= bit(hbits[k]);
                    return d;
                }();
                size_t cut = rest.size();
                for (size_t i = 0; i < rest.size(); ++i)
                    if (taken[i] && rest[i].kind == OP_U1 && (bit(rest[i].a) & dropped)) {
                        cut = i;
                        break;
                    }
                // this pass keeps the ops taken before the cut; the next
                // passes get the untaken ones and the taken ones from the
                // cut on, in their original order
                std::vector<Op> keep_ops, back;
                std::vector<OpSets> back_sets;
                for (size_t i = 0; i < rest.size(); ++i) {
                    if (taken[i] && i < cut) {
                        keep_ops.push_back(rest[i]);
                    } else {
                        back.push_back(rest[i]);
                        back_sets.push_back(rsets[i]);
                    }
                }
                ps.ops.swap(keep_ops);
                deferred.swap(back);
                dsets.swap(back_sets);
                S = low;
                for (const Op &o : ps.ops) S |= sets_of(o).target;
                nS = __builtin_popcountll(S);
            }
        }
        // pad the tile with the lowest unused bits (longer contiguous runs)
        for (int b = 0; b < n && nS < m; ++b)
            if (!(S & bit(b))) { S |= bit(b); ++nS; }
        // (forced dense blocks take runs of consecutive ops: they keep the
        // program order, whose runs stay on few bits)
        if (layered && opt.order_layers && opt.dense_force == 0) order_layered_pass(ps.ops);
        finish_tile_pass(n, ps, S);
        if (ps.ops.empty()) fail(SV_EDEVICE, "internal: planner made no progress");
        if (opt.dense4 && ps.m >= 4) fuse_dense4(ps, plan, opt.dense_force);
        plan.passes.push_back(std::move(ps));
        rest.swap(deferred);
        rsets.swap(dsets);
    }

    // 4. restore the layout
    bool ident = true;
    for (int i = 0; i < n; ++i) ident &= phys[i] == i;
    if (!ident) {
        // two tiles live in LDS at once: 2 * 2^perm_bits amplitudes (64 KiB)
        const int mp = std::min(n, std::max(l, std::min(opt.tile_bits, opt.perm_bits)));
        for (auto &inv : involutions(phys)) plan.passes.push_back(make_perm_pass(n, inv, mp, l));
    }
    return plan;
}

}  // namespace sv
