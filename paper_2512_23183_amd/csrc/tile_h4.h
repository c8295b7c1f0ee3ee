// Tile passes made only of uncontrolled one-qubit gates, ladders (merged
// controlled-phase runs) and diagonals -- the passes of the gate-based QFT
// (Alg. "Gate-Based QFT") and of layered random circuits.  The stages hold
// four register bits (16 amplitudes per thread) instead of three, so a pass
// of h mixing gates' bits takes ceil(h / 4) stages and ceil(h / 4) - 1 LDS
// round trips, and the op loop knows only these kinds.
#pragma once
#include <type_traits>

#include "device_common.h"

namespace sv {

template <int E>
__device__ __forceinline__ uint32_t loffx4(const uint32_t (&L)[4]) {
    return ((E & 1) ? L[0] : 0u) ^ ((E & 2) ? L[1] : 0u) ^ ((E & 4) ? L[2] : 0u) ^ ((E & 8) ? L[3] : 0u);
}
// LDS position of tile element j (the swizzle of h4_lane_order); linear
// over XOR, so the position of j0 | loff(e) is h4_swz(j0) ^ h4_swz(loff(e)).
__device__ __forceinline__ uint32_t h4_swz(uint32_t j) {
    return j ^ ((j >> 4) & 15u) ^ ((j >> 8) & 15u) ^ ((j >> 12) & 15u);
}
// Tile index of group index it: bit k of it goes to local bit lp[k].
__device__ __forceinline__ uint32_t h4_deposit(uint32_t it, uint64_t lp) {
    uint32_t j = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) j |= ((it >> k) & 1u) << ((uint32_t)(lp >> (4 * k)) & 15u);
    return j;
}
template <int E>
__device__ __forceinline__ uint64_t goff4(const uint64_t (&G)[4]) {
    return ((E & 1) ? G[0] : 0ull) | ((E & 2) ? G[1] : 0ull) | ((E & 4) ? G[2] : 0ull) | ((E & 8) ? G[3] : 0ull);
}

// Sums and differences on register slot I (the 1/sqrt 2 goes to the pass
// scale, as in the three-bit engine).
template <int I, typename R>
__device__ __forceinline__ void h4_had(V2<R> (&v)[16]) {
    static_for<0, 16>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        if constexpr (!(e & (1 << I))) {
            const V2<R> a = v[e], b = v[e | (1 << I)];
            v[e].x = a.x + b.x;
            v[e].y = a.y + b.y;
            v[e | (1 << I)].x = a.x - b.x;
            v[e | (1 << I)].y = a.y - b.y;
        }
    });
}

// Uncontrolled 2x2 on register slot I (an exchange for X).  K as in the
// three-bit engine: 0 complex matrix, 1 real matrix, 2 exchange, 4 / 5 the
// scaled rotations (coefficient in entry 5; their factor, like the
// Hadamard's, is in the pass scale).
template <int I, int K, typename R>
__device__ __forceinline__ void h4_u1(V2<R> (&v)[16], const DevOp<R> &op) {
    const V2<R> m0 = mat_at(op, (K == 4 || K == 5) ? 5 : 0), m1 = mat_at(op, 1), m2 = mat_at(op, 2),
                m3 = mat_at(op, 3);
    static_for<0, 16>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        if constexpr (!(e & (1 << I))) {
            constexpr int f = e | (1 << I);
            const V2<R> x = v[e], y = v[f];
            V2<R> nx, ny;
            if constexpr (K == 2) {
                nx = y;
                ny = x;
            } else if constexpr (K == 1) {
                nx.x = m0.x * x.x + m1.x * y.x;
                nx.y = m0.x * x.y + m1.x * y.y;
                ny.x = m2.x * x.x + m3.x * y.x;
                ny.y = m2.x * x.y + m3.x * y.y;
            } else if constexpr (K == 4) {
                nx.x = x.x - m0.x * y.x;
                nx.y = x.y - m0.x * y.y;
                ny.x = m0.x * x.x + y.x;
                ny.y = m0.x * x.y + y.y;
            } else if constexpr (K == 5) {
                nx.x = m0.x * x.x - y.x;
                nx.y = m0.x * x.y - y.y;
                ny.x = x.x + m0.x * y.x;
                ny.y = x.y + m0.x * y.y;
            } else {
                nx = cmac2(m0, x, m1, y);
                ny = cmac2(m2, x, m3, y);
            }
            v[e] = nx;
            v[f] = ny;
        }
    });
}

template <int K, typename R>
__device__ __forceinline__ void h4_u1_at(V2<R> (&v)[16], const DevOp<R> &op) {
    if (op.ra == 0) h4_u1<0, K, R>(v, op);
    else if (op.ra == 1) h4_u1<1, K, R>(v, op);
    else if (op.ra == 2) h4_u1<2, K, R>(v, op);
    else h4_u1<3, K, R>(v, op);
}

// Diagonal amplitude *= d[2 bit_a + bit_b] (d[bit_a] without b) where all
// control bits are set; each of a, b and the controls is a register slot
// (taken from e) or a bit of the group (taken from k0).
// The group-bit conditions differ between the lanes of a wave: they are
// applied as selects, not branches (a divergent branch around the sixteen
// amplitudes would make the compiler copy all of them at the join).
template <typename R>
__device__ __forceinline__ void h4_diag(V2<R> (&v)[16], V2<R> &acc, uint64_t k0, const uint64_t (&G)[4],
                                        const DevOp<R> &op) {
    const uint64_t regs = G[0] | G[1] | G[2] | G[3];
    const uint64_t gc = op.cmask & ~regs;
    const bool gon = (k0 & gc) == gc;
    const uint32_t ec = ((op.cmask & G[0]) ? 1u : 0u) | ((op.cmask & G[1]) ? 2u : 0u) |
                        ((op.cmask & G[2]) ? 4u : 0u) | ((op.cmask & G[3]) ? 8u : 0u);
    auto slot = [&](int bitpos) {
        const uint64_t m = 1ull << bitpos;
        return G[0] == m ? 0 : G[1] == m ? 1 : G[2] == m ? 2 : G[3] == m ? 3 : -1;
    };
    const int sa = slot(op.a), sb = op.b >= 0 ? slot(op.b) : -1;
    const uint32_t ga = (uint32_t)((k0 >> op.a) & 1), gb = op.b >= 0 ? (uint32_t)((k0 >> op.b) & 1) : 0u;
    const V2<R> d0 = mat_at(op, 0), d1 = mat_at(op, 1), d2 = mat_at(op, 2), d3 = mat_at(op, 3);
    if (sa < 0 && sb < 0 && ec == 0) {
        const V2<R> f = op.b >= 0 ? vsel(ga != 0, vsel(gb != 0, d3, d2), vsel(gb != 0, d1, d0)) : vsel(ga != 0, d1, d0);
        acc = vsel(gon, cmul(acc, f), acc);
        return;
    }
    static_for<0, 16>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        const uint32_t ba = sa >= 0 ? ((uint32_t)e >> sa) & 1u : ga;
        V2<R> f;
        if (op.b >= 0) {
            const uint32_t bb = sb >= 0 ? ((uint32_t)e >> sb) & 1u : gb;
            f = vsel(ba != 0, vsel(bb != 0, d3, d2), vsel(bb != 0, d1, d0));
        } else {
            f = vsel(ba != 0, d1, d0);
        }
        const bool on = gon && ((uint32_t)e & ec) == ec;
        v[e] = vsel(on, cmul(v[e], f), v[e]);
    });
}

// Scaled real rotation on register slot I: (x, y) <- (x - t y, y + t x)
// (t = 0: identity); the cosine factor is in the pass scale.
template <int I, typename R>
__device__ __forceinline__ void h4_rot(V2<R> (&v)[16], R t) {
    static_for<0, 16>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        if constexpr (!(e & (1 << I))) {
            constexpr int f = e | (1 << I);
            const V2<R> x = v[e], y = v[f];
            v[e].x = x.x - t * y.x;
            v[e].y = x.y - t * y.y;
            v[f].x = y.x + t * x.x;
            v[f].y = y.y + t * x.y;
        }
    });
}

// Factor of a diagonal on bits outside the registers for the group at k0
// (a select per lane, not a branch).
template <typename R>
__device__ __forceinline__ void diag_factor(V2<R> &acc, uint64_t k, const DevOp<R> &op) {
    const bool on = (k & op.cmask) == op.cmask;
    const uint32_t ba = (uint32_t)((k >> op.a) & 1);
    V2<R> f;
    if (op.b >= 0) {
        const uint32_t bb = (uint32_t)((k >> op.b) & 1);
        f = vsel(ba != 0, vsel(bb != 0, mat_at(op, 3), mat_at(op, 2)), vsel(bb != 0, mat_at(op, 1), mat_at(op, 0)));
    } else {
        f = vsel(ba != 0, mat_at(op, 1), mat_at(op, 0));
    }
    acc = vsel(on, cmul(acc, f), acc);
}

// Uncontrolled one-qubit diagonal diag(d0, d1) on register slot I: d0 goes
// to the group factor (nothing to do when it is 1: OPF_PAT), the elements
// with the bit set are multiplied by d1 / d0 (complex entry 4 of m).
template <int I, typename R>
__device__ __forceinline__ void h4_diag1(V2<R> (&v)[16], V2<R> &acc, const DevOp<R> &op) {
    if (!(op.flags & OPF_PAT)) acc = cmul(acc, mat_at(op, 0));
    const V2<R> r = mat_at(op, 4);
    static_for<0, 16>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        if constexpr ((e >> I) & 1) v[e] = cmul(v[e], r);
    });
}

// Gathered diagonals of a stage (OP_DIAG16): element e *= m[e], negated
// where e & c has odd parity, c_r = parity(k0 & M_r).  The parities become a
// 16-bit mask of the negated elements, xor-ed into the sign bits.
template <typename R>
__device__ __forceinline__ void h4_table(V2<R> (&v)[16], uint64_t k0, const DevOp<R> &op) {
    uint32_t neg = 0;
    if (op.flags & OPF_SGN) {
        const uint32_t c0 = __popcll(k0 & op.cmask) & 1, c1 = __popcll(k0 & op.lcmask) & 1,
                       c2 = __popcll(k0 & op.gcmask) & 1, c3 = __popcll(k0 & op.lmask) & 1;
        neg = (c0 ? 0xAAAAu : 0u) ^ (c1 ? 0xCCCCu : 0u) ^ (c2 ? 0xF0F0u : 0u) ^ (c3 ? 0xFF00u : 0u);
    }
    static_for<0, 16>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        V2<R> t = mat_at(op, e);
        if ((neg >> e) & 1) {
            t.x = -t.x;
            t.y = -t.y;
        }
        v[e] = cmul(v[e], t);
    });
}

// The same with the sign variant fixed at compile time; the signs go to
// the sign bits of the products (no select on the table entries).
template <bool SGN, typename R>
__device__ __forceinline__ void rl_table(V2<R> (&v)[16], uint64_t k0, const DevOp<R> &op) {
    using U = typename std::conditional<sizeof(R) == 4, uint32_t, uint64_t>::type;
    uint32_t neg = 0;
    if constexpr (SGN) {
        const uint32_t c0 = __popcll(k0 & op.cmask) & 1, c1 = __popcll(k0 & op.lcmask) & 1,
                       c2 = __popcll(k0 & op.gcmask) & 1, c3 = __popcll(k0 & op.lmask) & 1;
        neg = (c0 ? 0xAAAAu : 0u) ^ (c1 ? 0xCCCCu : 0u) ^ (c2 ? 0xF0F0u : 0u) ^ (c3 ? 0xFF00u : 0u);
    }
    static_for<0, 16>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        V2<R> w = cmul(v[e], mat_at(op, e));
        if constexpr (SGN) {
            const U sb = (U)((neg >> e) & 1u) << (8 * sizeof(R) - 1);
            w.x = __builtin_bit_cast(R, __builtin_bit_cast(U, w.x) ^ sb);
            w.y = __builtin_bit_cast(R, __builtin_bit_cast(U, w.y) ^ sb);
        }
        v[e] = w;
    });
}

// Ladder: where bit a is set, multiply by exp(2 pi i turns (k & lmask)) =
// (group phase from the tile-independent tables and the tile factor) x K_e
// (the phase of element e's register-bit offset, complex slot e of op.m).
// RA: register slot of a, or -1 when a is the same for the whole group.
template <int RA, typename R>
__device__ __forceinline__ void h4_ladder(V2<R> (&v)[16], uint32_t j0, uint64_t k0, const DevOp<R> &op,
                                          const TileCtx<R> &tc) {
    if (RA < 0 && !((k0 >> op.a) & 1)) return;
    const uint32_t i0 = j0 & ((1u << tc.lsa) - 1), i1 = (1 << tc.lsa) + ((j0 >> tc.lsa) & ((1u << tc.lsb) - 1)),
                   i2 = (1 << tc.lsa) + (1 << tc.lsb) + (j0 >> (tc.lsa + tc.lsb));
    V2<R> p;
    if (tc.ltl) {
        const SV_LDS R *T = tc.ltl + 2 * op.tab;
        p = cmul(cmul(lds_v2<R>(T, i0), lds_v2<R>(T, i1)), lds_v2<R>(T, i2));
    } else {
        const V2<R> *T = tc.ltabs + op.tab;
        p = cmul(cmul(T[i0], T[i1]), T[i2]);
    }
    if (tc.Gs) p = cmul(p, lds_v2<R>(tc.Gs, op.tslot));
    static_for<0, 16>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        if constexpr (RA < 0 || (e & (1 << (RA < 0 ? 0 : RA)))) v[e] = cmul(v[e], cmul(p, mat_at(op, e)));
    });
}

// Diagonal whose only factor differs from 1 on the all-ones pattern of
// (controls, a, b): that factor (-1 exactly with NEG) where all are set.
// The pattern splits into the group's bits (all set in k0, else nothing to
// do) and the register slots it covers (emask: all set in e).
// ACC (general stages): a diagonal that involves no register bit goes into
// acc, the group's factor (such diagonals commute with every op of the
// stage; it is applied once after them).
template <bool NEG, bool ACC, typename R>
__device__ __forceinline__ void h4_pat(V2<R> (&v)[16], V2<R> &acc, uint64_t k0, const uint64_t (&G)[4],
                                       const DevOp<R> &op) {
    const uint64_t all = op.cmask | (1ull << op.a) | (op.b >= 0 ? (1ull << op.b) : 0ull);
    const uint64_t gmask = all & ~(G[0] | G[1] | G[2] | G[3]);
    // per lane: a select in the stages with a group factor (ACC), a branch in
    // the Hadamard / ladder stages (measured faster there)
    if constexpr (!ACC) {
        if ((k0 & gmask) != gmask) return;
    }
    const bool gon = !ACC || (k0 & gmask) == gmask;
    const uint32_t emask = ((all & G[0]) ? 1u : 0u) | ((all & G[1]) ? 2u : 0u) | ((all & G[2]) ? 4u : 0u) |
                           ((all & G[3]) ? 8u : 0u);
    const V2<R> dl = op.b >= 0 ? mat_at(op, 3) : mat_at(op, 1);
    if (ACC && emask == 0) {
        if constexpr (NEG) {
            acc.x = gon ? -acc.x : acc.x;
            acc.y = gon ? -acc.y : acc.y;
        } else {
            acc = vsel(gon, cmul(acc, dl), acc);
        }
        return;
    }
    static_for<0, 16>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        const bool on = gon && ((uint32_t)e & emask) == emask;
        if constexpr (NEG) {
            v[e].x = on ? -v[e].x : v[e].x;
            v[e].y = on ? -v[e].y : v[e].y;
        } else {
            v[e] = vsel(on, cmul(v[e], dl), v[e]);
        }
    });
}

// One four-bit stage.  MODE bit 0: read the groups from global memory (or
// synthesise |0...0>), else from the LDS tile; MODE bit 1: write them to
// global memory (scaled by the pass scale), else to the LDS tile.
// KIND 1: any of the kinds above; 2: Hadamards, ladders and pattern
// diagonals only (the QFT's passes); 3: Hadamards, real rotations and
// diagonals only (layered circuits once their one-qubit gates are split
// into rotations and phases).  The smaller op loops of 2 and 3 keep the
// sixteen amplitudes and the op data in registers without spilling.
// ONE: the caller guarantees at most one group per thread (2^m / 16 <= TPB);
// the body then runs once with no loop around it, so nothing of the stage
// (its tables, rotation slopes and masks) is hoisted and kept live in
// scalar registers across iterations that never come.
template <typename R, int TPB, int MODE, int KIND, int RL = 0, bool ONE = false>
__device__ __forceinline__ void h4_stage(V2<R> *tile, V2<R> *__restrict__ gpsi, const TileCtx<R> &tc,
                                         const DevStage &S, const DevOp<R> *__restrict__ ops, int ovr_index,
                                         const DevOp<R> *ovr) {
    constexpr bool GEN = KIND != 2;
    const uint32_t nitems = (1u << tc.m) >> 4;
    const int r[4] = {S.r0, S.r1, S.r2, S.r3};
    // LDS positions of the register-bit offsets (swizzled tile)
    const uint32_t L[4] = {h4_swz(1u << r[0]), h4_swz(1u << r[1]), h4_swz(1u << r[2]), h4_swz(1u << r[3])};
    const uint64_t G[4] = {gbit(tc, r[0]), gbit(tc, r[1]), gbit(tc, r[2]), gbit(tc, r[3])};
    // complex64 with global bit 0 as register slot 0: elements 2i, 2i + 1
    // are adjacent in HBM and move as one 16-byte access
    const bool pairg = sizeof(R) == 4 && G[0] == 1ull;
    using P = typename Pair<R>::T;
    for (uint32_t it = threadIdx.x; it < nitems; it += TPB) {
        const uint32_t j0 = h4_deposit(it, S.lane_pos);
        const uint32_t p0 = h4_swz(j0);
        const uint64_t k0 = gaddr(tc, j0);
        V2<R> v[16];
        if constexpr (MODE & 1) {
            if (tc.zero) {
                static_for<0, 16>([&](auto EC) {
                    constexpr int e = decltype(EC)::value;
                    v[e].x = (k0 | goff4<e>(G)) == 0 ? (R)1 : (R)0;
                    v[e].y = 0;
                });
            } else if (pairg) {
                static_for<0, 8>([&](auto IC) {
                    constexpr int e = 2 * decltype(IC)::value;
                    const P w = *reinterpret_cast<const P *>(gpsi + SV_GIDX(k0 | goff4<e>(G), tc.dim));
                    v[e] = pair_lo(w);
                    v[e + 1] = pair_hi(w);
                });
            } else {
                static_for<0, 16>([&](auto EC) {
                    constexpr int e = decltype(EC)::value;
                    v[e] = gpsi[SV_GIDX(k0 | goff4<e>(G), tc.dim)];
                });
            }
        } else {
            static_for<0, 16>([&](auto EC) {
                constexpr int e = decltype(EC)::value;
                v[e] = tile[SV_LIDX(p0 ^ loffx4<e>(L), 1u << tc.m)];
            });
        }
        V2<R> acc;
        acc.x = (R)1;
        acc.y = (R)0;
        if constexpr (KIND == 4) {
            // a rotation layer: straight-line code, its variant (RL) fixed at
            // compile time
            if constexpr (RL & 4)
                for (int o = S.op_begin; o < S.op_end; ++o) diag_factor(acc, k0, ops[o]);
            if constexpr (RL & 1) rl_table<(RL & 2) != 0>(v, k0, ops[S.tpre]);
            const DevOp<R> &q = ops[S.rot];
            h4_rot<0>(v, q.m[0]);
            h4_rot<1>(v, q.m[2]);
            h4_rot<2>(v, q.m[4]);
            h4_rot<3>(v, q.m[6]);
            rl_table<(RL & 2) != 0>(v, k0, ops[S.tpost]);
        }
        for (int o = S.op_begin; KIND != 4 && o < S.op_end; ++o) {
            const DevOp<R> &op = (o == ovr_index) ? *ovr : ops[o];
            if constexpr (KIND == 3) {
                if (op.kind == OP_DIAG16) {
                    h4_table(v, k0, op);
                    continue;
                }
                if (op.kind == OP_U1) {
                    if (op.flags & OPF_HAD) {
                        if (op.ra == 0) h4_had<0, R>(v);
                        else if (op.ra == 1) h4_had<1, R>(v);
                        else if (op.ra == 2) h4_had<2, R>(v);
                        else h4_had<3, R>(v);
                    } else if (op.flags & OPF_ROTC) {
                        h4_u1_at<4>(v, op);
                    } else {
                        h4_u1_at<5>(v, op);
                    }
                } else if (op.flags & OPF_REG1) {
                    if (op.ra == 0) h4_diag1<0>(v, acc, op);
                    else if (op.ra == 1) h4_diag1<1>(v, acc, op);
                    else if (op.ra == 2) h4_diag1<2>(v, acc, op);
                    else h4_diag1<3>(v, acc, op);
                } else if (op.flags & OPF_PAT) {
                    if (op.flags & OPF_NEG) h4_pat<true, true>(v, acc, k0, G, op);
                    else h4_pat<false, true>(v, acc, k0, G, op);
                } else {
                    h4_diag(v, acc, k0, G, op);
                }
                continue;
            }
            if (op.kind == OP_U1) {
                if (!GEN || (op.flags & OPF_HAD)) {
                    if (op.ra == 0) h4_had<0, R>(v);
                    else if (op.ra == 1) h4_had<1, R>(v);
                    else if (op.ra == 2) h4_had<2, R>(v);
                    else h4_had<3, R>(v);
                } else if (op.flags & OPF_ROTC) {
                    h4_u1_at<4>(v, op);
                } else if (op.flags & OPF_ROTS) {
                    h4_u1_at<5>(v, op);
                } else if (op.flags & OPF_REAL) {
                    h4_u1_at<1>(v, op);
                } else {
                    h4_u1_at<0>(v, op);
                }
            } else if (GEN && op.kind == OP_XPERM) {
                h4_u1_at<2>(v, op);
            } else if (op.kind == OP_LADDER) {
                if (op.ra == 0) h4_ladder<0>(v, j0, k0, op, tc);
                else if (op.ra == 1) h4_ladder<1>(v, j0, k0, op, tc);
                else if (op.ra == 2) h4_ladder<2>(v, j0, k0, op, tc);
                else if (op.ra == 3) h4_ladder<3>(v, j0, k0, op, tc);
                else h4_ladder<-1>(v, j0, k0, op, tc);
            } else if (GEN && (op.flags & OPF_REG1)) {
                if (op.ra == 0) h4_diag1<0>(v, acc, op);
                else if (op.ra == 1) h4_diag1<1>(v, acc, op);
                else if (op.ra == 2) h4_diag1<2>(v, acc, op);
                else h4_diag1<3>(v, acc, op);
            } else if (!GEN || (op.flags & OPF_PAT)) {
                if (op.flags & OPF_NEG) h4_pat<true, GEN>(v, acc, k0, G, op);
                else h4_pat<false, GEN>(v, acc, k0, G, op);
            } else {
                h4_diag(v, acc, k0, G, op);
            }
        }
        if constexpr (KIND == 4) {
            if constexpr (RL & 4) {
                static_for<0, 16>([&](auto EC) {
                    constexpr int e = decltype(EC)::value;
                    v[e] = cmul(v[e], acc);
                });
            }
        } else if constexpr (GEN) {
            // acc is exactly 1 unless a diagonal of the stage contributed
            if (S.acc) {
                static_for<0, 16>([&](auto EC) {
                    constexpr int e = decltype(EC)::value;
                    v[e] = cmul(v[e], acc);
                });
            }
        }
        if constexpr (MODE & 2) {
            if (KIND == 4 && tc.has_tf) {
                static_for<0, 16>([&](auto EC) {
                    constexpr int e = decltype(EC)::value;
                    v[e] = cmul(v[e], tc.tf);
                });
            } else if (tc.scaled) {
                static_for<0, 16>([&](auto EC) {
                    constexpr int e = decltype(EC)::value;
                    v[e].x *= tc.scale;
                    v[e].y *= tc.scale;
                });
            }
            if (pairg) {
                static_for<0, 8>([&](auto IC) {
                    constexpr int e = 2 * decltype(IC)::value;
                    *reinterpret_cast<P *>(gpsi + SV_GIDX(k0 | goff4<e>(G), tc.dim)) = pair_join(v[e], v[e + 1]);
                });
            } else {
                static_for<0, 16>([&](auto EC) {
                    constexpr int e = decltype(EC)::value;
                    gpsi[SV_GIDX(k0 | goff4<e>(G), tc.dim)] = v[e];
                });
            }
        } else {
            static_for<0, 16>([&](auto EC) {
                constexpr int e = decltype(EC)::value;
                tile[SV_LIDX(p0 ^ loffx4<e>(L), 1u << tc.m)] = v[e];
            });
        }
        if constexpr (ONE) break;
    }
}

template <typename R, int TPB, int KIND, bool ONE = false>
__device__ __forceinline__ void run_stages_h4(V2<R> *tile, V2<R> *__restrict__ gpsi, const TileCtx<R> &tc,
                                              const DevStage *__restrict__ stages, int sb, int se,
                                              const DevOp<R> *__restrict__ ops, int ovr_index, const DevOp<R> *ovr) {
    for (int s = sb; s < se; ++s) {
        const DevStage &S = stages[s];
        const bool first = s == sb, last = s == se - 1;
        if constexpr (KIND == 4) {
            // one straight-line body per (first, last, variant): the choice
            // is made here, outside the loop over register groups
            auto go = [&](auto MC) {
                constexpr int MODE = decltype(MC)::value;
                switch (S.rl) {
                case 0: h4_stage<R, TPB, MODE, 4, 0, ONE>(tile, gpsi, tc, S, ops, ovr_index, ovr); break;
                case 1: h4_stage<R, TPB, MODE, 4, 1, ONE>(tile, gpsi, tc, S, ops, ovr_index, ovr); break;
                case 2: h4_stage<R, TPB, MODE, 4, 2, ONE>(tile, gpsi, tc, S, ops, ovr_index, ovr); break;
                case 3: h4_stage<R, TPB, MODE, 4, 3, ONE>(tile, gpsi, tc, S, ops, ovr_index, ovr); break;
                case 4: h4_stage<R, TPB, MODE, 4, 4, ONE>(tile, gpsi, tc, S, ops, ovr_index, ovr); break;
                case 5: h4_stage<R, TPB, MODE, 4, 5, ONE>(tile, gpsi, tc, S, ops, ovr_index, ovr); break;
                case 6: h4_stage<R, TPB, MODE, 4, 6, ONE>(tile, gpsi, tc, S, ops, ovr_index, ovr); break;
                default: h4_stage<R, TPB, MODE, 4, 7, ONE>(tile, gpsi, tc, S, ops, ovr_index, ovr); break;
                }
            };
            if (first && last) go(std::integral_constant<int, 3>{});
            else if (first) go(std::integral_constant<int, 1>{});
            else if (last) go(std::integral_constant<int, 2>{});
            else go(std::integral_constant<int, 0>{});
        } else {
            if (first && last) h4_stage<R, TPB, 3, KIND, 0, ONE>(tile, gpsi, tc, S, ops, ovr_index, ovr);
            else if (first) h4_stage<R, TPB, 1, KIND, 0, ONE>(tile, gpsi, tc, S, ops, ovr_index, ovr);
            else if (last) h4_stage<R, TPB, 2, KIND, 0, ONE>(tile, gpsi, tc, S, ops, ovr_index, ovr);
            else h4_stage<R, TPB, 0, KIND, 0, ONE>(tile, gpsi, tc, S, ops, ovr_index, ovr);
        }
        __syncthreads();
    }
}

}  // namespace sv
