// Device-side helpers shared by the HIP translation units: complex
// arithmetic on (re, im) pairs, index expansion, the ops applied to a tile in
// LDS, FP64 block reductions and the Pauli pair contribution.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "sv_internal.h"

namespace sv {


// Index checks of the debug kernel build (SV_DEBUG_BOUNDS, see
// build_debug.py): an index outside its array sets a bit in this
// translation unit's flag word and is replaced by 0, so the access stays
// inside the array (nothing traps); the API call that ran the kernel
// returns SV_EDEVICE.  In the regular build the checks are the index itself.
#ifdef SV_DEBUG_BOUNDS
static __device__ unsigned int sv_debug_bound_flags;
template <typename T>
__device__ __forceinline__ T dbg_idx(T i, T n, unsigned int bit) {
    if (i >= n) {
        atomicOr(&sv_debug_bound_flags, bit);
        return (T)0;
    }
    return i;
}
#define SV_GIDX(i, n) ::sv::dbg_idx<uint64_t>((uint64_t)(i), (uint64_t)(n), 1u)
#define SV_LIDX(i, n) ::sv::dbg_idx<uint32_t>((uint32_t)(i), (uint32_t)(n), 2u)
namespace {
uint32_t take_bound_flags_here() {
    uint32_t v = 0, z = 0;
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(sv_debug_bound_flags), sizeof v) != hipSuccess ||
        hipMemcpyToSymbol(HIP_SYMBOL(sv_debug_bound_flags), &z, sizeof z) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return v;
}
[[maybe_unused]] const bool bound_flags_registered = register_bound_flag_reader(&take_bound_flags_here);
}  // namespace
#else
#define SV_GIDX(i, n) (i)
#define SV_LIDX(i, n) (i)
#endif

template <typename R> struct VecOf;
template <> struct VecOf<float> { using T = float2; };
template <> struct VecOf<double> { using T = double2; };
template <typename R> using V2 = typename VecOf<R>::T;

template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// u*a + w*b
template <typename V>
__device__ __forceinline__ V cmac2(V u, V a, V w, V b) {
    V r;
    r.x = u.x * a.x - u.y * a.y + w.x * b.x - w.y * b.y;
    r.y = u.x * a.y + u.y * a.x + w.x * b.y + w.y * b.x;
    return r;
}

template <typename R>
__device__ __forceinline__ V2<R> mat_at(const DevOp<R> &op, int k) {
    V2<R> v;
    v.x = op.m[2 * k];
    v.y = op.m[2 * k + 1];
    return v;
}

__device__ __forceinline__ void sincos_turns(float t, float *s, float *c) {
    sincospif(2.0f * t, s, c);
}
__device__ __forceinline__ void sincos_turns(double t, double *s, double *c) {
    sincospi(2.0 * t, s, c);
}

// Phase factor exp(2 pi i * turns * v), reduced modulo one turn in FP64.
template <typename R>
__device__ __forceinline__ V2<R> ladder_phase(double turns, uint64_t v) {
    double t = turns * (double)v;
    t -= floor(t);
    R s, c;
    sincos_turns((R)t, &s, &c);
    V2<R> r;
    r.x = c;
    r.y = s;
    return r;
}

// Insert zero bits at ascending positions, then OR the fixed ones.
struct Ins {
    int npos;
    int pos[6];
    uint64_t ones;
};
__device__ __forceinline__ uint64_t expand(uint64_t r, const Ins &in) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        if (i < in.npos) {
            const int p = in.pos[i];
            r = ((r >> p) << (p + 1)) | (r & ((1ull << p) - 1));
        }
    }
    return r | in.ones;
}

inline Ins make_ins(std::vector<int> pos, uint64_t ones) {
    std::sort(pos.begin(), pos.end());
    Ins in{};
    in.npos = (int)pos.size();
    for (int i = 0; i < in.npos; ++i) in.pos[i] = pos[i];
    in.ones = ones;
    return in;
}

inline std::vector<int> bits_of(uint64_t m) {
    std::vector<int> v;
    for (int b = 0; b < 64; ++b)
        if (m & (1ull << b)) v.push_back(b);
    return v;
}

// ---------------------------------------------------------------------------
// Stage engine.  A tile holds 2^m amplitudes; local index j maps to the
// global index gaddr(j) = base | hi_off[j >> l] | (j & lowm) (or j itself for
// a whole state in LDS).  A stage takes 8-amplitude groups that differ only
// in its three register bits, loads each group into registers, applies the
// stage's ops there and stores it back -- one LDS (or HBM) round trip for
// up to three mixing gates and any number of diagonal ones.
// ---------------------------------------------------------------------------

// Pointers into LDS, typed so that reads through them compile to LDS
// instructions (a generic pointer gives flat loads, which also wait on the
// vector-memory counter of every global access still in flight).
#define SV_LDS __attribute__((address_space(3)))

template <typename R>
__device__ __forceinline__ V2<R> lds_v2(const SV_LDS R *p, uint32_t i) {
    V2<R> v;
    v.x = p[2 * i];
    v.y = p[2 * i + 1];
    return v;
}

template <typename R>
struct TileCtx {
    int m, l;
    uint32_t lowm;
    bool ident;               // global index == local index
    uint64_t base;            // global bits fixed for this tile
    const SV_LDS uint64_t *hi_off;  // global offset of the high local bits
    const SV_LDS R *ltl;      // ladder phase tables in LDS (re, im pairs), or null:
    const V2<R> *ltabs;       // then read here (global memory or LDS)
    const SV_LDS R *Gs;       // per-tile ladder factors by op.tslot (re, im pairs), null = 1
    int lsa, lsb;             // ladder table split of the local bits
    bool zero;                // first global read synthesises |0...0>
    V2<R> tf;                 // kind-4 passes: the tile's diagonal factor times
    bool has_tf;              // the pass scale, applied by the last store instead
    const uint32_t *paux;     // stage layout-map tables (memory), or
    const SV_LDS uint32_t *pauxl;  // their LDS copy (non-null) holding entries from paux_off
    int paux_off;
    const float *mtab;        // MFMA stage matrices
    uint64_t dim;             // amplitudes per state (debug index checks)
    R scale;                  // pass scale (OPF_SCALED factors), applied
    bool scaled;              // by the store of the pass's last stage
};

// Ladder tables split the m local bits into a low part of a bits, a middle
// part of b bits and a high part of m - a - b bits.
__host__ __device__ inline void ladder_split(int m, int &a, int &b) {
    a = m < 5 ? m : 5;
    b = (m - a + 1) / 2;
}
__host__ __device__ inline int ladder_entries(int m) {
    int a, b;
    ladder_split(m, a, b);
    return (1 << a) + (1 << b) + (1 << (m - a - b));
}

// LDS layout of a tile pass (byte offsets, 16-byte aligned parts); the
// host sizes the launch with the same function.
constexpr int LTAB_LDS_CAP = 2048;  // ladder table entries kept in LDS
struct LdsLayout {
    uint32_t gs, tabs, paux, tile, end;
    bool tabs_in_lds;
};
// paux_lds: 32-bit layout-map entries copied to LDS (0 = read from memory)
__host__ __device__ inline LdsLayout tile_lds_layout(uint32_t nhi, int nlad, int ltab_count, uint32_t amp,
                                                     int paux_lds = 0) {
    auto al = [](uint32_t x) { return (x + 15u) & ~15u; };
    LdsLayout L;
    L.gs = al(8 * nhi);
    L.tabs = L.gs + al(amp * (uint32_t)nlad);
    L.tabs_in_lds = ltab_count <= LTAB_LDS_CAP;
    L.paux = L.tabs + (L.tabs_in_lds ? al(amp * (uint32_t)ltab_count) : 0u);
    L.tile = L.paux + al(4u * (uint32_t)paux_lds);
    L.end = L.tile;
    return L;
}

template <typename R>
__device__ __forceinline__ uint64_t gaddr(const TileCtx<R> &tc, uint32_t j) {
    return tc.ident ? (uint64_t)j : (tc.base | tc.hi_off[j >> tc.l] | (uint64_t)(j & tc.lowm));
}

__device__ __forceinline__ uint32_t ins0(uint32_t x, int p) {
    return ((x >> p) << (p + 1)) | (x & ((1u << p) - 1));
}

// Global bit mask of local bit r.
template <typename R>
__device__ __forceinline__ uint64_t gbit(const TileCtx<R> &tc, int r) {
    if (tc.ident || r < tc.l) return 1ull << r;
    return tc.hi_off[1u << (r - tc.l)];
}

// Offset of element e (bits of e -> register bits 0, 1, 2) given the three
// per-register offsets; e is a constant after unrolling.
template <typename T>
__device__ __forceinline__ T eoff(int e, T o0, T o1, T o2) {
    return ((e & 1) ? o0 : (T)0) | ((e & 2) ? o1 : (T)0) | ((e & 4) ? o2 : (T)0);
}

template <typename V>
__device__ __forceinline__ V vsel(bool c, V a, V b) {
    V r;
    r.x = c ? a.x : b.x;
    r.y = c ? a.y : b.y;
    return r;
}

// One group of 8 amplitudes held in registers as eight named values (no
// array: an array indexed from several dispatch branches can be merged by
// the optimiser into a dynamically indexed stack object).
// Deposit the bits of t into the set bits of mask (ascending): the global
// index bits of tile t.  Uniform, so it runs on the scalar unit.
__device__ __forceinline__ uint64_t deposit(uint64_t t, uint64_t mask) {
    uint64_t r = 0;
    while (mask) {
        const uint64_t low = mask & (~mask + 1);
        if (t & 1) r |= low;
        t >>= 1;
        mask ^= low;
    }
    return r;
}

template <typename R>
struct Grp {
    V2<R> e0, e1, e2, e3, e4, e5, e6, e7;
    uint32_t j0;   // local index of element 0
    uint64_t k0;   // global index of element 0
    bool live;
};

template <int E, typename R>
__device__ __forceinline__ V2<R> &el(Grp<R> &g) {
    if constexpr (E == 0) return g.e0;
    else if constexpr (E == 1) return g.e1;
    else if constexpr (E == 2) return g.e2;
    else if constexpr (E == 3) return g.e3;
    else if constexpr (E == 4) return g.e4;
    else if constexpr (E == 5) return g.e5;
    else if constexpr (E == 6) return g.e6;
    else return g.e7;
}

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <int E>
__device__ __forceinline__ uint32_t loff(const uint32_t (&L)[3]) {
    return ((E & 1) ? L[0] : 0u) | ((E & 2) ? L[1] : 0u) | ((E & 4) ? L[2] : 0u);
}
template <int E>
__device__ __forceinline__ uint64_t goff(const uint64_t (&G)[3]) {
    return ((E & 1) ? G[0] : 0ull) | ((E & 2) ? G[1] : 0ull) | ((E & 4) ? G[2] : 0ull);
}

// 2x2 on register bit I.  K: 0 complex matrix, 1 real matrix, 2 exchange
// (X / CNOT).  CTRL: some control bits are local (checked per pair against
// lc); otherwise the op applies to every pair.
template <int I, int K, bool CTRL, typename R>
__device__ __forceinline__ void rg_u1(Grp<R> &g, uint32_t lc, const uint32_t (&L)[3], V2<R> m0, V2<R> m1,
                                      V2<R> m2, V2<R> m3) {
    static_for<0, 8>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        if constexpr (!(e & (1 << I))) {
            constexpr int f = e | (1 << I);
            V2<R> &px = el<e>(g), &py = el<f>(g);
            const V2<R> x = px, y = py;
            V2<R> nx, ny;
            if constexpr (K == 2) {
                nx = y;
                ny = x;
            } else if constexpr (K == 1) {
                nx.x = m0.x * x.x + m1.x * y.x;
                nx.y = m0.x * x.y + m1.x * y.y;
                ny.x = m2.x * x.x + m3.x * y.x;
                ny.y = m2.x * x.y + m3.x * y.y;
            } else if constexpr (K == 3) {  // OPF_HAD (unscaled)
                nx.x = x.x + y.x;
                nx.y = x.y + y.y;
                ny.x = x.x - y.x;
                ny.y = x.y - y.y;
            } else if constexpr (K == 4) {  // OPF_ROTC, t in m0.x
                nx.x = x.x - m0.x * y.x;
                nx.y = x.y - m0.x * y.y;
                ny.x = m0.x * x.x + y.x;
                ny.y = m0.x * x.y + y.y;
            } else if constexpr (K == 5) {  // OPF_ROTS, u in m0.x
                nx.x = m0.x * x.x - y.x;
                nx.y = m0.x * x.y - y.y;
                ny.x = x.x + m0.x * y.x;
                ny.y = x.y + m0.x * y.y;
            } else {
                nx = cmac2(m0, x, m1, y);
                ny = cmac2(m2, x, m3, y);
            }
            if constexpr (CTRL) {
                const bool ok = ((g.j0 | loff<e>(L)) & lc) == lc;
                nx = vsel(ok, nx, x);
                ny = vsel(ok, ny, y);
            }
            px = nx;
            py = ny;
        }
    });
}

template <int K, bool CTRL, typename R>
__device__ __forceinline__ void rg_u1_at(Grp<R> &g, uint32_t lc, const uint32_t (&L)[3], const DevOp<R> &op) {
    // K 4 / 5 (scaled rotations) take their one coefficient from entry 5
    const V2<R> m0 = mat_at(op, (K == 4 || K == 5) ? 5 : 0), m1 = mat_at(op, 1), m2 = mat_at(op, 2),
                m3 = mat_at(op, 3);
    if (op.ra == 0) rg_u1<0, K, CTRL>(g, lc, L, m0, m1, m2, m3);
    else if (op.ra == 1) rg_u1<1, K, CTRL>(g, lc, L, m0, m1, m2, m3);
    else rg_u1<2, K, CTRL>(g, lc, L, m0, m1, m2, m3);
}

template <int K, typename R>
__device__ __forceinline__ void rg_u1_dispatch(Grp<R> &g, const uint32_t (&L)[3], const DevOp<R> &op) {
    const uint32_t lc = (uint32_t)op.lcmask;
    if (lc) rg_u1_at<K, true>(g, lc, L, op);
    else rg_u1_at<K, false>(g, lc, L, op);
}

// 4x4 on register bits A (high matrix bit) and B; plain exchange when !W.
template <int A, int B, bool W, bool CTRL, typename R>
__device__ __forceinline__ void rg_u2(Grp<R> &g, uint32_t lc, const uint32_t (&L)[3], const DevOp<R> &op) {
    static_for<0, 8>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        if constexpr (!(e & ((1 << A) | (1 << B)))) {
            constexpr int i01 = e | (1 << B), i10 = e | (1 << A), i11 = e | (1 << A) | (1 << B);
            V2<R> &p0 = el<e>(g), &p1 = el<i01>(g), &p2 = el<i10>(g), &p3 = el<i11>(g);
            const V2<R> x0 = p0, x1 = p1, x2 = p2, x3 = p3;
            V2<R> w0, w1, w2, w3;
            if constexpr (!W) {
                w0 = x0;
                w1 = x2;
                w2 = x1;
                w3 = x3;
            } else {
                auto row = [&](int r) {
                    V2<R> acc = cmul(mat_at(op, 4 * r), x0);
                    V2<R> t = cmul(mat_at(op, 4 * r + 1), x1);
                    acc.x += t.x;
                    acc.y += t.y;
                    t = cmul(mat_at(op, 4 * r + 2), x2);
                    acc.x += t.x;
                    acc.y += t.y;
                    t = cmul(mat_at(op, 4 * r + 3), x3);
                    acc.x += t.x;
                    acc.y += t.y;
                    return acc;
                };
                w0 = row(0);
                w1 = row(1);
                w2 = row(2);
                w3 = row(3);
            }
            if constexpr (CTRL) {
                const bool ok = ((g.j0 | loff<e>(L)) & lc) == lc;
                w0 = vsel(ok, w0, x0);
                w1 = vsel(ok, w1, x1);
                w2 = vsel(ok, w2, x2);
                w3 = vsel(ok, w3, x3);
            }
            p0 = w0;
            p1 = w1;
            p2 = w2;
            p3 = w3;
        }
    });
}

template <bool W, bool CTRL, typename R>
__device__ __forceinline__ void rg_u2_at(Grp<R> &g, uint32_t lc, const uint32_t (&L)[3], const DevOp<R> &op) {
    switch (op.ra * 3 + op.rb) {
    case 1: rg_u2<0, 1, W, CTRL>(g, lc, L, op); break;
    case 2: rg_u2<0, 2, W, CTRL>(g, lc, L, op); break;
    case 3: rg_u2<1, 0, W, CTRL>(g, lc, L, op); break;
    case 5: rg_u2<1, 2, W, CTRL>(g, lc, L, op); break;
    case 6: rg_u2<2, 0, W, CTRL>(g, lc, L, op); break;
    case 7: rg_u2<2, 1, W, CTRL>(g, lc, L, op); break;
    default: break;
    }
}

template <bool W, typename R>
__device__ __forceinline__ void rg_u2_dispatch(Grp<R> &g, uint32_t lc, const uint32_t (&L)[3], const DevOp<R> &op) {
    if (lc) rg_u2_at<W, true>(g, lc, L, op);
    else rg_u2_at<W, false>(g, lc, L, op);
}

// Diagonal factor d[2*bit_a + bit_b] (or d[bit_a]) where all cmask bits
// set.  PAT: only the all-ones pattern has a factor != 1 (CZ, CP, controlled
// phases): then a single condition and multiply (a sign flip when NEG).
template <bool PAT, bool NEG, typename R>
__device__ __forceinline__ void rg_diag(Grp<R> &g, const uint64_t (&G)[3], const DevOp<R> &op) {
    const int a = op.a, b = op.b;
    const uint64_t cm = op.cmask;
    const uint64_t all = cm | (1ull << a) | (b >= 0 ? (1ull << b) : 0ull);
    const V2<R> d0 = mat_at(op, 0), d1 = mat_at(op, 1), d2 = mat_at(op, 2), d3 = mat_at(op, 3);
    const V2<R> dl = b >= 0 ? d3 : d1;
    static_for<0, 8>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        V2<R> &v = el<e>(g);
        const uint64_t k = g.k0 | goff<e>(G);
        if constexpr (PAT) {
            const bool on = (k & all) == all;
            if constexpr (NEG) {
                v.x = on ? -v.x : v.x;
                v.y = on ? -v.y : v.y;
            } else {
                v = vsel(on, cmul(v, dl), v);
            }
        } else {
            const bool ba = (k >> a) & 1;
            V2<R> f;
            if (b >= 0) {
                const bool bb = (k >> b) & 1;
                f = vsel(ba, vsel(bb, d3, d2), vsel(bb, d1, d0));
            } else {
                f = vsel(ba, d1, d0);
            }
            const bool on = (k & cm) == cm;
            v = vsel(on, cmul(v, f), v);
        }
    });
}

// Group factor of a DIAG op none of whose bits is a register bit: with k0
// the global index of the group's element 0, the factor is d[2 bit_a +
// bit_b] (or d[bit_a]) where all cmask bits are set, else 1.
template <typename R>
__device__ __forceinline__ V2<R> rg_diag_grp(V2<R> acc, uint64_t k0, const DevOp<R> &op) {
    const uint64_t cm = op.cmask;
    if ((k0 & cm) != cm) return acc;
    const bool ba = (k0 >> op.a) & 1;
    if (op.flags & OPF_NEG) {
        const bool on = ba && (op.b < 0 || ((k0 >> op.b) & 1));
        if (on) {
            acc.x = -acc.x;
            acc.y = -acc.y;
        }
        return acc;
    }
    V2<R> f;
    if (op.b >= 0) {
        const bool bb = (k0 >> op.b) & 1;
        f = vsel(ba, vsel(bb, mat_at(op, 3), mat_at(op, 2)), vsel(bb, mat_at(op, 1), mat_at(op, 0)));
    } else {
        f = vsel(ba, mat_at(op, 1), mat_at(op, 0));
    }
    return cmul(acc, f);
}

// Multiply the elements whose register bit RB is set by r.
template <int RB, typename R>
__device__ __forceinline__ void rg_bit_scale(Grp<R> &g, const V2<R> r) {
    static_for<0, 8>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        if constexpr ((e >> RB) & 1) el<e>(g) = cmul(el<e>(g), r);
    });
}

// Ladder: where bit a is set, multiply by exp(2 pi i turns (k & lmask)).
// For k = base | off(j0) | off(e) (tile bits, the group's base index, its
// register bits) the phase factors into G (per tile), the product of the
// three tile-independent tables at j0's low / middle / high local bits, and
// a constant K_e of the op's stage (m entries 8 + e).  When a is register
// bit RA (template), exactly the elements with that bit set are touched;
// otherwise (RA < 0) bit a is the same for the whole group.
template <int RA, typename R>
__device__ __forceinline__ void rg_ladder(Grp<R> &g, const DevOp<R> &op, const TileCtx<R> &tc) {
    if (RA < 0 && !((g.k0 >> op.a) & 1)) return;
    const uint32_t j = g.j0;
    const uint32_t i0 = j & ((1u << tc.lsa) - 1), i1 = (1 << tc.lsa) + ((j >> tc.lsa) & ((1u << tc.lsb) - 1)),
                   i2 = (1 << tc.lsa) + (1 << tc.lsb) + (j >> (tc.lsa + tc.lsb));
    V2<R> p;
    if (tc.ltl) {
        const SV_LDS R *T = tc.ltl + 2 * op.tab;
        p = cmul(cmul(lds_v2<R>(T, i0), lds_v2<R>(T, i1)), lds_v2<R>(T, i2));
    } else {
        const V2<R> *T = tc.ltabs + op.tab;
        p = cmul(cmul(T[i0], T[i1]), T[i2]);
    }
    if (tc.Gs) p = cmul(p, lds_v2<R>(tc.Gs, op.tslot));
    static_for<0, 8>([&](auto EC) {
        constexpr int e = decltype(EC)::value;
        if constexpr (RA < 0 || (e & (1 << (RA < 0 ? 0 : RA)))) {
            V2<R> &v = el<e>(g);
            v = cmul(v, cmul(p, mat_at(op, 8 + e)));
        }
    });
}

// Apply the ops [op_begin, op_end) of stage S to one register group.
template <typename R>
__device__ __forceinline__ void stage_ops(Grp<R> &g, const TileCtx<R> &tc, const DevStage &S,
                                          const uint32_t (&L)[3], const uint64_t (&G)[3],
                                          const DevOp<R> *__restrict__ ops, int ovr_index, const DevOp<R> *ovr) {
    // diagonal factor common to the whole group (OPF_GRP / OPF_REG1 ops):
    // diagonal ops commute with each other and with every op on other bits,
    // so it is applied once after the stage's ops
    V2<R> acc;
    acc.x = (R)1;
    acc.y = (R)0;
    for (int o = S.op_begin; o < S.op_end; ++o) {
        const DevOp<R> &op = (o == ovr_index) ? *ovr : ops[o];
        const int kind = op.kind;
        if (kind == OP_U1 || kind == OP_XPERM) {
            if ((tc.base & op.gcmask) != op.gcmask) continue;
            if (kind == OP_XPERM) rg_u1_dispatch<2>(g, L, op);
            else if (op.flags & OPF_HAD) rg_u1_dispatch<3>(g, L, op);
            else if (op.flags & OPF_ROTC) rg_u1_dispatch<4>(g, L, op);
            else if (op.flags & OPF_ROTS) rg_u1_dispatch<5>(g, L, op);
            else if (op.flags & OPF_REAL) rg_u1_dispatch<1>(g, L, op);
            else rg_u1_dispatch<0>(g, L, op);
        } else if (kind == OP_U2 || kind == OP_SWAP) {
            if ((tc.base & op.gcmask) != op.gcmask) continue;
            if (kind == OP_U2) rg_u2_dispatch<true>(g, (uint32_t)op.lcmask, L, op);
            else rg_u2_dispatch<false>(g, (uint32_t)op.lcmask, L, op);
        } else if (kind == OP_DIAG) {
            if (op.flags & OPF_GRP) acc = rg_diag_grp<R>(acc, g.k0, op);
            else if (op.flags & OPF_REG1) {
                acc = cmul(acc, mat_at(op, 0));
                const V2<R> r = mat_at(op, 4);
                if (op.ra == 0) rg_bit_scale<0>(g, r);
                else if (op.ra == 1) rg_bit_scale<1>(g, r);
                else rg_bit_scale<2>(g, r);
            }
            else if (op.flags & OPF_NEG) rg_diag<true, true>(g, G, op);
            else if (op.flags & OPF_PAT) rg_diag<true, false>(g, G, op);
            else rg_diag<false, false>(g, G, op);
        } else if (kind == OP_LADDER) {
            if (op.ra == 0) rg_ladder<0>(g, op, tc);
            else if (op.ra == 1) rg_ladder<1>(g, op, tc);
            else if (op.ra == 2) rg_ladder<2>(g, op, tc);
            else rg_ladder<-1>(g, op, tc);
        }
    }
    if (S.acc) {
        static_for<0, 8>([&](auto EC) {
            constexpr int e = decltype(EC)::value;
            el<e>(g) = cmul(el<e>(g), acc);
        });
    }
}

// MODE bit 0: read the groups from global memory (else from the LDS tile);
// MODE bit 1: write them to global memory (else to the LDS tile).  Each
// thread handles groups threadIdx.x, +TPB, ... one at a time.  Groups are
// logical: element e of a group is local index j0 | loff(e).  With S.perm
// the LDS holds local index j at position Q(j) = tab_lo[j & 127] ^
// tab_hi[j >> 7] ^ q (the layout left by CNOT runs folded out of earlier
// stages); loads and stores of a group use the same positions, so no
// thread writes where another has yet to read.
typedef float mfma_f32x16 __attribute__((ext_vector_type(16)));

// MFMA stage (complex64 only): the stage's 16 x 16 complex matrix U on
// register bits r0 < r1 < r2 < r3 as the real 32 x 32 matrix
// W = [[Re U, -Im U], [Im U, Re U]] (row-major at tc.mtab + S.wtab).  A wave
// takes 32 groups g of 16 amplitudes at a time: Y = W X with column g of X =
// (Re x_g, Im x_g), as 16 v_mfma_f32_32x32x2f32 steps (K = 2 each).  Lane
// l = j + 32 h (group j, half h) supplies operand A = W[j][2s + h] and B =
// component 2s + h of group j, i.e. Re / Im of amplitudes h, h + 2, ...,
// h + 14, so it loads those 8 amplitudes; its 16 results are rows (r / 4) 8
// + 4 h + r % 4 of column j: Re (r < 8) and Im (r + 8) of amplitudes
// 4 h .. 4 h + 3 and 8 + 4 h .. 11 + 4 h, which it stores.  Every load of a
// wave feeds the MFMAs before any of its stores, and waves own disjoint
// groups, so the stage runs in place.
template <typename R, int TPB, int MODE>
__device__ __forceinline__ void mfma_stage(V2<R> *tile, V2<R> *__restrict__ gpsi, const TileCtx<R> &tc,
                                           const DevStage &S) {
    if constexpr (sizeof(R) == 4) {
        const int r[4] = {S.r0, S.r1, S.r2, S.r3};
        uint32_t L4[4];
        uint64_t G4[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            L4[i] = 1u << r[i];
            G4[i] = gbit(tc, r[i]);
        }
        const uint32_t lane = threadIdx.x & 63, j = lane & 31, h = lane >> 5;
        const uint32_t wave = threadIdx.x >> 6;
        float w[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) w[s] = tc.mtab[S.wtab + 32 * j + 2 * s + h];
        auto loff = [&](uint32_t a) {
            return ((a & 1) ? L4[0] : 0u) | ((a & 2) ? L4[1] : 0u) | ((a & 4) ? L4[2] : 0u) | ((a & 8) ? L4[3] : 0u);
        };
        auto goff = [&](uint32_t a) {
            return ((a & 1) ? G4[0] : 0ull) | ((a & 2) ? G4[1] : 0ull) | ((a & 4) ? G4[2] : 0ull) |
                   ((a & 8) ? G4[3] : 0ull);
        };
        const uint32_t ngroups = 1u << (tc.m - 4);
        for (uint32_t g0 = wave * 32; g0 < ngroups; g0 += (TPB / 64) * 32) {
            const uint32_t gi = g0 + j;
            const bool live = gi < ngroups;
            const uint32_t j0 = ins0(ins0(ins0(ins0(live ? gi : 0u, r[0]), r[1]), r[2]), r[3]);
            const uint64_t k0 = gaddr(tc, j0);
            float bre[8], bim[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const uint32_t a = 2 * s + h;
                V2<R> v;
                v.x = 0;
                v.y = 0;
                if (live) {
                    if constexpr (MODE & 1) {
                        if (tc.zero) v.x = (k0 | goff(a)) == 0 ? (R)1 : (R)0;
                        else v = gpsi[SV_GIDX(k0 | goff(a), tc.dim)];
                    } else {
                        v = tile[SV_LIDX(j0 | loff(a), 1u << tc.m)];
                    }
                }
                bre[s] = v.x;
                bim[s] = v.y;
            }
            mfma_f32x16 acc;
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
#pragma unroll
            for (int s = 0; s < 16; ++s)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(w[s], s < 8 ? bre[s] : bim[s - 8], acc, 0, 0, 0);
            if (live) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint32_t a = (q / 4) * 8 + 4 * h + (q % 4);
                    V2<R> v;
                    v.x = acc[q];
                    v.y = acc[q + 8];
                    if constexpr (MODE & 2) {
                        if (tc.scaled) {
                            v.x *= tc.scale;
                            v.y *= tc.scale;
                        }
                        gpsi[SV_GIDX(k0 | goff(a), tc.dim)] = v;
                    } else {
                        tile[SV_LIDX(j0 | loff(a), 1u << tc.m)] = v;
                    }
                }
            }
        }
    }
}

// 16-byte access to two adjacent complex64 amplitudes / one complex128.
template <typename R> struct Pair;
template <> struct Pair<float> { using T = float4; };
template <> struct Pair<double> { using T = double2; };
__device__ __forceinline__ float2 pair_lo(float4 v) { return make_float2(v.x, v.y); }
__device__ __forceinline__ float2 pair_hi(float4 v) { return make_float2(v.z, v.w); }
__device__ __forceinline__ float4 pair_join(float2 a, float2 b) { return make_float4(a.x, a.y, b.x, b.y); }
// (complex128 never takes the paired path; these only keep it compiling)
__device__ __forceinline__ double2 pair_lo(double2 v) { return v; }
__device__ __forceinline__ double2 pair_hi(double2 v) { return v; }
__device__ __forceinline__ double2 pair_join(double2 a, double2) { return a; }

// Issue the HBM loads of the 8 elements of a group at global index k0 (the
// offsets of its register bits: G) into d.
template <typename R>
__device__ __forceinline__ void load_group(V2<R> (&d)[8], const V2<R> *__restrict__ gpsi, uint64_t k0,
                                           const uint64_t (&G)[3], bool pairg, uint64_t dim) {
    (void)dim;  // read by the debug build's index checks
    if (pairg) {
        static_for<0, 4>([&](auto IC) {
            constexpr int e = 2 * decltype(IC)::value;
            const typename Pair<R>::T v =
                *reinterpret_cast<const typename Pair<R>::T *>(gpsi + SV_GIDX(k0 | goff<e>(G), dim));
            d[e] = pair_lo(v);
            d[e + 1] = pair_hi(v);
        });
    } else {
        static_for<0, 8>([&](auto EC) {
            constexpr int e = decltype(EC)::value;
            d[e] = gpsi[SV_GIDX(k0 | goff<e>(G), dim)];
        });
    }
}

// One 3-bit stage over the tile.  MODE bit 0: read the groups from global
// memory (else from the LDS tile); MODE bit 1: write them to global memory
// (else to the LDS tile).  Each thread handles groups threadIdx.x, +TPB, ...
// one at a time (holding two at once spills registers; so does holding the
// next tile's first groups while this one is processed, and at three waves
// per SIMD that measured 25-70% slower).
template <typename R, int TPB, int MODE>
__device__ __forceinline__ void run_stage(V2<R> *tile, V2<R> *__restrict__ gpsi, const TileCtx<R> &tc,
                                          const DevStage &S, const DevOp<R> *__restrict__ ops,
                                          int ovr_index, const DevOp<R> *ovr) {
    if constexpr (sizeof(R) == 4) {
        if (S.mfma) {
            mfma_stage<R, TPB, MODE>(tile, gpsi, tc, S);
            return;
        }
    }
    const uint32_t nitems = (1u << tc.m) >> 3;
    const int r0 = S.r0, r1 = S.r1, r2 = S.r2;
    const uint32_t L[3] = {1u << r0, 1u << r1, 1u << r2};
    const uint64_t G[3] = {gbit(tc, r0), gbit(tc, r1), gbit(tc, r2)};
    const bool perm = S.perm != 0;
    // complex64 with global bit 0 as register bit r0: elements 2i, 2i + 1
    // are adjacent in HBM and move as one 16-byte access (in LDS, 16-byte
    // accesses measured slower)
    const bool pairg = sizeof(R) == 4 && G[0] == 1ull;
    auto group = [&](uint32_t it) {
        Grp<R> g;
        g.live = true;
        g.j0 = ins0(ins0(ins0(it, r0), r1), r2);
        g.k0 = gaddr(tc, g.j0);
        return g;
    };
    // LDS position of element e: pos0 ^ pd[e] (layout map) or j0 | loff(e)
    auto lpos0 = [&](const Grp<R> &g) -> uint32_t {
        if (!perm) return g.j0;
        if (tc.pauxl) {
            const int t = S.perm_tab - tc.paux_off;
            return tc.pauxl[t + (g.j0 & 127u)] ^ tc.pauxl[t + 128 + (g.j0 >> 7)];
        }
        return tc.paux[S.perm_tab + (g.j0 & 127u)] ^ tc.paux[S.perm_tab + 128 + (g.j0 >> 7)];
    };
    auto lpos = [&](uint32_t pos0, auto EC) {
        constexpr int e = decltype(EC)::value;
        return perm ? pos0 ^ (uint32_t)S.pd[e] : pos0 | loff<e>(L);
    };
    // the stage's ops, the pass scale on a store to HBM, the store
    auto finish = [&](Grp<R> &g, uint32_t pos0) {
        stage_ops<R>(g, tc, S, L, G, ops, ovr_index, ovr);
        if constexpr (MODE & 2) {
            if (tc.scaled) {
                static_for<0, 8>([&](auto EC) {
                    constexpr int e = decltype(EC)::value;
                    el<e>(g).x *= tc.scale;
                    el<e>(g).y *= tc.scale;
                });
            }
            if (pairg) {
                static_for<0, 4>([&](auto IC) {
                    constexpr int e = 2 * decltype(IC)::value;
                    *reinterpret_cast<typename Pair<R>::T *>(gpsi + SV_GIDX(g.k0 | goff<e>(G), tc.dim)) =
                        pair_join(el<e>(g), el<e + 1>(g));
                });
            } else {
                static_for<0, 8>([&](auto EC) {
                    constexpr int e = decltype(EC)::value;
                    gpsi[SV_GIDX(g.k0 | goff<e>(G), tc.dim)] = el<e>(g);
                });
            }
        } else {
            static_for<0, 8>([&](auto EC) {
                constexpr int e = decltype(EC)::value;
                tile[SV_LIDX(lpos(pos0, EC), 1u << tc.m)] = el<e>(g);
            });
        }
    };
    for (uint32_t it = threadIdx.x; it < nitems; it += TPB) {
        Grp<R> g = group(it);
        const uint32_t pos0 = lpos0(g);
        if constexpr (MODE & 1) {
            if (tc.zero) {
                static_for<0, 8>([&](auto EC) {
                    constexpr int e = decltype(EC)::value;
                    V2<R> z;
                    z.x = (g.k0 | goff<e>(G)) == 0 ? (R)1 : (R)0;
                    z.y = 0;
                    el<e>(g) = z;
                });
            } else {
                V2<R> d[8];
                load_group<R>(d, gpsi, g.k0, G, pairg, tc.dim);
                static_for<0, 8>([&](auto EC) {
                    constexpr int e = decltype(EC)::value;
                    el<e>(g) = d[e];
                });
            }
        } else {
            static_for<0, 8>([&](auto EC) {
                constexpr int e = decltype(EC)::value;
                el<e>(g) = tile[SV_LIDX(lpos(pos0, EC), 1u << tc.m)];
            });
        }
        finish(g, pos0);
    }
}

// Run stages [sb, se) of a tile.  With gpsi: a one-stage pass streams
// HBM -> registers -> HBM; in a multi-stage pass the first stage reads its
// groups from HBM and writes them to the LDS tile, the middle stages work in
// LDS and the last one writes its groups to HBM.  Without gpsi everything
// stays in the LDS tile.  A barrier follows every stage.
template <typename R, int TPB>
__device__ __forceinline__ void run_stages(V2<R> *tile, V2<R> *__restrict__ gpsi, const TileCtx<R> &tc,
                                           const DevStage *__restrict__ stages, int sb, int se,
                                           const DevOp<R> *__restrict__ ops, int ovr_index = -1,
                                           const DevOp<R> *ovr = nullptr) {
    for (int s = sb; s < se; ++s) {
        const DevStage &S = stages[s];
        const bool first = gpsi && s == sb, last = gpsi && s == se - 1;
        if (first && last) run_stage<R, TPB, 3>(tile, gpsi, tc, S, ops, ovr_index, ovr);
        else if (first) run_stage<R, TPB, 1>(tile, gpsi, tc, S, ops, ovr_index, ovr);
        else if (last) run_stage<R, TPB, 2>(tile, gpsi, tc, S, ops, ovr_index, ovr);
        else run_stage<R, TPB, 0>(tile, gpsi, tc, S, ops, ovr_index, ovr);
        __syncthreads();
    }
}

// Host: exp(2 pi i turns (v & lmask)) in FP64, rounded once.
template <typename R>
inline V2<R> host_phase(double turns, uint64_t v) {
    double t = turns * (double)v;
    t -= std::floor(t);
    V2<R> z;
    z.x = (R)std::cos(2.0 * M_PI * t);
    z.y = (R)std::sin(2.0 * M_PI * t);
    return z;
}

// In-tile global offset of a pattern of local bits.
inline uint64_t local_offset(uint32_t pattern, const std::vector<int> &local_bits) {
    uint64_t o = 0;
    for (size_t i = 0; i < local_bits.size(); ++i)
        if ((pattern >> i) & 1) o |= 1ull << local_bits[i];
    return o;
}

// Host: the tile-independent ladder tables of op d for a tile whose local
// bit i is global bit local_bits[i]: the phase of the in-tile offset of each
// pattern of the low a, middle b and high m - a - b local bits.
template <typename R>
inline void append_ladder_tables(DevOp<R> &d, const Op &op, const std::vector<int> &local_bits,
                                 std::vector<V2<R>> &ltab) {
    const int m = (int)local_bits.size();
    int a, b;
    ladder_split(m, a, b);
    d.tab = (int)ltab.size();
    for (uint32_t v = 0; v < (1u << a); ++v) ltab.push_back(host_phase<R>(op.turns, local_offset(v, local_bits) & op.lmask));
    for (uint32_t v = 0; v < (1u << b); ++v)
        ltab.push_back(host_phase<R>(op.turns, local_offset(v << a, local_bits) & op.lmask));
    for (uint32_t v = 0; v < (1u << (m - a - b)); ++v)
        ltab.push_back(host_phase<R>(op.turns, local_offset(v << (a + b), local_bits) & op.lmask));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Per-term FP64 sums of Pauli expectations over a tile in LDS (one wave per
// chunk of terms sharing an X/Y support).
constexpr int ESUM_CHUNK = 8;

// +1.0 or -1.0 by the parity of popcount(j & z)
__device__ __forceinline__ double parity_sign(uint32_t j, uint32_t z) {
    return __hiloint2double((int)((__popc(j & z) << 31) | 0x3ff00000u), 0);
}

// One wave's sums over a tile in LDS for CNT terms of one group chunk.
// MODE 0: diagonal, items = amplitudes j, value |psi_j|^2.  MODE 1/2: items
// = pairs (j, j ^ xl) with j's top bit of xl clear, value Re/Im conj(b) a.
// acc[q] += (-1)^popcount(j & zl[q]) value (exact sign flips).
//
// Lane l takes items l, l + 64, l + 128, ... (block k = item / 64).  Item
// 64k + l sits at j = B(k) + Lj(l) with B(k) a multiple of 64 (of 128 when
// the pair bit is below 6) common to the wave and Lj(l) < 64 (< 128), so
// the sign splits into a wave-uniform factor (-1)^popcount(B & z), applied
// per block, and a lane factor (-1)^popcount(Lj & z), applied once at the
// end; the partner is (B ^ xhi) + Lp(l).  Blocks go four at a time from a
// multiple of four, where B(k + u) = B(k) + B(u) with disjoint bits, so the
// uniform signs of the four come from one parity of B(k) and four per-group
// constants.  Per pair that leaves two LDS reads, the value and one FMA per
// term.  Blocks are summed in the order of their items.
template <typename R, int CNT, int MODE>
__device__ __forceinline__ void esum(const V2<R> *__restrict__ tile, uint32_t T, uint32_t xl,
                                     const uint32_t (&zl)[ESUM_CHUNK], double (&acc)[ESUM_CHUNK], uint32_t lane) {
    constexpr int U = 4;
    auto value = [&](const V2<R> &a, const V2<R> &b) {
        const double ax = a.x, ay = a.y;
        if (MODE == 0) return ax * ax + ay * ay;
        const double bx = b.x, by = b.y;
        return MODE == 1 ? bx * ax + by * ay : bx * ay - by * ax;
    };
    const uint32_t items = MODE == 0 ? T : T / 2;
    const int hb = MODE == 0 ? 0 : 31 - __clz(xl);  // the pair bit (top bit of xl)
    // lane parts of j and of its partner; the partner's block part is B ^ xhi
    uint32_t Lj = lane, Lp = 0, xhi = 0;
    if (MODE != 0) {
        if (hb <= 5) {
            Lj = ins0(lane, hb);
            Lp = Lj ^ xl;
        } else {
            Lp = lane ^ (xl & 63u);
            xhi = xl & ~63u;
        }
    }
    // B(k) = 64k (MODE 0), 128k (pair bit below 6), else 64k + (k >> (hb - 6)) 2^hb
    const bool wide = MODE != 0 && hb >= 6;
    const uint32_t sh1 = MODE != 0 && hb <= 5 ? 7u : 6u, s2 = wide ? (uint32_t)hb - 6u : 0u,
                   h2 = wide ? (uint32_t)hb : 0u, m2 = wide ? ~0u : 0u;
    auto base = [&](uint32_t k) -> uint32_t { return (k << sh1) + (((k >> s2) << h2) & m2); };
    // high words of +-1.0: sign bit = parity of (B(u) & z), u = 0..3
    uint32_t shi[CNT][U];
#pragma unroll
    for (int q = 0; q < CNT; ++q)
#pragma unroll
        for (int u = 0; u < U; ++u)
            shi[q][u] = ((uint32_t)__popc(base((uint32_t)u) & zl[q]) << 31) | 0x3ff00000u;
    double part[CNT];
#pragma unroll
    for (int q = 0; q < CNT; ++q) part[q] = 0.0;
    if (items >= 64 || lane < items) {
        const uint32_t nblk = items >= 64 ? items / 64 : 1;
        uint32_t k = 0;
        for (; k + U <= nblk; k += U) {
            const uint32_t Bk = base(k);
            V2<R> a[U], b[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t B = Bk + base((uint32_t)u);
                a[u] = tile[B + Lj];
                if (MODE != 0) b[u] = tile[(B ^ xhi) + Lp];
            }
            uint32_t flip[CNT];
#pragma unroll
            for (int q = 0; q < CNT; ++q) flip[q] = (uint32_t)__popc(Bk & zl[q]) << 31;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double v = value(a[u], MODE != 0 ? b[u] : a[u]);
#pragma unroll
                for (int q = 0; q < CNT; ++q)
                    part[q] = fma(__hiloint2double((int)(shi[q][u] ^ flip[q]), 0), v, part[q]);
            }
        }
        for (; k < nblk; ++k) {
            const uint32_t Bk = base(k);
            const V2<R> a = tile[Bk + Lj];
            const double v = value(a, MODE != 0 ? tile[(Bk ^ xhi) + Lp] : a);
#pragma unroll
            for (int q = 0; q < CNT; ++q) part[q] = fma(parity_sign(Bk, zl[q]), v, part[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < CNT; ++q) acc[q] = fma(parity_sign(Lj, zl[q]), part[q], acc[q]);
}

// esum for a chunk of cnt (1..ESUM_CHUNK) terms over a tile of T amplitudes:
// mode 0 diagonal, 1 / 2 pairs on X/Y support xl using Re / Im.
template <typename R>
__device__ __forceinline__ void esum_dispatch(const V2<R> *__restrict__ tile, uint32_t T, uint32_t xl, int mode,
                                              int cnt, const uint32_t (&zl)[ESUM_CHUNK],
                                              double (&acc)[ESUM_CHUNK], uint32_t lane) {
    switch (cnt * 3 + mode) {
#define SV_ESUM_CASE(C)                                                                            \
    case C * 3 + 0: esum<R, C, 0>(tile, T, 0u, zl, acc, lane); break;                              \
    case C * 3 + 1: esum<R, C, 1>(tile, T, xl, zl, acc, lane); break;                              \
    case C * 3 + 2: esum<R, C, 2>(tile, T, xl, zl, acc, lane); break;
        SV_ESUM_CASE(1)
        SV_ESUM_CASE(2)
        SV_ESUM_CASE(3)
        SV_ESUM_CASE(4)
        SV_ESUM_CASE(5)
        SV_ESUM_CASE(6)
        SV_ESUM_CASE(7)
        SV_ESUM_CASE(8)
#undef SV_ESUM_CASE
    default: break;
    }
}


// Block-wide sum in a fixed order; result valid in thread 0.
template <int TPB>
__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < TPB / 64; ++i) s += red[i];
    return s;
}

// Contribution of the pair (k, k^x) with amplitudes a = psi[k], b = psi[k^x]
// to <P> for a term (x, z, ny): s_k Re(i^ny conj(b) a) + s_k' Re(i^ny conj(a) b).
__device__ __forceinline__ double pair_contrib(double pre, double pim, uint64_t k, uint64_t k2,
                                               uint64_t z, int ny) {
    double v1, v2;  // Re(i^ny p), Re(i^ny conj p)
    switch (ny) {
    case 0: v1 = pre; v2 = pre; break;
    case 1: v1 = -pim; v2 = pim; break;
    case 2: v1 = -pre; v2 = -pre; break;
    default: v1 = pim; v2 = -pim; break;
    }
    const double s1 = (__popcll(k & z) & 1) ? -v1 : v1;
    const double s2 = (__popcll(k2 & z) & 1) ? -v2 : v2;
    return s1 + s2;
}


// ---------------------------------------------------------------------------
// Host helpers shared by the launchers
// ---------------------------------------------------------------------------

// A plan in device form: host arrays, then their device copies.
template <typename R>
struct DevPlanHost {
    std::vector<DevOp<R>> dops;
    std::vector<int> gate;        // source gate index of each op (-1 = merged)
    std::vector<DevPass> dpass;
    std::vector<DevStage> dstages;
    std::vector<uint64_t> aux;
    std::vector<uint32_t> aux32;
    std::vector<V2<R>> ltab;
    std::vector<float> mtab;      // 32x32 real matrices of MFMA stages
};
template <typename R>
struct DevPlanDev {
    const DevOp<R> *ops;
    const DevPass *pass;
    const DevStage *stages;
    const uint64_t *aux;
    const uint32_t *aux32;
    const V2<R> *ltab;
    const float *mtab;
};
// Tile-pass launch with TPB threads per workgroup (tile_t<TPB>.hip).
template <typename R, int TPB>
void launch_tile_tpb(Ctx *ctx, size_t lds, unsigned grid, V2<R> *slab, uint64_t dim, int nc, const int *ovr_idx,
                     const DevOp<R> *ovr, const DevPlanDev<R> &d, int pidx, uint64_t tiles, bool from_zero, int h4,
                     bool one);

// Workgroup size of a tile pass of m local bits: two 8-amplitude groups per
// thread per stage (measured fastest at every width: more independent
// workgroups per CU overlap one workgroup's HBM waits with another's stages).
inline int tile_tpb(int m) { return std::max(64, std::min(512, 1 << std::max(0, m - 4))); }

template <typename R>
inline void launch_tile(Ctx *ctx, int tpb, size_t lds, unsigned grid, V2<R> *slab, uint64_t dim, int nc,
                        const int *ovr_idx, const DevOp<R> *ovr, const DevPlanDev<R> &d, int pidx, uint64_t tiles,
                        bool from_zero, int h4, int m) {
    const bool one = (1u << m) / 16 <= (unsigned)tpb;
    switch (tpb) {
    case 64: launch_tile_tpb<R, 64>(ctx, lds, grid, slab, dim, nc, ovr_idx, ovr, d, pidx, tiles, from_zero, h4, one); break;
    case 128: launch_tile_tpb<R, 128>(ctx, lds, grid, slab, dim, nc, ovr_idx, ovr, d, pidx, tiles, from_zero, h4, one); break;
    case 256: launch_tile_tpb<R, 256>(ctx, lds, grid, slab, dim, nc, ovr_idx, ovr, d, pidx, tiles, from_zero, h4, one); break;
    default: launch_tile_tpb<R, 512>(ctx, lds, grid, slab, dim, nc, ovr_idx, ovr, d, pidx, tiles, from_zero, h4, one); break;
    }
}

template <typename R> DevPlanHost<R> build_dev_plan(const Plan &plan);
template <typename R> DevPlanDev<R> upload_dev_plan(Ctx *ctx, const DevPlanHost<R> &h, const std::string &slot);
// Run every pass of a plan over a slab of nc states.  nc_pass (host, one
// count per pass, non-decreasing, last = nc): only states [0, nc_pass[i])
// take part in pass i; states [nc_pass[i-1], nc_pass[i]) first receive a
// copy of state 0 (whose ops up to pass i they share).
template <typename R>
void launch_plan(Ctx *ctx, const Plan &plan, const DevPlanHost<R> &h, const DevPlanDev<R> &d, V2<R> *slab,
                 uint64_t dim, int nc, const int *ovr_idx, const DevOp<R> *ovr, bool from_zero,
                 const int *nc_pass = nullptr);

void upload(Ctx *ctx, void *dst, const void *src, size_t bytes);
unsigned grid_for(uint64_t items, int tpb, int cu);
void set_lds_limit(const void *fn, size_t bytes);
struct DevTerms;
void expectation_dev(Ctx *ctx, const void *psi, int n, int dtype, const DevTerms &dt, double *d_energy,
                     double *d_vals);

template <typename R>
inline DevOp<R> to_dev(const Op &op) {
    DevOp<R> d;
    std::memset(&d, 0, sizeof d);
    d.kind = op.kind;
    d.a = op.a;
    d.b = op.b;
    d.la = -1;
    d.lb = -1;
    d.cmask = op.cmask;
    d.lmask = op.lmask;
    d.turns = op.turns;
    d.tab = -1;
    for (int k = 0; k < 16; ++k) {
        d.m[2 * k] = (R)op.m[k].real();
        d.m[2 * k + 1] = (R)op.m[k].imag();
    }
    if (op.kind == OP_U1 && op.m[0].imag() == 0.0 && op.m[1].imag() == 0.0 && op.m[2].imag() == 0.0 &&
        op.m[3].imag() == 0.0) {
        d.flags |= OPF_REAL;
        const double m0 = op.m[0].real(), m1 = op.m[1].real(), m2 = op.m[2].real(), m3 = op.m[3].real();
        // value-dependent classes (Hadamard, all-ones pattern) are kept from
        // parameterised ops: a shifted copy of such an op replaces it on the
        // device without a new plan, and the pass kernel chosen from the
        // base op's class must still be right for the copy
        if (!op.param && op.cmask == 0 && m0 != 0.0 && m0 == m1 && m0 == m2 && m3 == -m0) {
            d.flags |= OPF_HAD;
            d.sfac = m0;
        } else if (op.cmask == 0 && m0 == m3 && m1 == -m2 && (m0 != 0.0 || m2 != 0.0)) {
            if (std::fabs(m0) >= std::fabs(m2)) {
                d.flags |= OPF_ROTC;
                d.sfac = m0;
                d.m[10] = (R)(m2 / m0);
            } else {
                d.flags |= OPF_ROTS;
                d.sfac = m2;
                d.m[10] = (R)(m0 / m2);
            }
        }
    }
    if (op.kind == OP_DIAG && op.b < 0 && op.m[0] != cd(0.0)) {
        const cd r = op.m[1] / op.m[0];
        d.m[8] = (R)r.real();
        d.m[9] = (R)r.imag();
    }
    // a parameterised gate whose shifted copies can leave the real-matrix
    // class (every one but RY and CRY)
    if (op.param && !op.real_family) d.flags |= OPF_PARAMC;
    if (op.kind == OP_DIAG && !op.param) {
        const int last = op.b >= 0 ? 3 : 1;
        bool pat = true;
        for (int k = 0; k < last; ++k) pat &= op.m[k] == cd(1.0);
        if (pat) d.flags |= OPF_PAT;
        if (pat && op.m[last] == cd(-1.0)) d.flags |= OPF_NEG;
    }
    return d;
}

// In-tile global offset of every combination of the local bits >= lt.
inline std::vector<uint64_t> hi_offsets(const std::vector<int> &local_bits, int lt) {
    const int m = (int)local_bits.size();
    std::vector<uint64_t> out(1u << (m - lt));
    for (uint32_t h = 0; h < out.size(); ++h) {
        uint64_t o = 0;
        for (int i = 0; i < m - lt; ++i)
            if ((h >> i) & 1) o |= 1ull << local_bits[lt + i];
        out[h] = o;
    }
    return out;
}

// Fill the tile-local fields of an op for a pass with local bits `lb`.
template <typename R>
inline void localise(DevOp<R> &d, const std::vector<int> &local_bits) {
    int pos[64];
    for (int i = 0; i < 64; ++i) pos[i] = -1;
    for (size_t i = 0; i < local_bits.size(); ++i) pos[local_bits[i]] = (int)i;
    if (d.kind == OP_DIAG || d.kind == OP_LADDER) d.la = d.a >= 0 ? pos[d.a] : -1;
    if (d.kind == OP_DIAG) {
        d.lb = d.b >= 0 ? pos[d.b] : -1;
        d.lcmask = 0;
        d.gcmask = 0;
        for (int b : bits_of(d.cmask)) {
            if (pos[b] >= 0) d.lcmask |= 1ull << pos[b];
            else d.gcmask |= 1ull << b;
        }
    }
    if (d.kind == OP_U1 || d.kind == OP_XPERM || d.kind == OP_U2 || d.kind == OP_SWAP) {
        d.la = pos[d.a];
        if (d.la < 0) fail(SV_EDEVICE, "internal: target bit outside tile");
        if (d.kind == OP_U2 || d.kind == OP_SWAP) {
            d.lb = pos[d.b];
            if (d.lb < 0) fail(SV_EDEVICE, "internal: target bit outside tile");
        }
        d.lcmask = 0;
        d.gcmask = 0;
        for (int b : bits_of(d.cmask)) {
            if (pos[b] >= 0) d.lcmask |= 1ull << pos[b];
            else d.gcmask |= 1ull << b;
        }
    }
}

// Device term layout: terms in group order plus the norm pseudo-term
// (x = z = 0, idx = T) appended to the x = 0 group (created if absent).

// Group the localised ops [ob, oe) of a tile (m local bits, m >= 3) into
// stages: a mixing op joins the current stage while the union of targets
// stays within three bits; diagonal ops always join.  A run of
// single-control CNOTs and
// X gates on local bits that would open a new stage after an earlier
// stage of the tile is not run at all: it only changes the LDS layout map
// Q of the following stages (Q <- Q o P for each op's index map P, an
// involution), whose tables go to aux32.  If the tile ends on such a run a
// stage without ops realises the layout (it must then write to global
// memory: folding needs final_to_global).  Fills ra / rb / tslot of every
// op that stays in a stage.
// Four-bit stages for a pass of uncontrolled one-qubit gates, ladders and
// diagonals only (h4_kind): a stage takes ops in order until a fifth
// distinct gate bit would be needed; its register bits are those gate
// bits, padded with the highest other local bits.  A ladder gets
// its register slot (or -1) and, in complex slots 0..15 of m, the phase of
// each element's register-bit offset.
// 0: not eligible; 1: general four-bit stages; 2: Hadamards, ladders and
// all-ones-pattern diagonals only (the QFT's passes, a smaller kernel);
// 3: Hadamards, real rotations and diagonals only.  A parameterised op
// whose shifted copies may fall outside a class (OPF_PARAMC) keeps its pass
// general.
template <typename R>
inline int h4_kind(const std::vector<DevOp<R>> &ops, int ob, int oe, int m) {
    if (m < 6 || m > 16 || oe <= ob) return 0;
    bool qft = true, rot = true;
    for (int o = ob; o < oe; ++o) {
        const DevOp<R> &d = ops[o];
        const bool mix = (d.kind == OP_U1 || d.kind == OP_XPERM) && d.cmask == 0;
        if (!mix && d.kind != OP_DIAG && d.kind != OP_LADDER) return 0;
        if ((d.kind == OP_U1 && !(d.flags & OPF_HAD)) || d.kind == OP_XPERM ||
            (d.kind == OP_DIAG && !(d.flags & OPF_PAT)))
            qft = false;
        if (d.kind == OP_XPERM || d.kind == OP_LADDER ||
            (d.kind == OP_U1 && (!(d.flags & (OPF_HAD | OPF_ROTC | OPF_ROTS)) || (d.flags & OPF_PARAMC))))
            rot = false;
    }
    return qft ? 2 : rot ? 3 : 1;
}

// Lane order of a four-bit stage.  The h4 engines keep the LDS tile
// XOR-swizzled: element j sits at j ^ (j >> 4 & 15) ^ (j >> 8 & 15) ^
// (j >> 12 & 15) (a bijection that folds the higher 4-bit digits onto the
// lowest), so local bit b lands on bank slot b mod 4.  A 16-byte access of
// 16 consecutive lanes then meets 16 distinct 16-byte bank slots when the
// four lowest bits of the group index take local bits of residues 0, 1, 2
// and 3 mod 4; the stage gives them the lowest non-register bits of those
// residues (where one exists), and the other bits follow in increasing
// order.  Packed 4 bits per index bit, from index bit 0.
inline uint64_t h4_lane_order(const DevStage &S, int m) {
    const int reg[4] = {S.r0, S.r1, S.r2, S.r3};
    std::vector<int> free_bits, order;
    for (int b = 0; b < m; ++b)
        if (std::find(reg, reg + 4, b) == reg + 4) free_bits.push_back(b);
    std::vector<char> used(free_bits.size(), 0);
    for (int res = 0; res < 4 && res < (int)free_bits.size(); ++res) {
        int pick = -1;
        for (size_t i = 0; i < free_bits.size() && pick < 0; ++i)
            if (!used[i] && free_bits[i] % 4 == res) pick = (int)i;
        for (size_t i = 0; i < free_bits.size() && pick < 0; ++i)
            if (!used[i]) pick = (int)i;
        used[pick] = 1;
        order.push_back(free_bits[pick]);
    }
    for (size_t i = 0; i < free_bits.size(); ++i)
        if (!used[i]) order.push_back(free_bits[i]);
    if (order.size() > 12) fail(SV_EDEVICE, "internal: four-bit stage wider than 16 bits");
    uint64_t lp = 0;
    for (size_t k = 0; k < order.size(); ++k) lp |= (uint64_t)order[k] << (4 * k);
    return lp;
}

template <typename R>
inline void build_stages_h4(std::vector<DevOp<R>> &ops, int ob, int oe, const std::vector<int> &local_bits,
                            std::vector<DevStage> &out, bool layers = false) {
    const int m = (int)local_bits.size();
    int start = ob;
    std::vector<int> regs;
    // layers: a stage also closes before a second mixing op on one bit, and
    // before a mixing op on a bit of a diagonal that follows a mixing op of
    // the stage on another of its bits (rotation-layer stages rotate each
    // register bit once, with every diagonal before or after the rotations
    // on its bits)
    uint64_t rotated = 0, post = 0;
    auto close = [&](int end) {
        if (end <= start) return;
        for (int b = m - 1; b >= 0 && (int)regs.size() < 4; --b)
            if (std::find(regs.begin(), regs.end(), b) == regs.end()) regs.push_back(b);
        std::sort(regs.begin(), regs.end());
        DevStage S;
        std::memset(&S, 0, sizeof S);
        S.r0 = regs[0];
        S.r1 = regs[1];
        S.r2 = regs[2];
        S.r3 = regs[3];
        S.op_begin = start;
        S.op_end = end;
        auto slot = [&](int lb) {
            const auto it = std::find(regs.begin(), regs.end(), lb);
            return it == regs.end() ? -1 : (int)(it - regs.begin());
        };
        uint64_t greg = 0;  // global positions of the register bits
        for (int r : regs) greg |= 1ull << local_bits[r];
        S.acc = 0;
        for (int o = start; o < end; ++o) {
            DevOp<R> &d = ops[o];
            d.flags &= ~OPF_PLACEMENT;
            if (d.kind == OP_U1 || d.kind == OP_XPERM) {
                d.ra = slot(d.la);
                if (d.ra < 0) fail(SV_EDEVICE, "internal: gate bit outside its stage");
            } else if (d.kind == OP_DIAG) {
                // which ops feed the group factor (acc) decides whether the
                // stage applies it: REG1 ops with d0 != 1, and diagonals
                // that involve no register bit
                const uint64_t all = d.cmask | (1ull << d.a) | (d.b >= 0 ? (1ull << d.b) : 0ull);
                if (d.b < 0 && d.cmask == 0 && d.la >= 0 && slot(d.la) >= 0) {
                    d.ra = slot(d.la);
                    d.flags |= OPF_REG1;
                    if (!(d.flags & OPF_PAT)) S.acc = 1;
                } else if ((all & greg) == 0) {
                    S.acc = 1;
                }
            } else if (d.kind == OP_LADDER) {
                d.ra = d.la >= 0 ? slot(d.la) : -1;
                for (int e = 0; e < 16; ++e) {
                    uint32_t lo = 0;
                    for (int i = 0; i < 4; ++i)
                        if ((e >> i) & 1) lo |= 1u << regs[i];
                    const V2<R> k = host_phase<R>(d.turns, local_offset(lo, local_bits) & d.lmask);
                    d.m[2 * e] = k.x;
                    d.m[2 * e + 1] = k.y;
                }
            }
        }
        out.push_back(S);
        start = end;
        regs.clear();
    };
    for (int o = ob; o < oe; ++o) {
        const DevOp<R> &d = ops[o];
        if (layers && d.kind == OP_DIAG) {
            const uint64_t bits = d.cmask | (1ull << d.a) | (d.b >= 0 ? (1ull << d.b) : 0ull);
            if (bits & rotated) post |= bits;
            continue;
        }
        if (d.kind != OP_U1 && d.kind != OP_XPERM) continue;
        const bool have = std::find(regs.begin(), regs.end(), d.la) != regs.end();
        if (layers && ((rotated | post) >> d.a) & 1) {
            close(o);
            rotated = post = 0;
        } else if (have) {
            continue;
        } else if ((int)regs.size() == 4) {
            close(o);
            rotated = post = 0;
        }
        if (std::find(regs.begin(), regs.end(), d.la) == regs.end()) regs.push_back(d.la);
        rotated |= 1ull << d.a;
    }
    close(oe);
}

// Diagonal tables for the four-bit stages of a pass of rotations and
// diagonals (h4 kind 3).  In each stage, every fixed diagonal whose bits are
// all register bits, and every fixed -1-on-the-all-ones-pattern diagonal
// (CZ) on one register bit and one bit outside the registers, leaves the op
// list and is gathered into an OP_DIAG16 op: the product of the factors on
// the 16 register-bit combinations (FP64, rounded once) and, per register
// slot, the outside bits whose parity negates the elements with that slot
// set.  A gathered diagonal may move anywhere between the mixing ops on its
// register bits that precede and follow it (diagonals commute with each
// other and with mixing ops on other bits); the tables go to the fewest
// points between the stage's mixing ops that give every diagonal a point
// inside its range (interval stabbing: take the ranges by right end, a new
// point at the right end of the first one not yet covered).
// pops: the FP64 ops of the pass (pops[i] is ops[ob + i]).  The pass's ops
// and gate list are rebuilt; stage op ranges and oe follow.
template <typename R>
inline void gather_stage_diagonals(std::vector<DevOp<R>> &ops, std::vector<int> &gate, const std::vector<Op> &pops,
                                   int ob, int &oe, std::vector<DevStage> &stages, int sb,
                                   const std::vector<int> &local_bits) {
    std::vector<DevOp<R>> out(ops.begin(), ops.begin() + ob);
    std::vector<int> gout(gate.begin(), gate.begin() + ob);
    for (int si = sb; si < (int)stages.size(); ++si) {
        DevStage &S = stages[si];
        const int regs[4] = {S.r0, S.r1, S.r2, S.r3};
        uint64_t greg[4];
        for (int i = 0; i < 4; ++i) greg[i] = 1ull << local_bits[regs[i]];
        const uint64_t gall = greg[0] | greg[1] | greg[2] | greg[3];
        struct Gathered {
            int o;          // op index
            uint32_t slots; // register slots it depends on
            int r;          // sign coupling: its slot (else -1)
            uint64_t outb;  // sign coupling: the outside bit
            int lo, hi, at; // allowed gaps and the chosen one
        };
        std::vector<Gathered> gd;
        std::vector<int> mix;           // op indices of the mixing ops, in order
        std::vector<int> gap_of;        // per op of the stage: mixing ops before it
        for (int o = S.op_begin; o < S.op_end; ++o) {
            const DevOp<R> &d = ops[o];
            const Op &src = pops[o - ob];
            gap_of.push_back((int)mix.size());
            if (d.kind == OP_U1 || d.kind == OP_XPERM) {
                mix.push_back(o);
                continue;
            }
            if (d.kind != OP_DIAG || src.param) continue;
            const uint64_t all = src.cmask | (1ull << src.a) | (src.b >= 0 ? (1ull << src.b) : 0ull);
            const uint64_t outb = all & ~gall;
            Gathered g{o, 0u, -1, 0ull, 0, 0, 0};
            for (int i = 0; i < 4; ++i)
                if (all & greg[i]) g.slots |= 1u << i;
            if (outb != 0) {
                const bool pat_neg = (d.flags & OPF_PAT) && (d.flags & OPF_NEG);
                if (!pat_neg || __builtin_popcount(g.slots) != 1 || __builtin_popcountll(outb) != 1) continue;
                g.r = __builtin_ctz(g.slots);
                g.outb = outb;
            }
            gd.push_back(g);
        }
        const int K = (int)mix.size();
        for (Gathered &g : gd) {
            const int j = gap_of[g.o - S.op_begin];
            g.lo = 0;
            for (int k = j - 1; k >= 0; --k)
                if ((g.slots >> ops[mix[k]].ra) & 1) { g.lo = k + 1; break; }
            g.hi = K;
            for (int k = j; k < K; ++k)
                if ((g.slots >> ops[mix[k]].ra) & 1) { g.hi = k; break; }
        }
        std::vector<int> order(gd.size());
        for (size_t i = 0; i < gd.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return gd[a].hi < gd[b].hi; });
        int point = -1;
        for (int i : order) {
            if (point < gd[i].lo) point = gd[i].hi;
            gd[i].at = point;
        }
        std::vector<char> gathered(S.op_end - S.op_begin, 0);
        for (const Gathered &g : gd) gathered[g.o - S.op_begin] = 1;
        // emit: per gap, its table, the ops left in place there, its mixing op
        const int nb = (int)out.size();
        auto emit_table = [&](int gap) {
            cd T[16];
            for (int e = 0; e < 16; ++e) T[e] = 1.0;
            uint64_t M[4] = {0, 0, 0, 0};
            bool any = false;
            for (const Gathered &g : gd) {
                if (g.at != gap) continue;
                any = true;
                if (g.r >= 0) {
                    M[g.r] ^= g.outb;
                    continue;
                }
                const Op &src = pops[g.o - ob];
                for (int e = 0; e < 16; ++e) {
                    uint64_t k = 0;
                    for (int i = 0; i < 4; ++i)
                        if ((e >> i) & 1) k |= greg[i];
                    if ((k & src.cmask) != src.cmask) continue;
                    const int ba = (k >> src.a) & 1;
                    T[e] *= src.b >= 0 ? src.m[2 * ba + (int)((k >> src.b) & 1)] : src.m[ba];
                }
            }
            if (!any) return;
            DevOp<R> t;
            std::memset(&t, 0, sizeof t);
            t.kind = OP_DIAG16;
            t.a = t.b = t.la = t.lb = t.ra = t.rb = -1;
            t.tab = -1;
            for (int e = 0; e < 16; ++e) {
                t.m[2 * e] = (R)T[e].real();
                t.m[2 * e + 1] = (R)T[e].imag();
            }
            t.cmask = M[0];
            t.lcmask = M[1];
            t.gcmask = M[2];
            t.lmask = M[3];
            if (M[0] | M[1] | M[2] | M[3]) t.flags |= OPF_SGN;
            out.push_back(t);
            gout.push_back(-1);
        };
        int next = S.op_begin;
        for (int gap = 0; gap <= K; ++gap) {
            emit_table(gap);
            const int stop = gap < K ? mix[gap] : S.op_end;
            for (; next < stop; ++next)
                if (!gathered[next - S.op_begin]) {
                    out.push_back(ops[next]);
                    gout.push_back(gate[next]);
                }
            if (gap < K) {
                out.push_back(ops[mix[gap]]);
                gout.push_back(gate[mix[gap]]);
                next = mix[gap] + 1;
            }
        }
        S.op_begin = nb;
        S.op_end = (int)out.size();
        // the group factor is needed only for what feeds it now
        S.acc = 0;
        for (int o = S.op_begin; o < S.op_end; ++o) {
            const DevOp<R> &d = out[o];
            if (d.kind != OP_DIAG) continue;
            const uint64_t all = d.cmask | (1ull << d.a) | (d.b >= 0 ? (1ull << d.b) : 0ull);
            if ((d.flags & OPF_REG1) ? !(d.flags & OPF_PAT) : (all & gall) == 0) S.acc = 1;
        }
    }
    for (int o = oe; o < (int)ops.size(); ++o) {
        out.push_back(ops[o]);
        gout.push_back(gate[o]);
    }
    oe = (int)out.size() - ((int)ops.size() - oe);
    ops.swap(out);
    gate.swap(gout);
}

// Rotation-layer stages (h4 kind 4): a pass of fixed real rotations and
// fixed diagonals whose stages each rotate every register slot at most once
// is rewritten so that each stage is straight-line code: a table of gathered
// diagonals (OP_DIAG16), the four rotations (OP_ROT4, each in the form
// c [[1, -t], [t, 1]] with c going to the pass scale), a second table, and
// the group factor of the diagonals left on bits outside the registers.
// Diagonals on bits outside the tile form one factor per tile, applied with
// the pass scale by the last store.  Every diagonal is placed inside its
// range: after the last rotation on one of its bits that precedes it and
// before the first that follows it (diagonals commute with each other and
// with rotations on other bits); placements that fold it into a table are
// preferred.  Returns false (nothing changed) when the pass does not have
// this form: then its stages keep the general loop (gather_stage_diagonals).
template <typename R>
inline bool build_rotation_layers(std::vector<DevOp<R>> &ops, std::vector<int> &gate, const std::vector<Op> &pops,
                                  int ob, int oe, std::vector<DevStage> &stages, int sb,
                                  const std::vector<int> &local_bits, DevPass &dp) {
    const int NS = (int)stages.size() - sb;
    if (NS <= 0) return false;
    uint64_t localm = 0;
    for (int b : local_bits) localm |= 1ull << b;
    std::vector<int> st_of(oe - ob, -1);
    for (int si = 0; si < NS; ++si)
        for (int o = stages[sb + si].op_begin; o < stages[sb + si].op_end; ++o) st_of[o - ob] = si;
    std::vector<uint64_t> regm(NS, 0);
    for (int si = 0; si < NS; ++si) {
        const DevStage &S = stages[sb + si];
        const int regs[4] = {S.r0, S.r1, S.r2, S.r3};
        for (int i = 0; i < 4; ++i) regm[si] |= 1ull << local_bits[regs[i]];
    }
    // rotations: t per (stage, slot), the pass scale and a bound on the growth
    // of the unscaled amplitudes
    std::vector<double> tv(4 * NS, 0.0);
    std::vector<char> used(4 * NS, 0);
    double scale = 1.0, growth = 1.0;
    for (int o = ob; o < oe; ++o) {
        const DevOp<R> &d = ops[o];
        const Op &src = pops[o - ob];
        if (st_of[o - ob] < 0 || src.param) return false;
        if (d.kind == OP_DIAG) continue;
        if (d.kind != OP_U1 || !(d.flags & (OPF_ROTC | OPF_ROTS))) return false;
        const double c = src.m[0].real(), sn = src.m[2].real();
        if (!(std::fabs(c) >= 1.0 / 4096.0 * std::fabs(sn)) || c == 0.0) return false;
        const int slot = st_of[o - ob] * 4 + d.ra;
        if (used[slot]) return false;
        used[slot] = 1;
        tv[slot] = sn / c;
        scale *= c;
        growth *= 1.0 + std::fabs(sn / c);
    }
    if (growth > (sizeof(R) == 4 ? 1e30 : 1e290)) return false;
    // placements of the diagonals: stage, and 0 = table before the
    // rotations, 1 = after them, 2 = group factor, 3 = tile factor
    struct Place { int o, stage, where, r; uint64_t outb; };
    std::vector<Place> pl;
    auto rot_bits = [&](int o) { return 1ull << ops[o].a; };
    for (int o = ob; o < oe; ++o) {
        if (ops[o].kind != OP_DIAG) continue;
        const Op &src = pops[o - ob];
        const uint64_t bits = src.cmask | (1ull << src.a) | (src.b >= 0 ? (1ull << src.b) : 0ull);
        if ((bits & localm) == 0) {
            pl.push_back({o, -1, 3, -1, 0});
            continue;
        }
        int s_lo = -1, s_hi = NS;
        for (int q = o - 1; q >= ob; --q)
            if (ops[q].kind == OP_U1 && (rot_bits(q) & bits)) { s_lo = st_of[q - ob]; break; }
        for (int q = o + 1; q < oe; ++q)
            if (ops[q].kind == OP_U1 && (rot_bits(q) & bits)) { s_hi = st_of[q - ob]; break; }
        if (s_lo >= 0 && s_lo == s_hi) return false;
        const bool pat_neg = (ops[o].flags & OPF_PAT) && (ops[o].flags & OPF_NEG);
        auto fold = [&](int si, int &r, uint64_t &outb) {
            const uint64_t A = bits & regm[si], B = bits & ~regm[si];
            if (B == 0) { r = -1; outb = 0; return true; }
            if (pat_neg && __builtin_popcountll(A) == 1 && __builtin_popcountll(B) == 1) {
                const DevStage &S = stages[sb + si];
                const int regs[4] = {S.r0, S.r1, S.r2, S.r3};
                for (int i = 0; i < 4; ++i)
                    if ((1ull << local_bits[regs[i]]) == A) r = i;
                outb = B;
                return true;
            }
            return false;
        };
        bool done = false;
        int r = -1;
        uint64_t outb = 0;
        // after the stage of its last preceding rotation, before the stage
        // of its next one, then any other table, then a group factor
        if (s_lo >= 0 && s_lo < s_hi && fold(s_lo, r, outb)) { pl.push_back({o, s_lo, 1, r, outb}); done = true; }
        if (!done && s_hi < NS && s_hi > s_lo && fold(s_hi, r, outb)) { pl.push_back({o, s_hi, 0, r, outb}); done = true; }
        for (int si = std::max(s_lo, 0); !done && si < std::min(s_hi, NS); ++si)
            if (si >= s_lo && fold(si, r, outb)) { pl.push_back({o, si, 1, r, outb}); done = true; }
        for (int si = s_lo + 1; !done && si <= std::min(s_hi, NS - 1); ++si)
            if (fold(si, r, outb)) { pl.push_back({o, si, 0, r, outb}); done = true; }
        for (int si = s_lo + 1; !done && si < std::min(s_hi, NS); ++si)
            if ((bits & regm[si]) == 0) { pl.push_back({o, si, 2, -1, 0}); done = true; }
        if (!done) return false;
    }
    // rebuild the pass's ops: per stage its group-factor diagonals, tables
    // and rotations; then the tile-factor diagonals
    std::vector<DevOp<R>> out(ops.begin(), ops.begin() + ob);
    std::vector<int> gout(gate.begin(), gate.begin() + ob);
    auto table = [&](int si, int where) -> int {
        cd T[16];
        for (int e = 0; e < 16; ++e) T[e] = 1.0;
        uint64_t M[4] = {0, 0, 0, 0};
        bool any = false;
        const DevStage &S = stages[sb + si];
        const int regs[4] = {S.r0, S.r1, S.r2, S.r3};
        for (const Place &p : pl) {
            if (p.stage != si || p.where != where) continue;
            any = true;
            if (p.r >= 0) {
                M[p.r] ^= p.outb;
                continue;
            }
            const Op &src = pops[p.o - ob];
            for (int e = 0; e < 16; ++e) {
                uint64_t k = 0;
                for (int i = 0; i < 4; ++i)
                    if ((e >> i) & 1) k |= 1ull << local_bits[regs[i]];
                if ((k & src.cmask) != src.cmask) continue;
                const int ba = (k >> src.a) & 1;
                T[e] *= src.b >= 0 ? src.m[2 * ba + (int)((k >> src.b) & 1)] : src.m[ba];
            }
        }
        if (!any) return -1;
        DevOp<R> t;
        std::memset(&t, 0, sizeof t);
        t.kind = OP_DIAG16;
        t.a = t.b = t.la = t.lb = t.ra = t.rb = -1;
        t.tab = -1;
        for (int e = 0; e < 16; ++e) {
            t.m[2 * e] = (R)T[e].real();
            t.m[2 * e + 1] = (R)T[e].imag();
        }
        t.cmask = M[0];
        t.lcmask = M[1];
        t.gcmask = M[2];
        t.lmask = M[3];
        if (M[0] | M[1] | M[2] | M[3]) t.flags |= OPF_SGN;
        out.push_back(t);
        gout.push_back(-1);
        return (int)out.size() - 1;
    };
    for (int si = 0; si < NS; ++si) {
        DevStage &S = stages[sb + si];
        S.op_begin = (int)out.size();
        for (const Place &p : pl)
            if (p.stage == si && p.where == 2) {
                out.push_back(ops[p.o]);
                gout.push_back(gate[p.o]);
            }
        S.op_end = (int)out.size();
        S.acc = S.op_end > S.op_begin ? 1 : 0;
        S.tpre = table(si, 0);
        S.tpost = table(si, 1);
        if (S.tpost < 0) {
            // every layer ends with a table (its code has no branch on it)
            DevOp<R> t;
            std::memset(&t, 0, sizeof t);
            t.kind = OP_DIAG16;
            t.a = t.b = t.la = t.lb = t.ra = t.rb = -1;
            t.tab = -1;
            for (int e = 0; e < 16; ++e) t.m[2 * e] = (R)1;
            out.push_back(t);
            gout.push_back(-1);
            S.tpost = (int)out.size() - 1;
        }
        const bool sgn = (out[S.tpost].flags & OPF_SGN) || (S.tpre >= 0 && (out[S.tpre].flags & OPF_SGN));
        S.rl = (S.tpre >= 0 ? 1 : 0) | (sgn ? 2 : 0) | (S.acc ? 4 : 0);
        DevOp<R> q;
        std::memset(&q, 0, sizeof q);
        q.kind = OP_ROT4;
        q.a = q.b = q.la = q.lb = q.ra = q.rb = -1;
        q.tab = -1;
        for (int i = 0; i < 4; ++i) q.m[2 * i] = (R)tv[4 * si + i];
        out.push_back(q);
        gout.push_back(-1);
        S.rot = (int)out.size() - 1;
    }
    dp.tf_begin = (int)out.size();
    for (const Place &p : pl)
        if (p.where == 3) {
            out.push_back(ops[p.o]);
            gout.push_back(gate[p.o]);
        }
    dp.tf_end = (int)out.size();
    for (int o = oe; o < (int)ops.size(); ++o) {
        out.push_back(ops[o]);
        gout.push_back(gate[o]);
    }
    dp.op_end = (int)out.size() - ((int)ops.size() - oe);
    dp.scale = scale;
    dp.h4 = 4;
    ops.swap(out);
    gate.swap(gout);
    return true;
}

template <typename R>
inline void build_stages(std::vector<DevOp<R>> &ops, int ob, int oe, const std::vector<int> &local_bits,
                         std::vector<DevStage> &out, std::vector<uint32_t> &aux32, bool final_to_global) {
    const int m = (int)local_bits.size();
    const bool can_fold = final_to_global && m <= 16;
    int start = ob;
    std::vector<int> regs;
    bool diag = false;
    int closed = 0;  // stages of this tile so far
    // layout map Q(j) = sum_i j_i col[i] ^ q over GF(2)
    uint32_t col[32];
    for (int i = 0; i < m; ++i) col[i] = 1u << i;
    uint32_t q = 0;
    bool ident = true;
    auto img = [&](uint32_t v) {
        uint32_t r = q;
        for (int i = 0; i < m; ++i)
            if ((v >> i) & 1) r ^= col[i];
        return r;
    };
    auto foldable = [](const DevOp<R> &d) {
        return d.kind == OP_XPERM && d.gcmask == 0 && __builtin_popcountll(d.lcmask) <= 1;
    };
    auto close = [&](int end, bool force) {
        if (end <= start && !force) return;
        // fill with the highest unused local bits (keeps the low bits on the
        // lanes, so global loads of a group stay coalesced)
        for (int b = m - 1; b >= 0 && (int)regs.size() < 3; --b)
            if (std::find(regs.begin(), regs.end(), b) == regs.end()) regs.push_back(b);
        std::sort(regs.begin(), regs.end());
        DevStage S;
        std::memset(&S, 0, sizeof S);
        S.r0 = regs[0];
        S.r1 = regs[1];
        S.r2 = regs[2];
        S.op_begin = start;
        S.op_end = end;
        S.has_diag = diag ? 1 : 0;
        for (int o = start; o < end; ++o) {
            DevOp<R> &d = ops[o];
            auto slot = [&](int lb) { return (int)(std::find(regs.begin(), regs.end(), lb) - regs.begin()); };
            if (d.kind == OP_U1 || d.kind == OP_XPERM || d.kind == OP_U2 || d.kind == OP_SWAP) d.ra = slot(d.la);
            if (d.kind == OP_U2 || d.kind == OP_SWAP) d.rb = slot(d.lb);
            if (d.kind == OP_LADDER) {
                const int sl = d.la >= 0 ? slot(d.la) : 3;
                d.ra = sl < 3 ? sl : -1;
                // K_e: phase of the register bits' in-tile offset
                for (int e = 0; e < 8; ++e) {
                    const uint32_t lo = ((e & 1) ? 1u << regs[0] : 0u) | ((e & 2) ? 1u << regs[1] : 0u) |
                                        ((e & 4) ? 1u << regs[2] : 0u);
                    const V2<R> k = host_phase<R>(d.turns, local_offset(lo, local_bits) & d.lmask);
                    d.m[2 * (8 + e)] = k.x;
                    d.m[2 * (8 + e) + 1] = k.y;
                }
            }
            if (d.kind == OP_DIAG) {
                d.flags &= ~OPF_PLACEMENT;
                const int sa = d.la >= 0 ? slot(d.la) : 3, sb = d.lb >= 0 ? slot(d.lb) : 3;
                d.ra = sa < 3 ? sa : -1;
                d.rb = sb < 3 ? sb : -1;
                uint64_t regmask = 0;
                for (int r : regs) regmask |= 1ull << r;
                const bool ctrl_reg = (d.lcmask & regmask) != 0;
                if (d.ra < 0 && d.rb < 0 && !ctrl_reg) {
                    d.flags |= OPF_GRP;
                    S.acc = 1;
                } else if (d.b < 0 && d.cmask == 0 && d.ra >= 0) {
                    d.flags |= OPF_REG1;
                    S.acc = 1;
                }
            }
        }
        if (!ident) {
            if (closed == 0) fail(SV_EDEVICE, "internal: layout map on the first stage of a tile");
            S.perm = 1;
            S.perm_tab = (int)aux32.size();
            const uint32_t q0 = q;
            q = 0;  // tables hold the linear part; pd[e] carries q
            for (uint32_t v = 0; v < 128; ++v) aux32.push_back(img(v & ((1u << m) - 1)));
            const uint32_t nh = m > 7 ? 1u << (m - 7) : 1u;
            for (uint32_t v = 0; v < nh; ++v) aux32.push_back(img(v << 7));
            q = q0;
            for (int e = 0; e < 8; ++e) {
                const uint32_t lo = ((e & 1) ? 1u << regs[0] : 0u) | ((e & 2) ? 1u << regs[1] : 0u) |
                                    ((e & 4) ? 1u << regs[2] : 0u);
                S.pd[e] = (uint16_t)img(lo);
            }
        }
        out.push_back(S);
        ++closed;
        start = end;
        regs.clear();
        diag = false;
    };
    bool pending = false;  // Q changed since the last closed stage
    for (int o = ob; o < oe; ++o) {
        const DevOp<R> &d = ops[o];
        if (d.kind == OP_DENSE4) {
            // a stage of its own on its four bits (layout maps are not folded
            // in passes that hold dense ops)
            if (!ident) fail(SV_EDEVICE, "internal: dense op after a folded permutation");
            close(o, false);
            DevStage S;
            std::memset(&S, 0, sizeof S);
            int r[4], k = 0;
            for (int b = 0; b < m && k < 4; ++b)
                if ((d.lcmask >> b) & 1) r[k++] = b;
            if (k != 4) fail(SV_EDEVICE, "internal: dense op without four local bits");
            S.r0 = r[0];
            S.r1 = r[1];
            S.r2 = r[2];
            S.r3 = r[3];
            S.op_begin = o;
            S.op_end = o + 1;
            S.mfma = 1;
            S.wtab = d.tab;
            out.push_back(S);
            ++closed;
            start = o + 1;
            continue;
        }
        std::vector<int> tg;
        if (d.kind == OP_U1 || d.kind == OP_XPERM) tg = {d.la};
        else if (d.kind == OP_U2 || d.kind == OP_SWAP) tg = {d.la, d.lb};
        int add = 0;
        for (int t : tg)
            if (std::find(regs.begin(), regs.end(), t) == regs.end()) ++add;
        const bool full = (int)regs.size() + add > 3;
        if (can_fold && foldable(d) && (full || start == o) && (closed > 0 || o > start)) {
            close(o, false);
            start = o + 1;
            // Q <- Q o P with P(j) = j ^ [control bit set] 2^t (no control: always)
            const int t = d.la;
            const uint32_t lc = (uint32_t)d.lcmask;
            if (lc) {
                const int cb = __builtin_ctz(lc);
                col[cb] ^= col[t];
            } else {
                q ^= col[t];
            }
            ident = false;
            for (int i = 0; i < m && ident; ++i) ident = col[i] == (1u << i);
            ident = ident && q == 0;
            pending = true;
            continue;
        }
        if (full) close(o, false);
        pending = false;
        for (int t : tg)
            if (std::find(regs.begin(), regs.end(), t) == regs.end()) regs.push_back(t);
        if (d.kind == OP_DIAG || d.kind == OP_LADDER) diag = true;
    }
    if (start < oe) close(oe, false);
    else if (pending && !ident) close(oe, true);  // realise the final layout
}

struct DevTerms {
    std::vector<DevTerm> terms;
    std::vector<int> gbeg, gend;
    std::vector<uint64_t> gx;
    std::vector<double> coeffs;  // by original index
    int T = 0;
};

inline DevTerms build_dev_terms(const TermGroups &tg) {
    DevTerms d;
    d.T = (int)tg.terms.size();
    int g0 = -1;
    for (size_t g = 0; g < tg.gx.size(); ++g)
        if (tg.gx[g] == 0) g0 = (int)g;
    auto push_group = [&](uint64_t x, int b, int e, bool add_norm) {
        d.gx.push_back(x);
        d.gbeg.push_back((int)d.terms.size());
        for (int i = b; i < e; ++i) {
            const Term &t = tg.terms[tg.order[i]];
            DevTerm dt;
            dt.x = t.x;
            dt.z = t.z;
            dt.ny = t.ny;
            dt.idx = tg.order[i];
            dt.c = t.c;
            d.terms.push_back(dt);
        }
        if (add_norm) {
            DevTerm dt;
            dt.x = 0;
            dt.z = 0;
            dt.ny = 0;
            dt.idx = d.T;
            dt.c = 0.0;
            d.terms.push_back(dt);
        }
        d.gend.push_back((int)d.terms.size());
    };
    if (g0 < 0) push_group(0, 0, 0, true);
    for (size_t g = 0; g < tg.gx.size(); ++g)
        push_group(tg.gx[g], tg.g_begin[g], tg.g_end[g], (int)g == g0);
    d.coeffs.resize(std::max(d.T, 1));
    for (int t = 0; t < d.T; ++t) d.coeffs[t] = tg.terms[t].c;
    return d;
}


// ---------------------------------------------------------------------------
// Expectation plans: passes of tile-resident Pauli groups (see expect.hip)
// ---------------------------------------------------------------------------

struct alignas(16) EPass {
    int32_t m, l;              // local bits, low contiguous run
    int32_t g_begin, g_end;    // group chunks
    int32_t hi_begin, nslots;  // hi-offset table in aux; terms (LDS slots)
    uint32_t vb;               // workgroups per circuit
    int32_t wide;              // 1: supports wider than a tile, read from HBM
    uint64_t free_mask, ntiles;  // wide: ntiles = pairs per workgroup
    uint64_t part_off;         // this pass's partials inside a circuit's row
};

struct alignas(16) EGroup {
    uint32_t xl;       // X/Y support in tile coordinates
    int32_t pim;       // uses Im (odd ny) instead of Re of conj(b) a
    int32_t tbeg, tend;
    uint64_t x, pad;   // X/Y support (global bits)
};

struct alignas(16) ETerm {
    uint64_t z;        // Z/Y support (global bits)
    uint32_t zl;       // its local part in tile coordinates
    uint16_t slot;
    uint8_t diag, neg;
};

struct ETermRef {
    uint64_t off;      // first partial in a circuit's row
    uint32_t stride, cnt;
};

struct EPlanHost {
    int n = 0, T = 0;
    bool ok = true;
    std::string why;
    std::vector<EPass> passes;
    std::vector<uint64_t> aux;
    std::vector<EGroup> groups;
    std::vector<ETerm> terms;
    std::vector<ETermRef> refs;  // by term index, T = norm
    std::vector<double> coeffs;
    uint64_t part_stride = 0;    // doubles per circuit
};

struct EPlanDev {
    const EPass *passes;
    const uint64_t *aux;
    const EGroup *groups;
    const ETerm *terms;
    const ETermRef *refs;
    const double *coeffs;
};

EPlanHost make_eplan(int n, int m_max, const DevTerms &dt);
EPlanDev upload_eplan(Ctx *ctx, const EPlanHost &E, const std::string &slot);
int expect_tile_bits(const Ctx *ctx, int dtype);
// FP64 partial-sum buffer for nc states of plan E (scratch slot `slot`).
double *expect_partials(Ctx *ctx, const EPlanHost &E, int nc, const std::string &slot);
// Launches only (no allocation or upload): part comes from expect_partials.
template <typename R>
void launch_expect(Ctx *ctx, const EPlanHost &E, const EPlanDev &d, const V2<R> *slab, uint64_t dim, int nc,
                   double *part, const int *d_out_slot, double *d_E, double *d_vals);

}  // namespace sv
