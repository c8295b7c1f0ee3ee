// Device-side helpers shared by the HIP translation units: complex
// arithmetic on (re, im) pairs, index expansion, the ops applied to a tile in
// LDS, FP64 block reductions and the Pauli pair contribution.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sv_internal.h"

namespace sv {


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
// Ops applied to a tile held in LDS.  `gidx(j)` maps a local index to the
// global amplitude index (diagonal ops use it).  Work assignment: element
// ops use j = tid + s*TPB, pair ops p = tid + s*TPB over the reduced space.
// ---------------------------------------------------------------------------

template <typename R, int TPB, typename GI>
__device__ __forceinline__ void lds_apply(V2<R> *tile, int m, const DevOp<R> &op, uint64_t tile_base,
                                          GI gidx) {
    const uint32_t T = 1u << m;
    const int tid = threadIdx.x;
    const int kind = op.kind;
    if (kind == OP_U1 || kind == OP_XPERM) {
        if ((tile_base & op.gcmask) != op.gcmask) return;
        const int la = op.la;
        const uint32_t lc = (uint32_t)op.lcmask;
        const uint32_t lo = (1u << la) - 1;
        if (kind == OP_XPERM) {
            for (uint32_t p = tid; p < T / 2; p += TPB) {
                const uint32_t i0 = ((p & ~lo) << 1) | (p & lo);
                if ((i0 & lc) != lc) continue;
                const uint32_t i1 = i0 | (1u << la);
                const V2<R> x = tile[i0], y = tile[i1];
                tile[i0] = y;
                tile[i1] = x;
            }
        } else {
            const V2<R> m0 = mat_at(op, 0), m1 = mat_at(op, 1), m2 = mat_at(op, 2), m3 = mat_at(op, 3);
            for (uint32_t p = tid; p < T / 2; p += TPB) {
                const uint32_t i0 = ((p & ~lo) << 1) | (p & lo);
                if ((i0 & lc) != lc) continue;
                const uint32_t i1 = i0 | (1u << la);
                const V2<R> x = tile[i0], y = tile[i1];
                tile[i0] = cmac2(m0, x, m1, y);
                tile[i1] = cmac2(m2, x, m3, y);
            }
        }
    } else if (kind == OP_U2 || kind == OP_SWAP) {
        if ((tile_base & op.gcmask) != op.gcmask) return;
        const int la = op.la, lb = op.lb;
        const int p0 = la < lb ? la : lb, p1 = la < lb ? lb : la;
        const uint32_t lc = (uint32_t)op.lcmask;
        for (uint32_t p = tid; p < T / 4; p += TPB) {
            uint32_t k = ((p >> p0) << (p0 + 1)) | (p & ((1u << p0) - 1));
            k = ((k >> p1) << (p1 + 1)) | (k & ((1u << p1) - 1));
            if ((k & lc) != lc) continue;
            if (kind == OP_SWAP) {
                const uint32_t i = k | (1u << la), j = k | (1u << lb);
                const V2<R> x = tile[i], y = tile[j];
                tile[i] = y;
                tile[j] = x;
            } else {
                const uint32_t idx[4] = {k, k | (1u << lb), k | (1u << la), k | (1u << la) | (1u << lb)};
                V2<R> v[4], w[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = tile[idx[i]];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    V2<R> acc = cmul(mat_at(op, 4 * i), v[0]);
#pragma unroll
                    for (int jj = 1; jj < 4; ++jj) {
                        V2<R> t = cmul(mat_at(op, 4 * i + jj), v[jj]);
                        acc.x += t.x;
                        acc.y += t.y;
                    }
                    w[i] = acc;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) tile[idx[i]] = w[i];
            }
        }
    } else if (kind == OP_DIAG) {
        const int a = op.a, b = op.b;
        const uint64_t cm = op.cmask;
        const V2<R> d0 = mat_at(op, 0), d1 = mat_at(op, 1), d2 = mat_at(op, 2), d3 = mat_at(op, 3);
        for (uint32_t j = tid; j < T; j += TPB) {
            const uint64_t k = gidx(j);
            if ((k & cm) != cm) continue;
            int idx = (int)((k >> a) & 1);
            if (b >= 0) idx = 2 * idx + (int)((k >> b) & 1);
            const V2<R> f = idx == 0 ? d0 : idx == 1 ? d1 : idx == 2 ? d2 : d3;
            tile[j] = cmul(tile[j], f);
        }
    } else if (kind == OP_LADDER) {
        const int a = op.a;
        const uint64_t lm = op.lmask;
        const double tu = op.turns;
        for (uint32_t j = tid; j < T; j += TPB) {
            const uint64_t k = gidx(j);
            if (!((k >> a) & 1)) continue;
            tile[j] = cmul(tile[j], ladder_phase<R>(tu, k & lm));
        }
    }
}

template <typename R, int TPB, typename GI>
__device__ __forceinline__ void lds_apply_list(V2<R> *tile, int m, const DevOp<R> *ops, int begin,
                                               int end, uint64_t tile_base, GI gidx,
                                               int ovr_index = -1, const DevOp<R> *ovr = nullptr) {
    bool prev_diag = false;
    for (int o = begin; o < end; ++o) {
        const DevOp<R> &op = (o == ovr_index) ? *ovr : ops[o];
        const bool d = op.kind == OP_DIAG || op.kind == OP_LADDER;
        if (!(d && prev_diag)) __syncthreads();
        lds_apply<R, TPB>(tile, m, op, tile_base, gidx);
        prev_diag = d;
    }
    __syncthreads();
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
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
    for (int k = 0; k < 16; ++k) {
        d.m[2 * k] = (R)op.m[k].real();
        d.m[2 * k + 1] = (R)op.m[k].imag();
    }
    return d;
}

// Fill the tile-local fields of an op for a pass with local bits `lb`.
template <typename R>
inline void localise(DevOp<R> &d, const std::vector<int> &local_bits) {
    int pos[64];
    for (int i = 0; i < 64; ++i) pos[i] = -1;
    for (size_t i = 0; i < local_bits.size(); ++i) pos[local_bits[i]] = (int)i;
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

}  // namespace sv
