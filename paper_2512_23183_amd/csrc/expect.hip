// FP64 Pauli-sum expectation values over one state or a slab of states.
//
// E = sum_t c_t <P_t> / <psi|psi>, with, for a term of X/Y support x, Z/Y
// support z and ny Y factors (qubit order as everywhere: qubit q is index
// bit n-1-q),
//   <P> = sum_k conj(psi[k ^ x]) i^ny (-1)^popcount(k & z) psi[k].
// Summing the pair {k, k ^ x} once (k with the top bit of x clear) gives
//   2 (-1)^popcount(k & z) * {Re, -Im, -Re, Im}[ny mod 4] (conj(psi[k ^ x]) psi[k])
// because popcount(x & z) = ny.  Diagonal terms (x = 0) reduce
// (-1)^popcount(k & z) |psi[k]|^2.  The norm <psi|psi> is the pseudo-term
// x = z = 0 that closes the diagonal group, so the quotient renormalises in
// FP64.
//
// Stage 1 (k_expect_tile): the terms are grouped by x; each pass holds the
// groups whose x lies inside a set of m local bits (the low coalescing bits
// included) and reads every state once, tile by tile, into LDS.  Each wave
// owns a fixed subset of the pass's group chunks and adds its wave-reduced
// FP64 sums into a per-workgroup LDS accumulator slot per term.  The tile's
// free-bit sign (-1)^popcount(base & z) and the factor 2 of a pair are
// applied there.  Workgroup b of circuit c handles tiles b, b + vb, ...
// with vb a function of the tile count only; gsplit workgroups share a
// tile and split its group chunks.  Each term is summed over the same
// tiles in the same order whatever gsplit and the number of circuits in
// the launch, so a circuit's result does not depend on what else shares
// the launch.
// Stage 2 (k_expect_final): per circuit, each term's vb partials are summed
// in ascending order, then E = (sum_t c_t v_t) / v_norm in term order.
#include "device_common.h"

#include <algorithm>
#include <cstring>
#include <numeric>

namespace sv {

namespace {

constexpr int EXPT_TPB = 512;  // 8 waves share a tile's groups (256: 16% slower on the 20-qubit 641-circuit gradient)
constexpr int EXPT_WAVES = EXPT_TPB / 64;
constexpr int EXPT_CHUNK = ESUM_CHUNK;  // terms per register block
constexpr int EXPT_SLOT_CAP = 1024;  // terms per pass (LDS accumulators)
constexpr uint64_t EXPT_VB_MAX = 2048;

}  // namespace

// Stage 1: grid = nc * vb workgroups of EXPT_TPB threads.
template <typename R>
__global__ __launch_bounds__(EXPT_TPB) void k_expect_tile(const V2<R> *__restrict__ slab, uint64_t dim,
                                                          const EPass *__restrict__ eps, int e,
                                                          const uint64_t *__restrict__ aux,
                                                          const EGroup *__restrict__ groups,
                                                          const ETerm *__restrict__ terms,
                                                          double *__restrict__ partial, uint64_t part_stride,
                                                          int gsplit) {
    extern __shared__ __align__(16) unsigned char smem[];
    const EPass &P = eps[e];
    const int m = P.m, l = P.l, nslots = P.nslots;
    const uint32_t T = 1u << m, lowm = (1u << l) - 1, nhi = 1u << (m - l);
    const uint32_t vb = P.vb;
    V2<R> *tile = reinterpret_cast<V2<R> *>(smem);
    uint64_t *hi_off = reinterpret_cast<uint64_t *>(smem + (sizeof(V2<R>) << m));
    double *acc_s = reinterpret_cast<double *>(hi_off + nhi);
    const uint32_t sl = blockIdx.x % (uint32_t)gsplit, cb = blockIdx.x / (uint32_t)gsplit;
    const uint64_t c = cb / vb;
    const uint32_t b = cb - (uint32_t)(c * vb);
    const V2<R> *__restrict__ psi = slab + c * dim;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    const int g0 = P.g_begin + (int)sl * EXPT_WAVES + wave, gstep = EXPT_WAVES * gsplit;
    for (uint32_t h = threadIdx.x; h < nhi; h += EXPT_TPB) hi_off[h] = aux[P.hi_begin + h];
    for (int s = threadIdx.x; s < nslots; s += EXPT_TPB) acc_s[s] = 0.0;
    __syncthreads();
    for (uint64_t t = b; t < P.ntiles; t += vb) {
        const uint64_t base = deposit(t, P.free_mask);
        for (uint32_t j = threadIdx.x; j < T; j += EXPT_TPB) tile[j] = psi[SV_GIDX(base | hi_off[j >> l] | (j & lowm), dim)];
        __syncthreads();
        for (int g = g0; g < P.g_end; g += gstep) {
            const EGroup G = groups[g];
            const int cnt = G.tend - G.tbeg;
            uint32_t zl[EXPT_CHUNK];
#pragma unroll
            for (int q = 0; q < EXPT_CHUNK; ++q) zl[q] = q < cnt ? terms[G.tbeg + q].zl : 0u;
            double acc[EXPT_CHUNK];
#pragma unroll
            for (int q = 0; q < EXPT_CHUNK; ++q) acc[q] = 0.0;
            esum_dispatch<R>(tile, T, G.xl, G.xl == 0 ? 0 : (G.pim ? 2 : 1), cnt, zl, acc, lane);
#pragma unroll
            for (int q = 0; q < EXPT_CHUNK; ++q) {
                if (q < cnt) {
                    const double s = wave_sum(acc[q]);
                    if (lane == 0) {
                        const ETerm &tm = terms[G.tbeg + q];
                        // tile sign, pair factor and the i^ny sign are exact scalings
                        const bool neg = ((__popcll(base & tm.z) & 1) != 0) != (tm.neg != 0);
                        const double v = tm.diag ? s : 2.0 * s;
                        acc_s[tm.slot] += neg ? -v : v;
                    }
                }
            }
        }
        __syncthreads();
    }
    // each slot has one owner (slice, wave): write the slots this wave summed
    double *out = partial + c * part_stride + P.part_off + (uint64_t)b * nslots;
    for (int g = g0; g < P.g_end; g += gstep) {
        const int tb = groups[g].tbeg, te = groups[g].tend;
        if ((int)lane < te - tb) {
            const int slot = terms[tb + lane].slot;
            out[slot] = acc_s[slot];
        }
    }
}

// Stage 1 for X/Y supports wider than any tile: pairs (k, k ^ x) straight
// from HBM.  Workgroup b of circuit c takes pairs [b * per, (b + 1) * per)
// of every group in the pass (per = P.ntiles); waves own groups as above.
template <typename R>
__global__ __launch_bounds__(EXPT_TPB) void k_expect_wide(const V2<R> *__restrict__ slab, uint64_t dim,
                                                          const EPass *__restrict__ eps, int e,
                                                          const EGroup *__restrict__ groups,
                                                          const ETerm *__restrict__ terms,
                                                          double *__restrict__ partial, uint64_t part_stride) {
    extern __shared__ __align__(16) unsigned char smem[];
    const EPass &P = eps[e];
    const int nslots = P.nslots;
    double *acc_s = reinterpret_cast<double *>(smem);
    const uint32_t vb = P.vb;
    const uint64_t c = blockIdx.x / vb;
    const uint32_t b = blockIdx.x - (uint32_t)(c * vb);
    const V2<R> *__restrict__ psi = slab + c * dim;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t per = P.ntiles, i0 = (uint64_t)b * per;
    const uint64_t i1 = i0 + per < dim / 2 ? i0 + per : dim / 2;
    for (int s = threadIdx.x; s < nslots; s += EXPT_TPB) acc_s[s] = 0.0;
    __syncthreads();
    for (int g = P.g_begin + wave; g < P.g_end; g += EXPT_WAVES) {
        const EGroup G = groups[g];
        const int cnt = G.tend - G.tbeg;
        const int hb = 63 - __clzll(G.x);
        const uint64_t below = (1ull << hb) - 1;
        uint64_t z[EXPT_CHUNK];
#pragma unroll
        for (int q = 0; q < EXPT_CHUNK; ++q) z[q] = q < cnt ? terms[G.tbeg + q].z : 0ull;
        double acc[EXPT_CHUNK];
#pragma unroll
        for (int q = 0; q < EXPT_CHUNK; ++q) acc[q] = 0.0;
        for (uint64_t it = i0 + lane; it < i1; it += 64) {
            const uint64_t k = ((it & ~below) << 1) | (it & below);
            const V2<R> a = psi[SV_GIDX(k, dim)], bb = psi[SV_GIDX(k ^ G.x, dim)];
            const double ax = a.x, ay = a.y, bx = bb.x, by = bb.y;
            const double u = G.pim ? bx * ay - by * ax : bx * ax + by * ay;
#pragma unroll
            for (int q = 0; q < EXPT_CHUNK; ++q)
                if (q < cnt) acc[q] += (__popcll(k & z[q]) & 1) ? -u : u;
        }
#pragma unroll
        for (int q = 0; q < EXPT_CHUNK; ++q) {
            if (q < cnt) {
                const double s = wave_sum(acc[q]);
                if (lane == 0) {
                    const ETerm &tm = terms[G.tbeg + q];
                    const double v = 2.0 * s;
                    acc_s[tm.slot] += tm.neg ? -v : v;
                }
            }
        }
    }
    __syncthreads();
    double *out = partial + c * part_stride + P.part_off + (uint64_t)b * nslots;
    for (int s = threadIdx.x; s < nslots; s += EXPT_TPB) out[s] = acc_s[s];
}

// Stage 2: one workgroup per circuit.  v_t = sum_b partial[t_off[t] +
// b * t_stride[t]] (ascending b); E = (sum_t c_t v_t) / v_T.  With vals,
// vals[c * (T + 1) + t] = v_t / v_T and vals[c * (T + 1) + T] = v_T.
__global__ void k_expect_final(double *__restrict__ partial, uint64_t part_stride, int nc,
                               const ETermRef *__restrict__ refs, int T, const double *__restrict__ coeffs,
                               const int *__restrict__ out_slot, double *__restrict__ E,
                               double *__restrict__ vals) {
    for (int c = blockIdx.x; c < nc; c += gridDim.x) {
        double *row = partial + (uint64_t)c * part_stride;
        for (int t = threadIdx.x; t <= T; t += blockDim.x) {
            const ETermRef r = refs[t];
            double v = 0.0;
            for (uint32_t i = 0; i < r.cnt; ++i) v += row[r.off + (uint64_t)i * r.stride];
            row[r.off] = v;
        }
        __threadfence_block();
        __syncthreads();
        const double norm = row[refs[T].off];
        if (threadIdx.x == 0) {
            double e = 0.0;
            for (int t = 0; t < T; ++t) e += coeffs[t] * row[refs[t].off];
            E[out_slot ? out_slot[c] : c] = e / norm;
        }
        if (vals) {
            double *vr = vals + (uint64_t)c * (T + 1);
            for (int t = threadIdx.x; t < T; t += blockDim.x) vr[t] = row[refs[t].off] / norm;
            if (threadIdx.x == 0) vr[T] = norm;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

EPlanHost make_eplan(int n, int m_max, const DevTerms &dt) {
    EPlanHost E;
    E.T = dt.T;
    E.n = n;
    E.coeffs = dt.coeffs;
    const int m = std::max(1, std::min(m_max, n));
    const int l0 = std::min(5, m);
    const uint64_t low = (1ull << l0) - 1;
    // split groups wider than a pass can hold
    struct Grp {
        uint64_t x;
        int b, e;
    };
    std::vector<Grp> gs;
    for (size_t g = 0; g < dt.gx.size(); ++g)
        for (int b = dt.gbeg[g]; b < dt.gend[g]; b += EXPT_SLOT_CAP)
            gs.push_back({dt.gx[g], b, std::min(dt.gend[g], b + EXPT_SLOT_CAP)});
    const int G = (int)gs.size();
    std::vector<int> order(G);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return __builtin_popcountll(gs[a].x) > __builtin_popcountll(gs[b].x);
    });
    std::vector<char> done(G, 0);
    int remaining = G;
    E.refs.assign(E.T + 1, ETermRef{0, 0, 0});
    uint64_t part = 0;
    // chunks of one group's terms that use the same part of conj(b) a
    auto add_chunks = [&](int g, const uint32_t xl, auto &&to_local, int &slot,
                          std::vector<std::pair<int, int>> &slot_of) {
        for (int pim = 0; pim < 2; ++pim) {
            std::vector<int> ts;
            for (int t = gs[g].b; t < gs[g].e; ++t)
                if (gs[g].x != 0 ? (dt.terms[t].ny & 1) == pim : pim == 0) ts.push_back(t);
            for (size_t i = 0; i < ts.size(); i += EXPT_CHUNK) {
                EGroup eg;
                std::memset(&eg, 0, sizeof eg);
                eg.xl = xl;
                eg.x = gs[g].x;
                eg.pim = pim;
                eg.tbeg = (int)E.terms.size();
                for (size_t k = i; k < std::min(ts.size(), i + EXPT_CHUNK); ++k) {
                    const DevTerm &d = dt.terms[ts[k]];
                    ETerm et;
                    std::memset(&et, 0, sizeof et);
                    et.z = d.z;
                    et.zl = to_local(d.z);
                    et.slot = (uint16_t)slot;
                    et.diag = gs[g].x == 0;
                    // ny mod 4 = 0: +Re, 1: -Im, 2: -Re, 3: +Im
                    et.neg = gs[g].x != 0 && (d.ny == 1 || d.ny == 2);
                    E.terms.push_back(et);
                    slot_of.push_back({d.idx, slot});
                    ++slot;
                }
                eg.tend = (int)E.terms.size();
                E.groups.push_back(eg);
            }
        }
    };
    // supports wider than the tile: passes that read pairs from HBM
    {
        const uint64_t pairs = n > 0 ? 1ull << (n - 1) : 1;
        const uint32_t vbw = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(EXPT_VB_MAX, pairs / 4096));
        auto none = [](uint64_t) { return 0u; };
        std::vector<int> wide;
        for (int g : order)
            if (__builtin_popcountll(gs[g].x) > m) wide.push_back(g);
        size_t i = 0;
        while (i < wide.size()) {
            EPass ep;
            std::memset(&ep, 0, sizeof ep);
            ep.wide = 1;
            ep.vb = vbw;
            ep.ntiles = (pairs + vbw - 1) / vbw;
            ep.g_begin = (int)E.groups.size();
            ep.part_off = part;
            int slot = 0;
            std::vector<std::pair<int, int>> slot_of;
            while (i < wide.size() && slot + (gs[wide[i]].e - gs[wide[i]].b) <= EXPT_SLOT_CAP) {
                const int g = wide[i++];
                done[g] = 1;
                --remaining;
                add_chunks(g, 0u, none, slot, slot_of);
            }
            ep.g_end = (int)E.groups.size();
            ep.nslots = slot;
            for (auto [idx, s] : slot_of) E.refs[idx] = ETermRef{part + (uint64_t)s, (uint32_t)slot, ep.vb};
            part += (uint64_t)slot * ep.vb;
            E.passes.push_back(ep);
        }
    }
    while (remaining > 0) {
        uint64_t S = low;
        int slots = 0;
        std::vector<int> chosen;
        for (int g : order) {
            if (done[g]) continue;
            const int cnt = gs[g].e - gs[g].b;
            const uint64_t need = gs[g].x & ~S;
            if (__builtin_popcountll(S) + __builtin_popcountll(need) <= m && slots + cnt <= EXPT_SLOT_CAP) {
                S |= gs[g].x;
                slots += cnt;
                chosen.push_back(g);
            }
        }
        if (chosen.empty()) {
            // the widest remaining support does not fit beside the low bits
            for (int g : order) {
                if (done[g]) continue;
                S = gs[g].x;
                chosen.push_back(g);
                break;
            }
        } else {
            // pad the greedy tile to m bits, then exchange one bit above the
            // low ones for an outside bit while more of the remaining terms
            // fit it (fewer passes over the states: each reads all of them)
            for (int bit = 0; bit < n && __builtin_popcountll(S) < m; ++bit) S |= 1ull << bit;
            auto fit = [&](uint64_t T) {
                int c = 0;
                for (int g : order)
                    if (!done[g] && (gs[g].x & ~T) == 0) c += gs[g].e - gs[g].b;
                return c;
            };
            int best = fit(S);
            // each round costs (remaining groups) x (tile bits) x (outside
            // bits) containment tests: skipped for very large Pauli sums
            const bool search = (uint64_t)remaining * (uint64_t)std::max(0, m - l0) * (uint64_t)std::max(0, n - m) <=
                                (1u << 20);
            for (int round = 0; search && round < 32; ++round) {
                int gain = 0;
                uint64_t bestS = S;
                for (int o = l0; o < n; ++o) {
                    if (!((S >> o) & 1)) continue;
                    for (int i = l0; i < n; ++i) {
                        if ((S >> i) & 1) continue;
                        const uint64_t T = (S & ~(1ull << o)) | (1ull << i);
                        const int c = fit(T);
                        if (c - best > gain) {
                            gain = c - best;
                            bestS = T;
                        }
                    }
                }
                if (gain <= 0) break;
                best += gain;
                S = bestS;
            }
            chosen.clear();
            slots = 0;
            for (int g : order) {
                if (done[g]) continue;
                const int cnt = gs[g].e - gs[g].b;
                if ((gs[g].x & ~S) == 0 && slots + cnt <= EXPT_SLOT_CAP) {
                    slots += cnt;
                    chosen.push_back(g);
                }
            }
        }
        for (int bit = 0; bit < n && __builtin_popcountll(S) < m; ++bit) S |= 1ull << bit;
        std::vector<int> local, freeb;
        int pos[64];
        for (int bit = 0; bit < n; ++bit) {
            if (S & (1ull << bit)) {
                pos[bit] = (int)local.size();
                local.push_back(bit);
            } else {
                pos[bit] = -1;
                freeb.push_back(bit);
            }
        }
        EPass ep;
        std::memset(&ep, 0, sizeof ep);
        ep.m = (int)local.size();
        int run = 0;
        while (run < ep.m && local[run] == run) ++run;
        ep.l = run;
        for (int bit : freeb) ep.free_mask |= 1ull << bit;
        ep.ntiles = 1ull << freeb.size();
        ep.vb = (uint32_t)std::min<uint64_t>(ep.ntiles, EXPT_VB_MAX);
        ep.hi_begin = (int)E.aux.size();
        for (uint32_t h = 0; h < (1u << (ep.m - ep.l)); ++h) {
            uint64_t o = 0;
            for (int i = 0; i < ep.m - ep.l; ++i)
                if ((h >> i) & 1) o |= 1ull << local[ep.l + i];
            E.aux.push_back(o);
        }
        auto to_local = [&](uint64_t mask) {
            uint32_t r = 0;
            for (int bit = 0; bit < n; ++bit)
                if ((mask >> bit) & 1 && pos[bit] >= 0) r |= 1u << pos[bit];
            return r;
        };
        ep.g_begin = (int)E.groups.size();
        ep.part_off = part;
        int slot = 0;
        std::vector<std::pair<int, int>> slot_of;  // (term idx, slot)
        for (int g : chosen) {
            done[g] = 1;
            --remaining;
            add_chunks(g, to_local(gs[g].x), to_local, slot, slot_of);
        }
        ep.g_end = (int)E.groups.size();
        ep.nslots = slot;
        for (auto [idx, s] : slot_of) E.refs[idx] = ETermRef{part + (uint64_t)s, (uint32_t)slot, ep.vb};
        part += (uint64_t)slot * ep.vb;
        E.passes.push_back(ep);
    }
    E.part_stride = part;
    return E;
}

EPlanDev upload_eplan(Ctx *ctx, const EPlanHost &E, const std::string &slot) {
    std::vector<unsigned char> host;
    auto put = [&](const void *p, size_t bytes) {
        const size_t off = (host.size() + 255) & ~(size_t)255;
        host.resize(off + bytes);
        if (bytes) std::memcpy(host.data() + off, p, bytes);
        return off;
    };
    const size_t o_p = put(E.passes.data(), E.passes.size() * sizeof(EPass));
    const size_t o_a = put(E.aux.data(), E.aux.size() * 8);
    const size_t o_g = put(E.groups.data(), E.groups.size() * sizeof(EGroup));
    const size_t o_t = put(E.terms.data(), E.terms.size() * sizeof(ETerm));
    const size_t o_r = put(E.refs.data(), E.refs.size() * sizeof(ETermRef));
    const size_t o_c = put(E.coeffs.data(), E.coeffs.size() * 8);
    char *base = (char *)scratch(ctx, slot, std::max<size_t>(host.size(), 256));
    upload(ctx, base, host.data(), host.size());
    EPlanDev d;
    d.passes = (const EPass *)(base + o_p);
    d.aux = (const uint64_t *)(base + o_a);
    d.groups = (const EGroup *)(base + o_g);
    d.terms = (const ETerm *)(base + o_t);
    d.refs = (const ETermRef *)(base + o_r);
    d.coeffs = (const double *)(base + o_c);
    return d;
}

size_t eplan_lds_bytes(const EPass &p, size_t amp_bytes) {
    return (amp_bytes << p.m) + 8 * ((size_t)1 << (p.m - p.l)) + 8 * (size_t)p.nslots;
}

double *expect_partials(Ctx *ctx, const EPlanHost &E, int nc, const std::string &slot) {
    return (double *)scratch(ctx, slot, 8 * std::max<uint64_t>(1, E.part_stride) * std::max(nc, 1));
}

template <typename R>
void launch_expect(Ctx *ctx, const EPlanHost &E, const EPlanDev &d, const V2<R> *slab, uint64_t dim, int nc,
                   double *part, const int *d_out_slot, double *d_E, double *d_vals) {
    if (!E.ok) fail(SV_EINVAL, E.why);
    for (size_t e = 0; e < E.passes.size(); ++e) {
        const EPass &p = E.passes[e];
        const uint64_t blocks = (uint64_t)p.vb * nc;
        if (blocks > 0x7fffffffull) fail(SV_EINVAL, "expectation launch too large");
        if (p.wide) {
            const size_t lds = 8 * (size_t)std::max(1, p.nslots);
            const int G = p.g_end - p.g_begin;
            LaunchScope ls(ctx, "expect_wide", 2.0 * sizeof(V2<R>) * (double)dim * nc * G);
            hipLaunchKernelGGL(k_expect_wide<R>, dim3((unsigned)blocks), dim3(EXPT_TPB), lds, ctx->stream, slab, dim,
                               d.passes, (int)e, d.groups, d.terms, part, E.part_stride);
        } else {
            const size_t lds = eplan_lds_bytes(p, sizeof(V2<R>));
            set_lds_limit((const void *)k_expect_tile<R>, lds);
            // enough workgroups to fill the chip: split the group chunks
            const uint64_t chunks = (uint64_t)(p.g_end - p.g_begin);
            const uint64_t max_split = std::max<uint64_t>(1, (chunks + EXPT_WAVES - 1) / EXPT_WAVES);
            const uint64_t want = (uint64_t)ctx->cu_count * 8;
            const uint64_t gsplit = std::min(max_split, std::max<uint64_t>(1, (want + blocks - 1) / blocks));
            if (blocks * gsplit > 0x7fffffffull) fail(SV_EINVAL, "expectation launch too large");
            LaunchScope ls(ctx, "expect_tile", (double)sizeof(V2<R>) * (double)dim * nc * gsplit);
            hipLaunchKernelGGL(k_expect_tile<R>, dim3((unsigned)(blocks * gsplit)), dim3(EXPT_TPB), lds, ctx->stream,
                               slab, dim, d.passes, (int)e, d.aux, d.groups, d.terms, part, E.part_stride,
                               (int)gsplit);
        }
        SV_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_expect_final, dim3((unsigned)std::min(nc, ctx->cu_count * 4)), dim3(256), 0, ctx->stream,
                       part, E.part_stride, nc, d.refs, E.T, d.coeffs, d_out_slot, d_E, d_vals);
    SV_HIP(hipGetLastError());
}
template void launch_expect<float>(Ctx *, const EPlanHost &, const EPlanDev &, const V2<float> *, uint64_t, int,
                                   double *, const int *, double *, double *);
template void launch_expect<double>(Ctx *, const EPlanHost &, const EPlanDev &, const V2<double> *, uint64_t, int,
                                    double *, const int *, double *, double *);

int expect_tile_bits(const Ctx *ctx, int dtype) {
    return ctx->expect_bits[dtype];
}

// One state: the energy goes to the device scalar d_energy, d_vals
// (nullable) receives the T + 1 values.
void expectation_dev(Ctx *ctx, const void *psi, int n, int dtype, const DevTerms &dt, double *d_energy,
                     double *d_vals) {
    EPlanHost E = make_eplan(n, expect_tile_bits(ctx, dtype), dt);
    EPlanDev d = upload_eplan(ctx, E, "exp_meta");
    double *part = expect_partials(ctx, E, 1, "exp_partial");
    if (dtype == SV_C64)
        launch_expect<float>(ctx, E, d, (const V2<float> *)psi, 1ull << n, 1, part, nullptr, d_energy, d_vals);
    else launch_expect<double>(ctx, E, d, (const V2<double> *)psi, 1ull << n, 1, part, nullptr, d_energy, d_vals);
}

void device_expectation(Ctx *ctx, const void *psi, int n, int dtype, const TermGroups &tg, double *energy,
                        double *term_values, double *norm2) {
    DevTerms dt = build_dev_terms(tg);
    const int T = dt.T;
    double *d_out = (double *)scratch(ctx, "exp_out", (size_t)(T + 2) * 8);
    expectation_dev(ctx, psi, n, dtype, dt, d_out, d_out + 1);
    std::vector<double> out(T + 2);
    SV_HIP(hipMemcpyAsync(out.data(), d_out, (T + 2) * 8, hipMemcpyDeviceToHost, ctx->stream));
    SV_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->profile) profile_collect(ctx);
    if (energy) *energy = out[0];
    if (term_values)
        for (int t = 0; t < T; ++t) term_values[t] = out[1 + t];
    if (norm2) *norm2 = out[1 + T];
}

void device_norm2(Ctx *ctx, const void *psi, int n, int dtype, double *out) {
    TermGroups empty;
    device_expectation(ctx, psi, n, dtype, empty, nullptr, nullptr, out);
}

}  // namespace sv
