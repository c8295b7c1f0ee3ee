// Batched execution of many independent circuits (parameter-shift copies,
// serving requests of mixed qubit counts), each from |0...0>.
//
//  * Circuits whose whole state fits one workgroup's LDS run in one
//    persistent launch: each workgroup repeatedly takes the next circuit
//    from a device counter (largest first), applies every op in LDS and
//    reduces the FP64 energy in place.  No HBM traffic for the state.
//  * Larger circuits run one at a time through the fused pass executor and
//    the two-stage FP64 expectation, energies staying on the device.
//  * The gradient is combined on the device in FP64 from the energies
//    (fixed summation order).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <numeric>

#include "device_common.h"

namespace sv {

struct alignas(16) DevCirc {
    int32_t n, op_begin, op_end, ovr_index;  // ovr_index: absolute op index or -1
    int32_t ovr_slot, grp_begin, grp_end, T;
    int32_t coeff_begin, out_slot, stage_begin, stage_end;
};

constexpr int SMALL_TPB = 256;

int small_batch_max_qubits(int dtype) { return dtype == SV_C64 ? 13 : 12; }

__global__ void k_fill_u32(unsigned *p, unsigned v, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// LDS: state[2^max_n], red[TPB/64], vals[max_T + 1], ladder tables.
template <typename R>
__global__ __launch_bounds__(SMALL_TPB) void k_small_batch(
    const DevCirc *__restrict__ circ, int ncirc, unsigned *__restrict__ counter,
    const DevOp<R> *__restrict__ ops, const DevStage *__restrict__ stages, const V2<R> *__restrict__ ltab,
    const DevOp<R> *__restrict__ ovr_ops,
    const DevTerm *__restrict__ terms, const int *__restrict__ gbeg, const int *__restrict__ gend,
    const uint64_t *__restrict__ gx, const double *__restrict__ coeffs, double *__restrict__ energies,
    int max_n, int max_T) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cur;
    V2<R> *st = reinterpret_cast<V2<R> *>(smem);
    double *red = reinterpret_cast<double *>(smem + (sizeof(V2<R>) << max_n));
    double *vals = red + SMALL_TPB / 64;
    V2<R> *tabs = reinterpret_cast<V2<R> *>(vals + ((max_T + 2) & ~1));
    for (;;) {
        if (threadIdx.x == 0) cur = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int c = cur;
        __syncthreads();
        if (c >= ncirc) break;
        const DevCirc &C = circ[c];
        const int n = C.n;
        const uint32_t N = 1u << n;
        for (uint32_t j = threadIdx.x; j < N; j += SMALL_TPB) {
            V2<R> v;
            v.x = j == 0 ? (R)1 : (R)0;
            v.y = 0;
            st[j] = v;
        }
        TileCtx<R> tc;
        tc.m = n;
        tc.l = n < 5 ? n : 5;
        tc.lowm = (1u << tc.l) - 1;
        tc.ident = true;
        tc.zero = false;
        tc.base = 0;
        tc.hi_off = nullptr;
        tc.tabs = tabs;
        tc.lt = ladder_split(n);
        tc.tstride = (1 << tc.lt) + (1 << (n - tc.lt));
        __syncthreads();
        run_stages<R, SMALL_TPB>(st, nullptr, tc, stages, C.stage_begin, C.stage_end, ops, ltab,
                                    C.ovr_index, ovr_ops + C.ovr_slot);
        for (int g = C.grp_begin; g < C.grp_end; ++g) {
            const uint64_t x = gx[g];
            const int hb = x ? 63 - __clzll(x) : -1;
            const uint32_t items = x ? N / 2 : N;
            for (int t = gbeg[g]; t < gend[g]; ++t) {
                const uint64_t z = terms[t].z;
                const int ny = terms[t].ny;
                double acc = 0.0;
                for (uint32_t it = threadIdx.x; it < items; it += SMALL_TPB) {
                    if (x == 0) {
                        const V2<R> a = st[it];
                        const double p = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
                        acc += (__popcll(it & z) & 1) ? -p : p;
                    } else {
                        const uint32_t k = ((it >> hb) << (hb + 1)) | (it & ((1u << hb) - 1));
                        const uint32_t k2 = k ^ (uint32_t)x;
                        const V2<R> a = st[k], b = st[k2];
                        const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
                        acc += pair_contrib(bx * ax + by * ay, bx * ay - by * ax, k, k2, z, ny);
                    }
                }
                const double s = block_sum<SMALL_TPB>(acc, red);
                if (threadIdx.x == 0) vals[terms[t].idx] = s;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double e = 0.0;
            for (int t = 0; t < C.T; ++t) e += coeffs[C.coeff_begin + t] * vals[t];
            energies[C.out_slot] = e / vals[C.T];
        }
        __syncthreads();
    }
}

// grad[i] = sum_j w[j] * E[circ[j]] for j in [beg[i], beg[i+1]) in order.
__global__ void k_combine(const double *__restrict__ E, const int *__restrict__ beg,
                          const int *__restrict__ circ, const double *__restrict__ w, int np,
                          double *__restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    double s = 0.0;
    for (int j = beg[i]; j < beg[i + 1]; ++j) s += w[j] * E[circ[j]];
    grad[i] = s;
}

namespace {

struct Blob {
    std::vector<unsigned char> host;
    size_t add(const void *src, size_t bytes) {
        const size_t off = (host.size() + 255) & ~(size_t)255;
        host.resize(off + std::max<size_t>(bytes, 16), 0);
        if (bytes && src) std::memcpy(host.data() + off, src, bytes);
        return off;
    }
};

constexpr size_t SMALL_VALS_MAX = 32 * 1024;  // LDS bytes for term values

template <typename R>
void launch_small(Ctx *ctx, const BatchSpec &spec, const std::vector<int> &idx, double *d_E) {
    if (idx.empty()) return;
    // op sets used by these circuits, uploaded once
    std::vector<int> set_begin(spec.op_sets.size(), -1), set_end(spec.op_sets.size(), -1);
    std::vector<DevOp<R>> dops;
    std::vector<int> all_local(64);
    std::iota(all_local.begin(), all_local.end(), 0);
    std::vector<int> ham_gb(spec.hams.size(), -1), ham_ge(spec.hams.size(), -1),
        ham_cb(spec.hams.size(), -1), ham_T(spec.hams.size(), 0);
    std::vector<DevTerm> terms;
    std::vector<int> gbeg, gend;
    std::vector<uint64_t> gx;
    std::vector<double> coeffs;
    std::vector<DevCirc> circ;
    std::vector<DevOp<R>> ovr;
    std::vector<DevStage> stages;
    std::vector<V2<R>> ltab;
    std::vector<int> set_sb(spec.op_sets.size(), -1), set_se(spec.op_sets.size(), -1);
    int max_n = 3, max_T = 0;
    for (int c : idx) {
        const BatchCircuit &bc = spec.circuits[c];
        // states of fewer than 3 qubits run as 3-qubit states whose extra
        // (most significant) bits stay |0>: energies are unchanged
        const int n_eff = std::max(bc.n, 3);
        if (set_begin[bc.op_set] < 0) {
            set_begin[bc.op_set] = (int)dops.size();
            std::vector<int> loc(all_local.begin(), all_local.begin() + n_eff);
            std::vector<uint64_t> hoff;
            for (const Op &op : spec.op_sets[bc.op_set]) {
                DevOp<R> d = to_dev<R>(op);
                localise(d, loc);
                if (op.kind == OP_LADDER) {
                    if (hoff.empty()) hoff = hi_offsets(loc, ladder_split(n_eff));
                    append_ladder_tables<R>(d, op, n_eff, hoff, ltab);
                }
                dops.push_back(d);
            }
            set_end[bc.op_set] = (int)dops.size();
            set_sb[bc.op_set] = (int)stages.size();
            build_stages<R>(dops, set_begin[bc.op_set], set_end[bc.op_set], n_eff, stages);
            set_se[bc.op_set] = (int)stages.size();
        }
        if (ham_gb[bc.ham] < 0) {
            DevTerms dt = build_dev_terms(spec.hams[bc.ham]);
            const int tb = (int)terms.size();
            ham_gb[bc.ham] = (int)gx.size();
            for (size_t g = 0; g < dt.gx.size(); ++g) {
                gx.push_back(dt.gx[g]);
                gbeg.push_back(tb + dt.gbeg[g]);
                gend.push_back(tb + dt.gend[g]);
            }
            ham_ge[bc.ham] = (int)gx.size();
            terms.insert(terms.end(), dt.terms.begin(), dt.terms.end());
            ham_cb[bc.ham] = (int)coeffs.size();
            coeffs.insert(coeffs.end(), dt.coeffs.begin(), dt.coeffs.end());
            ham_T[bc.ham] = dt.T;
        }
        DevCirc d;
        std::memset(&d, 0, sizeof d);
        d.n = n_eff;
        d.op_begin = set_begin[bc.op_set];
        d.op_end = set_end[bc.op_set];
        d.stage_begin = set_sb[bc.op_set];
        d.stage_end = set_se[bc.op_set];
        d.ovr_index = -1;
        d.ovr_slot = 0;
        if (bc.ovr_index >= 0) {
            d.ovr_index = d.op_begin + bc.ovr_index;
            d.ovr_slot = (int)ovr.size();
            const DevOp<R> &basep = dops[d.ovr_index];
            DevOp<R> o = to_dev<R>(bc.ovr_op);
            // same gate and qubits as the base op: reuse its placement
            o.la = basep.la;
            o.lb = basep.lb;
            o.ra = basep.ra;
            o.rb = basep.rb;
            o.tslot = basep.tslot;
            o.lcmask = basep.lcmask;
            o.gcmask = basep.gcmask;
            ovr.push_back(o);
        }
        d.grp_begin = ham_gb[bc.ham];
        d.grp_end = ham_ge[bc.ham];
        d.T = ham_T[bc.ham];
        d.coeff_begin = ham_cb[bc.ham];
        d.out_slot = bc.out_slot >= 0 ? bc.out_slot : c;
        circ.push_back(d);
        max_n = std::max(max_n, n_eff);
        max_T = std::max(max_T, d.T);
    }
    if (ovr.empty()) ovr.resize(1);
    // largest circuits first: better balance of the dynamic schedule
    std::stable_sort(circ.begin(), circ.end(), [](const DevCirc &a, const DevCirc &b) {
        return (a.op_end - a.op_begin) * (1ll << a.n) > (b.op_end - b.op_begin) * (1ll << b.n);
    });
    Blob blob;
    const size_t o_c = blob.add(circ.data(), circ.size() * sizeof(DevCirc));
    const size_t o_ops = blob.add(dops.data(), dops.size() * sizeof(DevOp<R>));
    const size_t o_stg = blob.add(stages.data(), stages.size() * sizeof(DevStage));
    const size_t o_lt = blob.add(ltab.data(), ltab.size() * sizeof(V2<R>));
    const size_t o_ovr = blob.add(ovr.data(), ovr.size() * sizeof(DevOp<R>));
    const size_t o_t = blob.add(terms.data(), terms.size() * sizeof(DevTerm));
    const size_t o_gb = blob.add(gbeg.data(), gbeg.size() * 4);
    const size_t o_ge = blob.add(gend.data(), gend.size() * 4);
    const size_t o_gx = blob.add(gx.data(), gx.size() * 8);
    const size_t o_cf = blob.add(coeffs.data(), coeffs.size() * 8);
    const size_t o_cnt = blob.add(nullptr, 16);
    char *base = (char *)scratch(ctx, "batch_small", blob.host.size());
    upload(ctx, base, blob.host.data(), blob.host.size());
    unsigned *d_cnt = (unsigned *)(base + o_cnt);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, ctx->stream, d_cnt, 0u, 1);
    const int lts = ladder_split(max_n);
    const size_t lds = (sizeof(V2<R>) << max_n) + 8 * (SMALL_TPB / 64) + 8 * ((max_T + 2) & ~1) +
                       STAGE_MAX_LADDERS * sizeof(V2<R>) * ((1u << lts) + (1u << (max_n - lts)) + 1);
    set_lds_limit((const void *)k_small_batch<R>, lds);
    const int nc = (int)circ.size();
    const int per_cu = lds <= 40 * 1024 ? 4 : lds <= 80 * 1024 ? 2 : 1;
    const int grid = std::max(1, std::min(nc, ctx->cu_count * per_cu));
    double bytes = 0;
    for (const DevCirc &d : circ) bytes += (double)(sizeof(V2<R>) << d.n);
    LaunchScope ls(ctx, "small_batch", bytes);
    hipLaunchKernelGGL(k_small_batch<R>, dim3(grid), dim3(SMALL_TPB), lds, ctx->stream,
                       (const DevCirc *)(base + o_c), nc, d_cnt, (const DevOp<R> *)(base + o_ops),
                       (const DevStage *)(base + o_stg), (const V2<R> *)(base + o_lt),
                       (const DevOp<R> *)(base + o_ovr),
                       (const DevTerm *)(base + o_t), (const int *)(base + o_gb), (const int *)(base + o_ge),
                       (const uint64_t *)(base + o_gx), (const double *)(base + o_cf), d_E, max_n, max_T);
    SV_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Batched expectation tile passes: read-only passes over a slab of states.
// Pass e holds the Pauli groups whose X/Y support lies inside its local
// bits; every workgroup reduces its tile's FP64 contribution to each of the
// pass's terms into partial[c][term slot][tile] (fixed order).
// ---------------------------------------------------------------------------

struct alignas(16) DevEPass {
    int32_t m, l, g_begin, g_end;
    int32_t hi_begin, part_off, pad0, pad1;
    uint64_t free_mask;
    uint64_t ntiles;
};

constexpr int EXPT_TPB = 256;
constexpr int EXPT_CHUNK = 8;

template <typename R>
__global__ __launch_bounds__(EXPT_TPB) void k_expect_tile(
    const V2<R> *__restrict__ slab, uint64_t dim, int nc, const DevEPass *__restrict__ eps, int e,
    const uint64_t *__restrict__ aux, const uint32_t *__restrict__ gxl, const int *__restrict__ gbeg,
    const int *__restrict__ gend, const DevTerm *__restrict__ terms, const int *__restrict__ tslot,
    uint64_t part_stride, double *__restrict__ partial) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[EXPT_TPB / 64];
    const DevEPass &P = eps[e];
    const int m = P.m, l = P.l;
    const uint32_t T = 1u << m, lowm = (1u << l) - 1;
    const uint32_t nhi = 1u << (m - l);
    V2<R> *tile = reinterpret_cast<V2<R> *>(smem);
    uint64_t *hi_off = reinterpret_cast<uint64_t *>(smem + (sizeof(V2<R>) << m));
    for (uint32_t h = threadIdx.x; h < nhi; h += EXPT_TPB) hi_off[h] = aux[P.hi_begin + h];
    __syncthreads();
    const uint64_t ntiles = P.ntiles, nw = (uint64_t)nc * ntiles;
    for (uint64_t w = blockIdx.x; w < nw; w += gridDim.x) {
        const uint64_t c = w / ntiles, t = w - c * ntiles;
        const uint64_t base = deposit(t, P.free_mask);
        const V2<R> *__restrict__ psi = slab + c * dim;
        for (uint32_t j = threadIdx.x; j < T; j += EXPT_TPB) tile[j] = psi[base | hi_off[j >> l] | (j & lowm)];
        __syncthreads();
        for (int g = P.g_begin; g < P.g_end; ++g) {
            const uint32_t xl = gxl[g];
            const int hb = xl ? 31 - __clz(xl) : -1;
            const uint32_t items = xl ? T / 2 : T;
            for (int t0 = gbeg[g]; t0 < gend[g]; t0 += EXPT_CHUNK) {
                const int cnt = min(EXPT_CHUNK, gend[g] - t0);
                double acc[EXPT_CHUNK];
#pragma unroll
                for (int q = 0; q < EXPT_CHUNK; ++q) acc[q] = 0.0;
                for (uint32_t it = threadIdx.x; it < items; it += EXPT_TPB) {
                    if (!xl) {
                        const V2<R> a = tile[it];
                        const uint64_t k = base | hi_off[it >> l] | (it & lowm);
                        const double pr = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
#pragma unroll
                        for (int q = 0; q < EXPT_CHUNK; ++q)
                            if (q < cnt) acc[q] += (__popcll(k & terms[t0 + q].z) & 1) ? -pr : pr;
                    } else {
                        const uint32_t j = ins0(it, hb), j2 = j ^ xl;
                        const V2<R> a = tile[j], b = tile[j2];
                        const uint64_t k = base | hi_off[j >> l] | (j & lowm);
                        const uint64_t k2 = base | hi_off[j2 >> l] | (j2 & lowm);
                        const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
                        const double pre = bx * ax + by * ay, pim = bx * ay - by * ax;
#pragma unroll
                        for (int q = 0; q < EXPT_CHUNK; ++q)
                            if (q < cnt) acc[q] += pair_contrib(pre, pim, k, k2, terms[t0 + q].z, terms[t0 + q].ny);
                    }
                }
#pragma unroll
                for (int q = 0; q < EXPT_CHUNK; ++q) {
                    if (q < cnt) {
                        const double sum = block_sum<EXPT_TPB>(acc[q], red);
                        if (threadIdx.x == 0)
                            partial[c * part_stride + P.part_off + (uint64_t)tslot[t0 + q] * ntiles + t] = sum;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// One workgroup per circuit: value[t] = sum of its partial row in order,
// E = (sum_t c_t value[t]) / value[T], written to E[out_slot[c]].
__global__ void k_expect_final(double *__restrict__ partial, uint64_t part_stride, int nc,
                               const int *__restrict__ t_off, const int *__restrict__ t_cnt, int T,
                               const double *__restrict__ coeffs, const int *__restrict__ out_slot,
                               double *__restrict__ E) {
    for (int c = blockIdx.x; c < nc; c += gridDim.x) {
        double *row = partial + (uint64_t)c * part_stride;
        for (int t = threadIdx.x; t <= T; t += blockDim.x) {
            double v = 0.0;
            for (int i = 0; i < t_cnt[t]; ++i) v += row[t_off[t] + i];
            row[t_off[t]] = v;
        }
        __threadfence_block();
        __syncthreads();
        if (threadIdx.x == 0) {
            double e = 0.0;
            for (int t = 0; t < T; ++t) e += coeffs[t] * row[t_off[t]];
            E[out_slot[c]] = e / row[t_off[T]];
        }
        __syncthreads();
    }
}

namespace {

// Expectation passes for a lowered Pauli sum: greedy cover of the X/Y
// supports by tile bit-sets that keep the low bits local.
struct EPlan {
    std::vector<DevEPass> eps;
    std::vector<uint64_t> aux;
    std::vector<uint32_t> gxl;
    std::vector<int> gbeg, gend, tslot;
    std::vector<DevTerm> terms;
    std::vector<int> t_off, t_cnt;  // per term index 0..T
    std::vector<double> coeffs;
    uint64_t part_stride = 0;
    int T = 0;
    bool ok = true;
};

EPlan make_eplan(int n, int m_max, const TermGroups &tg) {
    EPlan E;
    DevTerms dt = build_dev_terms(tg);
    E.T = dt.T;
    E.coeffs = dt.coeffs;
    const int m = std::min(m_max, n);
    const int l0 = std::min(5, m);
    const uint64_t low = (1ull << l0) - 1;
    const int G = (int)dt.gx.size();
    std::vector<int> order(G);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return __builtin_popcountll(dt.gx[a]) > __builtin_popcountll(dt.gx[b]);
    });
    std::vector<bool> done(G, false);
    int remaining = G;
    E.t_off.assign(E.T + 1, 0);
    E.t_cnt.assign(E.T + 1, 0);
    uint64_t part = 0;
    while (remaining > 0) {
        uint64_t S = low;
        std::vector<int> chosen;
        for (int g : order) {
            if (done[g]) continue;
            const uint64_t need = dt.gx[g] & ~S;
            if (__builtin_popcountll(S) + __builtin_popcountll(need) <= m) {
                S |= dt.gx[g];
                chosen.push_back(g);
            }
        }
        if (chosen.empty()) {
            // a support wider than the tile's free room: drop the low bits
            for (int g : order)
                if (!done[g]) {
                    if (__builtin_popcountll(dt.gx[g]) > m) {
                        E.ok = false;
                        return E;
                    }
                    S = dt.gx[g];
                    chosen.push_back(g);
                    break;
                }
        }
        for (int b = 0; b < n && __builtin_popcountll(S) < m; ++b) S |= 1ull << b;
        std::vector<int> local, freeb;
        int pos[64];
        for (int b = 0; b < n; ++b) {
            if (S & (1ull << b)) {
                pos[b] = (int)local.size();
                local.push_back(b);
            } else {
                pos[b] = -1;
                freeb.push_back(b);
            }
        }
        DevEPass ep;
        std::memset(&ep, 0, sizeof ep);
        ep.m = (int)local.size();
        int run = 0;
        while (run < ep.m && local[run] == run) ++run;
        ep.l = run;
        for (int b : freeb) ep.free_mask |= 1ull << b;
        ep.ntiles = 1ull << freeb.size();
        ep.hi_begin = (int)E.aux.size();
        for (uint32_t h = 0; h < (1u << (ep.m - ep.l)); ++h) {
            uint64_t o = 0;
            for (int i = 0; i < ep.m - ep.l; ++i)
                if ((h >> i) & 1) o |= 1ull << local[ep.l + i];
            E.aux.push_back(o);
        }
        ep.g_begin = (int)E.gxl.size();
        ep.part_off = (int)part;
        int slot = 0;
        for (int g : chosen) {
            done[g] = true;
            --remaining;
            uint32_t xl = 0;
            for (int b = 0; b < n; ++b)
                if (dt.gx[g] & (1ull << b)) xl |= 1u << pos[b];
            E.gxl.push_back(xl);
            E.gbeg.push_back((int)E.terms.size());
            for (int t = dt.gbeg[g]; t < dt.gend[g]; ++t) {
                E.terms.push_back(dt.terms[t]);
                E.tslot.push_back(slot);
                E.t_off[dt.terms[t].idx] = (int)(part + (uint64_t)slot * ep.ntiles);
                E.t_cnt[dt.terms[t].idx] = (int)ep.ntiles;
                ++slot;
            }
            E.gend.push_back((int)E.terms.size());
        }
        ep.g_end = (int)E.gxl.size();
        part += (uint64_t)slot * ep.ntiles;
        E.eps.push_back(ep);
    }
    E.part_stride = part;
    return E;
}

// Circuits too large for one workgroup, batched: one plan per (op set,
// Hamiltonian); per pass one launch over all (circuit, tile) items of a
// chunk of circuits held in a slab; then the batched expectation passes.
template <typename R>
void run_large_batched(Ctx *ctx, const BatchSpec &spec, const std::vector<int> &idx, double *d_E,
                       std::vector<int> &fallback) {
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int c : idx) groups[{spec.circuits[c].op_set, spec.circuits[c].ham}].push_back(c);
    for (auto &kv : groups) {
        const std::vector<int> &cs = kv.second;
        const int n = spec.circuits[cs[0]].n;
        PlanOptions po;
        po.tile_bits = spec.dtype == SV_C64 ? ctx->tile_bits_c64 : ctx->tile_bits_c128;
        po.perm_bits = spec.dtype == SV_C64 ? 12 : 11;
        const std::vector<Op> &ops = spec.op_sets[kv.first.first];
        Plan plan = make_plan(n, ops, po);
        EPlan E = make_eplan(n, po.tile_bits, spec.hams[kv.first.second]);
        bool plan_ok = !plan.passes.empty() && plan.passes[0].kind == PASS_TILE;
        for (const Pass &ps : plan.passes) plan_ok = plan_ok && ps.kind != PASS_SWEEP;
        if (!E.ok || !plan_ok) {
            fallback.insert(fallback.end(), cs.begin(), cs.end());
            continue;
        }
        DevPlanHost<R> h = build_dev_plan<R>(plan);
        DevPlanDev<R> d = upload_dev_plan<R>(ctx, h, "mp_plan");
        std::map<int, int> dop_of_gate;
        for (size_t i = 0; i < h.gate.size(); ++i)
            if (h.gate[i] >= 0) dop_of_gate[h.gate[i]] = (int)i;
        // expectation metadata (one upload)
        Blob eb;
        const size_t o_ep = eb.add(E.eps.data(), E.eps.size() * sizeof(DevEPass));
        const size_t o_aux = eb.add(E.aux.data(), E.aux.size() * 8);
        const size_t o_gxl = eb.add(E.gxl.data(), E.gxl.size() * 4);
        const size_t o_gb = eb.add(E.gbeg.data(), E.gbeg.size() * 4);
        const size_t o_ge = eb.add(E.gend.data(), E.gend.size() * 4);
        const size_t o_t = eb.add(E.terms.data(), E.terms.size() * sizeof(DevTerm));
        const size_t o_ts = eb.add(E.tslot.data(), E.tslot.size() * 4);
        const size_t o_to = eb.add(E.t_off.data(), E.t_off.size() * 4);
        const size_t o_tc = eb.add(E.t_cnt.data(), E.t_cnt.size() * 4);
        const size_t o_cf = eb.add(E.coeffs.data(), E.coeffs.size() * 8);
        char *ebase = (char *)scratch(ctx, "mp_eplan", eb.host.size());
        upload(ctx, ebase, eb.host.data(), eb.host.size());
        // chunks of circuits whose states fit the slab budget
        const uint64_t dim = 1ull << n;
        const size_t sbytes = sizeof(V2<R>) * dim;
        const size_t budget = (size_t)16 << 30, pbudget = (size_t)2 << 30;
        const size_t pbytes = 8 * E.part_stride;
        const int chunk = (int)std::max<size_t>(
            1, std::min<size_t>(cs.size(), std::min(budget / sbytes, pbudget / std::max<size_t>(pbytes, 1))));
        V2<R> *slab = (V2<R> *)scratch(ctx, "mp_slab", sbytes * chunk);
        double *part = (double *)scratch(ctx, "mp_partial", 8 * E.part_stride * chunk + 64);
        for (size_t c0 = 0; c0 < cs.size(); c0 += chunk) {
            const int nc = (int)std::min<size_t>(chunk, cs.size() - c0);
            std::vector<int> oidx(nc, -1), oslot(nc);
            std::vector<DevOp<R>> ovr(nc);
            for (int c = 0; c < nc; ++c) {
                const BatchCircuit &bc = spec.circuits[cs[c0 + c]];
                oslot[c] = bc.out_slot >= 0 ? bc.out_slot : cs[c0 + c];
                std::memset(&ovr[c], 0, sizeof(DevOp<R>));
                if (bc.ovr_index < 0) continue;
                auto it = dop_of_gate.find(bc.ovr_index);
                if (it == dop_of_gate.end()) fail(SV_EDEVICE, "internal: shifted gate not found in the plan");
                const DevOp<R> &bp = h.dops[it->second];
                DevOp<R> o = to_dev<R>(bc.ovr_op);
                // same gate and qubits: keep the base op's placement in the plan
                o.kind = bp.kind;
                o.a = bp.a;
                o.b = bp.b;
                o.la = bp.la;
                o.lb = bp.lb;
                o.ra = bp.ra;
                o.rb = bp.rb;
                o.tslot = bp.tslot;
                o.tab = bp.tab;
                o.cmask = bp.cmask;
                o.lcmask = bp.lcmask;
                o.gcmask = bp.gcmask;
                o.lmask = bp.lmask;
                ovr[c] = o;
                oidx[c] = it->second;
            }
            Blob ob;
            const size_t o_oi = ob.add(oidx.data(), nc * 4);
            const size_t o_ov = ob.add(ovr.data(), nc * sizeof(DevOp<R>));
            const size_t o_os = ob.add(oslot.data(), nc * 4);
            char *obase = (char *)scratch(ctx, "mp_ovr", ob.host.size());
            upload(ctx, obase, ob.host.data(), ob.host.size());
            launch_plan<R>(ctx, plan, h, d, slab, dim, nc, (const int *)(obase + o_oi),
                           (const DevOp<R> *)(obase + o_ov), true);
            for (size_t e = 0; e < E.eps.size(); ++e) {
                const DevEPass &ep = E.eps[e];
                const size_t lds = (sizeof(V2<R>) << ep.m) + 8 * (1u << (ep.m - ep.l));
                set_lds_limit((const void *)k_expect_tile<R>, lds);
                const unsigned grid =
                    (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ep.ntiles * nc, (uint64_t)ctx->cu_count * 8));
                LaunchScope ls(ctx, "expect_tile", (double)sbytes * nc);
                hipLaunchKernelGGL(k_expect_tile<R>, dim3(grid), dim3(EXPT_TPB), lds, ctx->stream, slab, dim, nc,
                                   (const DevEPass *)(ebase + o_ep), (int)e, (const uint64_t *)(ebase + o_aux),
                                   (const uint32_t *)(ebase + o_gxl), (const int *)(ebase + o_gb),
                                   (const int *)(ebase + o_ge), (const DevTerm *)(ebase + o_t),
                                   (const int *)(ebase + o_ts), E.part_stride, part);
                SV_HIP(hipGetLastError());
            }
            hipLaunchKernelGGL(k_expect_final, dim3(std::min(nc, ctx->cu_count * 4)), dim3(256), 0, ctx->stream, part,
                               E.part_stride, nc, (const int *)(ebase + o_to), (const int *)(ebase + o_tc), E.T,
                               (const double *)(ebase + o_cf), (const int *)(obase + o_os), d_E);
            SV_HIP(hipGetLastError());
        }
    }
}

}  // namespace

// Large circuits: one at a time through the pass executor.
void run_large_sequential(Ctx *ctx, const BatchSpec &spec, const std::vector<int> &idx, uint32_t flags,
                          double *d_E) {
    if (idx.empty()) return;
    int max_n = 0;
    for (int c : idx) max_n = std::max(max_n, spec.circuits[c].n);
    const size_t amp = spec.dtype == SV_C64 ? 8 : 16;
    void *buf = scratch(ctx, "batch_state", amp << max_n);
    std::vector<DevTerms> dts(spec.hams.size());
    std::vector<bool> have(spec.hams.size(), false);
    for (int c : idx) {
        const BatchCircuit &bc = spec.circuits[c];
        State st;
        st.ctx = ctx;
        st.n = bc.n;
        st.dtype = spec.dtype;
        st.ptr = buf;
        st.owned = false;
        set_zero_state(ctx, buf, bc.n, spec.dtype);
        std::vector<Op> ops = spec.op_sets[bc.op_set];
        if (bc.ovr_index >= 0) ops[bc.ovr_index] = bc.ovr_op;
        if (flags & SV_FLAG_UNFUSED) {
            run_unfused(ctx, &st, ops);
        } else {
            PlanOptions po;
            po.tile_bits = spec.dtype == SV_C64 ? ctx->tile_bits_c64 : ctx->tile_bits_c128;
            po.perm_bits = spec.dtype == SV_C64 ? 12 : 11;
            run_plan(ctx, &st, make_plan(bc.n, ops, po));
        }
        if (!have[bc.ham]) {
            dts[bc.ham] = build_dev_terms(spec.hams[bc.ham]);
            have[bc.ham] = true;
        }
        expectation_dev(ctx, buf, bc.n, spec.dtype, dts[bc.ham], d_E + (bc.out_slot >= 0 ? bc.out_slot : c),
                        nullptr);
    }
}

}  // namespace

void run_batch_dev(Ctx *ctx, const BatchSpec &spec, uint32_t flags, double *d_E) {
    const int nc = (int)spec.circuits.size();
    std::vector<int> small, large;
    const int smax = small_batch_max_qubits(spec.dtype);
    const bool sequential = (flags & (SV_FLAG_SEQUENTIAL | SV_FLAG_UNFUSED)) != 0;
    for (int c = 0; c < nc; ++c) {
        const BatchCircuit &bc = spec.circuits[c];
        const size_t vals = 8 * (spec.hams[bc.ham].terms.size() + 1);
        if (!sequential && bc.n <= smax && vals <= SMALL_VALS_MAX) small.push_back(c);
        else large.push_back(c);
    }
    if (spec.dtype == SV_C64) launch_small<float>(ctx, spec, small, d_E);
    else launch_small<double>(ctx, spec, small, d_E);
    if (sequential) {
        run_large_sequential(ctx, spec, large, flags, d_E);
    } else {
        std::vector<int> fallback;
        if (spec.dtype == SV_C64) run_large_batched<float>(ctx, spec, large, d_E, fallback);
        else run_large_batched<double>(ctx, spec, large, d_E, fallback);
        run_large_sequential(ctx, spec, fallback, flags, d_E);
    }
}

void combine_dev(Ctx *ctx, const double *d_E, const std::vector<int> &beg, const std::vector<int> &circ,
                 const std::vector<double> &w, double *d_grad) {
    const int np = beg.empty() ? 0 : (int)beg.size() - 1;
    if (np <= 0) return;
    Blob blob;
    const size_t o_b = blob.add(beg.data(), beg.size() * 4);
    const size_t o_c = blob.add(circ.data(), circ.size() * 4);
    const size_t o_w = blob.add(w.data(), w.size() * 8);
    char *base = (char *)scratch(ctx, "comb", blob.host.size());
    upload(ctx, base, blob.host.data(), blob.host.size());
    hipLaunchKernelGGL(k_combine, dim3((np + 255) / 256), dim3(256), 0, ctx->stream, d_E,
                       (const int *)(base + o_b), (const int *)(base + o_c), (const double *)(base + o_w), np,
                       d_grad);
    SV_HIP(hipGetLastError());
}

void run_batch(Ctx *ctx, const BatchSpec &spec, uint32_t flags, std::vector<double> &E,
               std::vector<double> &grad) {
    const int nc = (int)spec.circuits.size();
    const int np = spec.comb_begin.empty() ? 0 : (int)spec.comb_begin.size() - 1;
    double *d_E = (double *)scratch(ctx, "batch_E", (size_t)(std::max(nc, 1) + np) * 8);
    run_batch_dev(ctx, spec, flags, d_E);
    grad.assign(np, 0.0);
    if (np > 0) {
        combine_dev(ctx, d_E, spec.comb_begin, spec.comb_circ, spec.comb_w, d_E + nc);
        SV_HIP(hipMemcpyAsync(grad.data(), d_E + nc, (size_t)np * 8, hipMemcpyDeviceToHost, ctx->stream));
    }
    E.assign(nc, 0.0);
    if (nc) SV_HIP(hipMemcpyAsync(E.data(), d_E, (size_t)nc * 8, hipMemcpyDeviceToHost, ctx->stream));
    SV_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->profile) profile_collect(ctx);
}

}  // namespace sv
