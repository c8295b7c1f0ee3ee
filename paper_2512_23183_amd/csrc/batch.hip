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
    int32_t ovr_slot, ch_begin, ch_end, T;   // term chunks [ch_begin, ch_end)
    int32_t coeff_begin, out_slot, stage_begin, stage_end;
    int32_t paux_begin, paux_end, pad[2];    // the op set's layout-map tables
};

// LDS copy of one circuit's ops, stages and layout-map tables (offsets in
// bytes within the cache; counts are the maxima over the batch's op sets).
struct SmallCache {
    uint32_t ops, ovr, stages, paux, end;
};
template <typename R>
__host__ __device__ inline SmallCache small_cache_layout(uint32_t base, int max_ops, int max_stages, int max_paux) {
    auto al = [](uint32_t x) { return (x + 15u) & ~15u; };
    SmallCache c;
    c.ops = al(base);
    c.ovr = c.ops + al((uint32_t)sizeof(DevOp<R>) * (uint32_t)max_ops);
    c.stages = c.ovr + al((uint32_t)sizeof(DevOp<R>));
    c.paux = c.stages + al((uint32_t)sizeof(DevStage) * (uint32_t)max_stages);
    c.end = c.paux + al(4u * (uint32_t)max_paux);
    return c;
}

// Copy n16 16-byte words (all threads of the workgroup).
__device__ __forceinline__ void lds_copy16(void *dst, const void *src, uint32_t n16) {
    typedef uint32_t w4 __attribute__((ext_vector_type(4)));
    w4 *d = reinterpret_cast<w4 *>(dst);
    const w4 *s = reinterpret_cast<const w4 *>(src);
    for (uint32_t i = threadIdx.x; i < n16; i += blockDim.x) d[i] = s[i];
}

// Pauli terms of the small-circuit path in chunks of <= ESUM_CHUNK terms
// that share an X/Y support x (local = global bits) and the part (Re / Im)
// of conj(psi[k ^ x]) psi[k] they use: mode 0 diagonal, 1 Re, 2 Im.
struct alignas(16) SChunk {
    uint32_t x;
    int32_t mode, tbeg, tend;
};
struct alignas(16) STerm {
    uint32_t z;
    int32_t idx;   // value slot (term index; T = norm)
    int32_t neg;   // i^ny sign: ny mod 4 in {1, 2}
    int32_t diag;  // x = 0: no pair factor 2
};

constexpr int SMALL_TPB = 256;

int small_batch_max_qubits(int dtype) { return dtype == SV_C64 ? 13 : 12; }

__global__ void k_fill_u32(unsigned *p, unsigned v, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// LDS: state[2^max_n], red[TPB/64], vals[max_T + 1], then (cache != 0) a
// copy of the current circuit's ops, shifted op, stages and layout-map
// tables.  A circuit is a chain of dependent steps run by one workgroup; with
// its ops in LDS each step reads them at LDS latency instead of a cache miss
// to L2 per op.  Ladder tables are read from global memory.
template <typename R>
__global__ __launch_bounds__(SMALL_TPB) void k_small_batch(
    const DevCirc *__restrict__ circ, int ncirc, unsigned *__restrict__ counter,
    const DevOp<R> *__restrict__ ops, const DevStage *__restrict__ stages, const V2<R> *__restrict__ ltab,
    const uint32_t *__restrict__ paux, const DevOp<R> *__restrict__ ovr_ops,
    const SChunk *__restrict__ chunks, const STerm *__restrict__ sterms, const double *__restrict__ coeffs,
    double *__restrict__ energies, int max_n, int max_T, int cache, int max_ops, int max_stages, int max_paux) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cur;
    V2<R> *st = reinterpret_cast<V2<R> *>(smem);
    double *red = reinterpret_cast<double *>(smem + (sizeof(V2<R>) << max_n));
    double *vals = red + SMALL_TPB / 64;
    const SmallCache lay = small_cache_layout<R>((uint32_t)((sizeof(V2<R>) << max_n) + 8 * (SMALL_TPB / 64) +
                                                            8 * ((max_T + 2) & ~1)),
                                                 max_ops, max_stages, max_paux);
    DevOp<R> *c_ops = reinterpret_cast<DevOp<R> *>(smem + lay.ops);
    DevOp<R> *c_ovr = reinterpret_cast<DevOp<R> *>(smem + lay.ovr);
    DevStage *c_st = reinterpret_cast<DevStage *>(smem + lay.stages);
    uint32_t *c_paux = reinterpret_cast<uint32_t *>(smem + lay.paux);
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
        tc.paux = paux;
        tc.pauxl = nullptr;
        tc.paux_off = 0;
        tc.mtab = nullptr;
        tc.scale = (R)1;
        tc.scaled = false;
        tc.base = 0;
        tc.hi_off = nullptr;
        tc.ltl = nullptr;
        tc.ltabs = ltab;
        tc.Gs = nullptr;
        ladder_split(n, tc.lsa, tc.lsb);
        if (cache) {
            // ops, stages and tables of this circuit, renumbered from 0
            const int nops = C.op_end - C.op_begin, nst = C.stage_end - C.stage_begin;
            lds_copy16(c_ops, ops + C.op_begin, (uint32_t)(nops * sizeof(DevOp<R>) / 16));
            if (C.ovr_index >= 0) lds_copy16(c_ovr, ovr_ops + C.ovr_slot, (uint32_t)(sizeof(DevOp<R>) / 16));
            for (int i = threadIdx.x; i < C.paux_end - C.paux_begin; i += SMALL_TPB) c_paux[i] = paux[C.paux_begin + i];
            for (int i = threadIdx.x; i < nst; i += SMALL_TPB) {
                DevStage S = stages[C.stage_begin + i];
                S.op_begin -= C.op_begin;
                S.op_end -= C.op_begin;
                S.perm_tab -= C.paux_begin;
                c_st[i] = S;
            }
            tc.paux = c_paux;
            __syncthreads();
            run_stages<R, SMALL_TPB>(st, nullptr, tc, c_st, 0, nst, c_ops,
                                     C.ovr_index >= 0 ? C.ovr_index - C.op_begin : -1, c_ovr);
        } else {
            __syncthreads();
            run_stages<R, SMALL_TPB>(st, nullptr, tc, stages, C.stage_begin, C.stage_end, ops, C.ovr_index,
                                     ovr_ops + C.ovr_slot);
        }
        // one wave per chunk of terms; each term's value has one writer
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const uint32_t lane = threadIdx.x & 63;
        for (int ch = C.ch_begin + wave; ch < C.ch_end; ch += SMALL_TPB / 64) {
            const SChunk K = chunks[ch];
            const int cnt = K.tend - K.tbeg;
            uint32_t zl[ESUM_CHUNK];
            double acc[ESUM_CHUNK];
#pragma unroll
            for (int q = 0; q < ESUM_CHUNK; ++q) {
                zl[q] = q < cnt ? sterms[K.tbeg + q].z : 0u;
                acc[q] = 0.0;
            }
            esum_dispatch<R>(st, N, K.x, K.mode, cnt, zl, acc, lane);
#pragma unroll
            for (int q = 0; q < ESUM_CHUNK; ++q) {
                if (q < cnt) {
                    const double sum = wave_sum(acc[q]);
                    if (lane == 0) {
                        const STerm &tm = sterms[K.tbeg + q];
                        const double v = tm.diag ? sum : 2.0 * sum;
                        vals[tm.idx] = tm.neg ? -v : v;
                    }
                }
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
    std::vector<SChunk> chunks;
    std::vector<STerm> sterms;
    std::vector<double> coeffs;
    std::vector<DevCirc> circ;
    std::vector<DevOp<R>> ovr;
    std::vector<DevStage> stages;
    std::vector<V2<R>> ltab;
    std::vector<uint32_t> paux;
    std::vector<int> set_sb(spec.op_sets.size(), -1), set_se(spec.op_sets.size(), -1);
    std::vector<int> set_pb(spec.op_sets.size(), 0), set_pe(spec.op_sets.size(), 0);
    int max_n = 3, max_T = 0, max_ops = 0, max_stages = 0, max_paux = 0;
    for (int c : idx) {
        const BatchCircuit &bc = spec.circuits[c];
        // states of fewer than 3 qubits run as 3-qubit states whose extra
        // (most significant) bits stay |0>: energies are unchanged
        const int n_eff = std::max(bc.n, 3);
        if (set_begin[bc.op_set] < 0) {
            set_begin[bc.op_set] = (int)dops.size();
            std::vector<int> loc(all_local.begin(), all_local.begin() + n_eff);
            for (const Op &op : spec.op_sets[bc.op_set]) {
                DevOp<R> d = to_dev<R>(op);
                d.flags &= ~OPF_SCALED;  // no pass scale here: ops apply their full matrix
                localise(d, loc);
                if (op.kind == OP_LADDER) append_ladder_tables<R>(d, op, loc, ltab);  // read from global memory
                dops.push_back(d);
            }
            set_end[bc.op_set] = (int)dops.size();
            set_sb[bc.op_set] = (int)stages.size();
            set_pb[bc.op_set] = (int)paux.size();
            build_stages<R>(dops, set_begin[bc.op_set], set_end[bc.op_set], loc, stages, paux, false);
            set_se[bc.op_set] = (int)stages.size();
            set_pe[bc.op_set] = (int)paux.size();
            max_ops = std::max(max_ops, set_end[bc.op_set] - set_begin[bc.op_set]);
            max_stages = std::max(max_stages, set_se[bc.op_set] - set_sb[bc.op_set]);
            max_paux = std::max(max_paux, set_pe[bc.op_set] - set_pb[bc.op_set]);
        }
        if (ham_gb[bc.ham] < 0) {
            DevTerms dt = build_dev_terms(spec.hams[bc.ham]);
            ham_gb[bc.ham] = (int)chunks.size();
            for (size_t g = 0; g < dt.gx.size(); ++g) {
                const uint32_t x = (uint32_t)dt.gx[g];
                for (int pim = 0; pim < 2; ++pim) {
                    std::vector<int> ts;
                    for (int t = dt.gbeg[g]; t < dt.gend[g]; ++t)
                        if (x != 0 ? (dt.terms[t].ny & 1) == pim : pim == 0) ts.push_back(t);
                    for (size_t i = 0; i < ts.size(); i += ESUM_CHUNK) {
                        SChunk K;
                        K.x = x;
                        K.mode = x == 0 ? 0 : (pim ? 2 : 1);
                        K.tbeg = (int)sterms.size();
                        for (size_t k = i; k < std::min(ts.size(), i + ESUM_CHUNK); ++k) {
                            const DevTerm &d = dt.terms[ts[k]];
                            STerm st;
                            st.z = (uint32_t)d.z;
                            st.idx = d.idx;
                            st.neg = x != 0 && (d.ny == 1 || d.ny == 2);
                            st.diag = x == 0;
                            sterms.push_back(st);
                        }
                        K.tend = (int)sterms.size();
                        chunks.push_back(K);
                    }
                }
            }
            ham_ge[bc.ham] = (int)chunks.size();
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
        d.paux_begin = set_pb[bc.op_set];
        d.paux_end = set_pe[bc.op_set];
        d.ovr_index = -1;
        d.ovr_slot = 0;
        if (bc.ovr_index >= 0) {
            d.ovr_index = d.op_begin + bc.ovr_index;
            d.ovr_slot = (int)ovr.size();
            const DevOp<R> &basep = dops[d.ovr_index];
            DevOp<R> o = to_dev<R>(bc.ovr_op);
            o.flags &= ~OPF_SCALED;
            // same gate and qubits as the base op: reuse its placement
            o.la = basep.la;
            o.lb = basep.lb;
            o.ra = basep.ra;
            o.rb = basep.rb;
            o.tslot = basep.tslot;
            o.lcmask = basep.lcmask;
            o.gcmask = basep.gcmask;
            o.flags = (o.flags & ~OPF_PLACEMENT) | (basep.flags & OPF_PLACEMENT);
            ovr.push_back(o);
        }
        d.ch_begin = ham_gb[bc.ham];
        d.ch_end = ham_ge[bc.ham];
        d.T = ham_T[bc.ham];
        d.coeff_begin = ham_cb[bc.ham];
        d.out_slot = bc.out_slot >= 0 ? bc.out_slot : c;
        circ.push_back(d);
        max_n = std::max(max_n, n_eff);
        max_T = std::max(max_T, d.T);
    }
    if (ovr.empty()) ovr.resize(1);
    if (paux.empty()) paux.resize(1);
    // largest circuits first: better balance of the dynamic schedule
    std::stable_sort(circ.begin(), circ.end(), [](const DevCirc &a, const DevCirc &b) {
        return (a.op_end - a.op_begin) * (1ll << a.n) > (b.op_end - b.op_begin) * (1ll << b.n);
    });
    Blob blob;
    const size_t o_c = blob.add(circ.data(), circ.size() * sizeof(DevCirc));
    const size_t o_ops = blob.add(dops.data(), dops.size() * sizeof(DevOp<R>));
    const size_t o_stg = blob.add(stages.data(), stages.size() * sizeof(DevStage));
    const size_t o_lt = blob.add(ltab.data(), ltab.size() * sizeof(V2<R>));
    const size_t o_pa = blob.add(paux.data(), paux.size() * 4);
    const size_t o_ovr = blob.add(ovr.data(), ovr.size() * sizeof(DevOp<R>));
    const size_t o_ch = blob.add(chunks.data(), chunks.size() * sizeof(SChunk));
    const size_t o_st = blob.add(sterms.data(), sterms.size() * sizeof(STerm));
    const size_t o_cf = blob.add(coeffs.data(), coeffs.size() * 8);
    const size_t o_cnt = blob.add(nullptr, 16);
    char *base = (char *)scratch(ctx, "batch_small", blob.host.size());
    upload(ctx, base, blob.host.data(), blob.host.size());
    unsigned *d_cnt = (unsigned *)(base + o_cnt);
    const size_t lds0 = (sizeof(V2<R>) << max_n) + 8 * (SMALL_TPB / 64) + 8 * ((max_T + 2) & ~1);
    // the circuit's ops in LDS when they fit beside the state
    const SmallCache cl = small_cache_layout<R>((uint32_t)lds0, max_ops, max_stages, max_paux);
    const int cache = cl.end <= 96u * 1024u ? 1 : 0;
    const size_t lds = cache ? cl.end : lds0;
    set_lds_limit((const void *)k_small_batch<R>, lds);
    const int nc = (int)circ.size();
    const int per_cu = lds <= 40 * 1024 ? 4 : lds <= 80 * 1024 ? 2 : 1;
    const int grid = std::max(1, std::min(nc, ctx->cu_count * per_cu));
    double bytes = 0;
    for (const DevCirc &d : circ) bytes += (double)(sizeof(V2<R>) << d.n);
    launch_or_record(ctx, [=] {
        // the work counter is cleared by a kernel (graph-safe, no memset node)
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, ctx->stream, d_cnt, 0u, 1);
        LaunchScope ls(ctx, "small_batch", bytes);
        hipLaunchKernelGGL(k_small_batch<R>, dim3(grid), dim3(SMALL_TPB), lds, ctx->stream,
                           (const DevCirc *)(base + o_c), nc, d_cnt, (const DevOp<R> *)(base + o_ops),
                           (const DevStage *)(base + o_stg), (const V2<R> *)(base + o_lt),
                           (const uint32_t *)(base + o_pa), (const DevOp<R> *)(base + o_ovr),
                           (const SChunk *)(base + o_ch), (const STerm *)(base + o_st),
                           (const double *)(base + o_cf), d_E, max_n, max_T, cache, max_ops, max_stages,
                           max_paux);
        SV_HIP(hipGetLastError());
    });
}

namespace {

// Circuits too large for one workgroup, batched: one plan per (op set,
// Hamiltonian); per pass one launch over all (circuit, tile) items of a
// chunk of circuits held in a slab; then the batched expectation passes.
// Everything is planned and uploaded first (one scratch slot per group and
// chunk, the slab and the partial sums sized once for the largest group),
// so the launches can be recorded and replayed as one graph.
template <typename R>
struct LargeGroup {
    std::vector<int> cs;
    Plan plan;
    EPlanHost E;
    DevPlanHost<R> h;
    int chunk = 1;
};

template <typename R>
void run_large_batched(Ctx *ctx, const BatchSpec &spec, const std::vector<int> &idx, double *d_E,
                       std::vector<int> &fallback) {
    std::map<std::pair<int, int>, std::vector<int>> by_key;
    for (int c : idx) by_key[{spec.circuits[c].op_set, spec.circuits[c].ham}].push_back(c);
    std::vector<std::shared_ptr<LargeGroup<R>>> groups;
    size_t slab_bytes = 0, part_bytes = 0;
    for (auto &kv : by_key) {
        auto G = std::make_shared<LargeGroup<R>>();
        G->cs = kv.second;
        const int n = spec.circuits[G->cs[0]].n;
        PlanOptions po;
        po.tile_bits = ctx->tile_bits[spec.dtype];
        po.tile_bits_layers = ctx->tile_bits_layers[spec.dtype];
        po.perm_bits = ctx->perm_bits[spec.dtype];
        G->plan = make_plan(n, spec.op_sets[kv.first.first], po);
        G->E = make_eplan(n, expect_tile_bits(ctx, spec.dtype), build_dev_terms(spec.hams[kv.first.second]));
        bool plan_ok = !G->plan.passes.empty() && G->plan.passes[0].kind == PASS_TILE;
        for (const Pass &ps : G->plan.passes) plan_ok = plan_ok && ps.kind != PASS_SWEEP;
        if (!G->E.ok || !plan_ok) {
            fallback.insert(fallback.end(), G->cs.begin(), G->cs.end());
            continue;
        }
        G->h = build_dev_plan<R>(G->plan);
        // chunks of circuits whose states fit the slab budget
        const size_t sbytes = sizeof(V2<R>) << n;
        const size_t budget = (size_t)16 << 30, pbudget = (size_t)2 << 30;
        const size_t pbytes = 8 * std::max<uint64_t>(1, G->E.part_stride);
        G->chunk = (int)std::max<size_t>(
            1, std::min<size_t>(G->cs.size(), std::min(budget / sbytes, pbudget / pbytes)));
        slab_bytes = std::max(slab_bytes, sbytes * G->chunk);
        part_bytes = std::max(part_bytes, pbytes * G->chunk);
        groups.push_back(G);
    }
    if (groups.empty()) return;
    V2<R> *slab = (V2<R> *)scratch(ctx, "mp_slab", slab_bytes);
    double *part = (double *)scratch(ctx, "mp_partial", part_bytes);
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        std::shared_ptr<LargeGroup<R>> G = groups[gi];
        const std::string tag = "#" + std::to_string(gi);
        const DevPlanDev<R> d = upload_dev_plan<R>(ctx, G->h, "mp_plan" + tag);
        const EPlanDev ed = upload_eplan(ctx, G->E, "mp_eplan" + tag);
        std::map<int, int> dop_of_gate;
        for (size_t i = 0; i < G->h.gate.size(); ++i)
            if (G->h.gate[i] >= 0) dop_of_gate[G->h.gate[i]] = (int)i;
        // tile pass holding each plan op
        std::vector<int> pass_of_op(G->h.dops.size(), -1);
        for (size_t i = 0; i < G->plan.passes.size(); ++i)
            if (G->plan.passes[i].kind == PASS_TILE)
                for (int o = G->h.dpass[i].op_begin; o < G->h.dpass[i].op_end; ++o) pass_of_op[o] = (int)i;
        const int npass = (int)G->plan.passes.size();
        const std::vector<int> &cs = G->cs;
        const uint64_t dim = 1ull << G->plan.n;
        for (size_t c0 = 0; c0 < cs.size(); c0 += G->chunk) {
            const int nc = (int)std::min<size_t>(G->chunk, cs.size() - c0);
            std::vector<int> oidx(nc, -1), oslot(nc);
            std::vector<DevOp<R>> ovr(nc);
            for (int c = 0; c < nc; ++c) {
                const BatchCircuit &bc = spec.circuits[cs[c0 + c]];
                oslot[c] = bc.out_slot >= 0 ? bc.out_slot : cs[c0 + c];
                std::memset(&ovr[c], 0, sizeof(DevOp<R>));
                if (bc.ovr_index < 0) continue;
                auto it = dop_of_gate.find(bc.ovr_index);
                if (it == dop_of_gate.end()) fail(SV_EDEVICE, "internal: shifted gate not found in the plan");
                const DevOp<R> &bp = G->h.dops[it->second];
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
                o.flags = (o.flags & ~OPF_PLACEMENT) | (bp.flags & OPF_PLACEMENT);
                // the scale of its pass with o in place of the base op, in
                // the order build_dev_plan multiplies the factors
                o.pscale = 1.0;
                const int pi = pass_of_op[it->second];
                if (pi >= 0)
                    for (int q = G->h.dpass[pi].op_begin; q < G->h.dpass[pi].op_end; ++q) {
                        const DevOp<R> &oq = q == it->second ? o : G->h.dops[q];
                        if (oq.flags & OPF_SCALED) o.pscale *= oq.sfac;
                    }
                ovr[c] = o;
                oidx[c] = it->second;
            }
            // Shared prefixes: every circuit of a group runs the same ops
            // except its one shifted op, so before the pass that holds that
            // op its state equals the unshifted circuit's.  With an unshifted
            // circuit in the chunk, it goes first in the slab and the others
            // follow by the pass of their shifted op; a circuit joins at that
            // pass with a copy of the first one's state (bitwise the state it
            // would have computed itself) and skips the passes before it.
            std::vector<int> nc_pass;
            {
                int ref = -1;
                for (int c = 0; c < nc && ref < 0; ++c)
                    if (oidx[c] < 0) ref = c;
                if (ref >= 0 && npass > 1) {
                    std::vector<int> start(nc, 0);
                    for (int c = 0; c < nc; ++c) start[c] = oidx[c] < 0 ? 0 : std::max(0, pass_of_op[oidx[c]]);
                    std::vector<int> order;
                    order.reserve(nc);
                    order.push_back(ref);
                    for (int c = 0; c < nc; ++c)
                        if (c != ref) order.push_back(c);
                    std::stable_sort(order.begin() + 1, order.end(),
                                     [&](int a, int b) { return start[a] < start[b]; });
                    std::vector<int> oi2(nc), os2(nc);
                    std::vector<DevOp<R>> ov2(nc);
                    for (int k = 0; k < nc; ++k) {
                        oi2[k] = oidx[order[k]];
                        os2[k] = oslot[order[k]];
                        ov2[k] = ovr[order[k]];
                    }
                    oidx.swap(oi2);
                    oslot.swap(os2);
                    ovr.swap(ov2);
                    nc_pass.assign(npass, 0);
                    for (int k = 0; k < nc; ++k)
                        for (int i = start[order[k]]; i < npass; ++i) ++nc_pass[i];
                }
            }
            Blob ob;
            const size_t o_oi = ob.add(oidx.data(), nc * 4);
            const size_t o_ov = ob.add(ovr.data(), nc * sizeof(DevOp<R>));
            const size_t o_os = ob.add(oslot.data(), nc * 4);
            char *obase = (char *)scratch(ctx, "mp_ovr" + tag + "." + std::to_string(c0), ob.host.size());
            upload(ctx, obase, ob.host.data(), ob.host.size());
            launch_or_record(ctx, [=] {
                launch_plan<R>(ctx, G->plan, G->h, d, slab, dim, nc, (const int *)(obase + o_oi),
                               (const DevOp<R> *)(obase + o_ov), true, nc_pass.empty() ? nullptr : nc_pass.data());
                launch_expect<R>(ctx, G->E, ed, slab, dim, nc, part, (const int *)(obase + o_os), d_E, nullptr);
            });
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
            po.tile_bits = ctx->tile_bits[spec.dtype];
            po.tile_bits_layers = ctx->tile_bits_layers[spec.dtype];
            po.perm_bits = ctx->perm_bits[spec.dtype];
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

void run_batch_dev(Ctx *ctx, const BatchSpec &spec, uint32_t flags, double *d_E, double *d_grad) {
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
    const bool comb = d_grad && spec.comb_begin.size() > 1;
    if (sequential) {
        if (spec.dtype == SV_C64) launch_small<float>(ctx, spec, small, d_E);
        else launch_small<double>(ctx, spec, small, d_E);
        run_large_sequential(ctx, spec, large, flags, d_E);
        if (comb) combine_dev(ctx, d_E, spec.comb_begin, spec.comb_circ, spec.comb_w, d_grad);
        return;
    }
    // batched: uploads are enqueued now, launches are recorded and then run
    // as one graph (or directly when graphs are off or launches are timed)
    std::vector<std::function<void()>> work;
    const bool graph = ctx->graphs && !ctx->profile;
    if (graph) {
        ctx->record = &work;
        ctx->record_slots.clear();
    }
    std::vector<int> fallback;
    try {
        if (spec.dtype == SV_C64) launch_small<float>(ctx, spec, small, d_E);
        else launch_small<double>(ctx, spec, small, d_E);
        if (spec.dtype == SV_C64) run_large_batched<float>(ctx, spec, large, d_E, fallback);
        else run_large_batched<double>(ctx, spec, large, d_E, fallback);
        if (comb && fallback.empty()) combine_dev(ctx, d_E, spec.comb_begin, spec.comb_circ, spec.comb_w, d_grad);
    } catch (...) {
        ctx->record = nullptr;
        throw;
    }
    ctx->record = nullptr;
    if (graph) launch_recorded(ctx, work);
    // circuits the batched plan cannot take run one at a time afterwards
    run_large_sequential(ctx, spec, fallback, flags, d_E);
    if (comb && !fallback.empty()) combine_dev(ctx, d_E, spec.comb_begin, spec.comb_circ, spec.comb_w, d_grad);
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
    launch_or_record(ctx, [=] {
        hipLaunchKernelGGL(k_combine, dim3((np + 255) / 256), dim3(256), 0, ctx->stream, d_E,
                           (const int *)(base + o_b), (const int *)(base + o_c), (const double *)(base + o_w), np,
                           d_grad);
        SV_HIP(hipGetLastError());
    });
}

void run_batch(Ctx *ctx, const BatchSpec &spec, uint32_t flags, std::vector<double> &E,
               std::vector<double> &grad) {
    const int nc = (int)spec.circuits.size();
    const int np = spec.comb_begin.empty() ? 0 : (int)spec.comb_begin.size() - 1;
    double *d_E = (double *)scratch(ctx, "batch_E", (size_t)(std::max(nc, 1) + np) * 8);
    pinned_begin(ctx);
    try {
        run_batch_dev(ctx, spec, flags, d_E, np > 0 ? d_E + nc : nullptr);
    } catch (...) {
        (void)hipStreamSynchronize(ctx->stream);  // the arena may still feed copies
        pinned_end(ctx);
        throw;
    }
    // energies and gradient in one copy
    const size_t rb = (size_t)(nc + np) * 8;
    double *h = nullptr;
    if (ctx->pinned_on && ctx->pinned_used + rb <= ctx->pinned_cap) {
        h = reinterpret_cast<double *>(ctx->pinned + ctx->pinned_used);
        ctx->pinned_used += (rb + 255) & ~(size_t)255;
    }
    std::vector<double> hv;
    if (!h) {
        hv.resize(nc + np);
        h = hv.data();
    }
    if (rb) SV_HIP(hipMemcpyAsync(h, d_E, rb, hipMemcpyDeviceToHost, ctx->stream));
    const hipError_t se = hipStreamSynchronize(ctx->stream);
    pinned_end(ctx);
    SV_HIP(se);
    E.assign(h, h + nc);
    grad.assign(h + nc, h + nc + np);
    if (ctx->profile) profile_collect(ctx);
}

}  // namespace sv
