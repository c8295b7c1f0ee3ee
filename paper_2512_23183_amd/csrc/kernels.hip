// HIP kernels for gfx950 (wave64) and their host launchers.
//
//  * sweep kernels: one gate over the whole state, one launch per gate (the
//    plain path).  The loop runs over the reduced index space of the
//    amplitudes the gate actually touches (bit-mask loops of the paper's
//    direct state-vector gates): consecutive work-items map to consecutive
//    addresses on every bit above the target, so loads and stores of both
//    halves of a pair are coalesced.
//  * tile pass: one workgroup loads 2^m amplitudes (every index bit outside
//    the tile fixed) into LDS with coalesced runs over the low bits, applies
//    a list of ops in LDS and writes the tile back: one HBM round trip for
//    many gates.  Diagonal ops are evaluated from the global index and so may
//    touch any bit.
//  * permutation pass: in-place exchange of bit pairs (restores the layout
//    after the planner absorbed SWAP gates into a relabelling).
//  * expectation: stage 1 writes FP64 per-block partial sums per Pauli term
//    (amplitudes upcast to FP64 before any product); stage 2 reduces them in
//    a fixed order, so results are bitwise reproducible.
//  * small-state batch: one workgroup runs a whole circuit of <= 2^13
//    amplitudes in LDS and reduces its energy (parameter-shift batches).
#include <cstdio>

#include "device_common.h"

namespace sv {

// ---------------------------------------------------------------------------
// Sweep kernels (one gate per launch)
// ---------------------------------------------------------------------------

constexpr int SWEEP_TPB = 256;

enum SweepKind { SW_U1, SW_XPERM, SW_U2, SW_SWAP, SW_PHASE, SW_DIAG, SW_LADDER };
// How a thread reaches its amplitudes:
//  SWM_ONE   one amplitude per index (8 B complex64, 16 B complex128);
//  SWM_VEC2  complex64 with index bit 0 free: the thread takes reduced
//            indices 2t and 2t+1, whose amplitudes sit next to each other,
//            so every access is 16 bytes (two lanes' worth per load);
//  SWM_PAIR  complex64 one-qubit gate on bit 0: the pair (k, k+1) is one
//            16-byte access.
enum SweepMode { SWM_ONE, SWM_VEC2, SWM_PAIR };

template <typename R>
struct SweepArgs {
    DevOp<R> op;  // matrix entries (U1, U2, DIAG)
    V2<R> f;      // PHASE factor
    uint64_t flip, lmask;
    double turns;
    int a, b;
    uint64_t dim;  // amplitudes of the state (debug index checks)
};

constexpr int sweep_nidx(int kind) {
    return kind == SW_U2 ? 4 : (kind == SW_U1 || kind == SW_XPERM || kind == SW_SWAP) ? 2 : 1;
}

// Loads and stores of one amplitude (V2<R>) or of two adjacent complex64
// amplitudes; NT marks streaming accesses (data touched once per sweep).
template <bool NT, typename R>
__device__ __forceinline__ V2<R> sw_ld1(const V2<R> *p) {
    typedef R vec __attribute__((ext_vector_type(2)));
    const vec v = NT ? __builtin_nontemporal_load(reinterpret_cast<const vec *>(p)) : *reinterpret_cast<const vec *>(p);
    V2<R> r;
    r.x = v.x;
    r.y = v.y;
    return r;
}
template <bool NT, typename R>
__device__ __forceinline__ void sw_st1(V2<R> *p, V2<R> x) {
    typedef R vec __attribute__((ext_vector_type(2)));
    const vec v = {x.x, x.y};
    if (NT) __builtin_nontemporal_store(v, reinterpret_cast<vec *>(p));
    else *reinterpret_cast<vec *>(p) = v;
}
template <bool NT>
__device__ __forceinline__ void sw_ld2(const V2<float> *p, V2<float> &a, V2<float> &b) {
    typedef float vec __attribute__((ext_vector_type(4)));
    const vec v = NT ? __builtin_nontemporal_load(reinterpret_cast<const vec *>(p)) : *reinterpret_cast<const vec *>(p);
    a.x = v.x;
    a.y = v.y;
    b.x = v.z;
    b.y = v.w;
}
template <bool NT>
__device__ __forceinline__ void sw_st2(V2<float> *p, V2<float> a, V2<float> b) {
    typedef float vec __attribute__((ext_vector_type(4)));
    const vec v = {a.x, a.y, b.x, b.y};
    if (NT) __builtin_nontemporal_store(v, reinterpret_cast<vec *>(p));
    else *reinterpret_cast<vec *>(p) = v;
}

// The gate on the amplitudes of one index set (k = index of v[0]).
template <int KIND, typename R>
__device__ __forceinline__ void sweep_apply(V2<R> (&v)[sweep_nidx(KIND)], uint64_t k, const SweepArgs<R> &A) {
    if constexpr (KIND == SW_U1) {
        const V2<R> x = v[0], y = v[1];
        v[0] = cmac2(mat_at(A.op, 0), x, mat_at(A.op, 1), y);
        v[1] = cmac2(mat_at(A.op, 2), x, mat_at(A.op, 3), y);
    } else if constexpr (KIND == SW_XPERM || KIND == SW_SWAP) {
        const V2<R> x = v[0];
        v[0] = v[1];
        v[1] = x;
    } else if constexpr (KIND == SW_U2) {
        V2<R> w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            V2<R> acc = cmul(mat_at(A.op, 4 * i), v[0]);
#pragma unroll
            for (int j = 1; j < 4; ++j) {
                const V2<R> t = cmul(mat_at(A.op, 4 * i + j), v[j]);
                acc.x += t.x;
                acc.y += t.y;
            }
            w[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = w[i];
    } else if constexpr (KIND == SW_PHASE) {
        v[0] = cmul(v[0], A.f);
    } else if constexpr (KIND == SW_DIAG) {
        int idx = (int)((k >> A.a) & 1);
        if (A.b >= 0) idx = 2 * idx + (int)((k >> A.b) & 1);
        v[0] = cmul(v[0], mat_at(A.op, idx));
    } else {
        v[0] = cmul(v[0], ladder_phase<R>(A.turns, k & A.lmask));
    }
}

// Index set of one gate application from the smallest index k.
template <int KIND, typename R>
__device__ __forceinline__ void sweep_index(uint64_t (&idx)[sweep_nidx(KIND)], uint64_t k, const SweepArgs<R> &A) {
    idx[0] = k;
    if constexpr (KIND == SW_U1 || KIND == SW_XPERM) {
        idx[1] = k | (1ull << A.a);
    } else if constexpr (KIND == SW_SWAP) {
        idx[1] = k ^ A.flip;
    } else if constexpr (KIND == SW_U2) {
        idx[1] = k | (1ull << A.b);
        idx[2] = k | (1ull << A.a);
        idx[3] = k | (1ull << A.a) | (1ull << A.b);
    }
#ifdef SV_DEBUG_BOUNDS
    for (int i = 0; i < sweep_nidx(KIND); ++i) idx[i] = SV_GIDX(idx[i], A.dim);
#endif
}

// One gate over the whole state: thread t handles reduced index t (two
// adjacent ones in SWM_VEC2), expanded by `in` to the indices of the
// amplitudes the gate touches.  One thread per work item (exact grid): a
// grid-stride loop measured slower on these streaming sweeps.  With U > 1
// (index sets far apart) a thread takes U work items, 256 * W apart, so
// each stream of a wavefront has U accesses in flight; the grid then covers
// the items exactly (items a multiple of 256 * W * U).
template <typename R, int KIND, int MODE, bool NT, int U>
__global__ __launch_bounds__(SWEEP_TPB) void k_sweep(V2<R> *__restrict__ psi, uint64_t threads, Ins in,
                                                     SweepArgs<R> A) {
    constexpr int NI = sweep_nidx(KIND);
    if constexpr (U > 1) {
        static_assert(MODE != SWM_PAIR, "pair mode takes one item per thread");
        constexpr int W = MODE == SWM_VEC2 ? 2 : 1;
        const uint64_t rb = (uint64_t)blockIdx.x * (SWEEP_TPB * W * U) + W * threadIdx.x;
        uint64_t idx[U][NI];
        V2<R> v0[U][NI], v1[U][NI];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            sweep_index<KIND, R>(idx[u], expand(rb + (uint64_t)(SWEEP_TPB * W) * u, in), A);
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                if constexpr (W == 2) sw_ld2<NT>(psi + idx[u][i], v0[u][i], v1[u][i]);
                else v0[u][i] = sw_ld1<NT, R>(psi + idx[u][i]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            sweep_apply<KIND, R>(v0[u], idx[u][0], A);
            if constexpr (W == 2) sweep_apply<KIND, R>(v1[u], idx[u][0] + 1, A);
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                if constexpr (W == 2) sw_st2<NT>(psi + idx[u][i], v0[u][i], v1[u][i]);
                else sw_st1<NT, R>(psi + idx[u][i], v0[u][i]);
            }
        }
        return;
    }
    const uint64_t t = (uint64_t)blockIdx.x * SWEEP_TPB + threadIdx.x;
    if (t >= threads) return;
    if constexpr (MODE == SWM_PAIR) {
        const uint64_t k = SV_GIDX(expand(t, in), A.dim);  // bit 0 inserted as 0: the pair is (k, k + 1)
        V2<R> v[2];
        sw_ld2<NT>(psi + k, v[0], v[1]);
        sweep_apply<KIND, R>(v, k, A);
        sw_st2<NT>(psi + k, v[0], v[1]);
    } else if constexpr (MODE == SWM_VEC2) {
        const uint64_t k = expand(2 * t, in);  // bit 0 free: expand(2t + 1) = k + 1
        uint64_t idx[NI];
        sweep_index<KIND, R>(idx, k, A);
        V2<R> v0[NI], v1[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) sw_ld2<NT>(psi + idx[i], v0[i], v1[i]);
        sweep_apply<KIND, R>(v0, k, A);
        sweep_apply<KIND, R>(v1, k + 1, A);
#pragma unroll
        for (int i = 0; i < NI; ++i) sw_st2<NT>(psi + idx[i], v0[i], v1[i]);
    } else {
        const uint64_t k = expand(t, in);
        uint64_t idx[NI];
        sweep_index<KIND, R>(idx, k, A);
        V2<R> v[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) v[i] = sw_ld1<NT, R>(psi + idx[i]);
        sweep_apply<KIND, R>(v, k, A);
#pragma unroll
        for (int i = 0; i < NI; ++i) sw_st1<NT, R>(psi + idx[i], v[i]);
    }
}

template <typename R>
__global__ __launch_bounds__(SWEEP_TPB) void k_zero(V2<R> *__restrict__ psi, uint64_t dim) {
    const uint64_t stride = (uint64_t)gridDim.x * SWEEP_TPB;
    for (uint64_t k = (uint64_t)blockIdx.x * SWEEP_TPB + threadIdx.x; k < dim; k += stride) {
        V2<R> v;
        v.x = (k == 0) ? (R)1 : (R)0;
        v.y = 0;
        psi[k] = v;
    }
}

template <typename R>
__global__ __launch_bounds__(SWEEP_TPB) void k_scale(V2<R> *__restrict__ psi, uint64_t dim, double s) {
    const uint64_t stride = (uint64_t)gridDim.x * SWEEP_TPB;
    for (uint64_t k = (uint64_t)blockIdx.x * SWEEP_TPB + threadIdx.x; k < dim; k += stride) {
        V2<R> v = psi[k];
        v.x = (R)((double)v.x * s);
        v.y = (R)((double)v.y * s);
        psi[k] = v;
    }
}

constexpr int TILE_TPB = 512;

// LDS position of tile element x: XOR-swizzled within rows of 256 bytes
// (32 complex64 / 16 complex128) by two folds of the row index, so that the
// permuted (e.g. bit-reversed) reads of a wave spread over the banks.
template <typename R>
__device__ __forceinline__ uint32_t swz(uint32_t x) {
    constexpr int S = sizeof(V2<R>) == 8 ? 5 : 4;
    constexpr uint32_t M = (1u << S) - 1;
    return x ^ ((x >> S) & M) ^ ((x >> (2 * S)) & M);
}

// In-place involution on index bits.  The local bit set is closed under the
// involution, so tile v maps onto tile w = P(v); the workgroup owning
// min(v, w) exchanges both.  The local part of P is a bit permutation, so
// the image of local position j is lo[j & 63] ^ hi[j >> 6] (two 64-entry
// tables in LDS).  Software-pipelined: the loads of a workgroup's next item
// are issued before the LDS exchange and the stores of the current one, so
// HBM reads overlap the rest of the item.  MAXA = 16-byte accesses per
// thread and tile (2^m / (EPA * TILE_TPB), at most 4): the registers that
// hold two items scale with it.
template <typename R, int MAXA>
__global__ __launch_bounds__(TILE_TPB) void k_perm(V2<R> *__restrict__ slab, uint64_t dim, int nc,
                                                   const DevPass *__restrict__ passes, int pidx,
                                                   const uint64_t *__restrict__ aux,
                                                   const uint32_t *__restrict__ aux32, uint64_t ntiles) {
    extern __shared__ __align__(16) unsigned char smem[];
    const DevPass &P = passes[pidx];
    const int m = P.m, l = P.l;
    const uint32_t T = 1u << m;
    V2<R> *A = reinterpret_cast<V2<R> *>(smem);
    V2<R> *B = A + T;
    uint64_t *hi_off = reinterpret_cast<uint64_t *>(smem + 2 * (sizeof(V2<R>) << m));
    const uint32_t nhi = 1u << (m - l);
    uint32_t *plo = reinterpret_cast<uint32_t *>(hi_off + nhi);
    uint32_t *phi = plo + 64;
    const uint32_t lowm = (1u << l) - 1;
    for (uint32_t h = threadIdx.x; h < nhi; h += TILE_TPB) hi_off[h] = aux[P.hi_begin + h];
    const uint32_t *lperm = aux32 + P.lperm_begin;
    if (threadIdx.x < 64) {
        plo[threadIdx.x] = threadIdx.x < T ? lperm[threadIdx.x] : 0u;
        phi[threadIdx.x] = (threadIdx.x << 6) < T ? lperm[threadIdx.x << 6] : 0u;
    }
    const uint64_t fmask = P.free_mask;
    const int nfp = P.nfp;
    const int lt = __builtin_ctzll(ntiles);
    // the free bit pairs, as 32-bit words held in scalar registers (byte
    // loads inside the item loop would be vector loads, each waited out)
    uint32_t fpw[12];
    const uint32_t *fw = reinterpret_cast<const uint32_t *>(P.fpa);
#pragma unroll
    for (int i = 0; i < 12; ++i) fpw[i] = __builtin_amdgcn_readfirstlane(fw[i]);
    __syncthreads();
    // 16-byte register images of the accesses (two complex64 / one complex128)
    typedef float PT __attribute__((ext_vector_type(4)));
    constexpr int EPA = 16 / sizeof(V2<R>);
    auto half = [](PT v, int h) __attribute__((always_inline)) {
        V2<R> r;
        if constexpr (EPA == 2) {
            r.x = h ? v.z : v.x;
            r.y = h ? v.w : v.y;
        } else {
            __builtin_memcpy(&r, &v, 16);
        }
        return r;
    };
    auto join = [](V2<R> a, V2<R> b) __attribute__((always_inline)) {
        PT v;
        if constexpr (EPA == 2) {
            v.x = a.x;
            v.y = a.y;
            v.z = b.x;
            v.w = b.y;
        } else {
            __builtin_memcpy(&v, &a, 16);
        }
        return v;
    };
    const uint32_t nacc = T / EPA;
    const uint64_t nw = (uint64_t)nc * ntiles;
    struct Item {
        V2<R> *psi;
        uint64_t bv, bw;
    };
    // the item's tiles; false when the partner tile's workgroup owns it
    auto meta = [&](uint64_t w, Item &it) __attribute__((always_inline)) {
        // ntiles is a power of two: shift and mask (a 64-bit division is a
        // long scalar routine, run by every wave for every candidate item)
        const uint64_t c = w >> lt, t = w & (ntiles - 1);
        it.psi = slab + c * dim;
        it.bv = deposit(t, fmask);
        it.bw = it.bv;
#pragma unroll
        for (int i = 0; i < 24; ++i) {
            if (i >= nfp) break;  // unrolled: the words stay in scalar registers
            const int a = (int)((fpw[i >> 2] >> (8 * (i & 3))) & 255u);
            const int b = (int)((fpw[6 + (i >> 2)] >> (8 * (i & 3))) & 255u);
            if (((it.bv >> a) ^ (it.bv >> b)) & 1) it.bw ^= (1ull << a) | (1ull << b);
        }
        return it.bw >= it.bv;
    };
    auto load = [&](const Item &it, PT (&x)[MAXA], PT (&y)[MAXA]) __attribute__((always_inline)) {
        const bool two = it.bw != it.bv;
#pragma unroll
        for (int a = 0; a < MAXA; ++a) {
            const uint32_t q = threadIdx.x + (uint32_t)a * TILE_TPB;
            if (q < nacc) {
                const uint32_t j = q * EPA;
                const uint64_t off = hi_off[j >> l] | (j & lowm);
                x[a] = *reinterpret_cast<const PT *>(it.psi + SV_GIDX(it.bv | off, dim));
                if (two) y[a] = *reinterpret_cast<const PT *>(it.psi + SV_GIDX(it.bw | off, dim));
            }
        }
    };
    Item cur;
    PT xc[MAXA], yc[MAXA];
    uint64_t w = blockIdx.x;
    while (w < nw && !meta(w, cur)) w += gridDim.x;
    if (w < nw) load(cur, xc, yc);
    while (w < nw) {
        // next owned item: its loads go out before this item's exchange
        Item nxt;
        uint64_t wn = w + gridDim.x;
        while (wn < nw && !meta(wn, nxt)) wn += gridDim.x;
        PT xn[MAXA], yn[MAXA];
        if (wn < nw) load(nxt, xn, yn);
        const bool two = cur.bw != cur.bv;
#pragma unroll
        for (int a = 0; a < MAXA; ++a) {
            const uint32_t q = threadIdx.x + (uint32_t)a * TILE_TPB;
            if (q < nacc) {
                const uint32_t j = q * EPA;
                A[SV_LIDX(swz<R>(j), T)] = half(xc[a], 0);
                if (two) B[SV_LIDX(swz<R>(j), T)] = half(yc[a], 0);
                if constexpr (EPA == 2) {
                    A[SV_LIDX(swz<R>(j + 1), T)] = half(xc[a], 1);
                    if (two) B[SV_LIDX(swz<R>(j + 1), T)] = half(yc[a], 1);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < MAXA; ++a) {
            const uint32_t q = threadIdx.x + (uint32_t)a * TILE_TPB;
            if (q < nacc) {
                const uint32_t j = q * EPA;
                const uint64_t off = hi_off[j >> l] | (j & lowm);
                PT x, y;
                const uint32_t s0 = SV_LIDX(swz<R>(plo[j & 63] ^ phi[j >> 6]), T);
                if constexpr (EPA == 2) {
                    const uint32_t s1 = SV_LIDX(swz<R>(plo[(j + 1) & 63] ^ phi[(j + 1) >> 6]), T);
                    x = join(A[s0], A[s1]);
                    if (two) y = join(B[s0], B[s1]);
                } else {
                    x = join(A[s0], A[s0]);
                    if (two) y = join(B[s0], B[s0]);
                }
                if (two) {
                    *reinterpret_cast<PT *>(cur.psi + SV_GIDX(cur.bw | off, dim)) = x;
                    *reinterpret_cast<PT *>(cur.psi + SV_GIDX(cur.bv | off, dim)) = y;
                } else {
                    *reinterpret_cast<PT *>(cur.psi + SV_GIDX(cur.bv | off, dim)) = x;
                }
            }
        }
        __syncthreads();
        w = wn;
        cur = nxt;
#pragma unroll
        for (int a = 0; a < MAXA; ++a) {
            xc[a] = xn[a];
            yc[a] = yn[a];
        }
    }
}

// ===========================================================================
// Host side
// ===========================================================================

hipError_t dev_malloc(Ctx *ctx, void **p, size_t bytes) {
    const uint64_t k = ctx->n_allocs.fetch_add(1) + 1;
    if (ctx->fault_alloc > 0 && k == (uint64_t)ctx->fault_alloc) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

void *scratch(Ctx *ctx, const std::string &name, size_t bytes) {
    DeviceBuffer &b = ctx->scratch[name];
    if (ctx->record) {
        // a recorded launch holds this pointer until the graph runs: a slot
        // may be handed out once per recording
        for (const std::string &s : ctx->record_slots)
            if (s == name) fail(SV_EDEVICE, "internal: scratch slot " + name + " reused while recording");
        ctx->record_slots.push_back(name);
    }
    if (b.bytes < bytes) {
        if (b.ptr) {
            SV_HIP(hipStreamSynchronize(ctx->stream));
            SV_HIP(hipFree(b.ptr));
            b.ptr = nullptr;
            b.bytes = 0;
        }
        size_t want = std::max<size_t>(bytes, 4096);
        if (dev_malloc(ctx, &b.ptr, want) != hipSuccess) {
            (void)hipGetLastError();
            fail(SV_ENOMEM, "device allocation of " + std::to_string(want) + " bytes failed");
        }
        b.bytes = want;
    }
    return b.ptr;
}

void upload(Ctx *ctx, void *dst, const void *src, size_t bytes) {
    if (!bytes) return;
    if (ctx->pinned_on && ctx->pinned_used + bytes <= ctx->pinned_cap) {
        // through the batch call's pinned arena (a pageable copy stages
        // through driver buffers and costs more for these small blobs)
        char *p = ctx->pinned + ctx->pinned_used;
        ctx->pinned_used += (bytes + 255) & ~(size_t)255;
        std::memcpy(p, src, bytes);
        SV_HIP(hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, ctx->stream));
        return;
    }
    SV_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
}

void pinned_begin(Ctx *ctx) {
    constexpr size_t cap = (size_t)4 << 20;
    if (!ctx->pinned) {
        if (hipHostMalloc((void **)&ctx->pinned, cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            ctx->pinned = nullptr;
            return;  // pageable copies then
        }
        ctx->pinned_cap = cap;
    }
    ctx->pinned_used = 0;
    ctx->pinned_on = true;
}

void pinned_end(Ctx *ctx) { ctx->pinned_on = false; }

void release_pinned(Ctx *ctx) {
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_cap = ctx->pinned_used = 0;
    ctx->pinned_on = false;
}

void launch_or_record(Ctx *ctx, std::function<void()> f) {
    if (ctx->record) ctx->record->push_back(std::move(f));
    else f();
}

void release_graph(Ctx *ctx) {
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    ctx->graph_exec = nullptr;
}

// The uploads of a batch have been enqueued while it was recorded; the
// launches are captured from ctx->stream into a graph and run as one
// launch.  The instantiated graph is kept and updated in place while the
// next batch has the same shape (same kernels and grid; pointers and
// arguments may change), which skips the instantiation.
void launch_recorded(Ctx *ctx, std::vector<std::function<void()>> &work) {
    if (work.empty()) return;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        // the stream cannot be captured (e.g. the caller is capturing it):
        // launch the same kernels directly
        (void)hipGetLastError();
        for (auto &f : work) f();
        return;
    }
    try {
        for (auto &f : work) f();
    } catch (...) {
        (void)hipStreamEndCapture(ctx->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        throw;
    }
    SV_HIP(hipStreamEndCapture(ctx->stream, &g));
    bool updated = false;
    if (ctx->graph_exec) {
        // the previous replay must be over before its node arguments change
        SV_HIP(hipStreamSynchronize(ctx->stream));
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        updated = hipGraphExecUpdate(ctx->graph_exec, g, &bad, &res) == hipSuccess &&
                  res == hipGraphExecUpdateSuccess;
        if (!updated) {
            (void)hipGetLastError();
            release_graph(ctx);
        }
    }
    if (!updated) {
        const hipError_t e = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            ctx->graph_exec = nullptr;
            (void)hipGraphDestroy(g);
            fail(SV_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        ++ctx->graph_instantiations;
    }
    (void)hipGraphDestroy(g);
    SV_HIP(hipGraphLaunch(ctx->graph_exec, ctx->stream));
    ++ctx->graph_launches;
}

LaunchScope::LaunchScope(Ctx *c, const char *nm, double b) : ctx(c), name(nm), bytes(b) {
    if (!ctx->profile) return;
    if (ctx->free_events.size() >= 2) {
        e0 = ctx->free_events.back();
        ctx->free_events.pop_back();
        e1 = ctx->free_events.back();
        ctx->free_events.pop_back();
    } else {
        SV_HIP(hipEventCreate(&e0));
        SV_HIP(hipEventCreate(&e1));
    }
    SV_HIP(hipEventRecord(e0, ctx->stream));
}
LaunchScope::~LaunchScope() {
    if (!e0) return;
    if (hipEventRecord(e1, ctx->stream) != hipSuccess) return;
    ctx->pending.push_back({name, {e0, e1}});
    ctx->pending_bytes.push_back(bytes);
}

void profile_collect(Ctx *ctx) {
    for (size_t i = 0; i < ctx->pending.size(); ++i) {
        auto &p = ctx->pending[i];
        float ms = 0.f;
        SV_HIP(hipEventSynchronize(p.second.second));
        SV_HIP(hipEventElapsedTime(&ms, p.second.first, p.second.second));
        ProfileEntry &e = ctx->prof[p.first];
        e.ms += ms;
        e.launches += 1;
        e.bytes += ctx->pending_bytes[i];
        ctx->free_events.push_back(p.second.first);
        ctx->free_events.push_back(p.second.second);
    }
    ctx->pending.clear();
    ctx->pending_bytes.clear();
}

unsigned grid_for(uint64_t items, int tpb, int cu) {
    uint64_t g = (items + tpb - 1) / tpb;
    const uint64_t cap = (uint64_t)cu * 64;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

void set_lds_limit(const void *fn, size_t bytes) {
    static std::mutex mu;
    static int max_lds = 0;
    std::lock_guard<std::mutex> g(mu);
    if (max_lds == 0) {
        int dev = 0;
        SV_HIP(hipGetDevice(&dev));
        SV_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    }
    if (bytes > (size_t)max_lds)
        fail(SV_EDEVICE, "internal: LDS request of " + std::to_string(bytes) + " bytes exceeds the device limit of " +
                             std::to_string(max_lds));
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(SV_EDEVICE, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    }
}

// Device descriptor of a pass; appends its hi_off table (and for PERM
// passes the local permutation) to the auxiliary arrays.
static DevPass to_dev_pass(const Pass &ps, int op_begin, int op_end, std::vector<uint64_t> &aux,
                           std::vector<uint32_t> &aux32) {
    DevPass d;
    std::memset(&d, 0, sizeof d);
    d.kind = ps.kind;
    d.m = ps.m;
    d.l = ps.l;
    d.nfree = (int)ps.free_bits.size();
    d.op_begin = op_begin;
    d.op_end = op_end;
    for (int b : ps.free_bits) d.free_mask |= 1ull << b;
    d.hi_begin = (int)aux.size();
    const uint32_t nhi = 1u << (ps.m - ps.l);
    for (uint32_t h = 0; h < nhi; ++h) {
        uint64_t o = 0;
        for (int i = 0; i < ps.m - ps.l; ++i)
            if ((h >> i) & 1) o |= 1ull << ps.local_bits[ps.l + i];
        aux.push_back(o);
    }
    if (ps.kind == PASS_PERM) {
        int pos[64];
        for (int i = 0; i < 64; ++i) pos[i] = -1;
        for (size_t i = 0; i < ps.local_bits.size(); ++i) pos[ps.local_bits[i]] = (int)i;
        std::vector<std::pair<int, int>> local_pairs;
        for (auto &pr : ps.swaps) {
            if (pos[pr.first] >= 0 && pos[pr.second] >= 0) {
                local_pairs.push_back({pos[pr.first], pos[pr.second]});
            } else if (pos[pr.first] < 0 && pos[pr.second] < 0) {
                d.fpa[d.nfp] = (int8_t)pr.first;
                d.fpb[d.nfp] = (int8_t)pr.second;
                ++d.nfp;
            } else {
                fail(SV_EDEVICE, "internal: permutation pass tile not closed under its pairs");
            }
        }
        d.lperm_begin = (int)aux32.size();
        for (uint32_t j = 0; j < (1u << ps.m); ++j) {
            uint32_t s = j;
            for (auto &lp : local_pairs) {
                const uint32_t x = ((s >> lp.first) ^ (s >> lp.second)) & 1;
                s ^= (x << lp.first) | (x << lp.second);
            }
            aux32.push_back(s);
        }
    }
    return d;
}

static unsigned tile_grid(uint64_t tiles, int cu) {
    const uint64_t cap = (uint64_t)cu * 16;
    return (unsigned)std::max<uint64_t>(1, std::min(tiles, cap));
}

// One-qubit gate (U1 or X) on a low bit a whose partner sits in another
// lane of the same wavefront: each lane loads 16 contiguous bytes (two
// complex64 / one complex128 amplitude), so a wavefront reads and writes one
// contiguous kilobyte, and the partner amplitudes come from lane t ^ d by a
// cross-lane permute.  `in` inserts the control bits only; they all lie above
// the wavefront's span, and the thread count is a multiple of 64.
template <typename R, int KIND>
__global__ __launch_bounds__(SWEEP_TPB) void k_sweep_shfl(V2<R> *__restrict__ psi, uint64_t threads, Ins in,
                                                          SweepArgs<R> A, int d) {
    const uint64_t t = (uint64_t)blockIdx.x * SWEEP_TPB + threadIdx.x;
    if (t >= threads) return;  // whole wavefronts only
    constexpr int W = sizeof(R) == 4 ? 2 : 1;
    const uint64_t k = SV_GIDX(expand(t * W, in), A.dim);
    V2<R> own[W], par[W];
    if constexpr (W == 2) sw_ld2<true>(psi + k, own[0], own[1]);
    else own[0] = sw_ld1<true, R>(psi + k);
#pragma unroll
    for (int i = 0; i < W; ++i) {
        par[i].x = __shfl_xor(own[i].x, d);
        par[i].y = __shfl_xor(own[i].y, d);
    }
    if constexpr (KIND == SW_XPERM) {
#pragma unroll
        for (int i = 0; i < W; ++i) own[i] = par[i];
    } else {
        // own amplitude has bit a = b: new = m[b][b] * own + m[b][1-b] * partner
        const bool b = (k >> A.a) & 1;
        const V2<R> co = b ? mat_at(A.op, 3) : mat_at(A.op, 0), cp = b ? mat_at(A.op, 2) : mat_at(A.op, 1);
#pragma unroll
        for (int i = 0; i < W; ++i) own[i] = cmac2(co, own[i], cp, par[i]);
    }
    if constexpr (W == 2) sw_st2<true>(psi + k, own[0], own[1]);
    else sw_st1<true, R>(psi + k, own[0]);
}

// Launch one sweep: `pos` are the index bits inserted by `in` (controls and
// the bits a gate acts on), `low` the smallest distance in bytes between
// two amplitudes of one index set (0 when a set has one amplitude).
template <typename R, int KIND>
static void launch_sweep(Ctx *ctx, V2<R> *psi, int n, const std::vector<int> &pos, uint64_t ones,
                         const SweepArgs<R> &A, size_t low, const char *name, double bytes) {
    if constexpr (KIND == SW_U1 || KIND == SW_XPERM) {
        // partner in another lane of the wavefront (a below its span of 2^span
        // amplitudes; complex64 bit 0 is the 16-byte pair), controls above it
        constexpr int W = sizeof(R) == 4 ? 2 : 1, span = sizeof(R) == 4 ? 7 : 6;
        int cmin = 64;
        for (int p : pos)
            if (p != A.a) cmin = std::min(cmin, p);
        const int nc = (int)pos.size() - 1;
        if (A.a < span && (W == 1 || A.a >= 1) && cmin >= span && n - nc >= span) {
            std::vector<int> cpos;
            for (int p : pos)
                if (p != A.a) cpos.push_back(p);
            const Ins cin = make_ins(cpos, ones);
            const uint64_t threads = (1ull << (n - nc)) / W;
            const uint64_t blocks = (threads + SWEEP_TPB - 1) / SWEEP_TPB;
            if (blocks > 0x7fffffffull) fail(SV_EINVAL, "sweep launch too large");
            LaunchScope ls(ctx, name, bytes);
            hipLaunchKernelGGL((k_sweep_shfl<R, KIND>), dim3((unsigned)blocks), dim3(SWEEP_TPB), 0, ctx->stream, psi,
                               threads, cin, A, (1 << A.a) / W);
            return;
        }
    }
    const Ins in = make_ins(pos, ones);
    const uint64_t items = 1ull << (n - pos.size());
    bool bit0 = false;
    for (int p : pos) bit0 |= p == 0;
    int mode = SWM_ONE;
    if constexpr (sizeof(R) == 4) {
        if (!bit0 && items >= 2) mode = SWM_VEC2;
        else if ((KIND == SW_U1 || KIND == SW_XPERM) && A.a == 0 && !(ones & 1)) mode = SWM_PAIR;
    }
    // streaming (non-temporal) accesses unless the index set shares a cache
    // line (then the second access of a lane reuses the line of the first);
    // single amplitudes of complex64 stay plain (sparse patterns)
    const bool nt = (low == 0 || low >= 128) && (mode != SWM_ONE || sizeof(R) == 16);
    // index sets spread over 32 MiB and more: four items per thread
    const int W = mode == SWM_VEC2 ? 2 : 1;
    const bool wide = low >= ((size_t)32 << 20) && mode != SWM_PAIR && (mode != SWM_ONE || sizeof(R) == 16) &&
                      items % (uint64_t)(SWEEP_TPB * W * 4) == 0;
    const uint64_t threads = items / W;
    const uint64_t blocks = wide ? items / (SWEEP_TPB * W * 4) : (threads + SWEEP_TPB - 1) / SWEEP_TPB;
    if (blocks > 0x7fffffffull) fail(SV_EINVAL, "sweep launch too large");
    LaunchScope ls(ctx, name, bytes);
    auto go = [&](auto MODE_C, auto NT_C, auto U_C) {
        constexpr int M = decltype(MODE_C)::value;
        constexpr bool T = decltype(NT_C)::value;
        constexpr int UU = decltype(U_C)::value;
        hipLaunchKernelGGL((k_sweep<R, KIND, M, T, UU>), dim3((unsigned)blocks), dim3(SWEEP_TPB), 0, ctx->stream,
                           psi, threads, in, A);
    };
    using I0 = std::integral_constant<int, SWM_ONE>;
    using IT = std::true_type;
    using IF = std::false_type;
    using U1c = std::integral_constant<int, 1>;
    using U4c = std::integral_constant<int, 4>;
    if constexpr (sizeof(R) == 4) {
        using IV = std::integral_constant<int, SWM_VEC2>;
        if (mode == SWM_VEC2) {
            if (wide) go(IV{}, IT{}, U4c{});
            else if (nt) go(IV{}, IT{}, U1c{});
            else go(IV{}, IF{}, U1c{});
            return;
        }
        if constexpr (KIND == SW_U1 || KIND == SW_XPERM) {
            using IP = std::integral_constant<int, SWM_PAIR>;
            if (mode == SWM_PAIR) {
                go(IP{}, IT{}, U1c{});
                return;
            }
        }
        if (nt) go(I0{}, IT{}, U1c{});
        else go(I0{}, IF{}, U1c{});
    } else {
        if (wide) go(I0{}, IT{}, U4c{});
        else if (nt) go(I0{}, IT{}, U1c{});
        else go(I0{}, IF{}, U1c{});
    }
}

template <typename R>
void sweep_one(Ctx *ctx, V2<R> *psi, int n, const Op &op) {
    const size_t amp = sizeof(V2<R>);
    SweepArgs<R> A;
    std::memset(&A, 0, sizeof A);
    A.op = to_dev<R>(op);
    A.a = op.a;
    A.b = op.b;
    A.dim = 1ull << n;
    std::vector<int> cb = bits_of(op.cmask);
    switch (op.kind) {
    case OP_U1:
    case OP_XPERM: {
        std::vector<int> pos = cb;
        pos.push_back(op.a);
        const double bytes = 2.0 * amp * (double)(1ull << (n - cb.size()));
        if (op.kind == OP_U1)
            launch_sweep<R, SW_U1>(ctx, psi, n, pos, op.cmask, A, amp << op.a, "sweep_u1", bytes);
        else
            launch_sweep<R, SW_XPERM>(ctx, psi, n, pos, op.cmask, A, amp << op.a, "sweep_xperm", bytes);
        break;
    }
    case OP_U2: {
        std::vector<int> pos = cb;
        pos.push_back(op.a);
        pos.push_back(op.b);
        const double bytes = 2.0 * amp * (double)(1ull << (n - cb.size()));
        launch_sweep<R, SW_U2>(ctx, psi, n, pos, op.cmask, A, amp << std::min(op.a, op.b), "sweep_u2", bytes);
        break;
    }
    case OP_SWAP: {
        std::vector<int> pos = cb;
        pos.push_back(op.a);
        pos.push_back(op.b);
        A.flip = (1ull << op.a) | (1ull << op.b);
        // pairs (k, k ^ flip) with bit a set and bit b clear: half the state moves
        const double bytes = 2.0 * amp * (double)(1ull << (n - cb.size() - 1));
        launch_sweep<R, SW_SWAP>(ctx, psi, n, pos, op.cmask | (1ull << op.a), A, amp << std::min(op.a, op.b),
                                 "sweep_swap", bytes);
        break;
    }
    case OP_DIAG: {
        // phase-only on one pattern when the other entries are 1
        const bool one_b = op.b < 0;
        const int last = one_b ? 1 : 3;
        bool only_last = true;
        for (int k = 0; k < last; ++k) only_last &= op.m[k] == cd(1.0);
        if (only_last) {
            std::vector<int> pos = cb;
            uint64_t ones = op.cmask | (1ull << op.a);
            if (!(op.cmask & (1ull << op.a))) pos.push_back(op.a);
            if (!one_b) {
                if (!(ones & (1ull << op.b))) pos.push_back(op.b);
                ones |= 1ull << op.b;
            }
            A.f.x = (R)op.m[last].real();
            A.f.y = (R)op.m[last].imag();
            const double bytes = 2.0 * amp * (double)(1ull << (n - pos.size()));
            launch_sweep<R, SW_PHASE>(ctx, psi, n, pos, ones, A, 0, "sweep_phase", bytes);
        } else {
            const double bytes = 2.0 * amp * (double)(1ull << (n - cb.size()));
            launch_sweep<R, SW_DIAG>(ctx, psi, n, cb, op.cmask, A, 0, "sweep_diag", bytes);
        }
        break;
    }
    case OP_LADDER: {
        A.lmask = op.lmask;
        A.turns = op.turns;
        const double bytes = 2.0 * amp * (double)(1ull << (n - 1));
        launch_sweep<R, SW_LADDER>(ctx, psi, n, {op.a}, 1ull << op.a, A, 0, "sweep_ladder", bytes);
        break;
    }
    default:
        fail(SV_EDEVICE, "internal: bad op kind");
    }
    SV_HIP(hipGetLastError());
}

template <typename R>
DevPlanHost<R> build_dev_plan(const Plan &plan) {
    DevPlanHost<R> h;
    for (const Pass &ps : plan.passes) {
        if (ps.kind == PASS_SWEEP) {
            h.dpass.push_back(DevPass{});
            continue;
        }
        const int b = (int)h.dops.size();
        const int ltab_begin = (int)h.ltab.size();
        std::vector<int> ladders;
        for (const Op &op : ps.ops) {
            DevOp<R> d = to_dev<R>(op);
            localise(d, ps.local_bits);
            if (op.kind == OP_DENSE4) {
                // local positions of its four bits; W = [[Re U, -Im U], [Im U, Re U]]
                d.lcmask = 0;
                for (size_t i = 0; i < ps.local_bits.size(); ++i)
                    if ((op.lmask >> ps.local_bits[i]) & 1) d.lcmask |= 1ull << i;
                d.tab = (int)h.mtab.size();
                const std::vector<cd> &U = plan.dense[op.dense];
                for (int rr = 0; rr < 32; ++rr)
                    for (int cc = 0; cc < 32; ++cc) {
                        const cd u = U[16 * (rr % 16) + (cc % 16)];
                        const double v = rr < 16 ? (cc < 16 ? u.real() : -u.imag()) : (cc < 16 ? u.imag() : u.real());
                        h.mtab.push_back((float)v);
                    }
            }
            if (op.kind == OP_LADDER && ps.kind == PASS_TILE) {
                append_ladder_tables<R>(d, op, ps.local_bits, h.ltab);
                d.tab -= ltab_begin;  // tables are addressed from the pass's first one
                d.tslot = (int)ladders.size();
                ladders.push_back((int)h.dops.size());
            }
            h.gate.push_back(op.gate);
            h.dops.push_back(d);
        }
        DevPass dp = to_dev_pass(ps, b, (int)h.dops.size(), h.aux, h.aux32);
        dp.ltab_begin = ltab_begin;
        dp.ltab_count = (int)h.ltab.size() - ltab_begin;
        dp.nlad = (int)ladders.size();
        dp.lad_list = (int)h.aux32.size();
        for (int o : ladders) h.aux32.push_back((uint32_t)o);
        dp.scale = 1.0;
        for (int i = b; i < (int)h.dops.size(); ++i)
            if (h.dops[i].flags & OPF_SCALED) dp.scale *= h.dops[i].sfac;
        dp.stage_begin = (int)h.dstages.size();
        dp.paux_begin = (int)h.aux32.size();
        // passes of uncontrolled one-qubit gates, ladders and diagonals take
        // four-bit stages
        dp.h4 = ps.kind == PASS_TILE ? h4_kind<R>(h.dops, b, (int)h.dops.size(), ps.m) : 0;
        if (dp.h4) {
            build_stages_h4<R>(h.dops, b, (int)h.dops.size(), ps.local_bits, h.dstages, dp.h4 == 3);
            if (dp.h4 == 3 &&
                !build_rotation_layers<R>(h.dops, h.gate, ps.ops, b, (int)h.dops.size(), h.dstages, dp.stage_begin,
                                          ps.local_bits, dp)) {
                int oe = (int)h.dops.size();
                gather_stage_diagonals<R>(h.dops, h.gate, ps.ops, b, oe, h.dstages, dp.stage_begin, ps.local_bits);
                dp.op_end = oe;
            }
            for (size_t si = dp.stage_begin; si < h.dstages.size(); ++si)
                h.dstages[si].lane_pos = h4_lane_order(h.dstages[si], ps.m);
        } else if (ps.kind == PASS_TILE) {
            build_stages<R>(h.dops, b, (int)h.dops.size(), ps.local_bits, h.dstages, h.aux32, true);
        }
        dp.stage_end = (int)h.dstages.size();
        dp.paux_count = (int)h.aux32.size() - dp.paux_begin;
        // the layout-map tables go to LDS when the workgroup still fits
        // twice per CU (measured 1.3% faster on the 20-qubit 641-circuit gradient)
        if (ps.kind == PASS_TILE && dp.paux_count > 0) {
            const uint32_t nhi = 1u << (ps.m - ps.l);
            const size_t with = tile_lds_layout(nhi, dp.nlad, dp.ltab_count, sizeof(V2<R>), dp.paux_count).end +
                                (sizeof(V2<R>) << ps.m);
            dp.paux_lds = with <= (size_t)80 * 1024 ? 1 : 0;
        }
        h.dpass.push_back(dp);
    }
    return h;
}
template DevPlanHost<float> build_dev_plan<float>(const Plan &);
template DevPlanHost<double> build_dev_plan<double>(const Plan &);

// Host-side summary and text listing of a device plan (no device work).
template <typename R>
PlanSummary summarize_plan(const Plan &plan, std::string *text) {
    const DevPlanHost<R> h = build_dev_plan<R>(plan);
    PlanSummary sm;
    static const char *kname[] = {"U1", "U2", "DIAG", "LADDER", "SWAP", "XPERM", "DENSE4", "DIAG16"};
    char line[256];
    for (size_t i = 0; i < plan.passes.size(); ++i) {
        const Pass &ps = plan.passes[i];
        const DevPass &dp = h.dpass[i];
        if (ps.kind == PASS_SWEEP) {
            ++sm.sweep_passes;
            if (text) *text += "pass " + std::to_string(i) + " sweep\n";
            continue;
        }
        if (ps.kind == PASS_PERM) {
            ++sm.perm_passes;
            if (text) *text += "pass " + std::to_string(i) + " perm m=" + std::to_string(ps.m) + "\n";
            continue;
        }
        ++sm.tile_passes;
        sm.h4_passes[std::max(0, std::min(4, dp.h4))] += 1;
        sm.stages += dp.stage_end - dp.stage_begin;
        sm.ops += dp.op_end - dp.op_begin;
        if (dp.h4 == 4) sm.tile_factor_ops += dp.tf_end - dp.tf_begin;
        sm.min_scale = std::min(sm.min_scale, std::fabs(dp.scale));
        sm.max_scale = std::max(sm.max_scale, std::fabs(dp.scale));
        if (text) {
            std::snprintf(line, sizeof line, "pass %zu tile m=%d l=%d h4=%d ops=%d stages=%d scale=%.17g\n", i, ps.m,
                          ps.l, dp.h4, dp.op_end - dp.op_begin, dp.stage_end - dp.stage_begin, dp.scale);
            *text += line;
        }
        for (int s = dp.stage_begin; s < dp.stage_end; ++s) {
            const DevStage &S = h.dstages[s];
            if (text) {
                std::snprintf(line, sizeof line, "  stage regs=%d,%d,%d,%d ops=[%d,%d) acc=%d mfma=%d perm=%d\n", S.r0,
                              S.r1, S.r2, dp.h4 ? S.r3 : -1, S.op_begin, S.op_end, S.acc, S.mfma, S.perm);
                *text += line;
            }
            if (dp.h4 == 4) {
                // rotation layer: tables before and after the four rotations
                sm.tables += (S.tpre >= 0) + (S.tpost >= 0);
                if (text) {
                    const DevOp<R> &q = h.dops[S.rot];
                    std::snprintf(line, sizeof line, "    layer pre=%d t=(%.4g %.4g %.4g %.4g) post=%d\n",
                                  S.tpre >= 0 ? (h.dops[S.tpre].flags & OPF_SGN ? 2 : 1) : 0, (double)q.m[0],
                                  (double)q.m[2], (double)q.m[4], (double)q.m[6],
                                  S.tpost >= 0 ? (h.dops[S.tpost].flags & OPF_SGN ? 2 : 1) : 0);
                    *text += line;
                }
            }
            for (int o = S.op_begin; o < S.op_end; ++o) {
                const DevOp<R> &op = h.dops[o];
                if (op.kind == OP_DENSE4) ++sm.dense_blocks;
                if (op.kind == OP_DIAG16) ++sm.tables;
                if (text) {
                    std::snprintf(line, sizeof line, "    %s a=%d b=%d ra=%d flags=%d cmask=%llx gate=%d\n",
                                  op.kind >= 0 && op.kind < 8 ? kname[op.kind] : "?", op.a, op.b, op.ra, op.flags,
                                  (unsigned long long)op.cmask, h.gate[o]);
                    *text += line;
                }
            }
        }
    }
    return sm;
}
template PlanSummary summarize_plan<float>(const Plan &, std::string *);
template PlanSummary summarize_plan<double>(const Plan &, std::string *);

// Device image of a plan: every table at a 256-byte boundary of one block
// (dbase null: only the size of that block is computed).
template <typename R>
static size_t place_dev_plan(Ctx *ctx, const DevPlanHost<R> &h, char *dbase, DevPlanDev<R> *out) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t s_ops = al(h.dops.size() * sizeof(DevOp<R>) + 16), s_pass = al(h.dpass.size() * sizeof(DevPass) + 16);
    const size_t s_st = al(h.dstages.size() * sizeof(DevStage) + 16), s_aux = al(h.aux.size() * 8 + 16);
    const size_t s_aux32 = al(h.aux32.size() * 4 + 16), s_lt = al(h.ltab.size() * sizeof(V2<R>) + 16);
    const size_t s_mt = al(h.mtab.size() * 4 + 16);
    const size_t total = s_ops + s_pass + s_st + s_aux + s_aux32 + s_lt + s_mt;
    if (!dbase) return total;
    std::vector<unsigned char> host(total, 0);
    size_t off = 0;
    auto put = [&](const void *src, size_t bytes, size_t sz) {
        if (bytes) std::memcpy(host.data() + off, src, bytes);
        const size_t o = off;
        off += sz;
        return o;
    };
    const size_t o_ops = put(h.dops.data(), h.dops.size() * sizeof(DevOp<R>), s_ops);
    const size_t o_pass = put(h.dpass.data(), h.dpass.size() * sizeof(DevPass), s_pass);
    const size_t o_st = put(h.dstages.data(), h.dstages.size() * sizeof(DevStage), s_st);
    const size_t o_aux = put(h.aux.data(), h.aux.size() * 8, s_aux);
    const size_t o_aux32 = put(h.aux32.data(), h.aux32.size() * 4, s_aux32);
    const size_t o_lt = put(h.ltab.data(), h.ltab.size() * sizeof(V2<R>), s_lt);
    const size_t o_mt = put(h.mtab.data(), h.mtab.size() * 4, s_mt);
    upload(ctx, dbase, host.data(), host.size());
    DevPlanDev<R> &d = *out;
    d.ops = (const DevOp<R> *)(dbase + o_ops);
    d.pass = (const DevPass *)(dbase + o_pass);
    d.stages = (const DevStage *)(dbase + o_st);
    d.aux = (const uint64_t *)(dbase + o_aux);
    d.aux32 = (const uint32_t *)(dbase + o_aux32);
    d.ltab = (const V2<R> *)(dbase + o_lt);
    d.mtab = (const float *)(dbase + o_mt);
    return total;
}

template <typename R>
DevPlanDev<R> upload_dev_plan(Ctx *ctx, const DevPlanHost<R> &h, const std::string &slot) {
    DevPlanDev<R> d;
    char *dbase = (char *)scratch(ctx, slot, place_dev_plan<R>(ctx, h, nullptr, nullptr));
    place_dev_plan<R>(ctx, h, dbase, &d);
    return d;
}
template DevPlanDev<float> upload_dev_plan<float>(Ctx *, const DevPlanHost<float> &, const std::string &);
template DevPlanDev<double> upload_dev_plan<double>(Ctx *, const DevPlanHost<double> &, const std::string &);

// Launch every pass of a plan over a slab of nc states (dim amplitudes
// each).  Sweep passes (the plain path) only exist for nc == 1.  With
// from_zero the first pass synthesises |0...0> instead of reading memory
// (it must be a tile pass then).
// Copy state 0 of a slab (dim amplitudes per state) into states [c0, c1):
// 16-byte accesses, one grid row per destination state.
template <typename R>
__global__ void k_bcast(V2<R> *__restrict__ slab, uint64_t dim, int c0) {
    const uint64_t nacc = dim * sizeof(V2<R>) / 16;
    const uint4 *src = reinterpret_cast<const uint4 *>(slab);
    uint4 *dst = reinterpret_cast<uint4 *>(slab + (uint64_t)(c0 + (int)blockIdx.y) * dim);
    for (uint64_t a = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; a < nacc; a += (uint64_t)gridDim.x * blockDim.x)
        dst[a] = src[a];
}

template <typename R>
void launch_plan(Ctx *ctx, const Plan &plan, const DevPlanHost<R> &h, const DevPlanDev<R> &d, V2<R> *slab,
                 uint64_t dim, int nc_all, const int *ovr_idx, const DevOp<R> *ovr, bool from_zero,
                 const int *nc_pass) {
    int joined = 0;
    for (size_t i = 0; i < plan.passes.size(); ++i) {
        const Pass &ps = plan.passes[i];
        // circuits [joined, nc) enter at this pass with circuit 0's state
        const int nc = nc_pass ? nc_pass[i] : nc_all;
        if (nc_pass && i > 0 && nc > joined) {
            if ((dim * sizeof(V2<R>)) % 16 != 0) fail(SV_EDEVICE, "internal: state too small to share");
            const uint64_t nacc = dim * sizeof(V2<R>) / 16;
            const unsigned gx = (unsigned)std::min<uint64_t>((nacc + 255) / 256, (uint64_t)ctx->cu_count * 8);
            LaunchScope ls(ctx, "share", 2.0 * (double)sizeof(V2<R>) * (double)dim * (nc - joined));
            for (int c = joined; c < nc; c += 32768) {  // grid rows (y) per launch
                const unsigned rows = (unsigned)std::min(nc - c, 32768);
                hipLaunchKernelGGL((k_bcast<R>), dim3(gx, rows), dim3(256), 0, ctx->stream, slab, dim, c);
                SV_HIP(hipGetLastError());
            }
        }
        joined = nc;
        const double S = (double)sizeof(V2<R>) * (double)dim * nc;
        if (ps.kind == PASS_SWEEP) {
            if (nc != 1 || ovr_idx) fail(SV_EDEVICE, "internal: sweep pass in a batched plan");
            sweep_one<R>(ctx, slab, plan.n, ps.ops[0]);
            continue;
        }
        const uint64_t tiles = 1ull << ps.free_bits.size();
        const uint32_t nhi = 1u << (ps.m - ps.l);
        const unsigned grid = tile_grid(tiles * (uint64_t)nc, ctx->cu_count);
        if (ps.kind == PASS_TILE) {
            const DevPass &dp = h.dpass[i];
            size_t lds = tile_lds_layout(nhi, dp.nlad, dp.ltab_count, sizeof(V2<R>), dp.paux_lds ? dp.paux_count : 0).end;
            if (dp.stage_end - dp.stage_begin > 1) lds += sizeof(V2<R>) << ps.m;
            LaunchScope ls(ctx, "tile", 2.0 * S);
            launch_tile<R>(ctx, tile_tpb(ps.m), lds, grid, slab, dim, nc, ovr_idx, ovr, d, (int)i, tiles,
                           from_zero && i == 0, dp.h4, ps.m);
        } else {
            if (from_zero && i == 0) fail(SV_EDEVICE, "internal: plan starts with a permutation");
            // k_perm moves at most 4 accesses per thread per tile
            if ((1u << ps.m) > 4u * TILE_TPB * (16 / sizeof(V2<R>)))
                fail(SV_EDEVICE, "internal: permutation tile too wide");
            const size_t lds = 2 * (sizeof(V2<R>) << ps.m) + 8 * nhi + 2 * 64 * 4;
            const uint32_t acc = (1u << ps.m) / (16 / sizeof(V2<R>));
            const int maxa = acc <= TILE_TPB ? 1 : acc <= 2 * TILE_TPB ? 2 : 4;
            auto go = [&](auto MA) {
                constexpr int M = decltype(MA)::value;
                set_lds_limit((const void *)k_perm<R, M>, lds);
                LaunchScope ls(ctx, "perm", 2.0 * S);
                hipLaunchKernelGGL((k_perm<R, M>), dim3(grid), dim3(TILE_TPB), lds, ctx->stream, slab, dim, nc,
                                   d.pass, (int)i, d.aux, d.aux32, tiles);
            };
            if (maxa == 1) go(std::integral_constant<int, 1>{});
            else if (maxa == 2) go(std::integral_constant<int, 2>{});
            else go(std::integral_constant<int, 4>{});
        }
        SV_HIP(hipGetLastError());
    }
}
template void launch_plan<float>(Ctx *, const Plan &, const DevPlanHost<float> &, const DevPlanDev<float> &,
                                 V2<float> *, uint64_t, int, const int *, const DevOp<float> *, bool, const int *);
template void launch_plan<double>(Ctx *, const Plan &, const DevPlanHost<double> &, const DevPlanDev<double> &,
                                  V2<double> *, uint64_t, int, const int *, const DevOp<double> *, bool,
                                  const int *);

template <typename R>
static void run_plan_t(Ctx *ctx, State *st, const Plan &plan) {
    DevPlanHost<R> h = build_dev_plan<R>(plan);
    DevPlanDev<R> d = upload_dev_plan<R>(ctx, h, "plan");
    launch_plan<R>(ctx, plan, h, d, reinterpret_cast<V2<R> *>(st->ptr), 1ull << st->n, 1, nullptr, nullptr, false);
}

void run_plan(Ctx *ctx, State *st, const Plan &plan) {
    if (st->dtype == SV_C64) run_plan_t<float>(ctx, st, plan);
    else run_plan_t<double>(ctx, st, plan);
}

// As run_plan, with the plan's device tables in a caller-provided block of
// cap bytes instead of a context buffer (no device allocation).
template <typename R>
static void run_plan_in_t(Ctx *ctx, State *st, const Plan &plan, void *block, size_t cap) {
    DevPlanHost<R> h = build_dev_plan<R>(plan);
    const size_t need = place_dev_plan<R>(ctx, h, nullptr, nullptr);
    if (need > cap)
        fail(SV_EINVAL, "the circuit's plan needs " + std::to_string(need) + " bytes of device tables; at most " +
                            std::to_string(cap) + " fit the preallocated block");
    DevPlanDev<R> d;
    place_dev_plan<R>(ctx, h, (char *)block, &d);
    launch_plan<R>(ctx, plan, h, d, reinterpret_cast<V2<R> *>(st->ptr), 1ull << st->n, 1, nullptr, nullptr, false);
}

void run_plan_in(Ctx *ctx, State *st, const Plan &plan, void *block, size_t cap) {
    if (st->dtype == SV_C64) run_plan_in_t<float>(ctx, st, plan, block, cap);
    else run_plan_in_t<double>(ctx, st, plan, block, cap);
}

void run_unfused(Ctx *ctx, State *st, const std::vector<Op> &ops) {
    for (const Op &op : ops) {
        if (st->dtype == SV_C64) sweep_one<float>(ctx, (V2<float> *)st->ptr, st->n, op);
        else sweep_one<double>(ctx, (V2<double> *)st->ptr, st->n, op);
    }
}

void set_zero_state(Ctx *ctx, void *psi, int n, int dtype) {
    const uint64_t dim = 1ull << n;
    const unsigned g = grid_for(dim, SWEEP_TPB, ctx->cu_count);
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_zero<float>, dim3(g), dim3(SWEEP_TPB), 0, ctx->stream, (V2<float> *)psi, dim);
    else
        hipLaunchKernelGGL(k_zero<double>, dim3(g), dim3(SWEEP_TPB), 0, ctx->stream, (V2<double> *)psi, dim);
    SV_HIP(hipGetLastError());
}

#ifdef SV_DEBUG_BOUNDS
// Debug build: one thread forms index 1 of a one-element buffer; the check
// replaces it by 0 (the store stays in bounds) and must raise the HBM flag.
__global__ void k_debug_bounds_probe(unsigned int *p) { p[SV_GIDX(1, 1)] = 7u; }

void debug_bounds_probe(Ctx *ctx) {
    unsigned int *p = nullptr;
    if (hipMalloc(&p, sizeof *p) != hipSuccess) {
        (void)hipGetLastError();
        fail(SV_ENOMEM, "debug probe buffer");
    }
    (void)take_bound_flags();
    hipLaunchKernelGGL(k_debug_bounds_probe, dim3(1), dim3(1), 0, ctx->stream, p);
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(p);
    if (e != hipSuccess) fail(SV_EDEVICE, std::string("debug probe: ") + hipGetErrorString(e));
    if (!(take_bound_flags() & 1u)) fail(SV_EDEVICE, "debug build: index checks do not report");
}
#endif

void device_scale(Ctx *ctx, void *psi, int n, int dtype, double s) {
    const uint64_t dim = 1ull << n;
    const unsigned g = grid_for(dim, SWEEP_TPB, ctx->cu_count);
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_scale<float>, dim3(g), dim3(SWEEP_TPB), 0, ctx->stream, (V2<float> *)psi, dim, s);
    else
        hipLaunchKernelGGL(k_scale<double>, dim3(g), dim3(SWEEP_TPB), 0, ctx->stream, (V2<double> *)psi, dim, s);
    SV_HIP(hipGetLastError());
}


}  // namespace sv
