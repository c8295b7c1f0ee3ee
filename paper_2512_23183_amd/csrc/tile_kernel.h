// The tile-pass kernel, instantiated per workgroup size in tile_t*.hip.
#pragma once
#include "device_common.h"
#include "tile_h4.h"

namespace sv {

// Tile passes over a slab of nc states of dim amplitudes each (one state:
// nc = 1).  Each workgroup walks the work items w = blockIdx.x,
// +gridDim.x, ... with w = circuit * ntiles + tile, so neighbouring
// workgroups share a circuit.  Circuit c applies op ovr_idx[c] as ovr[c]
// (parameter-shift copies); from_zero makes the reads synthesise |0...0>.
// LDS layout (16-byte aligned parts): hi_off[2^(m-l)], the per-tile ladder
// factors Gs[nlad], the pass's ladder tables when they fit
// (ltab_count <= LTAB_LDS_CAP; else they are read from global memory), then
// the tile (2^m amplitudes, only for multi-stage passes).
// H4: 0 = three-bit register stages; four-bit stages (tile_h4.h) with
// 1 = one-qubit gates, ladders and diagonals, 2 = Hadamards, ladders and
// pattern diagonals only, 3 = Hadamards, real rotations and diagonals only,
// 4 = rotation layers (straight-line stages, see build_rotation_layers).
// ONE (four-bit stages): at most one group per thread, see h4_stage.
template <typename R, int TPB, int H4, bool ONE = false>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : (H4 >= 3 ? 2 : 1)))) void k_tile(V2<R> *__restrict__ slab, uint64_t dim, int nc,
                                                   const int *__restrict__ ovr_idx,
                                                   const DevOp<R> *__restrict__ ovr,
                                                   const DevPass *__restrict__ passes, int pidx,
                                                   const DevStage *__restrict__ stages,
                                                   const DevOp<R> *__restrict__ ops,
                                                   const uint64_t *__restrict__ aux,
                                                   const uint32_t *__restrict__ aux32,
                                                   const V2<R> *__restrict__ ltab,
                                                   const float *__restrict__ mtab, uint64_t ntiles, int from_zero) {
    extern __shared__ __align__(16) unsigned char smem[];
    const DevPass &P = passes[pidx];
    TileCtx<R> tc;
    tc.m = P.m;
    tc.l = P.l;
    tc.lowm = (1u << P.l) - 1;
    tc.ident = false;
    tc.zero = from_zero != 0;
    tc.paux = aux32;
    tc.mtab = mtab;
    tc.dim = dim;
    const uint32_t nhi = 1u << (P.m - P.l);
    uint64_t *hi_off = reinterpret_cast<uint64_t *>(smem);
    tc.hi_off = (const SV_LDS uint64_t *)hi_off;
    ladder_split(P.m, tc.lsa, tc.lsb);
    const LdsLayout lay = tile_lds_layout(nhi, P.nlad, P.ltab_count, sizeof(V2<R>), P.paux_lds ? P.paux_count : 0);
    V2<R> *Gs = reinterpret_cast<V2<R> *>(smem + lay.gs);
    V2<R> *ltl = reinterpret_cast<V2<R> *>(smem + lay.tabs);
    V2<R> *tile = reinterpret_cast<V2<R> *>(smem + lay.tile);
    tc.Gs = (const SV_LDS R *)Gs;
    tc.ltl = lay.tabs_in_lds ? (const SV_LDS R *)ltl : nullptr;
    tc.ltabs = ltab + P.ltab_begin;
    for (uint32_t h = threadIdx.x; h < nhi; h += TPB) hi_off[h] = aux[P.hi_begin + h];
    if (lay.tabs_in_lds)
        for (int i = threadIdx.x; i < P.ltab_count; i += TPB) ltl[i] = ltab[P.ltab_begin + i];
    tc.pauxl = nullptr;
    tc.paux_off = 0;
    if (P.paux_lds) {
        uint32_t *pl = reinterpret_cast<uint32_t *>(smem + lay.paux);
        for (int i = threadIdx.x; i < P.paux_count; i += TPB) pl[i] = aux32[P.paux_begin + i];
        tc.pauxl = (const SV_LDS uint32_t *)pl;
        tc.paux_off = P.paux_begin;
    }
    const uint64_t fmask = P.free_mask;
    const int sb = P.stage_begin, se = P.stage_end;
    __syncthreads();
    const uint64_t nw = (uint64_t)nc * ntiles;
    const int lt = __builtin_ctzll(ntiles);
    for (uint64_t w = blockIdx.x; w < nw; w += gridDim.x) {
        const uint64_t c = w >> lt, t = w & (ntiles - 1);  // ntiles: a power of two
        tc.base = deposit(t, fmask);
        if (P.nlad) {
            // the tile's factor of every ladder: the phase of its fixed bits
            for (int i = threadIdx.x; i < P.nlad; i += TPB) {
                const DevOp<R> &op = ops[aux32[P.lad_list + i]];
                Gs[i] = ladder_phase<R>(op.turns, tc.base & op.lmask);
            }
            __syncthreads();
        }
        const int oi = ovr_idx ? ovr_idx[c] : -1;
        // pass scale of this circuit: with its shifted op in this pass, the
        // product of the pass's factors taken with the shifted op's own
        // (formed on the host in op order, as for a one-circuit plan)
        const double sc = (oi >= P.op_begin && oi < P.op_end) ? ovr[c].pscale : P.scale;
        tc.scale = (R)sc;
        tc.scaled = sc != 1.0;
        tc.has_tf = false;
        if constexpr (H4 == 4) {
            // the tile's factor of the diagonals on bits outside it, times
            // the pass scale (one complex multiply in the last store)
            if (P.tf_end > P.tf_begin) {
                V2<R> f;
                f.x = (R)1;
                f.y = (R)0;
                for (int o = P.tf_begin; o < P.tf_end; ++o) diag_factor(f, tc.base, ops[o]);
                tc.tf.x = f.x * tc.scale;
                tc.tf.y = f.y * tc.scale;
                tc.has_tf = true;
            }
        }
        if constexpr (H4 != 0)
            run_stages_h4<R, TPB, H4, ONE>(tile, slab + c * dim, tc, stages, sb, se, ops, oi, ovr ? ovr + c : nullptr);
        else run_stages<R, TPB>(tile, slab + c * dim, tc, stages, sb, se, ops, oi, ovr ? ovr + c : nullptr);
    }
}


template <typename R, int TPB>
void launch_tile_tpb(Ctx *ctx, size_t lds, unsigned grid, V2<R> *slab, uint64_t dim, int nc, const int *ovr_idx,
                     const DevOp<R> *ovr, const DevPlanDev<R> &d, int pidx, uint64_t tiles, bool from_zero, int h4,
                     bool one) {
    // one: 2^m / 16 <= TPB (four-bit stages: true at every width with
    // fewer than 512 threads; at 512 threads up to m = 13)
    auto go = [&](auto H) {
        constexpr int H4 = decltype(H)::value;
        auto run = [&](auto O) {
            constexpr bool ONE = decltype(O)::value;
            set_lds_limit((const void *)k_tile<R, TPB, H4, ONE>, lds);
            hipLaunchKernelGGL((k_tile<R, TPB, H4, ONE>), dim3(grid), dim3(TPB), lds, ctx->stream, slab, dim, nc,
                               ovr_idx, ovr, d.pass, pidx, d.stages, d.ops, d.aux, d.aux32, d.ltab, d.mtab, tiles,
                               from_zero ? 1 : 0);
        };
        if constexpr (H4 == 0) run(std::false_type{});
        else if constexpr (TPB < 512) {
            if (!one) fail(SV_EDEVICE, "internal: more than one group per thread below 512 threads");
            run(std::true_type{});
        }
        else if (one) run(std::true_type{});
        else run(std::false_type{});
    };
    if (h4 == 1) go(std::integral_constant<int, 1>{});
    else if (h4 == 2) go(std::integral_constant<int, 2>{});
    else if (h4 == 3) go(std::integral_constant<int, 3>{});
    else if (h4 == 4) go(std::integral_constant<int, 4>{});
    else go(std::integral_constant<int, 0>{});
    SV_HIP(hipGetLastError());
}

#define SV_TILE_INSTANTIATE(TPB)                                                                              \
    template void launch_tile_tpb<float, TPB>(Ctx *, size_t, unsigned, V2<float> *, uint64_t, int, const int *, \
                                              const DevOp<float> *, const DevPlanDev<float> &, int, uint64_t,   \
                                              bool, int, bool);                                                \
    template void launch_tile_tpb<double, TPB>(Ctx *, size_t, unsigned, V2<double> *, uint64_t, int,           \
                                               const int *, const DevOp<double> *, const DevPlanDev<double> &,  \
                                               int, uint64_t, bool, int, bool);

}  // namespace sv
