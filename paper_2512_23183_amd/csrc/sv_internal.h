// Internal declarations of libsv: the lowered gate IR, the pass plan, the
// context / state objects and the kernel launchers.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <complex>
#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "sv.h"

namespace sv {

using cd = std::complex<double>;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------

struct Error {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const std::string &msg);
// Debug kernel build (SV_DEBUG_BOUNDS): each translation unit with kernels
// registers a reader that returns and clears its out-of-range flags
// (bit 0: an HBM index, bit 1: an LDS index); the API reports them.
bool register_bound_flag_reader(uint32_t (*reader)());
uint32_t take_bound_flags();
#ifdef SV_DEBUG_BOUNDS
struct Ctx;
void debug_bounds_probe(Ctx *ctx);  // at context creation: the checks must report
#endif
void set_last_error(const std::string &msg);

#define SV_HIP(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess)                                                 \
            ::sv::fail(SV_EDEVICE, std::string(#call) + ": " +                \
                                       hipGetErrorString(e_));                \
    } while (0)

// ---------------------------------------------------------------------------
// Lowered operations.  Every gate lowers to exactly one Op acting on index
// BIT positions (bit = n-1-qubit).  Matrices are computed on the host in FP64
// and rounded once to the state's precision when uploaded.
// ---------------------------------------------------------------------------

enum OpKind : int32_t {
    OP_U1 = 0,      // 2x2 matrix m[0..3] on bit a, where all cmask bits set
    OP_U2 = 1,      // 4x4 matrix m[0..15] on bits (a, b), a = high matrix bit
    OP_DIAG = 2,    // amplitude *= m[2*bit_a + bit_b] (b < 0: m[bit_a]), cmask
    OP_LADDER = 3,  // if bit a set: amplitude *= exp(2 pi i turns (k & lmask))
    OP_SWAP = 4,    // exchange bits a and b, where all cmask bits set
    OP_XPERM = 5,   // CNOT-like: swap pair on bit a where all cmask bits set
    OP_DENSE4 = 6,  // dense 16x16 matrix (Plan::dense[dense]) on the four bits
                    // of lmask, pattern bit k = the k-th lowest of them; made
                    // by the planner from runs of fixed gates (MFMA stages)
    OP_ROT4 = 8,    // device only: the four real rotations of a rotation-layer
                    // stage, slot i: (x, y) <- (x - t y, y + t x) with t in the
                    // real part of complex entry i (0 = none); their cosines are
                    // in the pass scale
    OP_DIAG16 = 7,  // device only: the gathered diagonals of a four-bit stage,
                    // element e of a register group *= m[e] (complex), negated
                    // where the parity of e & c is odd; bit r of c is the
                    // parity of k & M_r with M_0..3 in cmask, lcmask, gcmask,
                    // lmask (CZ-like couplings to bits outside the registers)
};

struct Op {
    int32_t kind = OP_U1;
    int32_t a = -1, b = -1;
    uint64_t cmask = 0;
    uint64_t lmask = 0;
    double turns = 0.0;
    double ang = 0.0;      // CP: its angle (kept exact for ladder merging)
    cd m[16];
    int32_t gate = -1;     // source gate index (-1 = synthesised)
    int32_t dense = -1;    // OP_DENSE4: index of its matrix in Plan::dense
    bool param = false;    // angle depends on the parameter vector
    bool real_family = false;  // real matrix at every angle (RY, CRY)
    bool diagonal() const { return kind == OP_DIAG || kind == OP_LADDER; }
};

// Device copy of an op in precision R (float for complex64, double for
// complex128).  la / lb are the tile-local positions of a / b in the pass
// that holds the op; lcmask / gcmask split cmask into tile-local (re-indexed)
// and fixed-per-tile parts.
template <typename R>
struct alignas(16) DevOp {
    int32_t kind, a, b, la, lb;
    int32_t ra, rb;   // register slots (0..2) of la / lb within the op's stage
    int32_t tslot;    // LADDER: phase-table slot within the stage
    uint64_t cmask;   // global positions
    uint64_t lcmask;  // local positions of the controls inside the tile
    uint64_t gcmask;  // controls outside the tile (constant per tile)
    uint64_t lmask;
    double turns;
    int32_t flags;    // OPF_* below
    int32_t tab;      // LADDER: offset of its host-built phase tables
    double sfac;      // OPF_HAD / OPF_ROTC / OPF_ROTS: factor taken out
    double pscale;    // replacement op of a batched circuit: the scale of the
                      // pass that holds it, with its own factor in its place
    R m[32];          // complex entries as (re, im)
};
enum {
    OPF_REAL = 1,  // 2x2 matrix with real entries (H, RY): cheaper butterfly
    OPF_PAT = 2,   // DIAG whose only factor != 1 is on the all-ones pattern
    OPF_NEG = 4,   // ... and that factor is exactly -1 (CZ)
    // placement flags (set per stage by the stage builder):
    OPF_GRP = 8,   // DIAG on bits outside the stage's registers: one factor
                   // per register group, accumulated and applied once
    OPF_REG1 = 16, // one-qubit DIAG without controls on register bit ra:
                   // d0 goes to the group factor, the elements with the bit
                   // set are multiplied by d1 / d0 (entry 4 of m)
    // uncontrolled real one-qubit ops with a factor sfac taken out, applied
    // once per tile pass (the pass scale):
    OPF_HAD = 32,  // s [[1, 1], [1, -1]]: sums and differences
    OPF_ROTC = 64, // c [[1, -t], [t, 1]], t = s / c (|t| <= 1) in m[10]
    OPF_ROTS = 128,// s [[u, -1], [1, u]], u = c / s (|u| < 1) in m[10]
    OPF_PARAMC = 256, // parameterised, and its matrix class may change with
                      // the parameter (not RY / CRY): decides pass kernels
    OPF_SGN = 512,    // OP_DIAG16 with sign couplings
};
constexpr int OPF_SCALED = OPF_HAD | OPF_ROTC | OPF_ROTS;
constexpr int OPF_PLACEMENT = OPF_GRP | OPF_REG1;

// Lower one validated gate (kind, qubits, effective angles, user matrix) to
// its op.  mat = 8 or 32 doubles for MAT1 / MAT2.
Op lower_gate(int n, const sv_gate &g, const double ang[3], const double *mat,
              int gate_index);

// Gate list of Alg. "Gate-Based QFT" over n qubits.
std::vector<sv_gate> qft_gates(int n);

// Effective angles of gate g (angle[k] + params[param_idx[k]]).
void effective_angles(const sv_gate &g, const double *params, double out[3]);

// ---------------------------------------------------------------------------
// Plan: passes over the state.  A TILE pass loads 2^m amplitudes whose index
// bits outside the tile are fixed (one workgroup per tile), runs its ops in
// LDS and writes the tile back.  A PERM pass exchanges bit pairs in place.
// ---------------------------------------------------------------------------

enum PassKind : int32_t { PASS_TILE = 0, PASS_PERM = 1, PASS_SWEEP = 2 };

struct Pass {
    int32_t kind = PASS_TILE;
    int32_t m = 0;                    // tile bits
    int32_t l = 0;                    // low identity bits (coalescing run)
    std::vector<int> local_bits;      // global bit of local bit i, i < m
    std::vector<int> free_bits;       // global bits outside the tile
    std::vector<Op> ops;              // ops of the pass, in order
    std::vector<std::pair<int, int>> swaps;  // PERM: disjoint bit pairs
};

struct PlanOptions {
    int tile_bits = 13;    // m
    int tile_bits_layers = 0;  // m of layered circuits (only uncontrolled one-qubit
                               // gates and diagonals; 0: tile_bits)
    int low_bits = 4;      // l: 128 B (complex64) / 256 B (complex128) contiguous runs
    int perm_bits = 11;    // tile width of permutation passes
    bool fuse = true;      // false: one sweep op per gate
    bool dense4 = false;   // fuse runs of fixed gates on four bits into OP_DENSE4
    int dense_force = 0;   // 2..4: every run of >= 2 fixed gates on <= k bits becomes a
                           // block (padded to four bits), whatever its cost
    bool order_layers = true;  // list-schedule the ops of layered passes into few stages
};

struct Plan {
    int n = 0;
    std::vector<Pass> passes;
    int n_gate_ops = 0;
    std::vector<std::vector<cd>> dense;  // 16x16 row-major matrices of OP_DENSE4 ops
};

// Build passes from ops.  SWAP ops are absorbed into a bit relabelling and
// the final layout is restored by PERM passes.
Plan make_plan(int n, const std::vector<Op> &ops, const PlanOptions &opt);

// A stage: ops [op_begin, op_end) applied to 8-amplitude register groups
// (register bits r0 < r1 < r2), then the group is stored.  With perm the
// store goes through P(j) = A j ^ c, the composition of the single-control
// CNOTs and X gates that follow the stage's ops (folded out of the op list):
// P(j0 | loff_e) = tab_lo[j0 & 127] ^ tab_hi[j0 >> 7] ^ pd[e], tables at
// perm_tab in the plan's 32-bit aux array.
struct alignas(16) DevStage {
    int32_t r0, r1, r2;
    int32_t op_begin, op_end;
    int32_t has_diag;
    int32_t perm;
    int32_t perm_tab;
    int32_t acc;      // some DIAG op uses the per-group factor
    int32_t mfma;     // 1: the stage is one OP_DENSE4 op on bits r0 < r1 < r2 < r3
    int32_t r3;
    int32_t wtab;     // MFMA stage: its 32x32 real matrix in the plan's float table
    // rotation-layer stages (four-bit kind 4): op indices of the table
    // applied before the rotations, of the one after them, and of the
    // OP_ROT4 op holding the four rotations (-1 = none); the stage's op
    // range then lists the diagonals that feed the group factor
    int32_t tpre, tpost, rot;
    int32_t rl;       // rotation-layer code variant: 1 = a table before the
                      // rotations, 2 = sign couplings in its tables, 4 = a
                      // group factor
    uint16_t pd[8];
    // four-bit stages: the local bit taken by each bit of a thread's group
    // index, 4 bits per entry from index bit 0 (see h4_lane_order)
    uint64_t lane_pos;
};

// Device pass descriptor.  Per-pass tables live in an auxiliary array:
// hi_off (global offset of each combination of the high local bits) and,
// for PERM passes, the local permutation of tile positions.
struct alignas(16) DevPass {
    int32_t kind, m, l, nfree;
    int32_t op_begin, op_end, stage_begin, stage_end;
    uint64_t free_mask;        // index bits outside the tile
    int32_t hi_begin;          // offset of hi_off in the 64-bit aux array
    int32_t lperm_begin;       // PERM: offset of the local permutation (32-bit aux)
    int32_t nfp;               // PERM: bit pairs outside the tile
    int32_t pad;
    int8_t fpa[24], fpb[24];   // PERM: those pairs
    double scale;              // TILE: product of the deferred factors sfac
    int32_t lad_list, nlad;    // TILE: ladder ops (indices in the 32-bit aux array)
    int32_t ltab_begin, ltab_count;  // TILE: their phase tables in the plan's table array
    int32_t paux_begin, paux_count;  // TILE: its stages' layout-map tables (32-bit aux array)
    int32_t paux_lds;                // TILE: 1 = those tables are copied to LDS
    int32_t h4;                      // TILE: four-bit stages (1 general, 2 Hadamard / ladder only,
                                     // 3 rotation / diagonal, 4 rotation layers)
    int32_t tf_begin, tf_end;        // kind 4: diagonals on bits outside the tile (one
                                     // factor per tile, applied with the pass scale)
};
// k_perm reads fpa and fpb as twelve consecutive 32-bit words
static_assert(offsetof(DevPass, fpa) % 4 == 0 && offsetof(DevPass, fpb) == offsetof(DevPass, fpa) + 24,
              "DevPass pair arrays must be word-aligned and adjacent");

// ---------------------------------------------------------------------------
// Pauli sums lowered to masks (bit positions).
// ---------------------------------------------------------------------------

struct Term {
    uint64_t x = 0, z = 0;  // bit masks of X/Y and Z/Y factors
    int ny = 0;             // number of Y factors (mod 4)
    double c = 0.0;
};

struct TermGroups {
    // terms sorted into groups sharing x; order inside a group = term order
    std::vector<uint64_t> gx;           // group x mask
    std::vector<int> g_begin, g_end;    // ranges into `order`
    std::vector<int> order;             // term indices
    std::vector<Term> terms;            // as given
};
TermGroups lower_pauli_sum(const sv_pauli_sum &h);

struct alignas(16) DevTerm {
    uint64_t x, z;
    int32_t ny, idx;    // idx = original term index
    double c;
};

// ---------------------------------------------------------------------------
// Context / state
// ---------------------------------------------------------------------------

struct ProfileEntry {
    double ms = 0.0;
    uint64_t launches = 0;
    double bytes = 0.0;
};

struct DeviceBuffer {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// Largest tile widths whose LDS footprint fits one workgroup (160 KiB):
// gate tiles hold 2^m amplitudes plus up to four ladder tables, expectation
// tiles 2^m amplitudes plus term accumulators, permutation passes two tiles.
constexpr int TILE_MAX[2] = {14, 12};
constexpr int EXPECT_MAX[2] = {14, 13};
constexpr int PERM_MAX[2] = {12, 11};

struct Ctx {
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    // widths in bits, indexed by dtype (0 = complex64, 1 = complex128):
    // gate tile passes, expectation passes, permutation passes
    // (ranges: TILE_MAX / EXPECT_MAX / PERM_MAX below, minimum 6)
    int tile_bits[2] = {12, 12};
    int tile_bits_layers[2] = {12, 12};  // layered circuits (see PlanOptions)
    int expect_bits[2] = {13, 12};
    int perm_bits[2] = {12, 11};
    bool dense4 = true;  // complex64 circuits: MFMA stages for dense four-qubit runs
    int dense_force = 0; // 2..4: blocks of width <= k on every run (measurement mode)
    std::mutex mu;
    // states created on this context and not yet freed (sv_shutdown refuses
    // to run while any is alive: they reference the context's stream)
    std::atomic<int> live_states{0};
    // fault injection (environment variable SV_FAULT_ALLOC=N at sv_init):
    // the context's N-th device allocation fails as if HBM were exhausted
    int fault_alloc = 0;
    std::atomic<uint64_t> n_allocs{0};
    // scratch buffers reused across calls (grown on demand)
    std::map<std::string, DeviceBuffer> scratch;
    // batched executor: the launches of one batch call are recorded and
    // replayed as one hipGraph launch (graph_exec is reused through
    // hipGraphExecUpdate while the launch sequence keeps its shape)
    bool graphs = true;
    std::vector<std::function<void()>> *record = nullptr;  // non-null while recording
    std::vector<std::string> record_slots;                  // scratch slots touched while recording
    hipGraphExec_t graph_exec = nullptr;
    uint64_t graph_launches = 0, graph_instantiations = 0;
    // pinned host staging for the uploads and results of one batch call
    // (run_batch synchronises before returning, so the arena is reused)
    char *pinned = nullptr;
    size_t pinned_cap = 0, pinned_used = 0;
    bool pinned_on = false;
    // profiling
    bool profile = false;
    std::map<std::string, ProfileEntry> prof;
    std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> free_events;
    std::vector<double> pending_bytes;
};

struct State {
    Ctx *ctx = nullptr;
    int n = 0;
    int dtype = SV_C64;
    void *ptr = nullptr;
    bool owned = true;
    size_t amp_bytes() const { return dtype == SV_C64 ? 8 : 16; }
    size_t bytes() const { return amp_bytes() << n; }
};

// Every device allocation of the library goes through here (counted per
// context, for the fault-injection hook).
hipError_t dev_malloc(Ctx *ctx, void **p, size_t bytes);
void *scratch(Ctx *ctx, const std::string &name, size_t bytes);
// Kernel launches of the batched executor go through here: run now, or
// appended to ctx->record (no allocation or upload may happen inside f).
void launch_or_record(Ctx *ctx, std::function<void()> f);
// Launch the recorded work as one hipGraph on ctx->stream.
void launch_recorded(Ctx *ctx, std::vector<std::function<void()>> &work);
void release_graph(Ctx *ctx);
// Pinned staging of a synchronous batch call: uploads between begin and end
// go through a pinned arena (released by release_pinned).
void pinned_begin(Ctx *ctx);
void pinned_end(Ctx *ctx);
void release_pinned(Ctx *ctx);

// Profiling hooks around a launch.
struct LaunchScope {
    Ctx *ctx;
    const char *name;
    double bytes;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LaunchScope(Ctx *c, const char *nm, double b);
    ~LaunchScope();
};
void profile_collect(Ctx *ctx);

// ---------------------------------------------------------------------------
// Executors (implemented in the .hip files)
// ---------------------------------------------------------------------------

// Run a plan on one state (ops uploaded per call).
void run_plan(Ctx *ctx, State *st, const Plan &plan);
// What a device plan holds (host only: sv_plan_info / sv_plan_dump).
struct PlanSummary {
    int sweep_passes = 0, tile_passes = 0, perm_passes = 0, stages = 0, ops = 0;
    int h4_passes[5] = {0, 0, 0, 0, 0};
    int dense_blocks = 0, tables = 0, tile_factor_ops = 0;
    double min_scale = 1e300, max_scale = 0.0;
};
template <typename R>
PlanSummary summarize_plan(const Plan &plan, std::string *text);

// As run_plan with the plan's device tables in a given block of cap bytes
// (SV_EINVAL, before any device work, if they do not fit).
void run_plan_in(Ctx *ctx, State *st, const Plan &plan, void *block, size_t cap);

// The preallocated block of the no-allocation entry point: its size, its
// per-device set-up (at context creation) and its device address.
constexpr size_t NOALLOC_BLOCK_BYTES = SV_NOALLOC_BLOCK_BYTES;
void noalloc_setup(int device);
void *noalloc_block(int device);
// One-gate-per-launch sweeps (the plain path).
void run_unfused(Ctx *ctx, State *st, const std::vector<Op> &ops);
void set_zero_state(Ctx *ctx, void *psi, int n, int dtype);
// Tile-width autotuner (tune.cpp): times candidates through the public
// entry points on the handle ctx_ (the same context as ctx).
void autotune(Ctx *ctx, sv_ctx *ctx_, int dtype, int n_qubits, const char *cache_path);
void device_norm2(Ctx *ctx, const void *psi, int n, int dtype, double *out);
void device_scale(Ctx *ctx, void *psi, int n, int dtype, double s);
// FP64 expectation of a lowered Pauli sum: fills per-term values (already
// divided by the norm) and the energy.
void device_expectation(Ctx *ctx, const void *psi, int n, int dtype,
                        const TermGroups &tg, double *energy,
                        double *term_values, double *norm2);

// Batched evaluation of many independent circuits, each from |0...0>.
// Circuit c runs op set `op_set`, with op `ovr_index` of that set replaced
// by `ovr_op` (-1 = none; the parameter-shift copies), and reduces the
// energy of Hamiltonian `ham`.
struct BatchCircuit {
    int n = 0;
    int op_set = 0;
    int ovr_index = -1;
    Op ovr_op;
    int ham = 0;
    int out_slot = -1;   // energy slot in the output array (-1 = own index)
};
struct BatchSpec {
    int dtype = SV_C64;
    std::vector<std::vector<Op>> op_sets;
    std::vector<TermGroups> hams;
    std::vector<BatchCircuit> circuits;
    // optional gradient combination: grad[i] = sum_j w[j] * E[circ[j]],
    // j in [comb_begin[i], comb_begin[i+1])
    std::vector<int> comb_begin, comb_circ;
    std::vector<double> comb_w;
};
// Energies of all circuits (and the combined gradient when requested).
void run_batch(Ctx *ctx, const BatchSpec &spec, uint32_t flags,
               std::vector<double> &energies, std::vector<double> &grad);
// Device-resident variant: energies go to d_E[out_slot] and, when d_grad is
// non-null, the combined gradient to d_grad; nothing is synchronised.
void run_batch_dev(Ctx *ctx, const BatchSpec &spec, uint32_t flags, double *d_E, double *d_grad = nullptr);
// grad[i] = sum_j w[j] * E[circ[j]] on the device (fixed order).
void combine_dev(Ctx *ctx, const double *d_E, const std::vector<int> &beg,
                 const std::vector<int> &circ, const std::vector<double> &w,
                 double *d_grad);
BatchSpec psr_spec(const sv_circuit *c, const double *params, size_t n_params,
                   const sv_pauli_sum *ham, int dtype, bool want_grad);
int small_batch_max_qubits(int dtype);

// Host validation shared by the entry points (lower.cpp).
void check_circuit(const sv_circuit *c, const double *params, size_t n_params);
void check_pauli_sum(const sv_pauli_sum *h, int n);
const std::string &last_error();
int gate_arity(int kind);
int gate_n_angles(int kind);

}  // namespace sv
