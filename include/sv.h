/*
 * sv.h -- C ABI of libsv.so, an MI355X (gfx950) state-vector simulator for
 * the gate / expectation / parameter-shift hot path of LogosQ
 * (arxiv 2512.23183).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an sv_status (0 = SV_OK, negative = error).  No
 *    C++ exception, abort or HIP error escapes the ABI.  On error a
 *    human-readable message is available from sv_last_error() (thread-local;
 *    valid until the next sv_* call on the same thread).
 *  - All arguments are validated on the host BEFORE any device work is
 *    enqueued; an invalid argument returns SV_EINVAL and leaves device state
 *    untouched.  The paper's unchecked insertion path (Sec. "Circuit Data
 *    Structure", add_operation_unchecked) is deliberately not mirrored.
 *  - Input arrays (gates, matrices, parameters, Pauli strings, host
 *    amplitudes) are borrowed for the duration of the call only; the library
 *    copies what it keeps.  Outputs are written to caller-owned buffers.
 *  - States are owned by the library (sv_alloc .. sv_free), except states
 *    made by sv_wrap, whose device memory stays owned by the caller.
 *  - Qubit q corresponds to amplitude-index bit n-1-q ("MSB-first"; Alg.
 *    "Direct State Vector CNOT" and the worked examples of App. A and B).
 *    Amplitudes are interleaved (re, im) pairs: float for SV_C64, double for
 *    SV_C128.
 *  - A non-finite energy or gradient is reported as SV_ENUMERIC, never
 *    returned silently (App. D: explicit error reporting instead of silent
 *    NaN or empty gradients).
 *  - Device work runs on the context's stream (sv_set_stream); calls that
 *    return host results synchronise that stream before returning.
 */
#ifndef SV_ABI_H_INCLUDED
#define SV_ABI_H_INCLUDED

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SV_OK = 0,
    SV_EINVAL = -1,     /* invalid argument (nothing was enqueued)          */
    SV_ENOMEM = -2,     /* device or host allocation failed                 */
    SV_EDEVICE = -3,    /* a HIP call failed                                */
    SV_EBUSY = -4,      /* request exceeds the queue's memory budget        */
    SV_ENUMERIC = -5,   /* result not finite                                */
    SV_ECANCELED = -6,  /* request was cancelled                            */
    SV_ENODEV = -7,     /* no usable gfx950 device                          */
    SV_ETIMEDOUT = -8   /* sv_queue_wait timed out (request still pending)  */
} sv_status;

/* Amplitude precision: complex64 = pair of float, complex128 = pair of double. */
typedef enum { SV_C64 = 0, SV_C128 = 1 } sv_dtype;

/*
 * Gate kinds.  Angles are the gate's effective angles (see sv_gate).
 *  H, X, Y, Z           fixed one-qubit gates (H as printed in App. C)
 *  RX, RY, RZ (t)       exp(-i t P / 2) (generator form given with
 *                       Eq. "parameter_shift"); RZ = diag(e^{-it/2}, e^{it/2})
 *  U3 (t, p, l)         OpenQASM 2 U3 (not defined in the paper; the paper
 *                       names OpenQASM as its circuit format)
 *  CNOT (c, t)          Alg. "Direct State Vector CNOT"
 *  CZ (a, b)            diag(1, 1, 1, -1)
 *  CP (a, b; p)         diag(1, 1, 1, e^{ip}); the controlled phase of Alg.
 *                       "Gate-Based QFT"
 *  SWAP (a, b)          exchange of two qubits (Alg. "Gate-Based QFT")
 *  CRX/CRY/CRZ (c, t; t) |0><0|_c x I + |1><1|_c x R_P(t)_t (App. D circuit)
 *  CCX (c1, c2, t)      Toffoli, Alg. "Direct State Vector Toffoli" (App. B)
 *  RXX/RYY/RZZ (a,b; t) exp(-i t/2 P x P), the Trotter two-qubit rotations
 *                       of Sec. "XYZ Heisenberg Model"
 *  MAT1 (q)             user 2x2 matrix (apply_single_qubit_matrix of
 *                       Sec. "Circuit Data Structure")
 *  MAT2 (a, b)          user 4x4 matrix (apply_two_qubit_matrix); the 4x4 row
 *                       / column index is 2*bit(a) + bit(b)
 */
typedef enum {
    SV_H = 0, SV_X = 1, SV_Y = 2, SV_Z = 3,
    SV_RX = 4, SV_RY = 5, SV_RZ = 6, SV_U3 = 7,
    SV_CNOT = 8, SV_CZ = 9, SV_CP = 10, SV_SWAP = 11,
    SV_CRX = 12, SV_CRY = 13, SV_CRZ = 14, SV_CCX = 15,
    SV_RXX = 16, SV_RYY = 17, SV_RZZ = 18,
    SV_MAT1 = 19, SV_MAT2 = 20,
    SV_NUM_GATE_KINDS = 21
} sv_gate_kind;

/*
 * One gate occurrence (Sec. "Circuit Data Structure", Operation), 56 bytes.
 *   kind        sv_gate_kind
 *   q[3]        qubit operands, controls first; unused slots ignored
 *   param_idx[3] for each angle slot: index into the parameter vector, or -1
 *   mat_idx     MAT1 / MAT2: row of sv_circuit.mats; otherwise ignored
 *   angle[3]    fixed angle (or offset) per slot
 * Effective angle k = angle[k] + (param_idx[k] >= 0 ? params[param_idx[k]] : 0)
 * -- the circuit-rebuilding model of Sec. "Circuit Rebuilding Architecture":
 * every evaluation instantiates its gates from the parameter vector.
 */
typedef struct sv_gate {
    int32_t kind;
    int32_t q[3];
    int32_t param_idx[3];
    int32_t mat_idx;
    double angle[3];
} sv_gate;

/*
 * A gate list (Sec. "Circuit Data Structure", Circuit; Sec. "Compile-Time
 * Type Safety", ParameterizedCircuit).
 *   n_qubits   1..SV_MAX_QUBITS
 *   n_params   length the parameter vector must have (the length assert of
 *              build_circuit becomes an SV_EINVAL)
 *   gates      n_gates records
 *   mats       n_mats rows of 32 doubles: a row-major complex matrix as
 *              (re, im) pairs; a 2x2 uses the first 8 doubles, a 4x4 all 32
 */
typedef struct sv_circuit {
    int32_t n_qubits;
    int32_t n_params;
    const sv_gate *gates;
    size_t n_gates;
    const double *mats;
    size_t n_mats;
} sv_circuit;

/*
 * H = sum_t coeffs[t] P_t with P_t a Pauli string (VQE "Problem
 * Formulation"; Eq. "xyz_hamiltonian" and Eq. "energy_expectation").
 * paulis holds n_terms rows of n_qubits characters from "IXYZ"; character q
 * of row t is the factor on qubit q.  No terminating NULs are needed.
 */
typedef struct sv_pauli_sum {
    int32_t n_qubits;
    size_t n_terms;
    const double *coeffs;
    const char *paulis;
} sv_pauli_sum;

#define SV_MAX_QUBITS 34       /* 2^34 complex128 = 256 GiB < 288 GB HBM  */
#define SV_MAX_GATES (1u << 24)
#define SV_MAX_TERMS (1u << 20)

typedef struct sv_ctx sv_ctx;
typedef struct sv_state sv_state;
typedef struct sv_queue sv_queue;

/* Execution options for sv_apply_circuit_ex / sv_param_shift_grad_ex. */
enum {
    SV_FLAG_UNFUSED = 1u << 0,    /* one kernel launch per gate (plain path) */
    SV_FLAG_SEQUENTIAL = 1u << 1  /* gradient / batch: one circuit at a time */
};

/*
 * Context: one device, one stream, the planner's tuning cache and buffer
 * pools.  device = HIP ordinal.  cfg may be NULL (defaults).  Returns
 * SV_ENODEV if the device is missing or not gfx950.
 */
typedef struct sv_config {
    int32_t tile_bits_c64;     /* gate tile pass width (bits), complex64: 6..14, 0 = default 12 */
    int32_t tile_bits_c128;    /* same for complex128: 6..12, 0 = default 12 */
    int32_t expect_bits_c64;   /* expectation pass tile width, complex64: 6..14, 0 = default 13 */
    int32_t expect_bits_c128;  /* same for complex128: 6..13, 0 = default 12 */
    int32_t perm_bits_c64;     /* permutation pass tile width, complex64: 6..12, 0 = default 12 */
    int32_t perm_bits_c128;    /* same for complex128: 6..11, 0 = default 11 */
    int32_t dense_fuse;        /* complex64 apply: runs of fixed gates on four qubits become
                                  one dense 16x16 block applied with MFMA; 0 = default (on),
                                  1 = on, -1 = off; 2..4 = measurement mode: every run of at
                                  least two fixed gates on at most k = dense_fuse qubits
                                  becomes a block (padded to four qubits), whatever its cost;
                                  other values are SV_EINVAL */
    int32_t graph_batch;       /* gradients, batch energies and queue ticks: record the batch's
                                  launches and replay them as one hipGraph launch (the
                                  instantiated graph is reused while the batch keeps its
                                  shape); 0 = default (on), 1 = on, -1 = off */
    int32_t tile_bits_layers_c64;  /* gate tile width of layered circuits (only fixed
                                      uncontrolled one-qubit gates and diagonals, no merged CP
                                      ladders: rotation layers with CZ / CP), complex64: 6..14,
                                      0 = default 12 */
    int32_t tile_bits_layers_c128; /* same for complex128: 6..12, 0 = default 12 */
} sv_config;

/* Fault injection for tests of the error paths: if the environment variable
 * SV_FAULT_ALLOC=N (N >= 1) is set when sv_init runs, the context's N-th
 * device allocation (states, scratch buffers, and separately each queue's
 * own allocations) fails as if HBM were exhausted, and the call that made
 * it returns SV_ENOMEM with nothing leaked. */
int sv_init(sv_ctx **out, int device, const sv_config *cfg);
/* Release the context.  Every state (sv_alloc, sv_wrap) and queue created on
 * it must have been released first (sv_free, sv_queue_destroy): while any is
 * alive the call changes nothing and returns SV_EBUSY, so no handle can
 * outlive the context it references. */
int sv_shutdown(sv_ctx *ctx);

/* Use the caller's HIP stream (e.g. PyTorch's current stream); NULL = the
 * context's own stream. */
int sv_set_stream(sv_ctx *ctx, void *hip_stream);
/* Block until all work on the context's stream has finished. */
int sv_synchronize(sv_ctx *ctx);

/*
 * State allocation: a contiguous 2^n amplitude vector in HBM initialised to
 * |0...0> (Sec. "Dense State Vector Representation", zero_state: allocated
 * once, no allocation during execution).
 */
int sv_alloc(sv_ctx *ctx, int n_qubits, int dtype, sv_state **out);
/* Adopt caller-owned device memory of 2^n amplitudes (e.g. a torch tensor);
 * the contents are left as they are. */
int sv_wrap(sv_ctx *ctx, void *dev_ptr, int n_qubits, int dtype,
            sv_state **out);
int sv_free(sv_state *st);
int sv_reset(sv_state *st);                     /* back to |0...0> */
int sv_state_info(const sv_state *st, int *n_qubits, int *dtype,
                  void **dev_ptr);
/* Host <-> device copies of all 2^n amplitudes in the state's dtype. */
int sv_set_amplitudes(sv_state *st, const void *host, size_t n_amps);
int sv_get_amplitudes(sv_state *st, void *host, size_t n_amps);

/*
 * Apply a gate list to the state: psi <- U_L ... U_1 psi (Sec. "Circuit
 * Data Structure", execute; gates by Sec. "Direct State Vector Gates").
 * The default path plans fused passes (LDS tiles, in-register runs,
 * diagonal gates folded in); SV_FLAG_UNFUSED applies one gate per launch.
 * params must hold circuit->n_params finite values.
 */
int sv_apply_circuit(sv_state *st, const sv_circuit *circuit,
                     const double *params, size_t n_params);
int sv_apply_circuit_ex(sv_state *st, const sv_circuit *circuit,
                        const double *params, size_t n_params, uint32_t flags);

/*
 * For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the
 * fused apply of sv_apply_circuit with no device allocation.  The plan's
 * device tables (ops, stages, ladder and layout tables) go to a block
 * preallocated per device when the library is loaded (SV_NOALLOC_BLOCK_BYTES,
 * held until the process ends) instead of a context buffer.  The state is
 * the caller's, as in sv_apply_circuit.  Returns SV_EINVAL, before any
 * device work, when the circuit's tables exceed the block (a plan holds
 * about 224 bytes per op at complex64, 352 at complex128, so circuits of
 * roughly 10^4 gates fit).  Every call on a device shares that
 * device's block: calls that overlap on one device (other streams, other
 * contexts, other threads) race and must be serialised by the caller; calls
 * in order on one stream are safe.  Results equal sv_apply_circuit's.
 */
#define SV_NOALLOC_BLOCK_BYTES ((size_t)4 << 20)
int sv_apply_circuit_noalloc(sv_state *st, const sv_circuit *circuit,
                             const double *params, size_t n_params);

/*
 * Quantum Fourier transform as the gate list of Alg. "Gate-Based QFT"
 * (H, controlled phases CP(pi/2^(j-i)), final swaps) run through the same
 * executor; equals sqrt(N) times the inverse DFT of the amplitudes
 * (Sec. "Quantum Fourier Transform Optimizations").
 */
int sv_qft(sv_state *st);
int sv_qft_ex(sv_state *st, uint32_t flags);

/* sum_k |psi_k|^2 in FP64, and scaling of psi to unit norm. */
int sv_norm2(sv_state *st, double *out);
int sv_normalize(sv_state *st);

/*
 * Energy E = sum_t c_t <psi|P_t|psi> / <psi|psi>, every product and sum in
 * FP64 (two-stage deterministic reduction; the division is the FP64
 * renormalisation).  term_values (nullable, n_terms doubles) receives each
 * <P_t> / <psi|psi>.  ham->n_qubits must equal the state's.
 */
int sv_expectation(sv_state *st, const sv_pauli_sum *ham, double *energy,
                   double *term_values);

/*
 * Parameter-shift gradient (Eq. "parameter_shift", s = pi/2; ParameterShift
 * of Sec. "Circuit Rebuilding Architecture"): every evaluation starts from a
 * fresh |0...0>.  Computes f(theta) into *energy and df/dtheta_i into
 * grad[0..n_params-1].  Rules per gate occurrence of parameter i (summed
 * over occurrences): two-term (s = pi/2) for RX/RY/RZ/U3/CP/RXX/RYY/RZZ;
 * four-term (shifts pi/2, 3pi/2) for CRX/CRY/CRZ.  All 1 + sum(shifts)
 * circuits run batched (one persistent launch) unless flags say otherwise;
 * the differences are taken in FP64 on the device.
 */
int sv_param_shift_grad(sv_ctx *ctx, int dtype, const sv_circuit *circuit,
                        const double *params, size_t n_params,
                        const sv_pauli_sum *ham, double *energy,
                        double *grad);
int sv_param_shift_grad_ex(sv_ctx *ctx, int dtype, const sv_circuit *circuit,
                           const double *params, size_t n_params,
                           const sv_pauli_sum *ham, uint32_t flags,
                           double *energy, double *grad);

/*
 * Variational eigensolver loop (Sec. "Variational Quantum Eigensolver"): minimise
 * E(theta) = <psi(theta)|H|psi(theta)> with Adam (Kingma and Ba: first and
 * second moment decay 0.9 and 0.999, denominator offset 1e-8, bias-corrected)
 * at learning rate lr, each step driven by one batched parameter-shift
 * gradient as in sv_param_shift_grad (same dtype and tolerances).  Iteration
 * t evaluates E_t and the gradient at the current parameters, records E_t in
 * energies[t - 1] (nullable; room for max_iters values) and stops when
 * t == max_iters or |E_t - E_{t-1}| < tol (t > 1); otherwise it takes the
 * Adam step.  params (n_params values) holds the initial parameters on entry
 * and, on return, those at which the last recorded energy was evaluated;
 * *iterations (nullable) receives the number of evaluations.  max_iters >= 1,
 * lr > 0 and tol >= 0 must be finite.  Errors as for sv_param_shift_grad;
 * on an error params are left unchanged (energies may hold the iterations
 * that completed).
 */
int sv_vqe_adam(sv_ctx *ctx, int dtype, const sv_circuit *circuit, double *params,
                size_t n_params, const sv_pauli_sum *ham, double lr, int max_iters,
                double tol, double *energies, int *iterations);

/*
 * Energies of many independent circuits of possibly different qubit counts
 * in one batched launch, each from |0...0>: energies[i] =
 * <psi_i|H_i|psi_i> for circuits[i], params[i], hams[i].
 */
int sv_batch_energies(sv_ctx *ctx, int dtype, size_t n_circuits,
                      const sv_circuit *circuits, const double *const *params,
                      const sv_pauli_sum *hams, double *energies);

/*
 * Serving queue: continuous batching of energy / gradient requests of mixed
 * qubit counts.  A scheduler thread admits requests while their state
 * slots fit in hbm_budget_bytes, runs every admitted circuit in shared
 * batched launches, and admits new work as slots free up.
 */
typedef struct sv_request {
    int32_t want_grad;        /* 0 = energy only, 1 = energy + gradient */
    int32_t dtype;            /* sv_dtype */
    sv_circuit circuit;
    const double *params;
    size_t n_params;
    sv_pauli_sum ham;
} sv_request;

typedef struct sv_queue_stats {
    uint64_t submitted, completed, failed, cancelled;
    uint64_t launches;         /* batched launches issued by the scheduler */
    uint64_t circuits_run;
    uint64_t peak_bytes;       /* largest resident footprint seen */
} sv_queue_stats;

int sv_queue_create(sv_ctx *ctx, size_t hbm_budget_bytes, sv_queue **out);
/* Copies the request; SV_EBUSY if one request alone exceeds the budget. */
int sv_queue_submit(sv_queue *q, const sv_request *req, uint64_t *ticket);
/* Wait up to timeout_ms (< 0 = forever).  grad may be NULL for energy-only
 * requests; grad_len must be >= the request's n_params otherwise.  The
 * ticket is released once a final status (OK or error) is returned.  If the
 * scheduler thread stops on an internal error, every request it had not
 * finished completes with that error (SV_EDEVICE unless the error carries
 * its own status) and later submissions return it too. */
int sv_queue_wait(sv_queue *q, uint64_t ticket, int timeout_ms,
                  double *energy, double *grad, size_t grad_len);
/* As sv_queue_wait; latency_s (nullable) receives the time from submission
 * to completion measured by the scheduler (steady clock). */
int sv_queue_wait_timed(sv_queue *q, uint64_t ticket, int timeout_ms,
                        double *energy, double *grad, size_t grad_len,
                        double *latency_s);
int sv_queue_cancel(sv_queue *q, uint64_t ticket);
/* Bound on the work of one scheduler tick, in amplitude updates (2^n x ops
 * per circuit; default 5e11, about 0.15 s of device work; 0 = no bound).  A
 * request whose remaining work exceeds an eighth of the bound is admitted
 * in pieces of at most the bound, after the small requests waiting at that
 * tick, so requests that arrive behind a large gradient wait for at most
 * one piece; each later piece of a gradient reruns its unshifted circuit
 * so that the piece's shifted circuits share that circuit's prefix.
 * SV_EINVAL for a negative or non-finite value. */
int sv_queue_set_tick_budget(sv_queue *q, double amplitude_updates);
int sv_queue_get_stats(sv_queue *q, sv_queue_stats *out);
int sv_queue_destroy(sv_queue *q);

/* Host-only validation used by every entry point (no device needed). */
int sv_check_circuit(const sv_circuit *circuit, const double *params,
                     size_t n_params);
int sv_check_pauli_sum(const sv_pauli_sum *ham, int n_qubits);

/*
 * Host-only inspection of the plan the fused apply would run for a circuit
 * (the lowering and fusion of Sec. "Circuit Data Structure"'s gate list; the
 * paper itself applies gates one at a time).  No device is needed: the
 * circuit is validated, lowered to FP64 gate records, planned into passes
 * and register stages with the widths of cfg (NULL = the library's
 * defaults) for dtype, and described.  sv_plan_dump writes a text listing
 * (one line per pass, stage and device op) into buf, truncated to buf_len
 * bytes including the terminating NUL; *needed (nullable) receives the full
 * length.  Errors as sv_apply_circuit's validation.
 */
typedef struct sv_plan_stats {
    int32_t tile_passes;       /* passes over the state through LDS tiles */
    int32_t perm_passes;       /* bit-relabelling passes (absorbed SWAPs) */
    int32_t sweep_passes;      /* one-gate sweeps (states of 1-2 qubits) */
    int32_t stages;            /* register stages over all tile passes */
    int32_t ops;               /* device ops over all tile passes */
    int32_t tile_passes_by_engine[5]; /* [0] three-bit stages, four-bit stages:
                                 [1] general, [2] Hadamard / ladder,
                                 [3] rotation / diagonal, [4] rotation layers */
    int32_t dense_blocks;      /* dense 16x16 blocks applied with MFMA */
    int32_t diagonal_tables;   /* gathered stage diagonals */
    double min_pass_scale, max_pass_scale; /* deferred real factors per pass */
} sv_plan_stats;
int sv_plan_info(const sv_circuit *circuit, const double *params, size_t n_params,
                 int dtype, const sv_config *cfg, sv_plan_stats *out);
int sv_plan_dump(const sv_circuit *circuit, const double *params, size_t n_params,
                 int dtype, const sv_config *cfg, char *buf, size_t buf_len,
                 size_t *needed);
/* Host-only: the batch that sv_param_shift_grad runs for these arguments
 * (Eq. "parameter_shift", one shifted pair per occurrence of a parameter;
 * the four-term rule for CRX / CRY / CRZ parameters): *circuits_out = 1 +
 * the shifted circuits; shifts_out (nullable, n_params entries) receives
 * how many shifted circuits each parameter's derivative combines (2 per
 * two-term occurrence, 4 per four-term one).  Errors as the gradient's
 * validation. */
int sv_psr_info(const sv_circuit *circuit, const double *params, size_t n_params,
                const sv_pauli_sum *ham, size_t *circuits_out, int32_t *shifts_out);

/* Optional per-kernel timing with HIP events recorded on the launching
 * stream around every launch (off by default).  name = kernel family. */
int sv_profile_enable(sv_ctx *ctx, int on);
int sv_profile_get(sv_ctx *ctx, const char *name, double *total_ms,
                   uint64_t *launches, double *bytes);
int sv_profile_reset(sv_ctx *ctx);

const char *sv_last_error(void);
/*
 * Autotuner: times, for dtype on synthetic work of n_qubits qubits clamped
 * to 8..30, the gate tile width (a gate-based QFT plus two RY/RZ +
 * CNOT-ladder layers), the layered-circuit tile width (sixteen layers of U3
 * on every qubit and CZ on a random matching), the permutation width and
 * the expectation tile width (a 2-local Pauli sum), one at a time, and
 * keeps the fastest in ctx; for complex64 it then times two layers of U3 +
 * CZ + RXX / RYY with and without dense four-qubit MFMA blocks (dense_fuse).
 * cache_path (nullable): a text file with one line per device, dtype and
 * size; a valid line is used without timing, a new result is appended.
 * chosen (nullable) receives every width of ctx afterwards.  Needs a free
 * state of the clamped size in HBM (16 GiB at 30 qubits complex128); takes
 * about a second at 28 qubits complex64, a few at 30 complex128.
 */
int sv_autotune(sv_ctx *ctx, int dtype, int n_qubits, const char *cache_path, sv_config *chosen);

/*
 * Counters of the context's batch graphs (nullable outputs): hipGraph
 * launches, and instantiations among them (the others reused the previous
 * executable graph, updated in place).  For the caller's diagnostics.
 */
int sv_graph_stats(sv_ctx *ctx, uint64_t *launches, uint64_t *instantiations);

const char *sv_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SV_ABI_H_INCLUDED */
