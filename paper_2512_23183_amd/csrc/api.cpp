// The C ABI (include/sv.h): argument validation first, then lowering,
// planning and device work.  Every entry point converts internal errors to
// an sv_status plus a thread-local message.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "sv_internal.h"

struct sv_ctx : sv::Ctx {};
struct sv_state : sv::State {};

namespace sv {
size_t queue_count(Ctx *ctx);

static std::vector<uint32_t (*)()> &bound_flag_readers() {
    static std::vector<uint32_t (*)()> r;
    return r;
}

bool register_bound_flag_reader(uint32_t (*reader)()) {
    bound_flag_readers().push_back(reader);
    return true;
}

uint32_t take_bound_flags() {
    uint32_t f = 0;
    for (auto r : bound_flag_readers()) f |= r();
    return f;
}
}  // namespace sv

using namespace sv;

namespace {

template <class F>
int guard(F &&f) {
    try {
        f();
#ifdef SV_DEBUG_BOUNDS
        // debug build: wait for the call's kernels and report any index
        // that fell outside its array
        if (hipDeviceSynchronize() != hipSuccess) (void)hipGetLastError();
        if (const uint32_t fl = take_bound_flags())
            fail(SV_EDEVICE, std::string("debug build: out-of-range index in a kernel (") +
                                 ((fl & 1) ? "HBM" : "") + ((fl & 3) == 3 ? ", " : "") + ((fl & 2) ? "LDS" : "") +
                                 ")");
#endif
        set_last_error("");
        return SV_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return SV_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(std::string("internal error: ") + e.what());
        return SV_EDEVICE;
    } catch (...) {
        set_last_error("internal error");
        return SV_EDEVICE;
    }
}

void need(bool cond, const char *msg) {
    if (!cond) fail(SV_EINVAL, msg);
}

void use_device(Ctx *ctx) { SV_HIP(hipSetDevice(ctx->device)); }

// Widths and switches of sv_config over the context's defaults (a field of
// 0 keeps the default; widths are clamped to their ranges).
void apply_config(Ctx *ctx, const sv_config *cfg) {
    if (!cfg) return;
    auto pick = [](int32_t v, int lo, int hi, int &dst) {
        if (v > 0) dst = std::max(lo, std::min(hi, (int)v));
    };
    pick(cfg->tile_bits_c64, 6, TILE_MAX[SV_C64], ctx->tile_bits[SV_C64]);
    pick(cfg->tile_bits_c128, 6, TILE_MAX[SV_C128], ctx->tile_bits[SV_C128]);
    pick(cfg->tile_bits_layers_c64, 6, TILE_MAX[SV_C64], ctx->tile_bits_layers[SV_C64]);
    pick(cfg->tile_bits_layers_c128, 6, TILE_MAX[SV_C128], ctx->tile_bits_layers[SV_C128]);
    pick(cfg->expect_bits_c64, 6, EXPECT_MAX[SV_C64], ctx->expect_bits[SV_C64]);
    pick(cfg->expect_bits_c128, 6, EXPECT_MAX[SV_C128], ctx->expect_bits[SV_C128]);
    pick(cfg->perm_bits_c64, 6, PERM_MAX[SV_C64], ctx->perm_bits[SV_C64]);
    pick(cfg->perm_bits_c128, 6, PERM_MAX[SV_C128], ctx->perm_bits[SV_C128]);
    need(cfg->dense_fuse >= -1 && cfg->dense_fuse <= 4,
         "dense_fuse must be -1 (off), 0 (default), 1 (on) or 2..4 (forced block width)");
    if (cfg->dense_fuse != 0) ctx->dense4 = cfg->dense_fuse > 0;
    ctx->dense_force = cfg->dense_fuse >= 2 ? cfg->dense_fuse : 0;
    if (cfg->graph_batch != 0) ctx->graphs = cfg->graph_batch > 0;
}

void check_dtype(int dtype) { need(dtype == SV_C64 || dtype == SV_C128, "dtype must be SV_C64 or SV_C128"); }

std::vector<Op> lower_circuit(const sv_circuit *c, const double *params) {
    std::vector<Op> ops;
    ops.reserve(c->n_gates);
    for (size_t i = 0; i < c->n_gates; ++i) {
        const sv_gate &g = c->gates[i];
        double ang[3];
        effective_angles(g, params, ang);
        const double *mat = (g.kind == SV_MAT1 || g.kind == SV_MAT2) ? c->mats + 32 * (size_t)g.mat_idx : nullptr;
        ops.push_back(lower_gate(c->n_qubits, g, ang, mat, (int)i));
    }
    return ops;
}

void apply_ops(State *st, const std::vector<Op> &ops, uint32_t flags) {
    Ctx *ctx = st->ctx;
    if (flags & SV_FLAG_UNFUSED) {
        run_unfused(ctx, st, ops);
    } else {
        PlanOptions po;
        po.tile_bits = ctx->tile_bits[st->dtype];
        po.tile_bits_layers = ctx->tile_bits_layers[st->dtype];
        po.perm_bits = ctx->perm_bits[st->dtype];
        po.dense4 = st->dtype == SV_C64 && ctx->dense4;
        po.dense_force = ctx->dense_force;
        run_plan(ctx, st, make_plan(st->n, ops, po));
    }
    if (ctx->profile) {
        SV_HIP(hipStreamSynchronize(ctx->stream));
        profile_collect(ctx);
    }
}

void check_finite(double v, const char *what) {
    if (!std::isfinite(v)) fail(SV_ENUMERIC, std::string(what) + " is not finite");
}

// Parameter-shift rule per gate kind: 2 = two-term (s = pi/2), 4 = four-term.
int shift_rule(int kind) {
    switch (kind) {
    case SV_RX: case SV_RY: case SV_RZ: case SV_U3: case SV_CP:
    case SV_RXX: case SV_RYY: case SV_RZZ:
        return 2;
    case SV_CRX: case SV_CRY: case SV_CRZ:
        return 4;
    default:
        return 0;
    }
}

}  // namespace

namespace sv {

// Build the 1 + sum(shifts) circuits of a parameter-shift gradient and the
// combination weights (Eq. "parameter_shift"; four-term rule for controlled
// rotations, see sv.h).
BatchSpec psr_spec(const sv_circuit *c, const double *params, size_t n_params, const sv_pauli_sum *ham,
                   int dtype, bool want_grad) {
    BatchSpec spec;
    spec.dtype = dtype;
    spec.op_sets.push_back(lower_circuit(c, params));
    spec.hams.push_back(lower_pauli_sum(*ham));
    BatchCircuit base;
    base.n = c->n_qubits;
    base.op_set = 0;
    base.ham = 0;
    spec.circuits.push_back(base);
    spec.comb_begin.push_back(0);
    if (!want_grad) return spec;
    const double s = M_PI / 2.0;
    const double d1 = (std::sqrt(2.0) + 1.0) / (4.0 * std::sqrt(2.0));
    const double d2 = (std::sqrt(2.0) - 1.0) / (4.0 * std::sqrt(2.0));
    // occurrences of each parameter (indices were validated < n_params)
    std::vector<std::vector<std::pair<int, int>>> occ(n_params);
    for (size_t g = 0; g < c->n_gates; ++g)
        for (int k = 0; k < 3; ++k) {
            const int p = c->gates[g].param_idx[k];
            if (p >= 0) {
                if ((size_t)p >= n_params) fail(SV_EINVAL, "param_idx out of range");
                occ[p].push_back({(int)g, k});
            }
        }
    for (size_t i = 0; i < n_params; ++i) {
        for (auto [g, k] : occ[i]) {
            const sv_gate &gt = c->gates[g];
            const int rule = shift_rule(gt.kind);
            if (rule == 0) fail(SV_EINVAL, "gate " + std::to_string(g) + " has no differentiable angle");
            std::vector<std::pair<double, double>> sw;  // (shift, weight)
            if (rule == 2) sw = {{+s, 0.5}, {-s, -0.5}};
            else sw = {{+s, d1}, {-s, -d1}, {+3 * s, -d2}, {-3 * s, d2}};
            for (auto [shift, w] : sw) {
                double ang[3];
                effective_angles(gt, params, ang);
                ang[k] += shift;
                const double *mat = nullptr;
                BatchCircuit bc = base;
                bc.ovr_index = g;
                bc.ovr_op = lower_gate(c->n_qubits, gt, ang, mat, g);
                spec.comb_circ.push_back((int)spec.circuits.size());
                spec.comb_w.push_back(w);
                spec.circuits.push_back(bc);
            }
        }
        spec.comb_begin.push_back((int)spec.comb_circ.size());
    }
    return spec;
}

}  // namespace sv

extern "C" {

const char *sv_last_error(void) { return last_error().c_str(); }

const char *sv_version(void) { return "sv-mi355x 0.1 (gfx950)"; }

int sv_check_circuit(const sv_circuit *circuit, const double *params, size_t n_params) {
    return guard([&] { check_circuit(circuit, params, n_params); });
}

int sv_check_pauli_sum(const sv_pauli_sum *ham, int n_qubits) {
    return guard([&] { check_pauli_sum(ham, n_qubits); });
}

namespace {
// The plan sv_apply_circuit would run for this circuit with these widths
// (host only: validation, lowering, planning and the device tables' layout).
PlanSummary plan_for(const sv_circuit *circuit, const double *params, size_t n_params, int dtype,
                     const sv_config *cfg, std::string *text) {
    check_circuit(circuit, params, n_params);
    check_dtype(dtype);
    Ctx opts;  // the library's default widths, then cfg's
    apply_config(&opts, cfg);
    PlanOptions po;
    po.tile_bits = opts.tile_bits[dtype];
    po.tile_bits_layers = opts.tile_bits_layers[dtype];
    po.perm_bits = opts.perm_bits[dtype];
    po.dense4 = dtype == SV_C64 && opts.dense4;
    po.dense_force = opts.dense_force;
    const Plan plan = make_plan(circuit->n_qubits, lower_circuit(circuit, params), po);
    return dtype == SV_C64 ? summarize_plan<float>(plan, text) : summarize_plan<double>(plan, text);
}
}  // namespace

int sv_plan_info(const sv_circuit *circuit, const double *params, size_t n_params, int dtype, const sv_config *cfg,
                 sv_plan_stats *out) {
    return guard([&] {
        need(out != nullptr, "out is NULL");
        const PlanSummary sm = plan_for(circuit, params, n_params, dtype, cfg, nullptr);
        std::memset(out, 0, sizeof *out);
        out->tile_passes = sm.tile_passes;
        out->perm_passes = sm.perm_passes;
        out->sweep_passes = sm.sweep_passes;
        out->stages = sm.stages;
        out->ops = sm.ops;
        for (int i = 0; i < 5; ++i) out->tile_passes_by_engine[i] = sm.h4_passes[i];
        out->dense_blocks = sm.dense_blocks;
        out->diagonal_tables = sm.tables;
        out->min_pass_scale = sm.tile_passes ? sm.min_scale : 1.0;
        out->max_pass_scale = sm.tile_passes ? sm.max_scale : 1.0;
    });
}

int sv_psr_info(const sv_circuit *circuit, const double *params, size_t n_params, const sv_pauli_sum *ham,
                size_t *circuits_out, int32_t *shifts_out) {
    return guard([&] {
        need(circuits_out != nullptr, "circuits_out is NULL");
        check_circuit(circuit, params, n_params);
        check_pauli_sum(ham, circuit->n_qubits);
        const BatchSpec spec = psr_spec(circuit, params, n_params, ham, SV_C128, true);
        *circuits_out = spec.circuits.size();
        if (shifts_out)
            for (size_t i = 0; i < n_params; ++i)
                shifts_out[i] = spec.comb_begin.size() > i + 1 ? spec.comb_begin[i + 1] - spec.comb_begin[i] : 0;
    });
}

int sv_plan_dump(const sv_circuit *circuit, const double *params, size_t n_params, int dtype, const sv_config *cfg,
                 char *buf, size_t buf_len, size_t *needed) {
    return guard([&] {
        std::string text;
        plan_for(circuit, params, n_params, dtype, cfg, &text);
        if (needed) *needed = text.size() + 1;
        if (buf && buf_len) {
            const size_t k = std::min(buf_len - 1, text.size());
            std::memcpy(buf, text.data(), k);
            buf[k] = 0;
        }
    });
}

int sv_init(sv_ctx **out, int device, const sv_config *cfg) {
    return guard([&] {
        need(out != nullptr, "out is NULL");
        *out = nullptr;
        {
            Ctx check;  // the configuration is validated before anything is created
            apply_config(&check, cfg);
        }
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
            (void)hipGetLastError();
            fail(SV_ENODEV, "no HIP device available");
        }
        if (device < 0 || device >= count) fail(SV_ENODEV, "device ordinal out of range");
        hipDeviceProp_t prop;
        SV_HIP(hipGetDeviceProperties(&prop, device));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            fail(SV_ENODEV, std::string("device is ") + prop.gcnArchName + "; this library targets gfx950");
        SV_HIP(hipSetDevice(device));
        noalloc_setup(device);
        sv_ctx *ctx = new sv_ctx();
        ctx->device = device;
        ctx->cu_count = prop.multiProcessorCount;
        if (hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            fail(SV_EDEVICE, "stream creation failed");
        }
        ctx->stream = ctx->own_stream;
        if (const char *fa = std::getenv("SV_FAULT_ALLOC")) ctx->fault_alloc = std::max(0, std::atoi(fa));
        apply_config(ctx, cfg);
#ifdef SV_DEBUG_BOUNDS
        try {
            debug_bounds_probe(ctx);
        } catch (...) {
            (void)hipStreamDestroy(ctx->own_stream);
            delete ctx;
            throw;
        }
#endif
        *out = ctx;
    });
}

int sv_shutdown(sv_ctx *ctx) {
    return guard([&] {
        need(ctx != nullptr, "ctx is NULL");
        // states and queues reference the context (its stream, its device):
        // they must be released first, so that no handle outlives it
        const int ns = ctx->live_states.load();
        const size_t nq = queue_count(ctx);
        if (ns > 0 || nq > 0)
            fail(SV_EBUSY, "context still has " + std::to_string(ns) + " live state(s) and " +
                               std::to_string(nq) + " queue(s); free them before sv_shutdown");
        use_device(ctx);
        (void)hipStreamSynchronize(ctx->stream);
        release_graph(ctx);
        release_pinned(ctx);
        for (auto &kv : ctx->scratch)
            if (kv.second.ptr) (void)hipFree(kv.second.ptr);
        for (auto &p : ctx->pending) {
            (void)hipEventDestroy(p.second.first);
            (void)hipEventDestroy(p.second.second);
        }
        for (hipEvent_t e : ctx->free_events) (void)hipEventDestroy(e);
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
        delete ctx;
    });
}

int sv_graph_stats(sv_ctx *ctx, uint64_t *launches, uint64_t *instantiations) {
    return guard([&] {
        need(ctx != nullptr, "ctx is NULL");
        if (launches) *launches = ctx->graph_launches;
        if (instantiations) *instantiations = ctx->graph_instantiations;
    });
}

int sv_set_stream(sv_ctx *ctx, void *hip_stream) {
    return guard([&] {
        need(ctx != nullptr, "ctx is NULL");
        ctx->stream = hip_stream ? (hipStream_t)hip_stream : ctx->own_stream;
    });
}

int sv_synchronize(sv_ctx *ctx) {
    return guard([&] {
        need(ctx != nullptr, "ctx is NULL");
        use_device(ctx);
        SV_HIP(hipStreamSynchronize(ctx->stream));
        if (ctx->profile) profile_collect(ctx);
    });
}

int sv_alloc(sv_ctx *ctx, int n_qubits, int dtype, sv_state **out) {
    return guard([&] {
        need(ctx != nullptr && out != nullptr, "ctx or out is NULL");
        *out = nullptr;
        need(n_qubits >= 1 && n_qubits <= SV_MAX_QUBITS, "n_qubits out of range");
        check_dtype(dtype);
        use_device(ctx);
        sv_state *st = new sv_state();
        st->ctx = ctx;
        st->n = n_qubits;
        st->dtype = dtype;
        if (dev_malloc(ctx, &st->ptr, st->bytes()) != hipSuccess) {
            (void)hipGetLastError();
            delete st;
            fail(SV_ENOMEM, "device allocation of the state failed");
        }
        try {
            set_zero_state(ctx, st->ptr, n_qubits, dtype);
        } catch (...) {
            (void)hipFree(st->ptr);
            delete st;
            throw;
        }
        ctx->live_states.fetch_add(1);
        *out = st;
    });
}

int sv_wrap(sv_ctx *ctx, void *dev_ptr, int n_qubits, int dtype, sv_state **out) {
    return guard([&] {
        need(ctx != nullptr && out != nullptr && dev_ptr != nullptr, "NULL argument");
        *out = nullptr;
        need(n_qubits >= 1 && n_qubits <= SV_MAX_QUBITS, "n_qubits out of range");
        check_dtype(dtype);
        need(((uintptr_t)dev_ptr & 15) == 0, "device pointer must be 16-byte aligned");
        sv_state *st = new sv_state();
        st->ctx = ctx;
        st->n = n_qubits;
        st->dtype = dtype;
        st->ptr = dev_ptr;
        st->owned = false;
        ctx->live_states.fetch_add(1);
        *out = st;
    });
}

int sv_free(sv_state *st) {
    return guard([&] {
        if (!st) return;
        use_device(st->ctx);
        if (st->owned && st->ptr) {
            (void)hipStreamSynchronize(st->ctx->stream);
            (void)hipFree(st->ptr);
        }
        st->ctx->live_states.fetch_sub(1);
        delete st;
    });
}

int sv_reset(sv_state *st) {
    return guard([&] {
        need(st != nullptr, "state is NULL");
        use_device(st->ctx);
        set_zero_state(st->ctx, st->ptr, st->n, st->dtype);
    });
}

int sv_state_info(const sv_state *st, int *n_qubits, int *dtype, void **dev_ptr) {
    return guard([&] {
        need(st != nullptr, "state is NULL");
        if (n_qubits) *n_qubits = st->n;
        if (dtype) *dtype = st->dtype;
        if (dev_ptr) *dev_ptr = st->ptr;
    });
}

int sv_set_amplitudes(sv_state *st, const void *host, size_t n_amps) {
    return guard([&] {
        need(st != nullptr && host != nullptr, "NULL argument");
        need(n_amps == (1ull << st->n), "n_amps must equal 2^n_qubits");
        use_device(st->ctx);
        SV_HIP(hipMemcpyAsync(st->ptr, host, st->bytes(), hipMemcpyHostToDevice, st->ctx->stream));
        SV_HIP(hipStreamSynchronize(st->ctx->stream));
    });
}

int sv_get_amplitudes(sv_state *st, void *host, size_t n_amps) {
    return guard([&] {
        need(st != nullptr && host != nullptr, "NULL argument");
        need(n_amps == (1ull << st->n), "n_amps must equal 2^n_qubits");
        use_device(st->ctx);
        SV_HIP(hipMemcpyAsync(host, st->ptr, st->bytes(), hipMemcpyDeviceToHost, st->ctx->stream));
        SV_HIP(hipStreamSynchronize(st->ctx->stream));
    });
}

int sv_apply_circuit_ex(sv_state *st, const sv_circuit *circuit, const double *params, size_t n_params,
                        uint32_t flags) {
    return guard([&] {
        need(st != nullptr, "state is NULL");
        check_circuit(circuit, params, n_params);
        need(circuit->n_qubits == st->n, "circuit and state qubit counts differ");
        use_device(st->ctx);
        apply_ops(st, lower_circuit(circuit, params), flags);
    });
}

int sv_apply_circuit(sv_state *st, const sv_circuit *circuit, const double *params, size_t n_params) {
    return sv_apply_circuit_ex(st, circuit, params, n_params, 0);
}

int sv_apply_circuit_noalloc(sv_state *st, const sv_circuit *circuit, const double *params, size_t n_params) {
    return guard([&] {
        need(st != nullptr, "state is NULL");
        check_circuit(circuit, params, n_params);
        need(circuit->n_qubits == st->n, "circuit and state qubit counts differ");
        Ctx *ctx = st->ctx;
        use_device(ctx);
        void *block = noalloc_block(ctx->device);
        PlanOptions po;
        po.tile_bits = ctx->tile_bits[st->dtype];
        po.tile_bits_layers = ctx->tile_bits_layers[st->dtype];
        po.perm_bits = ctx->perm_bits[st->dtype];
        po.dense4 = st->dtype == SV_C64 && ctx->dense4;
        po.dense_force = ctx->dense_force;
        run_plan_in(ctx, st, make_plan(st->n, lower_circuit(circuit, params), po), block, NOALLOC_BLOCK_BYTES);
    });
}

int sv_qft_ex(sv_state *st, uint32_t flags) {
    return guard([&] {
        need(st != nullptr, "state is NULL");
        use_device(st->ctx);
        std::vector<sv_gate> gates = qft_gates(st->n);
        std::vector<Op> ops;
        ops.reserve(gates.size());
        for (size_t i = 0; i < gates.size(); ++i) {
            double ang[3];
            effective_angles(gates[i], nullptr, ang);
            ops.push_back(lower_gate(st->n, gates[i], ang, nullptr, (int)i));
        }
        apply_ops(st, ops, flags);
    });
}

int sv_qft(sv_state *st) { return sv_qft_ex(st, 0); }

int sv_norm2(sv_state *st, double *out) {
    return guard([&] {
        need(st != nullptr && out != nullptr, "NULL argument");
        use_device(st->ctx);
        device_norm2(st->ctx, st->ptr, st->n, st->dtype, out);
        check_finite(*out, "norm");
    });
}

int sv_normalize(sv_state *st) {
    return guard([&] {
        need(st != nullptr, "state is NULL");
        use_device(st->ctx);
        double nn = 0.0;
        device_norm2(st->ctx, st->ptr, st->n, st->dtype, &nn);
        if (!(nn > 0.0) || !std::isfinite(nn)) fail(SV_ENUMERIC, "state norm is zero or not finite");
        device_scale(st->ctx, st->ptr, st->n, st->dtype, 1.0 / std::sqrt(nn));
    });
}

int sv_expectation(sv_state *st, const sv_pauli_sum *ham, double *energy, double *term_values) {
    return guard([&] {
        need(st != nullptr, "state is NULL");
        check_pauli_sum(ham, st->n);
        use_device(st->ctx);
        double e = 0.0, nn = 0.0;
        device_expectation(st->ctx, st->ptr, st->n, st->dtype, lower_pauli_sum(*ham), &e, term_values, &nn);
        if (!(nn > 0.0)) fail(SV_ENUMERIC, "state norm is zero");
        check_finite(e, "energy");
        if (energy) *energy = e;
    });
}

int sv_param_shift_grad_ex(sv_ctx *ctx, int dtype, const sv_circuit *circuit, const double *params,
                           size_t n_params, const sv_pauli_sum *ham, uint32_t flags, double *energy,
                           double *grad) {
    return guard([&] {
        need(ctx != nullptr, "ctx is NULL");
        check_dtype(dtype);
        check_circuit(circuit, params, n_params);
        check_pauli_sum(ham, circuit->n_qubits);
        need(n_params == 0 || grad != nullptr, "grad is NULL");
        use_device(ctx);
        BatchSpec spec = psr_spec(circuit, params, n_params, ham, dtype, true);
        std::vector<double> E, g;
        run_batch(ctx, spec, flags, E, g);
        check_finite(E[0], "energy");
        for (size_t i = 0; i < g.size(); ++i) check_finite(g[i], "gradient");
        if (energy) *energy = E[0];
        for (size_t i = 0; i < n_params; ++i) grad[i] = g[i];
    });
}

int sv_param_shift_grad(sv_ctx *ctx, int dtype, const sv_circuit *circuit, const double *params,
                        size_t n_params, const sv_pauli_sum *ham, double *energy, double *grad) {
    return sv_param_shift_grad_ex(ctx, dtype, circuit, params, n_params, ham, 0, energy, grad);
}

int sv_vqe_adam(sv_ctx *ctx, int dtype, const sv_circuit *circuit, double *params, size_t n_params,
                const sv_pauli_sum *ham, double lr, int max_iters, double tol, double *energies,
                int *iterations) {
    return guard([&] {
        need(ctx != nullptr, "ctx is NULL");
        check_dtype(dtype);
        check_circuit(circuit, params, n_params);
        check_pauli_sum(ham, circuit->n_qubits);
        need(max_iters >= 1, "max_iters must be at least 1");
        need(std::isfinite(lr) && lr > 0.0, "lr must be finite and positive");
        need(std::isfinite(tol) && tol >= 0.0, "tol must be finite and non-negative");
        use_device(ctx);
        if (iterations) *iterations = 0;
        // Adam moments (Kingma and Ba), bias-corrected
        const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
        std::vector<double> theta(params, params + n_params), m(n_params, 0.0), v(n_params, 0.0);
        double prev = 0.0, p1 = 1.0, p2 = 1.0;
        for (int t = 1; t <= max_iters; ++t) {
            BatchSpec spec = psr_spec(circuit, theta.data(), n_params, ham, dtype, true);
            std::vector<double> E, g;
            run_batch(ctx, spec, 0, E, g);
            check_finite(E[0], "energy");
            for (double x : g) check_finite(x, "gradient");
            if (energies) energies[t - 1] = E[0];
            if (iterations) *iterations = t;
            if (t == max_iters || (t > 1 && std::fabs(E[0] - prev) < tol)) break;
            prev = E[0];
            p1 *= b1;
            p2 *= b2;
            for (size_t i = 0; i < n_params; ++i) {
                m[i] = b1 * m[i] + (1.0 - b1) * g[i];
                v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
                const double mh = m[i] / (1.0 - p1), vh = v[i] / (1.0 - p2);
                theta[i] -= lr * mh / (std::sqrt(vh) + eps);
            }
        }
        std::copy(theta.begin(), theta.end(), params);
    });
}

int sv_batch_energies(sv_ctx *ctx, int dtype, size_t n_circuits, const sv_circuit *circuits,
                      const double *const *params, const sv_pauli_sum *hams, double *energies) {
    return guard([&] {
        need(ctx != nullptr, "ctx is NULL");
        check_dtype(dtype);
        need(n_circuits == 0 || (circuits && params && hams && energies), "NULL argument");
        for (size_t i = 0; i < n_circuits; ++i) {
            check_circuit(&circuits[i], params[i], circuits[i].n_params);
            check_pauli_sum(&hams[i], circuits[i].n_qubits);
        }
        use_device(ctx);
        BatchSpec spec;
        spec.dtype = dtype;
        for (size_t i = 0; i < n_circuits; ++i) {
            spec.op_sets.push_back(lower_circuit(&circuits[i], params[i]));
            spec.hams.push_back(lower_pauli_sum(hams[i]));
            BatchCircuit bc;
            bc.n = circuits[i].n_qubits;
            bc.op_set = (int)i;
            bc.ham = (int)i;
            spec.circuits.push_back(bc);
        }
        std::vector<double> E, g;
        run_batch(ctx, spec, 0, E, g);
        for (size_t i = 0; i < n_circuits; ++i) {
            check_finite(E[i], "energy");
            energies[i] = E[i];
        }
    });
}

int sv_profile_enable(sv_ctx *ctx, int on) {
    return guard([&] {
        need(ctx != nullptr, "ctx is NULL");
        ctx->profile = on != 0;
    });
}

int sv_profile_get(sv_ctx *ctx, const char *name, double *total_ms, uint64_t *launches, double *bytes) {
    return guard([&] {
        need(ctx != nullptr && name != nullptr, "NULL argument");
        use_device(ctx);
        SV_HIP(hipStreamSynchronize(ctx->stream));
        profile_collect(ctx);
        auto it = ctx->prof.find(name);
        ProfileEntry e;
        if (it != ctx->prof.end()) e = it->second;
        if (total_ms) *total_ms = e.ms;
        if (launches) *launches = e.launches;
        if (bytes) *bytes = e.bytes;
    });
}

int sv_profile_reset(sv_ctx *ctx) {
    return guard([&] {
        need(ctx != nullptr, "ctx is NULL");
        use_device(ctx);
        SV_HIP(hipStreamSynchronize(ctx->stream));
        profile_collect(ctx);
        ctx->prof.clear();
    });
}

int sv_autotune(sv_ctx *ctx, int dtype, int n_qubits, const char *cache_path, sv_config *chosen) {
    return guard([&] {
        need(ctx != nullptr, "ctx is NULL");
        check_dtype(dtype);
        use_device(ctx);
        autotune(ctx, ctx, dtype, n_qubits, cache_path);
        if (chosen) {
            std::memset(chosen, 0, sizeof *chosen);
            chosen->tile_bits_c64 = ctx->tile_bits[SV_C64];
            chosen->tile_bits_c128 = ctx->tile_bits[SV_C128];
            chosen->tile_bits_layers_c64 = ctx->tile_bits_layers[SV_C64];
            chosen->tile_bits_layers_c128 = ctx->tile_bits_layers[SV_C128];
            chosen->expect_bits_c64 = ctx->expect_bits[SV_C64];
            chosen->expect_bits_c128 = ctx->expect_bits[SV_C128];
            chosen->perm_bits_c64 = ctx->perm_bits[SV_C64];
            chosen->perm_bits_c128 = ctx->perm_bits[SV_C128];
            chosen->dense_fuse = ctx->dense4 ? (ctx->dense_force ? ctx->dense_force : 1) : -1;
        }
    });
}

}  // extern "C"
