// Serving queue: continuous batching of energy / gradient requests of mixed
// qubit counts on one device.
//
// A scheduler thread owns all device work of the queue.  Each request
// expands into circuits (1 for an energy, 1 + shifts for a gradient).  On
// every tick the scheduler admits circuits in arrival order while the
// resident footprint (state slots of the circuits in flight) stays within
// the HBM budget -- a large gradient is admitted piecewise, so it never
// blocks the queue -- runs all admitted circuits in one batched launch
// (small states in LDS, larger ones through the pass executor), and
// completes every request whose circuits have all finished.  Requests that
// arrive meanwhile join the next tick.  Each circuit's energy is reduced by
// itself in a fixed order, so a result does not depend on what else shared
// its launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>

#include "sv_internal.h"

struct sv_queue;

namespace sv {

namespace {

using clk = std::chrono::steady_clock;

struct Req {
    uint64_t ticket = 0;
    bool want_grad = false;
    int dtype = SV_C64;
    // owned copies of the request's arrays
    std::vector<sv_gate> gates;
    std::vector<double> mats, params, coeffs;
    std::vector<char> paulis;
    sv_circuit circ{};
    sv_pauli_sum ham{};
    BatchSpec spec;             // circuits of this request (op set 0, ham 0)
    size_t next = 0;            // next circuit to admit
    size_t done = 0;            // circuits finished
    int e_off = -1;             // slot range in the device energy pool
    int status = SV_OK;
    bool finished = false, cancelled = false;
    double energy = 0.0;
    std::vector<double> grad;
    std::string err;
    clk::time_point t_submit, t_done;
};

}  // namespace

struct QueueImpl {
    Ctx *parent = nullptr;   // the context the queue was created on
    Ctx *ctx = nullptr;      // the queue's own stream and scratch buffers
    size_t budget = 0;
    // work per tick, in amplitude updates (2^n x ops per circuit; 0 = no
    // bound): a large gradient is admitted in pieces of about this much, so
    // requests that arrive meanwhile wait for at most one piece
    double tick_budget = 5e11;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Req>> pending;
    std::map<uint64_t, std::shared_ptr<Req>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    // set when the scheduler thread ended on an exception: every request it
    // left was completed with dead_code, and later submissions fail
    bool dead = false;
    int dead_code = SV_OK;
    std::string dead_msg;
    sv_queue_stats stats{};
    // device energy pool: first-fit ranges
    double *d_pool = nullptr;
    int pool_cap = 0;
    std::map<int, int> free_ranges;  // offset -> length

    int pool_alloc(int len) {
        for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
            if (it->second >= len) {
                const int off = it->first, rem = it->second - len;
                free_ranges.erase(it);
                if (rem > 0) free_ranges[off + len] = rem;
                return off;
            }
        }
        return -1;
    }
    void pool_free(int off, int len) {
        auto it = free_ranges.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_ranges.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_ranges.erase(nx);
        }
        if (it != free_ranges.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_ranges.erase(it);
            }
        }
    }

    static size_t circuit_bytes(int n, int dtype) {
        // states held in LDS need no HBM slot; count their metadata only
        const size_t amp = dtype == SV_C64 ? 8 : 16;
        return n <= small_batch_max_qubits(dtype) ? 4096 : (amp << n);
    }

    // work of one circuit of r in amplitude updates (state size x ops)
    static double circuit_cost(const Req &r) {
        const double ops = r.spec.op_sets.empty() ? 1.0 : (double)std::max<size_t>(1, r.spec.op_sets[0].size());
        return std::ldexp(ops, r.circ.n_qubits);
    }

    void run();
    void fail_all(int code, const std::string &msg);
    void tick(std::vector<std::pair<std::shared_ptr<Req>, std::vector<int>>> &work);
};

void QueueImpl::tick(std::vector<std::pair<std::shared_ptr<Req>, std::vector<int>>> &work) {
    // one batched launch over the admitted circuits of all requests
    BatchSpec batch;
    batch.dtype = -1;
    std::vector<BatchSpec> by_dtype(2);
    for (auto &dt : by_dtype) dt.dtype = -1;
    for (int dt = 0; dt < 2; ++dt) {
        BatchSpec &b = by_dtype[dt];
        b.dtype = dt;
        for (auto &w : work) {
            Req &r = *w.first;
            if (r.dtype != dt) continue;
            const int set = (int)b.op_sets.size();
            b.op_sets.push_back(r.spec.op_sets[0]);
            b.hams.push_back(r.spec.hams[0]);
            // a later piece of a gradient runs the unshifted circuit again
            // (its energy, bitwise the same, rewrites its own slot) so that
            // the piece's shifted circuits share its prefix
            if (w.second.size() > 1 && r.spec.circuits[0].ovr_index < 0 &&
                std::find(w.second.begin(), w.second.end(), 0) == w.second.end()) {
                BatchCircuit bc = r.spec.circuits[0];
                bc.op_set = set;
                bc.ham = set;
                bc.out_slot = r.e_off;
                b.circuits.push_back(bc);
            }
            for (int ci : w.second) {
                BatchCircuit bc = r.spec.circuits[ci];
                bc.op_set = set;
                bc.ham = set;
                bc.out_slot = r.e_off + ci;
                b.circuits.push_back(bc);
            }
        }
        if (!b.circuits.empty()) run_batch_dev(ctx, b, 0, d_pool);
    }
    stats.launches += 1;
}

void QueueImpl::run() {
    (void)hipSetDevice(ctx->device);
    for (;;) {
        std::vector<std::pair<std::shared_ptr<Req>, std::vector<int>>> work;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !pending.empty(); });
            if (stop) return;
            // admission within the HBM budget and the tick's work bound:
            // first every request whose remaining work is small (an eighth
            // of the bound), in arrival order, then pieces of the large ones
            // in arrival order; a tick always takes at least one circuit
            size_t used = 0;
            size_t n_circ = 0;
            double cost = 0.0;
            const size_t max_circ = 1 << 14;
            const double small = tick_budget > 0.0 ? tick_budget / 8.0 : 0.0;
            bool full = false;
            for (int phase = 0; phase < 2 && !full; ++phase) {
                for (auto &rp : pending) {
                    Req &r = *rp;
                    if (r.cancelled || r.finished || r.next >= r.spec.circuits.size()) continue;
                    const double each = circuit_cost(r);
                    const double rest = each * (double)(r.spec.circuits.size() - r.next);
                    const bool is_small = tick_budget > 0.0 && rest <= small;
                    if ((phase == 0) != is_small) continue;
                    if (r.e_off < 0) {
                        r.e_off = pool_alloc((int)r.spec.circuits.size());
                        if (r.e_off < 0) {  // pool full: wait for completions
                            full = true;
                            break;
                        }
                    }
                    std::vector<int> take;
                    while (r.next < r.spec.circuits.size() && n_circ < max_circ) {
                        const size_t b = circuit_bytes(r.spec.circuits[r.next].n, r.dtype);
                        const bool first = n_circ == 0;
                        if (!first && used + b > budget) break;
                        if (!first && tick_budget > 0.0 && cost + each > tick_budget) break;
                        used += b;
                        cost += each;
                        take.push_back((int)r.next++);
                        ++n_circ;
                    }
                    if (!take.empty()) work.push_back({rp, std::move(take)});
                    if (used >= budget || n_circ >= max_circ || (tick_budget > 0.0 && cost >= tick_budget)) {
                        full = true;
                        break;
                    }
                }
            }
            if (used > stats.peak_bytes) stats.peak_bytes = used;
        }
        int err = SV_OK;
        std::string msg;
        try {
            tick(work);
            SV_HIP(hipStreamSynchronize(ctx->stream));
        } catch (const Error &e) {
            err = e.code;
            msg = e.msg;
        } catch (const std::bad_alloc &) {
            err = SV_ENOMEM;
            msg = "host allocation failed";
        } catch (const std::exception &e) {
            err = SV_EDEVICE;
            msg = std::string("internal error: ") + e.what();
        }
        // complete requests whose circuits are all done
        std::vector<std::shared_ptr<Req>> complete;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto &w : work) {
                Req &r = *w.first;
                r.done += w.second.size();
                stats.circuits_run += w.second.size();
                if (err != SV_OK) {
                    r.status = err;
                    r.err = msg;
                }
                if (r.done == r.spec.circuits.size() || err != SV_OK) complete.push_back(w.first);
            }
        }
        for (auto &rp : complete) {
            Req &r = *rp;
            if (r.status == SV_OK) {
                try {
                    const int np = r.want_grad ? (int)r.spec.comb_begin.size() - 1 : 0;
                    double *d_grad = (double *)scratch(ctx, "queue_grad", (size_t)std::max(np, 1) * 8);
                    if (np > 0) {
                        std::vector<int> circ = r.spec.comb_circ;
                        for (int &c : circ) c += r.e_off;
                        combine_dev(ctx, d_pool, r.spec.comb_begin, circ, r.spec.comb_w, d_grad);
                    }
                    r.grad.assign(np, 0.0);
                    SV_HIP(hipMemcpyAsync(&r.energy, d_pool + r.e_off, 8, hipMemcpyDeviceToHost, ctx->stream));
                    if (np > 0)
                        SV_HIP(hipMemcpyAsync(r.grad.data(), d_grad, (size_t)np * 8, hipMemcpyDeviceToHost,
                                              ctx->stream));
                    SV_HIP(hipStreamSynchronize(ctx->stream));
                    if (!std::isfinite(r.energy)) { r.status = SV_ENUMERIC; r.err = "energy not finite"; }
                    for (double g : r.grad)
                        if (!std::isfinite(g)) { r.status = SV_ENUMERIC; r.err = "gradient not finite"; }
                } catch (const Error &e) {
                    r.status = e.code;
                    r.err = e.msg;
                } catch (const std::exception &e) {
                    r.status = SV_EDEVICE;
                    r.err = std::string("internal error: ") + e.what();
                }
            }
            std::lock_guard<std::mutex> lk(mu);
            r.finished = true;
            r.t_done = clk::now();
            pool_free(r.e_off, (int)r.spec.circuits.size());
            if (r.status == SV_OK) stats.completed++;
            else stats.failed++;
            for (auto it = pending.begin(); it != pending.end(); ++it)
                if (it->get() == &r) { pending.erase(it); break; }
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            // drop cancelled requests that were never started
            for (auto it = pending.begin(); it != pending.end();) {
                Req &r = **it;
                if (r.cancelled && r.done == r.next) {
                    r.finished = true;
                    r.status = SV_ECANCELED;
                    r.t_done = clk::now();
                    if (r.e_off >= 0) pool_free(r.e_off, (int)r.spec.circuits.size());
                    stats.cancelled++;
                    it = pending.erase(it);
                } else {
                    ++it;
                }
            }
        }
        cv_done.notify_all();
    }
}

void QueueImpl::fail_all(int code, const std::string &msg) {
    {
        std::lock_guard<std::mutex> lk(mu);
        dead = true;
        dead_code = code;
        dead_msg = msg;
        for (auto &kv : all) {
            Req &r = *kv.second;
            if (r.finished) continue;
            r.finished = true;
            r.status = code;
            r.err = "queue scheduler stopped: " + msg;
            r.t_done = clk::now();
            stats.failed++;
        }
        pending.clear();
    }
    cv_done.notify_all();
}

static std::mutex g_queues_mu;
static std::multimap<Ctx *, QueueImpl *> g_queues;

void queue_destroy_impl(QueueImpl *q) {
    {
        std::lock_guard<std::mutex> lk(q->mu);
        q->stop = true;
    }
    q->cv_work.notify_all();
    if (q->worker.joinable()) q->worker.join();
    {
        std::lock_guard<std::mutex> lk(q->mu);
        for (auto &kv : q->all)
            if (!kv.second->finished) {
                kv.second->finished = true;
                kv.second->status = SV_ECANCELED;
            }
    }
    q->cv_done.notify_all();
    (void)hipSetDevice(q->ctx->device);
    (void)hipStreamSynchronize(q->ctx->stream);
    release_graph(q->ctx);
    release_pinned(q->ctx);
    if (q->d_pool) (void)hipFree(q->d_pool);
    for (auto &kv : q->ctx->scratch)
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    if (q->ctx->own_stream) (void)hipStreamDestroy(q->ctx->own_stream);
    delete q->ctx;
    delete q;
}

size_t queue_count(Ctx *ctx) {
    std::lock_guard<std::mutex> lk(g_queues_mu);
    return g_queues.count(ctx);
}

}  // namespace sv

static inline sv::QueueImpl *Q(sv_queue *q) { return reinterpret_cast<sv::QueueImpl *>(q); }

using namespace sv;

namespace {
template <class F>
int qguard(F &&f) {
    try {
        f();
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
    }
}
}  // namespace

extern "C" {

int sv_queue_create(sv_ctx *ctx_, size_t hbm_budget_bytes, sv_queue **out) {
    return qguard([&] {
        if (!ctx_ || !out) fail(SV_EINVAL, "NULL argument");
        if (hbm_budget_bytes < (1u << 20)) fail(SV_EINVAL, "budget must be at least 1 MiB");
        Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
        SV_HIP(hipSetDevice(ctx->device));
        QueueImpl *q = new QueueImpl();
        q->parent = ctx;
        q->ctx = new Ctx();
        q->ctx->device = ctx->device;
        q->ctx->cu_count = ctx->cu_count;
        for (int d = 0; d < 2; ++d) {
            q->ctx->tile_bits[d] = ctx->tile_bits[d];
            q->ctx->tile_bits_layers[d] = ctx->tile_bits_layers[d];
            q->ctx->expect_bits[d] = ctx->expect_bits[d];
            q->ctx->perm_bits[d] = ctx->perm_bits[d];
        }
        q->ctx->dense4 = ctx->dense4;
        q->ctx->dense_force = ctx->dense_force;
        q->ctx->graphs = ctx->graphs;
        q->ctx->fault_alloc = ctx->fault_alloc;
        if (hipStreamCreateWithFlags(&q->ctx->own_stream, hipStreamNonBlocking) != hipSuccess) {
            delete q->ctx;
            delete q;
            fail(SV_EDEVICE, "stream creation failed");
        }
        q->ctx->stream = q->ctx->own_stream;
        q->budget = hbm_budget_bytes;
        q->pool_cap = 1 << 22;
        if (dev_malloc(q->ctx, (void **)&q->d_pool, (size_t)q->pool_cap * 8) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipStreamDestroy(q->ctx->own_stream);
            delete q->ctx;
            delete q;
            fail(SV_ENOMEM, "energy pool allocation failed");
        }
        q->free_ranges[0] = q->pool_cap;
        q->worker = std::thread([q] {
            // whatever ends the scheduler completes every waiting request
            // with an error instead of leaving its waiter blocked
            try {
                q->run();
            } catch (const Error &e) {
                q->fail_all(e.code, e.msg);
            } catch (const std::exception &e) {
                q->fail_all(SV_EDEVICE, std::string("internal error: ") + e.what());
            } catch (...) {
                q->fail_all(SV_EDEVICE, "internal error: unknown exception");
            }
        });
        {
            std::lock_guard<std::mutex> lk(g_queues_mu);
            g_queues.emplace(ctx, q);
        }
        *out = reinterpret_cast<sv_queue *>(q);
    });
}

int sv_queue_submit(sv_queue *q_, const sv_request *req, uint64_t *ticket) {
    return qguard([&] {
        QueueImpl *q = Q(q_);
        if (!q || !req || !ticket) fail(SV_EINVAL, "NULL argument");
        if (req->dtype != SV_C64 && req->dtype != SV_C128) fail(SV_EINVAL, "bad dtype");
        check_circuit(&req->circuit, req->params, req->n_params);
        check_pauli_sum(&req->ham, req->circuit.n_qubits);
        auto r = std::make_shared<Req>();
        r->want_grad = req->want_grad != 0;
        r->dtype = req->dtype;
        r->gates.assign(req->circuit.gates, req->circuit.gates + req->circuit.n_gates);
        r->mats.assign(req->circuit.mats, req->circuit.mats + 32 * req->circuit.n_mats);
        r->params.assign(req->params, req->params + req->n_params);
        r->coeffs.assign(req->ham.coeffs, req->ham.coeffs + req->ham.n_terms);
        r->paulis.assign(req->ham.paulis, req->ham.paulis + req->ham.n_terms * (size_t)req->ham.n_qubits);
        r->circ = req->circuit;
        r->circ.gates = r->gates.data();
        r->circ.mats = r->mats.data();
        r->ham = req->ham;
        r->ham.coeffs = r->coeffs.data();
        r->ham.paulis = r->paulis.data();
        r->spec = psr_spec(&r->circ, r->params.data(), r->params.size(), &r->ham, r->dtype, r->want_grad);
        // one circuit alone must fit the budget
        const size_t one = QueueImpl::circuit_bytes(req->circuit.n_qubits, req->dtype);
        if (one > q->budget) fail(SV_EBUSY, "a single state of this request exceeds the queue budget");
        if ((int)r->spec.circuits.size() > q->pool_cap) fail(SV_EBUSY, "request has too many circuits");
        std::lock_guard<std::mutex> lk(q->mu);
        if (q->dead) fail(q->dead_code, "queue scheduler stopped: " + q->dead_msg);
        r->ticket = q->next_ticket++;
        r->t_submit = std::chrono::steady_clock::now();
        q->all[r->ticket] = r;
        q->pending.push_back(r);
        q->stats.submitted++;
        *ticket = r->ticket;
        q->cv_work.notify_one();
    });
}

int sv_queue_wait_timed(sv_queue *q_, uint64_t ticket, int timeout_ms, double *energy, double *grad,
                        size_t grad_len, double *latency_s) {
    return qguard([&] {
        QueueImpl *q = Q(q_);
        if (!q) fail(SV_EINVAL, "queue is NULL");
        std::unique_lock<std::mutex> lk(q->mu);
        auto it = q->all.find(ticket);
        if (it == q->all.end()) fail(SV_EINVAL, "unknown ticket");
        std::shared_ptr<Req> r = it->second;
        auto ready = [&] { return r->finished; };
        if (timeout_ms < 0) q->cv_done.wait(lk, ready);
        else if (!q->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
            fail(SV_ETIMEDOUT, "request still pending");
        q->all.erase(ticket);
        if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
        if (r->status != SV_OK) fail(r->status, r->err.empty() ? "request failed" : r->err);
        if (energy) *energy = r->energy;
        if (r->want_grad) {
            if (!grad || grad_len < r->grad.size()) fail(SV_EINVAL, "grad buffer too small");
            std::memcpy(grad, r->grad.data(), r->grad.size() * 8);
        }
    });
}

int sv_queue_wait(sv_queue *q, uint64_t ticket, int timeout_ms, double *energy, double *grad, size_t grad_len) {
    return sv_queue_wait_timed(q, ticket, timeout_ms, energy, grad, grad_len, nullptr);
}

int sv_queue_cancel(sv_queue *q_, uint64_t ticket) {
    return qguard([&] {
        QueueImpl *q = Q(q_);
        if (!q) fail(SV_EINVAL, "queue is NULL");
        std::lock_guard<std::mutex> lk(q->mu);
        auto it = q->all.find(ticket);
        if (it == q->all.end()) fail(SV_EINVAL, "unknown ticket");
        it->second->cancelled = true;
        q->cv_work.notify_one();
    });
}

int sv_queue_set_tick_budget(sv_queue *q_, double amplitude_updates) {
    return qguard([&] {
        QueueImpl *q = Q(q_);
        if (!q) fail(SV_EINVAL, "queue is NULL");
        if (!(amplitude_updates >= 0.0) || !std::isfinite(amplitude_updates))
            fail(SV_EINVAL, "tick budget must be finite and >= 0");
        std::lock_guard<std::mutex> lk(q->mu);
        q->tick_budget = amplitude_updates;
    });
}

int sv_queue_get_stats(sv_queue *q_, sv_queue_stats *out) {
    return qguard([&] {
        QueueImpl *q = Q(q_);
        if (!q || !out) fail(SV_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> lk(q->mu);
        *out = q->stats;
    });
}

int sv_queue_destroy(sv_queue *q_) {
    return qguard([&] {
        QueueImpl *q = Q(q_);
        if (!q) return;
        {
            std::lock_guard<std::mutex> lk(g_queues_mu);
            auto r = g_queues.equal_range(q->parent);
            for (auto it = r.first; it != r.second; ++it)
                if (it->second == q) {
                    g_queues.erase(it);
                    break;
                }
        }
        queue_destroy_impl(q);
    });
}

}  // extern "C"
