// Continuous-batching request server of the form-factor engine.
//
// Pipeline per request:
//   submit    copy the caller's inputs, assign a ticket, queue for prep
//   prep      (host worker pool) basis, pair precompute, screening and
//             packing; the exact device footprint is known afterwards
//   admit     (scheduler) strictly in ticket order: the head request starts
//             when its footprint fits the HBM budget next to everything in
//             flight and a run slot is free; requests arriving meanwhile
//             queue behind it, so no request starves
//   run       (batch runners, one HIP stream each) every admitted request
//             waiting for a runner joins its next batch: one graph-captured
//             launch sequence per batch (1D tables of each request, one
//             persistent grid kernel per kernel variant popping the
//             (request, tile) items of all its requests from a device queue,
//             split reductions, copies of the results into pinned staging
//             buffers of the server); two runners alternate, so one batch
//             is assembled while the other runs
//   copy      (copy threads) staging buffer -> the caller's host buffers;
//             the run slot and the device memory are released before this,
//             so the next request's kernels do not wait for host copies
//   complete  record latency (results in the caller's memory), wake waiters
// A failing request records its own status and never affects others.
// Contexts are pooled: a finished request hands its context back and the next
// prep reuses it (a context keeps every device buffer that is large enough,
// and its molecule: a request on the same molecule is given that context and
// skips the molecule load, a device-resident molecule cache),
// so in steady state a request allocates and frees no device memory and no
// thread ever waits for the whole device (freeing memory and destroying a
// context would).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/scarff.h"
#include "engine.h"

namespace {

using Clock = std::chrono::steady_clock;

enum class St { Queued, Ready, Running, Done, Cancelled };

// The molecule of a request (owned copies of its inputs).  Equal keys load
// equal device tables, so an idle context that holds one serves the next
// request on the same molecule without loading it again.
struct MolKey {
    std::vector<double> xyz, exps, coefs;
    std::vector<int> sh_atom, sh_l, sh_nprim;
    int normalise = 1;
    bool operator==(const MolKey& o) const {
        return normalise == o.normalise && sh_l == o.sh_l && sh_nprim == o.sh_nprim && sh_atom == o.sh_atom &&
               xyz == o.xyz && exps == o.exps && coefs == o.coefs;
    }
};
using MolPtr = std::shared_ptr<const MolKey>;

bool same_mol(const MolPtr& a, const MolPtr& b) { return a && b && (a == b || *a == *b); }

// an idle context and the molecule loaded on it (NULL: unknown)
struct Idle {
    scff_ctx* c = nullptr;
    MolPtr mol;
};

struct Req {
    unsigned long long ticket = 0;
    // owned copies of the inputs
    MolPtr mol;
    std::vector<double> T;
    int n_atoms = 0, n_shells = 0, n_states = 0, precision = 0;
    scff_grid grid{};
    double eps = 0.0, spin = 1.0;
    float* f = nullptr;
    float* f2 = nullptr;
    // execution state
    scff_ctx* ctx = nullptr;
    MolPtr ctx_mol;   // the molecule loaded on ctx
    size_t bytes = 0;
    St state = St::Queued;
    int status = SCFF_OK;
    bool waited = false;
    int queue_refs = 0;   // prep_q / admit_q entries still naming this ticket
    Clock::time_point t_submit, t_done;
    // stage times: prep start/end, run start/end (device results staged)
    Clock::time_point t_prep0, t_prep1, t_run0, t_run1;
};

}  // namespace

struct scff_server {
    int device = 0;
    bool fake = false;   // scheduler test mode: no device work
    size_t budget = 0;
    int max_inflight = 1;
    std::mutex mu;
    std::condition_variable cv_prep, cv_sched, cv_run, cv_done;
    std::deque<unsigned long long> prep_q;     // tickets waiting for prep
    std::deque<unsigned long long> admit_q;    // tickets in submit order, not yet admitted
    std::deque<unsigned long long> run_q;      // admitted, waiting for a run slot thread
    std::map<unsigned long long, std::unique_ptr<Req>> reqs;
    unsigned long long next_ticket = 1;
    size_t admitted = 0, peak_admitted = 0;
    int inflight = 0, peak_inflight = 0;
    long long n_submitted = 0, n_completed = 0, n_failed = 0, n_cancelled = 0;
    bool stop = false;
    std::vector<std::thread> threads;
    std::condition_variable cv_copy;
    std::deque<std::pair<unsigned long long, void*>> copy_q;   // (ticket, staging buffer) to copy out
    int copying = 0;                   // requests between the end of their run and completion
    std::multimap<size_t, void*> stage_free;   // pinned staging buffers by size
    std::map<void*, size_t> stage_size;        // size of every staging buffer
    std::vector<void*> stage_all;              // every staging buffer (freed at shutdown)
    std::vector<Idle> ctx_pool;        // idle contexts, device buffers and molecule kept
    long long n_mol_hits = 0;          // requests served by a context that held their molecule
    // stage times summed over completed requests (ns): waiting for a prep
    // thread, prep, waiting for admission and a run slot, run, host copy
    long long ns_stage[5] = {};
    std::vector<scff_ctx*> to_free;    // contexts to destroy outside the lock
    size_t pool_cap = 0;               // idle contexts kept at most
    size_t pool_ctx_max = 0;           // largest context (device bytes) kept idle
    size_t staged = 0;                 // device bytes of prepared requests waiting for admission
    long long batches = 0, batched_requests = 0;             // batch launches and the requests in them
    long long graphs_instantiated = 0, graphs_updated = 0;   // graph executables created / reused
    long long eager_batches = 0;       // batches run without a graph (capture failed)
    std::string last_failure;          // message of the most recent failed request
};

namespace {

int sfail(int code, const std::string& m) {
    scff::set_error(m);
    return code;
}

// caller holds s->mu: drop one queue reference; erase a request that was
// already handed back to its waiter and is no longer queued anywhere
void unref(scff_server* s, unsigned long long t) {
    auto it = s->reqs.find(t);
    if (it == s->reqs.end()) return;
    if (--it->second->queue_refs <= 0 && it->second->waited) s->reqs.erase(it);
}

Req* lookup(scff_server* s, unsigned long long t) {
    auto it = s->reqs.find(t);
    return it == s->reqs.end() ? nullptr : it->second.get();
}

// caller holds s->mu: an idle context, preferably one that holds molecule m
// (the most recently returned such context), else the most recently
// returned one; {NULL, NULL} when the pool is empty
Idle take_ctx(scff_server* s, const MolPtr& m) {
    if (s->ctx_pool.empty()) return Idle{};
    size_t k = s->ctx_pool.size() - 1;
    for (size_t i = s->ctx_pool.size(); i-- > 0;)
        if (same_mol(s->ctx_pool[i].mol, m)) {
            k = i;
            break;
        }
    Idle e = s->ctx_pool[k];
    s->ctx_pool.erase(s->ctx_pool.begin() + (long)k);
    return e;
}

// caller holds s->mu: return a context to the pool, or, when the pool is
// full or the context holds more device memory than an idle context may
// (idle contexts are not counted against the budget), queue it for
// destruction outside the lock (destroying waits for the device)
void give_ctx(scff_server* s, scff_ctx* c, MolPtr mol) {
    if (!c) return;
    if (s->ctx_pool.size() < s->pool_cap && scff::ctx_device_bytes(c) <= s->pool_ctx_max)
        s->ctx_pool.push_back(Idle{c, std::move(mol)});
    else
        s->to_free.push_back(c);
}

// output bytes of a request: f (complex64) and |f|^2 (float32), both staged
size_t out_points(const Req* r) {
    return (size_t)r->grid.n[0] * r->grid.n[1] * r->grid.n[2] * (size_t)r->n_states;
}

// a pinned staging buffer of at least `bytes`; caller does not hold s->mu.
// Sizes are rounded up to powers of two (at least 1 MiB) so buffers are
// reused across requests of similar size; when no idle buffer is large
// enough, the largest idle one is freed and a larger one allocated, so the
// server never holds more buffers than it has used at once (at most the
// requests running or waiting for their host copy, 2 x max_inflight).
void* take_stage(scff_server* s, size_t bytes) {
    size_t cls = (size_t)1 << 20;
    while (cls < bytes) cls <<= 1;
    void* drop = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->stage_free.lower_bound(cls);
        if (it != s->stage_free.end()) {
            void* p = it->second;
            s->stage_free.erase(it);
            return p;
        }
        if (!s->stage_free.empty()) {
            auto last = std::prev(s->stage_free.end());
            drop = last->second;
            s->stage_free.erase(last);
            s->stage_size.erase(drop);
            s->stage_all.erase(std::find(s->stage_all.begin(), s->stage_all.end(), drop));
        }
    }
    void* p = nullptr;
    {
        scff::GateShared g(scff::device_gate());
        if (drop) (void)hipHostFree(drop);   // idle: no copy uses it
        if (hipHostMalloc(&p, cls, hipHostMallocDefault) != hipSuccess) return nullptr;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->stage_all.push_back(p);
    s->stage_size[p] = cls;
    return p;
}

// destroy the queued contexts; caller does not hold s->mu
void drain_to_free(scff_server* s) {
    std::vector<scff_ctx*> v;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        v.swap(s->to_free);
    }
    for (scff_ctx* c : v) scff_destroy(c);
}

void finish(scff_server* s, Req* r, int status) {
    // caller holds s->mu
    r->status = status;
    r->state = St::Done;
    r->t_done = Clock::now();
    if (status == SCFF_OK) {
        ++s->n_completed;
        auto ns = [](Clock::time_point a, Clock::time_point b) {
            return (long long)std::chrono::duration_cast<std::chrono::nanoseconds>(b - a).count();
        };
        s->ns_stage[0] += ns(r->t_submit, r->t_prep0);
        s->ns_stage[1] += ns(r->t_prep0, r->t_prep1);
        s->ns_stage[2] += ns(r->t_prep1, r->t_run0);
        s->ns_stage[3] += ns(r->t_run0, r->t_run1);
        s->ns_stage[4] += ns(r->t_run1, r->t_done);
    } else {
        ++s->n_failed;
        s->last_failure = "ticket " + std::to_string(r->ticket) + ": " + scff_last_error();
    }
    s->cv_done.notify_all();
}

void prep_loop(scff_server* s) {
    // each prep thread stages its precompute on a stream of its own and waits
    // for it, so a prepared request is complete in device memory before a run
    // slot (another stream) evaluates it
    hipStream_t pst = nullptr;
    if (!s->fake) {
        (void)hipSetDevice(s->device);
        scff::GateShared g(scff::device_gate());
        if (hipStreamCreateWithFlags(&pst, hipStreamNonBlocking) != hipSuccess) pst = nullptr;
    }
    for (;;) {
        unsigned long long t;
        Req* r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            // a new prep starts while the admitted and the prepared-but-waiting
            // requests leave room in the budget (or nothing is prepared ahead)
            s->cv_prep.wait(lk, [&] {
                return s->stop || (!s->prep_q.empty() && (s->admitted + s->staged < s->budget || s->staged == 0));
            });
            if (s->stop) {
                if (pst) {
                    scff::GateShared g(scff::device_gate());
                    (void)hipStreamDestroy(pst);
                }
                return;
            }
            t = s->prep_q.front();
            s->prep_q.pop_front();
            r = lookup(s, t);
            if (!r) continue;
            if (r->state == St::Cancelled) {
                unref(s, t);
                continue;
            }
            ++r->queue_refs;   // held while prep runs unlocked
            r->t_prep0 = Clock::now();
        }
        int rc = SCFF_OK;
        size_t bytes = 0;
        scff_ctx* c = nullptr;
        MolPtr loaded;   // the molecule c holds
        std::string err;
        const MolKey& m = *r->mol;
        // validation common to both modes (host only); on a device the
        // molecule is validated by its load (or was, if a context holds it)
        {
            std::string e2;
            if (s->fake) {
                scff::Basis bchk;
                e2 = scff::build_basis(bchk, r->n_atoms, m.xyz.data(), r->n_shells, m.sh_atom.data(), m.sh_l.data(),
                                       m.sh_nprim.data(), m.exps.data(), m.coefs.data(), m.normalise);
            }
            if (e2.empty() && r->precision != SCFF_FP32 && r->precision != SCFF_BF16X3) e2 = "unknown precision";
            for (int a = 0; e2.empty() && a < 3; ++a)
                if (r->grid.n[a] < 1 || r->grid.n[a] > 4096) e2 = "grid n must be in 1..4096";
            if (!e2.empty()) {
                rc = SCFF_EINVAL;
                scff::set_error(e2);
            }
        }
        if (rc == SCFF_OK && !s->fake) {
            bool hit = false;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                Idle e = take_ctx(s, r->mol);
                c = e.c;
                hit = c && same_mol(e.mol, r->mol);
                if (hit) ++s->n_mol_hits;
            }
            if (!c) rc = scff_create(s->device, 0, &c);
            if (rc == SCFF_OK && !hit)
                rc = scff_load_molecule(c, r->n_atoms, m.xyz.data(), r->n_shells, m.sh_atom.data(), m.sh_l.data(),
                                        m.sh_nprim.data(), m.exps.data(), m.coefs.data(), m.normalise, nullptr);
            if (rc == SCFF_OK) loaded = r->mol;
            if (rc == SCFF_OK) rc = scff_load_transitions(c, r->n_states, r->T.data());
            if (rc == SCFF_OK) rc = scff_set_options(c, r->eps, r->spin);
            if (rc == SCFF_OK) rc = scff::ctx_prepare(c, &r->grid, r->precision, pst, &bytes);
        } else if (rc == SCFF_OK) {
            // scheduler test mode: footprint of the outputs only
            bytes = (size_t)r->grid.n[0] * r->grid.n[1] * r->grid.n[2] * (size_t)r->n_states * 12;
        }
        if (rc != SCFF_OK) err = scff_last_error();
        std::unique_lock<std::mutex> lk(s->mu);
        if (rc != SCFF_OK) {
            give_ctx(s, c, loaded);
            scff::set_error(err);
            // remove from the admission queue and fail alone
            for (auto it = s->admit_q.begin(); it != s->admit_q.end(); ++it)
                if (*it == t) {
                    s->admit_q.erase(it);
                    unref(s, t);
                    break;
                }
            if (r->state != St::Cancelled) finish(s, r, rc);
        } else if (r->state == St::Cancelled) {
            give_ctx(s, c, loaded);
        } else {
            r->ctx = c;
            r->ctx_mol = loaded;
            r->bytes = bytes;
            r->t_prep1 = Clock::now();
            r->state = St::Ready;
            s->staged += r->bytes;
        }
        unref(s, t);   // the prep reference
        unref(s, t);   // the prep_q entry
        s->cv_sched.notify_all();
        lk.unlock();
        drain_to_free(s);
    }
}

void sched_loop(scff_server* s) {
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (s->stop) return;
        bool progressed = false;
        while (!s->admit_q.empty()) {
            const unsigned long long t = s->admit_q.front();
            Req* r = lookup(s, t);
            if (!r || r->state == St::Cancelled || r->state == St::Done) {   // cancelled / failed in prep
                s->admit_q.pop_front();
                unref(s, t);
                progressed = true;
                continue;
            }
            if (r->state != St::Ready) break;                 // head not prepared yet
            if (r->bytes > s->budget) {                       // can never fit
                s->staged -= r->bytes;
                s->cv_prep.notify_all();
                s->admit_q.pop_front();
                unref(s, t);
                give_ctx(s, r->ctx, r->ctx_mol);
                r->ctx = nullptr;
                scff::set_error("request footprint exceeds the server's HBM budget");
                finish(s, r, SCFF_ENOMEM);
                progressed = true;
                continue;
            }
            // staged results waiting for their host copy hold pinned buffers:
            // bound them (and so the pinned memory) by the run slots
            if (s->inflight >= s->max_inflight || s->inflight + s->copying >= 2 * s->max_inflight ||
                s->admitted + r->bytes > s->budget)
                break;
            s->admit_q.pop_front();
            unref(s, t);
            r->state = St::Running;
            s->admitted += r->bytes;
            s->staged -= r->bytes;
            if (s->admitted > s->peak_admitted) s->peak_admitted = s->admitted;
            ++s->inflight;
            if (s->inflight > s->peak_inflight) s->peak_inflight = s->inflight;
            s->run_q.push_back(t);
            s->cv_run.notify_one();
            progressed = true;
        }
        if (!progressed) s->cv_sched.wait(lk);
    }
}

// A batch runner: takes the admitted requests waiting for it (up to half of
// max_inflight, rounded up), and runs them as one batch on its own stream:
//   reserve   each request's device buffers (tables, outputs, split sums)
//             and its grid-kernel descriptor, nothing launched yet;
//   capture   into a graph: upload of the descriptors and of the queue of
//             (request, tile) items, counter reset (a kernel), each
//             request's 1D tables, one persistent grid kernel per kernel
//             variant present, popping the items of all requests of that
//             variant from the queue, then each request's split reduction
//             and the copy of its results into its pinned staging buffer;
//   replay    the graph: an executable graph is kept per launch topology and
//             its parameters updated for the next batch of the same
//             topology (hipGraphExecUpdate), else one is instantiated.
// Two runners alternate, so one batch is assembled while the other runs.
struct Runner {
    hipStream_t st = nullptr;
    void* d_buf = nullptr;     // descriptors, then items
    size_t d_cap = 0;
    int* d_cnt = nullptr;      // one queue counter per kernel variant
    void* h_buf = nullptr;     // pinned staging of descriptors and items
    size_t h_cap = 0;
    std::vector<std::pair<std::string, hipGraphExec_t>> execs;   // by topology, most recent last
    long long graphs_instantiated = 0, graphs_updated = 0, eager_batches = 0;
};

constexpr size_t kMaxExecs = 32;
constexpr int kRunners = 2;
constexpr int kVariants = 4;

int grow_device(void** p, size_t* cap, size_t need) {
    if (*cap >= need) return SCFF_OK;
    size_t c = std::max<size_t>(need, 2 * *cap);
    c = std::max<size_t>(c, 4096);
    scff::GateShared g(scff::device_gate());
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc(p, c) != hipSuccess) return sfail(SCFF_ENOMEM, "batch queue allocation failed");
    *cap = c;
    return SCFF_OK;
}

int grow_pinned(void** p, size_t* cap, size_t need) {
    if (*cap >= need) return SCFF_OK;
    size_t c = std::max<size_t>(need, 2 * *cap);
    c = std::max<size_t>(c, 4096);
    scff::GateShared g(scff::device_gate());
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipHostMalloc(p, c, hipHostMallocDefault) != hipSuccess) return sfail(SCFF_ENOMEM, "pinned queue allocation failed");
    *cap = c;
    return SCFF_OK;
}

struct Member {
    Req* r;
    void* stage = nullptr;
    scff::BatchEval be;
    int rc = SCFF_OK;
    std::string err;
};

// Enqueues the batch's device work on R.st (the same calls whether the stream
// is being captured or not).
int enqueue_batch(Runner& R, std::vector<Member*>& live, const int off[], size_t need, std::string& err) {
    const auto* d_desc = (const scff::GridDesc*)R.d_buf;
    const size_t dbytes = (live.size() * sizeof(scff::GridDesc) + 255) & ~(size_t)255;
    const auto* d_items = (const int2*)((const char*)R.d_buf + dbytes);
    hipError_t e = hipMemcpyAsync(R.d_buf, R.h_buf, need, hipMemcpyHostToDevice, R.st);
    if (e == hipSuccess) e = scff::launch_zero_counters(R.d_cnt, kVariants, R.st);
    if (e != hipSuccess) {
        err = std::string("queue upload: ") + hipGetErrorString(e);
        return SCFF_EDEVICE;
    }
    for (Member* m : live)
        if (scff::ctx_batch_tables(m->r->ctx, &m->r->grid, R.st) != SCFF_OK) {
            err = scff_last_error();
            return SCFF_EDEVICE;
        }
    const int ncu = scff::ctx_n_cu(live[0]->r->ctx);
    for (int v = 0; v < kVariants; ++v) {
        const int n = off[v + 1] - off[v];
        if (n == 0) continue;
        const int wgs = std::min(n, ncu * scff::grid_wg_per_cu(v % 2 + 1, v / 2));
        e = scff::launch_grid_batch(v, d_desc, d_items + off[v], n, R.d_cnt + v, wgs, R.st);
        if (e != hipSuccess) {
            err = std::string("batch grid kernel: ") + hipGetErrorString(e);
            return SCFF_EDEVICE;
        }
    }
    for (Member* m : live) {
        const size_t np = m->be.nout;
        float* sf = m->r->f ? (float*)m->stage : nullptr;
        float* sf2 = m->r->f2 ? (float*)m->stage + 2 * np : nullptr;
        if (scff::ctx_batch_finish(m->r->ctx, &m->r->grid, m->be, sf, sf2, R.st) != SCFF_OK) {
            err = scff_last_error();
            return SCFF_EDEVICE;
        }
    }
    return SCFF_OK;
}

// Runs the batch's device work; returns SCFF_OK or the error of a launch (then
// every member that had not failed alone fails with it).  The launches are
// captured into a graph and replayed; if the capture itself fails (another
// thread's device-wide call can invalidate it), the same launches run
// eagerly on the stream.
int run_batch(scff_server* s, Runner& R, std::vector<Member>& ms) {
    (void)s;
    std::vector<Member*> live;
    for (Member& m : ms)
        if (m.rc == SCFF_OK) live.push_back(&m);
    if (live.empty()) return SCFF_OK;
    // queue of (descriptor, tile) items, grouped by kernel variant, requests in ticket order
    std::vector<int2> items;
    int off[kVariants + 1] = {};
    for (int v = 0; v < kVariants; ++v) {
        off[v] = (int)items.size();
        for (size_t i = 0; i < live.size(); ++i)
            if (live[i]->be.cls == v)
                for (long long b = 0; b < live[i]->be.blocks; ++b) items.push_back(make_int2((int)i, (int)b));
    }
    off[kVariants] = (int)items.size();
    const size_t dbytes = (live.size() * sizeof(scff::GridDesc) + 255) & ~(size_t)255;
    const size_t need = dbytes + items.size() * sizeof(int2);
    int rc;
    if ((rc = grow_device(&R.d_buf, &R.d_cap, need)) || (rc = grow_pinned(&R.h_buf, &R.h_cap, need))) return rc;
    for (size_t i = 0; i < live.size(); ++i)
        std::memcpy((char*)R.h_buf + i * sizeof(scff::GridDesc), &live[i]->be.desc, sizeof(scff::GridDesc));
    std::memcpy((char*)R.h_buf + dbytes, items.data(), items.size() * sizeof(int2));
    // launch topology: per member its variant, split and outputs; per variant whether it runs
    std::string topo;
    for (Member* m : live)
        topo += std::to_string(m->be.cls) + (m->be.n_split > 1 ? "s" : "u") + (m->r->f ? "f" : "-") +
                (m->r->f2 ? "g" : "-") + ";";
    for (int v = 0; v < kVariants; ++v)
        if (off[v + 1] > off[v]) topo += "k" + std::to_string(v);
    std::string err;
    hipGraph_t graph = nullptr;
    bool captured = false, began = false;
    {
        // no allocation, release or device synchronisation in any thread of
        // the process while the stream is captured
        std::unique_lock<std::shared_mutex> gate(scff::device_gate());
        if (hipStreamBeginCapture(R.st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            began = true;
            rc = enqueue_batch(R, live, off, need, err);
            const hipError_t e = hipStreamEndCapture(R.st, &graph);
            captured = rc == SCFF_OK && e == hipSuccess && graph;
            if (!captured && graph) {
                (void)hipGraphDestroy(graph);
                graph = nullptr;
            }
        }
        (void)hipGetLastError();   // a failed capture leaves its error behind
    }
    if (!captured && began) {
        // the stream of a failed capture may keep its error: run the eager
        // launches on a fresh one
        scff::GateShared g(scff::device_gate());
        hipStream_t fresh = nullptr;
        if (hipStreamCreateWithFlags(&fresh, hipStreamNonBlocking) == hipSuccess) {
            (void)hipStreamDestroy(R.st);
            R.st = fresh;
        }
        (void)hipGetLastError();
    }
    hipGraphExec_t exec = nullptr;
    if (captured) {
        // an executable graph of this topology: update it, else instantiate one
        for (size_t i = 0; i < R.execs.size(); ++i)
            if (R.execs[i].first == topo) {
                exec = R.execs[i].second;
                R.execs.erase(R.execs.begin() + (long)i);
                break;
            }
        if (exec) {
            hipGraphExecUpdateResult res;
            hipGraphNode_t bad = nullptr;
            if (hipGraphExecUpdate(exec, graph, &bad, &res) != hipSuccess || res != hipGraphExecUpdateSuccess) {
                (void)hipGetLastError();
                scff::GateShared g(scff::device_gate());
                (void)hipGraphExecDestroy(exec);
                exec = nullptr;
            } else {
                ++R.graphs_updated;
            }
        }
        if (!exec) {
            scff::GateShared g(scff::device_gate());
            if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
                ++R.graphs_instantiated;
            } else {
                (void)hipGetLastError();
                exec = nullptr;
            }
        }
        (void)hipGraphDestroy(graph);
    }
    hipError_t e;
    if (exec) {
        R.execs.emplace_back(topo, exec);
        if (R.execs.size() > kMaxExecs) {
            scff::GateShared g(scff::device_gate());
            (void)hipGraphExecDestroy(R.execs.front().second);
            R.execs.erase(R.execs.begin());
        }
        e = hipGraphLaunch(exec, R.st);
    } else {
        // no graph (capture or instantiation failed): the same launches, eagerly
        ++R.eager_batches;
        err.clear();
        if ((rc = enqueue_batch(R, live, off, need, err)) != SCFF_OK) {
            (void)hipStreamSynchronize(R.st);
            return sfail(rc, err);
        }
        e = hipSuccess;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(R.st);
    if (e != hipSuccess) return sfail(SCFF_EDEVICE, std::string("batch: ") + hipGetErrorString(e));
    return SCFF_OK;
}

void run_loop(scff_server* s) {
    Runner R;
    if (!s->fake) {
        (void)hipSetDevice(s->device);
        scff::GateShared g(scff::device_gate());
        if (hipStreamCreateWithFlags(&R.st, hipStreamNonBlocking) != hipSuccess) R.st = nullptr;
        if (hipMalloc((void**)&R.d_cnt, kVariants * sizeof(int)) != hipSuccess) R.d_cnt = nullptr;
    }
    for (;;) {
        std::vector<Member> ms;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_run.wait(lk, [&] { return s->stop || !s->run_q.empty(); });
            if (s->stop && s->run_q.empty()) break;
            const auto now = Clock::now();
            // at most half the in-flight cap per batch, so that the other
            // runner always has requests to run beside it: one batch's tail
            // (last tiles, reductions, result copies) overlaps the other's
            // grid kernels
            const int take = std::max(1, (s->max_inflight + kRunners - 1) / kRunners);
            while (!s->run_q.empty() && (int)ms.size() < take) {
                Req* r = lookup(s, s->run_q.front());
                s->run_q.pop_front();
                if (!r) continue;
                r->t_run0 = now;
                Member m;
                m.r = r;
                ms.push_back(std::move(m));
            }
            s->batches += ms.empty() ? 0 : 1;
            s->batched_requests += (long long)ms.size();
        }
        if (!s->fake) {
            for (Member& m : ms) {
                Req* r = m.r;
                if (!R.st || !R.d_cnt) {
                    m.rc = SCFF_EDEVICE;
                    m.err = "batch runner has no stream or queue counters";
                    continue;
                }
                m.stage = take_stage(s, out_points(r) * (sizeof(float) * 2 + sizeof(float)));
                if (!m.stage) {
                    m.rc = SCFF_ENOMEM;
                    m.err = "pinned staging buffer allocation failed";
                    continue;
                }
                m.rc = scff::ctx_batch_reserve(r->ctx, &r->grid, r->precision, r->f != nullptr, r->f2 != nullptr, &m.be);
                if (m.rc != SCFF_OK) m.err = scff_last_error();
            }
            const int brc = run_batch(s, R, ms);
            if (brc != SCFF_OK) {
                const std::string err = scff_last_error();
                for (Member& m : ms)
                    if (m.rc == SCFF_OK) {
                        m.rc = brc;
                        m.err = err;
                    }
            }
            for (Member& m : ms) scff::ctx_batch_done(m.r->ctx);
        } else {
            std::this_thread::sleep_for(std::chrono::milliseconds(2));
        }
        std::unique_lock<std::mutex> lk(s->mu);
        s->graphs_instantiated += R.graphs_instantiated;
        s->graphs_updated += R.graphs_updated;
        s->eager_batches += R.eager_batches;
        R.graphs_instantiated = R.graphs_updated = R.eager_batches = 0;
        for (Member& m : ms) {
            Req* r = m.r;
            r->t_run1 = Clock::now();
            give_ctx(s, r->ctx, r->ctx_mol);
            r->ctx = nullptr;
            s->admitted -= r->bytes;
            s->cv_prep.notify_all();
            --s->inflight;
            if (m.rc == SCFF_OK && m.stage) {
                // results are staged: the copy threads finish the request
                ++s->copying;
                s->copy_q.emplace_back(r->ticket, m.stage);
                s->cv_copy.notify_one();
            } else if (m.rc == SCFF_OK) {   // scheduler test mode
                finish(s, r, SCFF_OK);
            } else {
                if (m.stage) s->stage_free.emplace(s->stage_size[m.stage], m.stage);
                scff::set_error(m.err);
                finish(s, r, m.rc);
            }
        }
        s->cv_sched.notify_all();
        lk.unlock();
        drain_to_free(s);
    }
    scff::GateShared g(scff::device_gate());
    for (auto& x : R.execs) (void)hipGraphExecDestroy(x.second);
    if (R.d_buf) (void)hipFree(R.d_buf);
    if (R.d_cnt) (void)hipFree(R.d_cnt);
    if (R.h_buf) (void)hipHostFree(R.h_buf);
    if (R.st) (void)hipStreamDestroy(R.st);
}

void copy_loop(scff_server* s) {
    for (;;) {
        unsigned long long t;
        void* stage;
        Req* r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_copy.wait(lk, [&] { return s->stop || !s->copy_q.empty(); });
            if (s->copy_q.empty()) return;   // stop, nothing left
            t = s->copy_q.front().first;
            stage = s->copy_q.front().second;
            s->copy_q.pop_front();
            r = lookup(s, t);
        }
        // the request stays in the map while it is not Done (no waiter can take it)
        const size_t np = out_points(r);
        if (r->f) std::memcpy(r->f, stage, np * 2 * sizeof(float));
        if (r->f2) std::memcpy(r->f2, (const float*)stage + 2 * np, np * sizeof(float));
        std::lock_guard<std::mutex> lk(s->mu);
        s->stage_free.emplace(s->stage_size[stage], stage);
        --s->copying;
        finish(s, r, SCFF_OK);
        s->cv_sched.notify_all();
    }
}

template <class T>
void copy_in(std::vector<T>& dst, const T* src, size_t n) {
    dst.assign(src, src + n);
}

}  // namespace

extern "C" {

int scff_server_create(int device, size_t hbm_budget_bytes, int max_inflight, scff_server** out) {
    if (!out) return sfail(SCFF_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_inflight < 1 || max_inflight > 64) return sfail(SCFF_EINVAL, "max_inflight must be in 1..64");
    const bool fake = (device == -1);
    if (!fake) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return sfail(SCFF_EDEVICE, "no HIP device available");
        if (device < 0 || device >= n) return sfail(SCFF_EINVAL, "device index out of range");
    }
    scff_server* s = new scff_server();
    s->device = fake ? 0 : device;
    s->fake = fake;
    s->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)64 << 30;
    s->max_inflight = max_inflight;
    const int n_prep = 8;
    // every thread can hold one context; prepared requests waiting for
    // admission hold theirs until they run
    s->pool_cap = (size_t)(n_prep + max_inflight);
    s->pool_ctx_max = s->budget / (2 * s->pool_cap);
    for (int i = 0; i < n_prep; ++i) s->threads.emplace_back(prep_loop, s);
    s->threads.emplace_back(sched_loop, s);
    for (int i = 0; i < kRunners; ++i) s->threads.emplace_back(run_loop, s);
    for (int i = 0; i < 2; ++i) s->threads.emplace_back(copy_loop, s);
    *out = s;
    return SCFF_OK;
}

int scff_server_submit(scff_server* s, const scff_request* q, unsigned long long* ticket) {
    if (!s || !q || !ticket) return sfail(SCFF_EINVAL, "NULL argument");
    if (q->n_atoms <= 0 || q->n_shells <= 0 || !q->xyz_bohr || !q->shell_atom || !q->shell_l ||
        !q->shell_nprim || !q->exps || !q->coefs || !q->T)
        return sfail(SCFF_EINVAL, "malformed request (sizes or NULL arrays)");
    if (q->n_states < 1 || q->n_states > scff::kMaxStates) return sfail(SCFF_EINVAL, "n_states must be in 1..32");
    if (!q->f && !q->f2) return sfail(SCFF_EINVAL, "request has no output buffer");
    int nprim = 0, nbf = 0;
    for (int i = 0; i < q->n_shells; ++i) {
        if (q->shell_nprim[i] < 1 || q->shell_nprim[i] > 32) return sfail(SCFF_EINVAL, "shell_nprim out of range");
        if (q->shell_l[i] < 0 || q->shell_l[i] > 2) return sfail(SCFF_EINVAL, "shell_l must be 0..2");
        nprim += q->shell_nprim[i];
        nbf += (q->shell_l[i] + 1) * (q->shell_l[i] + 2) / 2;
    }
    auto r = std::make_unique<Req>();
    {
        auto m = std::make_shared<MolKey>();
        copy_in(m->xyz, q->xyz_bohr, (size_t)3 * q->n_atoms);
        copy_in(m->sh_atom, q->shell_atom, q->n_shells);
        copy_in(m->sh_l, q->shell_l, q->n_shells);
        copy_in(m->sh_nprim, q->shell_nprim, q->n_shells);
        copy_in(m->exps, q->exps, nprim);
        copy_in(m->coefs, q->coefs, nprim);
        m->normalise = q->normalise;
        r->mol = std::move(m);
    }
    copy_in(r->T, q->T, (size_t)q->n_states * nbf * nbf);
    r->n_atoms = q->n_atoms;
    r->n_shells = q->n_shells;
    r->n_states = q->n_states;
    r->precision = q->precision;
    r->grid = q->grid;
    r->eps = q->screen_eps;
    r->spin = q->spin_factor;
    r->f = q->f;
    r->f2 = q->f2;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    const unsigned long long t = s->next_ticket++;
    r->ticket = t;
    r->queue_refs = 2;   // prep_q + admit_q
    s->reqs[t] = std::move(r);
    s->prep_q.push_back(t);
    s->admit_q.push_back(t);
    ++s->n_submitted;
    *ticket = t;
    s->cv_prep.notify_one();
    return SCFF_OK;
}

int scff_server_wait(scff_server* s, unsigned long long ticket, long long timeout_ns, int* status,
                     long long* latency_ns) {
    if (!s) return sfail(SCFF_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second->waited) return sfail(SCFF_EINVAL, "unknown ticket");
    Req* r = it->second.get();
    auto done = [&] { return r->state == St::Done || r->state == St::Cancelled; };
    if (timeout_ns < 0)
        s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), done))
        return sfail(SCFF_EBUSY, "request not finished");
    const int st = r->state == St::Cancelled ? SCFF_ECANCELLED : r->status;
    if (status) *status = st;
    if (latency_ns)
        *latency_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(r->t_done - r->t_submit).count();
    r->waited = true;
    if (r->queue_refs <= 0) s->reqs.erase(it);
    return SCFF_OK;
}

int scff_server_cancel(scff_server* s, unsigned long long ticket) {
    if (!s) return sfail(SCFF_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return sfail(SCFF_EINVAL, "unknown ticket");
    Req* r = it->second.get();
    if (r->state == St::Running || r->state == St::Done) return sfail(SCFF_EBUSY, "request already running or finished");
    if (r->state == St::Ready) {
        s->staged -= r->bytes;
        s->cv_prep.notify_all();
    }
    r->state = St::Cancelled;
    r->t_done = Clock::now();
    give_ctx(s, r->ctx, r->ctx_mol);
    r->ctx = nullptr;
    ++s->n_cancelled;
    s->cv_done.notify_all();
    s->cv_sched.notify_all();
    return SCFF_OK;
}

int scff_server_stats_get(scff_server* s, scff_server_stats* o) {
    if (!s || !o) return sfail(SCFF_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    o->submitted = s->n_submitted;
    o->completed = s->n_completed;
    o->failed = s->n_failed;
    o->cancelled = s->n_cancelled;
    o->queued = (long long)s->admit_q.size();
    o->inflight = s->inflight;
    o->admitted_bytes = s->admitted;
    o->budget_bytes = s->budget;
    o->peak_admitted_bytes = s->peak_admitted;
    o->peak_inflight = s->peak_inflight;
    o->mol_cache_hits = s->n_mol_hits;
    for (int i = 0; i < 5; ++i) o->ns_stage[i] = s->ns_stage[i];
    o->batches = s->batches;
    o->batched_requests = s->batched_requests;
    o->graphs_instantiated = s->graphs_instantiated;
    o->graphs_updated = s->graphs_updated;
    o->eager_batches = s->eager_batches;
    return SCFF_OK;
}

int scff_server_last_failure(scff_server* s, char* buf, size_t len) {
    if (!s || !buf || len == 0) return sfail(SCFF_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    const size_t n = std::min(len - 1, s->last_failure.size());
    std::memcpy(buf, s->last_failure.data(), n);
    buf[n] = '\0';
    return SCFF_OK;
}

void scff_server_destroy(scff_server* s) {
    if (!s) return;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        // cancel everything not yet running, let running requests finish
        for (auto& kv : s->reqs)
            if (kv.second->state == St::Queued || kv.second->state == St::Ready)
                kv.second->state = St::Cancelled;   // contexts are freed below
        s->admit_q.clear();
        s->cv_done.wait(lk, [&] { return s->inflight == 0 && s->run_q.empty() && s->copying == 0; });
        s->stop = true;
    }
    s->cv_prep.notify_all();
    s->cv_sched.notify_all();
    s->cv_run.notify_all();
    s->cv_done.notify_all();
    s->cv_copy.notify_all();
    for (auto& t : s->threads) t.join();
    for (auto& kv : s->reqs)
        if (kv.second->ctx) scff_destroy(kv.second->ctx);
    for (Idle& e : s->ctx_pool) scff_destroy(e.c);
    for (scff_ctx* c : s->to_free) scff_destroy(c);
    {
        scff::GateShared g(scff::device_gate());
        for (void* p : s->stage_all) (void)hipHostFree(p);
    }
    delete s;
}

}  // extern "C"
