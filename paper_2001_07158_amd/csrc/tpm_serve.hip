// The serving loop (C ABI: tpm_server_*) and the batch engines behind tpm_batch_run.
//
// Two engines, both continuous batching over a resident graph:
//   * Row mode: one multi-query row (tpm_sieve.hip: k_step) of up to 64 lanes.  A lane
//     group is one (query, chunk of sieve points) with its own seed and level; every
//     row step advances each group one level in one sweep over the in-edge index.  A
//     group that ran its last level frees its lanes, and waiting requests take free
//     lanes at the next step: any request that fits, so a small request is not held
//     behind a large one (a request that does not fit may be overtaken 8 times, then
//     admission waits for it).  Extraction of a hit's path runs on its own thread and
//     stream, off the step loop.
//   * Pruned mode: each request runs alone on the subgraph of its own colours (the
//     paper's preprocessing step (i), section "Implementation"; exact, since a vertex
//     of another colour has z = 0).  Up to 4 worker threads, each with its own HIP
//     stream, subgraph arena, sieve workspace and a fixed share of the state budget,
//     hold requests at once; a request takes the widest chunk whose device memory
//     (estimated from the exact edge count of its colour pairs) fits the share.  One
//     worker uses the device at a time, while the others admit requests and extract
//     paths on the host; admission takes the least device work first unless the
//     oldest request has waited long.
// Results are bit-identical to the same query run alone: fingerprints depend only on
// (seed, tag, indices), never on lanes, steps, streams or subgraphs.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "tpm_internal.h"

namespace tpm {

void store_path_into(const tpm_query &q, const int32_t *pv, const int64_t *pe, tpm_result &r) {
    for (int i = 0; i < q.k; ++i) r.path_vertices[i] = pv[i];
    for (int i = 0; i + 1 < q.k; ++i) r.path_edges[i] = pe[i];
}

void extract_into(const Graph &G, const tpm_query &q, tpm_result &r, hipStream_t st,
                  const uint8_t *q_loc) {
    int64_t pe[16];
    int32_t pv[16];
    r.path_status = TPM_NOTFOUND;
    if (q.k >= 2) {
        r.path_status = q_loc ? extract_from_vertices(G, q.multiset, q.k, q_loc, kQuickDfsBudget, pv, pe)
                              : extract_vertexloc(G, q.multiset, q.k, q.seed, 2, pv, pe, nullptr,
                                                  kQuickDfsBudget);
    }
    if (r.path_status != TPM_OK) r.path_status = extract_path(G, q.multiset, q.k, q.seed, 8, pv, pe, st);
    if (r.path_status == TPM_OK) store_path_into(q, pv, pe, r);
}

}  // namespace tpm

using namespace tpm;

namespace {

constexpr int kMaxBypass = 8;     // times a waiting request may be overtaken
constexpr double kAgeMs = 750;    // pruned mode: a request waiting longer goes first
constexpr double kExpressShare = 0.05;  // serial servers: budget of the express workers
constexpr int kMaxStreams = 4;    // worker streams (the device serves 4 hardware queues)

struct SReq {
    tpm_query q{};
    std::vector<int32_t> ms;
    uint8_t *user_pp = nullptr;
    std::vector<uint8_t> pp;  // 2^k per-point values, filled as chunks finish
    uint64_t ticket = 0;
    double t_submit = 0, t_start = -1, deadline = 0;  // host clock, ms (deadline 0: none)
    std::atomic<int> cancel{0};
    std::atomic<bool> finished{false};
    bool want_path = false;
    int bypassed = 0;
    // pruned mode
    int64_t mk = 0;        // edges of its colour subgraph (whole graph for wildcards)
    bool whole = false;    // runs on the whole graph (wildcards)
    int C = 0;             // sieve points per pass chosen at admission
    int max_c = 1024;      // widest chunk allowed (halved after a failed allocation)
    int64_t est = 0;       // estimated device bytes at admission
    double cost = 0;       // estimated device work (bytes moved by its subgraph build and sieve)
    int tries = 0;
    // row mode
    int chunks_left = 0, next_chunk = 0, groups_live = 0;
    uint8_t total = 0;
};
using ReqP = std::shared_ptr<SReq>;

void check_query(const Graph &G, const tpm_query &q) {
    TPM_REQUIRE(q.multiset != nullptr, "query multiset must not be NULL");
    TPM_REQUIRE(q.k >= 1 && q.k <= 16, "k must be in [1, 16]");
    TPM_REQUIRE(q.deadline_ms >= 0, "deadline_ms must be >= 0");
    for (int i = 0; i < q.k; ++i)
        TPM_REQUIRE(q.multiset[i] >= -1 && q.multiset[i] < G.q, "multiset colour out of range");
}

// lane-group geometry of a query of size k on rows with W dwords per lane
int group_points(int k, int W) {
    const int pts = 1 << k;
    const int unit = 4 * W;
    return std::max(pts, unit);  // padded to whole lanes; padded points are ignored
}

struct WorkerMem {
    GraphArena *arena = nullptr;  // subgraph index and build temporaries
    Workspace *ws = nullptr;      // sieve state
    int64_t accounted = 0;        // bytes counted against the budget for this worker
    bool busy = false;
};

}  // namespace

struct tpm_server {
    const tpm_graph *g = nullptr;
    tpm_server_config cfg{};
    bool pruned = false;
    std::mutex mu;
    std::condition_variable cv;       // queue, memory or stop changed
    std::condition_variable cv_done;  // a result was produced
    std::deque<ReqP> queue;
    std::map<uint64_t, ReqP> live;    // submitted and not finished
    std::deque<tpm_result> done;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::string error;
    std::vector<std::thread> threads;
    // counters
    uint64_t steps = 0;
    int64_t completed = 0, cancelled = 0, rejected = 0;
    double prune_ms = 0, sieve_ms = 0, extract_ms = 0;
    int inflight = 0, inflight_peak = 0;
    int queued_peak = 0;  // most requests waiting for admission at once
    int64_t trims = 0;  // pruned mode: times a worker gave its device memory back
    double gpu_wait_ms = 0;
    // pruned mode, serial device use (servers): one worker uses the device at a time.
    // Worker 0 takes any request; the others ("express" workers) take only requests
    // that fit their small share at full width.  Between two levels of a sieve, worker 0
    // lends the device to a waiting express worker for one whole request, then takes
    // it back before any other express request.
    bool serial = false;
    std::mutex dev_mu;
    std::condition_variable dev_cv;
    int dev_owner = -1;      // worker holding the device
    int dev_exp_waiting = 0; // express workers waiting for it
    bool dev_lent = false;   // worker 0 has lent it in the middle of a sieve
    bool dev_back = false;   // the loan ended: worker 0 takes it next
    // row mode
    int W = 1, lanes = 64;
    int row_points_cap = 1024;  // widest row allowed (internal batches: the tuning's chunk)
    bool use_graph = false;
    std::deque<std::pair<ReqP, tpm_result>> ext_queue;  // hits waiting for a path
    std::condition_variable ext_cv;
    bool rows_done = false;  // the row loop has ended (the extraction thread may finish)
    // pruned mode
    int nstreams = 0;
    int64_t budget = 0, held = 0, held_peak = 0;
    std::vector<int64_t> share;  // per worker: its share of the budget
    std::vector<int64_t> pair_counts;  // q x q edge counts by colour pair (whole graphs)
    std::vector<WorkerMem> wm;
    // memory: pools owned by the server, or borrowed from the graph (internal batches)
    WorkspacePool *ppool = nullptr;
    GraphArena *arena = nullptr;      // row-mode extraction subgraphs
    bool own_pools = true;
};

namespace {

// ------------------------------------------------------------------ results
// Hands a finished request's result out (per-point bytes first, so a result that is
// visible to tpm_server_poll never has a half-written per-point buffer).
void finish(tpm_server *s, SReq &rq, tpm_result r) {
    if (rq.finished.exchange(true)) return;
    r.ticket = rq.ticket;
    r.t_submit_ms = rq.t_submit;
    r.t_start_ms = rq.t_start >= 0 ? rq.t_start : now_ms();
    r.t_done_ms = now_ms();
    if (r.status == TPM_OK && rq.user_pp && rq.pp.size() >= ((size_t)1 << rq.q.k))
        std::memcpy(rq.user_pp, rq.pp.data(), (size_t)1 << rq.q.k);
    std::lock_guard<std::mutex> lk(s->mu);
    s->live.erase(rq.ticket);
    s->done.push_back(r);
    s->completed++;
    if (r.status == TPM_ECANCELLED) s->cancelled++;
    if (r.status == TPM_ENOMEM) s->rejected++;
    s->cv_done.notify_all();
}

tpm_result status_result(tpm_status st) {
    tpm_result r;
    std::memset(&r, 0, sizeof(r));
    r.status = st;
    return r;
}

bool expired(const SReq &rq, double now) {
    return rq.cancel.load() != 0 || (rq.deadline > 0 && now > rq.deadline);
}

// Removes cancelled or expired requests from the queue; their results are produced by
// the caller after the lock is released.  Caller holds s->mu.
void purge_queue(tpm_server *s, std::vector<ReqP> &gone) {
    const double now = now_ms();
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        if (expired(**it, now)) {
            // a row-mode request with chunks on the row ends when those leave it
            if ((*it)->groups_live == 0) {
                if ((*it)->t_start >= 0) s->inflight--;
                gone.push_back(*it);
            }
            it = s->queue.erase(it);
        } else {
            ++it;
        }
    }
}

void finish_gone(tpm_server *s, std::vector<ReqP> &gone) {
    for (auto &rq : gone) finish(s, *rq, status_result(TPM_ECANCELLED));
    gone.clear();
}

// Wait bound while requests with deadlines are queued (expiry is noticed on wake-up).
bool any_deadline(tpm_server *s) {
    for (auto &rq : s->queue)
        if (rq->deadline > 0) return true;
    return false;
}

void record_error(tpm_server *s, const std::string &msg) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->error.empty()) s->error = msg;
    s->cv_done.notify_all();
}

// ------------------------------------------------------------------ pruned mode
// Estimated device bytes of one request on a worker: its subgraph's index and build
// temporaries (the parent's m bytes of keep flags and 4m of scan output, about 36
// bytes per kept edge, per-vertex arrays) and its sieve state (per-vertex rows of C
// points, two level buffers of R C bytes with R estimated from the parent's ratio of
// stored rows to edges plus a margin, localisation bytes).  Over-estimates are
// harmless; an under-estimate only lets the workers hold a little more than the
// budget.
int64_t est_request_bytes(const Graph &G, int64_t mk, bool whole, int k, int C, bool loc) {
    const int64_t n = G.n;
    const int64_t T = std::max<int32_t>(1, G.tile_auto ? auto_tile_edges(mk) : G.tile_edges);
    const int64_t tiles = 2 * mk / T + std::min<int64_t>(n, mk) + 1;
    int64_t arena = 0;
    if (!whole)
        // parent-sized: the kept-position rank records, their counts and bases (about
        // m / 7); per kept edge: six index arrays (seven with departure times), the
        // remapped read positions, the needed-position flags and their rank records; per
        // vertex: colours, in-list starts, vertex flags
        arena = G.m / 6 + (G.pdep ? 34 : 30) * mk + 44 * n + 12 * tiles + (int64_t(16) << 20);
    // stored rows per kept edge: colour subgraphs of the serving and batched workloads
    // keep the whole graph's ratio within 3 % (checked on samples); the 50 % margin
    // leaves room on the device (smaller margins let the largest requests take
    // 1024-point rows whose buffers filled the device and made regrowth slow)
    const double ratio = G.m ? (double)G.R / (double)G.m : 1.0;
    const int64_t R = whole ? G.R : std::min<int64_t>(mk, (int64_t)std::ceil(1.5 * ratio * (double)mk) + 1024);
    const int64_t rowb = std::max(C, 16);
    int64_t ws = 16 * n + n * rowb + (k > 2 ? 2 : 1) * R * rowb + 2 * (mk / T + 1) * rowb +
                 std::max<int64_t>(int64_t(1) << k, rowb) + 2 * n + (int64_t(1) << 20);
    // level 2's coefficient form: 20 bytes a row, 64 bytes per 256 positions
    if (k > 2) ws += 20 * R + (mk / 256 + 1) * 64 + (int64_t(1) << 20);
    if (loc) ws += mk;
    return arena + ws;
}

int64_t worker_bytes(const WorkerMem &w) {
    return arena_bytes(w.arena) + workspace_bytes(w.ws);
}

// Edge count of a request's colour subgraph from the pair counts (exact for whole graphs
// with at most 64 colours); wildcard queries use the whole graph.
void size_request(tpm_server *s, SReq &rq) {
    const Graph &G = s->g->G;
    rq.whole = false;
    for (int32_t c : rq.ms) rq.whole |= c < 0;
    if (rq.whole || s->pair_counts.empty()) {
        rq.mk = G.m;
        rq.whole = rq.whole || s->pair_counts.empty();
        return;
    }
    std::vector<uint8_t> in((size_t)G.q, 0);
    for (int32_t c : rq.ms) in[(size_t)c] = 1;
    int64_t mk = 0;
    for (int a = 0; a < G.q; ++a)
        if (in[(size_t)a])
            for (int b = 0; b < G.q; ++b)
                if (in[(size_t)b]) mk += s->pair_counts[(size_t)a * G.q + b];
    rq.mk = mk;
}

// Device work of a request, for ordering: its subgraph build scans the parent index
// (about 12 bytes per edge), its sieve moves about (k - 1) C bytes per kept edge and
// sieve point.
void cost_request(const Graph &G, SReq &rq) {
    const int k = rq.q.k;
    const double pts = (double)std::max(16, 1 << k);
    rq.cost = (rq.whole ? 0.0 : 12.0 * (double)G.m) + (double)rq.mk * std::max(1, k - 1) * pts;
}

int preferred_chunk(int k) { return std::max(16, std::min(1 << k, 1024)); }

// Widest chunk a request may take (halved after a failed allocation).
int max_chunk(const tpm_server *, const SReq &rq) { return std::max(16, std::min(rq.max_c, 1024)); }

// The widest chunk (a power of two of sieve points, from the preferred one down to 16)
// whose estimated bytes fit `cap`; 0 if none does.
int chunk_within(const tpm_server *s, const SReq &rq, int64_t cap) {
    const Graph &G = s->g->G;
    const bool loc = rq.want_path && rq.q.k >= 2;
    for (int C = std::min(preferred_chunk(rq.q.k), max_chunk(s, rq)); C >= 16; C >>= 1)
        if (est_request_bytes(G, rq.mk, rq.whole, rq.q.k, C, loc) <= cap) return C;
    return 0;
}

bool is_express(const tpm_server *s, int w) { return s->serial && w > 0; }

// Does the request fit worker 0's share of the budget (at some chunk size)?
bool fits_share(tpm_server *s, const SReq &rq) { return chunk_within(s, rq, s->share[0]) > 0; }

// Tries to admit `rq` on worker w.  Each worker owns a fixed share of the state budget,
// so a request sized to the share always fits beside the others and no worker ever
// waits for, or gives back, memory: it takes the widest chunk whose estimate fits the
// share.  An express worker takes only requests that fit its share at full width.  A
// request that does not fit a share at any chunk size runs only with every other
// worker idle, on whatever the others do not hold.  Caller holds s->mu.
bool admit_pruned(tpm_server *s, int w, SReq &rq) {
    const Graph &G = s->g->G;
    WorkerMem &me = s->wm[(size_t)w];
    const int64_t others = s->held - me.accounted;
    int C = chunk_within(s, rq, s->share[(size_t)w]);
    if (is_express(s, w) && C != std::min(preferred_chunk(rq.q.k), max_chunk(s, rq))) return false;
    if (C == 0) {
        for (size_t i = 0; i < s->wm.size(); ++i)
            if ((int)i != w && s->wm[i].busy) return false;
        C = chunk_within(s, rq, s->budget - others);
        if (C == 0) return false;
    }
    const bool loc = rq.want_path && rq.q.k >= 2;
    const int64_t est = est_request_bytes(G, rq.mk, rq.whole, rq.q.k, C, loc);
    const int64_t need = std::max(est, worker_bytes(me));
    if (others + need > s->budget) return false;
    rq.C = C;
    rq.est = est;
    s->held = others + need;
    me.accounted = need;
    s->held_peak = std::max(s->held_peak, s->held);
    return true;
}

// ------------------------------------------------------------------ device token
// Serial device use: dev_take blocks until worker w may use the device (an express
// worker waits while a loan is being returned; worker 0 lets waiting express workers go
// first); dev_give releases it (ending a loan); dev_lend, called by worker 0 between
// two levels of its sieve, lends it to a waiting express worker for one request and
// takes it back.
void dev_take(tpm_server *s, int w) {
    std::unique_lock<std::mutex> lk(s->dev_mu);
    const bool exp = is_express(s, w);
    if (exp) ++s->dev_exp_waiting;
    s->dev_cv.wait(lk, [&] {
        return s->stop || (s->dev_owner < 0 && (exp ? !s->dev_back : s->dev_exp_waiting == 0));
    });
    if (exp) --s->dev_exp_waiting;
    if (s->stop) throw Error{TPM_ECANCELLED, "server stopping"};
    s->dev_owner = w;
}

void dev_give(tpm_server *s) {
    std::lock_guard<std::mutex> lk(s->dev_mu);
    s->dev_owner = -1;
    if (s->dev_lent) {
        s->dev_lent = false;
        s->dev_back = true;
    }
    s->dev_cv.notify_all();
}

void dev_lend(tpm_server *s, int w, hipStream_t st) {
    {
        std::lock_guard<std::mutex> lk(s->dev_mu);
        if (s->dev_exp_waiting == 0) return;
    }
    // this worker's queued levels finish before the borrower's work starts
    TPM_HIP(hipStreamSynchronize(st));
    std::unique_lock<std::mutex> lk(s->dev_mu);
    s->dev_owner = -1;
    s->dev_lent = true;
    s->dev_cv.notify_all();
    s->dev_cv.wait(lk, [&] { return s->stop || (s->dev_owner < 0 && !s->dev_lent); });
    s->dev_back = false;
    s->dev_owner = w;
    if (s->stop) throw Error{TPM_ECANCELLED, "server stopping"};
}

// Holds the device for a scope (serial servers only).
struct DevHold {
    tpm_server *s;
    bool held = false;
    DevHold(tpm_server *srv, int w) : s(srv) {
        if (s->serial) {
            dev_take(s, w);
            held = true;
        }
    }
    void release() {
        if (held) dev_give(s);
        held = false;
    }
    ~DevHold() { release(); }
    DevHold(const DevHold &) = delete;
    DevHold &operator=(const DevHold &) = delete;
};

// Runs one request on worker w's stream; returns its result.
tpm_result run_pruned(tpm_server *s, int w, WorkerMem &wmem, SReq &rq, hipStream_t st) {
    const Graph &G = s->g->G;
    tpm_result r = status_result(TPM_OK);
    rq.q.multiset = rq.ms.data();
    const bool loc = rq.want_path && rq.q.k >= 2;
    SieveRequest req;
    req.multiset = rq.ms.data();
    req.k = rq.q.k;
    req.seed = rq.q.seed;
    req.chunk = rq.C;
    req.cancel = &rq.cancel;
    req.deadline_ms = rq.deadline;
    req.ws = wmem.ws;
    Graph P;
    struct Free {
        Graph &g;
        ~Free() {
            g.pool = nullptr;  // the server's
            free_graph(g);
        }
    } fr{P};
    const Graph *H = &G;
    const double t0 = now_ms();
    std::vector<uint8_t> qloc;
    double tg, t1, t2;
    {
        // serial servers use the device one request at a time: every device phase here
        // (subgraph build, sieve) is bound by HBM bandwidth, and two requests at once
        // measured slower than one after the other (two sieves at full serving size:
        // capacity 7.0 -> 5.2 queries/s; a subgraph build beside a sieve: 7.0 -> 6.1);
        // worker 0 lends the device between levels to the express workers' short requests
        DevHold dev(s, w);
        tg = now_ms();
        if (!rq.whole) {
            std::vector<uint8_t> keep((size_t)G.q, 0);
            for (int32_t c : rq.ms) keep[(size_t)c] = 1;
            PruneSpec spec;
            spec.keep_color = keep.data();
            spec.need_times = false;
            prune_graph(G, spec, P, wmem.arena, st);
            P.pool = s->ppool;
            H = &P;
        }
        t1 = now_ms();
        std::function<void(hipStream_t)> lend = [s, w](hipStream_t sst) { dev_lend(s, w, sst); };
        if (s->serial && w == 0) req.between_levels = &lend;
        if (loc) {
            qloc.resize((size_t)H->n);
            r.total = vertex_localise(*H, req, qloc.data(), st, &rq.pp);
        } else {
            SieveResult res;
            run_sieve(*H, req, res, st);
            r.total = res.total;
            rq.pp.swap(res.per_point);
        }
        t2 = now_ms();
    }
    r.found = r.total != 0;
    if (r.found && rq.want_path) {
        // the reverse DFS from the query's own localisation runs on the host; a fallback
        // that sieves again takes the device
        int64_t pe[16];
        int32_t pv[16];
        r.path_status = TPM_NOTFOUND;
        if (!qloc.empty())
            r.path_status = extract_from_vertices(*H, rq.ms.data(), rq.q.k, qloc.data(), kQuickDfsBudget, pv, pe);
        if (r.path_status == TPM_OK) {
            store_path_into(rq.q, pv, pe, r);
        } else {
            DevHold dev(s, w);
            extract_into(*H, rq.q, r, st, nullptr);
        }
    }
    const double t3 = now_ms();
    std::lock_guard<std::mutex> lk(s->mu);
    s->steps++;
    s->gpu_wait_ms += tg - t0;
    s->prune_ms += t1 - tg;
    s->sieve_ms += t2 - t1;
    s->extract_ms += t3 - t2;
    return r;
}

void pruned_worker(tpm_server *s, int w) {
    const Graph &G = s->g->G;
    (void)hipSetDevice(G.device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        record_error(s, "cannot create a worker stream");
        return;
    }
    WorkerMem &me = s->wm[(size_t)w];
    std::vector<ReqP> gone;
    for (;;) {
        ReqP rq;
        bool trim = false;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                if (s->stop) break;
                purge_queue(s, gone);
                if (!gone.empty()) break;  // results are produced outside the lock
                // admission: the oldest request; a request larger than one worker's
                // share waits for the device to itself, and later requests may overtake
                // it at most kMaxBypass times
                bool all_idle = true;
                for (auto &x : s->wm) all_idle &= !x.busy;
                const bool empty_dev = all_idle && s->held == me.accounted;
                // order: the oldest first if it has waited kAgeMs, else the least
                // device work first (short requests do not wait behind long ones; the
                // age bound keeps long ones from waiting behind a stream of short ones)
                std::vector<size_t> order(s->queue.size());
                for (size_t i = 0; i < order.size(); ++i) order[i] = i;
                const double tnow = now_ms();
                const bool aged = !s->queue.empty() && tnow - s->queue.front()->t_submit > kAgeMs;
                std::stable_sort(order.begin() + (aged ? 1 : 0), order.end(), [&](size_t a, size_t b) {
                    return s->queue[a]->cost < s->queue[b]->cost;
                });
                for (size_t oi = 0; oi < order.size(); ++oi) {
                    SReq &c = *s->queue[order[oi]];
                    const bool head = order[oi] == 0;
                    if (admit_pruned(s, w, c)) {
                        rq = s->queue[order[oi]];
                        s->queue.erase(s->queue.begin() + (std::ptrdiff_t)order[oi]);
                        break;
                    }
                    if (head && !fits_share(s, c)) {
                        // the oldest needs the device's memory to itself: later requests
                        // may overtake it kMaxBypass times, then nobody does
                        if (c.bypassed >= kMaxBypass) break;
                        ++c.bypassed;
                    }
                }
                if (rq) break;
                if (!s->queue.empty()) {
                    const bool big_head = !fits_share(s, *s->queue.front());
                    // the oldest needs more than a share: idle workers give their memory
                    // back; with every worker idle and nothing held, it never fits
                    if (big_head && !me.busy && worker_bytes(me) > 0 && !empty_dev) {
                        trim = true;
                        break;
                    }
                    // nothing fits an idle device for worker 0 (which takes any
                    // request): the oldest never will
                    if (empty_dev && !is_express(s, w)) {
                        gone.push_back(s->queue.front());
                        s->queue.pop_front();
                        break;
                    }
                }
                if (any_deadline(s)) s->cv.wait_for(lk, std::chrono::milliseconds(20));
                else s->cv.wait(lk);
            }
            if (s->stop && !rq) break;
            if (rq) {
                me.busy = true;
                s->inflight++;
                s->inflight_peak = std::max(s->inflight_peak, s->inflight);
            }
        }
        if (trim) {
            try {
                arena_trim(me.arena);
                workspace_trim(me.ws);
            } catch (const Error &e) {
                record_error(s, e.msg);
            }
            std::lock_guard<std::mutex> lk(s->mu);
            s->trims++;
            s->held -= me.accounted;
            me.accounted = 0;
            s->cv.notify_all();
            continue;
        }
        if (!gone.empty()) {
            // purged (cancelled / expired) requests, or a request that cannot fit
            for (auto &x : gone) {
                const bool never_fits = !expired(*x, now_ms());
                finish(s, *x, status_result(never_fits ? TPM_ENOMEM : TPM_ECANCELLED));
            }
            gone.clear();
            continue;
        }
        if (!rq) continue;
        rq->t_start = now_ms();
        tpm_result r;
        bool requeue = false;
        try {
            r = run_pruned(s, w, me, *rq, st);
        } catch (const Error &e) {
            (void)hipStreamSynchronize(st);
            r = status_result(e.code);
            if (e.code == TPM_ENOMEM && rq->tries++ == 0) requeue = true;  // retry once, alone
            if (e.code != TPM_ECANCELLED && e.code != TPM_ENOMEM) record_error(s, e.msg);
        } catch (const std::exception &e) {
            (void)hipStreamSynchronize(st);
            r = status_result(TPM_EDEVICE);
            record_error(s, e.what());
        }
        if (!requeue && worker_bytes(me) > s->share[(size_t)w]) {
            // after a request larger than a share: back to at most the share, so that an
            // idle worker never holds more than its share
            try {
                arena_trim(me.arena);
                workspace_trim(me.ws);
            } catch (const Error &e) {
                record_error(s, e.msg);
            }
            std::lock_guard<std::mutex> lk(s->mu);
            s->trims++;
        }
        const int64_t actual = worker_bytes(me);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            me.busy = false;
            s->inflight--;
            // the estimate is replaced by what the worker holds now
            s->held += actual - me.accounted;
            me.accounted = actual;
            s->held_peak = std::max(s->held_peak, s->held);
            if (requeue) {
                rq->bypassed = kMaxBypass;  // runs next, with half the chunk
                rq->max_c = std::max(16, rq->C / 2);
                s->queue.push_front(rq);
            }
            s->cv.notify_all();
        }
        if (requeue) {
            try {
                arena_trim(me.arena);
                workspace_trim(me.ws);
            } catch (const Error &) {
            }
            std::lock_guard<std::mutex> lk(s->mu);
            s->held -= me.accounted;
            me.accounted = 0;
            s->cv.notify_all();
            continue;
        }
        finish(s, *rq, r);
    }
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
}

// ------------------------------------------------------------------ row mode
struct Group {
    ReqP req;
    int lane0 = 0, nl = 0, gpts = 0, level = 2, chunk = 0;
};

// Extraction for a hit of the row engine: on the subgraph of the query's colours
// (built in the server's arena, same ids, so the same path certificate), or on the
// whole graph for queries with wildcards.
void extract_on_subgraph(tpm_server *s, const Graph &G, const tpm_query &q, tpm_result &r,
                         hipStream_t st) {
    bool wild = false;
    std::vector<uint8_t> keep((size_t)G.q, 0);
    for (int i = 0; i < q.k; ++i) {
        if (q.multiset[i] < 0) wild = true;
        else keep[(size_t)q.multiset[i]] = 1;
    }
    if (wild) {
        extract_into(G, q, r, st);
        return;
    }
    Graph P;
    struct Free {
        Graph &g;
        ~Free() {
            g.pool = nullptr;  // the server owns it
            free_graph(g);
        }
    } fr{P};
    PruneSpec spec;
    spec.keep_color = keep.data();
    spec.need_times = false;
    prune_graph(G, spec, P, s->arena, st);
    P.pool = s->ppool;
    extract_into(P, q, r, st);
}

// The extraction thread of the row engine: paths for hits, on its own stream.
void extraction_worker(tpm_server *s) {
    const Graph &G = s->g->G;
    (void)hipSetDevice(G.device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        record_error(s, "cannot create the extraction stream");
        return;
    }
    for (;;) {
        std::pair<ReqP, tpm_result> job;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->ext_cv.wait(lk, [&] { return s->stop || s->rows_done || !s->ext_queue.empty(); });
            if (s->ext_queue.empty()) break;  // stop, or the row loop ended with nothing left
            job = s->ext_queue.front();
            s->ext_queue.pop_front();
        }
        SReq &rq = *job.first;
        tpm_result &r = job.second;
        const double te = now_ms();
        try {
            if (rq.cancel.load()) {
                r = status_result(TPM_ECANCELLED);
            } else {
                rq.q.multiset = rq.ms.data();
                extract_on_subgraph(s, G, rq.q, r, st);
            }
        } catch (const Error &e) {
            (void)hipStreamSynchronize(st);
            r.path_status = TPM_NOTFOUND;
            if (e.code != TPM_ECANCELLED) record_error(s, e.msg);
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->extract_ms += now_ms() - te;
        }
        finish(s, rq, r);
    }
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
}

void row_loop(tpm_server *s) {
    const Graph &G = s->g->G;
    (void)hipSetDevice(G.device);
    hipStream_t st = nullptr;
    std::vector<ReqP> gone;
    try {
        TPM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        WorkspaceLease lease(G);
        MultiRow row;
        row.W = s->W;
        row.lanes = s->lanes;
        row.ws = lease.ws;
        multi_init(G, row, st);
        StepGraph sg;
        int rowpts = 1;  // largest power of two of points that fits the row
        while (rowpts * 2 <= row.rowb()) rowpts *= 2;
        std::vector<Group> groups;
        std::vector<char> used((size_t)row.lanes, 0);
        std::vector<uint8_t> rowbytes((size_t)row.rowb());
        auto alloc_lanes = [&](int nl) -> int {
            for (int a = 0; a + nl <= row.lanes; ++a) {
                bool ok = true;
                for (int t = a; t < a + nl && ok; ++t) ok = !used[(size_t)t];
                if (ok) {
                    for (int t = a; t < a + nl; ++t) used[(size_t)t] = 1;
                    return a;
                }
            }
            return -1;
        };
        auto free_lanes = [&](const Group &gr) {
            for (int t = gr.lane0; t < gr.lane0 + gr.nl; ++t) used[(size_t)t] = 0;
        };
        // a request whose chunks are all done: its result, or a path first
        auto complete = [&](const ReqP &rq) {
            tpm_result r = status_result(TPM_OK);
            r.total = rq->total;
            r.found = rq->total != 0;
            if (r.found && rq->want_path) {
                std::lock_guard<std::mutex> lk(s->mu);
                s->ext_queue.emplace_back(rq, r);
                s->ext_cv.notify_one();
                return;
            }
            finish(s, *rq, r);
        };
        for (;;) {
            std::vector<ReqP> alone;  // k = 1 or an edgeless graph: no levels to run
            std::vector<Group> fresh;
            {
                std::unique_lock<std::mutex> lk(s->mu);
                for (;;) {
                    purge_queue(s, gone);
                    if (s->stop || !groups.empty() || !s->queue.empty() || !gone.empty()) break;
                    if (any_deadline(s)) s->cv.wait_for(lk, std::chrono::milliseconds(20));
                    else s->cv.wait(lk);
                }
                if (s->stop) break;
                // ---- admission: waiting requests take free lanes (the chunks of a large
                // query in order); any request that fits, unless the oldest has been
                // overtaken kMaxBypass times
                for (auto it = s->queue.begin(); it != s->queue.end();) {
                    ReqP rq = *it;
                    const bool head = it == s->queue.begin();
                    if (rq->q.k == 1 || G.m == 0) {
                        alone.push_back(rq);
                        it = s->queue.erase(it);
                        continue;
                    }
                    const int pts = 1 << rq->q.k;
                    const int gpts = std::min(rowpts, group_points(rq->q.k, row.W));
                    const int nl = gpts / (4 * row.W);
                    bool admitted = false;
                    while (rq->next_chunk * gpts < pts) {
                        const int a = alloc_lanes(nl);
                        if (a < 0) break;
                        if (rq->t_start < 0) {
                            rq->t_start = now_ms();
                            rq->chunks_left = std::max(1, pts / gpts);
                            rq->pp.assign((size_t)pts, 0);
                            s->inflight++;
                            s->inflight_peak = std::max(s->inflight_peak, s->inflight);
                        }
                        Group gr;
                        gr.req = rq;
                        gr.lane0 = a;
                        gr.nl = nl;
                        gr.gpts = gpts;
                        gr.chunk = rq->next_chunk++;
                        rq->groups_live++;
                        fresh.push_back(gr);
                        admitted = true;
                    }
                    if (rq->next_chunk * gpts >= pts) {
                        it = s->queue.erase(it);
                        continue;
                    }
                    if (!admitted && head) {
                        if (rq->bypassed >= kMaxBypass) break;  // nobody overtakes it now
                        ++rq->bypassed;
                    }
                    ++it;
                }
            }
            finish_gone(s, gone);
            for (auto &rq : alone) {
                rq->t_start = now_ms();
                try {
                    SieveRequest req;
                    req.multiset = rq->ms.data();
                    req.k = rq->q.k;
                    req.seed = rq->q.seed;
                    SieveResult res;
                    run_sieve(G, req, res, st);
                    rq->pp.swap(res.per_point);
                    rq->total = res.total;
                    complete(rq);
                } catch (const Error &e) {
                    finish(s, *rq, status_result(e.code));
                }
            }
            // x rows and cleared accumulators of the groups that start now
            for (Group &gr : fresh) {
                multi_prepare(G, row, gr.lane0, gr.gpts, gr.req->ms.data(), gr.req->q.k,
                              gr.req->q.seed, (uint32_t)(gr.chunk * gr.gpts), nullptr, st);
                groups.push_back(gr);
            }
            // cancelled or expired requests leave the row before the step
            {
                const double now = now_ms();
                std::vector<Group> keep;
                std::vector<ReqP> ended;
                for (Group &gr : groups) {
                    if (!expired(*gr.req, now)) {
                        keep.push_back(gr);
                        continue;
                    }
                    free_lanes(gr);
                    if (--gr.req->groups_live == 0) ended.push_back(gr.req);
                }
                groups.swap(keep);
                for (auto &rq : ended) {
                    {
                        std::lock_guard<std::mutex> lk(s->mu);
                        // chunks not admitted yet are dropped with it
                        for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
                            if (*it == rq) {
                                s->queue.erase(it);
                                break;
                            }
                        s->inflight--;
                    }
                    finish(s, *rq, status_result(TPM_ECANCELLED));
                }
            }
            if (groups.empty()) continue;
            // ---- one step: every group advances one level
            std::vector<StepLane> lanes((size_t)64, StepLane{0, 0, 0, 0});
            for (const Group &gr : groups) {
                const int k = gr.req->q.k;
                const uint32_t flags = kLaneActive | (gr.level == 2 ? kLaneFromX : 0u) |
                                       (gr.level == k ? kLaneAcc : 0u);
                const uint64_t cm = colour_mask(G, gr.req->ms.data(), k);
                for (int t = 0; t < gr.nl; ++t)
                    lanes[(size_t)(gr.lane0 + t)] = {gr.req->q.seed, (uint32_t)(gr.level - 1), flags, cm};
            }
            const double ts = now_ms();
            if (s->use_graph) {
                multi_upload_tabs(row, lanes.data(), 1, st);
                multi_steps_graph(G, row, 1, sg, st);
            } else {
                multi_step(G, row, lanes.data(), st);
            }
            // ---- retire groups that ran their last level: one read of the row
            bool any_fin = false;
            for (const Group &gr : groups) any_fin |= gr.level == gr.req->q.k;
            if (any_fin) multi_read(G, row, 0, row.lanes, rowbytes.data(), st);
            std::vector<Group> keep;
            std::vector<ReqP> completed_now;
            for (Group &gr : groups) {
                if (gr.level == gr.req->q.k) {
                    SReq &rq = *gr.req;
                    const int pts = 1 << rq.q.k;
                    const uint8_t *src = rowbytes.data() + (size_t)gr.lane0 * 4 * row.W;
                    const int cnt = std::min(pts, gr.gpts);
                    std::memcpy(rq.pp.data() + (size_t)gr.chunk * gr.gpts, src, (size_t)cnt);
                    for (int b = 0; b < cnt; ++b) rq.total ^= src[b];
                    free_lanes(gr);
                    --rq.groups_live;
                    if (--rq.chunks_left == 0) completed_now.push_back(gr.req);
                } else {
                    gr.level++;
                    keep.push_back(gr);
                }
            }
            groups.swap(keep);
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->steps++;
                s->sieve_ms += now_ms() - ts;
                s->inflight -= (int)completed_now.size();
            }
            for (auto &rq : completed_now) complete(rq);
        }
    } catch (const Error &e) {
        record_error(s, e.msg);
    } catch (const std::exception &e) {
        record_error(s, e.what());
    }
    if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->rows_done = true;
    s->ext_cv.notify_all();
}

// ------------------------------------------------------------------ creation
void start_server(tpm_server *s, const tpm_graph *g, const tpm_server_config *cfg,
                  bool internal_batch) {
    s->g = g;
    if (cfg) s->cfg = *cfg;
    const Graph &G = g->G;
    TPM_REQUIRE(s->cfg.prune_queries == 0 || s->cfg.prune_queries == 1, "prune_queries must be 0 or 1");
    TPM_REQUIRE(s->cfg.streams >= 0 && s->cfg.streams <= kMaxStreams, "streams must be in [0, 4]");
    TPM_REQUIRE(s->cfg.state_bytes >= 0, "state_bytes must be >= 0");
    TPM_REQUIRE(s->cfg.max_lanes >= 0 && s->cfg.max_lanes <= 64, "max_lanes must be in [0, 64]");
    s->pruned = s->cfg.prune_queries != 0;
    DeviceGuard dg(G.device);
    // a batch borrows the graph's pools, so its memory stays with the graph across calls
    s->own_pools = !(internal_batch && G.pool && G.apool);
    s->ppool = s->own_pools ? new_workspace_pool() : G.pool;
    s->arena = new_graph_arena();
    size_t freeb = 0, totalb = 0;
    TPM_HIP(hipMemGetInfo(&freeb, &totalb));
    if (s->pruned) {
        // servers share the device serially (worker 0 and express workers); batches run
        // their queries on several streams at once
        s->serial = !internal_batch;
        s->nstreams = s->cfg.streams ? s->cfg.streams : (s->serial ? 2 : 3);
        if (G.q <= 64 && G.pcol) colour_pair_counts(G, s->pair_counts, nullptr);
        s->wm.resize((size_t)s->nstreams);
        int64_t held = 0;  // memory the borrowed worker buffers already hold
        for (int w = 0; w < s->nstreams; ++w) {
            WorkerMem &x = s->wm[(size_t)w];
            x.arena = s->own_pools ? new_graph_arena() : arena_take(G.apool);
            x.ws = s->own_pools ? new Workspace() : workspace_take(G.pool);
            x.accounted = worker_bytes(x);
            held += x.accounted;
        }
        s->held = held;
        s->budget = s->cfg.state_bytes > 0 ? s->cfg.state_bytes
                                           : (int64_t)(0.85 * (double)freeb) + held;
        s->share.assign((size_t)s->nstreams, s->budget / s->nstreams);
        if (s->serial && s->nstreams > 1) {
            // express workers: 5 % of the budget between them, worker 0 the rest
            const int64_t ex = (int64_t)(kExpressShare * (double)s->budget) / (s->nstreams - 1);
            for (int w = 1; w < s->nstreams; ++w) s->share[(size_t)w] = ex;
            s->share[0] = s->budget - ex * (s->nstreams - 1);
        }
        for (int w = 0; w < s->nstreams; ++w) s->threads.emplace_back(pruned_worker, s, w);
        return;
    }
    // row width: the widest of 1024 / 512 / 256 points whose two level buffers and
    // vertex rows fit the state budget (default: 85 % of free device memory)
    const double budget = s->cfg.state_bytes > 0 ? (double)s->cfg.state_bytes : 0.85 * (double)freeb;
    s->budget = (int64_t)budget;
    // bytes per lane-dword of a row: both level buffers, vertex rows, look-back words
    const double per_dword = (double)(2 * G.R + G.n + 2 * G.nslots) * 4.0;
    int W = 4;
    while (W > 1 && (per_dword * (64.0 * W) > budget || 256 * W > s->row_points_cap)) W >>= 1;
    // narrower rows (fewer lanes) when even one dword per lane does not fit
    const int fit = (int)std::min(64.0, std::floor(budget / per_dword));
    TPM_REQUIRE(fit >= 1, "not enough device memory for one serving lane");
    s->W = W;
    s->lanes = W > 1 ? 64 : fit;
    if (s->cfg.max_lanes > 0) s->lanes = std::min(s->lanes, s->cfg.max_lanes);
    s->threads.emplace_back(row_loop, s);
    s->threads.emplace_back(extraction_worker, s);
}

void stop_server(tpm_server *s) {
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->queue.clear();
    }
    s->cv.notify_all();
    s->ext_cv.notify_all();
    {
        std::lock_guard<std::mutex> lk(s->dev_mu);
        s->dev_cv.notify_all();
    }
    for (auto &t : s->threads)
        if (t.joinable()) t.join();
    (void)hipDeviceSynchronize();
    const Graph &G = s->g->G;
    for (auto &w : s->wm) {
        if (s->own_pools) {
            delete_graph_arena(w.arena);
            delete w.ws;
        } else {
            arena_give(G.apool, w.arena);
            workspace_give(G.pool, w.ws);
        }
    }
    s->wm.clear();
    if (s->own_pools) delete_workspace_pool(s->ppool);
    delete_graph_arena(s->arena);
    s->ppool = nullptr;
    s->arena = nullptr;
}

tpm_status submit(tpm_server *s, const tpm_query &q, uint64_t *ticket) {
    check_query(s->g->G, q);
    auto rq = std::make_shared<SReq>();
    rq->q = q;
    rq->ms.assign(q.multiset, q.multiset + q.k);
    rq->q.multiset = rq->ms.data();
    rq->user_pp = q.per_point;
    rq->t_submit = now_ms();
    rq->deadline = q.deadline_ms > 0 ? rq->t_submit + q.deadline_ms : 0;
    rq->want_path = q.want_path || s->cfg.extract_paths;
    if (s->pruned) {
        size_request(s, *rq);
        cost_request(s->g->G, *rq);
        // the smallest state this request can run with (16-point rows, no other request
        // holding memory) must fit the budget
        const int64_t least = est_request_bytes(s->g->G, rq->mk, rq->whole, rq->q.k,
                                                std::min(16, 1 << rq->q.k),
                                                rq->want_path && rq->q.k >= 2);
        if (least > s->budget) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->rejected++;
            throw Error{TPM_ENOMEM, "request cannot fit the server's state budget (needs about " +
                                        std::to_string(least) + " bytes, budget " +
                                        std::to_string(s->budget) + ")"};
        }
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return TPM_ECLOSED;
        if (!s->error.empty()) throw Error{TPM_EDEVICE, "server stopped: " + s->error};
        rq->ticket = s->next_ticket++;
        if (ticket) *ticket = rq->ticket;
        s->live[rq->ticket] = rq;
        s->queue.push_back(rq);
        s->queued_peak = std::max(s->queued_peak, (int)s->queue.size());
    }
    s->cv.notify_all();
    return TPM_OK;
}

}  // namespace

namespace tpm {

void batch_through_server(const tpm_graph *g, int32_t nq, const tpm_query *q, tpm_result *out,
                          bool pruned, int streams, int row_points, bool use_graph) {
    tpm_server s;
    tpm_server_config cfg{};
    cfg.prune_queries = pruned ? 1 : 0;
    cfg.streams = streams;
    s.use_graph = use_graph && !pruned;
    s.row_points_cap = row_points;
    start_server(&s, g, &cfg, true);
    struct Stop {
        tpm_server *s;
        ~Stop() { stop_server(s); }
    } stopper{&s};
    // largest first: long queries start early, short ones fill the gaps
    std::vector<int32_t> order((size_t)nq);
    for (int32_t i = 0; i < nq; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return q[a].k > q[b].k; });
    std::map<uint64_t, int32_t> slot;
    for (int32_t i : order) {
        tpm_query qq = q[i];
        qq.deadline_ms = 0;
        uint64_t t = 0;
        const tpm_status rc = submit(&s, qq, &t);
        if (rc != TPM_OK) throw Error{rc, "batch: submission failed"};
        slot[t] = i;
    }
    std::unique_lock<std::mutex> lk(s.mu);
    int32_t got = 0;
    while (got < nq) {
        s.cv_done.wait(lk, [&] { return !s.done.empty() || !s.error.empty(); });
        if (!s.error.empty()) throw Error{TPM_EDEVICE, "batch: " + s.error};
        while (!s.done.empty()) {
            tpm_result r = s.done.front();
            s.done.pop_front();
            const int32_t i = slot[r.ticket];
            if (r.status != TPM_OK)
                throw Error{r.status, "batch: query " + std::to_string(i) + " ended with status " +
                                          std::to_string(r.status)};
            r.ticket = 0;
            r.t_submit_ms = r.t_start_ms = r.t_done_ms = 0;
            out[i] = r;
            ++got;
        }
    }
}

}  // namespace tpm

extern "C" {

tpm_status tpm_server_create(const tpm_graph *g, const tpm_server_config *cfg, tpm_server **out) {
    return guarded_call([&]() -> tpm_status {
        TPM_REQUIRE(g && out, "NULL argument");
        *out = nullptr;
        std::unique_ptr<tpm_server> s(new tpm_server());
        start_server(s.get(), g, cfg, false);
        *out = s.release();
        return TPM_OK;
    });
}

tpm_status tpm_server_submit(tpm_server *s, const tpm_query *q, uint64_t *ticket) {
    return guarded_call([&]() -> tpm_status {
        TPM_REQUIRE(s && q, "NULL argument");
        return submit(s, *q, ticket);
    });
}

tpm_status tpm_server_poll(tpm_server *s, tpm_result *out, int32_t max, int32_t *n_out) {
    return guarded_call([&]() -> tpm_status {
        TPM_REQUIRE(s && n_out && (max == 0 || out), "NULL argument");
        TPM_REQUIRE(max >= 0, "max must be >= 0");
        std::lock_guard<std::mutex> lk(s->mu);
        int32_t n = 0;
        while (n < max && !s->done.empty()) {
            out[n++] = s->done.front();
            s->done.pop_front();
        }
        *n_out = n;
        if (n == 0 && !s->error.empty()) throw Error{TPM_EDEVICE, "server stopped: " + s->error};
        return n ? TPM_OK : TPM_PENDING;
    });
}

tpm_status tpm_server_cancel(tpm_server *s, uint64_t ticket) {
    return guarded_call([&]() -> tpm_status {
        TPM_REQUIRE(s, "NULL argument");
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->live.find(ticket);
        if (it == s->live.end()) return TPM_NOTFOUND;
        it->second->cancel.store(1);
        s->cv.notify_all();
        return TPM_OK;
    });
}

tpm_status tpm_server_stats_get(tpm_server *s, tpm_server_stats *out) {
    return guarded_call([&]() -> tpm_status {
        TPM_REQUIRE(s && out, "NULL argument");
        std::lock_guard<std::mutex> lk(s->mu);
        std::memset(out, 0, sizeof(*out));
        out->completed = s->completed;
        out->steps = (int64_t)s->steps;
        out->lanes = s->pruned ? 0 : s->lanes;
        int rp = 1;
        while (!s->pruned && rp * 2 <= 4 * s->W * s->lanes) rp *= 2;
        out->row_points = s->pruned ? 0 : rp;
        out->prune_ms = s->prune_ms;
        out->sieve_ms = s->sieve_ms;
        out->extract_ms = s->extract_ms;
        out->cancelled = s->cancelled;
        out->rejected = s->rejected;
        out->streams = s->pruned ? s->nstreams : 0;
        out->inflight_peak = s->inflight_peak;
        out->budget_bytes = s->budget;
        out->held_bytes_peak = s->held_peak;
        out->trims = s->trims;
        out->queued = (int32_t)s->queue.size();
        out->queued_peak = s->queued_peak;
        out->inflight = s->inflight;
        out->gpu_wait_ms = s->gpu_wait_ms;
        return TPM_OK;
    });
}

void tpm_server_destroy(tpm_server *s) {
    if (!s) return;
    stop_server(s);
    delete s;
}

}  // extern "C"
