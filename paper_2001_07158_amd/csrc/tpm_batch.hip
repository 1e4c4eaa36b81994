// Batched queries and the serving loop (C ABI: tpm_batch_run, tpm_server_*).
//
// Both run on multi-query rows (tpm_sieve.hip: k_step): a row of up to 64 lanes holds
// lane groups, each a (query, chunk of sieve points) with its own seed and level.
//   * Batch: queries of equal k are packed side by side and advance level by level
//     together, so a small query no longer pays a whole sweep over the graph for a
//     handful of lanes.  Queries with 2^k >= 1024 points already fill a row and take
//     the single-query path.
//   * Server: the row stays resident; every step advances each group one level, a
//     group that finished its last level frees its lanes, and queued requests are
//     admitted into free lanes at the next step (continuous batching).  A request
//     whose sieve is nonzero can have its witness extracted.
// Results are bit-identical to the same query run alone: fingerprints depend only on
// (seed, tag, indices), never on lanes or steps.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "tpm_internal.h"


using namespace tpm;

namespace {

template <class F>
tpm_status guarded2(F &&f) {
    try {
        clear_error();
        return f();
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return TPM_ENOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return TPM_EDEVICE;
    }
}

struct OwnedStream {
    hipStream_t s = nullptr;
    OwnedStream() = default;
    OwnedStream(const OwnedStream &) = delete;
    OwnedStream &operator=(const OwnedStream &) = delete;
    ~OwnedStream() {
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    }
};

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

void check_query(const Graph &G, const tpm_query &q) {
    TPM_REQUIRE(q.multiset != nullptr, "query multiset must not be NULL");
    TPM_REQUIRE(q.k >= 1 && q.k <= 16, "k must be in [1, 16]");
    for (int i = 0; i < q.k; ++i)
        TPM_REQUIRE(q.multiset[i] >= -1 && q.multiset[i] < G.q, "multiset colour out of range");
}


void store_path(const tpm_query &q, const int32_t *pv, const int64_t *pe, tpm_result &r) {
    for (int i = 0; i < q.k; ++i) r.path_vertices[i] = pv[i];
    for (int i = 0; i + 1 < q.k; ++i) r.path_edges[i] = pe[i];
}

// Extraction on a hit: vertex localisation + reverse temporal DFS (one sieve), else
// the localisation-guided self-reduction.  q_loc (nullable): the query's own vertex
// localisation, already computed by the sieve that found the hit.
void extract_into(const Graph &G, const tpm_query &q, tpm_result &r, hipStream_t st,
                  const uint8_t *q_loc = nullptr) {
    int64_t pe[16];
    int32_t pv[16];
    r.path_status = TPM_NOTFOUND;
    if (q.k >= 2) {
        r.path_status = q_loc ? extract_from_vertices(G, q.multiset, q.k, q_loc, kQuickDfsBudget, pv, pe)
                              : extract_vertexloc(G, q.multiset, q.k, q.seed, 2, pv, pe, nullptr,
                                                  kQuickDfsBudget);
    }
    if (r.path_status != TPM_OK) r.path_status = extract_path(G, q.multiset, q.k, q.seed, 8, pv, pe, st);
    if (r.path_status == TPM_OK) store_path(q, pv, pe, r);
}

void run_alone(const Graph &G, const tpm_query &q, tpm_result &r, hipStream_t st) {
    SieveRequest req;
    req.multiset = q.multiset;
    req.k = q.k;
    req.seed = q.seed;
    SieveResult res;
    run_sieve(G, req, res, st);
    r.total = res.total;
    r.found = res.total != 0;
}

// lane-group geometry of a query of size k on rows with W dwords per lane
int group_points(int k, int W) {
    const int pts = 1 << k;
    const int unit = 4 * W;
    return std::max(pts, unit);  // padded to whole lanes; padded points are ignored
}

}  // namespace

extern "C" {

tpm_status tpm_batch_run(const tpm_graph *g, int32_t nq, const tpm_query *q, tpm_result *out,
                         const tpm_tuning *tune) {
    return guarded2([&]() -> tpm_status {
        TPM_REQUIRE(g && (nq == 0 || (q && out)), "NULL argument");
        TPM_REQUIRE(nq >= 0, "nq must be >= 0");
        const Graph &G = g->G;
        for (int32_t i = 0; i < nq; ++i) check_query(G, q[i]);
        for (int32_t i = 0; i < nq; ++i) std::memset(&out[i], 0, sizeof(tpm_result));
        const int max_pts = (tune && tune->chunk) ? tune->chunk : 1024;
        TPM_REQUIRE(max_pts >= 256 && max_pts <= 1024 && (max_pts & (max_pts - 1)) == 0,
                    "batch row width (chunk) must be 256, 512 or 1024");
        TPM_REQUIRE(!tune || tune->use_graph == 0 || tune->use_graph == 1, "use_graph must be 0 or 1");
        const bool use_graph = tune && tune->use_graph;
        // graph replay needs a created stream; everything of this call runs on it
        OwnedStream own;
        if (use_graph) TPM_HIP(hipStreamCreateWithFlags(&own.s, hipStreamNonBlocking));
        hipStream_t st = own.s;
        std::map<std::pair<int, int>, std::unique_ptr<StepGraph>> graphs;
        TPM_REQUIRE(!tune || tune->prune == 0 || tune->prune == 1, "prune must be 0 or 1");
        if (tune && tune->prune) {
            // each query alone on the subgraph of its colours, extraction there too
            struct Ctx {
                const tpm_query *q;
                tpm_result *r;
                const SieveResult *res;
                hipStream_t st;
            };
            for (int32_t i = 0; i < nq; ++i) {
                SieveRequest req;
                req.multiset = q[i].multiset;
                req.k = q[i].k;
                req.seed = q[i].seed;
                SieveResult res;
                Ctx ctx{&q[i], &out[i], &res, st};
                run_sieve_pruned(
                    G, req, res, nullptr, st,
                    [](const Graph &P, void *c) {
                        Ctx &x = *(Ctx *)c;
                        x.r->total = x.res->total;
                        x.r->found = x.res->total != 0;
                        if (x.q->want_path && x.r->found) extract_into(P, *x.q, *x.r, x.st);
                    },
                    &ctx);
            }
            return TPM_OK;
        }

        // queries that fill a row on their own, or k = 1, take the single-query path
        std::map<int, std::vector<int32_t>> by_k;
        for (int32_t i = 0; i < nq; ++i) {
            if (q[i].k == 1 || (1 << q[i].k) >= max_pts) {
                run_alone(G, q[i], out[i], st);
            } else {
                by_k[q[i].k].push_back(i);
            }
        }
        if (!by_k.empty() && G.m > 0) {
            WorkspaceLease lease(G);
            for (auto &kv : by_k) {
                const int k = kv.first;
                const auto &ids = kv.second;
                const int W = std::min(4, std::max(1, (1 << k) / 4));
                const int W_row = std::min(W, max_pts / 256);
                const int gpts = group_points(k, W_row);
                const int lpg = gpts / (4 * W_row);  // lanes per query
                const int per_pass = 64 / lpg;
                for (size_t a = 0; a < ids.size(); a += per_pass) {
                    const int cnt = (int)std::min<size_t>(per_pass, ids.size() - a);
                    MultiRow row;
                    row.W = W_row;
                    row.lanes = cnt * lpg;
                    row.ws = lease.ws;
                    multi_init(G, row, st);
                    for (int j = 0; j < cnt; ++j) {
                        const tpm_query &qq = q[ids[a + j]];
                        multi_prepare(G, row, j * lpg, gpts, qq.multiset, k, qq.seed, 0, nullptr, st);
                    }
                    // lane tables of levels 2..k, 64 entries per level
                    std::vector<StepLane> lanes((size_t)(k - 1) * 64, StepLane{0, 0, 0, 0});
                    for (int l = 2; l <= k; ++l) {
                        uint32_t flags = kLaneActive | (l == 2 ? kLaneFromX : 0u) | (l == k ? kLaneAcc : 0u);
                        for (int j = 0; j < cnt; ++j) {
                            const tpm_query &qq = q[ids[a + j]];
                            const uint64_t cm = colour_mask(G, qq.multiset, k);
                            for (int t = 0; t < lpg; ++t)
                                lanes[(size_t)(l - 2) * 64 + (size_t)(j * lpg + t)] = {
                                    qq.seed, (uint32_t)(l - 1), flags, cm};
                        }
                    }
                    if (use_graph) {
                        multi_upload_tabs(row, lanes.data(), k - 1, st);
                        auto &sg = graphs[{k, row.lanes}];
                        if (!sg) sg.reset(new StepGraph);
                        multi_steps_graph(G, row, k - 1, *sg, st);
                    } else {
                        for (int l = 2; l <= k; ++l)
                            multi_step(G, row, lanes.data() + (size_t)(l - 2) * 64, st);
                    }
                    std::vector<uint8_t> pp((size_t)row.rowb());
                    multi_read(G, row, 0, row.lanes, pp.data(), st);
                    for (int j = 0; j < cnt; ++j) {
                        uint8_t t = 0;
                        for (int b = 0; b < (1 << k); ++b) t ^= pp[(size_t)j * gpts + b];
                        out[ids[a + j]].total = t;
                        out[ids[a + j]].found = t != 0;
                    }
                }
            }
        }
        for (int32_t i = 0; i < nq; ++i)
            if (q[i].want_path && out[i].found) extract_into(G, q[i], out[i], st);
        return TPM_OK;
    });
}

tpm_status tpm_rainbow_decide(const tpm_graph *g, int32_t k, uint64_t seed, int32_t reps,
                              int32_t *found, int32_t *colors) {
    return guarded2([&]() -> tpm_status {
        TPM_REQUIRE(g && found && colors, "NULL argument");
        const int32_t q = g->G.q;
        TPM_REQUIRE(k >= 1 && k <= 16 && k <= q, "k must be in [1, min(16, num_colors)]");
        TPM_REQUIRE(reps >= 1, "reps must be >= 1");
        double sets = 1;
        for (int i = 0; i < k; ++i) sets = sets * (q - i) / (i + 1);
        TPM_REQUIRE(sets <= (double)(1 << 20), "too many colour sets");
        *found = 0;
        std::vector<int32_t> comb((size_t)k);
        for (int i = 0; i < k; ++i) comb[(size_t)i] = i;
        bool more = true;
        auto next_comb = [&]() {  // lexicographic successor of comb, false at the end
            int i = k - 1;
            while (i >= 0 && comb[(size_t)i] == q - k + i) --i;
            if (i < 0) return false;
            ++comb[(size_t)i];
            for (int j = i + 1; j < k; ++j) comb[(size_t)j] = comb[(size_t)j - 1] + 1;
            return true;
        };
        while (more) {
            // one batch: up to 256 (set, repetition) queries
            std::vector<std::vector<int32_t>> sets_b;
            while (more && (int)sets_b.size() * reps < 256) {
                sets_b.push_back(comb);
                more = next_comb();
            }
            std::vector<tpm_query> qs;
            for (size_t i = 0; i < sets_b.size(); ++i)
                for (int32_t r = 0; r < reps; ++r) {
                    tpm_query q1{};
                    q1.multiset = sets_b[i].data();
                    q1.k = k;
                    q1.seed = seed + (uint64_t)r * 0x9E3779B97F4A7C15ull;
                    qs.push_back(q1);
                }
            std::vector<tpm_result> out(qs.size());
            const tpm_status rc = tpm_batch_run(g, (int32_t)qs.size(), qs.data(), out.data(), nullptr);
            if (rc != TPM_OK) return rc;
            for (size_t i = 0; i < qs.size(); ++i)
                if (out[i].found) {
                    *found = 1;
                    const auto &set = sets_b[i / (size_t)reps];
                    for (int j = 0; j < k; ++j) colors[j] = set[(size_t)j];
                    return TPM_OK;
                }
        }
        return TPM_OK;
    });
}

}  // extern "C"

// ------------------------------------------------------------------ serving loop
struct tpm_server {
    const tpm_graph *g = nullptr;
    tpm_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv;
    struct Req {
        tpm_query q;
        std::vector<int32_t> ms;
        uint64_t ticket = 0;
        double t_submit = 0, t_start = -1;
        int chunks_left = 0;     // chunks not yet finished
        int next_chunk = 0;      // next chunk to admit
        uint8_t total = 0;
    };
    std::deque<std::shared_ptr<Req>> queue;
    std::deque<tpm_result> done;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::string error;
    std::thread worker;
    // row geometry
    int W = 1, lanes = 64;
    uint64_t steps = 0;
    int64_t completed = 0;
    double prune_ms = 0, sieve_ms = 0, extract_ms = 0;
    // pruned mode: workspaces and index memory shared by the per-request subgraphs
    WorkspacePool *ppool = nullptr;
    GraphArena *arena = nullptr;
};

namespace {

struct Group {
    std::shared_ptr<tpm_server::Req> req;
    int lane0 = 0, nl = 0, gpts = 0, level = 2, chunk = 0;
};

// Pruned mode: requests in arrival order, each on the subgraph of its own colours
// (preprocessing step (i)); the subgraph's workspaces come from a pool kept for the
// server's lifetime, so steady state allocates nothing but the subgraph index.
// Extraction for a hit of the batching server: on the subgraph of the query's colours
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
    prune_graph(G, spec, P, s->arena);
    P.pool = s->ppool;
    extract_into(P, q, r, st);
}

void serve_pruned(tpm_server *s) {
    const Graph &G = s->g->G;
    (void)hipSetDevice(G.device);
    hipStream_t st = nullptr;
    try {
        for (;;) {
            std::shared_ptr<tpm_server::Req> rq;
            {
                std::unique_lock<std::mutex> lk(s->mu);
                s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
                if (s->stop) return;
                rq = s->queue.front();
                s->queue.pop_front();
            }
            rq->t_start = now_ms();
            rq->q.multiset = rq->ms.data();
            tpm_result r;
            std::memset(&r, 0, sizeof(r));
            std::vector<uint8_t> keep((size_t)G.q, 0);
            bool wild = false;
            for (int32_t c : rq->ms) {
                if (c < 0) wild = true;
                else keep[(size_t)c] = 1;
            }
            if (wild) std::fill(keep.begin(), keep.end(), (uint8_t)1);  // any vertex may match
            Graph P;
            struct Free {
                Graph &g;
                ~Free() {
                    g.pool = nullptr;  // the server owns it
                    free_graph(g);
                }
            } fr{P};
            const double t0 = now_ms();
            PruneSpec spec;
            spec.keep_color = keep.data();
            prune_graph(G, spec, P, s->arena);
            P.pool = s->ppool;
            const double t1 = now_ms();
            const bool want = rq->q.want_path || s->cfg.extract_paths;
            std::vector<uint8_t> qloc;
            if (want && rq->q.k >= 2) {
                // the sieve with vertex localisation: the total, and the end vertices
                // the extraction's DFS starts from
                qloc.resize((size_t)P.n);
                SieveRequest req;
                req.multiset = rq->q.multiset;
                req.k = rq->q.k;
                req.seed = rq->q.seed;
                r.total = vertex_localise(P, req, qloc.data(), st);
                r.found = r.total != 0;
            } else {
                run_alone(P, rq->q, r, st);
            }
            const double t2 = now_ms();
            if (r.found && want) extract_into(P, rq->q, r, st, qloc.empty() ? nullptr : qloc.data());
            const double t3 = now_ms();
            r.ticket = rq->ticket;
            r.t_submit_ms = rq->t_submit;
            r.t_start_ms = rq->t_start;
            r.t_done_ms = t3;
            std::lock_guard<std::mutex> lk(s->mu);
            s->done.push_back(r);
            s->steps++;
            s->completed++;
            s->prune_ms += t1 - t0;
            s->sieve_ms += t2 - t1;
            s->extract_ms += t3 - t2;
        }
    } catch (const Error &e) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->error = e.msg;
    } catch (const std::exception &e) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->error = e.what();
    }
}

void serve_loop(tpm_server *s) {
    const Graph &G = s->g->G;
    (void)hipSetDevice(G.device);
    hipStream_t st = nullptr;
    try {
        WorkspaceLease lease(G);
        MultiRow row;
        row.W = s->W;
        row.lanes = s->lanes;
        row.ws = lease.ws;
        multi_init(G, row, st);
        int rowpts = 1;  // largest power of two of points that fits the row
        while (rowpts * 2 <= row.rowb()) rowpts *= 2;
        std::vector<Group> groups;
        std::vector<char> used((size_t)row.lanes, 0);
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
        double ext_in_step = 0;
        auto finish = [&](const std::shared_ptr<tpm_server::Req> &rq) {
            tpm_result r;
            std::memset(&r, 0, sizeof(r));
            r.ticket = rq->ticket;
            r.total = rq->total;
            r.found = rq->total != 0;
            r.t_submit_ms = rq->t_submit;
            r.t_start_ms = rq->t_start;
            rq->q.multiset = rq->ms.data();
            const double te = now_ms();
            if (r.found && (rq->q.want_path || s->cfg.extract_paths))
                extract_on_subgraph(s, G, rq->q, r, st);
            r.t_done_ms = now_ms();
            ext_in_step += r.t_done_ms - te;
            std::lock_guard<std::mutex> lk(s->mu);
            s->done.push_back(r);
            s->completed++;
            s->extract_ms += r.t_done_ms - te;
        };
        for (;;) {
            // ---- admission: requests enter free lanes (chunks of large queries in order)
            {
                std::unique_lock<std::mutex> lk(s->mu);
                if (groups.empty())
                    s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
                if (s->stop) return;
            }
            for (;;) {
                std::shared_ptr<tpm_server::Req> rq;
                {
                    std::lock_guard<std::mutex> lk(s->mu);
                    if (s->queue.empty()) break;
                    rq = s->queue.front();
                }
                if (rq->q.k == 1 || G.m == 0) {  // no levels to run: single-query path
                    {
                        std::lock_guard<std::mutex> lk(s->mu);
                        s->queue.pop_front();
                    }
                    rq->t_start = now_ms();
                    tpm_result r0;
                    std::memset(&r0, 0, sizeof(r0));
                    rq->q.multiset = rq->ms.data();
                    run_alone(G, rq->q, r0, st);
                    rq->total = r0.total;
                    finish(rq);
                    continue;
                }
                const int pts = 1 << rq->q.k;
                const int gpts = std::min(rowpts, group_points(rq->q.k, row.W));
                const int nl = gpts / (4 * row.W);
                const int a = alloc_lanes(nl);
                if (a < 0) break;  // row full: wait for lanes to free up
                if (rq->t_start < 0) {
                    rq->t_start = now_ms();
                    rq->chunks_left = std::max(1, pts / gpts);
                }
                Group gr;
                gr.req = rq;
                gr.lane0 = a;
                gr.nl = nl;
                gr.gpts = gpts;
                gr.chunk = rq->next_chunk++;
                multi_prepare(G, row, a, gpts, rq->ms.data(), rq->q.k, rq->q.seed,
                              (uint32_t)(gr.chunk * gpts), nullptr, st);
                groups.push_back(gr);
                if (rq->next_chunk * gpts >= pts) {
                    std::lock_guard<std::mutex> lk(s->mu);
                    s->queue.pop_front();
                }
            }
            if (groups.empty()) continue;
            // ---- one step: every group advances one level
            std::vector<StepLane> lanes((size_t)row.lanes, StepLane{0, 0, 0, 0});
            for (const Group &gr : groups) {
                const int k = gr.req->q.k;
                uint32_t flags = kLaneActive | (gr.level == 2 ? kLaneFromX : 0u) |
                                 (gr.level == k ? kLaneAcc : 0u);
                const uint64_t cm = colour_mask(G, gr.req->ms.data(), k);
                for (int t = 0; t < gr.nl; ++t)
                    lanes[(size_t)(gr.lane0 + t)] = {gr.req->q.seed, (uint32_t)(gr.level - 1), flags, cm};
            }
            const double ts = now_ms();
            ext_in_step = 0;
            multi_step(G, row, lanes.data(), st);
            s->steps++;
            // ---- retire groups that ran their last level
            std::vector<Group> keep;
            for (Group &gr : groups) {
                if (gr.level == gr.req->q.k) {
                    std::vector<uint8_t> pp((size_t)gr.gpts);
                    multi_read(G, row, gr.lane0, gr.nl, pp.data(), st);
                    const int pts = 1 << gr.req->q.k;
                    for (int b = 0; b < std::min(pts, gr.gpts); ++b) gr.req->total ^= pp[(size_t)b];
                    for (int t = gr.lane0; t < gr.lane0 + gr.nl; ++t) used[(size_t)t] = 0;
                    if (--gr.req->chunks_left == 0) finish(gr.req);
                } else {
                    gr.level++;
                    keep.push_back(gr);
                }
            }
            groups.swap(keep);
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->sieve_ms += now_ms() - ts - ext_in_step;
            }
        }
    } catch (const Error &e) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->error = e.msg;
    } catch (const std::exception &e) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->error = e.what();
    }
}

}  // namespace

extern "C" {

tpm_status tpm_server_create(const tpm_graph *g, const tpm_server_config *cfg, tpm_server **out) {
    return guarded2([&]() -> tpm_status {
        TPM_REQUIRE(g && out, "NULL argument");
        *out = nullptr;
        auto *s = new tpm_server();
        s->g = g;
        if (cfg) s->cfg = *cfg;
        const Graph &G = g->G;
        TPM_REQUIRE(s->cfg.prune_queries == 0 || s->cfg.prune_queries == 1,
                    "prune_queries must be 0 or 1");
        // per-request subgraphs (pruned mode, and extraction in batching mode) live in
        // an arena with their own workspace pool
        s->ppool = new_workspace_pool();
        s->arena = new_graph_arena();
        if (s->cfg.prune_queries) {
            s->worker = std::thread(serve_pruned, s);
            *out = s;
            return TPM_OK;
        }
        // row width: the widest of 1024 / 512 / 256 points whose two level buffers and
        // vertex rows fit the state budget (default: 70 % of free device memory)
        size_t freeb = 0, totalb = 0;
        TPM_HIP(hipMemGetInfo(&freeb, &totalb));
        double budget = s->cfg.state_bytes > 0 ? (double)s->cfg.state_bytes : 0.7 * (double)freeb;
        // bytes per lane-dword of a row: both level buffers, vertex rows, look-back words
        const double per_dword = (double)(2 * G.R + G.n + 2 * G.nslots) * 4.0;
        int W = 4;
        while (W > 1 && per_dword * (64.0 * W) > budget) W >>= 1;
        // narrower rows (fewer lanes) when even one dword per lane does not fit
        const int fit = (int)std::min(64.0, std::floor(budget / per_dword));
        TPM_REQUIRE(fit >= 1, "not enough device memory for one serving lane");
        s->W = W;
        s->lanes = W > 1 ? 64 : fit;
        if (s->cfg.max_lanes > 0) s->lanes = std::min(s->lanes, s->cfg.max_lanes);
        s->worker = std::thread(serve_loop, s);
        *out = s;
        return TPM_OK;
    });
}

tpm_status tpm_server_submit(tpm_server *s, const tpm_query *q, uint64_t *ticket) {
    return guarded2([&]() -> tpm_status {
        TPM_REQUIRE(s && q, "NULL argument");
        check_query(s->g->G, *q);
        auto rq = std::make_shared<tpm_server::Req>();
        rq->q = *q;
        rq->ms.assign(q->multiset, q->multiset + q->k);
        rq->t_submit = now_ms();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->stop) return TPM_ECLOSED;
            if (!s->error.empty()) throw Error{TPM_EDEVICE, "server stopped: " + s->error};
            rq->ticket = s->next_ticket++;
            if (ticket) *ticket = rq->ticket;
            s->queue.push_back(rq);
        }
        s->cv.notify_one();
        return TPM_OK;
    });
}

tpm_status tpm_server_poll(tpm_server *s, tpm_result *out, int32_t max, int32_t *n_out) {
    return guarded2([&]() -> tpm_status {
        TPM_REQUIRE(s && n_out && (max == 0 || out), "NULL argument");
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

tpm_status tpm_server_stats_get(tpm_server *s, tpm_server_stats *out) {
    return guarded2([&]() -> tpm_status {
        TPM_REQUIRE(s && out, "NULL argument");
        std::lock_guard<std::mutex> lk(s->mu);
        out->completed = s->completed;
        out->steps = (int64_t)s->steps;
        const bool pruned = s->cfg.prune_queries != 0;
        out->lanes = pruned ? 0 : s->lanes;
        int rp = 1;
        while (!pruned && rp * 2 <= 4 * s->W * s->lanes) rp *= 2;
        out->row_points = pruned ? 0 : rp;
        out->prune_ms = s->prune_ms;
        out->sieve_ms = s->sieve_ms;
        out->extract_ms = s->extract_ms;
        return TPM_OK;
    });
}

void tpm_server_destroy(tpm_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->queue.clear();
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (s->ppool) {
        (void)hipDeviceSynchronize();
        delete_workspace_pool(s->ppool);
        delete_graph_arena(s->arena);
    }
    delete s;
}

}  // extern "C"
