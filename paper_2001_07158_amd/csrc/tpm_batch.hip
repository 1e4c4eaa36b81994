// Batched queries and the serving loop (C ABI: tpm_batch_run, tpm_server_*).
//
// First form: queries run one after another through the single-query path; the
// packed multi-query kernel replaces this loop.

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>

#include "tpm_internal.h"

namespace tpm {
tpm_status extract_path(const Graph &G, const int32_t *M, int32_t k, uint64_t seed,
                        int32_t max_reps, int32_t *path_vertices, int64_t *path_edges,
                        hipStream_t st);
}

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
    } catch (const std::exception &e) {
        set_error(e.what());
        return TPM_EDEVICE;
    }
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

void run_one(const Graph &G, const tpm_query &q, tpm_result &r, hipStream_t st) {
    SieveRequest req;
    req.multiset = q.multiset;
    req.k = q.k;
    req.seed = q.seed;
    SieveResult res;
    run_sieve(G, req, res, st);
    r.total = res.total;
    r.found = res.total != 0;
    r.path_status = 0;
    if (q.want_path && r.found) {
        int64_t pe[16];
        r.path_status = extract_path(G, q.multiset, q.k, q.seed, 8, r.path_vertices, pe, st);
        for (int i = 0; i + 1 < q.k; ++i) r.path_edges[i] = pe[i];
    }
}

}  // namespace

extern "C" {

tpm_status tpm_batch_run(const tpm_graph *g, int32_t nq, const tpm_query *q, tpm_result *out,
                         const tpm_tuning *tune) {
    return guarded2([&]() -> tpm_status {
        TPM_REQUIRE(g && (nq == 0 || (q && out)), "NULL argument");
        TPM_REQUIRE(nq >= 0, "nq must be >= 0");
        for (int32_t i = 0; i < nq; ++i) {
            std::memset(&out[i], 0, sizeof(tpm_result));
            run_one(g->G, q[i], out[i], nullptr);
        }
        return TPM_OK;
    });
}

struct tpm_server {
    const tpm_graph *g = nullptr;
    tpm_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv;
    struct Item {
        tpm_query q;
        std::vector<int32_t> ms;
        uint64_t ticket;
        double t_submit;
    };
    std::deque<Item> queue;
    std::deque<tpm_result> done;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
};

tpm_status tpm_server_create(const tpm_graph *g, const tpm_server_config *cfg, tpm_server **out) {
    return guarded2([&]() -> tpm_status {
        TPM_REQUIRE(g && out, "NULL argument");
        auto *s = new tpm_server();
        s->g = g;
        if (cfg) s->cfg = *cfg;
        s->worker = std::thread([s]() {
            int dev = s->g->G.device;
            (void)hipSetDevice(dev);
            for (;;) {
                tpm_server::Item it;
                {
                    std::unique_lock<std::mutex> lk(s->mu);
                    s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
                    if (s->queue.empty()) return;
                    it = std::move(s->queue.front());
                    s->queue.pop_front();
                }
                tpm_result r;
                std::memset(&r, 0, sizeof(r));
                r.ticket = it.ticket;
                r.t_submit_ms = it.t_submit;
                r.t_start_ms = now_ms();
                it.q.multiset = it.ms.data();
                it.q.want_path = it.q.want_path || s->cfg.extract_paths;
                try {
                    run_one(s->g->G, it.q, r, nullptr);
                } catch (const Error &e) {
                    r.path_status = e.code;
                }
                r.t_done_ms = now_ms();
                std::lock_guard<std::mutex> lk(s->mu);
                s->done.push_back(r);
            }
        });
        *out = s;
        return TPM_OK;
    });
}

tpm_status tpm_server_submit(tpm_server *s, const tpm_query *q, uint64_t *ticket) {
    return guarded2([&]() -> tpm_status {
        TPM_REQUIRE(s && q && q->multiset, "NULL argument");
        TPM_REQUIRE(q->k >= 1 && q->k <= 16, "k must be in [1, 16]");
        for (int i = 0; i < q->k; ++i)
            TPM_REQUIRE(q->multiset[i] >= 0 && q->multiset[i] < s->g->G.q, "multiset colour out of range");
        tpm_server::Item it;
        it.q = *q;
        it.ms.assign(q->multiset, q->multiset + q->k);
        it.t_submit = now_ms();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->stop) return TPM_ECLOSED;
            it.ticket = s->next_ticket++;
            if (ticket) *ticket = it.ticket;
            s->queue.push_back(std::move(it));
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
        return n ? TPM_OK : TPM_PENDING;
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
    delete s;
}

}  // extern "C"
