// Batched queries (C ABI: tpm_batch_run) and RAINBOW-PATH as batches of colour sets.
//
// A batch runs through the serving engines of tpm_serve.hip with every query queued at
// once, largest first:
//   * packed: lane groups of any k share resident multi-query rows (tpm_sieve.hip:
//     k_step); each row step advances every group one level, and lanes freed by a
//     finished group are refilled at the next step from the queries still waiting;
//   * pruned (tpm_tuning.prune): each query alone on the subgraph of its colours, up
//     to tpm_tuning.streams at once on their own streams, within a memory budget.
// Results are bit-identical to the same query run alone: fingerprints depend only on
// (seed, tag, indices), never on lanes, steps or streams.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "tpm_internal.h"

using namespace tpm;

extern "C" {

tpm_status tpm_batch_run(const tpm_graph *g, int32_t nq, const tpm_query *q, tpm_result *out,
                         const tpm_tuning *tune) {
    return guarded_call([&]() -> tpm_status {
        TPM_REQUIRE(g && (nq == 0 || (q && out)), "NULL argument");
        TPM_REQUIRE(nq >= 0, "nq must be >= 0");
        const Graph &G = g->G;
        for (int32_t i = 0; i < nq; ++i) {
            TPM_REQUIRE(q[i].multiset != nullptr, "query multiset must not be NULL");
            TPM_REQUIRE(q[i].k >= 1 && q[i].k <= 16, "k must be in [1, 16]");
            for (int j = 0; j < q[i].k; ++j)
                TPM_REQUIRE(q[i].multiset[j] >= -1 && q[i].multiset[j] < G.q,
                            "multiset colour out of range");
        }
        for (int32_t i = 0; i < nq; ++i) std::memset(&out[i], 0, sizeof(tpm_result));
        const int row_points = (tune && tune->chunk) ? tune->chunk : 1024;
        TPM_REQUIRE(row_points >= 256 && row_points <= 1024 && (row_points & (row_points - 1)) == 0,
                    "batch row width (chunk) must be 256, 512 or 1024");
        TPM_REQUIRE(!tune || tune->use_graph == 0 || tune->use_graph == 1, "use_graph must be 0 or 1");
        TPM_REQUIRE(!tune || tune->prune == 0 || tune->prune == 1, "prune must be 0 or 1");
        TPM_REQUIRE(!tune || (tune->streams >= 0 && tune->streams <= 4), "streams must be in [0, 4]");
        if (nq == 0) return TPM_OK;
        DeviceGuard dg(G.device);
        const bool pruned = tune && tune->prune;
        batch_through_server(g, nq, q, out, pruned, tune ? tune->streams : 0, row_points,
                             tune && tune->use_graph);
        return TPM_OK;
    });
}

tpm_status tpm_rainbow_decide(const tpm_graph *g, int32_t k, uint64_t seed, int32_t reps,
                              int32_t *found, int32_t *colors) {
    return guarded_call([&]() -> tpm_status {
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
