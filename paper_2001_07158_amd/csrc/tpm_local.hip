// Localised outputs of the sieve (C ABI: tpm_sieve_vertex, tpm_time_buckets,
// tpm_optimum_time).
//
// The last level of the sieve can keep, per CSR position, the XOR over all sieve
// points of that edge's contribution: the per-edge localisation L[e], nonzero only if
// a matching temporal path ends with e (section "Vertex-localization", at edge
// granularity).  Two reductions of L are built here:
//   * by destination vertex: Q_u = XOR of L[e] over u's in-edges, which is the
//     vertex-localised sieve sum_A P_{u,k,t}(z^A);
//   * by timestamp: B(t) = XOR of L[e] over edges with timestamp t.  A walk's last
//     edge carries its largest time, so XOR_{t' <= t} B(t') is the sieve over walks
//     that finish by t, and the first t with B(t) != 0 is the smallest t whose
//     restricted sieve is nonzero: one localised pass replaces the binary search of
//     decide calls of section "Finding optimum timestamp".

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "tpm_internal.h"

namespace tpm {
namespace {

// Q_u: positions are grouped by destination, so runs of equal dst are contiguous
// inside a wave.  Each lane folds the rest of its run with doubling shuffles; the
// first lane of each run issues one atomic.
__global__ void k_vertex_xor(int64_t lo, int64_t hi, const uint8_t *loc, const int32_t *pdst,
                             uint32_t *q32) {
    const int64_t p = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    uint32_t v = 0;
    int32_t d = -1;
    if (p < hi) {
        v = loc[p - lo];
        d = pdst[p];
    }
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t vo = __shfl_down(v, off);
        const int32_t dn = __shfl_down(d, off);
        if (lane + off < 64 && dn == d) v ^= vo;
    }
    const int32_t dprev = __shfl_up(d, 1);
    const bool head = lane == 0 || dprev != d;
    if (head && d >= 0 && v != 0) atomicXor(&q32[d >> 2], v << (8 * (d & 3)));
}

// B(t): bucket = rank of the position's timestamp among the distinct timestamps.
__global__ void k_time_xor(int64_t lo, int64_t hi, const uint8_t *loc, const int32_t *ptau,
                           const int32_t *ttab, int64_t nt, uint32_t *b32) {
    const int64_t p = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= hi) return;
    const uint32_t v = loc[p - lo];
    if (v == 0) return;
    const int32_t t = ptau[p];
    int64_t a = 0, b = nt;
    while (a < b) {
        const int64_t mid = (a + b) >> 1;
        if (ttab[mid] < t) a = mid + 1;
        else b = mid;
    }
    if (a < nt && ttab[a] == t) atomicXor(&b32[a >> 2], v << (8 * (a & 3)));
}

__global__ void k_first_nonzero(int64_t nt, const uint8_t *b, unsigned long long *best) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nt && b[i]) atomicMin(best, (unsigned long long)i);
}

unsigned grid_of(int64_t work, int block = 256) {
    return (unsigned)std::max<int64_t>(1, (work + block - 1) / block);
}

struct VertexSink : LocSink {
    uint8_t *out = nullptr;  // host, n bytes
    void consume(const Graph &G, Workspace &ws, const uint8_t *dloc, int64_t lo, int64_t hi,
                 hipStream_t st) override {
        const size_t words = ((size_t)G.n + 3) / 4;
        ws.aux.alloc(words * 4, st);
        TPM_HIP(hipMemsetAsync(ws.aux.p, 0, words * 4, st));
        if (hi > lo)
            k_vertex_xor<<<grid_of(hi - lo), 256, 0, st>>>(lo, hi, dloc, G.pdst, ws.aux.as<uint32_t>());
        TPM_HIP(hipMemcpyAsync(out, ws.aux.p, (size_t)G.n, hipMemcpyDeviceToHost, st));
    }
};

struct TimeSink : LocSink {
    uint8_t *buckets = nullptr;  // host, ntimes bytes (nullable)
    unsigned long long first = ~0ull;
    void consume(const Graph &G, Workspace &ws, const uint8_t *dloc, int64_t lo, int64_t hi,
                 hipStream_t st) override {
        const int64_t nt = G.ntimes;
        const size_t words = ((size_t)std::max<int64_t>(nt, 1) + 3) / 4;
        ws.aux.alloc(words * 4, st);
        TPM_HIP(hipMemsetAsync(ws.aux.p, 0, words * 4, st));
        if (hi > lo && nt > 0)
            k_time_xor<<<grid_of(hi - lo), 256, 0, st>>>(lo, hi, dloc, G.ptau, G.ttab, nt,
                                                         ws.aux.as<uint32_t>());
        ws.aux2.alloc(sizeof(unsigned long long), st);
        TPM_HIP(hipMemsetAsync(ws.aux2.p, 0xFF, sizeof(unsigned long long), st));
        if (nt > 0)
            k_first_nonzero<<<grid_of(nt), 256, 0, st>>>(nt, ws.aux.as<uint8_t>(),
                                                          ws.aux2.as<unsigned long long>());
        TPM_HIP(hipMemcpyAsync(&first, ws.aux2.p, sizeof(first), hipMemcpyDeviceToHost, st));
        if (buckets && nt > 0)
            TPM_HIP(hipMemcpyAsync(buckets, ws.aux.p, (size_t)nt, hipMemcpyDeviceToHost, st));
    }
};

void check_k(int32_t k) { TPM_REQUIRE(k >= 2 && k <= 16, "k must be in [2, 16]"); }

__global__ void k_live(int32_t n, const int32_t *color, const uint8_t *keepc, uint8_t *live) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) live[u] = keepc[color[u]];
}

__global__ void k_or_nonzero(int32_t n, const uint8_t *s, uint8_t *keep) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n && s[u]) keep[u] = 1;
}

// live vertices of a multiset: a colour of it, or every vertex with a wildcard entry
void live_vertices(const Graph &G, const int32_t *M, int32_t k, uint8_t *live) {
    TPM_REQUIRE(M != nullptr, "multiset must not be NULL");
    TPM_REQUIRE(k >= 1 && k <= 16, "k must be in [1, 16]");
    std::vector<uint8_t> keepc((size_t)G.q, 0);
    bool wild = false;
    for (int i = 0; i < k; ++i) {
        TPM_REQUIRE(M[i] >= -1 && M[i] < G.q, "multiset colour out of range");
        if (M[i] < 0) wild = true;
        else keepc[(size_t)M[i]] = 1;
    }
    if (wild) std::fill(keepc.begin(), keepc.end(), (uint8_t)1);
    DBuf kc;
    kc.alloc(std::max<size_t>(1, keepc.size()), nullptr);
    TPM_HIP(hipMemcpy(kc.p, keepc.data(), keepc.size(), hipMemcpyHostToDevice));
    k_live<<<grid_of(G.n), 256>>>(G.n, G.color, kc.as<uint8_t>(), live);
    TPM_HIP(hipDeviceSynchronize());
}

// room for the static sieve's rows: half of the free device memory
size_t static_budget() {
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) return size_t(1) << 30;
    return freeb / 2;
}

struct StaticHolder {
    StaticGraph S;
    ~StaticHolder() { free_static(S); }
};

}  // namespace

int32_t optimum_time(const Graph &G, const int32_t *M, int32_t k, uint64_t seed, int32_t reps) {
    check_k(k);
    TPM_REQUIRE(reps >= 1, "reps must be >= 1");
    int32_t best = -1;
    for (int32_t r = 0; r < reps; ++r) {
        SieveRequest req;
        req.multiset = M;
        req.k = k;
        req.seed = seed + (uint64_t)r * 0x9E3779B97F4A7C15ull;
        SieveResult res;
        if (G.m == 0) {
            run_sieve(G, req, res, nullptr);
            continue;
        }
        TimeSink sink;
        run_sieve_sink(G, req, res, sink, nullptr);
        if (sink.first != ~0ull && (int64_t)sink.first < G.ntimes) {
            const int32_t t = G.h_ttab[(size_t)sink.first];
            if (best < 0 || t < best) best = t;
        }
    }
    return best;
}

uint8_t vertex_localise(const Graph &G, const SieveRequest &req, uint8_t *q, hipStream_t st,
                        std::vector<uint8_t> *per_point) {
    SieveResult res;
    if (G.m == 0) {
        std::memset(q, 0, (size_t)G.n);
        run_sieve(G, req, res, st);  // argument checks; the total of k = 1
    } else {
        VertexSink sink;
        sink.out = q;
        run_sieve_sink(G, req, res, sink, st);
    }
    if (per_point) per_point->swap(res.per_point);
    return res.total;
}

}  // namespace tpm

using namespace tpm;

extern "C" {

tpm_status tpm_sieve_vertex(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                            const uint8_t *vertex_mask, uint8_t *q) {
    return guarded_call([&]() -> tpm_status {
        TPM_REQUIRE(g && q, "NULL argument");
        check_k(k);
        DeviceGuard dg(g->G.device);
        SieveRequest req;
        req.multiset = multiset;
        req.k = k;
        req.seed = seed;
        req.vertex_mask = vertex_mask;
        vertex_localise(g->G, req, q, nullptr);
        return TPM_OK;
    });
}

tpm_status tpm_time_buckets(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                            int32_t *times, uint8_t *buckets) {
    return guarded_call([&]() -> tpm_status {
        TPM_REQUIRE(g && (g->G.ntimes == 0 || (times && buckets)), "NULL argument");
        check_k(k);
        DeviceGuard dg(g->G.device);
        const Graph &G = g->G;
        SieveRequest req;
        req.multiset = multiset;
        req.k = k;
        req.seed = seed;
        SieveResult res;
        if (G.m == 0) {
            run_sieve(G, req, res, nullptr);
            return TPM_OK;
        }
        TimeSink sink;
        sink.buckets = buckets;
        run_sieve_sink(G, req, res, sink, nullptr);
        std::memcpy(times, G.h_ttab.data(), sizeof(int32_t) * (size_t)G.ntimes);
        return TPM_OK;
    });
}

tpm_status tpm_optimum_time(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                            int32_t reps, int32_t *t_out) {
    return guarded_call([&]() -> tpm_status {
        TPM_REQUIRE(g && t_out, "NULL argument");
        DeviceGuard dg(g->G.device);
        *t_out = optimum_time(g->G, multiset, k, seed, reps);
        return TPM_OK;
    });
}

tpm_status tpm_static_sieve(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                            uint8_t *s) {
    return guarded_call([&]() -> tpm_status {
        TPM_REQUIRE(g && s, "NULL argument");
        DeviceGuard dg(g->G.device);
        const Graph &G = g->G;
        DBuf live, sv;
        live.alloc((size_t)std::max<int32_t>(1, G.n), nullptr);
        live_vertices(G, multiset, k, live.as<uint8_t>());
        StaticHolder h;
        if (k >= 2) build_static(G, live.as<uint8_t>(), h.S);
        sv.alloc((size_t)std::max<int32_t>(1, G.n), nullptr);
        TPM_HIP(hipMemset(sv.p, 0, (size_t)G.n));
        static_sieve(G, h.S, multiset, k, seed, sv.as<uint8_t>(), static_budget(), nullptr);
        TPM_HIP(hipMemcpy(s, sv.p, (size_t)G.n, hipMemcpyDeviceToHost));
        return TPM_OK;
    });
}

tpm_status tpm_graph_prune_static(const tpm_graph *g, const int32_t *multiset, int32_t k,
                                  uint64_t seed, int32_t reps, tpm_graph **out) {
    return guarded_call([&]() -> tpm_status {
        TPM_REQUIRE(g && out, "NULL argument");
        TPM_REQUIRE(reps >= 1, "reps must be >= 1");
        *out = nullptr;
        DeviceGuard dg(g->G.device);
        const Graph &G = g->G;
        DBuf live, sv, keep;
        live.alloc((size_t)std::max<int32_t>(1, G.n), nullptr);
        live_vertices(G, multiset, k, live.as<uint8_t>());
        sv.alloc((size_t)std::max<int32_t>(1, G.n), nullptr);
        keep.alloc((size_t)std::max<int32_t>(1, G.n), nullptr);
        TPM_HIP(hipMemset(keep.p, 0, (size_t)G.n));
        {
            StaticHolder h;
            if (k >= 2) build_static(G, live.as<uint8_t>(), h.S);
            for (int32_t r = 0; r < reps; ++r) {
                TPM_HIP(hipMemset(sv.p, 0, (size_t)G.n));
                static_sieve(G, h.S, multiset, k, seed + (uint64_t)r * 0x9E3779B97F4A7C15ull,
                             sv.as<uint8_t>(), static_budget(), nullptr);
                k_or_nonzero<<<grid_of(G.n), 256>>>(G.n, sv.as<uint8_t>(), keep.as<uint8_t>());
            }
            TPM_HIP(hipDeviceSynchronize());
        }
        auto *hnd = new tpm_graph();
        try {
            PruneSpec spec;
            spec.vkeep = keep.as<uint8_t>();
            prune_graph(G, spec, hnd->G);
            hnd->G.pool = new_workspace_pool();
            hnd->G.apool = new_arena_pool();
        } catch (...) {
            delete hnd;
            throw;
        }
        *out = hnd;
        return TPM_OK;
    });
}

}  // extern "C"
