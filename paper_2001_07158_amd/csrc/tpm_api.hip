// C ABI entry points (include/tpm.h): argument checks, error reporting, decide and
// extraction by self-reduction.  No exception crosses the ABI.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <unordered_map>

#include "tpm_internal.h"

namespace tpm {

namespace {
thread_local std::string t_last_error;
template <class F>
tpm_status guarded(F &&f) {
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
    } catch (...) {
        set_error("unknown error");
        return TPM_EDEVICE;
    }
}

struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) TPM_HIP(hipSetDevice(dev));
        else prev = -1;
    }
    ~DeviceScope() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

uint64_t rep_seed(uint64_t seed, int64_t r) { return seed + (uint64_t)r * kGamma; }

// seeds of extraction step s (s = 0 is the first localised sieve), attempt r
uint64_t step_seed(uint64_t seed, int64_t s, int64_t r) {
    return seed + (uint64_t)(s * 1000003 + r) * kGamma;
}

}  // namespace

// ------------------------------------------------------------------ profiling
namespace {
std::atomic<int> g_profile{0};
std::mutex g_prof_mu;
std::vector<tpm_kernel_time> g_prof_done;
struct Pending {
    hipEvent_t a, b;
    int kind, level, chunk;
};
thread_local std::vector<Pending> t_pending;
}  // namespace

bool profile_on() { return g_profile.load() != 0; }

ProfileScope::ProfileScope(hipStream_t st, int kind_, int level_, int chunk_)
    : s(st), kind(kind_), level(level_), chunk(chunk_) {
    if (!profile_on()) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        a = b = nullptr;
        return;
    }
    (void)hipEventRecord(a, s);
}

ProfileScope::~ProfileScope() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    t_pending.push_back({a, b, kind, level, chunk});
}

void profile_collect() {
    if (t_pending.empty()) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &p : t_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess)
            g_prof_done.push_back({p.kind, p.level, p.chunk, 0, (double)ms});
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    t_pending.clear();
}

// ------------------------------------------------------------------ workspaces
struct WorkspacePool {
    std::mutex mu;
    std::vector<Workspace *> all, free_list;
    ~WorkspacePool() {
        for (Workspace *w : all) delete w;
    }
};

// Growth takes 1/8 more than asked when the device has it: a buffer of tens of GB costs
// about a second to allocate (measured: 62 GB in 0.7-1.8 s), and requests of a stream
// ask for sizes a few percent apart, so exact growth reallocated the largest buffers
// again and again.  Buffers sized to a budget (the row engine's) ask for `exact`: with
// the extra eighth they crowded out the memory the budget leaves to other work.
void DBuf::alloc(size_t bytes, hipStream_t st, bool exact) {
    bytes = std::max<size_t>(bytes, 16);
    if (bytes <= cap) return;
    if (p) {
        TPM_HIP(hipStreamSynchronize(st));
        (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    if (!exact) {
        const size_t roomy = bytes + bytes / 8;
        if (hipMalloc(&p, roomy) == hipSuccess) {
            cap = roomy;
            return;
        }
        (void)hipGetLastError();  // clears the failed attempt
        p = nullptr;
    }
    TPM_HIP(hipMalloc(&p, bytes));
    cap = bytes;
}

DBuf::~DBuf() {
    if (p) (void)hipFree(p);
}

WorkspaceLease::WorkspaceLease(const Graph &G) : pool(G.pool), ws(nullptr) {
    std::lock_guard<std::mutex> lk(pool->mu);
    if (!pool->free_list.empty()) {
        ws = pool->free_list.back();
        pool->free_list.pop_back();
    } else {
        ws = new Workspace();
        pool->all.push_back(ws);
    }
}

WorkspaceLease::~WorkspaceLease() {
    std::lock_guard<std::mutex> lk(pool->mu);
    pool->free_list.push_back(ws);
}

int64_t workspace_bytes(const Workspace *w) {
    if (!w) return 0;
    int64_t b = 0;
    for (const DBuf *d : {&w->ctl, &w->z, &w->xt, &w->s0, &w->s1, &w->pub, &w->pp, &w->tot,
                          &w->mask, &w->loc, &w->pick, &w->tabs, &w->aux, &w->aux2, &w->w2})
        b += (int64_t)d->cap;
    return b;
}

void workspace_trim(Workspace *w) {
    if (!w || workspace_bytes(w) == 0) return;
    TPM_HIP(hipDeviceSynchronize());
    for (DBuf *d : {&w->ctl, &w->z, &w->xt, &w->s0, &w->s1, &w->pub, &w->pp, &w->tot, &w->mask,
                    &w->loc, &w->pick, &w->tabs, &w->aux, &w->aux2, &w->w2}) {
        if (d->p) (void)hipFree(d->p);
        d->p = nullptr;
        d->cap = 0;
    }
}

Workspace *workspace_take(WorkspacePool *p) {
    std::lock_guard<std::mutex> lk(p->mu);
    if (!p->free_list.empty()) {
        Workspace *w = p->free_list.back();
        p->free_list.pop_back();
        return w;
    }
    Workspace *w = new Workspace();
    p->all.push_back(w);
    return w;
}

void workspace_give(WorkspacePool *p, Workspace *w) {
    std::lock_guard<std::mutex> lk(p->mu);
    p->free_list.push_back(w);
}

WorkspacePool *new_workspace_pool() { return new WorkspacePool(); }
void delete_workspace_pool(WorkspacePool *p) { delete p; }

void set_error(const std::string &msg) { t_last_error = msg; }
void clear_error() { t_last_error.clear(); }

// Verify a path using the device index (consecutive endpoints, distinct vertices,
// colours = M, and each edge leaving after the previous one arrived plus the
// vertex's delay: strictly increasing times in the plain problem).
bool verify_path(const Graph &G, const int32_t *M, int32_t k, const int32_t *verts,
                 const int64_t *edges_pos) {
    std::set<int32_t> seen;  // original vertices (layer copies of one vertex are one)
    std::map<int32_t, int32_t> have;
    for (int i = 0; i < k; ++i) {
        if (verts[i] < 0 || verts[i] >= G.n) return false;
        const int32_t orig = G.h_fid.empty() ? verts[i] : G.h_fid[(size_t)verts[i]];
        if (!seen.insert(orig).second) return false;
        have[G.h_color()[verts[i]]]++;
    }
    // colours = M, where a wildcard entry (-1) may be taken by any vertex
    for (int i = 0; i < k; ++i)
        if (M[i] >= 0 && --have[M[i]] < 0) return false;
    int64_t prev_arr = 0;
    for (int i = 0; i + 1 < k; ++i) {
        int32_t s, d, a, t;
        int64_t p = edges_pos[i];
        if (p < 0 || p >= G.m) return false;
        TPM_HIP(hipMemcpy(&s, G.psrc + p, 4, hipMemcpyDeviceToHost));
        TPM_HIP(hipMemcpy(&d, G.pdst + p, 4, hipMemcpyDeviceToHost));
        TPM_HIP(hipMemcpy(&a, G.ptau + p, 4, hipMemcpyDeviceToHost));
        t = a;
        if (G.pdep) TPM_HIP(hipMemcpy(&t, G.pdep + p, 4, hipMemcpyDeviceToHost));
        if (s != verts[i] || d != verts[i + 1]) return false;
        const int64_t dl = G.h_delay.empty() ? 1 : G.h_delay[(size_t)s];
        if (i > 0 && !(prev_arr <= (int64_t)t - dl)) return false;
        prev_arr = a;
    }
    return true;
}

// Self-reduction by per-edge localisation.  A nonzero localisation at position p
// (edge v -> u at time tau) certifies a matching path ending with that edge, hence a
// path ending at v before tau with colours M - {c(u)} that avoids u.  Each step sieves
// the smaller problem on the graph with the suffix's vertices deleted, counting only
// v's in-edges earlier than tau at the last level.  A zero answer can be a false
// negative, so each step retries with fresh seeds.
tpm_status extract_path(const Graph &G, const int32_t *M, int32_t k, uint64_t seed,
                        int32_t max_reps, int32_t *path_vertices, int64_t *path_edges,
                        hipStream_t st, int64_t *sieves) {
    int64_t nsieve = 0;
    struct Count {
        int64_t *out;
        int64_t &n;
        ~Count() {
            if (out) *out = n;
        }
    } count{sieves, nsieve};
    TPM_REQUIRE(k >= 1 && k <= 16, "k must be in [1, 16]");
    TPM_REQUIRE(max_reps >= 1, "max_reps must be >= 1");
    for (int i = 0; i < k; ++i) TPM_REQUIRE(M[i] >= -1 && M[i] < G.q, "multiset colour out of range");
    auto orig = [&](int32_t u) { return G.h_fid.empty() ? u : G.h_fid[(size_t)u]; };
    if (k == 1) {
        for (int32_t u = 0; u < G.n; ++u)
            if (G.h_color()[u] == M[0] || M[0] == -1) {
                path_vertices[0] = orig(u);
                return TPM_OK;
            }
        return TPM_NOTFOUND;
    }
    std::vector<uint8_t> mask((size_t)G.n, 1);
    std::vector<int32_t> cur(M, M + k);
    std::vector<int32_t> rverts;   // reversed path
    std::vector<int64_t> rpos;     // reversed edge positions
    std::vector<int64_t> reids;
    int64_t lo = 0, hi = 0;        // positions counted at the last level (all at step 0)
    int32_t end_v = -1;
    for (int step = 0; (int)cur.size() >= 2; ++step) {
        SieveResult res;
        bool got = false;
        for (int r = 0; r < max_reps && !got; ++r) {
            SieveRequest req;
            req.multiset = cur.data();
            req.k = (int32_t)cur.size();
            req.seed = step_seed(seed, step, r);
            req.vertex_mask = mask.data();
            req.fin_lo = lo;
            req.fin_hi = hi;
            req.want_pick = true;
            run_sieve(G, req, res, st);
            ++nsieve;
            got = res.pick_pos >= 0;
        }
        if (!got) return TPM_NOTFOUND;
        int32_t v, u, tau;  // tau: departure of the picked edge
        TPM_HIP(hipMemcpy(&v, G.psrc + res.pick_pos, 4, hipMemcpyDeviceToHost));
        TPM_HIP(hipMemcpy(&u, G.pdst + res.pick_pos, 4, hipMemcpyDeviceToHost));
        TPM_HIP(hipMemcpy(&tau, (G.pdep ? G.pdep : G.ptau) + res.pick_pos, 4, hipMemcpyDeviceToHost));
        if (end_v < 0) rverts.push_back(u);
        rpos.push_back(res.pick_pos);
        reids.push_back(res.pick_eid);
        rverts.push_back(v);
        end_v = v;
        // delete u (every layer copy of it), drop its colour
        mask[(size_t)u] = 0;
        if (!G.h_fid.empty())
            for (int32_t i = 0; i < G.n; ++i)
                if (G.h_fid[(size_t)i] == G.h_fid[(size_t)u]) mask[(size_t)i] = 0;
        auto it = std::find(cur.begin(), cur.end(), G.h_color()[u]);
        if (it == cur.end()) it = std::find(cur.begin(), cur.end(), -1);  // u took a wildcard
        if (it == cur.end()) return TPM_NOTFOUND;  // cannot happen for a certified edge
        cur.erase(it);
        // next: v's in-edges that arrived by tau - delay(v) (plain problem: earlier
        // than tau)
        int32_t ab[2];
        TPM_HIP(hipMemcpy(ab, G.inptr + v, 2 * sizeof(int32_t), hipMemcpyDeviceToHost));
        lo = ab[0];
        int64_t a = ab[0], b = ab[1];
        if (b > a) {
            std::vector<int32_t> taus((size_t)(b - a));
            TPM_HIP(hipMemcpy(taus.data(), G.ptau + a, sizeof(int32_t) * (b - a), hipMemcpyDeviceToHost));
            const int64_t th = (int64_t)tau - (G.h_delay.empty() ? 1 : G.h_delay[(size_t)v]) + 1;
            hi = a + (int64_t)(std::lower_bound(taus.begin(), taus.end(), th,
                                                [](int32_t x, int64_t y) { return (int64_t)x < y; }) -
                               taus.begin());
        } else {
            hi = a;
        }
        if ((int)cur.size() >= 2 && hi <= lo) return TPM_NOTFOUND;
    }
    // cur has one colour left: it must be v's colour
    if (cur.size() != 1 || (G.h_color()[end_v] != cur[0] && cur[0] != -1)) return TPM_NOTFOUND;
    std::reverse(rverts.begin(), rverts.end());
    std::reverse(rpos.begin(), rpos.end());
    std::reverse(reids.begin(), reids.end());
    if (!verify_path(G, M, k, rverts.data(), rpos.data()))
        throw Error{TPM_EDEVICE, "extracted path failed verification"};
    for (int i = 0; i < k; ++i) path_vertices[i] = orig(rverts[i]);
    for (int i = 0; i + 1 < k; ++i) path_edges[i] = reids[i];
    return TPM_OK;
}

// inc[u] = 1 for the endpoints of every edge
__global__ void k_incident(int64_t m, const int32_t *psrc, const int32_t *pdst, uint8_t *inc) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < m) {
        inc[psrc[p]] = 1;
        inc[pdst[p]] = 1;
    }
}

// Self-reducibility (section "Extracting a solution", first approach): delete vertex
// groups while the decision oracle stays YES, halving a group that cannot go (group
// testing, O(k log n) decisions), then find the path among the survivors by temporal
// DFS.  A decision is `reps` sieves with fresh seeds; YES is certain, so a deleted
// group never held the last matching path, and a false NO only keeps extra vertices.
tpm_status extract_selfreduce(const Graph &G, const int32_t *M, int32_t k, uint64_t seed,
                              int32_t reps, int32_t *path_vertices, int64_t *path_edges,
                              int64_t *sieves) {
    TPM_REQUIRE(k >= 2 && k <= 16, "k must be in [2, 16]");
    TPM_REQUIRE(reps >= 1, "max_reps must be >= 1");
    bool wild = false;
    std::vector<uint8_t> in_m((size_t)G.q, 0);
    for (int i = 0; i < k; ++i) {
        TPM_REQUIRE(M[i] >= -1 && M[i] < G.q, "multiset colour out of range");
        if (M[i] < 0) wild = true;
        else in_m[(size_t)M[i]] = 1;
    }
    // vertices of other colours, and vertices without edges, are on no matching path
    std::vector<uint8_t> inc((size_t)G.n, 0);
    if (G.m) {
        DBuf d;
        d.alloc((size_t)G.n, nullptr);
        TPM_HIP(hipMemset(d.p, 0, (size_t)G.n));
        k_incident<<<(unsigned)std::max<int64_t>(1, (G.m + 255) / 256), 256>>>(
            G.m, G.psrc, G.pdst, d.as<uint8_t>());
        TPM_HIP(hipMemcpy(inc.data(), d.p, (size_t)G.n, hipMemcpyDeviceToHost));
    }
    std::vector<uint8_t> mask((size_t)G.n, 0);
    std::vector<int32_t> cand;
    for (int32_t u = 0; u < G.n; ++u)
        if (inc[(size_t)u] && (wild || in_m[(size_t)G.h_color()[(size_t)u]])) {
            mask[(size_t)u] = 1;
            cand.push_back(u);
        }
    // Decisions run on the subgraph of the vertices still live (rebuilt each time the
    // live set halves): deleted vertices have z = 0 either way, so every sieve value is
    // the same, and later decisions touch fewer edges.
    Graph sub;
    bool have_sub = false;
    struct SubOwn {
        Graph &g;
        bool &have;
        ~SubOwn() {
            if (have) {
                g.pool = nullptr;  // borrowed
                free_graph(g);
            }
        }
    } sub_own{sub, have_sub};
    size_t live = cand.size(), live_at_build = cand.size();
    auto maybe_shrink = [&]() {
        if (G.m < 100000 || live * 2 > live_at_build) return;
        DBuf vk;
        vk.alloc((size_t)std::max<int32_t>(1, G.n), nullptr);
        TPM_HIP(hipMemcpy(vk.p, mask.data(), (size_t)G.n, hipMemcpyHostToDevice));
        Graph ng;
        PruneSpec spec;
        spec.vkeep = vk.as<uint8_t>();
        prune_graph(G, spec, ng);
        ng.pool = G.pool;
        if (have_sub) {
            sub.pool = nullptr;
            free_graph(sub);
        }
        sub = ng;
        have_sub = true;
        live_at_build = live;
    };
    int64_t calls = 0, nsieve = 0;
    auto decide = [&]() {
        const Graph &Gs = have_sub ? sub : G;
        for (int32_t r = 0; r < reps; ++r) {
            SieveRequest req;
            req.multiset = M;
            req.k = k;
            req.seed = step_seed(seed, 2000000 + calls, r);
            req.vertex_mask = mask.data();
            SieveResult res;
            run_sieve(Gs, req, res, nullptr);
            ++nsieve;
            if (res.total) {
                ++calls;
                return true;
            }
        }
        ++calls;
        return false;
    };
    struct Count {
        int64_t *out;
        int64_t &n;
        ~Count() {
            if (out) *out = n;
        }
    } count{sieves, nsieve};
    if (!decide()) return TPM_NOTFOUND;
    // group testing over the candidates, in halves
    std::vector<std::pair<size_t, size_t>> todo{{0, cand.size()}};
    while (!todo.empty()) {
        auto [a, b] = todo.back();
        todo.pop_back();
        if (a >= b) continue;
        for (size_t i = a; i < b; ++i) mask[(size_t)cand[i]] = 0;
        if (decide()) {  // the group goes
            live -= b - a;
            maybe_shrink();
            continue;
        }
        for (size_t i = a; i < b; ++i) mask[(size_t)cand[i]] = 1;
        if (b - a == 1) continue;  // an essential vertex
        const size_t mid = a + (b - a) / 2;
        todo.push_back({mid, b});
        todo.push_back({a, mid});
    }
    // ---- temporal DFS among the survivors (host; a handful of vertices)
    std::vector<int32_t> surv;
    for (int32_t u = 0; u < G.n; ++u)
        if (mask[(size_t)u]) surv.push_back(u);
    struct E {
        int32_t src, dst, arr, dep;
        int64_t pos, eid;
    };
    std::vector<std::vector<E>> out_edges((size_t)G.n);
    for (int32_t v : surv) {
        int32_t ab[2];
        TPM_HIP(hipMemcpy(ab, G.inptr + v, 2 * sizeof(int32_t), hipMemcpyDeviceToHost));
        const int64_t len = (int64_t)ab[1] - ab[0];
        if (len <= 0) continue;
        std::vector<int32_t> s((size_t)len), a((size_t)len), d((size_t)len), e((size_t)len);
        TPM_HIP(hipMemcpy(s.data(), G.psrc + ab[0], sizeof(int32_t) * len, hipMemcpyDeviceToHost));
        TPM_HIP(hipMemcpy(a.data(), G.ptau + ab[0], sizeof(int32_t) * len, hipMemcpyDeviceToHost));
        TPM_HIP(hipMemcpy(d.data(), (G.pdep ? G.pdep : G.ptau) + ab[0], sizeof(int32_t) * len,
                          hipMemcpyDeviceToHost));
        TPM_HIP(hipMemcpy(e.data(), G.peid + ab[0], sizeof(int32_t) * len, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < len; ++i)
            if (mask[(size_t)s[(size_t)i]])
                out_edges[(size_t)s[(size_t)i]].push_back(
                    {s[(size_t)i], v, a[(size_t)i], d[(size_t)i], ab[0] + i, e[(size_t)i]});
    }
    auto orig = [&](int32_t u) { return G.h_fid.empty() ? u : G.h_fid[(size_t)u]; };
    std::vector<int32_t> pv;
    std::vector<int64_t> pp, pe;
    std::vector<int32_t> used_orig;
    std::function<bool(int64_t)> dfs = [&](int64_t arr) -> bool {
        if ((int32_t)pv.size() == k)
            return verify_path(G, M, k, pv.data(), pp.data());
        const int32_t w = pv.back();
        const int64_t dl = G.h_delay.empty() ? 1 : G.h_delay[(size_t)w];
        for (const E &x : out_edges[(size_t)w]) {
            if (pv.size() > 1 && !(arr <= (int64_t)x.dep - dl)) continue;
            const int32_t o = orig(x.dst);
            if (std::find(used_orig.begin(), used_orig.end(), o) != used_orig.end()) continue;
            pv.push_back(x.dst);
            pp.push_back(x.pos);
            pe.push_back(x.eid);
            used_orig.push_back(o);
            if (dfs(x.arr)) return true;
            pv.pop_back();
            pp.pop_back();
            pe.pop_back();
            used_orig.pop_back();
        }
        return false;
    };
    for (int32_t u : surv) {
        pv.assign(1, u);
        pp.clear();
        pe.clear();
        used_orig.assign(1, orig(u));
        if (dfs(0)) {
            for (int i = 0; i < k; ++i) path_vertices[i] = orig(pv[(size_t)i]);
            for (int i = 0; i + 1 < k; ++i) path_edges[i] = pe[(size_t)i];
            return TPM_OK;
        }
    }
    return TPM_NOTFOUND;  // every group test said YES only by a path the DFS rules out: impossible
}

// Reverse temporal DFS (section "Extracting a solution", second approach): from the
// vertices u with q[u] != 0 (smallest id first; a nonzero Q_u certifies a matching path
// that ends at u) extend a path backwards through in-edges that arrive early enough
// for the edge already chosen to leave (latest arrival first), with distinct vertices
// and colours drawn from what is left of M.  The DFS is exhaustive per end vertex, so
// it finds a path from a certified u unless `budget` edge visits run out first.
tpm_status extract_from_vertices(const Graph &G, const int32_t *M, int32_t k, const uint8_t *q,
                                 int64_t budget, int32_t *path_vertices, int64_t *path_edges) {
    TPM_REQUIRE(k >= 2 && k <= 16, "k must be in [2, 16]");
    std::vector<int32_t> need((size_t)G.q, 0);
    int32_t wild = 0;
    for (int i = 0; i < k; ++i) {
        TPM_REQUIRE(M[i] >= -1 && M[i] < G.q, "multiset colour out of range");
        if (M[i] < 0) ++wild;
        else ++need[(size_t)M[i]];
    }
    auto orig = [&](int32_t u) { return G.h_fid.empty() ? u : G.h_fid[(size_t)u]; };
    // in-lists fetched on demand (positions in arrival order)
    struct InList {
        int64_t p0 = 0;
        std::vector<int32_t> src, arr, dep, eid;
    };
    std::unordered_map<int32_t, InList> cache;
    auto inlist = [&](int32_t w) -> const InList & {
        auto it = cache.find(w);
        if (it != cache.end()) return it->second;
        InList L;
        int32_t ab[2];
        TPM_HIP(hipMemcpy(ab, G.inptr + w, 2 * sizeof(int32_t), hipMemcpyDeviceToHost));
        L.p0 = ab[0];
        const int64_t len = (int64_t)ab[1] - ab[0];
        if (len > 0) {
            L.src.resize((size_t)len);
            L.arr.resize((size_t)len);
            L.eid.resize((size_t)len);
            TPM_HIP(hipMemcpy(L.src.data(), G.psrc + ab[0], 4 * len, hipMemcpyDeviceToHost));
            TPM_HIP(hipMemcpy(L.arr.data(), G.ptau + ab[0], 4 * len, hipMemcpyDeviceToHost));
            TPM_HIP(hipMemcpy(L.eid.data(), G.peid + ab[0], 4 * len, hipMemcpyDeviceToHost));
            if (G.pdep) {
                L.dep.resize((size_t)len);
                TPM_HIP(hipMemcpy(L.dep.data(), G.pdep + ab[0], 4 * len, hipMemcpyDeviceToHost));
            }
        }
        return cache.emplace(w, std::move(L)).first->second;
    };
    std::vector<int32_t> rv;    // the path, last vertex first
    std::vector<int64_t> rp;    // edge positions, last edge first
    std::vector<int32_t> reid;
    std::vector<int32_t> used;  // original ids on the path
    int64_t visits = 0;
    // a vertex of colour c takes its colour (alt 0) or a wildcard (alt 1)
    auto take = [&](int32_t c, int alt) -> bool {
        int32_t &slot = alt == 0 ? need[(size_t)c] : wild;
        if (slot <= 0) return false;
        --slot;
        return true;
    };
    auto give = [&](int32_t c, int alt) { ++(alt == 0 ? need[(size_t)c] : wild); };
    // extend backwards from rv.back(), whose outgoing path edge leaves at `dep`
    std::function<bool(int64_t)> dfs = [&](int64_t dep) -> bool {
        if ((int32_t)rv.size() == k) {
            std::vector<int32_t> pv(rv.rbegin(), rv.rend());
            std::vector<int64_t> pp(rp.rbegin(), rp.rend());
            return verify_path(G, M, k, pv.data(), pp.data());
        }
        const int32_t w = rv.back();
        const int64_t dl = G.h_delay.empty() ? 1 : G.h_delay[(size_t)w];
        const InList &L = inlist(w);
        // in-edges that arrive by dep - delay(w) (any, for the path's last vertex)
        int64_t hi = (int64_t)L.arr.size();
        if (rv.size() > 1) {
            const int64_t th = dep - dl + 1;  // arrival < th
            hi = std::lower_bound(L.arr.begin(), L.arr.end(), th,
                                  [](int32_t x, int64_t y) { return (int64_t)x < y; }) -
                 L.arr.begin();
        }
        for (int64_t i = hi - 1; i >= 0; --i) {
            if (++visits > budget) return false;
            const int32_t v = L.src[(size_t)i];
            const int32_t o = orig(v);
            if (std::find(used.begin(), used.end(), o) != used.end()) continue;
            const int32_t c = G.h_color()[(size_t)v];
            for (int alt = 0; alt < 2; ++alt) {
                if (!take(c, alt)) continue;
                rv.push_back(v);
                rp.push_back(L.p0 + i);
                reid.push_back(L.eid[(size_t)i]);
                used.push_back(o);
                const int64_t d = G.pdep ? (int64_t)L.dep[(size_t)i] : (int64_t)L.arr[(size_t)i];
                if (dfs(d)) return true;
                rv.pop_back();
                rp.pop_back();
                reid.pop_back();
                used.pop_back();
                give(c, alt);
                if (visits > budget) return false;
            }
        }
        return false;
    };
    for (int32_t u = 0; u < G.n; ++u) {
        if (!q[(size_t)u]) continue;
        const int32_t c = G.h_color()[(size_t)u];
        for (int alt = 0; alt < 2; ++alt) {
            if (!take(c, alt)) continue;
            rv.assign(1, u);
            rp.clear();
            reid.clear();
            used.assign(1, orig(u));
            const bool ok = dfs(0);
            give(c, alt);
            if (ok) {
                for (int i = 0; i < k; ++i) path_vertices[i] = orig(rv[(size_t)(k - 1 - i)]);
                for (int i = 0; i + 1 < k; ++i) path_edges[i] = reid[(size_t)(k - 2 - i)];
                return TPM_OK;
            }
            if (visits > budget) return TPM_NOTFOUND;
        }
    }
    return TPM_NOTFOUND;
}

// Extraction by vertex localisation: one localised sieve per seed, then the reverse
// temporal DFS from the certified end vertices.
tpm_status extract_vertexloc(const Graph &G, const int32_t *M, int32_t k, uint64_t seed,
                             int32_t max_reps, int32_t *path_vertices, int64_t *path_edges,
                             int64_t *sieves, int64_t budget) {
    TPM_REQUIRE(k >= 2 && k <= 16, "k must be in [2, 16]");
    TPM_REQUIRE(max_reps >= 1, "max_reps must be >= 1");
    int64_t nsieve = 0;
    struct Count {
        int64_t *out;
        int64_t &n;
        ~Count() {
            if (out) *out = n;
        }
    } count{sieves, nsieve};
    std::vector<uint8_t> q((size_t)G.n);
    int64_t left = budget;
    for (int32_t r = 0; r < max_reps; ++r) {
        SieveRequest req;
        req.multiset = M;
        req.k = k;
        req.seed = step_seed(seed, 0, r);
        const uint8_t total = vertex_localise(G, req, q.data(), nullptr);
        ++nsieve;
        if (!total) continue;
        const tpm_status st = extract_from_vertices(G, M, k, q.data(), left, path_vertices, path_edges);
        if (st == TPM_OK) return TPM_OK;
        return TPM_NOTFOUND;  // a certified end vertex and no path within the budget
    }
    (void)left;
    return TPM_NOTFOUND;
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ autotune cache
// Results of tpm_autotune by (GPU architecture, k, log2 m, log2 n): one process-wide
// table, also kept in the file named by TPM_AUTOTUNE_CACHE when that is set (one entry
// a line: arch k log2m log2n tile chunk; read once, appended to on every new entry).
struct TuneKey {
    std::string arch;
    int k = 0, mlog = 0, nlog = 0;
    bool operator<(const TuneKey &o) const {
        return std::tie(arch, k, mlog, nlog) < std::tie(o.arch, o.k, o.mlog, o.nlog);
    }
};
struct TuneVal {
    int tile = 0, chunk = 0;
};

std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
bool g_tune_loaded = false;

int log2_floor(int64_t v) {
    int b = 0;
    while (v > 1) {
        v >>= 1;
        ++b;
    }
    return b;
}

TuneKey tune_key(const Graph &G, int k) {
    hipDeviceProp_t prop{};
    TPM_HIP(hipGetDeviceProperties(&prop, G.device));
    TuneKey key;
    key.arch = prop.gcnArchName;
    key.arch = key.arch.substr(0, key.arch.find(':'));  // gfx950, without feature flags
    key.k = k;
    key.mlog = log2_floor(std::max<int64_t>(1, G.m));
    key.nlog = log2_floor(std::max<int64_t>(1, G.n));
    return key;
}

const char *tune_file() {
    const char *f = std::getenv("TPM_AUTOTUNE_CACHE");
    return (f && *f) ? f : nullptr;
}

// caller holds g_tune_mu
void tune_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *f = tune_file();
    if (!f) return;
    std::ifstream in(f);
    TuneKey key;
    TuneVal val;
    while (in >> key.arch >> key.k >> key.mlog >> key.nlog >> val.tile >> val.chunk)
        if (val.tile >= 1 && val.tile <= 4096 && val.chunk >= 4) g_tune[key] = val;
}

bool tune_lookup(const TuneKey &key, TuneVal &val) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load();
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    val = it->second;
    return true;
}

void tune_store(const TuneKey &key, const TuneVal &val) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load();
    g_tune[key] = val;
    if (const char *f = tune_file()) {
        std::ofstream o(f, std::ios::app);
        o << key.arch << ' ' << key.k << ' ' << key.mlog << ' ' << key.nlog << ' ' << val.tile << ' '
          << val.chunk << '\n';
    }
}

// Streaming read for counter calibration: every 16-byte word once (grid-stride), XOR
// of the words reduced per wave, one atomic per wave.
__global__ void k_stream_read(const uint4 *src, int64_t words, unsigned long long *out) {
    unsigned long long v = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint4 t = src[i];
        v ^= ((unsigned long long)t.y << 32 | t.x) ^ ((unsigned long long)t.w << 32 | t.z);
    }
    for (int off = 32; off >= 1; off >>= 1) v ^= __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0 && v) atomicXor(out, v);
}

__global__ void k_zero64(unsigned long long *p) { *p = 0; }

}  // namespace tpm

using namespace tpm;

extern "C" {

tpm_status tpm_stream_read(const void *src, int64_t bytes, uint64_t *out, void *hip_stream) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(src && out, "NULL argument");
        TPM_REQUIRE(bytes >= 0 && bytes % 16 == 0, "bytes must be a non-negative multiple of 16");
        TPM_REQUIRE(((uintptr_t)src & 15) == 0, "src must be 16-byte aligned");
        hipStream_t st = (hipStream_t)hip_stream;
        int dev = 0, cus = 0;
        TPM_HIP(hipGetDevice(&dev));
        TPM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const int64_t words = bytes / 16;
        const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * 8, (words + 255) / 256));
        k_zero64<<<1, 1, 0, st>>>((unsigned long long *)out);
        k_stream_read<<<(unsigned)grid, 256, 0, st>>>((const uint4 *)src, words, (unsigned long long *)out);
        TPM_HIP(hipGetLastError());
        return TPM_OK;
    });
}

const char *tpm_last_error(void) { return t_last_error.c_str(); }

const char *tpm_version(void) { return "tpm 0.1 (gfx950)"; }

tpm_status tpm_profile_enable(int32_t on) {
    g_profile.store(on ? 1 : 0);
    return TPM_OK;
}

tpm_status tpm_profile_read(tpm_kernel_time *out, int32_t max, int32_t *n_out) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(n_out && (max == 0 || out), "NULL argument");
        std::lock_guard<std::mutex> lk(g_prof_mu);
        int32_t n = std::min<int32_t>(max, (int32_t)g_prof_done.size());
        for (int32_t i = 0; i < n; ++i) out[i] = g_prof_done[i];
        g_prof_done.erase(g_prof_done.begin(), g_prof_done.begin() + n);
        *n_out = n;
        return TPM_OK;
    });
}

tpm_status tpm_graph_create_ex(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                               const int32_t *tau, const int32_t *color, int32_t num_colors,
                               uint32_t flags, const tpm_graph_options *opt, tpm_graph **out) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(out != nullptr, "out must not be NULL");
        *out = nullptr;
        auto *g = new tpm_graph();
        try {
            build_graph(g->G, n, m, src, dst, tau, color, num_colors, flags, opt);
            g->G.pool = new_workspace_pool();
            g->G.apool = new_arena_pool();
        } catch (...) {
            delete g;
            throw;
        }
        *out = g;
        return TPM_OK;
    });
}

tpm_status tpm_graph_create(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                            const int32_t *tau, const int32_t *color, int32_t num_colors,
                            uint32_t flags, tpm_graph **out) {
    return tpm_graph_create_ex(n, m, src, dst, tau, color, num_colors, flags, nullptr, out);
}

void tpm_graph_destroy(tpm_graph *g) {
    if (!g) return;
    int prev = -1;
    if (hipGetDevice(&prev) == hipSuccess && prev != g->G.device) (void)hipSetDevice(g->G.device);
    (void)hipDeviceSynchronize();
    delete_workspace_pool(g->G.pool);
    g->G.pool = nullptr;
    delete_arena_pool(g->G.apool);
    g->G.apool = nullptr;
    free_graph(g->G);
    if (prev >= 0 && prev != g->G.device) (void)hipSetDevice(prev);
    delete g;
}

tpm_status tpm_graph_prune(const tpm_graph *g, const int32_t *colors, int32_t ncolors,
                           tpm_graph **out) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(colors && ncolors >= 1, "colors must be given (ncolors >= 1)");
        return tpm_graph_prune_ex(g, colors, ncolors, nullptr, 0, out);
    });
}

tpm_status tpm_graph_prune_ex(const tpm_graph *g, const int32_t *colors, int32_t ncolors,
                              const int32_t *times, int32_t ntimes, tpm_graph **out) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(g && out, "NULL argument");
        *out = nullptr;
        TPM_REQUIRE(ncolors >= 0 && ntimes >= 0, "counts must be >= 0");
        TPM_REQUIRE(ncolors == 0 || colors, "colors must not be NULL");
        TPM_REQUIRE(ntimes == 0 || times, "times must not be NULL");
        std::vector<uint8_t> keep((size_t)g->G.q, ncolors ? 0 : 1);
        for (int32_t i = 0; i < ncolors; ++i) {
            TPM_REQUIRE(colors[i] >= 0 && colors[i] < g->G.q, "colour out of range");
            keep[(size_t)colors[i]] = 1;
        }
        std::vector<int32_t> ts(times, times + ntimes);
        std::sort(ts.begin(), ts.end());
        ts.erase(std::unique(ts.begin(), ts.end()), ts.end());
        DeviceScope ds(g->G.device);
        auto *h = new tpm_graph();
        try {
            PruneSpec spec;
            spec.keep_color = keep.data();
            spec.times = ntimes ? ts.data() : nullptr;
            spec.ntimes = (int32_t)ts.size();
            prune_graph(g->G, spec, h->G);
            h->G.pool = new_workspace_pool();
            h->G.apool = new_arena_pool();
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
        return TPM_OK;
    });
}

tpm_status tpm_graph_layer(const tpm_graph *g, const int32_t *tuple, int32_t k, tpm_graph **out) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(g && tuple && out, "NULL argument");
        *out = nullptr;
        DeviceScope ds(g->G.device);
        auto *h = new tpm_graph();
        try {
            layer_graph(g->G, tuple, k, h->G);
            h->G.pool = new_workspace_pool();
            h->G.apool = new_arena_pool();
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
        return TPM_OK;
    });
}

tpm_status tpm_extract_optimum(const tpm_graph *g, const int32_t *multiset, int32_t k,
                               uint64_t seed, int32_t reps, int32_t method, int32_t *t_out,
                               int32_t *path_vertices, int64_t *path_edges) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(g && multiset && t_out && path_vertices && path_edges, "NULL argument");
        TPM_REQUIRE(method >= 0 && method <= 2, "method must be 0, 1 or 2");
        DeviceScope ds(g->G.device);
        const Graph &G = g->G;
        *t_out = optimum_time(G, multiset, k, seed, reps);
        if (*t_out < 0) return TPM_NOTFOUND;
        // the subgraph of the edges that arrive by the optimum: every path in it finishes
        // by then, and it holds the optimal paths (same ids, so their fingerprints)
        Graph P;
        struct Own {
            Graph &g;
            ~Own() {
                g.pool = nullptr;  // borrowed
                free_graph(g);
            }
        } own{P};
        PruneSpec spec;
        spec.tcut = *t_out;
        prune_graph(G, spec, P);
        P.pool = G.pool;
        const uint64_t s2 = seed + 0x5851F42D4C957F2Dull;  // fresh seeds for the extraction
        if (method == 1)
            return extract_selfreduce(P, multiset, k, s2, reps, path_vertices, path_edges, nullptr);
        if (method == 2)
            return extract_vertexloc(P, multiset, k, s2, reps, path_vertices, path_edges, nullptr,
                                     kDfsBudget);
        return extract_path(P, multiset, k, s2, reps, path_vertices, path_edges, nullptr);
    });
}

tpm_status tpm_graph_sd(const tpm_graph *g, int32_t s, int32_t d, tpm_graph **out) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(g && out, "NULL argument");
        *out = nullptr;
        DeviceScope ds(g->G.device);
        auto *h = new tpm_graph();
        try {
            sd_graph(g->G, s, d, h->G);
            h->G.pool = new_workspace_pool();
            h->G.apool = new_arena_pool();
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
        return TPM_OK;
    });
}

tpm_status tpm_graph_vertex_ids(const tpm_graph *g, int32_t *ids) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(g && ids, "NULL argument");
        const Graph &G = g->G;
        for (int32_t i = 0; i < G.n; ++i) ids[i] = G.h_fid.empty() ? i : G.h_fid[(size_t)i];
        return TPM_OK;
    });
}

tpm_status tpm_graph_retile(tpm_graph *g, int32_t tile_edges) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(g != nullptr, "graph must not be NULL");
        DeviceScope ds(g->G.device);
        retile_graph(g->G, tile_edges);
        return TPM_OK;
    });
}

tpm_status tpm_autotune(tpm_graph *g, int32_t k, uint64_t seed, tpm_autotune_report *out) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(g && out, "NULL argument");
        TPM_REQUIRE(k >= 2 && k <= 16, "k must be in [2, 16]");
        DeviceScope ds(g->G.device);
        Graph &G = g->G;
        std::memset(out, 0, sizeof(*out));
        const TuneKey key = tune_key(G, k);
        TuneVal hit;
        if (tune_lookup(key, hit)) {
            retile_graph(G, hit.tile);
            out->tile_edges = hit.tile;
            out->chunk = hit.chunk;
            out->cached = 1;
            return TPM_OK;
        }
        int32_t M[16];
        for (int i = 0; i < k; ++i) M[i] = i % G.q;
        const int64_t npts = int64_t(1) << k;
        std::vector<int32_t> chunks;
        if (npts < 256) chunks.push_back((int32_t)npts);
        for (int32_t c : {256, 512, 1024})
            if (c <= npts) chunks.push_back(c);
        const int32_t tiles[4] = {256, 512, 1024, 2048};
        const int32_t cmp = chunks.front();  // points every candidate computes
        const int32_t orig_T = G.tile_edges;
        std::vector<uint8_t> first;
        double best = -1.0;
        try {
            for (int32_t T : tiles) {
                retile_graph(G, T);
                for (int32_t C : chunks) {
                    SieveRequest req;
                    req.multiset = M;
                    req.k = k;
                    req.seed = seed;
                    req.chunk = C;
                    req.max_chunks = 1;
                    SieveResult res;
                    run_sieve(G, req, res, nullptr);  // untimed: sizes the workspace
                    const double t0 = now_ms();
                    run_sieve(G, req, res, nullptr);
                    const double ms = std::max(now_ms() - t0, 1e-6);
                    if (first.empty()) {
                        first.assign(res.per_point.begin(), res.per_point.begin() + cmp);
                    } else if (!std::equal(first.begin(), first.end(), res.per_point.begin())) {
                        throw Error{TPM_EDEVICE, "autotune candidates disagree (tile " +
                                                     std::to_string(T) + ", chunk " +
                                                     std::to_string(C) + ")"};
                    }
                    const double rate = (double)G.m * (double)(k - 1) * (double)C / (ms * 1e-3);
                    const int i = out->ncand++;
                    out->cand_tile[i] = T;
                    out->cand_chunk[i] = C;
                    out->cand_rate[i] = rate;
                    if (rate > best) {
                        best = rate;
                        out->tile_edges = T;
                        out->chunk = C;
                    }
                }
            }
            retile_graph(G, out->tile_edges);
            tune_store(key, TuneVal{out->tile_edges, out->chunk});
        } catch (...) {
            try {
                retile_graph(G, orig_T);
            } catch (...) {
            }
            throw;
        }
        return TPM_OK;
    });
}

tpm_status tpm_graph_stats_get(const tpm_graph *g, tpm_graph_stats *out) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(g && out, "NULL argument");
        const Graph &G = g->G;
        out->n = G.n;
        out->m = G.m;
        out->num_colors = G.q;
        out->tmax = G.tmax;
        out->rows = G.R;
        out->tiles = G.ntiles;
        out->slots = G.nslots;
        out->max_in_degree = G.max_in_degree;
        out->device_bytes = G.device_bytes;
        out->gathers = G.gathers;
        out->segments = G.segments;
        out->times = G.ntimes;
        out->edge_ids = G.edge_ids;
        out->tile_edges = G.tile_edges;
        return TPM_OK;
    });
}

tpm_status tpm_sieve_ex(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                        const uint8_t *vertex_mask, const tpm_tuning *tune, uint8_t *per_point,
                        uint8_t *total, uint8_t *loc, void *hip_stream) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(g != nullptr, "graph must not be NULL");
        DeviceScope ds(g->G.device);
        SieveRequest req;
        req.multiset = multiset;
        req.k = k;
        req.seed = seed;
        req.vertex_mask = vertex_mask;
        req.chunk = tune ? tune->chunk : 0;
        TPM_REQUIRE(!tune || tune->prune == 0 || tune->prune == 1, "prune must be 0 or 1");
        SieveResult res;
        hipStream_t st = (hipStream_t)hip_stream;
        if (tune && tune->prune) run_sieve_pruned(g->G, req, res, loc, st);
        else if (loc) run_sieve_loc_all(g->G, req, res, loc, st);
        else run_sieve(g->G, req, res, st);
        if (per_point) std::memcpy(per_point, res.per_point.data(), res.per_point.size());
        if (total) *total = res.total;
        return TPM_OK;
    });
}

tpm_status tpm_sieve(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                     const uint8_t *vertex_mask, uint8_t *per_point, uint8_t *total,
                     void *hip_stream) {
    return tpm_sieve_ex(g, multiset, k, seed, vertex_mask, nullptr, per_point, total, nullptr,
                        hip_stream);
}

tpm_status tpm_decide(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                      int32_t reps, int32_t *found) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(g && found, "NULL argument");
        TPM_REQUIRE(reps >= 1, "reps must be >= 1");
        DeviceScope ds(g->G.device);
        *found = 0;
        for (int32_t r = 0; r < reps; ++r) {
            SieveRequest req;
            req.multiset = multiset;
            req.k = k;
            req.seed = rep_seed(seed, r);
            SieveResult res;
            run_sieve(g->G, req, res, nullptr);
            if (res.total) {
                *found = 1;
                break;
            }
        }
        return TPM_OK;
    });
}

tpm_status tpm_extract_ex(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                          int32_t max_reps, int32_t method, int32_t *path_vertices,
                          int64_t *path_edges, int64_t *sieves) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(g && multiset && path_vertices && (k < 2 || path_edges), "NULL argument");
        TPM_REQUIRE(method >= 0 && method <= 2, "method must be 0, 1 or 2");
        DeviceScope ds(g->G.device);
        if (method == 1 && k >= 2)
            return extract_selfreduce(g->G, multiset, k, seed, max_reps, path_vertices, path_edges,
                                      sieves);
        if (method == 2 && k >= 2)
            return extract_vertexloc(g->G, multiset, k, seed, max_reps, path_vertices, path_edges,
                                     sieves, kDfsBudget);
        return extract_path(g->G, multiset, k, seed, max_reps, path_vertices, path_edges, nullptr,
                            sieves);
    });
}

tpm_status tpm_extract(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                       int32_t max_reps, int32_t *path_vertices, int64_t *path_edges) {
    return guarded([&]() -> tpm_status {
        TPM_REQUIRE(g && multiset && path_vertices && (k < 2 || path_edges), "NULL argument");
        DeviceScope ds(g->G.device);
        // the vertex-localisation DFS (one sieve) with a bounded budget, then the
        // localisation-guided self-reduction
        if (k >= 2 && extract_vertexloc(g->G, multiset, k, seed, max_reps, path_vertices,
                                        path_edges, nullptr, kQuickDfsBudget) == TPM_OK)
            return TPM_OK;
        return extract_path(g->G, multiset, k, seed, max_reps, path_vertices, path_edges, nullptr);
    });
}

}  // extern "C"
