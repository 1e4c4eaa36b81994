// Internal declarations shared by the libtpm translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tpm.h"

namespace tpm {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
void clear_error();

struct Error {
    tpm_status code;
    std::string msg;
};

// Runs an entry point body: exceptions become status codes and tpm_last_error text.
template <class F>
tpm_status guarded_call(F &&f) {
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

// Makes `dev` current for a scope (restores the previous device).
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            if (hipSetDevice(dev) != hipSuccess) prev = -1;
        } else {
            prev = -1;
        }
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    DeviceGuard(const DeviceGuard &) = delete;
    DeviceGuard &operator=(const DeviceGuard &) = delete;
};

#define TPM_HIP(expr)                                                                 \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess)                                                         \
            throw ::tpm::Error{_e == hipErrorOutOfMemory ? TPM_ENOMEM : TPM_EDEVICE,  \
                               std::string(#expr) + ": " + hipGetErrorString(_e)};   \
    } while (0)

#define TPM_REQUIRE(cond, msg)                                                        \
    do {                                                                              \
        if (!(cond))                                                                  \
            throw ::tpm::Error{TPM_EINVAL, (msg)};                                    \
    } while (0)

// ------------------------------------------------------------------ GF(2^8)
// Power and logarithm tables of the generator alpha = x (0x02) of GF(2^8) with
// modulus x^8 + x^4 + x^3 + x^2 + 1, generated at compile time by repeated
// multiplication by x (shift, and fold x^8 back as 0x1D).
struct GfTables {
    uint8_t exp[512];  // exp[i] = alpha^(i mod 255)
    uint8_t log[256];  // log[v] = i with alpha^i = v; log[0] = 255 (marks zero)
};

constexpr GfTables make_gf_tables() {
    GfTables t{};
    unsigned v = 1;
    for (int i = 0; i < 255; ++i) {
        t.exp[i] = (uint8_t)v;
        t.log[v] = (uint8_t)i;
        v <<= 1;
        if (v & 0x100u) v ^= 0x11Du;
    }
    for (int i = 255; i < 512; ++i) t.exp[i] = t.exp[i - 255];
    t.log[0] = 255;
    return t;
}

inline constexpr GfTables kGf = make_gf_tables();

// Per-workgroup LDS tables of the sieve kernels.  gfx950's LDS serves 32 dword banks,
// so every entry is stored 32 times, once per bank, and lane L reads the copy in
// bank L mod 32: lookups never conflict whatever the looked-up values are.
//   LOG region, [0, 65536): row g (256 bytes) holds, in its first 128 bytes, 32
//     copies of the dword LOG7[g] = log(g) << 7 (kZero7 for g = 0); the second
//     half of each row is unused.
//   EXP region, [kExpBase, kExpBase + kExpRows * 128): row s holds 32 copies of the
//     dword alpha^(s mod 255) for s <= 762 and 0 for s = 763 (the clamp row).
// The product x * y * g of three field elements is then the low byte of EXP row
// min(log x + log y + log g, 763): one LOG read of g, one EXP read.
constexpr int kExpBase = 65536;
constexpr int kExpRows = 764;
constexpr int kClampRow = 763;
constexpr uint32_t kZero7 = 0x00100000u;  // LOG7 of zero: pushes any sum past the clamp
constexpr int kLdsBytes = kExpBase + kExpRows * 128;  // 163328 <= 160 KiB

// ------------------------------------------------------------------ workspaces
// A device buffer that keeps its allocation across calls and only grows.
struct DBuf {
    void *p = nullptr;
    size_t cap = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    // ensures capacity (synchronises on growth); takes 1/8 more when the device has it,
    // unless `exact` (buffers sized to a budget)
    void alloc(size_t bytes, hipStream_t st, bool exact = false);
    ~DBuf();
    template <class T>
    T *as() const { return (T *)p; }
};

// Device memory of one sieve call: level buffers, per-vertex rows, control words.
struct Workspace {
    DBuf ctl, z, xt, s0, s1, pub, pp, tot, mask, loc, pick, tabs, aux, aux2, w2;
};

// Workspaces of a graph: a call takes one (creating it if none is free) and
// returns it when its stream is synchronised, so concurrent calls never share one.
struct WorkspacePool;
struct GraphArena;
struct Graph;
WorkspacePool *new_workspace_pool();
void delete_workspace_pool(WorkspacePool *p);

// Arenas for per-query subgraphs of a graph: a call takes one (creating it if none is
// free) for the lifetime of its subgraph.
struct ArenaPool;
ArenaPool *new_arena_pool();
void delete_arena_pool(ArenaPool *p);

// Device bytes held by a workspace, and release of all of them (waits for the device).
int64_t workspace_bytes(const Workspace *w);
void workspace_trim(Workspace *w);

// Long leases (a worker's lifetime) of a pool's workspace / arena; returned for reuse.
Workspace *workspace_take(WorkspacePool *p);
void workspace_give(WorkspacePool *p, Workspace *w);
GraphArena *arena_take(ArenaPool *p);
void arena_give(ArenaPool *p, GraphArena *a);

struct WorkspaceLease {
    explicit WorkspaceLease(const Graph &G);
    ~WorkspaceLease();
    WorkspaceLease(const WorkspaceLease &) = delete;
    WorkspaceLease &operator=(const WorkspaceLease &) = delete;
    WorkspacePool *pool;
    Workspace *ws;
};

// ------------------------------------------------------------------ graph
struct Graph {
    int device = 0;
    int32_t n = 0;
    int64_t m = 0;
    int32_t q = 0;
    int32_t tmax = 0;
    int32_t tile_edges = 1024;
    bool tile_auto = true;     // tile_edges chosen from m (not set by the caller)
    int64_t R = 0;        // stored rows per level
    int64_t ntiles = 0;
    int64_t nslots = 0;
    int64_t max_in_degree = 0;
    int64_t gathers = 0;
    int64_t segments = 0;
    int64_t device_bytes = 0;
    int num_cu = 0;

    // device arrays (CSR order = edges sorted by (dst, tau, input id))
    int32_t *color = nullptr;  // [n]
    int32_t *pdst = nullptr;   // [m] dst of the edge at each position
    int32_t *psrc = nullptr;   // [m] src
    int32_t *ptau = nullptr;   // [m] timestamp
    int32_t *peid = nullptr;   // [m] input edge id
    int32_t *gsrc = nullptr;   // [m] state row read by the edge (last in-edge of src
                               //     earlier than tau), -1 if none
    int32_t *orow = nullptr;   // [m] state row written at this position, -1 if none
    int32_t *gposw = nullptr;  // [m] position whose row the edge reads, -1 if none
                               //     (whole graphs only: pruning remaps it)
    uint16_t *pcol = nullptr;  // [m] colours of the edge's source (low byte) and head
                               //     (high byte): whole graphs with <= 64 colours
    int32_t *inptr = nullptr;  // [n+1]
    // colour subgraphs (<= 64 colours): only vertices of these colours have edges, so
    // the level pipeline computes vertex rows for them alone; 0 = every vertex
    uint64_t edge_colors = 0;
    int32_t *tile_p0 = nullptr;   // [ntiles+1]
    int32_t *tile_pub = nullptr;  // [ntiles] slot this tile publishes to, -1 if none
    int32_t *tile_lb = nullptr;   // [ntiles] slot its look-back starts at, -1 if none
    uint8_t *lds_image = nullptr; // [kLdsBytes]
    int32_t *pdep = nullptr;      // [m] departure times when edges have transition times
                                  //     (ptau then holds arrivals), else null
    int32_t *vdelay = nullptr;    // [n] per-vertex delays, null = 1 everywhere
    int32_t *fid = nullptr;       // [n] original vertex of each vertex of a layered graph
                                  //     (keys its fingerprints), null = identity
    int32_t *ttab = nullptr;      // [ntimes] distinct timestamps, ascending
    int64_t ntimes = 0;
    int64_t edge_ids = 0;         // input edge ids are < edge_ids (m, or the parent's m
                                  // for a colour-pruned graph)

    WorkspacePool *pool = nullptr;  // owned (shared, not owned, by per-query subgraphs)
    ArenaPool *apool = nullptr;     // owned: memory of per-query subgraphs
    GraphArena *arena = nullptr;    // not owned: device arrays live there when set

    // host copies
    // [n] vertex colours; shared (not copied) by the per-query subgraphs of a graph
    std::shared_ptr<std::vector<int32_t>> h_color_sp;
    std::vector<int32_t> h_tile_p0; // [ntiles+1]
    std::vector<int32_t> h_ttab;    // [ntimes]
    std::vector<int32_t> h_delay;   // [n] when vdelay is set
    std::vector<int32_t> h_fid;     // [n] when fid is set

    const std::vector<int32_t> &h_color() const { return *h_color_sp; }
    std::vector<int32_t> &h_color_mut() {
        if (!h_color_sp) h_color_sp = std::make_shared<std::vector<int32_t>>();
        return *h_color_sp;
    }
};

// Builds all of the above; throws Error.
void build_graph(Graph &G, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                 const int32_t *tau, const int32_t *color, int32_t num_colors, uint32_t flags,
                 const tpm_graph_options *opt);
void free_graph(Graph &G);
// (Re)computes G.pcol from G.color for a whole graph with at most 64 colours.
void build_pcol(Graph &G, int64_t &acct);
// Default work-tile size: 1024 positions, fewer for small graphs so that the tiles
// (each walked by one wave) still outnumber the waves of the GPU.
int32_t auto_tile_edges(int64_t m);
// Rebuilds the work tiles with at most T positions each (results do not depend on
// T).  Waits for the device; must not overlap other calls on the same graph.
void retile_graph(Graph &G, int32_t T);
// Builds G as the subgraph of P on the edges whose two endpoints have a colour c with
// keep_color[c] != 0 (host, P.q bytes).  Vertex ids, colours and input edge ids are
// kept, so every fingerprint, and every sieve whose colours are all kept, is
// unchanged.  G must be empty; on error G is freed.
// Which edges a pruned graph keeps: both endpoints kept and every other condition met.
struct PruneSpec {
    const uint8_t *keep_color = nullptr;  // host [P.q]; nullable: every colour
    const int32_t *times = nullptr;       // host, sorted, distinct; nullable: every
    int32_t ntimes = 0;                   //   timestamp (else departures in the set)
    int32_t cut_in = -1, cut_out = -1;    // a vertex whose in- / out-edges go (-1: none)
    const uint8_t *vkeep = nullptr;       // device [P.n]; nullable: every vertex
    int32_t tcut = 0x7FFFFFFF;            // keep edges that arrive by tcut
    bool need_times = true;               // build the distinct-timestamp table (time
                                          // buckets, optimum time); off for subgraphs
                                          // that only run sieves and extraction
};
// With an arena, G's arrays and the build's temporaries live in the arena's grow-only
// buffers (reused by the next graph built there; G must be freed before that, and must
// not outlive P: it shares P's host colours and LDS image).  All device work runs on
// `st` and the call waits only for that stream, so prunes on other streams overlap.
// Vertex ids, colours, timestamps and input edge ids are P's.
void prune_graph(const Graph &P, const PruneSpec &spec, Graph &G, GraphArena *arena = nullptr,
                 hipStream_t st = nullptr);
// Device bytes held by an arena's buffers.
int64_t arena_bytes(const GraphArena *a);
// Releases every buffer of an arena (waits for the device).
void arena_trim(GraphArena *a);
// Edge counts by colour pair: out[a * q + b] = edges from a vertex of colour a to one of
// colour b (q = G.q <= 64; whole graphs only).  Synchronous on st.
void colour_pair_counts(const Graph &G, std::vector<int64_t> &out, hipStream_t st);
// (s,d)-COLORFUL-PATH: G = P with colour q on s and q + 1 on d (q + 2 colours), s's
// in-edges and d's out-edges removed.
void sd_graph(const Graph &P, int32_t s, int32_t d, Graph &G);
// VC-PATH-MOTIF: G = the layered graph of P for the colour tuple[0..k): vertex (u, l)
// for each layer l with c(u) = tuple[l-1] (fingerprints keyed by u), edges
// (v, l-1) -> (u, l) for P's edges v -> u with matching colours.
void layer_graph(const Graph &P, const int32_t *tuple, int32_t k, Graph &G);
GraphArena *new_graph_arena();
void delete_graph_arena(GraphArena *a);

// ------------------------------------------------------------------ sieve
// Block aggregate of the segmented XOR scan behind level 2's coefficient form (the
// sieve kernels): the block's value at its last position (back to its last segment
// start) and whether a segment starts in it.
struct W2Agg {
    uint4 v;
    uint32_t head;
    uint32_t pad[3];
};

// Inclusive scan of n block aggregates under (a, b) -> (b.head ? b.v : a.v ^ b.v,
// a.head | b.head) on st, in tmp (tmp_bytes); with tmp == nullptr only returns the bytes
// of temporary storage it needs.
size_t w2_scan(void *tmp, size_t tmp_bytes, const W2Agg *in, W2Agg *out, int64_t n, hipStream_t st);

struct SieveRequest {
    const int32_t *multiset = nullptr;
    int32_t k = 0;
    uint64_t seed = 0;
    const uint8_t *vertex_mask = nullptr;  // host, n bytes, nullable
    int32_t chunk = 0;
    // restrict the last level's contributions to CSR positions [fin_lo, fin_hi)
    // (all positions if fin_lo >= fin_hi)
    int64_t fin_lo = 0, fin_hi = 0;
    // localise over the contributing positions and pick the one with nonzero
    // localisation and the smallest input edge id
    bool want_pick = false;
    // run only the first chunk of sieve points (timing probes); 0 = all chunks
    int32_t max_chunks = 0;
    // nullable: checked before every level launch; when it is nonzero, or the host
    // clock (now_ms) has passed deadline_ms, the call stops launching, waits for the
    // stream and throws TPM_ECANCELLED
    const std::atomic<int> *cancel = nullptr;
    double deadline_ms = 0;  // 0 = none
    // nullable: run in this workspace (owned by the caller, used on one stream at a
    // time) instead of one leased from the graph's pool
    Workspace *ws = nullptr;
    // nullable: called on the host before every level launch (after the cancellation
    // check) with the call's stream; a server lends the device between levels with it
    const std::function<void(hipStream_t)> *between_levels = nullptr;
};

// Host clock in ms (steady clock), shared by the serving deadlines and timestamps.
double now_ms();

struct SieveResult {
    std::vector<uint8_t> per_point;  // 2^k
    uint8_t total = 0;
    int64_t pick_eid = -1, pick_pos = -1;
};

void run_sieve(const Graph &G, const SieveRequest &req, SieveResult &res, hipStream_t stream);

// Witness extraction by localisation-guided self-reduction (tpm_extract); sieves
// (nullable) receives the number of sieves run.
tpm_status extract_path(const Graph &G, const int32_t *M, int32_t k, uint64_t seed,
                        int32_t max_reps, int32_t *path_vertices, int64_t *path_edges,
                        hipStream_t st, int64_t *sieves = nullptr);

// Consumes the per-position localisation of a sieve (positions [lo, hi), device
// memory) on the sieve's stream, before the call's final synchronisation; results go
// to host memory the sink owns (copied asynchronously on st).  Scratch: ws.aux, ws.aux2.
struct LocSink {
    virtual ~LocSink() = default;
    virtual void consume(const Graph &G, Workspace &ws, const uint8_t *dloc, int64_t lo,
                         int64_t hi, hipStream_t st) = 0;
};
// The same sieve on the subgraph of the query's colours (preprocessing step (i));
// loc_by_edge (nullable, edge_ids bytes) as run_sieve_loc_all.  Queries with wildcard
// entries run on G.  `then` (nullable) runs on the subgraph before it is freed.
void run_sieve_pruned(const Graph &G, const SieveRequest &req, SieveResult &res,
                      uint8_t *loc_by_edge, hipStream_t st,
                      void (*then)(const Graph &, void *) = nullptr, void *ctx = nullptr);

// Sieve with localisation over the positions req.fin_lo..fin_hi (all when empty),
// handed to `sink`.
void run_sieve_sink(const Graph &G, const SieveRequest &req, SieveResult &res, LocSink &sink,
                    hipStream_t st);

// Vertex localisation of one sieve: q[u] (host, G.n bytes) = XOR of the per-edge
// localisation over u's in-edges (the sieve over walks ending at u).
// Optimum timestamp (smallest t whose time-restricted sieve is nonzero, minimised over
// reps seeds seed + r * 0x9E3779B97F4A7C15); -1 if no seed finds a path.
int32_t optimum_time(const Graph &G, const int32_t *M, int32_t k, uint64_t seed, int32_t reps);
// Returns the sieve total (the XOR of the q[u]); per_point (nullable) receives the
// 2^k per-point values of the same sieve.
uint8_t vertex_localise(const Graph &G, const SieveRequest &req, uint8_t *q, hipStream_t st,
                        std::vector<uint8_t> *per_point = nullptr);
// Extraction by vertex localisation (section "Extracting a solution", second
// approach): reverse temporal DFS from the vertices u with q[u] != 0 (q: host, G.n
// bytes, from vertex_localise), at most `budget` edge visits.  TPM_OK / TPM_NOTFOUND.
constexpr int64_t kDfsBudget = 50'000'000;
constexpr int64_t kQuickDfsBudget = 5'000'000;  // before falling back to self-reduction
tpm_status extract_from_vertices(const Graph &G, const int32_t *M, int32_t k, const uint8_t *q,
                                 int64_t budget, int32_t *path_vertices, int64_t *path_edges);
// One localised sieve per seed (step seeds of extraction), then the DFS.
tpm_status extract_vertexloc(const Graph &G, const int32_t *M, int32_t k, uint64_t seed,
                             int32_t max_reps, int32_t *path_vertices, int64_t *path_edges,
                             int64_t *sieves, int64_t budget);

// A whole sieve query enqueued on st with every buffer carved out of the device block
// [scratch, scratch + cap): no allocation and no host synchronisation.  Outputs go to
// device memory: *total, per_point[0 .. 2^k) (nullable) and *err (nullable: the
// look-back failure bits, 0 when none).  Rows are the widest power of two of points
// whose buffers fit; TPM_ENOMEM when even 16-point rows do not.  No vertex mask.
void enqueue_sieve_fixed(const Graph &G, const int32_t *M, int32_t k, uint64_t seed,
                         uint8_t *scratch, size_t cap, uint8_t *per_point, uint8_t *total,
                         uint32_t *err, hipStream_t st);
// bytes enqueue_sieve_fixed needs at its narrowest rows
size_t fixed_scratch_need(const Graph &G, int32_t k);


// Per-edge localisation over all edges, indexed by input edge id.
void run_sieve_loc_all(const Graph &G, const SieveRequest &req, SieveResult &res,
                       uint8_t *loc_by_edge, hipStream_t stream);

// ------------------------------------------------------------------ static instance
// The static instance of a temporal graph restricted to its live vertices (section
// "Preprocessing", step (ii)): one arc v -> u per ordered pair of live vertices with a
// temporal edge v -> u, v != u, keyed by the smallest input edge id among those
// edges.  Vertices on an arc get compact ids 0..n-1.  Arcs are listed twice: by
// (head, tail) for the forward pass of Eq. (1) and by (tail, head) for the backward
// pass; in each list, seg is the vertex whose row a position adds to, gat the vertex
// whose row it reads.
struct StaticGraph {
    int32_t n = 0;
    int64_t m = 0;
    int32_t *vid = nullptr;                                    // [n] vertex of compact id
    int32_t *in_seg = nullptr, *in_gat = nullptr, *in_key = nullptr;    // [m] by head
    int32_t *out_seg = nullptr, *out_gat = nullptr, *out_key = nullptr; // [m] by tail
};
// vlive: device [G.n], nonzero for live vertices.
void build_static(const Graph &G, const uint8_t *vlive, StaticGraph &S);
void free_static(StaticGraph &S);
// XOR-accumulates S_u (the static vertex-localised sieve: the sum over the 2^k points
// and the k walk positions l of F_{u,l} G_{u,l}) into sv[u] (device, G.n bytes) for
// the vertices of S.  x values are the temporal sieve's (same substitution and seed);
// arc variables y_{arc,l} = fp(seed, 4, l, arc key).  budget: bytes the level rows
// may take (rows get narrower when needed).
void static_sieve(const Graph &G, const StaticGraph &S, const int32_t *M, int32_t k, uint64_t seed,
                  uint8_t *sv, size_t budget, hipStream_t st);

// ------------------------------------------------------------------ multi-query steps
// Per-lane role in a multi-query step (device table, one entry per lane).
struct StepLane {
    uint64_t seed;
    uint32_t ylevel;  // walk position of y at this step = level - 1
    uint32_t flags;   // kLaneActive | kLaneFromX (level 2) | kLaneAcc (last level)
    uint64_t cmask;   // colours a vertex of a matching path can have (bit c); an edge
                      // with an endpoint outside adds nothing for this lane's query
};
// The colours of a multiset as a StepLane mask (every colour with a wildcard entry or
// more than 64 colours).
uint64_t colour_mask(const Graph &G, const int32_t *M, int32_t k);
constexpr uint32_t kLaneActive = 1, kLaneFromX = 2, kLaneAcc = 4;
// bits 8..10 of a lane's flags: its group in the step's fingerprint table (set by the
// library, ignored on input)
constexpr uint32_t kLaneGroupShift = 8;
constexpr int kMaxYGroups = 8;

// A multi-query row: W dwords per lane, `lanes` lanes, buffers from a workspace.
struct MultiRow {
    int W = 1, lanes = 64;
    int rowb() const { return 4 * W * lanes; }
    int parity = 0;  // steps read level buffer `parity` and write the other one
    Workspace *ws = nullptr;
};

// Sizes the buffers of `row` for graph G (W, lanes already set).
void multi_init(const Graph &G, MultiRow &row, hipStream_t st);
// Computes the x rows of query (M, k, seed) for points [base, base + npts) into lanes
// [lane0, lane0 + npts / (4 W)) and clears their accumulators.
void multi_prepare(const Graph &G, MultiRow &row, int lane0, int npts, const int32_t *M, int32_t k,
                   uint64_t seed, uint32_t base, const uint8_t *vertex_mask, hipStream_t st);
// One level for every lane group (lanes[i] for lane i; inactive lanes have flags 0).
void multi_step(const Graph &G, MultiRow &row, const StepLane *lanes, hipStream_t st);
// Device-resident lane tables, per step: 64 lanes, then a header (ylevel = shared
// level, flags = ymode | ngroups << 8), then kMaxYGroups (seed, level) group entries.
constexpr int kTabStride = 64 + 1 + kMaxYGroups;
// Copies the lane tables of nsteps steps (lanes[s * 64 + lane]) into the workspace.
// `lanes` must stay valid until the stream has passed the copy.
void multi_upload_tabs(MultiRow &row, const StepLane *lanes, int nsteps, hipStream_t st);
// nsteps steps whose lane tables were uploaded, replayed from a HIP graph that holds
// the (k_prep, k_step) launches; the graph is captured on first use and again when
// the row's geometry or buffers change.  st must not be the legacy null stream.
struct StepGraph {
    hipGraphExec_t exec = nullptr;
    int W = 0, lanes = 0, nsteps = 0, parity = 0;
    const void *key[8] = {};
    StepGraph() = default;
    StepGraph(const StepGraph &) = delete;
    StepGraph &operator=(const StepGraph &) = delete;
    ~StepGraph();
};
void multi_steps_graph(const Graph &G, MultiRow &row, int nsteps, StepGraph &sg, hipStream_t st);
// Copies the accumulators of lanes [lane0, lane0 + nl) (4 W bytes per lane) to host.
void multi_read(const Graph &G, MultiRow &row, int lane0, int nl, uint8_t *out, hipStream_t st);

// ------------------------------------------------------------------ batch and serving
// Extraction on a hit (batch and serving): vertex localisation + reverse temporal DFS
// (q_loc: the query's own vertex localisation when its sieve computed it), else the
// localisation-guided self-reduction; fills r.path_status and the path.
void extract_into(const Graph &G, const tpm_query &q, tpm_result &r, hipStream_t st,
                  const uint8_t *q_loc = nullptr);
// The continuous-batching engines behind tpm_batch_run: `pruned` runs each query alone
// on the subgraph of its colours, up to `streams` at once; otherwise queries share
// resident multi-query rows of row_points points (use_graph: steps replayed from HIP
// graphs).  Results (and per-point outputs) as tpm_batch_run.
void batch_through_server(const tpm_graph *g, int32_t nq, const tpm_query *q, tpm_result *out,
                          bool pruned, int streams, int row_points, bool use_graph);

// ------------------------------------------------------------------ profiling
bool profile_on();
// brackets a level kernel launch with events when profiling is enabled
struct ProfileScope {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s = nullptr;
    int kind = 0, level = 0, chunk = 0;
    ProfileScope(hipStream_t st, int kind, int level, int chunk);
    ~ProfileScope();
};
// resolves the pending events of this thread (call after the stream is synchronised)
void profile_collect();

}  // namespace tpm

struct tpm_graph {
    tpm::Graph G;
};
