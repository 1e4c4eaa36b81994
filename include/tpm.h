/*
 * tpm.h -- C ABI of the MI355X temporal path-motif sieve (libtpm.so).
 *
 * Problem (paper: Thejaswi, Gionis, Lauri, "Finding path motifs in large
 * temporal graphs using algebraic fingerprints", section "Path problems in
 * temporal graphs", problem PATH-MOTIF): given a directed temporal graph whose
 * vertices carry colours and a multiset M of k colours, decide whether a
 * temporal path (k distinct vertices, k-1 edges with strictly increasing
 * timestamps) exists whose vertex colours are exactly M, and extract one.
 *
 * Method (section "Algebraic algorithm"): evaluate the temporal generating
 * polynomial of Eq. (3) at the 2^k points of the constrained multilinear sieve
 * (Lemma "constrained multilinear sieving", Eq. (motif)) over GF(2^8) with
 * random fingerprints, and XOR the 2^k values into one field element Q.
 * Q != 0 certifies a matching path (no false positives); Q == 0 may be a false
 * negative with probability at most (3k-1)/256 per seed, so decisions repeat
 * with derived seeds.
 *
 * Conventions shared by every call:
 *   - Edge e is (src[e] -> dst[e]) at time tau[e] >= 1; e is its index in the
 *     caller's arrays.  Walks follow edges forward; consecutive edges need
 *     strictly increasing timestamps.  Duplicate edges and self-loops are
 *     accepted (each edge is its own variable; self-loops never lie on a path).
 *   - Field GF(2^8), modulus x^8 + x^4 + x^3 + x^2 + 1 (0x11D).
 *   - Sieve point A in [0, 2^k): bit j of A set <=> label j in A.
 *   - Fingerprints: fp(seed, tag, a, b) = low 8 bits of
 *       mix64(seed ^ mix64((tag << 56) ^ (a << 32) ^ b)),
 *     mix64 = the SplitMix64 output function.  y_{e,l} = fp(seed, 1, l, e)
 *     (walk position l = 1..k-1), v_{u,d} = fp(seed, 2, d, u), w_{d,j} =
 *     fp(seed, 3, d, j).  Slots: the distinct colours of M in ascending order,
 *     colour s owning mu(s) consecutive slot indices d.
 *   - Status codes: 0 = OK, > 0 = a non-error outcome, < 0 = error; on error
 *     tpm_last_error() describes it.  No C++ exception crosses this ABI.
 *   - Host pointers unless stated otherwise.  `hip_stream` arguments take a
 *     hipStream_t (NULL = the default stream).
 *   - A graph handle is immutable after creation; calls on one handle from
 *     several host threads are allowed (each call brings its own workspace).
 */
#ifndef TPM_H
#define TPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tpm_status;

#define TPM_OK 0
#define TPM_NOTFOUND 1   /* extraction: no path found within the repetitions */
#define TPM_PENDING 2    /* server poll: no result ready */
#define TPM_EINVAL (-1)  /* invalid argument or malformed input */
#define TPM_ENOMEM (-2)  /* device or host allocation failed */
#define TPM_EDEVICE (-3) /* HIP runtime error or a kernel-reported fault */
#define TPM_ECANCELLED (-4) /* server: the request was cancelled or passed its deadline */
#define TPM_ECLOSED (-5) /* server is shutting down */

/* graph creation flags */
#define TPM_DEVICE_PTRS 0x1u /* src/dst/tau/color are device pointers */
#define TPM_UNDIRECTED 0x2u  /* edge e is also the arc dst -> src at the same time (and
                                transition time), with input edge id e + m; needs
                                2m < 2^31 - 1 (the paper supports both kinds of graph) */

/* A multiset entry that any vertex may take (section "Including wildcard entries":
 * every vertex also carries one extra colour).  Multisets hold colours in
 * [0, num_colors) and TPM_WILDCARD; the path's vertex colours must equal the multiset
 * after some of them are replaced by wildcards.  Not accepted by tpm_graph_layer. */
#define TPM_WILDCARD (-1)

typedef struct tpm_graph tpm_graph;

/* Options of graph creation.  Zero / NULL fields take the default.
 * tile_edges: T, the work-tile size in CSR positions (1..4096; default
 *             min(1024, max(128, m / 4096)), so that small graphs still have more tiles
 *             than the GPU has waves; subgraphs built from a graph with the default
 *             choose it again for their own m).
 *             In-lists longer than T are cut into pieces of T positions that add the
 *             running value of their predecessors by look-back; shorter ones stay
 *             whole, grouped by the T-aligned window of their first position (a
 *             group spans fewer than 2T positions).
 * tile_held:  reserved, must be 0.
 * transit, delay: the variant with transition and delay times (section "Path motif
 *             problem with delays"); host arrays even with TPM_DEVICE_PTRS.
 *             transit[e] >= 0 (m entries): edge e = (u -> v, tau) reaches v at
 *             tau + transit[e] (< 2^31).  delay[v] >= 0 (n entries): a walk that
 *             reached v at time a may leave it by an edge of timestamp tau only if
 *             a <= tau - delay[v].  Defaults 0 and 1 give the plain problem (strictly
 *             increasing timestamps).  Time outputs (time buckets, optimum time) are
 *             then arrival times. */
typedef struct {
    int32_t tile_edges;
    int32_t tile_held;
    const int32_t *transit;
    const int32_t *delay;
} tpm_graph_options;

typedef struct {
    int32_t n;
    int64_t m;
    int32_t num_colors;
    int32_t tmax;
    int64_t rows;          /* R: CSR positions whose running value a later edge reads */
    int64_t tiles;         /* work tiles */
    int64_t slots;         /* tiles that publish a running value to a successor */
    int64_t max_in_degree;
    int64_t device_bytes;  /* device memory held by the index */
    int64_t gathers;       /* edges whose source has an earlier in-edge (rows read per level) */
    int64_t segments;      /* non-empty in-lists */
    int64_t times;         /* distinct timestamps (length of tpm_time_buckets output) */
    int64_t edge_ids;      /* input edge ids are < edge_ids: m, or the parent's m for a
                              graph made by tpm_graph_prune */
    int32_t tile_edges;    /* work-tile size in use */
} tpm_graph_stats;

/* Per-call tuning.  Every admissible setting gives bit-identical results.
 * chunk:     sieve points per pass (power of two, 4..1024; 0 = min(2^k, 1024));
 *            for tpm_batch_run the row width (256, 512 or 1024; 0 = 1024).
 * use_graph: tpm_batch_run only: 1 = each row step replays its launches from a HIP
 *            graph captured once per row shape (lane tables live in device memory),
 *            on a stream the call creates; 0 = plain launches.
 * prune:     tpm_sieve_ex and tpm_batch_run: 1 = each query runs alone on the
 *            subgraph of its own colours (as tpm_graph_prune; built in memory the
 *            graph keeps for this), which gives the same results; queries with
 *            wildcards run on the whole graph.  tpm_batch_run then runs up to
 *            `streams` such queries at once instead of packing rows. */
typedef struct {
    int32_t chunk;
    int32_t use_graph;
    int32_t prune;
    int32_t streams;  /* tpm_batch_run with prune = 1: queries in flight at once, each on
                         its own HIP stream (0 = 2, at most 4; as the server's pruned
                         mode, one of them sieves at a time) */
} tpm_tuning;

/* ---------------------------------------------------------------- graph --- */
/* Build the device-resident in-edge index of a temporal graph (the edge list of
 * the paper's terminology section, plus the vertex colouring of PATH-MOTIF).
 * n >= 1 vertices, m >= 0 edges (m < 2^31), arrays src/dst/tau of length m,
 * color of length n, 0 <= src, dst < n, tau >= 1, 0 <= color < num_colors.
 * Inputs are copied; with TPM_DEVICE_PTRS they are device pointers on the current
 * device.  `opt` may be NULL.  On success *out owns all device memory.
 * Errors: TPM_EINVAL (bad sizes or values), TPM_ENOMEM, TPM_EDEVICE. */
tpm_status tpm_graph_create(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                            const int32_t *tau, const int32_t *color, int32_t num_colors,
                            uint32_t flags, tpm_graph **out);
tpm_status tpm_graph_create_ex(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                               const int32_t *tau, const int32_t *color, int32_t num_colors,
                               uint32_t flags, const tpm_graph_options *opt, tpm_graph **out);

/* Rebuild the work tiles with at most tile_edges (1..4096) CSR positions each; the
 * sieve's results do not depend on it.  Waits for the device and must not run
 * while another call uses the same graph.  Errors: TPM_EINVAL, TPM_ENOMEM,
 * TPM_EDEVICE (the old tiles are kept on error). */
tpm_status tpm_graph_retile(tpm_graph *g, int32_t tile_edges);

/* Autotuner for the sieve on one graph (the launch shape is this project's, not
 * the paper's).  Times one chunk of a probe query of size k (colours 0, 1, ...,
 * taken modulo num_colors; seed `seed`) for every candidate pair of tile size
 * {256, 512, 1024, 2048} and chunk {256, 512, 1024} (chunks above 2^k dropped; for
 * 2^k < 256 the chunk is 2^k), after one untimed run per pair, and checks that
 * every candidate gives the same per-point bytes.  The fastest tile size is applied
 * to the graph (as tpm_graph_retile) and reported with the fastest chunk; pass
 * that chunk in tpm_tuning.  Same concurrency rule as tpm_graph_retile.  Results are
 * cached by (GPU architecture, k, floor(log2 m), floor(log2 n)) for the process, and in
 * the file named by the environment variable TPM_AUTOTUNE_CACHE when it is set (read
 * at the first call, appended to on each new result); a cached result is applied
 * without timing (cached = 1, no candidates).
 * Errors: TPM_EINVAL (k outside 2..16), TPM_EDEVICE (a candidate disagreed). */
typedef struct {
    int32_t tile_edges;      /* chosen and applied */
    int32_t chunk;           /* chosen */
    int32_t ncand;           /* candidates timed (<= 12) */
    int32_t cand_tile[12];
    int32_t cand_chunk[12];
    double cand_rate[12];    /* edge-level-point updates per second: m (k-1) C / time */
    int32_t cached;          /* 1: taken from the autotune cache, nothing timed */
} tpm_autotune_report;
tpm_status tpm_autotune(tpm_graph *g, int32_t k, uint64_t seed, tpm_autotune_report *out);

/* Colour pruning (the paper's preprocessing step (i), section "Implementation"): a
 * new graph holding the edges of g whose two endpoints both have a colour in
 * colors[0..ncolors).  Vertex ids, colours and input edge ids (those of g) are kept,
 * so for a multiset whose colours are all in the set every result (per-point values,
 * totals, localisation, extraction) equals g's bit for bit: a vertex of another
 * colour has z = 0 and no walk through it contributes.  Built on the device from
 * g's sorted index (no sort).  The new graph is independent of g afterwards.
 * Errors: TPM_EINVAL (colour out of range, ncolors < 1), TPM_ENOMEM, TPM_EDEVICE. */
tpm_status tpm_graph_prune(const tpm_graph *g, const int32_t *colors, int32_t ncolors,
                           tpm_graph **out);

/* As tpm_graph_prune, with an optional colour set (ncolors = 0: every colour) and an
 * optional timestamp set times[0..ntimes) (ntimes = 0: every timestamp; edges are
 * matched by their own timestamp, i.e. departure).  With the k - 1 timestamps
 * j_1 < ... < j_{k-1} of an EC-PATH-MOTIF query (section "Extending the framework":
 * edges at prescribed times, in order) the plain sieve on the result decides that
 * query: k - 1 strictly increasing times from a set of k - 1 values are that set in
 * order.  (With transition or delay times the kept edges follow the graph's rule.) */
tpm_status tpm_graph_prune_ex(const tpm_graph *g, const int32_t *colors, int32_t ncolors,
                              const int32_t *times, int32_t ntimes, tpm_graph **out);

/* VC-PATH-MOTIF (section "Extending the framework": the path's vertex colours must be
 * tuple[0], ..., tuple[k-1] in this order).  Builds a layered graph: one vertex per
 * (layer l, vertex u with colour tuple[l-1]) and the edges (v, l-1) -> (u, l) of g's
 * edges v -> u with colours (tuple[l-2], tuple[l-1]), with their timestamps,
 * transition / delay times and input edge ids.  Every copy of u keeps u's
 * fingerprints, so sieving the result with the tuple as multiset evaluates the paper's
 * VC polynomial (level-l vertices and edges restricted by colour): a nonzero total
 * certifies a temporal path whose l-th vertex has colour tuple[l-1].  Its vertex ids
 * are layer copies (map them with tpm_graph_vertex_ids); tpm_extract on it deletes
 * every copy of a picked vertex and returns original vertex ids.  Only the edges
 * between consecutive layers are kept, so it is about (k-1)/q^2 of g for q colours.
 * Errors: TPM_EINVAL (k outside 1..16, colour out of range), TPM_ENOMEM, TPM_EDEVICE. */
tpm_status tpm_graph_layer(const tpm_graph *g, const int32_t *tuple, int32_t k, tpm_graph **out);

/* (s,d)-COLORFUL-PATH (section "Solving COLORFUL-PATH and (s,d)-COLORFUL-PATH"): the
 * instance in which s gets the new colour num_colors and d the new colour
 * num_colors + 1 (the result has num_colors + 2 colours), s loses its in-edges and d
 * its out-edges.  Sieving it with M' = M + {num_colors, num_colors + 1} (k + 2 entries)
 * decides whether a temporal path s -> ... -> d exists whose k internal vertices have
 * the colours M: the new colours put s and d on the path exactly once, and the removed
 * edges make them its first and last vertex.  Every other vertex, edge, timestamp,
 * transition / delay time and input edge id is g's; tpm_extract on it returns such a
 * path.  Errors: TPM_EINVAL (s or d out of range, s == d), TPM_ENOMEM, TPM_EDEVICE. */
tpm_status tpm_graph_sd(const tpm_graph *g, int32_t s, int32_t d, tpm_graph **out);

/* ids[i] = the vertex of the original graph that vertex i stands for (n entries:
 * identity, except for graphs made by tpm_graph_layer). */
tpm_status tpm_graph_vertex_ids(const tpm_graph *g, int32_t *ids);

/* Free a graph and everything it owns.  NULL is accepted. */
void tpm_graph_destroy(tpm_graph *g);

/* Sizes of a built index.  Errors: TPM_EINVAL. */
tpm_status tpm_graph_stats_get(const tpm_graph *g, tpm_graph_stats *out);

/* ---------------------------------------------------------------- sieve --- */
/* Evaluate the sieve for one query (Lemma "constrained multilinear sieving"):
 * per_point[A] = P_{k,t}(z^A) for A in [0, 2^k) (nullable, 2^k bytes) and
 * *total = XOR of all of them (nullable).  multiset: k colour ids, 1 <= k <= 16.
 * vertex_mask (nullable, n bytes): 0 deletes the vertex (its variable x_u = 0).
 * Blocks until the results are on the host.
 * Errors: TPM_EINVAL (k out of range, colour out of range), TPM_ENOMEM,
 * TPM_EDEVICE. */
tpm_status tpm_sieve(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                     const uint8_t *vertex_mask, uint8_t *per_point, uint8_t *total,
                     void *hip_stream);

/* As tpm_sieve, plus tuning (nullable) and the per-edge localisation
 * loc[e] = sum over A of the level-k term of edge e (nullable; tpm_graph_stats.edge_ids
 * bytes indexed by input edge id, zero for ids not in the graph): loc[e] != 0
 * certifies a matching path whose last edge is e (the edge-level form of the
 * paper's vertex-localisation). */
tpm_status tpm_sieve_ex(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                        const uint8_t *vertex_mask, const tpm_tuning *tune, uint8_t *per_point,
                        uint8_t *total, uint8_t *loc, void *hip_stream);

/* tpm_sieve for callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops and harnesses that must not call hipMalloc.  Computes what
 * tpm_sieve computes (no vertex mask) and allocates nothing: every buffer of the query
 * lives in one fixed block of 256 MiB of device memory per GPU, reserved when the
 * library's code is loaded on that GPU and held until the process ends.  Rows are the
 * widest power of two of sieve points (16 .. 1024) whose buffers fit the block; graphs
 * whose state does not fit even 16-point rows (about 32 (n + R + S) bytes for k >= 3,
 * R and S = rows and slots of tpm_graph_stats) are refused with TPM_ENOMEM.
 * Asynchronous: only enqueues work on hip_stream (NULL = the default stream) and
 * returns; the outputs are DEVICE pointers, valid once the stream has reached them:
 *   total        1 byte, the XOR of all 2^k sieve values (required);
 *   per_point    2^k bytes, per_point[A] = P_{k,t}(z^A) (nullable);
 *   error_flags  4 bytes, 0, or nonzero if the kernels reported a look-back failure
 *                (the results are then invalid) (nullable).
 * Every call on one GPU uses that GPU's block, and a call's buffers keep their contents
 * until the next call: calls that overlap on one GPU (other host threads, or other
 * streams whose work has not finished) race and give wrong results; serialise them.
 * multiset is a host pointer, read before the call returns.
 * Errors: TPM_EINVAL (NULL graph or total, k out of range, colour out of range),
 * TPM_ENOMEM (the state does not fit the block), TPM_EDEVICE. */
tpm_status tpm_sieve_noalloc(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                             uint8_t *per_point, uint8_t *total, uint32_t *error_flags,
                             void *hip_stream);

/* Decide PATH-MOTIF: run up to `reps` sieves with seeds seed_r = seed + r *
 * 0x9E3779B97F4A7C15 and stop at the first nonzero total.  *found = 1 is
 * certain; *found = 0 means no sieve detected a path.  reps >= 1. */
tpm_status tpm_decide(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                      int32_t reps, int32_t *found);

/* Extract a matching temporal path (section "Extracting a solution"): first the
 * vertex-localisation approach (tpm_extract_ex method 2, with a DFS budget of 5e6
 * edge visits), then, if that finds nothing, the localisation-guided self-reduction
 * (method 0: localise the last edge (u' -> u, tau), delete u, drop c(u) from M, and
 * repeat on the in-edges of u' earlier than tau until one vertex is left).
 * On TPM_OK, path_vertices[0..k) and path_edges[0..k-1) (input edge ids) hold a
 * path that the library has verified (strictly increasing times, distinct
 * vertices, colours = M).  TPM_NOTFOUND: no path found within max_reps seeds
 * per step.  Deterministic for a fixed seed. */
tpm_status tpm_extract(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                       int32_t max_reps, int32_t *path_vertices, int64_t *path_edges);

/* As tpm_extract with a choice of method, and the number of sieves run (nullable).
 * method 0: the localisation-guided self-reduction (about k sieves).
 * method 1: the paper's self-reducibility (section "Extracting a solution", first
 *           approach): vertices of other colours are dropped, then vertex groups are
 *           deleted while a decision (max_reps sieves) stays YES, halving groups that
 *           cannot go (O(k log n) decisions), and a temporal DFS over the surviving
 *           vertices returns the path.  k >= 2.
 * method 2: the paper's vertex-localisation approach (same section, second
 *           approach): one localised sieve per seed gives the vertices u with a
 *           nonzero Q_u (tpm_sieve_vertex), each certified to end a matching path;
 *           from them, smallest id first, a reverse temporal DFS (in-edges by
 *           decreasing arrival, distinct vertices, colours from what is left of M)
 *           returns a path.  The DFS is exhaustive per end vertex within a budget of
 *           5e7 edge visits per call (TPM_NOTFOUND when it runs out).  k >= 2.
 * For k = 1 every method returns a vertex of the colour. */
tpm_status tpm_extract_ex(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                          int32_t max_reps, int32_t method, int32_t *path_vertices,
                          int64_t *path_edges, int64_t *sieves);

/* ------------------------------------------------------ localised sieves --- */
/* Vertex-localised sieve (section "Vertex-localization"): q[u] = sum over all 2^k
 * sieve points A of P_{u,k,t}(z^A), for every vertex u (q: n bytes, host).  q[u] != 0
 * certifies a matching temporal path that ends at u; the q[u] XOR to the sieve total.
 * Computed from the per-edge localisation (XOR over u's in-edges).  2 <= k <= 16;
 * vertex_mask as tpm_sieve.  Errors: TPM_EINVAL, TPM_ENOMEM, TPM_EDEVICE. */
tpm_status tpm_sieve_vertex(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                            const uint8_t *vertex_mask, uint8_t *q);

/* The sieve split by the time of a walk's last edge: times[i] = i-th distinct
 * timestamp (ascending), buckets[i] = XOR of the per-edge localisation over the
 * edges with timestamp times[i].  The XOR of buckets[0..i] is the sieve over walks
 * whose edges all have timestamps <= times[i].  Both arrays hold
 * tpm_graph_stats.times entries (host).  2 <= k <= 16. */
tpm_status tpm_time_buckets(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                            int32_t *times, uint8_t *buckets);

/* Optimum timestamp (section "Finding optimum timestamp"): the smallest t such that
 * the sieve over walks finishing by t is nonzero, minimised over `reps` seeds
 * seed_r = seed + r * 0x9E3779B97F4A7C15 (one localised sieve per seed instead of a
 * binary search of decides); *t_out = -1 if no seed found a path.  A returned t is
 * certain (a matching path with all timestamps <= t exists); it exceeds the optimum
 * only if every seed misses the optimal paths (one-sided error, as decide). */
tpm_status tpm_optimum_time(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                            int32_t reps, int32_t *t_out);

/* Static vertex-localised sieve (section "Preprocessing", step (ii), on the static
 * generating polynomial Eq. (1)).  The static instance has one arc v -> u per ordered
 * pair of vertices joined by a temporal edge (v != u), whose variables y_{vu,l} are
 * keyed by the smallest input edge id among those edges; x_u is the temporal
 * sieve's.  s[u] (host, n bytes) = sum over the 2^k points and the k walk positions l
 * of F_{u,l} G_{u,l}, where F runs Eq. (1) forward from F_{u,1} = x_u and G runs the
 * same walks backward from G_{u,k} = 1: the sieve of the k-vertex walks through u,
 * counted once per visit.  Paths through u count once and all other walks cancel,
 * so s[u] != 0 certifies a static path through u whose colours match the multiset
 * (and every temporal match is a static one).  1 <= k <= 16.
 * Errors: TPM_EINVAL, TPM_ENOMEM, TPM_EDEVICE. */
tpm_status tpm_static_sieve(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                            uint8_t *s);

/* Preprocessing steps (i) and (ii) together: the subgraph of g on the vertices u with
 * s[u] != 0 for some of `reps` seeds seed_r = seed + r * 0x9E3779B97F4A7C15
 * (tpm_static_sieve; a vertex of a colour outside the multiset always has s[u] = 0).
 * Vertex ids, colours, timestamps and input edge ids are g's.  When every vertex of
 * every temporal match is kept, the sieve total of the multiset on the result equals
 * g's for every seed; a vertex of a match is dropped only if all `reps` static sieves
 * miss it (probability at most ((2k - 1) / 256)^reps per vertex, the one-sided error
 * of the sieve).  Errors: TPM_EINVAL (bad multiset, reps < 1), TPM_ENOMEM,
 * TPM_EDEVICE. */
tpm_status tpm_graph_prune_static(const tpm_graph *g, const int32_t *multiset, int32_t k,
                                  uint64_t seed, int32_t reps, tpm_graph **out);

/* An optimum solution (sections "Finding optimum timestamp" and "Extracting a
 * solution"): *t_out = tpm_optimum_time(g, multiset, k, seed, reps); then a path is
 * extracted by `method` (as tpm_extract_ex, max_reps = reps, seeds derived from seed)
 * on the subgraph of the edges that arrive by *t_out, so the path finishes by *t_out,
 * the earliest finishing time unless every seed missed the earliest paths.  Returns
 * TPM_NOTFOUND with *t_out = -1 when no seed finds a path, or when extraction misses on
 * the subgraph.  2 <= k <= 16.  Errors: TPM_EINVAL, TPM_ENOMEM, TPM_EDEVICE. */
tpm_status tpm_extract_optimum(const tpm_graph *g, const int32_t *multiset, int32_t k,
                               uint64_t seed, int32_t reps, int32_t method, int32_t *t_out,
                               int32_t *path_vertices, int64_t *path_edges);

/* ---------------------------------------------------------------- batch --- */
typedef struct {
    const int32_t *multiset; /* k colours */
    int32_t k;
    uint64_t seed;
    int32_t want_path;       /* 1: extract a path when the sieve is nonzero */
    uint8_t *per_point;      /* nullable, host, 2^k bytes: receives P_{k,t}(z^A) for every
                                sieve point A, as tpm_sieve's per_point.  tpm_batch_run
                                writes it before returning; a server writes it before
                                tpm_server_poll hands out the result, so the buffer must
                                stay valid until then (it is left alone on a result whose
                                status is not TPM_OK) */
    double deadline_ms;      /* server only: the request ends with status TPM_ECANCELLED
                                if it has not finished this many ms after its submission
                                (checked while queued and between level launches; 0 =
                                no deadline) */
} tpm_query;

typedef struct {
    int32_t status;          /* TPM_OK, or (server) TPM_ECANCELLED (tpm_server_cancel or
                                the deadline), TPM_ENOMEM (the request did not fit the
                                state budget even alone), TPM_EDEVICE (a device error) */
    int32_t found;           /* 1 iff the sieve total was nonzero */
    uint8_t total;
    int32_t path_status;     /* TPM_OK / TPM_NOTFOUND / 0 when not requested */
    int32_t path_vertices[16];
    int64_t path_edges[15];
    uint64_t ticket;         /* server: the submit ticket */
    double t_submit_ms, t_start_ms, t_done_ms; /* server: host clock, ms */
} tpm_result;

/* Run nq queries against one graph.  Each result is bit-identical to the same
 * query run alone through tpm_sieve (same seed), per point when the query asks for
 * per-point output.  Without pruning the queries share resident multi-query rows
 * (lane groups of any k side by side; a finished group's lanes are refilled from the
 * queries still waiting, largest first); with tune->prune each query runs alone on
 * the subgraph of its colours, up to tune->streams at once on their own streams and
 * within a device-memory budget (85 % of the memory free at the call), as the
 * server's pruned mode.  tune may be
 * NULL.  Errors: TPM_EINVAL (bad query or tuning), TPM_ENOMEM, TPM_EDEVICE. */
tpm_status tpm_batch_run(const tpm_graph *g, int32_t nq, const tpm_query *q, tpm_result *out,
                         const tpm_tuning *tune);

/* RAINBOW-PATH (section "Extending the framework"): is there a temporal path with k
 * vertices of k different colours?  Decided, as in the paper, by the PATH-MOTIF
 * oracle over the C(num_colors, k) colour sets, here run as packed batches of up to
 * 256 queries with reps seeds each (seed_r as tpm_decide), stopping at the first hit.
 * On *found = 1, colors[0..k) holds a colour set with a path (certain); *found = 0:
 * no set was detected.  C(num_colors, k) must not exceed 2^20.
 * Errors: TPM_EINVAL (k outside 1..16 or > num_colors, too many sets). */
tpm_status tpm_rainbow_decide(const tpm_graph *g, int32_t k, uint64_t seed, int32_t reps,
                              int32_t *found, int32_t *colors);

/* ---------------------------------------------------------------- serve --- */
typedef struct tpm_server tpm_server;

/* Two modes, both continuous batching: requests that arrive while others run are
 * admitted as lanes or memory free up, and their work overlaps on the device.
 *   Row mode (prune_queries = 0): one resident multi-query row of up to 64 lanes over
 *     the whole graph; every row step advances each lane group one level, finished
 *     groups free their lanes and waiting requests (any that fit, not only the oldest)
 *     take them at the next step.  Extraction runs on its own thread and stream.
 *   Pruned mode (prune_queries = 1): each request runs alone on the subgraph of its
 *     colours (as tpm_graph_prune), up to `streams` requests at once, each on its own
 *     HIP stream and worker thread with a fixed share (budget / streams) of the state
 *     budget: a request takes the widest chunk of sieve points whose estimated device
 *     memory (subgraph index and sieve state, from the exact edge count of its colour
 *     pairs) fits the share; one larger than a share waits for the device to itself
 *     and may be overtaken by later requests at most 8 times.  One worker uses the
 *     device at a time (subgraph build and sieve; every such phase is bound by HBM
 *     bandwidth, and two at once measured slower than one after the other) while the
 *     others admit requests and extract paths on the host.  Admission takes the request
 *     with the least estimated device work first, unless the oldest has waited 750 ms.
 *     Extraction on a hit is the reverse DFS from the deciding sieve's own vertex
 *     localisation.
 * Results are identical in both modes, to the same query run alone. */
typedef struct {
    int64_t state_bytes;   /* device memory the server may use for query state (0 = 85 %
                              of the memory free at creation); pruned mode rejects a
                              request whose smallest state cannot fit it */
    int32_t max_lanes;     /* row mode: most sieve lanes resident at once (0 = auto) */
    int32_t extract_paths; /* 1: extract a witness for every YES */
    int32_t prune_queries; /* 1: pruned mode (above) */
    int32_t streams;       /* pruned mode: requests in flight at once (0 = 2; 1..4) */
} tpm_server_config;

tpm_status tpm_server_create(const tpm_graph *g, const tpm_server_config *cfg, tpm_server **out);
/* Queue a request (the multiset is copied).  Errors: TPM_EINVAL (bad query),
 * TPM_ENOMEM (pruned mode: the request cannot fit the state budget even alone),
 * TPM_ECLOSED, TPM_EDEVICE (the server stopped on a device error). */
tpm_status tpm_server_submit(tpm_server *s, const tpm_query *q, uint64_t *ticket);
/* Copy up to max finished results into out; *n_out = how many. TPM_PENDING if
 * none is ready yet. */
tpm_status tpm_server_poll(tpm_server *s, tpm_result *out, int32_t max, int32_t *n_out);
/* Cancel a request that has not finished: it ends with status TPM_ECANCELLED (a queued
 * request at once, a running one at its next level launch or row step).  TPM_NOTFOUND
 * if the ticket is unknown or its result is already out. */
tpm_status tpm_server_cancel(tpm_server *s, uint64_t ticket);
void tpm_server_destroy(tpm_server *s);

/* Counters of a server since creation (host clock, ms). */
typedef struct {
    int64_t completed;     /* results produced (every status) */
    int64_t steps;         /* row steps (row mode) or requests run (pruned mode) */
    int32_t row_points;    /* sieve points per resident row (row mode), else 0 */
    int32_t lanes;         /* lanes of the resident row (row mode), else 0 */
    double prune_ms;       /* building per-request subgraphs (pruned mode; summed over
                              streams) */
    double sieve_ms;       /* sieving: row steps, or per-request sieves (summed) */
    double extract_ms;     /* witness extraction (summed) */
    int64_t cancelled;     /* results with status TPM_ECANCELLED */
    int64_t rejected;      /* submissions refused with TPM_ENOMEM, plus results with
                              status TPM_ENOMEM */
    int32_t streams;       /* pruned mode: worker streams */
    int32_t inflight_peak; /* most requests running at once */
    int64_t budget_bytes;  /* state budget */
    int64_t held_bytes_peak; /* pruned mode: most device bytes held by the workers */
    int64_t trims;         /* pruned mode: times a worker released its device memory
                              (after a request larger than its share of the budget) */
    double gpu_wait_ms;    /* pruned mode: time workers waited for the device (one
                              request uses it at a time; summed) */
    int32_t queued;        /* requests waiting for admission now */
    int32_t queued_peak;   /* most requests waiting for admission at once */
    int32_t inflight;      /* requests admitted and not finished now */
    int32_t pad;
} tpm_server_stats;
tpm_status tpm_server_stats_get(tpm_server *s, tpm_server_stats *out);

/* ---------------------------------------------------------- diagnostics --- */
/* When enabled (process-wide), every sieve level kernel is bracketed by HIP events
 * recorded on the stream it is launched on; tpm_profile_read drains the measured
 * durations.  kind: 0 = level 2 (reads the per-vertex rows), 1 = a middle level
 * (3..k-1), 2 = the last level (reduction), 3 = a multi-query step (batched form
 * with plain launches, serving loop; chunk_points = row width).  Timing adds no
 * device work. */
typedef struct {
    int32_t kind;
    int32_t level;
    int32_t chunk_points;  /* sieve points per pass */
    int32_t pad;
    double ms;
} tpm_kernel_time;

tpm_status tpm_profile_enable(int32_t on);
tpm_status tpm_profile_read(tpm_kernel_time *out, int32_t max, int32_t *n_out);

/* A plain streaming read of `bytes` bytes of device memory at `src` (16-byte aligned,
 * bytes a multiple of 16), each byte read once with 16-byte loads, for scaling
 * profiler traffic counters against a kernel of known size; *out (device, 8 bytes)
 * receives the XOR of the buffer's 8-byte words.  Enqueued on hip_stream (NULL = the
 * default stream).  Errors: TPM_EINVAL (NULL, misaligned or bad size), TPM_EDEVICE. */
tpm_status tpm_stream_read(const void *src, int64_t bytes, uint64_t *out, void *hip_stream);

/* ---------------------------------------------------------------- misc --- */
/* Description of the last error on the calling thread ("" if none). */
const char *tpm_last_error(void);

/* Library version string. */
const char *tpm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TPM_H */
