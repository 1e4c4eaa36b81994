/*
 * tpm_oracle.c -- CPU oracle for constrained multilinear sieving of temporal
 * path motifs (Thejaswi, Gionis, Lauri: "Finding path motifs in large temporal
 * graphs using algebraic fingerprints").
 *
 * TEST INFRASTRUCTURE ONLY.  Loaded by the test-suite, by the smoke check and by
 * the bench's CPU-baseline leg.  The product library never links, loads or calls
 * it, and it shares no code, header or table with the product library.
 *
 * What it computes (all arithmetic exact, in GF(2^8)):
 *   For a vertex-coloured directed temporal graph (edge e = (src_e, dst_e, tau_e),
 *   e = index in the caller's arrays), a colour multiset M of size k and a
 *   fingerprint seed, the value P(A) of the temporal generating polynomial
 *   (Eq. (3), section "Generating polynomial for temporal walks") at the sieve
 *   point A (section "Multilinear sieving", Lemma on multilinear sieving), with
 *   the constrained substitution z_{u,j} = sum_{d in S_c(u)} v_{u,d} w_{d,j}
 *   (Eq. (motif), Lemma on constrained multilinear sieving).  The sum of P(A)
 *   over all 2^k points is the sieve value Q; Q != 0 certifies a temporal path
 *   whose colours equal M.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - v is in N_i(u) iff the directed edge (v -> u, i) exists: walks follow
 *     edges forward.
 *   - P_{u,1,0} = x_u (a first edge at time 1 is allowed; the worked example's
 *     level-2, time-1 panel shows it); P_{u,l,0} = 0 for l >= 2.
 *   - Every input edge is its own variable: y is keyed by (input index e,
 *     walk position l), l = 1..k-1.
 *   - Slots: the distinct colours of M in ascending order, colour s owning
 *     mu(s) consecutive slot indices; labels are 0..k-1; bit j of A <=> j in A.
 *   - The field is GF(2^8) with modulus x^8+x^4+x^3+x^2+1 (0x11D).
 *   - Fingerprints: low byte of SplitMix64's output mix (Steele, Lea, Flood,
 *     OOPSLA 2014) applied twice:
 *       fp(seed, tag, a, b) = low8(mix64(seed ^ mix64((tag<<56) ^ (a<<32) ^ b)))
 *     with tag 1 = y (a = l, b = e), 2 = v (a = d, b = u), 3 = w (a = d, b = j).
 *
 * The evaluation is Eq. (3) written edge by edge: P_{u,l,.} only changes at the
 * times of u's in-edges, so with c_l[e] = x_{dst_e} * y_{e,l-1} * P_{src_e,l-1,tau_e-1}
 * one has P_{v,l-1,tau-1} = sum of c_{l-1}[e'] over in-edges e' of v with
 * tau' < tau (for l-1 >= 2; x_v for l-1 = 1), and P_{k,t} = sum_e c_k[e].
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ------------------------------------------------------------------------- */
/* GF(2^8): addition is XOR; multiplication is the carry-less product reduced  */
/* modulo x^8 + x^4 + x^3 + x^2 + 1, here done bit by bit (shift and add).     */
/* ------------------------------------------------------------------------- */
uint8_t or_gf_mul_bits(uint8_t a, uint8_t b)
{
    uint8_t r = 0;
    for (int i = 0; i < 8; i++) {
        if (b & 1u)
            r ^= a;
        int carry = (a & 0x80u) != 0;
        a = (uint8_t)(a << 1);
        if (carry)
            a ^= 0x1Du; /* x^8 = x^4 + x^3 + x^2 + 1 */
        b >>= 1;
    }
    return r;
}

/* The same function tabulated (so the slow evaluations stay affordable). */
static uint8_t OR_MUL[256][256];
static int or_ready = 0;

void or_init(void)
{
    if (or_ready)
        return;
    for (int a = 0; a < 256; a++)
        for (int b = 0; b < 256; b++)
            OR_MUL[a][b] = or_gf_mul_bits((uint8_t)a, (uint8_t)b);
    or_ready = 1;
}

uint8_t or_gf_mul(uint8_t a, uint8_t b) { return OR_MUL[a][b]; }

void or_mul_table(uint8_t *out /* 65536 */) { memcpy(out, OR_MUL, sizeof(OR_MUL)); }

/* ------------------------------------------------------------------------- */
/* Fingerprints.                                                               */
/* ------------------------------------------------------------------------- */
uint64_t or_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint8_t or_fp(uint64_t seed, uint32_t tag, uint32_t a, uint32_t b)
{
    uint64_t key = ((uint64_t)tag << 56) ^ ((uint64_t)a << 32) ^ (uint64_t)b;
    return (uint8_t)(or_mix64(seed ^ or_mix64(key)) & 0xFFu);
}

/* ------------------------------------------------------------------------- */
/* Slots S_s and the substitution z (Eq. (motif)).                             */
/* ------------------------------------------------------------------------- */
/* Colour s (0 <= s < q) gets mu[s] slots starting at off[s]; colours not in M
 * get mu = 0.  Entries -1 of M are wildcards (section "Including wildcard entries":
 * every vertex also has an extra colour); they take the first slots, 0 .. wc - 1,
 * since the slots follow the colours of M in ascending order.  Returns -1 if M names
 * a colour outside [-1, q). */
int or_wildcards(const int32_t *M, int32_t k)
{
    int wc = 0;
    for (int i = 0; i < k; i++)
        wc += M[i] == -1;
    return wc;
}

int or_slots(const int32_t *M, int32_t k, int32_t q, int32_t *off, int32_t *mu)
{
    for (int s = 0; s < q; s++) {
        mu[s] = 0;
        off[s] = -1;
    }
    for (int i = 0; i < k; i++) {
        if (M[i] < -1 || M[i] >= q)
            return -1;
        if (M[i] >= 0)
            mu[M[i]]++;
    }
    int next = or_wildcards(M, k);
    for (int s = 0; s < q; s++) {
        if (mu[s]) {
            off[s] = next;
            next += mu[s];
        }
    }
    return 0;
}

/* z[u*k + j] = sum over d in S_c(u), and over the wildcard slots, of v_{u,d} w_{d,j};
 * zero when the vertex is deleted (mask[u] == 0) or has no slot. */
int or_z(int32_t n, const int32_t *color, int32_t q, const int32_t *M, int32_t k,
         uint64_t seed, const uint8_t *mask, uint8_t *z)
{
    or_init();
    int32_t *off = malloc(sizeof(int32_t) * (size_t)q);
    int32_t *mu = malloc(sizeof(int32_t) * (size_t)q);
    if (!off || !mu || or_slots(M, k, q, off, mu)) {
        free(off);
        free(mu);
        return -1;
    }
    uint8_t w[16][16];
    for (int d = 0; d < k; d++)
        for (int j = 0; j < k; j++)
            w[d][j] = or_fp(seed, 3, (uint32_t)d, (uint32_t)j);
    const int wc = or_wildcards(M, k);
    for (int32_t u = 0; u < n; u++) {
        int32_t c = color[u];
        for (int j = 0; j < k; j++)
            z[(size_t)u * k + j] = 0;
        if (mask && !mask[u])
            continue;
        const int own = (c >= 0 && c < q) ? mu[c] : 0;
        if (own == 0 && wc == 0)
            continue;
        for (int j = 0; j < k; j++) {
            uint8_t acc = 0;
            for (int d = 0; d < wc; d++)
                acc ^= OR_MUL[or_fp(seed, 2, (uint32_t)d, (uint32_t)u)][w[d][j]];
            for (int d = own ? off[c] : 0; d < (own ? off[c] + own : 0); d++)
                acc ^= OR_MUL[or_fp(seed, 2, (uint32_t)d, (uint32_t)u)][w[d][j]];
            z[(size_t)u * k + j] = acc;
        }
    }
    free(off);
    free(mu);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* In-edge lists sorted by time, and the predecessor position of every edge.  */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t n;
    int64_t m;
    const int32_t *src, *dst, *tau;
    int32_t *arr;   /* [m] arrival times tau + transit (owned; NULL when arrival = tau) */
    int64_t *start; /* [n+1]: in-list of v is order[start[v] .. start[v+1]) */
    int64_t *order; /* [m]: edge ids, grouped by dst, each group by (arrival, id) */
    int64_t *gpos;  /* [m]: position in `order` of the last in-edge e' of src_e whose
                       arrival is <= tau_e - delay(src_e) (delay 1: arrival < tau_e),
                       or -1 if there is none */
    const uint8_t *emask; /* [m] or NULL (borrowed): emask[e] == 0 removes edge e from
                             the graph (it keeps its index, so y of the others is as is) */
    const int32_t *eid;   /* [m] or NULL (borrowed): the fingerprint key of edge e (its
                             index in a larger graph this one keeps some edges of) */
} or_index;

static const int32_t *g_cmp_tau;
static int cmp_by_tau_then_id(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    if (g_cmp_tau[a] != g_cmp_tau[b])
        return g_cmp_tau[a] < g_cmp_tau[b] ? -1 : 1;
    return a < b ? -1 : (a > b);
}

void or_index_free(or_index *ix)
{
    if (!ix)
        return;
    free(ix->start);
    free(ix->order);
    free(ix->gpos);
    free(ix->arr);
    free(ix);
}

/* Section "Path motif problem with delays": an edge (v -> u, tau) with transition
 * time eps reaches u at tau + eps, and a walk may leave a vertex w at time tau only
 * if it arrived at w by tau - delay(w).  transit (per edge, >= 0) and delay (per
 * vertex, >= 0) are nullable: no transit means arrival = tau, no delay means 1 (the
 * strictly increasing times of the plain problem).  The arrays are borrowed and must
 * outlive the index. */
or_index *or_index_build_ex(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                            const int32_t *tau, const int32_t *transit, const int32_t *delay)
{
    or_index *ix = calloc(1, sizeof(or_index));
    if (!ix)
        return NULL;
    ix->n = n;
    ix->m = m;
    ix->src = src;
    ix->dst = dst;
    ix->tau = tau;
    const int32_t *arr = tau;
    if (transit) {
        ix->arr = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
        if (!ix->arr) {
            free(ix);
            return NULL;
        }
        for (int64_t e = 0; e < m; e++)
            ix->arr[e] = tau[e] + transit[e];
        arr = ix->arr;
    }
    ix->start = calloc((size_t)n + 1, sizeof(int64_t));
    ix->order = malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    ix->gpos = malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    if (!ix->start || !ix->order || !ix->gpos) {
        or_index_free(ix);
        return NULL;
    }
    for (int64_t e = 0; e < m; e++)
        ix->start[dst[e] + 1]++;
    for (int32_t v = 0; v < n; v++)
        ix->start[v + 1] += ix->start[v];
    int64_t *fill = malloc(sizeof(int64_t) * ((size_t)n + 1));
    memcpy(fill, ix->start, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t e = 0; e < m; e++)
        ix->order[fill[dst[e]]++] = e;
    free(fill);
    g_cmp_tau = arr; /* single-threaded build */
    for (int32_t v = 0; v < n; v++)
        qsort(ix->order + ix->start[v], (size_t)(ix->start[v + 1] - ix->start[v]),
              sizeof(int64_t), cmp_by_tau_then_id);
    for (int64_t e = 0; e < m; e++) {
        int32_t v = src[e];
        /* in-edges of v that arrived by tau_e - delay(v): arrival < th */
        int64_t th = (int64_t)tau[e] - (delay ? delay[v] : 1) + 1;
        int64_t lo = ix->start[v], hi = ix->start[v + 1]; /* first position with arrival >= th */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if ((int64_t)arr[ix->order[mid]] < th)
                lo = mid + 1;
            else
                hi = mid;
        }
        ix->gpos[e] = (lo > ix->start[v]) ? lo - 1 : -1;
    }
    return ix;
}

or_index *or_index_build(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                         const int32_t *tau)
{
    return or_index_build_ex(n, m, src, dst, tau, NULL, NULL);
}

/* y_{e,l} of the edge at index e is keyed by eid[e] instead of e (borrowed). */
void or_index_set_eid(or_index *ix, const int32_t *eid)
{
    ix->eid = eid;
}

/* ------------------------------------------------------------------------- */
/* Evaluation of P(A) (Eq. (3)) at a list of sieve points.                     */
/* ------------------------------------------------------------------------- */
/* z: [n*k] from or_z.  y is drawn here, per (walk position l, edge e).
 * out[i] = P(points[i]).  loc (nullable, [m]) receives, XOR-ed over the given
 * points, the contribution c_k[e] of walks whose last edge is e (the per-edge
 * form of vertex-localisation).  nthreads <= 0: OpenMP default. */
/* vc (nullable, k colours) with color: the VC-PATH-MOTIF polynomial (section "Extending
 * the framework"): P_{u,1} = x_u only if c(u) = vc[0], and level l takes only edges
 * (v -> u) with c(v) = vc[l-2], c(u) = vc[l-1]. */
static int or_eval_impl(const or_index *ix, const uint8_t *z, int32_t k, uint64_t seed,
                        const uint32_t *points, int64_t npoints, uint8_t *out, uint8_t *loc,
                        int nthreads, const int32_t *vc, const int32_t *color);

int or_eval(const or_index *ix, const uint8_t *z, int32_t k, uint64_t seed,
            const uint32_t *points, int64_t npoints, uint8_t *out, uint8_t *loc, int nthreads)
{
    return or_eval_impl(ix, z, k, seed, points, npoints, out, loc, nthreads, NULL, NULL);
}

static int or_eval_impl(const or_index *ix, const uint8_t *z, int32_t k, uint64_t seed,
                        const uint32_t *points, int64_t npoints, uint8_t *out, uint8_t *loc,
                        int nthreads, const int32_t *vc, const int32_t *color)
{
    or_init();
    if (k < 1 || k > 16)
        return -1;
    const int32_t n = ix->n;
    const int64_t m = ix->m;
    const int32_t *src = ix->src, *dst = ix->dst;
    /* y_{e,l} for l = 1..k-1, stored level-major. */
    uint8_t *Y = NULL;
    if (k >= 2) {
        Y = malloc((size_t)(k - 1) * (size_t)(m ? m : 1));
        if (!Y)
            return -2;
        for (int l = 1; l <= k - 1; l++)
            for (int64_t e = 0; e < m; e++)
                Y[(size_t)(l - 1) * m + e] =
                    or_fp(seed, 1, (uint32_t)l, (uint32_t)(ix->eid ? ix->eid[e] : e));
    }
    if (loc)
        memset(loc, 0, (size_t)m);
    int err = 0;
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
    {
        uint8_t *x = malloc((size_t)n + 1);
        uint8_t *prev = malloc((size_t)m + 1);
        uint8_t *cur = malloc((size_t)m + 1);
        uint8_t *pre = malloc((size_t)m + 1);
        uint8_t *myloc = loc ? calloc((size_t)m + 1, 1) : NULL;
        int ok = x && prev && cur && pre && (!loc || myloc);
        if (!ok) {
#pragma omp atomic write
            err = -2;
        }
        {
#pragma omp for schedule(dynamic, 1)
            for (int64_t i = 0; i < npoints; i++) {
                if (!ok)
                    continue;
                uint32_t A = points[i];
                /* z_u^A = sum_{j in A} z_{u,j} */
                for (int32_t u = 0; u < n; u++) {
                    uint8_t s = 0;
                    for (int j = 0; j < k; j++)
                        if ((A >> j) & 1u)
                            s ^= z[(size_t)u * k + j];
                    x[u] = s;
                }
                uint8_t r = 0;
                if (k == 1) {
                    for (int32_t u = 0; u < n; u++)
                        if (!vc || color[u] == vc[0])
                            r ^= x[u];
                    out[i] = r;
                    continue;
                }
                /* level 2: P_{src,1,tau-1} = x_src */
                for (int64_t e = 0; e < m; e++) {
                    prev[e] = OR_MUL[OR_MUL[x[dst[e]]][Y[e]]][x[src[e]]];
                    if (vc && (color[src[e]] != vc[0] || color[dst[e]] != vc[1]))
                        prev[e] = 0;
                    if (ix->emask && !ix->emask[e])
                        prev[e] = 0;
                }
                for (int l = 3; l <= k; l++) {
                    /* running sums along each in-list: P_{v,l-1,tau} */
                    for (int32_t v = 0; v < n; v++) {
                        uint8_t run = 0;
                        for (int64_t p = ix->start[v]; p < ix->start[v + 1]; p++) {
                            run ^= prev[ix->order[p]];
                            pre[p] = run;
                        }
                    }
                    const uint8_t *Yl = Y + (size_t)(l - 2) * m; /* y_{e,l-1} */
                    for (int64_t e = 0; e < m; e++) {
                        uint8_t h = ix->gpos[e] >= 0 ? pre[ix->gpos[e]] : 0;
                        cur[e] = OR_MUL[OR_MUL[x[dst[e]]][Yl[e]]][h];
                        if (vc && (color[src[e]] != vc[l - 2] || color[dst[e]] != vc[l - 1]))
                            cur[e] = 0;
                        if (ix->emask && !ix->emask[e])
                            cur[e] = 0;
                    }
                    uint8_t *t = prev;
                    prev = cur;
                    cur = t;
                }
                for (int64_t e = 0; e < m; e++)
                    r ^= prev[e];
                if (myloc)
                    for (int64_t e = 0; e < m; e++)
                        myloc[e] ^= prev[e];
                out[i] = r;
            }
            if (ok && myloc) {
#pragma omp critical
                for (int64_t e = 0; e < m; e++)
                    loc[e] ^= myloc[e];
            }
        }
        free(x);
        free(prev);
        free(cur);
        free(pre);
        free(myloc);
    }
    free(Y);
    return err;
}

/* One-shot convenience: index + z + evaluation, with optional transition times and
 * delays (as or_index_build_ex). */
int or_sieve_ex(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *tau,
                const int32_t *transit, const int32_t *delay, const int32_t *color, int32_t q,
                const int32_t *M, int32_t k, uint64_t seed, const uint8_t *mask,
                const uint32_t *points, int64_t npoints, uint8_t *out, uint8_t *loc, int nthreads);

int or_sieve(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *tau,
             const int32_t *color, int32_t q, const int32_t *M, int32_t k, uint64_t seed,
             const uint8_t *mask, const uint32_t *points, int64_t npoints, uint8_t *out,
             uint8_t *loc, int nthreads)
{
    return or_sieve_ex(n, m, src, dst, tau, NULL, NULL, color, q, M, k, seed, mask, points,
                       npoints, out, loc, nthreads);
}

int or_sieve_em(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *tau,
                const int32_t *transit, const int32_t *delay, const uint8_t *emask,
                const int32_t *color, int32_t q, const int32_t *M, int32_t k, uint64_t seed,
                const uint8_t *mask, const uint32_t *points, int64_t npoints, uint8_t *out,
                uint8_t *loc, int nthreads);

int or_sieve_ex(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *tau,
                const int32_t *transit, const int32_t *delay, const int32_t *color, int32_t q,
                const int32_t *M, int32_t k, uint64_t seed, const uint8_t *mask,
                const uint32_t *points, int64_t npoints, uint8_t *out, uint8_t *loc, int nthreads)
{
    return or_sieve_em(n, m, src, dst, tau, transit, delay, NULL, color, q, M, k, seed, mask,
                       points, npoints, out, loc, nthreads);
}

/* As or_sieve_ex on the graph without the edges e with emask[e] == 0 (the others keep
 * their indices, hence their y). */
int or_sieve_em(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *tau,
                const int32_t *transit, const int32_t *delay, const uint8_t *emask,
                const int32_t *color, int32_t q, const int32_t *M, int32_t k, uint64_t seed,
                const uint8_t *mask, const uint32_t *points, int64_t npoints, uint8_t *out,
                uint8_t *loc, int nthreads)
{
    or_init();
    if (n < 1 || m < 0 || k < 1 || k > 16)
        return -1;
    uint8_t *z = malloc((size_t)n * (size_t)k);
    if (!z)
        return -2;
    int rc = or_z(n, color, q, M, k, seed, mask, z);
    if (rc) {
        free(z);
        return rc;
    }
    or_index *ix = or_index_build_ex(n, m, src, dst, tau, transit, delay);
    if (!ix) {
        free(z);
        return -2;
    }
    ix->emask = emask;
    rc = or_eval(ix, z, k, seed, points, npoints, out, loc, nthreads);
    or_index_free(ix);
    free(z);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Exact existence of a temporal path whose k vertex colours are the k        */
/* DISTINCT colours of M (colourful query).  Distinct colours make any walk   */
/* using them a path, so an earliest-arrival table over (vertex, colour set)  */
/* decides it exactly; used to check decisions at sizes brute force cannot.  */
/* Returns 1 (exists), 0 (no), -1 (M has a repeated colour or bad input).     */
/* ------------------------------------------------------------------------- */
int or_colorful_exists(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                       const int32_t *tau, const int32_t *color, int32_t q, const int32_t *M,
                       int32_t k)
{
    if (k < 1 || k > 16)
        return -1;
    int32_t *bit = malloc(sizeof(int32_t) * (size_t)q);
    for (int s = 0; s < q; s++)
        bit[s] = -1;
    for (int i = 0; i < k; i++) {
        if (M[i] < 0 || M[i] >= q || bit[M[i]] >= 0) {
            free(bit);
            return -1;
        }
        bit[M[i]] = i;
    }
    const uint32_t full = (k == 32) ? 0xFFFFFFFFu : ((1u << k) - 1u);
    const int32_t INF = 0x7FFFFFFF;
    size_t S = (size_t)1 << k;
    /* best[v][set] = earliest time a walk ending at v with colour set `set`
       arrives at v (0 for the one-vertex walk). */
    int32_t *best = malloc(sizeof(int32_t) * (size_t)n * S);
    for (size_t i = 0; i < (size_t)n * S; i++)
        best[i] = INF;
    int found = 0;
    for (int32_t v = 0; v < n; v++)
        if (bit[color[v]] >= 0) {
            best[(size_t)v * S + (1u << bit[color[v]])] = 0;
            if ((1u << bit[color[v]]) == full)
                found = 1;
        }
    /* edges by increasing time; equal-time edges must not chain, so a group of
       equal timestamps reads only values written before the group. */
    int64_t *ord = malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    for (int64_t e = 0; e < m; e++)
        ord[e] = e;
    g_cmp_tau = tau;
    qsort(ord, (size_t)m, sizeof(int64_t), cmp_by_tau_then_id);
    typedef struct { int32_t v; uint32_t set; int32_t t; } upd;
    upd *pend = malloc(sizeof(upd) * 64);
    size_t npend = 0, cap = 64;
    int64_t a = 0;
    while (a < m && !found) {
        int64_t b = a;
        while (b < m && tau[ord[b]] == tau[ord[a]])
            b++;
        npend = 0;
        for (int64_t i = a; i < b; i++) {
            int64_t e = ord[i];
            int32_t u = src[e], v = dst[e], t = tau[e];
            if (bit[color[u]] < 0 || bit[color[v]] < 0)
                continue;
            uint32_t cb = 1u << bit[color[v]];
            for (uint32_t set = 0; set <= full; set++) {
                if (set & cb)
                    continue;
                if (best[(size_t)u * S + set] < t) {
                    if (npend == cap) {
                        cap *= 2;
                        pend = realloc(pend, sizeof(upd) * cap);
                    }
                    pend[npend].v = v;
                    pend[npend].set = set | cb;
                    pend[npend].t = t;
                    npend++;
                }
            }
        }
        for (size_t i = 0; i < npend; i++) {
            int32_t *slot = &best[(size_t)pend[i].v * S + pend[i].set];
            if (pend[i].t < *slot)
                *slot = pend[i].t;
            if (pend[i].set == full)
                found = 1;
        }
        a = b;
    }
    free(pend);
    free(ord);
    free(best);
    free(bit);
    return found;
}

/* VC-PATH-MOTIF: the sieve of the ordered-colour polynomial (see or_eval_impl); the
 * substitution is that of the multiset of the k colours of vc. */
int or_sieve_vc(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *tau,
                const int32_t *transit, const int32_t *delay, const int32_t *color, int32_t q,
                const int32_t *vc, int32_t k, uint64_t seed, const uint32_t *points,
                int64_t npoints, uint8_t *out, uint8_t *loc, int nthreads)
{
    or_init();
    if (n < 1 || m < 0 || k < 1 || k > 16)
        return -1;
    uint8_t *z = malloc((size_t)n * (size_t)k);
    if (!z)
        return -2;
    int rc = or_z(n, color, q, vc, k, seed, NULL, z);
    if (rc) {
        free(z);
        return rc;
    }
    or_index *ix = or_index_build_ex(n, m, src, dst, tau, transit, delay);
    if (!ix) {
        free(z);
        return -2;
    }
    rc = or_eval_impl(ix, z, k, seed, points, npoints, out, loc, nthreads, vc, color);
    or_index_free(ix);
    free(z);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Static vertex-localised sieve (section "Preprocessing", step (ii), with the */
/* static generating polynomial Eq. (1)).                                      */
/*                                                                             */
/* The static instance has one arc (v -> u) per ordered pair with at least one */
/* temporal edge v -> u, v != u (a path never uses a loop); the arc's variables */
/* y_{vu,l} are keyed by its smallest input edge id r:                          */
/*     y_{vu,l} = fp(seed, 4, l, r),  l = 1..k-1,                              */
/* and x_u is the temporal sieve's (same substitution, same seed).              */
/* Eq. (1) read forward gives F_{u,1} = x_u and                                */
/*     F_{u,l} = x_u * sum_{arcs v -> u} y_{vu,l-1} F_{v,l-1};                 */
/* the same walks read backward give G_{u,k} = 1 and                           */
/*     G_{u,l} = sum_{arcs u -> w} y_{uw,l} x_w G_{w,l+1},                     */
/* so F_{u,l} G_{u,l} sums the monomials of the k-vertex walks whose l-th       */
/* vertex is u.  S_u = sum over points A and over l of F_{u,l} G_{u,l} is the   */
/* sieve of the walks through u counted once per visit: a path through u counts */
/* once, every other walk cancels, so S_u != 0 certifies a static path through  */
/* u whose colours match M (the property the section asks of the vertex-        */
/* localised sieve: nonzero at vertices that are part of a match).             */
/* S[n] receives S_u.  Returns 0, or -1 / -2 on bad input / no memory.          */
/* ------------------------------------------------------------------------- */
static const int32_t *g_arc_src, *g_arc_dst;
static int cmp_arc(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    if (g_arc_src[a] != g_arc_src[b])
        return g_arc_src[a] < g_arc_src[b] ? -1 : 1;
    if (g_arc_dst[a] != g_arc_dst[b])
        return g_arc_dst[a] < g_arc_dst[b] ? -1 : 1;
    return a < b ? -1 : (a > b);
}

int or_static_sieve(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                    const int32_t *color, int32_t q, const int32_t *M, int32_t k, uint64_t seed,
                    const uint8_t *mask, uint8_t *S, int nthreads)
{
    or_init();
    if (n < 1 || m < 0 || k < 1 || k > 16)
        return -1;
    uint8_t *z = malloc((size_t)n * (size_t)k);
    if (!z)
        return -2;
    int rc = or_z(n, color, q, M, k, seed, mask, z);
    if (rc) {
        free(z);
        return rc;
    }
    /* arcs: edges sorted by (src, dst, id); the first of each pair is its
       representative */
    int64_t *ord = malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    int32_t *as = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    int32_t *ad = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    int64_t *ar = malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    if (!ord || !as || !ad || !ar) {
        free(z); free(ord); free(as); free(ad); free(ar);
        return -2;
    }
    for (int64_t e = 0; e < m; e++)
        ord[e] = e;
    g_arc_src = src;
    g_arc_dst = dst;
    qsort(ord, (size_t)m, sizeof(int64_t), cmp_arc);
    int64_t na = 0;
    for (int64_t i = 0; i < m; i++) {
        int64_t e = ord[i];
        if (src[e] == dst[e])
            continue;
        if (na > 0 && as[na - 1] == src[e] && ad[na - 1] == dst[e])
            continue;
        as[na] = src[e];
        ad[na] = dst[e];
        ar[na] = e;
        na++;
    }
    free(ord);
    /* y_{arc,l}, level-major */
    uint8_t *Y = malloc((size_t)(k > 1 ? k - 1 : 1) * (size_t)(na ? na : 1));
    if (!Y) {
        free(z); free(as); free(ad); free(ar);
        return -2;
    }
    for (int l = 1; l <= k - 1; l++)
        for (int64_t a = 0; a < na; a++)
            Y[(size_t)(l - 1) * na + a] = or_fp(seed, 4, (uint32_t)l, (uint32_t)ar[a]);
    memset(S, 0, (size_t)n);
    int err = 0;
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
    const int64_t npoints = (int64_t)1 << k;
#pragma omp parallel num_threads(nthreads)
    {
        uint8_t *x = malloc((size_t)n);
        uint8_t *F = malloc((size_t)k * (size_t)n); /* F[l-1][u] */
        uint8_t *Gc = malloc((size_t)n), *Gn = malloc((size_t)n);
        uint8_t *myS = calloc((size_t)n, 1);
        int ok = x && F && Gc && Gn && myS;
        if (!ok) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t A = 0; A < npoints; A++) {
            if (!ok)
                continue;
            for (int32_t u = 0; u < n; u++) {
                uint8_t s = 0;
                for (int j = 0; j < k; j++)
                    if ((A >> j) & 1)
                        s ^= z[(size_t)u * k + j];
                x[u] = s;
            }
            memcpy(F, x, (size_t)n);
            for (int l = 2; l <= k; l++) {
                uint8_t *Fl = F + (size_t)(l - 1) * n;
                const uint8_t *Fp = F + (size_t)(l - 2) * n;
                const uint8_t *Yl = Y + (size_t)(l - 2) * na; /* y_{.,l-1} */
                memset(Fl, 0, (size_t)n);
                for (int64_t a = 0; a < na; a++)
                    Fl[ad[a]] ^= OR_MUL[Yl[a]][Fp[as[a]]];
                for (int32_t u = 0; u < n; u++)
                    Fl[u] = OR_MUL[x[u]][Fl[u]];
            }
            /* l = k: G = 1 */
            for (int32_t u = 0; u < n; u++) {
                Gc[u] = 1;
                myS[u] ^= F[(size_t)(k - 1) * n + u];
            }
            for (int l = k - 1; l >= 1; l--) {
                const uint8_t *Yl = Y + (size_t)(l - 1) * na; /* y_{.,l} */
                memset(Gn, 0, (size_t)n);
                for (int64_t a = 0; a < na; a++)
                    Gn[as[a]] ^= OR_MUL[Yl[a]][OR_MUL[x[ad[a]]][Gc[ad[a]]]];
                for (int32_t u = 0; u < n; u++)
                    myS[u] ^= OR_MUL[F[(size_t)(l - 1) * n + u]][Gn[u]];
                uint8_t *t = Gc;
                Gc = Gn;
                Gn = t;
            }
        }
        if (ok) {
#pragma omp critical
            for (int32_t u = 0; u < n; u++)
                S[u] ^= myS[u];
        }
        free(x);
        free(F);
        free(Gc);
        free(Gn);
        free(myS);
    }
    free(Y);
    free(z);
    free(as);
    free(ad);
    free(ar);
    return err;
}
