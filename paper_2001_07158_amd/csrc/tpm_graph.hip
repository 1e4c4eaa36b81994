// Graph ingest and the device-resident in-edge index.
//
// The temporal graph (section "Terminology": temporal edges (u, v, j), j a positive
// integer) is stored as an in-edge CSR: positions sorted by (dst, tau, input id).
// Eq. (3) makes P_{u,l,.} a step function of time that changes only at u's in-edge
// times, so the running value after position p of u's in-list is P_{u,l,tau_p}.
// For the edge e = (v -> u, tau) at position p the recursion reads P_{v,l-1,tau-1}:
// the running value at the last position of v's in-list with tau' < tau, found here
// once per graph by binary search.  Only positions some edge reads ("rows") are ever
// stored by the sieve kernels; rows are numbered in CSR order.
//
// Work tiles: consecutive CSR positions, built on the device (k_tile_*).  An in-list
// longer than tile_edges (T) is cut into pieces of T positions whose running values
// are published to consecutive "slots" for the look-back; shorter in-lists are kept
// whole and grouped by the T-aligned window their first position falls in (a group
// spans less than 2T positions).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include <rocprim/rocprim.hpp>

#include "tpm_internal.h"

namespace tpm {

namespace {

__global__ void k_validate(int64_t m, int32_t n, const int32_t *src, const int32_t *dst,
                           const int32_t *tau, int32_t *bad, int32_t *tmax) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int32_t local_max = 0;
    for (; i < m; i += stride) {
        int32_t s = src[i], d = dst[i], t = tau[i];
        if (s < 0 || s >= n || d < 0 || d >= n || t < 1) atomicOr(bad, 1);
        local_max = max(local_max, t);
    }
    for (int off = 32; off >= 1; off >>= 1) local_max = max(local_max, __shfl_xor(local_max, off));
    if ((threadIdx.x & 63) == 0) atomicMax(tmax, local_max);
}

__global__ void k_validate_color(int32_t n, int32_t q, const int32_t *color, int32_t *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (color[i] < 0 || color[i] >= q)) atomicOr(bad, 2);
}

__global__ void k_keys(int64_t m, const int32_t *dst, const int32_t *tau, int tbits,
                       uint64_t *keys, int32_t *vals) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) {
        keys[e] = ((uint64_t)(uint32_t)dst[e] << tbits) | (uint64_t)(uint32_t)tau[e];
        vals[e] = (int32_t)e;
    }
}

// tau: the time that orders in-lists (arrival); dep (nullable): departure times
__global__ void k_apply(int64_t m, const int32_t *order, const int32_t *src, const int32_t *dst,
                        const int32_t *tau, const int32_t *dep, int32_t *psrc, int32_t *pdst,
                        int32_t *ptau, int32_t *pdep, int32_t *peid) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < m) {
        int32_t e = order[p];
        peid[p] = e;
        psrc[p] = src[e];
        pdst[p] = dst[e];
        ptau[p] = tau[e];
        if (dep) pdep[p] = dep[e];
    }
}

// arrival = departure + transition time; flag bit 4 on a negative transition time or an
// arrival past 2^31 - 1, and the largest arrival in *amax
__global__ void k_arrival(int64_t m, const int32_t *tau, const int32_t *transit, int32_t *arr,
                          int32_t *bad, int32_t *amax) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int32_t local = 0;
    for (; i < m; i += stride) {
        const int64_t a = (int64_t)tau[i] + transit[i];
        if (transit[i] < 0 || a > 0x7FFFFFFF) {
            atomicOr(bad, 4);
            arr[i] = tau[i];
        } else {
            arr[i] = (int32_t)a;
            local = max(local, (int32_t)a);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) local = max(local, __shfl_xor(local, off));
    if ((threadIdx.x & 63) == 0) atomicMax(amax, local);
}

// inptr[u] = first position whose dst >= u; every position writes the entries of
// the vertices between its predecessor's dst and its own (deterministic, no atomics).
__global__ void k_inptr(int64_t m, int32_t n, const int32_t *pdst, int32_t *inptr) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > m) return;
    int32_t lo = (p == 0) ? 0 : pdst[p - 1] + 1;
    int32_t hi = (p == m) ? n : pdst[p];
    for (int32_t u = lo; u <= hi; ++u) inptr[u] = (int32_t)p;
}

// ---- Position bitmaps with rank, in records of 128 bytes (one memory transfer): word
// 0 holds the record's base (set bits in the records before it), words 1..31 the flags
// of 992 positions (bit j of word 1 + i is position 992 r + 32 i + j).  rank(x), the
// number of set bits below x, then costs one record read; the structure takes m / 7.75
// bytes, where an int per position (exclusive counts) takes m x 4 and a scan to build.
constexpr int64_t kRecPos = 992;

int64_t rank_recs(int64_t m) { return (m + kRecPos - 1) / kRecPos; }

__device__ __forceinline__ int64_t rec_word(int64_t x) {
    const int64_t r = x / kRecPos;
    return r * 32 + 1 + ((x - r * kRecPos) >> 5);
}

__device__ __forceinline__ bool bit_at(const uint32_t *rec, int64_t x) {
    return (rec[rec_word(x)] >> ((x % kRecPos) & 31)) & 1u;
}

// Set bits below x, 0 <= x <= the bitmap's length (bits past the length are zero);
// total: the number of all set bits (read only for x at the end of the last record).
__device__ __forceinline__ int32_t bit_rank(const uint32_t *rec, int64_t nr, const int32_t *total,
                                            int64_t x) {
    const int64_t r = x / kRecPos;
    if (r >= nr) return *total;
    const int32_t o = (int32_t)(x - r * kRecPos);
    const int k = o >> 5, j = o & 31;
    const uint4 *w4 = (const uint4 *)(rec + r * 32);
    int32_t base = 0, c = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint4 v = w4[i];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int wi = 4 * i + t;
            if (wi == 0) {
                base = (int32_t)w[t];
            } else {
                const int bi = wi - 1;
                const uint32_t keep = bi < k ? 0xFFFFFFFFu : (bi == k ? (uint32_t)((1ull << j) - 1ull) : 0u);
                c += __popc(w[t] & keep);
            }
        }
    }
    return base + c;
}

// Blocks of 256 threads over quarters of records: block b covers positions 992 (b / 4) +
// 256 (b % 4) + t, t < 256 (the last quarter has 224).  wave_rank gives a thread's
// exclusive rank among the set bits from the record's base, the words before its wave's
// 64 positions and a ballot (no LDS).
__device__ __forceinline__ int64_t quarter_pos() {
    return (int64_t)(blockIdx.x >> 2) * kRecPos + 256 * (blockIdx.x & 3) + threadIdx.x;
}

__device__ __forceinline__ bool quarter_in(int64_t m, int64_t p) {
    return 256 * (blockIdx.x & 3) + threadIdx.x < kRecPos && p < m;
}

__device__ __forceinline__ int32_t wave_rank(const uint32_t *rec, bool f) {
    const uint32_t *w = rec + (int64_t)(blockIdx.x >> 2) * 32;
    const int first = 8 * (blockIdx.x & 3) + 2 * (threadIdx.x >> 6);  // bit word of lane 0
    int32_t c = (int32_t)w[0];
    for (int i = 0; i < first; ++i) c += __popc(w[1 + i]);
    const uint64_t b = __ballot(f);
    return c + __popcll(b & ((1ull << (threadIdx.x & 63)) - 1ull));
}

// Records written one wave per record: lane l < 31 gives word 1 + l (the flags of
// positions 992 r + 32 l ... + 31); the wave writes the 31 words and the record's count
// (and the zero count past the last record).  Word 0 (the base) is written by k_put_base
// after the scan of the counts.
__device__ __forceinline__ void put_record(uint32_t word, int lane, int64_t r, uint32_t *rec,
                                           int32_t *cnt, int64_t nr) {
    if (lane < 31) rec[r * 32 + 1 + lane] = word;
    int32_t c = __popc(word);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    if (lane == 0) {
        cnt[r] = c;
        if (r == nr - 1) cnt[nr] = 0;
    }
}

// word 0 of each record: its base, from the exclusive scan of the counts
__global__ void k_put_base(int64_t nr, const int32_t *base, uint32_t *rec) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nr) rec[r * 32] = (uint32_t)base[r];
}

// gpos[p] = last position q of src's in-list that arrived by the departure of p minus
// the delay of src (plain problem: arrival = departure = tau, delay 1, so tau[q] <
// tau[p]), or -1; needed[q] = 1 (every writer stores the same value).  pdep, vdelay
// nullable.
__global__ void k_gpos(int64_t m, const int32_t *psrc, const int32_t *ptau, const int32_t *pdep,
                       const int32_t *vdelay, const int32_t *inptr, int32_t *gpos,
                       uint8_t *needed) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    int32_t v = psrc[p];
    const int64_t th = (int64_t)(pdep ? pdep[p] : ptau[p]) - (vdelay ? vdelay[v] : 1) + 1;
    int32_t lo = inptr[v], hi = inptr[v + 1], base = lo;
    while (lo < hi) {
        int32_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)ptau[mid] < th) lo = mid + 1; else hi = mid;
    }
    int32_t q = (lo > base) ? lo - 1 : -1;
    gpos[p] = q;
    if (q >= 0) needed[q] = 1;
}

// Rank records of m byte flags, one wave per record (blocks of 256 = 4 records)
__global__ void __launch_bounds__(256) k_pack(int64_t m, int64_t nr, const uint8_t *flag,
                                              uint32_t *rec, int32_t *cnt) {
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (r >= nr) return;
    const int64_t p0 = r * kRecPos + 32 * (int64_t)lane;
    uint32_t w = 0;
    if (lane < 31 && p0 < m) {
        if (p0 + 32 <= m) {
            const uint4 *f4 = (const uint4 *)(flag + p0);
            const uint4 a = f4[0], b = f4[1];
            const uint32_t v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if ((v[i] >> (8 * j)) & 0xFFu) w |= 1u << (4 * i + j);
        } else {
            for (int j = 0; p0 + j < m; ++j)
                if (flag[p0 + j]) w |= 1u << j;
        }
    }
    put_record(w, lane, r, rec, cnt, nr);
}

// Rows are the needed positions, numbered in CSR order: orow[p] = rank of p among them
// (or -1), gsrc[p] = the row that p reads (or -1).  Blocks of 256 over record quarters.
__global__ void __launch_bounds__(256) k_rows(int64_t m, const int32_t *gpos, const uint32_t *needed,
                                              int64_t nr, const int32_t *total, int32_t *orow,
                                              int32_t *gsrc) {
    const int64_t p = quarter_pos();
    const bool in = quarter_in(m, p);
    const bool f = in && bit_at(needed, p);
    const int32_t r = wave_rank(needed, f);
    if (!in) return;
    orow[p] = f ? r : -1;
    const int32_t q = gpos[p];
    gsrc[p] = q >= 0 ? bit_rank(needed, nr, total, q) : -1;
}

__global__ void k_count_nonneg(int64_t m, const int32_t *a, unsigned long long *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long c = 0;
    for (; i < m; i += stride) c += a[i] >= 0;
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

// keep[p] = 1 when both endpoints of the edge at position p have a kept colour
// vkeep[u] = 1 when u's colour is kept
__global__ void k_vkeep(int32_t n, const int32_t *color, const uint8_t *keepc, uint8_t *vkeep) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) vkeep[u] = keepc[color[u]];
}

__global__ void k_vand(int32_t n, const uint8_t *a, uint8_t *b) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) b[u] = (a[u] != 0 && b[u] != 0) ? 1 : 0;
}

// keep[p] = 1 when both endpoints of the edge at position p are kept and, with a
// timestamp set ts[0..nts) (sorted), its timestamp is in the set
// vbits: one bit per vertex (bit u & 31 of word u >> 5), so that the random lookups of
// the sources stay in cache
__global__ void k_vbits(int32_t n, const uint8_t *vkeep, uint32_t *vbits) {
    int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= ((int64_t)n + 31) / 32) return;
    uint32_t b = 0;
    for (int j = 0; j < 32; ++j) {
        const int64_t u = w * 32 + j;
        if (u < n && vkeep[u]) b |= 1u << j;
    }
    vbits[w] = b;
}

__device__ __forceinline__ bool vbit(const uint32_t *vbits, int32_t u) {
    return (vbits[u >> 5] >> (u & 31)) & 1u;
}

// (cut_in: a vertex whose in-edges go, cut_out: one whose out-edges go; -1 for none;
// parr: arrival times, kept up to tcut)
__device__ __forceinline__ bool time_in(const int32_t *ts, int32_t nts, int32_t t) {
    int32_t a = 0, b = nts;
    while (a < b) {
        const int32_t mid = (a + b) >> 1;
        if (ts[mid] < t) a = mid + 1;
        else b = mid;
    }
    return a < nts && ts[a] == t;
}

// The kept positions as rank records with their counts, one wave per record (blocks of
// 256 = 4 records), lane l < 31 for the 32 positions of word 1 + l
__global__ void __launch_bounds__(256) k_keep(int64_t m, int64_t nr, const int32_t *psrc,
                                              const int32_t *pdst, const uint32_t *vbits,
                                              const int32_t *ptime, const int32_t *ts, int32_t nts,
                                              int32_t cut_in, int32_t cut_out, const int32_t *parr,
                                              int32_t tcut, uint32_t *keep, int32_t *kcnt) {
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (r >= nr) return;
    const int64_t p0 = r * kRecPos + 32 * (int64_t)lane;
    uint32_t w = 0;
    if (lane < 31)
        for (int j = 0; j < 32 && p0 + j < m; ++j) {
            const int64_t p = p0 + j;
            const int32_t s = psrc[p], d = pdst[p];
            bool k = vbit(vbits, s) && vbit(vbits, d) && d != cut_in && s != cut_out && parr[p] <= tcut;
            if (k && ts) k = time_in(ts, nts, ptime[p]);
            if (k) w |= 1u << j;
        }
    put_record(w, lane, r, keep, kcnt, nr);
}

// k_keep for a colour set only, from the colour pair of each position (2 bytes read
// per position instead of both endpoints and their vertex bits)
__global__ void __launch_bounds__(256) k_keep_pc(int64_t m, int64_t nr, const uint16_t *pcol,
                                                 uint64_t cmask, const int32_t *ptime,
                                                 const int32_t *ts, int32_t nts, const int32_t *parr,
                                                 int32_t tcut, uint32_t *keep, int32_t *kcnt) {
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (r >= nr) return;
    const int64_t p0 = r * kRecPos + 32 * (int64_t)lane;
    uint32_t w = 0;
    if (lane < 31 && p0 < m) {
        const int nv = (int)min<int64_t>(32, m - p0);
        if (nv == 32) {
            const uint4 *c4 = (const uint4 *)(pcol + p0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint4 v = c4[i];
                const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const uint32_t pc = (u[t] >> (16 * h)) & 0xFFFFu;
                        if ((cmask >> (pc & 0xFFu)) & (cmask >> (pc >> 8)) & 1ull)
                            w |= 1u << (8 * i + 2 * t + h);
                    }
            }
        } else {
            for (int j = 0; j < nv; ++j) {
                const uint32_t pc = pcol[p0 + j];
                if ((cmask >> (pc & 0xFFu)) & (cmask >> (pc >> 8)) & 1ull) w |= 1u << j;
            }
        }
        if (w && (tcut < 0x7FFFFFFF || ts)) {  // time restrictions, kept candidates only
            for (int j = 0; j < nv; ++j) {
                if (!((w >> j) & 1u)) continue;
                const int64_t p = p0 + j;
                bool k = tcut >= 0x7FFFFFFF || parr[p] <= tcut;
                if (k && ts) k = time_in(ts, nts, ptime[p]);
                if (!k) w &= ~(1u << j);
            }
        }
    }
    put_record(w, lane, r, keep, kcnt, nr);
}

// layer keep: edge at p goes from colour cs to colour cd
__global__ void k_layer_keep(int64_t m, const int32_t *psrc, const int32_t *pdst,
                             const int32_t *color, int32_t cs, int32_t cd, int32_t *keep) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < m) keep[p] = (color[psrc[p]] == cs && color[pdst[p]] == cd) ? 1 : 0;
}

// kept edges of one layer, renumbered: source in layer l-1 (base bs), head in layer l
// (base bd), placed from position off on
__global__ void k_layer_compact(int64_t m, const int32_t *keep, const int32_t *at, int32_t off,
                                const int32_t *psrc, const int32_t *pdst, const int32_t *ptau,
                                const int32_t *peid, const int32_t *pdep, const int32_t *rank,
                                int32_t bs, int32_t bd, int32_t *qsrc, int32_t *qdst,
                                int32_t *qtau, int32_t *qeid, int32_t *qdep) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < m && keep[p]) {
        const int64_t q = (int64_t)off + at[p];
        qsrc[q] = bs + rank[psrc[p]];
        qdst[q] = bd + rank[pdst[p]];
        qtau[q] = ptau[p];
        qeid[q] = peid[p];
        if (pdep) qdep[q] = pdep[p];
    }
}

__global__ void k_pcol(int64_t m, const int32_t *psrc, const int32_t *pdst, const int32_t *color,
                       uint16_t *pcol) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < m) pcol[p] = (uint16_t)(color[psrc[p]] | (color[pdst[p]] << 8));
}

// In-list starts of the subgraph: the kept positions before the parent's start
// (keep: the kept-position records, nr of them, total: their set bits).
__global__ void k_sub_inptr(int32_t n, const int32_t *pinptr, const uint32_t *keep, int64_t nr,
                            const int32_t *total, int32_t *inptr) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u > n) return;
    inptr[u] = bit_rank(keep, nr, total, pinptr[u]);
}

__global__ void k_needed(int64_t m, const int32_t *gpos, uint8_t *needed) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    const int32_t q = gpos[p];
    if (q >= 0) needed[q] = 1;  // every writer stores the same value
}

// Kept positions copied in order, one wave per record of `keep` (the kept-position
// records, nr of them; blocks of 256 = 4 records): the wave lists the record's kept
// offsets in LDS (lane l those of word 1 + l, at the exclusive count of the lanes
// before), then its lanes copy one kept position each per round, so that a wave moves
// only kept edges whatever the density (a wave walking the record 64 positions at a
// time without LDS measured 2 ms slower per request on the 1e9-edge graph).  pdep
// nullable; gpar (nullable): the parent's read position of each kept edge (k_remap maps
// it into the subgraph).
__global__ void __launch_bounds__(256) k_compact(
    int64_t nr, const uint32_t *keep, const int32_t *psrc, const int32_t *pdst,
    const int32_t *ptau, const int32_t *peid, const int32_t *pdep, const int32_t *gposw,
    int32_t *qsrc, int32_t *qdst, int32_t *qtau, int32_t *qeid, int32_t *qdep, int32_t *gpar) {
    __shared__ uint16_t lst[4][kRecPos];
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool ok = r < nr;
    uint32_t w = (ok && lane < 31) ? keep[r * 32 + 1 + lane] : 0u;
    const int32_t base = ok ? (int32_t)keep[r * 32] : 0;
    const int32_t c = __popc(w);
    int32_t x = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    const int32_t K = __shfl(x, 63);
    int32_t i = x - c;
    while (w) {
        const int j = __ffs(w) - 1;
        w &= w - 1u;
        lst[wv][i++] = (uint16_t)(32 * lane + j);
    }
    __syncthreads();
    for (int32_t k = lane; k < K; k += 64) {
        const int64_t p = r * kRecPos + lst[wv][k];
        const int32_t q = base + k;
        qsrc[q] = psrc[p];
        qdst[q] = pdst[p];
        qtau[q] = ptau[p];
        qeid[q] = peid[p];
        if (pdep) qdep[q] = pdep[p];
        if (gposw) gpar[q] = gposw[p];
    }
}

// Read positions of the subgraph's mk edges, in place of their parent read positions g:
// the last kept position at or before g (positions keep their order; keep: the parent's
// kept-position records, nr of them, total: their set bits), if that is still in the
// source's in-list (sub_inptr: the subgraph's in-list starts), -1 otherwise; needed[r] =
// 1 for every position read (one byte each).
__global__ void k_remap(int64_t mk, const int32_t *qsrc, const uint32_t *keep, int64_t nr,
                        const int32_t *total, const int32_t *sub_inptr, int32_t *gpos,
                        uint8_t *needed) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= mk) return;
    const int32_t g = gpos[q];
    int32_t r = -1;
    if (g >= 0) {
        const int32_t last = bit_rank(keep, nr, total, (int64_t)g + 1) - 1;
        if (last >= sub_inptr[qsrc[q]]) r = last;
    }
    gpos[q] = r;
    if (r >= 0) needed[r] = 1;  // every writer stores the same value
}

// ---- work tiles on the device.  Per vertex u with an in-list of L positions: a long
// list (L > T) gives ceil(L / T) pieces of T positions; every piece but the last
// publishes to a slot, every piece but the first looks back at its predecessor's.  A
// short list (0 < L <= T) starts a new tile when it is the first non-empty list, when
// the previous non-empty list is long, or when its first position falls in another
// T-aligned window than the previous list's; otherwise it joins that list's tile (so a
// tile of short lists spans less than 2T positions).
__global__ void k_tile_prev(int32_t n, const int32_t *inptr, int32_t *nz) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) nz[u] = inptr[u + 1] > inptr[u] ? (int32_t)u : -1;
}

// grid-stride over vertices (a bounded grid keeps the two statistics atomics few: one
// pair per wave)
__global__ void k_tile_count(int32_t n, const int32_t *inptr, int32_t T, const int32_t *prevmax,
                             int32_t *tcnt, int32_t *scnt, unsigned long long *stats) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long mx = 0, ne = 0;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        const int32_t a = inptr[u];
        const int32_t L = inptr[u + 1] - a;
        int32_t t = 0, sl = 0;
        if (L > T) {
            t = (L + T - 1) / T;
            sl = t - 1;
        } else if (L > 0) {
            const int32_t prev = u > 0 ? prevmax[u - 1] : -1;  // previous non-empty list
            if (prev < 0) {
                t = 1;
            } else {
                const int32_t pa = inptr[prev], pl = inptr[prev + 1] - pa;
                t = (pl > T || a / T != pa / T) ? 1 : 0;
            }
        }
        tcnt[u] = t;
        scnt[u] = sl;
        // in-degree statistics: largest and non-empty count
        mx = (unsigned long long)L > mx ? (unsigned long long)L : mx;
        ne += L > 0 ? 1ull : 0ull;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(mx, off);
        mx = o > mx ? o : mx;
        ne += __shfl_xor(ne, off);
    }
    if ((threadIdx.x & 63) == 0) {
        if (mx) atomicMax(&stats[0], mx);
        if (ne) atomicAdd(&stats[1], ne);
    }
}

__global__ void k_tile_fill(int32_t n, const int32_t *inptr, int32_t T, const int32_t *tcnt,
                            const int32_t *tbase, const int32_t *sbase, int32_t *p0, int32_t *pub,
                            int32_t *lb) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n || tcnt[u] == 0) return;
    const int32_t a = inptr[u], L = inptr[u + 1] - a, tb = tbase[u];
    if (L > T) {
        const int32_t np = tcnt[u], sb = sbase[u];
        for (int32_t j = 0; j < np; ++j) {
            p0[tb + j] = a + j * T;
            pub[tb + j] = j + 1 < np ? sb + j : -1;
            lb[tb + j] = j > 0 ? sb + j - 1 : -1;
        }
    } else {
        p0[tb] = a;
        pub[tb] = -1;
        lb[tb] = -1;
    }
}

__global__ void k_set1(int32_t *p, int32_t v) { *p = v; }

inline unsigned grid_for(int64_t work, int block = 256) {
    int64_t g = (work + block - 1) / block;
    return (unsigned)std::max<int64_t>(1, g);
}

template <class T>
T *dalloc(int64_t count, int64_t &acct) {
    void *p = nullptr;
    size_t bytes = (size_t)std::max<int64_t>(1, count) * sizeof(T);
    TPM_HIP(hipMalloc(&p, bytes));
    acct += (int64_t)bytes;
    return (T *)p;
}

int bits_for(uint64_t v) {  // bits needed to represent values 0..v
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return std::max(b, 1);
}

}  // namespace

// Slots of a graph arena: one grow-only buffer per index array and per temporary.
enum ArenaSlot {
    A_COLOR, A_PDST, A_PSRC, A_PTAU, A_PEID, A_GSRC, A_OROW, A_INPTR, A_TP0, A_TPUB,
    A_TLB, A_LDS, A_TTAB, A_KEEPC, A_KBITS, A_KCNT, A_KBASE, A_SCRATCH, A_GPOS, A_NBITS, A_NCNT,
    A_NBASE, A_TSORT, A_TUNIQ, A_TCOUNT, A_CNT, A_PDEP, A_VDELAY, A_VKEEP, A_TSET, A_FID, A_TNZ,
    A_TPM, A_TCNT, A_SCNT, A_TBASE, A_SBASE, A_TSTAT, A_VBITS, A_GPOSW, A_GPOSP, A_NFLAG, A_NFLAGP, A_NSLOTS
};

struct GraphArena {
    DBuf s[A_NSLOTS];
};

GraphArena *new_graph_arena() { return new GraphArena(); }
void delete_graph_arena(GraphArena *a) { delete a; }

int64_t arena_bytes(const GraphArena *a) {
    int64_t b = 0;
    if (a)
        for (const DBuf &d : a->s) b += (int64_t)d.cap;
    return b;
}

void arena_trim(GraphArena *a) {
    if (!a) return;
    bool any = false;
    for (DBuf &d : a->s) any |= d.p != nullptr;
    if (!any) return;
    TPM_HIP(hipDeviceSynchronize());
    for (DBuf &d : a->s) {
        if (d.p) (void)hipFree(d.p);
        d.p = nullptr;
        d.cap = 0;
    }
}

struct ArenaPool {
    std::mutex mu;
    std::vector<GraphArena *> all, free_list;
    ~ArenaPool() {
        for (GraphArena *a : all) delete a;
    }
};
ArenaPool *new_arena_pool() { return new ArenaPool(); }

GraphArena *arena_take(ArenaPool *p) {
    std::lock_guard<std::mutex> lk(p->mu);
    if (!p->free_list.empty()) {
        GraphArena *a = p->free_list.back();
        p->free_list.pop_back();
        return a;
    }
    GraphArena *a = new GraphArena();
    p->all.push_back(a);
    return a;
}

void arena_give(ArenaPool *p, GraphArena *a) {
    std::lock_guard<std::mutex> lk(p->mu);
    p->free_list.push_back(a);
}
void delete_arena_pool(ArenaPool *p) { delete p; }

void run_sieve_pruned(const Graph &G, const SieveRequest &req, SieveResult &res,
                      uint8_t *loc_by_edge, hipStream_t st, void (*then)(const Graph &, void *),
                      void *ctx) {
    TPM_REQUIRE(req.multiset != nullptr && req.k >= 1 && req.k <= 16, "bad query");
    std::vector<uint8_t> keep((size_t)G.q, 0);
    bool wild = false;
    for (int i = 0; i < req.k; ++i) {
        TPM_REQUIRE(req.multiset[i] >= -1 && req.multiset[i] < G.q, "multiset colour out of range");
        if (req.multiset[i] < 0) wild = true;
        else keep[(size_t)req.multiset[i]] = 1;
    }
    if (wild || !G.apool) {  // every vertex may match: nothing to prune
        if (loc_by_edge) run_sieve_loc_all(G, req, res, loc_by_edge, st);
        else run_sieve(G, req, res, st);
        if (then) then(G, ctx);
        return;
    }
    GraphArena *arena = nullptr;
    {
        std::lock_guard<std::mutex> lk(G.apool->mu);
        if (!G.apool->free_list.empty()) {
            arena = G.apool->free_list.back();
            G.apool->free_list.pop_back();
        } else {
            arena = new GraphArena();
            G.apool->all.push_back(arena);
        }
    }
    struct Back {
        ArenaPool *pool;
        GraphArena *a;
        Graph P;
        ~Back() {
            P.pool = nullptr;  // the parent's
            free_graph(P);
            std::lock_guard<std::mutex> lk(pool->mu);
            pool->free_list.push_back(a);
        }
    } b{G.apool, arena, Graph()};
    PruneSpec spec;
    spec.keep_color = keep.data();
    spec.need_times = false;
    prune_graph(G, spec, b.P, arena, st);
    b.P.pool = G.pool;
    if (loc_by_edge) run_sieve_loc_all(b.P, req, res, loc_by_edge, st);
    else run_sieve(b.P, req, res, st);
    if (then) then(b.P, ctx);
}

namespace {

// An array of the graph: its own allocation (freed with the graph), or the arena's
// slot when the graph lives in an arena.
template <class T>
T *galloc(Graph &G, int slot, int64_t count, int64_t &acct, hipStream_t st = nullptr) {
    if (G.arena) {
        DBuf &b = G.arena->s[slot];
        b.alloc((size_t)std::max<int64_t>(1, count) * sizeof(T), st);
        acct += (int64_t)b.cap;
        return (T *)b.p;
    }
    return dalloc<T>(count, acct);
}

// Temporaries of an index build: the arena's slots, or allocations freed at the end.
struct Temps {
    GraphArena *arena = nullptr;
    hipStream_t st = nullptr;
    std::vector<void *> own;
    explicit Temps(GraphArena *a, hipStream_t s = nullptr) : arena(a), st(s) {}
    Temps(const Temps &) = delete;
    Temps &operator=(const Temps &) = delete;
    void *raw(int slot, size_t bytes) {
        bytes = std::max<size_t>(bytes, 16);
        if (arena) {
            arena->s[slot].alloc(bytes, st);
            return arena->s[slot].p;
        }
        void *p = nullptr;
        TPM_HIP(hipMalloc(&p, bytes));
        own.push_back(p);
        return p;
    }
    template <class T>
    T *get(int slot, int64_t count) {
        return (T *)raw(slot, (size_t)std::max<int64_t>(1, count) * sizeof(T));
    }
    ~Temps() {
        if (!own.empty()) (void)hipStreamSynchronize(st);
        for (void *p : own) (void)hipFree(p);
    }
};

// Greedy tiles on the host (whole graphs, built once): short in-lists are packed
// while the tile stays within T positions, long ones are cut into pieces of T.  The
// device builder below groups short lists by window instead (per-query subgraphs,
// where build time matters); results do not depend on the tiling, and the greedy
// tiles measured a few percent faster in the level kernels.
void build_tiles(const std::vector<int32_t> &inptr, int32_t T, std::vector<int32_t> &p0,
                 std::vector<int32_t> &pub, std::vector<int32_t> &lb, int64_t &nslots) {
    const int32_t n = (int32_t)inptr.size() - 1;
    p0.clear();
    pub.clear();
    lb.clear();
    nslots = 0;
    int32_t cur_start = -1, cur_len = 0;
    auto close_pack = [&]() {
        if (cur_len > 0) {
            p0.push_back(cur_start);
            pub.push_back(-1);
            lb.push_back(-1);
        }
        cur_len = 0;
        cur_start = -1;
    };
    for (int32_t u = 0; u < n; ++u) {
        int32_t a = inptr[u], b = inptr[u + 1], L = b - a;
        if (L == 0) continue;
        if (L <= T) {
            if (cur_len > 0 && cur_len + L > T) close_pack();
            if (cur_len == 0) cur_start = a;
            cur_len += L;
            continue;
        }
        close_pack();
        // first piece: starts at the in-list head and publishes its running value;
        // every later piece looks back, and all but the last publish as well
        int32_t prev_slot = (int32_t)nslots++;
        p0.push_back(a);
        pub.push_back(prev_slot);
        lb.push_back(-1);
        for (int32_t q = a + T; q < b; q += T) {
            bool last = (q + T >= b);
            int32_t slot = last ? -1 : (int32_t)nslots++;
            p0.push_back(q);
            pub.push_back(slot);
            lb.push_back(prev_slot);
            prev_slot = slot;
        }
    }
    close_pack();
    p0.push_back(inptr[n]);
}

// Builds G.tile_p0/pub/lb (device), G.h_tile_p0, ntiles, nslots, max_in_degree and
// segments from G.inptr on the device (allocations through galloc unless `own` is set:
// then plain allocations the caller adopts).
void build_tiles_device(Graph &G, int32_t T, Temps &tmp, int64_t &acct, int32_t **tp0,
                        int32_t **tpub, int32_t **tlb, int64_t &ntiles, int64_t &nslots,
                        bool own, bool greedy, hipStream_t st) {
    const int32_t n = G.n;
    int32_t *nz = tmp.get<int32_t>(A_TNZ, n);
    int32_t *pm = tmp.get<int32_t>(A_TPM, n);
    int32_t *tcnt = tmp.get<int32_t>(A_TCNT, n);
    int32_t *scnt = tmp.get<int32_t>(A_SCNT, n);
    int32_t *tbase = tmp.get<int32_t>(A_TBASE, n);
    int32_t *sbase = tmp.get<int32_t>(A_SBASE, n);
    unsigned long long *stats = tmp.get<unsigned long long>(A_TSTAT, 2);
    TPM_HIP(hipMemsetAsync(stats, 0, 2 * sizeof(unsigned long long), st));
    k_tile_prev<<<grid_for(n), 256, 0, st>>>(n, G.inptr, nz);
    size_t b1 = 0, b2 = 0;
    TPM_HIP(rocprim::inclusive_scan(nullptr, b1, nz, pm, (size_t)n, rocprim::maximum<int32_t>(), st));
    TPM_HIP(rocprim::exclusive_scan(nullptr, b2, tcnt, tbase, 0, (size_t)n, rocprim::plus<int32_t>(), st));
    void *scratch = tmp.raw(A_SCRATCH, std::max(b1, b2));
    TPM_HIP(rocprim::inclusive_scan(scratch, b1, nz, pm, (size_t)n, rocprim::maximum<int32_t>(), st));
    k_tile_count<<<std::min<unsigned>(grid_for(n), 2048), 256, 0, st>>>(n, G.inptr, T, pm, tcnt, scnt, stats);
    TPM_HIP(rocprim::exclusive_scan(scratch, b2, tcnt, tbase, 0, (size_t)n, rocprim::plus<int32_t>(), st));
    TPM_HIP(rocprim::exclusive_scan(scratch, b2, scnt, sbase, 0, (size_t)n, rocprim::plus<int32_t>(), st));
    int32_t h[4] = {0, 0, 0, 0};
    TPM_HIP(hipMemcpyAsync(&h[0], tbase + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TPM_HIP(hipMemcpyAsync(&h[1], tcnt + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TPM_HIP(hipMemcpyAsync(&h[2], sbase + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TPM_HIP(hipMemcpyAsync(&h[3], scnt + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, st));
    unsigned long long hs[2] = {0, 0};
    TPM_HIP(hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, st));
    TPM_HIP(hipStreamSynchronize(st));
    ntiles = (int64_t)h[0] + h[1];
    nslots = (int64_t)h[2] + h[3];
    G.max_in_degree = (int64_t)hs[0];
    G.segments = (int64_t)hs[1];
    if (greedy) {  // whole graph: greedy packing on the host instead
        std::vector<int32_t> hin((size_t)n + 1), p0, pub, lb;
        TPM_HIP(hipMemcpyAsync(hin.data(), G.inptr, sizeof(int32_t) * ((size_t)n + 1),
                               hipMemcpyDeviceToHost, st));
        TPM_HIP(hipStreamSynchronize(st));
        build_tiles(hin, T, p0, pub, lb, nslots);
        ntiles = (int64_t)pub.size();
        if (own) {
            *tp0 = dalloc<int32_t>(ntiles + 1, acct);
            *tpub = dalloc<int32_t>(ntiles, acct);
            *tlb = dalloc<int32_t>(ntiles, acct);
        } else {
            *tp0 = galloc<int32_t>(G, A_TP0, ntiles + 1, acct, st);
            *tpub = galloc<int32_t>(G, A_TPUB, ntiles, acct, st);
            *tlb = galloc<int32_t>(G, A_TLB, ntiles, acct, st);
        }
        TPM_HIP(hipMemcpyAsync(*tp0, p0.data(), sizeof(int32_t) * p0.size(), hipMemcpyHostToDevice, st));
        if (ntiles) {
            TPM_HIP(hipMemcpyAsync(*tpub, pub.data(), sizeof(int32_t) * pub.size(),
                                   hipMemcpyHostToDevice, st));
            TPM_HIP(hipMemcpyAsync(*tlb, lb.data(), sizeof(int32_t) * lb.size(),
                                   hipMemcpyHostToDevice, st));
        }
        TPM_HIP(hipStreamSynchronize(st));  // the host vectors go out of scope
        G.h_tile_p0 = std::move(p0);
        return;
    }
    if (own) {
        *tp0 = dalloc<int32_t>(ntiles + 1, acct);
        *tpub = dalloc<int32_t>(ntiles, acct);
        *tlb = dalloc<int32_t>(ntiles, acct);
    } else {
        *tp0 = galloc<int32_t>(G, A_TP0, ntiles + 1, acct, st);
        *tpub = galloc<int32_t>(G, A_TPUB, ntiles, acct, st);
        *tlb = galloc<int32_t>(G, A_TLB, ntiles, acct, st);
    }
    k_tile_fill<<<grid_for(n), 256, 0, st>>>(n, G.inptr, T, tcnt, tbase, sbase, *tp0, *tpub, *tlb);
    k_set1<<<1, 1, 0, st>>>(*tp0 + ntiles, (int32_t)G.m);
    G.h_tile_p0.resize((size_t)ntiles + 1);
    TPM_HIP(hipMemcpyAsync(G.h_tile_p0.data(), *tp0, sizeof(int32_t) * ((size_t)ntiles + 1),
                           hipMemcpyDeviceToHost, st));
    TPM_HIP(hipStreamSynchronize(st));
}

// The bank-replicated LOG/EXP image (kLdsBytes), built once per process.
const std::vector<uint8_t> &lds_image_host() {
    static const std::vector<uint8_t> img = [] {
        std::vector<uint8_t> v(kLdsBytes, 0);
        auto put32 = [&](size_t off, uint32_t x) { std::memcpy(v.data() + off, &x, 4); };
        for (int g = 0; g < 256; ++g) {
            const uint32_t l7 = g ? ((uint32_t)kGf.log[g] << 7) : kZero7;
            for (int c = 0; c < 32; ++c) put32((size_t)g * 256 + c * 4, l7);
        }
        for (int r = 0; r < kExpRows; ++r) {
            const uint32_t e = (r <= 762) ? kGf.exp[r % 255] : 0u;
            for (int c = 0; c < 32; ++c) put32((size_t)kExpBase + (size_t)r * 128 + c * 4, e);
        }
        return v;
    }();
    return img;
}

}  // namespace

int32_t auto_tile_edges(int64_t m) {
    // a sweep of T = 64..1024 (k = 8 sieves): best 128 at m = 2e4 and 2e5, 512 at 2e6,
    // 1024 at 1e7 (k = 5) and above
    return (int32_t)std::min<int64_t>(1024, std::max<int64_t>(128, m / 4096));
}

void free_graph(Graph &G) {
    int32_t **ptrs[] = {&G.color, &G.pdst,  &G.psrc,    &G.ptau,     &G.peid,   &G.gsrc,
                        &G.orow,  &G.inptr, &G.tile_p0, &G.tile_pub, &G.tile_lb,
                        &G.ttab,  &G.pdep,  &G.vdelay, &G.fid,      &G.gposw};
    const bool own = G.arena == nullptr;  // arena memory stays with the arena
    for (auto pp : ptrs) {
        if (*pp && own) (void)hipFree(*pp);
        *pp = nullptr;
    }
    if (G.lds_image && own) (void)hipFree(G.lds_image);
    G.lds_image = nullptr;
    if (G.pcol && own) (void)hipFree(G.pcol);
    G.pcol = nullptr;
}

void build_pcol(Graph &G, int64_t &acct) {
    if (G.arena || G.q > 64 || G.m == 0) return;
    if (!G.pcol) G.pcol = dalloc<uint16_t>(G.m, acct);
    k_pcol<<<grid_for(G.m), 256>>>(G.m, G.psrc, G.pdst, G.color, G.pcol);
    TPM_HIP(hipDeviceSynchronize());
}

// Edge counts by (source colour, head colour) from the colour pairs of the positions:
// one LDS histogram per workgroup, merged with global atomics.
__global__ void k_pair_hist(int64_t m, const uint16_t *pcol, int32_t q,
                            unsigned long long *out) {
    __shared__ unsigned int h[64 * 64];
    const int nb = q * q;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += stride) {
        const uint32_t pc = pcol[p];
        atomicAdd(&h[(pc & 0xFFu) * q + (pc >> 8)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
        if (h[i]) atomicAdd(&out[i], (unsigned long long)h[i]);
}

void colour_pair_counts(const Graph &G, std::vector<int64_t> &out, hipStream_t st) {
    TPM_REQUIRE(G.q <= 64, "colour pair counts need at most 64 colours");
    const int nb = G.q * G.q;
    out.assign((size_t)nb, 0);
    if (G.m == 0) return;
    TPM_REQUIRE(G.pcol != nullptr, "colour pair counts need the colour pairs of a whole graph");
    unsigned long long *d = nullptr;
    TPM_HIP(hipMalloc(&d, sizeof(unsigned long long) * (size_t)nb));
    std::vector<unsigned long long> h((size_t)nb, 0);
    hipError_t e = hipMemcpyAsync(d, h.data(), sizeof(unsigned long long) * (size_t)nb,
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        const unsigned grid = std::min<unsigned>(grid_for(G.m), 4 * std::max(1, G.num_cu));
        k_pair_hist<<<grid, 256, 0, st>>>(G.m, G.pcol, G.q, d);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), d, sizeof(unsigned long long) * (size_t)nb,
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    TPM_HIP(e);
    for (int i = 0; i < nb; ++i) out[(size_t)i] = (int64_t)h[(size_t)i];
}

// Everything of the index that follows from the CSR arrays (pdst, psrc, ptau, peid
// sorted by (dst, tau, input id)), G.color and G.tmax: distinct timestamps, in-list
// offsets, gathered and stored rows, host copies, tiles and the LDS image.  taus:
// the m timestamps in any order (device).
// gpos_pre (nullable, device [m]): read positions already known (pruned graphs), with
// needed_pre (nullable, m bytes): the positions they read (1) and the others (0)
// lds_shared (nullable): an LDS image to use instead of a new one (subgraphs in an
// arena use their parent's); need_times = false skips the distinct-timestamp table.
void finish_index(Graph &G, int64_t &acct, const int32_t *taus, bool greedy_tiles,
                  const int32_t *gpos_pre = nullptr, hipStream_t st = nullptr,
                  bool need_times = true, uint8_t *lds_shared = nullptr,
                  uint8_t *needed_pre = nullptr) {
    const int64_t m = G.m;
    const int32_t n = G.n;
    const int32_t tmax = G.tmax;
    const int32_t T = G.tile_edges;
    Temps tmp(G.arena, st);
    if (m && need_times) {
        // ---- distinct timestamps, ascending (per-time splits of the sieve)
        const int tbits = bits_for((uint64_t)tmax);
        int32_t *tsort = tmp.get<int32_t>(A_TSORT, m);
        int32_t *tuniq = tmp.get<int32_t>(A_TUNIQ, m);
        int64_t *tcount = tmp.get<int64_t>(A_TCOUNT, 1);
        size_t sbytes = 0, ubytes = 0;
        TPM_HIP(rocprim::radix_sort_keys(nullptr, sbytes, taus, tsort, (size_t)m, 0,
                                         (unsigned)tbits, st));
        TPM_HIP(rocprim::unique(nullptr, ubytes, tsort, tuniq, tcount, (size_t)m,
                                rocprim::equal_to<int32_t>(), st));
        void *scratch = tmp.raw(A_SCRATCH, std::max(sbytes, ubytes));
        TPM_HIP(rocprim::radix_sort_keys(scratch, sbytes, taus, tsort, (size_t)m, 0,
                                         (unsigned)tbits, st));
        TPM_HIP(rocprim::unique(scratch, ubytes, tsort, tuniq, tcount, (size_t)m,
                                rocprim::equal_to<int32_t>(), st));
        int64_t nt = 0;
        TPM_HIP(hipMemcpyAsync(&nt, tcount, sizeof(nt), hipMemcpyDeviceToHost, st));
        TPM_HIP(hipStreamSynchronize(st));
        G.ntimes = nt;
        G.ttab = galloc<int32_t>(G, A_TTAB, nt, acct, st);
        TPM_HIP(hipMemcpyAsync(G.ttab, tuniq, sizeof(int32_t) * (size_t)nt, hipMemcpyDeviceToDevice, st));
        G.h_ttab.resize((size_t)nt);
        TPM_HIP(hipMemcpyAsync(G.h_ttab.data(), tuniq, sizeof(int32_t) * (size_t)nt,
                               hipMemcpyDeviceToHost, st));
    }
    k_inptr<<<grid_for(m + 1), 256, 0, st>>>(m, n, G.pdst, G.inptr);
    if (m) {
        // needed positions (some edge reads them) as byte flags, then rank records; rows
        // are their ranks
        const int64_t nr = rank_recs(m);
        uint8_t *flags = needed_pre;
        if (!flags) {
            uint8_t *nf = tmp.get<uint8_t>(A_NFLAG, m);
            TPM_HIP(hipMemsetAsync(nf, 0, (size_t)m, st));
            flags = nf;
        }
        const int32_t *gpos = gpos_pre;
        if (gpos) {
            if (!needed_pre) k_needed<<<grid_for(m), 256, 0, st>>>(m, gpos, flags);
        } else {
            int32_t *gp = tmp.get<int32_t>(A_GPOS, m);
            k_gpos<<<grid_for(m), 256, 0, st>>>(m, G.psrc, G.ptau, G.pdep, G.vdelay, G.inptr, gp,
                                                flags);
            gpos = gp;
        }
        uint32_t *needed = tmp.get<uint32_t>(A_NBITS, nr * 32);
        int32_t *ncnt = tmp.get<int32_t>(A_NCNT, nr + 1);
        int32_t *nbase = tmp.get<int32_t>(A_NBASE, nr + 1);
        k_pack<<<grid_for(nr * 64), 256, 0, st>>>(m, nr, flags, needed, ncnt);
        size_t sbytes = 0;
        TPM_HIP(rocprim::exclusive_scan(nullptr, sbytes, ncnt, nbase, 0, (size_t)(nr + 1),
                                        rocprim::plus<int32_t>(), st));
        void *scratch = tmp.raw(A_SCRATCH, sbytes);
        TPM_HIP(rocprim::exclusive_scan(scratch, sbytes, ncnt, nbase, 0, (size_t)(nr + 1),
                                        rocprim::plus<int32_t>(), st));
        k_put_base<<<grid_for(nr), 256, 0, st>>>(nr, nbase, needed);
        k_rows<<<(unsigned)(nr * 4), 256, 0, st>>>(m, gpos, needed, nr, nbase + nr, G.orow, G.gsrc);
        int32_t rows = 0;
        unsigned long long *cnt = tmp.get<unsigned long long>(A_CNT, 1);
        TPM_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), st));
        k_count_nonneg<<<std::min<unsigned>(grid_for(m), 4096), 256, 0, st>>>(m, G.gsrc, cnt);
        unsigned long long h = 0;
        TPM_HIP(hipMemcpyAsync(&rows, nbase + nr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        TPM_HIP(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, st));
        TPM_HIP(hipStreamSynchronize(st));
        G.R = (int64_t)rows;
        G.gathers = (int64_t)h;
        if (!G.arena) {  // whole graphs keep the read positions for pruning
            G.gposw = galloc<int32_t>(G, A_GPOSW, m, acct, st);
            TPM_HIP(hipMemcpyAsync(G.gposw, gpos, sizeof(int32_t) * (size_t)m,
                                   hipMemcpyDeviceToDevice, st));
        }
    }
    if (!G.h_color_sp || G.h_color().size() != (size_t)n) {
        G.h_color_mut().resize((size_t)n);
        TPM_HIP(hipMemcpyAsync(G.h_color_mut().data(), G.color, sizeof(int32_t) * (size_t)n,
                               hipMemcpyDeviceToHost, st));
    }
    // window grouping makes tiles of up to two windows: windows of T / 2 keep them
    // within T positions, as the greedy packing does
    build_tiles_device(G, greedy_tiles ? T : std::max<int32_t>(1, T / 2), tmp, acct, &G.tile_p0,
                       &G.tile_pub, &G.tile_lb, G.ntiles, G.nslots, false, greedy_tiles, st);

    if (lds_shared) {
        G.lds_image = lds_shared;  // the parent's (never freed through an arena graph)
    } else {
        G.lds_image = galloc<uint8_t>(G, A_LDS, kLdsBytes, acct, st);
        TPM_HIP(hipMemcpyAsync(G.lds_image, lds_image_host().data(), kLdsBytes,
                               hipMemcpyHostToDevice, st));
    }
    TPM_HIP(hipStreamSynchronize(st));
    build_pcol(G, acct);
}

void build_graph(Graph &G, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                 const int32_t *tau, const int32_t *color, int32_t num_colors, uint32_t flags,
                 const tpm_graph_options *opt) {
    TPM_REQUIRE(n >= 1, "n must be >= 1");
    TPM_REQUIRE(m >= 0 && m < (int64_t(1) << 31) - 1, "m must be in [0, 2^31 - 1)");
    TPM_REQUIRE(num_colors >= 1, "num_colors must be >= 1");
    TPM_REQUIRE(m == 0 || (src && dst && tau), "edge arrays must not be NULL");
    TPM_REQUIRE(color != nullptr, "color must not be NULL");
    int T = 0;  // 0: chosen from m below
    if (opt && opt->tile_edges) T = opt->tile_edges;
    TPM_REQUIRE(T == 0 || (T >= 1 && T <= 4096), "tile_edges must be in [1, 4096]");
    TPM_REQUIRE(!opt || opt->tile_held == 0, "tile_held is reserved and must be 0");
    const bool on_dev = (flags & TPM_DEVICE_PTRS) != 0;
    const bool undirected = (flags & TPM_UNDIRECTED) != 0;
    TPM_REQUIRE((flags & ~(TPM_DEVICE_PTRS | TPM_UNDIRECTED)) == 0, "unknown flag bits");
    TPM_REQUIRE(!undirected || 2 * m < (int64_t(1) << 31) - 1,
                "an undirected graph needs 2m < 2^31 - 1");

    const int32_t *transit = opt ? opt->transit : nullptr;  // host, per edge
    const int32_t *delay = opt ? opt->delay : nullptr;      // host, per vertex

    // ---- validation of host arrays happens before any device work
    int32_t tmax = 0;  // largest arrival time
    if (!on_dev) {
        for (int64_t e = 0; e < m; ++e) {
            int32_t s = src[e], d = dst[e], t = tau[e];
            TPM_REQUIRE(s >= 0 && s < n && d >= 0 && d < n, "edge endpoint out of range");
            TPM_REQUIRE(t >= 1, "timestamps must be >= 1");
            int64_t a = t;
            if (transit) {
                TPM_REQUIRE(transit[e] >= 0, "transition times must be >= 0");
                a += transit[e];
                TPM_REQUIRE(a <= 0x7FFFFFFF, "timestamp + transition time must be < 2^31");
            }
            tmax = std::max(tmax, (int32_t)a);
        }
        for (int32_t u = 0; u < n; ++u)
            TPM_REQUIRE(color[u] >= 0 && color[u] < num_colors, "colour out of range");
    }
    if (delay)
        for (int32_t u = 0; u < n; ++u)
            TPM_REQUIRE(delay[u] >= 0 && delay[u] <= (1 << 30), "delays must be in [0, 2^30]");
    // undirected: edge e is also the arc dst -> src, input id e + m, same time
    const int64_t m_in = m;
    std::vector<int32_t> transit2;
    if (undirected) {
        if (transit) {
            transit2.assign(transit, transit + m_in);
            transit2.insert(transit2.end(), transit, transit + m_in);
            transit = transit2.data();
        }
        m = 2 * m_in;
    }

    TPM_HIP(hipGetDevice(&G.device));
    hipDeviceProp_t prop;
    TPM_HIP(hipGetDeviceProperties(&prop, G.device));
    G.num_cu = prop.multiProcessorCount;
    G.n = n;
    G.m = m;
    G.q = num_colors;
    G.tile_auto = T == 0;
    G.tile_edges = T ? T : auto_tile_edges(m);
    G.edge_ids = m;
    int64_t acct = 0;
    hipStream_t st = nullptr;

    int32_t *d_src = nullptr, *d_dst = nullptr, *d_tau = nullptr, *d_arr = nullptr;
    int64_t tmp = 0;
    uint64_t *keys = nullptr, *keys2 = nullptr;
    int32_t *vals = nullptr, *vals2 = nullptr;
    void *scratch = nullptr;
    auto cleanup_tmp = [&]() {
        for (void *p : {(void *)d_src, (void *)d_dst, (void *)d_tau, (void *)d_arr, (void *)keys,
                        (void *)keys2, (void *)vals, (void *)vals2, scratch})
            if (p) (void)hipFree(p);
    };
    try {
        G.color = dalloc<int32_t>(n, acct);
        d_src = dalloc<int32_t>(m, tmp);
        d_dst = dalloc<int32_t>(m, tmp);
        d_tau = dalloc<int32_t>(m, tmp);
        hipMemcpyKind kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        TPM_HIP(hipMemcpy(G.color, color, sizeof(int32_t) * n, kind));
        if (m_in) {
            TPM_HIP(hipMemcpy(d_src, src, sizeof(int32_t) * m_in, kind));
            TPM_HIP(hipMemcpy(d_dst, dst, sizeof(int32_t) * m_in, kind));
            TPM_HIP(hipMemcpy(d_tau, tau, sizeof(int32_t) * m_in, kind));
            if (undirected) {
                TPM_HIP(hipMemcpy(d_src + m_in, dst, sizeof(int32_t) * m_in, kind));
                TPM_HIP(hipMemcpy(d_dst + m_in, src, sizeof(int32_t) * m_in, kind));
                TPM_HIP(hipMemcpy(d_tau + m_in, tau, sizeof(int32_t) * m_in, kind));
            }
        }
        if (on_dev) {
            int32_t *flagbuf = dalloc<int32_t>(2, tmp);
            TPM_HIP(hipMemset(flagbuf, 0, 2 * sizeof(int32_t)));
            if (m)
                k_validate<<<std::min<unsigned>(grid_for(m), 4096), 256, 0, st>>>(
                    m, n, d_src, d_dst, d_tau, flagbuf, flagbuf + 1);
            k_validate_color<<<grid_for(n), 256, 0, st>>>(n, num_colors, G.color, flagbuf);
            int32_t h[2];
            TPM_HIP(hipMemcpy(h, flagbuf, sizeof(h), hipMemcpyDeviceToHost));
            (void)hipFree(flagbuf);
            TPM_REQUIRE(!(h[0] & 1), "edge endpoint out of range or timestamp < 1");
            TPM_REQUIRE(!(h[0] & 2), "colour out of range");
            tmax = h[1];
        }
        // ---- transition times: in-lists are ordered by arrival, departures kept apart
        if (transit && m) {
            d_arr = dalloc<int32_t>(m, tmp);
            int32_t *flagbuf = dalloc<int32_t>(2, tmp);
            TPM_HIP(hipMemset(flagbuf, 0, 2 * sizeof(int32_t)));
            TPM_HIP(hipMemcpy(d_arr, transit, sizeof(int32_t) * m, hipMemcpyHostToDevice));
            k_arrival<<<std::min<unsigned>(grid_for(m), 4096), 256, 0, st>>>(m, d_tau, d_arr, d_arr,
                                                                            flagbuf, flagbuf + 1);
            int32_t h[2];
            TPM_HIP(hipMemcpy(h, flagbuf, sizeof(h), hipMemcpyDeviceToHost));
            (void)hipFree(flagbuf);
            TPM_REQUIRE(!(h[0] & 4), "transition times must be >= 0 with timestamp + transition < 2^31");
            tmax = std::max(tmax, h[1]);
            G.pdep = dalloc<int32_t>(m, acct);
        }
        if (delay) {
            G.vdelay = dalloc<int32_t>(n, acct);
            TPM_HIP(hipMemcpy(G.vdelay, delay, sizeof(int32_t) * n, hipMemcpyHostToDevice));
            G.h_delay.assign(delay, delay + n);
        }
        const int32_t *d_order_t = d_arr ? d_arr : d_tau;  // arrival times
        G.tmax = tmax;

        G.pdst = dalloc<int32_t>(m, acct);
        G.psrc = dalloc<int32_t>(m, acct);
        G.ptau = dalloc<int32_t>(m, acct);
        G.peid = dalloc<int32_t>(m, acct);
        G.gsrc = dalloc<int32_t>(m, acct);
        G.orow = dalloc<int32_t>(m, acct);
        G.inptr = dalloc<int32_t>((int64_t)n + 1, acct);

        if (m) {
            // ---- sort positions by (dst, tau, id): stable radix sort of (dst, tau) keys
            const int tbits = bits_for((uint64_t)tmax);
            const int nbits = bits_for((uint64_t)(n - 1));
            keys = dalloc<uint64_t>(m, tmp);
            keys2 = dalloc<uint64_t>(m, tmp);
            vals = dalloc<int32_t>(m, tmp);
            vals2 = dalloc<int32_t>(m, tmp);
            k_keys<<<grid_for(m), 256, 0, st>>>(m, d_dst, d_order_t, tbits, keys, vals);
            size_t sbytes = 0;
            TPM_HIP(rocprim::radix_sort_pairs(nullptr, sbytes, keys, keys2, vals, vals2, (size_t)m,
                                              0, (unsigned)(tbits + nbits), st));
            TPM_HIP(hipMalloc(&scratch, std::max<size_t>(sbytes, 16)));
            TPM_HIP(rocprim::radix_sort_pairs(scratch, sbytes, keys, keys2, vals, vals2, (size_t)m,
                                              0, (unsigned)(tbits + nbits), st));
            k_apply<<<grid_for(m), 256, 0, st>>>(m, vals2, d_src, d_dst, d_order_t,
                                                 d_arr ? d_tau : nullptr, G.psrc, G.pdst, G.ptau,
                                                 G.pdep, G.peid);
            (void)hipFree(keys);
            keys = nullptr;
            (void)hipFree(keys2);
            keys2 = nullptr;
            (void)hipFree(scratch);
            scratch = nullptr;
        }
        finish_index(G, acct, d_order_t, true);
        G.device_bytes = acct;
    } catch (...) {
        cleanup_tmp();
        free_graph(G);
        throw;
    }
    cleanup_tmp();
}

void prune_graph(const Graph &P, const PruneSpec &spec, Graph &G, GraphArena *arena,
                 hipStream_t st) {
    const uint8_t *keep_color = spec.keep_color, *vkeep_in = spec.vkeep;
    const int32_t *times = spec.times;
    const int32_t ntimes = spec.ntimes;
    TPM_HIP(hipSetDevice(P.device));
    G.device = P.device;
    G.num_cu = P.num_cu;
    G.n = P.n;
    G.q = P.q;
    G.tmax = P.tmax;
    G.tile_edges = P.tile_edges;
    G.edge_ids = P.edge_ids;
    G.arena = arena;
    G.h_color_sp = P.h_color_sp;  // shared: colours are P's
    G.h_delay = P.h_delay;
    G.h_fid = P.h_fid;
    int64_t acct = 0;
    try {
        int64_t mk = 0;
        uint32_t *keep = nullptr;  // kept-position records of the parent's m positions
        int32_t *kbase = nullptr;  // their bases (nrk + 1: the last one the total)
        const int64_t nrk = rank_recs(P.m);
        Temps outer(arena, st);
        int32_t *gpos_pre = nullptr;  // read positions mapped from the parent's
        uint8_t *needed_pre = nullptr;  // the positions they read (byte flags)
        {
            Temps tmp(arena, st);
            G.color = galloc<int32_t>(G, A_COLOR, P.n, acct, st);
            TPM_HIP(hipMemcpyAsync(G.color, P.color, sizeof(int32_t) * (size_t)P.n,
                                   hipMemcpyDeviceToDevice, st));
            if (P.m) {
                uint8_t *keepc = tmp.get<uint8_t>(A_KEEPC, P.q);
                if (keep_color) {
                    TPM_HIP(hipMemcpyAsync(keepc, keep_color, (size_t)P.q, hipMemcpyHostToDevice, st));
                } else {
                    TPM_HIP(hipMemsetAsync(keepc, 1, (size_t)P.q, st));
                }
                uint8_t *vkeep = tmp.get<uint8_t>(A_VKEEP, P.n);
                k_vkeep<<<grid_for(P.n), 256, 0, st>>>(P.n, P.color, keepc, vkeep);
                if (vkeep_in)
                    k_vand<<<grid_for(P.n), 256, 0, st>>>(P.n, vkeep_in, vkeep);
                uint32_t *vbits = tmp.get<uint32_t>(A_VBITS, ((int64_t)P.n + 31) / 32);
                k_vbits<<<grid_for(((int64_t)P.n + 31) / 32), 256, 0, st>>>(P.n, vkeep, vbits);
                int32_t *ts = nullptr;
                if (times) {
                    ts = tmp.get<int32_t>(A_TSET, ntimes);
                    TPM_HIP(hipMemcpyAsync(ts, times, sizeof(int32_t) * (size_t)ntimes,
                                           hipMemcpyHostToDevice, st));
                }
                keep = tmp.get<uint32_t>(A_KBITS, nrk * 32);
                int32_t *kcnt = tmp.get<int32_t>(A_KCNT, nrk + 1);
                kbase = tmp.get<int32_t>(A_KBASE, nrk + 1);
                // timestamps of the edges as given (departures when transit times exist)
                if (P.pcol && !vkeep_in && spec.cut_in < 0 && spec.cut_out < 0 && P.q <= 64) {
                    uint64_t cm = 0;
                    std::vector<uint8_t> kc((size_t)P.q, 1);
                    if (keep_color) std::copy(keep_color, keep_color + P.q, kc.begin());
                    for (int32_t c = 0; c < P.q; ++c)
                        if (kc[(size_t)c]) cm |= 1ull << c;
                    // both endpoints of every kept edge have a colour of cm
                    G.edge_colors = cm;
                    k_keep_pc<<<grid_for(nrk * 64), 256, 0, st>>>(P.m, nrk, P.pcol, cm,
                                                                   P.pdep ? P.pdep : P.ptau, ts,
                                                                   ntimes, P.ptau, spec.tcut, keep,
                                                                   kcnt);
                } else {
                    k_keep<<<grid_for(nrk * 64), 256, 0, st>>>(P.m, nrk, P.psrc, P.pdst, vbits,
                                                                P.pdep ? P.pdep : P.ptau, ts, ntimes,
                                                                spec.cut_in, spec.cut_out, P.ptau,
                                                                spec.tcut, keep, kcnt);
                }
                size_t sbytes = 0;
                TPM_HIP(rocprim::exclusive_scan(nullptr, sbytes, kcnt, kbase, 0, (size_t)(nrk + 1),
                                                rocprim::plus<int32_t>(), st));
                void *scratch = tmp.raw(A_SCRATCH, sbytes);
                TPM_HIP(rocprim::exclusive_scan(scratch, sbytes, kcnt, kbase, 0, (size_t)(nrk + 1),
                                                rocprim::plus<int32_t>(), st));
                k_put_base<<<grid_for(nrk), 256, 0, st>>>(nrk, kbase, keep);
                int32_t kept = 0;
                TPM_HIP(hipMemcpyAsync(&kept, kbase + nrk, sizeof(int32_t), hipMemcpyDeviceToHost, st));
                TPM_HIP(hipStreamSynchronize(st));
                mk = (int64_t)kept;
            }
            G.m = mk;
            G.tile_auto = P.tile_auto;
            if (P.tile_auto) G.tile_edges = auto_tile_edges(mk);
            G.pdst = galloc<int32_t>(G, A_PDST, mk, acct, st);
            G.psrc = galloc<int32_t>(G, A_PSRC, mk, acct, st);
            G.ptau = galloc<int32_t>(G, A_PTAU, mk, acct, st);
            G.peid = galloc<int32_t>(G, A_PEID, mk, acct, st);
            G.gsrc = galloc<int32_t>(G, A_GSRC, mk, acct, st);
            G.orow = galloc<int32_t>(G, A_OROW, mk, acct, st);
            G.inptr = galloc<int32_t>(G, A_INPTR, (int64_t)G.n + 1, acct, st);
            if (P.pdep) G.pdep = galloc<int32_t>(G, A_PDEP, mk, acct, st);
            if (P.fid) {
                G.fid = galloc<int32_t>(G, A_FID, P.n, acct, st);
                TPM_HIP(hipMemcpyAsync(G.fid, P.fid, sizeof(int32_t) * (size_t)P.n,
                                       hipMemcpyDeviceToDevice, st));
            }
            if (P.vdelay) {
                G.vdelay = galloc<int32_t>(G, A_VDELAY, P.n, acct, st);
                TPM_HIP(hipMemcpyAsync(G.vdelay, P.vdelay, sizeof(int32_t) * (size_t)P.n,
                                       hipMemcpyDeviceToDevice, st));
            }
            if (mk) {  // kept positions stay in (dst, arrival, id) order
                if (P.gposw) {  // read positions remapped from the parent's
                    gpos_pre = outer.get<int32_t>(A_GPOSP, mk);
                    needed_pre = outer.get<uint8_t>(A_NFLAGP, mk);
                    TPM_HIP(hipMemsetAsync(needed_pre, 0, (size_t)mk, st));
                    k_sub_inptr<<<grid_for((int64_t)P.n + 1), 256, 0, st>>>(P.n, P.inptr, keep,
                                                                            nrk, kbase + nrk, G.inptr);
                }
                k_compact<<<grid_for(nrk * 64), 256, 0, st>>>(nrk, keep, P.psrc, P.pdst,
                                                               P.ptau, P.peid, P.pdep, P.gposw,
                                                               G.psrc, G.pdst, G.ptau, G.peid,
                                                               G.pdep, gpos_pre);
                if (P.gposw)
                    k_remap<<<grid_for(mk), 256, 0, st>>>(mk, G.psrc, keep, nrk, kbase + nrk, G.inptr,
                                                          gpos_pre, needed_pre);
            }
            TPM_HIP(hipStreamSynchronize(st));
        }
        finish_index(G, acct, G.ptau, arena == nullptr, gpos_pre, st, spec.need_times,
                     arena ? P.lds_image : nullptr, needed_pre);
        G.device_bytes = acct;
    } catch (...) {
        free_graph(G);
        throw;
    }
}

namespace {
struct W2Op {
    __host__ __device__ W2Agg operator()(const W2Agg &a, const W2Agg &b) const {
        W2Agg o = b;
        if (!b.head) {
            o.v.x ^= a.v.x;
            o.v.y ^= a.v.y;
            o.v.z ^= a.v.z;
            o.v.w ^= a.v.w;
        }
        o.head = a.head | b.head;
        return o;
    }
};
}  // namespace

size_t w2_scan(void *tmp, size_t tmp_bytes, const W2Agg *in, W2Agg *out, int64_t n, hipStream_t st) {
    size_t bytes = 0;
    TPM_HIP(rocprim::inclusive_scan(nullptr, bytes, in, out, (size_t)std::max<int64_t>(1, n), W2Op(), st));
    if (!tmp) return bytes;
    TPM_REQUIRE(tmp_bytes >= bytes, "scan storage too small");
    TPM_HIP(rocprim::inclusive_scan(tmp, bytes, in, out, (size_t)n, W2Op(), st));
    return bytes;
}

void sd_graph(const Graph &P, int32_t s, int32_t d, Graph &G) {
    TPM_REQUIRE(s >= 0 && s < P.n && d >= 0 && d < P.n, "vertex out of range");
    TPM_REQUIRE(s != d, "s and d must differ");
    TPM_REQUIRE(P.q <= (int32_t)0x7FFFFFFD, "too many colours");
    PruneSpec spec;
    spec.cut_in = s;
    spec.cut_out = d;
    prune_graph(P, spec, G);
    try {
        G.q = P.q + 2;
        const int32_t cs = P.q, cd = P.q + 1;
        TPM_HIP(hipMemcpy(G.color + s, &cs, sizeof(int32_t), hipMemcpyHostToDevice));
        TPM_HIP(hipMemcpy(G.color + d, &cd, sizeof(int32_t), hipMemcpyHostToDevice));
        // own copy: s and d change colour
        G.h_color_sp = std::make_shared<std::vector<int32_t>>(P.h_color());
        G.h_color_mut()[(size_t)s] = cs;
        G.h_color_mut()[(size_t)d] = cd;
        int64_t acct = 0;
        if (G.q > 64 && G.pcol) {
            (void)hipFree(G.pcol);
            G.pcol = nullptr;
        }
        build_pcol(G, acct);
        G.device_bytes += acct;
    } catch (...) {
        free_graph(G);
        throw;
    }
}

void layer_graph(const Graph &P, const int32_t *tuple, int32_t k, Graph &G) {
    TPM_REQUIRE(k >= 1 && k <= 16, "k must be in [1, 16]");
    for (int i = 0; i < k; ++i) TPM_REQUIRE(tuple[i] >= 0 && tuple[i] < P.q, "colour out of range");
    TPM_HIP(hipSetDevice(P.device));
    // ---- vertices: layer l holds the vertices of colour tuple[l-1], in id order
    std::vector<int64_t> cnt((size_t)P.q, 0);
    std::vector<int32_t> rank((size_t)P.n);
    for (int32_t u = 0; u < P.n; ++u) rank[(size_t)u] = (int32_t)cnt[(size_t)P.h_color()[(size_t)u]]++;
    std::vector<int64_t> base((size_t)k + 1, 0);
    for (int l = 0; l < k; ++l) base[(size_t)l + 1] = base[(size_t)l] + cnt[(size_t)tuple[l]];
    int64_t nn = base[(size_t)k];
    TPM_REQUIRE(nn < (int64_t(1) << 31), "layered graph too large");
    G.device = P.device;
    G.num_cu = P.num_cu;
    G.q = P.q;
    G.tmax = P.tmax;
    G.tile_edges = P.tile_edges;
    G.edge_ids = P.edge_ids;
    std::vector<uint8_t> in_tuple((size_t)P.q, 0);
    for (int l = 0; l < k; ++l) in_tuple[(size_t)tuple[l]] = 1;
    if (nn == 0) {
        // no vertex has a colour of the tuple: one vertex of another colour, no edges
        int32_t other = 0;
        while (in_tuple[(size_t)other]) ++other;
        G.h_color_mut().assign(1, other);
        G.h_fid.assign(1, 0);
        if (!P.h_delay.empty()) G.h_delay.assign(1, 1);
        nn = 1;
    } else {
        G.h_color_mut().resize((size_t)nn);
        G.h_fid.resize((size_t)nn);
        if (!P.h_delay.empty()) G.h_delay.resize((size_t)nn);
        for (int l = 0; l < k; ++l)
            for (int32_t u = 0; u < P.n; ++u)
                if (P.h_color()[(size_t)u] == tuple[l]) {
                    const size_t i = (size_t)(base[(size_t)l] + rank[(size_t)u]);
                    G.h_color_mut()[i] = tuple[l];
                    G.h_fid[i] = P.h_fid.empty() ? u : P.h_fid[(size_t)u];
                    if (!P.h_delay.empty()) G.h_delay[i] = P.h_delay[(size_t)u];
                }
    }
    G.n = (int32_t)nn;
    int64_t acct = 0, tmp = 0;
    hipStream_t st = nullptr;
    int32_t *d_rank = nullptr, *keep = nullptr, *at = nullptr;
    void *scratch = nullptr;
    auto cleanup = [&]() {
        for (void *p : {(void *)d_rank, (void *)keep, (void *)at, scratch})
            if (p) (void)hipFree(p);
    };
    try {
        G.color = dalloc<int32_t>(G.n, acct);
        G.fid = dalloc<int32_t>(G.n, acct);
        TPM_HIP(hipMemcpy(G.color, G.h_color().data(), sizeof(int32_t) * (size_t)G.n, hipMemcpyHostToDevice));
        TPM_HIP(hipMemcpy(G.fid, G.h_fid.data(), sizeof(int32_t) * (size_t)G.n, hipMemcpyHostToDevice));
        if (!G.h_delay.empty()) {
            G.vdelay = dalloc<int32_t>(G.n, acct);
            TPM_HIP(hipMemcpy(G.vdelay, G.h_delay.data(), sizeof(int32_t) * (size_t)G.n,
                              hipMemcpyHostToDevice));
        }
        // ---- edges: layer l (2..k) takes P's edges v -> u with colours (tuple[l-2], tuple[l-1]),
        // in P's order (sorted by destination, then time), renumbered into the layers
        std::vector<int64_t> ml((size_t)k + 1, 0), off((size_t)k + 2, 0);
        if (P.m && nn > 1) {
            d_rank = dalloc<int32_t>(P.n, tmp);
            TPM_HIP(hipMemcpy(d_rank, rank.data(), sizeof(int32_t) * (size_t)P.n, hipMemcpyHostToDevice));
            keep = dalloc<int32_t>(P.m, tmp);
            at = dalloc<int32_t>(P.m, tmp);
            size_t sbytes = 0;
            TPM_HIP(rocprim::exclusive_scan(nullptr, sbytes, keep, at, 0, (size_t)P.m,
                                            rocprim::plus<int32_t>(), st));
            TPM_HIP(hipMalloc(&scratch, std::max<size_t>(sbytes, 16)));
            for (int l = 2; l <= k; ++l) {
                k_layer_keep<<<grid_for(P.m), 256, 0, st>>>(P.m, P.psrc, P.pdst, P.color,
                                                             tuple[l - 2], tuple[l - 1], keep);
                TPM_HIP(rocprim::exclusive_scan(scratch, sbytes, keep, at, 0, (size_t)P.m,
                                                rocprim::plus<int32_t>(), st));
                int32_t a = 0, b = 0;
                TPM_HIP(hipMemcpy(&a, at + (P.m - 1), sizeof(int32_t), hipMemcpyDeviceToHost));
                TPM_HIP(hipMemcpy(&b, keep + (P.m - 1), sizeof(int32_t), hipMemcpyDeviceToHost));
                ml[(size_t)l] = (int64_t)a + b;
            }
        }
        for (int l = 2; l <= k; ++l) off[(size_t)l + 1] = off[(size_t)l] + ml[(size_t)l];
        const int64_t mk = off[(size_t)k + 1];
        TPM_REQUIRE(mk < (int64_t(1) << 31) - 1, "layered graph has too many edges");
        G.m = mk;
        G.tile_auto = P.tile_auto;
        if (P.tile_auto) G.tile_edges = auto_tile_edges(mk);
        G.pdst = dalloc<int32_t>(mk, acct);
        G.psrc = dalloc<int32_t>(mk, acct);
        G.ptau = dalloc<int32_t>(mk, acct);
        G.peid = dalloc<int32_t>(mk, acct);
        G.gsrc = dalloc<int32_t>(mk, acct);
        G.orow = dalloc<int32_t>(mk, acct);
        G.inptr = dalloc<int32_t>((int64_t)G.n + 1, acct);
        if (P.pdep) G.pdep = dalloc<int32_t>(mk, acct);
        if (mk) {
            size_t sbytes = 0;
            TPM_HIP(rocprim::exclusive_scan(nullptr, sbytes, keep, at, 0, (size_t)P.m,
                                            rocprim::plus<int32_t>(), st));
            for (int l = 2; l <= k; ++l) {
                if (!ml[(size_t)l]) continue;
                k_layer_keep<<<grid_for(P.m), 256, 0, st>>>(P.m, P.psrc, P.pdst, P.color,
                                                             tuple[l - 2], tuple[l - 1], keep);
                TPM_HIP(rocprim::exclusive_scan(scratch, sbytes, keep, at, 0, (size_t)P.m,
                                                rocprim::plus<int32_t>(), st));
                k_layer_compact<<<grid_for(P.m), 256, 0, st>>>(
                    P.m, keep, at, (int32_t)off[(size_t)l], P.psrc, P.pdst, P.ptau, P.peid, P.pdep,
                    d_rank, (int32_t)base[(size_t)l - 2], (int32_t)base[(size_t)l - 1], G.psrc,
                    G.pdst, G.ptau, G.peid, G.pdep);
            }
        }
        TPM_HIP(hipDeviceSynchronize());
        cleanup();
        d_rank = keep = at = nullptr;
        scratch = nullptr;
        finish_index(G, acct, G.ptau, true);
        G.device_bytes = acct;
    } catch (...) {
        cleanup();
        free_graph(G);
        throw;
    }
}

void retile_graph(Graph &G, int32_t T) {
    TPM_REQUIRE(T >= 1 && T <= 4096, "tile_edges must be in [1, 4096]");
    if (T == G.tile_edges) return;
    TPM_REQUIRE(G.arena == nullptr, "graphs built in an arena are not retiled");
    TPM_HIP(hipSetDevice(G.device));
    int64_t acct = 0, nt = 0, nslots = 0;
    int32_t *p0 = nullptr, *pb = nullptr, *lb = nullptr;
    std::vector<int32_t> old_h = G.h_tile_p0;
    try {
        Temps tmp(nullptr);
        build_tiles_device(G, T, tmp, acct, &p0, &pb, &lb, nt, nslots, true, true, nullptr);
    } catch (...) {
        for (void *q : {(void *)p0, (void *)pb, (void *)lb})
            if (q) (void)hipFree(q);
        G.h_tile_p0 = std::move(old_h);
        throw;
    }
    // the old tile arrays may still be read by work queued on other streams
    TPM_HIP(hipDeviceSynchronize());
    const int64_t old_bytes = (int64_t)sizeof(int32_t) * (3 * G.ntiles + 1);
    for (int32_t **q : {&G.tile_p0, &G.tile_pub, &G.tile_lb}) {
        if (*q) (void)hipFree(*q);
    }
    G.tile_p0 = p0;
    G.tile_pub = pb;
    G.tile_lb = lb;
    G.ntiles = nt;
    G.nslots = nslots;
    G.tile_edges = T;
    G.tile_auto = false;
    G.device_bytes += acct - old_bytes;
}


// ------------------------------------------------------------------ static instance
namespace {

// live[p] = 1 for a position whose edge joins two live vertices and is not a loop
__global__ void k_arc_flag(int64_t m, const int32_t *psrc, const int32_t *pdst,
                           const uint8_t *vlive, int32_t *flag) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < m) {
        const int32_t s = psrc[p], d = pdst[p];
        flag[p] = (s != d && vlive[s] && vlive[d]) ? 1 : 0;
    }
}

// key (head << bt | tail) and input id of each flagged position, compacted
__global__ void k_arc_keys(int64_t m, const int32_t *psrc, const int32_t *pdst, const int32_t *peid,
                           const int32_t *flag, const int32_t *at, int bt, uint64_t *keys,
                           int32_t *ids) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < m && flag[p]) {
        const int32_t q = at[p];
        keys[q] = ((uint64_t)(uint32_t)pdst[p] << bt) | (uint64_t)(uint32_t)psrc[p];
        ids[q] = peid[p];
    }
}

__global__ void k_arc_mark(int64_t na, const uint64_t *keys, int bt, int32_t *on) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < na) {
        const uint64_t key = keys[a];
        on[key >> bt] = 1;
        on[key & ((uint64_t(1) << bt) - 1)] = 1;
    }
}

__global__ void k_vid(int32_t n, const int32_t *on, const int32_t *cid, int32_t *vid) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n && on[u]) vid[cid[u]] = (int32_t)u;
}

// by-head list in compact ids, and the swapped keys for the by-tail order
__global__ void k_arc_in(int64_t na, const uint64_t *keys, const int32_t *ids, const int32_t *cid,
                         int bt, int32_t *seg, int32_t *gat, int32_t *key, uint64_t *rkeys,
                         int32_t *ridx) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < na) {
        const uint64_t k = keys[a];
        const uint64_t head = k >> bt, tail = k & ((uint64_t(1) << bt) - 1);
        seg[a] = cid[head];
        gat[a] = cid[tail];
        key[a] = ids[a];
        rkeys[a] = (tail << bt) | head;
        ridx[a] = (int32_t)a;
    }
}

__global__ void k_arc_out(int64_t na, const uint64_t *rkeys, const int32_t *ridx, const int32_t *cid,
                          const int32_t *in_key, int bt, int32_t *seg, int32_t *gat, int32_t *key) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < na) {
        const uint64_t k = rkeys[a];
        seg[a] = cid[k >> bt];
        gat[a] = cid[k & ((uint64_t(1) << bt) - 1)];
        key[a] = in_key[ridx[a]];
    }
}

}  // namespace

void free_static(StaticGraph &S) {
    for (int32_t **q : {&S.vid, &S.in_seg, &S.in_gat, &S.in_key, &S.out_seg, &S.out_gat, &S.out_key}) {
        if (*q) (void)hipFree(*q);
        *q = nullptr;
    }
    S.n = 0;
    S.m = 0;
}

void build_static(const Graph &G, const uint8_t *vlive, StaticGraph &S) {
    TPM_HIP(hipSetDevice(G.device));
    hipStream_t st = nullptr;
    const int bt = std::max(1, bits_for((uint64_t)std::max<int32_t>(1, G.n - 1)));
    int64_t acct = 0;
    try {
        Temps tmp(nullptr);
        int64_t na = 0;
        uint64_t *keys = nullptr;
        int32_t *ids = nullptr;
        if (G.m) {
            int32_t *flag = tmp.get<int32_t>(0, G.m), *at = tmp.get<int32_t>(0, G.m);
            k_arc_flag<<<grid_for(G.m), 256, 0, st>>>(G.m, G.psrc, G.pdst, vlive, flag);
            size_t sb = 0;
            TPM_HIP(rocprim::exclusive_scan(nullptr, sb, flag, at, 0, (size_t)G.m,
                                            rocprim::plus<int32_t>(), st));
            void *scratch = tmp.raw(0, sb);
            TPM_HIP(rocprim::exclusive_scan(scratch, sb, flag, at, 0, (size_t)G.m,
                                            rocprim::plus<int32_t>(), st));
            int32_t h[2];
            TPM_HIP(hipMemcpy(&h[0], at + (G.m - 1), sizeof(int32_t), hipMemcpyDeviceToHost));
            TPM_HIP(hipMemcpy(&h[1], flag + (G.m - 1), sizeof(int32_t), hipMemcpyDeviceToHost));
            const int64_t ne = (int64_t)h[0] + h[1];
            if (ne) {
                uint64_t *k0 = tmp.get<uint64_t>(0, ne), *k1 = tmp.get<uint64_t>(0, ne);
                int32_t *v0 = tmp.get<int32_t>(0, ne), *v1 = tmp.get<int32_t>(0, ne);
                k_arc_keys<<<grid_for(G.m), 256, 0, st>>>(G.m, G.psrc, G.pdst, G.peid, flag, at,
                                                          bt, k0, v0);
                size_t rb = 0;
                TPM_HIP(rocprim::radix_sort_pairs(nullptr, rb, k0, k1, v0, v1, (size_t)ne, 0,
                                                  (unsigned)(2 * bt), st));
                void *rs = tmp.raw(0, rb);
                TPM_HIP(rocprim::radix_sort_pairs(rs, rb, k0, k1, v0, v1, (size_t)ne, 0,
                                                  (unsigned)(2 * bt), st));
                // one arc per (head, tail): the smallest input id of its edges
                int32_t *cnt = tmp.get<int32_t>(0, 1);
                size_t ub = 0;
                TPM_HIP(rocprim::reduce_by_key(nullptr, ub, k1, v1, (size_t)ne, k0, v0, cnt,
                                               rocprim::minimum<int32_t>(),
                                               rocprim::equal_to<uint64_t>(), st));
                void *us = tmp.raw(0, ub);
                TPM_HIP(rocprim::reduce_by_key(us, ub, k1, v1, (size_t)ne, k0, v0, cnt,
                                               rocprim::minimum<int32_t>(),
                                               rocprim::equal_to<uint64_t>(), st));
                int32_t c = 0;
                TPM_HIP(hipMemcpy(&c, cnt, sizeof(int32_t), hipMemcpyDeviceToHost));
                na = c;
                keys = k0;
                ids = v0;
            }
        }
        S.m = na;
        if (na == 0) {
            S.n = 0;
            TPM_HIP(hipDeviceSynchronize());
            return;
        }
        // compact ids of the vertices on an arc
        int32_t *on = tmp.get<int32_t>(0, G.n), *cid = tmp.get<int32_t>(0, G.n);
        TPM_HIP(hipMemsetAsync(on, 0, sizeof(int32_t) * (size_t)G.n, st));
        k_arc_mark<<<grid_for(na), 256, 0, st>>>(na, keys, bt, on);
        size_t sb = 0;
        TPM_HIP(rocprim::exclusive_scan(nullptr, sb, on, cid, 0, (size_t)G.n,
                                        rocprim::plus<int32_t>(), st));
        void *scratch = tmp.raw(0, sb);
        TPM_HIP(rocprim::exclusive_scan(scratch, sb, on, cid, 0, (size_t)G.n,
                                        rocprim::plus<int32_t>(), st));
        int32_t h[2];
        TPM_HIP(hipMemcpy(&h[0], cid + (G.n - 1), sizeof(int32_t), hipMemcpyDeviceToHost));
        TPM_HIP(hipMemcpy(&h[1], on + (G.n - 1), sizeof(int32_t), hipMemcpyDeviceToHost));
        S.n = h[0] + h[1];
        S.vid = dalloc<int32_t>(S.n, acct);
        k_vid<<<grid_for(G.n), 256, 0, st>>>(G.n, on, cid, S.vid);
        S.in_seg = dalloc<int32_t>(na, acct);
        S.in_gat = dalloc<int32_t>(na, acct);
        S.in_key = dalloc<int32_t>(na, acct);
        S.out_seg = dalloc<int32_t>(na, acct);
        S.out_gat = dalloc<int32_t>(na, acct);
        S.out_key = dalloc<int32_t>(na, acct);
        uint64_t *r0 = tmp.get<uint64_t>(0, na), *r1 = tmp.get<uint64_t>(0, na);
        int32_t *i0 = tmp.get<int32_t>(0, na), *i1 = tmp.get<int32_t>(0, na);
        k_arc_in<<<grid_for(na), 256, 0, st>>>(na, keys, ids, cid, bt, S.in_seg, S.in_gat, S.in_key,
                                               r0, i0);
        size_t rb = 0;
        TPM_HIP(rocprim::radix_sort_pairs(nullptr, rb, r0, r1, i0, i1, (size_t)na, 0,
                                          (unsigned)(2 * bt), st));
        void *rs = tmp.raw(0, rb);
        TPM_HIP(rocprim::radix_sort_pairs(rs, rb, r0, r1, i0, i1, (size_t)na, 0,
                                          (unsigned)(2 * bt), st));
        k_arc_out<<<grid_for(na), 256, 0, st>>>(na, r1, i1, cid, S.in_key, bt, S.out_seg,
                                                S.out_gat, S.out_key);
        TPM_HIP(hipDeviceSynchronize());
    } catch (...) {
        free_static(S);
        throw;
    }
}

}  // namespace tpm
