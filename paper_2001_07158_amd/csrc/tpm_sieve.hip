// Sieve kernels: evaluation of the temporal generating polynomial (Eq. (3)) at the
// points of the constrained multilinear sieve (Lemma "constrained multilinear
// sieving", Eq. (motif)) over GF(2^8), edge by edge over the in-edge CSR.
//
// Notation.  c_l[p] = x_u * y_{e,l-1} * H_{l-1}(p) for the edge e = (v -> u, tau) at
// CSR position p, where H_1 = x_v and, for l-1 >= 2, H_{l-1} = running XOR of c_{l-1}
// over v's in-list up to the last position earlier than tau (= P_{v,l-1,tau-1}).
// The running XOR after position p of u's in-list is P_{u,l,tau_p}; it is stored
// only at positions some later edge reads (its "row").  P_{k,t} = XOR_p c_k[p].
//
// Mapping.  One wavefront walks one tile of consecutive CSR positions; its 64 lanes
// hold the sieve points of the current chunk, 4*W points per lane (lanes = points,
// the paper's SIMD lanes over the 2^k evaluations).  For each edge all lanes gather
// the C-byte row of the predecessor value, multiply by x_u*y_e per point, and keep a
// per-lane running XOR (the segmented prefix over the in-list).
//
// Arithmetic.  Rows hold field elements (bytes).  The product x_u * y_e * g costs two
// LDS reads from bank-replicated tables: LOG7[g] (= log g << 7), then the EXP row
// min(log g + log x_u + log y_e, 763), where row 763 is zero and log 0 is so large
// that a zero factor always lands there.  log x_u is read once per in-list and
// log y_e once per edge, so a point costs one perm, one add3, one min and two
// conflict-free table reads.
//
// Long in-lists span several tiles.  Each tile of such a list publishes its running
// value as 64-bit words (epoch, status, value) — first AGGREGATE (this tile only),
// then INCLUSIVE (from the list head) — and later tiles add the values of earlier
// ones by walking back until an INCLUSIVE word (decoupled look-back, Merrill and
// Garland 2016).  Tiles are claimed from an atomic ticket, so a tile only ever waits
// for tiles claimed before it.  A continuation tile stores its rows without the
// carry, then adds the carry to them once the look-back has produced it.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "tpm_internal.h"

namespace tpm {

namespace {

__constant__ GfTables c_gf = make_gf_tables();

constexpr int kU = 8;                // edges per batch; two batches of gathers in flight
constexpr uint32_t kAgg = 1, kInc = 2;
constexpr uint32_t kSpinLimit = 1u << 24;

struct Ctl {
    uint32_t ticket;
    uint32_t epoch;
    uint32_t err;
    uint32_t pad;
};

struct QuerySlots {
    int32_t ncol;        // distinct colours of the multiset
    int32_t col[16];     // ascending
    int32_t off[16];     // first slot of the colour
    int32_t mu[16];      // multiplicity
};

struct LevelParams {
    const int32_t *gidx;   // row gathered by the edge at each position (-1: none)
    const uint8_t *gbase;  // gathered rows (log domain), rowb bytes each
    const int32_t *pdst;
    const int32_t *peid;
    const int32_t *orow;   // row stored at each position (-1: none)
    uint8_t *sout;         // stored rows
    const uint8_t *xt;     // per-vertex rows of x_u^A (bytes)
    const int32_t *tile_p0;
    const int32_t *tile_pub;
    const int32_t *tile_lb;
    int32_t tile_lo, tile_hi;
    int32_t pos_lo, pos_hi;  // last level: positions that contribute
    unsigned long long *pub;
    Ctl *ctl;
    uint32_t *fin;           // last level: per-point XOR accumulators (rowb/4 dwords)
    uint8_t *loc;            // last level: per-position localisation, index p - pos_lo
    const uint8_t *lds_image;
    uint64_t seed;
    uint32_t ylevel;         // walk position of y used at this level (= l - 1)
    int32_t rowb;            // bytes per row = sieve points per chunk
    int32_t lanes;           // lanes holding points = rowb / (4 W)
    int32_t valid_pts;       // points of the chunk that are sieve points (a row of 16
                             // points for 2^k < 16 repeats them; localisation skips the rest)
};

struct StepParams {
    const int32_t *psrc, *gsrc, *pdst, *peid, *orow;
    const uint16_t *pcol;  // colours of source and head per position; null: no skipping
    const uint8_t *xt;   // per-vertex rows of x for every lane group
    const uint8_t *sin;  // rows written by the previous step
    uint8_t *sout;       // rows written by this step
    const int32_t *tile_p0, *tile_pub, *tile_lb;
    int32_t ntiles;
    unsigned long long *pub;
    Ctl *ctl;
    uint32_t *fin;               // per-point accumulators of groups at their last level
    const uint8_t *lds_image;
    int32_t rowb, lanes;
    // How a lane finds y_{e, level} (see StepYPlan): 0 = its own full hash, 1 = the
    // inner hash is shared (one level, ylevel0), 2 = table of up to 8 (seed, level)
    // groups hashed once per 64 positions; the lane's group is in flags bits 8..10.
    int32_t ymode;
    uint32_t ylevel0;
    int32_t ngroups;
    uint32_t glevel[kMaxYGroups];
    uint64_t gseed[kMaxYGroups];
    uint64_t gmask[kMaxYGroups];  // colours the group's queries use (OR of their lanes)
    const StepLane *dtab;        // non-null: lane table and plan in device memory
                                 // (kTabStride entries), used instead of the above
    StepLane tab[64];            // per lane: seed, level, role
};

// SplitMix64 output function (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t fp8(uint64_t seed, uint32_t tag, uint32_t a, uint32_t b) {
    uint64_t key = ((uint64_t)tag << 56) ^ ((uint64_t)a << 32) ^ (uint64_t)b;
    return (uint32_t)(mix64(seed ^ mix64(key)) & 0xFFu);
}

__device__ __forceinline__ uint32_t gmul(uint32_t a, uint32_t b) {
    return (a && b) ? c_gf.exp[c_gf.log[a] + c_gf.log[b]] : 0u;
}

// LDS address of the LOG7 entry of byte i of g, in this lane's bank column:
// (g_i << 8) | lanebits (lanebits = (lane & 31) << 2).
template <int I>
__device__ __forceinline__ uint32_t log_addr(uint32_t lanebits, uint32_t g) {
    return __builtin_amdgcn_perm(lanebits, g, 0x0C0C0004u | ((uint32_t)I << 8));
}

__device__ __forceinline__ uint32_t lds32(const uint8_t *lds, uint32_t addr) {
    return *(const uint32_t *)(lds + addr);
}

// Four bytes (each zero-extended in a dword) packed low to high: two byte permutes
// and one shift-or.
__device__ __forceinline__ uint32_t pack4(uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3) {
    const uint32_t lo = __builtin_amdgcn_perm(b1, b0, 0x0C0C0400u);  // b0 | b1 << 8
    const uint32_t hi = __builtin_amdgcn_perm(b3, b2, 0x0C0C0400u);  // b2 | b3 << 8
    return lo | (hi << 16);
}

// x*y*g for the 4 points of dword g: lx7[i] = LOG7[x_i] + kExpBase + lanebits,
// ly7 = LOG7[y] (uniform), zc = clamp address of this lane.
__device__ __forceinline__ uint32_t mul4(const uint8_t *lds, uint32_t lanebits, uint32_t g,
                                         const uint32_t *lx7, uint32_t ly7, uint32_t zc) {
    uint32_t s0 = min(lds32(lds, log_addr<0>(lanebits, g)) + lx7[0] + ly7, zc);
    uint32_t s1 = min(lds32(lds, log_addr<1>(lanebits, g)) + lx7[1] + ly7, zc);
    uint32_t s2 = min(lds32(lds, log_addr<2>(lanebits, g)) + lx7[2] + ly7, zc);
    uint32_t s3 = min(lds32(lds, log_addr<3>(lanebits, g)) + lx7[3] + ly7, zc);
    return pack4(lds[s0], lds[s1], lds[s2], lds[s3]);
}

template <int W>
__device__ __forceinline__ void load_row(const uint8_t *base, int64_t row, int rowb, int lane,
                                         uint32_t (&v)[W]) {
    const uint8_t *p = base + row * (int64_t)rowb + (int64_t)lane * (4 * W);
    if constexpr (W == 4) {
        uint4 t = *(const uint4 *)p;
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else if constexpr (W == 2) {
        uint2 t = *(const uint2 *)p;
        v[0] = t.x; v[1] = t.y;
    } else {
        v[0] = *(const uint32_t *)p;
    }
}

template <int W>
__device__ __forceinline__ void store_row(uint8_t *base, int64_t row, int rowb, int lane,
                                          const uint32_t (&v)[W]) {
    uint8_t *p = base + row * (int64_t)rowb + (int64_t)lane * (4 * W);
    if constexpr (W == 4) {
        *(uint4 *)p = make_uint4(v[0], v[1], v[2], v[3]);
    } else if constexpr (W == 2) {
        *(uint2 *)p = make_uint2(v[0], v[1]);
    } else {
        *(uint32_t *)p = v[0];
    }
}

// Published words: slot s, dword w of the row, lane L at index s*rowd + w*lanes + L, so
// that one store instruction of a wave covers consecutive words.
template <int W>
__device__ __forceinline__ void publish(unsigned long long *pub, int32_t slot, int rowd, int lanes,
                                        int lane, uint32_t status, uint32_t epoch,
                                        const uint32_t (&v)[W]) {
    const unsigned long long hi = (unsigned long long)((epoch << 2) | status) << 32;
    unsigned long long *p = pub + (int64_t)slot * rowd + lane;
#pragma unroll
    for (int w = 0; w < W; ++w)
        __hip_atomic_store(p + w * lanes, hi | v[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int W>
__device__ __forceinline__ void lookback(unsigned long long *pub, int32_t slot, int rowd, int lanes,
                                         int lane, uint32_t epoch, Ctl *ctl, uint32_t (&carry)[W]) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint32_t c = 0;
        int32_t s = slot;
        for (;;) {
            unsigned long long *p = pub + (int64_t)s * rowd + w * lanes + lane;
            unsigned long long v;
            uint32_t spins = 0;
            bool ok = true;
            for (;;) {
                v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                uint32_t hi = (uint32_t)(v >> 32);
                if ((hi >> 2) == (epoch & 0x3FFFFFFFu) && (hi & 3u) != 0) break;
                if (++spins > kSpinLimit) {
                    atomicOr(&ctl->err, 2u);
                    ok = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            if (!ok) break;
            c ^= (uint32_t)v;
            if (((uint32_t)(v >> 32) & 3u) == kInc) break;
            if (s == 0) {
                atomicOr(&ctl->err, 4u);
                break;
            }
            --s;
        }
        carry[w] = c;
    }
}

// Per-position metadata of a window of 64 consecutive CSR positions, one position per
// lane: gathered row, destination vertex, stored row, LOG7 of the edge's y.  Windows
// are loaded one ahead so that no per-edge scalar value ever waits on memory.
struct Win {
    int32_t g, d, o;
    uint32_t y;  // input edge id until finish_win, then LOG7 of y_{e, ylevel}
};

template <bool FIN>
__device__ __forceinline__ Win load_win(const LevelParams &P, int32_t wb, int32_t p1, int lane) {
    Win m{-1, -1, -1, 0};
    const int32_t q = wb + lane;
    if (q < p1) {
        m.g = P.gidx[q];
        m.d = P.pdst[q];
        if constexpr (!FIN) m.o = P.orow[q];
        m.y = (uint32_t)P.peid[q];
    }
    return m;
}

__device__ __forceinline__ void finish_win(const LevelParams &P, const uint8_t *lds, Win &m,
                                           int32_t wb, int32_t p1, int lane, uint32_t lanebits) {
    if (wb + lane < p1) {
        uint32_t y = fp8(P.seed, 1u, P.ylevel, m.y);
        m.y = lds32(lds, (y << 8) | lanebits);
    } else {
        m.y = kZero7;
    }
}

template <int W>
__device__ __forceinline__ void gather_batch(const LevelParams &P, const Win &cw, const Win &nw,
                                             int32_t wb, int32_t pb, int32_t p1, bool act,
                                             int lane, uint32_t (&g)[kU][W]) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int32_t q = pb + u;
        int32_t r = -1;
        if (q < p1) {
            const int32_t i = q - wb;  // uniform
            r = (i < 64) ? __builtin_amdgcn_readlane(cw.g, i) : __builtin_amdgcn_readlane(nw.g, i - 64);
        }
        if (r >= 0 && act) {
            load_row<W>(P.gbase, r, P.rowb, lane, g[u]);
        } else {
#pragma unroll
            for (int w = 0; w < W; ++w) g[u][w] = 0;
        }
    }
}

template <int W, bool FIN>
__global__ void __launch_bounds__(1024) k_level(LevelParams P) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsBytes];
    {
        const uint4 *src = (const uint4 *)P.lds_image;
        uint4 *dst = (uint4 *)lds;
        for (int i = threadIdx.x; i < kLdsBytes / 16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const bool act = lane < P.lanes;
    const int rowd = P.rowb >> 2;
    const uint32_t lanebits = (uint32_t)(lane & 31) << 2;
    const uint32_t xbase = (uint32_t)kExpBase + lanebits;
    const uint32_t zc = (uint32_t)kExpBase + ((uint32_t)kClampRow << 7) + lanebits;
    const uint32_t epoch = __hip_atomic_load(&P.ctl->epoch, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) & 0x3FFFFFFFu;
    uint32_t fin[W];
#pragma unroll
    for (int w = 0; w < W; ++w) fin[w] = 0;

    // Tiles are claimed in ticket order.  The last level claims the next tile while
    // working on the current one (it has no look-back).  The scan levels claim a tile
    // only when they start it: a tile claimed early but not started would hold up the
    // look-back of every later piece of its in-list.
    uint32_t tk = 0;
    if (lane == 0) tk = atomicAdd(&P.ctl->ticket, 1u);
    tk = __builtin_amdgcn_readfirstlane(__shfl(tk, 0));
    for (;;) {
        const int32_t tile = P.tile_lo + (int32_t)tk;
        if (tile >= P.tile_hi) break;
        uint32_t tk_next = 0;
        if constexpr (FIN) {
            if (lane == 0) tk_next = atomicAdd(&P.ctl->ticket, 1u);
        }

        const int32_t p0 = P.tile_p0[tile], p1 = P.tile_p0[tile + 1];
        int32_t pubslot = -1, lbslot = -1;
        if constexpr (!FIN) {
            pubslot = P.tile_pub[tile];
            lbslot = P.tile_lb[tile];
        }
        const bool cont = lbslot >= 0;

        int32_t wb = p0;  // first position of the current window
        Win cw = load_win<FIN>(P, wb, p1, lane);
        Win nw = load_win<FIN>(P, wb + 64, p1, lane);
        finish_win(P, lds, cw, wb, p1, lane, lanebits);

        // x row (as LOG7 + base, per point) of the in-list being processed, and the raw
        // x row of the next in-list, loaded ahead
        const int32_t d0 = __builtin_amdgcn_readfirstlane(cw.d);
        int32_t cur_dst = -1, nxt_dst = d0;
        uint32_t lx7[4 * W], acc[W], xn[W];
        if (act) {
            load_row<W>(P.xt, d0, P.rowb, lane, xn);
        } else {
#pragma unroll
            for (int w = 0; w < W; ++w) xn[w] = 0;
        }
#pragma unroll
        for (int w = 0; w < W; ++w) acc[w] = 0;
#pragma unroll
        for (int i = 0; i < 4 * W; ++i) lx7[i] = kZero7;

        auto process = [&](const uint32_t (&g)[kU][W], int32_t pb) {
            const int nb = min(kU, p1 - pb);
            // last level with localisation: this lane's XOR of each position's points,
            // one byte per position, four positions to a dword
            uint32_t lp[kU / 4];
#pragma unroll
            for (int h = 0; h < kU / 4; ++h) lp[h] = 0;
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (u >= nb) break;
                const int32_t p = pb + u;
                const int32_t i = p - wb;  // lane of this position in the current window
                const int32_t d = __builtin_amdgcn_readlane(cw.d, i);
                if (d != cur_dst) {  // a new in-list (or the start of a continuation tile)
                    if (d != nxt_dst && act) load_row<W>(P.xt, d, P.rowb, lane, xn);
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        lx7[4 * w + 0] = lds32(lds, log_addr<0>(lanebits, xn[w])) + xbase;
                        lx7[4 * w + 1] = lds32(lds, log_addr<1>(lanebits, xn[w])) + xbase;
                        lx7[4 * w + 2] = lds32(lds, log_addr<2>(lanebits, xn[w])) + xbase;
                        lx7[4 * w + 3] = lds32(lds, log_addr<3>(lanebits, xn[w])) + xbase;
                        acc[w] = 0;
                    }
                    cur_dst = d;
                    // the next in-list of this tile, if it starts in this window or the next
                    uint64_t later = __ballot(cw.d != d && cw.d >= 0 && lane > i);
                    int32_t nd = -1;
                    if (later) {
                        nd = __builtin_amdgcn_readlane(cw.d, __ffsll((long long)later) - 1);
                    } else {
                        uint64_t l2 = __ballot(nw.d != d && nw.d >= 0);
                        if (l2) nd = __builtin_amdgcn_readlane(nw.d, __ffsll((long long)l2) - 1);
                    }
                    nxt_dst = nd;
                    if (nd >= 0 && act) load_row<W>(P.xt, nd, P.rowb, lane, xn);
                }
                const uint32_t ly7 = __builtin_amdgcn_readlane(cw.y, i);
                uint32_t c[W];
                if (ly7 < kZero7) {
#pragma unroll
                    for (int w = 0; w < W; ++w)
                        c[w] = mul4(lds, lanebits, g[u][w], &lx7[4 * w], ly7, zc);
                } else {  // y = 0: the edge adds nothing at this level
#pragma unroll
                    for (int w = 0; w < W; ++w) c[w] = 0;
                }
                if constexpr (FIN) {
                    if (p >= P.pos_lo && p < P.pos_hi) {
#pragma unroll
                        for (int w = 0; w < W; ++w) fin[w] ^= c[w];
                        if (P.loc) {
                            uint32_t x = 0;
#pragma unroll
                            for (int w = 0; w < W; ++w) x ^= c[w];
                            x ^= x >> 16;
                            x ^= x >> 8;
                            lp[u >> 2] |= (x & 0xFFu) << (8 * (u & 3));
                        }
                    }
                } else {
#pragma unroll
                    for (int w = 0; w < W; ++w) acc[w] ^= c[w];
                    const int32_t orow = __builtin_amdgcn_readlane(cw.o, i);
                    if (orow >= 0 && act) store_row<W>(P.sout, orow, P.rowb, lane, acc);
                }
            }
            if constexpr (FIN) {
                if (P.loc) {
                    // XOR across the wave, four positions at a time; lane j < nb then
                    // adds position pb + j's byte
#pragma unroll
                    for (int h = 0; h < kU / 4; ++h) {
                        if (4 * h >= nb) break;
#pragma unroll
                        for (int off = 32; off >= 1; off >>= 1) lp[h] ^= __shfl_xor(lp[h], off);
                    }
                    const int32_t p = pb + lane;
                    if (lane < nb && p >= P.pos_lo && p < P.pos_hi)
                        P.loc[p - P.pos_lo] ^= (uint8_t)(lp[(lane >> 2) & (kU / 4 - 1)] >> (8 * (lane & 3)));
                }
            }
            // advance the window after its last batch
            if (pb + kU - wb == 64 && pb + kU < p1) {
                wb += 64;
                cw = nw;
                finish_win(P, lds, cw, wb, p1, lane, lanebits);
                nw = load_win<FIN>(P, wb + 64, p1, lane);
            }
        };

        // two batches of gathers in flight: while one is multiplied, the next loads
        uint32_t ga[kU][W], gb[kU][W];
        gather_batch<W>(P, cw, nw, wb, p0, p1, act, lane, ga);
        for (int32_t pb = p0; pb < p1;) {
            gather_batch<W>(P, cw, nw, wb, pb + kU, p1, act, lane, gb);
            process(ga, pb);
            pb += kU;
            if (pb >= p1) break;
            gather_batch<W>(P, cw, nw, wb, pb + kU, p1, act, lane, ga);
            process(gb, pb);
            pb += kU;
        }

        if constexpr (!FIN) {
            if (act) {
                if (pubslot >= 0)
                    publish<W>(P.pub, pubslot, rowd, P.lanes, lane, cont ? kAgg : kInc, epoch, acc);
                if (cont) {
                    uint32_t carry[W];
                    lookback<W>(P.pub, lbslot, rowd, P.lanes, lane, epoch, P.ctl, carry);
                    if (pubslot >= 0) {
                        uint32_t inc[W];
#pragma unroll
                        for (int w = 0; w < W; ++w) inc[w] = acc[w] ^ carry[w];
                        publish<W>(P.pub, pubslot, rowd, P.lanes, lane, kInc, epoch, inc);
                    }
                    // rows of a continuation tile were stored without the carry of the
                    // earlier pieces: add it now (this wave's own stores are complete)
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                    for (int32_t p = p0; p < p1; ++p) {
                        const int32_t orow = P.orow[p];
                        if (orow >= 0) {
                            uint32_t v[W];
                            load_row<W>(P.sout, orow, P.rowb, lane, v);
#pragma unroll
                            for (int w = 0; w < W; ++w) v[w] ^= carry[w];
                            store_row<W>(P.sout, orow, P.rowb, lane, v);
                        }
                    }
                }
            }
        }
        if constexpr (!FIN) {
            if (lane == 0) tk_next = atomicAdd(&P.ctl->ticket, 1u);
        }
        tk = __builtin_amdgcn_readfirstlane(__shfl(tk_next, 0));
    }

    if constexpr (FIN) {
        if (act) {
#pragma unroll
            for (int w = 0; w < W; ++w)
                if (fin[w]) atomicXor(&P.fin[lane * W + w], fin[w]);
        }
    }
}

// ---------------------------------------------------------------------------------
// Narrow rows: C = 16 LP points (LP = 1..32 lanes per row, 16 points per lane).  A
// wave processes E = 64 / LP consecutive positions side by side, one per slot of LP
// lanes, so the per-edge fixed work (metadata, fingerprint, branch, address) is shared
// by E edges.  The running value of an in-list then comes from an inclusive segmented
// XOR-scan across the slots of a step (shuffles by multiples of LP lanes, a slot whose
// destination differs from the previous slot's starts a segment); the last slot's
// value carries into the next step.  Tiles, look-back and the carry fix-up of
// continuation pieces are those of k_level.
// ---------------------------------------------------------------------------------
// One step of the inclusive segmented XOR-scan, (f, v) <- (f | f', f ? v : v ^ v'),
// with (f', v') read through DPP control CTRL: a source outside the lane's 16-lane row,
// or a lane that ROWMASK leaves out, reads (0, 0), the identity of the step.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ void seg_step_dpp(uint32_t (&v)[4], uint32_t &f) {
    uint32_t vo[4];
#pragma unroll
    for (int w = 0; w < 4; ++w)
        vo[w] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[w], CTRL, ROWMASK, 0xF, true);
    const uint32_t fo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)f, CTRL, ROWMASK, 0xF, true);
#pragma unroll
    for (int w = 0; w < 4; ++w) v[w] = f ? v[w] : (v[w] ^ vo[w]);
    f |= fo;
}

// The same step across 16-lane rows for slots of LP lanes: a lane of a receiving row
// (ROWS: bit r set for row r) reads the last slot of row LASTROW of its own row's
// predecessor (LASTROW = -1: the row just below), lane sub of that slot, by shuffle.
template <int LP, int ROWS, int LASTROW>
__device__ __forceinline__ void seg_step_rows(uint32_t (&v)[4], uint32_t &f, int lane) {
    const int row = lane >> 4, sub = lane % LP;
    const int srow = LASTROW >= 0 ? LASTROW : row - 1;
    const int src = ((srow < 0 ? 0 : srow) << 4) + 16 - LP + sub;
    uint32_t vo[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) vo[w] = __shfl(v[w], src);
    const uint32_t fo = __shfl(f, src);
    if ((ROWS >> row) & 1) {
#pragma unroll
        for (int w = 0; w < 4; ++w) v[w] = f ? v[w] : (v[w] ^ vo[w]);
        f |= fo;
    }
}

// Inclusive segmented XOR-scan over the E = 64 / LP slots of a step (slot s holds lanes
// [s LP, s LP + LP)), f = 1 at a slot that starts a segment.  Within each 16-lane row:
// DPP row shifts of LP, 2 LP, .. 8 lanes.  Then across rows, as the last slot of a row
// holds the row's running value: rows 1 and 3 add the last slot of rows 0 and 2, then
// rows 2 and 3 add the last slot of row 1 (now rows 0-1): DPP row broadcasts for LP = 1
// (lane 15, lane 31), lane shuffles for wider slots.
template <int LP>
__device__ __forceinline__ void seg_scan(uint32_t (&v)[4], uint32_t &f, int lane) {
    static_assert(LP == 1 || LP == 2 || LP == 4 || LP == 8, "slots of 1..8 lanes");
    if constexpr (LP == 1) seg_step_dpp<0x111, 0xF>(v, f);
    if constexpr (LP <= 2) seg_step_dpp<0x110 + 2, 0xF>(v, f);
    if constexpr (LP <= 4) seg_step_dpp<0x110 + 4, 0xF>(v, f);
    if constexpr (LP <= 8) seg_step_dpp<0x110 + 8, 0xF>(v, f);
    if constexpr (LP == 1) {
        seg_step_dpp<0x142, 0xA>(v, f);  // row_bcast:15 into rows 1 and 3
        seg_step_dpp<0x143, 0xC>(v, f);  // row_bcast:31 into rows 2 and 3
    } else {
        seg_step_rows<LP, 0xA, -1>(v, f, lane);
        seg_step_rows<LP, 0xC, 1>(v, f, lane);
    }
}

template <int LP, bool FIN>
__global__ void __launch_bounds__(1024) k_narrow(LevelParams P) {
    constexpr int E = 64 / LP;           // positions per step
    constexpr int U = (E >= 64) ? 1 : 2;  // steps per batch; two batches in flight
    static_assert(64 % (U * E) == 0, "batches tile a window");
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsBytes];
    {
        const uint4 *src = (const uint4 *)P.lds_image;
        uint4 *dst = (uint4 *)lds;
        for (int i = threadIdx.x; i < kLdsBytes / 16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int slot = lane / LP, sub = lane % LP;
    const int rowd = P.rowb >> 2;
    const int64_t subofs = (int64_t)sub * 16;
    const uint32_t lanebits = (uint32_t)(lane & 31) << 2;
    const uint32_t xbase = (uint32_t)kExpBase + lanebits;
    const uint32_t zc = (uint32_t)kExpBase + ((uint32_t)kClampRow << 7) + lanebits;
    const uint32_t epoch = __hip_atomic_load(&P.ctl->epoch, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) & 0x3FFFFFFFu;
    uint32_t fin[4] = {0, 0, 0, 0};

    uint32_t tk = 0;
    if (lane == 0) tk = atomicAdd(&P.ctl->ticket, 1u);
    tk = __builtin_amdgcn_readfirstlane(__shfl(tk, 0));
    for (;;) {
        const int32_t tile = P.tile_lo + (int32_t)tk;
        if (tile >= P.tile_hi) break;
        uint32_t tk_next = 0;
        if constexpr (FIN) {
            if (lane == 0) tk_next = atomicAdd(&P.ctl->ticket, 1u);
        }
        const int32_t p0 = P.tile_p0[tile], p1 = P.tile_p0[tile + 1];
        int32_t pubslot = -1, lbslot = -1;
        if constexpr (!FIN) {
            pubslot = P.tile_pub[tile];
            lbslot = P.tile_lb[tile];
        }
        const bool cont = lbslot >= 0;

        int32_t wb = p0;
        Win cw = load_win<FIN>(P, wb, p1, lane);
        Win nw = load_win<FIN>(P, wb + 64, p1, lane);
        finish_win(P, lds, cw, wb, p1, lane, lanebits);

        uint32_t run[4] = {0, 0, 0, 0};  // running value after the last step (every slot)
        int32_t run_d = -1;              // its in-list
        int32_t cur_d = -1;              // in-list whose x row is in lx7 (per lane)
        int32_t gprev = -1;              // gather side: this slot's previous destination
        uint32_t lx7[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) lx7[i] = kZero7;

        // one batch: U steps from position pb; row of the gathered predecessor, and the
        // x row of the destination where it changes along this slot's positions
        auto gather = [&](int32_t pb, uint32_t (&g)[U][4], uint32_t (&xr)[U][4]) {
            const bool in_next = (pb - wb) >= 64;  // uniform
            const int base = (pb - wb) - (in_next ? 64 : 0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t q = pb + u * E + slot;
                const int li = base + u * E + slot;
                const int32_t r = in_next ? __shfl(nw.g, li) : __shfl(cw.g, li);
                const int32_t d = in_next ? __shfl(nw.d, li) : __shfl(cw.d, li);
                const bool valid = q < p1;
                if (valid && r >= 0) {
                    const uint4 t = *(const uint4 *)(P.gbase + (int64_t)r * P.rowb + subofs);
                    g[u][0] = t.x; g[u][1] = t.y; g[u][2] = t.z; g[u][3] = t.w;
                } else {
                    g[u][0] = g[u][1] = g[u][2] = g[u][3] = 0;
                }
                if (valid && d != gprev) {
                    const uint4 t = *(const uint4 *)(P.xt + (int64_t)d * P.rowb + subofs);
                    xr[u][0] = t.x; xr[u][1] = t.y; xr[u][2] = t.z; xr[u][3] = t.w;
                }
                if (valid) gprev = d;
            }
        };

        auto process = [&](int32_t pb, const uint32_t (&g)[U][4], const uint32_t (&xr)[U][4]) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t sb = pb + u * E;  // first position of the step (uniform)
                if (sb >= p1) break;
                const int nvalid = min(E, p1 - sb);
                const int li = (sb - wb) + slot;
                const int32_t d = __shfl(cw.d, li);
                const uint32_t ly7 = __shfl(cw.y, li);
                const bool valid = slot < nvalid;
                if (valid && d != cur_d) {
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        lx7[4 * w + 0] = lds32(lds, log_addr<0>(lanebits, xr[u][w])) + xbase;
                        lx7[4 * w + 1] = lds32(lds, log_addr<1>(lanebits, xr[u][w])) + xbase;
                        lx7[4 * w + 2] = lds32(lds, log_addr<2>(lanebits, xr[u][w])) + xbase;
                        lx7[4 * w + 3] = lds32(lds, log_addr<3>(lanebits, xr[u][w])) + xbase;
                    }
                    cur_d = d;
                }
                uint32_t c[4];
                if (valid && ly7 < kZero7) {
#pragma unroll
                    for (int w = 0; w < 4; ++w) c[w] = mul4(lds, lanebits, g[u][w], &lx7[4 * w], ly7, zc);
                } else {
                    c[0] = c[1] = c[2] = c[3] = 0;
                }
                if constexpr (FIN) {
                    const int32_t p = sb + slot;
                    const bool inr = valid && p >= P.pos_lo && p < P.pos_hi;
                    if (inr) {
#pragma unroll
                        for (int w = 0; w < 4; ++w) fin[w] ^= c[w];
                    }
                    if (P.loc) {
                        // only this chunk's real sieve points count
                        const int lim = P.valid_pts - sub * 16;
                        uint32_t x = 0;
#pragma unroll
                        for (int w = 0; w < 4; ++w) {
                            const int nb = min(4, max(0, lim - 4 * w));
                            const uint32_t keep = nb >= 4 ? 0xFFFFFFFFu : ((1u << (8 * nb)) - 1u);
                            x ^= c[w] & keep;
                        }
                        if (!inr) x = 0;
                        x ^= x >> 16;
                        x ^= x >> 8;
                        x &= 0xFFu;
#pragma unroll
                        for (int off = LP / 2; off >= 1; off >>= 1) x ^= __shfl_xor(x, off);
                        if (inr && sub == 0) P.loc[p - P.pos_lo] ^= (uint8_t)x;
                    }
                } else {
                    // inclusive segmented XOR-scan over the slots of this step
                    const int32_t dprev = __shfl_up(d, LP);
                    uint32_t fl = (valid && (slot == 0 ? d != run_d : d != dprev)) ? 1u : 0u;
                    uint32_t v[4] = {c[0], c[1], c[2], c[3]};
                    seg_scan<LP>(v, fl, lane);
                    const bool f = fl != 0;
                    // slots with no segment start at or below them continue run_d
                    uint32_t a[4];
#pragma unroll
                    for (int w = 0; w < 4; ++w) a[w] = f ? v[w] : (v[w] ^ run[w]);
                    const int32_t o = __shfl(cw.o, li);
                    if (valid && o >= 0)
                        *(uint4 *)(P.sout + (int64_t)o * P.rowb + subofs) = make_uint4(a[0], a[1], a[2], a[3]);
                    const int last = (nvalid - 1) * LP;
#pragma unroll
                    for (int w = 0; w < 4; ++w) run[w] = __shfl(a[w], last + sub);
                    run_d = __shfl(d, last);
                }
            }
            // advance the window after its last batch
            if (pb + U * E - wb == 64 && pb + U * E < p1) {
                wb += 64;
                cw = nw;
                finish_win(P, lds, cw, wb, p1, lane, lanebits);
                nw = load_win<FIN>(P, wb + 64, p1, lane);
            }
        };

        uint32_t ga[U][4], gb[U][4], xa[U][4], xb[U][4];
        gather(p0, ga, xa);
        for (int32_t pb = p0; pb < p1;) {
            gather(pb + U * E, gb, xb);
            process(pb, ga, xa);
            pb += U * E;
            if (pb >= p1) break;
            gather(pb + U * E, ga, xa);
            process(pb, gb, xb);
            pb += U * E;
        }

        if constexpr (!FIN) {
            if (pubslot >= 0 && lane < LP)
                publish<4>(P.pub, pubslot, rowd, LP, sub, cont ? kAgg : kInc, epoch, run);
            if (cont) {
                uint32_t carry[4] = {0, 0, 0, 0};
                if (lane < LP) lookback<4>(P.pub, lbslot, rowd, LP, sub, epoch, P.ctl, carry);
#pragma unroll
                for (int w = 0; w < 4; ++w) carry[w] = __shfl(carry[w], sub);
                if (pubslot >= 0 && lane < LP) {
                    uint32_t inc[4];
#pragma unroll
                    for (int w = 0; w < 4; ++w) inc[w] = run[w] ^ carry[w];
                    publish<4>(P.pub, pubslot, rowd, LP, sub, kInc, epoch, inc);
                }
                // rows of a continuation piece were stored without the carry
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                for (int32_t p = p0 + slot; p < p1; p += E) {
                    const int32_t orow = P.orow[p];
                    if (orow >= 0) {
                        uint4 *q = (uint4 *)(P.sout + (int64_t)orow * P.rowb + subofs);
                        uint4 t = *q;
                        t.x ^= carry[0]; t.y ^= carry[1]; t.z ^= carry[2]; t.w ^= carry[3];
                        *q = t;
                    }
                }
            }
            if (lane == 0) tk_next = atomicAdd(&P.ctl->ticket, 1u);
        }
        tk = __builtin_amdgcn_readfirstlane(__shfl(tk_next, 0));
    }

    if constexpr (FIN) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
#pragma unroll
            for (int off = LP; off < 64; off <<= 1) fin[w] ^= __shfl_xor(fin[w], off);
        }
        if (lane < LP) {
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (fin[w]) atomicXor(&P.fin[sub * 4 + w], fin[w]);
        }
    }
}

// ---------------------------------------------------------------------------------
// Slot tiles for narrow rows: each of the E = 64 / LP slots of a wave (LP lanes, 16
// points a lane) runs a tile of its own, one position per step, as k_level runs a
// tile with a whole wave: the running value of an in-list stays in the slot's lanes,
// so no scan across slots is needed.  A ticket claims E consecutive tiles.  Per-slot
// metadata comes from a window of LP positions held one per lane of the slot (the
// step's lane is the same in every slot); the x row of the first new destination of a
// batch is fetched with the batch's gathers, a second one in the same batch when it is
// reached.  Publication, look-back and the carry fix-up of continuation tiles are
// k_level's, per slot.
// ---------------------------------------------------------------------------------
template <bool FIN>
__device__ __forceinline__ Win load_slot_win(const LevelParams &P, int32_t q, int32_t p1) {
    Win m{-1, -1, -1, 0};
    if (q < p1) {
        m.g = P.gidx[q];
        m.d = P.pdst[q];
        if constexpr (!FIN) m.o = P.orow[q];
        m.y = (uint32_t)P.peid[q];
    }
    return m;
}

__device__ __forceinline__ void finish_slot_win(const LevelParams &P, const uint8_t *lds, Win &m,
                                                int32_t q, int32_t p1, uint32_t lanebits) {
    if (q < p1) {
        uint32_t y = fp8(P.seed, 1u, P.ylevel, m.y);
        m.y = lds32(lds, (y << 8) | lanebits);
    } else {
        m.y = kZero7;
    }
}

template <int LP, bool FIN>
__global__ void __launch_bounds__(1024) k_slot(LevelParams P) {
    constexpr int E = 64 / LP;  // slots (tiles) per wave
    constexpr int U = 4;        // steps per batch; two batches in flight
    static_assert(LP >= U && LP % U == 0, "batches tile a window");
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsBytes];
    {
        const uint4 *src = (const uint4 *)P.lds_image;
        uint4 *dst = (uint4 *)lds;
        for (int i = threadIdx.x; i < kLdsBytes / 16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int slot = lane / LP, sub = lane % LP;
    const int rowd = P.rowb >> 2;
    const int64_t subofs = (int64_t)sub * 16;
    const int sbase = slot * LP * 4;  // ds_bpermute address of the slot's first lane
    const uint32_t rowb = (uint32_t)P.rowb;
    const uint8_t *gsub = P.gbase + subofs, *xsub = P.xt + subofs;
    uint8_t *osub = P.sout + subofs;
    const uint32_t lanebits = (uint32_t)(lane & 31) << 2;
    const uint32_t xbase = (uint32_t)kExpBase + lanebits;
    const uint32_t zc = (uint32_t)kExpBase + ((uint32_t)kClampRow << 7) + lanebits;
    const uint32_t epoch = __hip_atomic_load(&P.ctl->epoch, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) & 0x3FFFFFFFu;
    uint32_t fin[4] = {0, 0, 0, 0};

    uint32_t tk = 0;
    if (lane == 0) tk = atomicAdd(&P.ctl->ticket, 1u);
    tk = __builtin_amdgcn_readfirstlane(__shfl(tk, 0));
    for (;;) {
        const int32_t tile0 = P.tile_lo + (int32_t)tk * E;
        if (tile0 >= P.tile_hi) break;
        uint32_t tk_next = 0;
        if constexpr (FIN) {
            if (lane == 0) tk_next = atomicAdd(&P.ctl->ticket, 1u);
        }
        const int32_t tile = tile0 + slot;
        const bool has = tile < P.tile_hi;
        const int32_t p0 = has ? P.tile_p0[tile] : 0;
        const int32_t p1 = has ? P.tile_p0[tile + 1] : 0;
        int32_t pubslot = -1, lbslot = -1;
        if constexpr (!FIN) {
            if (has) {
                pubslot = P.tile_pub[tile];
                lbslot = P.tile_lb[tile];
            }
        }
        const bool cont = lbslot >= 0;
        const int32_t len = p1 - p0;
        int32_t K = len;  // steps: the longest tile of the wave
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) K = max(K, __shfl_xor(K, off));
        K = __builtin_amdgcn_readfirstlane(K);

        int32_t wb = 0;  // first step of the current window (uniform)
        Win cw = load_slot_win<FIN>(P, p0 + sub, p1);
        Win nw = load_slot_win<FIN>(P, p0 + LP + sub, p1);
        finish_slot_win(P, lds, cw, p0 + sub, p1, lanebits);

        uint32_t acc[4] = {0, 0, 0, 0};  // running value of the slot's in-list
        int32_t cur_d = -1;               // in-list whose x row is in lx7
        int32_t gprev = -1;               // gather side: destination of the last step
        uint32_t lx7[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) lx7[i] = kZero7;

        // one batch: U steps from step kb; the gathered row, and the x row of the
        // destination where it changes
        auto gather = [&](int32_t kb, uint32_t (&g)[U][4], uint32_t (&xr)[4], int32_t &xd) {
            xd = -1;
            const bool in_next = (kb - wb) >= LP;  // uniform
            const int base = (kb - wb) - (in_next ? LP : 0);
            const int32_t wg = in_next ? nw.g : cw.g, wd = in_next ? nw.d : cw.d;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int a = sbase + 4 * (base + u);
                const int32_t r = __builtin_amdgcn_ds_bpermute(a, wg);
                const int32_t d = __builtin_amdgcn_ds_bpermute(a, wd);
                const bool valid = kb + u < len;
                if (valid && r >= 0) {
                    const uint4 t = *(const uint4 *)(gsub + (uint64_t)(uint32_t)r * rowb);
                    g[u][0] = t.x; g[u][1] = t.y; g[u][2] = t.z; g[u][3] = t.w;
                } else {
                    g[u][0] = g[u][1] = g[u][2] = g[u][3] = 0;
                }
                if (valid && d != gprev && xd < 0) {  // the batch's first new in-list
                    const uint4 t = *(const uint4 *)(xsub + (uint64_t)(uint32_t)d * rowb);
                    xr[0] = t.x; xr[1] = t.y; xr[2] = t.z; xr[3] = t.w;
                    xd = d;
                }
                if (valid) gprev = d;
            }
        };

        auto process = [&](int32_t kb, const uint32_t (&g)[U][4], const uint32_t (&xr)[4], int32_t xd) {
            // last level with localisation: this lane's XOR of each step's points, one
            // byte per step
            uint32_t lp = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t k = kb + u;
                if (k >= K) break;
                const int a = sbase + 4 * (k - wb);
                const int32_t d = __builtin_amdgcn_ds_bpermute(a, cw.d);
                const uint32_t ly7 = (uint32_t)__builtin_amdgcn_ds_bpermute(a, (int)cw.y);
                const bool valid = k < len;
                if (valid && d != cur_d) {  // a new in-list of this slot's tile
                    uint32_t x[4] = {xr[0], xr[1], xr[2], xr[3]};
                    if (d != xd) {  // a second new in-list in the batch: not fetched ahead
                        const uint4 t = *(const uint4 *)(xsub + (uint64_t)(uint32_t)d * rowb);
                        x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
                    }
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        lx7[4 * w + 0] = lds32(lds, log_addr<0>(lanebits, x[w])) + xbase;
                        lx7[4 * w + 1] = lds32(lds, log_addr<1>(lanebits, x[w])) + xbase;
                        lx7[4 * w + 2] = lds32(lds, log_addr<2>(lanebits, x[w])) + xbase;
                        lx7[4 * w + 3] = lds32(lds, log_addr<3>(lanebits, x[w])) + xbase;
                        acc[w] = 0;
                    }
                    cur_d = d;
                }
                // no test needed: y = 0 (LOG7 kZero7, also past the tile's end) and g = 0
                // both push every sum past the clamp, so the products come out zero
                uint32_t c[4];
#pragma unroll
                for (int w = 0; w < 4; ++w) c[w] = mul4(lds, lanebits, g[u][w], &lx7[4 * w], ly7, zc);
                if constexpr (FIN) {
                    const int32_t p = p0 + k;
                    const bool inr = valid && p >= P.pos_lo && p < P.pos_hi;
                    if (inr) {
#pragma unroll
                        for (int w = 0; w < 4; ++w) fin[w] ^= c[w];
                    }
                    if (P.loc) {
                        // only this chunk's real sieve points count
                        const int lim = P.valid_pts - sub * 16;
                        uint32_t x = 0;
#pragma unroll
                        for (int w = 0; w < 4; ++w) {
                            const int nb = min(4, max(0, lim - 4 * w));
                            const uint32_t keep = nb >= 4 ? 0xFFFFFFFFu : ((1u << (8 * nb)) - 1u);
                            x ^= c[w] & keep;
                        }
                        if (!inr) x = 0;
                        x ^= x >> 16;
                        x ^= x >> 8;
                        lp |= (x & 0xFFu) << (8 * u);
                    }
                } else {
#pragma unroll
                    for (int w = 0; w < 4; ++w) acc[w] ^= c[w];
                    const int32_t o = __builtin_amdgcn_ds_bpermute(a, cw.o);
                    if (valid && o >= 0)
                        *(uint4 *)(osub + (uint64_t)(uint32_t)o * rowb) = make_uint4(acc[0], acc[1], acc[2], acc[3]);
                }
            }
            if constexpr (FIN) {
                if (P.loc) {
                    // XOR across the slot's lanes, all steps of the batch at once; lane
                    // sub < U then adds step kb + sub's byte
#pragma unroll
                    for (int off = LP / 2; off >= 1; off >>= 1) lp ^= __shfl_xor(lp, off);
                    const int32_t p = p0 + kb + sub;
                    if (sub < U && kb + sub < len && p >= P.pos_lo && p < P.pos_hi)
                        P.loc[p - P.pos_lo] ^= (uint8_t)(lp >> (8 * (sub & (U - 1))));
                }
            }
            // advance the window after its last batch
            if (kb + U - wb == LP && kb + U < K) {
                wb += LP;
                cw = nw;
                finish_slot_win(P, lds, cw, p0 + wb + sub, p1, lanebits);
                nw = load_slot_win<FIN>(P, p0 + wb + LP + sub, p1);
            }
        };

        uint32_t ga[U][4], gb[U][4], xa[4], xb[4];
        int32_t xda, xdb;
        gather(0, ga, xa, xda);
        for (int32_t kb = 0; kb < K;) {
            gather(kb + U, gb, xb, xdb);
            process(kb, ga, xa, xda);
            kb += U;
            if (kb >= K) break;
            gather(kb + U, ga, xa, xda);
            process(kb, gb, xb, xdb);
            kb += U;
        }

        if constexpr (!FIN) {
            if (pubslot >= 0)
                publish<4>(P.pub, pubslot, rowd, LP, sub, cont ? kAgg : kInc, epoch, acc);
            if (cont) {
                uint32_t carry[4] = {0, 0, 0, 0};
                lookback<4>(P.pub, lbslot, rowd, LP, sub, epoch, P.ctl, carry);
                if (pubslot >= 0) {
                    uint32_t inc[4];
#pragma unroll
                    for (int w = 0; w < 4; ++w) inc[w] = acc[w] ^ carry[w];
                    publish<4>(P.pub, pubslot, rowd, LP, sub, kInc, epoch, inc);
                }
                // rows of a continuation tile were stored without the carry
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                for (int32_t p = p0; p < p1; ++p) {
                    const int32_t orow = P.orow[p];
                    if (orow >= 0) {
                        uint4 *q = (uint4 *)(P.sout + (int64_t)orow * P.rowb + subofs);
                        uint4 t = *q;
                        t.x ^= carry[0]; t.y ^= carry[1]; t.z ^= carry[2]; t.w ^= carry[3];
                        *q = t;
                    }
                }
            }
            if (lane == 0) tk_next = atomicAdd(&P.ctl->ticket, 1u);
        }
        tk = __builtin_amdgcn_readfirstlane(__shfl(tk_next, 0));
    }

    if constexpr (FIN) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
#pragma unroll
            for (int off = LP; off < 64; off <<= 1) fin[w] ^= __shfl_xor(fin[w], off);
        }
        if (lane < LP) {
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (fin[w]) atomicXor(&P.fin[sub * 4 + w], fin[w]);
        }
    }
}

__global__ void k_prep(Ctl *ctl, int bump_epoch) {
    ctl->ticket = 0;
    if (bump_epoch) ctl->epoch = (ctl->epoch + 1u) & 0x3FFFFFFFu;
}

// z[u][j] = sum over slots d of colour c(u) of v_{u,d} * w_{d,j} (Eq. (motif)), rows
// padded to 16 bytes; zero for a deleted vertex or a colour outside the multiset.
// fid (nullable): the vertex id that keys a vertex's fingerprints (layer copies of a
// vertex share the original's)
__global__ void k_z(int32_t n, int32_t k, const int32_t *color, const int32_t *fid, QuerySlots qs,
                    const uint8_t *mask, uint64_t seed, uint8_t *z) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int32_t c = color[u];
    int32_t off = 0, mu = 0;
    for (int i = 0; i < qs.ncol; ++i)
        if (qs.col[i] == c) {
            off = qs.off[i];
            mu = qs.mu[i];
        }
    // wildcard entries (colour -1, first slots) belong to every vertex
    const int32_t wmu = (qs.ncol > 0 && qs.col[0] == -1) ? qs.mu[0] : 0;
    const bool live = (mask == nullptr || mask[u] != 0) && (mu > 0 || wmu > 0);
    const uint32_t uid = fid ? (uint32_t)fid[u] : (uint32_t)u;
    uint32_t out[4] = {0, 0, 0, 0};
    for (int j = 0; j < k; ++j) {
        uint32_t acc = 0;
        if (live) {
            for (int d = 0; d < wmu; ++d)
                acc ^= gmul(fp8(seed, 2u, (uint32_t)d, uid), fp8(seed, 3u, (uint32_t)d, (uint32_t)j));
            for (int d = off; d < off + mu; ++d)
                acc ^= gmul(fp8(seed, 2u, (uint32_t)d, uid), fp8(seed, 3u, (uint32_t)d, (uint32_t)j));
        }
        out[j >> 2] |= acc << (8 * (j & 3));
    }
    ((uint4 *)z)[u] = make_uint4(out[0], out[1], out[2], out[3]);
}

// x_u^A = sum_{j in A} z_{u,j} for the points A = base + b, b in [0, npts), written to
// bytes [col, col + npts) of vertex u's row (stride bytes per row).  A thread writes
// 16 points: x^A = x^(A with its low 4 bits cleared) + x^(A's low 4 bits).
__global__ void k_xt(int32_t n, int32_t k, int32_t npts, int32_t stride, int32_t col, uint32_t base,
                     const uint8_t *z, uint8_t *xt, const int32_t *color, uint64_t colors) {
    const int32_t per_row = (npts + 15) >> 4;  // threads per vertex row
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * per_row) return;
    int64_t u = i / per_row;
    // colours != 0: the rows of vertices of other colours are never read (no edges)
    if (colors && !((colors >> color[u]) & 1ull)) return;
    int32_t part = (int32_t)(i - u * per_row);
    const uint4 zz4 = ((const uint4 *)z)[u];
    const uint32_t zw[4] = {zz4.x, zz4.y, zz4.z, zz4.w};
    auto zj = [&](int j) -> uint32_t { return (zw[j >> 2] >> (8 * (j & 3))) & 0xFFu; };
    const uint32_t A0 = base + (uint32_t)part * 16u;
    uint32_t hi = 0;
    for (int j = 4; j < k; ++j)
        if ((A0 >> j) & 1u) hi ^= zj(j);
    uint32_t lo[16];
    lo[0] = 0;
    for (int b = 1; b < 16; ++b) {
        int j = __builtin_ctz(b);
        lo[b] = lo[b & (b - 1)] ^ (j < k ? zj(j) : 0u);
    }
    const int cnt = min(16, npts - part * 16);
    uint32_t out[4] = {0, 0, 0, 0};
    for (int b = 0; b < cnt; ++b) {
        uint32_t A = A0 + (uint32_t)b;
        uint32_t x = ((A >> 4) == (A0 >> 4)) ? (hi ^ lo[A & 15u]) : 0u;
        out[b >> 2] |= x << (8 * (b & 3));
    }
    uint8_t *row = xt + u * (int64_t)stride + col + (int64_t)part * 16;
    if (cnt == 16 && ((stride | col) & 15) == 0) {
        *(uint4 *)row = make_uint4(out[0], out[1], out[2], out[3]);
    } else {
        for (int b = 0; b < cnt; b += 4) *(uint32_t *)(row + b) = out[b >> 2];
    }
}

// k = 1: P(A) = sum_u x_u^A, A in {0, 1}; x^0 = 0, x^1 = z_{u,0}.
__global__ void k_single(int32_t n, const uint8_t *z, uint32_t *out) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t v = (u < n) ? ((uint32_t)z[u * 16] << 8) : 0u;
    for (int off = 32; off >= 1; off >>= 1) v ^= __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0 && v) atomicXor(out, v);
}

// total = XOR of all per-point bytes
__global__ void k_total(int32_t npts, const uint8_t *pp, uint8_t *total) {
    uint32_t v = 0;
    for (int32_t i = threadIdx.x; i < npts; i += blockDim.x) v ^= pp[i];
    for (int off = 32; off >= 1; off >>= 1) v ^= __shfl_xor(v, off);
    __shared__ uint32_t part[16];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t ^= part[i];
        *total = (uint8_t)t;
    }
}

// p[0 .. words) = v (grid-stride); clears device words without a memset node
__global__ void k_fill32(uint32_t *p, int64_t words, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Outputs of a sieve on caller buffers: total = XOR of the npts per-point bytes,
// out[0 .. npts) = pp (out nullable), *err = the look-back failure bits (nullable).
// One workgroup of 256 threads.
__global__ void k_fixed_out(int32_t npts, const uint8_t *pp, uint8_t *out, uint8_t *total,
                            const Ctl *ctl, uint32_t *err) {
    uint32_t v = 0;
    for (int32_t i = threadIdx.x; i < npts; i += blockDim.x) {
        const uint8_t b = pp[i];
        v ^= b;
        if (out) out[i] = b;
    }
    for (int off = 32; off >= 1; off >>= 1) v ^= __shfl_xor(v, off);
    __shared__ uint32_t part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        *total = (uint8_t)(part[0] ^ part[1] ^ part[2] ^ part[3]);
        if (err) *err = ctl->err;
    }
}

// smallest (input edge id, position) over positions whose localisation is nonzero;
// each wave reduces its 64 candidates first, so the shared word sees one atomic per wave
__global__ void k_pick(int32_t lo, int32_t hi, const uint8_t *loc, const int32_t *peid,
                       unsigned long long *best) {
    int64_t p = (int64_t)lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v = ~0ull;
    if (p < hi && loc[p - lo])
        v = ((unsigned long long)(uint32_t)peid[p] << 32) | (unsigned long long)p;
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    if ((threadIdx.x & 63) == 0 && v != ~0ull) atomicMin(best, v);
}

inline unsigned grid_for(int64_t work, int block = 256) {
    return (unsigned)std::max<int64_t>(1, (work + block - 1) / block);
}

// ---------------------------------------------------------------------------------
// Multi-query step.  The row holds several lane groups, each a (query, chunk) with
// its own seed and its own level: a group at level 2 gathers the x row of the edge's
// source, later levels gather the previous step's rows, and a group at its last
// level accumulates instead of storing.  One launch advances every group one level,
// so groups can start and finish independently (continuous batching), and queries of
// any size share one sweep over the graph.
// ---------------------------------------------------------------------------------
struct WinS {
    int32_t g, s, d, o;
    uint32_t pc;      // colours of source (low byte) and head (high byte)
    uint32_t e;       // input edge id
    uint32_t h0, h1;  // ymode 1: inner fingerprint hash of (tag y, ylevel0, e), low and
                      // high words; ymode 2: log y of groups 0..3 and 4..7, one byte
                      // each (255 for y = 0)
};

// does a query with colour mask cmask use an edge with colours pc (source low byte,
// head high byte)
__device__ __forceinline__ bool lane_uses(uint64_t cmask, uint32_t pc) {
    return ((cmask >> (pc & 0xFFu)) & (cmask >> (pc >> 8)) & 1ull) != 0;
}

struct YPlan {
    int ymode, ngroups;
    uint32_t ylevel0;
    const uint64_t *gs;  // group seeds, levels and colour masks, in LDS (shared by the
    const uint32_t *gl;  // workgroup)
    const uint64_t *gm;
};

__device__ __forceinline__ WinS load_wins(const StepParams &P, int32_t wb, int32_t p1, int lane,
                                          const YPlan &Y, const uint8_t *lds, uint32_t lanebits) {
    WinS m{-1, -1, -1, -1, 0, 0, 0, 0};
    const int32_t q = wb + lane;
    if (q < p1) {
        m.g = P.gsrc[q];
        m.s = P.psrc[q];
        m.d = P.pdst[q];
        m.o = P.orow[q];
        if (P.pcol) m.pc = P.pcol[q];
        m.e = (uint32_t)P.peid[q];
        if (Y.ymode == 1) {
            const uint64_t h = mix64((1ull << 56) ^ ((uint64_t)Y.ylevel0 << 32) ^ (uint64_t)m.e);
            m.h0 = (uint32_t)h;
            m.h1 = (uint32_t)(h >> 32);
        } else if (Y.ymode == 2) {
            // groups are sorted by level: the inner hash changes only with the level; a
            // group whose queries do not use this edge's colours gets y = 0 unhashed
            uint64_t inner = 0;
            uint32_t prev = ~0u;
#pragma unroll 1
            for (int g = 0; g < Y.ngroups; ++g) {
                uint32_t lb = 255u;
                if (!P.pcol || lane_uses(Y.gm[g], m.pc)) {
                    const uint32_t lv = Y.gl[g];
                    if (lv != prev) inner = mix64((1ull << 56) ^ ((uint64_t)lv << 32) ^ (uint64_t)m.e);
                    prev = lv;
                    const uint32_t y = (uint32_t)(mix64(Y.gs[g] ^ inner) & 0xFFu);
                    const uint32_t l7 = lds32(lds, (y << 8) | lanebits);
                    lb = l7 >= kZero7 ? 255u : (l7 >> 7);
                }
                if (g < 4) m.h0 |= lb << (8 * g);
                else m.h1 |= lb << (8 * (g - 4));
            }
        }
    }
    return m;
}

template <int W, int U>
__device__ __forceinline__ void gather_step(const StepParams &P, const WinS &cw, const WinS &nw,
                                            int32_t wb, int32_t pb, int32_t p1, bool act,
                                            bool from_x, uint64_t cmask, int lane,
                                            uint32_t (&g)[U][W]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int32_t q = pb + u;
        int32_t rg = -1, rs = -1;
        uint32_t pc = 0;
        if (q < p1) {
            const int32_t i = q - wb;  // uniform
            rg = (i < 64) ? __builtin_amdgcn_readlane(cw.g, i) : __builtin_amdgcn_readlane(nw.g, i - 64);
            rs = (i < 64) ? __builtin_amdgcn_readlane(cw.s, i) : __builtin_amdgcn_readlane(nw.s, i - 64);
            pc = (i < 64) ? __builtin_amdgcn_readlane(cw.pc, i) : __builtin_amdgcn_readlane(nw.pc, i - 64);
        }
        // both candidate rows are uniform: form their addresses in scalar registers
        // and let each lane pick by its role; a lane whose query has no vertex of one
        // of the edge's colours reads nothing (its contribution is zero)
        const uint8_t *px = P.xt + (int64_t)rs * P.rowb;
        const uint8_t *ps = P.sin + (int64_t)rg * P.rowb;
        if ((from_x ? rs : rg) >= 0 && act && lane_uses(cmask, pc)) {
            load_row<W>(from_x ? px : ps, 0, P.rowb, lane, g[u]);
        } else {
#pragma unroll
            for (int w = 0; w < W; ++w) g[u][w] = 0;
        }
    }
}

template <int W>
__global__ void __launch_bounds__(1024) k_step(StepParams P) {
    constexpr int U = (W == 4) ? 4 : kU;  // edges per batch (register budget)
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsBytes];
    __shared__ uint64_t s_gseed[kMaxYGroups];
    __shared__ uint32_t s_glevel[kMaxYGroups];
    __shared__ uint64_t s_gmask[kMaxYGroups];
    {
        const uint4 *src = (const uint4 *)P.lds_image;
        uint4 *dst = (uint4 *)lds;
        for (int i = threadIdx.x; i < kLdsBytes / 16; i += blockDim.x) dst[i] = src[i];
        if (threadIdx.x < kMaxYGroups) {
            const int g = threadIdx.x;
            s_gseed[g] = P.dtab ? P.dtab[65 + g].seed : P.gseed[g];
            s_glevel[g] = P.dtab ? P.dtab[65 + g].ylevel : P.glevel[g];
            s_gmask[g] = P.dtab ? P.dtab[65 + g].cmask : P.gmask[g];
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    StepLane L{0, 0, 0};
    YPlan Y;
    Y.gs = s_gseed;
    Y.gl = s_glevel;
    Y.gm = s_gmask;
    if (P.dtab) {
        if (lane < P.lanes) L = P.dtab[lane];
        const StepLane h = P.dtab[64];
        Y.ymode = (int)(h.flags & 0xFFu);
        Y.ngroups = (int)(h.flags >> 8);
        Y.ylevel0 = h.ylevel;
    } else {
        if (lane < P.lanes) L = P.tab[lane];
        Y.ymode = P.ymode;
        Y.ngroups = P.ngroups;
        Y.ylevel0 = P.ylevel0;
    }
    const bool act = (L.flags & kLaneActive) != 0;
    const bool from_x = (L.flags & kLaneFromX) != 0;
    const bool accm = (L.flags & kLaneAcc) != 0;
    // without colour pairs every edge counts for every lane (the pair 0|0 is tested
    // against a mask of all colours)
    const uint64_t cmask = P.pcol ? L.cmask : ~0ull;
    const uint32_t grp = (L.flags >> kLaneGroupShift) & (kMaxYGroups - 1);
    const bool grp_hi = grp >= 4;
    const uint32_t grp_shift = 8 * (grp & 3);
    const int rowd = P.rowb >> 2;
    const uint32_t lanebits = (uint32_t)(lane & 31) << 2;
    const uint32_t xbase = (uint32_t)kExpBase + lanebits;
    const uint32_t zc = (uint32_t)kExpBase + ((uint32_t)kClampRow << 7) + lanebits;
    const uint32_t epoch = __hip_atomic_load(&P.ctl->epoch, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) & 0x3FFFFFFFu;
    uint32_t fin[W];
#pragma unroll
    for (int w = 0; w < W; ++w) fin[w] = 0;

    uint32_t tk = 0;
    if (lane == 0) tk = atomicAdd(&P.ctl->ticket, 1u);
    tk = __builtin_amdgcn_readfirstlane(__shfl(tk, 0));
    for (;;) {
        const int32_t tile = (int32_t)tk;
        if (tile >= P.ntiles) break;
        const int32_t p0 = P.tile_p0[tile], p1 = P.tile_p0[tile + 1];
        const int32_t pubslot = P.tile_pub[tile], lbslot = P.tile_lb[tile];
        const bool cont = lbslot >= 0;

        int32_t wb = p0;
        WinS cw = load_wins(P, wb, p1, lane, Y, lds, lanebits);
        WinS nw = load_wins(P, wb + 64, p1, lane, Y, lds, lanebits);

        const int32_t d0 = __builtin_amdgcn_readfirstlane(cw.d);
        int32_t cur_dst = -1, nxt_dst = d0;
        uint32_t lx7[4 * W], acc[W], xn[W];
        if (act) {
            load_row<W>(P.xt, d0, P.rowb, lane, xn);
        } else {
#pragma unroll
            for (int w = 0; w < W; ++w) xn[w] = 0;
        }
#pragma unroll
        for (int w = 0; w < W; ++w) acc[w] = 0;
#pragma unroll
        for (int i = 0; i < 4 * W; ++i) lx7[i] = kZero7;

        auto process = [&](const uint32_t (&g)[U][W], int32_t pb) {
            const int nb = min(U, p1 - pb);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (u >= nb) break;
                const int32_t p = pb + u;
                const int32_t i = p - wb;
                const int32_t d = __builtin_amdgcn_readlane(cw.d, i);
                if (d != cur_dst) {
                    if (d != nxt_dst && act) load_row<W>(P.xt, d, P.rowb, lane, xn);
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        lx7[4 * w + 0] = lds32(lds, log_addr<0>(lanebits, xn[w])) + xbase;
                        lx7[4 * w + 1] = lds32(lds, log_addr<1>(lanebits, xn[w])) + xbase;
                        lx7[4 * w + 2] = lds32(lds, log_addr<2>(lanebits, xn[w])) + xbase;
                        lx7[4 * w + 3] = lds32(lds, log_addr<3>(lanebits, xn[w])) + xbase;
                        acc[w] = 0;
                    }
                    cur_dst = d;
                    uint64_t later = __ballot(cw.d != d && cw.d >= 0 && lane > i);
                    int32_t nd = -1;
                    if (later) {
                        nd = __builtin_amdgcn_readlane(cw.d, __ffsll((long long)later) - 1);
                    } else {
                        uint64_t l2 = __ballot(nw.d != d && nw.d >= 0);
                        if (l2) nd = __builtin_amdgcn_readlane(nw.d, __ffsll((long long)l2) - 1);
                    }
                    nxt_dst = nd;
                    if (nd >= 0 && act) load_row<W>(P.xt, nd, P.rowb, lane, xn);
                }
                // lanes whose query uses the edge (the others gathered nothing: their
                // g is zero); a head of a colour outside a query's multiset never feeds
                // a later edge of that query, so its rows are not stored for it
                const uint32_t pc = (uint32_t)__builtin_amdgcn_readlane(cw.pc, i);
                const bool uses = act && lane_uses(cmask, pc);
                const bool head_used = ((cmask >> (pc >> 8)) & 1ull) != 0;
                if (__ballot(uses)) {
                    // y_{e, level-1} of this lane's query
                    uint32_t ly7;
                    if (Y.ymode == 2) {
                        const uint32_t w0 = (uint32_t)__builtin_amdgcn_readlane(cw.h0, i);
                        const uint32_t w1 = (uint32_t)__builtin_amdgcn_readlane(cw.h1, i);
                        const uint32_t lb = ((grp_hi ? w1 : w0) >> grp_shift) & 0xFFu;
                        ly7 = lb == 255u ? kZero7 : (lb << 7);
                    } else {
                        uint32_t y;
                        if (Y.ymode == 1) {
                            const uint64_t inner =
                                ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(cw.h1, i) << 32) |
                                (uint64_t)(uint32_t)__builtin_amdgcn_readlane(cw.h0, i);
                            y = (uint32_t)(mix64(L.seed ^ inner) & 0xFFu);
                        } else {
                            const uint32_t eid = __builtin_amdgcn_readlane(cw.e, i);
                            y = fp8(L.seed, 1u, L.ylevel, eid);
                        }
                        ly7 = lds32(lds, (y << 8) | lanebits);
                    }
                    uint32_t c[W];
#pragma unroll
                    for (int w = 0; w < W; ++w) c[w] = mul4(lds, lanebits, g[u][w], &lx7[4 * w], ly7, zc);
                    if (accm) {
#pragma unroll
                        for (int w = 0; w < W; ++w) fin[w] ^= c[w];
                    } else {
#pragma unroll
                        for (int w = 0; w < W; ++w) acc[w] ^= c[w];
                    }
                }
                const int32_t orow = __builtin_amdgcn_readlane(cw.o, i);
                if (orow >= 0 && act && !accm && head_used) store_row<W>(P.sout, orow, P.rowb, lane, acc);
            }
            if (pb + U - wb == 64 && pb + U < p1) {
                wb += 64;
                cw = nw;
                nw = load_wins(P, wb + 64, p1, lane, Y, lds, lanebits);
            }
        };

        uint32_t ga[U][W], gb[U][W];
        gather_step<W, U>(P, cw, nw, wb, p0, p1, act, from_x, cmask, lane, ga);
        for (int32_t pb = p0; pb < p1;) {
            gather_step<W, U>(P, cw, nw, wb, pb + U, p1, act, from_x, cmask, lane, gb);
            process(ga, pb);
            pb += U;
            if (pb >= p1) break;
            gather_step<W, U>(P, cw, nw, wb, pb + U, p1, act, from_x, cmask, lane, ga);
            process(gb, pb);
            pb += U;
        }

        if (lane < P.lanes) {
            if (pubslot >= 0)
                publish<W>(P.pub, pubslot, rowd, P.lanes, lane, cont ? kAgg : kInc, epoch, acc);
            if (cont) {
                uint32_t carry[W];
                lookback<W>(P.pub, lbslot, rowd, P.lanes, lane, epoch, P.ctl, carry);
                if (pubslot >= 0) {
                    uint32_t inc[W];
#pragma unroll
                    for (int w = 0; w < W; ++w) inc[w] = acc[w] ^ carry[w];
                    publish<W>(P.pub, pubslot, rowd, P.lanes, lane, kInc, epoch, inc);
                }
                if (act && !accm) {
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                    for (int32_t p = p0; p < p1; ++p) {
                        const int32_t orow = P.orow[p];
                        if (orow >= 0) {
                            uint32_t v[W];
                            load_row<W>(P.sout, orow, P.rowb, lane, v);
#pragma unroll
                            for (int w = 0; w < W; ++w) v[w] ^= carry[w];
                            store_row<W>(P.sout, orow, P.rowb, lane, v);
                        }
                    }
                }
            }
        }
        uint32_t tk_next = 0;
        if (lane == 0) tk_next = atomicAdd(&P.ctl->ticket, 1u);
        tk = __builtin_amdgcn_readfirstlane(__shfl(tk_next, 0));
    }

    if (act && accm) {
#pragma unroll
        for (int w = 0; w < W; ++w)
            if (fin[w]) atomicXor(&P.fin[lane * W + w], fin[w]);
    }
}

// ---------------------------------------------------------------------------------
// Static instance (preprocessing step (ii)): each vertex of the instance has a row of
// rowb sieve points (lanes * 4 W bytes), stored in compact vertex order.
// ---------------------------------------------------------------------------------
constexpr int kStaticTile = 256;  // positions per tile of k_sgather

// Product of two dwords of field elements, byte by byte, through the LDS tables.
__device__ __forceinline__ uint32_t gmul4(const uint8_t *lds, uint32_t lanebits, uint32_t a,
                                          uint32_t b, uint32_t xbase, uint32_t zc) {
    uint32_t s0 = min(lds32(lds, log_addr<0>(lanebits, a)) + lds32(lds, log_addr<0>(lanebits, b)) + xbase, zc);
    uint32_t s1 = min(lds32(lds, log_addr<1>(lanebits, a)) + lds32(lds, log_addr<1>(lanebits, b)) + xbase, zc);
    uint32_t s2 = min(lds32(lds, log_addr<2>(lanebits, a)) + lds32(lds, log_addr<2>(lanebits, b)) + xbase, zc);
    uint32_t s3 = min(lds32(lds, log_addr<3>(lanebits, a)) + lds32(lds, log_addr<3>(lanebits, b)) + xbase, zc);
    return pack4(lds[s0], lds[s1], lds[s2], lds[s3]);
}

__device__ __forceinline__ void load_lds_image(uint8_t *lds, const uint8_t *image) {
    const uint4 *src = (const uint4 *)image;
    uint4 *dst = (uint4 *)lds;
    for (int i = threadIdx.x; i < kLdsBytes / 16; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

// sum[seg] = sum over the positions p of seg's list of y_{key[p], ylevel} * rows[gat[p]]
// (the sum of Eq. (1) before the factor x; ylevel is the walk position of the arc).
// One wave per tile of kStaticTile positions.  A list that a tile boundary cuts adds
// its parts with atomic XOR into a row the caller cleared; a list inside one tile is
// stored.
template <int W>
__global__ void __launch_bounds__(1024) k_sgather(int64_t m, const int32_t *seg, const int32_t *gat,
                                                  const int32_t *key, const uint8_t *rows,
                                                  uint8_t *sum, int32_t rowb, int32_t lanes,
                                                  uint64_t seed, uint32_t ylevel,
                                                  const uint8_t *lds_image) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsBytes];
    load_lds_image(lds, lds_image);
    const int lane = threadIdx.x & 63;
    const bool act = lane < lanes;
    const uint32_t lanebits = (uint32_t)(lane & 31) << 2;
    const uint32_t xbase = (uint32_t)kExpBase + lanebits;
    const uint32_t zc = (uint32_t)kExpBase + ((uint32_t)kClampRow << 7) + lanebits;
    uint32_t lx7[4 * W];
#pragma unroll
    for (int i = 0; i < 4 * W; ++i) lx7[i] = xbase;  // x = 1
    const int64_t ntiles = (m + kStaticTile - 1) / kStaticTile;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    auto flush = [&](int32_t d, const uint32_t (&acc)[W], bool shared) {
        if (!act) return;
        if (shared) {
            uint32_t *row = (uint32_t *)(sum + (int64_t)d * rowb + (int64_t)lane * (4 * W));
#pragma unroll
            for (int w = 0; w < W; ++w)
                if (acc[w]) atomicXor(row + w, acc[w]);
        } else {
            store_row<W>(sum, d, rowb, lane, acc);
        }
    };
    for (int64_t t = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); t < ntiles;
         t += nwaves) {
        const int64_t p0 = t * kStaticTile, p1 = min(p0 + (int64_t)kStaticTile, m);
        const int32_t sfirst = seg[p0], slast = seg[p1 - 1];
        const bool open_l = p0 > 0 && seg[p0 - 1] == sfirst;
        const bool open_r = p1 < m && seg[p1] == slast;
        uint32_t acc[W];
#pragma unroll
        for (int w = 0; w < W; ++w) acc[w] = 0;
        int32_t cur = sfirst;
        bool shared = open_l;
        for (int64_t wb = p0; wb < p1; wb += 64) {
            const int nb = (int)min<int64_t>(64, p1 - wb);
            int32_t ms = -1, mg = -1;
            uint32_t ly = kZero7;
            if (lane < nb) {
                ms = seg[wb + lane];
                mg = gat[wb + lane];
                const uint32_t y = fp8(seed, 4u, ylevel, (uint32_t)key[wb + lane]);
                ly = lds32(lds, (y << 8) | lanebits);
            }
            for (int i0 = 0; i0 < nb; i0 += kU) {
                uint32_t g[kU][W];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int i = min(i0 + u, 63);
                    const int32_t r = __builtin_amdgcn_readlane(mg, i);
                    if (i0 + u < nb && r >= 0 && act) {
                        load_row<W>(rows, r, rowb, lane, g[u]);
                    } else {
#pragma unroll
                        for (int w = 0; w < W; ++w) g[u][w] = 0;
                    }
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    if (i0 + u >= nb) break;
                    const int i = i0 + u;
                    const int32_t d = __builtin_amdgcn_readlane(ms, i);
                    if (d != cur) {
                        flush(cur, acc, shared);
#pragma unroll
                        for (int w = 0; w < W; ++w) acc[w] = 0;
                        cur = d;
                        shared = false;
                    }
                    const uint32_t ly7 = __builtin_amdgcn_readlane(ly, i);
#pragma unroll
                    for (int w = 0; w < W; ++w) acc[w] ^= mul4(lds, lanebits, g[u][w], &lx7[4 * w], ly7, zc);
                }
            }
        }
        flush(cur, acc, shared || open_r);
    }
}

// Per vertex u of the instance (one wave per row): prod = x_u * g_u with g_u = sum[u]
// (1 when sum is null); out[u] = prod (out nullable); sv[vid[u]] ^= the XOR over the
// row's points of prod (with_prod) and of fin[u] * g_u (fin nullable).
template <int W>
__global__ void __launch_bounds__(1024) k_svertex(int32_t n, const uint8_t *sum, const uint8_t *x,
                                                  const uint8_t *fin, uint8_t *out, int with_prod,
                                                  const int32_t *vid, uint8_t *sv, int32_t rowb,
                                                  int32_t lanes, const uint8_t *lds_image) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsBytes];
    load_lds_image(lds, lds_image);
    const int lane = threadIdx.x & 63;
    const bool act = lane < lanes;
    const uint32_t lanebits = (uint32_t)(lane & 31) << 2;
    const uint32_t xbase = (uint32_t)kExpBase + lanebits;
    const uint32_t zc = (uint32_t)kExpBase + ((uint32_t)kClampRow << 7) + lanebits;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); u < n; u += nwaves) {
        uint32_t r = 0;
        if (act) {
            uint32_t xv[W], gv[W], pv[W];
            load_row<W>(x, u, rowb, lane, xv);
            if (sum) {
                load_row<W>(sum, u, rowb, lane, gv);
#pragma unroll
                for (int w = 0; w < W; ++w) pv[w] = gmul4(lds, lanebits, xv[w], gv[w], xbase, zc);
            } else {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    gv[w] = 0x01010101u;
                    pv[w] = xv[w];
                }
            }
            if (out) store_row<W>(out, u, rowb, lane, pv);
            if (with_prod) {
#pragma unroll
                for (int w = 0; w < W; ++w) r ^= pv[w];
            }
            if (fin) {
                uint32_t fv[W];
                load_row<W>(fin, u, rowb, lane, fv);
#pragma unroll
                for (int w = 0; w < W; ++w) r ^= gmul4(lds, lanebits, fv[w], gv[w], xbase, zc);
            }
        }
        r ^= r >> 16;
        r ^= r >> 8;
        r &= 0xFFu;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) r ^= __shfl_xor(r, off);
        if (lane == 0 && r) sv[vid[u]] ^= (uint8_t)r;
    }
}

// zs[i] = z[vid[i]] (16-byte rows)
__global__ void k_zgather(int32_t n, const int32_t *vid, const uint8_t *z, uint8_t *zs) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ((uint4 *)zs)[i] = ((const uint4 *)z)[vid[i]];
}

// k = 1: sv[u] ^= x_u at the point {0} = z_{u,0}
__global__ void k_single_v(int32_t n, const uint8_t *z, uint8_t *sv) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) sv[u] ^= z[u * 16];
}

QuerySlots make_slots(const Graph &G, const int32_t *M, int32_t k) {
    TPM_REQUIRE(M != nullptr, "multiset must not be NULL");
    TPM_REQUIRE(k >= 1 && k <= 16, "k must be in [1, 16]");
    int32_t cols[16];
    for (int i = 0; i < k; ++i) {
        TPM_REQUIRE(M[i] >= -1 && M[i] < G.q, "multiset colour out of range");
        cols[i] = M[i];  // -1: wildcard (sorts first, so it owns the first slots)
    }
    std::sort(cols, cols + k);
    QuerySlots qs{};
    int next = 0;
    for (int i = 0; i < k;) {
        int j = i;
        while (j < k && cols[j] == cols[i]) ++j;
        qs.col[qs.ncol] = cols[i];
        qs.off[qs.ncol] = next;
        qs.mu[qs.ncol] = j - i;
        next += j - i;
        ++qs.ncol;
        i = j;
    }
    return qs;
}

// Persistent grid: one 1024-thread workgroup per CU (a small launch still spreads its
// tiles over as many CUs as it has)
unsigned persistent_grid(const Graph &G, int64_t tiles) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(G.num_cu, tiles));
}

template <int W, bool FIN>
void launch_level(const Graph &G, const LevelParams &P, hipStream_t st) {
    hipLaunchKernelGGL((k_level<W, FIN>), dim3(persistent_grid(G, P.tile_hi - P.tile_lo)),
                       dim3(1024), 0, st, P);
}

// 128- to 512-point rows run slot tiles (k_slot), smaller rows the scan kernel
// (k_narrow).  Per middle level of a 1e8-edge graph: 512 points 13.3 ms (k_level with
// 2 dwords a lane: 14.9), 256 points 7.4 ms (k_narrow 9.5), 128 points 4.6 ms (k_narrow
// 5.4), but 64 points 4.3 against 3.2 ms for k_narrow (sixteen tiles per ticket leave
// too few tickets per wave to balance).  At 1024 points a single slot matches k_level
// (25.8 ms) and k_level stays.
template <int LP>
void launch_narrow(bool fin, const Graph &G, const LevelParams &P, hipStream_t st) {
    if constexpr (LP >= 8) {
        constexpr int E = 64 / LP;
        const dim3 grid(persistent_grid(G, (P.tile_hi - P.tile_lo + E - 1) / E));
        if (fin) hipLaunchKernelGGL((k_slot<LP, true>), grid, dim3(1024), 0, st, P);
        else hipLaunchKernelGGL((k_slot<LP, false>), grid, dim3(1024), 0, st, P);
    } else {
        const dim3 grid(persistent_grid(G, P.tile_hi - P.tile_lo));
        if (fin) hipLaunchKernelGGL((k_narrow<LP, true>), grid, dim3(1024), 0, st, P);
        else hipLaunchKernelGGL((k_narrow<LP, false>), grid, dim3(1024), 0, st, P);
    }
}

// rows of 16..512 points run several positions per wave (k_slot, k_narrow); rows of
// 1024 points run one position per wave (k_level).  Rows of 16..256 points:
bool is_narrow(int rowb) { return rowb >= 16 && rowb <= 256; }

void launch_level_any(int rowb, bool fin, const Graph &G, const LevelParams &P, hipStream_t st) {
    if (rowb == 512) {  // two slots of 32 lanes per wave
        launch_narrow<32>(fin, G, P, st);
        return;
    }
    switch (is_narrow(rowb) ? rowb / 16 : 0) {
        case 1: launch_narrow<1>(fin, G, P, st); break;
        case 2: launch_narrow<2>(fin, G, P, st); break;
        case 4: launch_narrow<4>(fin, G, P, st); break;
        case 8: launch_narrow<8>(fin, G, P, st); break;
        case 16: launch_narrow<16>(fin, G, P, st); break;
        default:
            TPM_REQUIRE(rowb == 1024, "sieve rows hold 16..1024 points");
            fin ? launch_level<4, true>(G, P, st) : launch_level<4, false>(G, P, st);
    }
}

void launch_step_w(int W, const Graph &G, const StepParams &P, hipStream_t st) {
    const dim3 grid(persistent_grid(G, P.ntiles));
    if (W == 4) hipLaunchKernelGGL((k_step<4>), grid, dim3(1024), 0, st, P);
    else if (W == 2) hipLaunchKernelGGL((k_step<2>), grid, dim3(1024), 0, st, P);
    else hipLaunchKernelGGL((k_step<1>), grid, dim3(1024), 0, st, P);
}

int pick_chunk(const Graph &G, int32_t k, int32_t requested) {
    const int64_t npts = int64_t(1) << k;
    int64_t c = requested > 0 ? requested : std::min<int64_t>(npts, 1024);
    TPM_REQUIRE((c & (c - 1)) == 0 && c >= 4 && c <= 1024, "chunk must be a power of two in [4, 1024]");
    c = std::min<int64_t>(c, std::max<int64_t>(npts, 16));
    // fit the two level buffers (and level 2's coefficients, 20 bytes a row) into free
    // device memory
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) == hipSuccess && requested <= 0) {
        const double fixed = k > 2 ? 20.0 * (double)G.R : 0.0;
        while (c > 16 && (double)(2 * G.R + G.n + 2 * G.nslots) * c + fixed > 0.85 * (double)freeb) c >>= 1;
    }
    // rows hold at least 16 points (one lane): smaller queries repeat their points
    return (int)std::max<int64_t>(c, 16);
}

}  // namespace

// A cancelled (or expired) request stops between launches: the work already queued
// on the stream completes before the error leaves, so no kernel outlives its buffers.
void check_cancel(const SieveRequest &req, hipStream_t st) {
    const bool c = req.cancel && req.cancel->load(std::memory_order_relaxed) != 0;
    const bool late = req.deadline_ms > 0 && now_ms() > req.deadline_ms;
    if (c || late) {
        (void)hipStreamSynchronize(st);
        throw Error{TPM_ECANCELLED, c ? "request cancelled" : "request deadline passed"};
    }
}

namespace {
// Device buffers of one sieve query: per-vertex z and x rows, the two level buffers,
// published look-back words, control words, per-point accumulators (zeroed by the
// caller) and, nullable, per-position localisation bytes of the last level.
// ---------------------------------------------------------------------------------
// Level 2 from coefficients.  x_u^A = XOR over j in A of z_u[j] is linear in A's
// indicator, and GF(2^8) multiplication distributes over XOR, so the level-2 running
// value of v's in-list after position p is
//     x_v^A * (XOR over j in A of W_p[j]),   W_p[j] = XOR over q <= p in the list of
//                                                    y_q * z_{src q}[j]:
// k bytes per position instead of a row of 2^k points.  W is a segmented XOR scan
// over the in-edge order (a segment per in-list), in blocks of 256 positions whose
// carries are scanned apart; a stored row is then expanded once per chunk from W, z_v
// and the LDS tables.  Bit for bit the level kernel's rows, without its gather of the
// 1 KB x row of every edge's source.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ uint4 xor4(uint4 a, uint4 b) {
    return make_uint4(a.x ^ b.x, a.y ^ b.y, a.z ^ b.z, a.w ^ b.w);
}

// The field's log and exp tables in LDS for a block (768 bytes; the constant-memory
// copy costs a vector memory load per lookup).  Every thread must call it.
struct W2Tabs {
    uint8_t exp[512];
    uint8_t log[256];
};

__device__ __forceinline__ void w2_tabs_load(W2Tabs &t) {
    for (int i = threadIdx.x; i < 512; i += blockDim.x) t.exp[i] = c_gf.exp[i];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) t.log[i] = c_gf.log[i];
    __syncthreads();
}

// y_p * z_{src p}, bytewise (z rows hold zeros past byte k - 1)
__device__ __forceinline__ uint4 w2_term(const W2Tabs &tb, const int32_t *psrc, const int32_t *peid,
                                         const uint8_t *z, uint64_t seed, int64_t p) {
    const uint32_t y = fp8(seed, 1u, 1u, (uint32_t)peid[p]);
    const uint4 zz = ((const uint4 *)z)[psrc[p]];
    uint32_t w[4] = {zz.x, zz.y, zz.z, zz.w};
    if (y == 0) return make_uint4(0, 0, 0, 0);
    const uint32_t ly = tb.log[y];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint32_t o = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uint32_t b = (w[i] >> (8 * t)) & 0xFFu;
            if (b) o |= (uint32_t)tb.exp[ly + tb.log[b]] << (8 * t);
        }
        w[i] = o;
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Inclusive XOR scan of v over the block of 256 threads within segments (a segment
// starts where head is set); open: no head from the block's first position to this
// one.  Every thread of the block must call it.
__device__ __forceinline__ uint4 w2_block_scan(uint4 v, bool head, bool &open) {
    __shared__ uint4 wv[4];
    __shared__ uint32_t wf[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool f = head;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint4 o;
        o.x = __shfl_up(v.x, off);
        o.y = __shfl_up(v.y, off);
        o.z = __shfl_up(v.z, off);
        o.w = __shfl_up(v.w, off);
        const int of = __shfl_up((int)f, off);
        if (lane >= off) {
            if (!f) v = xor4(v, o);
            f = f || of;
        }
    }
    if (lane == 63) {
        wv[wave] = v;
        wf[wave] = f ? 1u : 0u;
    }
    __syncthreads();
    for (int u = wave - 1; u >= 0 && !f; --u) {
        v = xor4(v, wv[u]);
        f = wf[u] != 0;
    }
    open = !f;
    return v;
}

__device__ __forceinline__ uint4 w2_position(int64_t m, const int32_t *pdst, const int32_t *psrc,
                                             const int32_t *peid, const uint8_t *z, uint64_t seed,
                                             int64_t p, bool &open) {
    __shared__ W2Tabs tb;
    w2_tabs_load(tb);
    uint4 v = make_uint4(0, 0, 0, 0);
    bool head = true;  // past the end: empty segments
    if (p < m) {
        v = w2_term(tb, psrc, peid, z, seed, p);
        head = p == 0 || pdst[p] != pdst[p - 1];
    }
    return w2_block_scan(v, head, open);
}

// per block of 256 positions: its value at its last position and whether a segment
// starts in it
__global__ void __launch_bounds__(256) k_w2_blocks(int64_t m, const int32_t *pdst, const int32_t *psrc,
                                                   const int32_t *peid, const uint8_t *z, uint64_t seed,
                                                   W2Agg *agg) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool open;
    const uint4 v = w2_position(m, pdst, psrc, peid, z, seed, p, open);
    if (threadIdx.x == 255) {
        W2Agg a{};
        a.v = v;
        a.head = open ? 0u : 1u;
        agg[blockIdx.x] = a;
    }
}

// W and the in-list's vertex at every needed position (row r = orow[p]); scanned: the
// inclusive scan of the block aggregates (carry into block b: scanned[b - 1])
__global__ void __launch_bounds__(256) k_w2_final(int64_t m, const int32_t *pdst, const int32_t *psrc,
                                                  const int32_t *peid, const uint8_t *z, uint64_t seed,
                                                  const W2Agg *scanned, const int32_t *orow,
                                                  uint4 *W, int32_t *V) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool open;
    uint4 v = w2_position(m, pdst, psrc, peid, z, seed, p, open);
    if (p >= m) return;
    if (open && blockIdx.x > 0) v = xor4(v, scanned[blockIdx.x - 1].v);
    const int32_t r = orow[p];
    if (r >= 0) {
        W[r] = v;
        V[r] = pdst[p];
    }
}

// Rows of the chunk of rowb points from base: row r, points A = base + i, byte i =
// x_{V[r]}^A * (XOR over j in A, j < k, of W[r][j]) (bits of A from k on are ignored,
// as in the x rows).  Persistent grid of 1024-thread blocks (the LDS tables fill the
// CU); a thread makes 16 points of a row, four rows' worth of loads in flight (W, V,
// then z of V: a dependent pair of loads per row that one row at a time left waiting).
__device__ __forceinline__ uint4 w2_expand(const uint8_t *lds, uint32_t lanebits, uint32_t ebase,
                                           uint32_t zc, int32_t k, uint32_t A0, uint4 w4, uint4 z4) {
    const uint32_t ww[4] = {w4.x, w4.y, w4.z, w4.w}, zw[4] = {z4.x, z4.y, z4.z, z4.w};
    uint32_t xh = 0, sh = 0;
    for (int j = 4; j < k; ++j)
        if ((A0 >> j) & 1u) {
            xh ^= (zw[j >> 2] >> (8 * (j & 3))) & 0xFFu;
            sh ^= (ww[j >> 2] >> (8 * (j & 3))) & 0xFFu;
        }
    uint32_t xl[16], sl[16];
    xl[0] = sl[0] = 0;
#pragma unroll
    for (int b = 1; b < 16; ++b) {
        const int j = __builtin_ctz(b);  // j < 4: bytes of the first dword
        const uint32_t zj = j < k ? (zw[0] >> (8 * j)) & 0xFFu : 0u;
        const uint32_t wj = j < k ? (ww[0] >> (8 * j)) & 0xFFu : 0u;
        xl[b] = xl[b & (b - 1)] ^ zj;
        sl[b] = sl[b & (b - 1)] ^ wj;
    }
    uint32_t out[4] = {0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        const uint32_t x = xh ^ xl[b], s = sh ^ sl[b];
        const uint32_t a = min(lds32(lds, (x << 8) | lanebits) + lds32(lds, (s << 8) | lanebits) + ebase, zc);
        out[b >> 2] |= (uint32_t)lds[a] << (8 * (b & 3));
    }
    return make_uint4(out[0], out[1], out[2], out[3]);
}

__global__ void __launch_bounds__(1024) k_w2_rows(int64_t R, int32_t k, int32_t rowb, uint32_t base,
                                                  const uint4 *W, const int32_t *V, const uint8_t *z,
                                                  const uint8_t *lds_image, uint8_t *rows) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsBytes];
    {
        const uint4 *src = (const uint4 *)lds_image;
        uint4 *dst = (uint4 *)lds;
        for (int i = threadIdx.x; i < kLdsBytes / 16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    constexpr int UR = 4;  // rows per thread per round
    const uint32_t lanebits = (uint32_t)(threadIdx.x & 31) << 2;
    const uint32_t ebase = (uint32_t)kExpBase + lanebits;
    const uint32_t zc = (uint32_t)kExpBase + ((uint32_t)kClampRow << 7) + lanebits;
    const int lp = __builtin_ctz((uint32_t)(rowb >> 4));  // parts per row: a power of two
    const int64_t items = R << lp;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t it0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it0 < items; it0 += UR * stride) {
        uint4 w[UR], zz[UR];
        int32_t v[UR];
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const int64_t it = it0 + u * stride;
            if (it < items) {
                w[u] = W[it >> lp];
                v[u] = V[it >> lp];
            }
        }
#pragma unroll
        for (int u = 0; u < UR; ++u)
            if (it0 + u * stride < items) zz[u] = ((const uint4 *)z)[v[u]];
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const int64_t it = it0 + u * stride;
            if (it < items) {
                const int64_t r = it >> lp;
                const uint32_t part = (uint32_t)(it & ((1 << lp) - 1));
                const uint4 o = w2_expand(lds, lanebits, ebase, zc, k, base + part * 16u, w[u], zz[u]);
                *(uint4 *)(rows + r * (int64_t)rowb + (int64_t)part * 16) = o;
            }
        }
    }
}

// Rows of P = 2^k points of a query of 4 <= k <= 10 (one chunk).  A row has P / 16
// lanes; lane l of a row makes points A = 16 l + b: the bits of l are variables 4..k-1
// (the lane's part H), those of b variables 0..3 (B), and with x_H = XOR over j in H of
// z_j and S_H likewise of W_j,
//   x^A S^A = K + XOR over i in B of L_i + XOR over i < j in B of q_ij,
//   K = x_H S_H,  L_i = z_i (S_H + W_i) + x_H W_i,  q_ij = z_i W_j + z_j W_i:
// 21 products a lane instead of 16 per group of 16 points, then the points by XOR.  W,
// V and z of 64 rows are loaded together, one row per lane, and passed to the lanes of
// each row by shuffles, the next 64 loaded while these are made.  Products by the LDS
// tables (persistent grid of 1024-thread blocks).
__global__ void __launch_bounds__(1024) k_w2_rows_q(int64_t R, int32_t k, const uint4 *W,
                                                    const int32_t *V, const uint8_t *z,
                                                    const uint8_t *lds_image, uint8_t *rows) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[kLdsBytes];
    {
        const uint4 *src = (const uint4 *)lds_image;
        uint4 *dst = (uint4 *)lds;
        for (int i = threadIdx.x; i < kLdsBytes / 16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint32_t lanebits = (uint32_t)(lane & 31) << 2;
    const uint32_t ebase = (uint32_t)kExpBase + lanebits;
    const uint32_t zc = (uint32_t)kExpBase + ((uint32_t)kClampRow << 7) + lanebits;
    auto lg = [&](uint32_t g) -> uint32_t { return lds32(lds, (g << 8) | lanebits); };
    auto ex = [&](uint32_t l1, uint32_t l2) -> uint32_t { return lds[min(l1 + l2 + ebase, zc)]; };
    const int nh = k - 4;                // variables from the lane's index in its row
    const int lr = 1 << nh;              // lanes per row
    const int rpw = 64 >> nh;            // rows a wave makes per round
    const int grp = lane >> nh, li = lane & (lr - 1);
    const int64_t P = (int64_t)lr * 16;  // points (bytes) per row
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    uint4 w4 = make_uint4(0, 0, 0, 0), z4 = make_uint4(0, 0, 0, 0);
    if (gw * 64 + lane < R) {
        w4 = W[gw * 64 + lane];
        z4 = ((const uint4 *)z)[V[gw * 64 + lane]];
    }
    for (int64_t bi = gw; bi * 64 < R; bi += nw) {
        // the next 64 rows' W and V now, their z half-way through these
        const int64_t rn = (bi + nw) * 64 + lane;
        const bool hn = rn < R;
        uint4 wn = make_uint4(0, 0, 0, 0), zn = make_uint4(0, 0, 0, 0);
        int32_t vn = 0;
        bool zdone = false;
        if (hn) {
            wn = W[rn];
            vn = V[rn];
        }
        const int nrows = (int)min<int64_t>(64, R - bi * 64);
        for (int t0 = 0; t0 < nrows; t0 += rpw) {
            if (t0 >= 32 && !zdone) {
                if (hn) zn = ((const uint4 *)z)[vn];
                zdone = true;
            }
            const int src = t0 + grp;  // the lane that holds this lane's row
            const uint32_t z0 = (uint32_t)__shfl((int)z4.x, src), z1 = (uint32_t)__shfl((int)z4.y, src);
            const uint32_t z2 = (uint32_t)__shfl((int)z4.z, src);
            const uint32_t w0 = (uint32_t)__shfl((int)w4.x, src), w1 = (uint32_t)__shfl((int)w4.y, src);
            const uint32_t w2 = (uint32_t)__shfl((int)w4.z, src);
            // variables 4..k-1: bytes 0..3 of dword 1 and 0..1 of dword 2
            uint32_t xh = 0, sh = 0;
#pragma unroll
            for (int h = 0; h < 6; ++h) {
                const uint32_t zb = ((h < 4 ? z1 : z2) >> (8 * (h & 3))) & 0xFFu;
                const uint32_t wb = ((h < 4 ? w1 : w2) >> (8 * (h & 3))) & 0xFFu;
                const bool on = h < nh && ((li >> h) & 1);
                xh ^= on ? zb : 0u;
                sh ^= on ? wb : 0u;
            }
            const uint32_t lxh = lg(xh), lsh = lg(sh);
            uint32_t lz[4], lw[4], Lc[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t zi = (z0 >> (8 * i)) & 0xFFu, wi = (w0 >> (8 * i)) & 0xFFu;
                lz[i] = lg(zi);
                lw[i] = lg(wi);
                Lc[i] = ex(lz[i], lg(sh ^ wi)) ^ ex(lxh, lw[i]);
            }
            uint32_t q[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = a + 1; b < 4; ++b) q[a][b] = ex(lz[a], lw[b]) ^ ex(lz[b], lw[a]);
            uint32_t val[16];
            val[0] = ex(lxh, lsh);
#pragma unroll
            for (int b = 1; b < 16; ++b) {
                const int lo = __builtin_ctz(b), rest = b & (b - 1);
                uint32_t u2 = Lc[lo];
#pragma unroll
                for (int j = lo + 1; j < 4; ++j)
                    if ((rest >> j) & 1) u2 ^= q[lo][j];
                val[b] = val[rest] ^ u2;
            }
            uint32_t out[4];
#pragma unroll
            for (int d = 0; d < 4; ++d)
                out[d] = pack4(val[4 * d], val[4 * d + 1], val[4 * d + 2], val[4 * d + 3]);
            if (src < nrows)
                *(uint4 *)(rows + (bi * 64 + src) * P + (int64_t)li * 16) =
                    make_uint4(out[0], out[1], out[2], out[3]);
        }
        if (hn && !zdone) zn = ((const uint4 *)z)[vn];
        w4 = wn;
        z4 = zn;
    }
}

struct LevelBufs {
    uint8_t *z = nullptr, *xt = nullptr, *s0 = nullptr, *s1 = nullptr, *pp = nullptr;
    unsigned long long *pub = nullptr;
    Ctl *ctl = nullptr;
    uint8_t *loc = nullptr;
    // level 2 from coefficients (nullable: level 2 gathers x rows): W and V per row,
    // block aggregates and their scan, the scan's temporary storage
    uint4 *w2W = nullptr;
    int32_t *w2V = nullptr;
    W2Agg *w2agg = nullptr, *w2scan = nullptr;
    void *w2tmp = nullptr;
    size_t w2tmp_bytes = 0;
};

// Bytes of the coefficient form of level 2 for a graph: W and V per row, two block
// aggregates per 256 positions, the scan's temporary storage (aligned).
size_t w2_bytes(const Graph &G, size_t &tmp_bytes) {
    const int64_t nb = (G.m + 255) / 256;
    tmp_bytes = w2_scan(nullptr, 0, nullptr, nullptr, nb, nullptr);
    return (size_t)std::max<int64_t>(1, G.R) * 20 + 256 + (size_t)nb * 2 * sizeof(W2Agg) + 256 +
           tmp_bytes;
}

// Points the LevelBufs at a w2_bytes block.
void w2_place(const Graph &G, uint8_t *blk, size_t tmp_bytes, LevelBufs &B) {
    const int64_t nb = (G.m + 255) / 256;
    const size_t R = (size_t)std::max<int64_t>(1, G.R);
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t o = 0;
    B.w2W = (uint4 *)(blk + o);
    o += R * 16;
    B.w2V = (int32_t *)(blk + o);
    o = up(o + R * 4);
    B.w2agg = (W2Agg *)(blk + o);
    B.w2scan = B.w2agg + nb;
    o = up(o + (size_t)nb * 2 * sizeof(W2Agg));
    B.w2tmp = blk + o;
    B.w2tmp_bytes = tmp_bytes;
}

// Enqueues levels 2..k of every chunk of rowb points in [0, pts_end) on st: the x rows
// of the chunk, then one level kernel per level, the last one accumulating into
// pp[base ..] (positions [lo, hi) contribute; its tiles are [fin_tlo, fin_thi)).  z must
// hold the query's z rows.  With a request, cancellation is checked between launches.
void enqueue_chunks(const Graph &G, int32_t k, uint64_t seed, int rowb, int64_t pts_end,
                    const LevelBufs &B, int64_t lo, int64_t hi, int32_t fin_tlo, int32_t fin_thi,
                    const SieveRequest *req, bool profile, hipStream_t st) {
    const int64_t npts = int64_t(1) << k;
    // lanes holding points: 64 lanes of 16 points for 1024-point rows, else one 16-point
    // lane per 16 points of a narrow row (its 1024 / rowb slots repeat the same lanes)
    const int lanes = std::max(1, rowb / 16);
    // level 2 from coefficients: W once for every chunk
    const bool w2 = B.w2W != nullptr && k >= 3 && G.m > 0;
    if (w2) {
        const int64_t nb = (G.m + 255) / 256;
        k_w2_blocks<<<(unsigned)nb, 256, 0, st>>>(G.m, G.pdst, G.psrc, G.peid, B.z, seed, B.w2agg);
        w2_scan(B.w2tmp, B.w2tmp_bytes, B.w2agg, B.w2scan, nb, st);
        k_w2_final<<<(unsigned)nb, 256, 0, st>>>(G.m, G.pdst, G.psrc, G.peid, B.z, seed, B.w2scan,
                                                  G.orow, B.w2W, B.w2V);
    }
    for (int64_t base = 0; base < pts_end; base += rowb) {
        k_xt<<<grid_for((int64_t)G.n * ((rowb + 15) / 16)), 256, 0, st>>>(
            G.n, k, rowb, rowb, 0, (uint32_t)base, B.z, B.xt, G.color, G.edge_colors);
        for (int l = 2; l <= k; ++l) {
            if (req) {
                check_cancel(*req, st);
                if (req->between_levels) (*req->between_levels)(st);
            }
            const bool fin = (l == k);
            if (l == 2 && w2) {  // rows expanded from W into s0, the level-2 output
                const int64_t items = G.R * (rowb / 16);
                if (items > 0) {
                    const unsigned grid = (unsigned)std::max<int64_t>(
                        1, std::min<int64_t>(G.num_cu, (items + 1023) / 1024));
                    // one chunk of 2^k points, 4 <= k <= 10: the quadratic form per lane
                    const bool quad = k >= 4 && k <= 10 && rowb == (1 << k);
                    const unsigned gq = (unsigned)std::max<int64_t>(
                        1, std::min<int64_t>(G.num_cu, (G.R + 1023) / 1024));
                    std::unique_ptr<ProfileScope> prof;
                    if (profile) prof.reset(new ProfileScope(st, 0, l, rowb));
                    if (quad)
                        k_w2_rows_q<<<gq, 1024, 0, st>>>(G.R, k, B.w2W, B.w2V, B.z, G.lds_image, B.s0);
                    else
                        k_w2_rows<<<grid, 1024, 0, st>>>(G.R, k, rowb, (uint32_t)base, B.w2W, B.w2V,
                                                         B.z, G.lds_image, B.s0);
                }
                continue;
            }
            LevelParams P{};
            P.gidx = (l == 2) ? G.psrc : G.gsrc;
            P.gbase = (l == 2) ? B.xt : ((l & 1) ? B.s0 : B.s1);
            P.pdst = G.pdst;
            P.peid = G.peid;
            P.orow = G.orow;
            P.sout = (l & 1) ? B.s1 : B.s0;
            P.xt = B.xt;
            P.tile_p0 = G.tile_p0;
            P.tile_pub = G.tile_pub;
            P.tile_lb = G.tile_lb;
            P.tile_lo = fin ? fin_tlo : 0;
            P.tile_hi = fin ? fin_thi : (int32_t)G.ntiles;
            P.pos_lo = (int32_t)lo;
            P.pos_hi = (int32_t)hi;
            P.pub = B.pub;
            P.ctl = B.ctl;
            P.fin = (uint32_t *)(B.pp + base);
            P.loc = B.loc;
            P.lds_image = G.lds_image;
            P.seed = seed;
            P.ylevel = (uint32_t)(l - 1);
            P.rowb = rowb;
            P.lanes = lanes;
            P.valid_pts = (int32_t)std::min<int64_t>(rowb, npts - base);
            k_prep<<<1, 1, 0, st>>>(B.ctl, fin ? 0 : 1);
            if (profile) {
                ProfileScope prof(st, fin ? 2 : (l == 2 ? 0 : 1), l, rowb);
                launch_level_any(rowb, fin, G, P, st);
            } else {
                launch_level_any(rowb, fin, G, P, st);
            }
        }
    }
}
}  // namespace

// Positions [lo, hi) of the last level contribute (all when fin_lo >= fin_hi).  With
// want_loc, the per-position localisation over that range is computed on the device;
// loc_host (nullable, hi - lo bytes) receives it, and res.pick_eid / res.pick_pos get
// the contributing position with nonzero localisation and the smallest input edge id
// (-1 if none).
void run_sieve_impl(const Graph &G, const SieveRequest &req, SieveResult &res, bool want_loc,
                    uint8_t *loc_host, hipStream_t st, LocSink *sink = nullptr) {
    const int32_t k = req.k;
    QuerySlots qs = make_slots(G, req.multiset, k);
    const int64_t npts = int64_t(1) << k;
    const int rowb = (k == 1) ? 4 : pick_chunk(G, k, req.chunk);
    const int rowd = rowb / 4;
    const int64_t ppbytes = std::max<int64_t>(npts, rowb);

    std::unique_ptr<WorkspaceLease> lease;
    if (!req.ws) lease.reset(new WorkspaceLease(G));
    Workspace &ws = req.ws ? *req.ws : *lease->ws;
    DBuf &ctl = ws.ctl, &z = ws.z, &xt = ws.xt, &s0 = ws.s0, &s1 = ws.s1, &pub = ws.pub,
         &pp = ws.pp, &tot = ws.tot, &mask = ws.mask, &loc = ws.loc, &pick = ws.pick;
    ctl.alloc(sizeof(Ctl), st);
    TPM_HIP(hipMemsetAsync(ctl.p, 0, sizeof(Ctl), st));
    z.alloc((size_t)G.n * 16, st);
    pp.alloc((size_t)ppbytes, st);
    TPM_HIP(hipMemsetAsync(pp.p, 0, (size_t)ppbytes, st));
    tot.alloc(4, st);
    const uint8_t *dmask = nullptr;
    if (req.vertex_mask) {
        mask.alloc((size_t)G.n, st);
        TPM_HIP(hipMemcpyAsync(mask.p, req.vertex_mask, (size_t)G.n, hipMemcpyHostToDevice, st));
        dmask = mask.as<uint8_t>();
    }
    k_z<<<grid_for(G.n), 256, 0, st>>>(G.n, k, G.color, G.fid, qs, dmask, req.seed, z.as<uint8_t>());

    int64_t lo = 0, hi = G.m;
    if (req.fin_lo < req.fin_hi) {
        lo = std::max<int64_t>(0, req.fin_lo);
        hi = std::min<int64_t>(G.m, req.fin_hi);
    }
    if (want_loc) {
        loc.alloc((size_t)std::max<int64_t>(1, hi - lo), st);
        TPM_HIP(hipMemsetAsync(loc.p, 0, (size_t)std::max<int64_t>(1, hi - lo), st));
        pick.alloc(sizeof(unsigned long long), st);
        TPM_HIP(hipMemsetAsync(pick.p, 0xFF, sizeof(unsigned long long), st));
    }

    if (k == 1) {
        k_single<<<grid_for(G.n), 256, 0, st>>>(G.n, z.as<uint8_t>(), pp.as<uint32_t>());
    } else if (G.m > 0) {
        xt.alloc((size_t)G.n * rowb, st);
        s0.alloc((size_t)std::max<int64_t>(1, G.R) * rowb, st);
        if (k > 2) s1.alloc((size_t)std::max<int64_t>(1, G.R) * rowb, st);
        if (k > 2 && G.nslots) {
            // published words carry a per-launch epoch; start every query from zero so
            // that a reused allocation never holds a word with a current epoch
            pub.alloc((size_t)G.nslots * rowd * 8, st);
            TPM_HIP(hipMemsetAsync(pub.p, 0, (size_t)G.nslots * rowd * 8, st));
        }
        // tiles covering the contributing positions of the last level
        const auto &tp = G.h_tile_p0;
        int32_t fin_tlo = 0, fin_thi = (int32_t)G.ntiles;
        if (lo > 0 || hi < G.m) {
            fin_tlo = (int32_t)(std::upper_bound(tp.begin(), tp.end(), (int32_t)lo) - tp.begin()) - 1;
            fin_thi = (int32_t)(std::lower_bound(tp.begin(), tp.end(), (int32_t)hi) - tp.begin());
            fin_tlo = std::max(0, fin_tlo);
            fin_thi = std::min<int32_t>((int32_t)G.ntiles, fin_thi);
        }
        const int64_t pts_end =
            req.max_chunks > 0 ? std::min<int64_t>(npts, (int64_t)req.max_chunks * rowb) : npts;
        LevelBufs B;
        B.z = z.as<uint8_t>();
        B.xt = xt.as<uint8_t>();
        B.s0 = s0.as<uint8_t>();
        B.s1 = s1.as<uint8_t>();
        B.pp = pp.as<uint8_t>();
        B.pub = pub.as<unsigned long long>();
        B.ctl = ctl.as<Ctl>();
        B.loc = want_loc ? loc.as<uint8_t>() : nullptr;
        if (k > 2) {
            size_t tb = 0;
            ws.w2.alloc(w2_bytes(G, tb), st);
            w2_place(G, ws.w2.as<uint8_t>(), tb, B);
        }
        enqueue_chunks(G, k, req.seed, rowb, pts_end, B, lo, hi, fin_tlo, fin_thi, &req, true, st);
    }
    k_total<<<1, 256, 0, st>>>((int32_t)npts, pp.as<uint8_t>(), tot.as<uint8_t>());
    unsigned long long hpick = ~0ull;
    if (want_loc && req.want_pick && hi > lo) {
        k_pick<<<grid_for(hi - lo), 256, 0, st>>>((int32_t)lo, (int32_t)hi, loc.as<uint8_t>(), G.peid,
                                                  pick.as<unsigned long long>());
        TPM_HIP(hipMemcpyAsync(&hpick, pick.p, sizeof(hpick), hipMemcpyDeviceToHost, st));
    }
    if (sink && want_loc) sink->consume(G, ws, loc.as<uint8_t>(), lo, hi, st);
    TPM_HIP(hipGetLastError());
    res.per_point.resize((size_t)npts);
    Ctl hctl{};
    TPM_HIP(hipMemcpyAsync(res.per_point.data(), pp.p, (size_t)npts, hipMemcpyDeviceToHost, st));
    TPM_HIP(hipMemcpyAsync(&res.total, tot.p, 1, hipMemcpyDeviceToHost, st));
    TPM_HIP(hipMemcpyAsync(&hctl, ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    if (want_loc && loc_host && hi > lo)
        TPM_HIP(hipMemcpyAsync(loc_host, loc.p, (size_t)(hi - lo), hipMemcpyDeviceToHost, st));
    TPM_HIP(hipStreamSynchronize(st));
    profile_collect();
    res.pick_eid = -1;
    res.pick_pos = -1;
    if (hpick != ~0ull) {
        res.pick_eid = (int64_t)(hpick >> 32);
        res.pick_pos = (int64_t)(hpick & 0xFFFFFFFFull);
    }
    if (hctl.err)
        throw Error{TPM_EDEVICE, "sieve kernel reported a look-back failure (code " +
                                     std::to_string(hctl.err) + ")"};
}

uint64_t colour_mask(const Graph &G, const int32_t *M, int32_t k) {
    if (G.q > 64) return ~0ull;
    uint64_t m = 0;
    for (int i = 0; i < k; ++i) {
        if (M[i] < 0) return ~0ull;  // a wildcard: any vertex
        m |= 1ull << M[i];
    }
    return m;
}

void run_sieve(const Graph &G, const SieveRequest &req, SieveResult &res, hipStream_t st) {
    run_sieve_impl(G, req, res, req.want_pick, nullptr, st);
}

void run_sieve_sink(const Graph &G, const SieveRequest &req, SieveResult &res, LocSink &sink,
                    hipStream_t st) {
    run_sieve_impl(G, req, res, true, nullptr, st, &sink);
}

void run_sieve_loc_all(const Graph &G, const SieveRequest &req, SieveResult &res,
                       uint8_t *loc_by_edge, hipStream_t st) {
    std::vector<uint8_t> bypos((size_t)std::max<int64_t>(1, G.m));
    SieveRequest r2 = req;
    r2.fin_lo = 0;
    r2.fin_hi = 0;
    run_sieve_impl(G, r2, res, true, bypos.data(), st);
    std::memset(loc_by_edge, 0, (size_t)G.edge_ids);
    if (G.m) {
        std::vector<int32_t> peid((size_t)G.m);
        TPM_HIP(hipMemcpy(peid.data(), G.peid, sizeof(int32_t) * G.m, hipMemcpyDeviceToHost));
        for (int64_t p = 0; p < G.m; ++p) loc_by_edge[peid[p]] = bypos[p];
    }
}

// ---------------------------------------------------------------- fixed scratch
namespace {
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Carving of one sieve query's buffers out of a block of `cap` bytes: the widest row
// (a power of two of points in [16, min(1024, 2^k)]) whose buffers fit.
struct FixedLayout {
    int rowb = 0;
    size_t ctl = 0, z = 0, xt = 0, s0 = 0, s1 = 0, pub = 0, pp = 0, end = 0;
};

FixedLayout fixed_layout(const Graph &G, int32_t k, int rowb) {
    const int64_t npts = int64_t(1) << k;
    FixedLayout L;
    L.rowb = rowb;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t off = at;
        at = align_up(at + std::max<size_t>(bytes, 1));
        return off;
    };
    L.ctl = take(sizeof(Ctl));
    L.z = take((size_t)G.n * 16);
    L.pp = take((size_t)std::max<int64_t>(npts, rowb));
    if (k >= 2 && G.m > 0) {
        const size_t R = (size_t)std::max<int64_t>(1, G.R);
        L.xt = take((size_t)G.n * rowb);
        L.s0 = take(R * rowb);
        if (k > 2) L.s1 = take(R * rowb);
        if (k > 2 && G.nslots) L.pub = take((size_t)G.nslots * (rowb / 4) * 8);
    }
    L.end = at;
    return L;
}

void fill_words(void *p, size_t bytes, hipStream_t st) {
    const int64_t words = (int64_t)(bytes / 4);
    if (words <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>(1024, (words + 255) / 256);
    k_fill32<<<grid, 256, 0, st>>>((uint32_t *)p, words, 0u);
}
}  // namespace

size_t fixed_scratch_need(const Graph &G, int32_t k) {
    return fixed_layout(G, k, k == 1 ? 4 : 16).end;
}

void enqueue_sieve_fixed(const Graph &G, const int32_t *M, int32_t k, uint64_t seed,
                         uint8_t *scratch, size_t cap, uint8_t *per_point, uint8_t *total,
                         uint32_t *err, hipStream_t st) {
    TPM_REQUIRE(total != nullptr, "total must not be NULL");
    QuerySlots qs = make_slots(G, M, k);
    const int64_t npts = int64_t(1) << k;
    FixedLayout L;
    if (k == 1) {
        L = fixed_layout(G, k, 4);
    } else {
        for (int rowb = (int)std::min<int64_t>(1024, std::max<int64_t>(npts, 16)); rowb >= 16; rowb >>= 1) {
            L = fixed_layout(G, k, rowb);
            if (L.end <= cap) break;
        }
    }
    if (L.end > cap)
        throw Error{TPM_ENOMEM, "query needs " + std::to_string(L.end) +
                                    " bytes of sieve state at its narrowest rows; the fixed scratch holds " +
                                    std::to_string(cap)};
    uint8_t *base = scratch;
    Ctl *ctl = (Ctl *)(base + L.ctl);
    uint8_t *z = base + L.z, *pp = base + L.pp;
    const int64_t ppbytes = std::max<int64_t>(npts, L.rowb);
    // the scratch keeps the previous call's contents: clear what must start at zero
    fill_words(ctl, sizeof(Ctl), st);
    fill_words(pp, (size_t)ppbytes, st);
    k_z<<<grid_for(G.n), 256, 0, st>>>(G.n, k, G.color, G.fid, qs, nullptr, seed, z);
    if (k == 1) {
        k_single<<<grid_for(G.n), 256, 0, st>>>(G.n, z, (uint32_t *)pp);
    } else if (G.m > 0) {
        if (L.pub) fill_words(base + L.pub, (size_t)G.nslots * (L.rowb / 4) * 8, st);
        LevelBufs B;
        B.z = z;
        B.xt = base + L.xt;
        B.s0 = base + L.s0;
        B.s1 = k > 2 ? base + L.s1 : nullptr;
        B.pp = pp;
        B.pub = L.pub ? (unsigned long long *)(base + L.pub) : nullptr;
        B.ctl = ctl;
        enqueue_chunks(G, k, seed, L.rowb, npts, B, 0, G.m, 0, (int32_t)G.ntiles, nullptr, false, st);
    }
    k_fixed_out<<<1, 256, 0, st>>>((int32_t)npts, pp, per_point, total, ctl, err);
    TPM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- static instance
namespace {
unsigned static_grid(const Graph &G, int64_t waves) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(G.num_cu, (waves + 15) / 16));
}
}  // namespace

void static_sieve(const Graph &G, const StaticGraph &S, const int32_t *M, int32_t k, uint64_t seed,
                  uint8_t *sv, size_t budget, hipStream_t st) {
    QuerySlots qs = make_slots(G, M, k);
    TPM_HIP(hipSetDevice(G.device));
    DBuf z;
    z.alloc((size_t)std::max<int32_t>(1, G.n) * 16, st);
    k_z<<<grid_for(G.n), 256, 0, st>>>(G.n, k, G.color, G.fid, qs, nullptr, seed, z.as<uint8_t>());
    if (k == 1) {  // one-vertex paths: S_u = sum over A of x_u^A = z_{u,0}
        k_single_v<<<grid_for(G.n), 256, 0, st>>>(G.n, z.as<uint8_t>(), sv);
        TPM_HIP(hipStreamSynchronize(st));
        return;
    }
    if (S.n == 0 || S.m == 0) {
        TPM_HIP(hipStreamSynchronize(st));
        return;
    }
    const int64_t npts = int64_t(1) << k;
    int64_t C = std::min<int64_t>(std::max<int64_t>(npts, 16), 1024);
    // rows: x, the sum, two backward rows and the forward rows F_2 .. F_{k-1}
    const int64_t nrows = (int64_t)k + 2;
    while (C > 16 && (double)nrows * S.n * C > (double)budget) C >>= 1;
    const int W = C >= 1024 ? 4 : (C >= 512 ? 2 : 1);
    const int lanes = (int)(C / (4 * W));
    const int64_t valid = std::min<int64_t>(npts, C);
    const size_t rowbytes = (size_t)S.n * (size_t)C;
    DBuf zs, X, sum, H0, H1, F;
    zs.alloc((size_t)S.n * 16, st);
    X.alloc(rowbytes, st);
    sum.alloc(rowbytes, st);
    H0.alloc(rowbytes, st);
    H1.alloc(rowbytes, st);
    F.alloc(rowbytes * (size_t)std::max(1, k - 2), st);
    k_zgather<<<grid_for(S.n), 256, 0, st>>>(S.n, S.vid, z.as<uint8_t>(), zs.as<uint8_t>());
    auto Frow = [&](int l) { return F.as<uint8_t>() + rowbytes * (size_t)(l - 2); };  // l = 2..k-1
    const uint8_t *lds_image = G.lds_image;
    auto gather = [&](bool fwd, const uint8_t *rows, uint32_t ylevel) {
        TPM_HIP(hipMemsetAsync(sum.p, 0, rowbytes, st));
        const int32_t *sg = fwd ? S.in_seg : S.out_seg, *gt = fwd ? S.in_gat : S.out_gat,
                      *ky = fwd ? S.in_key : S.out_key;
        const dim3 grid(static_grid(G, (S.m + kStaticTile - 1) / kStaticTile)), block(1024);
        uint8_t *sm = sum.as<uint8_t>();
        const int32_t rb = (int32_t)C;
        if (W == 4)
            hipLaunchKernelGGL((k_sgather<4>), grid, block, 0, st, S.m, sg, gt, ky, rows, sm, rb, lanes, seed, ylevel, lds_image);
        else if (W == 2)
            hipLaunchKernelGGL((k_sgather<2>), grid, block, 0, st, S.m, sg, gt, ky, rows, sm, rb, lanes, seed, ylevel, lds_image);
        else
            hipLaunchKernelGGL((k_sgather<1>), grid, block, 0, st, S.m, sg, gt, ky, rows, sm, rb, lanes, seed, ylevel, lds_image);
        TPM_HIP(hipGetLastError());
    };
    auto vertex = [&](const uint8_t *fin, uint8_t *out, int with_prod) {
        const uint8_t *sm = sum.as<uint8_t>(), *xr = X.as<uint8_t>();
        const dim3 grid(static_grid(G, S.n)), block(1024);
        const int32_t rb = (int32_t)C;
        if (W == 4)
            hipLaunchKernelGGL((k_svertex<4>), grid, block, 0, st, S.n, sm, xr, fin, out, with_prod, S.vid, sv, rb, lanes, lds_image);
        else if (W == 2)
            hipLaunchKernelGGL((k_svertex<2>), grid, block, 0, st, S.n, sm, xr, fin, out, with_prod, S.vid, sv, rb, lanes, lds_image);
        else
            hipLaunchKernelGGL((k_svertex<1>), grid, block, 0, st, S.n, sm, xr, fin, out, with_prod, S.vid, sv, rb, lanes, lds_image);
        TPM_HIP(hipGetLastError());
    };
    for (int64_t base = 0; base < npts; base += C) {
        if (valid < C) TPM_HIP(hipMemsetAsync(X.p, 0, rowbytes, st));
        const int32_t per_row = (int32_t)((valid + 15) / 16);
        k_xt<<<grid_for((int64_t)S.n * per_row), 256, 0, st>>>(S.n, k, (int32_t)valid, (int32_t)C, 0,
                                                                (uint32_t)base, zs.as<uint8_t>(),
                                                                X.as<uint8_t>(), nullptr, 0);
        // forward, Eq. (1): F_l = x * sum over in-arcs of y_{., l-1} F_{l-1}; the last
        // level adds sum_A F_k (G_k = 1)
        const uint8_t *prev = X.as<uint8_t>();
        for (int l = 2; l <= k; ++l) {
            gather(true, prev, (uint32_t)(l - 1));
            uint8_t *out = (l < k) ? Frow(l) : nullptr;
            vertex(nullptr, out, l == k ? 1 : 0);
            prev = out;
        }
        // backward: G_l = sum over out-arcs of y_{., l} x_w G_{w, l+1}, with H_l = x G_l
        // (H_k = x); adds sum_A F_l G_l
        const uint8_t *h = X.as<uint8_t>();
        for (int l = k - 1; l >= 1; --l) {
            gather(false, h, (uint32_t)l);
            uint8_t *hout = (l >= 2) ? ((l & 1) ? H1.as<uint8_t>() : H0.as<uint8_t>()) : nullptr;
            vertex(l == 1 ? X.as<uint8_t>() : Frow(l), hout, 0);
            h = hout;
        }
    }
    TPM_HIP(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------- multi-query rows
void multi_init(const Graph &G, MultiRow &row, hipStream_t st) {
    TPM_REQUIRE(row.ws != nullptr, "multi-query row without workspace");
    TPM_REQUIRE(row.W == 1 || row.W == 2 || row.W == 4, "W must be 1, 2 or 4");
    TPM_REQUIRE(row.lanes >= 1 && row.lanes <= 64, "lanes must be in [1, 64]");
    Workspace &ws = *row.ws;
    const int rowb = row.rowb(), rowd = rowb / 4;
    ws.ctl.alloc(sizeof(Ctl), st);
    TPM_HIP(hipMemsetAsync(ws.ctl.p, 0, sizeof(Ctl), st));
    ws.z.alloc((size_t)G.n * 16, st);
    // sized to the server's state budget: exact
    ws.xt.alloc((size_t)G.n * rowb, st, true);
    ws.s0.alloc((size_t)std::max<int64_t>(1, G.R) * rowb, st, true);
    ws.s1.alloc((size_t)std::max<int64_t>(1, G.R) * rowb, st, true);
    if (G.nslots) {
        ws.pub.alloc((size_t)G.nslots * rowd * 8, st, true);
        TPM_HIP(hipMemsetAsync(ws.pub.p, 0, (size_t)G.nslots * rowd * 8, st));
    }
    ws.pp.alloc((size_t)rowb, st);
    TPM_HIP(hipMemsetAsync(ws.pp.p, 0, (size_t)rowb, st));
    row.parity = 0;
}

void multi_prepare(const Graph &G, MultiRow &row, int lane0, int npts, const int32_t *M, int32_t k,
                   uint64_t seed, uint32_t base, const uint8_t *vertex_mask, hipStream_t st) {
    TPM_REQUIRE(k >= 2, "multi-query rows need k >= 2");
    TPM_REQUIRE(npts % (4 * row.W) == 0 && npts > 0, "group size must be whole lanes");
    TPM_REQUIRE(lane0 >= 0 && lane0 + npts / (4 * row.W) <= row.lanes, "group outside the row");
    TPM_REQUIRE(vertex_mask == nullptr, "vertex masks are not supported in multi-query rows");
    Workspace &ws = *row.ws;
    QuerySlots qs = make_slots(G, M, k);
    const int rowb = row.rowb();
    const int col = lane0 * 4 * row.W;
    k_z<<<grid_for(G.n), 256, 0, st>>>(G.n, k, G.color, G.fid, qs, nullptr, seed, ws.z.as<uint8_t>());
    k_xt<<<grid_for((int64_t)G.n * ((npts + 15) / 16)), 256, 0, st>>>(
        G.n, k, npts, rowb, col, base, ws.z.as<uint8_t>(), ws.xt.as<uint8_t>(), nullptr, 0);
    TPM_HIP(hipMemsetAsync(ws.pp.as<uint8_t>() + col, 0, (size_t)npts, st));
    TPM_HIP(hipGetLastError());
}

namespace {
void fill_step_params(const Graph &G, const MultiRow &row, StepParams &P) {
    Workspace &ws = *row.ws;
    P.psrc = G.psrc;
    P.gsrc = G.gsrc;
    P.pdst = G.pdst;
    P.peid = G.peid;
    P.orow = G.orow;
    P.pcol = G.pcol;
    P.xt = ws.xt.as<uint8_t>();
    P.sin = (row.parity ? ws.s1 : ws.s0).as<uint8_t>();
    P.sout = (row.parity ? ws.s0 : ws.s1).as<uint8_t>();
    P.tile_p0 = G.tile_p0;
    P.tile_pub = G.tile_pub;
    P.tile_lb = G.tile_lb;
    P.ntiles = (int32_t)G.ntiles;
    P.pub = ws.pub.as<unsigned long long>();
    P.ctl = ws.ctl.as<Ctl>();
    P.fin = ws.pp.as<uint32_t>();
    P.lds_image = G.lds_image;
    P.rowb = row.rowb();
    P.lanes = row.lanes;
    P.dtab = nullptr;
}

// How the lanes of one step find their y fingerprints: up to kMaxYGroups distinct
// (seed, level) pairs become a table that the kernel hashes once per window of 64
// positions (ymode 2, group index written into each lane's flags); otherwise a shared
// level lets lanes share the inner hash (ymode 1); otherwise every lane hashes alone.
struct StepYPlan {
    int32_t ymode = 0, ngroups = 0;
    uint32_t ylevel0 = 0;
    uint32_t glevel[kMaxYGroups] = {};
    uint64_t gseed[kMaxYGroups] = {};
    uint64_t gmask[kMaxYGroups] = {};
};

StepYPlan plan_y(StepLane *lanes, int nl) {
    StepYPlan Y;
    std::vector<std::pair<uint32_t, uint64_t>> groups;  // (level, seed)
    int32_t lvl = -1;
    bool same = true;
    for (int i = 0; i < nl; ++i) {
        lanes[i].flags &= ~(uint32_t)((kMaxYGroups - 1) << kLaneGroupShift);
        if (!(lanes[i].flags & kLaneActive)) continue;
        if (lvl < 0) lvl = (int32_t)lanes[i].ylevel;
        else same &= (int32_t)lanes[i].ylevel == lvl;
        const std::pair<uint32_t, uint64_t> key{lanes[i].ylevel, lanes[i].seed};
        if (std::find(groups.begin(), groups.end(), key) == groups.end()) groups.push_back(key);
    }
    if (!groups.empty() && groups.size() <= (size_t)kMaxYGroups) {
        std::sort(groups.begin(), groups.end());
        Y.ymode = 2;
        Y.ngroups = (int32_t)groups.size();
        for (int g = 0; g < Y.ngroups; ++g) {
            Y.glevel[g] = groups[(size_t)g].first;
            Y.gseed[g] = groups[(size_t)g].second;
        }
        for (int i = 0; i < nl; ++i) {
            if (!(lanes[i].flags & kLaneActive)) continue;
            const std::pair<uint32_t, uint64_t> key{lanes[i].ylevel, lanes[i].seed};
            const uint32_t g = (uint32_t)(std::find(groups.begin(), groups.end(), key) - groups.begin());
            lanes[i].flags |= g << kLaneGroupShift;
            Y.gmask[g] |= lanes[i].cmask;
        }
    } else if (same && lvl >= 0) {
        Y.ymode = 1;
        Y.ylevel0 = (uint32_t)lvl;
    }
    return Y;
}
}  // namespace

void multi_step(const Graph &G, MultiRow &row, const StepLane *lanes, hipStream_t st) {
    if (G.m == 0) return;
    Workspace &ws = *row.ws;
    StepParams P{};
    fill_step_params(G, row, P);
    for (int i = 0; i < 64; ++i) P.tab[i] = (i < row.lanes) ? lanes[i] : StepLane{0, 0, 0};
    const StepYPlan Y = plan_y(P.tab, row.lanes);
    P.ymode = Y.ymode;
    P.ngroups = Y.ngroups;
    P.ylevel0 = Y.ylevel0;
    for (int g = 0; g < kMaxYGroups; ++g) {
        P.glevel[g] = Y.glevel[g];
        P.gseed[g] = Y.gseed[g];
        P.gmask[g] = Y.gmask[g];
    }
    k_prep<<<1, 1, 0, st>>>(ws.ctl.as<Ctl>(), 1);
    {
        ProfileScope prof(st, 3, 0, row.rowb());
        launch_step_w(row.W, G, P, st);
    }
    TPM_HIP(hipGetLastError());
    row.parity ^= 1;
}

void multi_upload_tabs(MultiRow &row, const StepLane *lanes, int nsteps, hipStream_t st) {
    TPM_REQUIRE(nsteps >= 1 && nsteps <= 16, "steps per upload must be in [1, 16]");
    Workspace &ws = *row.ws;
    ws.tabs.alloc(sizeof(StepLane) * kTabStride * 16, st);
    thread_local std::vector<StepLane> host;
    host.assign((size_t)kTabStride * nsteps, StepLane{0, 0, 0});
    for (int s = 0; s < nsteps; ++s) {
        StepLane *dst = host.data() + (size_t)s * kTabStride;
        const StepLane *src = lanes + (size_t)s * 64;
        for (int i = 0; i < row.lanes; ++i) dst[i] = src[i];
        const StepYPlan Y = plan_y(dst, row.lanes);
        dst[64] = StepLane{0, Y.ylevel0, (uint32_t)Y.ymode | ((uint32_t)Y.ngroups << 8)};
        for (int g = 0; g < kMaxYGroups; ++g)
            dst[65 + g] = StepLane{Y.gseed[g], Y.glevel[g], 0, Y.gmask[g]};
    }
    TPM_HIP(hipMemcpyAsync(ws.tabs.p, host.data(), sizeof(StepLane) * host.size(),
                           hipMemcpyHostToDevice, st));
    // the host table is reused by the next upload on this thread
    TPM_HIP(hipStreamSynchronize(st));
}

StepGraph::~StepGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
}

void multi_steps_graph(const Graph &G, MultiRow &row, int nsteps, StepGraph &sg, hipStream_t st) {
    if (G.m == 0) return;
    TPM_REQUIRE(st != nullptr, "graph replay needs a created stream");
    TPM_REQUIRE(nsteps >= 1 && nsteps <= 16, "steps per graph must be in [1, 16]");
    Workspace &ws = *row.ws;
    TPM_REQUIRE(ws.tabs.p != nullptr, "lane tables were not uploaded");
    const void *key[8] = {ws.xt.p, ws.s0.p, ws.s1.p, ws.pub.p, ws.ctl.p, ws.pp.p, ws.tabs.p,
                          G.tile_p0};
    bool same = sg.exec && sg.W == row.W && sg.lanes == row.lanes && sg.nsteps == nsteps &&
                sg.parity == row.parity;
    for (int i = 0; i < 8 && same; ++i) same = sg.key[i] == key[i];
    if (!same) {
        if (sg.exec) TPM_HIP(hipGraphExecDestroy(sg.exec));
        sg.exec = nullptr;
        // only kernels are recorded (no memset or copy nodes)
        TPM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        hipGraph_t graph = nullptr;
        hipError_t err = hipSuccess;
        int parity = row.parity;
        for (int s = 0; s < nsteps && err == hipSuccess; ++s) {
            StepParams P{};
            MultiRow r2 = row;
            r2.parity = parity;
            fill_step_params(G, r2, P);
            P.dtab = ws.tabs.as<StepLane>() + (size_t)s * kTabStride;
            k_prep<<<1, 1, 0, st>>>(ws.ctl.as<Ctl>(), 1);
            launch_step_w(row.W, G, P, st);
            err = hipGetLastError();
            parity ^= 1;
        }
        hipError_t e2 = hipStreamEndCapture(st, &graph);
        if (err == hipSuccess) err = e2;
        if (err == hipSuccess) err = hipGraphInstantiate(&sg.exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        TPM_HIP(err);
        sg.W = row.W;
        sg.lanes = row.lanes;
        sg.nsteps = nsteps;
        sg.parity = row.parity;
        for (int i = 0; i < 8; ++i) sg.key[i] = key[i];
    }
    TPM_HIP(hipGraphLaunch(sg.exec, st));
    row.parity ^= (nsteps & 1);
}

void multi_read(const Graph &G, MultiRow &row, int lane0, int nl, uint8_t *out, hipStream_t st) {
    (void)G;
    const int lb = 4 * row.W;
    Ctl hctl{};
    TPM_HIP(hipMemcpyAsync(out, row.ws->pp.as<uint8_t>() + lane0 * lb, (size_t)nl * lb,
                           hipMemcpyDeviceToHost, st));
    TPM_HIP(hipMemcpyAsync(&hctl, row.ws->ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    TPM_HIP(hipStreamSynchronize(st));
    profile_collect();
    if (hctl.err)
        throw Error{TPM_EDEVICE, "step kernel reported a look-back failure (code " +
                                     std::to_string(hctl.err) + ")"};
}

}  // namespace tpm
